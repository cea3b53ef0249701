"""Shared helpers for the GPU tests: seeded problems and the parity rule."""
from __future__ import annotations

import numpy as np

from oracle import model as M
from paper_2506_12787_amd import synth

TOL_REL = 1e-5  # normwise relative L-infinity bound of the FP32 path vs the FP64 oracle


def problem(n, H, W, seed, scale_range=(1.0, 12.0)):
    g = synth.gaussians(n, H, W, seed=seed, scale_range=scale_range)
    return g, M.Scene.from_arrays(g, H, W)


def mlp_f64(Ws, bs):
    return M.MLP([w.astype(np.float64) for w in Ws], [b.astype(np.float64) for b in bs])


def parity(gpu: np.ndarray, res: M.RenderResult, tol_rel=TOL_REL):
    """Decision-ambiguity parity: every pixel must lie within tol of one of the
    oracle's reachable values (tol plus the oracle's bound for unforked flags).
    Returns a report dict; raises AssertionError on failure."""
    g = np.asarray(gpu, np.float64).ravel()
    scale = float(np.abs(res.C).max()) if len(res.C) else 0.0
    tol = tol_rel * scale
    err_primary = np.abs(g - res.C)
    ML = res.leaves.shape[1]
    idx = np.arange(ML)[None, :] < res.nleaves[:, None]
    lerr = np.where(idx, np.abs(res.leaves - g[:, None]), np.inf).min(axis=1)
    ok = (err_primary <= tol) | (lerr <= tol) | (err_primary <= tol + res.bound)
    flagged = res.nflags > 0
    rep = dict(
        pixels=len(g), scale=scale, tol=tol,
        flagged_pixels=int(flagged.sum()),
        took_other_branch=int(((err_primary > tol) & ok).sum()),
        worst_unflagged=float(err_primary[~flagged].max()) if (~flagged).any() else 0.0,
        worst_unflagged_rel=float(err_primary[~flagged].max() / scale) if (~flagged).any() and scale > 0 else 0.0,
        overflow_pixels=int((res.overflow > 0).sum()),
        failures=int((~ok).sum()),
    )
    if not ok.all():
        bad = np.nonzero(~ok)[0][:10]
        raise AssertionError(f"parity failed at {rep['failures']} pixels; first {bad.tolist()} "
                             f"gpu={g[bad].tolist()} oracle={res.C[bad].tolist()} report={rep}")
    return rep


# ---------------------------------------------------------------------------
# Hand-worked fixtures under tests/golden/: expected values are closed forms
# written as small arithmetic expressions (numbers, + - * / **, exp, sqrt, and
# names bound by the case's "let").
# ---------------------------------------------------------------------------
GOLDEN_DIR = __import__("os").path.join(__import__("os").path.dirname(__file__), "golden")


def golden(name: str) -> dict:
    import json
    import os
    with open(os.path.join(GOLDEN_DIR, name)) as f:
        return json.load(f)


def closed_form(expr: str, env: dict | None = None) -> float:
    """Evaluate a fixture's closed form in float64 (no other names or calls)."""
    import ast
    import math
    funcs = {"exp": math.exp, "sqrt": math.sqrt}
    env = env or {}
    ops = {ast.Add: lambda a, b: a + b, ast.Sub: lambda a, b: a - b, ast.Mult: lambda a, b: a * b,
           ast.Div: lambda a, b: a / b, ast.Pow: lambda a, b: a ** b}

    def ev(n):
        if isinstance(n, ast.Expression):
            return ev(n.body)
        if isinstance(n, ast.Constant) and isinstance(n.value, (int, float)):
            return float(n.value)
        if isinstance(n, ast.BinOp) and type(n.op) in ops:
            return ops[type(n.op)](ev(n.left), ev(n.right))
        if isinstance(n, ast.UnaryOp) and isinstance(n.op, (ast.USub, ast.UAdd)):
            v = ev(n.operand)
            return -v if isinstance(n.op, ast.USub) else v
        if isinstance(n, ast.Name) and n.id in env:
            return env[n.id]
        if isinstance(n, ast.Call) and isinstance(n.func, ast.Name) and n.func.id in funcs and len(n.args) == 1:
            return funcs[n.func.id](ev(n.args[0]))
        raise ValueError(f"unsupported closed form: {expr!r}")

    return ev(ast.parse(expr, mode="eval"))


def golden_pixel(px: dict) -> tuple:
    """(C, T) of one fixture pixel, its 'let' names bound first."""
    env = {k: closed_form(v) for k, v in px.get("let", {}).items()}
    return closed_form(px["C"], env), closed_form(px["T"], env)


def golden_scene(case: dict) -> dict:
    return {k: np.asarray(v, np.float32) for k, v in case["gaussians"].items()}
