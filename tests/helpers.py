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


# ---------------------------------------------------------------------------
# Gradient checks with derived componentwise bounds (the GPU backward against
# the oracle's FP64 analytic gradient, Sec. 3.2 blending rule differentiated
# with decisions held). The unit roundoffs: FP32 2^-24, BF16 operands 2^-8.
U32, U16 = 2.0 ** -24, 2.0 ** -8


def unflagged_weights(scene: M.Scene, deltas, seed, pix_per_query=None):
    """One weight array of H*W per query: random normal weights on (sampled, or
    all) pixels whose every decision, for these residuals (None: static), is
    clear of its threshold; zero elsewhere. Returns (weights, kept pixels)."""
    H, W = scene.H, scene.W
    rng = np.random.default_rng(seed)
    order = M.depth_order(scene.depth)
    out, kept = [], 0
    for d in deltas:
        idx = (rng.choice(H * W, pix_per_query, replace=False) if pix_per_query else np.arange(H * W))
        px, py = (idx % W).astype(np.int32), (idx // W).astype(np.int32)
        res = M.composite(M.gaussians_for_raster(M.deform(scene, d), scene.depth), order, px, py)
        ok = idx[res.nflags == 0]
        w = np.zeros(H * W)
        w[ok] = rng.normal(0, 1, len(ok))
        out.append(w)
        kept += len(ok)
    return out, kept


def gradient_bound_factors(ref: dict, n_layers: int, pairs: int, bf16: bool):
    """(c_r, c_mlp): bound = c_r * magnitude sum of the compositing and covariance
    part, c_mlp * magnitude sum of the network's part.
      c_r = (3 m + 32) u32, m the longest composited run at a weighted pixel (the
          replay divides T by (1 - alpha) once per entry, the forward multiplied
          once per entry; 32 covers q, exp and the chain);
      c_mlp = 3 (L + 1) u + L K u32 + 4 sqrt(P) u32 + c_r, u the unit roundoff of
          the network's operands, K = 256 (FP32 accumulation inside each
          product), P pairs summed per weight (blocked FP32 sums)."""
    m = ref["replay"]
    c_r = (3 * m + 32) * U32
    c_mlp = 3 * (n_layers + 1) * (U16 if bf16 else U32) + n_layers * 256 * U32 + 4 * np.sqrt(pairs) * U32 + c_r
    return c_r, c_mlp


def within_bound(name, got, ref, bound):
    """Worst componentwise |got - ref| / bound (printed)."""
    got = np.asarray(got, np.float64)
    err = np.abs(got - ref)
    scale = max(float(np.abs(ref).max()), 1e-300)
    ratio = float((err / np.maximum(bound, 1e-300)).max())
    print(f"  {name}: normwise err {err.max() / scale:.2e}, worst err / bound {ratio:.3f}", flush=True)
    return ratio


def check_gradients(got: dict, ref: dict, params, n_layers: int, pairs: int, bf16: bool):
    """Every component of every block within its derived bound: the rounding
    terms above plus the oracle's allowance for the network's decisions and
    operands (W_flip, b_flip, pe_flip; with the implementation's ReLU pattern
    held only the operand differences within binary32 slack remain)."""
    assert not ref["flagged"].any()
    c_r, c_mlp = gradient_bound_factors(ref, n_layers, pairs, bf16)
    print(f"  longest run {ref['replay']}: bound factors {c_r:.2e} / {c_mlp:.2e}", flush=True)
    worst = {}
    for j, k in enumerate(params):
        bound = c_r * ref["base_abs"][:, j]
        if j < 2 and n_layers:
            bound = bound + c_mlp * ref["pe_abs"][:, j] + ref["pe_flip"][:, j]
        worst[k] = within_bound(k, got[k], ref["base"][:, j], bound + 1e-300)
    for l in range(n_layers):
        worst[f"W{l}"] = within_bound(f"W{l}", got["weight"][l], ref["W"][l],
                                      c_mlp * ref["W_abs"][l] + ref["W_flip"][l])
        worst[f"b{l}"] = within_bound(f"b{l}", got["bias"][l], ref["b"][l], c_mlp * ref["b_abs"][l] + ref["b_flip"][l])
    bad = {k: v for k, v in worst.items() if not v <= 1.0}
    assert not bad, bad
    return worst
