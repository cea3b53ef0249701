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
