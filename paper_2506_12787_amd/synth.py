"""Seeded synthetic inputs for the render path.

This module only draws random inputs (Gaussian parameters, transceiver
positions, MLP weights). It holds none of the method's arithmetic, and both the
HIP path's tests and the FP64 oracle consume its output.

Workload recipe (stand-in for the paper's indoor scenes, which are not
available): means uniform over the pixel grid; log-scales uniform in
[log a, log b] pixels; rotation uniform in [0, pi); opacity logit ~ N(0, 1);
amplitude uniform in [0, 1); depth uniform in [0.5, 10); transceiver positions
uniform in a 6 x 6 x 3 m room. MLP weights are Xavier-uniform (gain 1) with zero
biases, and the output layer is multiplied by `out_scale` (0.01 by default).
"""
from __future__ import annotations

import numpy as np

PARAM_NAMES = ("mean_x", "mean_y", "log_scale_x", "log_scale_y", "rotation", "opacity_logit", "amplitude", "depth")


def gaussians(n: int, H: int, W: int, seed: int, scale_range=(1.0, 12.0), depth_range=(0.5, 10.0)) -> dict:
    """n canonical 2D Gaussians as FP32 arrays (pixel units)."""
    rng = np.random.default_rng(seed)
    lo, hi = np.log(scale_range[0]), np.log(scale_range[1])
    d = {
        "mean_x": rng.uniform(0.0, W, n),
        "mean_y": rng.uniform(0.0, H, n),
        "log_scale_x": rng.uniform(lo, hi, n),
        "log_scale_y": rng.uniform(lo, hi, n),
        "rotation": rng.uniform(0.0, np.pi, n),
        "opacity_logit": rng.normal(0.0, 1.0, n),
        "amplitude": rng.uniform(0.0, 1.0, n),
        "depth": rng.uniform(depth_range[0], depth_range[1], n),
    }
    return {k: np.ascontiguousarray(v, dtype=np.float32) for k, v in d.items()}


def tx_positions(b: int, seed: int, room=((0.0, 0.0, 0.0), (6.0, 6.0, 3.0))) -> np.ndarray:
    rng = np.random.default_rng(seed)
    lo = np.asarray(room[0], np.float64)
    hi = np.asarray(room[1], np.float64)
    return np.ascontiguousarray(lo + (hi - lo) * rng.uniform(0.0, 1.0, (b, 3)), dtype=np.float32)


def mlp_weights(seed: int, mean_bands: int = 6, tx_bands: int = 10, hidden: int = 256, n_hidden: int = 4,
                out_dim: int = 7, out_scale: float = 0.01):
    """FP32 weights [W_l (out, in)] and biases [b_l] of the deformation MLP."""
    rng = np.random.default_rng(seed)
    d_in = 2 * (2 * mean_bands + 1) + 3 * (2 * tx_bands + 1)
    dims = [d_in] + [hidden] * n_hidden + [out_dim]
    Ws, bs = [], []
    for l in range(len(dims) - 1):
        fan_in, fan_out = dims[l], dims[l + 1]
        bound = np.sqrt(6.0 / (fan_in + fan_out))
        w = rng.uniform(-bound, bound, (fan_out, fan_in))
        if l == len(dims) - 2:
            w = w * out_scale
        Ws.append(np.ascontiguousarray(w, dtype=np.float32))
        bs.append(np.zeros(fan_out, dtype=np.float32))
    return Ws, bs


def targets_like(shape, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(rng.uniform(0.0, 1.0, shape), dtype=np.float32)
