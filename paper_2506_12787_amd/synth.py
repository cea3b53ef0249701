"""Seeded synthetic inputs for the render path.

This module only draws random inputs (Gaussian parameters, transceiver
positions, MLP weights). It holds none of the method's arithmetic, and both the
HIP path's tests and the FP64 oracle consume its output.

Workload recipe (stand-in for the paper's indoor scenes, which are not
available; multipath() stands in for ray-traced path lists): means uniform over the pixel grid; log-scales uniform in
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


def multipath(b: int, seed: int, rx=(3.0, 0.5, 1.2), room=((0.0, 0.0, 0.0), (6.0, 6.0, 3.0)), max_order: int = 2,
              gamma: float = 0.6, jitter: float = 0.05):
    """Multipath lists of b transmitter positions seen from a fixed receiver in
    a box room (a stand-in for ray-traced path lists): the line-of-sight path
    and the specular reflections off the six walls up to `max_order` bounces,
    by mirror images of the transmitter. Path l arrives from the direction of
    its image source; its power coefficient is gamma^bounces / length times a
    seeded factor in [1 - jitter, 1 + jitter]. Returns (paths, counts, tx):
    paths float32 [b][L][3] = (rho, azimuth in [0, 2 pi), elevation in
    [0, pi/2]) with unused slots zero, counts int32 [b], tx float32 [b][3].
    Elevation is the angle above the array plane; a source below it arrives at
    the mirrored elevation (a planar array cannot tell them apart)."""
    rng = np.random.default_rng(seed)
    lo = np.asarray(room[0], np.float64)
    hi = np.asarray(room[1], np.float64)
    rx = np.asarray(rx, np.float64)
    tx = lo + (hi - lo) * rng.uniform(0.05, 0.95, (b, 3))
    images = [((0, 0, 0), 0)]
    # image index k per axis (|k| reflections off that axis' two walls); total bounces = |kx| + |ky| + |kz|
    for kx in range(-max_order, max_order + 1):
        for ky in range(-max_order, max_order + 1):
            for kz in range(-max_order, max_order + 1):
                if (kx, ky, kz) == (0, 0, 0):
                    continue
                if abs(kx) + abs(ky) + abs(kz) <= max_order:
                    images.append(((kx, ky, kz), abs(kx) + abs(ky) + abs(kz)))
    L = len(images)
    paths = np.zeros((b, L, 3), np.float64)
    for i in range(b):
        for l, (k, order) in enumerate(images):
            src = np.empty(3)
            for a in range(3):
                size = hi[a] - lo[a]
                x = tx[i, a] - lo[a]
                # mirror images of a point in [0, size]: for k even x + k size, for k odd (k + 1) size - x
                src[a] = lo[a] + (k[a] * size + x if k[a] % 2 == 0 else (k[a] + 1) * size - x)
            d = src - rx
            dist = float(np.linalg.norm(d))
            rho = gamma ** order / dist * rng.uniform(1.0 - jitter, 1.0 + jitter)
            az = np.arctan2(d[1], d[0]) % (2.0 * np.pi)
            el = abs(np.arctan2(d[2], np.hypot(d[0], d[1])))
            paths[i, l] = (rho, az, el)
    counts = np.full(b, L, np.int32)
    return (np.ascontiguousarray(paths, dtype=np.float32), counts,
            np.ascontiguousarray(tx, dtype=np.float32))


PAPER_KEYS = ("center_x", "center_y", "chol_l1", "chol_l2", "chol_l3", "atten_logit", "psi_re", "psi_im")
# (out, in) of the paper MLP's layers: 81 inputs (10 centre bands, 6 position bands), eight layers of 156 whose
# layers 3, 5 and 7 also take the 81 inputs, and an output layer of 5
PAPER_LAYER_SHAPES = ((156, 81), (156, 156), (156, 237), (156, 156), (156, 237), (156, 156), (156, 237), (156, 156),
                      (5, 156))


def paper_gaussians(n: int, seed: int, diag=(1.0, 8.0)) -> dict:
    """n raw paper-model Gaussians: centres whose tanh map spreads them over the grid, Cholesky diagonals of
    `diag` pixels with random signs and shears in [-3, 3], gate logits ~ N(0, 1), complex responses ~ N(0, 1)^2."""
    rng = np.random.default_rng(seed)
    u = lambda lo, hi: rng.uniform(lo, hi, n)
    sgn = lambda: np.where(rng.uniform(size=n) < 0.5, -1.0, 1.0)
    g = {"center_x": np.arctanh(u(-0.98, 0.98)), "center_y": np.arctanh(u(-0.97, 0.97)),
         "chol_l1": sgn() * u(*diag), "chol_l2": u(-3, 3), "chol_l3": sgn() * u(*diag),
         "atten_logit": rng.normal(0, 1, n), "psi_re": rng.normal(0, 1, n), "psi_im": rng.normal(0, 1, n)}
    return {k: np.ascontiguousarray(v, np.float32) for k, v in g.items()}


def paper_mlp_weights(seed: int, out_scale: float = 1.0, bias_std: float = 0.05):
    """Xavier-uniform weights of the paper MLP (output layer times out_scale) and N(0, bias_std) biases."""
    rng = np.random.default_rng(seed)
    Ws, bs = [], []
    for o, i in PAPER_LAYER_SHAPES:
        bound = np.sqrt(6.0 / (o + i))
        w = rng.uniform(-bound, bound, (o, i)) * (out_scale if o == 5 else 1.0)
        Ws.append(np.ascontiguousarray(w, np.float32))
        bs.append(np.ascontiguousarray(rng.normal(0, bias_std, o), np.float32))
    return Ws, bs
