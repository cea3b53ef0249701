"""FP64 reference model of the SwiftWRF render path (the oracle).

TEST INFRASTRUCTURE ONLY. Only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark import this package. The product path (the
HIP library and its Python binding) never imports, links or calls it, and this
package imports nothing from the product path. Everything here is written from
the paper's definitions, step by step, in float64:

  * positional encoding gamma(.)          -- Sec. 4.2, eq. (posenc)
  * deformation MLP F_theta                -- Sec. 4.2, residual prediction eq.
  * deformed primitive set G^s = G^0 + dG  -- Sec. 4.2, GOP reference + residuals
  * 2D Gaussian kernel K = delta exp(-q/2) -- Sec. 4.1, kernel-weight eq.
  * front-to-back compositing              -- Sec. 3.2, alpha-blending eq.

Where the paper is silent the readings listed in the design notes are used:
log-scale + rotation covariance, opacity as sigmoid(logit), one real amplitude,
a per-Gaussian depth that fixes the blending order, the 3-sigma cutoff q <= 9,
the alpha clamp 0.99, the alpha skip 1/255 and the transmittance floor 1e-4.

Parity status: no function here is checked against a value printed in the
paper (the paper prints no worked example). Each is pinned by closed forms,
special cases, brute force and finite differences in tests/test_oracle_*.py.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

# FP32 constants of the blending rule, widened exactly to FP64.
ALPHA_MAX = float(np.float32(0.99))
ALPHA_MIN = float(np.float32(1.0) / np.float32(255.0))
T_MIN = float(np.float32(1e-4))
Q_MAX = 9.0
# Binning superset margin added to the 3-sigma half extent (pixels).
EXTENT_EPS = float(np.float32(1e-3))

# Relative flag margins for the decision-ambiguity rule (q vs 9, alpha vs
# 1/255, T' vs 1e-4).
DEFAULT_MARGINS = (1e-4, 1e-4, 1e-3)

MEAN_BANDS = 6   # PE frequency bands of the 2D canonical mean
TX_BANDS = 10    # PE frequency bands of the 3D transceiver position
DEFAULT_ROOM = ((0.0, 0.0, 0.0), (6.0, 6.0, 3.0))

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle_raster.so")
_lib = None


def build_raster(force: bool = False) -> str:
    """Compile raster.c with gcc (OpenMP) into liboracle_raster.so."""
    src = os.path.join(_HERE, "raster.c")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, src, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _raster():
    global _lib
    if _lib is None:
        build_raster()
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        lib.oracle_render.argtypes = [ctypes.c_int64] + [P] * 10 + [P, ctypes.c_int64] + [P] * 13
        lib.oracle_render.restype = None
        lib.oracle_grad.argtypes = [ctypes.c_int64] + [P] * 11 + [ctypes.c_int64] + [P] * 6
        lib.oracle_grad.restype = None
        lib.oracle_max_leaves.restype = ctypes.c_int
        lib.oracle_set_threads.argtypes = [ctypes.c_int]
        lib.oracle_set_threads.restype = ctypes.c_int
        lib.oracle_render_held.argtypes = [ctypes.c_int64] + [P] * 16 + [ctypes.c_int64] + [P] * 3
        lib.oracle_render_held.restype = None
        _lib = lib
    return _lib


def set_threads(n: int = 0) -> int:
    """Set the compositor's OpenMP thread count (n <= 0 leaves it); returns the count in effect."""
    return int(_raster().oracle_set_threads(int(n)))


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


# ---------------------------------------------------------------------------
# Positional encoding (Sec. 4.2, eq. posenc)
# ---------------------------------------------------------------------------
def posenc(v: np.ndarray, L: int) -> np.ndarray:
    """gamma(v) = [v, sin(2^0 pi v) .. sin(2^{L-1} pi v), cos(2^0 pi v) .. cos(2^{L-1} pi v)].

    The sine and cosine act element-wise on the d components; within each
    frequency block the components keep their order. Output width d(2L+1).
    """
    v = np.asarray(v, dtype=np.float64)
    parts = [v]
    for k in range(L):
        parts.append(np.sin((2.0 ** k) * np.pi * v))
    for k in range(L):
        parts.append(np.cos((2.0 ** k) * np.pi * v))
    return np.concatenate(parts, axis=-1)


def normalize_tx(tx: np.ndarray, room=DEFAULT_ROOM) -> np.ndarray:
    lo = np.asarray(room[0], np.float64)
    hi = np.asarray(room[1], np.float64)
    return (np.asarray(tx, np.float64) - lo) / (hi - lo)


def normalize_mean(mx, my, H: int, W: int) -> np.ndarray:
    return np.stack([np.asarray(mx, np.float64) / W, np.asarray(my, np.float64) / H], axis=-1)


# ---------------------------------------------------------------------------
# Deformation MLP (Sec. 4.2): inputs [gamma(mu_hat) | gamma(s_hat)], ReLU hidden
# layers, linear output of 7 residuals (d_mu 2, d_logscale 2, d_rot 1,
# d_logit 1, d_amp 1).
# ---------------------------------------------------------------------------
def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round to the nearest bfloat16 value (8 significant bits), ties to even."""
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)               # x = m * 2^e, 0.5 <= |m| < 1
    m = np.rint(m * 256.0) / 256.0   # numpy rint rounds half to even
    return np.ldexp(m, e)


@dataclass
class MLP:
    W: list  # W[l]: (out, in) float64
    b: list  # b[l]: (out,) float64

    @property
    def n_layers(self):
        return len(self.W)


def mlp_forward(x_mean: np.ndarray, x_tx: np.ndarray, mlp: MLP, bf16: bool = False, relu_masks=None):
    """Run F_theta on rows. x_mean: (R, 26) gamma of the canonical mean; x_tx:
    (R, 63) or (63,) gamma of the transceiver position. Returns (out, pre, act)
    where pre[l] / act[l] are the pre-activation and post-ReLU of hidden l.

    bf16=True emulates the BF16 kernel's operand rounding: the mean features,
    all weight matrices acting on activations and every hidden activation are
    rounded to bfloat16 (ties to even); the transceiver part of layer 1, the
    biases and all accumulation stay exact (float64 here).

    relu_masks (one boolean array per hidden layer, shaped like its
    pre-activation) replaces each ReLU by multiplication with the given mask:
    the network with its activation pattern held, used by finite differences
    of the decisions-held objective."""
    d_mean = x_mean.shape[-1]
    W1 = mlp.W[0]
    W1m, W1s = W1[:, :d_mean], W1[:, d_mean:]
    rnd = bf16_round if bf16 else (lambda a: a)
    xs = np.atleast_2d(x_tx)
    relu = (lambda p, l: np.maximum(p, 0.0)) if relu_masks is None else (lambda p, l: p * relu_masks[l])
    pre0 = rnd(x_mean) @ rnd(W1m).T + xs @ W1s.T + mlp.b[0]
    pres, acts = [pre0], [relu(pre0, 0)]
    h = acts[-1]
    for l in range(1, mlp.n_layers - 1):
        p = rnd(h) @ rnd(mlp.W[l]).T + mlp.b[l]
        pres.append(p)
        acts.append(relu(p, l))
        h = acts[-1]
    out = rnd(h) @ rnd(mlp.W[-1]).T + mlp.b[-1]
    return out, pres, acts


# ---------------------------------------------------------------------------
# Scene and deformation (Sec. 4.2: G^s = {mu^0 + d_mu, Sigma, psi^0 + d_psi, ...})
# ---------------------------------------------------------------------------
@dataclass
class Scene:
    """Canonical Gaussians in FP64 (the FP32 inputs widened exactly)."""
    mx: np.ndarray
    my: np.ndarray
    lsx: np.ndarray
    lsy: np.ndarray
    rot: np.ndarray
    logit: np.ndarray
    amp: np.ndarray
    depth: np.ndarray
    H: int
    W: int

    @property
    def n(self):
        return len(self.mx)

    @staticmethod
    def from_arrays(d: dict, H: int, W: int) -> "Scene":
        f = lambda k: np.asarray(d[k], dtype=np.float32).astype(np.float64)
        return Scene(f("mean_x"), f("mean_y"), f("log_scale_x"), f("log_scale_y"), f("rotation"),
                     f("opacity_logit"), f("amplitude"), f("depth"), int(H), int(W))


def deform(scene: Scene, delta: np.ndarray | None) -> dict:
    """Deformed per-Gaussian parameters for one query (delta: (n, 7) or None)."""
    if delta is None:
        delta = np.zeros((scene.n, 7))
    mx = scene.mx + delta[:, 0]
    my = scene.my + delta[:, 1]
    lsx = scene.lsx + delta[:, 2]
    lsy = scene.lsy + delta[:, 3]
    rot = scene.rot + delta[:, 4]
    logit = scene.logit + delta[:, 5]
    amp = scene.amp + delta[:, 6]
    opacity = 1.0 / (1.0 + np.exp(-logit))
    return dict(mx=mx, my=my, lsx=lsx, lsy=lsy, rot=rot, logit=logit, opacity=opacity, amp=amp)


def deltas(scene: Scene, mlp: MLP | None, tx: np.ndarray, room=DEFAULT_ROOM, bf16=False):
    """Residuals F_theta(gamma(mu_n), gamma(s)) for every Gaussian at one TX."""
    if mlp is None:
        return None
    xm = posenc(normalize_mean(scene.mx, scene.my, scene.H, scene.W), MEAN_BANDS)
    xs = posenc(normalize_tx(tx, room), TX_BANDS)
    out, _, _ = mlp_forward(xm, xs, mlp, bf16=bf16)
    return out


# ---------------------------------------------------------------------------
# Covariance and its inverse
# ---------------------------------------------------------------------------
def covariance(lsx, lsy, rot):
    """Sigma = R diag(e^{2 lsx}, e^{2 lsy}) R^T with R the rotation by `rot`."""
    with np.errstate(invalid="ignore", over="ignore"):
        c, s = np.cos(rot), np.sin(rot)
        ex, ey = np.exp(2.0 * lsx), np.exp(2.0 * lsy)
        sxx = c * c * ex + s * s * ey
        sxy = c * s * (ex - ey)
        syy = s * s * ex + c * c * ey
    return sxx, sxy, syy


def inverse2(sxx, sxy, syy):
    """Inverse of the symmetric 2x2 matrix [[sxx, sxy], [sxy, syy]].
    Returns (ixx, ixy, iyy, det, live) with live = finite and det > 0."""
    det = sxx * syy - sxy * sxy
    with np.errstate(divide="ignore", invalid="ignore"):
        ixx = syy / det
        ixy = -sxy / det
        iyy = sxx / det
    live = np.isfinite(det) & (det > 0) & np.isfinite(ixx) & np.isfinite(ixy) & np.isfinite(iyy)
    return ixx, ixy, iyy, det, live


def depth_order(depth: np.ndarray) -> np.ndarray:
    """Indices in ascending (depth as its FP32 value, id); NaN depths last."""
    d = np.asarray(depth, np.float32).astype(np.float64)
    ids = np.arange(len(d))
    nan = np.isnan(d)
    d = np.where(nan, np.inf, d)
    return np.lexsort((ids, d, nan.astype(np.int8)))


def depth_bits(depth: np.ndarray) -> np.ndarray:
    """Order-preserving map of FP32 depth to uint32 (-0 is mapped like +0)."""
    f = np.asarray(depth, np.float32).copy()
    f[f == 0] = 0.0
    u = f.view(np.uint32).astype(np.uint64)
    neg = (u >> 31) == 1
    out = np.where(neg, (~u) & 0xFFFFFFFF, u | 0x80000000)
    return out.astype(np.uint32)


# ---------------------------------------------------------------------------
# Rendering
# ---------------------------------------------------------------------------
@dataclass
class RenderResult:
    C: np.ndarray        # (npix,) primary value
    T: np.ndarray        # (npix,) primary final transmittance
    ncontrib: np.ndarray
    last: np.ndarray
    sig: np.ndarray
    mono: np.ndarray
    nflags: np.ndarray
    leaves: np.ndarray   # (npix, max_leaves)
    nleaves: np.ndarray
    bound: np.ndarray
    overflow: np.ndarray


def gaussians_for_raster(g: dict, depth=None):
    """Per-Gaussian arrays the compositor needs, from deformed parameters.
    A Gaussian takes part if its parameters are finite, det Sigma > 0 and its
    depth (when given) is not NaN."""
    sxx, sxy, syy = covariance(g["lsx"], g["lsy"], g["rot"])
    ixx, ixy, iyy, det, live = inverse2(sxx, sxy, syy)
    fin = np.isfinite(g["mx"]) & np.isfinite(g["my"]) & np.isfinite(g["opacity"]) & np.isfinite(g["amp"])
    if depth is not None:
        fin &= ~np.isnan(np.asarray(depth, np.float64))
    live = live & fin
    z = lambda a: np.ascontiguousarray(np.where(live, a, 0.0), np.float64)
    return dict(mx=z(g["mx"]), my=z(g["my"]), ixx=z(ixx), ixy=z(ixy), iyy=z(iyy), op=z(g["opacity"]),
                amp=z(g["amp"]), live=np.ascontiguousarray(live.astype(np.int8)), sxx=sxx, sxy=sxy, syy=syy)


def full_grid(H: int, W: int):
    ys, xs = np.meshgrid(np.arange(H, dtype=np.int32), np.arange(W, dtype=np.int32), indexing="ij")
    return xs.ravel().copy(), ys.ravel().copy()


def composite(rg: dict, order: np.ndarray, pix_x: np.ndarray, pix_y: np.ndarray,
              margins=DEFAULT_MARGINS, period: float = 0.0) -> RenderResult:
    """FP64 brute-force compositing of the listed pixels (see raster.c). period:
    the grid width W when azimuth wraps around (nearest image of each mean), 0
    for a plain plane."""
    lib = _raster()
    n = len(rg["mx"])
    npix = len(pix_x)
    ML = lib.oracle_max_leaves()
    order = np.ascontiguousarray(order, np.int64)
    px = np.ascontiguousarray(pix_x, np.int32)
    py = np.ascontiguousarray(pix_y, np.int32)
    consts = np.array([ALPHA_MAX, ALPHA_MIN, T_MIN, Q_MAX, float(period)], np.float64)
    marg = None if margins is None else np.array(margins, np.float64)
    C = np.zeros(npix); T = np.zeros(npix)
    nc = np.zeros(npix, np.int64); last = np.zeros(npix, np.int64)
    sig = np.zeros(npix, np.uint64); mono = np.zeros(npix, np.int8)
    nflags = np.zeros(npix, np.int32); leaves = np.zeros((npix, ML)); nleaves = np.zeros(npix, np.int32)
    bound = np.zeros(npix); overflow = np.zeros(npix, np.int32)
    lib.oracle_render(n, _ptr(rg["mx"]), _ptr(rg["my"]), _ptr(rg["ixx"]), _ptr(rg["ixy"]), _ptr(rg["iyy"]),
                      _ptr(rg["op"]), _ptr(rg["amp"]), _ptr(rg["live"]), _ptr(order), _ptr(consts),
                      None if marg is None else _ptr(marg), npix, _ptr(px), _ptr(py), _ptr(C), _ptr(T),
                      _ptr(nc), _ptr(last), _ptr(sig), _ptr(mono), _ptr(nflags), _ptr(leaves),
                      _ptr(nleaves), _ptr(bound), _ptr(overflow))
    return RenderResult(C, T, nc, last, sig, mono, nflags, leaves, nleaves, bound, overflow)


def composite_held(rg0: dict, rg: dict, order: np.ndarray, pix_x: np.ndarray, pix_y: np.ndarray,
                   period: float = 0.0) -> np.ndarray:
    """Composite with every decision taken on rg0 and every value on rg (see
    oracle_render_held in raster.c). Returns C per listed pixel."""
    lib = _raster()
    n = len(rg["mx"])
    order = np.ascontiguousarray(order, np.int64)
    px = np.ascontiguousarray(pix_x, np.int32)
    py = np.ascontiguousarray(pix_y, np.int32)
    consts = np.array([ALPHA_MAX, ALPHA_MIN, T_MIN, Q_MAX, float(period)], np.float64)
    C = np.zeros(len(px))
    a0 = [np.ascontiguousarray(rg0[k], np.float64) for k in ("mx", "my", "ixx", "ixy", "iyy", "op")]
    a1 = [np.ascontiguousarray(rg[k], np.float64) for k in ("mx", "my", "ixx", "ixy", "iyy", "op", "amp")]
    lib.oracle_render_held(n, *[_ptr(a) for a in a0], *[_ptr(a) for a in a1], _ptr(rg0["live"]), _ptr(order),
                           _ptr(consts), len(px), _ptr(px), _ptr(py), _ptr(C))
    return C


def at_grid(g: dict, rg: dict, sx: float, sy: float):
    """The deformed Gaussians seen on another resolution of the same field of view: pixel coordinates scale by
    (sx, sy), so the means do and Sigma' = S Sigma S (S = diag(sx, sy))."""
    g2 = dict(g)
    g2["mx"] = g["mx"] * sx
    g2["my"] = g["my"] * sy
    r2 = dict(rg)
    r2["mx"], r2["my"] = rg["mx"] * sx, rg["my"] * sy
    r2["ixx"], r2["ixy"], r2["iyy"] = rg["ixx"] / (sx * sx), rg["ixy"] / (sx * sy), rg["iyy"] / (sy * sy)
    r2["sxx"], r2["sxy"], r2["syy"] = rg["sxx"] * sx * sx, rg["sxy"] * sx * sy, rg["syy"] * sy * sy
    return g2, r2


def render_query(scene: Scene, mlp: MLP | None, tx, room=DEFAULT_ROOM, pix=None, margins=DEFAULT_MARGINS,
                 bf16=False, delta=None, wrap=False, grid=None):
    """Render one spectrum (the listed pixels, default the full H x W grid).
    wrap: azimuth is periodic with period W (each Gaussian acts through the
    image of its mean nearest to the pixel). grid: (H', W'), another
    resolution of the same field of view (the scene's own by default)."""
    if delta is None:
        delta = deltas(scene, mlp, tx, room, bf16=bf16) if mlp is not None else None
    g = deform(scene, delta)
    rg = gaussians_for_raster(g, scene.depth)
    H, W = scene.H, scene.W
    if grid is not None and tuple(grid) != (H, W):
        H, W = grid
        g, rg = at_grid(g, rg, W / scene.W, H / scene.H)
    order = depth_order(scene.depth)
    if pix is None:
        pix = full_grid(H, W)
    res = composite(rg, order, pix[0], pix[1], margins, period=W if wrap else 0.0)
    return res, g, rg, delta


# ---------------------------------------------------------------------------
# Tile binning and keys (gsplat-style tile lists; Sec. 4.1 tile partitioning)
# ---------------------------------------------------------------------------
def _rect_at(mx, my, hx, hy, H, W, tile, wrap=False):
    TW, TH = -(-W // tile), -(-H // tile)
    x0, x1, y0, y1 = mx - hx, mx + hx, my - hy, my + hy
    with np.errstate(invalid="ignore"):
        culled = (y1 < 0) | (y0 > H - 1)
        if not wrap:
            culled = culled | (x1 < 0) | (x0 > W - 1)
            tx0 = np.clip(np.floor(x0 / tile), 0, TW - 1)
            tx1 = np.clip(np.floor(x1 / tile), 0, TW - 1)
        else:
            # periodic azimuth: the box's columns taken modulo W. Folded so that
            # its left edge lies in [0, W); a box whose right edge then passes W
            # continues at column 0 (encoded as tx1 < tx0); a box at least W wide,
            # or whose two pieces meet, covers every column.
            k = np.floor(x0 / W)
            a, b = x0 - k * W, x1 - k * W
            tx0 = np.minimum(np.floor(a / tile), TW - 1)
            tx1 = np.where(b < W, np.minimum(np.floor(b / tile), TW - 1), np.floor((b - W) / tile))
            full = (x1 - x0 >= W) | ((b >= W) & (tx1 >= tx0 - 1))
            tx0 = np.where(full, 0, tx0)
            tx1 = np.where(full, TW - 1, tx1)
        ty0 = np.clip(np.floor(y0 / tile), 0, TH - 1)
        ty1 = np.clip(np.floor(y1 / tile), 0, TH - 1)
        bad = ~(np.isfinite(x0) & np.isfinite(x1) & np.isfinite(y0) & np.isfinite(y1))
        culled = culled | bad
        r = np.stack([np.where(culled, -1, v) for v in (tx0, ty0, tx1, ty1)], axis=-1).astype(np.int64)
    return r


def tile_rects(g: dict, rg: dict, H: int, W: int, tile: int = 16, rel_margin: float = 2.0 ** -19, wrap=False):
    """Tile rectangle [tx0, tx1] x [ty0, ty1] of every Gaussian (-1 if culled).

    The half extents are 3 sqrt(Sigma_xx) + eps and 3 sqrt(Sigma_yy) + eps (the
    bounding box of the q <= 9 ellipse plus a small binning margin). A Gaussian
    whose box misses [0, W-1] x [0, H-1] is culled. Returns (rect, flagged, alts)
    where a Gaussian is flagged if moving any of its four box edges by the FP32
    margin could change its rectangle; alts[i] lists every such rectangle.
    wrap: periodic azimuth (see _rect_at); a wrapped rectangle has tx1 < tx0 and
    covers columns tx0 .. TW-1 and 0 .. tx1."""
    live = rg["live"].astype(bool)
    with np.errstate(invalid="ignore"):
        hx = 3.0 * np.sqrt(np.where(live, rg["sxx"], 0.0)) + EXTENT_EPS
        hy = 3.0 * np.sqrt(np.where(live, rg["syy"], 0.0)) + EXTENT_EPS
    mx, my = g["mx"], g["my"]
    rect = _rect_at(mx, my, hx, hy, H, W, tile, wrap)
    rect[~live] = -1
    mxm = rel_margin * (np.abs(mx) + hx + tile)
    mym = rel_margin * (np.abs(my) + hy + tile)
    alts_all = []
    for sx0 in (-1, 1):
        for sx1 in (-1, 1):
            for sy0 in (-1, 1):
                for sy1 in (-1, 1):
                    # move each edge independently: x0 = mx - hx + sx0*m, etc.
                    x0 = mx - hx + sx0 * mxm
                    x1 = mx + hx + sx1 * mxm
                    y0 = my - hy + sy0 * mym
                    y1 = my + hy + sy1 * mym
                    cx, cy = 0.5 * (x0 + x1), 0.5 * (y0 + y1)
                    r = _rect_at(cx, cy, 0.5 * (x1 - x0), 0.5 * (y1 - y0), H, W, tile, wrap)
                    r[~live] = -1
                    alts_all.append(r)
    A = np.stack(alts_all, axis=1)  # (n, 16, 4)
    flagged = np.any(np.any(A != rect[:, None, :], axis=-1), axis=-1)
    alts = {}
    for i in np.nonzero(flagged)[0]:
        alts[int(i)] = sorted({tuple(int(v) for v in a) for a in A[i]})
    return rect, flagged, alts


def rect_count(rect: np.ndarray, TW: int | None = None) -> np.ndarray:
    """Tiles per rectangle (0 if culled); a wrapped one (tx1 < tx0, periodic
    azimuth) spans TW - tx0 + tx1 + 1 columns."""
    w = rect[:, 2] - rect[:, 0] + 1
    if TW is not None:
        w = np.where(rect[:, 2] < rect[:, 0], TW - rect[:, 0] + rect[:, 2] + 1, w)
    c = w * (rect[:, 3] - rect[:, 1] + 1)
    return np.where(rect[:, 0] < 0, 0, c).astype(np.int64)


def key_list(rect: np.ndarray, depth: np.ndarray, H: int, W: int, tile: int = 16, slot: int = 0,
             tile_base: int = 0):
    """Sorted (gtile, depth_bits, id) triples of one query, plus per-tile ranges.

    Every Gaussian emits one entry per tile of its rectangle (a wrapped one,
    tx1 < tx0, covers columns tx0 .. TW-1 and 0 .. tx1), with
    gtile = tile_base + ty * TW + tx. Sorting by (gtile, depth_bits, id) gives the
    per-tile front-to-back lists."""
    TW, TH = -(-W // tile), -(-H // tile)
    db = depth_bits(depth).astype(np.uint64)
    gt, dk, ids = [], [], []
    for i in range(len(rect)):
        tx0, ty0, tx1, ty1 = rect[i]
        if tx0 < 0:
            continue
        cols = range(tx0, tx1 + 1) if tx1 >= tx0 else list(range(tx0, TW)) + list(range(0, tx1 + 1))
        for ty in range(ty0, ty1 + 1):
            for tx in cols:
                gt.append(tile_base + ty * TW + tx)
                dk.append(db[i])
                ids.append(i)
    gt = np.array(gt, np.uint64); dk = np.array(dk, np.uint64); ids = np.array(ids, np.int64)
    o = np.lexsort((ids, dk, gt))
    gt, dk, ids = gt[o], dk[o], ids[o]
    ranges = np.zeros((TW * TH, 2), np.int64)
    for t in range(TW * TH):
        g = tile_base + t
        ranges[t, 0] = np.searchsorted(gt, g, side="left")
        ranges[t, 1] = np.searchsorted(gt, g, side="right")
    return gt, dk, ids, ranges


def exclusive_scan(counts: np.ndarray) -> tuple:
    """Exclusive prefix sum with a 64-bit running total: (offsets, total)."""
    out = np.zeros(len(counts), np.uint64)
    run = 0
    for i, c in enumerate(np.asarray(counts, np.uint64)):
        out[i] = run
        run += int(c)
    return out, run
