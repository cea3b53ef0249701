"""Python binding of libswiftwrf.so (ctypes): argument marshalling only.

Every step of the render path runs in the HIP library; PyTorch provides device
memory and the current stream. Loading fails loudly when the library has not
been built (there is no CPU fallback).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libswiftwrf.so")

# render flags (include/swiftwrf.h)
MLP_FP32 = 0
MLP_BF16 = 1 << 0
NO_DEFORM = 1 << 1
KEEP_AUX = 1 << 2
FULL_SORT = 1 << 3
TILE8 = 1 << 4
PAPER_DEFORM = 1 << 5
WRAP_AZIMUTH = 1 << 6
DETERMINISTIC = 1 << 7

STAGES = ("tx_features", "mlp_preprocess", "scan", "emit_keys", "radix_sort", "tile_ranges", "blend",
          "blend_backward", "preprocess_backward", "mlp_backward")
MAX_LAYERS = 8
PARAMS = ("mean_x", "mean_y", "log_scale_x", "log_scale_y", "rotation", "opacity_logit", "amplitude", "depth")

_fp = ctypes.POINTER(ctypes.c_float)


class _Config(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("mlp_pairs_per_wave", ctypes.c_int32),
                ("max_list_entries", ctypes.c_uint32), ("reserved", ctypes.c_int32 * 5)]


class _Gaussians(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32)] + [(k, ctypes.c_void_p) for k in PARAMS]


class _Mlp(ctypes.Structure):
    _fields_ = [("mean_bands", ctypes.c_int32), ("tx_bands", ctypes.c_int32), ("hidden", ctypes.c_int32),
                ("n_hidden", ctypes.c_int32), ("weight", ctypes.c_void_p * MAX_LAYERS),
                ("bias", ctypes.c_void_p * MAX_LAYERS), ("room_lo", ctypes.c_float * 3),
                ("room_hi", ctypes.c_float * 3)]


PAPER_KEYS = ("center_x", "center_y", "chol_l1", "chol_l2", "chol_l3", "atten_logit", "psi_re", "psi_im")


class _PaperGaussians(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32)] + [(k, ctypes.c_void_p) for k in PAPER_KEYS]


class _PaperMlp(ctypes.Structure):
    _fields_ = [("weight", ctypes.c_void_p * 9), ("bias", ctypes.c_void_p * 9), ("room_lo", ctypes.c_float * 3),
                ("room_hi", ctypes.c_float * 3)]


class _Grads(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in PARAMS[:7]] + [("weight", ctypes.c_void_p * MAX_LAYERS),
                                                             ("bias", ctypes.c_void_p * MAX_LAYERS)]


class _ServeCfg(ctypes.Structure):
    _fields_ = [("max_batch", ctypes.c_int32), ("n_slots", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("key_factor", ctypes.c_float), ("hbm_budget", ctypes.c_uint64), ("use_graphs", ctypes.c_int32),
                ("mixed", ctypes.c_int32), ("reserved", ctypes.c_int32 * 4)]


class _ReqStats(ctypes.Structure):
    _fields_ = [("queue_us", ctypes.c_double), ("service_us", ctypes.c_double), ("total_us", ctypes.c_double),
                ("batch", ctypes.c_int32), ("bucket", ctypes.c_int32), ("fallback", ctypes.c_int32),
                ("slot", ctypes.c_int32)]


class _DevStatus(ctypes.Structure):
    _fields_ = [("flags", ctypes.c_uint32), ("rerenders", ctypes.c_uint32), ("pairs", ctypes.c_uint64),
                ("culled_nonfinite", ctypes.c_uint64), ("culled_offgrid", ctypes.c_uint64),
                ("list_entries", ctypes.c_uint64), ("reserved", ctypes.c_uint64 * 3)]


DEV_KEY_OVERFLOW, DEV_RERENDERED, DEV_CULLED_NONFINITE, DEV_CULLED_OFFGRID, DEV_BWD_REUSED, DEV_CHUNKED = (
    1, 2, 4, 8, 16, 32)

SERVE_COUNTERS = ("launches", "completed", "fallbacks", "graph_builds", "budget_shrinks", "workspace_bytes",
                  "mixed_launches", "mixed_scenes")
PENDING = -7

_lib = None


def lib():
    """The loaded native library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(the render path has no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        P, I32, I64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        sig = {
            "swf_create": [P, P],
            "swf_destroy": [P],
            "swf_last_error": [P],
            "swf_status_string": [I32],
            "swf_scene_upload": [P, P, P, I32, I32, I32, P],
            "swf_scene_release": [P, I32],
            "swf_scene_update": [P, I32, P, P, I32, P],
            "swf_scene_bytes": [P, I32, P],
            "swf_render": [P, I32, P, I32, I32, P, P, P],
            "swf_render_backward": [P, I32, P, I32, I32, P, P, P, P],
            "swf_l1_loss": [P, P, P, I64, P, P, P],
            "swf_adam_step": [P, P, P, P, P, P, P, I32, ctypes.c_float, ctypes.c_float, ctypes.c_float, I32, P],
            "swf_anneal_tx": [P, P, P, I32, I32, ctypes.c_float, I32, I32, P, P, P, P],
            "swf_hybrid_loss": [P, P, P, I32, I32, I32, ctypes.c_float, P, P, P],
            "swf_scene_upload_paper": [P, P, P, I32, I32, I32, P],
            "swf_render_paper": [P, I32, P, I32, I32, P, P, P],
            "swf_render_mixed": [P, P, P, I32, I32, P, P, P],
            "swf_render_at": [P, I32, P, I32, I32, I32, I32, P, P, P],
            "swf_render_rssi": [P, I32, P, I32, I32, P, P, P, P],
            "swf_render_rssi_backward": [P, I32, P, I32, I32, P, P, P, P],
            "swf_beamscan": [P, P, P, I32, I32, I32, ctypes.c_float, I32, I32, P, P],
            "swf_stage_timing": [P, I32],
            "swf_stage_times": [P, P, P, P],
            "swf_debug_deform": [P, I32, P, I32, I32, P, P],
            "swf_debug_keys": [P, P, P, P, P, P, P, ctypes.c_uint64],
            "swf_debug_blend_work": [P, P, P, P],
            "swf_debug_blend_executed": [P, P],
            "swf_debug_rects": [P, P, ctypes.c_uint64],
            "swf_debug_relu_pattern": [P, P, ctypes.c_uint64],
            "swf_last_device_status": [P, P],
            "swf_measure_peaks": [P, P, P, P],
            "swf_radix_sort": [P, P, P, I64, I32, I32, I32, P],
            "swf_exclusive_scan": [P, P, P, P, I64, P],
            "swf_exclusive_scan_noalloc": [P, P, P, P, I64, P],
            "swf_serve_start": [P, P],
            "swf_serve_submit": [P, I32, P, P, ctypes.c_double, P],
            "swf_serve_poll": [P, ctypes.c_uint64, P],
            "swf_serve_wait": [P, ctypes.c_uint64, P],
            "swf_serve_stop": [P],
            "swf_serve_counters": [P, P, I32],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int32
        L.swf_last_error.restype = ctypes.c_char_p
        L.swf_serve_clock.argtypes = []
        L.swf_serve_clock.restype = ctypes.c_double
        L.swf_status_string.restype = ctypes.c_char_p
        _lib = L
    return _lib


class SwfError(RuntimeError):
    pass


def _ptr(t):
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Context:
    """One libswiftwrf context on one GPU."""

    def __init__(self, device: int = 0, mlp_pairs_per_wave: int = 0, max_list_entries: int = 0):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)
        self._L = lib()
        h = ctypes.c_void_p()
        cfg = _Config(device=device, mlp_pairs_per_wave=mlp_pairs_per_wave, max_list_entries=max_list_entries)
        self._check(self._L.swf_create(ctypes.byref(h), ctypes.byref(cfg)), ctx=False)
        self._h = h
        self._keep = {}
        self._rooms = {}
        self._serve_out = {}

    def _check(self, st, ctx=True):
        if st != 0:
            msg = self._L.swf_status_string(st).decode()
            if ctx and getattr(self, "_h", None):
                msg += ": " + self._L.swf_last_error(self._h).decode()
            raise SwfError(f"libswiftwrf status {st} ({msg})")

    def close(self):
        if getattr(self, "_h", None):
            self._L.swf_destroy(self._h)
            self._h = None
            self._serve_out = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- scenes -------------------------------------------------------------
    def upload_scene(self, gaussians: dict, H: int, W: int, mlp=None, room=((0, 0, 0), (6, 6, 3))) -> int:
        """Upload FP32 Gaussians (numpy arrays, host) and optional MLP weights
        (Ws, bs) lists of FP32 arrays with W_l of shape (out, in)."""
        cols = {k: np.ascontiguousarray(gaussians[k], dtype=np.float32) for k in PARAMS}
        n = len(cols["mean_x"])
        g = _Gaussians(n=n, **{k: cols[k].ctypes.data for k in PARAMS})
        m = None
        keep = [cols]
        if mlp is not None:
            Ws, bs = mlp
            Ws = [np.ascontiguousarray(w, dtype=np.float32) for w in Ws]
            bs = [np.ascontiguousarray(b, dtype=np.float32) for b in bs]
            keep += [Ws, bs]
            m = _Mlp(mean_bands=6, tx_bands=10, hidden=Ws[0].shape[0], n_hidden=len(Ws) - 1)
            for l in range(len(Ws)):
                m.weight[l] = Ws[l].ctypes.data
                m.bias[l] = bs[l].ctypes.data
            for k in range(3):
                m.room_lo[k] = room[0][k]
                m.room_hi[k] = room[1][k]
        sid = ctypes.c_int32()
        self._check(self._L.swf_scene_upload(self._h, ctypes.byref(g), ctypes.byref(m) if m is not None else None,
                                             H, W, 0, ctypes.byref(sid)))
        self._keep[sid.value] = (H, W, n, mlp is not None)
        self._rooms[sid.value] = room
        return sid.value

    def update_scene(self, sid: int, gaussians: dict | None = None, mlp=None):
        """Replace parameters of a resident scene from CUDA tensors (float32,
        contiguous): gaussians keyed like PARAMS[:7] (depth is kept), mlp as
        (Ws, bs) lists. The scene keeps its (depth, id) order."""
        g = m = None
        keep = []
        if gaussians is not None:
            cols = {k: gaussians[k].contiguous() for k in PARAMS[:7]}
            keep.append(cols)
            n = self._keep[sid][2]
            g = _Gaussians(n=n, **{k: cols[k].data_ptr() for k in PARAMS[:7]}, depth=None)
        if mlp is not None:
            Ws, bs = [w.contiguous() for w in mlp[0]], [b.contiguous() for b in mlp[1]]
            keep += [Ws, bs]
            m = _Mlp(mean_bands=6, tx_bands=10, hidden=Ws[0].shape[0], n_hidden=len(Ws) - 1)
            for l in range(len(Ws)):
                m.weight[l] = Ws[l].data_ptr()
                m.bias[l] = bs[l].data_ptr()
            room = self._rooms[sid]
            for k in range(3):
                m.room_lo[k] = room[0][k]
                m.room_hi[k] = room[1][k]
        self._check(self._L.swf_scene_update(self._h, sid, ctypes.byref(g) if g is not None else None,
                                             ctypes.byref(m) if m is not None else None, 1, _stream()))

    def upload_paper_scene(self, gaussians: dict, H: int, W: int, mlp=None, room=((0, 0, 0), (6, 6, 3))) -> int:
        """Upload a paper-model scene: FP32 host arrays keyed by PAPER_KEYS, optional paper MLP (Ws, bs) of nine
        layers (W_l of shape (out, in))."""
        cols = {k: np.ascontiguousarray(gaussians[k], dtype=np.float32) for k in PAPER_KEYS}
        n = len(cols["center_x"])
        g = _PaperGaussians(n=n, **{k: cols[k].ctypes.data for k in PAPER_KEYS})
        m = None
        if mlp is not None:
            Ws = [np.ascontiguousarray(w, dtype=np.float32) for w in mlp[0]]
            bs = [np.ascontiguousarray(b, dtype=np.float32) for b in mlp[1]]
            assert len(Ws) == 9 and len(bs) == 9
            m = _PaperMlp()
            for l in range(9):
                m.weight[l] = Ws[l].ctypes.data
                m.bias[l] = bs[l].ctypes.data
            for k in range(3):
                m.room_lo[k] = room[0][k]
                m.room_hi[k] = room[1][k]
        sid = ctypes.c_int32()
        self._check(self._L.swf_scene_upload_paper(self._h, ctypes.byref(g), ctypes.byref(m) if m is not None else None,
                                                   H, W, 0, ctypes.byref(sid)))
        self._keep[sid.value] = (H, W, n, mlp is not None)
        self._rooms[sid.value] = room
        return sid.value

    def render_paper(self, sid: int, tx=None, flags: int = 0, batch: int | None = None, out=None, channels=True):
        """Paper-model spectra (batch, H, W) = |GMM sum| and, with channels, the (batch, 2, H, W) real and imaginary
        sums."""
        torch = self.torch
        H, W, n, _ = self._keep[sid]
        if tx is not None:
            assert tx.is_cuda and tx.dtype == torch.float32 and tx.is_contiguous() and tx.shape[-1] == 3
            batch = tx.shape[0]
        batch = batch or 1
        if out is None:
            out = torch.empty((batch, H, W), device=self.device, dtype=torch.float32)
        ch = torch.empty((batch, 2, H, W), device=self.device, dtype=torch.float32) if channels else None
        self._check(self._L.swf_render_paper(self._h, sid, _ptr(tx), batch, flags, _ptr(out), _ptr(ch), _stream()))
        return out, ch

    def debug_deform_paper(self, sid: int, tx):
        """The paper MLP's residuals (batch, n, 5) for a paper-model scene."""
        torch = self.torch
        H, W, n, _ = self._keep[sid]
        d = torch.empty((tx.shape[0], n, 5), device=self.device, dtype=torch.float32)
        self._check(self._L.swf_debug_deform(self._h, sid, _ptr(tx), tx.shape[0], MLP_FP32, _ptr(d), _stream()))
        return d

    def release_scene(self, sid: int):
        self._check(self._L.swf_scene_release(self._h, sid))
        self._keep.pop(sid, None)

    def scene_bytes(self, sid: int) -> int:
        v = ctypes.c_uint64()
        self._check(self._L.swf_scene_bytes(self._h, sid, ctypes.byref(v)))
        return v.value

    def scene_shape(self, sid: int):
        return self._keep[sid]

    # ---- render ---------------------------------------------------------------
    def render(self, sid: int, tx=None, flags: int = 0, batch: int | None = None, out=None, aux=None):
        torch = self.torch
        H, W, n, _ = self._keep[sid]
        if tx is not None:
            assert tx.is_cuda and tx.dtype == torch.float32 and tx.is_contiguous() and tx.shape[-1] == 3
            batch = tx.shape[0]
        batch = batch or 1
        if out is None:
            out = torch.empty((batch, H, W), device=self.device, dtype=torch.float32)
        if (flags & KEEP_AUX) and aux is None:
            aux = torch.empty((2, batch, H, W), device=self.device, dtype=torch.float32)
        self._check(self._L.swf_render(self._h, sid, _ptr(tx), batch, flags, _ptr(out), _ptr(aux), _stream()))
        return (out, aux) if (flags & KEEP_AUX) else out

    def render_at(self, sid: int, height: int, width: int, tx=None, flags: int = 0, batch: int | None = None,
                  out=None):
        """Render on another resolution (height x width) of the scene's field of view."""
        torch = self.torch
        if tx is not None:
            assert tx.is_cuda and tx.dtype == torch.float32 and tx.is_contiguous() and tx.shape[-1] == 3
            batch = tx.shape[0]
        batch = batch or 1
        if out is None:
            out = torch.empty((batch, height, width), device=self.device, dtype=torch.float32)
        self._check(self._L.swf_render_at(self._h, sid, _ptr(tx), batch, height, width, flags, _ptr(out), None,
                                          _stream()))
        return out

    def render_mixed(self, scene_ids, tx=None, flags: int = MLP_BF16):
        """Queries over several scenes in one launch sequence: returns the list of per-query spectra (H_b, W_b),
        views into one flat device buffer."""
        torch = self.torch
        ids = np.ascontiguousarray(scene_ids, dtype=np.int32)
        B_ = len(ids)
        # an unknown scene id gets no room here: the library rejects the batch (SWF_E_NOT_FOUND)
        sizes = [self._keep[int(s)][0] * self._keep[int(s)][1] if int(s) in self._keep else 0 for s in ids]
        out = torch.empty(max(int(sum(sizes)), 1), device=self.device, dtype=torch.float32)
        offs = np.zeros(B_ + 1, np.uint64)
        if tx is not None:
            assert tx.is_cuda and tx.dtype == torch.float32 and tx.is_contiguous() and tx.shape == (B_, 3)
        self._check(self._L.swf_render_mixed(self._h, ids.ctypes.data_as(ctypes.c_void_p), _ptr(tx), B_, flags,
                                             _ptr(out), offs.ctypes.data_as(ctypes.c_void_p), _stream()))
        res = []
        for b, s in enumerate(ids):
            H, W = self._keep[int(s)][:2]
            res.append(out[int(offs[b]):int(offs[b + 1])].view(H, W))
        return res

    def render_backward(self, sid: int, tx, flags: int, grad_out, aux, grads: dict):
        """Gradients of sum(grad_out * out) into the caller's device tensors in
        `grads` (keys of PARAMS[:7], and optionally 'weight' / 'bias' lists)."""
        gr = _Grads()
        for k in PARAMS[:7]:
            setattr(gr, k, grads[k].data_ptr() if grads.get(k) is not None else None)
        for l, w in enumerate(grads.get("weight", []) or []):
            gr.weight[l] = w.data_ptr() if w is not None else None
        for l, b in enumerate(grads.get("bias", []) or []):
            gr.bias[l] = b.data_ptr() if b is not None else None
        torch = self.torch
        H, W, n, _ = self._keep[sid]
        batch = tx.shape[0] if tx is not None else grad_out.shape[0]
        if grad_out.dtype != torch.float32 or not grad_out.is_contiguous() or grad_out.numel() != batch * H * W:
            raise SwfError(f"grad_out must be contiguous float32 with {batch}*{H}*{W} values")
        if aux is None or not aux.is_contiguous() or aux.numel() * aux.element_size() != 8 * batch * H * W:
            raise SwfError(f"aux must be the contiguous {8 * batch * H * W}-byte buffer of the forward render")
        for k in PARAMS[:7]:
            t = grads.get(k)
            if t is not None and (t.dtype != torch.float32 or not t.is_contiguous() or t.numel() != n):
                raise SwfError(f"grads[{k!r}] must be contiguous float32 with {n} values")
        self._check(self._L.swf_render_backward(self._h, sid, _ptr(tx), batch, flags, _ptr(grad_out), _ptr(aux),
                                                ctypes.byref(gr), _stream()))

    def render_rssi(self, sid: int, tx, flags: int = 0, out=None, aux=None, keep_spectrum: bool = False):
        """RSSI per query (global average of the rendered spectrum). Returns rssi (batch,), plus the spectrum if
        keep_spectrum (or out) is given, plus aux with KEEP_AUX."""
        torch = self.torch
        H, W, n, _ = self._keep[sid]
        assert tx.is_cuda and tx.dtype == torch.float32 and tx.is_contiguous() and tx.shape[-1] == 3
        batch = tx.shape[0]
        rssi = torch.empty((batch,), device=self.device, dtype=torch.float32)
        if out is None and keep_spectrum:
            out = torch.empty((batch, H, W), device=self.device, dtype=torch.float32)
        if out is not None:
            assert out.dtype == torch.float32 and out.is_contiguous() and out.numel() == batch * H * W
        if (flags & KEEP_AUX) and aux is None:
            aux = torch.empty((2, batch, H, W), device=self.device, dtype=torch.float32)
        self._check(self._L.swf_render_rssi(self._h, sid, _ptr(tx), batch, flags, _ptr(rssi), _ptr(out), _ptr(aux),
                                            _stream()))
        res = (rssi,)
        if out is not None:
            res += (out,)
        if flags & KEEP_AUX:
            res += (aux,)
        return res[0] if len(res) == 1 else res

    def render_rssi_backward(self, sid: int, tx, flags: int, grad_rssi, aux, grads: dict):
        """Gradients of sum(grad_rssi * rssi) into the device tensors of `grads` (as render_backward)."""
        torch = self.torch
        H, W, n, _ = self._keep[sid]
        batch = tx.shape[0]
        if grad_rssi.dtype != torch.float32 or not grad_rssi.is_contiguous() or grad_rssi.numel() != batch:
            raise SwfError(f"grad_rssi must be contiguous float32 with {batch} values")
        if aux is None or not aux.is_contiguous() or aux.numel() * aux.element_size() != 8 * batch * H * W:
            raise SwfError(f"aux must be the contiguous {8 * batch * H * W}-byte buffer of the forward render")
        gr = self._grads_struct(grads, n)
        self._check(self._L.swf_render_rssi_backward(self._h, sid, _ptr(tx), batch, flags, _ptr(grad_rssi),
                                                     _ptr(aux), ctypes.byref(gr), _stream()))

    def _grads_struct(self, grads: dict, n: int):
        torch = self.torch
        gr = _Grads()
        for k in PARAMS[:7]:
            t = grads.get(k)
            if t is not None and (t.dtype != torch.float32 or not t.is_contiguous() or t.numel() != n):
                raise SwfError(f"grads[{k!r}] must be contiguous float32 with {n} values")
            setattr(gr, k, t.data_ptr() if t is not None else None)
        for l, w in enumerate(grads.get("weight", []) or []):
            gr.weight[l] = w.data_ptr() if w is not None else None
        for l, b in enumerate(grads.get("bias", []) or []):
            gr.bias[l] = b.data_ptr() if b is not None else None
        return gr

    def hybrid_loss(self, pred, target, lambda1: float = 0.7, want_grad=True):
        """(loss (3,) = total, l1, ssim; grad or None) of lambda1 * l1 + (1 - lambda1) * (1 - SSIM) over a batch of
        spectra (B, H, W)."""
        torch = self.torch
        assert pred.dtype == torch.float32 and pred.is_contiguous() and pred.dim() == 3 and pred.is_cuda
        assert target.shape == pred.shape and target.dtype == torch.float32 and target.is_contiguous()
        loss = torch.empty(3, device=self.device, dtype=torch.float32)
        grad = torch.empty_like(pred) if want_grad else None
        B_, H, W = pred.shape
        self._check(self._L.swf_hybrid_loss(self._h, _ptr(pred), _ptr(target), B_, H, W, float(lambda1), _ptr(loss),
                                            _ptr(grad), _stream()))
        return loss, grad

    def adam_step(self, params, grads, m, v, lrs, step: int, beta1=0.9, beta2=0.999, eps=1e-8):
        """In-place Adam update of lists of contiguous float32 device tensors (one learning rate each)."""
        n = len(params)
        for ts in (params, grads, m, v):
            assert len(ts) == n and all(t.is_contiguous() and t.dtype == self.torch.float32 for t in ts)
        P = ctypes.c_void_p * max(n, 1)
        arr = [P(*[t.data_ptr() for t in ts]) for ts in (params, grads, m, v)]
        sizes = (ctypes.c_int64 * max(n, 1))(*[t.numel() for t in params])
        lr = (ctypes.c_float * max(n, 1))(*[float(x) for x in lrs])
        self._check(self._L.swf_adam_step(self._h, *arr, sizes, lr, n, float(beta1), float(beta2), float(eps),
                                          int(step), _stream()))

    def anneal_tx(self, tx, noise, it: int, n_positions: int, gamma=1.0, tau=10_000,
                  room=((0.0, 0.0, 0.0), (6.0, 6.0, 3.0)), out=None):
        """Anneal-smoothed positions (batch, 3) from standard normal noise (batch, 3), both device float32."""
        torch = self.torch
        assert tx.is_contiguous() and noise.is_contiguous() and tx.shape == noise.shape and tx.shape[-1] == 3
        out = torch.empty_like(tx) if out is None else out
        lo = (ctypes.c_float * 3)(*room[0])
        hi = (ctypes.c_float * 3)(*room[1])
        self._check(self._L.swf_anneal_tx(self._h, _ptr(tx), _ptr(noise), tx.shape[0], int(it), float(gamma),
                                          int(tau), int(n_positions), lo, hi, _ptr(out), _stream()))
        return out

    def l1_loss(self, pred, target, want_grad=True):
        torch = self.torch
        loss = torch.empty((), device=self.device, dtype=torch.float32)
        grad = torch.empty_like(pred) if want_grad else None
        self._check(self._L.swf_l1_loss(self._h, _ptr(pred), _ptr(target), pred.numel(), _ptr(loss), _ptr(grad),
                                        _stream()))
        return loss, grad

    def beamscan(self, paths, counts, H: int, W: int, side: int = 4, spacing_over_lambda: float = 0.5, out=None):
        """Beam-scan spectra (batch, H, W) from device multipath lists: paths float32 (batch, max_paths, 3) of
        (rho, azimuth, elevation), counts int32 (batch,)."""
        torch = self.torch
        assert paths.is_cuda and paths.dtype == torch.float32 and paths.is_contiguous() and paths.dim() == 3
        assert paths.shape[2] == 3
        assert counts.is_cuda and counts.dtype == torch.int32 and counts.is_contiguous()
        batch, max_paths = paths.shape[0], paths.shape[1]
        assert counts.numel() == batch
        if out is None:
            out = torch.empty((batch, H, W), device=self.device, dtype=torch.float32)
        assert out.dtype == torch.float32 and out.is_contiguous() and out.numel() == batch * H * W
        self._check(self._L.swf_beamscan(self._h, _ptr(paths), _ptr(counts), batch, max_paths, side,
                                         float(spacing_over_lambda), H, W, _ptr(out), _stream()))
        return out

    # ---- timing ---------------------------------------------------------------
    def stage_timing(self, enable: bool):
        self._check(self._L.swf_stage_timing(self._h, 1 if enable else 0))

    def stage_times(self):
        ms = (ctypes.c_double * len(STAGES))()
        cnt = (ctypes.c_int64 * len(STAGES))()
        n = ctypes.c_int32(len(STAGES))
        self._check(self._L.swf_stage_times(self._h, ms, cnt, ctypes.byref(n)))
        return {STAGES[i]: (ms[i], cnt[i]) for i in range(n.value)}

    # ---- debug / step-level ------------------------------------------------------
    def debug_deform(self, sid: int, tx, flags: int = 0):
        torch = self.torch
        H, W, n, _ = self._keep[sid]
        d = torch.empty((tx.shape[0], n, 7), device=self.device, dtype=torch.float32)
        self._check(self._L.swf_debug_deform(self._h, sid, _ptr(tx), tx.shape[0], flags, _ptr(d), _stream()))
        return d

    def debug_relu_pattern(self, batch: int, n: int, layers: int):
        """ReLU decisions of the hidden units the last backward used, (batch, n, layers, 256) bool, original ids."""
        r = np.zeros((batch, n, layers, 256), np.uint8)
        self._check(self._L.swf_debug_relu_pattern(self._h, r.ctypes.data_as(ctypes.c_void_p), r.size))
        return r.astype(bool)

    def debug_rects(self, batch: int, n: int):
        """Tile rectangles of the last render's pairs, (batch, n, 4) int32 (tx0, ty0, tx1, ty1; -1 if culled)."""
        r = np.zeros((batch, n, 4), np.int32)
        self._check(self._L.swf_debug_rects(self._h, r.ctypes.data_as(ctypes.c_void_p), batch * n))
        return r

    def debug_keys(self, batch: int, n: int, tiles: int, capacity: int | None = None):
        self.torch.cuda.synchronize()
        nk = ctypes.c_uint64()
        self._check(self._L.swf_debug_keys(self._h, None, None, None, None, None, ctypes.byref(nk), 0))
        nkeys = nk.value
        counts = np.zeros(batch * n, np.uint32)
        offsets = np.zeros(batch * n, np.uint32)
        keys = np.zeros(max(nkeys, 1), np.uint64)
        vals = np.zeros(max(nkeys, 1), np.uint64)
        ranges = np.zeros((batch * tiles, 2), np.uint32)
        P = lambda a: a.ctypes.data_as(ctypes.c_void_p)
        self._check(self._L.swf_debug_keys(self._h, P(counts), P(offsets), P(keys), P(vals), P(ranges),
                                           ctypes.byref(nk), nkeys))
        return dict(counts=counts, offsets=offsets, keys=keys[:nkeys], values=vals[:nkeys], ranges=ranges)

    def blend_work(self):
        """Work of the last render's blend: (pixel, entry) evaluations inside the 3-sigma cutoff before the pixel
        ends, staged records, list entries."""
        ev, st, ne, ex = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
        self._check(self._L.swf_debug_blend_work(self._h, ctypes.byref(ev), ctypes.byref(st), ctypes.byref(ne)))
        self._check(self._L.swf_debug_blend_executed(self._h, ctypes.byref(ex)))
        return dict(evaluations=ev.value, staged=st.value, entries=ne.value, executed=ex.value)

    def device_status(self):
        """What the device saw during the last render: flags (DEV_* bits), exact-size re-renders, pairs, culled
        pairs (non-finite, off the grid) and list entries. Waits for that render."""
        st = _DevStatus()
        self._check(self._L.swf_last_device_status(self._h, ctypes.byref(st)))
        return dict(flags=st.flags, rerenders=st.rerenders, pairs=st.pairs, culled_nonfinite=st.culled_nonfinite,
                    culled_offgrid=st.culled_offgrid, list_entries=st.list_entries)

    def measure_peaks(self):
        """On-device peaks: BF16 MFMA TFLOP/s, FP32 FMA T lane-ops/s, LDS read TB/s (plain loops)."""
        m, f, l = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        self._check(self._L.swf_measure_peaks(self._h, ctypes.byref(m), ctypes.byref(f), ctypes.byref(l)))
        return dict(mfma_bf16_tflops=m.value, fma_tops=f.value, lds_tbps=l.value)

    def radix_sort(self, keys, values, begin_bit=0, end_bit=None):
        kb = keys.element_size()
        end_bit = 8 * kb if end_bit is None else end_bit
        self._check(self._L.swf_radix_sort(self._h, _ptr(keys), _ptr(values), keys.numel(), kb, begin_bit, end_bit,
                                           _stream()))

    def exclusive_scan(self, counts):
        torch = self.torch
        off = torch.empty_like(counts)
        tot = torch.zeros(1, device=self.device, dtype=torch.int64)
        self._check(self._L.swf_exclusive_scan(self._h, _ptr(counts), _ptr(off), _ptr(tot), counts.numel(), _stream()))
        return off, tot

    def exclusive_scan_noalloc(self, counts, off, tot):
        """The allocation-free scan into caller-owned off (uint32 like counts) and tot (one int64)."""
        torch = self.torch
        assert counts.dtype == torch.int32 and off.dtype == torch.int32 and off.numel() >= counts.numel()
        assert tot.dtype == torch.int64 and tot.numel() >= 1 and counts.is_contiguous() and off.is_contiguous()
        self._check(self._L.swf_exclusive_scan_noalloc(self._h, _ptr(counts), _ptr(off), _ptr(tot), counts.numel(),
                                                       _stream()))

    # ---- serving ------------------------------------------------------------------
    def serve_start(self, max_batch=64, n_slots=3, flags=MLP_BF16, key_factor=1.5, hbm_budget=0, use_graphs=True,
                    mixed=True):
        cfg = _ServeCfg(max_batch=max_batch, n_slots=n_slots, flags=flags, key_factor=key_factor,
                        hbm_budget=hbm_budget, use_graphs=1 if use_graphs else 0, mixed=1 if mixed else 0)
        self._check(self._L.swf_serve_start(self._h, ctypes.byref(cfg)))

    def serve_submit(self, sid: int, tx, out: np.ndarray, arrival: float = 0.0) -> int:
        """Queue one query; `out` (H x W float32, C-contiguous) receives the result."""
        assert out.dtype == np.float32 and out.flags["C_CONTIGUOUS"]
        t = (ctypes.c_float * 3)(*[float(v) for v in tx])
        tk = ctypes.c_uint64()
        st = self._L.swf_serve_submit(self._h, sid, t, out.ctypes.data_as(ctypes.c_void_p), float(arrival),
                                      ctypes.byref(tk))
        if st != 0:
            raise SwfError(f"serve_submit status {st} ({self._L.swf_status_string(st).decode()})")
        self._serve_out[tk.value] = out
        return tk.value

    def _stats(self, tk, st, rs):
        self._serve_out.pop(tk, None)
        if st != 0:
            raise SwfError(f"request {tk} failed with status {st} ({self._L.swf_status_string(st).decode()})")
        return {"queue_us": rs.queue_us, "service_us": rs.service_us, "total_us": rs.total_us, "batch": rs.batch,
                "bucket": rs.bucket, "fallback": rs.fallback, "slot": rs.slot}

    def serve_poll(self, ticket: int):
        rs = _ReqStats()
        st = self._L.swf_serve_poll(self._h, ticket, ctypes.byref(rs))
        if st == PENDING:
            return None
        return self._stats(ticket, st, rs)

    def serve_wait(self, ticket: int):
        rs = _ReqStats()
        st = self._L.swf_serve_wait(self._h, ticket, ctypes.byref(rs))
        return self._stats(ticket, st, rs)

    def serve_stop(self):
        self._check(self._L.swf_serve_stop(self._h))

    def serve_counters(self):
        v = (ctypes.c_uint64 * len(SERVE_COUNTERS))()
        self._check(self._L.swf_serve_counters(self._h, v, len(SERVE_COUNTERS)))
        return dict(zip(SERVE_COUNTERS, list(v)))

    def clock(self) -> float:
        return self._L.swf_serve_clock()
