"""ctypes binding of libesom (include/esom.h): argument marshalling only.

The functions named ``esom_*`` mirror the C entry points one to one and take
raw device pointers (ints) and sizes.  ``Context`` adds torch conveniences:
it takes device tensors, passes their ``data_ptr()`` and the current HIP
stream, and raises ``EsomError`` on any non-zero status.  Every computation
runs in the library's kernels; if the library is missing, loading fails
loudly instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libesom.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "esom.h")

ESOM_OK = 0
ESOM_EINVAL = -1
ESOM_ENOMEM = -2
ESOM_EDEVICE = -3
ESOM_EBUSY = -4
ESOM_ETIMEOUT = -5
ESOM_ENOTFOUND = -6
ESOM_MODE_FP32 = 0
ESOM_MODE_BF16_RESCORE = 1
MODES = {"fp32": ESOM_MODE_FP32, "bf16": ESOM_MODE_BF16_RESCORE}


class esom_params(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("boost", ctypes.c_float), ("adjust", ctypes.c_float),
                ("cutoff", ctypes.c_float), ("gravity", ctypes.c_float), ("mode", ctypes.c_int32),
                ("candidates", ctypes.c_int32)]


class esom_stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in (
        "n_points", "n_fallback", "n_uncertified", "n_near_tie", "n_illcond", "n_degenerate",
        "n_candidates", "n_slowpath", "n_timed")] + [
        (n, ctypes.c_double) for n in ("ms_prep", "ms_main", "ms_exact")]

    def as_dict(self):
        return {n: (float if t is ctypes.c_double else int)(getattr(self, n))
                for n, t in self._fields_}


class esom_request_info(ctypes.Structure):
    _fields_ = [("submit_ms", ctypes.c_double), ("start_ms", ctypes.c_double),
                ("done_ms", ctypes.c_double), ("n", ctypes.c_int64), ("cache_hit", ctypes.c_int32),
                ("graph_replay", ctypes.c_int32), ("status", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_ if n != "reserved"}


class esom_serve_stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in (
        "completed", "failed", "rejected", "points", "cache_hits", "graph_replays", "queued",
        "in_flight", "slots", "budget_bytes", "resident_bytes", "held_bytes", "peak_bytes",
        "admission_waits", "max_queued")] + [
        ("now_ms", ctypes.c_double)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class esom_layout_params(ctypes.Structure):
    _fields_ = [("scale", ctypes.c_float), ("repulsion", ctypes.c_float),
                ("softening", ctypes.c_float), ("step", ctypes.c_float),
                ("max_move", ctypes.c_float)]


class EsomError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("esom error %d: %s" % (code, msg))
        self.code = code


_lib = None
_vp, _i32, _i64, _f32, _sz = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float,
                              ctypes.c_size_t)


def load(path: str = LIB_PATH):
    """Loads libesom.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libesom.so not found at %s: build it with "
                           "`python -m paper_2201_00701_amd.build`" % path)
    lib = ctypes.CDLL(path)
    lib.esom_default_params.argtypes = [ctypes.POINTER(esom_params)]
    lib.esom_default_params.restype = None
    lib.esom_create.argtypes = [ctypes.c_int, _sz, ctypes.POINTER(_vp)]
    lib.esom_create.restype = ctypes.c_int
    lib.esom_destroy.argtypes = [_vp]
    lib.esom_destroy.restype = None
    lib.esom_last_error.argtypes = []
    lib.esom_last_error.restype = ctypes.c_char_p
    lib.esom_embed.argtypes = [_vp, _vp, _i64, _i32, _i64, _vp, _vp, _i32,
                               ctypes.POINTER(esom_params), _vp, _vp, _vp, _vp]
    lib.esom_embed.restype = ctypes.c_int
    lib.esom_embed_noalloc.argtypes = [_vp, _i64, _i32, _i64, _vp, _vp, _i32,
                                       ctypes.POINTER(esom_params), _vp, _vp, _vp, _vp]
    lib.esom_embed_noalloc.restype = ctypes.c_int
    lib.esom_landmark_update.argtypes = [_vp, _vp, _i64, _i32, _i64, _vp, _vp, _i32, _i32, _f32,
                                         _f32, _vp, _i64, _vp, _vp]
    lib.esom_landmark_update.restype = ctypes.c_int
    lib.esom_som_train.argtypes = [_vp, _vp, _i64, _i32, _i64, _vp, _vp, _i32, _vp, _i32, _i32,
                                   ctypes.POINTER(_f32), ctypes.POINTER(_f32), _vp, _vp]
    lib.esom_som_train.restype = ctypes.c_int
    lib.esom_fit_landmarks.argtypes = [_vp, _vp, _i32, _i32, _vp, _i32, _i32, _f32, _vp, _vp]
    lib.esom_fit_landmarks.restype = ctypes.c_int
    lib.esom_embed3.argtypes = [_vp, _vp, _i64, _i32, _i64, _vp, _vp, _i32,
                                ctypes.POINTER(esom_params), _vp, _vp, _vp]
    lib.esom_embed3.restype = ctypes.c_int
    lib.esom_landmark_graph.argtypes = [_vp, _i32, _i32, _i32, _vp, _vp, _vp]
    lib.esom_landmark_graph.restype = ctypes.c_int
    lib.esom_default_layout_params.argtypes = [ctypes.POINTER(esom_layout_params)]
    lib.esom_default_layout_params.restype = None
    lib.esom_graph_layout.argtypes = [_vp, _vp, _i32, _i32, _vp, _i32, _vp, _vp, _i32,
                                      ctypes.POINTER(esom_layout_params), _vp]
    lib.esom_graph_layout.restype = ctypes.c_int
    lib.esom_landmark_duplicate.argtypes = [_vp, _vp, _i32, _i32, _i32, _f32, _f32, _vp]
    lib.esom_landmark_duplicate.restype = ctypes.c_int
    lib.esom_landmark_remove.argtypes = [_vp, _vp, _i32, _i32, _i32, _vp]
    lib.esom_landmark_remove.restype = ctypes.c_int
    lib.esom_ablation_knn.argtypes = [_i32, _vp, _i64, _i32, _vp, _i32, _i32, _vp, _vp, _vp]
    lib.esom_ablation_knn.restype = ctypes.c_int
    lib.esom_ablation_project.argtypes = [_i32, _vp, _i64, _i32, _vp, _vp, _i32,
                                          ctypes.POINTER(esom_params), _vp, _vp, _vp, _vp]
    lib.esom_ablation_project.restype = ctypes.c_int
    lib.esom_sync.argtypes = [_vp, _vp]
    lib.esom_sync.restype = ctypes.c_int
    lib.esom_get_stats.argtypes = [_vp, _vp, ctypes.POINTER(esom_stats), _i32]
    lib.esom_get_stats.restype = ctypes.c_int
    lib.esom_get_fallback.argtypes = [_vp, _vp, _vp, _vp, _i64, ctypes.POINTER(_i64)]
    lib.esom_get_fallback.restype = ctypes.c_int
    lib.esom_set_timing.argtypes = [_vp, _i32]
    lib.esom_set_timing.restype = ctypes.c_int
    u64p = ctypes.POINTER(ctypes.c_uint64)
    lib.esom_serve_create.argtypes = [ctypes.c_int, _sz, _i32, ctypes.POINTER(_vp)]
    lib.esom_serve_create.restype = ctypes.c_int
    lib.esom_serve_destroy.argtypes = [_vp]
    lib.esom_serve_destroy.restype = None
    lib.esom_serve_dataset_put.argtypes = [_vp, _vp, _i64, _i32, u64p]
    lib.esom_serve_dataset_put.restype = ctypes.c_int
    lib.esom_serve_dataset_drop.argtypes = [_vp, ctypes.c_uint64]
    lib.esom_serve_dataset_drop.restype = ctypes.c_int
    lib.esom_serve_submit.argtypes = [_vp, ctypes.c_uint64, _vp, _i64, _i32, _vp, _vp, _i32,
                                      ctypes.POINTER(esom_params), _vp, u64p]
    lib.esom_serve_submit.restype = ctypes.c_int
    lib.esom_serve_wait.argtypes = [_vp, ctypes.c_uint64, _i32, ctypes.POINTER(esom_request_info)]
    lib.esom_serve_wait.restype = ctypes.c_int
    lib.esom_serve_get_stats.argtypes = [_vp, ctypes.POINTER(esom_serve_stats)]
    lib.esom_serve_get_stats.restype = ctypes.c_int
    _lib = lib
    return lib


def header_functions(header: str = HEADER):
    """Names of the functions include/esom.h declares."""
    txt = open(header).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(esom_[a-z_0-9]+)\s*\(", txt)))


def _check(rc):
    if rc != ESOM_OK:
        raise EsomError(rc, load().esom_last_error().decode())
    return rc


# ---- same-name wrappers (raw pointers) -------------------------------------------

def esom_default_params(**over) -> esom_params:
    p = esom_params()
    load().esom_default_params(ctypes.byref(p))
    for k, v in over.items():
        setattr(p, k, MODES.get(v, v) if k == "mode" else v)
    return p


def esom_create(device: int = 0, hbm_budget_bytes: int = 0) -> int:
    h = _vp()
    _check(load().esom_create(device, hbm_budget_bytes, ctypes.byref(h)))
    return h.value


def esom_destroy(ctx: int) -> None:
    load().esom_destroy(ctx)


def esom_last_error() -> str:
    return load().esom_last_error().decode()


def esom_embed(ctx, X, n, d, ldx, L_hd, L_2d, g, params, out, knn_idx=0, knn_dist2=0,
               stream=0) -> int:
    return load().esom_embed(ctx, X, n, d, ldx, L_hd, L_2d, g, ctypes.byref(params), out,
                             knn_idx or None, knn_dist2 or None, stream or None)


def esom_embed_noalloc(X, n, d, ldx, L_hd, L_2d, g, params, out, knn_idx=0, knn_dist2=0,
                       stream=0) -> int:
    return load().esom_embed_noalloc(X, n, d, ldx, L_hd, L_2d, g, ctypes.byref(params), out,
                                     knn_idx or None, knn_dist2 or None, stream or None)


def esom_landmark_update(ctx, X, n, d, ldx, L_hd, L_2d, g, kind, alpha, sigma, nearest=0,
                         nearest_ld=1, counts=0, stream=0) -> int:
    return load().esom_landmark_update(ctx, X, n, d, ldx, L_hd, L_2d or None, g, kind, alpha,
                                       sigma, nearest or None, nearest_ld, counts or None,
                                       stream or None)


def esom_som_train(ctx, X, n, d, ldx, L_hd, L_2d, g, batch_idx, batch, steps, sigma, alpha,
                   frozen=0, stream=0) -> int:
    """sigma, alpha: host sequences of `steps` floats."""
    sg = (_f32 * max(steps, 1))(*[float(v) for v in sigma])
    al = (_f32 * max(steps, 1))(*[float(v) for v in alpha])
    return load().esom_som_train(ctx, X, n, d, ldx, L_hd, L_2d, g, batch_idx, batch, steps, sg, al,
                                 frozen or None, stream or None)


def esom_fit_landmarks(L_hd, L_2d, g, d, p_2d, m, kfit, sigma, L_new, stream=0) -> int:
    return load().esom_fit_landmarks(L_hd, L_2d, g, d, p_2d, m, kfit, sigma, L_new, stream or None)


def esom_embed3(ctx, X, n, d, ldx, L_hd, L_3d, g, params, out, knn_idx=0, stream=0) -> int:
    return load().esom_embed3(ctx, X, n, d, ldx, L_hd, L_3d, g, ctypes.byref(params), out,
                              knn_idx or None, stream or None)


def esom_landmark_graph(L_hd, g, d, kg, nbr, dist2=0, stream=0) -> int:
    return load().esom_landmark_graph(L_hd, g, d, kg, nbr, dist2 or None, stream or None)


def esom_default_layout_params(**over) -> esom_layout_params:
    p = esom_layout_params()
    load().esom_default_layout_params(ctypes.byref(p))
    for k, v in over.items():
        setattr(p, k, v)
    return p


def esom_graph_layout(ctx, L_hd, g, d, nbr, kg, L_2d, fixed, steps, params, stream=0) -> int:
    return load().esom_graph_layout(ctx, L_hd, g, d, nbr, kg, L_2d, fixed or None, steps,
                                    ctypes.byref(params), stream or None)


def esom_landmark_duplicate(L_hd, L_2d, g, d, j, dx=0.0, dy=0.0, stream=0) -> int:
    return load().esom_landmark_duplicate(L_hd, L_2d, g, d, j, dx, dy, stream or None)


def esom_landmark_remove(L_hd, L_2d, g, d, j, stream=0) -> int:
    return load().esom_landmark_remove(L_hd, L_2d, g, d, j, stream or None)


ABL_KNN = {"base": 0, "shared": 1, "gridinsert": 2, "bitonic": 3}
ABL_PROJ = {"base": 0, "shared": 1, "aligned": 2, "registers": 3}


def esom_ablation_knn(algo, X, n, d, L_hd, g, k, knn_idx, knn_dist2, stream=0) -> int:
    return load().esom_ablation_knn(algo, X, n, d, L_hd, g, k, knn_idx, knn_dist2, stream or None)


def esom_ablation_project(algo, X, n, d, L_hd, L_2d, g, params, knn_idx, knn_dist2, out,
                          stream=0) -> int:
    return load().esom_ablation_project(algo, X, n, d, L_hd, L_2d, g, ctypes.byref(params), knn_idx,
                                        knn_dist2, out, stream or None)


def ablation_knn(algo, X, L, k, stream=None):
    """(idx n x k int32, dist2 n x k float32) from the named ablation kernel."""
    import torch
    X = _dev_f32(X, "X").contiguous()
    L = _dev_f32(L, "L", X.shape[1]).contiguous()
    n, d = X.shape
    idx = torch.empty((n, k), dtype=torch.int32, device=X.device)
    d2 = torch.empty((n, k), dtype=torch.float32, device=X.device)
    _check(esom_ablation_knn(ABL_KNN[algo], X.data_ptr(), n, d, L.data_ptr(), L.shape[0], k,
                             idx.data_ptr(), d2.data_ptr(), Context._stream(stream)))
    return idx, d2


def ablation_project(algo, X, L, l, idx, d2, out=None, stream=None, **params):
    """Projection (n x 2) from given neighbours with the named ablation kernel."""
    import torch
    X = _dev_f32(X, "X").contiguous()
    L = _dev_f32(L, "L", X.shape[1]).contiguous()
    l = _dev_f32(l, "l", 2).contiguous()
    n, d = X.shape
    k = idx.shape[1]
    if out is None:
        out = torch.empty((n, 2), dtype=torch.float32, device=X.device)
    p = esom_default_params(k=k, **params)
    _check(esom_ablation_project(ABL_PROJ[algo], X.data_ptr(), n, d, L.data_ptr(), l.data_ptr(),
                                 L.shape[0], p, idx.data_ptr(), d2.data_ptr(), out.data_ptr(),
                                 Context._stream(stream)))
    return out


def esom_sync(ctx, stream=0) -> int:
    return load().esom_sync(ctx, stream or None)


def esom_get_stats(ctx, stream=0, reset=False) -> dict:
    st = esom_stats()
    _check(load().esom_get_stats(ctx, stream or None, ctypes.byref(st), 1 if reset else 0))
    return st.as_dict()


def esom_get_fallback(ctx, stream=0, points=0, reasons=0, cap=0):
    """Returns (status, count); points / reasons are host addresses (or 0)."""
    cnt = _i64()
    rc = load().esom_get_fallback(ctx, stream or None, points or None, reasons or None, cap,
                                  ctypes.byref(cnt))
    return rc, cnt.value


def esom_set_timing(ctx, enable=True) -> int:
    return load().esom_set_timing(ctx, 1 if enable else 0)


# ---- torch convenience ------------------------------------------------------------

def _dev_f32(t, name, cols=None):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float32:
        raise TypeError("%s must be a float32 device tensor" % name)
    if t.dim() != 2 or (cols is not None and t.shape[1] != cols) or t.stride(1) != 1:
        raise ValueError("%s must be 2-D with unit column stride%s" %
                         (name, "" if cols is None else " and %d columns" % cols))
    return t


class Context:
    """Owns an esom context on one device; methods take torch device tensors."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        self.device = device
        self.handle = esom_create(device, hbm_budget_bytes)

    def close(self):
        if self.handle:
            esom_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _stream(stream):
        import torch
        if stream is None:
            return torch.cuda.current_stream().cuda_stream
        return getattr(stream, "cuda_stream", stream)

    def embed(self, X, L, l, k=16, mode="fp32", boost=1.0, adjust=1.0, cutoff=10.0,
              gravity=1e-5, candidates=0, out=None, knn=False, stream=None):
        """Returns out (n x 2), or (out, knn_idx n x k, knn_dist2 n x k) with knn=True."""
        import torch
        X = _dev_f32(X, "X")
        L = _dev_f32(L, "L", X.shape[1]).contiguous()
        l = _dev_f32(l, "l", 2).contiguous()
        n, d = X.shape
        g = L.shape[0]
        if out is None:
            out = torch.empty((n, 2), dtype=torch.float32, device=X.device)
        idx = dist = None
        if knn:
            idx = torch.empty((n, k), dtype=torch.int32, device=X.device)
            dist = torch.empty((n, k), dtype=torch.float32, device=X.device)
        p = esom_default_params(k=k, boost=boost, adjust=adjust, cutoff=cutoff, gravity=gravity,
                                mode=mode, candidates=candidates)
        _check(esom_embed(self.handle, X.data_ptr(), n, d, X.stride(0), L.data_ptr(),
                          l.data_ptr(), g, p, out.data_ptr(),
                          idx.data_ptr() if knn else 0, dist.data_ptr() if knn else 0,
                          self._stream(stream)))
        return (out, idx, dist) if knn else out

    def landmark_update(self, X, L, l, kind="kmeans", alpha=0.1, sigma=1.0, nearest=None,
                        counts=False, stream=None):
        """Updates L in place (stream-ordered); returns the counts tensor if asked."""
        import torch
        X = _dev_f32(X, "X")
        L = _dev_f32(L, "L", X.shape[1])
        if not L.is_contiguous():
            raise ValueError("L must be contiguous (it is updated in place)")
        n, d = X.shape
        g = L.shape[0]
        lp = _dev_f32(l, "l", 2).contiguous().data_ptr() if l is not None else 0
        cnt = torch.empty(g, dtype=torch.int32, device=X.device) if counts else None
        np_, nld = 0, 1
        if nearest is not None:
            # a 1-D int32 tensor of n entries at any stride (e.g. knn_idx[:, 0])
            if nearest.dtype != torch.int32 or nearest.dim() != 1 or nearest.shape[0] != n:
                raise TypeError("nearest must be a 1-D int32 tensor of n entries")
            np_, nld = nearest.data_ptr(), nearest.stride(0)
        _check(esom_landmark_update(self.handle, X.data_ptr(), n, d, X.stride(0), L.data_ptr(), lp,
                                    g, {"kmeans": 0, "som": 1}[kind], alpha, sigma, np_, nld,
                                    cnt.data_ptr() if counts else 0, self._stream(stream)))
        return cnt

    def som_train(self, X, L, l, batch_idx, sigma, alpha, frozen=None, stream=None):
        """Online SOM steps (see esom_som_train): trains L in place.  batch_idx is a
        steps x batch int32 device tensor; sigma and alpha are host sequences."""
        import torch
        X = _dev_f32(X, "X")
        L = _dev_f32(L, "L", X.shape[1])
        if not L.is_contiguous():
            raise ValueError("L must be contiguous (it is trained in place)")
        l = _dev_f32(l, "l", 2).contiguous()
        if (batch_idx.dtype != torch.int32 or batch_idx.dim() != 2 or not batch_idx.is_contiguous()
                or not batch_idx.is_cuda):
            raise TypeError("batch_idx must be a contiguous steps x batch int32 device tensor")
        steps, batch = batch_idx.shape
        if len(sigma) != steps or len(alpha) != steps:
            raise ValueError("sigma and alpha need one entry per step")
        fz = 0
        if frozen is not None:
            if frozen.dtype != torch.uint8 or frozen.numel() != L.shape[0] or not frozen.is_contiguous():
                raise TypeError("frozen must be a contiguous uint8 tensor of g entries")
            fz = frozen.data_ptr()
        _check(esom_som_train(self.handle, X.data_ptr(), X.shape[0], X.shape[1], X.stride(0),
                              L.data_ptr(), l.data_ptr(), L.shape[0], batch_idx.data_ptr(), batch,
                              steps, sigma, alpha, fz, self._stream(stream)))

    def embed3(self, X, L, l3, k=16, mode="fp32", boost=1.0, adjust=1.0, cutoff=10.0,
               gravity=1e-5, candidates=0, knn=False, stream=None):
        """3-D projection: returns out (n x 3), or (out, knn_idx n x k) with knn=True."""
        import torch
        X = _dev_f32(X, "X")
        L = _dev_f32(L, "L", X.shape[1]).contiguous()
        l3 = _dev_f32(l3, "l3", 3).contiguous()
        n, d = X.shape
        out = torch.empty((n, 3), dtype=torch.float32, device=X.device)
        idx = torch.empty((n, k), dtype=torch.int32, device=X.device) if knn else None
        p = esom_default_params(k=k, boost=boost, adjust=adjust, cutoff=cutoff, gravity=gravity,
                                mode=mode, candidates=candidates)
        _check(esom_embed3(self.handle, X.data_ptr(), n, d, X.stride(0), L.data_ptr(),
                           l3.data_ptr(), L.shape[0], p, out.data_ptr(),
                           idx.data_ptr() if knn else 0, self._stream(stream)))
        return (out, idx) if knn else out

    def graph_layout(self, L, nbr, l, steps=1, fixed=None, stream=None, **params):
        """Runs layout steps on l (g x 2 float32 device tensor, in place)."""
        import torch
        L = _dev_f32(L, "L").contiguous()
        l = _dev_f32(l, "l", 2)
        if not l.is_contiguous():
            raise ValueError("l must be contiguous (it is updated in place)")
        if nbr.dtype != torch.int32 or nbr.dim() != 2 or not nbr.is_contiguous():
            raise TypeError("nbr must be a contiguous g x kg int32 tensor")
        fz = 0
        if fixed is not None:
            if fixed.dtype != torch.uint8 or fixed.numel() != L.shape[0] or not fixed.is_contiguous():
                raise TypeError("fixed must be a contiguous uint8 tensor of g entries")
            fz = fixed.data_ptr()
        p = esom_default_layout_params(**params)
        _check(esom_graph_layout(self.handle, L.data_ptr(), L.shape[0], L.shape[1], nbr.data_ptr(),
                                 nbr.shape[1], l.data_ptr(), fz, steps, p, self._stream(stream)))

    def set_timing(self, enable=True):
        _check(esom_set_timing(self.handle, enable))

    def sync(self, stream=None):
        _check(esom_sync(self.handle, self._stream(stream)))

    def stats(self, reset=False, stream=None):
        return esom_get_stats(self.handle, self._stream(stream), reset)

    def fallback(self, stream=None):
        """(points int32, reasons uint8): the last call's exact-path list."""
        import numpy as np
        rc, n = esom_get_fallback(self.handle, self._stream(stream))
        _check(rc)
        pts = np.empty(n, np.int32)
        rsn = np.empty(n, np.uint8)
        rc, n2 = esom_get_fallback(self.handle, self._stream(stream), pts.ctypes.data,
                                   rsn.ctypes.data, n)
        _check(rc)
        return pts[:min(n, n2)], rsn[:min(n, n2)]


def landmark_graph(L, kg, stream=None):
    """(nbr g x kg int32, dist2 g x kg float32) device tensors: the kg nearest other
    landmarks of every landmark (see esom_landmark_graph)."""
    import torch
    L = _dev_f32(L, "L").contiguous()
    g, d = L.shape
    nbr = torch.empty((g, kg), dtype=torch.int32, device=L.device)
    dist = torch.empty((g, kg), dtype=torch.float32, device=L.device)
    _check(esom_landmark_graph(L.data_ptr(), g, d, kg, nbr.data_ptr(), dist.data_ptr(),
                               Context._stream(stream)))
    return nbr, dist


def fit_landmarks(L, l, p, kfit=8, sigma=1.0, stream=None):
    """High-dimensional positions (m x d device tensor) of landmarks added at the
    2-D positions p (m x 2 device tensor); see esom_fit_landmarks."""
    import torch
    L = _dev_f32(L, "L").contiguous()
    l = _dev_f32(l, "l", 2).contiguous()
    p = _dev_f32(p, "p", 2).contiguous()
    out = torch.empty((p.shape[0], L.shape[1]), dtype=torch.float32, device=L.device)
    st = Context._stream(stream)
    _check(esom_fit_landmarks(L.data_ptr(), l.data_ptr(), L.shape[0], L.shape[1], p.data_ptr(),
                              p.shape[0], kfit, sigma, out.data_ptr(), st))
    return out


# ---- serving (host arrays) ----------------------------------------------------------

def esom_serve_create(device=0, hbm_budget_bytes=0, n_slots=4) -> int:
    h = _vp()
    _check(load().esom_serve_create(device, hbm_budget_bytes, n_slots, ctypes.byref(h)))
    return h.value


def esom_serve_destroy(srv) -> None:
    load().esom_serve_destroy(srv)


def esom_serve_dataset_put(srv, X_ptr, n, d) -> int:
    did = ctypes.c_uint64()
    _check(load().esom_serve_dataset_put(srv, X_ptr, n, d, ctypes.byref(did)))
    return did.value


def esom_serve_dataset_drop(srv, dataset_id) -> int:
    return load().esom_serve_dataset_drop(srv, dataset_id)


def esom_serve_submit(srv, dataset_id, X_ptr, n, d, L_ptr, l_ptr, g, params, out_ptr):
    rid = ctypes.c_uint64()
    rc = load().esom_serve_submit(srv, dataset_id, X_ptr or None, n, d, L_ptr, l_ptr, g,
                                  ctypes.byref(params), out_ptr, ctypes.byref(rid))
    return rc, rid.value


def esom_serve_wait(srv, request_id, timeout_ms=-1):
    info = esom_request_info()
    rc = load().esom_serve_wait(srv, request_id, timeout_ms, ctypes.byref(info))
    return rc, info.as_dict()


def esom_serve_get_stats(srv) -> dict:
    st = esom_serve_stats()
    _check(load().esom_serve_get_stats(srv, ctypes.byref(st)))
    return st.as_dict()


class Server:
    """Serving runtime on host numpy arrays (float32, C-contiguous)."""

    def __init__(self, device=0, hbm_budget_bytes=0, n_slots=4):
        self.handle = esom_serve_create(device, hbm_budget_bytes, n_slots)
        self._keep = {}

    def close(self):
        if self.handle:
            esom_serve_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _f32(a, name):
        import numpy as np
        a = np.asarray(a)
        if a.dtype != np.float32 or not a.flags.c_contiguous or a.ndim != 2:
            raise TypeError("%s must be a C-contiguous 2-D float32 array" % name)
        return a

    def put(self, X):
        X = self._f32(X, "X")
        return esom_serve_dataset_put(self.handle, X.ctypes.data, X.shape[0], X.shape[1])

    def drop(self, dataset_id):
        _check(esom_serve_dataset_drop(self.handle, dataset_id))

    def submit(self, L, l, k=16, mode="fp32", dataset=0, X=None, out=None, **params):
        import numpy as np
        L = self._f32(L, "L")
        l = self._f32(l, "l")
        if dataset:
            n = None
        else:
            X = self._f32(X, "X")
            n = X.shape[0]
        p = esom_default_params(k=k, mode=mode, **params)
        if out is None:
            if n is None:
                raise ValueError("pass out= (n x 2 float32) for a resident dataset")
            out = np.empty((n, 2), np.float32)
        out = self._f32(out, "out")
        rc, rid = esom_serve_submit(self.handle, dataset, 0 if dataset else X.ctypes.data,
                                    0 if dataset else X.shape[0], L.shape[1], L.ctypes.data,
                                    l.ctypes.data, L.shape[0], p, out.ctypes.data)
        _check(rc)
        self._keep[rid] = (X, out, L, l)
        return rid

    def wait(self, rid, timeout_ms=-1):
        rc, info = esom_serve_wait(self.handle, rid, timeout_ms)
        if rc == ESOM_ETIMEOUT:
            return None
        keep = self._keep.pop(rid, None)
        _check(rc)
        info["out"] = keep[1]
        return info

    def stats(self):
        return esom_serve_get_stats(self.handle)
