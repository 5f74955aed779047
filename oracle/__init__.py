"""Plain FP64 CPU EmbedSOM oracle -- TEST INFRASTRUCTURE ONLY.

The arithmetic lives in ``esom_oracle.c`` (plain C, double precision, direct
differences, sorted insertion, Cramer's rule).  This module only compiles it
with gcc and marshals numpy arrays through ctypes.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never does, and this
package never imports the GPU library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "esom_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

DEFAULT_BOOST = 1.0
DEFAULT_ADJUST = 1.0
DEFAULT_CUTOFF = 10.0
DEFAULT_GRAVITY = 1e-5


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no FMA contraction, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fPIC", "-shared",
               "-pthread", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        f32p = ctypes.POINTER(ctypes.c_float)
        f64p = ctypes.POINTER(ctypes.c_double)
        i32p = ctypes.POINTER(ctypes.c_int32)
        i64p = ctypes.POINTER(ctypes.c_int64)
        i64, i32, dbl = ctypes.c_int64, ctypes.c_int, ctypes.c_double
        u8p = ctypes.POINTER(ctypes.c_uint8)
        lib.oracle_scores.argtypes = [f64p, i32, i32, dbl, dbl, f64p]
        lib.oracle_scores.restype = i32
        lib.oracle_knn.argtypes = [f32p, i64, i32, i64, f32p, i32, i32, i32p, f64p, i32]
        lib.oracle_knn.restype = i32
        lib.oracle_embed.argtypes = [f32p, i64, i32, i64, f32p, f32p, i32, i32, dbl, dbl,
                                     dbl, dbl, f64p, i32p, f64p, i64p, i32]
        lib.oracle_embed.restype = i32
        lib.oracle_landmark_update.argtypes = [f32p, i64, i32, i64, f32p, f32p, i32, i32,
                                               dbl, dbl, f64p, i64p, i32]
        lib.oracle_landmark_update.restype = i32
        lib.oracle_som_train.argtypes = [f32p, i64, i32, i64, f32p, f32p, i32, i32p, i32, i32,
                                         f64p, f64p, u8p]
        lib.oracle_som_train.restype = i32
        lib.oracle_fit_landmarks.argtypes = [f32p, f32p, i32, i32, f32p, i32, i32, dbl, f64p]
        lib.oracle_fit_landmarks.restype = i32
        lib.oracle_embed3.argtypes = lib.oracle_embed.argtypes
        lib.oracle_embed3.restype = i32
        lib.oracle_landmark_graph.argtypes = [f32p, i32, i32, i32, i32p, f64p]
        lib.oracle_landmark_graph.restype = i32
        lib.oracle_layout_step.argtypes = [f32p, i32, i32, i32p, i32, f32p, u8p, dbl, dbl, dbl,
                                           dbl, dbl]
        lib.oracle_layout_step.restype = i32
        _lib = lib
    return _lib


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _f32_rows(X):
    X = np.asarray(X)
    if X.dtype != np.float32:
        raise TypeError("oracle inputs must already be float32 (the GPU's inputs)")
    if X.ndim != 2:
        raise ValueError("expected a 2-D float32 array")
    if X.strides[1] != 4 or X.strides[0] % 4 or X.strides[0] < 4 * X.shape[1]:
        X = np.ascontiguousarray(X)
    return X, X.strides[0] // 4


def scores(delta, g, boost=DEFAULT_BOOST, cutoff=DEFAULT_CUTOFF):
    """Scores of sorted neighbour distances (Euclidean).  Returns (s, degenerate)."""
    lib = _load()
    d = np.ascontiguousarray(delta, dtype=np.float64)
    s = np.zeros_like(d)
    rc = lib.oracle_scores(_ptr(d, ctypes.c_double), len(d), int(g), float(boost),
                           float(cutoff), _ptr(s, ctypes.c_double))
    if rc < 0:
        raise ValueError("oracle_scores: invalid arguments")
    return s, bool(rc == 1)


def knn(X, L, m, threads=1):
    """The m nearest landmarks of every row of X: (idx int32 n x m, d2 float64 n x m)."""
    lib = _load()
    X, ldx = _f32_rows(X)
    L = np.ascontiguousarray(L, dtype=np.float32)
    n, d = X.shape
    g = L.shape[0]
    idx = np.empty((n, m), np.int32)
    d2 = np.empty((n, m), np.float64)
    rc = lib.oracle_knn(_ptr(X, ctypes.c_float), n, d, ldx, _ptr(L, ctypes.c_float), g, m,
                        _ptr(idx, ctypes.c_int32), _ptr(d2, ctypes.c_double), threads)
    if rc != 0:
        raise ValueError("oracle_knn failed (%d)" % rc)
    return idx, d2


def embed(X, L, l, k, boost=DEFAULT_BOOST, adjust=DEFAULT_ADJUST, cutoff=DEFAULT_CUTOFF,
          gravity=DEFAULT_GRAVITY, threads=1):
    """EmbedSOM projection.  Returns dict(out n x 2 f64, idx n x (k+1), d2 n x (k+1),
    n_degenerate)."""
    lib = _load()
    X, ldx = _f32_rows(X)
    L = np.ascontiguousarray(L, dtype=np.float32)
    l = np.ascontiguousarray(l, dtype=np.float32)
    n, d = X.shape
    g = L.shape[0]
    if L.shape[1] != d or l.shape != (g, 2):
        raise ValueError("shape mismatch")
    out = np.empty((n, 2), np.float64)
    idx = np.empty((n, k + 1), np.int32)
    d2 = np.empty((n, k + 1), np.float64)
    ndeg = ctypes.c_int64(0)
    rc = lib.oracle_embed(_ptr(X, ctypes.c_float), n, d, ldx, _ptr(L, ctypes.c_float),
                          _ptr(l, ctypes.c_float), g, int(k), float(boost), float(adjust),
                          float(cutoff), float(gravity), _ptr(out, ctypes.c_double),
                          _ptr(idx, ctypes.c_int32), _ptr(d2, ctypes.c_double),
                          ctypes.byref(ndeg), int(threads))
    if rc != 0:
        raise ValueError("oracle_embed failed (%d)" % rc)
    return {"out": out, "idx": idx, "d2": d2, "n_degenerate": int(ndeg.value)}


def landmark_update(X, L, l, kind, alpha, sigma=0.0, threads=1):
    """One batch landmark step (kind 'kmeans' or 'som').  Returns (L_new f64, counts)."""
    lib = _load()
    X, ldx = _f32_rows(X)
    L = np.ascontiguousarray(L, dtype=np.float32)
    l = np.ascontiguousarray(l, dtype=np.float32)
    n, d = X.shape
    g = L.shape[0]
    kid = {"kmeans": 0, "som": 1}[kind]
    Lout = np.empty((g, d), np.float64)
    counts = np.empty(g, np.int64)
    rc = lib.oracle_landmark_update(_ptr(X, ctypes.c_float), n, d, ldx,
                                    _ptr(L, ctypes.c_float), _ptr(l, ctypes.c_float), g, kid,
                                    float(alpha), float(sigma), _ptr(Lout, ctypes.c_double),
                                    _ptr(counts, ctypes.c_int64), int(threads))
    if rc != 0:
        raise ValueError("oracle_landmark_update failed (%d)" % rc)
    return Lout, counts


def som_train(X, L, l, batch_idx, sigma, alpha, frozen=None):
    """Online SOM training steps (mini-batch form of the online rule).  batch_idx
    is T x B int32 (rows of X per step); sigma, alpha have T entries.  Returns
    the trained landmarks (float32 g x d, a new array)."""
    lib = _load()
    X, ldx = _f32_rows(X)
    Lw = np.array(L, dtype=np.float32, order="C", copy=True)
    l = np.ascontiguousarray(l, dtype=np.float32)
    bi = np.ascontiguousarray(batch_idx, dtype=np.int32)
    T, B = bi.shape
    sg = np.ascontiguousarray(sigma, dtype=np.float64)
    al = np.ascontiguousarray(alpha, dtype=np.float64)
    if sg.shape != (T,) or al.shape != (T,):
        raise ValueError("sigma and alpha need one entry per step")
    fz = None
    if frozen is not None:
        fz = np.ascontiguousarray(frozen, dtype=np.uint8)
    n, d = X.shape
    rc = lib.oracle_som_train(_ptr(X, ctypes.c_float), n, d, ldx, _ptr(Lw, ctypes.c_float),
                              _ptr(l, ctypes.c_float), len(Lw), _ptr(bi, ctypes.c_int32), B, T,
                              _ptr(sg, ctypes.c_double), _ptr(al, ctypes.c_double),
                              _ptr(fz, ctypes.c_uint8) if fz is not None else None)
    if rc != 0:
        raise ValueError("oracle_som_train failed (%d)" % rc)
    return Lw


def fit_landmarks(L, l, p, kfit=8, sigma=1.0):
    """High-dimensional positions (m x d float64) of landmarks added at the 2-D
    positions p (m x 2), fitted from their kfit nearest 2-D landmarks."""
    lib = _load()
    L = np.ascontiguousarray(L, dtype=np.float32)
    l = np.ascontiguousarray(l, dtype=np.float32)
    p = np.ascontiguousarray(p, dtype=np.float32).reshape(-1, 2)
    g, d = L.shape
    out = np.empty((len(p), d), np.float64)
    rc = lib.oracle_fit_landmarks(_ptr(L, ctypes.c_float), _ptr(l, ctypes.c_float), g, d,
                                  _ptr(p, ctypes.c_float), len(p), int(kfit), float(sigma),
                                  _ptr(out, ctypes.c_double))
    if rc != 0:
        raise ValueError("oracle_fit_landmarks failed (%d)" % rc)
    return out


def embed3(X, L, l3, k, boost=DEFAULT_BOOST, adjust=DEFAULT_ADJUST, cutoff=DEFAULT_CUTOFF,
           gravity=DEFAULT_GRAVITY, threads=1):
    """The projection with 3-D landmark positions l3 (g x 3).  Returns dict(out n x 3
    f64, idx n x (k+1), d2 n x (k+1), n_degenerate)."""
    lib = _load()
    X, ldx = _f32_rows(X)
    L = np.ascontiguousarray(L, dtype=np.float32)
    l3 = np.ascontiguousarray(l3, dtype=np.float32)
    n, d = X.shape
    g = L.shape[0]
    if L.shape[1] != d or l3.shape != (g, 3):
        raise ValueError("shape mismatch")
    out = np.empty((n, 3), np.float64)
    idx = np.empty((n, k + 1), np.int32)
    d2 = np.empty((n, k + 1), np.float64)
    ndeg = ctypes.c_int64(0)
    rc = lib.oracle_embed3(_ptr(X, ctypes.c_float), n, d, ldx, _ptr(L, ctypes.c_float),
                           _ptr(l3, ctypes.c_float), g, int(k), float(boost), float(adjust),
                           float(cutoff), float(gravity), _ptr(out, ctypes.c_double),
                           _ptr(idx, ctypes.c_int32), _ptr(d2, ctypes.c_double),
                           ctypes.byref(ndeg), int(threads))
    if rc != 0:
        raise ValueError("oracle_embed3 failed (%d)" % rc)
    return {"out": out, "idx": idx, "d2": d2, "n_degenerate": int(ndeg.value)}


def landmark_graph(L, kg):
    """kg nearest other landmarks of every landmark: (nbr int32 g x kg, d2 f64 g x kg)."""
    lib = _load()
    L = np.ascontiguousarray(L, dtype=np.float32)
    g, d = L.shape
    nbr = np.empty((g, kg), np.int32)
    d2 = np.empty((g, kg), np.float64)
    rc = lib.oracle_landmark_graph(_ptr(L, ctypes.c_float), g, d, int(kg),
                                   _ptr(nbr, ctypes.c_int32), _ptr(d2, ctypes.c_double))
    if rc != 0:
        raise ValueError("oracle_landmark_graph failed (%d)" % rc)
    return nbr, d2


def layout(L, nbr, l, steps=1, fixed=None, scale=1.0, repulsion=0.0, soft=1.0, step=0.1,
           max_move=1.0):
    """`steps` synchronous force-layout steps of the 2-D positions l (g x 2) on the
    landmark graph nbr.  Returns the new positions (float32 g x 2, a new array)."""
    lib = _load()
    L = np.ascontiguousarray(L, dtype=np.float32)
    nb = np.ascontiguousarray(nbr, dtype=np.int32)
    lw = np.array(l, dtype=np.float32, order="C", copy=True)
    g, d = L.shape
    fz = None if fixed is None else np.ascontiguousarray(fixed, dtype=np.uint8)
    for _ in range(steps):
        rc = lib.oracle_layout_step(_ptr(L, ctypes.c_float), g, d, _ptr(nb, ctypes.c_int32),
                                    nb.shape[1], _ptr(lw, ctypes.c_float),
                                    _ptr(fz, ctypes.c_uint8) if fz is not None else None,
                                    float(scale), float(repulsion), float(soft), float(step),
                                    float(max_move))
        if rc != 0:
            raise ValueError("oracle_layout_step failed (%d)" % rc)
    return lw
