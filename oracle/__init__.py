"""CPU oracle for the generalised-entropy MI metric (arXiv 1909.10690).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package; the product library
and its Python binding never do.  It shares no code with the GPU path.

The arithmetic lives in ``mi_oracle.c`` (plain loops, 128-bit integers,
long-double entropies); this module builds it with gcc and wraps it with
ctypes.  Every function cites the passage of the paper it follows:

* Eq. (1) Shannon entropies, Eq. (2) MI, Discussion (one histogram serves
  Shannon and Tsallis), Fig. 1 (transform -> metric pipeline).  Transforms
  are physical fixed -> moving 3x4 matrices (mm); each volume carries its
  voxel spacing and origin, and ``compose`` gives the index-space matrix.
* Tsallis entropy, trilinear interpolation, binning, overlap rule and the
  Parzen/B-spline variant are not printed in the paper; they follow the
  readings recorded in the repository's design notes.

* Random subsampling (Discussion: Mattes' MI samples voxels at random):
  SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) from its published
  definition decides, per fixed voxel, whether it takes part.

Parity status: every function is pinned by tests in ``tests/test_oracle_*``
against closed forms, library routines and exact rational brute force.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mi_oracle.c")
_LIB = os.path.join(_HERE, "libmi_oracle.so")

U8, U16, I16, F32 = 0, 1, 2, 3
EXCLUDE, CLAMP = 0, 1
ADDITIVE, PSEUDOADDITIVE = 0, 1

_DTYPES = {np.dtype(np.uint8): U8, np.dtype(np.uint16): U16,
           np.dtype(np.int16): I16, np.dtype(np.float32): F32}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
                               "-std=gnu11", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Volume(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("nz", ctypes.c_int32), ("dtype", ctypes.c_int32), ("lo", ctypes.c_double),
                ("hi", ctypes.c_double), ("spacing", ctypes.c_double * 3), ("origin", ctypes.c_double * 3)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        vp = P(_Volume)
        dp = P(ctypes.c_double)
        lib.or_compose.argtypes = [vp, vp, dp, dp]
        lib.or_quantize.argtypes = [dp, P(ctypes.c_int64)]
        lib.or_quantize.restype = ctypes.c_int
        lib.or_hist_hard.argtypes = [vp, vp, dp, ctypes.c_int, ctypes.c_int, P(ctypes.c_uint32)]
        lib.or_hist_hard.restype = ctypes.c_int64
        lib.or_mi_from_counts.argtypes = [P(ctypes.c_uint32), ctypes.c_int, ctypes.c_int64, dp,
                                          ctypes.c_int, ctypes.c_int, dp]
        lib.or_mi_from_table.argtypes = [dp, ctypes.c_int, ctypes.c_double, dp, ctypes.c_int,
                                         ctypes.c_int, dp]
        lib.or_eval_hard.argtypes = [vp, vp, dp, ctypes.c_int, ctypes.c_int, dp, ctypes.c_int,
                                     ctypes.c_int, ctypes.c_int, dp, P(ctypes.c_int64),
                                     P(ctypes.c_uint32)]
        lib.or_beta3.argtypes = [ctypes.c_double]
        lib.or_beta3.restype = ctypes.c_double
        lib.or_dbeta3.argtypes = [ctypes.c_double]
        lib.or_dbeta3.restype = ctypes.c_double
        lib.or_parzen_table.argtypes = [vp, vp, dp, ctypes.c_int, ctypes.c_int, dp]
        lib.or_parzen_table.restype = ctypes.c_int64
        lib.or_parzen_grad.argtypes = [vp, vp, dp, ctypes.c_int, dp, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_int, dp, dp]
        lib.or_parzen_grad.restype = ctypes.c_int64
        lib.or_grad_batch.argtypes = [vp, vp, dp, ctypes.c_int, ctypes.c_int, dp, ctypes.c_int,
                                      ctypes.c_int, ctypes.c_int, dp, dp]
        lib.or_eval_parzen.argtypes = [vp, vp, dp, ctypes.c_int, ctypes.c_int, dp, ctypes.c_int,
                                       ctypes.c_int, ctypes.c_int, dp, P(ctypes.c_int64)]
        u64 = ctypes.c_uint64
        lib.or_splitmix64.argtypes = [u64, u64]
        lib.or_splitmix64.restype = u64
        lib.or_hist_hard_sampled.argtypes = [vp, vp, dp, ctypes.c_int, ctypes.c_int, ctypes.c_double, u64,
                                             P(ctypes.c_uint32)]
        lib.or_hist_hard_sampled.restype = ctypes.c_int64
        lib.or_eval_hard_sampled.argtypes = [vp, vp, dp, ctypes.c_int, ctypes.c_int, dp, ctypes.c_int,
                                             ctypes.c_int, ctypes.c_int, ctypes.c_double, u64, dp,
                                             P(ctypes.c_int64), P(ctypes.c_uint32)]
        lib.or_parzen_table_sampled.argtypes = [vp, vp, dp, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                                u64, dp]
        lib.or_parzen_table_sampled.restype = ctypes.c_int64
        lib.or_eval_parzen_sampled.argtypes = [vp, vp, dp, ctypes.c_int, ctypes.c_int, dp, ctypes.c_int,
                                               ctypes.c_int, ctypes.c_int, ctypes.c_double, u64, dp,
                                               P(ctypes.c_int64)]
        lib.or_num_threads.restype = ctypes.c_int
        lib.or_set_num_threads.argtypes = [ctypes.c_int]
        _lib = lib
    return _lib


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def volume(arr: np.ndarray, lo: float, hi: float, spacing=(1.0, 1.0, 1.0), origin=(0.0, 0.0, 0.0)) -> tuple:
    """Describe a C-order [nz][ny][nx] array with its voxel spacing and the
    position of voxel (0, 0, 0) (mm, x y z); keeps the array alive."""
    arr = np.ascontiguousarray(arr)
    if arr.ndim != 3 or arr.dtype not in _DTYPES:
        raise ValueError("volume must be a 3-D uint8/uint16/int16/float32 array")
    nz, ny, nx = arr.shape
    sp = (ctypes.c_double * 3)(*[float(x) for x in spacing])
    og = (ctypes.c_double * 3)(*[float(x) for x in origin])
    v = _Volume(arr.ctypes.data, nx, ny, nz, _DTYPES[arr.dtype], float(lo), float(hi), sp, og)
    return (v, arr)


def _mats(M) -> np.ndarray:
    M = np.ascontiguousarray(np.asarray(M, dtype=np.float64).reshape(-1, 12))
    return M


def _qs(q) -> np.ndarray:
    return np.ascontiguousarray(np.atleast_1d(np.asarray(q, dtype=np.float64)))


def compose(fixed, moving, P) -> np.ndarray:
    """Index-space 3x4 matrix (fixed voxel index -> moving continuous index)
    of one physical fixed -> moving matrix P, for the volumes' spacings and
    origins (Fig. 1 Transform block; transforms in mm, Methodology)."""
    lib = _load()
    P = _mats(P)[0].copy()
    out = np.zeros(12)
    lib.or_compose(ctypes.byref(fixed[0]), ctypes.byref(moving[0]), _ptr(P, ctypes.c_double),
                   _ptr(out, ctypes.c_double))
    return out.reshape(3, 4)


def quantize(M) -> tuple[np.ndarray, int]:
    """Q32 quantisation of one index-space 3x4 matrix; returns (Mq, status)."""
    lib = _load()
    M = _mats(M)[0].copy()
    out = np.zeros(12, dtype=np.int64)
    st = lib.or_quantize(_ptr(M, ctypes.c_double), _ptr(out, ctypes.c_int64))
    return out, int(st)


def hist_hard(fixed, moving, M, bins: int, boundary: int = EXCLUDE) -> tuple[np.ndarray, int]:
    """Hard-binned joint histogram [bins][bins] (row = fixed bin) and overlap
    count of one physical transform M.  ``fixed``/``moving`` come from
    :func:`volume`."""
    lib = _load()
    M = _mats(M)[0].copy()
    h = np.zeros((bins, bins), dtype=np.uint32)
    n = lib.or_hist_hard(ctypes.byref(fixed[0]), ctypes.byref(moving[0]), _ptr(M, ctypes.c_double),
                         bins, boundary, _ptr(h, ctypes.c_uint32))
    return h, int(n)


def mi_from_counts(hist: np.ndarray, q, form: int = ADDITIVE) -> np.ndarray:
    """MI for every q of a count histogram (Eq. (1), Eq. (2); q == 1 is Shannon)."""
    lib = _load()
    hist = np.ascontiguousarray(hist, dtype=np.uint32)
    bins = hist.shape[0]
    qs = _qs(q)
    out = np.zeros(len(qs))
    lib.or_mi_from_counts(_ptr(hist, ctypes.c_uint32), bins, int(hist.sum(dtype=np.int64)),
                          _ptr(qs, ctypes.c_double), len(qs), form, _ptr(out, ctypes.c_double))
    return out


def mi_from_table(table: np.ndarray, N: float, q, form: int = ADDITIVE) -> np.ndarray:
    """MI for every q of a real joint table normalised by N."""
    lib = _load()
    table = np.ascontiguousarray(table, dtype=np.float64)
    qs = _qs(q)
    out = np.zeros(len(qs))
    lib.or_mi_from_table(_ptr(table, ctypes.c_double), table.shape[0], float(N),
                         _ptr(qs, ctypes.c_double), len(qs), form, _ptr(out, ctypes.c_double))
    return out


def splitmix64(seed: int, i: int) -> int:
    """SplitMix64 output for counter i of the stream seeded with ``seed``."""
    return int(_load().or_splitmix64(seed & (2 ** 64 - 1), i))


def eval_hard(fixed, moving, M, bins: int, q, boundary: int = EXCLUDE, form: int = ADDITIVE,
              want_hist: bool = False, sample=None):
    """Hard-binned MI of a batch of transforms: (mi[n][nq], overlap[n], hist or None).
    ``sample`` = (fraction, seed) keeps each fixed voxel by the random
    subsampling rule (Discussion); None keeps every voxel."""
    lib = _load()
    M = _mats(M)
    n = M.shape[0]
    qs = _qs(q)
    mi = np.zeros((n, len(qs)))
    ov = np.zeros(n, dtype=np.int64)
    hist = np.zeros((n, bins, bins), dtype=np.uint32) if want_hist else None
    frac, seed = (1.0, 0) if sample is None else (float(sample[0]), int(sample[1]))
    lib.or_eval_hard_sampled(ctypes.byref(fixed[0]), ctypes.byref(moving[0]), _ptr(M, ctypes.c_double), n,
                             bins, _ptr(qs, ctypes.c_double), len(qs), boundary, form, frac, seed,
                             _ptr(mi, ctypes.c_double), _ptr(ov, ctypes.c_int64),
                             _ptr(hist, ctypes.c_uint32) if want_hist else None)
    return mi, ov, hist


def beta3(t: float) -> float:
    return _load().or_beta3(float(t))


def dbeta3(t: float) -> float:
    return _load().or_dbeta3(float(t))


def parzen_table(fixed, moving, M, bins: int, boundary: int = CLAMP, sample=None) -> tuple[np.ndarray, int]:
    """Unnormalised Parzen joint table [bins][bins] and normaliser N
    (``sample`` = (fraction, seed) as in :func:`eval_hard`)."""
    lib = _load()
    M = _mats(M)[0].copy()
    h = np.zeros((bins, bins))
    frac, seed = (1.0, 0) if sample is None else (float(sample[0]), int(sample[1]))
    n = lib.or_parzen_table_sampled(ctypes.byref(fixed[0]), ctypes.byref(moving[0]),
                                    _ptr(M, ctypes.c_double), bins, boundary, frac, seed,
                                    _ptr(h, ctypes.c_double))
    return h, int(n)


def hist_hard_sampled(fixed, moving, M, bins: int, boundary: int, fraction: float, seed: int):
    """Hard-binned joint histogram and overlap count of one transform over the
    fixed voxels the random subsampling rule keeps."""
    lib = _load()
    M = _mats(M)[0].copy()
    h = np.zeros((bins, bins), dtype=np.uint32)
    n = lib.or_hist_hard_sampled(ctypes.byref(fixed[0]), ctypes.byref(moving[0]), _ptr(M, ctypes.c_double),
                                 bins, boundary, float(fraction), int(seed), _ptr(h, ctypes.c_uint32))
    return h, int(n)


def parzen_grad(fixed, moving, M, bins: int, q, boundary: int = CLAMP, form: int = ADDITIVE):
    """Parzen MI [n][nq] and gradient [n][nq][12] w.r.t. the entries of the
    physical matrix."""
    lib = _load()
    M = _mats(M)
    n = M.shape[0]
    qs = _qs(q)
    mi = np.zeros((n, len(qs)))
    g = np.zeros((n, len(qs), 12))
    lib.or_grad_batch(ctypes.byref(fixed[0]), ctypes.byref(moving[0]), _ptr(M, ctypes.c_double), n,
                      bins, _ptr(qs, ctypes.c_double), len(qs), boundary, form,
                      _ptr(mi, ctypes.c_double), _ptr(g, ctypes.c_double))
    return mi, g


def eval_parzen(fixed, moving, M, bins: int, q, boundary: int = CLAMP, form: int = ADDITIVE, sample=None):
    """Parzen MI [n][nq] and normaliser [n] of a batch of transforms
    (``sample`` = (fraction, seed) as in :func:`eval_hard`)."""
    lib = _load()
    M = _mats(M)
    n = M.shape[0]
    qs = _qs(q)
    mi = np.zeros((n, len(qs)))
    ov = np.zeros(n, dtype=np.int64)
    frac, seed = (1.0, 0) if sample is None else (float(sample[0]), int(sample[1]))
    lib.or_eval_parzen_sampled(ctypes.byref(fixed[0]), ctypes.byref(moving[0]), _ptr(M, ctypes.c_double),
                               n, bins, _ptr(qs, ctypes.c_double), len(qs), boundary, form, frac, seed,
                               _ptr(mi, ctypes.c_double), _ptr(ov, ctypes.c_int64))
    return mi, ov


def num_threads() -> int:
    return int(_load().or_num_threads())


def set_num_threads(n: int) -> None:
    """OpenMP threads of later oracle calls (results do not depend on it)."""
    _load().or_set_num_threads(int(n))
