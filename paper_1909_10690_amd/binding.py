"""Python binding of libgemi.so (include/gemi.h): argument marshalling only.

Torch tensors provide device memory and the current HIP stream; every step
of the metric runs in the library's HIP kernels.  There is no fallback: if
the library is not built, or no gfx950 device is present, calls raise.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgemi.so")

# status codes, dtypes and flags (mirror include/gemi.h)
MI_OK = 0
MI_ERR_NULL, MI_ERR_DIMS, MI_ERR_DTYPE, MI_ERR_BINS, MI_ERR_RANGE = -1, -2, -3, -4, -5
MI_ERR_Q, MI_ERR_WORKSPACE, MI_ERR_UNSUPPORTED, MI_ERR_FLAGS, MI_ERR_COUNT = -6, -7, -8, -9, -10
MI_ERR_SAMPLE, MI_ERR_TOO_LARGE, MI_ERR_GEOMETRY = -11, -12, -13
NOALLOC_SCRATCH_BYTES = 64 << 20  # MI_NOALLOC_SCRATCH_BYTES
MI_ERR_HIP, MI_ERR_NO_DEVICE = -20, -21
U8, U16, I16, F32 = 0, 1, 2, 3
BOUNDARY_EXCLUDE, BOUNDARY_CLAMP = 0x0, 0x1
TSALLIS_ADDITIVE, TSALLIS_PSEUDOADDITIVE = 0x0, 0x10
HIST_HARD, HIST_PARZEN = 0x0, 0x100
USE_GRAPH = 0x1000
VOLUMES_UNCHANGED = 0x2000  # reuse the workspace's prepared volumes (see include/gemi.h)
SAMPLED = 0x4000  # workspace sizing for eval_sampled
COMPACT_SLABS = 0x8000  # hint: bricks instead of thin slabs (rotation-heavy batches)
GRADIENT = 0x10000  # workspace sizing for grad
TIMER_HARD, TIMER_PARZEN_FWD, TIMER_PARZEN_BWD, TIMER_PAIRS, TIMER_REDUCE = 0, 1, 2, 3, 4

_TORCH_DTYPES = {torch.uint8: U8, torch.uint16: U16, torch.int16: I16, torch.float32: F32}


class GemiError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: status {status}: {status_string(status)}")


class MiVolume(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("nz", ctypes.c_int32), ("dtype", ctypes.c_int32), ("spacing", ctypes.c_double * 3),
                ("origin", ctypes.c_double * 3), ("lo", ctypes.c_double), ("hi", ctypes.c_double)]


class MiPair(ctypes.Structure):
    _fields_ = [("fixed", MiVolume), ("moving", MiVolume), ("transforms", ctypes.c_void_p),
                ("n_transforms", ctypes.c_int32)]


EXPORTS = ["mi_create", "mi_destroy", "mi_workspace_size", "mi_eval", "mi_eval_sampled", "mi_grad",
           "mi_pairs_workspace_size", "mi_eval_pairs", "mi_tune", "mi_timing_enable",
           "mi_timing_read", "mi_probe_lds_atomics", "mi_map_paths", "mi_eval_noalloc", "mi_tune_pairs",
           "mi_status_string"]

_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Loads libgemi.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    P, vp, sz = ctypes.POINTER, ctypes.c_void_p, ctypes.c_size_t
    i32, dp = ctypes.c_int32, P(ctypes.c_double)
    lib.mi_create.argtypes = [P(vp), ctypes.c_int]
    lib.mi_destroy.argtypes = [vp]
    lib.mi_workspace_size.argtypes = [vp, P(MiVolume), P(MiVolume), i32, i32, i32, i32, P(sz)]
    lib.mi_eval.argtypes = [vp, P(MiVolume), P(MiVolume), vp, i32, i32, dp, i32, i32, vp, vp, vp,
                            vp, sz, vp]
    lib.mi_eval_noalloc.argtypes = [vp, P(MiVolume), P(MiVolume), vp, i32, i32, dp, i32, i32, vp, vp, vp, vp]
    lib.mi_eval_sampled.argtypes = [vp, P(MiVolume), P(MiVolume), vp, i32, i32, dp, i32, i32,
                                    ctypes.c_double, ctypes.c_uint64, vp, vp, vp, vp, sz, vp]
    lib.mi_grad.argtypes = [vp, P(MiVolume), P(MiVolume), vp, i32, i32, dp, i32, i32, vp, vp, vp,
                            sz, vp]
    lib.mi_pairs_workspace_size.argtypes = [P(MiPair), i32, i32, i32, i32, P(sz)]
    lib.mi_eval_pairs.argtypes = [vp, P(MiPair), i32, i32, dp, i32, i32, vp, vp, sz, vp]
    lib.mi_tune.argtypes = [vp, P(MiVolume), P(MiVolume), vp, i32, i32, i32, vp, sz, vp]
    lib.mi_tune_pairs.argtypes = [vp, P(MiPair), i32, i32, i32, vp, sz, vp]
    lib.mi_timing_enable.argtypes = [vp, ctypes.c_int]
    lib.mi_timing_read.argtypes = [vp, ctypes.c_int, dp, P(ctypes.c_int64)]
    lib.mi_probe_lds_atomics.argtypes = [vp, vp, sz, vp, dp]
    lib.mi_map_paths.argtypes = [vp, vp, i32, i32, i32, i32, i32, i32, i32, vp, vp, vp, vp]
    lib.mi_status_string.argtypes = [ctypes.c_int]
    lib.mi_status_string.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name != "mi_status_string":
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def status_string(status: int) -> str:
    return load().mi_status_string(int(status)).decode()


def _check(status: int, where: str) -> None:
    if status != MI_OK:
        raise GemiError(status, where)


def _ptr(t) -> int | None:
    return None if t is None else t.data_ptr()


class Volume:
    """A device volume [nz][ny][nx] with the intensity range mapped onto bins,
    its voxel spacing (mm, x y z) and the position of voxel (0, 0, 0)."""

    def __init__(self, tensor: torch.Tensor, lo: float, hi: float, spacing=(1.0, 1.0, 1.0),
                 origin=(0.0, 0.0, 0.0)):
        if tensor.dim() != 3:
            raise ValueError("volume must be 3-D [nz][ny][nx]")
        if tensor.dtype not in _TORCH_DTYPES:
            raise ValueError(f"unsupported dtype {tensor.dtype}")
        self.tensor = tensor.contiguous()
        self.lo, self.hi = float(lo), float(hi)
        self.spacing = tuple(float(x) for x in spacing)
        self.origin = tuple(float(x) for x in origin)
        if len(self.spacing) != 3 or len(self.origin) != 3:
            raise ValueError("spacing and origin take three values (x, y, z)")

    @classmethod
    def from_numpy(cls, arr: np.ndarray, lo: float, hi: float, device="cuda", spacing=(1.0, 1.0, 1.0),
                   origin=(0.0, 0.0, 0.0)) -> "Volume":
        t = torch.from_numpy(np.ascontiguousarray(arr))
        return cls(t.to(device), lo, hi, spacing, origin)

    def c(self) -> MiVolume:
        nz, ny, nx = self.tensor.shape
        return MiVolume(self.tensor.data_ptr(), nx, ny, nz, _TORCH_DTYPES[self.tensor.dtype],
                        (ctypes.c_double * 3)(*self.spacing), (ctypes.c_double * 3)(*self.origin),
                        self.lo, self.hi)


def _qarr(q) -> tuple:
    qs = np.ascontiguousarray(np.atleast_1d(np.asarray(q, dtype=np.float64)))
    return qs, qs.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def flags_of(boundary: str = "exclude", tsallis: str = "additive", parzen: bool = False) -> int:
    f = {"exclude": BOUNDARY_EXCLUDE, "clamp": BOUNDARY_CLAMP}[boundary]
    f |= {"additive": TSALLIS_ADDITIVE, "pseudoadditive": TSALLIS_PSEUDOADDITIVE}[tsallis]
    if parzen:
        f |= HIST_PARZEN
    return f


# Field names of the three kinds of line in an MI_TUNE_CACHE file (the
# problem-class key, then the launch shape), as the library writes them.
_TUNE_FIELDS = {
    "gemi-tune": ("fnx", "fny", "fnz", "mnx", "mny", "mnz", "mdtype", "bins", "clamp", "n_bucket", "oct8",
                  "block", "slab_major", "chunks", "packed"),
    "gemi-tune-parzen": ("fnx", "fny", "fnz", "mnx", "mny", "mnz", "mdtype", "bins", "clamp", "n_bucket",
                         "fwd_block", "fwd_lds_kib", "bwd_block", "bwd_lds_kib", "chunk_shift"),
    "gemi-tune-pairs": ("pairs_bucket", "voxels_bucket", "transforms_bucket", "bins", "clamp", "oct8",
                        "block", "slab_voxels", "packed", "transform_major"),
}


def read_tune_cache(path: str) -> list[dict]:
    """The entries of an MI_TUNE_CACHE file as dicts ({"kind": tag, field:
    value, ...}); lines of another form are skipped."""
    out = []
    try:
        with open(path) as fh:
            lines = fh.read().splitlines()
    except OSError:
        return out
    for line in lines:
        parts = line.split()
        if not parts or parts[0] not in _TUNE_FIELDS:
            continue
        names = _TUNE_FIELDS[parts[0]]
        try:
            vals = [int(v) for v in parts[1:]]
        except ValueError:
            continue
        if len(vals) == len(names):
            out.append({"kind": parts[0], **dict(zip(names, vals))})
    return out


class Context:
    """A libgemi context on one HIP device."""

    def __init__(self, device: int = 0):
        self.lib = load()
        self.device = device
        h = ctypes.c_void_p()
        _check(self.lib.mi_create(ctypes.byref(h), device), "mi_create")
        self.handle = h
        self._ws = None

    def probe_lds_atomics(self, stream=None) -> float:
        """Measured peak rate of conflict-free LDS atomic adds (lane-atomics/s)."""
        scratch = self.workspace(4 << 20)
        rate = ctypes.c_double()
        _check(self.lib.mi_probe_lds_atomics(self.handle, _ptr(scratch), scratch.numel(), self._stream(stream),
                                              ctypes.byref(rate)), "mi_probe_lds_atomics")
        return rate.value

    def close(self) -> None:
        if self.handle:
            self.lib.mi_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _stream(self, stream) -> int:
        s = torch.cuda.current_stream(self.device) if stream is None else stream
        return s.cuda_stream

    def workspace(self, nbytes: int) -> torch.Tensor:
        """A cached device workspace of at least ``nbytes`` bytes."""
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=f"cuda:{self.device}")
        return self._ws

    def workspace_size(self, fixed: Volume, moving: Volume, n: int, bins: int, n_q: int,
                       flags: int = 0) -> int:
        """Workspace bytes of eval (``flags``), eval_sampled (| SAMPLED) or
        grad (| GRADIENT)."""
        out = ctypes.c_size_t()
        f, m = fixed.c(), moving.c()
        _check(self.lib.mi_workspace_size(self.handle, ctypes.byref(f), ctypes.byref(m), n, bins, n_q, flags,
                                          ctypes.byref(out)), "mi_workspace_size")
        return out.value

    def eval(self, fixed: Volume, moving: Volume, transforms: torch.Tensor, bins: int, q=(1.0,),
             flags: int = 0, want_hist: bool = False, want_overlap: bool = True, out=None,
             workspace: torch.Tensor | None = None, stream=None):
        """MI[n][n_q] (+ overlap[n], hist[n][bins][bins]) of n transforms."""
        dev = fixed.tensor.device
        transforms = transforms.to(device=dev, dtype=torch.float64).reshape(-1, 12).contiguous()
        n = transforms.shape[0]
        qs, qp = _qarr(q)
        mi = out if out is not None else torch.empty((n, len(qs)), dtype=torch.float64, device=dev)
        ov = torch.empty(n, dtype=torch.int64, device=dev) if want_overlap else None
        hist = torch.empty((n, bins, bins), dtype=torch.int32, device=dev) if want_hist else None
        if workspace is None:
            workspace = self.workspace(self.workspace_size(fixed, moving, n, bins, len(qs), flags))
        f, m = fixed.c(), moving.c()
        st = self.lib.mi_eval(self.handle, ctypes.byref(f), ctypes.byref(m), _ptr(transforms), n,
                              bins, qp, len(qs), flags, _ptr(mi), _ptr(ov), _ptr(hist),
                              _ptr(workspace), workspace.numel(), self._stream(stream))
        _check(st, "mi_eval")
        return mi, ov, hist

    def eval_noalloc(self, fixed: Volume, moving: Volume, transforms: torch.Tensor, bins: int, q=(1.0,),
                     flags: int = 0, out=None, overlap=None, hist=None, stream=None):
        """mi_eval through the allocation-free entry point (include/gemi.h,
        mi_eval_noalloc): the library's fixed device scratch instead of a
        workspace.  The caller may pass the outputs (``out`` [n][n_q] float64,
        ``overlap`` [n] int64, ``hist`` [n][bins][bins] int32) so that the
        call itself allocates nothing; missing ones are allocated here."""
        dev = fixed.tensor.device
        transforms = transforms.to(device=dev, dtype=torch.float64).reshape(-1, 12).contiguous()
        n = transforms.shape[0]
        qs, qp = _qarr(q)
        mi = out if out is not None else torch.empty((n, len(qs)), dtype=torch.float64, device=dev)
        f, m = fixed.c(), moving.c()
        st = self.lib.mi_eval_noalloc(self.handle, ctypes.byref(f), ctypes.byref(m), _ptr(transforms), n, bins,
                                      qp, len(qs), flags, _ptr(mi), _ptr(overlap), _ptr(hist),
                                      self._stream(stream))
        _check(st, "mi_eval_noalloc")
        return mi, overlap, hist

    def eval_sampled(self, fixed: Volume, moving: Volume, transforms: torch.Tensor, bins: int, q=(1.0,),
                     fraction: float = 0.1, seed: int = 0, flags: int = 0, want_hist: bool = False,
                     want_overlap: bool = True, out=None, workspace: torch.Tensor | None = None, stream=None):
        """MI[n][n_q] (+ overlap[n], hist) over a random subsample of the fixed
        voxels (include/gemi.h, mi_eval_sampled): each kept with probability
        ``fraction``, decided by SplitMix64 from (``seed``, voxel index)."""
        dev = fixed.tensor.device
        transforms = transforms.to(device=dev, dtype=torch.float64).reshape(-1, 12).contiguous()
        n = transforms.shape[0]
        qs, qp = _qarr(q)
        mi = out if out is not None else torch.empty((n, len(qs)), dtype=torch.float64, device=dev)
        ov = torch.empty(n, dtype=torch.int64, device=dev) if want_overlap else None
        hist = torch.empty((n, bins, bins), dtype=torch.int32, device=dev) if want_hist else None
        if workspace is None:
            workspace = self.workspace(self.workspace_size(fixed, moving, n, bins, len(qs), flags | SAMPLED))
        f, m = fixed.c(), moving.c()
        st = self.lib.mi_eval_sampled(self.handle, ctypes.byref(f), ctypes.byref(m), _ptr(transforms), n, bins,
                                      qp, len(qs), flags, float(fraction), int(seed) & (2 ** 64 - 1), _ptr(mi),
                                      _ptr(ov), _ptr(hist), _ptr(workspace), workspace.numel(),
                                      self._stream(stream))
        _check(st, "mi_eval_sampled")
        return mi, ov, hist

    def grad(self, fixed: Volume, moving: Volume, transforms: torch.Tensor, bins: int, q=(1.0,),
             flags: int = BOUNDARY_CLAMP, workspace: torch.Tensor | None = None, stream=None,
             out: tuple | None = None):
        """Parzen MI[n][n_q] and dMI/dP[n][n_q][12] with respect to the physical
        matrices (into ``out`` = (mi, grad) if given)."""
        dev = fixed.tensor.device
        transforms = transforms.to(device=dev, dtype=torch.float64).reshape(-1, 12).contiguous()
        n = transforms.shape[0]
        qs, qp = _qarr(q)
        if out is not None:
            mi, g = out
            if mi.shape != (n, len(qs)) or g.shape != (n, len(qs), 12) or mi.dtype != torch.float64 \
                    or g.dtype != torch.float64 or not mi.is_contiguous() or not g.is_contiguous():
                raise ValueError("out must be contiguous float64 tensors [n][n_q] and [n][n_q][12]")
        else:
            mi = torch.empty((n, len(qs)), dtype=torch.float64, device=dev)
            g = torch.empty((n, len(qs), 12), dtype=torch.float64, device=dev)
        if workspace is None:
            workspace = self.workspace(self.workspace_size(fixed, moving, n, bins, len(qs),
                                                           flags | HIST_PARZEN | GRADIENT))
        f, m = fixed.c(), moving.c()
        st = self.lib.mi_grad(self.handle, ctypes.byref(f), ctypes.byref(m), _ptr(transforms), n,
                              bins, qp, len(qs), flags, _ptr(mi), _ptr(g), _ptr(workspace),
                              workspace.numel(), self._stream(stream))
        _check(st, "mi_grad")
        return mi, g

    def grad_fn(self, fixed: Volume, moving: Volume, transforms: torch.Tensor, bins: int, q, flags: int,
                workspace: torch.Tensor, out: tuple, stream=None):
        """A function f(extra_flags) that runs :meth:`grad` on these arguments
        (device tensors, kept alive by the function) with ``flags |
        extra_flags``: the arguments are checked and marshalled once, for
        loops that call the same evaluation many times."""
        dev = fixed.tensor.device
        n = transforms.shape[0]
        qs, qp = _qarr(q)
        mi, g = out
        if transforms.dtype != torch.float64 or not transforms.is_contiguous() or transforms.device != dev \
                or transforms.shape != (n, 12):
            raise ValueError("transforms must be a contiguous float64 device tensor [n][12]")
        if mi.shape != (n, len(qs)) or g.shape != (n, len(qs), 12) or mi.dtype != torch.float64 \
                or g.dtype != torch.float64 or not mi.is_contiguous() or not g.is_contiguous():
            raise ValueError("out must be contiguous float64 tensors [n][n_q] and [n][n_q][12]")
        f, m = fixed.c(), moving.c()
        args = (self.handle, ctypes.byref(f), ctypes.byref(m), _ptr(transforms), n, bins, qp, len(qs))
        tail = (_ptr(mi), _ptr(g), _ptr(workspace), workspace.numel(), self._stream(stream))
        call, keep = self.lib.mi_grad, (f, m, qs, qp, transforms, mi, g, workspace)

        def run(extra_flags: int = 0):
            _check(call(*args, flags | extra_flags, *tail), "mi_grad")
            return keep[5], keep[6]
        return run

    @staticmethod
    def _pair_array(pairs):
        arr = (MiPair * len(pairs))()
        keep, total, dev = [], 0, None
        for i, (fv, mv, tr) in enumerate(pairs):
            tr = tr.to(device=fv.tensor.device, dtype=torch.float64).reshape(-1, 12).contiguous()
            keep.append(tr)
            dev = fv.tensor.device
            arr[i].fixed = fv.c()
            arr[i].moving = mv.c()
            arr[i].transforms = tr.data_ptr()
            arr[i].n_transforms = tr.shape[0]
            total += tr.shape[0]
        return arr, keep, total, dev

    def pairs_workspace_size(self, pairs, bins: int, n_q: int = 1, flags: int = 0) -> int:
        arr, _keep, _, _ = self._pair_array(pairs)
        nb = ctypes.c_size_t()
        _check(self.lib.mi_pairs_workspace_size(arr, len(pairs), bins, n_q, flags, ctypes.byref(nb)),
               "mi_pairs_workspace_size")
        return nb.value

    def eval_pairs(self, pairs, bins: int, q=(1.0,), flags: int = 0,
                   workspace: torch.Tensor | None = None, stream=None, out=None):
        """Hard MI of many (fixed, moving, transforms) pairs in one launch;
        returns MI[sum n][n_q] with the pairs' rows concatenated (into
        ``out`` if given)."""
        qs, qp = _qarr(q)
        if not pairs:
            return torch.zeros((0, len(qs)), dtype=torch.float64)
        arr, _keep, total, dev = self._pair_array(pairs)
        mi = out if out is not None else torch.empty((total, len(qs)), dtype=torch.float64, device=dev)
        if workspace is None:
            workspace = self.workspace(self.pairs_workspace_size(pairs, bins, len(qs), flags))
        st = self.lib.mi_eval_pairs(self.handle, arr, len(pairs), bins, qp, len(qs), flags,
                                    _ptr(mi), _ptr(workspace), workspace.numel(),
                                    self._stream(stream))
        _check(st, "mi_eval_pairs")
        return mi

    def tune_pairs(self, pairs, bins: int, flags: int = 0, workspace: torch.Tensor | None = None,
                   stream=None) -> None:
        """Autotunes the persistent multi-pair sweep's launch shape for this
        class of pair set (synchronous; results are unaffected)."""
        if not pairs:
            return
        arr, _keep, _, _ = self._pair_array(pairs)
        if workspace is None:
            workspace = self.workspace(self.pairs_workspace_size(pairs, bins, 1, flags))
        _check(self.lib.mi_tune_pairs(self.handle, arr, len(pairs), bins, flags, _ptr(workspace),
                                      workspace.numel(), self._stream(stream)), "mi_tune_pairs")

    def tune(self, fixed: Volume, moving: Volume, transforms: torch.Tensor, bins: int, flags: int = 0,
             workspace: torch.Tensor | None = None, stream=None) -> None:
        """Autotunes the launch shape of the hard-binned sweep, or with
        HIST_PARZEN in ``flags`` of the Parzen sweeps, for this problem class
        (synchronous; hard results are unaffected, Parzen ones only in the
        last bits)."""
        transforms = transforms.to(device=fixed.tensor.device, dtype=torch.float64).reshape(-1, 12).contiguous()
        n = transforms.shape[0]
        if workspace is None:
            if flags & HIST_PARZEN:
                workspace = self.workspace(self.workspace_size(fixed, moving, n, bins, 2, flags | GRADIENT))
            else:
                workspace = self.workspace(self.workspace_size(fixed, moving, n, bins, 1, flags))
        f, m = fixed.c(), moving.c()
        _check(self.lib.mi_tune(self.handle, ctypes.byref(f), ctypes.byref(m), _ptr(transforms), n, bins,
                                flags, _ptr(workspace), workspace.numel(), self._stream(stream)), "mi_tune")

    def map_paths(self, values: torch.Tensor, direction: int = 1, centre=None, stream=None):
        """Discrete gradient paths on a [nz][ny][nx] map (include/gemi.h,
        mi_map_paths): returns (next, sink) int32 tensors of the map's shape
        and stats int64[4] = (extrema, sink of the centre, its basin size,
        capture radius), all on the map's device.  ``centre`` = (cx, cy, cz),
        the grid centre by default."""
        if values.dim() != 3:
            raise ValueError("values must be a 3D [nz][ny][nx] map")
        if values.device.type != "cuda":
            raise ValueError("values must be a device (cuda) tensor")
        values = values.to(dtype=torch.float64).contiguous()
        nz, ny, nx = values.shape
        cx, cy, cz = ((nx - 1) // 2, (ny - 1) // 2, (nz - 1) // 2) if centre is None else centre
        nxt = torch.empty(values.shape, dtype=torch.int32, device=values.device)
        sink = torch.empty(values.shape, dtype=torch.int32, device=values.device)
        stats = torch.empty(4, dtype=torch.int64, device=values.device)
        _check(self.lib.mi_map_paths(self.handle, _ptr(values), nx, ny, nz, int(direction), int(cx), int(cy),
                                     int(cz), _ptr(nxt), _ptr(sink), _ptr(stats), self._stream(stream)),
               "mi_map_paths")
        return nxt, sink, stats

    def timing(self, enable: bool) -> None:
        _check(self.lib.mi_timing_enable(self.handle, int(enable)), "mi_timing_enable")

    def timing_read(self, which: int) -> tuple[float, int]:
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        _check(self.lib.mi_timing_read(self.handle, which, ctypes.byref(ms), ctypes.byref(n)),
               "mi_timing_read")
        return ms.value, n.value
