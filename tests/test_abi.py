"""CPU tests of the C ABI boundary: the library loads, exports every entry
point include/gemi.h declares, and rejects invalid arguments with the
documented status before touching a GPU (no device is needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1909_10690_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gemi.h")

FAKE = 0x10000  # a non-NULL address that validation must never dereference


def header_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:int|const char \*)\s*(mi_\w+)\(", text, re.M)))


def test_header_declares_expected_entry_points():
    assert header_functions() == sorted(B.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = B.load()
    for name in header_functions():
        assert hasattr(lib, name), name


def header_signatures():
    text = open(HEADER).read()
    sigs = {}
    for name, params in re.findall(r"^(?:int|const char \*)\s*(mi_\w+)\(([^)]*)\);", text, re.M | re.S):
        sigs[name] = [p.strip() for p in params.replace("\n", " ").split(",") if p.strip()]
    return sigs


def test_binding_declares_argument_types_of_every_entry_point():
    """Every entry point has ctypes argtypes matching its C parameters: a
    pointer or size_t passed without them would travel as a 32-bit int and
    reach the library truncated."""
    import ctypes
    lib = B.load()
    sigs = header_signatures()
    assert sorted(sigs) == sorted(B.EXPORTS)
    for name, params in sigs.items():
        at = getattr(lib, name).argtypes
        assert at is not None, name
        assert len(at) == len(params), (name, at, params)
        for p, t in zip(params, at):
            if "*" in p or "size_t" in p:
                wide = t in (ctypes.c_void_p, ctypes.c_size_t, ctypes.c_char_p) or issubclass(t, ctypes._Pointer)
                assert wide, (name, p, t)
            elif p.startswith("double"):
                assert t is ctypes.c_double, (name, p, t)
            elif p.startswith("uint64_t"):
                assert t is ctypes.c_uint64, (name, p, t)
            else:
                assert t in (ctypes.c_int, ctypes.c_int32), (name, p, t)


def test_header_constants_match_binding():
    text = open(HEADER).read()
    consts = dict((k, int(v, 0)) for k, v in re.findall(r"#define (MI_\w+) \(?(-?\w+)\)?", text))
    assert consts["MI_ERR_NULL"] == B.MI_ERR_NULL and consts["MI_ERR_HIP"] == B.MI_ERR_HIP
    assert consts["MI_ERR_COUNT"] == B.MI_ERR_COUNT and consts["MI_ERR_NO_DEVICE"] == B.MI_ERR_NO_DEVICE
    assert consts["MI_HIST_PARZEN"] == B.HIST_PARZEN and consts["MI_BOUNDARY_CLAMP"] == B.BOUNDARY_CLAMP
    assert consts["MI_TSALLIS_PSEUDOADDITIVE"] == B.TSALLIS_PSEUDOADDITIVE
    assert consts["MI_USE_GRAPH"] == B.USE_GRAPH
    assert consts["MI_SAMPLED"] == B.SAMPLED and consts["MI_ERR_SAMPLE"] == B.MI_ERR_SAMPLE
    assert consts["MI_COMPACT_SLABS"] == B.COMPACT_SLABS
    assert consts["MI_GRADIENT"] == B.GRADIENT and consts["MI_ERR_GEOMETRY"] == B.MI_ERR_GEOMETRY
    assert consts["MI_ERR_TOO_LARGE"] == B.MI_ERR_TOO_LARGE
    # data, nx, ny, nz, dtype, spacing[3], origin[3], lo, hi
    assert ctypes.sizeof(B.MiVolume) == 88 and B.MiVolume.lo.offset == 72


def test_status_strings():
    for s in [0, -1, -2, -3, -4, -5, -6, -7, -8, -9, -10, -11, -12, -13, -20, -21, 12345]:
        assert isinstance(B.status_string(s), str) and B.status_string(s)
    assert B.status_string(0) == "ok"


def vol(nx=8, ny=8, nz=8, dtype=B.U8, lo=0.0, hi=255.0, data=FAKE, spacing=(1.0, 1.0, 1.0),
        origin=(0.0, 0.0, 0.0)):
    return B.MiVolume(data, nx, ny, nz, dtype, (ctypes.c_double * 3)(*spacing), (ctypes.c_double * 3)(*origin),
                      lo, hi)


def call_eval(f, m, n=4, bins=32, q=(1.0,), flags=0, transforms=FAKE, mi=FAKE, ws=FAKE,
              ws_bytes=1 << 40, hist=None, ctx=None):
    lib = B.load()
    qs = np.asarray(q, dtype=np.float64) if q is not None else None
    qp = qs.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if q is not None else None
    return lib.mi_eval(ctx, ctypes.byref(f), ctypes.byref(m), transforms, n, bins, qp,
                       0 if q is None else len(qs), flags, mi, None, hist, ws, ws_bytes, None)


def test_valid_arguments_reach_the_context_check():
    # everything valid but the context: MI_ERR_NULL, nothing launched
    assert call_eval(vol(), vol()) == B.MI_ERR_NULL


@pytest.mark.parametrize("kw,status", [
    (dict(nx=1), B.MI_ERR_DIMS), (dict(ny=4097), B.MI_ERR_DIMS), (dict(nz=0), B.MI_ERR_DIMS),
    (dict(nx=4096, ny=4096, nz=17), B.MI_ERR_DIMS),
    (dict(dtype=7), B.MI_ERR_DTYPE), (dict(dtype=-1), B.MI_ERR_DTYPE),
    (dict(lo=5.0, hi=5.0), B.MI_ERR_RANGE), (dict(lo=0.5), B.MI_ERR_RANGE),
    (dict(hi=float("nan")), B.MI_ERR_RANGE), (dict(lo=0.0, hi=65536.0), B.MI_ERR_RANGE),
    (dict(data=None), B.MI_ERR_NULL),
    (dict(spacing=(1.0, 0.0, 1.0)), B.MI_ERR_GEOMETRY), (dict(spacing=(-2.0, 1.0, 1.0)), B.MI_ERR_GEOMETRY),
    (dict(spacing=(1.0, 1.0, float("inf"))), B.MI_ERR_GEOMETRY),
    (dict(spacing=(1.0, float("nan"), 1.0)), B.MI_ERR_GEOMETRY),
    (dict(origin=(0.0, float("nan"), 0.0)), B.MI_ERR_GEOMETRY),
    (dict(origin=(float("-inf"), 0.0, 0.0)), B.MI_ERR_GEOMETRY),
    (dict(spacing=(0.25, 3.0, 1e-3), origin=(-120.5, 7.0, 1e6)), B.MI_ERR_NULL),
])
def test_volume_validation(kw, status):
    assert call_eval(vol(**kw), vol()) == status
    assert call_eval(vol(), vol(**kw)) == status


def test_moving_gather_layout_limit():
    """A fixed volume may hold 2^28 voxels; a moving one stays below 2^28
    (integer: 16-byte oct volume) or below 2^28 voxels including one extra
    slice (float, Parzen: 16-byte fp32 quads), so its gather layout fits
    32-bit buffer offsets."""
    big = dict(nx=4096, ny=4096, nz=16)
    assert call_eval(vol(**big), vol()) == B.MI_ERR_NULL
    assert call_eval(vol(), vol(**big)) == B.MI_ERR_DIMS
    assert call_eval(vol(), vol(nx=4096, ny=4095, nz=16)) == B.MI_ERR_NULL
    fbig = dict(nx=4096, ny=4096, nz=15, dtype=B.F32, lo=0.0, hi=1.0)   # 15 + 1 slices = 2^28
    assert call_eval(vol(), vol(**fbig), flags=B.HIST_PARZEN) == B.MI_ERR_DIMS
    fok = dict(nx=4096, ny=4095, nz=15, dtype=B.F32, lo=0.0, hi=1.0)
    assert call_eval(vol(), vol(**fok), flags=B.HIST_PARZEN) == B.MI_ERR_NULL


def test_float_moving_needs_parzen():
    assert call_eval(vol(), vol(dtype=B.F32, lo=0.0, hi=1.0)) == B.MI_ERR_DTYPE
    assert call_eval(vol(dtype=B.F32, lo=0.0, hi=1.0), vol()) == B.MI_ERR_NULL  # fixed f32 is fine
    assert call_eval(vol(), vol(dtype=B.F32, lo=0.0, hi=0.5), flags=B.HIST_PARZEN) == B.MI_ERR_NULL


def test_full_u16_range_is_valid():
    assert call_eval(vol(dtype=B.U16, lo=0.0, hi=65535.0), vol(dtype=B.I16, lo=-32768.0, hi=32767.0)) == B.MI_ERR_NULL


@pytest.mark.parametrize("bins,flags,status", [
    (1, 0, B.MI_ERR_BINS), (257, 0, B.MI_ERR_BINS), (2, 0, B.MI_ERR_NULL), (256, 0, B.MI_ERR_NULL),
    (7, B.HIST_PARZEN, B.MI_ERR_BINS), (8, B.HIST_PARZEN, B.MI_ERR_NULL),
])
def test_bins_validation(bins, flags, status):
    assert call_eval(vol(), vol(), bins=bins, flags=flags) == status


@pytest.mark.parametrize("q,status", [
    ((), B.MI_ERR_Q), ((0.0,), B.MI_ERR_Q), ((-1.0,), B.MI_ERR_Q), ((float("nan"),), B.MI_ERR_Q),
    ((float("inf"),), B.MI_ERR_Q), (tuple([1.0] * 17), B.MI_ERR_Q), (tuple([1.5] * 16), B.MI_ERR_NULL),
])
def test_q_validation(q, status):
    assert call_eval(vol(), vol(), q=q) == status


def test_q_null():
    assert call_eval(vol(), vol(), q=None) == B.MI_ERR_Q


def test_flags_count_pointers_workspace():
    assert call_eval(vol(), vol(), flags=0x2) == B.MI_ERR_FLAGS
    assert call_eval(vol(), vol(), n=-1) == B.MI_ERR_COUNT
    assert call_eval(vol(), vol(), n=(1 << 24) + 1) == B.MI_ERR_COUNT
    assert call_eval(vol(), vol(), transforms=None) == B.MI_ERR_NULL
    assert call_eval(vol(), vol(), ws=None) == B.MI_ERR_WORKSPACE
    assert call_eval(vol(), vol(), ws_bytes=100) == B.MI_ERR_WORKSPACE
    assert call_eval(vol(), vol(), hist=FAKE, flags=B.HIST_PARZEN) == B.MI_ERR_UNSUPPORTED


def ws_size(f, m, n, bins, n_q, flags=0):
    out = ctypes.c_size_t()
    st = B.load().mi_workspace_size(None, ctypes.byref(f), ctypes.byref(m), n, bins, n_q, flags,
                                    ctypes.byref(out))
    return st, out.value


def test_workspace_size_layout():
    a = lambda x: (x + 255) // 256 * 256
    # MI partial sums: per transform, slice (min(1024 // n, B // 8) for
    # B >= 16) and entropy, three compensated pairs of doubles
    part = a(5 * min(1024 // 5, 32 // 8) * 2 * 3 * 16)
    # the index-space matrices composed from the physical ones, then the hard
    # sweep's processing order (u32 per transform)
    xf = a(5 * 96) + a(5 * 4)
    st, n = ws_size(vol(10, 11, 12), vol(9, 8, 7), 5, 32, 2)
    # moving range <= 256: oct volume of 8-bit corners, 8 bytes per voxel;
    # histograms; N per transform
    assert st == 0 and n == xf + a(10 * 11 * 12) + a(9 * 8 * 7 * 8) + a(5 * 32 * 32 * 4) + a(5 * 8) + part
    # a wider range: 16-bit corners, 16 bytes per voxel
    st, n = ws_size(vol(10, 11, 12), vol(9, 8, 7, dtype=B.U16, lo=0.0, hi=4095.0), 5, 32, 2)
    assert st == 0 and n == xf + a(10 * 11 * 12) + a(9 * 8 * 7 * 16) + a(5 * 32 * 32 * 4) + a(5 * 8) + part
    octs = a(8 * 8 * 9 * 8)  # Parzen: 16-bit quads, 8 bytes per voxel, one extra slice
    # occupied fixed-bin rows (used, row_of_slot, slot_of_row, n_slots), then
    # one u32 slot-group mask per 16 x 4 wave tile of the fixed volume and
    # one per row group (4 rows of a slice)
    rowmap = a(3 * 256 * 4 + 4) + a(4 * ((11 + 3) // 4) * 12 * ((10 + 15) // 16 + 1))
    st, n = ws_size(vol(10, 11, 12), vol(), 5, 32, 2, B.HIST_PARZEN)
    assert st == 0 and n == xf + a(1320) + octs + rowmap + a(5 * 32 * 32 * 8) + a(5 * 8) + part
    st, n = ws_size(vol(10, 11, 12), vol(), 5, 32, 2, B.GRADIENT)
    # gradient: + the table marginals f64[n][2B] + dMI/dp tables f32[n][n_q][B][B]
    assert st == 0 and n == (xf + a(1320) + octs + rowmap + a(5 * 32 * 32 * 8) + a(5 * 8) + part + a(5 * 2 * 32 * 8)
                             + a(5 * 2 * 32 * 32 * 4))
    # a float moving volume keeps fp32 quads: 16 bytes per voxel, one extra slice
    st, n = ws_size(vol(10, 11, 12), vol(dtype=B.F32, lo=0.0, hi=1.0), 5, 32, 2, B.HIST_PARZEN)
    assert st == 0 and n == xf + a(1320) + a(8 * 8 * 9 * 16) + rowmap + a(5 * 32 * 32 * 8) + a(5 * 8) + part
    assert ws_size(vol(), vol(), 5, 1, 1)[0] == B.MI_ERR_BINS
    assert ws_size(vol(), vol(), 5, 32, 0)[0] == B.MI_ERR_Q


def test_create_without_gpu_reports_no_device():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    assert B.load().mi_create(ctypes.byref(h), 0) == B.MI_ERR_NO_DEVICE
    assert B.load().mi_destroy(None) == 0


def test_timing_and_pairs_null_checks():
    lib = B.load()
    assert lib.mi_timing_enable(None, 1) == B.MI_ERR_NULL
    ms, n = ctypes.c_double(), ctypes.c_int64()
    assert lib.mi_timing_read(None, 0, ctypes.byref(ms), ctypes.byref(n)) == B.MI_ERR_NULL


@pytest.mark.parametrize("dims,centre,direction,status", [
    ((51, 51, 51), (25, 25, 25), 1, B.MI_ERR_NULL),       # valid: reaches the context check
    ((1, 1, 1), (0, 0, 0), -1, B.MI_ERR_NULL),
    ((4096, 4096, 1), (0, 4095, 0), 1, B.MI_ERR_NULL),
    ((0, 5, 5), (0, 0, 0), 1, B.MI_ERR_DIMS),
    ((4097, 1, 1), (0, 0, 0), 1, B.MI_ERR_DIMS),
    ((4096, 4096, 128), (0, 0, 0), 1, B.MI_ERR_DIMS),    # 2^31 points
    ((5, 5, 5), (5, 0, 0), 1, B.MI_ERR_DIMS),
    ((5, 5, 5), (0, -1, 0), 1, B.MI_ERR_DIMS),
    ((5, 5, 5), (2, 2, 2), 0, B.MI_ERR_FLAGS),
    ((5, 5, 5), (2, 2, 2), 2, B.MI_ERR_FLAGS),
])
def test_map_paths_validation(dims, centre, direction, status):
    lib = B.load()
    nx, ny, nz = dims
    cx, cy, cz = centre
    assert lib.mi_map_paths(None, FAKE, nx, ny, nz, direction, cx, cy, cz, FAKE, FAKE, FAKE, None) == status


def test_map_paths_null_buffers():
    lib = B.load()
    for k in range(4):
        ptrs = [FAKE] * 4
        ptrs[k] = None
        v, nx_, sk, st = ptrs
        assert lib.mi_map_paths(None, v, 5, 5, 5, 1, 2, 2, 2, nx_, sk, st, None) == B.MI_ERR_NULL


def test_graph_flag_accepted_and_unknown_bits_rejected():
    assert call_eval(vol(), vol(), flags=B.USE_GRAPH) == B.MI_ERR_NULL
    assert call_eval(vol(), vol(), flags=B.USE_GRAPH | B.HIST_PARZEN) == B.MI_ERR_NULL
    assert call_eval(vol(), vol(), flags=B.VOLUMES_UNCHANGED | B.HIST_PARZEN) == B.MI_ERR_NULL
    assert call_eval(vol(), vol(), flags=B.SAMPLED) == B.MI_ERR_FLAGS  # mi_eval_sampled's flag
    assert call_eval(vol(), vol(), flags=B.COMPACT_SLABS) == B.MI_ERR_NULL  # a hint: accepted
    assert call_eval(vol(), vol(), flags=B.COMPACT_SLABS | B.HIST_PARZEN) == B.MI_ERR_NULL
    assert call_eval(vol(), vol(), flags=B.GRADIENT) == B.MI_ERR_FLAGS  # mi_grad's sizing flag
    assert call_eval(vol(), vol(), flags=0x20000) == B.MI_ERR_FLAGS


def call_sampled(f, m, fraction=0.25, seed=7, n=4, bins=32, flags=0, ws_bytes=1 << 40, hist=None, ws=FAKE):
    lib = B.load()
    qs = np.asarray((1.0, 2.0), dtype=np.float64)
    return lib.mi_eval_sampled(None, ctypes.byref(f), ctypes.byref(m), FAKE, n, bins,
                               qs.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 2, flags, fraction, seed,
                               FAKE, None, hist, ws, ws_bytes, None)


def test_sampled_validation():
    assert call_sampled(vol(), vol()) == B.MI_ERR_NULL            # valid: reaches the context check
    assert call_sampled(vol(), vol(), fraction=1.0, seed=2 ** 64 - 1) == B.MI_ERR_NULL
    assert call_sampled(vol(), vol(), fraction=3.0) == B.MI_ERR_NULL   # >= 1 keeps every voxel
    assert call_sampled(vol(), vol(), flags=B.SAMPLED | B.HIST_PARZEN) == B.MI_ERR_NULL
    for bad in (0.0, -0.5, float("nan"), float("inf")):
        assert call_sampled(vol(), vol(), fraction=bad) == B.MI_ERR_SAMPLE
    assert call_sampled(vol(), vol(), flags=0x20000) == B.MI_ERR_FLAGS
    assert call_sampled(vol(), vol(), flags=B.GRADIENT) == B.MI_ERR_FLAGS
    assert call_sampled(vol(), vol(), flags=B.HIST_PARZEN, hist=FAKE) == B.MI_ERR_UNSUPPORTED
    assert call_sampled(vol(), vol(), ws=None) == B.MI_ERR_WORKSPACE
    # the plain workspace is too small: the sample list is missing
    st, plain = ws_size(vol(), vol(), 4, 32, 2)
    st2, sampled = ws_size(vol(), vol(), 4, 32, 2, B.SAMPLED)
    assert st == st2 == 0 and sampled == plain + 8 * 8 * 8 * 8 + 256
    assert call_sampled(vol(), vol(), ws_bytes=plain) == B.MI_ERR_WORKSPACE
    assert call_sampled(vol(), vol(), ws_bytes=sampled) == B.MI_ERR_NULL
    # no sampled gradient
    assert ws_size(vol(), vol(), 4, 32, 2, B.SAMPLED | B.GRADIENT)[0] == B.MI_ERR_UNSUPPORTED


def test_tune_validation():
    lib = B.load()
    f, m = vol(), vol()
    assert lib.mi_tune(None, ctypes.byref(f), ctypes.byref(m), FAKE, 4, 32, 0, FAKE, 1 << 40, None) == B.MI_ERR_NULL
    # Parzen tuning: valid arguments reach the context check; a workspace
    # sized for one entropy's gradient is too small (it needs n_q = 2)
    assert lib.mi_tune(None, ctypes.byref(f), ctypes.byref(m), FAKE, 4, 32, B.HIST_PARZEN, FAKE, 1 << 40,
                       None) == B.MI_ERR_NULL
    st, one = ws_size(f, m, 4, 32, 1, B.HIST_PARZEN | B.GRADIENT)
    st2, two = ws_size(f, m, 4, 32, 2, B.HIST_PARZEN | B.GRADIENT)
    assert st == st2 == 0 and two > one
    assert lib.mi_tune(None, ctypes.byref(f), ctypes.byref(m), FAKE, 4, 32, B.HIST_PARZEN, FAKE, one,
                       None) == B.MI_ERR_WORKSPACE
    assert lib.mi_tune(None, ctypes.byref(f), ctypes.byref(m), FAKE, 4, 32, B.HIST_PARZEN, FAKE, two,
                       None) == B.MI_ERR_NULL
    assert lib.mi_tune(None, ctypes.byref(f), ctypes.byref(m), FAKE, 4, 32, B.SAMPLED, FAKE, 1 << 40,
                       None) == B.MI_ERR_FLAGS
    assert lib.mi_tune(None, ctypes.byref(f), ctypes.byref(m), FAKE, 4, 1, 0, FAKE, 1 << 40, None) == B.MI_ERR_BINS


def pairs_ws(pairs, bins=32, n_q=1, flags=0):
    arr = (B.MiPair * len(pairs))(*pairs)
    out = ctypes.c_size_t()
    st = B.load().mi_pairs_workspace_size(arr, len(pairs), bins, n_q, flags, ctypes.byref(out))
    return st, out.value


def test_pairs_validation_and_layout():
    p1 = B.MiPair(vol(8, 8, 8), vol(9, 8, 7), FAKE, 3)
    p2 = B.MiPair(vol(16, 4, 2), vol(5, 6, 7, dtype=B.U16, lo=0.0, hi=4095.0), FAKE, 0)
    st, n = pairs_ws([p1, p2], bins=32, n_q=2)
    assert st == 0 and n > 0
    # per-pair fixed bins + oct volumes (16-bit corners: p2's range exceeds
    # 256) + 3 transforms' histograms are included
    assert n >= 8 * 8 * 8 + 9 * 8 * 7 * 16 + 16 * 4 * 2 + 5 * 6 * 7 * 16 + 3 * 32 * 32 * 4
    bad = B.MiPair(vol(8, 8, 8), vol(dtype=B.F32, lo=0.0, hi=1.0), FAKE, 3)
    assert pairs_ws([p1, bad])[0] == B.MI_ERR_DTYPE
    assert pairs_ws([B.MiPair(vol(), vol(), None, 3)])[0] == B.MI_ERR_NULL
    assert pairs_ws([B.MiPair(vol(), vol(), FAKE, -1)])[0] == B.MI_ERR_COUNT
    assert pairs_ws([p1], bins=300)[0] == B.MI_ERR_BINS
    assert pairs_ws([p1], flags=B.HIST_PARZEN)[0] == B.MI_ERR_FLAGS
    assert pairs_ws([])[0] == 0


def test_registration_checkpoint_roundtrip(tmp_path):
    from paper_1909_10690_amd.register import RegState
    s = RegState(params=[1.0, 0, 0, 0, 1.0, 0, 0, 0, 1.0, 0.5, -0.25, 2.0], step=7,
                 m=[0.1] * 12, v=[0.2] * 12, history=[(1, [0.3, 0.4])])
    p = tmp_path / "state.json"
    s.save(str(p))
    r = RegState.load(str(p))
    assert r.params == s.params and r.step == 7 and r.m == s.m and r.v == s.v
    assert [tuple(h) if not isinstance(h, tuple) else h for h in r.history][0][0] == 1


def test_tune_pairs_validation():
    lib = B.load()
    p1 = B.MiPair(vol(8, 8, 8), vol(9, 8, 7), FAKE, 3)
    arr = (B.MiPair * 1)(p1)
    ok = lib.mi_tune_pairs(None, arr, 1, 32, 0, FAKE, 1 << 40, None)
    assert ok == B.MI_ERR_NULL  # valid: reaches the context check
    assert lib.mi_tune_pairs(None, arr, 1, 32, B.USE_GRAPH, FAKE, 1 << 40, None) == B.MI_ERR_FLAGS
    assert lib.mi_tune_pairs(None, arr, 1, 32, B.VOLUMES_UNCHANGED, FAKE, 1 << 40, None) == B.MI_ERR_FLAGS
    assert lib.mi_tune_pairs(None, arr, 1, 300, 0, FAKE, 1 << 40, None) == B.MI_ERR_BINS
    assert lib.mi_tune_pairs(None, arr, 1, 32, 0, None, 1 << 40, None) == B.MI_ERR_WORKSPACE
    # mi_eval_pairs takes MI_VOLUMES_UNCHANGED
    assert pairs_ws([p1], flags=B.VOLUMES_UNCHANGED)[0] == 0
