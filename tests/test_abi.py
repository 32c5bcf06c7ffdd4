"""CPU-side checks of the C ABI: the library loads, exports every symbol that
include/fft.h declares, and rejects bad arguments before touching the GPU.
Also the host-only plan logic (decomposition choice) and the autotune cache
format.  No compute call is made here."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "fft.h")).read()
    return sorted(set(re.findall(r"^(?:fft_status|const char \*|size_t)\s*(fft_\w+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def fftlib():
    import paper_2308_00497_amd as m
    return m


@pytest.fixture(scope="module")
def lib(fftlib):
    return fftlib.lib


def test_header_declares_the_boundary():
    names = header_functions()
    for required in ("fft_plan_create", "fft_execute", "fft_execute_backward", "fft_plan_destroy",
                     "fft_plan_create_ragged", "fft_plan_workspace_bytes", "fft_plan_set_workspace",
                     "fft_status_string"):
        assert required in names


def test_every_declared_symbol_is_exported(fftlib):
    so = ctypes.CDLL(fftlib._lib.LIB_PATH)
    for name in header_functions():
        assert hasattr(so, name), name
    assert sorted(header_functions()) == sorted(fftlib._lib.EXPORTS)


def test_status_strings(lib):
    for code in range(8):
        s = lib.fft_status_string(code).decode()
        assert s.startswith("FFT_")
    assert b"unknown" in lib.fft_status_string(99)


def _create(lib, n, batch, layout=0, direction=-1):
    h = ctypes.c_void_p()
    rc = lib.fft_plan_create(ctypes.byref(h), n, batch, layout, direction)
    return rc, h


@pytest.mark.parametrize("n", [0, -4, 3, 12, 1000, 1 << 25, (1 << 24) + 1])
def test_rejects_bad_sizes(lib, n):
    rc, h = _create(lib, n, 1)
    assert rc == 1 and h.value is None  # FFT_ERR_INVALID_SIZE


@pytest.mark.parametrize("batch,layout,direction", [(0, 0, -1), (-1, 0, -1), (1, 2, -1), (1, 0, 0), (1, 0, 2)])
def test_rejects_bad_args(lib, batch, layout, direction):
    rc, h = _create(lib, 64, batch, layout, direction)
    assert rc == 2 and h.value is None  # FFT_ERR_INVALID_ARG


def test_null_out_pointer(lib):
    assert lib.fft_plan_create(None, 64, 1, 0, -1) == 3


def test_explicit_decomposition_validation(lib):
    h = ctypes.c_void_p()
    assert lib.fft_plan_create_explicit(ctypes.byref(h), 4096, 1, 0, -1, b"garbage") == 2
    assert lib.fft_plan_create_explicit(ctypes.byref(h), 4096, 1, 0, -1, b"multi:8c4,5c4") == 7
    assert lib.fft_plan_create_explicit(ctypes.byref(h), 4096, 1, 0, -1, b"single:e5:w256:g2:r1") == 7
    assert lib.fft_plan_create_explicit(ctypes.byref(h), 4096, 1, 0, -1, b"single:e4:w256") == 2
    assert lib.fft_plan_create_explicit(ctypes.byref(h), 4096, 1, 0, -1, b"single:e4:w256:g0:r1") == 2
    assert lib.fft_plan_create_explicit(ctypes.byref(h), 4096, 1, 0, -1, b"single:e4:w256:g2:r1x") == 2
    assert lib.fft_plan_create_explicit(ctypes.byref(h), 4096, 1, 0, -1, None) == 3


@pytest.mark.parametrize("dec,status", [
    (b"multi:8c5,8c5i,8c5x", 2),    # trailing garbage after the in-place flag
    (b"multi:8c5,8c5ii,8c5", 2),    # one flag per pass
    (b"multi:8c5i,8c5,8c5", 7),     # the first pass reads the caller's input: never in place
    (b"multi:8c5,8c5,8c5i", 7),     # the last pass writes the caller's output: never in place
    (b"multi:12c2i,12c2", 7),       # a two-pass chain has no middle pass
    (b"multi:6c6,11c2i,7c7", 7),    # the last pass would read runs of 2^6 < 2^7 columns
    (b"multi:6c4,6c4i,6c4,6c4", 7), # only the penultimate pass may run in place
])
def test_in_place_pass_validation(lib, dec, status):
    """The in-place flag ("i" after a pass) parses only as one letter per pass
    and is accepted only on the penultimate pass of three or more, with the
    last pass's runs long enough for its tile; all checked before any device
    call."""
    h = ctypes.c_void_p()
    assert lib.fft_plan_create_explicit(ctypes.byref(h), 1 << 24, 1, 0, -1, dec) == status, dec
    if status == 7:
        # the same chain without the flag passes validation (it then fails, or
        # succeeds, only at the first device call): the flag is what is refused
        plain = re.sub(rb"(\d)i", rb"\1", dec)
        assert lib.fft_plan_create_explicit(ctypes.byref(h), 1 << 24, 1, 0, -1, plain) not in (2, 7), plain
        if h.value:
            lib.fft_plan_destroy(h)


def test_in_place_chains_round_trip_as_text(fftlib):
    """Every candidate, the in-place chains included, prints back as it
    parses, and the three-pass defaults carry the flag on the middle pass."""
    for log2n in (19, 21, 24):
        for layout in ("interleaved", "split"):
            q = fftlib.query_decomposition(1 << log2n, layout, "fp32")
            ip = [d for d in q["candidates"] if "i," in d]
            assert ip, (log2n, layout)
            for d in ip:
                parts = d.split(":")[1].split(",")
                assert len(parts) >= 3 and parts[-2].endswith("i") and not parts[-1].endswith("i")
            if q["default"].count(",") == 2:
                assert q["default"].split(",")[1].endswith("i"), q["default"]


def test_prefetch_decomposition_strings(lib, fftlib):
    """":p1" selects the prefetching single-pass kernel; it exists only where
    compiled (FP32 2^13, 2^14; FP64 2^12, 2^13) and ":p0" is not a spelling."""
    h = ctypes.c_void_p()
    ex = lib.fft_plan_create_ex
    assert ex(ctypes.byref(h), 4096, 1, 0, -1, 0, b"single:e4:w256:g2:r1:p0") == 2
    assert ex(ctypes.byref(h), 4096, 1, 0, -1, 0, b"single:e4:w256:g2:r1:p2") == 2
    assert ex(ctypes.byref(h), 4096, 1, 0, -1, 0, b"single:e4:w256:g2:r1:p1") == 7
    assert ex(ctypes.byref(h), 1 << 14, 1, 0, -1, 1, b"single:e4:w256:g1:r0:p1") == 7   # FP64 has no 2^14
    q32 = fftlib.query_decomposition(1 << 14, "split", "fp32")
    assert any(c.endswith(":p1") for c in q32["candidates"])
    q64 = fftlib.query_decomposition(1 << 12, "interleaved", "fp64")
    assert q64["default"] == "single:e3:w256:g1:r1:p1"


def test_half_exchange_decomposition_strings(lib, fftlib):
    """":h1" selects the single-pass kernel whose stages exchange one real part
    at a time; it exists only where compiled (FP32 2^12 .. 2^14, FP64 2^12 and
    2^13), is not combined with another variant, and is the FP32 2^14 default
    (16 points per thread interleaved, 32 split, both with the recurrence
    twiddles)."""
    h = ctypes.c_void_p()
    ex = lib.fft_plan_create_ex
    assert ex(ctypes.byref(h), 4096, 1, 0, -1, 0, b"single:e4:w256:g2:r1:h2") == 2
    assert ex(ctypes.byref(h), 4096, 1, 0, -1, 0, b"single:e4:w256:g2:r1:h1:p1") == 2
    assert ex(ctypes.byref(h), 1024, 1, 0, -1, 0, b"single:e4:w256:g2:r1:h1") == 7      # not compiled at 2^10
    assert ex(ctypes.byref(h), 1 << 11, 1, 0, -1, 1, b"single:e3:w256:g2:r0:h1") == 7   # nor FP64 2^11
    for layout in ("interleaved", "split"):
        q = fftlib.query_decomposition(1 << 14, layout, "fp32")
        want = "single:e5:w256:g4:r2:h1" if layout == "split" else "single:e4:w256:g8:r2:h1"
        assert q["default"] == want, q["default"]
        hs = [c for c in q["candidates"] if c.endswith(":h1")]
        assert hs and all(c.startswith(("single:e4:w256:", "single:e5:w256:")) for c in hs)
        # 32 points per thread (radix-32 stages) exists with half-width exchanges only
        e5 = [c for c in q["candidates"] if c.startswith("single:e5:")]
        assert e5 and all(c.endswith((":r0:h1", ":r2:h1")) for c in e5), e5


def test_recurrence_twiddle_decomposition_strings(lib, fftlib):
    """":r2" selects stage twiddles formed from one FP64 table value per
    butterfly, compiled for the largest single-pass sizes only (complex FP32
    2^13 and 2^14, FP64 2^12 and 2^13 in some shapes; real half lengths FP32
    2^13 and 2^14, FP64 2^12 and 2^13); r3 is not a spelling."""
    h = ctypes.c_void_p()
    ex = lib.fft_plan_create_ex
    assert ex(ctypes.byref(h), 1 << 14, 1, 0, -1, 0, b"single:e4:w256:g8:r3:h1") == 2
    assert ex(ctypes.byref(h), 1 << 12, 1, 0, -1, 0, b"single:e4:w256:g2:r2") == 7    # not compiled at 2^12
    assert ex(ctypes.byref(h), 1 << 13, 1, 0, -1, 1, b"single:e4:w256:g4:r2") == 7    # nor in FP64
    real = lib.fft_plan_create_real
    assert real(ctypes.byref(h), 1 << 12, 1, 0, -1, 0, b"single:e4:w256:g8:r2") == 7   # half length 2^11
    assert real(ctypes.byref(h), 1 << 15, 1, 0, -1, 0, b"single:e4:w256:g8:r2:h1") == 7  # no half-width real kernel
    assert real(ctypes.byref(h), 1 << 15, 1, 0, -1, 0, b"single:e4:w256:g8:r2:s1") == 7  # staged kernels: registers
    for log2n, want in ((14, ("single:e4:w256:g8:r2:h1", "single:e5:w256:g8:r2:h1")),
                        (13, ("single:e4:w256:g4:r2", "single:e5:w256:g4:r2:h1"))):
        for layout in ("interleaved", "split"):
            c = fftlib.query_decomposition(1 << log2n, layout, "fp32")["candidates"]
            for w in want:
                assert w in c, (log2n, layout, w)


def test_staged_decomposition_strings(lib, fftlib):
    """":s1" selects the staged small-transform kernel (FP32, N = 2 .. 512);
    ":s0" is not a spelling and a kernel cannot be staged and prefetching."""
    h = ctypes.c_void_p()
    ex = lib.fft_plan_create_ex
    for bad in (b"single:e4:w256:g2:r1:s0", b"single:e4:w256:g2:r1:s2", b"single:e4:w256:g2:r1:p1:s1",
                b"single:e4:w256:g2:r1:s1:p1", b"single:e4:w256:g2:r1:s1x"):
        assert ex(ctypes.byref(h), 16, 1, 0, -1, 0, bad) == 2, bad
    assert ex(ctypes.byref(h), 4096, 1, 0, -1, 0, b"single:e4:w256:g2:r1:s1") == 7   # not compiled there
    assert ex(ctypes.byref(h), 16, 1, 0, -1, 1, b"single:e4:w256:g2:r1:s1") == 7     # nor in FP64
    for n in (2, 16, 32, 64, 512):
        c = fftlib.query_decomposition(n, "split", "fp32")["candidates"]
        assert any(x.endswith(":s1") for x in c), n
    assert not any(x.endswith(":s1") for x in fftlib.query_decomposition(1024, "split", "fp32")["candidates"])


def test_create_ex_validation(lib):
    """Precision argument: unknown values are rejected; FP64 has its own kernel
    set (single-pass up to 2^13, 8-column pass tiles), checked before any HIP call."""
    h = ctypes.c_void_p()
    ex = lib.fft_plan_create_ex
    assert ex(ctypes.byref(h), 4096, 1, 0, -1, 2, None) == 2
    assert ex(ctypes.byref(h), 4096, 1, 0, -1, -1, b"single:e4:w256:g2:r1") == 2
    assert ex(ctypes.byref(h), 100, 1, 0, -1, 1, None) == 1
    assert ex(ctypes.byref(h), 1 << 14, 1, 0, -1, 1, b"single:e4:w256:g8:r0") == 7   # FP64 LDS limit
    assert ex(ctypes.byref(h), 1 << 13, 1, 0, -1, 1, b"single:e3:w256:g1:r1") == 7   # spills: not compiled
    assert ex(ctypes.byref(h), 1 << 24, 1, 0, -1, 1, b"multi:12c2,12c2") == 7        # FP64 tile too wide
    assert ex(ctypes.byref(h), 1 << 24, 1, 0, -1, 0, b"multi:12c2,12c2x") == 2
    assert ex(None, 64, 1, 0, -1, 1, None) == 3


def test_create_real_validation(lib):
    """Real-input plans: size, enum and decomposition checks before any HIP call."""
    h = ctypes.c_void_p()
    cr = lib.fft_plan_create_real
    assert cr(ctypes.byref(h), 100, 1, 0, -1, 0, None) == 1
    assert cr(ctypes.byref(h), 1 << 25, 1, 0, -1, 0, None) == 1
    assert cr(ctypes.byref(h), 64, 0, 0, -1, 0, None) == 2
    assert cr(ctypes.byref(h), 64, 1, 3, -1, 0, None) == 2
    assert cr(ctypes.byref(h), 64, 1, 0, 0, 0, None) == 2
    assert cr(ctypes.byref(h), 64, 1, 0, -1, 5, None) == 2
    assert cr(ctypes.byref(h), 64, 1, 0, -1, 0, b"nonsense") == 2
    assert cr(ctypes.byref(h), 64, 1, 0, -1, 0, b"multi:3c1,2c1") == 7   # sums to log2 n, not log2 n/2
    assert cr(ctypes.byref(h), 64, 1, 0, -1, 0, b"copy") == 7            # copy is n = 2 only
    assert cr(ctypes.byref(h), 1, 1, 0, -1, 0, b"copy") == 7             # n = 1 takes none
    assert cr(ctypes.byref(h), 1 << 16, 1, 1, 1, 1, b"single:e4:w256:g2:r1") == 7   # FP64 half 2^15
    assert cr(None, 64, 1, 0, -1, 0, None) == 3


@pytest.mark.parametrize("precision", [0, 1])
def test_real_defaults_pass_validation(lib, precision):
    """Every real-input size's default decomposition (fused kernel up to half
    length 2^14 FP32 / 2^13 FP64, among them the recurrence-twiddle shapes,
    else the half-length chain) names compiled kernels in both layouts and
    directions: plan creation gets past every check made before the first HIP
    call (here, without a GPU, it then fails at that call)."""
    h = ctypes.c_void_p()
    for log2n in range(1, 25):
        for layout in (0, 1):
            for direction in (-1, 1):
                rc = lib.fft_plan_create_real(ctypes.byref(h), 1 << log2n, 2, layout, direction, precision, None)
                assert rc not in (1, 2, 7), (log2n, layout, direction, precision, rc)
                if rc == 0:
                    lib.fft_plan_destroy(h)
    explicit = [(14, 1, -1, 0, b"single:e4:w256:g8:r2"), (15, 1, -1, 0, b"single:e4:w256:g1:r2"),
                (14, 1, -1, 0, b"single:e3:w256:g8:r2"), (13, 0, 1, 1, b"single:e4:w256:g8:r2"),
                (14, 0, 1, 1, b"single:e4:w256:g1:r2"), (14, 0, 1, 1, b"single:e3:w256:g1:r2")]
    for log2n, layout, direction, prec, dec in explicit:
        rc = lib.fft_plan_create_real(ctypes.byref(h), 1 << log2n, 2, layout, direction, prec, dec)
        assert rc not in (1, 2, 7), (dec, rc)
        if rc == 0:
            lib.fft_plan_destroy(h)


def test_create_nd_validation(lib):
    """Multi-dimensional plans: rank, dims and limits checked before any HIP call."""
    h = ctypes.c_void_p()
    nd = lib.fft_plan_create_nd

    def dims(*d):
        return (ctypes.c_int64 * len(d))(*d)
    assert nd(ctypes.byref(h), 2, None, 1, 0, -1, 0) == 3
    assert nd(ctypes.byref(h), 0, dims(4), 1, 0, -1, 0) == 2
    assert nd(ctypes.byref(h), 4, dims(4, 4, 4, 4), 1, 0, -1, 0) == 2
    assert nd(ctypes.byref(h), 2, dims(4, 6), 1, 0, -1, 0) == 1
    assert nd(ctypes.byref(h), 2, dims(8192, 4), 1, 0, -1, 0) == 1     # strided axis above 2^12
    assert nd(ctypes.byref(h), 2, dims(4, 1 << 25), 1, 0, -1, 0) == 1  # last axis above 2^24
    assert nd(ctypes.byref(h), 3, dims(4, 4, 4), 0, 0, -1, 0) == 2
    assert nd(ctypes.byref(h), 3, dims(4, 4, 4), 1, 0, -1, 9) == 2
    assert nd(ctypes.byref(h), 3, dims(4096, 4096, 4096), 1 << 10, 0, -1, 0) == 2  # element bound
    assert nd(None, 2, dims(4, 4), 1, 0, -1, 0) == 3


def test_ragged_validation(lib):
    h = ctypes.c_void_p()
    arr = (ctypes.c_int64 * 3)(64, 100, 256)
    assert lib.fft_plan_create_ragged(ctypes.byref(h), arr, 3, 0, -1) == 1
    arr = (ctypes.c_int64 * 2)(64, 256)
    assert lib.fft_plan_create_ragged(ctypes.byref(h), arr, 0, 0, -1) == 2
    assert lib.fft_plan_create_ragged(ctypes.byref(h), None, 2, 0, -1) == 3
    assert lib.fft_plan_create_ragged(ctypes.byref(h), arr, 2, 7, -1) == 2
    # explicit configurations that do not parse are rejected before any device call
    for bad in (b"bogus", b"ragged:p9:g8:o0", b"ragged:p5:g8:o0", b"ragged:p8:g0:o0", b"ragged:p8:g8:o2",
                b"ragged:p8:g8:o0:w4", b"ragged:p8:g8:o0:w", b"ragged:p8:g8:o0:w64x", b"ragged:p8:g8",
                b"ragged:p8:g8:o0:s12", b"ragged:p8:g8:o0:s15", b"ragged:p8:g8:o0:s", b"ragged:p8:g8:o0:s13:w8",
                b"ragged:p8:g8:o0:w8:s13x", b"ragged:p8:g8:o0:w8:s13:s14"):
        assert lib.fft_plan_create_ragged_ex(ctypes.byref(h), arr, 2, 0, -1, bad) == 2, bad


def test_execute_rejects_null_plan(lib):
    assert lib.fft_execute(None, 16, 16, 32, 32, None) == 2
    assert lib.fft_execute_backward(None, 16, 16, 32, 32, None) == 2
    assert lib.fft_plan_destroy(None) == 0
    n = ctypes.c_size_t()
    assert lib.fft_plan_workspace_bytes(None, ctypes.byref(n)) == 2
    assert lib.fft_plan_set_workspace(None, None) == 2


def test_copy_validation(lib):
    assert lib.fft_copy_device(None, 16, 16, None) == 3
    assert lib.fft_copy_device(16, 64, 17, None) == 4   # size not a multiple of 16
    assert lib.fft_copy_device(8, 64, 16, None) == 4    # misaligned source
    assert lib.fft_copy_device(16, 32, 64, None) == 2   # overlap


@pytest.mark.parametrize("precision,single_max", [("fp32", 14), ("fp64", 13)])
@pytest.mark.parametrize("log2n", range(0, 25))
def test_default_decomposition_covers_every_size(fftlib, log2n, precision, single_max):
    for layout in ("interleaved", "split"):
        q = fftlib.query_decomposition(1 << log2n, layout, precision)
        assert q["available"], q
        assert q["precision"] == precision
        assert q["default"] in q["candidates"]
        if log2n == 0:
            assert q["default"] == "copy"
        elif log2n <= single_max:
            assert q["default"].startswith("single:")
        else:
            parts = q["default"].split(":")[1].split(",")
            assert sum(int(p.split("c")[0]) for p in parts) == log2n


def test_query_rejects_bad_args(lib):
    buf = ctypes.create_string_buffer(256)
    assert lib.fft_query_decomposition(12, 0, 0, buf, 256) == 1
    assert lib.fft_query_decomposition(16, 9, 0, buf, 256) == 2
    assert lib.fft_query_decomposition(16, 0, 7, buf, 256) == 2


def test_query_truncates(lib):
    buf = ctypes.create_string_buffer(8)
    assert lib.fft_query_decomposition(1 << 24, 0, 0, buf, 8) == 0
    assert len(buf.value) == 7


def test_no_kernel_spills_or_uses_scratch():
    """Every kernel of the last build keeps its state in registers: no VGPR or
    SGPR spills and no per-lane scratch (the compiler's resource report, kept
    by the build next to the library)."""
    path = os.path.join(ROOT, "_build", "kernel_resources.json")
    if not os.path.exists(path):
        pytest.skip("no resource report: the library was built without one")
    import json
    report = json.load(open(path))
    assert report["arch"] == "gfx950"
    kernels = report["kernels"]
    assert len(kernels) > 100
    bad = [k["name"] for k in kernels
           if k.get("VGPRs Spill", 0) or k.get("SGPRs Spill", 0) or k.get("ScratchSize [bytes/lane]", 0)]
    assert not bad, f"{len(bad)} kernels spill or use scratch, e.g. {bad[:3]}"
    assert all(k.get("VGPRs", 0) <= 512 for k in kernels)
