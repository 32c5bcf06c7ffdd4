"""fft_execute_no_alloc: fft_execute on the library's static scratch buffer.

Called through the C ABI (ctypes) and compared with fft_execute of the same
plan on the same inputs (bitwise: the same kernels run on the same data, only
the workspace address differs) and with the FP64 oracle (relative L2 <= 1e-5
per transform).  Two calls in a row share the one scratch array of the GPU,
the second on a smaller input, so stale contents of the first call would show.
"""
import ctypes

import numpy as np
import pytest

import workloads
from fftcheck import TOL, TOL64, assert_parity, from_device, oracle_ref, to_device

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

FFT_OK, FFT_ERR_INVALID_SIZE, FFT_ERR_NOT_SUPPORTED = 0, 1, 7


@pytest.fixture(scope="module")
def fftlib():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2308_00497_amd as m
    return m


def _ptrs(x, layout):
    if layout == "split":
        return x[0].data_ptr(), x[1].data_ptr()
    return x.data_ptr(), None


def _run(fftlib, plan, x, layout, no_alloc):
    lib = fftlib._lib.lib
    out = (torch.empty_like(x[0]), torch.empty_like(x[1])) if layout == "split" else torch.empty_like(x)
    ia, ib = _ptrs(x, layout)
    oa, ob = _ptrs(out, layout)
    stream = torch.cuda.current_stream().cuda_stream
    fn = lib.fft_execute_no_alloc if no_alloc else lib.fft_execute
    rc = fn(plan._handle, ia, ib, oa, ob, stream)
    assert rc == FFT_OK, (rc, lib.fft_last_error_detail())
    return out


def _same(a, b, layout):
    if layout == "split":
        return bool(torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]))
    return bool(torch.equal(a, b))


# (n, batch, layout, precision, decomposition): multi-pass plans whose
# workspace fits the scratch buffer, the larger first
CASES = [
    [(1 << 20, 2, "split", "fp32", "multi:7c7,7c6,6c6"), (1 << 16, 4, "split", "fp32", None)],
    [(1 << 21, 2, "interleaved", "fp32", "multi:7c6,7c6i,7c6"), (1 << 15, 3, "interleaved", "fp32", None)],
    [(1 << 19, 3, "interleaved", "fp64", None), (1 << 12, 5, "interleaved", "fp64", None)],
]


@pytest.mark.parametrize("pair", CASES, ids=lambda c: f"{c[0][0]}x{c[0][1]}-{c[0][2]}-{c[0][3]}")
def test_no_alloc_matches_execute(fftlib, pair):
    cap = fftlib._lib.lib.fft_no_alloc_scratch_bytes()
    assert cap == 64 << 20
    for call, (n, batch, layout, prec, dec) in enumerate(pair):
        print(f"[no_alloc] call {call}: n={n} batch={batch} {layout} {prec} {dec}", flush=True)
        dt = np.float32 if prec == "fp32" else np.float64
        re, im = workloads.normal_complex((batch, n), seed=7100 + call + n % 97, dtype=dt)
        x = to_device(re, im, layout)
        with fftlib.Plan(n, batch, layout, "forward", decomposition=dec, precision=prec) as plan:
            assert 0 < plan.workspace_bytes <= cap or n <= 1 << 14
            y0 = _run(fftlib, plan, x, layout, no_alloc=False)
            y1 = _run(fftlib, plan, x, layout, no_alloc=True)
            torch.cuda.synchronize()
            assert _same(y0, y1, layout), f"call {call}: no-alloc output differs from fft_execute"
            ref = oracle_ref(re, im, "forward")
            assert_parity(from_device(y1, layout), ref, f"no_alloc call {call} n={n} b={batch} {layout} {prec}",
                          tol=TOL if prec == "fp32" else TOL64)


def test_no_alloc_rejects_oversize_and_ragged(fftlib):
    lib = fftlib._lib.lib
    n, batch = 1 << 22, 4            # workspace 2 x 128 MiB > 64 MiB
    x = torch.zeros(n * batch, dtype=torch.complex64, device="cuda")
    y = torch.empty_like(x)
    with fftlib.Plan(n, batch, "interleaved", "forward", decomposition="multi:8c4,8c5,6c6") as plan:
        assert plan.workspace_bytes > lib.fft_no_alloc_scratch_bytes()
        rc = lib.fft_execute_no_alloc(plan._handle, x.data_ptr(), None, y.data_ptr(), None,
                                      torch.cuda.current_stream().cuda_stream)
        assert rc == FFT_ERR_INVALID_SIZE
        assert b"scratch" in lib.fft_last_error_detail()
    sizes = [64, 128, 1 << 15]
    xr = torch.zeros(sum(sizes), dtype=torch.complex64, device="cuda")
    yr = torch.empty_like(xr)
    with fftlib.RaggedPlan(sizes, "interleaved", "forward") as rp:
        rc = lib.fft_execute_no_alloc(rp._handle, xr.data_ptr(), None, yr.data_ptr(), None,
                                      torch.cuda.current_stream().cuda_stream)
        assert rc == FFT_ERR_NOT_SUPPORTED
    torch.cuda.synchronize()
