"""Plans replayed from a captured graph.

`fft_execute` allocates nothing and waits for nothing (tables and workspace
belong to the plan), so a caller may capture it on a stream and replay it.
Each case captures one execute with torch's graph API, then replays it three
times on fresh inputs copied into the captured buffers, with eager work and
synchronisations between the replays, and checks every replay against the
FP64 oracle.  Multi-pass plans reuse the plan's workspace on every replay.
Complex, real (R2C and C2R captured together) and multi-dimensional plans.
"""
import numpy as np
import pytest

import oracle
import workloads
from fftcheck import SIGN, TOL, TOL64, assert_parity, from_device, oracle_ref, to_device

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def fftlib():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2308_00497_amd as m
    return m


CASES = [
    # log2 N, batch, layout, direction, precision
    (5, 301, "interleaved", "forward", "fp32"),     # several transforms per workgroup, ragged tail
    (12, 64, "interleaved", "inverse", "fp32"),
    (12, 64, "split", "forward", "fp32"),
    (16, 3, "split", "inverse", "fp32"),            # two passes through the plan's workspace
    (20, 1, "interleaved", "forward", "fp32"),      # three passes
    (12, 16, "interleaved", "forward", "fp64"),
    (14, 8, "interleaved", "forward", "fp32"),      # recurrence twiddles, half-width exchanges
    (14, 8, "split", "inverse", "fp32"),            # the same with 32 points per thread
    (13, 8, "split", "inverse", "fp64"),            # FP64 recurrence twiddles
]


def _load(dst, re, im, layout):
    src = to_device(re, im, layout)
    if layout == "split":
        dst[0].copy_(src[0])
        dst[1].copy_(src[1])
    else:
        dst.copy_(src)


@pytest.mark.parametrize("log2n,batch,layout,direction,precision", CASES)
def test_plan_replayed_from_graph(fftlib, log2n, batch, layout, direction, precision):
    n = 1 << log2n
    dtype = "float64" if precision == "fp64" else "float32"
    tol = TOL64 if precision == "fp64" else TOL
    what = f"graph N=2^{log2n} b={batch} {layout} {direction} {precision}"
    print(f"[case] {what}", flush=True)
    re, im = workloads.normal_complex((batch, n), seed=7000 + log2n, dtype=dtype)
    with fftlib.Plan(n, batch, layout, direction, precision=precision) as plan:
        x = to_device(re, im, layout)
        y = plan.execute(x)          # eager run: allocates the output the graph will write
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            plan.execute(x, out=y)
        for rep in range(3):
            re, im = workloads.normal_complex((batch, n), seed=7100 + 10 * log2n + rep, dtype=dtype)
            _load(x, re, im, layout)
            torch.cuda.synchronize()
            g.replay()
            got = from_device(y, layout)
            assert_parity(got, oracle_ref(re, im, direction), f"{what} replay {rep}", tol=tol)
        del g


REAL_CASES = [
    # log2 N, batch, layout, precision
    (15, 4, "split", "fp32"),          # fused kernel, recurrence twiddles
    (12, 16, "interleaved", "fp32"),   # fused kernel, register twiddles
    (14, 4, "interleaved", "fp64"),    # FP64 fused kernel, recurrence twiddles
    (18, 2, "split", "fp32"),          # half-length pass chain through the plan's workspace
]


@pytest.mark.parametrize("log2n,batch,layout,precision", REAL_CASES)
def test_real_plans_replayed_from_graph(fftlib, log2n, batch, layout, precision):
    """R2C and C2R plans captured once and replayed on fresh inputs."""
    n, h = 1 << log2n, (1 << (log2n - 1)) + 1
    dt = np.float64 if precision == "fp64" else np.float32
    tol = TOL64 if precision == "fp64" else TOL
    what = f"real graph N=2^{log2n} b={batch} {layout} {precision}"
    print(f"[case] {what}", flush=True)
    rng = np.random.default_rng(7300 + log2n)
    with fftlib.RealPlan(n, batch, layout, "forward", precision) as pf, \
            fftlib.RealPlan(n, batch, layout, "inverse", precision) as pi:
        x = torch.from_numpy(rng.standard_normal((batch, n)).astype(dt)).cuda()
        re, im = workloads.normal_complex((batch, h), seed=7350 + log2n, dtype=dt)
        z = to_device(re, im, layout)
        y = pf.execute(x)
        r = pi.execute(z)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            pf.execute(x, out=y)
            pi.execute(z, out=r)
        for rep in range(3):
            xs = rng.standard_normal((batch, n)).astype(dt)
            re, im = workloads.normal_complex((batch, h), seed=7400 + 10 * log2n + rep, dtype=dt)
            x.copy_(torch.from_numpy(xs).cuda())
            _load(z, re, im, layout)
            torch.cuda.synchronize()
            g.replay()
            assert_parity(from_device(y, layout), oracle.rfft(xs, threads=8), f"{what} R2C replay {rep}", tol)
            ref_i = oracle.irfft(re.astype(np.float64) + 1j * im.astype(np.float64), n, threads=8)
            torch.cuda.synchronize()
            assert_parity(r.cpu().numpy().astype(np.float64), ref_i, f"{what} C2R replay {rep}", tol)
        del g


ND_CASES = [
    # shape, batch, layout
    ((64, 4096), 2, "split"),          # one strided column pass over the row plan's output
    ((4096, 128), 2, "interleaved"),   # long columns as two passes through the plan's workspace
    ((32, 16, 64), 2, "interleaved"),  # rank 3
]


@pytest.mark.parametrize("shape,batch,layout", ND_CASES)
def test_nd_plans_replayed_from_graph(fftlib, shape, batch, layout):
    what = f"nd graph {shape} b={batch} {layout}"
    print(f"[case] {what}", flush=True)
    re, im = workloads.normal_complex((batch,) + shape, seed=7500 + sum(shape))
    with fftlib.PlanND(shape, batch, layout, "forward") as p:
        x = to_device(re, im, layout)
        y = p.execute(x)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            p.execute(x, out=y)
        for rep in range(3):
            re, im = workloads.normal_complex((batch,) + shape, seed=7600 + sum(shape) + rep)
            _load(x, re, im, layout)
            torch.cuda.synchronize()
            g.replay()
            got = from_device(y, layout).reshape(batch, -1)
            ref = oracle.fftn(re.astype(np.float64) + 1j * im.astype(np.float64), len(shape), SIGN["forward"],
                              threads=8)
            assert_parity(got, ref.reshape(batch, -1), f"{what} replay {rep}", TOL)
        del g
