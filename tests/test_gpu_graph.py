"""Plans replayed from a captured graph.

`fft_execute` allocates nothing and waits for nothing (tables and workspace
belong to the plan), so a caller may capture it on a stream and replay it.
Each case captures one execute with torch's graph API, then replays it three
times on fresh inputs copied into the captured buffers, with eager work and
synchronisations between the replays, and checks every replay against the
FP64 oracle.  Multi-pass plans reuse the plan's workspace on every replay.
"""
import pytest

import workloads
from fftcheck import TOL, TOL64, assert_parity, from_device, oracle_ref, to_device

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
