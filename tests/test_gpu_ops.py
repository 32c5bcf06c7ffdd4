"""GPU parity of the per-operator baseline ("ops:r<log2 R>"): Table 1's
operators (Permute, FusedIKMV, Mul, FusedMKIV) as one kernel each, composed
by Eq. 1 with radix R, against the FP64 oracle."""
import numpy as np
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


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("log2r", [1, 2, 3, 4])
@pytest.mark.parametrize("log2n", [1, 2, 3, 5, 8, 11, 12, 13, 16, 20])
def test_ops_baseline(fftlib, log2n, log2r, precision):
    n = 1 << log2n
    batch = max(1, min(9, (1 << 18) // n))
    dt = np.float64 if precision == "fp64" else np.float32
    tol = TOL64 if precision == "fp64" else TOL
    re, im = workloads.normal_complex((batch, n), seed=9000 + log2n, dtype=dt)
    for direction in ("forward", "inverse"):
        with fftlib.Plan(n, batch, "interleaved", direction, decomposition=f"ops:r{log2r}",
                         precision=precision) as p:
            y = from_device(p.execute(to_device(re, im, "interleaved")), "interleaved")
        assert_parity(y, oracle_ref(re, im, direction), f"ops:r{log2r} {precision} N=2^{log2n} {direction}", tol)


def test_ops_in_place_and_split_rejected(fftlib):
    n, batch = 4096, 3
    re, im = workloads.normal_complex((batch, n), seed=9100)
    x = to_device(re, im, "interleaved")
    with fftlib.Plan(n, batch, "interleaved", "forward", decomposition="ops:r4") as p:
        y = p.execute(x, out=x)
    assert_parity(from_device(y, "interleaved"), oracle_ref(re, im, "forward"), "ops:r4 in place")
    with pytest.raises(fftlib.FFTError):
        fftlib.Plan(n, batch, "split", "forward", decomposition="ops:r4")
