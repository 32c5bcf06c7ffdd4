"""GPU parity of the FP64 path (the precision of the paper's evaluation,
section 4): the same kernels over double2 elements, against the FP64 oracle
with a per-transform relative L2 bound of 1e-13."""
import numpy as np
import pytest

import oracle
import workloads
from fftcheck import SIGN, TOL64, assert_parity, from_device, multi_candidates, oracle_ref, to_device, widen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

F64 = np.float64


@pytest.fixture(scope="module")
def fftlib():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2308_00497_amd as m
    return m


def sweep_batch(n: int) -> int:
    return max(1, min(37, (1 << 20) // n))


@pytest.mark.parametrize("direction", ["forward", "inverse"])
@pytest.mark.parametrize("layout", ["interleaved", "split"])
@pytest.mark.parametrize("log2n", range(0, 25))
def test_sweep_fp64(fftlib, log2n, layout, direction):
    n = 1 << log2n
    batch = sweep_batch(n)
    re, im = workloads.normal_complex((batch, n), seed=7000 + log2n, dtype=F64)
    with fftlib.Plan(n, batch, layout, direction, precision="fp64") as plan:
        y = from_device(plan.execute(to_device(re, im, layout)), layout)
        desc = plan.describe()
    assert desc["precision"] == "fp64"
    assert_parity(y, oracle_ref(re, im, direction), f"FP64 N=2^{log2n} b={batch} {layout} {direction} "
                  f"{desc['decomposition']}", tol=TOL64)


def candidates(fftlib, log2n, layout):
    return fftlib.query_decomposition(1 << log2n, layout, "fp64")["candidates"]


@pytest.mark.parametrize("layout", ["interleaved", "split"])
@pytest.mark.parametrize("log2n", range(1, 14))
def test_every_single_pass_variant_fp64(fftlib, log2n, layout):
    n = 1 << log2n
    batch = max(3, min(41, (1 << 17) // n))
    re, im = workloads.uniform_complex((batch, n), seed=7100 + log2n, dtype=F64)
    ref = oracle_ref(re, im, "forward")
    seen = 0
    for dec in candidates(fftlib, log2n, layout):
        if not dec.startswith("single"):
            continue
        with fftlib.Plan(n, batch, layout, "forward", decomposition=dec, precision="fp64") as plan:
            y = from_device(plan.execute(to_device(re, im, layout)), layout)
        assert_parity(y, ref, f"FP64 N=2^{log2n} {layout} {dec}", tol=TOL64)
        seen += 1
    assert seen > 0


@pytest.mark.parametrize("layout", ["interleaved", "split"])
@pytest.mark.parametrize("log2n", [12, 13, 14, 15, 16, 17, 18, 20, 24])
def test_every_multi_pass_variant_fp64(fftlib, log2n, layout):
    n = 1 << log2n
    batch = max(1, min(3, (1 << 20) // n))
    direction = "inverse" if log2n % 2 else "forward"
    re, im = workloads.uniform_complex((batch, n), seed=7200 + log2n, dtype=F64)
    ref = oracle_ref(re, im, direction)
    seen = 0
    q = fftlib.query_decomposition(n, layout, "fp64")
    # 2^24: a spread of the ~400 chains (every pass kernel runs at the smaller sizes)
    for dec in multi_candidates(q["candidates"], q["default"], 48 if log2n >= 24 else 10**6):
        with fftlib.Plan(n, batch, layout, direction, decomposition=dec, precision="fp64") as plan:
            y = from_device(plan.execute(to_device(re, im, layout)), layout)
        assert_parity(y, ref, f"FP64 N=2^{log2n} {layout} {direction} {dec}", tol=TOL64)
        seen += 1
    assert seen > 0


@pytest.mark.parametrize("layout", ["interleaved", "split"])
@pytest.mark.parametrize("log2n", [0, 5, 12, 13, 14, 18, 22])
def test_in_place_and_backward_fp64(fftlib, log2n, layout):
    n = 1 << log2n
    batch = max(1, min(7, (1 << 20) // n))
    re, im = workloads.normal_complex((batch, n), seed=7300 + log2n, dtype=F64)
    x = to_device(re, im, layout)
    with fftlib.Plan(n, batch, layout, "forward", precision="fp64") as plan:
        g = from_device(plan.backward(x), layout)
        y = plan.execute(x, out=x)
    assert_parity(g, oracle_ref(re, im, "inverse"), f"FP64 backward N=2^{log2n} {layout}", tol=TOL64)
    assert_parity(from_device(y, layout), oracle_ref(re, im, "forward"), f"FP64 in-place N=2^{log2n} {layout}",
                  tol=TOL64)


def test_round_trip_fp64(fftlib):
    """ifft(fft(x)) = N x to FP64 rounding."""
    for log2n in (10, 16, 21):
        n = 1 << log2n
        re, im = workloads.normal_complex((2, n), seed=7400 + log2n, dtype=F64)
        z = torch.from_numpy(workloads.interleave(re, im)).cuda()
        back = fftlib.ifft(fftlib.fft(z)).cpu().numpy() / n
        err = oracle.rel_l2(back.reshape(-1), widen(re, im).reshape(-1))
        print(f"[parity] FP64 round trip N=2^{log2n}: rel-L2 {err:.3e}")
        assert err <= TOL64


def test_c2_shape_fp64_sampled(fftlib):
    """The batched N=4096 x 8192 workload in FP64 (1 GiB of input), 64 sampled
    transforms against the oracle, both layouts."""
    batch, n = 8192, 4096
    re, im = workloads.normal_complex((batch, n), seed=workloads.SEEDS["c2"], dtype=F64)
    rows = np.sort(np.random.default_rng(77).choice(batch, size=64, replace=False))
    ref = oracle.fft(widen(re[rows], im[rows]), SIGN["forward"], threads=8)
    for layout in ("interleaved", "split"):
        with fftlib.Plan(n, batch, layout, "forward", precision="fp64") as plan:
            yd = plan.execute(to_device(re, im, layout))
            torch.cuda.synchronize()
            if layout == "split":
                y = yd[0][rows].cpu().numpy() + 1j * yd[1][rows].cpu().numpy()
            else:
                y = yd[rows].cpu().numpy()
            del yd
        assert_parity(y, ref, f"FP64 C2 shape {layout} (64 sampled rows)", tol=TOL64)


def test_c3_shape_fp64(fftlib):
    """N = 2^24 split in FP64: full transform against the oracle, and the
    eight cosine spikes at their frequencies."""
    n = 1 << 24
    _, _, nr, ni, freqs = workloads.c3(n)
    tones = np.zeros(n)
    j = np.arange(n, dtype=np.int64)
    for f in freqs:
        tones += np.cos(2.0 * np.pi * ((int(f) * j) % n) / n)
    re = (nr + tones).astype(F64)
    im = ni.astype(F64)
    with fftlib.Plan(n, 1, "split", "forward", precision="fp64") as plan:
        y = from_device(plan.execute(to_device(re, im, "split")), "split").reshape(1, n)
    ref = oracle_ref(re.reshape(1, n), im.reshape(1, n), "forward")
    assert_parity(y, ref, "FP64 C3 N=2^24", tol=TOL64)
    mag = np.abs(y[0])
    for f in freqs:
        assert mag[f] > n / 2 - 8 * np.sqrt(n)


def test_fp64_autograd_gradient(fftlib):
    """complex128 autograd: z.grad = F^H(2 w y) against the oracle gradient."""
    batch, n = 16, 4096
    rng = np.random.default_rng(7500)
    re = rng.standard_normal((batch, n))
    im = rng.standard_normal((batch, n))
    w = rng.uniform(0.0, 1.0, (batch, n))
    z = torch.from_numpy(workloads.interleave(re, im)).cuda().requires_grad_(True)
    wt = torch.from_numpy(w).cuda()
    y = fftlib.fft_autograd(z)
    (wt * y.abs() ** 2).sum().backward()
    torch.cuda.synchronize()
    g = z.grad.cpu().numpy()
    worst = 0.0
    for r in range(batch):
        worst = max(worst, oracle.rel_l2(g[r], oracle.wpower_grad(re[r] + 1j * im[r], w[r])))
    print(f"[parity] FP64 autograd gradient: max rel-L2 {worst:.3e}")
    assert worst <= TOL64


def test_dtype_checks(fftlib):
    with fftlib.Plan(64, 2, "interleaved", "forward", precision="fp64") as plan:
        with pytest.raises(TypeError):
            plan.execute(torch.zeros(128, dtype=torch.complex64, device="cuda"))
    with fftlib.Plan(64, 2, "split", "forward", precision="fp32") as plan:
        with pytest.raises(TypeError):
            plan.execute((torch.zeros(128, dtype=torch.float64, device="cuda"),
                          torch.zeros(128, dtype=torch.float64, device="cuda")))
    with pytest.raises(ValueError):
        fftlib.Plan(64, 2, precision="fp16")
