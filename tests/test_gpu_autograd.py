"""GPU parity of the differentiable FFT: torch.autograd through the adjoint
kernel, against the FP64 oracle gradient and FP64 finite differences."""
import numpy as np
import pytest

import oracle
import workloads
from fftcheck import TOL

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def fftlib():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2308_00497_amd as m
    return m


def c5_grad(fftlib, batch=1024, n=4096):
    re, im, w = workloads.c5(batch=batch, n=n)
    xre = torch.from_numpy(re).cuda().requires_grad_(True)
    xim = torch.from_numpy(im).cuda().requires_grad_(True)
    wt = torch.from_numpy(w).cuda()
    yre, yim = fftlib.FFTFunction.apply(xre, xim)  # transforms along the last axis (N)
    loss = (wt * (yre * yre + yim * yim)).sum()
    loss.backward()
    torch.cuda.synchronize()
    g = xre.grad.cpu().numpy().astype(np.float64) + 1j * xim.grad.cpu().numpy().astype(np.float64)
    return re, im, w, g.reshape(batch, n), loss.item()


def test_c5_gradient_against_oracle(fftlib):
    """batch 1024 x N=4096 split, loss = sum(w |FFT(x)|^2): every transform's
    gradient against the oracle's analytic gradient 2 F^H (w F x), element by
    element, per transform."""
    re, im, w, g, _ = c5_grad(fftlib)
    errs = np.empty(re.shape[0])
    for r in range(re.shape[0]):
        x = re[r].astype(np.float64) + 1j * im[r].astype(np.float64)
        ref = oracle.wpower_grad(x, w[r].astype(np.float64))
        errs[r] = oracle.rel_l2(g[r], ref)
    print(f"[parity] C5 gradient, all {len(errs)} transforms: max per-transform rel-L2 {errs.max():.3e}")
    assert errs.max() <= TOL


def test_c5_gradient_against_finite_differences(fftlib):
    """FP64 central differences of the oracle loss on 256 seeded coordinates
    (Re and Im) of transform 0; the loss is quadratic, so the difference quotient
    is exact up to rounding."""
    re, im, w, g, _ = c5_grad(fftlib, batch=4)
    x = re[0].astype(np.float64) + 1j * im[0].astype(np.float64)
    wt = w[0].astype(np.float64)
    n = x.shape[0]
    rng = np.random.default_rng(56)
    coords = rng.choice(n, size=128, replace=False)
    h = 1e-3
    scale = np.abs(g[0]).max()
    worst = 0.0
    for idx in coords:
        for part in (1.0, 1j):
            e = np.zeros(n, dtype=complex)
            e[idx] = part * h
            fd = (oracle.wpower_loss(x + e, wt) - oracle.wpower_loss(x - e, wt)) / (2 * h)
            gpu = g[0, idx].real if part == 1.0 else g[0, idx].imag
            worst = max(worst, abs(fd - gpu) / scale)
    print(f"[parity] C5 gradient vs FP64 finite differences: max |diff| / max|g| = {worst:.3e}")
    assert worst <= 1e-5


def test_autograd_equals_direct_kernels(fftlib):
    """Forward + backward through autograd equal the two kernels called directly."""
    batch, n = 64, 4096
    re, im, w = workloads.c5(batch=batch, n=n)
    xre, xim = torch.from_numpy(re).cuda(), torch.from_numpy(im).cuda()
    wt = torch.from_numpy(w).cuda()
    a = xre.clone().requires_grad_(True)
    b = xim.clone().requires_grad_(True)
    yre, yim = fftlib.FFTFunction.apply(a, b)
    (wt * (yre * yre + yim * yim)).sum().backward()
    with fftlib.Plan(n, batch, "split", "forward") as p:
        dre, dim = p.execute((xre, xim))
        gre, gim = p.backward((2 * wt * dre, 2 * wt * dim))
    torch.cuda.synchronize()
    assert torch.equal(yre, dre) and torch.equal(yim, dim)
    assert torch.allclose(a.grad, gre, rtol=0, atol=0) and torch.allclose(b.grad, gim, rtol=0, atol=0)


def test_complex_autograd(fftlib):
    """complex64 input: z.grad = dL/dRe z + i dL/dIm z = F^H(2 w y)."""
    batch, n = 8, 1024
    re, im, w = workloads.c5(batch=batch, n=n)
    z = torch.from_numpy(workloads.interleave(re, im)).cuda().requires_grad_(True)
    wt = torch.from_numpy(w).cuda()
    y = fftlib.fft_autograd(z)
    (wt * y.abs() ** 2).sum().backward()
    torch.cuda.synchronize()
    g = z.grad.cpu().numpy().astype(np.complex128)
    for r in range(batch):
        x = re[r].astype(np.float64) + 1j * im[r].astype(np.float64)
        assert oracle.rel_l2(g[r], oracle.wpower_grad(x, w[r].astype(np.float64))) <= TOL
