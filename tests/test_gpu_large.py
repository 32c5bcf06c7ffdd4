"""Transforms whose element count passes 2^31 (64-bit indexing everywhere):
batched single-pass and multi-pass plans over more than 16 GiB of input,
checked on sampled rows, including the last ones, against the oracle.
Inputs are drawn on the device by torch's seeded generator (never by the
library), and the sampled rows are copied back for the oracle."""
import numpy as np
import pytest

import oracle
from fftcheck import SIGN, TOL, assert_parity

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def fftlib():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2308_00497_amd as m
    return m


def seeded_complex(count, seed):
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    return torch.randn(count, dtype=torch.complex64, device="cuda", generator=g)


@pytest.mark.parametrize("n,batch,layout", [(4096, (1 << 19) + 3, "interleaved"), (4096, (1 << 19) + 3, "split"),
                                            (1 << 20, (1 << 11) + 1, "interleaved")])
def test_more_than_2_31_elements(fftlib, n, batch, layout):
    total = n * batch
    assert total > (1 << 31)
    z = seeded_complex(total, 9700 + n % 97)
    rows = sorted({0, 1, batch // 2, batch - 3, batch - 2, batch - 1})
    x_rows = torch.stack([z[r * n:(r + 1) * n] for r in rows]).cpu().numpy().astype(np.complex128)
    with fftlib.Plan(n, batch, layout, "forward") as p:
        if layout == "split":
            re = z.real.contiguous()
            im = z.imag.contiguous()
            del z
            yre, yim = p.execute((re, im))
            del re, im
            torch.cuda.synchronize()
            y_rows = np.stack([yre[r * n:(r + 1) * n].cpu().numpy() + 1j * yim[r * n:(r + 1) * n].cpu().numpy()
                               for r in rows])
            del yre, yim
        else:
            y = p.execute(z)
            del z
            torch.cuda.synchronize()
            y_rows = np.stack([y[r * n:(r + 1) * n].cpu().numpy() for r in rows])
            del y
    torch.cuda.empty_cache()
    ref = oracle.fft(x_rows, SIGN["forward"], threads=8)
    assert_parity(y_rows, ref, f"N={n} batch={batch} ({total} elements) {layout}, rows {rows}", TOL)
