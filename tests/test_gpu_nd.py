"""GPU parity of batched 2D and 3D transforms (the last axis by the 1D plan,
the other axes by column passes) against the oracle's multi-dimensional DFT."""
import numpy as np
import pytest

import oracle
import workloads
from fftcheck import SIGN, TOL, TOL64, assert_parity

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def fftlib():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2308_00497_amd as m
    return m


def to_dev(re, im, layout):
    if layout == "split":
        return (torch.from_numpy(np.ascontiguousarray(re)).cuda(), torch.from_numpy(np.ascontiguousarray(im)).cuda())
    return torch.from_numpy(workloads.interleave(re, im)).cuda()


def from_dev(y, layout):
    torch.cuda.synchronize()
    if layout == "split":
        return y[0].cpu().numpy().astype(np.float64) + 1j * y[1].cpu().numpy().astype(np.float64)
    return y.cpu().numpy().astype(np.complex128)


SHAPES = [(2, 2), (4, 64), (16, 1024), (64, 64), (256, 128), (4096, 4), (32, 1 << 14), (1024, 1024),
          (2, 4, 8), (8, 8, 8), (16, 32, 64), (64, 64, 64), (128, 16, 2), (4, 4096, 2),
          # long columns (2^10 .. 2^12) as two passes of the pass kernel, and
          # the ones too narrow for it (one column pass)
          (2048, 64), (4096, 512), (1024, 256), (1024, 2), (2048, 4, 32), (4096, 2, 2)]


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("layout", ["interleaved", "split"])
@pytest.mark.parametrize("shape", SHAPES)
def test_nd_against_oracle(fftlib, shape, layout, precision):
    size = int(np.prod(shape))
    batch = max(1, min(3, (1 << 20) // size))
    dt = np.float64 if precision == "fp64" else np.float32
    tol = TOL64 if precision == "fp64" else TOL
    re, im = workloads.normal_complex((batch,) + shape, seed=9500 + size % 1000, dtype=dt)
    x64 = re.astype(np.float64) + 1j * im.astype(np.float64)
    for direction in ("forward", "inverse"):
        with fftlib.PlanND(shape, batch, layout, direction, precision) as p:
            y = from_dev(p.execute(to_dev(re, im, layout)), layout)
            g = from_dev(p.backward(to_dev(re, im, layout)), layout)
            desc = p.describe()
        ref = oracle.fftn(x64, len(shape), SIGN[direction], threads=8)
        adj = oracle.fftn(x64, len(shape), -SIGN[direction], threads=8)
        what = f"{precision} {shape} b={batch} {layout} {direction}"
        assert_parity(y.reshape(batch, -1), ref.reshape(batch, -1), what, tol)
        assert_parity(g.reshape(batch, -1), adj.reshape(batch, -1), what + " adjoint", tol)
        assert desc["rank"] == len(shape)
        two_pass = [c for c in desc["column_passes"] if "passes" in c]
        print(f"[case] {shape}: column passes {desc['column_passes']}", flush=True)
        if shape in ((2048, 64), (4096, 512), (2048, 4, 32)) or (shape == (1024, 256) and
                                                                  (layout == "split" or precision == "fp64")):
            assert two_pass, desc


def test_nd_in_place_and_tensor_functions(fftlib):
    shape = (64, 256)
    re, im = workloads.normal_complex((2,) + shape, seed=9600)
    z = torch.from_numpy(workloads.interleave(re, im)).cuda()
    ref = oracle.fftn(re.astype(np.float64) + 1j * im.astype(np.float64), 2)
    with fftlib.PlanND(shape, 2) as p:
        zi = z.clone()
        y = p.execute(zi, out=zi)
    assert_parity(from_dev(y, "interleaved").reshape(2, -1), ref.reshape(2, -1), "2D in place")
    y2 = from_dev(fftlib.fftn(z, 2), "interleaved")
    assert_parity(y2.reshape(2, -1), ref.reshape(2, -1), "fftn()")
    back = from_dev(fftlib.ifftn(fftlib.fftn(z, 2), 2), "interleaved") / np.prod(shape)
    assert oracle.rel_l2(back, re.astype(np.float64) + 1j * im.astype(np.float64)) <= TOL


def test_nd_rejects_long_strided_axis(fftlib):
    with pytest.raises(fftlib.FFTError):
        fftlib.PlanND((8192, 4), 1)


@pytest.mark.parametrize("layout", ["interleaved", "split"])
def test_nd_two_pass_columns_with_caller_workspace(fftlib, layout):
    """A plan whose long columns run as two passes needs a workspace of the
    whole array (shared with its last-axis plan); a caller-owned one works the
    same, and None returns the plan to its own."""
    shape, batch = (4096, 128), 2
    re, im = workloads.normal_complex((batch,) + shape, seed=9700)
    ref = oracle.fftn(re.astype(np.float64) + 1j * im.astype(np.float64), 2, threads=8)
    with fftlib.PlanND(shape, batch, layout) as p:
        assert any("passes" in c for c in p.describe()["column_passes"])
        nb = p.workspace_bytes
        assert nb >= batch * 4096 * 128 * 8
        ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
        p.set_workspace(ws)
        y1 = from_dev(p.execute(to_dev(re, im, layout)), layout)
        p.set_workspace(None)
        y2 = from_dev(p.execute(to_dev(re, im, layout)), layout)
    for y, what in ((y1, "caller workspace"), (y2, "own workspace")):
        assert_parity(y.reshape(batch, -1), ref.reshape(batch, -1), f"2D two-pass columns {layout} {what}")
