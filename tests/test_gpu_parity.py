"""GPU parity: the HIP path against the FP64 oracle, element by element.

Every test calls the library through the C ABI (the ctypes binding) on
seeded inputs and compares per transform: relative L2 error <= 1e-5.
"""
import os

import numpy as np
import pytest

import oracle
import workloads
from fftcheck import SIGN, TOL, assert_parity, from_device, multi_candidates, oracle_ref, to_device, widen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def fftlib():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2308_00497_amd as m
    return m


def sweep_batch(n: int) -> int:
    # odd transform counts, so the last workgroup is partly empty
    return max(1, min(37, (1 << 20) // n))


@pytest.mark.parametrize("direction", ["forward", "inverse"])
@pytest.mark.parametrize("layout", ["interleaved", "split"])
@pytest.mark.parametrize("log2n", range(0, 25))
def test_sweep(fftlib, log2n, layout, direction):
    n = 1 << log2n
    batch = sweep_batch(n)
    re, im = workloads.normal_complex((batch, n), seed=1000 + log2n)
    with fftlib.Plan(n, batch, layout, direction) as plan:
        y = from_device(plan.execute(to_device(re, im, layout)), layout)
        desc = plan.describe()["decomposition"]
    assert_parity(y, oracle_ref(re, im, direction), f"N=2^{log2n} b={batch} {layout} {direction} {desc}")


def candidates(fftlib, log2n, layout, limit=None):
    c = fftlib.query_decomposition(1 << log2n, layout)["candidates"]
    return c if limit is None else c[:limit]


@pytest.mark.parametrize("layout", ["interleaved", "split"])
@pytest.mark.parametrize("log2n", range(1, 15))
def test_every_single_pass_variant(fftlib, log2n, layout):
    n = 1 << log2n
    batch = max(3, min(41, (1 << 18) // n))
    re, im = workloads.uniform_complex((batch, n), seed=2000 + log2n)
    ref = oracle_ref(re, im, "forward")
    for dec in candidates(fftlib, log2n, layout):
        if not dec.startswith("single"):
            continue
        with fftlib.Plan(n, batch, layout, "forward", decomposition=dec) as plan:
            y = from_device(plan.execute(to_device(re, im, layout)), layout)
        assert_parity(y, ref, f"N=2^{log2n} {layout} {dec}")


@pytest.mark.parametrize("layout", ["interleaved", "split"])
@pytest.mark.parametrize("log2n", [13, 14])
def test_radix32_single_pass(fftlib, log2n, layout):
    """32 points per thread: radix-32 register DFTs (Eq. 1 with K = 4, M = 8
    inside each thread), every grid size, both directions, a batch that
    leaves the persistent grid a ragged last round."""
    n = 1 << log2n
    batch = 1029 if log2n == 13 else 515
    re, im = workloads.normal_complex((batch, n), seed=2100 + log2n)
    decs = [c for c in candidates(fftlib, log2n, layout) if c.startswith("single:e5:")]
    assert decs
    for direction in ("forward", "inverse"):
        ref = oracle_ref(re, im, direction)
        for dec in decs:
            with fftlib.Plan(n, batch, layout, direction, decomposition=dec) as plan:
                y = from_device(plan.execute(to_device(re, im, layout)), layout)
            assert_parity(y, ref, f"N=2^{log2n} b={batch} {layout} {direction} {dec}")


@pytest.mark.parametrize("layout", ["interleaved", "split"])
@pytest.mark.parametrize("log2n", [12, 13, 14, 15, 16, 17, 18, 20, 24])
def test_every_multi_pass_variant(fftlib, log2n, layout):
    n = 1 << log2n
    batch = max(1, min(3, (1 << 20) // n))
    re, im = workloads.uniform_complex((batch, n), seed=3000 + log2n)
    ref = oracle_ref(re, im, "inverse" if log2n % 2 else "forward")
    direction = "inverse" if log2n % 2 else "forward"
    seen = 0
    q = fftlib.query_decomposition(n, layout)
    # 2^24: a spread of the ~400 chains (every pass kernel runs at the smaller sizes)
    for dec in multi_candidates(q["candidates"], q["default"], 48 if log2n >= 24 else 10**6):
        with fftlib.Plan(n, batch, layout, direction, decomposition=dec) as plan:
            y = from_device(plan.execute(to_device(re, im, layout)), layout)
        assert_parity(y, ref, f"N=2^{log2n} {layout} {direction} {dec}")
        seen += 1
    assert seen > 0


@pytest.mark.parametrize("layout", ["interleaved", "split"])
@pytest.mark.parametrize("chain,batch", [("multi:6c6,6c6,6c6", 5), ("multi:8c5,6c6,5c8", 3),
                                         ("multi:8c5,7c5,6c6", 2), ("multi:8c5,8c5,8c5", 1),
                                         ("multi:6c4,6c4,6c4,6c4", 1)])
def test_in_place_middle_pass_is_bitwise_stockham(fftlib, chain, batch, layout):
    """A chain whose penultimate pass writes over its own input differs from
    the Stockham chain of the same lengths only in addresses (the last pass
    reads the permuted layout): both directions must give bit-identical
    results, and the oracle's within the tolerance."""
    parts = chain.split(":")[1].split(",")
    parts[-2] += "i"
    twin = "multi:" + ",".join(parts)
    log2n = sum(int(p.split("c")[0]) for p in parts)
    n = 1 << log2n
    re, im = workloads.normal_complex((batch, n), seed=4100 + log2n)
    for direction in ("forward", "inverse"):
        ys = []
        for dec in (chain, twin):
            with fftlib.Plan(n, batch, layout, direction, decomposition=dec) as plan:
                y = plan.execute(to_device(re, im, layout))
                torch.cuda.synchronize()
                ys.append(torch.cat(y) if layout == "split" else y)
                if dec == twin:
                    assert plan.workspace_bytes == n * batch * 8 * (1 if len(parts) == 3 else 2)
        assert torch.equal(ys[0], ys[1]), f"{twin} {layout} {direction} differs from {chain}"
        assert_parity(from_device(ys[1].chunk(2) if layout == "split" else ys[1], layout),
                      oracle_ref(re, im, direction), f"{twin} {layout} {direction}")


@pytest.mark.parametrize("layout", ["interleaved", "split"])
@pytest.mark.parametrize("log2n", [0, 4, 10, 12, 14, 16, 20])
def test_in_place(fftlib, log2n, layout):
    n = 1 << log2n
    batch = max(1, min(9, (1 << 20) // n))
    re, im = workloads.normal_complex((batch, n), seed=4000 + log2n)
    x = to_device(re, im, layout)
    with fftlib.Plan(n, batch, layout, "forward") as plan:
        y = plan.execute(x, out=x)
    assert_parity(from_device(y, layout), oracle_ref(re, im, "forward"), f"in-place N=2^{log2n} {layout}")


@pytest.mark.parametrize("layout", ["interleaved", "split"])
@pytest.mark.parametrize("log2n", [3, 8, 12, 16, 22])
def test_backward_is_adjoint(fftlib, log2n, layout):
    """fft_execute_backward applies F^H for a forward plan and F for an inverse plan."""
    n = 1 << log2n
    batch = max(1, min(5, (1 << 20) // n))
    re, im = workloads.normal_complex((batch, n), seed=5000 + log2n)
    g = to_device(re, im, layout)
    for direction, want in (("forward", "inverse"), ("inverse", "forward")):
        with fftlib.Plan(n, batch, layout, direction) as plan:
            y = from_device(plan.backward(g), layout)
        assert_parity(y, oracle_ref(re, im, want), f"backward of {direction} plan N=2^{log2n} {layout}")


def test_dot_product_adjoint(fftlib):
    n, batch = 4096, 4
    xr, xi = workloads.normal_complex((batch, n), seed=6001)
    gr, gi = workloads.normal_complex((batch, n), seed=6002)
    with fftlib.Plan(n, batch, "interleaved", "forward") as plan:
        fx = from_device(plan.execute(to_device(xr, xi, "interleaved")), "interleaved")
        fhg = from_device(plan.backward(to_device(gr, gi, "interleaved")), "interleaved")
    lhs = np.vdot(widen(gr, gi), fx)
    rhs = np.vdot(fhg, widen(xr, xi))
    assert abs(lhs - rhs) / abs(lhs) < 1e-5


def test_round_trip(fftlib):
    n, batch = 1 << 15, 3
    re, im = workloads.normal_complex((batch, n), seed=6100)
    x = to_device(re, im, "split")
    with fftlib.Plan(n, batch, "split", "forward") as f, fftlib.Plan(n, batch, "split", "inverse") as b:
        back = from_device(b.execute(f.execute(x)), "split")
    assert_parity(back, n * widen(re, im), "inverse(forward(x)) = N x")


@pytest.mark.parametrize("log2n", [4, 12, 14, 18])
def test_deterministic(fftlib, log2n):
    n = 1 << log2n
    batch = max(1, (1 << 20) // n)
    re, im = workloads.normal_complex((batch, n), seed=7000 + log2n)
    x = to_device(re, im, "interleaved")
    with fftlib.Plan(n, batch, "interleaved", "forward") as plan:
        a = plan.execute(x)
        b = plan.execute(x)
        torch.cuda.synchronize()
    assert torch.equal(a.view(torch.float32), b.view(torch.float32))


def test_c1_against_dense_dft(fftlib):
    """N=1024, batch 16, split, U[-1,1), seed 1: against the O(N^2) definition."""
    re, im = workloads.c1()
    with fftlib.Plan(1024, 16, "split", "forward") as plan:
        y = from_device(plan.execute(to_device(re, im, "split")), "split")
    assert_parity(y, oracle.dft(widen(re, im)), "C1 vs dense DFT")


@pytest.mark.parametrize("layout", ["interleaved", "split"])
@pytest.mark.parametrize("direction", ["forward", "inverse"])
def test_c2_full_size(fftlib, layout, direction):
    """N=4096, batch 8192 (the benchmark launch, its default plan): every one of
    the 8192 transforms against the threaded oracle, element by element."""
    n, batch = 4096, 8192
    re, im = workloads.c2()
    x = to_device(re, im, layout)
    with fftlib.Plan(n, batch, layout, direction) as plan:
        y = from_device(plan.execute(x), layout).reshape(batch, n)
        desc = plan.describe()["decomposition"]
    del x
    ref = oracle_ref(re, im, direction, threads=16)
    assert_parity(y, ref, f"C2 all {batch} rows {layout} {direction} {desc}")


def test_c3_spikes_and_oracle(fftlib):
    """N=2^24 split: noise + 8 cosines; full oracle comparison and the closed-form spikes."""
    n = 1 << 24
    re, im, nr, ni, freqs = workloads.c3()
    with fftlib.Plan(n, 1, "split", "forward") as plan:
        y = from_device(plan.execute(to_device(re, im, "split")), "split")
        desc = plan.describe()["decomposition"]
    ref = oracle_ref(re, im, "forward", threads=1)
    assert_parity(y[None], ref[None], f"C3 N=2^24 split {desc}")
    # spikes: the tone part equals N/2 at f and N-f; the noise part comes from linearity
    noise_spec = oracle.fft(nr + 1j * ni)
    for f in freqs:
        for k in (int(f), n - int(f)):
            assert abs(y[k] - noise_spec[k] - n / 2) < 1e-6 * n / 2, (k, y[k] - noise_spec[k])


def test_workspace_override(fftlib):
    n, batch = 1 << 16, 2
    re, im = workloads.normal_complex((batch, n), seed=8000)
    x = to_device(re, im, "interleaved")
    with fftlib.Plan(n, batch, "interleaved", "forward") as plan:
        nbytes = plan.workspace_bytes
        assert nbytes >= n * batch * 8
        ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        plan.set_workspace(ws)
        y = from_device(plan.execute(x), "interleaved")
        plan.set_workspace(None)
        y2 = from_device(plan.execute(x), "interleaved")
    assert_parity(y, oracle_ref(re, im, "forward"), "caller workspace")
    assert np.array_equal(y, y2)


def test_execute_argument_errors(fftlib):
    n, batch = 256, 4
    with fftlib.Plan(n, batch, "interleaved", "forward") as plan:
        buf = torch.zeros(2 * n * batch + 8, dtype=torch.float32, device="cuda")
        base = buf.data_ptr()
        h = plan._handle
        lib = fftlib.lib
        assert lib.fft_execute(h, base + 4, None, base + 4096 * 8, None, None) == 4      # misaligned
        assert lib.fft_execute(h, None, None, base, None, None) == 3                      # null
        assert lib.fft_execute(h, base, None, base + 16, None, None) == 2                 # partial overlap
        torch.cuda.synchronize()
    with fftlib.Plan(n, batch, "split", "forward") as plan:
        a = torch.zeros(4 * n * batch, dtype=torch.float32, device="cuda")
        p = a.data_ptr()
        lib = fftlib.lib
        assert lib.fft_execute(plan._handle, p, None, p + 4 * n * batch * 2, p + 4 * n * batch * 3, None) == 3
        # output imaginary array overlapping the input real array
        assert lib.fft_execute(plan._handle, p, p + 4 * n * batch, p + 4 * n * batch * 2, p, None) == 2


def test_autotune_cache(fftlib, tmp_path, monkeypatch):
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("FFT_AUTOTUNE", "1")
    monkeypatch.setenv("FFT_AUTOTUNE_CACHE", str(cache))
    n, batch = 1 << 13, 64
    re, im = workloads.normal_complex((batch, n), seed=9000)
    with fftlib.Plan(n, batch, "split", "forward") as plan:
        d = plan.describe()
        assert d["source"] == "autotune"
        y = from_device(plan.execute(to_device(re, im, "split")), "split")
    assert_parity(y, oracle_ref(re, im, "forward"), f"autotuned {d['decomposition']}")
    text = cache.read_text()
    assert d["decomposition"] in text and "n13" in text
    monkeypatch.setenv("FFT_AUTOTUNE", "0")
    with fftlib.Plan(n, batch, "split", "forward") as plan:
        assert plan.describe()["source"] == "cache"
        assert plan.describe()["decomposition"] == d["decomposition"]


def test_alloc_failure_is_reported():
    """FFT_TEST_FAIL_ALLOC makes the first device allocation fail: FFT_ERR_ALLOC, no plan.
    Runs in a child process so the hook does not affect this one."""
    import subprocess
    import sys
    code = (
        "import ctypes, paper_2308_00497_amd as f\n"
        "h = ctypes.c_void_p()\n"
        "rc = f.lib.fft_plan_create(ctypes.byref(h), 4096, 8, 0, -1)\n"
        "print(rc, h.value)\n"
        "rc2 = f.lib.fft_plan_create(ctypes.byref(h), 4096, 8, 0, -1)\n"
        "print(rc2, h.value is not None)\n"
        "f.lib.fft_plan_destroy(h)\n"
    )
    env = dict(os.environ, FFT_TEST_FAIL_ALLOC="1")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", code], env=env, cwd=root, capture_output=True, text=True, timeout=300)
    lines = r.stdout.split("\n")
    assert lines[0] == "5 None", r.stdout + r.stderr
    assert lines[1] == "0 True", r.stdout + r.stderr


@pytest.mark.parametrize("nbytes", [16, 4096, 4096 * 3 + 48, 1 << 24, (1 << 24) + 4096 * 5 + 32])
def test_copy_device(fftlib, nbytes):
    """The streaming copy entry point (the benchmark's HBM ceiling) copies exactly."""
    src = torch.randint(0, 255, (nbytes,), dtype=torch.uint8, device="cuda")
    dst = torch.zeros(nbytes + 16, dtype=torch.uint8, device="cuda")
    fftlib.copy_device(src, dst)
    torch.cuda.synchronize()
    assert torch.equal(dst[:nbytes], src)
    assert int(dst[nbytes:].sum()) == 0
