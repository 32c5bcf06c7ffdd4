"""Pins for the FP64 oracle: it is checked against things other than itself.

Each test names the passage of the paper (or the piece of mathematics) it
relies on.  Together they are chosen so that a plausible slip in the oracle (a
flipped sign, a dropped term, a wrong or transposed index, a missing twiddle)
fails at least one of them; ``test_mutants_are_caught`` plants such slips in a
copy of ``oracle.c`` and checks exactly that.
"""
import cmath
import math
import os
import shutil
import tempfile

import numpy as np
import pytest

import oracle
import workloads

RNG = np.random.default_rng(12345)


def rand_c(shape, rng=RNG):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


# ---------------------------------------------------------------------------
# Eq. 1 and Table 1, built independently of the oracle
# ---------------------------------------------------------------------------

def stride_perm(n, k):
    """Pi^N_K, read as the stride-K gather z[M*n2 + n1] = x[K*n1 + n2] (M = N/K)."""
    m = n // k
    p = np.zeros((n, n))
    for n1 in range(m):
        for n2 in range(k):
            p[m * n2 + n1, k * n1 + n2] = 1.0
    return p


def twiddle_diag(n, m):
    """D^N_M: entry M*n2 + k1 holds w_N^(n2*k1), w_N = exp(-2 pi i / N)."""
    k = n // m
    d = np.zeros(n, dtype=complex)
    for n2 in range(k):
        for k1 in range(m):
            d[m * n2 + k1] = np.exp(-2j * np.pi * n2 * k1 / n)
    return np.diag(d)


def eq1_matrix(n):
    """DFT_N assembled from DFT_2 = [[1, 1], [1, -1]] by Eq. 1, splitting N = M*K."""
    if n == 1:
        return np.ones((1, 1), dtype=complex)
    if n == 2:
        return np.array([[1, 1], [1, -1]], dtype=complex)
    # alternate the split so both the M and the K factors recurse
    k = 2 if (n.bit_length() % 2) else 4
    k = min(k, n // 2)
    m = n // k
    dk, dm = eq1_matrix(k), eq1_matrix(m)
    return (np.kron(dk, np.eye(m)) @ twiddle_diag(n, m) @ np.kron(np.eye(k), dm)
            @ stride_perm(n, k))


def fused_mkiv(a, n, x):
    """Table 1, FusedMKIV(A, n, X) = (A_m (x) I_n) X: A applied to every stride-n slice."""
    m = a.shape[0]
    y = np.empty(m * n, dtype=complex)
    for i in range(n):
        y[i:i + m * n:n] = a @ x[i:i + m * n:n]
    return y


def fused_ikmv(a, m, x):
    """Table 1, FusedIKMV(A, n, X) = (I_m (x) A_n) X: A applied to each contiguous block."""
    n = a.shape[0]
    y = np.empty(m * n, dtype=complex)
    for i in range(m):
        y[i * n:i * n + n] = a @ x[i * n:i * n + n]
    return y


def permute(m, mn, x):
    """Table 1, Permute(m, mn, X): Y[i + m*j] = X[n*i + j], i < m, j < n (a pure copy)."""
    n = mn // m
    y = np.empty(mn, dtype=complex)
    for i in range(m):
        for j in range(n):
            y[i + m * j] = x[n * i + j]
    return y


def fused_pkiv(m, mn, k, x):
    """Table 1, FusedPKIV(m, mn, k, X) = (Pi_m^mn (x) I_k) X: blocks of k moved as Permute moves scalars."""
    n = mn // m
    y = np.empty(mn * k, dtype=complex)
    for i in range(m):
        for j in range(n):
            y[k * (i + m * j):k * (i + m * j) + k] = x[k * (n * i + j):k * (n * i + j) + k]
    return y


def mul(d, x):
    """Table 1, Mul(TwiddleCoe, X): element-wise product over all N entries."""
    return d * x


def table1_fft(x):
    """FFT of x through the Table 1 operators composed as Eq. 1 (M = N/2, K = 2)."""
    n = x.shape[0]
    if n == 1:
        return x.copy()
    k, m = 2, n // 2
    z = permute(m, n, x)                        # Pi^N_K with the Table 1 loop
    sub = np.empty(n, dtype=complex)
    for b in range(k):                          # (I_K (x) DFT_M) by recursion
        sub[b * m:(b + 1) * m] = table1_fft(z[b * m:(b + 1) * m])
    d = np.diag(twiddle_diag(n, m))
    t = mul(d, sub)
    return fused_mkiv(np.array([[1, 1], [1, -1]], dtype=complex), m, t)


@pytest.mark.parametrize("n", [1, 2, 4, 8, 16, 32, 64, 128])
def test_dft_equals_eq1_factorisation(n):
    """Paper section 3, Eq. 1 (with the stride-gather and twiddle-diagonal readings)."""
    eye = np.eye(n, dtype=complex)
    f_oracle = oracle.dft(eye).T          # column j = DFT of e_j
    np.testing.assert_allclose(f_oracle, eq1_matrix(n), rtol=0, atol=1e-12 * max(n, 1))


@pytest.mark.parametrize("n", [2, 4, 8, 16, 64, 256])
def test_dft_equals_table1_operators(n):
    """Paper Table 1: FusedMKIV, FusedIKMV (as recursion), Mul and Permute compose to DFT_N."""
    x = rand_c(n)
    np.testing.assert_allclose(oracle.dft(x), table1_fft(x), rtol=0, atol=1e-11 * n)
    np.testing.assert_allclose(oracle.fft(x), table1_fft(x), rtol=0, atol=1e-11 * n)


def test_table1_readings_consistent():
    """Table 1 readings: FusedPKIV is Permute lifted to blocks, FusedIKMV/FusedMKIV are the Kronecker forms."""
    m, n, k = 4, 3, 5
    x = rand_c(m * n * k)
    p = stride_perm(m * n, n)  # Permute(m, mn) == Pi^{mn}_n in the gather reading
    np.testing.assert_allclose(permute(m, m * n, x[:m * n]), p @ x[:m * n])
    np.testing.assert_allclose(fused_pkiv(m, m * n, k, x), np.kron(p, np.eye(k)) @ x)
    a = rand_c((m, m))
    np.testing.assert_allclose(fused_mkiv(a, n, x[:m * n]), np.kron(a, np.eye(n)) @ x[:m * n])
    b = rand_c((n, n))
    np.testing.assert_allclose(fused_ikmv(b, m, x[:m * n]), np.kron(np.eye(m), b) @ x[:m * n])


# ---------------------------------------------------------------------------
# Golden fixtures (closed forms, written out by hand)
# ---------------------------------------------------------------------------

def test_dft4_golden(golden_dir):
    rows = np.loadtxt(os.path.join(golden_dir, "dft4_matrix.txt"))
    f = np.zeros((4, 4), dtype=complex)
    for k, j, re, im in rows:
        f[int(k), int(j)] = re + 1j * im
    np.testing.assert_allclose(oracle.dft(np.eye(4)).T, f, atol=1e-15)
    np.testing.assert_allclose(oracle.fft(np.eye(4)).T, f, atol=1e-15)


def test_ramp_golden(golden_dir):
    rows = np.loadtxt(os.path.join(golden_dir, "dft8_ramp.txt"))
    want = rows[:, 1] + 1j * rows[:, 2]
    x = np.arange(8, dtype=float)
    np.testing.assert_allclose(oracle.dft(x), want, rtol=0, atol=1e-13)
    np.testing.assert_allclose(oracle.fft(x), want, rtol=0, atol=1e-13)


@pytest.mark.parametrize("n", [16, 256, 4096])
def test_ramp_closed_form(n):
    """X[k] = -N/2 + i (N/2) cot(pi k / N), X[0] = N(N-1)/2 (arithmetic-geometric series)."""
    x = np.arange(n, dtype=float)
    k = np.arange(1, n)
    want = np.empty(n, dtype=complex)
    want[0] = n * (n - 1) / 2
    want[1:] = -n / 2 + 1j * (n / 2) / np.tan(np.pi * k / n)
    y = oracle.fft(x)
    assert oracle.rel_l2(y, want) < 1e-13


# ---------------------------------------------------------------------------
# Brute force and library cross-checks
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("log2n", range(0, 12))
def test_r2_equals_dft(log2n):
    n = 1 << log2n
    x = rand_c((3, n))
    for sign in (-1, +1):
        assert oracle.rel_l2(oracle.fft(x, sign), oracle.dft(x, sign)) < 1e-13


@pytest.mark.parametrize("log2n", list(range(0, 13)) + [16, 20])
def test_against_numpy_pocketfft(log2n):
    """numpy.fft.fft (pocketfft, FP64) is an independent library routine."""
    n = 1 << log2n
    x = rand_c((2, n))
    assert oracle.rel_l2(oracle.fft(x), np.fft.fft(x)) < 1e-13
    assert oracle.rel_l2(oracle.fft(x, +1), n * np.fft.ifft(x)) < 1e-13
    if log2n <= 10:
        assert oracle.rel_l2(oracle.dft(x), np.fft.fft(x)) < 1e-13


@pytest.mark.parametrize("log2n", range(4, 13))
def test_paper_error_metric(log2n):
    """Paper section 4: random inputs, N = 16 .. 4096, |result - NumPy| / N < 1e-7 (FP64)."""
    n = 1 << log2n
    x = rand_c(n)
    ref = np.fft.fft(x)
    for y in (oracle.fft(x), oracle.dft(x)):
        assert np.max(np.abs(y - ref)) / n < 1e-7
        assert np.linalg.norm(y - ref) / n < 1e-7


# ---------------------------------------------------------------------------
# Closed forms
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n", [1, 2, 16, 1024, 1 << 14])
def test_impulse_at_zero_gives_ones(n):
    x = np.zeros(n)
    x[0] = 1.0
    assert np.array_equal(oracle.fft(x), np.ones(n, dtype=complex))
    if n <= 1024:
        assert np.array_equal(oracle.dft(x), np.ones(n, dtype=complex))


@pytest.mark.parametrize("n", [1, 8, 4096])
def test_constant_gives_dc_spike(n):
    want = np.zeros(n, dtype=complex)
    want[0] = n
    np.testing.assert_allclose(oracle.fft(np.ones(n)), want, atol=1e-12 * n)
    np.testing.assert_allclose(oracle.dft(np.ones(n)), want, atol=1e-12 * n)


@pytest.mark.parametrize("n,f", [(8, 1), (64, 5), (1024, 17), (4096, 1000), (4096, 0), (4096, 2048)])
def test_cosine_gives_two_spikes(n, f):
    j = np.arange(n)
    x = np.cos(2 * np.pi * ((f * j) % n) / n)
    want = np.zeros(n, dtype=complex)
    if f == 0 or 2 * f == n:
        want[f] = n
    else:
        want[f] = want[n - f] = n / 2
    np.testing.assert_allclose(oracle.fft(x), want, atol=1e-10)
    if n <= 1024:
        np.testing.assert_allclose(oracle.dft(x), want, atol=1e-10)


def test_c3_style_spikes_small():
    """Sum of 8 seeded cosines plus noise: spikes of N/2 at f and N - f on top of the noise spectrum."""
    n = 1 << 16
    re, im, nr, ni, freqs = workloads.c3(n)
    spec_noise = oracle.fft(nr + 1j * ni)
    j = np.arange(n)
    tones = sum(np.cos(2 * np.pi * ((int(f) * j) % n) / n) for f in freqs)
    spec = oracle.fft(nr + tones + 1j * ni)
    want = spec_noise.copy()
    for f in freqs:
        want[f] += n / 2
        want[n - f] += n / 2
    assert oracle.rel_l2(spec, want) < 1e-13
    assert len(set(int(f) for f in freqs)) == 8


# ---------------------------------------------------------------------------
# Invariants
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n", [4, 256, 4096])
def test_parseval(n):
    x = rand_c(n)
    y = oracle.fft(x)
    np.testing.assert_allclose(np.sum(np.abs(y) ** 2), n * np.sum(np.abs(x) ** 2), rtol=1e-12)


def test_linearity():
    n = 512
    x, y = rand_c(n), rand_c(n)
    a, b = 0.3 - 1.2j, -2.0 + 0.5j
    lhs = oracle.fft(a * x + b * y)
    rhs = a * oracle.fft(x) + b * oracle.fft(y)
    assert oracle.rel_l2(lhs, rhs) < 1e-13


@pytest.mark.parametrize("n", [1, 2, 64, 4096])
def test_round_trip_is_n_times_identity(n):
    x = rand_c((2, n))
    back = oracle.fft(oracle.fft(x), +1)
    assert oracle.rel_l2(back, n * x) < 1e-13


@pytest.mark.parametrize("n", [8, 1024])
def test_involution(n):
    """(F F x)[j] = N x[-j mod N] and F^4 = N^2 I."""
    x = rand_c(n)
    ffx = oracle.fft(oracle.fft(x))
    rev = x[(-np.arange(n)) % n]
    assert oracle.rel_l2(ffx, n * rev) < 1e-13
    assert oracle.rel_l2(oracle.fft(oracle.fft(ffx)), n * n * x) < 1e-13


@pytest.mark.parametrize("s", [1, 7, 100])
def test_shift_theorem(s):
    n = 256
    x = rand_c(n)
    k = np.arange(n)
    lhs = oracle.fft(np.roll(x, s))
    rhs = np.exp(-2j * np.pi * ((k * s) % n) / n) * oracle.fft(x)
    assert oracle.rel_l2(lhs, rhs) < 1e-13


def test_hermitian_symmetry_for_real_input():
    n = 2048
    x = RNG.standard_normal(n)
    y = oracle.fft(x)
    k = np.arange(1, n)
    np.testing.assert_allclose(y[n - k], np.conj(y[k]), atol=1e-10)
    assert abs(y[0].imag) < 1e-10 and abs(y[n // 2].imag) < 1e-10


def test_adjoint_dot_product():
    """<F x, y> = <x, F^H y> with F^H the unnormalised inverse."""
    n = 4096
    x, y = rand_c(n), rand_c(n)
    lhs = np.vdot(y, oracle.fft(x))
    rhs = np.vdot(oracle.fft(y, +1), x)
    assert abs(lhs - rhs) / abs(lhs) < 1e-12


# ---------------------------------------------------------------------------
# Gradient of the weighted spectral power
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n", [16, 256])
def test_gradient_against_central_differences(n):
    """FP64 central differences on seeded coordinates of Re x and Im x.

    L is exactly quadratic in (Re x, Im x), so the central difference has no
    truncation error; only rounding remains, about eps * L / h.  The tolerance
    is that term with a safety factor, plus a 1e-9 relative floor.
    """
    rng = np.random.default_rng(77)
    x = rand_c(n, rng)
    w = rng.uniform(0, 1, n)
    g = oracle.wpower_grad(x, w)
    loss = oracle.wpower_loss(x, w)
    coords = rng.choice(n, size=min(n, 32), replace=False)
    for h in (1e-6, 1e-3):
        tol_abs = 64 * np.finfo(float).eps * loss / h
        for idx in coords:
            for part in (1.0, 1j):
                e = np.zeros(n, dtype=complex)
                e[idx] = part * h
                fd = (oracle.wpower_loss(x + e, w) - oracle.wpower_loss(x - e, w)) / (2 * h)
                an = g[idx].real if part == 1.0 else g[idx].imag
                assert abs(fd - an) <= tol_abs + 1e-9 * abs(an), (h, idx, part, fd, an)


def test_gradient_closed_form_for_uniform_weight():
    """w = 1: L = N ||x||^2 (Parseval), so the gradient is 2 N x."""
    n = 512
    x = rand_c(n)
    g = oracle.wpower_grad(x, np.ones(n))
    assert oracle.rel_l2(g, 2 * n * x) < 1e-13


# ---------------------------------------------------------------------------
# Argument checking
# ---------------------------------------------------------------------------

def test_rejects_non_power_of_two():
    with pytest.raises(ValueError):
        oracle.fft(np.ones(12))


def test_rejects_bad_sign():
    with pytest.raises(ValueError):
        oracle.fft(np.ones(8), sign=2)


# ---------------------------------------------------------------------------
# Real sequences: R2C (the half k = 0 .. N/2 of the DFT of a real row) and
# C2R (real part of the unnormalised inverse DFT of the Hermitian extension)
# ---------------------------------------------------------------------------

def brute_rfft(x):
    """Direct sum over n, pure Python loops (tiny sizes only)."""
    n = len(x)
    out = []
    for k in range(n // 2 + 1):
        acc = 0j
        for m in range(n):
            acc += x[m] * cmath.exp(-2j * math.pi * ((k * m) % n) / n)
        out.append(acc)
    return np.array(out)


def brute_irfft(xh, n):
    """Direct sum over the Hermitian extension, real part (tiny sizes only)."""
    ext = [xh[k] if k <= n // 2 else xh[n - k].conjugate() for k in range(n)]
    out = []
    for m in range(n):
        acc = 0j
        for k in range(n):
            acc += ext[k] * cmath.exp(2j * math.pi * ((k * m) % n) / n)
        out.append(acc.real)
    return np.array(out)


@pytest.mark.parametrize("n", [1, 2, 4, 8, 16, 32])
def test_rfft_brute_force(n):
    x = np.random.default_rng(900 + n).standard_normal((3, n))
    got = oracle.rfft(x)
    assert got.shape == (3, n // 2 + 1)
    for r in range(3):
        assert np.abs(got[r] - brute_rfft(list(x[r]))).max() <= 1e-12 * max(n, 1)


@pytest.mark.parametrize("n", [1, 2, 4, 8, 16, 32])
def test_irfft_brute_force(n):
    """Random half-spectra, with non-zero imaginary parts at DC and Nyquist
    (they drop out of the real part)."""
    rng = np.random.default_rng(950 + n)
    h = n // 2 + 1
    xh = rng.standard_normal((3, h)) + 1j * rng.standard_normal((3, h))
    got = oracle.irfft(xh, n)
    for r in range(3):
        assert np.abs(got[r] - brute_irfft(list(xh[r]), n)).max() <= 1e-12 * max(n, 1)


@pytest.mark.parametrize("log2n", range(0, 13))
def test_rfft_against_numpy(log2n):
    n = 1 << log2n
    x = np.random.default_rng(1000 + log2n).standard_normal((4, n))
    ref = np.fft.rfft(x)
    assert oracle.rel_l2(oracle.rfft(x), ref) <= 1e-14 * max(log2n, 1)


@pytest.mark.parametrize("log2n", range(0, 13))
def test_irfft_against_numpy(log2n):
    n = 1 << log2n
    rng = np.random.default_rng(1100 + log2n)
    xh = rng.standard_normal((4, n // 2 + 1)) + 1j * rng.standard_normal((4, n // 2 + 1))
    ref = n * np.fft.irfft(xh, n)
    assert oracle.rel_l2(oracle.irfft(xh, n), ref) <= 1e-14 * max(log2n, 1)


@pytest.mark.parametrize("n,f", [(64, 5), (256, 100), (1024, 1), (16, 7)])
def test_rfft_cosine_and_sine_closed_form(n, f):
    """cos(2 pi f m / n) -> n/2 at k = f; sin -> -i n/2 at k = f; zero elsewhere."""
    m = np.arange(n)
    ph = 2 * np.pi * ((f * m) % n) / n
    for sig, val in ((np.cos(ph), n / 2), (np.sin(ph), -1j * n / 2)):
        want = np.zeros(n // 2 + 1, dtype=complex)
        want[f] = val
        assert np.abs(oracle.rfft(sig[None])[0] - want).max() <= 1e-12 * n


@pytest.mark.parametrize("n", [2, 8, 512])
def test_rfft_dc_and_nyquist(n):
    got = oracle.rfft(np.stack([np.ones(n), (-1.0) ** np.arange(n)]))
    want = np.zeros((2, n // 2 + 1), dtype=complex)
    want[0, 0] = n
    want[1, n // 2] += n
    assert np.abs(got - want).max() <= 1e-12 * n
    assert np.all(got[:, 0].imag == 0) and np.all(got[:, -1].imag == 0)


@pytest.mark.parametrize("n", [1, 2, 4, 16, 64])
def test_real_vjp_references(n):
    """The references the GPU tests hold the backward of real plans to.
    R2C: the definition-based product equals the brute-force vector-Jacobian
    product (Jacobian rows from rfft of unit vectors), and satisfies
    Re<rfft x, g> = <x, vjp(g)>.  C2R: the brute-force product satisfies
    <irfft X, g> = Re<X, vjp(g)> and has real DC and Nyquist bins.  Both also
    match the forms the kernels use: C2R of g with bins 1 .. n/2-1 halved, and
    R2C of g with those bins doubled."""
    from fftcheck import c2r_vjp_bruteforce, r2c_vjp_definition
    rng = np.random.default_rng(1300 + n)
    h = n // 2 + 1
    g = rng.standard_normal((3, h)) + 1j * rng.standard_normal((3, h))
    x = rng.standard_normal((3, n))
    jac = oracle.rfft(np.eye(n))                            # (n, h): dX_k/dx_m
    brute = np.real(np.conj(g) @ jac.T)                     # torch convention
    vjp = r2c_vjp_definition(g, n)
    assert np.abs(vjp - brute).max() <= 1e-12 * n
    lhs = np.sum(np.real(np.conj(oracle.rfft(x)) * g))
    assert abs(lhs - np.sum(x * vjp)) <= 1e-10 * n
    half = g.copy()
    half[:, 1:n // 2] *= 0.5
    assert np.abs(oracle.irfft(half, n) - vjp).max() <= 1e-12 * n
    gr = rng.standard_normal((3, n))
    G = c2r_vjp_bruteforce(gr, n)
    X = rng.standard_normal((3, h)) + 1j * rng.standard_normal((3, h))
    assert abs(np.sum(oracle.irfft(X, n) * gr) - np.sum(np.real(np.conj(X) * G))) <= 1e-10 * n
    assert np.abs(G[:, 0].imag).max() <= 1e-12 and np.abs(G[:, -1].imag).max() <= 1e-12
    dbl = oracle.rfft(gr)
    dbl[:, 1:n // 2] *= 2.0
    assert np.abs(dbl - G).max() <= 1e-12 * n


@pytest.mark.parametrize("n", [1, 2, 64, 4096])
def test_real_round_trip(n):
    x = np.random.default_rng(1200 + n).standard_normal((3, n))
    assert np.abs(oracle.irfft(oracle.rfft(x), n) - n * x).max() <= 1e-12 * n


# ---------------------------------------------------------------------------
# Multi-dimensional DFT (2D / 3D batched)
# ---------------------------------------------------------------------------

def brute_dftn(x, sign=-1):
    """The d-dimensional DFT summed term by term (tiny shapes only)."""
    shape = x.shape
    out = np.zeros(shape, dtype=complex)
    idx = list(np.ndindex(*shape))
    for k in idx:
        acc = 0j
        for nn in idx:
            ph = sum(((kj * nj) % sj) / sj for kj, nj, sj in zip(k, nn, shape))
            acc += x[nn] * cmath.exp(sign * 2j * math.pi * ph)
        out[k] = acc
    return out


@pytest.mark.parametrize("shape", [(2, 4), (4, 8), (8, 2), (2, 2, 4), (4, 2, 8)])
@pytest.mark.parametrize("sign", [-1, 1])
def test_fftn_brute_force(shape, sign):
    x = rand_c(shape, np.random.default_rng(1300 + len(shape)))
    got = oracle.fftn(x[None], len(shape), sign)[0]
    assert np.abs(got - brute_dftn(x, sign)).max() <= 1e-12 * x.size


@pytest.mark.parametrize("shape", [(16, 64), (64, 32, 8), (128, 256)])
def test_fftn_against_numpy(shape):
    x = rand_c((3,) + shape, np.random.default_rng(1400 + len(shape)))
    axes = tuple(range(1, len(shape) + 1))
    assert oracle.rel_l2(oracle.fftn(x, len(shape)), np.fft.fftn(x, axes=axes)) <= 1e-14
    assert oracle.rel_l2(oracle.fftn(x, len(shape), +1), np.fft.ifftn(x, axes=axes) * np.prod(shape)) <= 1e-14


def test_fftn_separable_plane_wave():
    """exp(2 pi i (f0 n0 / N0 + f1 n1 / N1)) -> N0 N1 at (f0, f1), zero elsewhere."""
    n0, n1, f0, f1 = 32, 16, 5, 11
    a = np.arange(n0)[:, None]
    b = np.arange(n1)[None, :]
    x = np.exp(2j * np.pi * (((f0 * a) % n0) / n0 + ((f1 * b) % n1) / n1))
    want = np.zeros((n0, n1), dtype=complex)
    want[f0, f1] = n0 * n1
    assert np.abs(oracle.fftn(x[None], 2)[0] - want).max() <= 1e-10


# ---------------------------------------------------------------------------
# Planted mistakes: every one must be caught by some pin above
# ---------------------------------------------------------------------------

MUTANTS = {
    # sign of the twiddle's imaginary part in the radix-2 combine
    "r2_twiddle_sign": ("double wi = sign * s[k * tstep];", "double wi = -sign * s[k * tstep];"),
    # a dropped cross term in the complex product of the dense sum
    "dft_dropped_term": ("acc_r += xr[j] * wr - xi[j] * wi;", "acc_r += xr[j] * wr;"),
    # the odd half recursing on the even samples (index slip)
    "r2_odd_index": ("r2_rec(xr + stride, xi + stride, 2 * stride, h,",
                     "r2_rec(xr, xi, 2 * stride, h,"),
    # twiddle table stepped at the wrong rate
    "r2_twiddle_step": ("double wr = c[k * tstep];", "double wr = c[k];"),
    # exponent reduced with k + j instead of k * j
    "dft_exponent": ("(unsigned __int128)k * (unsigned __int128)j", "(unsigned __int128)(k + j)"),
    # butterfly outputs swapped (transposed halves)
    "r2_halves_swapped": ("yr[k] = er + orr;", "yr[k] = er - orr;"),
    # C2R: Hermitian extension without the conjugate
    "irfft_conj_dropped": ("ei[b * n + k] = -xi[b * h + (n - k)];", "ei[b * n + k] = xi[b * h + (n - k)];"),
    # C2R: mirrored index off by one
    "irfft_mirror_index": ("er[b * n + k] = xr[b * h + (n - k)];", "er[b * n + k] = xr[b * h + (n - k - 1)];"),
    # R2C: conjugated output (sign slip on the imaginary part)
    "rfft_imag_sign": ("yi[b * h + k] = fi[b * n + k];", "yi[b * h + k] = -fi[b * n + k];"),
    # R2C: inverse exponent
    "rfft_exponent_sign": ("rc = oracle_fft_r2_batch(n, batch, -1, x, zi, fr, fi, nthreads);",
                           "rc = oracle_fft_r2_batch(n, batch, 1, x, zi, fr, fi, nthreads);"),
}


def _pins_pass(lib_path) -> bool:
    """Run a compact set of the pins above against another compiled oracle."""
    oracle.use_library(lib_path)
    try:
        checks = [
            lambda: test_dft_equals_eq1_factorisation(16),
            lambda: test_dft_equals_table1_operators(16),
            lambda: test_r2_equals_dft(5),
            lambda: test_against_numpy_pocketfft(6),
            lambda: test_cosine_gives_two_spikes(64, 5),
            lambda: test_round_trip_is_n_times_identity(64),
            lambda: test_rfft_brute_force(16),
            lambda: test_irfft_brute_force(16),
            lambda: test_rfft_cosine_and_sine_closed_form(64, 5),
        ]
        for c in checks:
            try:
                c()
            except AssertionError:
                return False
        return True
    finally:
        oracle.use_library(None)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutants_are_caught(name):
    src = open(os.path.join(os.path.dirname(oracle.__file__), "oracle.c")).read()
    old, new = MUTANTS[name]
    assert src.count(old) == 1, "mutation site not found: " + old
    tmp = tempfile.mkdtemp(prefix="oracle_mutant_")
    try:
        path = os.path.join(tmp, "mutant.c")
        with open(path, "w") as f:
            f.write(src.replace(old, new))
        lib = oracle.compile_source(path, os.path.join(tmp, "libmutant.so"))
        assert not _pins_pass(lib), f"mutant {name} slipped past every pin"
    finally:
        shutil.rmtree(tmp, ignore_errors=True)


def test_unmutated_copy_passes_pins():
    tmp = tempfile.mkdtemp(prefix="oracle_copy_")
    try:
        src = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")
        lib = oracle.compile_source(src, os.path.join(tmp, "libcopy.so"))
        assert _pins_pass(lib)
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
