"""Helpers shared by the GPU tests: host <-> device marshalling and oracle references."""
from __future__ import annotations

import numpy as np

import oracle
import workloads

# per-transform relative L2 bound against the FP64 oracle: FP32 path
TOL = 1e-5
# FP64 path: the rounding error of a radix-2^k FFT grows like eps * log2 N
# (eps = 2^-53); at N = 2^24 with a few units of twiddle error that is
# ~1e-14, so 1e-13 leaves headroom while an FP32-rounded twiddle or value
# anywhere (~1e-7) fails it by six orders of magnitude
TOL64 = 1e-13
SIGN = {"forward": -1, "inverse": +1}


def to_device(re: np.ndarray, im: np.ndarray, layout: str):
    import torch
    if layout == "split":
        return (torch.from_numpy(np.ascontiguousarray(re)).cuda(), torch.from_numpy(np.ascontiguousarray(im)).cuda())
    return torch.from_numpy(workloads.interleave(re, im)).cuda()


def from_device(y, layout: str) -> np.ndarray:
    import torch
    torch.cuda.synchronize()
    if layout == "split":
        re, im = y
        return re.cpu().numpy().astype(np.float64) + 1j * im.cpu().numpy().astype(np.float64)
    return y.cpu().numpy().astype(np.complex128)


def widen(re: np.ndarray, im: np.ndarray) -> np.ndarray:
    """The float32 (or float64) input, widened exactly to complex128."""
    return re.astype(np.float64) + 1j * im.astype(np.float64)


def oracle_ref(re: np.ndarray, im: np.ndarray, direction: str, threads: int = 8) -> np.ndarray:
    return oracle.fft(widen(re, im), SIGN[direction], threads=threads)


def assert_parity(y: np.ndarray, ref: np.ndarray, what: str, tol: float = TOL) -> float:
    y = y.reshape(ref.shape)
    errs = oracle.rel_l2_rows(y.reshape(-1, ref.shape[-1]), ref.reshape(-1, ref.shape[-1]))
    worst = float(errs.max())
    print(f"[parity] {what}: max per-transform rel-L2 {worst:.3e}", flush=True)
    assert worst <= tol, f"{what}: rel-L2 {worst:.3e} > {tol}"
    return worst


def r2c_vjp_definition(g: np.ndarray, n: int) -> np.ndarray:
    """x[m] = Re sum_{k=0..n/2} g[k] exp(+2 pi i k m / n): the vector-Jacobian
    product of R2C from its definition (dX_k/dx_m = exp(-2 pi i k m / n)),
    through the oracle's complex DFT of g padded with zeros to length n."""
    b = g.shape[0]
    pad = np.zeros((b, n), dtype=np.complex128)
    pad[:, :n // 2 + 1] = g[:, :n // 2 + 1]
    return oracle.fft(pad, +1, threads=8).real


def c2r_vjp_bruteforce(g: np.ndarray, n: int) -> np.ndarray:
    """The vector-Jacobian product of C2R by brute force: column k of the
    Jacobian is the oracle's irfft of the unit vector e_k (real part) or
    i e_k (imaginary part), so G_k = <g, irfft(e_k)> + i <g, irfft(i e_k)>."""
    h = n // 2 + 1
    units = np.concatenate([np.eye(h), 1j * np.eye(h)]).astype(np.complex128)
    cols = oracle.irfft(units, n, threads=8)  # (2h, n)
    dots = g.astype(np.float64) @ cols.T      # (b, 2h)
    return dots[:, :h] + 1j * dots[:, h:]


def multi_candidates(cands: list[str], default: str, limit: int) -> list[str]:
    """The multi-pass decompositions among `cands`: all of them when there are
    at most `limit`, else an evenly spaced subset of `limit` plus the default
    (the sizes below the largest run every candidate, so every compiled pass
    kernel is still exercised)."""
    multi = [d for d in cands if d.startswith("multi")]
    if len(multi) <= limit:
        return multi
    step = len(multi) / limit
    pick = [multi[int(i * step)] for i in range(limit)]
    if default.startswith("multi") and default not in pick:
        pick.append(default)
    return pick
