"""Batched 1D complex-to-complex FFT (FP32 and FP64) for the AMD MI355X (gfx950).

Python binding over the C ABI of ``include/fft.h`` (the HIP library in
``lib/libfft_mi355x.so``).  Torch tensors supply device memory and the HIP
stream (``torch.cuda.current_stream()``); every step of the transform runs in
the library's kernels.  Conventions follow the paper's DFT (section 3, Eq. 1;
signs as the FFTW comparison of section 4): forward exp(-2 pi i k n / N),
inverse exp(+2 pi i k n / N), neither scaled.

    Plan(n, batch, layout="interleaved" | "split", direction="forward" | "inverse",
         precision="fp32" | "fp64")
    RaggedPlan(sizes, layout, direction)          (FP32)
    RealPlan(n, batch, layout, direction, precision)  R2C (forward) / C2R (inverse)
    PlanND(dims, batch, layout, direction, precision) 2D / 3D transforms
    fftn(x, ndim), ifftn(x, ndim)   over the last ndim (2 or 3) axes
    fft(x), ifft(x)                 complex64/complex128 tensors or (re, im) float32/float64 tuples
    rfft(x), irfft(X, n)            real tensors [..., n] <-> complex [..., n/2 + 1]
    FFTFunction.apply(re, im)       differentiable split-layout forward FFT
    fft_autograd(z)                 differentiable complex forward FFT
"""
from __future__ import annotations

import ctypes
import json

import torch

from ._lib import (FFT_FORWARD, FFT_INVERSE, FFT_LAYOUT_INTERLEAVED, FFT_LAYOUT_SPLIT, FFT_PRECISION_FP32,
                   FFT_PRECISION_FP64, FFTError, check, lib)

__all__ = ["Plan", "RaggedPlan", "RealPlan", "PlanND", "fft", "ifft", "rfft", "irfft", "fftn", "ifftn",
           "FFTFunction", "fft_autograd", "rfft_autograd", "irfft_autograd", "copy_device", "query_decomposition",
           "FFTError"]

_LAYOUTS = {"interleaved": FFT_LAYOUT_INTERLEAVED, "split": FFT_LAYOUT_SPLIT}
_DIRS = {"forward": FFT_FORWARD, "inverse": FFT_INVERSE}
_PRECISIONS = {"fp32": FFT_PRECISION_FP32, "fp64": FFT_PRECISION_FP64}
# precision -> (real dtype, complex dtype)
_DTYPES = {"fp32": (torch.float32, torch.complex64), "fp64": (torch.float64, torch.complex128)}


def _precision_of(dtype: torch.dtype) -> str:
    if dtype in (torch.float32, torch.complex64):
        return "fp32"
    if dtype in (torch.float64, torch.complex128):
        return "fp64"
    raise TypeError(f"unsupported dtype {dtype}: float32/complex64 or float64/complex128")


def _stream_handle(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _ptr(t: torch.Tensor | None) -> int | None:
    return None if t is None else t.data_ptr()


class _PlanBase:
    _handle: ctypes.c_void_p | None = None

    def __init__(self, layout: str, direction: str, precision: str = "fp32"):
        if layout not in _LAYOUTS:
            raise ValueError(f"layout must be one of {sorted(_LAYOUTS)}")
        if direction not in _DIRS:
            raise ValueError(f"direction must be one of {sorted(_DIRS)}")
        if precision not in _PRECISIONS:
            raise ValueError(f"precision must be one of {sorted(_PRECISIONS)}")
        self.layout = layout
        self.direction = direction
        self.precision = precision
        self.split = layout == "split"

    # --- introspection -------------------------------------------------
    def sizes(self) -> tuple[int, int, float]:
        t, e, f = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_double()
        check(lib.fft_plan_sizes(self._handle, ctypes.byref(t), ctypes.byref(e), ctypes.byref(f)), "fft_plan_sizes")
        return t.value, e.value, f.value

    @property
    def elements(self) -> int:
        return self.sizes()[1]

    @property
    def nominal_flops(self) -> float:
        """Sum of 5 N log2 N over the transforms (the paper's flop model, section 4)."""
        return self.sizes()[2]

    def describe(self) -> dict:
        buf = ctypes.create_string_buffer(1 << 16)
        check(lib.fft_plan_describe(self._handle, buf, len(buf)), "fft_plan_describe")
        return json.loads(buf.value.decode())

    @property
    def workspace_bytes(self) -> int:
        n = ctypes.c_size_t()
        check(lib.fft_plan_workspace_bytes(self._handle, ctypes.byref(n)), "fft_plan_workspace_bytes")
        return n.value

    def set_workspace(self, buf: torch.Tensor | None) -> None:
        """Use a caller-owned device buffer (>= workspace_bytes) as the workspace; None reverts."""
        if buf is not None:
            if not buf.is_cuda or buf.numel() * buf.element_size() < self.workspace_bytes:
                raise ValueError("workspace must be a device tensor of at least workspace_bytes bytes")
        self._ws_ref = buf
        check(lib.fft_plan_set_workspace(self._handle, _ptr(buf)), "fft_plan_set_workspace")

    # --- execution -------------------------------------------------------
    def _io(self, x, out):
        rdt, cdt = _DTYPES[self.precision]
        if self.split:
            if not (isinstance(x, (tuple, list)) and len(x) == 2):
                raise TypeError(f"split layout takes (re, im) {rdt} tensors")
            re, im = x
            for t in (re, im):
                if t.dtype != rdt or not t.is_cuda or not t.is_contiguous():
                    raise TypeError(f"split inputs must be contiguous {rdt} CUDA tensors")
                if t.numel() != self.elements:
                    raise ValueError(f"expected {self.elements} elements, got {t.numel()}")
            if out is None:
                out = (torch.empty_like(re), torch.empty_like(im))
            ore, oim = out
            return _ptr(re), _ptr(im), _ptr(ore), _ptr(oim), out
        if x.dtype != cdt or not x.is_cuda or not x.is_contiguous():
            raise TypeError(f"interleaved input must be a contiguous {cdt} CUDA tensor")
        if x.numel() != self.elements:
            raise ValueError(f"expected {self.elements} elements, got {x.numel()}")
        if out is None:
            out = torch.empty_like(x)
        return _ptr(x), None, _ptr(out), None, out

    def execute(self, x, out=None, stream=None):
        """y = F x (or the inverse, per the plan's direction).  `out` may be `x` (in place)."""
        ia, ib, oa, ob, out = self._io(x, out)
        check(lib.fft_execute(self._handle, ia, ib, oa, ob, _stream_handle(stream)), "fft_execute")
        return out

    def execute_no_alloc(self, x, out, stream=None):
        """execute() on the library's static scratch buffer (fft_execute_no_alloc):
        the call allocates nothing; `out` must be supplied."""
        if out is None:
            raise ValueError("execute_no_alloc needs a caller-supplied output")
        ia, ib, oa, ob, out = self._io(x, out)
        check(lib.fft_execute_no_alloc(self._handle, ia, ib, oa, ob, _stream_handle(stream)),
              "fft_execute_no_alloc")
        return out

    def backward(self, g, out=None, stream=None):
        """Adjoint of execute (unnormalised): F^H g for a forward plan, F g for an inverse plan."""
        ia, ib, oa, ob, out = self._io(g, out)
        check(lib.fft_execute_backward(self._handle, ia, ib, oa, ob, _stream_handle(stream)),
              "fft_execute_backward")
        return out

    __call__ = execute

    def close(self) -> None:
        if self._handle:
            check(lib.fft_plan_destroy(self._handle), "fft_plan_destroy")
            self._handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Plan(_PlanBase):
    """`batch` contiguous transforms of size n (a power of two up to 2^24), in
    FP32 (float32 / complex64 data) or FP64 (float64 / complex128 data)."""

    def __init__(self, n: int, batch: int = 1, layout: str = "interleaved", direction: str = "forward",
                 decomposition: str | None = None, precision: str = "fp32"):
        super().__init__(layout, direction, precision)
        h = ctypes.c_void_p()
        check(lib.fft_plan_create_ex(ctypes.byref(h), int(n), int(batch), _LAYOUTS[layout], _DIRS[direction],
                                     _PRECISIONS[precision],
                                     None if decomposition is None else decomposition.encode()),
              "fft_plan_create_ex")
        self._handle = h
        self.n = int(n)
        self.batch = int(batch)


class PlanND(_PlanBase):
    """`batch` arrays of shape `dims` (rank 1..3, row-major, powers of two; the
    last axis up to 2^24, the others up to 2^12), transformed over all axes."""

    def __init__(self, dims, batch: int = 1, layout: str = "interleaved", direction: str = "forward",
                 precision: str = "fp32"):
        super().__init__(layout, direction, precision)
        dims = [int(d) for d in dims]
        arr = (ctypes.c_int64 * len(dims))(*dims)
        h = ctypes.c_void_p()
        check(lib.fft_plan_create_nd(ctypes.byref(h), len(dims), arr, int(batch), _LAYOUTS[layout],
                                     _DIRS[direction], _PRECISIONS[precision]), "fft_plan_create_nd")
        self._handle = h
        self.dims = dims
        self.batch = int(batch)


class RaggedPlan(_PlanBase):
    """Transforms of the given power-of-two sizes packed back to back, one graph launch.

    `config` ("ragged:p8:g8:o0[:w64][:s13]") fixes the plan's configuration instead
    of the cached, default or autotuned one."""

    def __init__(self, sizes, layout: str = "interleaved", direction: str = "forward", config: str | None = None):
        super().__init__(layout, direction)
        sizes = [int(s) for s in sizes]
        arr = (ctypes.c_int64 * len(sizes))(*sizes)
        h = ctypes.c_void_p()
        check(lib.fft_plan_create_ragged_ex(ctypes.byref(h), arr, len(sizes), _LAYOUTS[layout], _DIRS[direction],
                                            None if config is None else config.encode()),
              "fft_plan_create_ragged_ex")
        self._handle = h
        self.sizes_list = sizes


class RealPlan(_PlanBase):
    """`batch` rows of n real values (n a power of two up to 2^24).

    direction "forward" is real-to-complex: real [batch][n] -> complex
    [batch][n/2 + 1] (X[k] for k = 0 .. n/2); "inverse" is complex-to-real,
    unnormalised (C2R(R2C(x)) = n x).  `layout` is the complex side's
    (interleaved complex tensor, or a (re, im) pair).  `backward` applies the
    adjoint (the vector-Jacobian product): R2C's maps a complex gradient to a
    real one, C2R's a real gradient to a complex one.
    """

    def __init__(self, n: int, batch: int = 1, layout: str = "interleaved", direction: str = "forward",
                 precision: str = "fp32", decomposition: str | None = None):
        super().__init__(layout, direction, precision)
        h = ctypes.c_void_p()
        check(lib.fft_plan_create_real(ctypes.byref(h), int(n), int(batch), _LAYOUTS[layout], _DIRS[direction],
                                       _PRECISIONS[precision],
                                       None if decomposition is None else decomposition.encode()),
              "fft_plan_create_real")
        self._handle = h
        self.n = int(n)
        self.batch = int(batch)
        self.half = self.n // 2 + 1

    def _check_real(self, t, count):
        rdt, _ = _DTYPES[self.precision]
        if t.dtype != rdt or not t.is_cuda or not t.is_contiguous():
            raise TypeError(f"real data must be a contiguous {rdt} CUDA tensor")
        if t.numel() != count:
            raise ValueError(f"expected {count} real values, got {t.numel()}")

    def _check_complex(self, x, count):
        rdt, cdt = _DTYPES[self.precision]
        if self.split:
            if not (isinstance(x, (tuple, list)) and len(x) == 2):
                raise TypeError(f"split layout takes (re, im) {rdt} tensors")
            for t in x:
                self._check_real(t, count)
            return _ptr(x[0]), _ptr(x[1])
        if x.dtype != cdt or not x.is_cuda or not x.is_contiguous():
            raise TypeError(f"interleaved data must be a contiguous {cdt} CUDA tensor")
        if x.numel() != count:
            raise ValueError(f"expected {count} complex values, got {x.numel()}")
        return _ptr(x), None

    def _run(self, fn, name, x, out, stream, real_in):
        rdt, cdt = _DTYPES[self.precision]
        nc = self.half * self.batch
        if real_in:
            self._check_real(x, self.n * self.batch)
            if out is None:
                shape = tuple(x.shape[:-1]) + (self.half,)
                if self.split:
                    out = (torch.empty(shape, dtype=rdt, device=x.device),
                           torch.empty(shape, dtype=rdt, device=x.device))
                else:
                    out = torch.empty(shape, dtype=cdt, device=x.device)
            oa, ob = self._check_complex(out, nc)
            ia, ib = _ptr(x), None
        else:
            ia, ib = self._check_complex(x, nc)
            if out is None:
                ref = x[0] if self.split else x
                out = torch.empty(tuple(ref.shape[:-1]) + (self.n,), dtype=rdt, device=ref.device)
            self._check_real(out, self.n * self.batch)
            oa, ob = _ptr(out), None
        check(fn(self._handle, ia, ib, oa, ob, _stream_handle(stream)), name)
        return out

    def execute(self, x, out=None, stream=None):
        return self._run(lib.fft_execute, "fft_execute", x, out, stream, self.direction == "forward")

    __call__ = execute

    def backward(self, g, out=None, stream=None):
        """Adjoint of execute: complex gradient -> real (R2C plan), real -> complex (C2R plan)."""
        return self._run(lib.fft_execute_backward, "fft_execute_backward", g, out, stream,
                         self.direction == "inverse")


_plan_cache: dict = {}


def _cached_plan(n: int, batch: int, layout: str, direction: str, precision: str = "fp32") -> Plan:
    key = (n, batch, layout, direction, precision, torch.cuda.current_device())
    p = _plan_cache.get(key)
    if p is None:
        p = Plan(n, batch, layout, direction, precision=precision)
        _plan_cache[key] = p
    return p


def _transform(x, direction: str):
    if isinstance(x, (tuple, list)):
        re, im = x
        n = re.shape[-1]
        plan = _cached_plan(n, re.numel() // n, "split", direction, _precision_of(re.dtype))
        return plan.execute((re.contiguous(), im.contiguous()))
    n = x.shape[-1]
    return _cached_plan(n, x.numel() // n, "interleaved", direction, _precision_of(x.dtype)).execute(x.contiguous())


def fft(x):
    """Forward FFT along the last axis (unnormalised)."""
    return _transform(x, "forward")


def _cached_real_plan(n: int, batch: int, direction: str, precision: str) -> RealPlan:
    key = ("real", n, batch, direction, precision, torch.cuda.current_device())
    p = _plan_cache.get(key)
    if p is None:
        p = RealPlan(n, batch, "interleaved", direction, precision)
        _plan_cache[key] = p
    return p


def _transform_nd(x, ndim: int, direction: str):
    if ndim < 1 or ndim > 3:
        raise ValueError("ndim must be 1, 2 or 3")
    split = isinstance(x, (tuple, list))
    ref = x[0] if split else x
    dims = tuple(int(d) for d in ref.shape[-ndim:])
    count = 1
    for d in dims:
        count *= d
    key = ("nd", dims, ref.numel() // count, "split" if split else "interleaved", direction,
           _precision_of(ref.dtype), torch.cuda.current_device())
    p = _plan_cache.get(key)
    if p is None:
        p = PlanND(dims, ref.numel() // count, key[3], direction, key[5])
        _plan_cache[key] = p
    return p.execute((x[0].contiguous(), x[1].contiguous()) if split else x.contiguous())


def fftn(x, ndim: int = 2):
    """Forward DFT over the last `ndim` axes (unnormalised)."""
    return _transform_nd(x, ndim, "forward")


def ifftn(x, ndim: int = 2):
    """Inverse DFT over the last `ndim` axes, unnormalised."""
    return _transform_nd(x, ndim, "inverse")


def rfft(x: torch.Tensor) -> torch.Tensor:
    """Real-to-complex FFT along the last axis: [..., n] real -> [..., n/2 + 1] complex."""
    n = x.shape[-1]
    x = x.contiguous()
    return _cached_real_plan(n, x.numel() // n, "forward", _precision_of(x.dtype)).execute(x)


def irfft(x: torch.Tensor, n: int) -> torch.Tensor:
    """Complex-to-real along the last axis, unnormalised: [..., n/2 + 1] -> [..., n]
    (irfft(rfft(x), n) = n x)."""
    if x.shape[-1] != n // 2 + 1:
        raise ValueError(f"last axis must hold n/2 + 1 = {n // 2 + 1} values")
    x = x.contiguous()
    return _cached_real_plan(n, x.numel() // (n // 2 + 1), "inverse", _precision_of(x.dtype)).execute(x)


def ifft(x):
    """Inverse FFT along the last axis, unnormalised (ifft(fft(x)) = N x)."""
    return _transform(x, "inverse")


class FFTFunction(torch.autograd.Function):
    """Differentiable forward FFT of split (re, im) tensors of shape [..., N].

    Forward: y = F x.  Backward: the vector-Jacobian product of the linear map
    F on the real pair (Re x, Im x) is F^H g, g = dL/dRe(y) + i dL/dIm(y),
    computed by the adjoint (unnormalised inverse) kernel.
    """

    @staticmethod
    def forward(ctx, re: torch.Tensor, im: torch.Tensor):
        n = re.shape[-1]
        plan = _cached_plan(n, re.numel() // n, "split", "forward", _precision_of(re.dtype))
        ctx.plan = plan
        yre, yim = plan.execute((re.contiguous(), im.contiguous()))
        return yre, yim

    @staticmethod
    def backward(ctx, gre: torch.Tensor, gim: torch.Tensor):
        if gre is None:
            gre = torch.zeros_like(gim)
        if gim is None:
            gim = torch.zeros_like(gre)
        xre, xim = ctx.plan.backward((gre.contiguous(), gim.contiguous()))
        return xre, xim


class _ComplexFFTFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, z: torch.Tensor):
        n = z.shape[-1]
        plan = _cached_plan(n, z.numel() // n, "interleaved", "forward", _precision_of(z.dtype))
        ctx.plan = plan
        return plan.execute(z.contiguous())

    @staticmethod
    def backward(ctx, g: torch.Tensor):
        return ctx.plan.backward(g.contiguous())


def fft_autograd(z: torch.Tensor) -> torch.Tensor:
    """Differentiable forward FFT of a complex64 or complex128 tensor [..., N]."""
    return _ComplexFFTFunction.apply(z)


class _RFFTFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x: torch.Tensor):
        n = x.shape[-1]
        plan = _cached_real_plan(n, x.numel() // n, "forward", _precision_of(x.dtype))
        ctx.plan = plan
        return plan.execute(x.contiguous())

    @staticmethod
    def backward(ctx, g: torch.Tensor):
        return ctx.plan.backward(g.contiguous())


class _IRFFTFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, z: torch.Tensor, n: int):
        plan = _cached_real_plan(n, z.numel() // (n // 2 + 1), "inverse", _precision_of(z.dtype))
        ctx.plan = plan
        return plan.execute(z.contiguous())

    @staticmethod
    def backward(ctx, g: torch.Tensor):
        return ctx.plan.backward(g.contiguous()), None


def rfft_autograd(x: torch.Tensor) -> torch.Tensor:
    """Differentiable R2C of a float32/float64 tensor [..., n] -> complex [..., n/2 + 1].
    The gradient of a real loss L is x_grad[m] = Re sum_k g[k] exp(+2 pi i k m / n),
    g = dL/dRe X + i dL/dIm X (torch's convention), from the adjoint kernel."""
    return _RFFTFunction.apply(x)


def irfft_autograd(z: torch.Tensor, n: int) -> torch.Tensor:
    """Differentiable C2R (unnormalised) of a complex tensor [..., n/2 + 1] -> real [..., n]."""
    if z.shape[-1] != n // 2 + 1:
        raise ValueError(f"last axis must hold n/2 + 1 = {n // 2 + 1} values")
    return _IRFFTFunction.apply(z, n)


def copy_device(src: torch.Tensor, dst: torch.Tensor, stream=None) -> None:
    """Streaming device copy with the library's copy kernel (HBM ceiling reference)."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() < nbytes:
        raise ValueError("destination too small")
    check(lib.fft_copy_device(_ptr(src), _ptr(dst), nbytes, _stream_handle(stream)), "fft_copy_device")


def query_decomposition(n: int, layout: str = "interleaved", precision: str = "fp32") -> dict:
    """Decomposition a plan for n would use, and the autotuner's candidates (host only)."""
    if precision not in _PRECISIONS:
        raise ValueError(f"precision must be one of {sorted(_PRECISIONS)}")
    buf = ctypes.create_string_buffer(1 << 16)
    check(lib.fft_query_decomposition(int(n), _LAYOUTS[layout], _PRECISIONS[precision], buf, len(buf)),
          "fft_query_decomposition")
    return json.loads(buf.value.decode())
