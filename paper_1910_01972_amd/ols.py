"""Python binding of the overlap-and-save library (argument marshalling only).

Paper: overlap-and-save convolution of a long signal with K short filters
(sec. 3.2), fused into one kernel per segment tile (sec. 3.4, Alg. 2).
PyTorch provides device memory and streams; all arithmetic runs in libols.so.
"""

from __future__ import annotations

import ctypes

import torch

from ._lib import OLSError, check, lib  # noqa: F401  (OLSError re-exported)


def _stream_handle(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _check_c64(t: torch.Tensor, name: str, ndim: int, dtype=torch.complex64) -> None:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on a GPU device")
    if t.dim() != ndim:
        raise ValueError(f"{name} must have {ndim} dimension(s)")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


# Stencils of the non-local stage, as (weights[J][T], left): the backward
# difference, and the cubic (four-point Lagrange) midpoint interpolation that
# writes each sample followed by the value half a sample later.
DIFFERENCE_STENCIL = ([[-1.0, 1.0]], 1)
MIDPOINT_CUBIC_STENCIL = ([[0.0, 1.0, 0.0, 0.0], [-1.0 / 16, 9.0 / 16, 9.0 / 16, -1.0 / 16]], 1)


class OLSPlan:
    """Filter bank h[K][M] (complex64, on the GPU) prepared for FFT length N.

    N = 0 lets the library choose.  The plan owns the filter spectra.
    derivative / power select the fused post-processing of sec. 4: the
    backward first difference of each output row (folded into the spectra)
    and the per-element power |y|^2 (float32 output).  A float32 filter bank
    makes a real-to-real (R2R) plan: the signal and the output are float32.
    stencil = (weights[J][T], left) adds the non-local stage of sec. 4 (see
    set_stencil).
    """

    def __init__(self, h: torch.Tensor, N: int = 0, stream=None, derivative: bool = False, power: bool = False,
                 stencil=None):
        self.real = isinstance(h, torch.Tensor) and h.dtype == torch.float32
        self._in_dtype = torch.float32 if self.real else torch.complex64
        _check_c64(h, "h", 2, self._in_dtype)
        self._handle = ctypes.c_void_p()
        self.K, self.M = int(h.shape[0]), int(h.shape[1])
        self.device = h.device
        self.post = (1 if derivative else 0) | (2 if power else 0)
        self.flags = self.post | (4 if self.real else 0)
        self._out_dtype = torch.float32 if (self.real or power) else torch.complex64
        with torch.cuda.device(h.device):
            check(lib().ols_plan_ex(ctypes.byref(self._handle), ctypes.c_void_p(h.data_ptr()), self.K, self.M, int(N),
                                    self.flags, _stream_handle(stream)), "ols_plan_ex")
        self._remember_filters(h)
        self.phases = 1
        if stencil is not None:
            self.set_stencil(*stencil)

    def set_stencil(self, weights, left: int = 0) -> None:
        """Non-local post-processing inside the forward kernel (sec. 4): every
        output sample n yields J values z[J n + j] = sum_d w[j][d + left] *
        y[n + d], d = -left .. T-1-left, from the segment's outputs staged on
        chip (zero history before 0, the convolution's tail past N_s).
        forward() then returns rows of J * N_s samples.  weights=None removes
        the stencil.  Resets the hop and the workgroups per CU."""
        if weights is None:
            check(lib().ols_plan_set_stencil(self.handle, 0, 0, 0, None), "ols_plan_set_stencil")
            self.phases = 1
            return
        rows = [[float(v) for v in row] for row in weights]
        J, T = len(rows), len(rows[0]) if rows else 0
        if J == 0 or T == 0 or any(len(r) != T for r in rows):
            raise ValueError("weights must be a non-empty J x T table")
        buf = (ctypes.c_float * (J * T))(*[v for r in rows for v in r])
        check(lib().ols_plan_set_stencil(self.handle, J, int(left), T - 1 - int(left), buf), "ols_plan_set_stencil")
        self.phases = J

    def _remember_filters(self, h: torch.Tensor) -> None:
        # a reference keeps the memory from being reused by another tensor, so
        # (address, version counter) identifies the contents the spectra hold
        self._src = h.detach()
        self._src_version = h._version

    def filters_current(self, h: torch.Tensor) -> bool:
        """True if the plan's spectra were computed from h's present contents
        (same memory, no in-place change since)."""
        src = getattr(self, "_src", None)
        return (src is not None and h.data_ptr() == src.data_ptr() and tuple(h.shape) == tuple(src.shape)
                and h._version == self._src_version)

    def ensure_filters(self, h: torch.Tensor, stream=None) -> None:
        """Recompute the spectra from h unless they already hold its contents."""
        if not self.filters_current(h):
            self.update_filters(h, stream=stream)

    def __del__(self):
        self.close()

    def close(self) -> None:
        h = getattr(self, "_handle", None)
        if h is not None and h.value:
            lib().ols_plan_destroy(h)
            self._handle = ctypes.c_void_p()

    @property
    def handle(self) -> ctypes.c_void_p:
        if not self._handle.value:
            raise RuntimeError("plan has been destroyed")
        return self._handle

    def info(self) -> dict:
        v = [ctypes.c_int32() for _ in range(5)]
        check(lib().ols_plan_get_info(self.handle, *[ctypes.byref(x) for x in v]), "ols_plan_get_info")
        return dict(zip(("N", "H", "D", "K", "M"), (x.value for x in v)))

    def launch(self) -> dict:
        v = [ctypes.c_int32() for _ in range(3)]
        check(lib().ols_plan_get_launch(self.handle, *[ctypes.byref(x) for x in v]), "ols_plan_get_launch")
        return dict(zip(("grid", "block", "cus"), (x.value for x in v)))

    def set_tiling(self, filters_per_unit: int = 0, workgroups_per_cu: int = 0) -> None:
        """Forward-kernel tiling (filters per work unit, persistent workgroups
        per CU); 0 restores the library's choice.  Results change at most by
        float rounding (filters per unit) or not at all (workgroups)."""
        check(lib().ols_plan_set_tiling(self.handle, int(filters_per_unit), int(workgroups_per_cu)),
              "ols_plan_set_tiling")

    def fft_length(self) -> int:
        N = ctypes.c_int32()
        check(lib().ols_plan_get_fft_length(self.handle, ctypes.byref(N)), "ols_plan_get_fft_length")
        return N.value

    def tiling(self) -> dict:
        v = [ctypes.c_int32() for _ in range(3)]
        check(lib().ols_plan_get_tiling(self.handle, *[ctypes.byref(x) for x in v]), "ols_plan_get_tiling")
        return dict(zip(("filters_per_unit", "workgroups_per_cu", "max_workgroups_per_cu"), (x.value for x in v)))

    def set_hop(self, H: int) -> None:
        check(lib().ols_plan_set_hop(self.handle, int(H)), "ols_plan_set_hop")

    def update_filters(self, h: torch.Tensor, stream=None) -> None:
        _check_c64(h, "h", 2, self._in_dtype)
        if tuple(h.shape) != (self.K, self.M):
            raise ValueError("filter bank shape must stay (K, M)")
        check(lib().ols_plan_update_filters(self.handle, ctypes.c_void_p(h.data_ptr()), _stream_handle(stream)),
              "ols_plan_update_filters")
        self._remember_filters(h)

    def spectra(self, stream=None) -> torch.Tensor:
        """Filter spectra in natural frequency order, FFT(pad h)/N, shape (K, N)."""
        N = self.info()["N"]
        out = torch.empty((self.K, N), dtype=torch.complex64, device=self.device)
        check(lib().ols_plan_get_spectra(self.handle, ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)),
              "ols_plan_get_spectra")
        return out

    def forward(self, s: torch.Tensor, y: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """y[K][N_s] = eq. (1) of s with every filter (zero history),
        post-processed as the plan's flags and stencil say ([K][J N_s] with a
        stencil of J phases)."""
        _check_c64(s, "s", 1, self._in_dtype)
        Ns = int(s.shape[0])
        out_dtype = self._out_dtype
        cols = self.phases * Ns  # J outputs per sample with a stencil
        if y is None:
            y = torch.empty((self.K, cols), dtype=out_dtype, device=s.device)
        else:
            if y.dtype != out_dtype or y.device.type != "cuda" or not y.is_contiguous():
                raise ValueError(f"y must be a contiguous {out_dtype} GPU tensor")
            if tuple(y.shape) != (self.K, cols):
                raise ValueError("y must have shape (K, J * N_s)")
        check(lib().ols_forward(self.handle, ctypes.c_void_p(s.data_ptr()), Ns, ctypes.c_void_p(y.data_ptr()),
                                _stream_handle(stream)), "ols_forward")
        return y

    __call__ = forward

    def reserve_backward(self) -> None:
        """Allocate the backward workspace now (later backward calls allocate nothing)."""
        check(lib().ols_plan_reserve_backward(self.handle), "ols_plan_reserve_backward")

    def backward(self, s: torch.Tensor, gy: torch.Tensor, need_ds: bool = True, need_dh: bool = True,
                 ds: torch.Tensor | None = None, dh: torch.Tensor | None = None, stream=None,
                 static_scratch: bool = False):
        """Adjoint of forward: (ds [N_s], dh [K][M]) for upstream gradient gy [K][N_s].

        static_scratch=True calls ols_backward_static: the library allocates
        nothing (pass ds/dh to avoid the allocations here too)."""
        _check_c64(s, "s", 1)
        _check_c64(gy, "gy", 2)
        Ns = int(s.shape[0])
        if tuple(gy.shape) != (self.K, Ns):
            raise ValueError("gy must have shape (K, N_s)")
        if need_ds and ds is None:
            ds = torch.empty(Ns, dtype=torch.complex64, device=s.device)
        elif need_ds:
            _check_c64(ds, "ds", 1)
            if int(ds.shape[0]) != Ns:
                raise ValueError("ds must have shape (N_s,)")
        if need_dh and dh is None:
            dh = torch.empty((self.K, self.M), dtype=torch.complex64, device=s.device)
        elif need_dh:
            _check_c64(dh, "dh", 2)
            if tuple(dh.shape) != (self.K, self.M):
                raise ValueError("dh must have shape (K, M)")
        p_ds = ctypes.c_void_p(ds.data_ptr()) if need_ds else ctypes.c_void_p()
        p_dh = ctypes.c_void_p(dh.data_ptr()) if need_dh else ctypes.c_void_p()
        name = "ols_backward_static" if static_scratch else "ols_backward"
        check(getattr(lib(), name)(self.handle, ctypes.c_void_p(s.data_ptr()), Ns, ctypes.c_void_p(gy.data_ptr()),
                                   p_ds, p_dh, _stream_handle(stream)), name)
        return (ds if need_ds else None), (dh if need_dh else None)


class OLSConvFunction(torch.autograd.Function):
    """y = s * h (eq. 1) for a bank of learnable filters; gradients by the
    library's adjoint kernel (segment spectra recomputed, nothing stored but
    the inputs)."""

    @staticmethod
    def forward(ctx, s, h, plan):
        plan.ensure_filters(h.detach().contiguous())
        y = plan.forward(s.detach().contiguous())
        ctx.save_for_backward(s, h)
        ctx.plan = plan
        return y

    @staticmethod
    def backward(ctx, gy):
        s, h = ctx.saved_tensors
        plan = ctx.plan
        # recomputed only if the plan has seen other filters since this forward
        plan.ensure_filters(h.detach().contiguous())
        ds, dh = plan.backward(s.detach().contiguous(), gy.contiguous(), need_ds=ctx.needs_input_grad[0],
                               need_dh=ctx.needs_input_grad[1])
        return ds, dh, None


class OLSConv(torch.nn.Module):
    """K learnable complex64 filters of length M applied to a long signal by
    overlap-and-save; output [K][N_s]."""

    def __init__(self, h_init: torch.Tensor, N: int = 0):
        super().__init__()
        _check_c64(h_init, "h_init", 2)
        self.h = torch.nn.Parameter(h_init.detach().clone())
        self.plan = OLSPlan(self.h.detach(), N=N)

    def forward(self, s: torch.Tensor) -> torch.Tensor:
        return OLSConvFunction.apply(s, self.h, self.plan)


class OLSBatch:
    """Many signals with their own filter banks in one persistent launch.

    items: sequence of (s [N_s] complex64, h [K][M] complex64[, N]) on the GPU;
    N = 0 (or omitted) lets the library choose, a callable fft_length(M, K)
    (e.g. the tuner's) may choose instead.  Outputs y_i [K_i][N_s_i] are
    allocated here (or passed as `outputs`) and rewritten by every run().
    """

    def __init__(self, items, outputs=None, fft_length=None, stream=None):
        from ._lib import BatchItem
        n = len(items)
        if n < 1:
            raise ValueError("empty batch")
        if outputs is not None and len(outputs) != n:
            raise ValueError(f"{len(outputs)} outputs for {n} items")
        arr = (BatchItem * n)()
        self.inputs, self.outputs = [], []
        for i, it in enumerate(items):
            s, h = it[0], it[1]
            N = int(it[2]) if len(it) > 2 else 0
            _check_c64(s, "s", 1)
            _check_c64(h, "h", 2)
            K, M = int(h.shape[0]), int(h.shape[1])
            if N == 0 and fft_length is not None:
                N = int(fft_length(M, K))
            y = outputs[i] if outputs is not None else torch.empty((K, s.shape[0]), dtype=torch.complex64,
                                                                   device=s.device)
            _check_c64(y, "y", 2)
            if tuple(y.shape) != (K, int(s.shape[0])):
                raise ValueError(f"output {i} must have shape (K, N_s) = ({K}, {int(s.shape[0])}), "
                                 f"got {tuple(y.shape)}")
            if y.device != s.device or h.device != s.device:
                raise ValueError(f"item {i}: s, h and y must be on the same device")
            self.inputs.append((s, h))
            self.outputs.append(y)
            arr[i] = BatchItem(s.data_ptr(), int(s.shape[0]), h.data_ptr(), K, M, N, y.data_ptr())
        nbytes = ctypes.c_size_t()
        check(lib().ols_batched_workspace_size(arr, n, ctypes.byref(nbytes)), "ols_batched_workspace_size")
        self.workspace_bytes = int(nbytes.value)
        self._handle = ctypes.c_void_p()
        check(lib().ols_batch_plan(ctypes.byref(self._handle), arr, n, _stream_handle(stream)), "ols_batch_plan")
        self.n = n

    def info(self) -> dict:
        u, g, n = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32()
        check(lib().ols_batch_get_info(self._handle, ctypes.byref(u), ctypes.byref(g), ctypes.byref(n)),
              "ols_batch_get_info")
        return {"units": u.value, "grid": g.value, "n": n.value}

    def item(self, i: int) -> dict:
        v = [ctypes.c_int32() for _ in range(3)]
        check(lib().ols_batch_get_item(self._handle, int(i), *[ctypes.byref(x) for x in v]), "ols_batch_get_item")
        return dict(zip(("N", "H", "D"), (x.value for x in v)))

    def run(self, stream=None):
        """One persistent launch over every item; returns the outputs."""
        check(lib().ols_batch_run(self._handle, _stream_handle(stream)), "ols_batch_run")
        return self.outputs

    def close(self) -> None:
        h = getattr(self, "_handle", None)
        if h is not None and h.value:
            lib().ols_batch_destroy(h)
            self._handle = ctypes.c_void_p()

    def __del__(self):
        self.close()


class OLSBatched:
    """The single-call batched path (ols_batched): the item table lives in
    device memory and the caller owns the workspace, so one call -- setup,
    filter spectra and the persistent forward -- allocates nothing and can be
    captured in a hipGraph; every call reads the items (and the filters)
    again.

    items: sequence of (s [N_s], h [K][M][, N]) complex64 GPU tensors, as for
    OLSBatch; outputs y_i [K_i][N_s_i] are allocated here or passed.
    workspace: a uint8 GPU tensor of at least workspace_bytes, or None to
    allocate one here.
    """

    def __init__(self, items, outputs=None, workspace=None):
        from ._lib import BatchItem
        n = len(items)
        if n < 1:
            raise ValueError("empty batch")
        if outputs is not None and len(outputs) != n:
            raise ValueError(f"{len(outputs)} outputs for {n} items")
        arr = (BatchItem * n)()
        self.inputs, self.outputs = [], []
        device = None
        for i, it in enumerate(items):
            s, h = it[0], it[1]
            N = int(it[2]) if len(it) > 2 else 0
            _check_c64(s, "s", 1)
            _check_c64(h, "h", 2)
            K = int(h.shape[0])
            y = outputs[i] if outputs is not None else torch.empty((K, s.shape[0]), dtype=torch.complex64,
                                                                   device=s.device)
            _check_c64(y, "y", 2)
            if tuple(y.shape) != (K, int(s.shape[0])):
                raise ValueError(f"output {i} must have shape (K, N_s) = ({K}, {int(s.shape[0])}), "
                                 f"got {tuple(y.shape)}")
            if y.device != s.device or h.device != s.device or (device is not None and s.device != device):
                raise ValueError(f"item {i}: all tensors must be on one device")
            device = s.device
            self.inputs.append((s, h))
            self.outputs.append(y)
            arr[i] = BatchItem(s.data_ptr(), int(s.shape[0]), h.data_ptr(), K, int(h.shape[1]), N, y.data_ptr())
        nbytes = ctypes.c_size_t()
        check(lib().ols_batched_workspace_size(arr, n, ctypes.byref(nbytes)), "ols_batched_workspace_size")
        self.workspace_bytes = int(nbytes.value)
        raw = bytes(arr)
        self.dev_items = torch.frombuffer(bytearray(raw), dtype=torch.uint8).to(device)
        if workspace is None:
            workspace = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=device)
        if workspace.dtype != torch.uint8 or workspace.device != device or not workspace.is_contiguous():
            raise ValueError("workspace must be a contiguous uint8 tensor on the items' device")
        if workspace.numel() < self.workspace_bytes:
            raise ValueError(f"workspace holds {workspace.numel()} bytes, {self.workspace_bytes} needed")
        self.workspace = workspace
        self.n = n

    def run(self, stream=None):
        """One ols_batched call (three launches, no allocation); returns the outputs."""
        check(lib().ols_batched(ctypes.c_void_p(self.dev_items.data_ptr()), self.n,
                                ctypes.c_void_p(self.workspace.data_ptr()), self.workspace.numel(),
                                _stream_handle(stream)), "ols_batched")
        return self.outputs

    def status(self, stream=None) -> tuple:
        """(status, first bad item or -1) of the last call's device-side checks."""
        st, bad = ctypes.c_int32(), ctypes.c_int32()
        check(lib().ols_batched_status(ctypes.c_void_p(self.workspace.data_ptr()), _stream_handle(stream),
                                       ctypes.byref(st), ctypes.byref(bad)), "ols_batched_status")
        return st.value, bad.value


def ols_conv(s: torch.Tensor, h: torch.Tensor, N: int = 0, stream=None, derivative: bool = False,
             power: bool = False, stencil=None) -> torch.Tensor:
    """One-shot overlap-and-save convolution: y[K][N_s] (post-processed as
    OLSPlan's flags and stencil select)."""
    plan = OLSPlan(h, N=N, stream=stream, derivative=derivative, power=power, stencil=stencil)
    try:
        return plan.forward(s, stream=stream)
    finally:
        # the forward is stream ordered; destroying the plan frees its spectra,
        # so wait for the kernel first
        (stream or torch.cuda.current_stream()).synchronize()
        plan.close()


def calibration_copy(dst: torch.Tensor, src: torch.Tensor, stream=None) -> None:
    """Plain device copy with the library's own kernel (HBM counter calibration)."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("size mismatch")
    check(lib().ols_calibration_copy(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()), nbytes,
                                     _stream_handle(stream)), "ols_calibration_copy")
