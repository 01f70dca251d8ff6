"""MI355X-native explicit RK2 finite-volume step of the 3D ideal-gas Euler
equations, the data-parallel hot path of the Riemann-problem example in
Budiardja & Cardall, "Targeting GPUs with OpenMP Directives on Summit"
(arXiv:1812.07977, Section 3, Algorithm 1), in FP64 or in a compensated FP32
form.

Python view of libgs_fluid.so: `Fluid` marshals torch tensors (device memory)
and the current stream into the C ABI; all arithmetic runs in the library's
HIP kernels.  An FP64 state is a float64 GPU tensor of shape (5, nz, ny, nx),
fields (rho, m_x, m_y, m_z, E), x fastest.  An FP32 state is a float32 GPU
tensor of shape (2, 5, nz, ny, nx): [0] the head, [1] the Kahan compensation;
it represents head - compensation.
"""
import ctypes

from . import _lib

__all__ = ["Fluid", "GSError", "NonPhysicalError", "OUTFLOW", "PERIODIC", "F64", "F32",
           "stream_probe", "advance_noalloc"]

OUTFLOW = _lib.GS_BC_OUTFLOW
PERIODIC = _lib.GS_BC_PERIODIC
F64 = _lib.GS_F64
F32 = _lib.GS_F32

_DTYPE_NAMES = {"f64": F64, "f32": F32, F64: F64, F32: F32}

_BC_NAMES = {"outflow": OUTFLOW, "periodic": PERIODIC, OUTFLOW: OUTFLOW, PERIODIC: PERIODIC}


class GSError(RuntimeError):
    """A non-OK status from the library."""

    def __init__(self, status, message):
        super().__init__(f"gs_fluid status {status}: {message}")
        self.status = status


class NonPhysicalError(GSError):
    """A state with non-positive or non-finite density or pressure was read."""


def _check(status, handle=None):
    if status == _lib.GS_OK:
        return
    msg = _lib.lib().gs_fluid_last_error(handle).decode(errors="replace")
    if status == _lib.GS_ERR_NONPHYSICAL:
        raise NonPhysicalError(status, msg)
    raise GSError(status, msg)


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class Fluid:
    """Solver for one mesh of nx*ny*nz proper cells.

    shape   (nx, ny, nz)
    spacing (dx, dy, dz); default 1/max(shape) in every direction
    gamma   ratio of specific heats (> 1)
    cfl     Courant number in (0, 1]
    bc      "outflow" or "periodic"
    dtype   "f64" or "f32" (the compensated FP32 form)
    stream  torch stream for all work (default: the current stream)
    """

    def __init__(self, shape, spacing=None, gamma=1.4, cfl=0.5, bc="outflow", dtype="f64",
                 stream=None):
        nx, ny, nz = (int(n) for n in shape)
        if spacing is None:
            h = 1.0 / max(nx, ny, nz)
            spacing = (h, h, h)
        if bc not in _BC_NAMES:
            raise ValueError(f"unknown boundary kind {bc!r}")
        if dtype not in _DTYPE_NAMES:
            raise ValueError(f"unknown dtype {dtype!r}")
        self.shape = (nx, ny, nz)
        self.spacing = tuple(float(s) for s in spacing)
        self.gamma = float(gamma)
        self.cfl = float(cfl)
        self.bc = _BC_NAMES[bc]
        self.dtype = _DTYPE_NAMES[dtype]
        L = _lib.lib()
        handle = ctypes.c_void_p()
        st = _stream_ptr(stream)
        _check(L.gs_fluid_create(nx, ny, nz, *self.spacing, self.gamma, self.cfl, self.bc,
                                 self.dtype, st, ctypes.byref(handle)))
        self._h = handle
        self._stream = st

    # -- marshalling ------------------------------------------------------------
    def state_shape(self):
        nx, ny, nz = self.shape
        return (5, nz, ny, nx) if self.dtype == F64 else (2, 5, nz, ny, nx)

    def _state_ptr(self, U):
        import torch
        if not isinstance(U, torch.Tensor):
            raise TypeError("U must be a torch tensor")
        want = torch.float64 if self.dtype == F64 else torch.float32
        if U.dtype != want or not U.is_cuda:
            raise TypeError(f"U must be a {want} tensor on the GPU")
        if tuple(U.shape) != self.state_shape() or not U.is_contiguous():
            raise ValueError(f"U must be contiguous with shape {self.state_shape()}")
        return ctypes.c_void_p(U.data_ptr())

    def state_from(self, U):
        """A device state of this solver's form from FP64 conserved data U
        (array or tensor of shape (5, nz, ny, nx)).  FP32 form: head = U
        rounded to FP32, compensation = (head - U) rounded to FP32, so that
        head - compensation keeps U to about 48 bits."""
        import torch
        u = torch.as_tensor(U, dtype=torch.float64)
        if tuple(u.shape) != self.state_shape()[-4:]:
            raise ValueError(f"U must have shape {self.state_shape()[-4:]}")
        u = u.to("cuda")
        if self.dtype == F64:
            return u.contiguous()
        head = u.to(torch.float32)
        comp = (head.to(torch.float64) - u).to(torch.float32)
        return torch.stack([head, comp]).contiguous()

    def to_f64(self, S):
        """FP64 values of a device state of this solver's form (for the FP32
        form head - compensation, exact in FP64)."""
        import torch
        if self.dtype == F64:
            return S
        return S[0].to(torch.float64) - S[1].to(torch.float64)

    def _handle(self):
        if self._h is None:
            raise RuntimeError("Fluid is closed")
        return self._h

    # -- the C ABI ----------------------------------------------------------------
    def dt(self, U):
        """CFL time step of state U (waits for the stream)."""
        out = ctypes.c_double()
        h = self._handle()
        _check(_lib.lib().gs_fluid_dt(h, self._state_ptr(U), ctypes.byref(out)), h)
        return out.value

    def dt_last(self):
        """CFL time step of the state the last advance or step_dt wrote, from
        the max its last step computed while writing it (no reduction;
        waits)."""
        out = ctypes.c_double()
        h = self._handle()
        _check(_lib.lib().gs_fluid_dt_last(h, ctypes.byref(out)), h)
        return out.value

    def step(self, U, dt):
        """One RK2 step of size dt, in place (asynchronous)."""
        h = self._handle()
        _check(_lib.lib().gs_fluid_step(h, self._state_ptr(U), float(dt)), h)

    def step_dt(self, U, dt):
        """One RK2 step of size dt in place, then the CFL time step of the
        new state from the max the step took while writing it (waits)."""
        out = ctypes.c_double()
        h = self._handle()
        _check(_lib.lib().gs_fluid_step_dt(h, self._state_ptr(U), float(dt), ctypes.byref(out)), h)
        return out.value

    def advance(self, U, nsteps, t_end=0.0, dt_log=None):
        """nsteps RK2 steps with device-computed dt (asynchronous).  dt_log:
        optional float64 GPU tensor of >= nsteps elements receiving each dt."""
        import torch
        h = self._handle()
        ptr = None
        if dt_log is not None:
            if (dt_log.dtype != torch.float64 or not dt_log.is_cuda or not dt_log.is_contiguous()
                    or dt_log.numel() < nsteps):
                raise ValueError("dt_log must be a contiguous float64 GPU tensor of >= nsteps")
            ptr = ctypes.c_void_p(dt_log.data_ptr())
        _check(_lib.lib().gs_fluid_advance(h, self._state_ptr(U), int(nsteps), float(t_end), ptr), h)

    def totals(self, U):
        """Conserved totals (5 FP64 sums over cells) of state U; waits."""
        out = (ctypes.c_double * 5)()
        h = self._handle()
        _check(_lib.lib().gs_fluid_totals(h, self._state_ptr(U), out), h)
        return [out[i] for i in range(5)]

    def sync(self):
        h = self._handle()
        _check(_lib.lib().gs_fluid_sync(h), h)

    @property
    def time(self):
        t = ctypes.c_double()
        h = self._handle()
        _check(_lib.lib().gs_fluid_get_time(h, ctypes.byref(t)), h)
        return t.value

    @time.setter
    def time(self, t):
        h = self._handle()
        _check(_lib.lib().gs_fluid_set_time(h, float(t)), h)

    def set_stream(self, stream):
        h = self._handle()
        st = _stream_ptr(stream)
        _check(_lib.lib().gs_fluid_set_stream(h, st), h)
        self._stream = st

    def set_launch(self, tile_y=0, chunk_z=0):
        h = self._handle()
        _check(_lib.lib().gs_fluid_set_launch(h, int(tile_y), int(chunk_z)), h)

    def profile(self, enable=True):
        h = self._handle()
        _check(_lib.lib().gs_fluid_profile(h, 1 if enable else 0), h)

    def kernel_ms(self, kernel):
        """(total ms, launches) of kernel 0 (substep 1), 1 (substep 2) or 2
        (dt reduction) since the last call; waits for the stream."""
        ms = ctypes.c_double()
        n = ctypes.c_int()
        h = self._handle()
        _check(_lib.lib().gs_fluid_kernel_ms(h, int(kernel), ctypes.byref(ms), ctypes.byref(n)), h)
        return ms.value, n.value

    @staticmethod
    def workspace_bytes(shape, dtype="f64"):
        nx, ny, nz = shape
        return _lib.lib().gs_fluid_workspace_bytes(nx, ny, nz, _DTYPE_NAMES[dtype])

    def close(self):
        """Wait for queued work, then release the handle."""
        if getattr(self, "_h", None) is not None:
            L = _lib.lib()
            L.gs_fluid_sync(self._h)
            L.gs_fluid_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def stream_probe(a, c, b=None, nontemporal=False, stream=None):
    """Queue the HBM streaming probe on `stream` (default: the current
    stream): c = a, or c = a + b when b is given.  a, b, c: contiguous
    float64 GPU tensors of the same even number of elements."""
    import torch
    ts = [a, c] + ([b] if b is not None else [])
    for t in ts:
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda \
                or not t.is_contiguous() or t.numel() != a.numel():
            raise ValueError("a, b, c must be contiguous float64 GPU tensors of one size")
    bp = ctypes.c_void_p(b.data_ptr()) if b is not None else None
    _check(_lib.lib().gs_fluid_stream_probe(ctypes.c_void_p(a.data_ptr()), bp,
                                            ctypes.c_void_p(c.data_ptr()), int(a.numel()),
                                            1 if nontemporal else 0, _stream_ptr(stream)))


def advance_noalloc(U, nsteps, spacing=None, gamma=1.4, cfl=0.5, bc="outflow", t0=0.0,
                    t_end=0.0, dt_log=None, t_out=None, flags_out=None, stream=None):
    """gs_fluid_advance_noalloc: nsteps device-dt RK2 steps of state U in
    place with the library's own workspace (no device allocation, no handle).
    U: float64 (5, nz, ny, nx) or float32 (2, 5, nz, ny, nx) contiguous GPU
    tensor; dt_log (float64, >= nsteps), t_out (float64, >= 1) and flags_out
    (int32, >= 1): optional GPU tensors written on the stream."""
    import torch
    if not isinstance(U, torch.Tensor) or not U.is_cuda or not U.is_contiguous():
        raise TypeError("U must be a contiguous GPU tensor")
    if U.dtype == torch.float64 and U.dim() == 4:
        dtype = F64
    elif U.dtype == torch.float32 and U.dim() == 5 and U.shape[0] == 2:
        dtype = F32
    else:
        raise ValueError("U must be float64 (5, nz, ny, nx) or float32 (2, 5, nz, ny, nx)")
    if U.shape[-4] != 5:
        raise ValueError("U must hold 5 fields")
    nz, ny, nx = (int(n) for n in U.shape[-3:])
    if spacing is None:
        h = 1.0 / max(nx, ny, nz)
        spacing = (h, h, h)
    if bc not in _BC_NAMES:
        raise ValueError(f"unknown boundary kind {bc!r}")

    def ptr(t, want, n, name):
        if t is None:
            return None
        if t.dtype != want or not t.is_cuda or not t.is_contiguous() or t.numel() < n:
            raise ValueError(f"{name} must be a contiguous {want} GPU tensor of >= {n} elements")
        return ctypes.c_void_p(t.data_ptr())

    _check(_lib.lib().gs_fluid_advance_noalloc(
        nx, ny, nz, *(float(s) for s in spacing), float(gamma), float(cfl), _BC_NAMES[bc], dtype,
        ctypes.c_void_p(U.data_ptr()), int(nsteps), float(t0), float(t_end),
        ptr(dt_log, torch.float64, nsteps, "dt_log"), ptr(t_out, torch.float64, 1, "t_out"),
        ptr(flags_out, torch.int32, 1, "flags_out"), _stream_ptr(stream)))
