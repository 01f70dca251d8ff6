"""Learned-correction form: Python view of the network kernels in
libgs_fluid.so (include/gs_cnn.h).

`CorrectionNet` marshals torch tensors into the C ABI; the network, its
training and the correction of a state run in the library's kernels.  A
coarse state is an FP32-form pair (torch float32, shape (2, 5, nz, ny, nx));
fine states are float64 (5, 2nz, 2ny, 2nx).
"""
import ctypes

import numpy as np

from . import _lib
from . import GSError, NonPhysicalError, OUTFLOW, PERIODIC, _stream_ptr  # noqa: F401

_BC = {"outflow": OUTFLOW, "periodic": PERIODIC, OUTFLOW: OUTFLOW, PERIODIC: PERIODIC}

HIDDEN = 32
FIELDS = 5
TAPS = 27
SHAPES = [(HIDDEN, FIELDS, 3, 3, 3), (HIDDEN,), (HIDDEN, HIDDEN, 3, 3, 3), (HIDDEN,),
          (FIELDS, HIDDEN, 3, 3, 3), (FIELDS,)]


def _check(status, handle=None):
    if status == _lib.GS_OK:
        return
    msg = _lib.lib().gs_cnn_last_error(handle).decode(errors="replace")
    if status == _lib.GS_ERR_NONPHYSICAL:
        raise NonPhysicalError(status, msg)
    raise GSError(status, msg)


def param_count():
    return _lib.lib().gs_cnn_param_count()


def split_params(flat):
    """The flat parameter vector as [W1, b1, W2, b2, W3, b3] views."""
    out, o = [], 0
    for s in SHAPES:
        n = int(np.prod(s))
        out.append(flat[o:o + n].reshape(s))
        o += n
    return out


def init_params(seed, out_scale=0.1):
    """He-normal weights (std sqrt(2 / fan_in)) for the ReLU layers, the
    output layer scaled by out_scale, zero biases; float32."""
    rng = np.random.default_rng(seed)
    parts = []
    for k, s in enumerate(SHAPES):
        if len(s) == 1:
            parts.append(np.zeros(s, dtype=np.float32))
            continue
        fan_in = s[1] * TAPS
        w = rng.standard_normal(s) * np.sqrt(2.0 / fan_in)
        if k == 4:
            w *= out_scale
        parts.append(w.astype(np.float32))
    return np.concatenate([p.ravel() for p in parts])


class CorrectionNet:
    """The 5 -> 32 -> 32 -> 5 correction network for an nx*ny*nz coarse mesh."""

    def __init__(self, shape, bc="periodic", gamma=1.4, stream=None):
        nx, ny, nz = (int(n) for n in shape)
        if bc not in _BC:
            raise ValueError(f"unknown boundary kind {bc!r}")
        self.shape = (nx, ny, nz)
        self.bc = _BC[bc]
        h = ctypes.c_void_p()
        _check(_lib.lib().gs_cnn_create(nx, ny, nz, self.bc, float(gamma), _stream_ptr(stream),
                                        ctypes.byref(h)))
        self._h = h

    def _handle(self):
        if self._h is None:
            raise RuntimeError("CorrectionNet is closed")
        return self._h

    def _ptr(self, t, dtype, shape):
        import torch
        if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dtype:
            raise TypeError(f"expected a {dtype} GPU tensor")
        if tuple(t.shape) != tuple(shape) or not t.is_contiguous():
            raise ValueError(f"expected a contiguous tensor of shape {shape}")
        return ctypes.c_void_p(t.data_ptr())

    def _coarse(self, U):
        import torch
        nx, ny, nz = self.shape
        return self._ptr(U, torch.float32, (2, 5, nz, ny, nx))

    def _field(self, y):
        import torch
        nx, ny, nz = self.shape
        return self._ptr(y, torch.float32, (5, nz, ny, nx))

    def _fine(self, F):
        import torch
        nx, ny, nz = self.shape
        return self._ptr(F, torch.float64, (5, 2 * nz, 2 * ny, 2 * nx))

    # -- parameters -----------------------------------------------------------
    def set_params(self, flat):
        a = np.ascontiguousarray(flat, dtype=np.float32)
        if a.size != param_count():
            raise ValueError("wrong parameter count")
        h = self._handle()
        _check(_lib.lib().gs_cnn_set_params(h, a.ctypes.data_as(ctypes.c_void_p)), h)

    def get_params(self):
        a = np.empty(param_count(), dtype=np.float32)
        h = self._handle()
        _check(_lib.lib().gs_cnn_get_params(h, a.ctypes.data_as(ctypes.c_void_p)), h)
        return a

    def set_norm(self, mu, sigma, tau):
        arrs = [np.ascontiguousarray(v, dtype=np.float64) for v in (mu, sigma, tau)]
        P = ctypes.POINTER(ctypes.c_double)
        h = self._handle()
        _check(_lib.lib().gs_cnn_set_norm(h, *[a.ctypes.data_as(P) for a in arrs]), h)
        self._norm = arrs

    # -- kernels --------------------------------------------------------------
    def forward(self, U):
        import torch
        nx, ny, nz = self.shape
        y = torch.empty((5, nz, ny, nx), dtype=torch.float32, device="cuda")
        h = self._handle()
        _check(_lib.lib().gs_cnn_forward(h, self._coarse(U), self._field(y)), h)
        return y

    def restrict(self, fine):
        import torch
        nx, ny, nz = self.shape
        U = torch.empty((2, 5, nz, ny, nx), dtype=torch.float32, device="cuda")
        h = self._handle()
        _check(_lib.lib().gs_cnn_restrict(h, self._fine(fine), self._coarse(U)), h)
        return U

    def make_target(self, fine, U):
        import torch
        nx, ny, nz = self.shape
        t = torch.empty((5, nz, ny, nx), dtype=torch.float32, device="cuda")
        h = self._handle()
        _check(_lib.lib().gs_cnn_make_target(h, self._fine(fine), self._coarse(U), self._field(t)), h)
        return t

    def gradients(self, U, target):
        g = np.empty(param_count(), dtype=np.float32)
        loss = ctypes.c_double()
        h = self._handle()
        _check(_lib.lib().gs_cnn_gradients(h, self._coarse(U), self._field(target),
                                           g.ctypes.data_as(ctypes.c_void_p), ctypes.byref(loss)), h)
        return loss.value, g

    def train_step(self, U, target, lr, want_loss=False):
        loss = ctypes.c_double()
        h = self._handle()
        _check(_lib.lib().gs_cnn_train_step(h, self._coarse(U), self._field(target), float(lr),
                                            ctypes.byref(loss) if want_loss else None), h)
        return loss.value if want_loss else None

    def correct(self, U):
        h = self._handle()
        _check(_lib.lib().gs_cnn_correct(h, self._coarse(U)), h)

    def counts(self):
        a, f = ctypes.c_int(), ctypes.c_int()
        h = self._handle()
        _check(_lib.lib().gs_cnn_counts(h, ctypes.byref(a), ctypes.byref(f)), h)
        return a.value, f.value

    def close(self):
        if getattr(self, "_h", None) is not None:
            import torch
            torch.cuda.synchronize()
            _lib.lib().gs_cnn_destroy(self._h)
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
