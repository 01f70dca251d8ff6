"""Batched form: Python view of gs_batch_* in libgs_fluid.so
(include/gs_batch.h).  Many independent problems, each with its own mesh and
device time step, advanced together; all arithmetic runs in the library's
kernels."""
import ctypes

from . import _lib
from . import GSError, NonPhysicalError, OUTFLOW, PERIODIC, F64, F32, _stream_ptr  # noqa: F401

_BC = {"outflow": OUTFLOW, "periodic": PERIODIC, OUTFLOW: OUTFLOW, PERIODIC: PERIODIC}
_DT = {"f64": F64, "f32": F32, F64: F64, F32: F32}


def _check(status, handle=None):
    if status == _lib.GS_OK:
        return
    msg = _lib.lib().gs_batch_last_error(handle).decode(errors="replace")
    if status == _lib.GS_ERR_NONPHYSICAL:
        raise NonPhysicalError(status, msg)
    raise GSError(status, msg)


class Batch:
    """count problems with meshes dims[i] = (nx, ny, nz) and caller-owned
    device states (torch tensors in the layout of the dtype: FP64
    (5, nz, ny, nx), FP32 (2, 5, nz, ny, nx)); the tensors must stay alive
    and in place for the life of the batch."""

    def __init__(self, dims, states, gamma=1.4, cfl=0.5, bc="periodic", dtype="f64", stream=None):
        import torch
        if bc not in _BC or dtype not in _DT:
            raise ValueError("unknown boundary kind or dtype")
        self.dims = [tuple(int(v) for v in d) for d in dims]
        self.dtype = _DT[dtype]
        want = torch.float64 if self.dtype == F64 else torch.float32
        for (nx, ny, nz), S in zip(self.dims, states):
            shape = (5, nz, ny, nx) if self.dtype == F64 else (2, 5, nz, ny, nx)
            if not isinstance(S, torch.Tensor) or S.dtype != want or not S.is_cuda:
                raise TypeError(f"states must be {want} GPU tensors")
            if tuple(S.shape) != shape or not S.is_contiguous():
                raise ValueError(f"a state must be contiguous with shape {shape}")
        if len(states) != len(self.dims):
            raise ValueError("one state per problem")
        self.states = list(states)
        n = len(self.dims)
        flat = (ctypes.c_int * (3 * n))(*[v for d in self.dims for v in d])
        ptrs = (ctypes.c_void_p * n)(*[S.data_ptr() for S in self.states])
        h = ctypes.c_void_p()
        _check(_lib.lib().gs_batch_create(n, flat, float(gamma), float(cfl), _BC[bc], self.dtype,
                                          ptrs, _stream_ptr(stream), ctypes.byref(h)))
        self._h = h

    def _handle(self):
        if self._h is None:
            raise RuntimeError("Batch is closed")
        return self._h

    def set_launch(self, tile_y=0, chunk_z=0):
        h = self._handle()
        _check(_lib.lib().gs_batch_set_launch(h, int(tile_y), int(chunk_z)), h)

    def autotune(self, cache_path=None):
        """Pick the fastest launch shape (timed on scratch copies, or read
        from the cache file); returns (tile_y, chunk_z, from_cache)."""
        ty, kz, hit = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        h = self._handle()
        path = None if cache_path is None else str(cache_path).encode()
        _check(_lib.lib().gs_batch_autotune(h, path, ctypes.byref(ty), ctypes.byref(kz),
                                            ctypes.byref(hit)), h)
        return ty.value, kz.value, bool(hit.value)

    def advance(self, nsteps, t_end=0.0, graph=True):
        h = self._handle()
        _check(_lib.lib().gs_batch_advance(h, int(nsteps), float(t_end), 1 if graph else 0), h)

    def times(self):
        t = (ctypes.c_double * len(self.dims))()
        h = self._handle()
        _check(_lib.lib().gs_batch_times(h, t), h)
        return [t[i] for i in range(len(self.dims))]

    def sync(self):
        h = self._handle()
        _check(_lib.lib().gs_batch_sync(h), h)

    def close(self):
        if getattr(self, "_h", None) is not None:
            _lib.lib().gs_batch_sync(self._h)
            _lib.lib().gs_batch_destroy(self._h)
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
