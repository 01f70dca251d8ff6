"""CPU FP64 oracle of the RK2 finite-volume Euler step (test infrastructure).

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
package.  It is a ctypes view of libgs_oracle.so (built from gs_oracle.c by
build.py) plus the exact Riemann solver in exact_riemann.py; it imports
nothing from the GPU library and the GPU library imports nothing from it.

Arrays are numpy float64 of shape (5, nz, ny, nx): conserved fields
(rho, m_x, m_y, m_z, E), x fastest.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# GS_ORACLE_LIB selects another build of the same source (the sanitizer
# build of build.py --sanitize)
LIB_PATH = os.environ.get("GS_ORACLE_LIB") or os.path.join(HERE, "libgs_oracle.so")

_lib = None

_D = ctypes.c_double
_I = ctypes.c_int
_P = ctypes.POINTER(ctypes.c_double)


def lib():
    """Load (building first if absent) the oracle's shared library."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _build
            _build.build()
        L = ctypes.CDLL(LIB_PATH)
        L.ora_c2p.argtypes = [_D, _P, _P]
        L.ora_p2c.argtypes = [_D, _P, _P]
        L.ora_minmod.argtypes = [_D, _D]
        L.ora_minmod.restype = _D
        L.ora_hll.argtypes = [_D, _I, _P, _P, _P, _P]
        L.ora_differences_line.argtypes = [_I, _P, _P]
        L.ora_reconstruction_line.argtypes = [_I, _P, _P, _P, _P, _P]
        L.ora_time_step.argtypes = [_I, _I, _I, _D, _D, _D, _D, _D, _P]
        L.ora_time_step.restype = _D
        L.ora_run.argtypes = [_I, _I, _I, _D, _D, _D, _D, _D, _I, _P, _I, _D, _P]
        L.ora_run.restype = _I
        L.ora_step.argtypes = [_I, _I, _I, _D, _D, _D, _D, _I, _P, _D]
        L.ora_step.restype = _I
        L.ora_step_window.argtypes = [_I, _I, _I, _D, _D, _D, _D, _P, _D,
                                      _I, _I, _I, _I, _I, _I, _P]
        L.ora_step_window.restype = _I
        L.ora_fill_ghosts.argtypes = [_I, _I, _I, _I, _P, _P]
        L.ora_fill_ghosts.restype = _I
        L.ora_threads.restype = _I
        L.ora_set_threads.argtypes = [_I]
        L.ora_set_threads.restype = None
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(_P)


def _vec5(x):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(5))
    return a


OUTFLOW, PERIODIC = 0, 1


def c2p(gamma, U):
    """Conserved -> primitive for one cell."""
    U = _vec5(U)
    W = np.empty(5)
    lib().ora_c2p(gamma, _ptr(U), _ptr(W))
    return W


def p2c(gamma, W):
    """Primitive -> conserved for one cell."""
    W = _vec5(W)
    U = np.empty(5)
    lib().ora_p2c(gamma, _ptr(W), _ptr(U))
    return U


def minmod(a, b):
    return lib().ora_minmod(float(a), float(b))


def hll(gamma, axis, WL, WR):
    """HLL flux through a face normal to `axis`; returns (F, (S_L, S_R))."""
    WL, WR = _vec5(WL), _vec5(WR)
    F = np.empty(5)
    S = np.empty(2)
    lib().ora_hll(gamma, int(axis), _ptr(WL), _ptr(WR), _ptr(F), _ptr(S))
    return F, (S[0], S[1])


def differences_line(V):
    """ComputeDifferences on one ghosted line V[-2 .. n+1] (length n+4)."""
    V = np.ascontiguousarray(V, dtype=np.float64)
    n = V.size - 4
    dV = np.full_like(V, np.nan)
    lib().ora_differences_line(n, _ptr(V), _ptr(dV))
    return dV


def reconstruction_line(V, dV):
    """ComputeReconstruction on one ghosted line; returns (sigma, V_L, V_R)."""
    V = np.ascontiguousarray(V, dtype=np.float64)
    dV = np.ascontiguousarray(dV, dtype=np.float64)
    n = V.size - 4
    sg, VL, VR = (np.full_like(V, np.nan) for _ in range(3))
    lib().ora_reconstruction_line(n, _ptr(V), _ptr(dV), _ptr(sg), _ptr(VL), _ptr(VR))
    return sg, VL, VR


def _shape(U):
    assert U.dtype == np.float64 and U.flags.c_contiguous and U.ndim == 4 and U.shape[0] == 5
    _, nz, ny, nx = U.shape
    return nx, ny, nz


def time_step(U, spacing, gamma, cfl):
    nx, ny, nz = _shape(U)
    return lib().ora_time_step(nx, ny, nz, *spacing, gamma, cfl, _ptr(U))


def run(U, spacing, gamma, cfl, bc, nsteps, t_end=0.0):
    """Advance U in place by up to nsteps RK2 steps (Algorithm 1), clipping
    the last step to reach t_end when t_end > 0.  Returns the TimeSteps."""
    nx, ny, nz = _shape(U)
    dts = np.zeros(max(nsteps, 1))
    taken = lib().ora_run(nx, ny, nz, *spacing, gamma, cfl, bc, _ptr(U),
                          nsteps, t_end, _ptr(dts))
    if taken < 0:
        raise ValueError("oracle rejected the arguments or ran out of memory")
    return dts[:taken]


def step(U, spacing, gamma, bc, dt):
    """One RK2 step in place with the given TimeStep."""
    nx, ny, nz = _shape(U)
    if lib().ora_step(nx, ny, nz, *spacing, gamma, bc, _ptr(U), dt) != 0:
        raise ValueError("oracle rejected the arguments or ran out of memory")


def step_window(U, spacing, gamma, dt, origin, size):
    """One periodic RK2 step evaluated on a window only: returns the window
    [5][wz][wy][wx] of what step() would produce.  origin = (i0, j0, k0)."""
    nx, ny, nz = _shape(U)
    wx, wy, wz = size
    out = np.empty((5, wz, wy, wx))
    r = lib().ora_step_window(nx, ny, nz, *spacing, gamma, _ptr(U), dt,
                              *origin, wx, wy, wz, _ptr(out))
    if r != 0:
        raise ValueError("oracle rejected the arguments or ran out of memory")
    return out


def fill_ghosts(U, bc):
    """GhostExchange alone: returns the ghosted array [5][nz+4][ny+4][nx+4]."""
    nx, ny, nz = _shape(U)
    G = np.empty((5, nz + 4, ny + 4, nx + 4))
    if lib().ora_fill_ghosts(nx, ny, nz, bc, _ptr(U), _ptr(G)) != 0:
        raise ValueError("oracle rejected the arguments")
    return G


def threads():
    return lib().ora_threads()


def set_threads(n):
    """Number of OpenMP threads for the mesh-level entry points."""
    lib().ora_set_threads(int(n))
