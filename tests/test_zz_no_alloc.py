"""The allocation-free advance (gs_fluid_advance_noalloc) against the
handle-based gs_fluid_advance, through the C ABI: the same kernels and
launch shape on the same input, so U, every step's dt and the final time
must be bit-identical.  Two calls in a row, the second on a smaller mesh, so
that the second call runs on the workspace contents the first one left;
both forms (FP64, FP32 pair), both boundary kinds; then the non-physical
flag of a bad state, and a following good call that must not see it.
"""
import ctypes
import sys

import numpy as np
import pytest

import workloads as wl
from paper_1812_07977_amd import F32, F64, OUTFLOW, PERIODIC, Fluid, _lib

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _noalloc(U, shape, bc, dtype, nsteps, t0, t_end, dt_log, t_out, flags):
    import torch
    nx, ny, nz = shape
    h = 1.0 / max(shape)
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    r = _lib.lib().gs_fluid_advance_noalloc(
        nx, ny, nz, h, h, h, 1.4, 0.5, bc, dtype, ctypes.c_void_p(U.data_ptr()), nsteps, t0,
        t_end, ctypes.c_void_p(dt_log.data_ptr()), ctypes.c_void_p(t_out.data_ptr()),
        ctypes.c_void_p(flags.data_ptr()), st)
    assert r == _lib.GS_OK, _lib.lib().gs_fluid_last_error(None).decode()


def _one_case(U0, shape, bc, dtype, nsteps, t0, t_end):
    import torch
    bcn = "periodic" if bc == PERIODIC else "outflow"
    dtn = "f32" if dtype == F32 else "f64"
    _say(f"case: noalloc {dtn} {shape} {bcn}, {nsteps} steps, t0 {t0}, t_end {t_end}")
    with Fluid(shape, bc=bcn, dtype=dtn) as F:
        Ua = F.state_from(U0)
        Ub = Ua.clone()
        F.time = t0
        log_a = torch.zeros(nsteps, dtype=torch.float64, device="cuda")
        F.advance(Ua, nsteps, t_end, log_a)
        ta = F.time
    log_b = torch.full((nsteps,), -1.0, dtype=torch.float64, device="cuda")
    t_b = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
    flags = torch.full((1,), 7, dtype=torch.int32, device="cuda")
    _noalloc(Ub, shape, bc, dtype, nsteps, t0, t_end, log_b, t_b, flags)
    torch.cuda.synchronize()
    assert torch.equal(Ua, Ub), (Ua - Ub).abs().max().item()
    assert torch.equal(log_a, log_b)
    assert t_b.item() == ta
    assert flags.item() == 0
    return Ub


@pytest.mark.parametrize("dtype", [F64, F32])
def test_two_calls_in_a_row_match_the_handle_path(dtype):
    # first call: 40 x 24 x 20 random plane, outflow, started at t0 = 0.25
    big = (40, 24, 20)
    _one_case(wl.random_plane(*big, seed=3), big, OUTFLOW, dtype, 6, 0.25, 0.0)
    # second call: smaller periodic mesh with an end time inside the run, so
    # the last steps are clipped and then stand still
    small = (17, 9, 5)
    U0 = wl.sine_wave(*small)
    _one_case(U0, small, PERIODIC, dtype, 5, 0.0, 0.004)


@pytest.mark.parametrize("dtype", [F64, F32])
def test_whole_tile_mesh_after_a_ragged_one(dtype):
    # 32 x 48 is whole for both tile shapes: the kernels without the
    # inactive-lane branch, on the workspace a ragged mesh used just before
    _one_case(wl.random_plane(37, 20, 9, seed=23), (37, 20, 9), OUTFLOW, dtype, 3, 0.0, 0.0)
    _one_case(wl.random_plane(32, 48, 10, seed=24, v=(0.2, -0.4, 0.3)), (32, 48, 10), PERIODIC,
              dtype, 4, 0.125, 0.0)


@pytest.mark.parametrize("dtype", [F64, F32])
def test_largest_mesh_that_fits_the_workspace(dtype):
    # 136^3 = 2,515,456 cells: 40 B per cell of the 2,516,582-cell workspace,
    # nearly all of it; periodic, so every ghost mapping wraps
    shape = (136, 136, 136)
    assert 136 ** 3 <= 2516582
    _one_case(wl.random_plane(*shape, seed=11, v=(0.2, 0.1, -0.3)), shape, PERIODIC, dtype, 3, 0.0, 0.0)


@pytest.mark.parametrize("dtype", [F64, F32])
def test_zero_steps_report_t0_and_leave_the_state(dtype):
    import torch
    shape = (14, 9, 7)
    U0 = wl.random_plane(*shape, seed=8)
    _say(f"case: noalloc zero steps, dtype {dtype}, {shape}")
    with Fluid(shape, bc="outflow", dtype="f32" if dtype == F32 else "f64") as F:
        U = F.state_from(U0)
    before = U.clone()
    log = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
    t = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
    flags = torch.full((1,), 7, dtype=torch.int32, device="cuda")
    _noalloc(U, shape, OUTFLOW, dtype, 0, 0.375, 0.0, log, t, flags)
    torch.cuda.synchronize()
    assert torch.equal(U, before)
    assert t.item() == 0.375
    assert flags.item() == 0
    assert log.item() == -1.0        # no step, no dt written


def test_nonphysical_flag_and_the_next_call():
    import torch
    shape = (12, 10, 8)
    U0 = wl.uniform(*shape)
    U0[4, 3, 4, 5] = -1.0            # negative total energy: negative pressure
    U = torch.from_numpy(U0).to("cuda")
    log = torch.zeros(1, dtype=torch.float64, device="cuda")
    t = torch.zeros(1, dtype=torch.float64, device="cuda")
    flags = torch.zeros(1, dtype=torch.int32, device="cuda")
    _say("case: noalloc non-physical 12x10x8, 1 step")
    _noalloc(U, shape, OUTFLOW, F64, 1, 0.0, 0.0, log, t, flags)
    torch.cuda.synchronize()
    assert flags.item() & 1
    # the next call starts from cleared device words
    _one_case(wl.uniform(*shape, v=(0.3, -0.2, 0.1)), shape, OUTFLOW, F64, 2, 0.0, 0.0)


def test_python_binding_marshals_to_the_same_call():
    import torch
    from paper_1812_07977_amd import advance_noalloc
    shape = (20, 16, 12)
    U0 = wl.random_plane(*shape, seed=5)
    with Fluid(shape, bc="outflow") as F:
        Ua = F.state_from(U0)
        F.advance(Ua, 3)
        F.sync()
    Ub = torch.from_numpy(U0).to("cuda")
    advance_noalloc(Ub, 3, bc="outflow")
    torch.cuda.synchronize()
    assert torch.equal(Ua, Ub)
