"""GPU parity: the HIP library against the CPU oracle on the same seeded
inputs, through the C ABI.

Bar: every conserved field within 1e-12 relative L-infinity of the oracle
(max |gpu - oracle| / max |oracle| per field, a zero field scaled by the
largest field), and every step's dt within 1e-14 relative.  The GPU divides
with a refined hardware reciprocal and takes square roots through a refined
reciprocal square root; both are accurate to a few ulp, and every operation
of the scheme is Lipschitz (minmod, min/max speeds, the clamped HLL
average), so differences stay at the rounding level.  Where a result must be
bit-identical (uniform states, tile shapes, repeated runs, the two dt paths)
the test says so.
"""
import math
import sys

import numpy as np
import pytest

import oracle
import workloads as wl
from tests.parity import (CFL, GAMMA, gpu_run_device_dt, gpu_run_host_dt, oracle_run, rel_linf,
                          to_cpu, to_gpu)

pytestmark = pytest.mark.gpu

TOL = 1e-12
DT_TOL = 1e-14


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _assert_parity(gpu, ref, tol=TOL, what=""):
    errs = rel_linf(gpu, ref)
    assert max(errs) <= tol, (what, errs)
    return errs


def _assert_dts(gdt, odt, tol=DT_TOL):
    assert len(gdt) == len(odt)
    rel = np.abs(np.asarray(gdt) - np.asarray(odt)) / np.abs(np.asarray(odt))
    _say(f"dt: max relative difference {float(np.max(rel)):.3e} over {len(rel)} steps (bound {tol:g})")
    assert np.all(rel <= tol), rel


# ---------------------------------------------------------------------------
# the small configuration: 32^3 diagonal Riemann problem, outflow, 20 steps
# ---------------------------------------------------------------------------

def test_diagonal_32_host_dt_matches_oracle():
    _say("case: diagonal_riemann 32^3 outflow, 20 steps, host dt")
    U0 = wl.diagonal_riemann(32)
    ref, odt = oracle_run(U0, "outflow", 20)
    out, gdt = gpu_run_host_dt(U0, "outflow", 20)
    _assert_dts(gdt, odt)
    _assert_parity(out, ref)


def test_diagonal_32_device_dt_matches_host_dt_bitwise():
    _say("case: diagonal_riemann 32^3 outflow, 20 steps, device dt")
    U0 = wl.diagonal_riemann(32)
    a, adt = gpu_run_host_dt(U0, "outflow", 20)
    b, bdt, t = gpu_run_device_dt(U0, "outflow", 20)
    assert np.array_equal(adt, bdt)
    assert np.array_equal(a, b)
    assert t == pytest.approx(math.fsum(bdt), rel=1e-15)


# ---------------------------------------------------------------------------
# periodic cubes with both workloads of the per-GPU configuration, small
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("case", ["sine", "plane0", "plane1"])
def test_periodic_64_matches_oracle(case):
    n, steps = 64, 100
    _say(f"case: {case} {n}^3 periodic, {steps} steps, device dt")
    U0 = wl.sine_wave(n, n, n) if case == "sine" else wl.random_plane(n, n, n, seed=int(case[-1]))
    ref, odt = oracle_run(U0, "periodic", steps)
    out, gdt, _ = gpu_run_device_dt(U0, "periodic", steps)
    _assert_dts(gdt, odt)
    _assert_parity(out, ref)


# ---------------------------------------------------------------------------
# ragged and odd meshes, both boundary kinds, several launch shapes
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("bc", ["outflow", "periodic"])
@pytest.mark.parametrize("shape", [(37, 20, 9), (5, 33, 17), (1, 1, 7), (64, 1, 1), (2, 2, 2),
                                   (17, 16, 40)])
def test_ragged_meshes_match_oracle(shape, bc):
    nx, ny, nz = shape
    _say(f"case: random_plane {shape} {bc}, 6 steps, host dt")
    U0 = wl.random_plane(nx, ny, nz, seed=7)
    ref, odt = oracle_run(U0, bc, 6)
    out, gdt = gpu_run_host_dt(U0, bc, 6)
    _assert_dts(gdt, odt)
    _assert_parity(out, ref)


@pytest.mark.parametrize("bc", ["outflow", "periodic"])
@pytest.mark.parametrize("shape,launch", [((16, 16, 1), (16, 0)), ((32, 16, 3), (16, 0)),
                                          ((32, 8, 2), (8, 0)), ((64, 16, 5), (8, 2))])
def test_small_whole_tile_meshes_match_oracle(shape, launch, bc):
    # one or two whole tiles and one to five planes: the whole-tile kernels
    # with every ghost plane and column mapped back into the mesh
    nx, ny, nz = shape
    _say(f"case: random_plane {shape} {bc}, 6 steps, device dt, launch {launch}")
    U0 = wl.random_plane(nx, ny, nz, seed=19, v=(0.3, 0.2, -0.4))
    ref, odt = oracle_run(U0, bc, 6)
    out, gdt, _ = gpu_run_device_dt(U0, bc, 6, launch=launch)
    _assert_dts(gdt, odt)
    _assert_parity(out, ref)


@pytest.mark.parametrize("bc", ["outflow", "periodic"])
@pytest.mark.parametrize("sign", [1, -1])
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_supersonic_flow_takes_the_one_sided_hll_branches(axis, sign, bc):
    # Mach 3 along one axis: on every face normal to it both signal speeds
    # have the flow's sign, so the oracle returns F_L (sign +1) or F_R (sign
    # -1) through its branches, while the GPU evaluates the clamped single
    # expression with S_L or S_R clamped to 0
    _say(f"case: supersonic contact axis {axis} sign {sign} {bc}, 8 steps, host dt")
    U0 = wl.supersonic_contact(24, 20, 18, axis, sign)
    ref, odt = oracle_run(U0, bc, 8)
    out, gdt = gpu_run_host_dt(U0, bc, 8)
    _assert_dts(gdt, odt)
    _assert_parity(out, ref)
    # the contact moved downstream: the first face column upstream of the
    # jump changed, the state is not the initial one
    assert not np.array_equal(out, U0)


@pytest.mark.parametrize("launch", [(16, 0), (8, 0), (16, 1), (8, 3), (16, 64), (8, 7)])
@pytest.mark.parametrize("boost", [(0.0, 0.0, 0.0), (0.9, -0.6, 0.4)])
def test_launch_shapes_give_identical_results(launch, boost):
    # with a background velocity the kinetic energy is a large part of E, so
    # a tile-edge face evaluated with a different rounding than the same face
    # inside a tile would show up in the last bits
    _say(f"case: random_plane (40,24,20) v={boost} outflow, 5 steps, launch {launch}")
    U0 = wl.random_plane(40, 24, 20, seed=11, v=boost)
    base, bdt = gpu_run_host_dt(U0, "outflow", 5, launch=(16, 0))
    out, odt = gpu_run_host_dt(U0, "outflow", 5, launch=launch)
    assert np.array_equal(bdt, odt)
    assert np.array_equal(base, out)


@pytest.mark.parametrize("bc", ["outflow", "periodic"])
def test_whole_tile_kernels_match_the_ragged_tile_kernels(bc):
    # 48 x 32 is a whole number of 16 x 16 tiles (the kernels without an
    # inactive-lane branch) but not of 32 x 8 tiles (the kernels with it):
    # the two launches must agree bit for bit, in both substeps, on both
    # the device-dt and the host-dt path
    _say(f"case: random_plane (48,32,12) {bc}, 6 steps, 16x16 whole tiles vs 32x8 ragged")
    U0 = wl.random_plane(48, 32, 12, seed=17, v=(0.5, -0.3, 0.2))
    a, adt, ta = gpu_run_device_dt(U0, bc, 6, launch=(16, 0))
    b, bdt, tb = gpu_run_device_dt(U0, bc, 6, launch=(8, 0))
    assert np.array_equal(adt, bdt) and ta == tb
    assert np.array_equal(a, b)
    c, cdt = gpu_run_host_dt(U0, bc, 6, launch=(16, 0))
    d, ddt = gpu_run_host_dt(U0, bc, 6, launch=(8, 0))
    assert np.array_equal(cdt, ddt)
    assert np.array_equal(c, d)
    ref, odt = oracle_run(U0, bc, 6)
    _assert_dts(adt, odt)
    _assert_parity(a, ref)


def test_repeated_runs_are_bitwise_identical():
    _say("case: random_plane 48^3 periodic, 10 steps, twice")
    U0 = wl.random_plane(48, 48, 48, seed=2)
    a, adt, _ = gpu_run_device_dt(U0, "periodic", 10)
    b, bdt, _ = gpu_run_device_dt(U0, "periodic", 10)
    assert np.array_equal(adt, bdt)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_aligned_sod_to_end_time_matches_oracle(axis):
    _say(f"case: sod axis {axis}, 64 x 4 x 4, t_end 0.1, device dt")
    U0 = wl.sod(64, axis, 4)
    ref, odt = oracle_run(U0, "outflow", 10000, t_end=0.1)
    out, gdt, t = gpu_run_device_dt(U0, "outflow", len(odt) + 3, t_end=0.1)
    # steps after the end time are exact no-ops (dt = 0)
    assert np.all(gdt[len(odt):] == 0.0)
    # the last step is clipped to the end time: its dt is the end time minus
    # the accumulated time, a difference of nearly equal numbers, so it is
    # compared in absolute terms (a few units in the last place of t_end)
    _assert_dts(gdt[:len(odt) - 1], odt[:-1])
    assert abs(gdt[len(odt) - 1] - odt[-1]) <= 1e-15
    assert t == pytest.approx(0.1, abs=1e-15)
    _assert_parity(out, ref)


@pytest.mark.parametrize("bc", ["outflow", "periodic"])
def test_uniform_state_stays_bitwise_uniform(bc):
    _say(f"case: uniform (19, 18, 21) {bc}")
    U0 = wl.uniform(19, 18, 21, rho=0.7, v=(0.3, -1.1, 0.25), p=2.5)
    out, _ = gpu_run_host_dt(U0, bc, 5)
    assert np.array_equal(out, U0)


def test_periodic_conservation_on_gpu():
    _say("case: random_plane 48^3 periodic conservation, 30 steps")
    U0 = wl.random_plane(48, 48, 48, seed=4)
    U0[1] += 0.3 * U0[0]
    U0[4] += 0.045 * U0[0]
    out, _, _ = gpu_run_device_dt(U0, "periodic", 30)
    totals = [math.fsum(U0[f].ravel()) for f in range(5)]
    scale = max(abs(t) for t in totals)
    for f in range(5):
        assert abs(math.fsum(out[f].ravel()) - totals[f]) <= 1e-13 * scale, f


# ---------------------------------------------------------------------------
# error paths (forced from the host; every kernel exits normally)
# ---------------------------------------------------------------------------

def test_nonphysical_input_is_reported_once():
    from paper_1812_07977_amd import Fluid, NonPhysicalError
    _say("case: negative density in one cell")
    U0 = wl.uniform(16, 16, 16)
    U0[0, 3, 4, 5] = -1.0
    U = to_gpu(U0)
    with Fluid((16, 16, 16)) as F:
        with pytest.raises(NonPhysicalError):
            F.dt(U)
        F.sync()  # reported once, then cleared
        F.step(U, 1e-3)
        with pytest.raises(NonPhysicalError):
            F.sync()


def test_nan_energy_is_reported():
    from paper_1812_07977_amd import Fluid, NonPhysicalError
    _say("case: NaN energy in one cell")
    U0 = wl.uniform(8, 9, 10)
    U0[4, 9, 8, 7] = np.nan
    U = to_gpu(U0)
    with Fluid((8, 9, 10), bc="periodic") as F:
        with pytest.raises(NonPhysicalError):
            F.dt(U)


def test_bad_arguments_raise_before_launch():
    import torch
    from paper_1812_07977_amd import Fluid, GSError
    with Fluid((8, 8, 8)) as F:
        U = to_gpu(wl.uniform(8, 8, 8))
        with pytest.raises(GSError):
            F.step(U, -1.0)
        with pytest.raises(GSError):
            F.step(U, float("nan"))
        with pytest.raises(ValueError):
            F.step(torch.zeros((5, 8, 8, 9), dtype=torch.float64, device="cuda"), 0.1)
        with pytest.raises(TypeError):
            F.step(U.float(), 0.1)
        with pytest.raises(GSError):
            F.set_launch(tile_y=5)
        F.sync()


def test_time_set_and_read():
    from paper_1812_07977_amd import Fluid
    U = to_gpu(wl.uniform(8, 8, 8))
    with Fluid((8, 8, 8)) as F:
        F.time = 0.25
        assert F.time == 0.25
        F.step(U, 0.125)
        assert F.time == 0.375


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_zero_steps_change_nothing(dtype):
    import torch
    from paper_1812_07977_amd import Fluid
    shape = (19, 13, 11)
    U0 = wl.random_plane(*shape, seed=21)
    _say(f"case: zero-step advance {dtype} {shape} outflow")
    with Fluid(shape, bc="outflow", dtype=dtype) as F:
        U = F.state_from(U0)
        before = U.clone()
        F.time = 0.125
        F.advance(U, 0)
        F.sync()
        assert torch.equal(U, before)
        assert F.time == 0.125
        # the call left the handle as it was: two steps now equal two steps
        # on a fresh handle from the same state and time
        F.advance(U, 2)
        ta = F.time
    with Fluid(shape, bc="outflow", dtype=dtype) as G:
        V = G.state_from(U0)
        G.time = 0.125
        G.advance(V, 2)
        tb = G.time
    assert torch.equal(U, V)
    assert ta == tb


def test_profiling_counts_launches():
    from paper_1812_07977_amd import Fluid
    U = to_gpu(wl.sine_wave(32, 32, 32))
    with Fluid((32, 32, 32), bc="periodic") as F:
        F.profile(True)
        F.advance(U, 3)
        ms1, n1 = F.kernel_ms(0)
        ms2, n2 = F.kernel_ms(1)
        ms3, n3 = F.kernel_ms(2)
        assert (n1, n2, n3) == (3, 3, 1)
        assert ms1 > 0 and ms2 > 0 and ms3 > 0
        assert F.kernel_ms(0) == (0.0, 0)


# ---------------------------------------------------------------------------
# full sizes, in the launch configuration of the benchmark (device dt)
# ---------------------------------------------------------------------------

def test_full_256_sine_matches_oracle_everywhere():
    n, steps = 256, 10
    _say(f"case: sine {n}^3 periodic, {steps} steps, full comparison")
    U0 = wl.sine_wave(n, n, n)
    out, gdt, _ = gpu_run_device_dt(U0, "periodic", steps)
    ref, odt = oracle_run(U0, "periodic", steps)
    _assert_dts(gdt, odt)
    _assert_parity(out, ref)


@pytest.mark.parametrize("case", ["sine", "plane0"])
def test_full_512_sampled_windows_match_oracle(case):
    n = 512
    _say(f"case: {case} {n}^3 periodic, 1 step, sampled windows")
    U0 = wl.sine_wave(n, n, n) if case == "sine" else wl.random_plane(n, n, n, seed=0)
    out, gdt, _ = gpu_run_device_dt(U0, "periodic", 1)
    h = 1.0 / n
    dt = oracle.time_step(U0, (h, h, h), GAMMA, CFL)
    _assert_dts(gdt, [dt])
    rng = np.random.default_rng(123)
    origins = [(0, 0, 0), (n - 3, n - 2, n - 4), (255, 256, 250)]
    origins += [tuple(int(v) for v in rng.integers(0, n, 3)) for _ in range(5)]
    size = (6, 5, 4)
    scale = np.max(np.abs(U0), axis=(1, 2, 3))
    for o in origins:
        win = oracle.step_window(U0, (h, h, h), GAMMA, dt, o, size)
        ii = [(o[0] + i) % n for i in range(size[0])]
        jj = [(o[1] + j) % n for j in range(size[1])]
        kk = [(o[2] + k) % n for k in range(size[2])]
        g = out[:, kk][:, :, jj][:, :, :, ii]
        for f in range(5):
            s = scale[f] if scale[f] > 0 else np.max(scale)
            assert np.max(np.abs(g[f] - win[f])) / s <= TOL, (o, f)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_largest_plane_matches_the_tiled_small_mesh(dtype):
    # The create call accepts planes of fewer than 2^29 cells: the FP64
    # kernels address a field plane through a buffer resource, whose range
    # ends at byte 2^32 - 1.  This mesh has planes of 2^29 - 1 = 233 x 1103 x
    # 2089 cells (256999 x 2089), so the last cell of an FP64 plane starts at
    # byte 2^32 - 16.  A periodic state that repeats one 233 x 2089 x 2 block
    # along x gives, cell for cell and bit for bit, that block's own result
    # on its 233 x 2089 x 2 periodic mesh with the same cell widths (every
    # stencil sees the same values and dt is the same maximum); the small
    # FP64 mesh is checked against the oracle.  The FP32 form (global
    # addressing) runs the same comparison of its pairs.  About 95 GB of
    # device memory, compared on the device.
    import torch
    from paper_1812_07977_amd import Fluid
    bx, ny, nz, steps = 233, 2089, 2, 2
    reps = 1103
    NX = bx * reps
    assert NX * ny == (1 << 29) - 1
    h = 1.0 / ny
    _say(f"case: {dtype} plane1 block {bx} x {ny} x {nz} tiled to {NX} x {ny} x {nz}, periodic, {steps} steps")
    U0 = wl.random_plane(bx, ny, nz, seed=1, v=(0.3, -0.2, 0.1))
    kw = dict(spacing=(h, h, h), gamma=GAMMA, cfl=CFL, bc="periodic", dtype=dtype)
    small_log = torch.zeros(steps, dtype=torch.float64, device="cuda")
    with Fluid((bx, ny, nz), **kw) as F:
        S = F.state_from(U0)
        F.advance(S, steps, 0.0, small_log)
        F.sync()
    if dtype == "f64":
        ref, odt = oracle_run(U0, "periodic", steps, spacing=(h, h, h))
        _assert_dts(small_log.cpu().numpy(), odt)
        _assert_parity(S.cpu().numpy(), ref)
    big_log = torch.zeros(steps, dtype=torch.float64, device="cuda")
    with Fluid((bx, ny, nz), **kw) as F:
        B = F.state_from(U0)
    reps_shape = (1,) * (B.dim() - 1) + (reps,)
    B = B.repeat(*reps_shape).contiguous()
    try:
        with Fluid((NX, ny, nz), **kw) as F:
            F.advance(B, steps, 0.0, big_log)
            F.sync()
        assert torch.equal(big_log, small_log)
        lead = tuple(B.shape[:-1])
        tiles = B.view(*lead, reps, bx)
        assert torch.eq(tiles, S.view(*lead, 1, bx)).all().item()
        # the highest offsets of the plane, separately
        assert torch.equal(B[..., -bx:], S)
    finally:
        del B
        torch.cuda.empty_cache()


def test_full_512_three_steps_match_oracle_everywhere():
    # the full per-GPU size, every cell (the oracle holds about 66 GB of
    # ghosted arrays on the host)
    n, steps = 512, 3
    _say(f"case: plane0 {n}^3 periodic, {steps} steps, full comparison")
    U0 = wl.random_plane(n, n, n, seed=0)
    out, gdt, _ = gpu_run_device_dt(U0, "periodic", steps)
    ref, odt = oracle_run(U0, "periodic", steps)
    del U0
    _assert_dts(gdt, odt)
    _assert_parity(out, ref)


def test_full_512_random_plane_conservation():
    n = 512
    _say(f"case: plane1 {n}^3 periodic, 3 steps, conservation")
    U0 = wl.random_plane(n, n, n, seed=1)
    import torch
    U = to_gpu(U0)
    before = U.sum(dim=(1, 2, 3)).cpu().numpy()
    from paper_1812_07977_amd import Fluid
    with Fluid((n, n, n), bc="periodic") as F:
        F.advance(U, 3)
        F.sync()
    after = U.sum(dim=(1, 2, 3)).cpu().numpy()
    scale = np.max(np.abs(before))
    assert np.max(np.abs(after - before)) <= 1e-12 * scale


def test_checkpoint_restart_is_bitwise_identical():
    # The caller owns U, so a checkpoint is (U, t): stepping N, saving,
    # restoring into a fresh handle and stepping M equals stepping N + M.
    import torch
    from paper_1812_07977_amd import Fluid
    _say("case: random_plane 40^3 periodic, 7 + 5 steps vs 12, device dt")
    U0 = wl.random_plane(40, 40, 40, seed=6)
    n, m = 7, 5
    A = to_gpu(U0)
    logA = torch.zeros(n + m, dtype=torch.float64, device="cuda")
    with Fluid((40, 40, 40), bc="periodic") as F:
        F.advance(A, n + m, 0.0, logA)
        tA = F.time
    B = to_gpu(U0)
    log1 = torch.zeros(n, dtype=torch.float64, device="cuda")
    with Fluid((40, 40, 40), bc="periodic") as F:
        F.advance(B, n, 0.0, log1)
        t_saved = F.time
    saved = to_cpu(B).copy()
    C = to_gpu(saved)
    log2 = torch.zeros(m, dtype=torch.float64, device="cuda")
    with Fluid((40, 40, 40), bc="periodic") as F:
        F.time = t_saved
        F.advance(C, m, 0.0, log2)
        tC = F.time
    assert np.array_equal(to_cpu(C), to_cpu(A))
    assert np.array_equal(np.concatenate([log1.cpu().numpy(), log2.cpu().numpy()]), logA.cpu().numpy())
    assert tC == tA


def test_host_dt_and_device_dt_interleave():
    # Mixing the two ways of driving the step on one handle gives the same
    # state as either alone.
    from paper_1812_07977_amd import Fluid
    _say("case: diagonal_riemann 32^3, step/advance interleaved")
    U0 = wl.diagonal_riemann(32)
    ref, rdt = gpu_run_host_dt(U0, "outflow", 6)
    U = to_gpu(U0)
    with Fluid((32, 32, 32), bc="outflow") as F:
        for _ in range(2):
            F.step(U, F.dt(U))
        F.advance(U, 2)
        for _ in range(2):
            F.step(U, F.dt(U))
        F.sync()
    assert np.array_equal(to_cpu(U), ref)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_dt_last_equals_a_reduction_of_the_state_written(dtype):
    # the max fused into a step's second substep gives the time step of the
    # state it wrote exactly as a reduction pass over that state does
    from paper_1812_07977_amd import GSError, Fluid
    _say(f"case: dt_last, {dtype} 40x24x20 random plane outflow, 5 steps")
    U0 = wl.random_plane(40, 24, 20, seed=2, v=(0.4, -0.2, 0.1))
    with Fluid((40, 24, 20), bc="outflow", dtype=dtype) as F:
        S = F.state_from(U0)
        with pytest.raises(GSError):
            F.dt_last()                      # nothing stepped yet
        dt = F.dt(S)
        for _ in range(5):
            dt = F.step_dt(S, dt)
            assert dt == F.dt(S) == F.dt_last()
        F.advance(S, 3)
        assert F.dt_last() == F.dt(S)
        F.step(S, dt)
        with pytest.raises(GSError):
            F.dt_last()                      # a plain step takes no max
        F.advance(S, 1)
        F.time = 0.0
        with pytest.raises(GSError):
            F.dt_last()                      # time reset: no step since


def test_two_handles_on_two_streams_match_each_alone():
    # two solvers with their own streams, device words and workspaces, their
    # advances queued concurrently (FP64 and FP32, different meshes), give
    # the states each gives alone
    import torch
    from paper_1812_07977_amd import Fluid
    cases = [((48, 40, 36), "f64", wl.random_plane(48, 40, 36, seed=5, v=(0.2, 0.1, -0.3))),
             ((40, 32, 24), "f32", wl.random_plane(40, 32, 24, seed=6))]
    _say("case: two handles on two streams, 12 steps each, f64 48x40x36 and f32 40x32x24")
    alone = []
    for shape, dtype, U0 in cases:
        with Fluid(shape, bc="periodic", dtype=dtype) as F:
            S = F.state_from(U0)
            F.advance(S, 12)
            alone.append((to_cpu(S), F.time))
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    solvers = [Fluid(shape, bc="periodic", dtype=dtype, stream=s)
               for (shape, dtype, _), s in zip(cases, streams)]
    try:
        states = [F.state_from(U0) for F, (_, _, U0) in zip(solvers, cases)]
        torch.cuda.synchronize()
        for _ in range(3):
            for F, S in zip(solvers, states):
                F.advance(S, 4)
        for F in solvers:
            F.sync()
        for (ref, t), F, S in zip(alone, solvers, states):
            assert np.array_equal(to_cpu(S), ref)
            assert F.time == t
    finally:
        for F in solvers:
            F.close()
