"""GPU tests of the FP32 form: FP32 state and reconstruction/HLL arithmetic,
Kahan-compensated RK2 combine, FP64 primitive recovery, time step and
conserved totals.  Compared, through the C ABI, with the FP64 oracle on the
same seeded inputs.

Error bound.  The FP32 form is not the FP64 scheme rounded once: the state
is held as an FP32 pair, the stencil reads its FP32 head (relative error
<= u/2, u = 2^-24 the FP32 unit roundoff), and the face fluxes are evaluated
in FP32, a chain of a few tens of operations whose rounding enters each
step's increment.  Every operation of the scheme is Lipschitz (minmod, min/max
signal speeds, the clamped HLL average) with a per-step constant near 1 at
CFL 0.5, so the difference from the FP64 oracle after N steps is bounded by a
representation term plus a term linear in N:
    relative L-infinity per field <= (A_LINF + B_LINF N) u,
    relative L1 per field         <= (A_L1 + B_L1 N) u.
The compensation is what keeps the growth at most linear: without it every
step would add a rounding of U itself, and increments below half an ulp of U
would be lost.  Measured (max over the cases below): L-infinity 0.8 u after
1 step (512^3), 1.8 u after 20, 3.1 u after 30, 2.8 u after 100; L1 1.4 u
after 20, 1.5 u after 100.  The constants leave three to ten times that.
"""
import json
import math
import sys

import numpy as np
import pytest

import oracle
import workloads as wl
from tests.parity import (CFL, GAMMA, f32_run, gpu_run_device_dt, oracle_run, rel_l1, rel_linf,
                          to_cpu)

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
A_LINF, B_LINF = 4.0, 0.25
A_L1, B_L1 = 2.0, 0.1


def linf_bound(n):
    return (A_LINF + B_LINF * n) * U32


def l1_bound(n):
    return (A_L1 + B_L1 * n) * U32


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _report(name, nsteps, l1, linf, dt_rel):
    _say("f32-error " + json.dumps({"case": name, "steps": nsteps,
                                    "l1_rel": [float(f"{v:.3e}") for v in l1],
                                    "linf_rel": [float(f"{v:.3e}") for v in linf],
                                    "linf_over_uN": round(max(linf) / (U32 * nsteps), 3),
                                    "l1_over_uN": round(max(l1) / (U32 * nsteps), 3),
                                    "dt_rel_max": float(f"{dt_rel:.3e}")}))


CASES = {
    "diagonal32": (lambda: wl.diagonal_riemann(32), "outflow", 20),
    "sine64": (lambda: wl.sine_wave(64, 64, 64), "periodic", 100),
    "plane0_64": (lambda: wl.random_plane(64, 64, 64, seed=0), "periodic", 100),
    "plane1_64": (lambda: wl.random_plane(64, 64, 64, seed=1), "periodic", 100),
    "boosted_ragged": (lambda: wl.random_plane(40, 24, 20, seed=7, v=(0.7, -0.45, 0.3)),
                       "outflow", 30),
}
# Mach 3 along each axis and sign (both one-sided HLL branches), both
# boundary kinds
for _ax in range(3):
    for _sg in (1, -1):
        for _bc in ("outflow", "periodic"):
            CASES[f"supersonic_{'xyz'[_ax]}{'+' if _sg > 0 else '-'}_{_bc}"] = (
                (lambda a=_ax, s=_sg: wl.supersonic_contact(24, 20, 18, a, s)), _bc, 8)


@pytest.mark.parametrize("case", sorted(CASES))
def test_f32_matches_fp64_oracle_within_bound(case):
    make, bc, n = CASES[case]
    U0 = make()
    _say(f"case: f32 {case} {U0.shape[1:]} {bc}, {n} steps, device dt")
    ref, odt = oracle_run(U0, bc, n)
    out, gdt, _, _ = f32_run(U0, bc, n, mode="device")
    dt_rel = float(np.max(np.abs(gdt - odt) / odt))
    l1, linf = rel_l1(out, ref), rel_linf(out, ref)
    _report(case, n, l1, linf, dt_rel)
    assert dt_rel <= linf_bound(n)
    assert max(linf) <= linf_bound(n), linf
    assert max(l1) <= l1_bound(n), l1


def test_f32_large_mesh_matches_fp64_oracle_within_bound():
    # 192^3: the FP32 state (5 fields x 7.1 M cells x 4 B) exceeds 128 MiB,
    # so the substeps take the non-temporal loads and stores, as at 512^3.
    # A bulk velocity gives every field an O(1) magnitude: at rest, the
    # momentum after 8 steps is nonzero only near the discontinuity, and its
    # relative L1 error would measure the rounding of rho and E instead
    U0 = wl.random_plane(192, 192, 192, seed=3, v=(0.5, -0.4, 0.3))
    n = 8
    _say(f"case: f32 plane3 192^3 periodic, {n} steps, device dt (non-temporal path)")
    ref, odt = oracle_run(U0, "periodic", n)
    out, gdt, _, _ = f32_run(U0, "periodic", n, mode="device")
    dt_rel = float(np.max(np.abs(gdt - odt) / odt))
    l1, linf = rel_l1(out, ref), rel_linf(out, ref)
    _report("plane3_192", n, l1, linf, dt_rel)
    assert dt_rel <= linf_bound(n)
    assert max(linf) <= linf_bound(n), linf
    assert max(l1) <= l1_bound(n), l1


def test_f32_with_the_oracle_time_steps():
    # the same dt sequence on both sides isolates the arithmetic
    U0 = wl.random_plane(48, 40, 36, seed=2)
    n = 40
    _say(f"case: f32 plane2 (48,40,36) periodic, {n} steps, the oracle's dts")
    ref, odt = oracle_run(U0, "periodic", n)
    out, _, _, _ = f32_run(U0, "periodic", n, mode="given", dts=odt)
    l1, linf = rel_l1(out, ref), rel_linf(out, ref)
    _report("plane2_given_dt", n, l1, linf, 0.0)
    assert max(linf) <= linf_bound(n), linf
    assert max(l1) <= l1_bound(n), l1


def test_f32_host_dt_and_device_dt_are_bitwise_identical():
    U0 = wl.diagonal_riemann(32)
    _say("case: f32 diagonal 32^3, host dt vs device dt, 8 steps")
    a, adt, _, pa = f32_run(U0, "outflow", 8, mode="host")
    b, bdt, _, pb = f32_run(U0, "outflow", 8, mode="device")
    assert np.array_equal(adt, bdt)
    assert np.array_equal(pa, pb)


@pytest.mark.parametrize("launch", [(8, 0), (16, 1), (8, 3), (16, 64)])
def test_f32_launch_shapes_give_identical_results(launch):
    U0 = wl.random_plane(40, 24, 20, seed=11, v=(0.9, -0.6, 0.4))
    _say(f"case: f32 boosted plane (40,24,20) outflow, 5 steps, launch {launch}")
    _, bdt, _, base = f32_run(U0, "outflow", 5, launch=(16, 0))
    _, odt, _, other = f32_run(U0, "outflow", 5, launch=launch)
    assert np.array_equal(bdt, odt)
    assert np.array_equal(base, other)


@pytest.mark.parametrize("bc", ["outflow", "periodic"])
def test_f32_whole_tile_kernels_match_the_ragged_tile_kernels(bc):
    # 48 x 32: whole 16 x 16 tiles, ragged 32 x 8 tiles
    U0 = wl.random_plane(48, 32, 12, seed=17, v=(0.5, -0.3, 0.2))
    _say(f"case: f32 plane (48,32,12) {bc}, 6 steps, 16x16 whole tiles vs 32x8 ragged")
    _, adt, _, a = f32_run(U0, bc, 6, launch=(16, 0))
    _, bdt, _, b = f32_run(U0, bc, 6, launch=(8, 0))
    assert np.array_equal(adt, bdt)
    assert np.array_equal(a, b)


def test_f32_repeated_runs_are_bitwise_identical():
    U0 = wl.random_plane(48, 48, 48, seed=3)
    _, adt, _, a = f32_run(U0, "periodic", 6)
    _, bdt, _, b = f32_run(U0, "periodic", 6)
    assert np.array_equal(adt, bdt)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("bc", ["outflow", "periodic"])
def test_f32_uniform_state_stays_bitwise_uniform(bc):
    # every face sees the same two states, so every increment is exactly
    # zero and the compensated sum leaves head and compensation unchanged
    U0 = wl.uniform(12, 10, 9, rho=1.3, v=(0.3, -0.2, 0.1), p=0.7)
    from paper_1812_07977_amd import Fluid
    with Fluid((12, 10, 9), bc=bc, dtype="f32") as F:
        start = to_cpu(F.state_from(U0))
    _, _, _, pair = f32_run(U0, bc, 5)
    assert np.array_equal(pair, start)


def test_f32_totals_are_conserved_with_periodic_boundaries():
    from paper_1812_07977_amd import Fluid
    U0 = wl.random_plane(48, 48, 48, seed=4, v=(0.3, 0.0, 0.0))
    n = 30
    _say(f"case: f32 boosted plane4 48^3 periodic, {n} steps, totals")
    with Fluid((48, 48, 48), bc="periodic", dtype="f32") as F:
        S = F.state_from(U0)
        before = np.array(F.totals(S))
        F.advance(S, n)
        after = np.array(F.totals(S))
    exact = np.array([math.fsum(U0[f].ravel()) for f in range(5)])
    scale = np.max(np.abs(exact))
    drift = float(np.max(np.abs(after - before)) / scale)
    # the fluxes telescope, but each cell's FP32 increment is rounded
    # independently: a random walk of about sqrt(cells) roundings of size
    # u max|U| per step
    est = n * math.sqrt(U0[0].size) * U32 * np.max(np.abs(U0)) / scale
    _say(f"f32 totals drift over {n} steps: {drift:.3e} of the largest total "
         f"(estimate {est:.1e})")
    # the initial pair holds U0 to about 48 bits
    assert np.max(np.abs(before - exact)) <= 1e-13 * scale
    assert drift <= est


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_totals_match_exact_sums(dtype):
    from paper_1812_07977_amd import Fluid
    rng = np.random.default_rng(5)
    shape = (37, 29, 23)
    U0 = wl.random_plane(*shape, seed=9, v=(0.2, -0.1, 0.05))
    U0 *= 1.0 + 0.01 * rng.standard_normal(U0.shape)
    with Fluid(shape, bc="periodic", dtype=dtype) as F:
        S = F.state_from(U0)
        got = np.array(F.totals(S))
        vals = to_cpu(F.to_f64(S))
    for f in range(5):
        exact = math.fsum(vals[f].ravel())
        assert abs(got[f] - exact) <= 4 * np.finfo(np.float64).eps * abs(exact), (f, got[f], exact)


def test_f32_compensation_keeps_increments_below_the_rounding_of_u():
    # a density wave of relative amplitude 1e-5 advected at CFL 0.02: every
    # step's increment (about 2e-8) is below half an FP32 ulp of rho ~ 1
    # (6e-8), so a plain FP32 update would leave the state unchanged; the
    # compensated form must follow the FP64 oracle's change
    from paper_1812_07977_amd import Fluid
    import torch
    n, steps, cfl = 32, 200, 0.02
    U0 = wl.sine_wave(n, n, n, amp=1e-5)
    h = 1.0 / n
    _say(f"case: f32 sine amp 1e-5 {n}^3 periodic, CFL {cfl}, {steps} steps")
    ref = U0.copy()
    dts = oracle.run(ref, (h, h, h), GAMMA, cfl, oracle.PERIODIC, steps)
    with Fluid((n, n, n), bc="periodic", cfl=cfl, dtype="f32") as F:
        S = F.state_from(U0)
        for dt in dts:
            F.step(S, float(dt))
        out = to_cpu(F.to_f64(S))
        head = to_cpu(S[0].to(torch.float64))
    for f in (0, 1, 4):
        change = np.sum(np.abs(ref[f] - U0[f]))
        err = np.sum(np.abs(out[f] - ref[f]))
        err_head = np.sum(np.abs(head[f] - ref[f]))
        _say(f"field {f}: change {change:.3e}, error {err:.3e} ({err / change:.3f}), "
             f"head alone {err_head / change:.3f}")
        assert err <= 0.1 * change, (f, err, change)


def test_f32_nonphysical_input_is_reported():
    from paper_1812_07977_amd import Fluid, NonPhysicalError
    U0 = wl.uniform(16, 16, 16)
    U0[0, 3, 4, 5] = -1.0
    with Fluid((16, 16, 16), dtype="f32") as F:
        S = F.state_from(U0)
        with pytest.raises(NonPhysicalError):
            F.dt(S)
        F.sync()


def test_f32_bad_arguments():
    import torch
    from paper_1812_07977_amd import Fluid
    with Fluid((8, 8, 8), dtype="f32") as F:
        S = F.state_from(wl.uniform(8, 8, 8))
        with pytest.raises(TypeError):
            F.step(S.double(), 0.1)
        with pytest.raises(ValueError):
            F.step(S[0].contiguous(), 0.1)
        F.sync()


def test_f32_checkpoint_restart_is_bitwise_identical():
    # the state pair and the device time are the whole checkpoint
    import torch
    from paper_1812_07977_amd import Fluid
    U0 = wl.random_plane(40, 40, 40, seed=6)
    with Fluid((40, 40, 40), bc="periodic", dtype="f32") as F:
        A = F.state_from(U0)
        F.advance(A, 12)
        tA = F.time
    with Fluid((40, 40, 40), bc="periodic", dtype="f32") as F:
        B = F.state_from(U0)
        F.advance(B, 7)
        t_saved = F.time
    saved = to_cpu(B).copy()
    with Fluid((40, 40, 40), bc="periodic", dtype="f32") as F:
        C = torch.from_numpy(saved).to("cuda")
        F.time = t_saved
        F.advance(C, 5)
        tC = F.time
    assert np.array_equal(to_cpu(C), to_cpu(A))
    assert tC == tA


# ---------------------------------------------------------------------------
# full size, in the launch configuration of the benchmark (device dt)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("case", ["sine", "plane0"])
def test_f32_full_512_sampled_windows_within_bound(case):
    from paper_1812_07977_amd import Fluid
    import torch
    n = 512
    _say(f"case: f32 {case} {n}^3 periodic, 1 step, sampled windows")
    U0 = wl.sine_wave(n, n, n) if case == "sine" else wl.random_plane(n, n, n, seed=0)
    log = torch.zeros(1, dtype=torch.float64, device="cuda")
    with Fluid((n, n, n), bc="periodic", dtype="f32") as F:
        S = F.state_from(U0)
        F.advance(S, 1, 0.0, log)
        out = to_cpu(F.to_f64(S))
        del S
    gdt = float(log.cpu()[0])
    h = 1.0 / n
    odt = oracle.time_step(U0, (h, h, h), GAMMA, CFL)
    assert abs(gdt - odt) <= linf_bound(1) * odt
    rng = np.random.default_rng(321)
    origins = [(0, 0, 0), (n - 3, n - 2, n - 4), (255, 256, 250)]
    origins += [tuple(int(v) for v in rng.integers(0, n, 3)) for _ in range(5)]
    size = (6, 5, 4)
    scale = np.max(np.abs(U0), axis=(1, 2, 3))
    worst = 0.0
    for o in origins:
        # the oracle's step with the FP32 form's own dt
        win = oracle.step_window(U0, (h, h, h), GAMMA, gdt, o, size)
        ii = [(o[0] + i) % n for i in range(size[0])]
        jj = [(o[1] + j) % n for j in range(size[1])]
        kk = [(o[2] + k) % n for k in range(size[2])]
        g = out[:, kk][:, :, jj][:, :, :, ii]
        for f in range(5):
            s = scale[f] if scale[f] > 0 else np.max(scale)
            worst = max(worst, float(np.max(np.abs(g[f] - win[f])) / s))
    _say(f"f32 512^3 {case}: worst windowed rel error {worst:.3e} = {worst / U32:.2f} u")
    assert worst <= linf_bound(1)
