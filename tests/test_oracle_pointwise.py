"""Pins of the oracle's pointwise physics and its line kernels.

Every expected value here is a worked example, a closed form or a special
case derived by hand, never a retyping of the oracle's formulas: a dropped
term, a wrong sign, a swapped index or a transposed operand in the oracle
fails at least one of them.
"""
import math

import numpy as np
import pytest

import oracle

# gamma = 1.5 makes gamma - 1 = 1/2 exact, so the worked examples below are
# exact in binary floating point.
G15 = 1.5


# ---------------------------------------------------------------------------
# conserved <-> primitive
# ---------------------------------------------------------------------------

def test_p2c_worked_example_exact():
    # rho = 2, v = (1, -2, 3), p = 4: m = (2, -4, 6); E = 4/0.5 + 0.5*2*14 = 22
    U = oracle.p2c(G15, [2.0, 1.0, -2.0, 3.0, 4.0])
    assert list(U) == [2.0, 2.0, -4.0, 6.0, 22.0]


def test_c2p_worked_example_exact():
    W = oracle.c2p(G15, [2.0, 2.0, -4.0, 6.0, 22.0])
    assert list(W) == [2.0, 1.0, -2.0, 3.0, 4.0]


def test_c2p_pressure_uses_gamma_minus_one():
    # at rest: p = (gamma-1) E, so gamma = 5/3 and E = 3 give p = 2
    W = oracle.c2p(5.0 / 3.0, [1.0, 0.0, 0.0, 0.0, 3.0])
    assert W[4] == pytest.approx(2.0, rel=4e-16)


def test_c2p_p2c_round_trip_random():
    rng = np.random.default_rng(7)
    for _ in range(200):
        W = np.array([10 ** rng.uniform(-3, 3), *rng.normal(0, 3, 3), 10 ** rng.uniform(-3, 3)])
        back = oracle.c2p(1.4, oracle.p2c(1.4, W))
        assert np.allclose(back[:4], W[:4], rtol=4 * 2.2e-16, atol=0)
        # pressure is recovered from a difference E - kinetic; its rounding
        # error is relative to E, not to p
        E = oracle.p2c(1.4, W)[4]
        assert abs(back[4] - W[4]) <= 8 * 2.2e-16 * E


# ---------------------------------------------------------------------------
# minmod
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("a,b,expected", [
    (1.0, 2.0, 1.0), (2.0, 1.0, 1.0), (-1.0, -2.0, -1.0), (-2.0, -1.0, -1.0),
    (1.0, -1.0, 0.0), (-1.0, 1.0, 0.0), (0.0, 1.0, 0.0), (1.0, 0.0, 0.0),
    (0.0, -1.0, 0.0), (-1.0, 0.0, 0.0), (0.0, 0.0, 0.0), (3.0, 3.0, 3.0),
    # products that underflow: the sign test must not depend on a*b
    (1e-200, 1e-200, 1e-200), (-1e-200, -3e-200, -1e-200),
])
def test_minmod_truth_table(a, b, expected):
    assert oracle.minmod(a, b) == expected


# ---------------------------------------------------------------------------
# line kernels: differences and reconstruction
# ---------------------------------------------------------------------------

def test_difference_index_range_follows_listing():
    # The paper's listing (Section 3) computes dV(i) = V(i) - V(i-1) for
    # i = 0 .. nX+2 on arrays with bounds -1 .. nX+2; in 0-based array
    # positions that is 1 .. n+3: only position 0 is left untouched.
    n = 6
    V = np.arange(n + 4, dtype=float) ** 2
    dV = oracle.differences_line(V)
    assert np.isnan(dV[0])
    assert list(dV[1:]) == [V[i] - V[i - 1] for i in range(1, n + 4)]


def test_reconstruction_exact_on_linear_data():
    n = 8
    a, b = 3.0, -0.25
    x = np.arange(-2, n + 2, dtype=float)
    V = a + b * x
    dV = oracle.differences_line(V)
    sg, VL, VR = oracle.reconstruction_line(V, dV)
    # slopes for cells -1 .. n (positions 1 .. n+2) equal b exactly
    assert np.all(sg[1:n + 3] == b)
    assert np.isnan(sg[0]) and np.isnan(sg[n + 3])
    # faces i+1/2 for i = -1 .. n-1 (positions 1 .. n+1): both states equal
    # the line's value at the face
    face = a + b * (x[1:n + 2] + 0.5)
    assert np.all(VL[1:n + 2] == face)
    assert np.all(VR[1:n + 2] == face)
    assert np.isnan(VL[n + 2]) and np.isnan(VR[0])


def test_reconstruction_flattens_at_extremum_and_jump():
    # peak at position 4: slope there is zero, so both its face states equal it
    V = np.array([0.0, 1.0, 2.0, 3.0, 4.0, 3.0, 2.0, 1.0, 0.0, -1.0])
    dV = oracle.differences_line(V)
    sg, VL, VR = oracle.reconstruction_line(V, dV)
    assert sg[4] == 0.0
    assert VL[4] == 4.0 and VR[3] == 4.0
    # monotone part: slope 1, face states interpolate
    assert sg[2] == 1.0 and VL[2] == 2.5 and VR[1] == 1.5
    # step: every slope is zero, face states are the cell values (first order)
    S = np.array([1.0] * 5 + [0.0] * 5)
    sg, VL, VR = oracle.reconstruction_line(S, oracle.differences_line(S))
    assert np.all(sg[1:9] == 0.0)
    assert np.all(VL[1:8] == S[1:8]) and np.all(VR[1:8] == S[2:9])


def test_reconstruction_is_limited_to_smaller_slope():
    # convex data: the left difference is the smaller one
    V = np.array([0.0, 1.0, 4.0, 9.0, 16.0, 25.0, 36.0])
    sg, VL, VR = oracle.reconstruction_line(V, oracle.differences_line(V))
    # cell at position 3 (value 9): differences 5 and 7 -> slope 5
    assert sg[3] == 5.0
    assert VL[3] == 11.5 and VR[2] == 6.5


# ---------------------------------------------------------------------------
# HLL
# ---------------------------------------------------------------------------

W0 = [2.0, 1.0, -2.0, 3.0, 4.0]   # gamma 1.5: c = sqrt(3), E = 22


def test_hll_consistency_worked_example_x():
    # along x: u_n = 1 with c = sqrt(3) -> subsonic, formula branch
    F, (SL, SR) = oracle.hll(G15, 0, W0, W0)
    expected = [2.0, 6.0, -4.0, 6.0, 26.0]   # rho u, rho u^2 + p, rho v u, rho w u, (E+p) u
    assert np.allclose(F, expected, rtol=4 * 2.2e-16, atol=1e-15)
    assert SL == pytest.approx(1.0 - math.sqrt(3.0), rel=1e-15)
    assert SR == pytest.approx(1.0 + math.sqrt(3.0), rel=1e-15)


def test_hll_consistency_worked_example_y():
    F, _ = oracle.hll(G15, 1, W0, W0)
    expected = [-4.0, -4.0, 12.0, -12.0, -52.0]
    assert np.allclose(F, expected, rtol=4 * 2.2e-16, atol=1e-15)


def test_hll_supersonic_takes_left_flux_exactly():
    # along z: u_n = 3 > c = sqrt(3): S_L > 0, so F = F_L without rounding
    WR = [0.5, 0.0, 0.0, 2.0, 1.0]
    F, (SL, SR) = oracle.hll(G15, 2, W0, WR)
    assert SL > 0.0
    assert list(F) == [6.0, 6.0, -12.0, 22.0, 78.0]


def test_hll_supersonic_leftward_takes_right_flux_exactly():
    WL = [1.0, -3.0, 0.0, 0.0, 1.0]    # c = sqrt(1.5) < 3 = |u_n|
    WR = [2.0, -3.0, 1.0, -2.0, 4.0]   # c = sqrt(3) < 3 = |u_n|
    F, (SL, SR) = oracle.hll(G15, 0, WL, WR)
    assert SR < 0.0
    # rho u = -6, rho u^2 + p = 22, rho v u = -6, rho w u = 12, (E+p) u with
    # E = 8 + 0.5*2*14 = 22 -> -78
    assert list(F) == [-6.0, 22.0, -6.0, 12.0, -78.0]


def test_hll_stationary_contact_closed_form():
    # v = 0, equal p, densities 1 | 1/2, gamma 1.4: S_R = -S_L = c_R = sqrt(2.8),
    # mass flux = -S_L S_R (rho_R - rho_L) / (S_R - S_L) = c_R / 4,
    # momentum flux = p = 1, energy flux = 0 (E_R = E_L).
    F, (SL, SR) = oracle.hll(1.4, 0, [1.0, 0.0, 0.0, 0.0, 1.0], [0.5, 0.0, 0.0, 0.0, 1.0])
    c = math.sqrt(2.8)
    assert SL == pytest.approx(-c, rel=1e-15) and SR == pytest.approx(c, rel=1e-15)
    assert F[0] == pytest.approx(c / 4.0, rel=1e-14)
    assert F[1] == pytest.approx(1.0, rel=1e-15)
    assert F[2] == 0.0 and F[3] == 0.0
    assert abs(F[4]) < 1e-15


def test_hll_davis_speeds_use_each_side():
    WL = [1.0, 0.3, 0.0, 0.0, 1.0]
    WR = [0.125, -0.2, 0.0, 0.0, 0.1]
    _, (SL, SR) = oracle.hll(1.4, 0, WL, WR)
    cL, cR = math.sqrt(1.4), math.sqrt(1.4 * 0.1 / 0.125)
    assert SL == pytest.approx(min(0.3 - cL, -0.2 - cR), rel=1e-15)
    assert SR == pytest.approx(max(0.3 + cL, -0.2 + cR), rel=1e-15)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_hll_mirror_symmetry(axis):
    # Reflecting the normal axis swaps the sides and negates normal velocity:
    # mass, transverse-momentum and energy fluxes change sign, the normal
    # momentum flux does not.
    rng = np.random.default_rng(11 + axis)
    for _ in range(50):
        WL = np.array([10 ** rng.uniform(-1, 1), *rng.normal(0, 1, 3), 10 ** rng.uniform(-1, 1)])
        WR = np.array([10 ** rng.uniform(-1, 1), *rng.normal(0, 1, 3), 10 ** rng.uniform(-1, 1)])
        F, _ = oracle.hll(1.4, axis, WL, WR)
        mL, mR = WR.copy(), WL.copy()
        mL[1 + axis] *= -1.0
        mR[1 + axis] *= -1.0
        Fm, _ = oracle.hll(1.4, axis, mL, mR)
        sign = np.array([-1.0, -1.0, -1.0, -1.0, -1.0])
        sign[1 + axis] = 1.0
        assert np.allclose(Fm, sign * F, rtol=1e-13, atol=1e-13)


def test_hll_galilean_transverse_velocity_only_advects():
    # Adding the same transverse velocity w to both sides leaves mass and
    # normal-momentum fluxes unchanged and adds w * mass flux to the
    # transverse-momentum flux.
    WL = np.array([1.0, 0.2, 0.0, 0.0, 1.0])
    WR = np.array([0.4, -0.1, 0.0, 0.0, 0.3])
    F0, _ = oracle.hll(1.4, 0, WL, WR)
    w = 0.75
    WL2, WR2 = WL.copy(), WR.copy()
    WL2[2] = WR2[2] = w
    F1, _ = oracle.hll(1.4, 0, WL2, WR2)
    assert F1[0] == pytest.approx(F0[0], rel=1e-14)
    assert F1[1] == pytest.approx(F0[1], rel=1e-14)
    assert F1[2] == pytest.approx(w * F0[0], rel=1e-13)
    assert F1[3] == 0.0
