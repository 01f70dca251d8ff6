"""Pins of the exact Riemann solver that the oracle is later judged by.

The solver is checked against published star states and, independently of
how it finds them, against the jump conditions the solution must satisfy:
Rankine-Hugoniot across shocks, isentropy and the Riemann invariant across
rarefactions.
"""
import math
import os

import numpy as np
import pytest

from oracle.exact_riemann import RiemannSolution

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
G = 1.4


def _read_pairs(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                k, v = line.split()
                out[k] = float(v)
    return out


def _read_rows(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append([float(x) for x in line.split()])
    return rows


def test_sod_star_state_matches_published_values():
    ref = _read_pairs("sod_star_state.txt")
    s = RiemannSolution((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), G)
    assert s.p_star == pytest.approx(ref["p_star"], abs=1e-5)
    assert s.u_star == pytest.approx(ref["u_star"], abs=1e-5)
    assert s.rho_starL == pytest.approx(ref["rho_star_left"], abs=1e-5)
    assert s.rho_starR == pytest.approx(ref["rho_star_right"], abs=1e-5)


@pytest.mark.parametrize("row", _read_rows("toro_tests.txt"))
def test_other_published_star_states(row):
    rl, ul, pl, rr, ur, pr, ps, us = row
    s = RiemannSolution((rl, ul, pl), (rr, ur, pr), G)
    assert s.p_star == pytest.approx(ps, rel=1e-4, abs=1e-5)
    assert s.u_star == pytest.approx(us, rel=1e-4, abs=1e-5)


def _energy(rho, u, p):
    return p / (G - 1.0) + 0.5 * rho * u * u


def _rh_residuals(pre, post, S):
    """Jumps of mass, momentum and energy fluxes in the frame of speed S."""
    (r0, u0, p0), (r1, u1, p1) = pre, post
    mass = r0 * (u0 - S) - r1 * (u1 - S)
    mom = (r0 * u0 * (u0 - S) + p0) - (r1 * u1 * (u1 - S) + p1)
    en = (_energy(r0, u0, p0) * (u0 - S) + p0 * u0) - (_energy(r1, u1, p1) * (u1 - S) + p1 * u1)
    return mass, mom, en


@pytest.mark.parametrize("left,right", [
    ((1.0, 0.0, 1.0), (0.125, 0.0, 0.1)),        # Sod: right shock
    ((0.125, 0.0, 0.1), (1.0, 0.0, 1.0)),        # mirrored: left shock
    ((1.0, 0.5, 2.0), (0.3, -0.4, 0.2)),         # colliding, two shocks
    ((1.0, 0.0, 1000.0), (1.0, 0.0, 0.01)),      # strong shock
])
def test_shocks_satisfy_rankine_hugoniot(left, right):
    s = RiemannSolution(left, right, G)
    checked = 0
    if s.p_star > s.pR:
        S = s.right_wave()[0]
        res = _rh_residuals(right, (s.rho_starR, s.u_star, s.p_star), S)
        scale = max(abs(s.p_star), 1.0)
        assert max(abs(r) for r in res) < 1e-11 * scale
        checked += 1
    if s.p_star > s.pL:
        S = s.left_wave()[0]
        res = _rh_residuals(left, (s.rho_starL, s.u_star, s.p_star), S)
        scale = max(abs(s.p_star), 1.0)
        assert max(abs(r) for r in res) < 1e-11 * scale
        checked += 1
    assert checked >= 1


@pytest.mark.parametrize("left,right", [
    ((1.0, 0.0, 1.0), (0.125, 0.0, 0.1)),
    ((1.0, -2.0, 0.4), (1.0, 2.0, 0.4)),
])
def test_left_rarefaction_is_isentropic_with_constant_invariant(left, right):
    s = RiemannSolution(left, right, G)
    head, tail = s.left_wave()
    assert head < tail
    entropy0 = s.pL / s.rhoL ** G
    j0 = s.uL + 2.0 * math.sqrt(G * s.pL / s.rhoL) / (G - 1.0)
    for xi in np.linspace(head, tail, 9):
        rho, u, p = s.sample(xi)
        assert p / rho ** G == pytest.approx(entropy0, rel=1e-12)
        c = math.sqrt(G * p / rho)
        assert u + 2.0 * c / (G - 1.0) == pytest.approx(j0, rel=1e-12)
    # characteristic condition inside the fan: xi = u - c
    rho, u, p = s.sample(0.5 * (head + tail))
    assert u - math.sqrt(G * p / rho) == pytest.approx(0.5 * (head + tail), abs=1e-12)
    # the fan's tail reaches the star state continuously
    rho, u, p = s.sample(tail - 1e-12)
    assert rho == pytest.approx(s.rho_starL, rel=1e-9)
    assert p == pytest.approx(s.p_star, rel=1e-9)


def test_cell_averages_of_constant_pieces_are_constant():
    s = RiemannSolution((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), G)
    edges = np.array([0.0, 0.1, 0.2, 0.95, 1.0])
    avg = s.cell_averages(edges, 0.25)
    assert avg[0] == pytest.approx(1.0, rel=1e-15)    # untouched left state
    assert avg[1] == pytest.approx(1.0, rel=1e-15)
    assert avg[3] == pytest.approx(0.125, rel=1e-15)  # ahead of the shock
    # shock at 0.5 + 1.75216*0.25 = 0.938 lies inside [0.2, 0.95]
    assert 0.125 < avg[2] < 1.0
