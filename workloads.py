"""Seeded synthetic initial data for the Euler finite-volume step.

This module only builds inputs: it holds no part of the step itself, and both
the GPU library's tests/benchmark and the CPU oracle's tests take their
inputs from here.  Every array is numpy float64 of shape (5, nz, ny, nx):
conserved fields (rho, m_x, m_y, m_z, E), x fastest, for an ideal gas with
E = p/(gamma-1) + rho |v|^2 / 2.

Mesh convention: cells are cubes of width h = 1/max(nx, ny, nz), so a cubic
mesh spans the unit cube; cell (i, j, k) has centre ((i+1/2)h, (j+1/2)h,
(k+1/2)h).  Discontinuous data take the value at the cell centre (strict "<"
for the left state); smooth data are exact cell averages.

Workloads (the paper's problem is a 3D extension of Sod's shock tube evolved
to t = 0.25, Section 3; its performance runs use 256^3 cells per GPU,
Section 4):
  diagonal_riemann   32^3 outflow problem: left state where x+y+z < 1.5
  sod                grid-aligned Sod tube along one axis
  sine_wave          smooth density wave advected at uniform v, p
  random_plane       seeded random discontinuity plane, rho and p ratios
                     log-uniform in [1, 100]
  supersonic_contact a density jump carried by a uniform flow that is
                     supersonic along one axis in every cell
  uniform            constant state
"""
import math

import numpy as np

GAMMA = 1.4


def spacing(nx, ny, nz):
    h = 1.0 / max(nx, ny, nz)
    return (h, h, h)


def centres(nx, ny, nz):
    """Cell-centre coordinates broadcastable to (nz, ny, nx)."""
    h = spacing(nx, ny, nz)[0]
    x = ((np.arange(nx) + 0.5) * h)[None, None, :]
    y = ((np.arange(ny) + 0.5) * h)[None, :, None]
    z = ((np.arange(nz) + 0.5) * h)[:, None, None]
    return x, y, z


def conserved(rho, vx, vy, vz, p, shape, gamma=GAMMA):
    """Conserved fields from primitive initial data (arrays or scalars)."""
    nz, ny, nx = shape
    U = np.empty((5, nz, ny, nx))
    rho = np.broadcast_to(np.asarray(rho, dtype=np.float64), shape)
    vel = [np.broadcast_to(np.asarray(v, dtype=np.float64), shape) for v in (vx, vy, vz)]
    p = np.broadcast_to(np.asarray(p, dtype=np.float64), shape)
    U[0] = rho
    for d in range(3):
        U[1 + d] = rho * vel[d]
    U[4] = p / (gamma - 1.0) + 0.5 * rho * (vel[0] ** 2 + vel[1] ** 2 + vel[2] ** 2)
    return U


def uniform(nx, ny, nz, rho=1.0, v=(0.0, 0.0, 0.0), p=1.0, gamma=GAMMA):
    return conserved(rho, *v, p, (nz, ny, nx), gamma)


def _two_state(left_mask, left, right, gamma):
    """left/right = (rho, p); velocity zero."""
    shape = left_mask.shape
    rho = np.where(left_mask, left[0], right[0])
    p = np.where(left_mask, left[1], right[1])
    return conserved(rho, 0.0, 0.0, 0.0, p, shape, gamma)


def diagonal_riemann(n=32, gamma=GAMMA):
    """The 32^3 outflow problem: (rho, p) = (1, 1) where x+y+z < 1.5, else
    (0.125, 0.1); v = 0."""
    x, y, z = centres(n, n, n)
    mask = np.broadcast_to(x + y + z < 1.5, (n, n, n))
    return _two_state(mask, (1.0, 1.0), (0.125, 0.1), gamma)


SOD_LEFT = (1.0, 0.0, 1.0)     # rho, u, p
SOD_RIGHT = (0.125, 0.0, 0.1)


def sod(n, axis=0, transverse=4, gamma=GAMMA):
    """Sod's tube along `axis`: n cells along it, `transverse` cells across,
    discontinuity at 1/2 (h = 1/n)."""
    dims = [transverse] * 3
    dims[axis] = n
    nx, ny, nz = dims
    c = centres(nx, ny, nz)
    mask = np.broadcast_to(c[axis] < 0.5, (nz, ny, nx))
    return _two_state(mask, (SOD_LEFT[0], SOD_LEFT[2]), (SOD_RIGHT[0], SOD_RIGHT[2]), gamma)


def _cell_sine(nx, ny, nz, k, shift):
    """Cell averages of sin(2 pi (k . x - shift)) on the mesh."""
    h = spacing(nx, ny, nz)[0]
    x, y, z = centres(nx, ny, nz)
    phase = 2.0 * math.pi * (k[0] * x + k[1] * y + k[2] * z - shift)
    damp = 1.0
    for kd in k:
        a = math.pi * kd * h
        damp *= math.sin(a) / a if kd != 0 else 1.0
    return damp * np.sin(phase)


def sine_density(nx, ny, nz, k=(1, 1, 1), v=(1.0, 1.0, 1.0), amp=0.2, t=0.0):
    """Exact cell averages of rho(x, t) = 1 + amp sin(2 pi k.(x - v t))."""
    shift = t * (k[0] * v[0] + k[1] * v[1] + k[2] * v[2])
    return 1.0 + amp * _cell_sine(nx, ny, nz, k, shift)


def sine_wave(nx, ny, nz, k=(1, 1, 1), v=(1.0, 1.0, 1.0), amp=0.2, p=1.0, gamma=GAMMA):
    """Smooth periodic case: rho = 1 + amp sin(2 pi k.x) (cell averages),
    uniform v and p; the momentum and energy are the exact cell averages
    too since v and p are constant."""
    rho = sine_density(nx, ny, nz, k, v, amp)
    return conserved(rho, *v, p, (nz, ny, nx), gamma)


def random_plane_params(seed):
    """Draws, in this order from numpy's default_rng(seed): the plane normal
    (3 standard normals, normalised), the plane's offset from the cube centre
    along the normal (uniform in [-0.2, 0.2]), then log10 of the density and
    pressure ratios (each uniform in [0, 2])."""
    rng = np.random.default_rng(seed)
    nrm = rng.standard_normal(3)
    nrm /= np.linalg.norm(nrm)
    off = rng.uniform(-0.2, 0.2)
    r_rho = 10.0 ** rng.uniform(0.0, 2.0)
    r_p = 10.0 ** rng.uniform(0.0, 2.0)
    d = float(nrm @ np.array([0.5, 0.5, 0.5])) + off
    return nrm, d, r_rho, r_p


def random_plane(nx, ny, nz, seed, gamma=GAMMA, v=(0.0, 0.0, 0.0)):
    """Seeded Riemann problem: (rho, p) = (1, 1) where n.x < d, and
    (1/r_rho, 1/r_p) on the other side; uniform velocity v (default 0; a
    non-zero v is the same problem seen from a moving frame)."""
    nrm, d, r_rho, r_p = random_plane_params(seed)
    x, y, z = centres(nx, ny, nz)
    mask = np.broadcast_to(nrm[0] * x + nrm[1] * y + nrm[2] * z < d, (nz, ny, nx))
    rho = np.where(mask, 1.0, 1.0 / r_rho)
    p = np.where(mask, 1.0, 1.0 / r_p)
    return conserved(rho, *v, p, (nz, ny, nx), gamma)


def supersonic_contact(nx, ny, nz, axis, sign, mach=3.0, gamma=GAMMA):
    """A contact discontinuity in a uniform supersonic flow: p = 1, rho = 1
    on the side a + 0.25 b + 0.15 c < 0.55 of a tilted plane (a the
    coordinate along `axis`, b and c the other two in cyclic order) and 0.2
    beyond it, velocity sign * mach * c_max along `axis` with c_max the sound
    speed of the lighter gas.  Every face state a minmod reconstruction can
    form lies between the two gases, so along `axis` both of a face's signal
    speeds have the flow's sign."""
    x, y, z = centres(nx, ny, nz)
    c = [x, y, z]
    a, b, cc = c[axis], c[(axis + 1) % 3], c[(axis + 2) % 3]
    mask = np.broadcast_to(a + 0.25 * b + 0.15 * cc < 0.55, (nz, ny, nx))
    rho = np.where(mask, 1.0, 0.2)
    speed = sign * mach * math.sqrt(gamma * 1.0 / 0.2)
    v = [0.0, 0.0, 0.0]
    v[axis] = speed
    return conserved(rho, *v, 1.0, (nz, ny, nx), gamma)


def random_batch_dims(count, seed, lo=32, hi=160):
    """Mesh sizes of a batch: each of nx, ny, nz drawn uniformly from the
    integers [lo, hi] with numpy's default_rng(seed) (non-cubic meshes)."""
    rng = np.random.default_rng(seed)
    return [tuple(int(v) for v in rng.integers(lo, hi + 1, 3)) for _ in range(count)]


def random_batch(count, seed, lo=32, hi=160, gamma=GAMMA):
    """A batch of seeded random-plane Riemann problems: mesh sizes from
    random_batch_dims(count, seed, lo, hi); problem i is
    random_plane(nx, ny, nz, seed=1000 * seed + i) on its own mesh."""
    dims = random_batch_dims(count, seed, lo, hi)
    return dims, [random_plane(nx, ny, nz, seed=1000 * seed + i, gamma=gamma)
                  for i, (nx, ny, nz) in enumerate(dims)]
