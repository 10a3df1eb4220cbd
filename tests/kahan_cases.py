"""Scenes and closed forms for the compensated-integration checks of the FP32
cell-relative form (shared by the GPU test and its CPU emulation).

Every case steps with dt = 2^-14 s and FP32-exact velocities, accelerations or
density rates, so each update adds one FP32-exact increment and the state after N
steps is known exactly in FP64.  With plain FP32 additions the rounding of each
add (up to half an ulp of the running value) accumulates over the steps; the
compensated sums keep it within a few ulp of the running value.
"""
import math

import numpy as np

from paper_1702_07760_amd import inputs

DT = 2.0 ** -14
NSTEPS = 100_000
BOX = 0.25          # periodic box side (m)
H = 0.01            # smoothing length (m): cells of (2 + skin) h = 0.021 m -> 11 per side
U0 = np.float32([0.9, -0.53, 0.31]).astype(np.float64)
G0 = np.float32([0.21, -0.37, 0.13]).astype(np.float64)


def cell_size():
    reach = 2.1 * H
    return BOX / math.floor(BOX / reach)


def drifting_particles(gravity=False):
    """64 fluid particles 0.0625 m apart (beyond 2h: no neighbours) in a periodic box,
    all at the velocity U0, under no gravity or the gravity G0."""
    k = np.arange(4)
    grid = np.stack(np.meshgrid(k, k, k, indexing="ij"), -1).reshape(-1, 3)
    x = (grid + 0.37) * (BOX / 4)
    n = len(x)
    p = inputs.default_params(3, H)
    p.update(lo=[0.0] * 3, hi=[BOX] * 3, periodic=[1, 1, 1], dt_fixed=DT, renorm_every=0,
             gravity=list(G0) if gravity else [0.0, 0.0, 0.0])
    return inputs.Scene("drift", 3, [p], [[(1000.0, 1e-6, 10.0)]], x, np.tile(U0, (n, 1)),
                        np.full(n, 1000.0), np.full(n, 1e-6), np.zeros(n, np.uint8),
                        np.zeros(n, np.uint8), np.array([0, n], np.int64), [H / 1.3], None)


def wall_lattice():
    """A periodic 2D lattice of boundary particles (fixed positions and velocities) with
    u_x = A sin(2 pi x / L): under the mass form of the continuity equation (Eq. (5))
    every density rate is constant in time, so rho grows linearly."""
    n, dx = 24, 1e-3
    s = inputs.lattice_box(2, n, dx, periodic=True)
    L = n * dx
    s.kind[:] = inputs.WALL
    s.u[:, 0] = 2e-4 * np.sin(2 * math.pi * s.x[:, 0] / L)
    s.rho[:] = 1000.0
    return s.with_params(cont_form=1, renorm_every=0, dt_fixed=DT)


def wrap_error(x, want, period):
    """x - want taken to the nearest periodic image."""
    d = x - want
    return d - period * np.round(d / period)
