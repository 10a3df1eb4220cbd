"""Seeded synthetic scenes for the two-phase WCSPH hot path.

This module only lays particles out: lattices, jitter, phase tags, particle
kinds, masses and the hydrostatic initial density.  It contains none of the
per-step arithmetic of the method (no kernel, no neighbour search, no rates,
no integration), so it can feed both the GPU library and the FP64 oracle.

Recipe (shared by every scene):

* cell-centred square/cubic lattice, spacing ``dx``, fluid at ``(i+1/2) dx``;
* three layers of fixed boundary particles at ``-(k+1/2) dx`` outside the
  bottom and the side walls (the dynamic boundary condition of Dalrymple and
  Knio, Sec. III), rising to ``1.2 H``; the top is open;
* fluid positions get seeded uniform jitter in ``[-0.05 dx, 0.05 dx]`` per
  component, boundary particles none;
* oil = unjittered lattice points inside the drop/slick; boundary particles
  carry water properties (Sec. III);
* particle mass ``rho0_phase * dx**dim``;
* hydrostatic pressure ``rho0_w * g * (H - z)`` (zero above the surface)
  turned into density by inverting the Tait law of Eqs. (3)-(4);
* smoothing length ``h = 1.3 dx``, sound speed ``c0 = 10 sqrt(g H)`` for both
  phases, ``gamma = 7``, ``delta = 0.1 h`` (Eq. (9)).

``perturb=True`` adds seeded velocities ``U[-0.05, 0.05] c0`` to fluid
particles and a ``+-0.5 %`` density perturbation to every particle, so that
every term of the rates is non-trivial in parity checks.
"""
from __future__ import annotations

import dataclasses
import itertools
import math
from typing import List, Optional

import numpy as np

FLUID, WALL, MOVING = 0, 1, 2
WATER, OIL = 0, 1
SEED_BASE = 17020776
GAMMA = 7.0
G = 9.81


def default_params(dim: int, h: float) -> dict:
    """Parameter dictionary shared by the oracle and the GPU library."""
    return dict(
        dim=dim, h=h, gamma=GAMMA, delta_coef=0.1, alpha_s=0.0,
        gravity=[0.0, 0.0, 0.0], lo=[0.0, 0.0, 0.0], hi=[1.0, 1.0, 1.0],
        periodic=[0, 0, 0], skin_coef=0.1,
        c_cfl=0.25, c_force=0.25, c_visc=0.125, c_st=0.25, dt_fixed=0.0,
        visc_form=0, cont_form=0, renorm_every=1,
        piston_a=[], piston_w=[], piston_phi=[], piston_t_end=0.0,
    )


@dataclasses.dataclass
class Scene:
    """A set of independent instances, particles concatenated per instance."""
    name: str
    dim: int
    params: List[dict]            # one dict per instance
    phases: List[list]            # per instance: list of (rho0, nu, c0)
    x: np.ndarray                 # (n, 3) float64, unused components zero
    u: np.ndarray                 # (n, 3) float64
    rho: np.ndarray               # (n,) float64
    m: np.ndarray                 # (n,) float64
    phase: np.ndarray             # (n,) uint8
    kind: np.ndarray              # (n,) uint8
    inst_offsets: np.ndarray      # (ninst+1,) int64
    dx: List[float]
    seed: Optional[int] = None

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    @property
    def ninst(self) -> int:
        return len(self.params)

    def instance(self, b: int) -> "Scene":
        a, e = int(self.inst_offsets[b]), int(self.inst_offsets[b + 1])
        return Scene(f"{self.name}[{b}]", self.dim, [self.params[b]], [self.phases[b]],
                     self.x[a:e].copy(), self.u[a:e].copy(), self.rho[a:e].copy(),
                     self.m[a:e].copy(), self.phase[a:e].copy(), self.kind[a:e].copy(),
                     np.array([0, e - a], np.int64), [self.dx[b]], self.seed)

    def with_params(self, **kw) -> "Scene":
        s = dataclasses.replace(self)
        s.params = [dict(p, **kw) for p in self.params]
        return s


def concat(name: str, scenes: List[Scene]) -> Scene:
    offs = np.cumsum([0] + [s.n for s in scenes]).astype(np.int64)
    return Scene(name, scenes[0].dim, [s.params[0] for s in scenes],
                 [s.phases[0] for s in scenes],
                 np.concatenate([s.x for s in scenes]), np.concatenate([s.u for s in scenes]),
                 np.concatenate([s.rho for s in scenes]), np.concatenate([s.m for s in scenes]),
                 np.concatenate([s.phase for s in scenes]), np.concatenate([s.kind for s in scenes]),
                 offs, [s.dx[0] for s in scenes], None)


def _grid(ranges):
    """All integer tuples in the product of ``ranges`` (list of (lo, hi))."""
    axes = [np.arange(a, b) for a, b in ranges]
    mesh = np.meshgrid(*axes, indexing="ij")
    return np.stack([m.ravel() for m in mesh], axis=1)


def _hydrostatic_rho(z, H, rho0, rho0_w, c0, g):
    """Density from the Tait law at the hydrostatic pressure of a water column."""
    p0 = rho0_w * g * np.maximum(H - z, 0.0)
    beta = rho0 * c0 * c0 / GAMMA
    return rho0 * (1.0 + p0 / beta) ** (1.0 / GAMMA)


def tank(dim: int, width, height: float, dx: float, *, seed: int, oil=None,
         rho_w=1000.0, mu_w=1e-3, rho_o=900.0, mu_o=5e-3, alpha_s=0.02,
         nlayers=3, wall_top=1.2, headroom=1.5, jitter=0.05, perturb=False,
         name="tank") -> Scene:
    """Still water tank, walls on the bottom and the sides, open top.

    ``width`` is the horizontal extent (a float in 2D, a pair in 3D), ``height``
    the water depth H.  The vertical axis is the last active dimension.
    ``oil(points) -> bool mask`` marks oil lattice points (unjittered positions).
    """
    rng = np.random.default_rng(seed)
    widths = [width] if dim == 2 else list(width)
    nh = [int(round(w / dx)) for w in widths]
    nz = int(round(height / dx))
    H = nz * dx
    c0 = 10.0 * math.sqrt(G * H)
    h = 1.3 * dx

    # fluid lattice
    fl = _grid([(0, k) for k in nh] + [(0, nz)]).astype(np.float64)
    xf = (fl + 0.5) * dx
    # boundary: every lattice site of the enlarged box that is outside the fluid box
    nwz = int(round(wall_top * height / dx))
    wl = _grid([(-nlayers, k + nlayers) for k in nh] + [(-nlayers, nwz)]).astype(np.float64)
    inside = np.all([(wl[:, d] >= 0) & (wl[:, d] < nh[d]) for d in range(dim - 1)], axis=0) \
        & (wl[:, dim - 1] >= 0)
    wl = wl[~inside]
    xw = (wl + 0.5) * dx

    ph_f = np.zeros(len(xf), np.uint8)
    if oil is not None:
        ph_f[oil(xf)] = OIL
    xf = xf + rng.uniform(-jitter * dx, jitter * dx, size=xf.shape)

    x = np.zeros((len(xf) + len(xw), 3))
    x[:len(xf), :dim] = xf
    x[len(xf):, :dim] = xw
    n = len(x)
    phase = np.concatenate([ph_f, np.zeros(len(xw), np.uint8)])
    kind = np.concatenate([np.full(len(xf), FLUID, np.uint8), np.full(len(xw), WALL, np.uint8)])
    rho0 = np.where(phase == OIL, rho_o, rho_w)
    rho = _hydrostatic_rho(x[:, dim - 1], H, rho0, rho_w, c0, G)
    m = rho0 * dx ** dim
    u = np.zeros((n, 3))
    if perturb:
        fluid = kind == FLUID
        u[fluid, :dim] = rng.uniform(-0.05 * c0, 0.05 * c0, size=(int(fluid.sum()), dim))
        rho = rho * (1.0 + rng.uniform(-0.005, 0.005, size=n))

    p = default_params(dim, h)
    p["alpha_s"] = alpha_s if oil is not None else 0.0
    grav = [0.0, 0.0, 0.0]
    grav[dim - 1] = -G
    p["gravity"] = grav
    lo = [0.0, 0.0, 0.0]
    hi = [0.0, 0.0, 0.0]
    for d in range(dim - 1):
        lo[d] = -nlayers * dx
        hi[d] = (nh[d] + nlayers) * dx
    lo[dim - 1] = -nlayers * dx
    hi[dim - 1] = headroom * H
    p["lo"], p["hi"] = lo, hi
    phases = [(rho_w, mu_w / rho_w, c0), (rho_o, mu_o / rho_o, c0)]
    return Scene(name, dim, [p], [phases], x, u, rho, m, phase, kind,
                 np.array([0, n], np.int64), [dx], seed)


def drop(dim, centre, R):
    c = np.asarray(centre, float)

    def mask(pts):
        return np.sum((pts - c[None, :dim]) ** 2, axis=1) < R * R
    return mask


def drop2d(k_seed: int = 0, *, dx=2.5e-3, perturb=False, **kw) -> Scene:
    """2D oil drop rising in still water: 0.1 x 0.1 m tank, R = 0.01 m at (0.05, 0.03)."""
    return tank(2, 0.1, 0.1, dx, seed=SEED_BASE + k_seed, oil=drop(2, (0.05, 0.03), 0.01),
                perturb=perturb, name="drop2d", **kw)


def drop3d(k_seed: int = 1, *, dx=1e-3, scale=1.0, perturb=False, **kw) -> Scene:
    """3D oil drop rising: box 0.05 x 0.05 x 0.1 m, sphere R = 5 mm at z = 0.015 m.

    ``scale`` shrinks the box and the drop together at fixed ``dx`` (smaller
    parity cases with the same structure)."""
    Wd, H, R = 0.05 * scale, 0.1 * scale, 5e-3 * scale
    return tank(3, (Wd, Wd), H, dx, seed=SEED_BASE + k_seed,
                oil=drop(3, (Wd / 2, Wd / 2, 0.015 * scale), R), perturb=perturb,
                name="drop3d", **kw)


def paper_drop(shape: str = "sphere", k_seed: int = 5, *, dx=5e-3, perturb=False, **kw) -> Scene:
    """The paper's two drop tests (Sec. III): a still water tank 0.2 m on a side filled
    to 0.2 m, particle size 5 mm (40^3 = 64,000 fluid particles), interfacial tension
    0.05 N/m, an oil sphere of diameter 0.04 m or an oil cube of side 0.04 m whose
    centre lies 0.16 m below the free surface.  Oil density and viscosity are not
    given there; the tank's defaults stand in for them."""
    side, depth, size = 0.2, 0.2, 0.04
    H = int(round(depth / dx)) * dx
    c = np.array([side / 2, side / 2, H - 0.16])
    if shape == "sphere":
        oil = drop(3, c, size / 2)
    elif shape == "cube":
        def oil(pts):
            return np.all(np.abs(pts - c[None, :3]) < size / 2, axis=1)
    else:
        raise ValueError("shape must be 'sphere' or 'cube'")
    kw.setdefault("alpha_s", 0.05)
    return tank(3, (side, side), depth, dx, seed=SEED_BASE + k_seed, oil=oil, perturb=perturb,
                name=f"paper_{shape}", **kw)


def still_tank(dim=2, *, dx=2.5e-3, width=0.1, height=0.1, seed=SEED_BASE, **kw) -> Scene:
    """Single-phase still water tank (hydrostatic column)."""
    wd = width if dim == 2 else (width, width)
    return tank(dim, wd, height, dx, seed=seed, oil=None, name="still_tank", **kw)


def lattice_box(dim: int, n: int, dx: float = 1.0, *, rho0=1000.0, nu=1e-6, c0=10.0,
                periodic=True, oil=None, rho_o=900.0, nu_o=5e-6) -> Scene:
    """Perfect ``n**dim`` lattice in a periodic box of side ``n*dx``, no walls, g = 0."""
    pts = _grid([(0, n)] * dim).astype(np.float64)
    xs = (pts + 0.5) * dx
    x = np.zeros((len(xs), 3))
    x[:, :dim] = xs
    phase = np.zeros(len(xs), np.uint8)
    if oil is not None:
        phase[oil(xs)] = OIL
    kind = np.zeros(len(xs), np.uint8)
    r0 = np.where(phase == OIL, rho_o, rho0)
    p = default_params(dim, 1.3 * dx)
    p["lo"] = [0.0, 0.0, 0.0]
    p["hi"] = [n * dx if d < dim else 0.0 for d in range(3)]
    p["periodic"] = [1 if (periodic and d < dim) else 0 for d in range(3)]
    phases = [(rho0, nu, c0), (rho_o, nu_o, c0)]
    return Scene("lattice", dim, [p], [phases], x, np.zeros_like(x), r0.copy(),
                 r0 * dx ** dim, phase, kind, np.array([0, len(xs)], np.int64), [dx], None)


def laplace_drop2d(*, dx=1e-3, R=0.02, box=0.08, alpha_s=0.02, mu=0.05, c0=1.0,
                   seed=SEED_BASE + 100) -> Scene:
    """Static 2D drop in a closed walled box full of fluid, g = 0, equal densities.

    Used for the Laplace pressure jump ``p_in - p_out = alpha_s / R``."""
    rng = np.random.default_rng(seed)
    nb = int(round(box / dx))
    fl = _grid([(0, nb), (0, nb)]).astype(np.float64)
    xf = (fl + 0.5) * dx
    wl = _grid([(-3, nb + 3), (-3, nb + 3)]).astype(np.float64)
    inside = (wl[:, 0] >= 0) & (wl[:, 0] < nb) & (wl[:, 1] >= 0) & (wl[:, 1] < nb)
    xw = (wl[~inside] + 0.5) * dx
    c = np.array([box / 2, box / 2])
    ph = (np.sum((xf - c) ** 2, axis=1) < R * R).astype(np.uint8)
    xf = xf + rng.uniform(-0.01 * dx, 0.01 * dx, size=xf.shape)
    x = np.zeros((len(xf) + len(xw), 3))
    x[:len(xf), :2] = xf
    x[len(xf):, :2] = xw
    n = len(x)
    phase = np.concatenate([ph, np.zeros(len(xw), np.uint8)])
    kind = np.concatenate([np.zeros(len(xf), np.uint8), np.ones(len(xw), np.uint8)])
    rho = np.full(n, 1000.0)
    m = rho * dx * dx
    p = default_params(2, 1.3 * dx)
    p["alpha_s"] = alpha_s
    p["lo"] = [-3 * dx, -3 * dx, 0.0]
    p["hi"] = [(nb + 3) * dx, (nb + 3) * dx, 0.0]
    phases = [(1000.0, mu / 1000.0, c0), (1000.0, mu / 1000.0, c0)]
    return Scene("laplace2d", 2, [p], [phases], x, np.zeros((n, 3)), rho, m, phase, kind,
                 np.array([0, n], np.int64), [dx], seed)


def isolated_particles(dim=3, n=1, *, spacing=1.0, h=0.01, u0=(0.3, -0.2, 0.5)) -> Scene:
    """Particles too far apart to interact: each moves under gravity alone."""
    x = np.zeros((n, 3))
    x[:, 0] = np.arange(n) * spacing + 0.5
    x[:, 1] = 0.5
    if dim == 3:
        x[:, 2] = 0.5
    u = np.zeros((n, 3))
    u[:, :dim] = np.asarray(u0[:dim])
    p = default_params(dim, h)
    grav = [0.0, 0.0, 0.0]
    grav[dim - 1] = -G
    p["gravity"] = grav
    p["lo"] = [-100.0, -100.0, -100.0 if dim == 3 else 0.0]
    p["hi"] = [100.0, 100.0, 100.0 if dim == 3 else 0.0]
    phases = [(1000.0, 1e-6, 10.0)]
    return Scene("isolated", dim, [p], [phases], x, u, np.full(n, 1000.0), np.full(n, 1e-3),
                 np.zeros(n, np.uint8), np.zeros(n, np.uint8), np.array([0, n], np.int64),
                 [h / 1.3], None)


# ----------------------------------------------------------------- flumes

def _dispersion_k(omega, depth):
    """Wavenumber of linear gravity waves, omega^2 = g k tanh(k depth) (Newton)."""
    k = omega * omega / G
    for _ in range(60):
        f = G * k * math.tanh(k * depth) - omega * omega
        df = G * math.tanh(k * depth) + G * k * depth / math.cosh(k * depth) ** 2
        k -= f / df
    return k


def focused_piston(seed: int, depth: float, x_focus: float, amplitude=0.08, ncomp=8,
                   periods=(0.7, 1.2)):
    """Piston displacement d(t) = sum a_k (cos(w_k t + phi_k) - cos phi_k) whose
    components reach x_focus in phase.  Component wave amplitudes are equal and sum to
    ``amplitude``; each paddle amplitude follows the linear piston transfer function
    H/S = 2 (cosh 2kh - 1) / (sinh 2kh + 2kh).  The focus time is the arrival of the
    slowest group.  Returns the piston entries of a parameter dictionary."""
    rng = np.random.default_rng(seed)
    T = np.sort(rng.uniform(periods[0], periods[1], ncomp))
    w = 2 * math.pi / T
    ks = np.array([_dispersion_k(wi, depth) for wi in w])
    kh = ks * depth
    transfer = 2 * (np.cosh(2 * kh) - 1) / (np.sinh(2 * kh) + 2 * kh)
    A = amplitude / ncomp
    ap = A / transfer                       # paddle amplitude = (H/2) / (H/S)
    cg = 0.5 * (w / ks) * (1 + 2 * kh / np.sinh(2 * kh))
    t_f = x_focus / cg.min()
    theta = w * t_f - ks * x_focus          # crest phase at the paddle
    # paddle x(t) = ap sin(w t - theta) = ap cos(w t - theta - pi/2)
    phi = -theta - math.pi / 2
    return dict(piston_a=list(ap), piston_w=list(w), piston_phi=list(phi),
                piston_t_end=1e30), dict(t_focus=t_f, periods=list(T), paddle=list(ap))


def flume(dim: int, length: float, depth: float, dx: float, *, seed: int, width=None,
          slick=None, rho_o=850.0, mu_o=0.01, alpha_s=0.02, piston=None, nlayers=3,
          wall_top=1.2, headroom=1.6, back=0.1, jitter=0.05, name="flume") -> Scene:
    """Wave flume: piston (MOVING) at x = 0, end wall at x = length, bottom wall, open
    top; in 3D the width is periodic.  ``slick(points) -> mask`` marks oil lattice
    points.  ``back`` is room behind the piston for its backward stroke."""
    rng = np.random.default_rng(seed)
    nx = int(round(length / dx))
    nz = int(round(depth / dx))
    H = nz * dx
    c0 = 10.0 * math.sqrt(G * H)
    h = 1.3 * dx
    ny = int(round(width / dx)) if dim == 3 else 1
    if dim == 2:
        fl = _grid([(0, nx), (0, nz)]).astype(np.float64)
    else:
        fl = _grid([(0, nx), (0, ny), (0, nz)]).astype(np.float64)
    xf = (fl + 0.5) * dx
    nwz = int(round(wall_top * depth / dx))
    zax = dim - 1
    # bottom: under the whole flume and under the piston/end wall columns
    if dim == 2:
        bot = _grid([(-nlayers, nx + nlayers), (-nlayers, 0)])
        end = _grid([(nx, nx + nlayers), (0, nwz)])
        pis = _grid([(-nlayers, 0), (0, nwz)])
    else:
        bot = _grid([(-nlayers, nx + nlayers), (0, ny), (-nlayers, 0)])
        end = _grid([(nx, nx + nlayers), (0, ny), (0, nwz)])
        pis = _grid([(-nlayers, 0), (0, ny), (0, nwz)])
    xw = (np.concatenate([bot, end]).astype(np.float64) + 0.5) * dx
    xp = (pis.astype(np.float64) + 0.5) * dx
    ph_f = np.zeros(len(xf), np.uint8)
    if slick is not None:
        ph_f[slick(xf)] = OIL
    xf = xf + rng.uniform(-jitter * dx, jitter * dx, size=xf.shape)
    if dim == 3:
        xf[:, 1] = np.mod(xf[:, 1], ny * dx)
    n = len(xf) + len(xw) + len(xp)
    x = np.zeros((n, 3))
    x[:len(xf), :dim] = xf
    x[len(xf):len(xf) + len(xw), :dim] = xw
    x[len(xf) + len(xw):, :dim] = xp
    phase = np.concatenate([ph_f, np.zeros(len(xw) + len(xp), np.uint8)])
    kind = np.concatenate([np.full(len(xf), FLUID, np.uint8), np.full(len(xw), WALL, np.uint8),
                           np.full(len(xp), MOVING, np.uint8)])
    rho0 = np.where(phase == OIL, rho_o, 1000.0)
    rho = _hydrostatic_rho(x[:, zax], H, rho0, 1000.0, c0, G)
    m = rho0 * dx ** dim
    p = default_params(dim, h)
    p["alpha_s"] = alpha_s if slick is not None else 0.0
    grav = [0.0, 0.0, 0.0]
    grav[zax] = -G
    p["gravity"] = grav
    lo, hi, per = [0.0] * 3, [0.0] * 3, [0, 0, 0]
    lo[0], hi[0] = -nlayers * dx - back, (nx + nlayers) * dx
    if dim == 3:
        lo[1], hi[1], per[1] = 0.0, ny * dx, 1
    lo[zax], hi[zax] = -nlayers * dx, headroom * H
    p["lo"], p["hi"], p["periodic"] = lo, hi, per
    if piston:
        p.update(piston)
    phases = [(1000.0, 1e-3 / 1000.0, c0), (rho_o, mu_o / rho_o, c0)]
    return Scene(name, dim, [p], [phases], x, np.zeros((n, 3)), rho, m, phase, kind,
                 np.array([0, n], np.int64), [dx], seed)


def flume2d(k_seed: int = 2, *, dx=5e-3, length=8.0, depth=0.5, x_focus=5.0) -> Scene:
    """2D breaking-wave flume: 8 m, depth 0.5 m, focused piston wave at x = 5 m; oil
    layer 4 particles thick, 0.5 m long, centred at x_focus (rho 850, mu 0.01, sigma 0.02)."""
    seed = SEED_BASE + k_seed
    piston, _ = focused_piston(seed, depth, x_focus)
    H = int(round(depth / dx)) * dx

    def slick(pts):
        return (np.abs(pts[:, 0] - x_focus) < 0.25) & (pts[:, 1] > H - 4 * dx)
    return flume(2, length, depth, dx, seed=seed, slick=slick, piston=piston, name="flume2d")


def flume3d(k_seed: int = 3, *, dx=4e-3, length=4.0, width=0.1, depth=0.5,
            x_focus=2.5) -> Scene:
    """3D flume section: 4 m x 0.1 m (periodic in y), depth 0.5 m, focused piston wave
    (focus inside the section, x = 2.5 m); oil slick 3 particles thick over
    0.3 x 0.1 m centred at the focus."""
    seed = SEED_BASE + k_seed
    piston, _ = focused_piston(seed, depth, x_focus)
    H = int(round(depth / dx)) * dx

    def slick(pts):
        return (np.abs(pts[:, 0] - x_focus) < 0.15) & (pts[:, 2] > H - 3 * dx)
    return flume(3, length, depth, dx, seed=seed, width=width, slick=slick, piston=piston,
                 name="flume3d")


def lab_flume(dim: int = 2, *, dx=5e-3, width=0.05, seed=SEED_BASE + 10) -> Scene:
    """The paper's laboratory flume (Sec. IV): 6 m long and 0.6 m high, water depth
    0.25 m, piston at x = 0.55 m driven by Eq. (18) (stroke 45.72 cm at 0.75 Hz,
    t <= 2/3 s), oil slick 25.4 cm long and 0.5 mm thick (one particle layer at this
    resolution) centred at x = 1.5 m, interfacial tension 0.019 N/m; in 3D a narrowed
    periodic width.  The piston and end wall are the flume's height; the domain reaches
    0.75 m, so that water running up the piston stays inside it."""
    stroke = 0.4572
    piston = dict(piston_a=[-stroke / 2], piston_w=[2 * math.pi * 0.75], piston_phi=[0.0],
                  piston_t_end=2.0 / 3.0)
    length = 6.0 - 0.55
    depth = 0.25
    H = int(round(depth / dx)) * dx
    xs = 1.5 - 0.55                         # slick centre in flume coordinates

    def slick(pts):
        top = pts[:, dim - 1] > H - max(5e-4, dx)
        return (np.abs(pts[:, 0] - xs) < 0.127) & top
    return flume(dim, length, depth, dx, seed=seed, width=width if dim == 3 else None,
                 slick=slick, piston=piston, rho_o=900.0, mu_o=5e-3, alpha_s=0.019,
                 back=0.05, wall_top=0.6 / depth, headroom=0.75 / depth, name="lab_flume")


def batched_drops(k_seed: int = 4, ninst: int = 256, nmin=2000, nmax=40000) -> Scene:
    """Independent 2D drop tanks of uneven sizes: each 0.1 x 0.1 m with
    dx = 0.1 / round(sqrt(n_fluid)), n_fluid ~ U[nmin, nmax]; drop radius U[5, 15] mm at
    (0.05, 0.03); oil density U[800, 950], viscosity U[1e-3, 2e-2], tension U[0.01, 0.05]."""
    ss = np.random.SeedSequence(SEED_BASE + k_seed)
    parts = []
    for b, child in enumerate(ss.spawn(ninst)):
        rng = np.random.default_rng(child)
        nf = int(rng.integers(nmin, nmax + 1))
        side = max(int(round(math.sqrt(nf))), 8)
        dx = 0.1 / side
        R = float(rng.uniform(5e-3, 15e-3))
        rho_o = float(rng.uniform(800.0, 950.0))
        mu_o = float(rng.uniform(1e-3, 2e-2))
        alpha = float(rng.uniform(0.01, 0.05))
        seed = int(rng.integers(0, 2 ** 31))
        parts.append(tank(2, 0.1, 0.1, dx, seed=seed, oil=drop(2, (0.05, 0.03), R),
                          rho_o=rho_o, mu_o=mu_o, alpha_s=alpha, name=f"tank{b}"))
    return concat("batched_drops", parts)
