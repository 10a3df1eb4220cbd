"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test ties one oracle function to something other than itself: a closed
form, an integral identity, a lattice sum of the closed-form kernel
(``tests/golden/lattice_constants.json``), an invariance or scaling law, a
brute-force search, or the numbers the paper prints (Eq. (18)).  Every test
here runs on the CPU.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy import integrate

import oracle
from paper_1702_07760_amd import inputs

HERE = os.path.dirname(os.path.abspath(__file__))
with open(os.path.join(HERE, "golden", "lattice_constants.json")) as fh:
    LAT = json.load(fh)
with open(os.path.join(HERE, "golden", "wavemaker_eq18.json")) as fh:
    EQ18 = json.load(fh)


def kappa(dim):
    return LAT[f"{dim}d"]["moment"]


def block(dim, n, dx=1.0, **kw):
    """Non-periodic perfect lattice block, g = 0; interior = >= 2h from every face."""
    s = inputs.lattice_box(dim, n, dx, periodic=False, **kw)
    h = 1.3 * dx
    x = s.x[:, :dim]
    interior = np.all((x > 2 * h) & (x < n * dx - 2 * h), axis=1)
    return s, interior


# ---------------------------------------------------------------- kernel W

@pytest.mark.parametrize("dim", [2, 3])
def test_kernel_normalised(dim):
    h = 0.37
    shell = (lambda r: 2 * math.pi * r) if dim == 2 else (lambda r: 4 * math.pi * r * r)
    val, _ = integrate.quad(lambda r: oracle.kernel_w(dim, h, r) * shell(r), 0, 2 * h,
                            epsabs=1e-14, epsrel=1e-13)
    assert abs(val - 1.0) < 1e-11


@pytest.mark.parametrize("dim", [2, 3])
def test_kernel_gradient_matches_finite_difference(dim):
    h = 0.37
    for q in (0.05, 0.3, 0.9, 1.4, 1.9):
        r = q * h
        e = 1e-6 * h
        dwdr = (oracle.kernel_w(dim, h, r + e) - oracle.kernel_w(dim, h, r - e)) / (2 * e)
        # grad_i W_ij = F r_ij, so dW/dr = F r
        assert oracle.kernel_f(dim, h, r) * r == pytest.approx(dwdr, rel=1e-7)


@pytest.mark.parametrize("dim", [2, 3])
def test_kernel_compact_support(dim):
    h = 0.5
    assert oracle.kernel_w(dim, h, 2 * h) == 0.0
    assert oracle.kernel_f(dim, h, 2 * h) == 0.0
    assert oracle.kernel_w(dim, h, 2 * h * (1 - 1e-9)) > 0.0
    assert oracle.kernel_f(dim, h, 0.0) < 0.0   # finite at r = 0, no 1/r


# ----------------------------------------------------------- neighbours

@pytest.mark.parametrize("dim", [2, 3])
def test_lattice_neighbour_count(dim):
    s = inputs.lattice_box(dim, 12, 1.0, periodic=True)
    o = oracle.Oracle(s)
    off, _ = o.neighbors()
    assert np.all(np.diff(off) == LAT[f"{dim}d"]["count"])


def _numpy_pairs(s):
    p = s.params[0]
    dim = s.dim
    x = s.x[:, :dim]
    r = x[:, None, :] - x[None, :, :]
    for d in range(dim):
        if p["periodic"][d]:
            L = p["hi"][d] - p["lo"][d]
            r[..., d] = np.where(r[..., d] > 0.5 * L, r[..., d] - L,
                                 np.where(r[..., d] < -0.5 * L, r[..., d] + L, r[..., d]))
    r2 = (r ** 2).sum(-1)
    np.fill_diagonal(r2, np.inf)
    return r2 < 4 * p["h"] ** 2


@pytest.mark.parametrize("case", ["drop2d", "periodic3d", "drop3d_small"])
def test_neighbours_brute_cells_numpy_agree(case):
    if case == "drop2d":
        s = inputs.drop2d(perturb=True)
    elif case == "periodic3d":
        s = inputs.lattice_box(3, 10, 1.0, periodic=True)
        rng = np.random.default_rng(5)
        s.x[:, :3] = np.mod(s.x[:, :3] + rng.uniform(-0.3, 0.3, s.x[:, :3].shape), 10.0)
    else:
        s = inputs.drop3d(scale=0.25)
    o = oracle.Oracle(s)
    o.set_neighbor_method(1)
    off_b, idx_b = o.neighbors()
    o.set_neighbor_method(2)
    off_c, idx_c = o.neighbors()
    assert np.array_equal(off_b, off_c) and np.array_equal(idx_b, idx_c)
    if s.n <= 4000:
        mask = _numpy_pairs(s)
        for i in range(0, s.n, 7):
            assert np.array_equal(np.nonzero(mask[i])[0], idx_b[off_b[i]:off_b[i + 1]])


# --------------------------------------------------- Eq. (7) renormalisation

def test_renormalisation_preserves_uniform_density_any_support():
    s = inputs.drop2d()             # free surface, walls, drop: truncated kernels everywhere
    s.rho[:] = 1234.5
    o = oracle.Oracle(s)
    o.renormalize()
    assert np.max(np.abs(o.get(oracle.RHO) / 1234.5 - 1)) < 1e-14


def test_renormalisation_is_a_convex_combination_of_same_phase_densities():
    s = inputs.drop2d(perturb=True)
    o = oracle.Oracle(s)
    off, idx = o.neighbors()
    rho0 = s.rho.copy()
    o.renormalize()
    rn = o.get(oracle.RHO)
    for i in range(s.n):
        js = idx[off[i]:off[i + 1]]
        js = np.concatenate([[i], js[s.phase[js] == s.phase[i]]])
        assert rho0[js].min() * (1 - 1e-15) <= rn[i] <= rho0[js].max() * (1 + 1e-15)


def test_renormalisation_keeps_phases_apart_and_includes_self():
    # a flat water/oil interface at uniform per-phase density: each phase keeps its
    # own density (mixing the phases would pull both towards the average)
    s, _ = block(2, 16, oil=lambda p: p[:, 1] > 8)
    s.rho[:] = np.where(s.phase == 1, 900.0, 1000.0)
    o = oracle.Oracle(s)
    o.renormalize()
    rn = o.get(oracle.RHO)
    assert np.allclose(rn, s.rho, rtol=1e-14, atol=0)
    # an isolated particle (no neighbour): only the self term, density unchanged
    iso = inputs.isolated_particles(2, 3)
    iso.rho[:] = [990.0, 1000.0, 1010.0]
    oi = oracle.Oracle(iso)
    oi.renormalize()
    assert np.allclose(oi.get(oracle.RHO), iso.rho, rtol=1e-15, atol=0)


@pytest.mark.parametrize("dim", [2, 3])
def test_renormalisation_weights_on_a_lattice(dim):
    """Eq. (7) weights each same-phase j by m_j W_ij (numerator) and m_j W_ij / rho_j
    (denominator).  On a perfect lattice (spacing 1), with s_j = |x_j - x_c|, a mass field
    m_j = m0 (1 + a s_j^2) and a specific-volume field 1/rho_j = (1 + b s_j^2) / rho0 give
    at the centre site c, with the kernel-weighted lattice moments M2, M4 (self included):
        rho_c = rho0 (1 + a M2) / (1 + (a + b) M2 + a b M4)
    and, with a = 0, at a site i offset by s_i from c (the odd moments vanish):
        rho_i = rho0 / (1 + b (s_i^2 + M2))."""
    n = 12
    m2, m4 = LAT[f"{dim}d"]["m2"], LAT[f"{dim}d"]["m4"]
    rho0, a, b = 1000.0, 0.03, 0.02
    s = inputs.lattice_box(dim, n, 1.0, periodic=True)
    xc = np.full(dim, n / 2 + 0.5)
    d = s.x[:, :dim] - xc
    s2 = (d ** 2).sum(1)
    c = int(np.argmin(s2))
    assert s2[c] == 0.0
    s.m[:] = 1.0 * (1 + a * s2)
    s.rho[:] = rho0 / (1 + b * s2)
    o = oracle.Oracle(s)
    o.renormalize()
    want = rho0 * (1 + a * m2) / (1 + (a + b) * m2 + a * b * m4)
    assert o.get(oracle.RHO)[c] == pytest.approx(want, rel=1e-13)
    # uniform mass: every site whose support does not reach the wrap of the field
    s.m[:] = 1.0
    o = oracle.Oracle(s)
    o.renormalize()
    near = np.all(np.abs(d) <= 2.0, axis=1)
    assert near.sum() == 5 ** dim
    want = rho0 / (1 + b * (s2 + m2))
    assert np.allclose(o.get(oracle.RHO)[near], want[near], rtol=1e-13, atol=0)


# ------------------------------------------------------------- Eqs. (3)-(4)

def test_tait_equation_of_state():
    rho0, c0 = 1000.0, 9.905
    assert oracle.eos(rho0, rho0, c0) == 0.0
    e = 1e-4
    dpdrho = (oracle.eos(rho0 + e, rho0, c0) - oracle.eos(rho0 - e, rho0, c0)) / (2 * e)
    assert dpdrho == pytest.approx(c0 * c0, rel=1e-7)   # sound speed at rho0
    beta = rho0 * c0 * c0 / 7.0
    for p in (-50.0, 10.0, 981.0, 5e4):
        rho = rho0 * (1 + p / beta) ** (1 / 7)          # inverse of the Tait law
        assert oracle.eos(rho, rho0, c0) == pytest.approx(p, rel=1e-10)


# ------------------------------------------------------ Eq. (6) continuity

@pytest.mark.parametrize("dim", [2, 3])
def test_continuity_linear_velocity_gives_minus_rho_div_u(dim):
    s, interior = block(dim, 12 if dim == 3 else 20)
    A = np.array([[0.3, -0.2, 0.1], [0.05, 0.7, -0.4], [0.2, 0.1, -0.25]])[:dim, :dim]
    u = np.zeros((s.n, 3))
    u[:, :dim] = s.x[:, :dim] @ A.T
    o = oracle.Oracle(s)
    o.set(oracle.U, u)
    o.rates()
    drho = o.get(oracle.DRHO)
    want = -kappa(dim) * s.rho * np.trace(A)
    assert np.allclose(drho[interior], want[interior], rtol=1e-11)
    assert abs(kappa(dim) - 1.0) < 0.03       # lattice moment ~ continuum identity


def test_continuity_translation_and_rotation():
    s = inputs.drop2d(perturb=True)
    o = oracle.Oracle(s)
    o.set(oracle.U, np.tile([0.31, -0.12, 0.0], (s.n, 1)))
    o.rates()
    assert np.all(o.get(oracle.DRHO) == 0.0)          # u_ij = 0 exactly
    x = s.x
    u = np.zeros_like(x)
    u[:, 0], u[:, 1] = -(x[:, 1] - 0.05) * 2.0, (x[:, 0] - 0.05) * 2.0
    o.set(oracle.U, u)
    o.rates()
    # u_ij . r_ij = 0: only rounding is left, far below rho |grad u| = 1000 * 2
    assert np.max(np.abs(o.get(oracle.DRHO))) < 1e-12 * 1000.0 * 2.0


def test_volume_form_is_phase_blind_mass_form_is_not():
    # Eq. (6) uses neighbour volumes: across an oil/water interface at lattice volumes
    # it gives the same -kappa rho div u as in the bulk.  Eq. (5) weighs by mass and does not.
    s, interior = block(2, 20, oil=lambda p: p[:, 1] > 10)
    s.rho[:] = np.where(s.phase == 1, 900.0, 1000.0)
    s.m[:] = s.rho
    A = np.diag([0.4, -0.1])
    u = np.zeros((s.n, 3))
    u[:, :2] = s.x[:, :2] @ A.T
    o = oracle.Oracle(s)
    o.set(oracle.U, u)
    o.rates()
    want = -kappa(2) * s.rho * np.trace(A)
    assert np.allclose(o.get(oracle.DRHO)[interior], want[interior], rtol=1e-11)
    s5 = s.with_params(cont_form=1)
    o5 = oracle.Oracle(s5)
    o5.set(oracle.U, u)
    o5.rates()
    d5 = o5.get(oracle.DRHO)
    bulk = interior & (np.abs(s.x[:, 1] - 10) > 3)
    near = interior & (np.abs(s.x[:, 1] - 10) < 1)
    assert np.allclose(d5[bulk], want[bulk], rtol=1e-11)
    assert np.max(np.abs(d5[near] / want[near] - 1)) > 1e-3


# ------------------------------------------------------------ Eq. (8) pressure

@pytest.mark.parametrize("dim", [2, 3])
def test_pressure_gradient_of_linear_field(dim):
    s, interior = block(dim, 12 if dim == 3 else 20, dx=0.01)
    rho0, c0 = 1000.0, 100.0
    s.phases = [[(rho0, 1e-6, c0)]]
    beta = rho0 * c0 * c0 / 7.0
    G = np.array([120.0, -300.0, 450.0])[:dim]
    P = 50.0 + s.x[:, :dim] @ G
    s.rho[:] = rho0 * (1 + P / beta) ** (1 / 7)
    o = oracle.Oracle(s)
    o.rates()
    ap = o.get(oracle.AP)[:, :dim]
    want = -kappa(dim) * G[None, :] / s.rho[:, None]
    assert np.allclose(ap[interior], want[interior], rtol=1e-4, atol=0)


def _all_pairs(o):
    off, idx = o.neighbors()
    for i in range(o.n):
        for j in idx[off[i]:off[i + 1]]:
            if j > i:
                yield i, int(j)


@pytest.mark.parametrize("visc_form", [0, 1])
def test_pair_terms_exactly_antisymmetric(visc_form):
    s = inputs.drop2d(perturb=True).with_params(visc_form=visc_form)
    o = oracle.Oracle(s)
    o.rates()
    assert np.abs(o.get(oracle.GRADC)).max() > 0        # the surface-tension path is live
    checked = 0
    for i, j in _all_pairs(o):
        tij, tji = o.pair_terms(i, j), o.pair_terms(j, i)
        assert np.array_equal(tij[0:3], -tji[0:3])      # Eq. (8)
        assert np.array_equal(tij[6:9], -tji[6:9])      # Eq. (17)
        if visc_form == 1:
            assert np.array_equal(tij[3:6], -tji[3:6])  # Eq. (11)
        checked += 1
    assert checked > 10000


def test_total_momentum_of_internal_forces_vanishes():
    # periodic two-phase box, no walls: every particle is fluid, so the pressure,
    # Eq. (11) viscosity and surface-tension forces must sum to zero
    s = inputs.lattice_box(2, 24, 1e-3, periodic=True, oil=inputs.drop(2, (0.012, 0.012), 0.005))
    rng = np.random.default_rng(3)
    s.x[:, :2] = np.mod(s.x[:, :2] + rng.uniform(-1e-4, 1e-4, (s.n, 2)), 0.024)
    s.u[:, :2] = rng.uniform(-0.1, 0.1, (s.n, 2))
    s.rho *= 1 + rng.uniform(-0.005, 0.005, s.n)
    s = s.with_params(visc_form=1, alpha_s=0.02)
    o = oracle.Oracle(s)
    o.rates()
    assert np.abs(o.get(oracle.AS)).max() > 0
    for f, sf in ((oracle.AP, oracle.SAP), (oracle.AV, oracle.SAV), (oracle.AS, oracle.SAS)):
        tot = np.abs((s.m[:, None] * o.get(f)).sum(0))
        bound = (s.m * o.get(sf)).sum()
        assert np.all(tot <= 1e-12 * bound)


# ------------------------------------------------------------ viscosity

@pytest.mark.parametrize("dim", [2, 3])
def test_viscosity_linear_shear_and_quadratic_profile(dim):
    s, interior = block(dim, 12 if dim == 3 else 20, dx=1e-3)
    nu = s.phases[0][0][1]
    o = oracle.Oracle(s)
    u = np.zeros((s.n, 3))
    u[:, 0] = 3.0 * s.x[:, 1]                  # linear shear: Laplacian 0
    o.set(oracle.U, u)
    o.rates()
    av = o.get(oracle.AV)
    assert np.max(np.abs(av[interior])) < 1e-12 * o.get(oracle.SAV).max()
    u[:, 0] = s.x[:, 1] ** 2 * 1e3             # Laplacian of u_x = 2e3
    o.set(oracle.U, u)
    o.rates()
    ratio = o.get(oracle.AV)[interior, 0] / (nu * 2e3)
    # nu lap u times the lattice moment, reduced by r^2/(r^2+delta^2) <= 1
    assert np.all(ratio > 0.97 * kappa(dim)) and np.all(ratio < kappa(dim))


def test_viscosity_uses_harmonic_mean_of_the_two_phases():
    # sparse water particles (4 dx apart) in oil: each water particle only sees oil,
    # so its viscous term equals a one-phase term with the harmonic-mean viscosity
    s, interior = block(2, 20, dx=1e-3)
    ij = np.round(s.x[:, :2] / 1e-3 - 0.5).astype(int)
    water = (ij[:, 0] % 4 == 0) & (ij[:, 1] % 4 == 0)
    s.phase[:] = 1
    s.phase[water] = 0
    s.rho[:] = 1000.0
    s.m[:] = 1000.0 * 1e-6
    nu_w, nu_o = 1e-6, 9e-6
    s.phases = [[(1000.0, nu_w, 10.0), (1000.0, nu_o, 10.0)]]
    u = np.zeros((s.n, 3))
    u[:, 0] = s.x[:, 1] ** 2 * 1e3
    o = oracle.Oracle(s)
    o.set(oracle.U, u)
    o.rates()
    sel = water & interior
    assert sel.sum() >= 9
    nu_h = 2 * nu_w * nu_o / (nu_w + nu_o)           # Eq. (12)
    s1 = inputs.lattice_box(2, 20, 1e-3, periodic=False)
    s1.phases = [[(1000.0, nu_h, 10.0)]]
    o1 = oracle.Oracle(s1)
    o1.set(oracle.U, u)
    o1.rates()
    assert np.allclose(o.get(oracle.AV)[sel], o1.get(oracle.AV)[sel], rtol=1e-13, atol=0)
    # arithmetic mean would be 5e-6, harmonic 1.8e-6: the two are far apart
    s2 = inputs.lattice_box(2, 20, 1e-3, periodic=False)
    s2.phases = [[(1000.0, 0.5 * (nu_w + nu_o), 10.0)]]
    o2 = oracle.Oracle(s2)
    o2.set(oracle.U, u)
    o2.rates()
    assert not np.allclose(o.get(oracle.AV)[sel], o2.get(oracle.AV)[sel], rtol=0.1)


def test_viscosity_delta_regularises_close_pairs():
    # two particles at r ~ delta: the term carries r^2 / (r^2 + delta^2), delta = 0.1 h
    h = 0.01
    delta = 0.1 * h
    vals = {}
    for r in (delta, 2 * delta):
        s = inputs.isolated_particles(2, 2, spacing=1.0, h=h)
        s.x[1, 0] = s.x[0, 0] + r
        s.u[1, :] = 0.0
        o = oracle.Oracle(s)
        o.rates()
        vals[r] = o.get(oracle.AV)[0, 0] / oracle.kernel_f(2, h, r)
    assert vals[2 * delta] / vals[delta] == pytest.approx((4.0 / 5.0) / (1.0 / 2.0), rel=1e-12)


def test_dynamic_viscosity_form_matches_kinematic_form_for_one_phase_at_rest_density():
    s = inputs.drop2d(perturb=True)
    s.phase[:] = 0
    s.rho[:] = 1000.0
    u = s.u.copy()
    o10 = oracle.Oracle(s)
    o10.rates()
    o11 = oracle.Oracle(s.with_params(visc_form=1))
    o11.rates()
    a10, a11 = o10.get(oracle.AV), o11.get(oracle.AV)
    assert np.abs(u).max() > 0
    assert np.max(np.abs(a10 - a11)) < 1e-13 * o10.get(oracle.SAV).max()


# ----------------------------------------------- Eqs. (14)-(17) surface tension

def _flat_interface(dim=2, n=24):
    s = inputs.lattice_box(dim, n, 1.0, periodic=False, oil=lambda p: p[:, dim - 1] > n / 2)
    s.params[0]["periodic"] = [1 if d < dim - 1 else 0 for d in range(3)]
    s.rho[:] = np.where(s.phase == 1, 900.0, 1000.0)
    s.params[0]["alpha_s"] = 0.02
    return s


@pytest.mark.parametrize("dim", [2, 3])
def test_colour_gradient_has_unit_jump_across_flat_interface(dim):
    s = _flat_interface(dim, 24 if dim == 2 else 12)
    o = oracle.Oracle(s)
    o.rates()
    g = o.get(oracle.GRADC)
    c = s.x[:, :dim - 1]
    col = np.all(np.abs(c - c[0]) < 1e-12, axis=1)
    water, oil = col & (s.phase == 0), col & (s.phase == 1)
    up = g[:, dim - 1]
    assert (up[water].sum() - up[oil].sum()) == pytest.approx(kappa(dim), rel=1e-12)
    assert up[water].sum() == pytest.approx(-up[oil].sum(), rel=1e-12)
    assert np.all(up[water] >= 0) and np.all(up[oil] <= 0)   # towards the other phase
    assert np.all(np.abs(g[:, :dim - 1]) < 1e-15)
    far = np.abs(s.x[:, dim - 1] - 12.0 * (24 if dim == 2 else 12) / 24) > 3
    assert np.all(g[far] == 0.0)


def test_colour_gradient_scales_with_number_densities():
    s = _flat_interface(2, 24)
    o = oracle.Oracle(s)
    o.rates()
    g0 = o.get(oracle.GRADC)
    k = 1.7
    s2 = _flat_interface(2, 24)
    s2.m[s2.phase == 1] *= k        # sigma_oil = rho/m shrinks by k
    o2 = oracle.Oracle(s2)
    o2.rates()
    g2 = o2.get(oracle.GRADC)
    w, oi = s.phase == 0, s.phase == 1
    tiny = 1e-15 * np.abs(g0).max()
    assert np.allclose(g2[w], k * k * g0[w], rtol=1e-14, atol=tiny)     # sigma_j^-2
    assert np.allclose(g2[oi], g0[oi] / k, rtol=1e-14, atol=tiny)       # sigma_i


@pytest.mark.parametrize("dim", [2, 3])
def test_surface_stress_tensor_is_traceless_and_projects_normal(dim):
    s = inputs.drop2d(perturb=True) if dim == 2 else inputs.drop3d(scale=0.3, perturb=True)
    o = oracle.Oracle(s)
    o.rates()
    g = o.get(oracle.GRADC)
    T = o.get(oracle.TENSOR)
    a = s.params[0]["alpha_s"]
    gn = np.linalg.norm(g, axis=1)
    live = gn > 0
    assert live.sum() > 10
    assert np.all(np.abs(np.trace(T, axis1=1, axis2=2)[live]) < 1e-13 * a * gn[live])
    Tg = np.einsum("kab,kb->ka", T, g)
    want = a * gn[:, None] * (1.0 / dim - 1.0) * g
    assert np.allclose(Tg[live], want[live], rtol=1e-12, atol=1e-12 * a)
    assert np.allclose(T, np.transpose(T, (0, 2, 1)), rtol=0, atol=0)
    assert np.all(T[~live] == 0.0)


def test_surface_tension_force_on_a_circle_static():
    s = inputs.laplace_drop2d(c0=10.0)
    s.x[:, :2] = np.round(s.x[:, :2] / 1e-3 - 0.5) * 1e-3 + 0.5e-3   # perfect lattice
    o = oracle.Oracle(s)
    o.rates()
    x, aS = o.get(oracle.X), o.get(oracle.AS)
    d = x[:, :2] - 0.04
    r = np.linalg.norm(d, axis=1)
    fr = s.m * np.sum(aS[:, :2] * d / r[:, None], axis=1)
    line = (fr / r).sum() / (2 * math.pi)       # int F_r dr, = -alpha/R in the continuum
    assert -1.15 < line < -0.85
    s2 = inputs.laplace_drop2d(c0=10.0, alpha_s=0.04)
    s2.x[:] = s.x
    o2 = oracle.Oracle(s2)
    o2.rates()
    assert np.allclose(o2.get(oracle.AS), 2 * aS, rtol=1e-14, atol=1e-300)


@pytest.mark.slow
def test_laplace_pressure_jump_of_static_drop():
    s = inputs.laplace_drop2d(c0=10.0)
    o = oracle.Oracle(s)
    o.set_neighbor_method(2)
    fl = s.kind == 0
    R, h = 0.02, 1.3e-3
    jumps = []
    for k in range(12):
        o.step(100)
        o.rates()
        x, P = o.get(oracle.X), o.get(oracle.P)
        r = np.linalg.norm(x[:, :2] - 0.04, axis=1)
        jumps.append(P[fl & (r < R - 2 * h)].mean() - P[fl & (r > R + 2 * h) & (r < R + 6 * h)].mean())
    dp = np.mean(jumps[4:])
    assert 0.8 * 0.02 / R < dp < 1.1 * 0.02 / R    # alpha_s / R, p_in > p_out


# ------------------------------------------------ integration and time step

def test_isolated_particle_follows_the_free_fall_parabola():
    s = inputs.isolated_particles(3, 2).with_params(dt_fixed=1e-3)
    o = oracle.Oracle(s)
    o.step(25)
    t = 25e-3
    g = np.array(s.params[0]["gravity"])
    want = s.x + s.u * t + 0.5 * g * t * t
    assert np.allclose(o.get(oracle.X), want, rtol=0, atol=1e-14)
    assert np.allclose(o.get(oracle.U), s.u + g * t, rtol=0, atol=1e-14)
    assert o.t == pytest.approx(t, rel=1e-14)


def test_walls_stay_fixed_and_their_density_evolves():
    s = inputs.drop2d(perturb=True)
    o = oracle.Oracle(s)
    o.step(3)
    w = s.kind == 1
    assert np.array_equal(o.get(oracle.X)[w], s.x[w])
    assert np.array_equal(o.get(oracle.U)[w], s.u[w])
    assert not np.array_equal(o.get(oracle.RHO)[w], s.rho[w])


def test_time_step_respects_every_limit():
    s = inputs.drop2d(perturb=True)
    o = oracle.Oracle(s)
    o.renormalize()
    o.rates()
    dt = o.dt()
    p = s.params[0]
    h = p["h"]
    fl = s.kind == 0
    umax = np.linalg.norm(s.u[fl], axis=1).max()
    amax = np.linalg.norm(o.get(oracle.A)[fl], axis=1).max()
    c0 = max(ph[2] for ph in s.phases[0])
    assert dt * (c0 + umax) <= 0.25 * h * (1 + 1e-15)
    assert dt <= 0.25 * math.sqrt(h / amax) * (1 + 1e-15)
    nu = max(ph[1] for ph in s.phases[0])
    assert dt <= 0.125 * h * h / nu
    assert dt == pytest.approx(min(0.25 * h / (c0 + umax), 0.25 * math.sqrt(h / amax),
                                   0.125 * h * h / nu,
                                   0.25 * math.sqrt(900 * h ** 3 / (2 * math.pi * 0.02))), rel=1e-15)
    # the neighbour skin of the GPU lists is no limit of the method: the step ignores it
    o2 = oracle.Oracle(s.with_params(skin_coef=1e-6))
    o2.renormalize()
    o2.rates()
    assert o2.dt() == dt


def test_wavemaker_eq18():
    stroke, f = EQ18["stroke_m"], EQ18["frequency_hz"]
    p = inputs.default_params(2, 0.01)
    p.update(piston_a=[-stroke / 2], piston_w=[2 * math.pi * f], piston_phi=[0.0],
             piston_t_end=EQ18["t_end_s"])
    for t, want in EQ18["points"]:
        d, _ = oracle.piston(p, t)
        assert d == pytest.approx(want, abs=1e-12)
    _, v = oracle.piston(p, EQ18["peak_velocity_t_s"])
    assert v == pytest.approx(EQ18["peak_velocity_m_s"], abs=1e-4)
    d_end, v_end = oracle.piston(p, 2.0)
    assert d_end == pytest.approx(stroke, abs=1e-12) and v_end == 0.0


def _piston_params(a, w, phi, t_end):
    p = inputs.default_params(2, 0.01)
    p.update(piston_a=list(a), piston_w=list(w), piston_phi=list(phi), piston_t_end=t_end)
    return p


def test_piston_series_with_phases():
    """The focused-wave series: several components with non-zero phases start from rest
    position, the velocity is the time derivative of the displacement, the piston stops
    at t_end, and a phase phi_k = w_k tau is a time advance by tau."""
    rng = np.random.default_rng(11)
    a = rng.uniform(-0.05, 0.05, 5)
    w = 2 * math.pi / rng.uniform(0.7, 1.2, 5)
    phi = rng.uniform(-math.pi, math.pi, 5)
    t_end = 3.7
    p = _piston_params(a, w, phi, t_end)
    d0, _ = oracle.piston(p, 0.0)
    assert abs(d0) < 1e-16                                 # x(0) = x0 for any phases
    e = 1e-6
    for t in (0.1, 0.83, 1.9, 3.1):
        d, v = oracle.piston(p, t)
        dp, _ = oracle.piston(p, t + e)
        dm, _ = oracle.piston(p, t - e)
        assert v == pytest.approx((dp - dm) / (2 * e), rel=1e-7, abs=1e-9)
        assert abs(v) > 1e-3
    d_end, _ = oracle.piston(p, t_end)
    for t in (t_end + 0.01, t_end + 5.0):
        d, v = oracle.piston(p, t)
        assert d == d_end and v == 0.0
    # phase = time advance: d_phi(t) = d_0(t + tau) - d_0(tau), the same for v
    tau = 0.37
    p0 = _piston_params(a, w, [0.0] * 5, 100.0)
    pt = _piston_params(a, w, list(w * tau), 100.0)
    dz_tau, _ = oracle.piston(p0, tau)
    for t in (0.0, 0.21, 1.3, 2.9):
        d, v = oracle.piston(pt, t)
        ds, vs = oracle.piston(p0, t + tau)
        assert d == pytest.approx(ds - dz_tau, abs=1e-14)
        assert v == pytest.approx(vs, abs=1e-13)


@pytest.mark.slow
def test_hydrostatic_column_time_averaged_pressure():
    s = inputs.still_tank(2)
    o = oracle.Oracle(s)
    o.set_neighbor_method(2)
    H, dx = 0.1, 2.5e-3
    fl = s.kind == 0
    o.step(200)
    prof = []
    for k in range(60):
        o.step(25)
        o.rates()
        z = o.get(oracle.X)[fl, 1]
        b = np.floor(z / (4 * dx)).astype(int)
        P = o.get(oracle.P)[fl]
        prof.append(np.bincount(b, weights=P, minlength=10)[:9] / np.bincount(b, minlength=10)[:9])
    zc = (np.arange(9) * 4 + 2) * dx
    ratio = np.mean(prof, axis=0) / (1000.0 * 9.81 * (H - zc))
    assert np.all(np.abs(ratio - 1) < 0.05)
    u = o.get(oracle.U)[fl]
    assert np.abs(u).max() < 0.1 * math.sqrt(9.81 * H)


def test_oracle_is_deterministic():
    s = inputs.drop2d(perturb=True)
    a, b = oracle.Oracle(s), oracle.Oracle(s)
    oracle.set_threads(1)
    a.step(2)
    oracle.set_threads(os.cpu_count() or 1)
    b.step(2)
    for f in (oracle.X, oracle.U, oracle.RHO):
        assert np.array_equal(a.get(f), b.get(f))


def test_set_moving_prescribes_a_linear_motion():
    # after so_set_moving(disp, vel) the MOVING particles sit at x0 + disp + vel (t - t_call)
    # with velocity vel at every later step, whatever the piston series says; the fluid
    # still moves with its own velocity
    s = inputs.flume2d(dx=0.02, length=2.0, depth=0.3, x_focus=1.0)
    mov = s.kind == inputs.MOVING
    x0 = s.x[mov].copy()
    o = oracle.Oracle(s)
    o.step(2)
    t_call = o.t
    disp, vel = np.array([0.004, -0.001, 0.0]), np.array([0.15, 0.05, 0.0])
    o.set_moving(disp, vel)
    # placed on the new motion at once
    assert np.allclose(o.get(oracle.X)[mov], x0 + disp, rtol=0, atol=1e-15)
    assert np.all(o.get(oracle.U)[mov] == vel)
    o.step(3)
    t = o.t
    x, u = o.get(oracle.X), o.get(oracle.U)
    want = x0 + (disp + vel * (t - t_call))
    assert np.allclose(x[mov], want, rtol=0, atol=1e-15)
    assert np.all(u[mov] == vel)
    assert not np.allclose(u[~mov], 0.0)
    # a second call restarts the line from the time of that call
    t2 = o.t
    o.set_moving([0.0, 0.0, 0.0], [-0.1, 0.0, 0.0])
    o.step(2)
    assert np.allclose(o.get(oracle.X)[mov], x0 + np.array([-0.1, 0.0, 0.0]) * (o.t - t2), rtol=0, atol=1e-15)
