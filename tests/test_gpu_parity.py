"""GPU library against the FP64 oracle, through the C ABI.

Bars: neighbour sets bit-exact in the FP64 form; rates and one full step
within 1e-12 (FP64) and 1e-5 (FP32 cell-relative) in the E-norm of
``tests/parity.py`` (positions in units of dx, density relative to rho0,
velocity relative to the largest oracle speed).
"""
import numpy as np
import pytest

import oracle
from paper_1702_07760_amd import binding, inputs

from parity import enorm, rel_to

pytestmark = pytest.mark.gpu

TOL = {binding.FP64: 1e-12, binding.FP32_CELLREL: 1e-5}
PRECS = [binding.FP64, binding.FP32_CELLREL]


def periodic_drop(dim, n=24, seed=11):
    """Periodic two-phase box, jittered, with seeded velocities (no walls)."""
    dx = 1e-3
    c = (n * dx / 2,) * dim
    s = inputs.lattice_box(dim, n, dx, periodic=True, oil=inputs.drop(dim, c, n * dx / 5),
                           c0=5.0)
    rng = np.random.default_rng(seed)
    L = n * dx
    s.x[:, :dim] = np.mod(s.x[:, :dim] + rng.uniform(-0.1 * dx, 0.1 * dx, (s.n, dim)), L)
    s.u[:, :dim] = rng.uniform(-0.2, 0.2, (s.n, dim))
    s.rho *= 1 + rng.uniform(-0.005, 0.005, s.n)
    s.params[0]["alpha_s"] = 0.02
    s.params[0]["gravity"] = [0.0, -9.81, 0.0] if dim == 2 else [0.0, 0.0, -9.81]
    return s


def jitter_mass(s, seed=21, amp=0.01):
    """Per-particle masses m (1 + U[-amp, amp]): no instance has one mass per phase."""
    rng = np.random.default_rng(seed)
    s.m = s.m * (1 + rng.uniform(-amp, amp, s.n))
    return s


SCENES = {
    "drop2d": lambda: inputs.drop2d(perturb=True),
    "drop2d_varmass": lambda: jitter_mass(inputs.drop2d(perturb=True)),
    "drop3d_varmass": lambda: jitter_mass(inputs.drop3d(scale=0.3, perturb=True)),
    "drop3d_small": lambda: inputs.drop3d(scale=0.3, perturb=True),
    "periodic2d": lambda: periodic_drop(2),
    "periodic3d": lambda: periodic_drop(3, 14),
    "drop2d_eq11_eq5": lambda: inputs.drop2d(perturb=True).with_params(visc_form=1, cont_form=1),
}


@pytest.fixture(scope="module")
def oracle_rates():
    cache = {}

    def get(name):
        if name not in cache:
            s = SCENES[name]()
            o = oracle.Oracle(s)
            o.renormalize()
            o.rates()
            cache[name] = (s, {f: o.get(f) for f in (oracle.RHO, oracle.DRHO, oracle.A, oracle.AP,
                                                      oracle.AV, oracle.AS, oracle.SDRHO,
                                                      oracle.SAP, oracle.SAV, oracle.SAS,
                                                      oracle.GRADC, oracle.P)}, o.neighbors())
        return cache[name]
    return get


@pytest.mark.parametrize("name", ["drop2d", "drop3d_small", "periodic2d", "periodic3d"])
def test_neighbour_sets_bit_exact_fp64(name, oracle_rates):
    s, _, (off, ids) = oracle_rates(name)
    print(f"case neighbours {name} n={s.n}", flush=True)
    sim = binding.Sim(s, precision=binding.FP64)
    goff, gids = sim.get_neighbors()
    assert np.array_equal(goff, off)
    assert np.array_equal(gids, ids)


@pytest.mark.parametrize("name", ["drop2d", "drop3d_small", "periodic2d", "periodic3d"])
def test_neighbour_sets_fp32_cell_relative(name, oracle_rates):
    # FP32 offsets may move a pair across the cutoff only within rounding of 2h
    s, _, (off, ids) = oracle_rates(name)
    sim = binding.Sim(s, precision=binding.FP32_CELLREL)
    goff, gids = sim.get_neighbors()
    a = {(i, int(j)) for i in range(s.n) for j in ids[off[i]:off[i + 1]]}
    b = {(i, int(j)) for i in range(s.n) for j in gids[goff[i]:goff[i + 1]]}
    diff = a ^ b
    x = s.x
    h = s.params[0]["h"]
    for i, j in diff:
        r = np.linalg.norm(x[i] - x[j])
        assert abs(r - 2 * h) < 1e-5 * h
    assert len(diff) <= 1e-4 * len(a)


@pytest.mark.parametrize("lanes", [1, 2, 4])
@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("name", list(SCENES))
def test_rates_match_oracle(name, prec, lanes, oracle_rates):
    s, ref, _ = oracle_rates(name)
    print(f"case rates {name} precision={prec} lanes={lanes} n={s.n}", flush=True)
    sim = binding.Sim(s, precision=prec)
    sim.set_option(binding.OPT_LANES, lanes)
    sim.set_option(binding.OPT_FORCE_LANES, lanes)
    sim.set_option(binding.OPT_DEBUG_TERMS, 1)
    sim.renormalize_density()
    sim.compute_forces()
    sim.sync()
    tol = TOL[prec]
    rho0 = max(p[0] for p in s.phases[0])
    assert rel_to(sim.get_field(binding.F_RHO), ref[oracle.RHO], rho0) < tol
    assert enorm(sim.get_field(binding.F_DRHO), ref[oracle.DRHO], ref[oracle.SDRHO]) < tol
    for f, g, sc in ((binding.F_AP, oracle.AP, oracle.SAP), (binding.F_AV, oracle.AV, oracle.SAV),
                     (binding.F_AS, oracle.AS, oracle.SAS)):
        if np.max(ref[sc]) > 0:
            assert enorm(sim.get_field(f), ref[g], ref[sc]) < tol, f
    total_scale = ref[oracle.SAP] + ref[oracle.SAV] + ref[oracle.SAS]
    assert enorm(sim.get_field(binding.F_A), ref[oracle.A], total_scale) < tol
    gref = ref[oracle.GRADC]
    if np.abs(gref).max() > 0:
        assert rel_to(sim.get_field(binding.F_GRADC), gref, np.abs(gref).max()) < 10 * tol
    P = sim.get_field(binding.F_P)
    assert rel_to(P, ref[oracle.P], np.abs(ref[oracle.P]).max()) < 10 * tol


def test_colour_walks_cover_both_forms():
    # the colour pass (Eq. (16)) walks its work list with a whole wave per particle when
    # the list fits the launch that way (count * 64 lanes within the colour blocks of the
    # derive launch: 8 threads per particle, at most 1024 blocks of 256), else with 8
    # lanes per particle grid-stride; the scenes of the rate tests take both forms
    forms = {}
    for name in ("drop2d", "periodic2d", "periodic3d", "drop3d_small"):
        s = SCENES[name]()
        sim = binding.Sim(s, precision=binding.FP64)
        count = sim.stats()["colour_particles"]
        nthr = min(-(-8 * s.n // 256), 1024) * 256
        forms[name] = count * 64 <= nthr
        print(f"  {name}: n={s.n} colour list {count}: {'wave per particle' if forms[name] else '8 lanes'}",
              flush=True)
        assert 0 < count < s.n
        sim.close()
    assert set(forms.values()) == {True, False}


def _one_step(scene, prec, nsteps=1, lanes=1):
    o = oracle.Oracle(scene)
    o.step(nsteps)
    sim = binding.Sim(scene, precision=prec)
    sim.set_option(binding.OPT_LANES, lanes)
    sim.set_option(binding.OPT_FORCE_LANES, lanes)
    sim.step(nsteps)
    sim.sync()
    return o, sim


@pytest.mark.parametrize("lanes", [1, 4])
@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("name", ["drop2d", "drop3d_small", "periodic3d", "drop2d_eq11_eq5", "drop2d_varmass"])
def test_one_step_matches_oracle(name, prec, lanes):
    s = SCENES[name]()
    print(f"case step {name} precision={prec} lanes={lanes} n={s.n}", flush=True)
    o, sim = _one_step(s, prec, lanes=lanes)
    dx = s.dx[0]
    rho0 = max(p[0] for p in s.phases[0])
    ur = np.abs(o.get(oracle.U)).max()
    tol = TOL[prec]
    assert abs(sim.stats()["t"] - o.t) <= 1e-6 * o.t if prec else abs(sim.stats()["t"] - o.t) <= 1e-13 * o.t
    assert rel_to(sim.get_field(binding.F_X), o.get(oracle.X), dx) < tol
    assert rel_to(sim.get_field(binding.F_U), o.get(oracle.U), ur) < tol
    assert rel_to(sim.get_field(binding.F_RHO), o.get(oracle.RHO), rho0) < tol


def test_neighbour_sets_stay_exact_after_gpu_steps():
    # after GPU steps, the oracle rebuilt at the GPU's own positions finds the same sets
    s = inputs.drop2d(perturb=True)
    sim = binding.Sim(s, precision=binding.FP64)
    sim.step(5)
    s2 = inputs.drop2d(perturb=True)
    s2.x[:] = sim.get_field(binding.F_X)
    o = oracle.Oracle(s2)
    off, ids = o.neighbors()
    goff, gids = sim.get_neighbors()
    assert np.array_equal(goff, off) and np.array_equal(gids, ids)


def _blob_lists(blob, s):
    """Positions, velocities (sorted order) and the neighbour list of an FP64 state blob:
    a 48-byte header, then pos, vel, aux (32 B per particle each), key, id, info (4 B),
    the cell table (4 B per cell + 1), the run block (64 B per instance), acc and gc
    (32 B), the list (entry e of particle i at 4 (e s + i), s = n rounded up to 32) and
    the counts (4 B)."""
    n = int(np.frombuffer(blob, np.int64, 1, 24)[0])
    ncell = int(np.frombuffer(blob, np.uint32, 1, 32)[0])
    cap = int(np.frombuffer(blob, np.uint32, 1, 40)[0])
    at = 48
    pos = np.frombuffer(blob, np.float64, 4 * n, at).reshape(n, 4)[:, :3]
    vel = np.frombuffer(blob, np.float64, 4 * n, at + 32 * n).reshape(n, 4)[:, :3]
    at += 96 * n + 12 * n + 4 * (ncell + 1) + 64 * s.ninst + 64 * n
    ls = (n + 31) // 32 * 32
    nbl = np.frombuffer(blob, np.uint32, ls * cap, at).reshape(cap, ls)
    nbc = np.frombuffer(blob, np.uint32, n, at + 4 * ls * cap)
    return pos, vel, nbl, nbc, cap


def _missing_pairs(pos, nbl, nbc, cap, s):
    """Pairs (i, j) within 2h (minimal image in a periodic box) that are not in i's list."""
    h = s.params[0]["h"]
    span = np.array(s.params[0]["hi"]) - np.array(s.params[0]["lo"])
    per = np.array(s.params[0]["periodic"], bool)
    d = pos[:, None, :] - pos[None, :, :]
    for a in range(3):
        if per[a]:
            d[..., a] -= span[a] * np.round(d[..., a] / span[a])
    near = (d ** 2).sum(-1) < 4 * h * h
    np.fill_diagonal(near, False)
    listed = np.zeros_like(near)
    for i in range(len(pos)):
        if nbc[i] <= cap:
            listed[i, nbl[:nbc[i], i] & ((1 << 25) - 1)] = True
        else:
            listed[i] = True          # the stencil walk serves an overflowed list
    return int((near & ~listed).sum())


@pytest.mark.parametrize("name", ["periodic2d", "periodic3d"])
def test_list_holds_every_pair_between_rebuilds(name):
    # the rebuild rule: a list serves the states S^n and S* of every step until the next
    # build, so every pair within 2h at those states must be in it.  Fast particles
    # (rebuilds every few steps); after each step the state blob gives the positions and
    # the list, and when the next step rebuilds nothing, the pairs within 2h at its S^n
    # and at its predicted state x + dt/2 u (no walls or pistons here) are all listed
    s = SCENES[name]()
    rng = np.random.default_rng(5)
    s.u[:, :s.dim] = rng.uniform(-0.15, 0.15, (s.n, s.dim))
    print(f"case list coverage {name} n={s.n}", flush=True)
    sim = binding.Sim(s, precision=binding.FP64)
    sim.set_option(binding.OPT_GRAPH, 0)
    checked, rebuilt = 0, 0
    for _ in range(40):
        pos, vel, nbl, nbc, cap = _blob_lists(sim.get_state(), s)
        b0 = sim.stats()["builds"]
        sim.step(1)
        st = sim.stats()
        if st["builds"] != b0:
            rebuilt += 1
            continue
        assert _missing_pairs(pos, nbl, nbc, cap, s) == 0
        assert _missing_pairs(pos + 0.5 * st["dt"] * vel, nbl, nbc, cap, s) == 0
        checked += 1
    print(f"  steps checked {checked}, steps that rebuilt {rebuilt}", flush=True)
    assert checked >= 10 and rebuilt >= 3


@pytest.mark.parametrize("lanes", [1, 4])
@pytest.mark.parametrize("prec", PRECS)
def test_steps_are_deterministic_and_graph_matches_eager(prec, lanes):
    s = inputs.drop2d(perturb=True)
    a = binding.Sim(s, precision=prec)
    b = binding.Sim(s, precision=prec)
    c = binding.Sim(s, precision=prec, graph=False)
    for sim in (a, b, c):
        sim.set_option(binding.OPT_LANES, lanes)
        sim.set_option(binding.OPT_FORCE_LANES, lanes)
        sim.step(6)
        sim.sync()
    for f in (binding.F_X, binding.F_U, binding.F_RHO):
        assert np.array_equal(a.get_field(f), b.get_field(f))
        assert np.array_equal(a.get_field(f), c.get_field(f))


@pytest.mark.parametrize("prec", PRECS)
def test_multi_step_graph_replays_match_eager_steps(prec):
    # chunks of 8 run as one replay of the eight-step graph, the rest step by step; the
    # fields are read (eager copies, a synchronisation) between replays, and every
    # chunk is checked against the eager context
    s = inputs.drop2d(perturb=True)
    a = binding.Sim(s, precision=prec)
    c = binding.Sim(s, precision=prec, graph=False)
    for chunk in (8, 3, 8, 9, 16):
        a.step(chunk)
        c.step(chunk)
        for f in (binding.F_X, binding.F_U, binding.F_RHO):
            assert np.array_equal(a.get_field(f), c.get_field(f)), (chunk, f)
    assert a.stats()["steps"] == c.stats()["steps"] == 44
    assert a.stats()["builds"] == c.stats()["builds"] > 1


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("name", ["drop2d", "periodic3d", "batch"])
def test_one_launch_build_matches_seven_launches(name, prec):
    # the neighbour build as one launch with grid barriers against the seven-launch form:
    # same states and lists, bit for bit, across steps with rebuilds
    if name == "batch":
        s = inputs.concat("batch", [inputs.drop2d(perturb=True, dx=dx) for dx in (2.5e-3, 4e-3)])
    else:
        s = SCENES[name]()
    print(f"case one-launch build {name} precision={prec} n={s.n}", flush=True)
    a = binding.Sim(s, precision=prec)
    b = binding.Sim(s, precision=prec)
    b.set_option(binding.OPT_ONE_LAUNCH_BUILD, 0)
    b_two = b.stats()["two_level_builds"]   # the build at creation ran as one launch
    for chunk in (1, 12, 20):
        a.step(chunk)
        b.step(chunk)
        for f in (binding.F_X, binding.F_U, binding.F_RHO):
            assert np.array_equal(a.get_field(f), b.get_field(f)), (chunk, f)
        oa, ia = a.get_neighbors()
        ob, ib = b.get_neighbors()
        assert np.array_equal(oa, ob) and np.array_equal(ia, ib)
    assert a.stats()["builds"] == b.stats()["builds"] > 1
    # every one-launch rebuild took the two-level barrier (the blocks of each residue mod 8
    # share an XCD on this device); the seven launches have no grid barrier
    assert a.stats()["two_level_builds"] == a.stats()["builds"]
    assert b.stats()["two_level_builds"] == b_two


def _expect(code, call):
    with pytest.raises(binding.SphxError) as e:
        call()
    assert e.value.code == code, str(e.value)


def _same_course(a, b, chunks=(1, 12, 20)):
    for chunk in chunks:
        a.step(chunk)
        b.step(chunk)
        for f in (binding.F_X, binding.F_U, binding.F_RHO):
            assert np.array_equal(a.get_field(f), b.get_field(f)), (chunk, f)
    oa, ia = a.get_neighbors()
    ob, ib = b.get_neighbors()
    assert np.array_equal(oa, ob) and np.array_equal(ia, ib)


def _same_state(a, b):
    for f in (binding.F_X, binding.F_U, binding.F_RHO):
        assert np.array_equal(a.get_field(f), b.get_field(f)), f
    assert a.stats()["steps"] == b.stats()["steps"] and a.stats()["t"] == b.stats()["t"]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("barrier", [1, 2, 3, 4, 5])
def test_stalled_build_keeps_the_state(barrier, prec):
    # a grid barrier of the one-launch build forced to time out (the host-side test hook,
    # so every wave exits at once): the build stops part-way, the next sync reports it and
    # rebuilds with seven launches from the state the build found, and the context steps
    # on bit-identically to one that restored the same state and never stalled
    s = inputs.drop2d(perturb=True)
    print(f"case stalled build barrier={barrier} precision={prec}", flush=True)
    a = binding.Sim(s, precision=prec)
    a.step(3)
    b = binding.Sim(s, precision=prec)
    b.set_option(binding.OPT_ONE_LAUNCH_BUILD, 0)
    b.set_state(a.get_state())
    a.set_option(binding.OPT_FORCE_STALL, barrier)
    a.build_neighbors()
    _expect(9, a.sync)
    assert a.get_option(binding.OPT_ONE_LAUNCH_BUILD) == 0
    b.build_neighbors()
    _same_state(a, b)
    _same_course(a, b)
    assert a.stats()["builds"] == b.stats()["builds"]


@pytest.mark.parametrize("prec", PRECS)
def test_stall_inside_step_graphs_skips_the_rest(prec):
    # the stall during replayed step graphs (a rebuild falls due on its own): the passes
    # after it return without work, the next sync reports it, and once the skipped steps
    # are taken the context matches one that built with seven launches all along
    s = inputs.drop2d(perturb=True)
    print(f"case stall in step graphs precision={prec}", flush=True)
    a = binding.Sim(s, precision=prec)
    c = binding.Sim(s, precision=prec)
    c.set_option(binding.OPT_ONE_LAUNCH_BUILD, 0)
    builds0 = c.stats()["builds"]
    c.step(40)
    assert c.stats()["builds"] > builds0   # a rebuild falls due within the 40 steps
    a.set_option(binding.OPT_FORCE_STALL, 3)
    a.step(40)
    _expect(9, a.sync)
    done = a.stats()["steps"]
    print(f"  steps taken before the stall: {done}", flush=True)
    assert 0 < done < 40
    a.step(40 - done)
    _same_state(a, c)
    _same_course(a, c)


@pytest.mark.parametrize("prec", PRECS)
def test_stall_in_the_first_build_of_init(prec):
    s = inputs.drop2d(perturb=True)
    print(f"case stalled first build precision={prec}", flush=True)
    a = binding.Sim(s, precision=prec)
    a.set_option(binding.OPT_FORCE_STALL, 4)
    _expect(9, a.init_particles)
    b = binding.Sim(s, precision=prec)
    b.set_option(binding.OPT_ONE_LAUNCH_BUILD, 0)
    b.init_particles()
    _same_state(a, b)
    _same_course(a, b)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("name", ["drop2d", "flume2d"])
def test_init_particles_again_matches_a_fresh_context(name, prec):
    # a second upload into a context that has stepped starts it over exactly; the
    # flume's piston particles need the reference positions, which a first upload
    # without them would have switched off
    s = SCENES["drop2d"]() if name == "drop2d" else small_flume2d()
    print(f"case init twice {name} precision={prec} n={s.n}", flush=True)
    a = binding.Sim(s, precision=prec)
    a.step(5)
    a.init_particles()
    b = binding.Sim(s, precision=prec)
    _same_course(a, b)


def test_set_state_rejects_out_of_range_indices():
    # the state blob's layout (header, then the spans of state_spans in the library):
    # a 48-byte header holding n at byte 24 and the cell count at byte 32, then in FP32
    # pos, vel, aux (16 B per particle each), key, id, info (4 B), the cell table
    # (4 B per cell + 1), the run block (64 B per instance), acc and gc (16 B) and the
    # list, entry e of particle i at 4 (e s + i) with s = n rounded up to 32
    s = inputs.drop2d(perturb=True)
    print("case set_state validation", flush=True)
    a = binding.Sim(s, precision=binding.FP32_CELLREL)
    a.step(2)
    good = a.get_state()
    n = int(np.frombuffer(good, np.int64, 1, 24)[0])
    ncell = int(np.frombuffer(good, np.uint32, 1, 32)[0])
    assert n == s.n and ncell == a.stats()["ncells"]
    key_at = 48 + 48 * n
    nbl_at = key_at + 12 * n + 4 * (ncell + 1) + 64 * s.ninst + 32 * n
    assert np.frombuffer(good, np.uint32, 1, key_at)[0] < ncell
    assert (np.frombuffer(good, np.uint32, 1, nbl_at)[0] & ((1 << 25) - 1)) < n
    for at, bad in ((nbl_at, n), (key_at, ncell)):
        blob = bytearray(good)
        blob[at:at + 4] = np.uint32(bad).tobytes()
        _expect(1, lambda: a.set_state(bytes(blob)))
    x = a.get_field(binding.F_X)
    a.set_state(good)          # the rejected blobs changed nothing
    assert np.array_equal(a.get_field(binding.F_X), x)
    a.step(1)


@pytest.mark.parametrize("every", [0, 3])
@pytest.mark.parametrize("prec", PRECS)
def test_steps_without_renormalisation_match_oracle(prec, every):
    # Eq. (7) never (0) or every third step: the steps between take the derive and
    # colour passes from the stored density and put m P / rho^2 back in the position record
    s = inputs.drop2d(perturb=True).with_params(renorm_every=every)
    print(f"case renorm_every={every} precision={prec}", flush=True)
    o, sim = _one_step(s, prec, nsteps=5)
    tol = TOL[prec]
    assert rel_to(sim.get_field(binding.F_X), o.get(oracle.X), s.dx[0]) < tol
    assert rel_to(sim.get_field(binding.F_RHO), o.get(oracle.RHO), 1000.0) < tol
    umax = np.abs(o.get(oracle.U)).max()
    assert rel_to(sim.get_field(binding.F_U), o.get(oracle.U), umax) < 10 * tol


@pytest.mark.parametrize("prec", PRECS)
def test_rates_after_steps_without_renormalisation(prec):
    # compute_forces straight after steps: the position record still holds the
    # renormalisation field and must get m P / rho^2 back before the force pass
    s = inputs.drop2d(perturb=True)
    o = oracle.Oracle(s)
    o.step(3)
    o.rates()
    sim = binding.Sim(s, precision=prec)
    sim.step(3)
    sim.compute_forces()
    tol = TOL[prec]
    scale = o.get(oracle.SAP) + o.get(oracle.SAV) + o.get(oracle.SAS)
    ea = enorm(sim.get_field(binding.F_A), o.get(oracle.A), scale)
    ed = enorm(sim.get_field(binding.F_DRHO), o.get(oracle.DRHO), o.get(oracle.SDRHO))
    print(f"rates after 3 steps: E-norm a {ea:.3e}, Drho {ed:.3e}", flush=True)
    assert ea < tol and ed < tol


@pytest.mark.parametrize("prec", PRECS)
def test_checkpoint_round_trip_is_bit_identical(prec):
    s = inputs.drop2d(perturb=True)
    a = binding.Sim(s, precision=prec)
    a.step(8)
    b = binding.Sim(s, precision=prec)
    b.step(4)
    blob = b.get_state()
    c = binding.Sim(s, precision=prec)
    c.set_state(blob)
    c.step(4)
    for f in (binding.F_X, binding.F_U, binding.F_RHO):
        assert np.array_equal(a.get_field(f), c.get_field(f))
    assert a.stats()["steps"] == c.stats()["steps"] == 8


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("name", ["drop2d", "drop3d_small", "periodic3d"])
def test_both_forms_of_eq7_match_the_oracle(name, prec, oracle_rates):
    # right after set-up the renormalisation reads q = (rho - rho0) / rho from the
    # position record (one record per neighbour, masses uniform per phase); after a rate
    # evaluation it reads m_j and V_j from the aux record instead.  Both are Eq. (7).
    s, ref, _ = oracle_rates(name)
    a = binding.Sim(s, precision=prec)
    a.renormalize_density()
    b = binding.Sim(s, precision=prec)
    b.compute_forces()
    b.renormalize_density()
    rho0 = max(p[0] for p in s.phases[0])
    ra, rb = a.get_field(binding.F_RHO), b.get_field(binding.F_RHO)
    assert rel_to(ra, ref[oracle.RHO], rho0) < TOL[prec]
    assert rel_to(rb, ref[oracle.RHO], rho0) < TOL[prec]


@pytest.mark.parametrize("prec", PRECS)
def test_restored_state_brings_its_own_masses(prec):
    # a context set up with one mass per phase takes a checkpoint whose masses vary per
    # particle: it must then step exactly as the context that wrote the checkpoint
    s = inputs.drop2d(perturb=True)
    v = jitter_mass(inputs.drop2d(perturb=True))
    a = binding.Sim(v, precision=prec)
    a.step(2)
    blob = a.get_state()
    a.step(3)
    b = binding.Sim(s, precision=prec)
    b.set_state(blob)
    b.step(3)
    for f in (binding.F_X, binding.F_U, binding.F_RHO):
        assert np.array_equal(a.get_field(f), b.get_field(f))


@pytest.mark.parametrize("prec", PRECS)
def test_batched_instances_with_and_without_one_mass_per_phase(prec):
    # instance 1 has per-particle masses, instances 0 and 2 one mass per phase
    parts = [inputs.drop2d(perturb=True, dx=dx) for dx in (2.5e-3, 3.3e-3, 4e-3)]
    jitter_mass(parts[1])
    scene = inputs.concat("batch_mass", parts)
    sim = binding.Sim(scene, precision=prec)
    sim.step(2)
    sim.sync()
    x = sim.get_field(binding.F_X)
    rho = sim.get_field(binding.F_RHO)
    for b, part in enumerate(parts):
        o = oracle.Oracle(part)
        o.step(2)
        a, e = scene.inst_offsets[b], scene.inst_offsets[b + 1]
        assert rel_to(x[a:e], o.get(oracle.X), part.dx[0]) < TOL[prec]
        assert rel_to(rho[a:e], o.get(oracle.RHO), 1000.0) < TOL[prec]


@pytest.mark.parametrize("prec", PRECS)
def test_manual_calls_equal_one_step(prec):
    # build / renormalise / forces / integrate through the separate entry points
    s = inputs.drop2d(perturb=True)
    a = binding.Sim(s, precision=prec)
    a.step(1)
    b = binding.Sim(s, precision=prec)
    b.build_neighbors()
    b.renormalize_density()
    b.compute_forces()
    b.integrate_step(0.0)
    for f in (binding.F_X, binding.F_U, binding.F_RHO):
        assert np.array_equal(a.get_field(f), b.get_field(f))


@pytest.mark.parametrize("prec", PRECS)
def test_batched_instances_match_their_own_oracles(prec):
    parts = [inputs.drop2d(perturb=True, dx=dx) for dx in (2.5e-3, 3.3e-3, 4e-3)]
    parts[1].params[0]["alpha_s"] = 0.04
    parts[2].phases[0][1] = (850.0, 1e-5, parts[2].phases[0][1][2])
    scene = inputs.concat("batch", parts)
    sim = binding.Sim(scene, precision=prec)
    sim.step(2)
    sim.sync()
    x = sim.get_field(binding.F_X)
    rho = sim.get_field(binding.F_RHO)
    for b, part in enumerate(parts):
        o = oracle.Oracle(part)
        o.step(2)
        a, e = scene.inst_offsets[b], scene.inst_offsets[b + 1]
        assert rel_to(x[a:e], o.get(oracle.X), part.dx[0]) < TOL[prec]
        assert rel_to(rho[a:e], o.get(oracle.RHO), 1000.0) < TOL[prec]


def test_invalid_particles_are_rejected():
    s = inputs.drop2d()
    s.x[5, 0] = np.nan
    with pytest.raises(binding.SphxError) as e:
        binding.Sim(s)
    assert e.value.code == 1
    s = inputs.drop2d()
    s.phase[s.kind == 1] = 1                       # walls must be water
    with pytest.raises(binding.SphxError):
        binding.Sim(s)


def test_fixed_dt_violating_the_skin_is_reported():
    s = inputs.drop2d(perturb=True).with_params(dt_fixed=1e-3)   # dt*max|u| >> skin
    sim = binding.Sim(s, precision=binding.FP64)
    sim.step(1)
    with pytest.raises(binding.SphxError) as e:
        sim.sync()
    assert e.value.code == 8
    sim.sync()                                      # sticky bits cleared by the report


def clumped2d(extra=40, seed=3):
    """Periodic 2D box with a tight clump of extra particles: the particles around the
    clump overflow the neighbour-list capacity and take the stencil path."""
    s = periodic_drop(2, 20)
    rng = np.random.default_rng(seed)
    c = np.array([0.01, 0.01])
    xc = np.zeros((extra, 3))
    xc[:, :2] = c + rng.uniform(-0.4e-3, 0.4e-3, (extra, 2))
    uc = np.zeros((extra, 3))
    uc[:, :2] = rng.uniform(-0.1, 0.1, (extra, 2))
    s.x = np.concatenate([s.x, xc])
    s.u = np.concatenate([s.u, uc])
    s.rho = np.concatenate([s.rho, np.full(extra, 1001.0)])
    s.m = np.concatenate([s.m, np.full(extra, 1e-3)])
    s.phase = np.concatenate([s.phase, np.zeros(extra, np.uint8)])
    s.kind = np.concatenate([s.kind, np.zeros(extra, np.uint8)])
    s.inst_offsets = np.array([0, s.x.shape[0]], np.int64)
    return s


SCENES["clumped2d"] = clumped2d


@pytest.mark.parametrize("lanes", [1, 4])
@pytest.mark.parametrize("prec", PRECS)
def test_list_overflow_falls_back_to_the_stencil(prec, lanes, oracle_rates):
    s, ref, (off, ids) = oracle_rates("clumped2d")
    assert np.diff(off).max() > 48                  # beyond the 2D list capacity
    print(f"case overflow precision={prec} lanes={lanes}", flush=True)
    sim = binding.Sim(s, precision=prec)
    sim.set_option(binding.OPT_LANES, lanes)
    sim.set_option(binding.OPT_FORCE_LANES, lanes)
    if prec == binding.FP64:
        goff, gids = sim.get_neighbors()
        assert np.array_equal(goff, off) and np.array_equal(gids, ids)
    sim.renormalize_density()
    sim.compute_forces()
    tol = TOL[prec]
    assert rel_to(sim.get_field(binding.F_RHO), ref[oracle.RHO], 1000.0) < tol
    total_scale = ref[oracle.SAP] + ref[oracle.SAV] + ref[oracle.SAS]
    assert enorm(sim.get_field(binding.F_A), ref[oracle.A], total_scale) < tol
    assert enorm(sim.get_field(binding.F_DRHO), ref[oracle.DRHO], ref[oracle.SDRHO]) < tol


# ---- flumes: piston (MOVING) particles, periodic width in 3D, oil slick at the surface

def small_flume2d():
    return inputs.flume2d(dx=0.02, length=2.0, depth=0.3, x_focus=1.0)


def small_flume3d():
    return inputs.flume3d(dx=0.02, length=1.0, width=0.2, depth=0.2, x_focus=0.5)


def small_lab_flume():
    return inputs.lab_flume(2, dx=0.02)


FLUMES = {"flume2d": small_flume2d, "flume3d": small_flume3d, "lab_flume": small_lab_flume}


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("name", list(FLUMES))
def test_flume_steps_match_oracle(name, prec):
    s = FLUMES[name]()
    print(f"case flume {name} precision={prec} n={s.n}", flush=True)
    nsteps = 3
    o, sim = _one_step(s, prec, nsteps)
    dx = s.dx[0]
    tol = TOL[prec]
    x, xo = sim.get_field(binding.F_X), o.get(oracle.X)
    assert rel_to(x, xo, dx) < tol
    assert rel_to(sim.get_field(binding.F_RHO), o.get(oracle.RHO), 1000.0) < tol
    ur = np.abs(o.get(oracle.U)).max()
    assert rel_to(sim.get_field(binding.F_U), o.get(oracle.U), ur) < tol
    piston = s.kind == inputs.MOVING
    d, _ = oracle.piston(s.params[0], o.t)
    assert np.allclose(xo[piston, 0], s.x[piston, 0] + d, rtol=0, atol=1e-12)
    assert np.abs(x[piston, 0] - xo[piston, 0]).max() < (1e-12 if prec == 0 else 1e-6) + 0.0


def test_flume3d_neighbours_bit_exact_across_the_periodic_width():
    s = small_flume3d()
    o = oracle.Oracle(s)
    off, ids = o.neighbors()
    sim = binding.Sim(s, precision=binding.FP64)
    goff, gids = sim.get_neighbors()
    assert np.array_equal(goff, off) and np.array_equal(gids, ids)
    # pairs across the periodic faces exist
    y = s.x[:, 1]
    L = s.params[0]["hi"][1] - s.params[0]["lo"][1]
    wrapped = 0
    for i in range(0, s.n, 17):
        js = ids[off[i]:off[i + 1]]
        wrapped += int(np.sum(np.abs(y[js] - y[i]) > 0.5 * L))
    assert wrapped > 0


def test_drift_over_1000_steps_is_reported():
    """Drift of both GPU forms against the oracle over 1000 steps of the 2D drop
    (reported, loose bounds: particle trajectories separate chaotically)."""
    import json
    s = inputs.drop2d()
    o = oracle.Oracle(s)
    o.set_neighbor_method(2)
    sims = {p: binding.Sim(s, precision=p) for p in PRECS}
    dx = s.dx[0]
    rows = []
    for k in range(10):
        o.step(100)
        xo, uo, ro = o.get(oracle.X), o.get(oracle.U), o.get(oracle.RHO)
        row = {"steps": 100 * (k + 1), "t": o.t}
        for p, sim in sims.items():
            sim.step(100)
            tag = "fp64" if p == 0 else "fp32"
            row[f"{tag}_x_over_dx"] = rel_to(sim.get_field(binding.F_X), xo, dx)
            row[f"{tag}_u_rel"] = rel_to(sim.get_field(binding.F_U), uo, np.abs(uo).max())
            row[f"{tag}_rho_rel"] = rel_to(sim.get_field(binding.F_RHO), ro, 1000.0)
        rows.append(row)
        print(json.dumps(row), flush=True)
    assert rows[0]["fp64_x_over_dx"] < 1e-9
    assert rows[-1]["fp32_x_over_dx"] < 0.5


@pytest.mark.parametrize("prec", PRECS)
def test_lists_stay_exact_between_conditional_rebuilds(prec):
    """The sort and the neighbour list are rebuilt only once a particle has moved a
    quarter of the skin; between rebuilds the sets filtered from the list must equal
    the oracle's sets at the current positions (FP64), every few steps."""
    s = inputs.drop2d(perturb=True)
    sim = binding.Sim(s, precision=prec)
    builds = [sim.stats()["builds"]]
    for k in range(6):
        sim.step(7)
        builds.append(sim.stats()["builds"])
        if prec == binding.FP64:
            s2 = inputs.drop2d(perturb=True)
            s2.x[:] = sim.get_field(binding.F_X)
            off, ids = oracle.Oracle(s2).neighbors()
            goff, gids = sim.get_neighbors()
            assert np.array_equal(goff, off) and np.array_equal(gids, ids)
    assert builds[-1] - builds[0] < 42          # not every step
    assert builds[-1] - builds[0] >= 5          # this fast scene does need rebuilds


def test_still_tank_rebuilds_rarely():
    sim = binding.Sim(inputs.drop2d(), precision=binding.FP32_CELLREL)
    b0 = sim.stats()["builds"]
    sim.step(40)
    assert sim.stats()["builds"] - b0 <= 4


@pytest.mark.parametrize("block", [128, 192, 256])
def test_rates_with_other_block_sizes(block, oracle_rates):
    s, ref, _ = oracle_rates("drop3d_small")
    print(f"case rates block={block}", flush=True)
    sim = binding.Sim(s, precision=binding.FP32_CELLREL)
    sim.set_option(binding.OPT_BLOCK, block)
    sim.renormalize_density()
    sim.compute_forces()
    sim.sync()
    tol = TOL[binding.FP32_CELLREL]
    assert rel_to(sim.get_field(binding.F_RHO), ref[oracle.RHO], 1000.0) < tol
    total_scale = ref[oracle.SAP] + ref[oracle.SAV] + ref[oracle.SAS]
    assert enorm(sim.get_field(binding.F_A), ref[oracle.A], total_scale) < tol


def test_blocks_above_256_are_rejected():
    sim = binding.Sim(inputs.drop2d(), precision=binding.FP64)
    with pytest.raises(binding.SphxError, match="block"):
        sim.set_option(binding.OPT_BLOCK, 512)
    sim.set_option(binding.OPT_BLOCK, 256)


def test_tuner_returns_a_working_option_set():
    from paper_1702_07760_amd import tune
    s = inputs.drop2d(perturb=True)
    best = tune.tune(s, binding.FP32_CELLREL, steps=2, warmup=1, repeats=1, blocks=(64, 256),
                     remaps=(1, 16), save=False, log=None)
    assert best["ms_per_step"] > 0
    assert best["block"] in (64, 256) and best["xcd_remap"] in (1, 4, 16)
    sim = binding.Sim(s, precision=binding.FP32_CELLREL, tuned=False)
    sim.set_launch(block=best["block"], xcd_remap=best["xcd_remap"])
    assert sim.launch_options()["block"] == best["block"]
    sim.step(2)
    sim.sync()


@pytest.mark.parametrize("prec", PRECS)
def test_tuned_launch_shapes_give_bit_identical_runs(prec):
    # the options the tuner searches (block size, tile order) must not change any result
    s = inputs.drop3d(scale=0.3, perturb=True)
    print(f"case tuned launch precision={prec} n={s.n}", flush=True)
    runs = []
    for block, remap in ((None, None), (64, 16), (256, 1), (192, 0), (128, -16)):
        sim = binding.Sim(s, precision=prec, tuned=False)
        sim.set_launch(block=block, xcd_remap=remap)
        sim.step(12)
        sim.sync()
        runs.append([sim.get_field(f) for f in (binding.F_X, binding.F_U, binding.F_RHO, binding.F_A)]
                    + [sim.stats()["interactions"]])
        sim.close()
    for r in runs[1:]:
        for a, b in zip(runs[0], r):
            assert np.array_equal(a, b)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("name", ["drop3d_small", "periodic2d"])
def test_colour_pass_at_the_predicted_state_in_either_launch(name, prec):
    # the colour pass at S* beside the predictor (computing the predicted states itself)
    # or in its own launch after it: bit-identical runs; periodic2d's colour list is long
    # against its launch (8 lanes per particle), drop3d_small's short (a wave each)
    s = SCENES[name]()
    print(f"case colour in predict {name} precision={prec} n={s.n}", flush=True)
    runs = []
    for inside in (1, 0):
        sim = binding.Sim(s, precision=prec, tuned=False)
        sim.set_launch(colour_in_predict=inside)
        assert sim.launch_options()["colour_in_predict"] == inside
        sim.step(12)
        sim.sync()
        runs.append([sim.get_field(f) for f in (binding.F_X, binding.F_U, binding.F_RHO, binding.F_GRADC)])
        sim.close()
    for a, b in zip(*runs):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("remap", [0, 1, 16, -4])
def test_rates_with_other_tile_orders(remap, oracle_rates):
    s, ref, _ = oracle_rates("drop3d_small")
    print(f"case rates remap={remap}", flush=True)
    sim = binding.Sim(s, precision=binding.FP32_CELLREL)
    sim.set_option(binding.OPT_XCD_REMAP, remap)
    sim.renormalize_density()
    sim.compute_forces()
    sim.sync()
    tol = TOL[binding.FP32_CELLREL]
    assert rel_to(sim.get_field(binding.F_RHO), ref[oracle.RHO], 1000.0) < tol
    total_scale = ref[oracle.SAP] + ref[oracle.SAV] + ref[oracle.SAS]
    assert enorm(sim.get_field(binding.F_A), ref[oracle.A], total_scale) < tol
    for bad in (3, -1, -3, 128):
        with pytest.raises(binding.SphxError, match="xcd_remap"):
            sim.set_option(binding.OPT_XCD_REMAP, bad)


def test_tile_orders_give_identical_rates_on_the_full_drop():
    # every particle's sums are independent of which workgroup computes them, so the
    # tile permutations (full 32 K chunks only exist at this size) change nothing
    s = inputs.drop3d()
    out = []
    for remap in (1, 4, 16, -4, -16):
        sim = binding.Sim(s, precision=binding.FP32_CELLREL)
        sim.set_option(binding.OPT_XCD_REMAP, remap)
        sim.renormalize_density()
        sim.compute_forces()
        sim.sync()
        out.append([sim.get_field(f) for f in (binding.F_RHO, binding.F_A, binding.F_DRHO)])
        sim.close()
    for other in out[1:]:
        for a, b in zip(out[0], other):
            assert np.array_equal(a, b)


# ---- edge cases: one particle, ragged sizes, one phase only, exact cutoff ties

@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("n", [1, 63, 65])
def test_isolated_particles_fall_freely(n, prec):
    s = inputs.isolated_particles(dim=3, n=n, spacing=3.0, h=1.0)
    k = np.arange(n)
    s.x[:, 0] = 0.5 + 3.0 * (k % 8)          # an 8-wide grid, 3 m (> 2h) apart, inside the box
    s.x[:, 1] = 0.5 + 3.0 * (k // 8)
    print(f"case isolated n={n} precision={prec}", flush=True)
    o, sim = _one_step(s, prec, nsteps=3)
    assert sim.stats()["interactions"] == 0
    assert rel_to(sim.get_field(binding.F_X), o.get(oracle.X), 1e-3) < TOL[prec]
    assert rel_to(sim.get_field(binding.F_U), o.get(oracle.U), 1.0) < TOL[prec]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("dim,side", [(2, 9), (3, 9)])
def test_ragged_lattices_match_oracle(dim, side, prec):
    # 81 and 729 particles: whole waves plus a partial one, with an oil region
    s = inputs.lattice_box(dim, side, 1e-3, periodic=True,
                           oil=lambda x: x[:, 0] < side * 1e-3 / 2)
    rng = np.random.default_rng(5)
    s.u[:, :dim] = rng.uniform(-0.2, 0.2, (s.n, dim))
    # a parity state perturbs the density too: at exactly rho0 the pressure is the
    # rounding noise of (rho/rho0)^7 - 1 on both sides, and its E-norm is meaningless
    s.rho *= 1 + rng.uniform(-0.005, 0.005, s.n)
    s.params[0]["alpha_s"] = 0.02
    print(f"case ragged dim={dim} n={s.n} precision={prec}", flush=True)
    o = oracle.Oracle(s)
    o.renormalize()
    o.rates()
    sim = binding.Sim(s, precision=prec)
    sim.renormalize_density()
    sim.compute_forces()
    tol = TOL[prec]
    assert rel_to(sim.get_field(binding.F_RHO), o.get(oracle.RHO), 1000.0) < tol
    scale = o.get(oracle.SAP) + o.get(oracle.SAV) + o.get(oracle.SAS)
    assert enorm(sim.get_field(binding.F_A), o.get(oracle.A), scale) < tol
    assert enorm(sim.get_field(binding.F_DRHO), o.get(oracle.DRHO), o.get(oracle.SDRHO)) < tol


@pytest.mark.parametrize("prec", PRECS)
def test_single_phase_tank_has_no_interface(prec):
    s = inputs.still_tank(2)
    print(f"case single phase precision={prec}", flush=True)
    o, sim = _one_step(s, prec, nsteps=2)
    assert np.all(sim.get_field(binding.F_GRADC) == 0.0)
    assert rel_to(sim.get_field(binding.F_X), o.get(oracle.X), s.dx[0]) < TOL[prec]
    assert rel_to(sim.get_field(binding.F_RHO), o.get(oracle.RHO), 1000.0) < TOL[prec]


def test_pairs_exactly_at_the_cutoff_are_not_neighbours():
    # h = 0.25: a pair exactly 2h = 0.5 apart (r^2 == 4h^2 in FP64) is excluded, a pair one
    # ulp (of the coordinate) closer is included, on both sides
    s = inputs.isolated_particles(dim=2, n=4, spacing=3.0, h=0.25, u0=(0.0, 0.0))
    s.x[1] = s.x[0] + [0.5, 0.0, 0.0]
    s.x[3] = s.x[2] + [0.5, 0.0, 0.0]
    s.x[3, 0] = np.nextafter(s.x[3, 0], 0.0)
    assert (s.x[1, 0] - s.x[0, 0]) ** 2 == 4 * 0.25 ** 2
    assert (s.x[3, 0] - s.x[2, 0]) ** 2 < 4 * 0.25 ** 2
    o = oracle.Oracle(s)
    off, ids = o.neighbors()
    sim = binding.Sim(s, precision=binding.FP64)
    goff, gids = sim.get_neighbors()
    assert np.array_equal(goff, off) and np.array_equal(gids, ids)
    assert list(np.diff(goff)) == [0, 0, 1, 1]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("name", ["flume2d", "flume3d"])
def test_set_moving_matches_the_oracle(name, prec):
    # the wavemaker driven from outside: the same set_moving calls between steps on the
    # GPU and on the oracle (in 3D the width is periodic, so the motion stays in x-z)
    s = FLUMES[name]()
    print(f"case set_moving {name} precision={prec} n={s.n}", flush=True)
    mov = s.kind == inputs.MOVING
    x0 = s.x[mov].copy()
    o = oracle.Oracle(s)
    sim = binding.Sim(s, precision=prec)
    calls = [([0.004, 0.0, 0.0], [0.15, 0.0, 0.0]), ([0.006, 0.0, -0.001], [-0.1, 0.0, 0.02])]
    if s.dim == 2:
        calls = [(d[:1] + [d[2], 0.0], v[:1] + [v[2], 0.0]) for d, v in calls]
    for disp, vel in calls:
        o.step(2)
        sim.step(2)
        sim.set_moving(0, disp, vel)
        o.set_moving(disp, vel)
    t0 = o.t
    o.step(3)
    sim.step(3)
    sim.sync()
    tol = TOL[prec]
    dx = s.dx[0]
    x = sim.get_field(binding.F_X)
    assert rel_to(x, o.get(oracle.X), dx) < tol
    assert rel_to(sim.get_field(binding.F_RHO), o.get(oracle.RHO), 1000.0) < tol
    ur = np.abs(o.get(oracle.U)).max()
    assert rel_to(sim.get_field(binding.F_U), o.get(oracle.U), ur) < tol
    disp, vel = np.array(calls[-1][0]), np.array(calls[-1][1])
    want = x0 + (disp + vel * (o.t - t0))
    assert np.abs(x[mov] - want).max() < (1e-12 if prec == binding.FP64 else 1e-6)


def test_set_moving_rejects_what_it_cannot_do():
    s = FLUMES["flume3d"]()
    sim = binding.Sim(s, precision=binding.FP32_CELLREL)
    _expect(1, lambda: sim.set_moving(1, [0, 0, 0], [0, 0, 0]))            # no instance 1
    _expect(1, lambda: sim.set_moving(0, [0, 0, 0], [0, 0.1, 0]))          # periodic width
    _expect(1, lambda: sim.set_moving(0, [np.nan, 0, 0], [0, 0, 0]))
    still = binding.Sim(inputs.drop2d(), precision=binding.FP32_CELLREL)
    _expect(5, lambda: still.set_moving(0, [0, 0, 0], [0.1, 0, 0]))        # nothing MOVING
    sim.set_moving(0, [0.0, 0.0, 0.0], [0.05, 0.0, 0.0])
    sim.step(2)
    sim.sync()


@pytest.mark.parametrize("prec", PRECS)
def test_set_moving_acts_on_its_instance_only(prec):
    # two flumes in one context: instance 1 gets a motion from outside, instance 0 keeps
    # its piston series; each is compared with an oracle of its own
    a = small_flume2d()
    b = inputs.flume2d(dx=0.025, length=2.0, depth=0.3, x_focus=1.0)
    s = inputs.concat("two_flumes", [a, b])
    print(f"case set_moving batched precision={prec} n={s.n}", flush=True)
    sim = binding.Sim(s, precision=prec)
    oa, ob = oracle.Oracle(a), oracle.Oracle(b)
    disp, vel = [0.003, 0.0, 0.0], [0.12, 0.0, 0.0]
    sim.step(2)
    oa.step(2)
    ob.step(2)
    sim.set_moving(1, disp, vel)
    ob.set_moving(disp, vel)
    sim.step(3)
    oa.step(3)
    ob.step(3)
    sim.sync()
    x = sim.get_field(binding.F_X)
    u = sim.get_field(binding.F_U)
    tol = TOL[prec]
    for o, part, (lo, hi) in ((oa, a, s.inst_offsets[0:2]), (ob, b, s.inst_offsets[1:3])):
        assert rel_to(x[lo:hi], o.get(oracle.X), part.dx[0]) < tol
        ur = np.abs(o.get(oracle.U)).max()
        assert rel_to(u[lo:hi], o.get(oracle.U), ur) < tol
    mov_b = b.kind == inputs.MOVING
    lo = int(s.inst_offsets[1])
    assert np.allclose(u[lo:][mov_b][:, 0], vel[0], rtol=0, atol=1e-6)
