"""GPU against the FP64 oracle at the full sizes of the benchmark workloads, in the
launch configuration the benchmark times (default options, graph-replayed steps).

The 3D drop (335,728 particles) and the 2D flume (165,538) are compared whole after one
step, the paper's sphere and cube drop tests (95,116) after three; the 3D periodic flume (3,222,950) in the FP32 form the benchmark reports; the
256-tank batch (5,961,716 particles) runs whole on the GPU and a sample of 8 tanks is
stepped by the oracle, one tank at a time (tanks are independent).
"""
import numpy as np
import pytest

import oracle
from paper_1702_07760_amd import binding, inputs

from parity import rel_to

pytestmark = pytest.mark.gpu

TOL = {binding.FP64: 1e-12, binding.FP32_CELLREL: 1e-5}


def _compare(scene, sim, o, prec, offsets=None):
    a, e = offsets if offsets is not None else (0, scene.n)
    dx = scene.dx[0]
    rho0 = max(p[0] for p in scene.phases[0])
    uo = o.get(oracle.U)
    ur = max(np.abs(uo).max(), 1e-30)
    x = sim.get_field(binding.F_X)[a:e]
    u = sim.get_field(binding.F_U)[a:e]
    r = sim.get_field(binding.F_RHO)[a:e]
    errs = (rel_to(x, o.get(oracle.X), dx), rel_to(u, uo, ur), rel_to(r, o.get(oracle.RHO), rho0))
    print(f"  errors x/dx {errs[0]:.3e}  u {errs[1]:.3e}  rho {errs[2]:.3e}", flush=True)
    assert max(errs) < TOL[prec]


@pytest.mark.parametrize("prec", [binding.FP64, binding.FP32_CELLREL])
@pytest.mark.parametrize("name", ["drop3d", "flume2d"])
def test_full_size_step_matches_oracle(name, prec):
    s = getattr(inputs, name)()
    print(f"case full {name} n={s.n} precision={prec}", flush=True)
    o = oracle.Oracle(s)
    o.set_neighbor_method(2)
    o.step(1)
    sim = binding.Sim(s, precision=prec)
    sim.step(1)
    sim.sync()
    assert abs(sim.stats()["t"] - o.t) <= 1e-6 * o.t
    _compare(s, sim, o, prec)


@pytest.mark.parametrize("prec", [binding.FP64, binding.FP32_CELLREL])
@pytest.mark.parametrize("shape", ["sphere", "cube"])
def test_paper_drop_cases_match_oracle(shape, prec):
    # the paper's two drop tests (64,000 fluid particles) with seeded velocity and
    # density perturbations, three steps
    s = inputs.paper_drop(shape, perturb=True)
    print(f"case paper drop {shape} n={s.n} precision={prec}", flush=True)
    o = oracle.Oracle(s)
    o.set_neighbor_method(2)
    o.step(3)
    sim = binding.Sim(s, precision=prec)
    sim.step(3)
    sim.sync()
    assert abs(sim.stats()["t"] - o.t) <= 1e-6 * o.t
    _compare(s, sim, o, prec)


def test_full_size_periodic_flume3d_fp32():
    s = inputs.flume3d()
    print(f"case full flume3d n={s.n}", flush=True)
    o = oracle.Oracle(s)
    o.set_neighbor_method(2)
    o.step(1)
    sim = binding.Sim(s, precision=binding.FP32_CELLREL)
    sim.step(1)
    sim.sync()
    _compare(s, sim, o, binding.FP32_CELLREL)


@pytest.mark.parametrize("prec", [binding.FP64, binding.FP32_CELLREL])
def test_full_batch_sampled_tanks_match_their_oracles(prec):
    s = inputs.batched_drops()
    print(f"case full batch n={s.n} instances={s.ninst} precision={prec}", flush=True)
    sim = binding.Sim(s, precision=prec)
    sim.step(2)
    sim.sync()
    for b in np.linspace(0, s.ninst - 1, 8).astype(int):
        part = s.instance(int(b))
        o = oracle.Oracle(part)
        o.set_neighbor_method(2)
        o.step(2)
        print(f" tank {b}: n={part.n}", flush=True)
        _compare(part, sim, o, prec, (int(s.inst_offsets[b]), int(s.inst_offsets[b + 1])))
