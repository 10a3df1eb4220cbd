"""Compensated integration of the FP32 cell-relative form over 10^5 steps.

Each case has an exact FP64 answer (``tests/kahan_cases.py``): positions drifting
through about 240 cells of a periodic box, velocities under constant gravity, and
densities under constant density rates.  The bound is 4 ulp of the running FP32
value.  ``tests/test_kahan_emulation_cpu.py`` replays the same FP32 operations on
the CPU and shows that plain additions miss these bounds by three to four orders of
magnitude.
"""
import numpy as np
import pytest

from paper_1702_07760_amd import binding

import kahan_cases as K

pytestmark = pytest.mark.gpu


def _run(scene, nsteps):
    sim = binding.Sim(scene, precision=binding.FP32_CELLREL)
    sim.step(nsteps)
    sim.sync()
    return sim


def test_positions_drift_exactly_through_many_cells():
    s = K.drifting_particles()
    print(f"case kahan positions n={s.n} steps={K.NSTEPS}", flush=True)
    sim = _run(s, K.NSTEPS)
    t = K.NSTEPS * K.DT
    assert sim.stats()["t"] == t
    cells = t * abs(K.U0[0]) / K.cell_size()
    assert cells > 200
    x = sim.get_field(binding.F_X)
    err = K.wrap_error(x, s.x + K.U0 * t, K.BOX)
    bound = 4 * float(np.spacing(np.float32(K.cell_size())))
    print(f"max position error {np.abs(err).max():.3e} m, bound {bound:.3e} m, {cells:.0f} cells crossed")
    assert np.abs(err).max() <= bound
    assert np.array_equal(sim.get_field(binding.F_U), np.tile(K.U0, (s.n, 1)))
    sim.close()


def test_velocities_follow_constant_gravity_exactly():
    s = K.drifting_particles(gravity=True)
    print(f"case kahan velocities n={s.n} steps={K.NSTEPS}", flush=True)
    sim = _run(s, K.NSTEPS)
    t = K.NSTEPS * K.DT
    u = sim.get_field(binding.F_U)
    want = K.U0 + K.G0 * t
    bound = 4 * float(np.spacing(np.float32(np.abs(want).max())))
    err = np.abs(u - want).max()
    print(f"max velocity error {err:.3e} m/s, bound {bound:.3e} m/s")
    assert err <= bound
    sim.close()


def test_densities_follow_constant_rates_exactly():
    s = K.wall_lattice()
    print(f"case kahan densities n={s.n} steps={K.NSTEPS}", flush=True)
    sim = _run(s, 1)
    rate = sim.get_field(binding.F_DRHO)
    assert np.abs(rate).max() > 10.0
    sim.step(K.NSTEPS - 1)
    sim.sync()
    assert np.array_equal(sim.get_field(binding.F_DRHO), rate)   # the rates never change
    rho = sim.get_field(binding.F_RHO)
    want = s.rho + K.NSTEPS * K.DT * rate
    bound = 4 * float(np.spacing(np.float32(np.abs(want - 1000.0).max())))
    err = np.abs(rho - want).max()
    print(f"max density error {err:.3e} kg/m^3, bound {bound:.3e}, largest change {np.abs(want - 1000).max():.1f}")
    assert err <= bound
    assert np.abs(sim.get_field(binding.F_X)[:, :2] - s.x[:, :2]).max() <= 1e-15
    sim.close()
