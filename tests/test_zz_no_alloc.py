"""sphx_bind_static_workspace: the same runs on the library's static per-device
workspace as on caller memory, bit for bit, for two contexts in a row (the second
smaller, on what the first left there); a second binding takes the workspace away
from the first context; contexts beyond its size are refused."""
import numpy as np
import pytest

from paper_1702_07760_amd import binding, inputs

pytestmark = pytest.mark.gpu

FIELDS = (binding.F_X, binding.F_U, binding.F_RHO, binding.F_A, binding.F_DRHO, binding.F_P,
          binding.F_GRADC)


def _run(scene, prec, static, steps):
    sim = binding.Sim(scene, precision=prec, static_workspace=static)
    sim.step(steps)
    sim.sync()
    out = {f: sim.get_field(f) for f in FIELDS}
    st = sim.stats()
    sim.close()
    return out, st


def test_static_workspace_gives_the_caller_workspace_results():
    cases = [("drop3d_small", inputs.drop3d(scale=0.3, perturb=True), binding.FP32_CELLREL),
             ("drop2d", inputs.drop2d(perturb=True), binding.FP64)]
    assert cases[1][1].n < cases[0][1].n
    for name, scene, prec in cases:
        assert binding.workspace_size(scene, prec) <= 64 << 20
        print(f"case static workspace {name} precision={prec} n={scene.n}", flush=True)
        ref, st_ref = _run(scene, prec, False, 12)
        got, st_got = _run(scene, prec, True, 12)
        assert st_got["steps"] == st_ref["steps"] == 12
        assert st_got["t"] == st_ref["t"] and st_got["interactions"] == st_ref["interactions"]
        for f in FIELDS:
            assert np.array_equal(got[f], ref[f]), (name, f)


def test_second_binding_takes_the_static_workspace():
    s = inputs.drop2d(dx=5e-3, perturb=True)
    print(f"case static workspace takeover n={s.n}", flush=True)
    a = binding.Sim(s, precision=binding.FP32_CELLREL, static_workspace=True)
    a.step(2)
    a.sync()
    b = binding.Sim(s, precision=binding.FP32_CELLREL, static_workspace=True)
    with pytest.raises(binding.SphxError) as e:
        a.step(1)
    assert e.value.code == 4
    b.step(2)
    b.sync()
    assert b.stats()["steps"] == 2
    b.close()
    a.close()


def test_static_workspace_refuses_a_context_beyond_its_size():
    s = inputs.drop3d()
    assert binding.workspace_size(s, binding.FP32_CELLREL) > 64 << 20
    with pytest.raises(binding.SphxError) as e:
        binding.Sim(s, precision=binding.FP32_CELLREL, static_workspace=True)
    assert e.value.code == 4 and "static workspace holds" in str(e.value)
