"""Host-side checks of the seeded scene generators against the sizes the paper states."""
import numpy as np
import pytest

from paper_1702_07760_amd import inputs


@pytest.mark.parametrize("shape", ["sphere", "cube"])
def test_paper_drop_cases_have_the_stated_sizes(shape):
    # Sec. III: tank 0.2 m on a side, water depth 0.2 m, particle size 5 mm (the paper
    # quotes 64k particles), drop 0.04 m across, centre 0.16 m below the surface
    s = inputs.paper_drop(shape)
    fluid = s.kind == inputs.FLUID
    oil = s.phase == inputs.OIL
    assert fluid.sum() == 40 ** 3 == 64000
    assert s.params[0]["alpha_s"] == 0.05
    assert np.all(s.kind[oil] == inputs.FLUID)
    xf = s.x[fluid]
    assert xf[:, 2].max() < 0.2 and xf[:, 2].min() > 0.0
    assert np.allclose(s.x[oil].mean(axis=0), [0.1, 0.1, 0.2 - 0.16], atol=1e-5)
    if shape == "cube":
        want = 8 ** 3   # 0.04 / 0.005 lattice sites per side
    else:
        # lattice sites (i + 1/2) dx within 4 dx of a centre that sits on a cell corner:
        # odd a, b, c (twice the offsets in dx) with a^2 + b^2 + c^2 < 8^2
        odd = np.arange(-7, 8, 2)
        a, b, c = np.meshgrid(odd, odd, odd, indexing="ij")
        want = int(np.sum(a * a + b * b + c * c < 64))
        assert abs(want - 4 / 3 * np.pi * 4 ** 3) < 0.1 * want
    assert oil.sum() == want


def test_paper_drop_rejects_unknown_shapes():
    with pytest.raises(ValueError):
        inputs.paper_drop("torus")
