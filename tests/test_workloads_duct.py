"""The straight-duct inputs (the paper's table of regions, embedded in a 36 cm square): every
resolution carries the same source (36 cm^2) and absorber (sigma 0.5 over 828 cm^2), the layout is
mirror-symmetric about both centre lines, and sample points fall in the right regions."""
import numpy as np
import pytest

from workloads import duct_inputs


@pytest.mark.parametrize("dx", [0.8, 0.4, 0.2, 0.1])
def test_duct_totals_and_symmetry(dx):
    N, L, st, ss, src = duct_inputs(dx)
    assert N * dx == pytest.approx(36.0)
    assert st.sum() * dx * dx == pytest.approx(0.5 * (22.0 * 36.0 + 36.0), rel=1e-12)
    assert src.sum() * dx * dx == pytest.approx(36.0, rel=1e-12)
    assert np.allclose(st[0], st[0][:, ::-1]) and np.allclose(st[0], st[0][::-1])
    assert not ss.any()


def test_duct_regions_at_points():
    dx = 0.1
    N, L, st, ss, src = duct_inputs(dx)
    def at(x, y):   # x in the 28 cm frame, y in [0, 36]; cell-average values, to rounding
        j, i = int(y / dx), int((x + 4.0) / dx)
        return pytest.approx((st[0, j, i], src[0, j, i]), abs=1e-12)
    assert (0.5, 1.0) == at(14.0, 18.0)      # source
    assert (0.0, 0.0) == at(14.0, 5.0)       # duct below the source
    assert (0.0, 0.0) == at(14.0, 30.0)      # duct above
    assert (0.5, 0.0) == at(5.0, 18.0)       # absorber left
    assert (0.5, 0.0) == at(25.0, 2.0)       # absorber right
    assert (0.0, 0.0) == at(-2.0, 18.0)      # padding outside the 28 cm domain
