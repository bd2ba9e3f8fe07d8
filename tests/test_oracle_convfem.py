"""Pins of the oracle's ConvFEM / upwind filters against the paper (CPU only).

* Appendix A prints the linear, quadratic and cubic filters to 3 significant figures: the exact
  averaged-row construction must reproduce every printed entry (readings: the printed linear
  w_x, w_y are twice the construction; the printed quadratic w_y has its first row at the -y
  offset while the linear and upwind w_y have it at +y; the 1/dy^2 in front of w_m is a misprint
  since its entries already sum to one).
* The worked example of the "conv_filter" figure fixes the cross-correlation semantics.
* Consistency moments (sum m = 1, sum u d = 1, sum u^2 k = -2) and symmetry.
"""
import numpy as np
import pytest

from oracle.convfem import (apply_filter, filters_2d, printed_orientation, stencils_1d,
                            upwind_filters)
from golden_io import read_blocks

PRINTED = read_blocks("appendix_filters.txt")


def _printed(name, p):
    for key, arr in PRINTED.items():
        parts = key.split()
        if parts[0] == name and int(parts[1]) == p:
            return arr
    raise KeyError((name, p))


def _close_to_printed(ours, printed):
    """Every printed entry is the exact value rounded to 3 significant figures."""
    assert ours.shape == printed.shape
    zero = printed == 0.0
    assert np.all(np.abs(ours[zero]) < 1e-15)
    rel = np.abs(ours[~zero] - printed[~zero]) / np.abs(printed[~zero])
    assert rel.max() < 5e-3, rel.max()


@pytest.mark.parametrize("p", [1, 2])
def test_diffusion_and_mass_filters_match_appendix(p):
    F = filters_2d(p, 1.0, 1.0)
    # symmetric in both axes: orientation does not matter for these three
    _close_to_printed(F["wDxx"], _printed("wDxx", p))
    _close_to_printed(F["wDyy"], _printed("wDyy", p))
    _close_to_printed(F["wm"], _printed("wm", p))


def test_quadratic_and_cubic_wx_match_appendix():
    _close_to_printed(filters_2d(2, 1.0, 1.0)["wx"], _printed("wx", 2))
    _close_to_printed(filters_2d(3, 1.0, 1.0)["wx"], _printed("wx", 3))


def test_quadratic_wy_printed_in_array_orientation():
    ours = filters_2d(2, 1.0, 1.0)["wy"]            # +d/dy, first row = offset -2
    _close_to_printed(ours, _printed("wy", 2))
    # read with its first row at +y it would be -d/dy
    assert np.allclose(printed_orientation(_printed("wy", 2)), -_printed("wy", 2)[:, :])


def test_linear_advection_filters_are_twice_the_construction():
    F = filters_2d(1, 1.0, 1.0)
    _close_to_printed(2.0 * F["wx"], _printed("wx", 1))
    _close_to_printed(2.0 * F["wy"], printed_orientation(_printed("wy", 1)))


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_consistency_moments_and_symmetry(p):
    m, d, k = stencils_1d(p)
    u = range(-p, p + 1)
    assert sum(m) == 1
    assert sum(x * ui for x, ui in zip(d, u)) == 1
    assert sum(x * ui * ui for x, ui in zip(k, u)) == -2
    assert sum(d) == 0 and sum(k) == 0
    assert m == m[::-1] and k == k[::-1] and d == [-x for x in d[::-1]]
    assert len(m) == 2 * p + 1


def test_linear_stencils_are_classical_bilinear_fem():
    # for linear elements ConvFEM is the classical bilinear FEM (section "ConvFEM")
    m, d, k = stencils_1d(1)
    assert [float(x) for x in m] == [1 / 6, 2 / 3, 1 / 6]
    assert [float(x) for x in d] == [-0.5, 0.0, 0.5]
    assert [float(x) for x in k] == [-1.0, 2.0, -1.0]


def test_worked_example_conv_filter():
    ex = read_blocks("conv_filter_example.txt")
    inp, w = ex["input"], ex["filter"]
    # printed first row = +y; convert both to offset order (rows = increasing y)
    inp_o, w_o = printed_orientation(inp), printed_orientation(w)
    out = apply_filter(inp_o, w_o)
    assert out.shape == (3, 3)
    assert out[1, 1] == ex["sum"][0, 0]
    prods = w_o * inp_o[1:4, 1:4]
    assert np.array_equal(printed_orientation(prods), ex["products"])


def test_cross_correlation_orientation():
    # a one-tap filter at offset (v, u) = (+1, -1) picks Psi[j+1, i-1]
    a = np.arange(25.0).reshape(5, 5)
    w = np.zeros((3, 3))
    w[2, 0] = 1.0
    out = apply_filter(a, w)
    assert out[1, 1] == a[3, 1]


def test_upwind_filters_orientation():
    # mu > 0: (psi_i - psi_{i-1})/dx; nu < 0: (psi_{j+1} - psi_j)/dy (eq. discretised_hfm)
    a = np.random.default_rng(0).normal(size=(5, 5))
    wx, wy = upwind_filters(0.5, -0.3, 0.1, 0.2)
    assert np.isclose(apply_filter(a, wx)[1, 1], (a[2, 2] - a[2, 1]) / 0.1)
    assert np.isclose(apply_filter(a, wy)[1, 1], (a[3, 2] - a[2, 2]) / 0.2)
    wx, wy = upwind_filters(-0.5, 0.3, 0.1, 0.2)
    assert np.isclose(apply_filter(a, wx)[1, 1], (a[2, 3] - a[2, 2]) / 0.1)
    assert np.isclose(apply_filter(a, wy)[1, 1], (a[2, 2] - a[1, 2]) / 0.2)
