"""Behaviour of the paper's sawtooth iteration on the ConvFEM + PG equations, measured on the oracle
(CPU): the spectral radius of the cycle's iteration matrix with the diffusivities frozen at a
uniform value, for one ordinate.  With one ordinate patch per face (na = 1) and no scattering the
ordinates decouple and the matrix restricted to one ordinate is assembled column by column from
the oracle's own cycle.  These are not pins of correctness: they record why the non-linear PG
iteration does not converge on optically thin cells (the cycle only contracts where there is
enough dissipation, from absorption or from k), which the solver's documentation states.

Regimes (p = element degree, k_max = h |mu| per axis, sigma h = cell optical thickness):
* k = k_max on thin cells: contracts at p = 1; at p >= 2 only with the 1/2 of the analytic k-Diff
  identity (k-Diff is linear in k, so that reading at k_max is this one at k_max / 2);
* k = 0 (the limiter's value on smooth fields): at p >= 2 the cycle grows errors on thin cells for
  every number of smoothing sweeps, and contracts on thick ones."""
import numpy as np
import pytest

from oracle import multigrid as omg


def _frozen_problem(N, p, sigma_h, kfrac, n_j=2, n_pg=2):
    L = 1.0
    st = np.full((1, N, N), sigma_h * N / L)
    prob = omg.Problem(N, L, p, 1, st, np.zeros((1, 1, 1, N, N)), np.zeros((1, N, N)), disc=omg.PG_FROZEN,
                       n_jacobi=n_j, n_pg=n_pg)
    h, q, shape = prob.h, prob.quad, prob.shape()
    kx = np.broadcast_to((kfrac * h * np.abs(q["mu"]))[None, :, None, None], shape).copy()
    ky = np.broadcast_to((kfrac * h * np.abs(q["nu"]))[None, :, None, None], shape).copy()
    prob.k_frozen = (kx, ky)
    return prob


def _cycle_radius(prob, n=0):
    """Spectral radius of e -> cycle(e) (homogeneous problem) on ordinate n."""
    _, _, Ny, Nx = prob.shape()
    M = np.zeros((Ny * Nx, Ny * Nx))
    for j in range(Ny * Nx):
        e = np.zeros(prob.shape())
        e[0, n].flat[j] = 1.0
        M[:, j] = omg.sawtooth_cycle(prob, e)[0, n].ravel()
    return float(np.max(np.abs(np.linalg.eigvals(M))))


def test_cycle_contracts_at_full_dissipation_for_bilinear_elements():
    assert _cycle_radius(_frozen_problem(8, 1, 0.03, 1.0)) < 0.7


@pytest.mark.parametrize("kfrac,lo,hi", [(1.0, 1.5, None), (0.5, None, 0.6)])
def test_biquadratic_full_dissipation_needs_the_half(kfrac, lo, hi):
    r = _cycle_radius(_frozen_problem(8, 2, 0.0, kfrac))
    assert (lo is None or r > lo) and (hi is None or r < hi), r


def test_central_biquadratic_cycle_grows_errors_on_void_cells():
    # k = 0, sigma = 0 at N = 16 (N = 8 is too coarse to show it)
    assert _cycle_radius(_frozen_problem(16, 2, 0.0, 0.0)) > 1.05


@pytest.mark.parametrize("n_j,n_pg", [(1, 0), (2, 0), (2, 2), (3, 3)])
def test_central_bicubic_cycle_grows_errors_for_any_sweep_count(n_j, n_pg):
    assert _cycle_radius(_frozen_problem(8, 3, 0.0, 0.0, n_j, n_pg)) > 1.1


@pytest.mark.parametrize("p", [2, 3])
def test_central_cycle_contracts_on_thick_cells(p):
    assert _cycle_radius(_frozen_problem(8, p, 1.0, 0.0)) < 0.6
