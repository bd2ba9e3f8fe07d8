"""Pins of the oracle's multigrid, smoothers and independent solvers (CPU only).

* pure absorber (upwind, vacuum x-sides, zero-gradient y-sides): the discrete solution is the
  closed-form recurrence psi_i = S/(4 pi s)(1 - r^(i+1)), r = 1/(1 + s h/mu), and converges at
  first order to the continuum S/(4 pi s)(1 - exp(-s x/mu));
* global balance of the converged upwind solution: h^2 sum(sigma_a phi - S) + leakage = 0;
* nilpotency: N_x + N_y - 1 upwind Jacobi sweeps reproduce the exact transport sweep;
* restriction / UpSamp identities: R(P(e)) = e and conservation of sum p h^2 rho;
* the multigrid solve agrees with dense LU and with sweep-preconditioned GMRES, and the exact
  solution is a fixed point of the sawtooth cycle;
* infinite medium solved from zero reaches the closed form.
"""
import numpy as np
import pytest

from oracle import quadrature as qd
from oracle.direct import dense_solve, gmres_solve, transport_sweep
from oracle.multigrid import (PG, PG_FROZEN, UPWIND, Problem, finest_residual, rel_residual,
                              restrict, sawtooth_cycle, solve, upsample, upwind_jacobi)
from oracle.transport import VACUUM, ZERO_GRADIENT, pg_diffusivity, weighted_norm
from workloads import WORKLOADS, make_inputs, scaled

VAC = (VACUUM,) * 4
ZG = (ZERO_GRADIENT,) * 4


def _absorber(N, s=1.5, S=1.0, na=1):
    st = np.full((1, N, N), s)
    ss = np.zeros((1, 1, 1, N, N))
    src = np.full((1, N, N), S)
    return Problem(N, 1.0, 1, na, st, ss, src, bc=(VACUUM, VACUUM, ZERO_GRADIENT, ZERO_GRADIENT),
                   disc=UPWIND)


def test_pure_absorber_discrete_closed_form():
    N, s, S = 16, 1.5, 1.0
    prob = _absorber(N, s, S, na=2)
    psi, hist, ok = solve(prob, rtol=1e-14, max_cycles=300)
    assert ok
    h = prob.h
    for n in range(len(prob.quad["p"])):
        mu = prob.quad["mu"][n]
        r = 1.0 / (1.0 + s * h / abs(mu))
        k = np.arange(N) if mu > 0 else np.arange(N)[::-1]
        exact = S / (4 * np.pi * s) * (1 - r ** (k + 1))
        assert np.allclose(psi[0, n], exact[None, :], rtol=1e-12, atol=0)


def test_pure_absorber_first_order_convergence():
    errs = []
    s, S = 1.5, 1.0
    for N in (32, 64, 128):
        prob = _absorber(N, s, S)
        x = transport_sweep(prob, np.broadcast_to(S / (4 * np.pi), prob.shape()).copy())
        h = prob.h
        xc = (np.arange(N) + 0.5) * h
        n = 0
        mu = prob.quad["mu"][n]
        cont = S / (4 * np.pi * s) * (1 - np.exp(-s * (xc + 0.5 * h) / mu))
        errs.append(np.abs(x[0, n, 0] - cont).max())
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all((orders > 0.85) & (orders < 1.15)), orders


def _c0_small(N=16, na=2, disc=UPWIND, L=1.0, p=1, **kw):
    w = scaled(WORKLOADS["c0_plain_fp64"], N)
    st, ss, src = make_inputs(w)
    return Problem(N, L, p, na, st, ss, src, disc=disc, **kw)


def test_upwind_global_balance():
    prob = _c0_small()
    psi, hist, ok = solve(prob, rtol=1e-13, max_cycles=200)
    assert ok
    h, q = prob.h, prob.quad
    phi = np.einsum("gnji,n->gji", psi, q["p"])
    sig_a = prob.sigma_t - prob.sigma_s[0].sum(axis=0)
    absorbed = h * h * np.sum(sig_a * phi - prob.source)
    mu, nu, p = q["mu"], q["nu"], q["p"]
    leak = 0.0
    for n in range(len(p)):
        col = psi[0, n, :, -1] if mu[n] > 0 else psi[0, n, :, 0]
        row = psi[0, n, -1, :] if nu[n] > 0 else psi[0, n, 0, :]
        leak += h * p[n] * (abs(mu[n]) * col.sum() + abs(nu[n]) * row.sum())
    assert abs(absorbed + leak) < 1e-11 * h * h * np.sum(prob.source)


def test_jacobi_nilpotent_without_scattering():
    prob = _c0_small(N=8, na=1)
    prob.sigma_s[:] = 0.0
    rng = np.random.default_rng(0)
    s = rng.normal(size=prob.shape())
    e0 = rng.normal(size=prob.shape())
    exact = transport_sweep(prob, s)
    e = upwind_jacobi(prob, 0, e0, s, 8 + 8 - 1)
    assert np.abs(e - exact).max() < 1e-12 * np.abs(exact).max()
    e_short = upwind_jacobi(prob, 0, e0, s, 8 + 8 - 2)
    assert np.abs(e_short - exact).max() > 1e-6


def test_restriction_prolongation_identities():
    prob = _c0_small(N=16, na=4)
    rng = np.random.default_rng(1)
    for l in range(len(prob.levels) - 1):
        lf, lc = prob.levels[l], prob.levels[l + 1]
        ec = rng.normal(size=prob.shape(l + 1))
        assert np.allclose(restrict(upsample(ec, lf), lf, lc), ec, rtol=1e-14, atol=1e-14)
        rho = rng.normal(size=prob.shape(l))
        rc = restrict(rho, lf, lc)
        fine = np.einsum("gnji,n->", rho, lf.quad["p"]) * lf.h ** 2
        coarse = np.einsum("gnji,n->", rc, lc.quad["p"]) * lc.h ** 2
        assert abs(fine - coarse) < 1e-12 * np.abs(rho).sum() * lf.h ** 2


def test_level_hierarchy():
    prob = _c0_small(N=32, na=4)
    assert [(lv.N, lv.quad["na"]) for lv in prob.levels] == [(32, 4), (16, 2), (8, 1), (4, 1), (2, 1)]
    odd = _c0_small(N=24, na=2)
    assert [lv.N for lv in odd.levels] == [24, 12, 6, 3]


def test_tiny_dense_lu_matches_gmres_and_multigrid():
    prob = _c0_small(N=4, na=1)
    x_lu = dense_solve(prob)
    x_gm, rel = gmres_solve(prob, tol=1e-14)
    assert rel < 1e-13
    assert np.abs(x_lu - x_gm).max() < 1e-12 * np.abs(x_lu).max()
    psi, hist, ok = solve(prob, rtol=1e-14, max_cycles=200)
    assert ok and np.abs(psi - x_lu).max() < 1e-11 * np.abs(x_lu).max()


def test_tiny_frozen_pg_dense_matches_gmres():
    prob = _c0_small(N=6, na=1, disc=PG_FROZEN, p=2)
    rng = np.random.default_rng(4)
    prob.k_frozen = pg_diffusivity(rng.uniform(size=prob.shape()), prob.quad, prob.h, prob.h, 2, prob.bc)
    x_lu = dense_solve(prob)
    x_gm, rel = gmres_solve(prob, tol=1e-14)
    assert rel < 1e-12
    assert np.abs(x_lu - x_gm).max() < 1e-10 * np.abs(x_lu).max()
    # rho(x_lu) = 0 for the frozen discretisation
    assert rel_residual(prob, finest_residual(prob, x_lu)) < 1e-12


def test_multigrid_solution_matches_gmres_and_is_a_fixed_point():
    prob = _c0_small(N=16, na=2)
    x_gm, rel = gmres_solve(prob, tol=1e-14)
    psi, hist, ok = solve(prob, rtol=1e-13, max_cycles=200)
    assert ok
    assert weighted_norm(psi - x_gm, prob.quad, prob.h, prob.h) < 1e-11 * weighted_norm(x_gm, prob.quad, prob.h, prob.h)
    nxt = sawtooth_cycle(prob, x_gm)
    assert np.abs(nxt - x_gm).max() < 1e-11 * np.abs(x_gm).max()


@pytest.mark.parametrize("disc,p", [(UPWIND, 1), (PG, 1), (PG, 2)])
def test_infinite_medium_solve_reaches_closed_form(disc, p):
    N, st, c, S = 8, 1.0, 0.5, 1.0
    sigma_t = np.full((1, N, N), st)
    prob = Problem(N, 8.0, p, 1, sigma_t, (c * sigma_t)[None, None], np.full((1, N, N), S),
                   bc=ZG, disc=disc)
    psi, hist, ok = solve(prob, rtol=1e-12, max_cycles=400)
    assert ok
    assert np.allclose(psi, S / (4 * np.pi * st * (1 - c)), rtol=1e-10)


def test_pg_converges_on_optically_thick_cells():
    # sigma_t h in [0.5, 2]: the sawtooth cycle with the non-linear PG reaches a tight residual
    prob = _c0_small(N=16, na=2, disc=PG, L=16.0, p=2)
    psi, hist, ok = solve(prob, rtol=1e-9, max_cycles=120)
    assert ok, hist[-5:]


@pytest.mark.parametrize("disc", [UPWIND, PG])
def test_solution_is_even_in_xi(disc):
    """In 2D the equations see only (mu, nu); every ordinate of face f (xi > 0) has a mirror on
    face f + 4 with the same (mu, nu) and weight, so the cycle keeps psi even in xi (the reading
    behind solving on the xi > 0 half with doubled weights)."""
    from workloads import Workload
    w = Workload("mirror", 16, 16.0, 2, 2, 1, 4, "iso", "box_center8", (0.3, 0.9), 3)
    st, ss, src = make_inputs(w)
    prob = Problem(w.N, w.L, w.p, w.na, st, ss, src, disc=disc)
    q = prob.quad
    half = 4 * w.na * w.na
    assert np.array_equal(q["mu"][:half], q["mu"][half:]) and np.array_equal(q["nu"][:half], q["nu"][half:])
    assert np.allclose(q["p"][:half], q["p"][half:], rtol=1e-14, atol=0)
    psi = np.zeros(prob.shape())
    for _ in range(4):
        psi = sawtooth_cycle(prob, psi)
    assert np.abs(psi[:, :half] - psi[:, half:]).max() <= 1e-13 * np.abs(psi).max()


def _scattering_dominated(N=32, seed=4):
    from workloads import Workload
    w = Workload("coupled", N, 32.0, 2, 2, 1, max(1, N // 32), "iso", "box_quarter_phys", (0.8, 0.99), seed)
    return w, make_inputs(w)


def test_coupled_sweep_closed_form_in_infinite_medium():
    """Zero-gradient sides, uniform sigma_t and c, e uniform and isotropic: the streaming term
    vanishes, S e = c sigma_t e (sum p = 4 pi), so one coupled sweep gives
    e + (s + c sigma_t e - sigma_t e) / (|mu|/h + |nu|/h + sigma_t) per ordinate."""
    N, s_t, c = 8, 1.3, 0.7
    st = np.full((1, N, N), s_t)
    ss = np.full((1, 1, 1, N, N), c * s_t)
    prob = Problem(N, 4.0, 1, 2, st, ss, np.zeros((1, N, N)), bc=ZG, disc=UPWIND, coupled=True)
    lv = prob.levels[1]
    e0, s0 = 0.25, 0.1
    e = np.full(prob.shape(1), e0)
    s = np.full(prob.shape(1), s0)
    got = upwind_jacobi(prob, 1, e, s, 1)
    d = np.abs(lv.quad["mu"]) / lv.h + np.abs(lv.quad["nu"]) / lv.h + s_t
    ref = e0 + (s0 + c * s_t * e0 - s_t * e0) / d
    assert np.allclose(got[0], ref[:, None, None], rtol=1e-13, atol=0)


def test_upsampled_moments_are_upsampled_coarse_moments():
    """sum_n p_n Y(n) UpSamp(e)[n] on the fine level equals the coarse moments of e copied to the
    2 x 2 children (coarse p_N = sum of children, coarse direction = p-weighted mean): the identity
    that lets a correction sweep take the moments of UpSamp(e) from the coarse level."""
    from oracle.transport import moments
    w, (st, ss, src) = _scattering_dominated(N=16)
    prob = Problem(w.N, w.L, w.p, 4, st, ss, src, disc=UPWIND)
    rng = np.random.default_rng(3)
    for l in range(len(prob.levels) - 1):
        e = rng.uniform(-1.0, 1.0, prob.shape(l + 1))
        fine = moments(upsample(e, prob.levels[l]), prob.levels[l].quad)
        coarse = moments(e, prob.levels[l + 1].quad)
        up = np.repeat(np.repeat(coarse, 2, axis=2), 2, axis=3)
        assert np.allclose(fine, up, rtol=1e-13, atol=1e-13 * np.abs(up).max())


def test_coupled_cycles_reach_the_same_solution_faster():
    """Scattering-dominated medium (c in [0.8, 0.99], 32 mean free paths): the coupled cycle reaches
    the solution of the plain cycle (the discrete equations are unchanged) in far fewer cycles."""
    w, (st, ss, src) = _scattering_dominated(N=32)
    plain = Problem(w.N, w.L, w.p, w.na, st, ss, src, disc=UPWIND)
    coupled = Problem(w.N, w.L, w.p, w.na, st, ss, src, disc=UPWIND, coupled=True)
    xp, hp, okp = solve(plain, rtol=1e-10, max_cycles=400)
    xc, hc, okc = solve(coupled, rtol=1e-10, max_cycles=400)
    assert okp and okc
    assert len(hc) < len(hp) / 2, (len(hc), len(hp))
    assert np.abs(xc - xp).max() <= 1e-8 * np.abs(xp).max()


def test_coupled_tiny_solve_matches_dense_lu():
    from workloads import Workload
    w = Workload("tinyc", 8, 8.0, 2, 1, 1, 2, "iso", "box_center8", (0.8, 0.99), 9)
    st, ss, src = make_inputs(w)
    prob = Problem(w.N, w.L, w.p, w.na, st, ss, src, disc=UPWIND, coupled=True)
    x_ref = dense_solve(prob)
    x, hist, ok = solve(prob, rtol=1e-13, max_cycles=400)
    assert ok
    assert np.abs(x - x_ref).max() <= 1e-11 * np.abs(x_ref).max()
