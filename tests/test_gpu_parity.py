"""Parity of the HIP library (through its C-ABI) with the CPU oracle, element by element, on seeded
inputs whose grids span several 16 x 16 tiles with a ragged tail.

Tolerances (float64 path): operator-level results agree to 1e-12 of the largest magnitude
(summation order only); solutions to 1e-10 relative in the weighted norm ||.||_W.
"""
import numpy as np
import pytest

from oracle import multigrid as omg
from oracle.transport import emission, moments, pg_diffusivity
from pairs import make_pair, rel_w, to_dev, to_host, workload
from workloads import random_field

pytestmark = pytest.mark.gpu


def _ctf():
    from paper_2301_09991_amd import ctf
    return ctf


def _maxrel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


CASES = [
    # (name, workload kwargs, disc, bc)
    ("upwind_iso", dict(G=1, scatter="iso"), "upwind", "vac"),
    ("upwind_down_zg", dict(G=2, scatter="downscatter"), "upwind", "mixed"),
    ("pg1_iso", dict(p=1, G=1, scatter="iso"), "pg", "vac"),
    ("pg2_down", dict(p=2, G=2, scatter="downscatter"), "pg", "vac"),
    ("pg3_p1", dict(p=3, G=2, scatter="p1"), "pg", "mixed"),
    ("pg2_zg", dict(p=2, G=1, scatter="iso"), "pg", "zg"),
]


def test_levels_match_oracle():
    op, gp = make_pair(workload(N=40, na=4), "pg", "vac")
    assert len(gp.levels) == len(op.levels)
    for l, lv in enumerate(op.levels):
        mu, nu, w = gp.level_quadrature(l)
        assert np.abs(mu - lv.quad["mu"]).max() < 1e-13
        assert np.abs(nu - lv.quad["nu"]).max() < 1e-13
        assert np.abs(w - lv.quad["p"]).max() < 1e-13
        st = to_host(gp.level_sigma_t(l))
        assert _maxrel(st, lv.sigma_t) < 1e-14
        assert gp.levels[l].n == lv.N


@pytest.mark.parametrize("name,wk,disc,bc", CASES, ids=[c[0] for c in CASES])
def test_apply_operator(name, wk, disc, bc):
    ctf = _ctf()
    w = workload(**wk)
    op, gp = make_pair(w, disc, bc)
    psi = random_field(op.shape(), seed=7, lo=0.0, hi=1.0)
    if disc == "pg_frozen":
        op.freeze_k(psi)
    ref = omg.finest_residual(op, psi)
    out = gp.empty()
    gp.apply_operator(to_dev(psi), out, ctf.OP_RESIDUAL)
    assert _maxrel(to_host(out), ref) < 1e-12, name
    gp.apply_operator(to_dev(psi), out, ctf.OP_APPLY)
    assert _maxrel(to_host(out), omg.apply_operator(op, psi)) < 1e-12, name


def test_frozen_k_operator_and_diffusivities():
    ctf = _ctf()
    w = workload(p=2, G=2, scatter="downscatter")
    op, gp = make_pair(w, "pg_frozen", "vac")
    psi_k = random_field(op.shape(), seed=3, lo=0.0, hi=1.0)
    psi = random_field(op.shape(), seed=4, lo=0.0, hi=1.0)
    kx, ky = gp.empty(), gp.empty()
    gp.freeze_k(to_dev(psi_k), kx, ky)
    okx, oky = pg_diffusivity(psi_k, op.quad, op.h, op.h, op.p, op.bc)
    scale = op.h * 1.0
    assert np.abs(to_host(kx) - okx).max() < 1e-12 * scale
    assert np.abs(to_host(ky) - oky).max() < 1e-12 * scale
    op.freeze_k(psi_k)
    out = gp.empty()
    gp.apply_operator(to_dev(psi), out, ctf.OP_RESIDUAL)
    assert _maxrel(to_host(out), omg.finest_residual(op, psi)) < 1e-12


def test_moments_and_emission_inputs():
    w = workload(p=2, G=2, scatter="p1")
    op, gp = make_pair(w, "pg", "vac")
    psi = random_field(op.shape(), seed=8)
    phi = gp.torch.empty((2, 3, w.N, w.N), dtype=gp.torch.float64, device="cuda")
    gp.moments(to_dev(psi), phi)
    assert _maxrel(to_host(phi), moments(psi, op.quad)) < 1e-13


def test_restrict_and_prolong_every_level():
    w = workload(N=48, na=4, G=2, scatter="downscatter")
    op, gp = make_pair(w, "pg", "vac")
    for l in range(len(op.levels) - 1):
        fine = random_field(op.shape(l), seed=20 + l)
        coarse = gp.empty(l + 1)
        gp.restrict(l, to_dev(fine), coarse)
        assert _maxrel(to_host(coarse), omg.restrict(fine, op.levels[l], op.levels[l + 1])) < 1e-13
        c = random_field(op.shape(l + 1), seed=40 + l)
        f = gp.empty(l)
        gp.prolong(l, to_dev(c), f)
        assert np.array_equal(to_host(f), omg.upsample(c, op.levels[l]))


@pytest.mark.parametrize("level", [0, 1, 2])
def test_upwind_smoothing_on_a_level(level):
    ctf = _ctf()
    w = workload(N=40, na=4, G=2, scatter="downscatter")
    op, gp = make_pair(w, "pg", "mixed")
    x = random_field(op.shape(level), seed=50 + level)
    s = random_field(op.shape(level), seed=60 + level)
    for nsw in (1, 2, 3, 4):   # single sweeps, pairs in one pass, a pair and a single, two pairs
        xd = to_dev(x)
        gp.smooth(level, ctf.SMOOTH_UPWIND, xd, to_dev(s), nsw)
        ref = omg.upwind_jacobi(op, level, x, s, nsw)
        assert _maxrel(to_host(xd), ref) < 1e-12


@pytest.mark.parametrize("disc,p", [("upwind", 1), ("pg", 1), ("pg", 3)])
def test_finest_smoothing(disc, p):
    ctf = _ctf()
    w = workload(p=p, G=2, scatter="downscatter")
    op, gp = make_pair(w, disc, "vac")
    psi = random_field(op.shape(), seed=70, lo=0.0, hi=1.0)
    for nsw in (1, 2):
        xd = to_dev(psi)
        gp.smooth(0, ctf.SMOOTH_FINEST, xd, None, nsw)
        assert _maxrel(to_host(xd), omg.finest_jacobi(op, psi, nsw)) < 1e-12


@pytest.mark.parametrize("disc,wk,bc", [
    ("upwind", dict(G=1, scatter="iso"), "vac"),
    ("pg", dict(p=1, G=1, scatter="iso"), "vac"),
    ("pg", dict(p=2, G=2, scatter="p1"), "mixed"),
    ("pg", dict(p=3, G=1, scatter="iso", N=24), "vac"),
])
def test_mg_cycle_iterates(disc, wk, bc):
    wkk = dict(N=40, na=4)
    wkk.update(wk)
    op, gp = make_pair(workload(**wkk), disc, bc)
    psi = np.zeros(op.shape())
    pd = to_dev(psi)
    for c in range(3):
        rel_o = omg.rel_residual(op, omg.finest_residual(op, psi))
        psi = omg.sawtooth_cycle(op, psi)
        rel_g = gp.mg_cycle(pd, want_residual=True)
        assert abs(rel_g - rel_o) <= 1e-12 * rel_o
        assert rel_w(to_host(pd), psi, op.quad, op.h) < 1e-12, c


@pytest.mark.parametrize("n_jacobi", [1, 3])
def test_mg_cycle_iterates_odd_sweep_counts(n_jacobi):
    """Odd numbers of correction sweeps per level (pairs run as one pass, the last one alone)."""
    op, gp = make_pair(workload(N=40, na=4, G=2, scatter="downscatter"), "upwind", "mixed", n_jacobi=n_jacobi)
    psi = np.zeros(op.shape())
    pd = to_dev(psi)
    for c in range(3):
        psi = omg.sawtooth_cycle(op, psi)
        gp.mg_cycle(pd)
        assert rel_w(to_host(pd), psi, op.quad, op.h) < 1e-12, c


def test_solve_upwind_plain_fp64_config():
    """The 32 x 32, p = 1, 128-ordinate, 1-group workload with the upwind discretisation, solved
    to 1e-12 on the GPU, against the oracle's preconditioned-GMRES solution."""
    from oracle.direct import gmres_solve
    from workloads import WORKLOADS
    w = WORKLOADS["c0_plain_fp64"]
    op, gp = make_pair(w, "upwind", "vac")
    x_ref, rel = gmres_solve(op, tol=1e-13)
    assert rel < 1e-12
    pd = gp.zeros()
    info = gp.solve(pd, 1e-12, 200, history_len=200)
    assert info["converged"], info
    assert rel_w(to_host(pd), x_ref, op.quad, op.h) < 1e-10
    # the residual history matches the oracle's cycle by cycle
    _, hist, ok = omg.solve(op, rtol=1e-12, max_cycles=200)
    n = min(len(hist), len(info["history"]))
    assert np.allclose(info["history"][:n], hist[:n], rtol=1e-9, atol=1e-15)


def test_solve_pg_optically_thick():
    """Non-linear PG (p = 2) on optically thick cells, where the sawtooth cycle converges: the
    GPU and the oracle reach the same solution."""
    w = workload(N=32, na=2, p=2, L=32.0, patch=4, source="box_center8", seed=0)
    op, gp = make_pair(w, "pg", "vac")
    psi_o, hist, ok = omg.solve(op, rtol=1e-10, max_cycles=150)
    assert ok
    pd = gp.zeros()
    info = gp.solve(pd, 1e-10, 150)
    assert info["converged"]
    assert rel_w(to_host(pd), psi_o, op.quad, op.h) < 1e-9


def test_mixed_precision_refinement_reaches_fp64_solution():
    ctf = _ctf()
    from workloads import WORKLOADS
    w = WORKLOADS["c0_plain_fp64"]
    op, gp = make_pair(w, "upwind", "vac", precision=ctf.FP32_IR, n_inner=2)
    psi_o, hist, ok = omg.solve(op, rtol=1e-13, max_cycles=300)
    assert ok
    pd = gp.zeros()
    info = gp.solve(pd, 1e-10, 300)
    assert info["converged"] and info["outer_steps"] > 0
    assert info["rel_residual"] <= 1e-10
    assert rel_w(to_host(pd), psi_o, op.quad, op.h) < 1e-8


def test_error_paths():
    ctf = _ctf()
    op, gp = make_pair(workload(N=16, na=1, p=2), "pg_frozen", "vac")
    psi = gp.zeros()
    out = gp.empty()
    with pytest.raises(ctf.CtfError):
        gp.apply_operator(psi, out, ctf.OP_RESIDUAL)       # no diffusivities held yet
    with pytest.raises(ctf.CtfError):
        gp.apply_operator(psi, psi, ctf.OP_RESIDUAL)       # aliasing
    with pytest.raises(ctf.CtfError):
        gp.restrict(len(gp.levels) - 1, psi, out)          # no coarser level
    with pytest.raises(ctf.CtfError):
        gp.smooth(0, ctf.SMOOTH_FINEST, psi, out, 1)       # finest smoothing takes no rhs
