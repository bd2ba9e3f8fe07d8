"""The xi > 0 half of the ordinate set with doubled weights (ctf_config.hemisphere) against the
oracle's full set: in 2D the flux is even in xi (pinned on the oracle by
test_solution_is_even_in_xi), so every result on the kept ordinates must equal the full set's.

Tolerances as the float64 parity tests: operators 1e-12 of the largest magnitude, solutions 1e-10
relative in the weighted norm (float32 refinement: 1e-8)."""
import numpy as np
import pytest

from oracle import multigrid as omg
from pairs import make_pair, rel_w, to_dev, to_host, workload
from workloads import random_field

pytestmark = pytest.mark.gpu


def _half(op):
    return 4 * op.quad["na"] ** 2


def _upper(q, half):
    return {"mu": q["mu"][:half], "nu": q["nu"][:half], "p": q["p"][:half], "na": q["na"]}


def test_half_set_quadrature_every_level():
    op, gp = make_pair(workload(N=40, na=4), "pg", "vac", hemisphere=True)
    assert len(gp.levels) == len(op.levels)
    for l, lv in enumerate(op.levels):
        half = 4 * lv.quad["na"] ** 2
        mu, nu, w = gp.level_quadrature(l)
        assert len(w) == half
        assert np.abs(mu - lv.quad["mu"][:half]).max() < 1e-13
        assert np.abs(nu - lv.quad["nu"][:half]).max() < 1e-13
        assert np.abs(w - 2.0 * lv.quad["p"][:half]).max() < 1e-13


@pytest.mark.parametrize("disc,wk,bc", [
    ("upwind", dict(G=2, scatter="downscatter"), "mixed"),
    ("pg", dict(p=2, G=2, scatter="p1"), "vac"),
    ("pg", dict(p=3, G=1, scatter="iso"), "zg"),
])
def test_half_set_operator(disc, wk, bc):
    from paper_2301_09991_amd import ctf
    op, gp = make_pair(workload(**wk), disc, bc, hemisphere=True)
    half = _half(op)
    upper = random_field((op.shape()[0], half) + op.shape()[2:], seed=5, lo=0.0, hi=1.0)
    full = np.concatenate([upper, upper], axis=1)
    ref = omg.finest_residual(op, full)[:, :half]
    out = gp.empty()
    gp.apply_operator(to_dev(upper), out, ctf.OP_RESIDUAL)
    got = to_host(out)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("disc,wk", [
    ("upwind", dict(N=40, na=4, G=2, scatter="downscatter")),
    ("pg", dict(N=32, na=2, p=2, L=32.0, patch=4, source="box_center8", seed=0)),
])
def test_half_set_solve(disc, wk):
    op, gp = make_pair(workload(**wk), disc, "vac", hemisphere=True)
    half = _half(op)
    psi_o, hist, ok = omg.solve(op, rtol=1e-12, max_cycles=300)
    assert ok
    pd = gp.zeros()
    info = gp.solve(pd, 1e-12, 300)
    assert info["converged"]
    assert rel_w(to_host(pd), psi_o[:, :half], _upper(op.quad, half), op.h) < 1e-10


def test_half_set_mixed_precision():
    from paper_2301_09991_amd import ctf
    op, gp = make_pair(workload(N=40, na=4, G=1), "upwind", "vac", precision=ctf.FP32_IR, hemisphere=True)
    half = _half(op)
    psi_o, hist, ok = omg.solve(op, rtol=1e-13, max_cycles=300)
    pd = gp.zeros()
    info = gp.solve(pd, 1e-10, 300)
    assert info["converged"] and info["rel_residual"] <= 1e-10
    assert rel_w(to_host(pd), psi_o[:, :half], _upper(op.quad, half), op.h) < 1e-8
