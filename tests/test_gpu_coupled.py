"""Scattering-coupled correction sweeps (ctf_config.coupled_scatter) against the oracle's
coupled cycle: iterates cycle by cycle (1e-12 in the weighted norm), solutions (1e-10), the
float32 refinement (1e-8), and the batched graph path (bit-identical to individual solves)."""
import numpy as np
import pytest

from oracle import multigrid as omg
from pairs import make_pair, rel_w, to_dev, to_host, workload
from workloads import Workload

pytestmark = pytest.mark.gpu


def _scattering_dominated(N=32, seed=4, na=2):
    return Workload("coupled", N, 32.0, 2, na, 1, max(1, N // 32), "iso", "box_quarter_phys", (0.8, 0.99), seed)


@pytest.mark.parametrize("disc,wk,bc", [
    ("upwind", dict(N=40, na=4, G=2, scatter="downscatter"), "vac"),
    ("pg", dict(N=40, na=2, p=2, G=2, scatter="p1"), "mixed"),
    ("upwind", dict(N=48, na=2, G=1, scatter="iso", L=24.0, c_range=(0.8, 0.99)), "zg"),
])
def test_coupled_cycle_iterates(disc, wk, bc):
    op, gp = make_pair(workload(**wk), disc, bc, coupled=True)
    psi = np.zeros(op.shape())
    pd = to_dev(psi)
    for c in range(3):
        rel_o = omg.rel_residual(op, omg.finest_residual(op, psi))
        psi = omg.sawtooth_cycle(op, psi)
        rel_g = gp.mg_cycle(pd, want_residual=True)
        assert abs(rel_g - rel_o) <= 1e-12 * rel_o
        assert rel_w(to_host(pd), psi, op.quad, op.h) < 1e-12, c


def test_coupled_solve_fewer_cycles_same_solution():
    w = _scattering_dominated(N=64)
    op, gp = make_pair(w, "upwind", "vac", coupled=True)
    _, gplain = make_pair(w, "upwind", "vac")
    psi_o, hist, ok = omg.solve(op, rtol=1e-10, max_cycles=400)
    assert ok
    pd = gp.zeros()
    info = gp.solve(pd, 1e-10, 400)
    pp = gplain.zeros()
    info_p = gplain.solve(pp, 1e-10, 400)
    assert info["converged"] and info_p["converged"]
    assert info["cycles"] == len(hist) - 1
    assert info["cycles"] < info_p["cycles"] / 2, (info["cycles"], info_p["cycles"])
    assert rel_w(to_host(pd), psi_o, op.quad, op.h) < 1e-10
    assert rel_w(to_host(pp), psi_o, op.quad, op.h) < 1e-9


def test_coupled_mixed_precision_refinement():
    from paper_2301_09991_amd import ctf
    w = _scattering_dominated(N=64)
    op, gp = make_pair(w, "upwind", "vac", precision=ctf.FP32_IR, coupled=True)
    psi_o, hist, ok = omg.solve(op, rtol=1e-12, max_cycles=400)
    pd = gp.zeros()
    info = gp.solve(pd, 1e-10, 400)
    assert info["converged"] and info["rel_residual"] <= 1e-10
    assert rel_w(to_host(pd), psi_o, op.quad, op.h) < 1e-8


def test_coupled_batch_equals_individual():
    import torch
    from paper_2301_09991_amd import ctf
    ws = [_scattering_dominated(N=N, seed=s) for N, s in ((32, 5), (64, 6), (48, 7))]
    pairs_ = [make_pair(w, "upwind", "vac", precision=ctf.FP32_IR, coupled=True) for w in ws]
    gps = [g for _, g in pairs_]
    psis = [g.zeros() for g in gps]
    ok, infos = ctf.solve_batch(gps, psis, 1e-8, 300, 2)
    assert ok
    for w, info, psi in zip(ws, infos, psis):
        _, g1 = make_pair(w, "upwind", "vac", precision=ctf.FP32_IR, coupled=True)
        x = g1.zeros()
        i1 = g1.solve(x, 1e-8, 300)
        assert i1["converged"]
        assert torch.equal(x, psi)
