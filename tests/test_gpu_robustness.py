"""Failure handling, determinism and warm starts through the C-ABI: a non-finite flux or
cross-section is reported (CTF_ENONFINITE) instead of iterated on; a step budget that runs out is
reported as not converged; two identical solves agree bit for bit (fixed-order reductions, no
atomics); and a solve resumed from a saved flux continues exactly as an uninterrupted one."""
import numpy as np
import pytest

from pairs import make_pair, workload
from workloads import make_inputs

pytestmark = pytest.mark.gpu


def test_non_finite_flux_is_reported():
    from paper_2301_09991_amd import ctf
    _, gp = make_pair(workload(N=24, na=2, p=2), "upwind", "vac")
    psi = gp.zeros()
    psi[0, 3, 5, 7] = float("nan")
    with pytest.raises(ctf.CtfError) as e:
        gp.solve(psi, 1e-8, 10)
    assert e.value.code == ctf.CTF_ENONFINITE


def test_non_finite_cross_section_is_reported():
    from paper_2301_09991_amd import ctf
    w = workload(N=24, na=2, p=2)
    st, ss, src = make_inputs(w)
    st[0, 4, 4] = float("inf")
    cfg = ctf.default_config(n=w.N, length=w.L, p=w.p, na=w.na, ngroups=w.G, scatter_order=0,
                             discretisation=ctf.UPWIND)
    gp = ctf.Problem(cfg, st, ss, src)
    psi = gp.zeros()
    psi.fill_(1.0)
    with pytest.raises(ctf.CtfError) as e:
        gp.solve(psi, 1e-8, 10)
    assert e.value.code == ctf.CTF_ENONFINITE


def test_step_budget_reports_not_converged():
    _, gp = make_pair(workload(N=32, na=2, p=2), "upwind", "vac")
    psi = gp.zeros()
    info = gp.solve(psi, 1e-14, 3)
    assert not info["converged"] and info["cycles"] == 3


@pytest.mark.parametrize("disc,precision", [("pg", 1), ("upwind", 0)])
def test_two_solves_agree_bit_for_bit(disc, precision):
    import torch
    w = workload(N=40, na=2, p=2, G=2, scatter="downscatter")
    runs = []
    for _ in range(2):
        _, gp = make_pair(w, disc, "vac", precision=precision)
        psi = gp.zeros()
        info = gp.solve(psi, 1e-30, 6, history_len=16)
        runs.append((psi, info["history"]))
    assert torch.equal(runs[0][0], runs[1][0])
    assert np.array_equal(runs[0][1], runs[1][1])


@pytest.mark.parametrize("precision", [0, 1])
def test_resume_from_saved_flux(precision):
    import torch
    w = workload(N=40, na=2, p=2)
    _, g1 = make_pair(w, "upwind", "vac", precision=precision)
    x = g1.zeros()
    g1.solve(x, 1e-30, 4)
    saved = x.clone()                       # checkpoint: the float64 flux is the whole state
    _, g2 = make_pair(w, "upwind", "vac", precision=precision)
    y = saved.clone()
    g2.solve(y, 1e-30, 4)                   # resumed in a fresh problem
    _, g3 = make_pair(w, "upwind", "vac", precision=precision)
    z = g3.zeros()
    g3.solve(z, 1e-30, 8)                   # uninterrupted
    assert torch.equal(y, z)
