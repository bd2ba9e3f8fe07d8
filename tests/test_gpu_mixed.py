"""Mixed precision on the GPU: float32 cycles with float64 refinement, and the bf16 MFMA moment
contraction, against the float64 oracle.

Tolerance of the bf16 contraction (derived from its arithmetic): psi is rounded to bf16 once
(relative error <= 2^-9), the weights keep ~16 bits as a bf16 hi + lo pair (<= 2^-16), and the
float32 accumulation over n_dir terms adds <= n_dir 2^-24; so per cell
|Phi_mfma - Phi| <= (2^-9 + 2^-16 + n_dir 2^-24) sum_n |W_mn psi_n|.
"""
import numpy as np
import pytest

from oracle import multigrid as omg
from oracle.transport import moments
from pairs import make_pair, rel_w, to_dev, to_host, workload
from workloads import WORKLOADS, random_field, scaled

pytestmark = pytest.mark.gpu


def _ctf():
    from paper_2301_09991_amd import ctf
    return ctf


def _abs_moment_bound(psi, quad):
    w = quad["p"]
    return np.stack([np.einsum("gnji,n->gji", np.abs(psi), np.abs(w * c))
                     for c in (np.ones_like(w), quad["mu"], quad["nu"])], axis=1)


@pytest.mark.parametrize("na,N", [(2, 40), (8, 24)])
def test_bf16_mfma_moments_within_bound(na, N):
    import torch
    ctf = _ctf()
    w = workload(N=N, na=na, G=2, scatter="downscatter")
    op, gp = make_pair(w, "pg", "vac", precision=ctf.FP32_IR_BF16_MOMENTS)
    psi = random_field(op.shape(), seed=12, lo=-1.0, hi=1.0).astype(np.float32)
    ref = moments(psi.astype(np.float64), op.quad)
    bound = _abs_moment_bound(psi.astype(np.float64), op.quad)
    nd = op.shape()[1]
    out_m = torch.empty((2, 3, N, N), dtype=torch.float32, device="cuda")
    out_v = torch.empty_like(out_m)
    pd = torch.as_tensor(psi, device="cuda")
    gp.moments_f32(pd, out_m, use_mfma=True)
    gp.moments_f32(pd, out_v, use_mfma=False)
    m, v = to_host(out_m).astype(np.float64), to_host(out_v).astype(np.float64)
    tol_m = (2.0 ** -9 + 2.0 ** -16 + nd * 2.0 ** -24) * bound
    tol_v = (nd * 2.0 ** -24 + 2.0 ** -24) * bound
    assert np.all(np.abs(m - ref) <= tol_m)
    assert np.all(np.abs(v - ref) <= tol_v)
    # the MFMA path really rounds psi to bf16 (it is not the float32 vector path)
    assert np.abs(m - v).max() > 0


def test_bf16_moments_refinement_reaches_fp64_solution():
    ctf = _ctf()
    w = WORKLOADS["c0_plain_fp64"]
    op, gp = make_pair(w, "upwind", "vac", precision=ctf.FP32_IR_BF16_MOMENTS, n_inner=2)
    psi_o, hist, ok = omg.solve(op, rtol=1e-13, max_cycles=300)
    assert ok
    pd = gp.zeros()
    gp.timing_enable(True, 4096)
    info = gp.solve(pd, 1e-10, 400)
    t = gp.timing_read()
    gp.timing_enable(False)
    assert info["converged"] and info["rel_residual"] <= 1e-10
    # every float32 moment contraction ran on MFMA (the float64 outer residual keeps its own)
    assert t["moments_mfma"][1] >= info["cycles"]
    assert rel_w(to_host(pd), psi_o, op.quad, op.h) < 1e-8


def test_pg_mixed_refinement_on_thick_cells():
    """Non-linear PG with float32 cycles in full-approximation form (optically thick cells, where
    the cycle converges), run into its floor: the full-approximation form evaluates the whole
    operator in float32, so the float64 residual levels off where it is one float32 rounding of the
    operator's largest terms (measured 4.7e-7 relative here, after ~70 cycles).  At that floor the
    solution is within 1e-6 relative L2 of the float64 oracle's converged solution (measured 8e-8)."""
    ctf = _ctf()
    w = workload(N=32, na=2, p=2, L=32.0, patch=4, source="box_center8", seed=0)
    op, gp = make_pair(w, "pg", "vac", precision=ctf.FP32_IR, n_inner=2)
    psi_o, hist, ok = omg.solve(op, rtol=1e-12, max_cycles=250)
    assert ok
    pd = gp.zeros()
    info = gp.solve(pd, 1e-6, 300)
    assert info["converged"], info
    info = gp.solve(pd, 1e-9, 60)           # on to the float32 floor
    assert info["rel_residual"] < 1e-6
    assert rel_w(to_host(pd), psi_o, op.quad, op.h) < 1e-6


def test_mixed_precision_downscaled_mixed_workload():
    """The mixed-precision recipe (p = 2, 2 groups with downscatter) on a 32 x 32 grid with 128
    ordinates, upwind discretisation: float32 cycles + float64 refinement to 1e-10 against the
    float64 oracle solution."""
    ctf = _ctf()
    w = scaled(WORKLOADS["c1_mixed"], 32, na=4)
    op, gp = make_pair(w, "upwind", "vac", precision=ctf.FP32_IR)
    psi_o, hist, ok = omg.solve(op, rtol=1e-13, max_cycles=300)
    assert ok
    pd = gp.zeros()
    info = gp.solve(pd, 1e-10, 300)
    assert info["converged"]
    assert rel_w(to_host(pd), psi_o, op.quad, op.h) < 1e-8


@pytest.mark.parametrize("n_pg", [0, 1, 2, 3])
def test_full_approximation_step_follows_the_fp64_cycle(n_pg):
    """A refinement step with one float32 cycle in full-approximation form is the float64 sawtooth
    cycle up to float32 rounding (optically thick cells, where the cycle contracts).  n_pg = 0
    takes the separate update pass; otherwise the last finest sweep applies psi64 += u - fl32(psi64),
    and odd counts end in the other buffer.  An error in that bookkeeping (a lost or doubled
    update, a stale float copy of psi) moves the iterate by far more than the bound."""
    ctf = _ctf()
    w = workload(N=32, na=2, p=2, L=32.0, patch=4, source="box_center8", seed=0)
    op, gp = make_pair(w, "pg", "vac", precision=ctf.FP32_IR, n_inner=1, n_pg=n_pg)
    psi = np.zeros(op.shape())
    pd = to_dev(psi)
    for c in range(3):
        psi = omg.sawtooth_cycle(op, psi)
        gp.mg_cycle(pd)
        assert rel_w(to_host(pd), psi, op.quad, op.h) < 1e-4, c
