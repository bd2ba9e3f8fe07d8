"""Full-size checks on the benchmark's workload (256 x 256 nodes, p = 2, 512 ordinates, two groups
with downscatter) in the launch configuration the benchmark times: the float64 residual on sampled
ordinates of a random flux against the oracle, and properties of the refinement step at any size."""
import numpy as np
import pytest

from oracle import multigrid as omg
from oracle.transport import emission, pg_residual
from workloads import WORKLOADS, make_inputs, random_field

pytestmark = pytest.mark.gpu


def _problem(precision, disc=None):
    from paper_2301_09991_amd import ctf
    w = WORKLOADS["c1_mixed"]
    st, ss, src = make_inputs(w)
    cfg = ctf.default_config(n=w.N, length=w.L, p=w.p, na=w.na, ngroups=w.G, scatter_order=0,
                             discretisation=ctf.CONVFEM_PG if disc is None else disc,
                             precision=precision, n_inner=2)
    return w, (st, ss, src), ctf.Problem(cfg, st, ss, src)


def test_fullsize_residual_on_sampled_ordinates():
    import torch
    from paper_2301_09991_amd import ctf
    w, (st, ss, src), gp = _problem(ctf.FP32_IR)
    op = omg.Problem(w.N, w.L, w.p, w.na, st, ss, src, disc=omg.PG, max_levels=1)
    psi = random_field(op.shape(), seed=17, lo=0.0, hi=1.0)
    out = gp.empty()
    gp.apply_operator(torch.as_tensor(psi, device="cuda"), out, ctf.OP_RESIDUAL)
    q = op.quad
    # emission from the full moments; the residual of a few ordinates of every face, both groups
    sel = np.array([f * 64 + k for f in range(8) for k in (0, 27, 63)])
    qs = {"mu": q["mu"][sel], "nu": q["nu"][sel], "p": q["p"][sel], "na": q["na"]}
    em = emission(psi, q, op.sigma_s, op.source)[:, sel]
    ref = pg_residual(psi[:, sel], em, op.sigma_t, qs, op.h, op.h, op.p, op.bc)
    got = out[:, torch.as_tensor(sel, device="cuda")].cpu().numpy()
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_fullsize_refinement_steps():
    """From psi = 0 the first float64 residual is ||b||; the non-linear PG steps stay finite and
    bounded (on these optically thin cells the PG iteration does not contract, as in float64), and
    with the upwind discretisation the same steps contract the float64 residual."""
    from paper_2301_09991_amd import ctf
    _, _, gp = _problem(ctf.FP32_IR)
    psi = gp.zeros()
    rels = [gp.mg_cycle(psi, want_residual=True) for _ in range(4)]
    assert rels[0] == pytest.approx(1.0, rel=1e-12)
    assert all(np.isfinite(rels)) and max(rels) < 1.5
    del gp, psi
    _, _, gu = _problem(ctf.FP32_IR, disc=ctf.UPWIND)
    psi = gu.zeros()
    rels = [gu.mg_cycle(psi, want_residual=True) for _ in range(4)]
    assert all(b < a for a, b in zip(rels, rels[1:])) and rels[-1] < 0.5
