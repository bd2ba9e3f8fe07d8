"""The low- and high-degree residual estimates of the isotropic non-linear PG diffusivity
(ctf_config.pg_r_estimate) against the oracle: diffusivities (1e-12 h), operator (1e-12 of the
largest magnitude), float64 cycle iterates (1e-12 in the weighted norm), and float32 cycles with
float64 refinement on optically thick cells, where the iteration converges."""
import sys

import numpy as np
import pytest

from oracle import multigrid as omg
from oracle.transport import pg_diffusivity_isotropic
from pairs import make_pair, rel_w, to_dev, to_host, workload
from workloads import random_field

pytestmark = pytest.mark.gpu

# (p, estimate): low needs p >= 2; high uses the filters of degree p + 1 <= 4
CASES = [(2, "low"), (3, "low"), (4, "low"), (1, "high"), (2, "high"), (3, "high")]


def _maxrel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("p,est", CASES)
def test_estimate_diffusivities(p, est):
    """150 x 150 nodes: several 64-column strips with a ragged last one, two row strips."""
    print(f"diffusivities p={p} {est}", file=sys.stderr, flush=True)
    op, gp = make_pair(workload(N=150, na=2, p=p, G=1), "pg_frozen", "mixed", isotropic=True, r_estimate=est)
    psi = random_field(op.shape(), seed=40 + p, lo=0.0, hi=1.0)
    kx, ky = gp.empty(), gp.empty()
    gp.freeze_k(to_dev(psi), kx, ky)
    ok, _ = pg_diffusivity_isotropic(psi, op.quad, op.h, op.h, op.p, op.bc, r_estimate=est)
    got = to_host(kx)
    assert np.abs(got - ok).max() < 1e-12 * op.h
    assert np.array_equal(got, to_host(ky))
    # the estimate is not the mixed-mass one
    om, _ = pg_diffusivity_isotropic(psi, op.quad, op.h, op.h, op.p, op.bc)
    assert np.abs(got - om).max() > 1e-3 * op.h


@pytest.mark.parametrize("case,bc", list(zip(CASES, ["vac", "zg", "mixed", "mixed", "vac", "zg"])))
def test_estimate_operator(case, bc):
    from paper_2301_09991_amd import ctf
    p, est = case
    print(f"operator p={p} {est} {bc}", file=sys.stderr, flush=True)
    op, gp = make_pair(workload(N=72, na=2, p=p, G=2, scatter="p1"), "pg", bc, isotropic=True, r_estimate=est)
    psi = random_field(op.shape(), seed=50 + p, lo=0.0, hi=1.0)
    out = gp.empty()
    gp.apply_operator(to_dev(psi), out, ctf.OP_RESIDUAL)
    assert _maxrel(to_host(out), omg.finest_residual(op, psi)) < 1e-12
    # the fused and the two-pass kernels give the same bits
    outs = []
    for shape in ((128, 256, 1), (32, 256, 0)):
        gp.set_launch_shape(*shape)
        o = gp.empty()
        gp.apply_operator(to_dev(psi), o, ctf.OP_RESIDUAL)
        outs.append(to_host(o))
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("p,est", [(2, "low"), (1, "high")])
def test_estimate_cycle_iterates(p, est):
    print(f"cycles p={p} {est}", file=sys.stderr, flush=True)
    op, gp = make_pair(workload(N=40, na=2, p=p, G=1), "pg", "vac", isotropic=True, r_estimate=est)
    psi = np.zeros(op.shape())
    pd = to_dev(psi)
    for c in range(3):
        psi = omg.sawtooth_cycle(op, psi)
        gp.mg_cycle(pd)
        assert rel_w(to_host(pd), psi, op.quad, op.h) < 1e-12, c


def test_low_estimate_mixed_refinement_on_thick_cells():
    """p = 2 with the low-degree estimate, float32 cycles in full-approximation form (the
    diffusivities formed by the float32 kernel) with float64 refinement, on optically thick cells:
    the float64 residual falls below 1e-6 and, at the float32 floor, the solution is within 1e-6 of
    the float64 oracle's."""
    from paper_2301_09991_amd import ctf
    print("mixed refinement p=2 low", file=sys.stderr, flush=True)
    w = workload(N=32, na=2, p=2, L=32.0, patch=4, source="box_center8", seed=0)
    op, gp = make_pair(w, "pg", "vac", precision=ctf.FP32_IR, n_inner=2, isotropic=True, r_estimate="low")
    psi_o, hist, ok = omg.solve(op, rtol=1e-12, max_cycles=250)
    assert ok
    pd = gp.zeros()
    info = gp.solve(pd, 1e-6, 300)
    assert info["converged"], info
    info = gp.solve(pd, 1e-9, 60)           # on to the float32 floor of the full-approximation form
    assert info["rel_residual"] < 1e-6
    assert rel_w(to_host(pd), psi_o, op.quad, op.h) < 1e-6
