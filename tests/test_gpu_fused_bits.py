"""The fused single-pass PG kernel and the two-pass form (diffusivities stored, then read back) give
the same bits: the finest operator and two cycles, in float64 and in the float32 refinement, for the
anisotropic and isotropic diffusivities (every residual estimate) with P1 scattering, whose emission
e0 + mu e1 + nu e2 enters every residual.  Both forms share the helpers that evaluate the bounds, the
estimates and the emission exactly as written."""
import sys

import numpy as np
import pytest

from pairs import make_pair, to_dev, to_host, workload
from workloads import random_field

pytestmark = pytest.mark.gpu

CASES = [(False, "mixed", 2), (True, "mixed", 1), (True, "low", 2), (True, "high", 2), (False, "mixed", 3),
         (True, "low", 3)]


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("iso,est,p", CASES)
def test_fused_and_two_pass_agree_bitwise(iso, est, p, precision):
    from paper_2301_09991_amd import ctf
    print(f"fused vs two-pass p={p} iso={iso} {est} precision={precision}", file=sys.stderr, flush=True)
    op, gp = make_pair(workload(N=72, na=2, p=p, G=2, scatter="p1"), "pg", "mixed", precision=precision,
                       isotropic=iso, r_estimate=est)
    psi = random_field(op.shape(), seed=60 + p, lo=0.0, hi=1.0)
    outs = []
    for shape in ((128, 256, 1), (32, 256, 0)):
        gp.set_launch_shape(*shape)
        out = gp.empty()
        gp.apply_operator(to_dev(psi), out, ctf.OP_RESIDUAL)
        x = to_dev(psi)
        for _ in range(2):
            gp.mg_cycle(x)
        outs.append((to_host(out), to_host(x)))
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1])
    assert np.isfinite(outs[0][1]).all()


@pytest.mark.parametrize("N,p,est", [(2, 2, "low"), (2, 1, "high"), (5, 2, "high"), (5, 3, "low"), (9, 4, "low")])
def test_estimates_on_grids_narrower_than_the_halo(N, p, est):
    """Grids narrower than the fused kernel's 4p-wide halo: both forms against the oracle's operator."""
    from oracle import multigrid as omg
    from paper_2301_09991_amd import ctf
    print(f"narrow N={N} p={p} {est}", file=sys.stderr, flush=True)
    op, gp = make_pair(workload(N=N, na=2, p=p, G=1, scatter="p1"), "pg", "mixed", isotropic=True, r_estimate=est)
    psi = random_field(op.shape(), seed=70 + N, lo=0.0, hi=1.0)
    ref = omg.finest_residual(op, psi)
    for shape in ((128, 256, 1), (32, 256, 0)):
        gp.set_launch_shape(*shape)
        out = gp.empty()
        gp.apply_operator(to_dev(psi), out, ctf.OP_RESIDUAL)
        assert np.abs(to_host(out) - ref).max() <= 1e-12 * np.abs(ref).max(), shape
