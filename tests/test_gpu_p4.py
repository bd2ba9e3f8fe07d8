"""Degree p = 4 ConvFEM filters (9 x 9, formal order 6) on the GPU against the oracle: the
operator (anisotropic and isotropic PG, vacuum and zero-gradient sides), cycle iterates, and the
fused / two-pass kernels bit for bit."""
import numpy as np
import pytest

from oracle import multigrid as omg
from pairs import make_pair, rel_w, to_dev, to_host, workload
from workloads import random_field

pytestmark = pytest.mark.gpu


def _maxrel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("bc,iso,prec", [("vac", False, 0), ("zg", True, 0), ("mixed", False, 1)])
def test_p4_operator(bc, iso, prec):
    from paper_2301_09991_amd import ctf
    op, gp = make_pair(workload(N=40, na=2, p=4, G=2, scatter="p1"), "pg", bc, precision=prec, isotropic=iso)
    psi = random_field(op.shape(), seed=31, lo=0.0, hi=1.0)
    out = gp.empty()
    gp.apply_operator(to_dev(psi), out, ctf.OP_RESIDUAL)
    assert _maxrel(to_host(out), omg.finest_residual(op, psi)) < 1e-12


def test_p4_cycles_and_launch_shapes():
    from paper_2301_09991_amd import ctf
    op, gp = make_pair(workload(N=48, na=2, p=4, G=1), "pg", "vac")
    psi = np.zeros(op.shape())
    pd = to_dev(psi)
    for c in range(2):
        psi = omg.sawtooth_cycle(op, psi)
        gp.mg_cycle(pd)
        assert rel_w(to_host(pd), psi, op.quad, op.h) < 1e-12, c
    x = random_field(op.shape(), seed=32, lo=0.0, hi=1.0)
    outs = []
    for shape in ((128, 256, 1), (32, 256, 0)):
        gp.set_launch_shape(*shape)
        out = gp.empty()
        gp.apply_operator(to_dev(x), out, ctf.OP_RESIDUAL)
        outs.append(to_host(out))
    assert np.array_equal(outs[0], outs[1])
