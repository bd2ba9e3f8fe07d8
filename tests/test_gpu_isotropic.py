"""The isotropic non-linear PG diffusivity (ctf_config.pg_isotropic) against the oracle's
pg_diffusivity_isotropic: diffusivities, operator (1e-12 of the largest magnitude), cycle iterates
(1e-12 in the weighted norm), and the fused / two-pass kernels bit for bit."""
import numpy as np
import pytest

from oracle import multigrid as omg
from oracle.transport import pg_diffusivity_isotropic
from pairs import make_pair, rel_w, to_dev, to_host, workload
from workloads import random_field

pytestmark = pytest.mark.gpu


def _maxrel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def test_isotropic_diffusivities():
    w = workload(p=2, G=2, scatter="downscatter")
    op, gp = make_pair(w, "pg_frozen", "mixed", isotropic=True)
    psi = random_field(op.shape(), seed=13, lo=0.0, hi=1.0)
    kx, ky = gp.empty(), gp.empty()
    gp.freeze_k(to_dev(psi), kx, ky)
    ok, _ = pg_diffusivity_isotropic(psi, op.quad, op.h, op.h, op.p, op.bc)
    assert np.abs(to_host(kx) - ok).max() < 1e-12 * op.h
    assert np.array_equal(to_host(kx), to_host(ky))


@pytest.mark.parametrize("wk,bc", [
    (dict(p=1, G=1, scatter="iso"), "vac"),
    (dict(p=2, G=2, scatter="p1"), "mixed"),
    (dict(p=3, G=1, scatter="iso"), "zg"),
])
def test_isotropic_operator(wk, bc):
    from paper_2301_09991_amd import ctf
    op, gp = make_pair(workload(**wk), "pg", bc, isotropic=True)
    psi = random_field(op.shape(), seed=8, lo=0.0, hi=1.0)
    out = gp.empty()
    gp.apply_operator(to_dev(psi), out, ctf.OP_RESIDUAL)
    assert _maxrel(to_host(out), omg.finest_residual(op, psi)) < 1e-12


def test_isotropic_cycle_iterates_and_launch_shapes():
    from paper_2301_09991_amd import ctf
    w = workload(N=40, na=2, p=2, G=1)
    op, gp = make_pair(w, "pg", "vac", isotropic=True)
    psi = np.zeros(op.shape())
    pd = to_dev(psi)
    for c in range(3):
        psi = omg.sawtooth_cycle(op, psi)
        gp.mg_cycle(pd)
        assert rel_w(to_host(pd), psi, op.quad, op.h) < 1e-12, c
    # the fused and the two-pass kernels give the same bits
    x = random_field(op.shape(), seed=9, lo=0.0, hi=1.0)
    outs = []
    for shape in ((128, 256, 1), (32, 256, 0)):
        gp.set_launch_shape(*shape)
        out = gp.empty()
        gp.apply_operator(to_dev(x), out, ctf.OP_RESIDUAL)
        outs.append(to_host(out))
    assert np.array_equal(outs[0], outs[1])
