"""Degenerate sizes against the oracle: one ordinate per face (na = 1, with the full and the half
ordinate set), a single-level grid of odd size, and 2 x 2 grids narrower than the ConvFEM halo.
Operators to 1e-12 of the largest magnitude, cycle iterates to 1e-12 in the weighted norm."""
import sys

import numpy as np
import pytest

from oracle import multigrid as omg
from pairs import make_pair, rel_w, to_dev, to_host, workload
from workloads import random_field

pytestmark = pytest.mark.gpu


def _maxrel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _cycles(op, gp, n=3, kept=None):
    """n sawtooth cycles from zero on both sides; kept: the GPU problem holds only the first kept
    ordinates (half set), compared with the oracle's full-set iterate there."""
    psi = np.zeros(op.shape())
    nd = op.shape()[1] if kept is None else kept
    pd = to_dev(psi[:, :nd])
    quad = op.quad if kept is None else {k: (v[:kept] if k != "na" else v) for k, v in op.quad.items()}
    for c in range(n):
        psi = omg.sawtooth_cycle(op, psi)
        gp.mg_cycle(pd)
        assert rel_w(to_host(pd), psi[:, :nd], quad, op.h) < 1e-12, c


@pytest.mark.parametrize("disc,N,bc,half", [
    ("upwind", 12, "mixed", False),   # 8 ordinates: one per face, levels 12 -> 6 -> 3
    ("upwind", 12, "vac", True),      # the 4 ordinates with xi > 0 (half set)
    ("pg", 12, "zg", False),
])
def test_one_ordinate_per_face(disc, N, bc, half):
    """The half set is compared on its ordinates with the oracle's full set (the 2D flux is even
    in xi): a field even in xi in, the kept half of the oracle's results out."""
    from paper_2301_09991_amd import ctf
    print(f"na=1 {disc} N={N} {bc} half={half}", file=sys.stderr, flush=True)
    op, gp = make_pair(workload(N=N, na=1, p=2, G=2, scatter="downscatter"), disc, bc, hemisphere=half)
    kept = 4 if half else None
    upper = random_field((op.shape()[0], kept or op.shape()[1]) + op.shape()[2:], seed=70, lo=0.0, hi=1.0)
    full = np.concatenate([upper, upper], axis=1) if half else upper
    ref = omg.finest_residual(op, full)[:, :upper.shape[1]]
    out = gp.empty()
    gp.apply_operator(to_dev(upper), out, ctf.OP_RESIDUAL)
    assert _maxrel(to_host(out), ref) < 1e-12
    _cycles(op, gp, kept=kept)


@pytest.mark.parametrize("disc", ["upwind", "pg"])
def test_single_level_odd_grid(disc):
    """N = 7 cannot be coarsened: the cycle is the coarsest-level sweeps from zero on the finest grid,
    then the finest smoothing."""
    print(f"N=7 {disc}", file=sys.stderr, flush=True)
    op, gp = make_pair(workload(N=7, na=2, p=1, G=1), disc, "mixed")
    assert len(op.levels) == 1 and len(gp.levels) == 1
    _cycles(op, gp)


@pytest.mark.parametrize("p", [1, 2])
def test_grid_narrower_than_the_halo(p):
    """2 x 2 nodes: the 2p-wide psi halo and the p-wide k halo are wider than the grid."""
    from paper_2301_09991_amd import ctf
    print(f"N=2 p={p}", file=sys.stderr, flush=True)
    op, gp = make_pair(workload(N=2, na=2, p=p, G=1), "pg", "mixed")
    psi = random_field(op.shape(), seed=71, lo=0.0, hi=1.0)
    out = gp.empty()
    gp.apply_operator(to_dev(psi), out, ctf.OP_RESIDUAL)
    assert _maxrel(to_host(out), omg.finest_residual(op, psi)) < 1e-12
    _cycles(op, gp, 2)
