"""Batched solves in one captured HIP graph, launch-shape independence, and the autotuner."""
import os
import tempfile

import numpy as np
import pytest

from pairs import make_pair, workload
from workloads import Workload, batch_workloads, make_inputs, random_field

pytestmark = pytest.mark.gpu


def _ctf():
    from paper_2301_09991_amd import ctf
    return ctf


def _problem(w, precision, disc=0):
    ctf = _ctf()
    st, ss, src = make_inputs(w)
    cfg = ctf.default_config(n=w.N, length=w.L, p=w.p, na=w.na, ngroups=w.G, scatter_order=0,
                             discretisation=disc, precision=precision)
    return ctf.Problem(cfg, st, ss, src)


@pytest.mark.parametrize("precision,steps_per_graph", [(0, 1), (1, 3)])
def test_batch_equals_individual_solves(precision, steps_per_graph):
    """Uneven problems (batched recipe: p = 2, 4x4-cell patches, central source) solved together
    by graph replays give exactly the iterates of their individual solves, every problem stopping
    at its own convergence step."""
    ctf = _ctf()
    sizes = [16, 24, 32, 48, 40, 20]
    ws = [Workload(f"b{k}", N, 1.0, 2, 2, 1, 4, "iso", "box_quarter", seed=3000 + k) for k, N in enumerate(sizes)]
    probs = [_problem(w, precision) for w in ws]
    psis = [p.zeros() for p in probs]
    ok, infos = ctf.solve_batch(probs, psis, 1e-6, 400, steps_per_graph)
    assert ok
    for w, psi, info in zip(ws, psis, infos):
        ref = _problem(w, precision)
        x = ref.zeros()
        r = ref.solve(x, 1e-6, 400)
        assert r["converged"] and info["rel_residual"] <= 1e-6
        assert info["cycles"] == r["cycles"]
        assert abs(info["rel_residual"] - r["rel_residual"]) <= 1e-12 * r["rel_residual"]
        assert np.array_equal(psi.cpu().numpy(), x.cpu().numpy())


@pytest.mark.parametrize("precision,rtol,tol", [(0, 1e-12, 1e-10), (1, 1e-10, 1e-8)])
def test_batch_solutions_match_the_oracle(precision, rtol, tol):
    """Uneven problems solved together by replays of one graph, in float64 and in float32 cycles
    with float64 refinement, reach the oracle's own solution of each: the discrete equations solved
    by restarted GMRES with the exact upwind transport sweep as preconditioner (no multigrid), to
    1e-13.  The batch stops each problem at its own residual rtol; the error bound allows the
    inverse operator's gain (at most ~1/sigma_a here) on that residual, with a factor 100 margin."""
    import sys
    from oracle import direct as odir
    from oracle import multigrid as omg
    from pairs import rel_w
    ctf = _ctf()
    sizes = [8, 12, 16, 10, 14]
    ws = [Workload(f"bo{k}", N, 1.0, 2, 2, 1, 2, "iso", "box_quarter", seed=3100 + k) for k, N in enumerate(sizes)]
    probs = [_problem(w, precision) for w in ws]
    psis = [p.zeros() for p in probs]
    print(f"[batch-oracle] precision={precision} sizes={sizes}", file=sys.stderr, flush=True)
    ok, infos = ctf.solve_batch(probs, psis, rtol, 600, 2)
    assert ok
    for w, psi, info in zip(ws, psis, infos):
        st, ss, src = make_inputs(w)
        op = omg.Problem(w.N, w.L, w.p, w.na, st, ss, src, disc=omg.UPWIND)
        ref, res = odir.gmres_solve(op, tol=1e-13)
        assert res < 1e-12
        assert info["rel_residual"] <= rtol
        err = rel_w(psi.cpu().numpy(), ref, op.quad, op.h)
        assert err < tol, (w.N, err)


def test_batch_workload_sizes():
    ws = batch_workloads()
    assert len(ws) == 64
    assert set(w.N for w in ws) <= {64, 96, 128, 192, 256, 384}
    assert len(set(w.seed for w in ws)) == 64


@pytest.mark.parametrize("disc,precision", [(1, 0), (1, 1), (2, 0)])
def test_results_do_not_depend_on_launch_shape(disc, precision):
    """The strip height and the sweep block size change only the launch decomposition: operator,
    sweeps and cycles agree bit for bit."""
    ctf = _ctf()
    names = {0: "upwind", 1: "pg", 2: "pg_frozen"}
    op, gp = make_pair(workload(N=72, na=2, G=2, scatter="downscatter"), names[disc], "vac",
                       precision=precision)
    psi = gp.empty()
    psi.copy_(__import__("torch").as_tensor(random_field(op.shape(), seed=4, lo=0.0, hi=1.0)))
    if disc == 2:
        gp.freeze_k(psi)
    outs = []
    for strip_h, block, fused in ((32, 256, 0), (8, 64, 1), (128, 1024, 1), (16, 512, 0)):
        gp.set_launch_shape(strip_h, block, fused)
        out = gp.empty()
        gp.apply_operator(psi, out, ctf.OP_RESIDUAL)
        x = psi.clone()
        for _ in range(2):
            gp.mg_cycle(x)
        outs.append((out.cpu().numpy(), x.cpu().numpy()))
    for o, x in outs[1:]:
        assert np.array_equal(o, outs[0][0]) and np.array_equal(x, outs[0][1])


@pytest.mark.parametrize("precision,p,scatter,G", [(0, 2, "iso", 1), (1, 2, "iso", 1), (2, 3, "p1", 2)])
def test_tall_strips_on_a_ragged_grid(precision, p, scatter, G):
    """Strips of 256 rows (the default once a launch fills the chip eight times over) on a grid of
    592 nodes (two full strips and a ragged one of 80 rows, levels down to 37), and of 512 rows (one
    full strip and a ragged one): PG operator and cycles give the bits of strips of 128 and of 32
    rows, fused and two-pass.  Also at p = 3 with P1 scattering over two groups and the bf16 MFMA
    moments (the largest workload's recipe)."""
    import torch
    ctf = _ctf()
    op, gp = make_pair(workload(N=592, na=1, G=G, scatter=scatter, p=p), "pg", "vac", precision=precision)
    psi = torch.as_tensor(random_field(op.shape(), seed=23, lo=0.0, hi=1.0), device="cuda")
    outs = []
    for strip_h, block, fused in ((256, 256, 1), (128, 256, 1), (32, 512, 0), (256, 1024, 0), (512, 256, 1)):
        gp.set_launch_shape(strip_h, block, fused)
        out = gp.empty()
        gp.apply_operator(psi, out, ctf.OP_RESIDUAL)
        x = psi.clone()
        for _ in range(2):
            gp.mg_cycle(x)
        outs.append((out.cpu().numpy(), x.cpu().numpy()))
    for o, x in outs[1:]:
        assert np.array_equal(o, outs[0][0]) and np.array_equal(x, outs[0][1])


@pytest.mark.parametrize("precision", [0, 1])
def test_wide_sweep_blocks_give_the_same_bits(precision):
    """Sweep blocks of 1024 and of 256 threads on a ragged grid wider than 256 nodes (288): the
    same cycle iterates, bit for bit."""
    import torch
    ctf = _ctf()
    op, gp = make_pair(workload(N=288, na=1, G=1), "upwind", "vac", precision=precision)
    psi0 = torch.as_tensor(random_field(op.shape(), seed=9, lo=0.0, hi=1.0), device="cuda")
    outs = []
    for block in (256, 1024):
        gp.set_launch_shape(128, block, 1)
        x = psi0.clone()
        for _ in range(2):
            gp.mg_cycle(x)
        outs.append(x.cpu().numpy())
    assert np.array_equal(outs[0], outs[1])


def test_autotune_picks_and_caches_a_shape():
    ctf = _ctf()
    w = Workload("tune", 96, 1.0, 2, 4, 1, 8, "iso", "box_quarter", seed=3)
    prob = _problem(w, ctf.FP32_IR, disc=ctf.CONVFEM_PG)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "tune.json")
        h, b, f = prob.autotune(path)
        assert h in (8, 16, 32, 64, 128, 256, 512) and b in (64, 128, 256, 512, 1024) and f in (0, 1)
        assert os.path.exists(path)
        text = open(path).read()
        assert '"strip_h": %d' % h in text
        other = _problem(w, ctf.FP32_IR, disc=ctf.CONVFEM_PG)
        assert other.autotune(path) == (h, b, f)
        assert other.launch_shape() == (h, b, f)


def test_launch_shape_limits():
    """Strip heights 8..512, sweep blocks that are multiples of 64 up to 1024 and pg_fused 0/1 are
    accepted; anything else is refused with CTF_EINVAL and leaves the shape as it was."""
    ctf = _ctf()
    w = Workload("shape", 32, 1.0, 2, 1, 1, 4, "iso", "box_quarter", seed=5)
    prob = _problem(w, ctf.FP64, disc=ctf.CONVFEM_PG)
    prob.set_launch_shape(512, 1024, 0)
    assert prob.launch_shape() == (512, 1024, 0)
    prob.set_launch_shape(8, 64, 1)
    for bad in ((7, 256, 1), (513, 256, 1), (128, 96, 1), (128, 1088, 1), (128, 0, 1), (128, 256, 2)):
        with pytest.raises(ctf.CtfError) as e:
            prob.set_launch_shape(*bad)
        assert e.value.code == ctf.CTF_EINVAL
        assert prob.launch_shape() == (8, 64, 1)
