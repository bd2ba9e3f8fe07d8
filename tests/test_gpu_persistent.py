"""The persistent batched solve: one launch of the work-queue kernel against the graph-replay
batch (same iterates, bit for bit), against the oracle's solutions, its step limit and what it
refuses."""
import ctypes
import sys

import numpy as np
import pytest

from workloads import Workload, make_inputs

pytestmark = pytest.mark.gpu


def _ctf():
    from paper_2301_09991_amd import ctf
    return ctf


def _problem(w, precision, disc=0, **kw):
    ctf = _ctf()
    st, ss, src = make_inputs(w)
    cfg = ctf.default_config(n=w.N, length=w.L, p=w.p, na=w.na, ngroups=w.G,
                             scatter_order=1 if w.scatter == "p1" else 0, discretisation=disc,
                             precision=precision, **kw)
    return ctf.Problem(cfg, st, ss, src)


def _uneven(tag, sizes, seed0, na=2, G=1, scatter="iso"):
    return [Workload(f"{tag}{k}", N, 1.0, 2, na, G, 4, scatter, "box_quarter", seed=seed0 + k)
            for k, N in enumerate(sizes)]


def _both(ws, precision, max_steps, items_per_block=0, rtol=1e-6, **kw):
    """Solve the set by graph replays (one step per replay) and by the persistent kernel."""
    ctf = _ctf()
    out = []
    for persistent in (False, True):
        probs = [_problem(w, precision, **kw) for w in ws]
        psis = [p.zeros() for p in probs]
        print(f"[persistent] precision={precision} persistent={persistent} sizes={[w.N for w in ws]} "
              f"items_per_block={items_per_block} kw={kw}", file=sys.stderr, flush=True)
        if persistent:
            ok, infos = ctf.solve_batch_persistent(probs, psis, rtol, max_steps, items_per_block)
        else:
            ok, infos = ctf.solve_batch(probs, psis, rtol, max_steps, 1)
        out.append((ok, infos, [x.cpu().numpy() for x in psis]))
    return out


def _same(a, b):
    (ok_a, inf_a, x_a), (ok_b, inf_b, x_b) = a, b
    assert ok_a == ok_b
    for ia, ib, xa, xb in zip(inf_a, inf_b, x_a, x_b):
        assert ia["cycles"] == ib["cycles"] and ia["outer_steps"] == ib["outer_steps"]
        assert ia["rel_residual"] == ib["rel_residual"]
        assert np.array_equal(xa, xb)


@pytest.mark.parametrize("precision", [0, 1, 2])
def test_persistent_equals_graph_batch(precision):
    """Uneven problems (p = 2 recipe, 4x4-cell patches, central source): the single persistent
    launch reproduces the graph-replay batch exactly — iterates, final norms and step counts —
    in float64, in float32 cycles with float64 refinement, and with the bf16 MFMA moments."""
    ws = _uneven("pe", [16, 24, 32, 48, 40, 20], 3200)
    a, b = _both(ws, precision, 400)
    assert a[0]
    _same(a, b)


@pytest.mark.parametrize("items_per_block", [1, 8])
def test_persistent_other_shapes(items_per_block):
    """Odd sweep counts (a single sweep after the paired one), P1 scattering over two groups,
    mixed ordinate sets and the hemisphere, under other work-item sizes: still the graph batch's
    iterates bit for bit."""
    ws = _uneven("po", [12, 20, 28], 3300, na=2, G=2, scatter="p1") + _uneven("pq", [16, 24], 3310, na=4)
    a, b = _both(ws, 1, 300, items_per_block, n_jacobi=3, n_pg=1)
    assert a[0]
    _same(a, b)
    ws = _uneven("ph", [16, 36], 3320)
    a, b = _both(ws, 0, 300, items_per_block, hemisphere=1)
    assert a[0]
    _same(a, b)


def test_persistent_step_limit():
    """With too few steps allowed, the launch ends after exactly that many steps of every
    problem, reports no convergence, and leaves the graph batch's iterates of that many steps."""
    ws = _uneven("pl", [24, 40, 16], 3400)
    a, b = _both(ws, 1, 3)
    assert not a[0]
    _same(a, b)
    for info in b[1]:
        assert info["outer_steps"] == 3 and info["cycles"] == 3 * 4


@pytest.mark.parametrize("precision,rtol,tol", [(0, 1e-12, 1e-10), (1, 1e-10, 1e-8)])
def test_persistent_solutions_match_the_oracle(precision, rtol, tol):
    """Each problem of a persistent batch reaches the oracle's solution of its discrete equations
    (restarted GMRES with the exact upwind sweep as preconditioner, to 1e-13); the bound is that of
    the graph-batch test (inverse-operator gain on the residual rtol, factor 100 margin)."""
    from oracle import direct as odir
    from oracle import multigrid as omg
    from pairs import rel_w
    ctf = _ctf()
    ws = _uneven("pg", [8, 12, 16, 10, 14], 3500)
    probs = [_problem(w, precision) for w in ws]
    psis = [p.zeros() for p in probs]
    print(f"[persistent-oracle] precision={precision}", file=sys.stderr, flush=True)
    ok, infos = ctf.solve_batch_persistent(probs, psis, rtol, 600)
    assert ok
    for w, psi, info in zip(ws, psis, infos):
        st, ss, src = make_inputs(w)
        op = omg.Problem(w.N, w.L, w.p, w.na, st, ss, src, disc=omg.UPWIND)
        ref, res = odir.gmres_solve(op, tol=1e-13)
        assert res < 1e-12
        assert info["rel_residual"] <= rtol
        err = rel_w(psi.cpu().numpy(), ref, op.quad, op.h)
        assert err < tol, (w.N, err)


def test_persistent_refusals():
    """PG problems are refused (sizing and solve, CTF_EUNSUPPORTED from the solve), and so is a
    workspace that is too small (CTF_ENOMEM); neither launches anything."""
    ctf = _ctf()
    lib = ctf.load()
    w = _uneven("pr", [16], 3600)[0]
    pg = _problem(w, 1, disc=ctf.CONVFEM_PG)
    up = _problem(w, 1)
    with pytest.raises(ctf.CtfError, match="upwind"):
        ctf.solve_batch_persistent([pg], [pg.zeros()], 1e-6, 10)
    import torch
    ws = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    for prob, expect in ((pg, ctf.CTF_EUNSUPPORTED), (up, ctf.CTF_ENOMEM)):
        x = prob.zeros()
        hs = (ctypes.c_void_p * 1)(prob.handle.value)
        ps = (ctypes.c_void_p * 1)(x.data_ptr())
        infos = (ctf.SolveInfo * 1)()
        nb = 256 if expect == ctf.CTF_ENOMEM else ws.numel()
        rc = lib.ctf_solve_batch_persistent(hs, 1, ps, 1e-6, 10, 0, ctypes.c_void_p(ws.data_ptr()), nb, infos)
        assert rc == expect
        assert float(x.abs().max()) == 0.0


@pytest.mark.parametrize("persistent", [False, True])
def test_problems_stay_usable_after_a_batch(persistent):
    """A batch leaves every problem active: a cycle afterwards gives the bits of the same cycle on a
    fresh problem (regression: converged problems kept their flag cleared, so every later kernel of
    theirs returned at once)."""
    ctf = _ctf()
    ws = _uneven("pu", [16, 24], 3700)
    probs = [_problem(w, 1) for w in ws]
    psis = [p.zeros() for p in probs]
    if persistent:
        ok, _ = ctf.solve_batch_persistent(probs, psis, 1e-6, 200)
    else:
        ok, _ = ctf.solve_batch(probs, psis, 1e-6, 200, 2)
    assert ok
    for w, prob, psi in zip(ws, probs, psis):
        x = psi.clone()
        prob.mg_cycle(x)
        fresh = _problem(w, 1)
        y = psi.clone()
        fresh.mg_cycle(y)
        assert not np.array_equal(x.cpu().numpy(), psi.cpu().numpy())
        assert np.array_equal(x.cpu().numpy(), y.cpu().numpy())


@pytest.mark.parametrize("persistent", [False, True])
def test_non_finite_residual_ends_the_batch(persistent):
    """A NaN in one problem's starting flux makes its first residual norm non-finite: both batch
    forms stop and report CTF_ENONFINITE (the persistent kernel through its device error flag), and
    the problems stay usable."""
    ctf = _ctf()
    ws = _uneven("pn", [16, 24], 3800)
    probs = [_problem(w, 1) for w in ws]
    psis = [p.zeros() for p in probs]
    psis[1][0, 3, 5, 7] = float("nan")
    with pytest.raises(ctf.CtfError) as e:
        if persistent:
            ctf.solve_batch_persistent(probs, psis, 1e-6, 50)
        else:
            ctf.solve_batch(probs, psis, 1e-6, 50, 2)
    assert e.value.code == ctf.CTF_ENONFINITE
    x = probs[0].zeros()
    probs[0].mg_cycle(x)
    assert float(x.abs().max()) > 0.0


@pytest.mark.parametrize("rtol", [1e-6, 2.0])
def test_single_problem_and_immediate_convergence(rtol):
    """A batch of one problem, and a tolerance the starting flux already meets (rtol = 2 with
    psi = 0, whose relative residual is 1): both forms agree bit for bit, the latter after the one
    step that evaluates the first residual."""
    ws = _uneven("ps", [20], 3900)
    a, b = _both(ws, 1, 200, rtol=rtol)
    assert a[0] and b[0]
    _same(a, b)
    if rtol > 1:
        assert b[1][0]["outer_steps"] <= 1


@pytest.mark.parametrize("persistent", [False, True])
def test_a_problem_twice_in_a_batch_is_refused(persistent):
    """The same problem twice in one batch (its steps would race on one set of buffers) is refused
    with CTF_EINVAL before anything runs."""
    ctf = _ctf()
    w = _uneven("pd", [16], 4000)[0]
    prob = _problem(w, 1)
    psis = [prob.zeros(), prob.zeros()]
    with pytest.raises(ctf.CtfError) as e:
        if persistent:
            ctf.solve_batch_persistent([prob, prob], psis, 1e-6, 10)
        else:
            ctf.solve_batch([prob, prob], psis, 1e-6, 10, 1)
    assert e.value.code == ctf.CTF_EINVAL
    assert all(float(x.abs().max()) == 0.0 for x in psis)
