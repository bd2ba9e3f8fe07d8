"""Independent solvers for the finest-level discrete equations (no multigrid).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The sawtooth multigrid is an iterative method; its converged result is the psi* with
rho(psi*) = 0 at every interior node, ordinate and group.  These routines reach that psi* by other
algorithms, so that the multigrid (oracle and HIP) can be pinned to it:

* ``assemble_dense`` / ``dense_solve``: the linear operator (upwind or frozen-k Petrov-Galerkin,
  scattering included) assembled column by column and solved with LAPACK LU (tiny grids);
* ``transport_sweep``: the exact solve of (A_up + sigma_t) x = r per ordinate by the classical
  serial upwind sweep in the downstream order of the ordinate's octant (the serial sweep the paper
  contrasts its data-parallel multigrid with);
* ``gmres_solve``: restarted GMRES on the full linear operator, preconditioned by that sweep;
* ``picard_solve``: the non-linear Petrov-Galerkin equations by Picard iteration on k.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from .multigrid import PG, PG_FROZEN, UPWIND, apply_operator
from .transport import VACUUM, pg_diffusivity


def _linear(prob):
    if prob.disc == PG:
        raise ValueError("the non-linear PG operator is not linear: freeze k or use picard_solve")
    return lambda x: apply_operator(prob, x)


def assemble_dense(prob):
    """Dense matrix of A (no external source) by applying it to every unit vector."""
    shape = prob.shape()
    n = int(np.prod(shape))
    A = np.zeros((n, n))
    op = _linear(prob)
    e = np.zeros(n)
    for c in range(n):
        e[c] = 1.0
        A[:, c] = op(e.reshape(shape)).ravel()
        e[c] = 0.0
    return A


def rhs(prob):
    """b[g, n, j, i] = S_g / 4 pi."""
    return np.broadcast_to(prob.source[:, None] / (4 * np.pi), prob.shape()).copy()


def dense_solve(prob):
    A = assemble_dense(prob)
    lu = sla.lu_factor(A)
    return sla.lu_solve(lu, rhs(prob).ravel()).reshape(prob.shape())


def transport_sweep(prob, r):
    """Exact solution x of (A_up + sigma_t) x = r, ordinate by ordinate, by marching through the
    nodes in the downstream order of each octant (all ordinates of one octant face share that
    order, so they are marched together).  Halo rule as for the residual: incoming halo 0 (vacuum)
    or a copy of the boundary node (zero gradient), in which case that boundary term vanishes
    from the node's equation."""
    G, nd, N, _ = r.shape
    h = prob.h
    mu, nu = prob.quad["mu"], prob.quad["nu"]
    nf = nd // 8
    x = np.zeros_like(r)
    for f in range(8):
        sl = slice(f * nf, (f + 1) * nf)
        m0, n0 = mu[f * nf], nu[f * nf]
        ax = (np.abs(mu[sl]) / h)[None, :]
        ay = (np.abs(nu[sl]) / h)[None, :]
        irange = range(N) if m0 > 0 else range(N - 1, -1, -1)
        jrange = range(N) if n0 > 0 else range(N - 1, -1, -1)
        di = -1 if m0 > 0 else 1
        dj = -1 if n0 > 0 else 1
        xbc = prob.bc[0] if m0 > 0 else prob.bc[1]
        ybc = prob.bc[2] if n0 > 0 else prob.bc[3]
        for j in jrange:
            for i in irange:
                diag = prob.sigma_t[:, j, i][:, None] + 0.0 * ax
                rhs_ = r[:, sl, j, i].copy()
                iu, ju = i + di, j + dj
                if 0 <= iu < N:
                    diag = diag + ax
                    rhs_ += ax * x[:, sl, j, iu]
                elif xbc == VACUUM:
                    diag = diag + ax    # upstream halo value is 0
                # zero gradient: the halo copies this node, the x-term is zero
                if 0 <= ju < N:
                    diag = diag + ay
                    rhs_ += ay * x[:, sl, ju, i]
                elif ybc == VACUUM:
                    diag = diag + ay
                x[:, sl, j, i] = rhs_ / diag
    return x


def gmres_solve(prob, tol=1e-13, restart=60, max_restarts=400, x0=None):
    """Right-preconditioned restarted GMRES (own implementation on top of numpy) for A psi = b.

    Returns (psi, relative true residual ||b - A psi|| / ||b|| in the plain 2-norm).
    """
    op = _linear(prob)
    shape = prob.shape()
    b = rhs(prob).ravel()
    bn = np.linalg.norm(b)
    x = np.zeros_like(b) if x0 is None else x0.ravel().copy()
    Aop = lambda v: op(v.reshape(shape)).ravel()
    Minv = lambda v: transport_sweep(prob, v.reshape(shape)).ravel()
    for _ in range(max_restarts):
        r = b - Aop(x)
        beta = np.linalg.norm(r)
        if beta <= tol * bn:
            break
        V = np.zeros((restart + 1, b.size))
        Z = np.zeros((restart, b.size))
        H = np.zeros((restart + 1, restart))
        V[0] = r / beta
        k_used = 0
        for k in range(restart):
            Z[k] = Minv(V[k])
            w = Aop(Z[k])
            for i in range(k + 1):           # modified Gram-Schmidt, twice
                H[i, k] = V[i] @ w
                w = w - H[i, k] * V[i]
            for i in range(k + 1):
                c = V[i] @ w
                H[i, k] += c
                w = w - c * V[i]
            H[k + 1, k] = np.linalg.norm(w)
            k_used = k + 1
            e1 = np.zeros(k + 2)
            e1[0] = beta
            y, *_ = np.linalg.lstsq(H[:k + 2, :k + 1], e1, rcond=None)
            res = np.linalg.norm(H[:k + 2, :k + 1] @ y - e1)
            if H[k + 1, k] == 0.0 or res <= 0.1 * tol * bn:
                break
            V[k + 1] = w / H[k + 1, k]
        x = x + Z[:k_used].T @ y
    rel = np.linalg.norm(b - Aop(x)) / bn
    return x.reshape(shape), rel


def picard_solve(prob, psi0, tol=1e-12, max_iter=200, inner=gmres_solve):
    """Non-linear PG: psi_{m+1} = solution of the frozen-k equations with k = k(psi_m).

    Returns (psi, list of relative changes ||psi_{m+1} - psi_m|| / ||psi_{m+1}||, converged)."""
    disc = prob.disc
    psi = psi0.copy()
    hist = []
    try:
        prob.disc = PG_FROZEN
        for _ in range(max_iter):
            prob.k_frozen = pg_diffusivity(psi, prob.quad, prob.h, prob.h, prob.p, prob.bc)
            new, _ = inner(prob, x0=psi) if inner is gmres_solve else (inner(prob), None)
            ch = np.linalg.norm(new - psi) / max(np.linalg.norm(new), 1e-300)
            hist.append(ch)
            psi = new
            if ch <= tol:
                return psi, hist, True
        return psi, hist, False
    finally:
        prob.disc = disc
        prob.k_frozen = None
