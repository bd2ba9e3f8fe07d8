"""Space-angle multigrid: hierarchy, restriction, UpSamp, Jacobi smoothers, sawtooth cycle, solve
(paper, section "Space-Angle Multigrid", eq. matrix_full, and the sawtooth-cycle figure).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Readings adopted where the paper is silent:
* hierarchy: halve x, y and both face-angle indices per level (N_a stops at 1); stop once N is odd
  or N <= 2 (or at ``max_levels``);
* coarse materials: harmonic mean of the 2x2 children of sigma_t (0 if any child is 0);
* coarse ordinates: patches added (p summed, p-weighted mean direction);
* restriction: the paper's two stages (multiply by p_n dx dy; 2x2 ones filter, here in all four
  dimensions) followed by division by the coarse p_N H^2, so that every level's equation is per
  unit volume and solid angle like the finest one;
* smoothing counts: n_j upwind Jacobi sweeps on every level (the coarsest from zero), then on the
  finest level psi += e_0 followed by n_pg Petrov-Galerkin Jacobi sweeps with beta = 3 (the upwind
  discretisation uses beta = 1 there);
* the emission (scattering and group coupling) is re-evaluated in every finest-level residual;
  the correction sweeps are transport only.
"""
import numpy as np

from . import quadrature as qd
from .transport import (VACUUM, emission, pg_diffusivity, pg_diffusivity_isotropic, pg_residual, source_norm,
                        upwind_advection, upwind_diagonal, upwind_residual, weighted_norm)

UPWIND = "upwind"
PG = "pg"
PG_FROZEN = "pg_frozen"


def harmonic_coarsen(sig):
    """Harmonic mean of the 2x2 children over the last two axes; 0 where any child is 0."""
    c = [sig[..., 0::2, 0::2], sig[..., 1::2, 0::2], sig[..., 0::2, 1::2], sig[..., 1::2, 1::2]]
    zero = np.zeros(c[0].shape, dtype=bool)
    for x in c:
        zero |= (x == 0.0)
    safe = [np.where(zero, 1.0, x) for x in c]
    hm = 4.0 / (1.0 / safe[0] + 1.0 / safe[1] + 1.0 / safe[2] + 1.0 / safe[3])
    return np.where(zero, 0.0, hm)


class Level:
    def __init__(self, N, h, quad, sigma_t, sigma_s):
        self.N, self.h, self.quad, self.sigma_t, self.sigma_s = N, h, quad, sigma_t, sigma_s


class Problem:
    """A fixed-source problem on the square [0, L]^2 with N x N nodes (h = L / N)."""

    def __init__(self, N, L, p, na, sigma_t, sigma_s, source, bc=(VACUUM,) * 4, disc=PG,
                 n_jacobi=2, n_pg=None, max_levels=0, beta_pg=3.0, quad=None, coupled=False,
                 isotropic=False, r_estimate="mixed"):
        self.N, self.L, self.p, self.na = N, L, p, na
        self.h = L / N
        self.sigma_t = np.asarray(sigma_t, dtype=float)
        self.sigma_s = np.asarray(sigma_s, dtype=float)
        self.source = np.asarray(source, dtype=float)
        self.G = self.sigma_t.shape[0]
        self.bc, self.disc = tuple(bc), disc
        self.n_jacobi = n_jacobi
        self.n_pg = n_jacobi if n_pg is None else n_pg
        self.beta_pg = beta_pg
        self.k_frozen = None
        # extension (the paper is silent): correction sweeps that include the scattering of the
        # correction on every level
        self.coupled = coupled
        self.isotropic = isotropic   # the isotropic PG diffusivity instead of the anisotropic one
        self.r_estimate = r_estimate  # its residual estimate: "mixed", "low" or "high"
        q0 = quad if quad is not None else qd.quadrature(na)
        self.levels = [Level(N, self.h, q0, self.sigma_t, self.sigma_s)]
        while True:
            lv = self.levels[-1]
            if lv.N % 2 or lv.N <= 2 or (max_levels and len(self.levels) >= max_levels):
                break
            self.levels.append(Level(lv.N // 2, 2 * lv.h, qd.coarsen(lv.quad), harmonic_coarsen(lv.sigma_t),
                                     harmonic_coarsen(lv.sigma_s)))

    @property
    def quad(self):
        return self.levels[0].quad

    def shape(self, level=0):
        lv = self.levels[level]
        return (self.G, len(lv.quad["p"]), lv.N, lv.N)

    def freeze_k(self, psi):
        """Hold k_x, k_y of psi for the PG_FROZEN discretisation."""
        if self.isotropic:
            self.k_frozen = pg_diffusivity_isotropic(psi, self.quad, self.h, self.h, self.p, self.bc,
                                                     r_estimate=self.r_estimate)
        else:
            self.k_frozen = pg_diffusivity(psi, self.quad, self.h, self.h, self.p, self.bc)


# ----------------------------------------------------------------------------------------------
def finest_residual(prob, psi, source=None):
    """rho_0 = b - A(psi) of the finest discretisation, with the emission of the current psi."""
    src = prob.source if source is None else source
    q = emission(psi, prob.quad, prob.sigma_s, src)
    h = prob.h
    if prob.disc == UPWIND:
        return upwind_residual(psi, q, prob.sigma_t, prob.quad, h, h, prob.bc)
    k = prob.k_frozen if prob.disc == PG_FROZEN else None
    if prob.disc == PG_FROZEN and k is None:
        raise ValueError("PG_FROZEN needs freeze_k first")
    return pg_residual(psi, q, prob.sigma_t, prob.quad, h, h, prob.p, prob.bc, k=k, isotropic=prob.isotropic,
                       r_estimate=prob.r_estimate)


def apply_operator(prob, psi):
    """A(psi) without the external source (transport, dissipation, removal, minus scattering)."""
    return -finest_residual(prob, psi, source=np.zeros_like(prob.source))


def restrict(rho, lf, lc):
    """Restriction of section "Space-Angle Multigrid": r_mod = p_n r dx dy, then the 2x2 ones
    filter (stride 2) in space and the sum over the 2x2 child patches in angle; divided by the
    coarse p_N H^2 (per unit volume / solid angle form)."""
    qf, qc = lf.quad, lc.quad
    mod = rho * qf["p"][None, :, None, None] * lf.h * lf.h
    sp = mod[..., 0::2, 0::2] + mod[..., 1::2, 0::2] + mod[..., 0::2, 1::2] + mod[..., 1::2, 1::2]
    out = np.zeros((rho.shape[0], len(qc["p"])) + sp.shape[2:])
    for n in range(rho.shape[1]):
        out[:, qd.parent_index(n, qf["na"])] += sp[:, n]
    return out / (qc["p"][None, :, None, None] * lc.h * lc.h)


def upsample(e_c, lf):
    """UpSamp: copy each coarse value to its 2x2 spatial and 2x2 angular children."""
    na = lf.quad["na"]
    nd = len(lf.quad["p"])
    out = np.zeros((e_c.shape[0], nd, 2 * e_c.shape[2], 2 * e_c.shape[3]))
    for n in range(nd):
        c = e_c[:, qd.parent_index(n, na)]
        out[:, n] = np.repeat(np.repeat(c, 2, axis=-1), 2, axis=-2)
    return out


def upwind_jacobi(prob, level, e, s, nsweeps, beta=1.0):
    """e <- e + (s - A_up e - sigma_t e) / (beta d) on one level (eq. matrix_full with the upwind
    system; beta = 1 on every grid for the upwind scheme).

    With ``prob.coupled`` (an extension; the paper is silent) the sweep also adds the scattering
    of the correction, the emission of e with no external source on the level's own ordinates and
    (harmonically averaged) sigma_s: e <- e + (s + S e - A_up e - sigma_t e) / (beta d), d as above."""
    lv = prob.levels[level]
    d = beta * upwind_diagonal(lv.sigma_t, lv.quad, lv.h, lv.h)
    for _ in range(nsweeps):
        r = s - upwind_advection(e, lv.quad, lv.h, lv.h, prob.bc) - lv.sigma_t[:, None] * e
        if prob.coupled:
            r = r + emission(e, lv.quad, lv.sigma_s, np.zeros_like(lv.sigma_t))
        e = e + r / d
    return e


def finest_jacobi(prob, psi, nsweeps):
    """Finest-level Jacobi on the full equations: psi <- psi + rho(psi) / (beta d_0), beta = 3 for
    the Petrov-Galerkin discretisation, 1 for the upwind one."""
    lv = prob.levels[0]
    beta = 1.0 if prob.disc == UPWIND else prob.beta_pg
    d = beta * upwind_diagonal(lv.sigma_t, lv.quad, lv.h, lv.h)
    for _ in range(nsweeps):
        psi = psi + finest_residual(prob, psi) / d
    return psi


def sawtooth_cycle(prob, psi, rho0=None):
    """One sawtooth cycle: restrict the finest residual to every level, Jacobi from zero on the
    coarsest, then UpSamp + Jacobi level by level up to the finest, update psi, finest smoothing."""
    L = len(prob.levels)
    rho = [finest_residual(prob, psi) if rho0 is None else rho0]
    for l in range(1, L):
        rho.append(restrict(rho[-1], prob.levels[l - 1], prob.levels[l]))
    e = upwind_jacobi(prob, L - 1, np.zeros(prob.shape(L - 1)), rho[L - 1], prob.n_jacobi)
    for l in range(L - 2, -1, -1):
        e = upsample(e, prob.levels[l])
        e = upwind_jacobi(prob, l, e, rho[l], prob.n_jacobi)
    psi = psi + e
    return finest_jacobi(prob, psi, prob.n_pg)


def rel_residual(prob, rho):
    return weighted_norm(rho, prob.quad, prob.h, prob.h) / source_norm(prob.source, prob.quad, prob.h, prob.h)


def solve(prob, psi=None, rtol=1e-8, max_cycles=200):
    """Repeat sawtooth cycles from psi (default 0) until ||rho||_W / ||b||_W <= rtol.

    Returns (psi, history of relative residuals, converged flag); the residual checked is the one
    the next cycle starts from.
    """
    psi = np.zeros(prob.shape()) if psi is None else psi.copy()
    hist = []
    for c in range(max_cycles + 1):
        rho = finest_residual(prob, psi)
        rel = rel_residual(prob, rho)
        hist.append(rel)
        if rel <= rtol:
            return psi, hist, True
        if c == max_cycles:
            break
        psi = sawtooth_cycle(prob, psi, rho0=rho)
    return psi, hist, False
