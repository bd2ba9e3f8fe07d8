"""Finest-level discrete transport operators (paper, sections "Boltzmann Transport Equation",
"Discrete Ordinates", "Discretisation in Cartesian space", "Optimised Anisotropic Non-Linear
Petrov-Galerkin Dissipation").

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Arrays: psi[g, n, j, i] (group, ordinate, y node, x node); N_y x N_x interior nodes at cell centres
of a uniform grid, plus halos outside (reading of the garbled index ranges of eq. discretised_hfm).
Materials sigma_t[g, j, i], sigma_s[l, g_to, g_from, j, i] (l = 0 isotropic, l = 1 linearly
anisotropic), isotropic external source S[g, j, i].

Sign convention: rho = b - A(psi) (the paper's residual r of eq. Petrov is A psi - b = -rho).
"""
import numpy as np

from .convfem import apply_filter, filters_2d, upwind_filters

VACUUM = "vacuum"
ZERO_GRADIENT = "zero_gradient"

# Petrov-Galerkin constants stated in the paper: eps_k = 0.001, alpha_kabs = 2^p/16,
# alpha_ksquare = 2^p/2 (eq. scalars_alpha) and beta_r = 3 (mixed-mass residual); alpha_r of the
# anisotropic residuals is not defined separately and is read as beta_r.
EPS_K = 1.0e-3
ALPHA_R = 3.0


def alpha_kabs(p):
    return 2.0**p / 16.0


def alpha_ksquare(p):
    return 2.0**p / 2.0


# ----------------------------------------------------------------------------------------------
# halo rule (section "Discretisation in Cartesian space": incoming halo values are zero (bare
# surface); outgoing halo values copy the solution just inside the domain; eq. diff-reflect gives
# the zero-normal-gradient boundary used by the closed-form tests)
def halo_extend(psi, mu, nu, width, bc):
    """Pad the last two axes of psi[..., n, j, i] by ``width`` halo layers.

    bc = (x-, x+, y-, y+), each VACUUM or ZERO_GRADIENT.  The x-halos of the interior rows are
    filled first, then the y-halos across the full padded width (which sets the corners).
    """
    ny, nx = psi.shape[-2:]
    W = width
    ext = np.zeros(psi.shape[:-2] + (ny + 2 * W, nx + 2 * W))
    ext[..., W:W + ny, W:W + nx] = psi
    for n in range(psi.shape[-3]):
        # x- side: a direction with mu > 0 enters the domain there
        if not (bc[0] == VACUUM and mu[n] > 0):
            ext[..., n, W:W + ny, :W] = psi[..., n, :, 0:1]
        if not (bc[1] == VACUUM and mu[n] < 0):
            ext[..., n, W:W + ny, W + nx:] = psi[..., n, :, nx - 1:nx]
        if not (bc[2] == VACUUM and nu[n] > 0):
            ext[..., n, :W, :] = ext[..., n, W:W + 1, :]
        if not (bc[3] == VACUUM and nu[n] < 0):
            ext[..., n, W + ny:, :] = ext[..., n, W + ny - 1:W + ny, :]
    return ext


def clamp_extend(a, width):
    """Copy-extend the last two axes (each halo value = the nearest interior value)."""
    return np.pad(a, [(0, 0)] * (a.ndim - 2) + [(width, width), (width, width)], mode="edge")


# ----------------------------------------------------------------------------------------------
# moments and emission (scalar flux phi_g = sum_n p_n psi_{n,g}; isotropic emission (sigma_s phi + S)
# / 4pi, the reading of the garbled psi~ = p_n phi / p_n line that keeps phi = S / sigma_a in an
# infinite medium; linearly anisotropic scattering adds 3/(4 pi) sigma_s1 (mu Phi_1 + nu Phi_2))
def moments(psi, quad):
    """Phi[g, m, j, i] for m = 0 (sum p psi), 1 (sum p mu psi), 2 (sum p nu psi)."""
    p, mu, nu = quad["p"], quad["mu"], quad["nu"]
    return np.stack([
        np.einsum("gnji,n->gji", psi, p),
        np.einsum("gnji,n->gji", psi, p * mu),
        np.einsum("gnji,n->gji", psi, p * nu),
    ], axis=1)


def emission(psi, quad, sigma_s, source):
    """q[g, n, j, i] = [S_g + sum_g' s0(g'->g) Phi0_g' + 3 sum_g' s1(g'->g)(mu_n Phi1 + nu_n Phi2)]/4pi."""
    return emission_from_moments(moments(psi, quad), quad, sigma_s, source)


def emission_from_moments(Phi, quad, sigma_s, source):
    """The emission above from given moments Phi[g, m, j, i], for the ordinates of ``quad`` (which
    may be a subset of the set the moments were summed over)."""
    G = Phi.shape[0]
    nd = len(quad["mu"])
    q = np.zeros((G, nd) + Phi.shape[2:])
    for g in range(G):
        iso = source[g].copy()
        for gp in range(G):
            iso = iso + sigma_s[0, g, gp] * Phi[gp, 0]
        q[g] = iso[None, :, :]
        if sigma_s.shape[0] > 1:
            for gp in range(G):
                for n in range(nd):
                    q[g, n] += 3.0 * sigma_s[1, g, gp] * (quad["mu"][n] * Phi[gp, 1] + quad["nu"][n] * Phi[gp, 2])
    return q / (4.0 * np.pi)


# ----------------------------------------------------------------------------------------------
# upwind operator (eq. discretised_hfm with the upwind filters of section "Neural network filters")
def upwind_advection(psi, quad, dx, dy, bc):
    """mu f(psi; w_x^up) + nu f(psi; w_y^up), filters chosen per ordinate by the signs."""
    mu, nu = quad["mu"], quad["nu"]
    ext = halo_extend(psi, mu, nu, 1, bc)
    out = np.zeros(psi.shape)
    for n in range(psi.shape[1]):
        wx, wy = upwind_filters(mu[n], nu[n], dx, dy)
        out[:, n] = mu[n] * apply_filter(ext[:, n], wx) + nu[n] * apply_filter(ext[:, n], wy)
    return out


def upwind_residual(psi, q, sigma_t, quad, dx, dy, bc):
    """rho = q - A_up psi - sigma_t psi (q = emission, already divided by 4 pi)."""
    return q - upwind_advection(psi, quad, dx, dy, bc) - sigma_t[:, None] * psi


def upwind_diagonal(sigma_t, quad, dx, dy):
    """Diagonal d[g, n, j, i] = |mu|/dx + |nu|/dy + sigma_t of the upwind filter system."""
    a = np.abs(quad["mu"]) / dx + np.abs(quad["nu"]) / dy
    return a[None, :, None, None] + sigma_t[:, None, :, :]


# ----------------------------------------------------------------------------------------------
# Petrov-Galerkin (eq. Petrov with k-Diff of eqs. kxx/kyy and the anisotropic k of eq. ano-k)
def pg_gradients(psi, quad, dx, dy, p, bc):
    """Psi_x = f(psi; w_x), Psi_y = f(psi; w_y) on the interior plus a p-wide ring.

    psi gets a 2p-wide halo so that the ring values exist (halo width not stated in the paper).
    """
    F = filters_2d(p, dx, dy)
    ext = halo_extend(psi, quad["mu"], quad["nu"], 2 * p, bc)
    return apply_filter(ext, F["wx"]), apply_filter(ext, F["wy"]), ext


def pg_diffusivity(psi, quad, dx, dy, p, bc, alpha_r=ALPHA_R, eps_k=EPS_K):
    """Anisotropic non-linear PG diffusivities (k_x, k_y) on the interior (eq. ano-k)."""
    F = filters_2d(p, dx, dy)
    Px, Py, _ = pg_gradients(psi, quad, dx, dy, p, bc)
    mu = quad["mu"][None, :, None, None]
    nu = quad["nu"][None, :, None, None]
    Px_i = Px[..., p:-p, p:-p]
    Py_i = Py[..., p:-p, p:-p]
    # residual estimates from the mixed mass: f(f(psi; w_x); m_L^-1 m - I)
    Rx = alpha_r * mu * (apply_filter(Px, F["wm"]) - Px_i)
    Ry = alpha_r * nu * (apply_filter(Py, F["wm"]) - Py_i)
    akabs, aksq = alpha_kabs(p), alpha_ksquare(p)
    kx_abs = akabs * np.abs(Rx) * dx / (eps_k + np.abs(Px_i))
    ky_abs = akabs * np.abs(Ry) * dy / (eps_k + np.abs(Py_i))
    kx_sq = aksq * Rx**2 * dx / (eps_k + np.abs(mu) * Px_i**2)
    ky_sq = aksq * Ry**2 * dy / (eps_k + np.abs(nu) * Py_i**2)
    kx_max = dx * np.abs(mu) + 0 * kx_abs
    ky_max = dy * np.abs(nu) + 0 * ky_abs
    kx = np.minimum(np.minimum(kx_max, kx_abs), kx_sq)
    ky = np.minimum(np.minimum(ky_max, ky_abs), ky_sq)
    return kx, ky


R_MIXED, R_LOW, R_HIGH = "mixed", "low", "high"


def advection_estimate(psi, quad, dx, dy, p, bc):
    """mu f(psi; w_x) + nu f(psi; w_y) with the ConvFEM filters of degree p, on the interior
    (psi gets a halo of width p by the halo rule)."""
    F = filters_2d(p, dx, dy)
    ext = halo_extend(psi, quad["mu"], quad["nu"], p, bc)
    mu = quad["mu"][None, :, None, None]
    nu = quad["nu"][None, :, None, None]
    return mu * apply_filter(ext, F["wx"]) + nu * apply_filter(ext, F["wy"])


def isotropic_residual_estimate(psi, quad, dx, dy, p, bc, r_estimate=R_MIXED, beta_r=ALPHA_R):
    """The residual estimate R of the isotropic diffusivity on the interior, one of the three of
    section "Non-Linear Petrov-Galerkin Dissipation", with Psi_x = f(psi; w_x), Psi_y = f(psi; w_y)
    of degree p:
        mixed: R = beta_r f(mu Psi_x + nu Psi_y; m_L^-1 m - I)   (beta_r read as alpha_r = 3)
        low:   R = (mu Psi_x + nu Psi_y) - (the same with the filters of degree p - 1),   p >= 2
        high:  R = (the same with the filters of degree p + 1) - (mu Psi_x + nu Psi_y)
    No coefficient is printed for the low and high estimates and none is applied.
    Returns (R, Psi_x, Psi_y) on the interior."""
    F = filters_2d(p, dx, dy)
    Px, Py, _ = pg_gradients(psi, quad, dx, dy, p, bc)
    mu = quad["mu"][None, :, None, None]
    nu = quad["nu"][None, :, None, None]
    Px_i = Px[..., p:-p, p:-p]
    Py_i = Py[..., p:-p, p:-p]
    if r_estimate == R_MIXED:
        adv = mu * Px + nu * Py
        R = beta_r * (apply_filter(adv, F["wm"]) - adv[..., p:-p, p:-p])
    elif r_estimate == R_LOW:
        if p < 2:
            raise ValueError("the low-order residual estimate needs p >= 2")
        R = (mu * Px_i + nu * Py_i) - advection_estimate(psi, quad, dx, dy, p - 1, bc)
    elif r_estimate == R_HIGH:
        R = advection_estimate(psi, quad, dx, dy, p + 1, bc) - (mu * Px_i + nu * Py_i)
    else:
        raise ValueError(r_estimate)
    return R, Px_i, Py_i


def pg_diffusivity_isotropic(psi, quad, dx, dy, p, bc, beta_r=ALPHA_R, eps_k=EPS_K, r_estimate=R_MIXED):
    """Isotropic non-linear PG diffusivity, the paper's first residual-based form (section
    "Non-Linear Petrov-Galerkin Dissipation"):

        k_abs = akabs |R| h / (eps + (|Psi_x| + |Psi_y|) / D),                        D = 2
        q = (mu Psi_x + nu Psi_y) / (eps + Psi_x^2 + Psi_y^2)
        k_square = aksq R^2 h / (eps + (|q Psi_x| + |q Psi_y|) / D (Psi_x^2 + Psi_y^2))
        k_max = sqrt((dx mu)^2 + (dy nu)^2),   k = min(k_max, k_abs, k_square),   h = (dx + dy) / 2

    on the interior, R from isotropic_residual_estimate.  The same k acts in x and y: returns (k, k)."""
    R, Px_i, Py_i = isotropic_residual_estimate(psi, quad, dx, dy, p, bc, r_estimate, beta_r)
    mu = quad["mu"][None, :, None, None]
    nu = quad["nu"][None, :, None, None]
    h = 0.5 * (dx + dy)
    akabs, aksq = alpha_kabs(p), alpha_ksquare(p)
    k_abs = akabs * np.abs(R) * h / (eps_k + (np.abs(Px_i) + np.abs(Py_i)) / 2.0)
    q = (mu * Px_i + nu * Py_i) / (eps_k + Px_i**2 + Py_i**2)
    k_sq = aksq * R**2 * h / (eps_k + (np.abs(q * Px_i) + np.abs(q * Py_i)) / 2.0 * (Px_i**2 + Py_i**2))
    k_max = np.sqrt((dx * mu) ** 2 + (dy * nu) ** 2) + 0 * k_abs
    k = np.minimum(np.minimum(k_max, k_abs), k_sq)
    return k, k


def k_diff(psi_ext_p, k, w, p):
    """f^{k-Diff}(Psi; k, w) = f(k.Psi; w) + k.f(Psi; w) - Psi.f(k; w) (eqs. kxx, kyy), taken as
    the definition (the 1/2 of the analytic identity is not in it).  psi_ext_p has a p-wide halo;
    k is interior-only and gets a copied p-wide halo (reading: halo values of k are not stated)."""
    k_ext = clamp_extend(k, p)
    psi_i = psi_ext_p[..., p:-p, p:-p]
    return apply_filter(k_ext * psi_ext_p, w) + k * apply_filter(psi_ext_p, w) - psi_i * apply_filter(k_ext, w)


def pg_residual(psi, q, sigma_t, quad, dx, dy, p, bc, k=None, isotropic=False, r_estimate=R_MIXED):
    """rho = q - mu Psi_x - nu Psi_y - kDiff_x - kDiff_y - sigma_t psi (lumped mass, w_ml = 1 in
    the per-unit-volume normalisation of the printed filters).

    k = None: non-linear PG, k from psi (anisotropic, eq. ano-k; or the isotropic form with the
    residual estimate r_estimate).
    k = (kx, ky): frozen diffusivities.
    """
    F = filters_2d(p, dx, dy)
    if k is None:
        if isotropic:
            k = pg_diffusivity_isotropic(psi, quad, dx, dy, p, bc, r_estimate=r_estimate)
        else:
            k = pg_diffusivity(psi, quad, dx, dy, p, bc)
    kx, ky = k
    Px, Py, ext = pg_gradients(psi, quad, dx, dy, p, bc)
    mu = quad["mu"][None, :, None, None]
    nu = quad["nu"][None, :, None, None]
    ext_p = ext[..., p:-p, p:-p]
    Dx = k_diff(ext_p, kx, F["wDxx"], p)
    Dy = k_diff(ext_p, ky, F["wDyy"], p)
    return (q - mu * Px[..., p:-p, p:-p] - nu * Py[..., p:-p, p:-p] - Dx - Dy
            - sigma_t[:, None] * psi)


# ----------------------------------------------------------------------------------------------
def weighted_norm(v, quad, dx, dy):
    """||v||_W = sqrt(sum_{g,n,j,i} p_n dx dy v^2)."""
    return float(np.sqrt(np.einsum("gnji,n->", v * v, quad["p"]) * dx * dy))


def source_norm(source, quad, dx, dy):
    """||b||_W of b_{g,n} = S_g / 4 pi."""
    b = np.broadcast_to(source[:, None] / (4.0 * np.pi), (source.shape[0], len(quad["p"])) + source.shape[1:])
    return weighted_norm(np.ascontiguousarray(b), quad, dx, dy)
