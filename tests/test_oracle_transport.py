"""Pins of the oracle's transport operators against closed forms (CPU only).

* infinite medium (zero-gradient halos everywhere, uniform data): psi = S / (4 pi sigma_a) makes
  every residual vanish, for the upwind and the Petrov-Galerkin discretisations of every degree;
  with downscatter the group fluxes follow by forward substitution;
* manufactured solution: the truncation error of the PG residual falls with the formal order of
  the ConvFEM stencils (2 / 4 / 4 for p = 1 / 2 / 3);
* halo rule: incoming halo 0 and outgoing copy, checked node by node on a small grid;
* the P1 emission leaves the particle balance unchanged (sum p mu = sum p nu = 0).
"""
import numpy as np
import pytest

from oracle import quadrature as qd
from oracle.convfem import filters_2d
from oracle.transport import (VACUUM, ZERO_GRADIENT, emission, halo_extend, moments,
                              pg_diffusivity, pg_residual, upwind_residual, weighted_norm)

ZG = (ZERO_GRADIENT,) * 4
VAC = (VACUUM,) * 4


def _uniform(G, N, val):
    return np.full((G, N, N), float(val))


@pytest.mark.parametrize("p", [1, 2, 3])
def test_infinite_medium_residual_vanishes(p):
    N, na = 12, 2
    quad = qd.quadrature(na)
    st, c, S = 1.3, 0.7, 2.0
    sigma_t = _uniform(1, N, st)
    sigma_s = (c * sigma_t)[None, None]
    source = _uniform(1, N, S)
    psi = np.full((1, 8 * na * na, N, N), S / (4 * np.pi * (st - c * st)))
    q = emission(psi, quad, sigma_s, source)
    for r in (upwind_residual(psi, q, sigma_t, quad, 0.1, 0.1, ZG),
              pg_residual(psi, q, sigma_t, quad, 0.1, 0.1, p, ZG)):
        assert np.abs(r).max() < 1e-13 * np.abs(q).max()


def test_infinite_medium_downscatter_closed_form():
    # sigma_t0 phi0 = S0 + s00 phi0 ; sigma_t1 phi1 = s10 phi0 + s11 phi1 (forward substitution)
    N, na = 8, 1
    quad = qd.quadrature(na)
    st0, st1, s00, s10, s11, S0 = 1.5, 0.8, 0.4, 0.5, 0.6, 1.0
    phi0 = S0 / (st0 - s00)
    phi1 = s10 * phi0 / (st1 - s11)
    sigma_t = np.stack([_uniform(1, N, st0)[0], _uniform(1, N, st1)[0]])
    sigma_s = np.zeros((1, 2, 2, N, N))
    sigma_s[0, 0, 0], sigma_s[0, 1, 0], sigma_s[0, 1, 1] = s00, s10, s11
    source = np.stack([_uniform(1, N, S0)[0], np.zeros((N, N))])
    psi = np.zeros((2, 8, N, N))
    psi[0], psi[1] = phi0 / (4 * np.pi), phi1 / (4 * np.pi)
    q = emission(psi, quad, sigma_s, source)
    for p in (1, 2):
        r = pg_residual(psi, q, sigma_t, quad, 0.25, 0.25, p, ZG)
        assert np.abs(r).max() < 1e-14


def test_p1_emission_conserves_particles():
    N, na = 6, 2
    quad = qd.quadrature(na)
    rng = np.random.default_rng(3)
    psi = rng.uniform(size=(1, 32, N, N))
    ss = np.zeros((2, 1, 1, N, N))
    ss[0, 0, 0] = 0.5
    ss1 = ss.copy()
    ss1[1, 0, 0] = 0.3
    q0 = emission(psi, quad, ss, np.zeros((1, N, N)))
    q1 = emission(psi, quad, ss1, np.zeros((1, N, N)))
    # the P1 part adds nothing to sum_n p_n q_n
    assert np.allclose(np.einsum("gnji,n->gji", q1 - q0, quad["p"]), 0, atol=1e-15)
    # and is 3/(4 pi) s1 (mu Phi1 + nu Phi2) for a purely linear angular flux psi = mu_n
    lin = np.broadcast_to(quad["mu"][None, :, None, None], (1, 32, N, N)).copy()
    Phi = moments(lin, quad)
    assert np.allclose(Phi[0, 0], 0, atol=1e-14)
    assert np.allclose(Phi[0, 1], np.dot(quad["p"], quad["mu"] ** 2))


def test_halo_rule_vacuum_and_copy():
    quad = qd.quadrature(1)
    N = 4
    psi = np.arange(1.0, 1 + 8 * N * N).reshape(1, 8, N, N)
    ext = halo_extend(psi, quad["mu"], quad["nu"], 2, VAC)
    for n in range(8):
        mu, nu = quad["mu"][n], quad["nu"][n]
        # x- side: zero when entering (mu > 0), else copy of column 0 on interior rows
        left = ext[0, n, 2:2 + N, :2]
        expect = 0 * left if mu > 0 else np.repeat(psi[0, n, :, :1], 2, axis=1)
        assert np.array_equal(left, expect)
        right = ext[0, n, 2:2 + N, 2 + N:]
        expect = 0 * right if mu < 0 else np.repeat(psi[0, n, :, -1:], 2, axis=1)
        assert np.array_equal(right, expect)
        # corner: zero when entering through either side, else the corner node
        corner = ext[0, n, 0, 0]
        assert corner == (0.0 if (mu > 0 or nu > 0) else psi[0, n, 0, 0])
        corner = ext[0, n, -1, -1]
        assert corner == (0.0 if (mu < 0 or nu < 0) else psi[0, n, -1, -1])


def test_upwind_residual_by_hand():
    quad = qd.quadrature(1)
    N, h = 3, 0.5
    rng = np.random.default_rng(1)
    psi = rng.normal(size=(1, 8, N, N))
    st = rng.uniform(0.5, 2, size=(1, N, N))
    q = rng.normal(size=(1, 8, N, N))
    r = upwind_residual(psi, q, st, quad, h, h, VAC)
    for n in range(8):
        mu, nu = quad["mu"][n], quad["nu"][n]
        for j in range(N):
            for i in range(N):
                def val(jj, ii):
                    return psi[0, n, jj, ii] if (0 <= ii < N and 0 <= jj < N) else 0.0
                if mu > 0:
                    ax = mu * (val(j, i) - val(j, i - 1)) / h
                else:
                    ax = mu * (val(j, i + 1) - val(j, i)) / h
                if nu > 0:
                    ay = nu * (val(j, i) - val(j - 1, i)) / h
                else:
                    ay = nu * (val(j + 1, i) - val(j, i)) / h
                ref = q[0, n, j, i] - ax - ay - st[0, j, i] * psi[0, n, j, i]
                assert np.isclose(r[0, n, j, i], ref, rtol=1e-13, atol=1e-13)


def _bump(x):
    y = np.zeros_like(x)
    t = (x - 0.2) / 0.6
    m = (t > 0) & (t < 1)
    y[m] = np.exp(-1.0 / (t[m] * (1 - t[m])) + 4.0)
    return y


def _dbump(x):
    y = np.zeros_like(x)
    t = (x - 0.2) / 0.6
    m = (t > 0) & (t < 1)
    tt = t[m]
    y[m] = np.exp(-1.0 / (tt * (1 - tt)) + 4.0) * (1 - 2 * tt) / (tt * (1 - tt)) ** 2 / 0.6
    return y


def _mms_truncation(p, N, quad):
    """||rho(psi_ms)||_W with the continuum source of a smooth compactly supported solution."""
    h = 1.0 / N
    xc = (np.arange(N) + 0.5) * h
    X, Y = np.meshgrid(xc, xc, indexing="xy")
    B, Bx, By = _bump(X) * _bump(Y), _dbump(X) * _bump(Y), _bump(X) * _dbump(Y)
    mu, nu = quad["mu"], quad["nu"]
    ang = 1 + 0.3 * mu + 0.2 * nu
    psi = (B[None] * ang[:, None, None])[None]
    sig = np.ones((1, N, N))
    q = (psi * sig[:, None] + (mu * ang)[None, :, None, None] * Bx[None, None]
         + (nu * ang)[None, :, None, None] * By[None, None])
    r = pg_residual(psi, q, sig, quad, h, h, p, VAC)
    return weighted_norm(r, quad, h, h)


@pytest.mark.parametrize("p,order_lo,order_hi,n", [(1, 1.85, 2.15, 64), (2, 3.6, 4.4, 64), (3, 3.4, 4.4, 64),
                                                     (4, 5.0, 6.6, 128)])
def test_manufactured_solution_truncation_order(p, order_lo, order_hi, n):
    # p = 4 (formal order 6) is pre-asymptotic below N = 128 on this bump: the limiter's
    # dissipation still acts there (orders 2.6 and 9.1 between 32, 64 and 128)
    quad = qd.quadrature(1)
    e1 = _mms_truncation(p, n, quad)
    e2 = _mms_truncation(p, 2 * n, quad)
    order = np.log2(e1 / e2)
    assert order_lo < order < order_hi, order


def test_pg_diffusivity_limits():
    # k never exceeds k_max = dx |mu| and vanishes on a linear field (R = 0 there)
    quad = qd.quadrature(2)
    N, h = 10, 0.1
    rng = np.random.default_rng(5)
    psi = rng.uniform(size=(1, 32, N, N))
    kx, ky = pg_diffusivity(psi, quad, h, h, 2, VAC)
    assert np.all(kx <= h * np.abs(quad["mu"])[None, :, None, None] + 1e-15)
    assert np.all(ky <= h * np.abs(quad["nu"])[None, :, None, None] + 1e-15)
    assert np.all(kx >= 0) and np.all(ky >= 0)
    N = 12
    xc = (np.arange(N) + 0.5) * h
    lin = np.broadcast_to((1 + xc)[None, None, None, :], (1, 32, N, N)).copy()
    kx, ky = pg_diffusivity(lin, quad, h, h, 2, ZG)
    # nodes at least 2p from the copied halo see an exactly linear field
    assert np.abs(kx[..., 4:-4, 4:-4]).max() < 1e-12
    assert np.abs(ky).max() < 1e-12


def test_kdiff_symmetric_form():
    # f(k psi; w) + k f(psi; w) - psi f(k; w) = sum_o w_o (k_c + k_o)(psi_o - psi_c), as sum w = 0
    from oracle.transport import clamp_extend, k_diff
    rng = np.random.default_rng(2)
    p, n = 2, 5
    w = filters_2d(p, 1.0, 1.0)["wDxx"]
    assert abs(w.sum()) < 1e-14
    ext = rng.normal(size=(1, 1, n + 2 * p, n + 2 * p))
    k = rng.uniform(size=(1, 1, n, n))
    kd = k_diff(ext, k, w, p)
    kext = clamp_extend(k, p)
    psi_c = ext[..., p:p + n, p:p + n]
    ref = np.zeros_like(kd)
    for v in range(-p, p + 1):
        for u in range(-p, p + 1):
            psi_o = ext[..., p + v:p + v + n, p + u:p + u + n]
            k_o = kext[..., p + v:p + v + n, p + u:p + u + n]
            ref += w[v + p, u + p] * (k + k_o) * (psi_o - psi_c)
    assert np.allclose(kd, ref, atol=1e-12)


def test_isotropic_pg_diffusivity_limits():
    # 0 <= k <= k_max = sqrt((h mu)^2 + (h nu)^2); k = 0 on a linear field; k_x = k_y
    from oracle.transport import pg_diffusivity_isotropic
    quad = qd.quadrature(2)
    N, h = 10, 0.1
    rng = np.random.default_rng(6)
    psi = rng.uniform(size=(1, 32, N, N))
    kx, ky = pg_diffusivity_isotropic(psi, quad, h, h, 2, VAC)
    kmax = h * np.sqrt(quad["mu"] ** 2 + quad["nu"] ** 2)[None, :, None, None]
    assert np.array_equal(kx, ky)
    assert np.all(kx <= kmax + 1e-15) and np.all(kx >= 0)
    N = 12
    xc = (np.arange(N) + 0.5) * h
    lin = np.broadcast_to((1 + 2 * xc)[None, None, None, :], (1, 32, N, N)).copy()
    kx, _ = pg_diffusivity_isotropic(lin, quad, h, h, 2, ZG)
    assert np.abs(kx[..., 4:-4, 4:-4]).max() < 1e-12


def test_isotropic_pg_diffusivity_cubic_closed_form():
    """psi = x^3 with the linear (p = 1) filters, where every quantity has a closed form:
    Psi_x = ((x+h)^3 - (x-h)^3) / 2h = 3x^2 + h^2, Psi_y = 0, and the mass filter m = [1/6, 2/3, 1/6]
    maps 3x^2 + h^2 to 3x^2 + 2h^2, so R = beta_r mu h^2; k from the three bounds."""
    from oracle.transport import pg_diffusivity_isotropic
    quad = qd.quadrature(2)
    mu, nu = quad["mu"][:, None], quad["nu"][:, None]
    N, h, eps, beta_r = 12, 0.3, 1e-3, 3.0
    x = (np.arange(N) + 0.5) * h
    psi = np.broadcast_to((x ** 3)[None, None, None, :], (1, 32, N, N)).copy()
    k, _ = pg_diffusivity_isotropic(psi, quad, h, h, 1, ZG)
    xi = x[2:-2][None, :]
    Px = 3 * xi ** 2 + h ** 2
    R = beta_r * mu * h ** 2
    akabs, aksq = 2.0 / 16.0, 2.0 / 2.0
    k_abs = akabs * np.abs(R) * h / (eps + Px / 2.0)
    q = mu * Px / (eps + Px ** 2)
    k_sq = aksq * R ** 2 * h / (eps + np.abs(q * Px) / 2.0 * Px ** 2)
    k_max = h * np.sqrt(mu ** 2 + nu ** 2)
    ref = np.minimum(np.minimum(k_max, k_abs), k_sq)
    got = k[0, :, 2:-2, 2:-2]
    assert np.allclose(got, ref[:, None, :], rtol=1e-10, atol=1e-15)


def _poly_field(N, h, deg, axis, G=1, nd=32):
    c = (np.arange(N) + 0.5) * h
    f = c ** deg
    shape = (1, 1, 1, N) if axis == "x" else (1, 1, N, 1)
    return np.broadcast_to(f.reshape(shape), (G, nd, N, N)).copy(), c


# R for psi = x^deg (or y^deg) from the moments sum_u u^q d[u] of the 1D derivative stencils:
# d_1 applied to x^3 gives 3x^2 + h^2; d_2 is exact on quintics less -4 h^4 (5x^4 - 4h^4 for x^5);
# d_3 gives 5x^4 + 3h^4 for x^5; d_2, d_3 are exact on cubics and d_4 on quintics.  The mass
# filter along the other axis acts on a constant (sum m = 1).
@pytest.mark.parametrize("p,est,deg,coef,hp", [
    (1, "high", 3, -1.0, 2),   # d_2 - d_1 on x^3: 3x^2 - (3x^2 + h^2)
    (2, "low", 3, -1.0, 2),    # d_2 - d_1 on x^3
    (3, "low", 5, 7.0, 4),     # d_3 - d_2 on x^5: (5x^4 + 3h^4) - (5x^4 - 4h^4)
    (3, "high", 5, -3.0, 4),   # d_4 - d_3 on x^5: 5x^4 - (5x^4 + 3h^4)
    (2, "high", 5, 7.0, 4),    # d_3 - d_2 on x^5, the pair of p = 3 low
])
@pytest.mark.parametrize("axis", ["x", "y"])
def test_low_high_residual_estimates_closed_form(p, est, deg, coef, hp, axis):
    """The low / high residual estimates of the isotropic diffusivity on psi = x^deg (or y^deg):
    R = coef * (mu or nu) * h^hp on nodes whose filters stay inside the domain.  Pins which degree
    is low and which high, the sign and the absence of a coefficient."""
    from oracle.transport import isotropic_residual_estimate
    quad = qd.quadrature(2)
    N, h = 16, 0.25
    psi, _ = _poly_field(N, h, deg, axis)
    R, _, _ = isotropic_residual_estimate(psi, quad, h, h, p, ZG, r_estimate=est)
    s = quad["mu"] if axis == "x" else quad["nu"]
    ref = coef * s[:, None, None] * h ** hp
    r = p + 1
    got = R[0][:, r:-r, r:-r]
    assert np.allclose(got, np.broadcast_to(ref, got.shape), rtol=1e-9, atol=1e-12 * h ** hp)


def test_low_estimate_diffusivity_closed_form():
    """psi = x^3, p = 2, low estimate: Psi_x = 3x^2 exactly, Psi_y = 0, R = -mu h^2; k from the
    three bounds with akabs = 4/16, aksq = 4/2."""
    from oracle.transport import pg_diffusivity_isotropic
    quad = qd.quadrature(2)
    mu, nu = quad["mu"][:, None], quad["nu"][:, None]
    N, h, eps = 16, 0.3, 1e-3
    psi, x = _poly_field(N, h, 3, "x")
    k, _ = pg_diffusivity_isotropic(psi, quad, h, h, 2, ZG, r_estimate="low")
    r = 3
    xi = x[r:-r][None, :]
    Px = 3 * xi ** 2
    R = -mu * h ** 2
    k_abs = 0.25 * np.abs(R) * h / (eps + Px / 2.0)
    q = mu * Px / (eps + Px ** 2)
    k_sq = 2.0 * R ** 2 * h / (eps + np.abs(q * Px) / 2.0 * Px ** 2)
    k_max = h * np.sqrt(mu ** 2 + nu ** 2)
    ref = np.minimum(np.minimum(k_max, k_abs), k_sq)
    got = k[0][:, r:-r, r:-r]
    assert np.allclose(got, np.broadcast_to(ref[:, None, :], got.shape), rtol=1e-10, atol=1e-15)


def test_low_high_estimates_vanish_on_linear_fields():
    """Every degree differentiates a linear field exactly, so both estimates vanish (and so does
    k) away from the boundary; on a random field they differ from each other and from zero."""
    from oracle.transport import isotropic_residual_estimate
    quad = qd.quadrature(2)
    N, h = 14, 0.2
    c = (np.arange(N) + 0.5) * h
    lin = np.broadcast_to((2.0 * c[None, :] - 0.7 * c[:, None] + 1.0)[None, None], (1, 32, N, N)).copy()
    for p, est in ((2, "low"), (3, "low"), (1, "high"), (2, "high"), (3, "high")):
        R, _, _ = isotropic_residual_estimate(lin, quad, h, h, p, ZG, r_estimate=est)
        r = p + 1
        assert np.abs(R[..., r:-r, r:-r]).max() < 1e-11, (p, est)
    rng = np.random.default_rng(3)
    psi = rng.uniform(0.0, 1.0, (1, 32, N, N))
    Rl, _, _ = isotropic_residual_estimate(psi, quad, h, h, 2, VAC, r_estimate="low")
    Rh, _, _ = isotropic_residual_estimate(psi, quad, h, h, 2, VAC, r_estimate="high")
    assert np.abs(Rl).max() > 1e-3 and np.abs(Rh).max() > 1e-3
    assert np.abs(Rl - Rh).max() > 1e-3


@pytest.mark.parametrize("axis", ["x", "y"])
def test_anisotropic_pg_diffusivity_cubic_closed_form(axis):
    """Eq. ano-k on psi = x^3 (or y^3) with the linear filters and dx != dy, every quantity in
    closed form.  Along the field's axis (spacing a, direction cosine c = mu or nu):
    Psi = ((s+a)^3 - (s-a)^3) / 2a = 3s^2 + a^2 (the mass along the other axis acts on a constant),
    the mass filter [1/6, 2/3, 1/6] maps it to 3s^2 + 2a^2, so R = alpha_r c a^2 with alpha_r = 3;
    k = min(a |c|, akabs |R| a / (eps + |Psi|), aksq R^2 a / (eps + |c| Psi^2)), akabs = 1/8,
    aksq = 1.  Across the field Psi = R = 0, so k = 0 there.  On this grid k_abs is the minimum near
    the low edge and k_square further out, so swapping the two constants, taking the other axis'
    spacing, or dropping |c| from the k_square denominator all change the result."""
    quad = qd.quadrature(2)
    mu, nu = quad["mu"][:, None], quad["nu"][:, None]
    N, dx, dy, eps = 12, 0.3, 0.2, 1e-3
    a, c = (dx, mu) if axis == "x" else (dy, nu)
    s = (np.arange(N) + 0.5) * a
    shape = (1, 1, 1, N) if axis == "x" else (1, 1, N, 1)
    psi = np.broadcast_to((s ** 3).reshape(shape), (1, 32, N, N)).copy()
    kx, ky = pg_diffusivity(psi, quad, dx, dy, 1, ZG)
    si = s[2:-2][None, :]
    P = 3 * si ** 2 + a ** 2
    R = 3.0 * c * a ** 2
    k_abs = (2.0 / 16.0) * np.abs(R) * a / (eps + P)
    k_sq = (2.0 / 2.0) * R ** 2 * a / (eps + np.abs(c) * P ** 2)
    ref = np.minimum(np.minimum(a * np.abs(c), k_abs), k_sq)
    assert (k_abs < k_sq).any() and (k_sq < k_abs).any()     # both bounds are active somewhere
    along, across = (kx, ky) if axis == "x" else (ky, kx)
    got = along[0, :, 2:-2, 2:-2] if axis == "x" else np.swapaxes(along[0, :, 2:-2, 2:-2], 1, 2)
    assert np.allclose(got, ref[:, None, :], rtol=1e-10, atol=1e-16)
    assert np.abs(across).max() < 1e-20      # rounding only: Psi and R vanish across the field


@pytest.mark.parametrize("na,ref", [(4, 0.978), (8, 0.994), (16, 0.9986)])
def test_p1_emission_scale(na, ref):
    """Linearly anisotropic emission on psi_n = mu_n (uniform in space): Phi_0 = Phi_2 = 0 and
    Phi_1 = sum p mu^2, so q_n = 3 sigma_s1 mu_n sum p mu^2 / (4 pi) and q_n / (sigma_s1 mu_n) =
    sum p mu^2 / (4 pi / 3).  For the octahedral patch sets that ratio is 0.978, 0.994 and 0.9986 at
    na = 4, 8, 16 (3 s.f.) and tends to the continuum value 1 (the integral of mu^2 over the sphere
    is 4 pi / 3); without the factor 3 it would be near 1/3."""
    quad = qd.quadrature(na)
    N, s1 = 3, 0.7
    nd = 8 * na * na
    psi = np.broadcast_to(quad["mu"][None, :, None, None], (1, nd, N, N)).copy()
    sigma_s = np.zeros((2, 1, 1, N, N))
    sigma_s[1] = s1
    q = emission(psi, quad, sigma_s, np.zeros((1, N, N)))
    sel = np.abs(quad["mu"]) > 0.05
    ratio = q[0, sel, 1, 1] / (s1 * quad["mu"][sel])
    assert np.allclose(ratio, ratio[0], rtol=1e-12)
    assert abs(ratio[0] - ref) < 1.5e-3
    assert 1.0 - 0.03 < ratio[0] < 1.0
