"""Octahedral patch quadrature (paper, section "Discrete Ordinates").

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The unit sphere is split into the 8 faces of an octahedron; an N_a x N_a grid with one collapsed
edge is placed on each face; every grid cell (patch) is projected radially onto the sphere and
gives one discrete ordinate.  Its weight p_n is the patch area, its direction the area-mean of
the unit vector over the patch; the weights are finally rescaled so that they sum to 4*pi.

Reading (the exact map lives in an external repository the paper points to, so it is unpinned
against the paper's own numbers): on the face with octant signs (sx, sy, sz) the point of the
flat face is

    P(s, t) = (1-s)(1-t) sx e1 + (1-s) t sy e2 + s sz e3,    (s, t) in [0,1]^2,

the edge s = 1 collapsing to the pole sz e3.  Patch (a, b) is
[a/N_a, (a+1)/N_a] x [b/N_a, (b+1)/N_a]: a runs towards the pole, b along the azimuth.  The area
element of the radial projection is |P . (P_s x P_t)| / |P|^3 ds dt.  In 2D the directions used
are (mu_n, nu_n) = the x and y parts of the mean direction, not renormalised.

Face index f: bit 0 set <=> sx < 0, bit 1 <=> sy < 0, bit 2 <=> sz < 0.
Direction index n = f * N_a^2 + a * N_a + b.
"""
import numpy as np

# tensor Gauss-Legendre points per patch side; the integrand is analytic on each patch
NQ_DEFAULT = 32


def face_signs(f):
    """Octant signs (sx, sy, sz) of face f (bit 0 -> x negative, bit 1 -> y, bit 2 -> z)."""
    return (-1.0 if f & 1 else 1.0, -1.0 if f & 2 else 1.0, -1.0 if f & 4 else 1.0)


def face_point(signs, s, t):
    """P(s, t) on the flat octahedron face, last axis = xyz."""
    sx, sy, sz = signs
    return np.stack([sx * (1 - s) * (1 - t), sy * (1 - s) * t, sz * s + 0 * t], axis=-1)


def _patch_integrals(signs, s0, s1, t0, t1, nq):
    """Area and area-weighted unit vector of one patch by tensor Gauss-Legendre quadrature."""
    x, w = np.polynomial.legendre.leggauss(nq)
    s = s0 + (s1 - s0) * (x + 1) / 2
    t = t0 + (t1 - t0) * (x + 1) / 2
    ws = w * (s1 - s0) / 2
    wt = w * (t1 - t0) / 2
    S, T = np.meshgrid(s, t, indexing="ij")
    W = np.outer(ws, wt)
    sx, sy, sz = signs
    P = face_point(signs, S, T)
    # partial derivatives of P with respect to s and t
    Ps = np.stack([-sx * (1 - T), -sy * T, sz + 0 * T], axis=-1)
    Pt = np.stack([-sx * (1 - S), sy * (1 - S), 0 * S], axis=-1)
    r = np.linalg.norm(P, axis=-1)
    jac = np.abs(np.einsum("...k,...k->...", P, np.cross(Ps, Pt))) / r**3
    area = np.sum(W * jac)
    first = np.einsum("ij,ijk->k", W * jac, P / r[..., None])
    return area, first


def raw_patches(na, nq=NQ_DEFAULT):
    """Un-normalised patch areas p[n] and area-weighted direction sums Ω*p [n, 3]."""
    nd = 8 * na * na
    area = np.zeros(nd)
    first = np.zeros((nd, 3))
    for f in range(8):
        sg = face_signs(f)
        for a in range(na):
            for b in range(na):
                n = f * na * na + a * na + b
                area[n], first[n] = _patch_integrals(sg, a / na, (a + 1) / na, b / na, (b + 1) / na, nq)
    return area, first


def quadrature(na, nq=NQ_DEFAULT):
    """Finest-level ordinates: returns dict(mu, nu, xi, p) with sum(p) = 4*pi.

    The mean direction of patch n is (integral of the unit vector) / (patch area); p is then
    rescaled to sum to 4*pi (the normalisation the paper applies to absorb quadrature error).
    """
    area, first = raw_patches(na, nq)
    omega = first / area[:, None]
    p = area * (4.0 * np.pi / area.sum())
    return {"mu": omega[:, 0].copy(), "nu": omega[:, 1].copy(), "xi": omega[:, 2].copy(), "p": p, "na": na}


def parent_index(n, na_fine):
    """Coarse ordinate of fine ordinate n: (f, a, b) -> (f, a//2, b//2); identity once N_a = 1."""
    if na_fine == 1:
        return n
    f, rem = divmod(n, na_fine * na_fine)
    a, b = divmod(rem, na_fine)
    nc = na_fine // 2
    return f * nc * nc + (a // 2) * nc + (b // 2)


def coarsen(q):
    """Coarse ordinates by adding patches: p_N = sum of children p, direction = p-weighted mean
    of the children's directions (section "Space-Angle Multigrid": directions/patches are added
    together to form the coarser discrete ordinate equations)."""
    na = q["na"]
    nc = max(na // 2, 1)
    ndc = 8 * nc * nc
    p = np.zeros(ndc)
    pm = np.zeros(ndc)
    pn = np.zeros(ndc)
    px = np.zeros(ndc)
    for n in range(8 * na * na):
        N = parent_index(n, na)
        p[N] += q["p"][n]
        pm[N] += q["p"][n] * q["mu"][n]
        pn[N] += q["p"][n] * q["nu"][n]
        px[N] += q["p"][n] * q["xi"][n]
    return {"mu": pm / p, "nu": pn / p, "xi": px / p, "p": p, "na": nc}
