"""Pins of the oracle's octahedral patch quadrature (section "Discrete Ordinates"), CPU only.

Each patch is the radial projection of a flat quadrilateral (a triangle on the collapsed edge)
of the octahedron face, so it is a spherical polygon with great-circle edges.  Its area has the
closed form of Van Oosterom & Strackee (solid angle of a spherical triangle), and its first
moment  int r dS = 1/2 sum_edges theta_e n_e  (theta_e the arc angle, n_e the unit normal of the
edge's great-circle plane, edges counter-clockwise seen from outside).  Both are exact, so they
pin the Jacobian and the direction averaging of the Gauss-Legendre patch integrals.
"""
import numpy as np
import pytest

from oracle import quadrature as qd


def _unit(v):
    return v / np.linalg.norm(v)


def _tri_solid_angle(a, b, c):
    num = abs(np.dot(a, np.cross(b, c)))
    den = 1.0 + np.dot(a, b) + np.dot(b, c) + np.dot(c, a)
    return 2.0 * np.arctan2(num, den)


def _polygon_exact(verts):
    """Area and first moment of a convex spherical polygon with great-circle edges."""
    # orient counter-clockwise seen from outside
    c = _unit(sum(verts))
    if np.dot(np.cross(verts[1] - verts[0], verts[2] - verts[0]), c) < 0:
        verts = verts[::-1]
    area = sum(_tri_solid_angle(verts[0], verts[i], verts[i + 1]) for i in range(1, len(verts) - 1))
    first = np.zeros(3)
    for i in range(len(verts)):
        a, b = verts[i], verts[(i + 1) % len(verts)]
        theta = np.arccos(np.clip(np.dot(a, b), -1, 1))
        first += 0.5 * theta * _unit(np.cross(a, b))
    return area, first


def _vertices(signs, a, b, na):
    s0, s1, t0, t1 = a / na, (a + 1) / na, b / na, (b + 1) / na
    pts = [qd.face_point(signs, np.array(s), np.array(t)) for s, t in
           [(s0, t0), (s1, t0), (s1, t1), (s0, t1)]]
    pts = [_unit(np.asarray(p, dtype=float)) for p in pts]
    if a == na - 1:          # collapsed edge: the two vertices at s = 1 coincide (the pole)
        pts = [pts[0], pts[1], pts[3]]
    return pts


@pytest.mark.parametrize("na", [1, 2, 4])
def test_patch_integrals_match_spherical_polygon_closed_forms(na):
    area, first = qd.raw_patches(na)
    for f in range(8):
        sg = qd.face_signs(f)
        for a in range(na):
            for b in range(na):
                n = f * na * na + a * na + b
                A, F = _polygon_exact(_vertices(sg, a, b, na))
                assert abs(area[n] - A) <= 1e-12 * A
                assert np.allclose(first[n], F, rtol=0, atol=1e-12)


@pytest.mark.parametrize("na", [1, 2, 4, 8])
def test_quadrature_invariants(na):
    q = qd.quadrature(na)
    raw, _ = qd.raw_patches(na)
    assert abs(raw.sum() - 4 * np.pi) < 1e-11           # octants tile the sphere
    assert abs(q["p"].sum() - 4 * np.pi) < 1e-12
    assert abs(np.dot(q["p"], q["mu"])) < 1e-13 and abs(np.dot(q["p"], q["nu"])) < 1e-13
    nf = na * na
    for f in range(8):
        sx, sy, sz = qd.face_signs(f)
        sl = slice(f * nf, (f + 1) * nf)
        assert np.all(np.sign(q["mu"][sl]) == sx) and np.all(np.sign(q["nu"][sl]) == sy)
        assert np.all(np.sign(q["xi"][sl]) == sz)
        # an octant's area is pi/2 and int x dS over it is pi/4 (exact)
        assert abs(raw[sl].sum() - np.pi / 2) < 1e-12
    # mean directions lie inside the unit ball
    r = np.sqrt(q["mu"] ** 2 + q["nu"] ** 2 + q["xi"] ** 2)
    assert np.all(r < 1.0) and np.all(r > 0.86)


def test_single_patch_per_face_is_the_octant_mean():
    # N_a = 1: the mean unit vector over an octant is (pi/4)(sx, sy, sz) / (pi/2)
    q = qd.quadrature(1)
    for f in range(8):
        assert np.allclose([q["mu"][f], q["nu"][f], q["xi"][f]], 0.5 * np.array(qd.face_signs(f)),
                           atol=1e-14)
        assert abs(q["p"][f] - np.pi / 2) < 1e-13


def test_second_moment_approaches_sphere_value():
    # sum p mu^2 -> int mu^2 dS = 4 pi / 3 as the patches shrink
    errs = []
    for na in (2, 4, 8, 16):
        q = qd.quadrature(na)
        errs.append(abs(np.dot(q["p"], q["mu"] ** 2) - 4 * np.pi / 3))
    assert all(e2 < e1 for e1, e2 in zip(errs, errs[1:]))
    assert errs[-1] < 0.01 * 4 * np.pi / 3


@pytest.mark.parametrize("na", [2, 4, 8])
def test_coarsening_adds_children(na):
    q = qd.quadrature(na)
    c = qd.coarsen(q)
    assert c["na"] == na // 2
    assert abs(c["p"].sum() - 4 * np.pi) < 1e-12
    # a coarse patch is the union of its 2x2 children: its exact raw integrals add up too
    raw, first = qd.raw_patches(na)
    rawc, firstc = qd.raw_patches(na // 2)
    for N in range(len(c["p"])):
        kids = [n for n in range(len(q["p"])) if qd.parent_index(n, na) == N]
        assert len(kids) == 4
        assert abs(raw[kids].sum() - rawc[N]) < 1e-13
        assert np.allclose(first[kids].sum(axis=0), firstc[N], atol=1e-13)
    c1 = qd.coarsen(qd.quadrature(1))
    assert np.allclose(c1["p"], qd.quadrature(1)["p"]) and np.allclose(c1["mu"], qd.quadrature(1)["mu"])
