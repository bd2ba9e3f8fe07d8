"""ConvFEM filters (paper, section "Neural Network Filters for the Convolutional Finite Element
Method", Appendix A) and the upwind filters (section "Neural network filters").

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

ConvFEM: the assembled finite-element equations of the different node types of a degree-p
Lagrange element (vertex node, p-1 interior nodes) have different stencils; averaging them gives
one stencil valid at every node.  In 1D this is done here in exact rational arithmetic:

* element matrices on nodes 0..p (unit spacing): M = int N_a N_b, C = int N_a N_b', K = int N_a' N_b'
* the assembled row of the vertex node = last row of the left element (offsets -p..0) plus the
  first row of the right element (offsets 0..p); interior node a: row a at offsets -a..p-a
* average the p rows, divide by the sum of the averaged mass row (lumped mass)

giving m (sum 1), d (first derivative, times 1/h) and k (minus the second derivative, times
1/h^2).  A 2D tensor-product element averages over all node-type pairs, so the 2D filters are
outer products:  w_x = m(y) (x) d(x) / dx,  w_y = d(y) (x) m(x) / dy,  w_Diffxx = m(y) (x) k(x) / dx^2,
w_Diffyy = k(y) (x) m(x) / dy^2,  w_m = m (x) m.

Orientation: every 2D filter here is an array w[v + l, u + l] indexed by the y-offset v (rows) and
x-offset u (columns) and applied as the cross-correlation f(Psi; w)[j, i] = sum w[v,u] Psi[j+v, i+u]
(the paper's conv sum, read with the offsets the printed formula leaves out).  The Appendix prints
the quadratic w_y with its first row at v = -l; the linear w_y and the upwind w_y are printed with
their first row at v = +l; the filters here are all defined by the operator they discretise
(+d/dy), see ``printed_orientation`` for the conversion used by the tests.
"""
from fractions import Fraction
import numpy as np


# ----------------------------------------------------------------------------------------------
# exact polynomial helpers (coefficient lists, lowest power first)
def _pmul(a, b):
    out = [Fraction(0)] * (len(a) + len(b) - 1)
    for i, x in enumerate(a):
        for j, y in enumerate(b):
            out[i + j] += x * y
    return out


def _pder(a):
    return [i * a[i] for i in range(1, len(a))] or [Fraction(0)]


def _pint(a, lo, hi):
    return sum(c * (Fraction(hi) ** (i + 1) - Fraction(lo) ** (i + 1)) / (i + 1) for i, c in enumerate(a))


def lagrange_basis(p):
    """Degree-p Lagrange basis on the equispaced nodes 0..p."""
    basis = []
    for a in range(p + 1):
        poly = [Fraction(1)]
        for b in range(p + 1):
            if b != a:
                poly = _pmul(poly, [Fraction(-b, a - b), Fraction(1, a - b)])
        basis.append(poly)
    return basis


def element_matrices(p):
    """Exact M, C, K of one degree-p element with unit node spacing (element length p)."""
    N = lagrange_basis(p)
    dN = [_pder(x) for x in N]
    M = [[_pint(_pmul(N[a], N[b]), 0, p) for b in range(p + 1)] for a in range(p + 1)]
    C = [[_pint(_pmul(N[a], dN[b]), 0, p) for b in range(p + 1)] for a in range(p + 1)]
    K = [[_pint(_pmul(dN[a], dN[b]), 0, p) for b in range(p + 1)] for a in range(p + 1)]
    return M, C, K


def _averaged_row(E, p):
    """Average over the p node types of the assembled row of element matrix E (offsets -p..p)."""
    avg = [Fraction(0)] * (2 * p + 1)
    for a in range(p):
        if a == 0:
            # vertex node: local node p of the left element and local node 0 of the right one
            for b in range(p + 1):
                avg[p + (b - p)] += E[p][b]
                avg[p + b] += E[0][b]
        else:
            for b in range(p + 1):
                avg[p + (b - a)] += E[a][b]
    return [x / p for x in avg]


def stencils_1d(p):
    """Exact 1D ConvFEM stencils (m, d, k) over offsets -p..p, as lists of Fractions."""
    M, C, K = element_matrices(p)
    mrow = _averaged_row(M, p)
    lump = sum(mrow)
    m = [x / lump for x in mrow]
    d = [x / lump for x in _averaged_row(C, p)]
    k = [x / lump for x in _averaged_row(K, p)]
    return m, d, k


def stencils_1d_float(p):
    m, d, k = stencils_1d(p)
    return (np.array([float(x) for x in m]), np.array([float(x) for x in d]),
            np.array([float(x) for x in k]))


def filters_2d(p, dx, dy):
    """The ConvFEM 2D filters of degree p, offset-indexed [v + p, u + p] (see module doc)."""
    m, d, k = stencils_1d_float(p)
    return {
        "wx": np.outer(m, d) / dx,
        "wy": np.outer(d, m) / dy,
        "wDxx": np.outer(m, k) / dx**2,
        "wDyy": np.outer(k, m) / dy**2,
        "wm": np.outer(m, m),
    }


def upwind_filters(mu, nu, dx, dy):
    """Upwind advection filters of the paper, as printed (first row = +y), for the signs of one
    face, converted to offset-indexed arrays [v + 1, u + 1]."""
    if mu > 0:
        wx_printed = np.array([[0, 0, 0], [-1 / dx, 1 / dx, 0], [0, 0, 0]])
    else:
        wx_printed = np.array([[0, 0, 0], [0, -1 / dx, 1 / dx], [0, 0, 0]])
    if nu > 0:
        wy_printed = np.array([[0, 0, 0], [0, 1 / dy, 0], [0, -1 / dy, 0]])
    else:
        wy_printed = np.array([[0, 1 / dy, 0], [0, -1 / dy, 0], [0, 0, 0]])
    return printed_orientation(wx_printed), printed_orientation(wy_printed)


def printed_orientation(w_printed_top_is_plus_y):
    """A filter printed with its first row at v = +l -> offset-indexed array (first row v = -l)."""
    return np.asarray(w_printed_top_is_plus_y, dtype=float)[::-1, :].copy()


def apply_filter(ext, w):
    """Cross-correlation of the last two axes of ``ext`` with the offset-indexed filter w.

    The output shrinks by l = (w.shape[0]-1)/2 on every side:
    out[..., j, i] = sum_{v,u} w[v+l, u+l] * ext[..., j+l+v, i+l+u].
    """
    l = (w.shape[0] - 1) // 2
    ny = ext.shape[-2] - 2 * l
    nx = ext.shape[-1] - 2 * l
    out = np.zeros(ext.shape[:-2] + (ny, nx))
    for v in range(-l, l + 1):
        for u in range(-l, l + 1):
            c = w[v + l, u + l]
            if c != 0.0:
                out += c * ext[..., l + v:l + v + ny, l + u:l + u + nx]
    return out
