// One-time host setup in float64: octahedral ordinates and ConvFEM stencils.
#include <cmath>
#include <vector>

#include "internal.h"

namespace ctf {

namespace {

// Gauss-Legendre nodes/weights on [-1, 1] by Newton iteration on the Legendre recurrence.
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < (n + 1) / 2; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double pk = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = pk;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-17) break;
    }
    {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double pk = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = pk;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
    }
    x[i] = -z;
    x[n - 1 - i] = z;
    w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

constexpr int kPatchGauss = 32;

// Area and area-weighted mean unit vector of the radial projection of one patch of the face with
// octant signs (sx, sy, sz): flat face point P(s,t) = (1-s)(1-t) sx e1 + (1-s) t sy e2 + s sz e3,
// solid-angle element |P . (P_s x P_t)| / |P|^3 ds dt.
void patch(double sx, double sy, double sz, double s0, double s1, double t0, double t1,
           const std::vector<double>& gx, const std::vector<double>& gw, double& area,
           double first[3]) {
  area = 0.0;
  first[0] = first[1] = first[2] = 0.0;
  const int n = static_cast<int>(gx.size());
  for (int a = 0; a < n; ++a) {
    const double s = s0 + (s1 - s0) * 0.5 * (gx[a] + 1.0);
    const double ws = gw[a] * 0.5 * (s1 - s0);
    for (int b = 0; b < n; ++b) {
      const double t = t0 + (t1 - t0) * 0.5 * (gx[b] + 1.0);
      const double wt = gw[b] * 0.5 * (t1 - t0);
      const double P[3] = {sx * (1 - s) * (1 - t), sy * (1 - s) * t, sz * s};
      const double Ps[3] = {-sx * (1 - t), -sy * t, sz};
      const double Pt[3] = {-sx * (1 - s), sy * (1 - s), 0.0};
      const double c[3] = {Ps[1] * Pt[2] - Ps[2] * Pt[1], Ps[2] * Pt[0] - Ps[0] * Pt[2],
                           Ps[0] * Pt[1] - Ps[1] * Pt[0]};
      const double r = std::sqrt(P[0] * P[0] + P[1] * P[1] + P[2] * P[2]);
      const double jac = std::fabs(P[0] * c[0] + P[1] * c[1] + P[2] * c[2]) / (r * r * r);
      const double wgt = ws * wt * jac;
      area += wgt;
      for (int k = 0; k < 3; ++k) first[k] += wgt * P[k] / r;
    }
  }
}

}  // namespace

Quadrature build_quadrature(int na, int faces) {
  std::vector<double> gx, gw;
  gauss_legendre(kPatchGauss, gx, gw);
  const int nd = faces * na * na;
  Quadrature q;
  q.na = na;
  q.faces = faces;
  q.mu.resize(nd);
  q.nu.resize(nd);
  q.xi.resize(nd);
  q.w.resize(nd);
  double total = 0.0;
  for (int f = 0; f < faces; ++f) {
    const double sx = (f & 1) ? -1.0 : 1.0, sy = (f & 2) ? -1.0 : 1.0, sz = (f & 4) ? -1.0 : 1.0;
    for (int a = 0; a < na; ++a)
      for (int b = 0; b < na; ++b) {
        const int n = f * na * na + a * na + b;
        double area, first[3];
        patch(sx, sy, sz, double(a) / na, double(a + 1) / na, double(b) / na, double(b + 1) / na,
              gx, gw, area, first);
        q.w[n] = area;
        q.mu[n] = first[0] / area;
        q.nu[n] = first[1] / area;
        q.xi[n] = first[2] / area;
        total += area;
      }
  }
  const double scale = 4.0 * M_PI / total;
  for (double& x : q.w) x *= scale;
  return q;
}

Quadrature coarsen_quadrature(const Quadrature& q) {
  const int na = q.na, nc = na > 1 ? na / 2 : 1, ndc = q.faces * nc * nc;
  Quadrature c;
  c.na = nc;
  c.faces = q.faces;
  c.w.assign(ndc, 0.0);
  c.mu.assign(ndc, 0.0);
  c.nu.assign(ndc, 0.0);
  c.xi.assign(ndc, 0.0);
  for (int n = 0; n < q.faces * na * na; ++n) {
    const int N = parent_dir(n, na);
    c.w[N] += q.w[n];
    c.mu[N] += q.w[n] * q.mu[n];
    c.nu[N] += q.w[n] * q.nu[n];
    c.xi[N] += q.w[n] * q.xi[n];
  }
  for (int N = 0; N < ndc; ++N) {
    c.mu[N] /= c.w[N];
    c.nu[N] /= c.w[N];
    c.xi[N] /= c.w[N];
  }
  return c;
}

// ConvFEM: average over the p node types of a degree-p Lagrange element (one vertex node, p-1
// interior nodes) of their assembled mass / advection / stiffness rows, normalised by the sum of
// the averaged mass row.  Element integrals by Gauss-Legendre (exact for these polynomials).
void convfem_stencils(int p, double* m, double* d, double* k) {
  std::vector<double> gx, gw;
  gauss_legendre(8, gx, gw);
  auto basis = [p](int a, double x) {
    double v = 1.0;
    for (int b = 0; b <= p; ++b)
      if (b != a) v *= (x - b) / double(a - b);
    return v;
  };
  auto dbasis = [p](int a, double x) {
    double s = 0.0;
    for (int c = 0; c <= p; ++c) {
      if (c == a) continue;
      double v = 1.0 / double(a - c);
      for (int b = 0; b <= p; ++b)
        if (b != a && b != c) v *= (x - b) / double(a - b);
      s += v;
    }
    return s;
  };
  double M[kMaxP + 1][kMaxP + 1] = {}, C[kMaxP + 1][kMaxP + 1] = {}, K[kMaxP + 1][kMaxP + 1] = {};
  for (int q = 0; q < static_cast<int>(gx.size()); ++q) {
    const double x = 0.5 * p * (gx[q] + 1.0), wq = 0.5 * p * gw[q];
    for (int a = 0; a <= p; ++a)
      for (int b = 0; b <= p; ++b) {
        M[a][b] += wq * basis(a, x) * basis(b, x);
        C[a][b] += wq * basis(a, x) * dbasis(b, x);
        K[a][b] += wq * dbasis(a, x) * dbasis(b, x);
      }
  }
  const int W = 2 * p + 1;
  double am[2 * kMaxP + 1] = {}, ad[2 * kMaxP + 1] = {}, ak[2 * kMaxP + 1] = {};
  for (int a = 0; a < p; ++a) {
    for (int b = 0; b <= p; ++b) {
      if (a == 0) {  // vertex: local node p of the left element + local node 0 of the right one
        am[p + b - p] += M[p][b];
        ad[p + b - p] += C[p][b];
        ak[p + b - p] += K[p][b];
        am[p + b] += M[0][b];
        ad[p + b] += C[0][b];
        ak[p + b] += K[0][b];
      } else {
        am[p + b - a] += M[a][b];
        ad[p + b - a] += C[a][b];
        ak[p + b - a] += K[a][b];
      }
    }
  }
  double lump = 0.0;
  for (int i = 0; i < W; ++i) lump += am[i];
  for (int i = 0; i < W; ++i) {
    m[i] = am[i] / lump;
    d[i] = ad[i] / lump;
    k[i] = ak[i] / lump;
  }
}

}  // namespace ctf
