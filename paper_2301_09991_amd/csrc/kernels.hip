// HIP kernels (gfx950, wave64) of the ConvFEM space-angle multigrid transport solver.
//
// Layout of every angular-flux-shaped array: [G][n_dir][n][n], x fastest; 64-bit offsets.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace ctf {

namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

template <typename T>
__device__ __forceinline__ T tabs(T x) { return x < T(0) ? -x : x; }

template <typename T>
__device__ __forceinline__ T tmin(T a, T b) { return b < a ? b : a; }

__device__ __forceinline__ int parent_dir_dev(int n, int na) {
  if (na == 1) return n;
  const int na2 = na * na;
  const int f = n / na2, r = n - f * na2;
  const int a = r / na, b = r - a * na, nc = na >> 1;
  return f * nc * nc + (a >> 1) * nc + (b >> 1);
}

// Is the halo position (gi, gj) outside the domain on a side through which ordinate (mu, nu)
// enters, with a vacuum condition there?  Such halo values are zero; all other halo values copy
// the nearest interior node (section "Discretisation in Cartesian space").
template <typename T>
__device__ __forceinline__ bool halo_zero(int gi, int gj, int n, T mu, T nu, int bc_vac) {
  return (gi < 0 && (bc_vac & 1) && mu > T(0)) || (gi >= n && (bc_vac & 2) && mu < T(0)) ||
         (gj < 0 && (bc_vac & 4) && nu > T(0)) || (gj >= n && (bc_vac & 8) && nu < T(0));
}

// ---------------------------------------------------------------------------------------------
// moments: phi[g][m][cell] = sum_n w_n Y_m(n) psi[g][n][cell], Y = (1, mu, nu)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_moments(LevelData<T> L, const T* __restrict__ psi,
                                                     T* __restrict__ phi, int nmom) {
  const size_t ncell = size_t(L.dims.n) * L.dims.n;
  const size_t t = size_t(blockIdx.x) * kBlock + threadIdx.x;
  const int g = blockIdx.y;
  if (t >= ncell) return;
  const T* src = psi + size_t(g) * L.dims.nd * ncell + t;
  T a0 = 0, a1 = 0, a2 = 0;
  for (int d = 0; d < L.dims.nd; ++d) {
    const T v = src[size_t(d) * ncell];
    const T w = L.w[d];
    a0 += w * v;
    if (nmom > 1) {
      a1 += (w * L.mu[d]) * v;
      a2 += (w * L.nu[d]) * v;
    }
  }
  T* dst = phi + size_t(g) * nmom * ncell + t;
  dst[0] = a0;
  if (nmom > 1) {
    dst[ncell] = a1;
    dst[2 * ncell] = a2;
  }
}

// emission E[g][m][cell]: q_n = E0 + mu_n E1 + nu_n E2, all divided by 4 pi
template <typename T>
__global__ __launch_bounds__(kBlock) void k_emission(LevelDims d, const T* __restrict__ phi,
                                                      const T* __restrict__ ss, int nl,
                                                      const T* __restrict__ src, T* __restrict__ E) {
  const size_t ncell = size_t(d.n) * d.n;
  const size_t t = size_t(blockIdx.x) * kBlock + threadIdx.x;
  const int g = blockIdx.y, G = d.G;
  if (t >= ncell) return;
  const int nmom = nl > 1 ? 3 : 1;
  T e0 = src ? src[size_t(g) * ncell + t] : T(0), e1 = 0, e2 = 0;
  for (int gp = 0; gp < G; ++gp) {
    const T s0 = ss[(size_t(g) * G + gp) * ncell + t];
    e0 += s0 * phi[(size_t(gp) * nmom) * ncell + t];
    if (nl > 1) {
      const T s1 = ss[((size_t(G) + g) * G + gp) * ncell + t];
      e1 += s1 * phi[(size_t(gp) * nmom + 1) * ncell + t];
      e2 += s1 * phi[(size_t(gp) * nmom + 2) * ncell + t];
    }
  }
  const T inv4pi = T(0.07957747154594767);  // 1 / (4 pi)
  T* dst = E + size_t(g) * nmom * ncell + t;
  dst[0] = e0 * inv4pi;
  if (nl > 1) {
    dst[ncell] = T(3) * e1 * inv4pi;
    dst[2 * ncell] = T(3) * e2 * inv4pi;
  }
}

// ---------------------------------------------------------------------------------------------
// ConvFEM Petrov-Galerkin residual (eq. Petrov) of one 16 x 16 tile, one ordinate, one group.
//   psi is staged with a 3P halo (halo rule above); Psi_x = f(psi; m (x) d), Psi_y = f(psi; d (x) m)
//   on the tile + 2P ring; the anisotropic diffusivities (eq. ano-k) on the tile + P ring at the
//   clamped position (the k halo copies the nearest interior value); then
//   rho = q - mu Psi_x - nu Psi_y - kDiff_x - kDiff_y - sigma_t psi  with
//   kDiff(psi; k, w) = sum_o w_o (k_c + k_o)(psi_o - psi_c)  (= f(k psi; w) + k f(psi; w) - psi f(k; w)
//   since every w_Diff sums to zero).
constexpr int kTile = 16;

template <typename T>
struct PGArgs {
  LevelData<T> L;
  Stencils<T> st;
  T alpha_r, eps_k, akabs, aksq, beta;
  int bc_vac;
  const T* psi;
  const T* E;
  int nmomE;
  const T* kx_in;
  const T* ky_in;
  T* out;
  T* kx_out;
  T* ky_out;
  const T* rhs;
  int mode;
  T sign;
  int ntx;
};

template <int P, typename T>
__global__ __launch_bounds__(kBlock) void k_pg(PGArgs<T> a) {
  constexpr int EXT = kTile + 6 * P;
  constexpr int GR = kTile + 4 * P;
  constexpr int KR = kTile + 2 * P;
  __shared__ T sp[EXT * EXT];
  __shared__ T sgx[GR * GR];
  __shared__ T sgy[GR * GR];
  __shared__ T skx[KR * KR];
  __shared__ T sky[KR * KR];

  const int n = a.L.dims.n;
  const int dir = blockIdx.y, g = blockIdx.z;
  const int tid = threadIdx.x;
  const int i0 = (blockIdx.x % a.ntx) * kTile, j0 = (blockIdx.x / a.ntx) * kTile;
  const size_t ncell = size_t(n) * n;
  const size_t base = (size_t(g) * a.L.dims.nd + dir) * ncell;
  const T mu = a.L.mu[dir], nu = a.L.nu[dir];
  const T h = T(a.L.dims.h);
  const T* __restrict__ psi = a.psi + base;

  for (int idx = tid; idx < EXT * EXT; idx += kBlock) {
    const int ly = idx / EXT, lx = idx - ly * EXT;
    const int gi = i0 - 3 * P + lx, gj = j0 - 3 * P + ly;
    T v = T(0);
    if (!halo_zero(gi, gj, n, mu, nu, a.bc_vac))
      v = psi[size_t(clampi(gj, 0, n - 1)) * n + clampi(gi, 0, n - 1)];
    sp[idx] = v;
  }
  __syncthreads();

  for (int idx = tid; idx < GR * GR; idx += kBlock) {
    const int ly = idx / GR, lx = idx - ly * GR;
    T gx = 0, gy = 0;
#pragma unroll
    for (int v = -P; v <= P; ++v) {
      const T* row = sp + (ly + P + v) * EXT + lx + P;
#pragma unroll
      for (int u = -P; u <= P; ++u) {
        const T val = row[u];
        gx += a.st.m[v + P] * a.st.d[u + P] * val;
        gy += a.st.d[v + P] * a.st.m[u + P] * val;
      }
    }
    sgx[idx] = gx;
    sgy[idx] = gy;
  }
  __syncthreads();

  for (int idx = tid; idx < KR * KR; idx += kBlock) {
    const int ly = idx / KR, lx = idx - ly * KR;
    const int ci = clampi(i0 - P + lx, 0, n - 1), cj = clampi(j0 - P + ly, 0, n - 1);
    T kx, ky;
    if (a.kx_in) {
      kx = a.kx_in[base + size_t(cj) * n + ci];
      ky = a.ky_in[base + size_t(cj) * n + ci];
    } else {
      const int cx = ci - i0 + 2 * P, cy = cj - j0 + 2 * P;
      T mx = 0, my = 0;
#pragma unroll
      for (int v = -P; v <= P; ++v)
#pragma unroll
        for (int u = -P; u <= P; ++u) {
          const T mm = a.st.m[v + P] * a.st.m[u + P];
          mx += mm * sgx[(cy + v) * GR + cx + u];
          my += mm * sgy[(cy + v) * GR + cx + u];
        }
      const T px = sgx[cy * GR + cx], py = sgy[cy * GR + cx];
      const T rx = a.alpha_r * mu * (mx - px);
      const T ry = a.alpha_r * nu * (my - py);
      const T kxabs = a.akabs * tabs(rx) * h / (a.eps_k + tabs(px));
      const T kyabs = a.akabs * tabs(ry) * h / (a.eps_k + tabs(py));
      const T kxsq = a.aksq * rx * rx * h / (a.eps_k + tabs(mu) * px * px);
      const T kysq = a.aksq * ry * ry * h / (a.eps_k + tabs(nu) * py * py);
      kx = tmin(tmin(h * tabs(mu), kxabs), kxsq);
      ky = tmin(tmin(h * tabs(nu), kyabs), kysq);
    }
    skx[idx] = kx;
    sky[idx] = ky;
  }
  __syncthreads();

  {
    const int ly = tid / kTile, lx = tid - ly * kTile;
    const int gi = i0 + lx, gj = j0 + ly;
    if (gi < n && gj < n) {
      const T pc = sp[(ly + 3 * P) * EXT + lx + 3 * P];
      const T kxc = skx[(ly + P) * KR + lx + P], kyc = sky[(ly + P) * KR + lx + P];
      T dx = 0, dy = 0;
#pragma unroll
      for (int v = -P; v <= P; ++v)
#pragma unroll
        for (int u = -P; u <= P; ++u) {
          const T dp = sp[(ly + 3 * P + v) * EXT + lx + 3 * P + u] - pc;
          const int kk = (ly + P + v) * KR + lx + P + u;
          dx += a.st.m[v + P] * a.st.k[u + P] * (kxc + skx[kk]) * dp;
          dy += a.st.k[v + P] * a.st.m[u + P] * (kyc + sky[kk]) * dp;
        }
      const size_t cell = size_t(gj) * n + gi;
      const size_t eb = size_t(g) * a.nmomE * ncell + cell;
      T q = a.E[eb];
      if (a.nmomE > 1) q += mu * a.E[eb + ncell] + nu * a.E[eb + 2 * ncell];
      if (a.rhs) q += a.rhs[base + cell];
      const T sig = a.L.sigma_t[size_t(g) * ncell + cell];
      const T px = sgx[(ly + 2 * P) * GR + lx + 2 * P], py = sgy[(ly + 2 * P) * GR + lx + 2 * P];
      const T rho = q - mu * px - nu * py - dx - dy - sig * pc;
      if (a.mode == 0) {
        a.out[base + cell] = a.sign * rho;
        if (a.kx_out) {
          a.kx_out[base + cell] = kxc;
          a.ky_out[base + cell] = kyc;
        }
      } else {
        const T diag = a.beta * (tabs(mu) / h + tabs(nu) / h + sig);
        a.out[base + cell] = pc + rho / diag;
      }
    }
  }
}

// ---------------------------------------------------------------------------------------------
// finest upwind operator (eq. discretised_hfm): rho = q - A_up psi - sigma_t psi
template <typename T>
__global__ __launch_bounds__(kBlock) void k_upwind_full(LevelData<T> L, int bc_vac,
                                                         const T* __restrict__ psi,
                                                         const T* __restrict__ E, int nmomE,
                                                         T* __restrict__ out, int mode, T sign,
                                                         const T* __restrict__ rhs) {
  const int n = L.dims.n, nd = L.dims.nd;
  const size_t ncell = size_t(n) * n;
  const size_t total = ncell * nd * L.dims.G;
  const size_t idx = size_t(blockIdx.x) * kBlock + threadIdx.x;
  if (idx >= total) return;
  const size_t gn = idx / ncell, cell = idx - gn * ncell;
  const int g = int(gn / nd), dir = int(gn - size_t(g) * nd);
  const int j = int(cell / n), i = int(cell - size_t(j) * n);
  const T mu = L.mu[dir], nu = L.nu[dir], h = T(L.dims.h);
  const T pc = psi[idx];
  T px, py;
  if (mu > T(0)) px = i > 0 ? psi[idx - 1] : ((bc_vac & 1) ? T(0) : pc);
  else px = i < n - 1 ? psi[idx + 1] : ((bc_vac & 2) ? T(0) : pc);
  if (nu > T(0)) py = j > 0 ? psi[idx - n] : ((bc_vac & 4) ? T(0) : pc);
  else py = j < n - 1 ? psi[idx + n] : ((bc_vac & 8) ? T(0) : pc);
  const T amu = tabs(mu) / h, anu = tabs(nu) / h;
  const size_t eb = size_t(g) * nmomE * ncell + cell;
  T q = E[eb];
  if (nmomE > 1) q += mu * E[eb + ncell] + nu * E[eb + 2 * ncell];
  if (rhs) q += rhs[idx];
  const T sig = L.sigma_t[size_t(g) * ncell + cell];
  const T rho = q - amu * (pc - px) - anu * (pc - py) - sig * pc;
  if (mode == 0) out[idx] = sign * rho;
  else out[idx] = pc + rho / (amu + anu + sig);
}

// correction sweep on one level: e_new = e + (rhs - A_up e - sigma_t e) / d
template <typename T, int XMODE>
__global__ __launch_bounds__(kBlock) void k_upwind_corr(LevelData<T> L, int bc_vac,
                                                         const T* __restrict__ xin, int nac,
                                                         const T* __restrict__ rhs,
                                                         T* __restrict__ xout, T* __restrict__ acc) {
  const int n = L.dims.n, nd = L.dims.nd;
  const size_t ncell = size_t(n) * n;
  const size_t total = ncell * nd * L.dims.G;
  const size_t idx = size_t(blockIdx.x) * kBlock + threadIdx.x;
  if (idx >= total) return;
  const size_t gn = idx / ncell, cell = idx - gn * ncell;
  const int g = int(gn / nd), dir = int(gn - size_t(g) * nd);
  const int j = int(cell / n), i = int(cell - size_t(j) * n);
  const T mu = L.mu[dir], nu = L.nu[dir], h = T(L.dims.h);
  const int iu = mu > T(0) ? i - 1 : i + 1;
  const int ju = nu > T(0) ? j - 1 : j + 1;
  const bool xin_dom = iu >= 0 && iu < n, yin_dom = ju >= 0 && ju < n;
  const bool xvac = mu > T(0) ? (bc_vac & 1) : (bc_vac & 2);
  const bool yvac = nu > T(0) ? (bc_vac & 4) : (bc_vac & 8);
  T ec = 0, ex = 0, ey = 0;
  if (XMODE == 0) {
    ec = xin[idx];
    ex = xin_dom ? xin[idx + (iu - i)] : (xvac ? T(0) : ec);
    ey = yin_dom ? xin[idx + ptrdiff_t(ju - j) * n] : (yvac ? T(0) : ec);
  } else if (XMODE == 1) {
    const int nc = n >> 1;
    const T* src = xin + (size_t(g) * (size_t(8) * (nac * nac)) + parent_dir_dev(dir, L.dims.na)) *
                             (size_t(nc) * nc);
    ec = src[size_t(j >> 1) * nc + (i >> 1)];
    ex = xin_dom ? src[size_t(j >> 1) * nc + (iu >> 1)] : (xvac ? T(0) : ec);
    ey = yin_dom ? src[size_t(ju >> 1) * nc + (i >> 1)] : (yvac ? T(0) : ec);
  }
  const T amu = tabs(mu) / h, anu = tabs(nu) / h;
  const T sig = L.sigma_t[size_t(g) * ncell + cell];
  const T r = rhs[idx] - amu * (ec - ex) - anu * (ec - ey) - sig * ec;
  const T enew = ec + r / (amu + anu + sig);
  if (acc) acc[idx] += enew;
  else xout[idx] = enew;
}

// restriction: coarse = sum_{child ordinates, 2x2 cells} w_n rho h^2 / (w_N H^2)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_restrict(LevelData<T> Lf, LevelData<T> Lc,
                                                      const T* __restrict__ fine,
                                                      T* __restrict__ coarse) {
  const int nc = Lc.dims.n, ndc = Lc.dims.nd, nf = Lf.dims.n, naf = Lf.dims.na;
  const size_t nccell = size_t(nc) * nc, nfcell = size_t(nf) * nf;
  const size_t total = nccell * ndc * Lc.dims.G;
  const size_t idx = size_t(blockIdx.x) * kBlock + threadIdx.x;
  if (idx >= total) return;
  const size_t gn = idx / nccell, cell = idx - gn * nccell;
  const int g = int(gn / ndc), N = int(gn - size_t(g) * ndc);
  const int J = int(cell / nc), I = int(cell - size_t(J) * nc);
  int kids[4], nk = 0;
  if (naf == 1) {
    kids[nk++] = N;
  } else {
    const int ncs = naf >> 1, ncs2 = ncs * ncs;
    const int f = N / ncs2, r = N - f * ncs2, A = r / ncs, B = r - A * ncs;
    for (int da = 0; da < 2; ++da)
      for (int db = 0; db < 2; ++db) kids[nk++] = f * naf * naf + (2 * A + da) * naf + 2 * B + db;
  }
  T s = 0;
  for (int c = 0; c < nk; ++c) {
    const T* src = fine + (size_t(g) * Lf.dims.nd + kids[c]) * nfcell + size_t(2 * J) * nf + 2 * I;
    s += Lf.w[kids[c]] * ((src[0] + src[nf]) + (src[1] + src[nf + 1]));
  }
  const T hf = T(Lf.dims.h), hc = T(Lc.dims.h);
  coarse[idx] = s * (hf * hf) / (Lc.w[N] * (hc * hc));
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_prolong(LevelData<T> Lf, int nac,
                                                     const T* __restrict__ coarse,
                                                     T* __restrict__ fine) {
  const int n = Lf.dims.n, nd = Lf.dims.nd;
  const size_t ncell = size_t(n) * n;
  const size_t total = ncell * nd * Lf.dims.G;
  const size_t idx = size_t(blockIdx.x) * kBlock + threadIdx.x;
  if (idx >= total) return;
  const size_t gn = idx / ncell, cell = idx - gn * ncell;
  const int g = int(gn / nd), dir = int(gn - size_t(g) * nd);
  const int j = int(cell / n), i = int(cell - size_t(j) * n);
  const int nc = n >> 1;
  fine[idx] = coarse[(size_t(g) * (size_t(8) * nac * nac) + parent_dir_dev(dir, Lf.dims.na)) *
                         (size_t(nc) * nc) + size_t(j >> 1) * nc + (i >> 1)];
}

// weighted squared norm, two deterministic passes
constexpr int kNormBlocks = 1024;

template <typename T>
__global__ __launch_bounds__(kBlock) void k_wnorm2_partial(LevelData<T> L, const T* __restrict__ v,
                                                            double* __restrict__ partial) {
  const size_t ncell = size_t(L.dims.n) * L.dims.n;
  const size_t total = ncell * L.dims.nd * L.dims.G;
  double acc = 0.0;
  for (size_t idx = size_t(blockIdx.x) * kBlock + threadIdx.x; idx < total;
       idx += size_t(gridDim.x) * kBlock) {
    const int dir = int((idx / ncell) % L.dims.nd);
    const double x = double(v[idx]);
    acc += double(L.w[dir]) * x * x;
  }
  __shared__ double red[kBlock];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0] * L.dims.h * L.dims.h;
}

__global__ __launch_bounds__(kBlock) void k_sum_partials(const double* __restrict__ partial, int np,
                                                          double* __restrict__ out) {
  __shared__ double red[kBlock];
  double acc = 0.0;
  for (int i = threadIdx.x; i < np; i += kBlock) acc += partial[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_axpy(T* __restrict__ y, const T* __restrict__ x, T a,
                                                  size_t n) {
  const size_t i = size_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i < n) y[i] += a * x[i];
}

__global__ __launch_bounds__(kBlock) void k_harmonic(const double* __restrict__ f,
                                                      double* __restrict__ c, int G, int nc) {
  const size_t ncc = size_t(nc) * nc;
  const size_t idx = size_t(blockIdx.x) * kBlock + threadIdx.x;
  if (idx >= ncc * G) return;
  const size_t g = idx / ncc, cell = idx - g * ncc;
  const int J = int(cell / nc), I = int(cell - size_t(J) * nc), nf = 2 * nc;
  const double* s = f + g * size_t(nf) * nf + size_t(2 * J) * nf + 2 * I;
  const double a = s[0], b = s[nf], cc = s[1], d = s[nf + 1];
  c[idx] = (a == 0.0 || b == 0.0 || cc == 0.0 || d == 0.0)
               ? 0.0
               : 4.0 / (1.0 / a + 1.0 / b + 1.0 / cc + 1.0 / d);
}

__global__ __launch_bounds__(kBlock) void k_d2f(const double* __restrict__ in, float* __restrict__ out,
                                                 size_t n) {
  const size_t i = size_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i < n) out[i] = float(in[i]);
}
__global__ __launch_bounds__(kBlock) void k_f2d(const float* __restrict__ in, double* __restrict__ out,
                                                 size_t n) {
  const size_t i = size_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i < n) out[i] = double(in[i]);
}
__global__ __launch_bounds__(kBlock) void k_add_f2d(double* __restrict__ y, const float* __restrict__ x,
                                                     size_t n) {
  const size_t i = size_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i < n) y[i] += double(x[i]);
}

inline unsigned nblocks(size_t total) { return unsigned((total + kBlock - 1) / kBlock); }

}  // namespace

// ---------------------------------------------------------------------------------------------
template <typename T>
hipError_t launch_moments(const LevelData<T>& L, const T* psi, T* phi, int nmom, hipStream_t s) {
  const size_t ncell = size_t(L.dims.n) * L.dims.n;
  hipLaunchKernelGGL(k_moments<T>, dim3(nblocks(ncell), L.dims.G), dim3(kBlock), 0, s, L, psi, phi,
                     nmom);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_emission(const LevelDims& d, const T* phi, const T* ss, int nl, const T* src,
                           T* E, hipStream_t s) {
  const size_t ncell = size_t(d.n) * d.n;
  hipLaunchKernelGGL(k_emission<T>, dim3(nblocks(ncell), d.G), dim3(kBlock), 0, s, d, phi, ss, nl,
                     src, E);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_pg(int p, const LevelData<T>& L, const Stencils<T>& st, const PGParams& pp,
                     const T* psi, const T* E, int nmomE, const T* kx, const T* ky, T* out,
                     T* kx_out, T* ky_out, int mode, T sign, const T* rhs, hipStream_t s) {
  PGArgs<T> a;
  a.rhs = rhs;
  a.L = L;
  a.st = st;
  a.alpha_r = T(pp.alpha_r);
  a.eps_k = T(pp.eps_k);
  a.akabs = T(pp.alpha_kabs);
  a.aksq = T(pp.alpha_ksq);
  a.beta = T(pp.beta);
  a.bc_vac = pp.bc_vac;
  a.psi = psi;
  a.E = E;
  a.nmomE = nmomE;
  a.kx_in = kx;
  a.ky_in = ky;
  a.out = out;
  a.kx_out = kx_out;
  a.ky_out = ky_out;
  a.mode = mode;
  a.sign = sign;
  const int nt = (L.dims.n + kTile - 1) / kTile;
  a.ntx = nt;
  dim3 grid(nt * nt, L.dims.nd, L.dims.G);
  switch (p) {
    case 1: hipLaunchKernelGGL((k_pg<1, T>), grid, dim3(kBlock), 0, s, a); break;
    case 2: hipLaunchKernelGGL((k_pg<2, T>), grid, dim3(kBlock), 0, s, a); break;
    case 3: hipLaunchKernelGGL((k_pg<3, T>), grid, dim3(kBlock), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_upwind_full(const LevelData<T>& L, int bc_vac, const T* psi, const T* E, int nmomE,
                              T* out, int mode, T sign, const T* rhs, hipStream_t s) {
  const size_t total = size_t(L.dims.n) * L.dims.n * L.dims.nd * L.dims.G;
  hipLaunchKernelGGL(k_upwind_full<T>, dim3(nblocks(total)), dim3(kBlock), 0, s, L, bc_vac, psi, E,
                     nmomE, out, mode, sign, rhs);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_upwind_correction(const LevelData<T>& L, int bc_vac, const T* x_in, int xmode,
                                    int nac, const T* rhs, T* x_out, T* psi_acc, hipStream_t s) {
  const size_t total = size_t(L.dims.n) * L.dims.n * L.dims.nd * L.dims.G;
  const dim3 grid(nblocks(total)), blk(kBlock);
  if (xmode == 0)
    hipLaunchKernelGGL((k_upwind_corr<T, 0>), grid, blk, 0, s, L, bc_vac, x_in, nac, rhs, x_out, psi_acc);
  else if (xmode == 1)
    hipLaunchKernelGGL((k_upwind_corr<T, 1>), grid, blk, 0, s, L, bc_vac, x_in, nac, rhs, x_out, psi_acc);
  else
    hipLaunchKernelGGL((k_upwind_corr<T, 2>), grid, blk, 0, s, L, bc_vac, x_in, nac, rhs, x_out, psi_acc);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_restrict(const LevelData<T>& Lf, const LevelData<T>& Lc, const T* fine, T* coarse,
                           hipStream_t s) {
  const size_t total = size_t(Lc.dims.n) * Lc.dims.n * Lc.dims.nd * Lc.dims.G;
  hipLaunchKernelGGL(k_restrict<T>, dim3(nblocks(total)), dim3(kBlock), 0, s, Lf, Lc, fine, coarse);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_prolong(const LevelData<T>& Lf, int nac, const T* coarse, T* fine, hipStream_t s) {
  const size_t total = size_t(Lf.dims.n) * Lf.dims.n * Lf.dims.nd * Lf.dims.G;
  hipLaunchKernelGGL(k_prolong<T>, dim3(nblocks(total)), dim3(kBlock), 0, s, Lf, nac, coarse, fine);
  return hipGetLastError();
}

int wnorm2_partials(const LevelDims&) { return kNormBlocks; }

template <typename T>
hipError_t launch_wnorm2(const LevelData<T>& L, const T* v, double* partial, int npartial,
                         double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_wnorm2_partial<T>, dim3(npartial), dim3(kBlock), 0, s, L, v, partial);
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kBlock), 0, s, partial, npartial, out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_axpy(T* y, const T* x, T a, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_axpy<T>, dim3(nblocks(n)), dim3(kBlock), 0, s, y, x, a, n);
  return hipGetLastError();
}

hipError_t launch_harmonic_coarsen(const double* fine, double* coarse, int G, int nc, hipStream_t s) {
  hipLaunchKernelGGL(k_harmonic, dim3(nblocks(size_t(nc) * nc * G)), dim3(kBlock), 0, s, fine,
                     coarse, G, nc);
  return hipGetLastError();
}

hipError_t launch_convert_d2f(const double* in, float* out, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_d2f, dim3(nblocks(n)), dim3(kBlock), 0, s, in, out, n);
  return hipGetLastError();
}
hipError_t launch_convert_f2d(const float* in, double* out, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_f2d, dim3(nblocks(n)), dim3(kBlock), 0, s, in, out, n);
  return hipGetLastError();
}
hipError_t launch_add_f2d(double* y, const float* x, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_add_f2d, dim3(nblocks(n)), dim3(kBlock), 0, s, y, x, n);
  return hipGetLastError();
}

#define CTF_INSTANTIATE(T)                                                                          \
  template hipError_t launch_moments<T>(const LevelData<T>&, const T*, T*, int, hipStream_t);       \
  template hipError_t launch_emission<T>(const LevelDims&, const T*, const T*, int, const T*, T*,   \
                                         hipStream_t);                                              \
  template hipError_t launch_pg<T>(int, const LevelData<T>&, const Stencils<T>&, const PGParams&,   \
                                   const T*, const T*, int, const T*, const T*, T*, T*, T*, int, T, \
                                   const T*, hipStream_t);                                          \
  template hipError_t launch_upwind_full<T>(const LevelData<T>&, int, const T*, const T*, int, T*,  \
                                            int, T, const T*, hipStream_t);                         \
  template hipError_t launch_upwind_correction<T>(const LevelData<T>&, int, const T*, int, int,     \
                                                  const T*, T*, T*, hipStream_t);                   \
  template hipError_t launch_restrict<T>(const LevelData<T>&, const LevelData<T>&, const T*, T*,    \
                                         hipStream_t);                                              \
  template hipError_t launch_prolong<T>(const LevelData<T>&, int, const T*, T*, hipStream_t);       \
  template hipError_t launch_wnorm2<T>(const LevelData<T>&, const T*, double*, int, double*,        \
                                       hipStream_t);                                                \
  template hipError_t launch_axpy<T>(T*, const T*, T, size_t, hipStream_t);

CTF_INSTANTIATE(double)
CTF_INSTANTIATE(float)

}  // namespace ctf
