// HIP kernels (gfx950, wave64) of the ConvFEM space-angle multigrid transport solver.
//
// Layout of every angular-flux-shaped array: [G][n_dir][n][n], x fastest; 64-bit offsets.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <type_traits>

#include "internal.h"

namespace ctf {

namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ bool idle(const int* active) { return active && *active == 0; }

// A block's place in its grid: the hardware's for a kernel launched on its own, or one tile of an
// operation run by the persistent batched kernel (bd: threads per block).
struct VBlk {
  unsigned x, y, z, gx, gy, gz, bd;
};
__device__ __forceinline__ VBlk hw_blk() {
  return VBlk{blockIdx.x, blockIdx.y, blockIdx.z, gridDim.x, gridDim.y, gridDim.z, blockDim.x};
}

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// |x| as a source modifier and min as one instruction (the operands here are never NaN)
__device__ __forceinline__ float tabs(float x) { return __builtin_fabsf(x); }
__device__ __forceinline__ double tabs(double x) { return __builtin_fabs(x); }
__device__ __forceinline__ float tmin(float a, float b) { return __builtin_fminf(a, b); }
__device__ __forceinline__ double tmin(double a, double b) { return __builtin_fmin(a, b); }
__device__ __forceinline__ float tfma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double tfma(double a, double b, double c) { return __builtin_fma(a, b, c); }

// a / b for b > 0: float32 as a times the hardware reciprocal (within 2 ulp; the float32 kernels
// serve the refinement's inner cycles), float64 exactly rounded.
__device__ __forceinline__ float qdiv(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ double qdiv(double a, double b) { return a / b; }
// a / b with the reciprocal rb of b formed once for several quotients by the same b: float32 as
// a * rb (rb = qrcp(b), within 2 ulp), float64 exactly rounded (rb unused)
__device__ __forceinline__ float qrcp(float b) { return __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ double qrcp(double) { return 0.0; }
__device__ __forceinline__ float qdivr(float a, float, float rb) { return a * rb; }
__device__ __forceinline__ double qdivr(double a, double b, double) { return a / b; }

// Element at a 32-bit byte offset from a wave-uniform row pointer, so that the access is a scalar
// base plus a 32-bit vector offset (no 64-bit vector address arithmetic per access).
template <typename T>
__device__ __forceinline__ const T& at(const T* row, unsigned boff) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(row) + boff);
}
template <typename T>
__device__ __forceinline__ T& at(T* row, unsigned boff) {
  return *reinterpret_cast<T*>(reinterpret_cast<char*>(row) + boff);
}

// Raw buffer access to one plane of `bytes` bytes (< 2^31): a 32-bit vector byte offset (the
// column) plus a 32-bit scalar byte offset (the row), so that a load costs no vector address
// arithmetic at all; offsets past the plane read 0 (never reached: every offset is clamped).
// Resource word 3 is the raw-buffer format of the gfx9 family.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const void* p, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, int(bytes), 0x00020000);
}
template <typename T>
__device__ __forceinline__ T bload(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff);
template <>
__device__ __forceinline__ float bload<float>(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
template <>
__device__ __forceinline__ double bload<double>(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
__device__ __forceinline__ void bstore(float v, __amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, soff, 0);
}
__device__ __forceinline__ void bstore(double v, __amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  typedef unsigned u2 __attribute__((ext_vector_type(2)));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), r, voff, soff, 0);
}

// Anisotropic diffusivity of one direction component (eq. ano-k):
//   k = min(h|mu|, akabs |R| h / (eps + |Psi|), aksq R^2 h / (eps + |mu| Psi^2))
// with the per-ordinate constants kmax = h |mu|, amu = |mu|, cabs = akabs h and csq = aksq h formed
// once per block.  The diffusivity helpers evaluate exactly as written: contraction is off inside
// them and the fused multiply-adds are explicit (a contraction left to the compiler depends on the
// surrounding code), so that every kernel forming k gives the same bits.
template <typename T>
__device__ __forceinline__ T pg_k(T kmax, T amu, T R, T Psi, T cabs, T csq, T eps) {
#pragma clang fp contract(off)
  return tmin(tmin(kmax, qdiv(cabs * tabs(R), eps + tabs(Psi))), qdiv(csq * R * R, tfma(amu * Psi, Psi, eps)));
}

template <typename T>
__device__ __forceinline__ T dot2(T a, T b, T c, T d) {
#pragma clang fp contract(off)
  return tfma(a, b, c * d);
}

// Isotropic diffusivity (the residual-based form with the mixed-mass residual R = R_x + R_y):
//   k = min(sqrt((h mu)^2 + (h nu)^2), akabs |R| h / (eps + (|Psi_x| + |Psi_y|)/2),
//           aksq R^2 h / (eps + (|q Psi_x| + |q Psi_y|)/2 (Psi_x^2 + Psi_y^2))),
//   q = (mu Psi_x + nu Psi_y) / (eps + Psi_x^2 + Psi_y^2)
// with kmax = sqrt((h mu)^2 + (h nu)^2) (pg_kmax_iso), cabs = akabs h and csq = aksq h.
template <typename T>
__device__ __forceinline__ T pg_kmax_iso(T mu, T nu, T h) {
#pragma clang fp contract(off)
  const T hm = h * mu, hn = h * nu;
  return T(sqrt(dot2(hm, hm, hn, hn)));
}
template <typename T>
__device__ __forceinline__ T pg_k_iso(T mu, T nu, T R, T px, T py, T kmax, T cabs, T csq, T eps) {
#pragma clang fp contract(off)
  const T s2 = dot2(px, px, py, py);
  const T q = qdiv(dot2(mu, px, nu, py), eps + s2);
  const T kabs = qdiv(cabs * tabs(R), tfma(tabs(px) + tabs(py), T(0.5), eps));
  const T ksq = qdiv(csq * R * R, tfma((tabs(q * px) + tabs(q * py)) * T(0.5), s2, eps));
  return tmin(tmin(kmax, kabs), ksq);
}

// Emission of one ordinate from the flux moments: e0 + mu e1 + nu e2 (evaluated as written, so that
// every kernel gives the same bits)
template <typename T>
__device__ __forceinline__ T emission_p1(T e0, T e1, T e2, T mu, T nu) {
#pragma clang fp contract(off)
  return e0 + dot2(mu, e1, nu, e2);
}

// The mixed-mass estimate of the isotropic form, R = R_x + R_y (the two terms rounded as formed)
template <typename T>
__device__ __forceinline__ T pg_r_mixed(T rx, T ry) {
#pragma clang fp contract(off)
  return rx + ry;
}

// Residual estimate of the isotropic form from the difference of the advection estimates
// mu Psi_x + nu Psi_y of degree P (px, py) and of the other degree (qx, qy): RE 1 takes the degree
// P - 1 (R^Low = degree P minus degree P - 1), RE 2 the degree P + 1 (R^High = degree P + 1 minus
// degree P).
template <int RE, typename T>
__device__ __forceinline__ T pg_r_other_degree(T mu, T nu, T px, T py, T qx, T qy) {
#pragma clang fp contract(off)
  const T adv = dot2(mu, px, nu, py), advq = dot2(mu, qx, nu, qy);
  return RE == 1 ? adv - advq : advq - adv;
}

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
// moments: phi[g][m][cell] = sum_n w_n Y_m(n) psi[g][n][cell], Y = (1, mu, nu).
// A block covers 64 cells; its four waves each sum a contiguous quarter of the ordinates
// (four loads in flight per lane), and the quarters are added in a fixed order.
constexpr int kMomCells = 64;

template <typename T>
__device__ __forceinline__ void b_moments(const VBlk& vb, LevelData<T> L, const T* __restrict__ psi,
                                                     T* __restrict__ phi, int nmom) {
  if (idle(L.dims.active)) return;
  const int ncell = L.dims.n * L.dims.n;
  const int lane = threadIdx.x % kMomCells, q = threadIdx.x / kMomCells;
  const int cell = vb.x * kMomCells + lane;
  const int g = vb.y;
  const int nd = L.dims.nd, per = nd / 4;
  __shared__ T red[3][4][kMomCells];
  T a0 = 0, a1 = 0, a2 = 0;
  if (cell < ncell) {
    const T* src = psi + (size_t(g) * nd + size_t(q) * per) * ncell + cell;
    const T* w = L.w + q * per;
    const T* mu = L.mu + q * per;
    const T* nu = L.nu + q * per;
    int d = 0;
    for (; d + 4 <= per; d += 4) {
      const T v0 = src[size_t(d) * ncell], v1 = src[size_t(d + 1) * ncell];
      const T v2 = src[size_t(d + 2) * ncell], v3 = src[size_t(d + 3) * ncell];
      a0 += w[d] * v0;
      a0 += w[d + 1] * v1;
      a0 += w[d + 2] * v2;
      a0 += w[d + 3] * v3;
      if (nmom > 1) {
        a1 += (w[d] * mu[d]) * v0;
        a1 += (w[d + 1] * mu[d + 1]) * v1;
        a1 += (w[d + 2] * mu[d + 2]) * v2;
        a1 += (w[d + 3] * mu[d + 3]) * v3;
        a2 += (w[d] * nu[d]) * v0;
        a2 += (w[d + 1] * nu[d + 1]) * v1;
        a2 += (w[d + 2] * nu[d + 2]) * v2;
        a2 += (w[d + 3] * nu[d + 3]) * v3;
      }
    }
    for (; d < per; ++d) {
      const T v = src[size_t(d) * ncell];
      a0 += w[d] * v;
      if (nmom > 1) {
        a1 += (w[d] * mu[d]) * v;
        a2 += (w[d] * nu[d]) * v;
      }
    }
  }
  red[0][q][lane] = a0;
  red[1][q][lane] = a1;
  red[2][q][lane] = a2;
  __syncthreads();
  if (q == 0 && cell < ncell) {
    T* dst = phi + size_t(g) * nmom * ncell + cell;
    for (int m = 0; m < nmom; ++m)
      dst[size_t(m) * ncell] = (red[m][0][lane] + red[m][1][lane]) + (red[m][2][lane] + red[m][3][lane]);
  }
}
template <typename T>
__global__ __launch_bounds__(kBlock) void k_moments(LevelData<T> L, const T* __restrict__ psi, T* __restrict__ phi, int nmom) {
  b_moments<T>(hw_blk(), L, psi, phi, nmom);
}

// BF16 MFMA form of the moment contraction (float32 psi in memory):
//   Phi[m][cell] = sum_n W[m][n] psi[n][cell],  W = (w, w mu, w nu),
// as a [16 x n_dir] x [n_dir x cells] product on gfx950's v_mfma_f32_16x16x32_bf16 (K = 32
// ordinates per instruction) with float32 accumulation (rows 3..15 of W are zero).  psi is
// rounded to bf16 once; the weights are carried as a bf16 pair (hi + lo, two MFMAs per K-chunk)
// so that they keep ~16 bits.  A block owns 64 cells (four 16-cell MFMA tiles); its four waves
// each take a quarter of the ordinates, and the quarters are summed in a fixed order through LDS.
typedef short v8s_t __attribute__((ext_vector_type(8)));
typedef __bf16 v8bf_t __attribute__((ext_vector_type(8)));
typedef float v4f_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ v8bf_t as_bf16x8(v8s_t v) { return __builtin_bit_cast(v8bf_t, v); }

__device__ __forceinline__ unsigned short bf16_rne(float x) {
  unsigned int u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return static_cast<unsigned short>(u >> 16);
}
__device__ __forceinline__ float bf16_to_float(unsigned short b) {
  return __uint_as_float(static_cast<unsigned int>(b) << 16);
}

__device__ __forceinline__ void b_moments_mfma(const VBlk& vb, LevelData<float> L, const float* __restrict__ psi,
                                                          float* __restrict__ phi, int nmom) {
  if (idle(L.dims.active)) return;
  const int ncell = L.dims.n * L.dims.n;
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  const int c0 = vb.x * 64;
  const int g = vb.y;
  const int nd = L.dims.nd;
  const int per = nd / 4;                     // ordinates of this wave (a multiple of 2 at least)
  const int i = lane % 16, kq = lane / 16;    // A row / B column, and the K eighth-block of the lane
  v4f_t acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = v4f_t{0.f, 0.f, 0.f, 0.f};
  const float* base = psi + size_t(g) * nd * ncell;
  // K = 32 ordinates per MFMA: lane (i, kq) holds ordinates n0 + 8 kq .. n0 + 8 kq + 7
  for (int n0 = wave * per; n0 < (wave + 1) * per; n0 += 32) {
    v8s_t ahi, alo;
    v8s_t b[4];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int n = n0 + 8 * kq + j;
      const bool inK = n < (wave + 1) * per;
      float wv = 0.f;
      if (inK && i < 3) wv = L.w[n] * (i == 0 ? 1.f : (i == 1 ? L.mu[n] : L.nu[n]));
      const unsigned short hi = bf16_rne(wv);
      ahi[j] = static_cast<short>(hi);
      alo[j] = static_cast<short>(bf16_rne(wv - bf16_to_float(hi)));
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int c = c0 + 16 * t + i;
        const float v = (inK && c < ncell) ? base[size_t(n) * ncell + c] : 0.f;
        b[t][j] = static_cast<short>(bf16_rne(v));
      }
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(ahi), as_bf16x8(b[t]), acc[t], 0, 0, 0);
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(alo), as_bf16x8(b[t]), acc[t], 0, 0, 0);
    }
  }
  // D layout: lane holds rows 4*(lane/16) .. +3 of column lane % 16; rows 0..2 are the moments
  __shared__ float red[4][3][64];
  if (kq == 0) {
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int m = 0; m < 3; ++m) red[wave][m][16 * t + i] = acc[t][m];
  }
  __syncthreads();
  if (wave == 0) {
    const int c = c0 + lane;
    if (c < ncell)
      for (int m = 0; m < nmom; ++m)
        phi[(size_t(g) * nmom + m) * ncell + c] =
            (red[0][m][lane] + red[1][m][lane]) + (red[2][m][lane] + red[3][m][lane]);
  }
}
__global__ __launch_bounds__(kBlock) void k_moments_mfma(LevelData<float> L, const float* __restrict__ psi, float* __restrict__ phi, int nmom) {
  b_moments_mfma(hw_blk(), L, psi, phi, nmom);
}

// emission E[g][m][cell]: q_n = E0 + mu_n E1 + nu_n E2, all divided by 4 pi
template <typename T>
// phi_coarse: phi is given on the grid of half the size (the moments of UpSamp(e) are those of e
// on its own level, copied to the 2 x 2 children), read at the parent cell.
__device__ __forceinline__ void b_emission(const VBlk& vb, LevelDims d, const T* __restrict__ phi,
                                                      const T* __restrict__ ss, int nl,
                                                      const T* __restrict__ src, T* __restrict__ E,
                                                      int phi_coarse) {
  if (idle(d.active)) return;
  const size_t ncell = size_t(d.n) * d.n;
  const size_t t = size_t(vb.x) * kBlock + threadIdx.x;
  const int g = vb.y, G = d.G;
  if (t >= ncell) return;
  size_t tp = t, np = ncell;
  if (phi_coarse) {
    const int j = int(t / d.n), i = int(t % d.n), nh = d.n >> 1;
    tp = size_t(j >> 1) * nh + (i >> 1);
    np = size_t(nh) * nh;
  }
  const int nmom = nl > 1 ? 3 : 1;
  T e0 = src ? src[size_t(g) * ncell + t] : T(0), e1 = 0, e2 = 0;
  for (int gp = 0; gp < G; ++gp) {
    const T s0 = ss[(size_t(g) * G + gp) * ncell + t];
    e0 += s0 * phi[(size_t(gp) * nmom) * np + tp];
    if (nl > 1) {
      const T s1 = ss[((size_t(G) + g) * G + gp) * ncell + t];
      e1 += s1 * phi[(size_t(gp) * nmom + 1) * np + tp];
      e2 += s1 * phi[(size_t(gp) * nmom + 2) * np + tp];
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
template <typename T>
__global__ __launch_bounds__(kBlock) void k_emission(LevelDims d, const T* __restrict__ phi, const T* __restrict__ ss, int nl, const T* __restrict__ src, T* __restrict__ E, int phi_coarse) {
  b_emission<T>(hw_blk(), d, phi, ss, nl, src, E, phi_coarse);
}

// ---------------------------------------------------------------------------------------------
// ConvFEM Petrov-Galerkin operator (eq. Petrov, eqs. kxx/kyy, eq. ano-k), arguments.
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
  T rhs_sign;         // the rhs enters as rhs_sign * rhs (+1 or -1)
  int mode;
  T sign;
  int ntx;
  int strip_h;
  float* out_f;       // optional float copy of the output (mode 0)
  double* partial;    // optional per-block sum of w_n h^2 out^2 (mode 0)
  float* kx_out_f;    // optional float copies of the computed diffusivities
  float* ky_out_f;
  float* psi_f;       // optional float copy of psi at the output cells
  double* acc64;      // mode 1, optional: acc64 += out - float(acc64) at the output cells
};

// ---------------------------------------------------------------------------------------------
// Streaming forms of the ConvFEM Petrov-Galerkin operator.  One wavefront owns a strip of 64
// columns and marches down its rows; every filter is applied as an x-pass on the current row
// (row buffer in LDS) followed by a y-pass over a rolling window of x-pass results held in
// registers, so every input value is read from HBM about once.
constexpr int kStripW = 64;

// Logical block of a strip kernel (grid: strips x ordinates x groups; strip = strip row * ntx +
// strip column).  The hardware hands out workgroups round-robin over the 8 XCDs by linear block
// id; the blocks one XCD receives get a contiguous range of logical ids, taken in the order strip
// column (fastest), ordinate, strip row, group.  So one XCD runs the strips of one strip row side
// by side, and its own L2 keeps the psi rows neighbouring strips share, and it goes through the
// ordinates of that strip row while the row's per-cell planes (emission, sigma_t) stay in its L2.
constexpr unsigned kXcds = 8;
struct StripBlock {
  int strip, dir, g;
};
__device__ __forceinline__ StripBlock strip_block(unsigned ntx) {
  const unsigned nb = gridDim.x * gridDim.y * gridDim.z;
  const unsigned b = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
  const unsigned x = b % kXcds, k = b / kXcds, q = nb / kXcds, rm = nb % kXcds;
  const unsigned L = x * q + (x < rm ? x : rm) + k;
  const unsigned r1 = L / ntx, r2 = r1 / gridDim.y, nrow = gridDim.x / ntx;
  return StripBlock{int((r2 % nrow) * ntx + L % ntx), int(r1 % gridDim.y), int(r2 / nrow)};
}

template <typename T, int W>
__device__ __forceinline__ void push(T (&w)[W], T v) {
#pragma unroll
  for (int t = 0; t < W - 1; ++t) w[t] = w[t + 1];
  w[W - 1] = v;
}

template <typename T, int W>
__device__ __forceinline__ T ypass(const T (&w)[W], const T* c) {
  T s = 0;
#pragma unroll
  for (int t = 0; t < W; ++t) s += c[t] * w[t];
  return s;
}

// y-pass over a window filled in rotation: slot t holds the newest row, slot (t + 1) % W the
// oldest.  Called with t a constant of a fully unrolled loop, so every index is static and the
// window stays in registers without the moves of push().
template <typename T, int W>
__device__ __forceinline__ T yrot(const T (&w)[W], const T* c, int t) {
  T s = 0;
#pragma unroll
  for (int u = 0; u < W; ++u) s += c[u] * w[(t + 1 + u) % W];
  return s;
}

// x-pass of an antisymmetric stencil (c[P] = 0, c[P + u] = -c[P - u] in exact arithmetic: the
// first-derivative stencils) at the centre v[P] of the row values v[0 .. 2P]:
// sum_u c[P + u] (v[P + u] - v[P - u]), one instruction less than the full W-tap sum
template <int P, typename T>
__device__ __forceinline__ T xanti(const T* v, const T* c) {
  T s = c[P + 1] * (v[P + 1] - v[P - 1]);
#pragma unroll
  for (int u = 2; u <= P; ++u) s = tfma(c[P + u], v[P + u] - v[P - u], s);
  return s;
}

// the same as a y-pass over a rotating window (the slot order of yrot)
template <typename T, int W>
__device__ __forceinline__ T yanti(const T (&w)[W], const T* c, int t) {
  constexpr int P = (W - 1) / 2;
  T s = c[P + 1] * (w[(t + 2 + P) % W] - w[(t + P) % W]);
#pragma unroll
  for (int u = 2; u <= P; ++u) s = tfma(c[P + u], w[(t + 1 + P + u) % W] - w[(t + 1 + P - u) % W], s);
  return s;
}

// The k-Diff term of eqs. kxx / kyy, k_c f(psi; w) + f(k psi; w) - psi_c f(k; w) with w = x-pass (x)
// y-pass, from the windows of the three x-passes (a1 = psi, a2 = k psi, a3 = k): one y-pass over
// the rows a2 + k_c a1 - psi_c a3 (k_c, psi_c are the output node's values)
template <typename T, int W>
__device__ __forceinline__ T ykdiff(const T (&a1)[W], const T (&a2)[W], const T (&a3)[W], const T* c, int t, T kc,
                                    T pc) {
  T s = 0;
#pragma unroll
  for (int u = 0; u < W; ++u) {
    const int j = (t + 1 + u) % W;
    s += c[u] * tfma(-pc, a3[j], tfma(kc, a1[j], a2[j]));
  }
  return s;
}

// Residual with given diffusivities (k_x, k_y read with a copied halo):
//   rho = rhs_sign rhs + q - mu Psi_x - nu Psi_y - D_x - D_y - sigma_t psi,
//   D = k_c f(psi; w) + f(k psi; w) - psi_c f(k; w)   (eqs. kxx, kyy as written).
// ACC: a.acc64 is given (mode 1), its values are prefetched with the other per-cell data.
template <int P, typename T, bool ACC>
__global__ __launch_bounds__(kStripW) void k_pg_stream(PGArgs<T> a) {
  if (idle(a.L.dims.active)) return;
  constexpr int W = 2 * P + 1;
  constexpr int RW = kStripW + 2 * P;
  constexpr int D = P + 2;   // LDS ring of input rows: the current row and the P rows above it
  __shared__ T s_row[D][3][RW];   // psi, k_x, k_y side by side (one base address per row)
  const int n = a.L.dims.n;
  const int lane = threadIdx.x;
  const StripBlock sb = strip_block(unsigned(a.ntx));
  const int x0 = (sb.strip % a.ntx) * kStripW, y0 = (sb.strip / a.ntx) * a.strip_h;
  const int dir = sb.dir, g = sb.g;
  const size_t ncell = size_t(n) * n;
  const size_t base = (size_t(g) * a.L.dims.nd + dir) * ncell;
  const T mu = a.L.mu[dir], nu = a.L.nu[dir];
  const T h = T(a.L.dims.h);
  const T* __restrict__ psi = a.psi + base;
  const T* __restrict__ kxin = a.kx_in + base;
  const T* __restrict__ kyin = a.ky_in + base;
  T cm[W], cd[W], ck[W];
#pragma unroll
  for (int t = 0; t < W; ++t) {
    cm[t] = a.st.m[t];
    cd[t] = a.st.d[t];
    ck[t] = a.st.k[t];
    if constexpr (sizeof(T) == 8 && P == 3) {
      // float64 at p = 3: taps in vector registers (two waves per SIMD either way), so the loop's
      // scalar values do not spill into vector lanes
      asm volatile("" : "+v"(cm[t]));
      asm volatile("" : "+v"(cd[t]));
      asm volatile("" : "+v"(ck[t]));
    }
  }
  // x-pass results of the last W rows, slot = (row - first row) % W
  T wXd[W] = {}, wXm[W] = {}, wXk[W] = {}, wA2x[W] = {}, wA3x[W] = {}, wA2y[W] = {}, wA3y[W] = {};
  const int gi = x0 + lane;
  const int c0 = x0 - P + lane, c1 = c0 + kStripW;
  const int cc0 = clampi(c0, 0, n - 1), cc1 = clampi(c1, 0, n - 1);
  const bool zx0 = (c0 < 0 && (a.bc_vac & 1) && mu > T(0)) || (c0 >= n && (a.bc_vac & 2) && mu < T(0));
  const bool zx1 = (c1 < 0 && (a.bc_vac & 1) && mu > T(0)) || (c1 >= n && (a.bc_vac & 2) && mu < T(0));
  const int yend = min(y0 + a.strip_h, n);
  const T diag = a.beta * (tabs(mu) / h + tabs(nu) / h);
  double acc = 0.0;
  // Row values are loaded one row ahead so that the loads overlap the filtering of a row; so are
  // the per-cell values of the output row they complete (emission, rhs, sigma_t).  Every load is
  // unconditional, from a clamped (in-bounds) address, and the halo rule and unused values are
  // applied at the use: a load under a branch would make the wave wait for it at the join.
  T p0, k0, q0, p1, k1, q1;
  T fe0, fe1, fe2, frh, fs;   // emission moments, rhs, sigma_t of output row r - P
  double fy = 0.0;             // acc64 of output row r - P (ACC)
  const double* __restrict__ yp = ACC ? a.acc64 + base : nullptr;
  const unsigned b64 = unsigned(min(gi, n - 1)) * 8u;
  const bool has_rhs = a.rhs != nullptr, p1mom = a.nmomE > 1;
  const T rsg = a.rhs_sign;
  const T* __restrict__ Eg = a.E + size_t(g) * a.nmomE * ncell;
  const T* __restrict__ E1g = p1mom ? Eg + ncell : Eg;
  const T* __restrict__ E2g = p1mom ? Eg + 2 * ncell : Eg;
  const T* __restrict__ sigg = a.L.sigma_t + size_t(g) * ncell;
  const T* __restrict__ rhsp = has_rhs ? a.rhs + base : Eg;
  const unsigned b0 = unsigned(cc0) * sizeof(T), b1 = unsigned(cc1) * sizeof(T);
  const unsigned bc = unsigned(min(gi, n - 1)) * sizeof(T);
  const unsigned bo = unsigned(gi) * sizeof(T), bof = unsigned(gi) * sizeof(float);
  auto load_row = [&](int r) {
    const unsigned ro = unsigned(clampi(r, 0, n - 1)) * unsigned(n);   // 32-bit in-plane offsets
    p0 = at(psi + ro, b0);
    k0 = at(kxin + ro, b0);
    q0 = at(kyin + ro, b0);
    p1 = at(psi + ro, b1);
    k1 = at(kxin + ro, b1);
    q1 = at(kyin + ro, b1);
    const unsigned co = unsigned(clampi(r - P, y0, yend - 1)) * unsigned(n);   // rows of this strip only
    fe0 = at(Eg + co, bc);
    fe1 = at(E1g + co, bc);
    fe2 = at(E2g + co, bc);
    frh = at(rhsp + co, bc);
    fs = at(sigg + co, bc);
    if (ACC) fy = at(yp + co, b64);
  };
  const int rbeg = y0 - P, rend = yend + P;
  load_row(rbeg);
  int ring = 0;   // ring slot of the current row
  for (int r0 = rbeg; r0 < rend; r0 += W) {
#pragma unroll
    for (int t = 0; t < W; ++t) {
      const int r = r0 + t;
      if (r >= rend) break;
      T* const rp = s_row[ring][0];
      T* const rk = s_row[ring][1];
      T* const rq = s_row[ring][2];
      const bool zy = (r < 0 && (a.bc_vac & 4) && nu > T(0)) || (r >= n && (a.bc_vac & 8) && nu < T(0));
      rp[lane] = (zy || zx0) ? T(0) : p0;
      rk[lane] = k0;
      rq[lane] = q0;
      if (lane < 2 * P) {
        rp[kStripW + lane] = (zy || zx1) ? T(0) : p1;
        rk[kStripW + lane] = k1;
        rq[kStripW + lane] = q1;
      }
      const T e0 = fe0, e1 = fe1, e2 = fe2, rh = frh, sig = fs;
      const double y64 = fy;
      load_row(r + 1);   // past the last row this reloads a clamped row, unused
      __syncthreads();
      const T xd = xanti<P>(rp + lane, cd);
      T xm = 0, xk = 0, a2x = 0, a3x = 0, a2y = 0, a3y = 0;
#pragma unroll
      for (int u = 0; u < W; ++u) {
        const T v = rp[lane + u], kv = rk[lane + u], qv = rq[lane + u];
        xm += cm[u] * v;
        xk += ck[u] * v;
        a2x += ck[u] * (kv * v);
        a3x += ck[u] * kv;
        a2y += cm[u] * (qv * v);
        a3y += cm[u] * qv;
      }
      wXd[t] = xd;
      wXm[t] = xm;
      wXk[t] = xk;
      wA2x[t] = a2x;
      wA3x[t] = a3x;
      wA2y[t] = a2y;
      wA3y[t] = a3y;
      const int o = r - P;
      if (o >= y0 && gi < n) {
        const int cs = ring >= P ? ring - P : ring + D - P;   // ring slot of row o
        const T pc = s_row[cs][0][lane + P], kxc = s_row[cs][1][lane + P], kyc = s_row[cs][2][lane + P];
        const T px = yrot(wXd, cm, t), py = yanti(wXm, cd, t);
        const T dx = ykdiff(wXk, wA2x, wA3x, cm, t, kxc, pc);
        const T dy = ykdiff(wXm, wA2y, wA3y, ck, t, kyc, pc);
        const size_t ro = base + size_t(o) * n;
        T q = e0;
        if (p1mom) q = emission_p1(q, e1, e2, mu, nu);
        if (has_rhs) q = tfma(rsg, rh, q);
        const T rho = q - mu * px - nu * py - dx - dy - sig * pc;
        if (a.psi_f) at(a.psi_f + ro, bof) = float(pc);
        if (a.mode == 0) {
          const T val = a.sign * rho;
          if (a.out) at(a.out + ro, bo) = val;
          if (a.out_f) at(a.out_f + ro, bof) = float(val);
          if constexpr (sizeof(T) == 8) acc += double(val) * double(val);
        } else {
          const T un = pc + qdiv(rho, diag + a.beta * sig);
          at(a.out + ro, bo) = un;
          if (ACC) at(a.acc64 + ro, unsigned(gi) * 8u) = y64 + (double(un) - double(float(y64)));
        }
      }
      ring = ring + 1 == D ? 0 : ring + 1;
    }
  }
  // norms are float64 only (a float32 launch with partial sums is refused by launch_pg)
  if (sizeof(T) == 8 && a.partial) {
    // wave-level reduction in a fixed order (deterministic)
    __shared__ double red[kStripW];
    red[lane] = acc;
    __syncthreads();
    for (int s = kStripW / 2; s > 0; s >>= 1) {
      if (lane < s) red[lane] += red[lane + s];
      __syncthreads();
    }
    if (lane == 0) {
      const size_t b = blockIdx.x + size_t(gridDim.x) * (blockIdx.y + size_t(gridDim.y) * blockIdx.z);
      a.partial[b] = red[0] * double(a.L.w[dir]) * a.L.dims.h * a.L.dims.h;
    }
  }
}

// Anisotropic diffusivities of psi (eq. ano-k) on the interior:
//   Psi_x = f(psi; m (x) d), Psi_y = f(psi; d (x) m) (psi with its halo rule),
//   R = alpha_r mu (f(Psi; m (x) m) - Psi),  k = min(h|mu|, akabs |R| h/(eps+|Psi|), aksq R^2 h/(eps+|mu| Psi^2)).
// The strip reads 64 + 4P columns, and writes k for its inner 64 - 2P columns.
// RE selects the diffusivity: 0 anisotropic (above); the isotropic form with R from the mixed mass
// (3) or from the difference of the advection estimates mu Psi_x + nu Psi_y of degrees P and
// P - 1 / P + 1 (1 / 2; section "Non-Linear Petrov-Galerkin Dissipation").  The other degree Q = P -+ 1 is x-passed on every
// psi row into windows of 2P + Q + 1 rows, long enough to reach back to row o - Q when row o is
// written.
template <int P, int RE, typename T>
__global__ __launch_bounds__(kStripW) void k_pg_diffusivity(PGArgs<T> a) {
  if (idle(a.L.dims.active)) return;
  static_assert(RE == 0 || RE == 3 || (RE == 1 && P >= 2) || (RE == 2 && P + 1 <= kMaxP),
                "residual estimate degree");
  constexpr bool MIXED = RE == 0 || RE == 3;   // R from the mixed mass (anisotropic or isotropic k)
  constexpr int W = 2 * P + 1;
  constexpr int PQ = RE == 1 ? P - 1 : (RE == 2 ? P + 1 : 0);   // the other degree
  constexpr int WQ = 2 * PQ + 1;
  constexpr int KQ = MIXED ? 1 : 2 * P + PQ + 1;
  constexpr int RW = kStripW + 2 * P;
  constexpr int OW = kStripW - 2 * P;   // columns written per strip
  // LDS ring of Psi rows (the newest and the P rows above it), as deep as the unrolled pass and
  // numbered from the strip's first row: the Psi row formed at step t of a pass sits in slot t
  constexpr int D = W;
  __shared__ T s_psi[RW];
  __shared__ T s_g[D][2][kStripW];   // Psi_x, Psi_y side by side
  const int n = a.L.dims.n;
  const int lane = threadIdx.x;
  const StripBlock sb = strip_block(unsigned(a.ntx));
  const int xs = (sb.strip % a.ntx) * OW, y0 = (sb.strip / a.ntx) * a.strip_h;
  const int x0 = xs - P;                 // column of lane 0 (Psi is formed for x0 .. x0 + 63)
  const int dir = sb.dir, g = sb.g;
  const size_t ncell = size_t(n) * n;
  const size_t base = (size_t(g) * a.L.dims.nd + dir) * ncell;
  const T mu = a.L.mu[dir], nu = a.L.nu[dir];
  const T h = T(a.L.dims.h);
  const T* __restrict__ psi = a.psi + base;
  T cm[W], cd[W];
#pragma unroll
  for (int t = 0; t < W; ++t) {
    cm[t] = a.st.m[t];
    cd[t] = a.st.d[t];
  }
  T cmq[WQ], cdq[WQ];
#pragma unroll
  for (int t = 0; t < WQ; ++t) {
    cmq[t] = a.st.mr[t];
    cdq[t] = a.st.dr[t];
  }
  // rotating windows (slot = step % W): x-passes of psi rows, x-passes of Psi rows
  T wXd[W] = {}, wXm[W] = {}, wMx[W] = {}, wMy[W] = {};
  // shifted windows (newest row last) of the other degree's x-passes
  T wQd[KQ] = {}, wQm[KQ] = {};
  const int c0 = x0 - P + lane, c1 = c0 + kStripW;
  const int cc0 = clampi(c0, 0, n - 1), cc1 = clampi(c1, 0, n - 1);
  const bool zx0 = (c0 < 0 && (a.bc_vac & 1) && mu > T(0)) || (c0 >= n && (a.bc_vac & 2) && mu < T(0));
  const bool zx1 = (c1 < 0 && (a.bc_vac & 1) && mu > T(0)) || (c1 >= n && (a.bc_vac & 2) && mu < T(0));
  const int gi = x0 + lane;
  const bool writer = lane >= P && lane < kStripW - P && gi < n && gi < xs + OW;
  const int yend = min(y0 + a.strip_h, n);
  const T eps = a.eps_k, ar = a.alpha_r;
  const T cabs = a.akabs * h, csq = a.aksq * h, amu = tabs(mu), anu = tabs(nu);
  const T kmx = h * amu, kmy = h * anu, kmi = pg_kmax_iso(mu, nu, h);
  // rows are loaded one ahead, unconditionally from clamped addresses (the halo rule is applied
  // when the row is written to LDS), so that no join waits for a load in flight
  T p0, p1;
  const unsigned b0 = unsigned(cc0) * sizeof(T), b1 = unsigned(cc1) * sizeof(T);
  const unsigned bo = unsigned(gi) * sizeof(T), bof = unsigned(gi) * sizeof(float);
  // FAST: row r needs no clamping
  auto load_row = [&](int r, auto fast) {
    constexpr bool FAST = decltype(fast)::value;
    const unsigned ro = unsigned(FAST ? r : clampi(r, 0, n - 1)) * unsigned(n);   // 32-bit in-plane offsets
    p0 = at(psi + ro, b0);
    p1 = at(psi + ro, b1);
  };
  const int rbeg = y0 - 2 * P, rend = yend + 2 * P;
  load_row(rbeg, std::false_type{});
  // One row step (t: its place in the unrolled pass).  FAST: a row of the strip's interior, where
  // row r + 1 lies inside the domain and the output row is written.
  auto step = [&](const int r, const int t, auto fast) __attribute__((always_inline)) {
    constexpr bool FAST = decltype(fast)::value;
    const bool zy = !FAST && ((r < 0 && (a.bc_vac & 4) && nu > T(0)) || (r >= n && (a.bc_vac & 8) && nu < T(0)));
    s_psi[lane] = (zy || zx0) ? T(0) : p0;
    if (lane < 2 * P) s_psi[kStripW + lane] = (zy || zx1) ? T(0) : p1;
    load_row(r + 1, fast);   // past the last row this reloads a clamped row, unused
    __syncthreads();
    const T xd = xanti<P>(s_psi + lane, cd);
    T xm = 0;
#pragma unroll
    for (int u = 0; u < W; ++u) xm += cm[u] * s_psi[lane + u];
    wXd[t] = xd;
    wXm[t] = xm;
    if constexpr (!MIXED) {
      // taps lq - 1 .. lq + 2P + 1 (degree P + 1) stay inside the row buffer; lq = lane for
      // every lane that writes
      const int lq = RE == 2 ? clampi(lane, 1, kStripW - 2) : lane;
      T qd = 0, qm = 0;
#pragma unroll
      for (int u = 0; u < WQ; ++u) {
        const T v = s_psi[lq + P - PQ + u];
        qd += cdq[u] * v;
        qm += cmq[u] * v;
      }
      push(wQd, qd);
      push(wQm, qm);
    }
    // Psi on row r - P (meaningful once the window is full)
    T* const gxr = s_g[t][0];
    T* const gyr = s_g[t][1];
    gxr[lane] = yrot(wXd, cm, t);
    gyr[lane] = yanti(wXm, cd, t);
    __syncthreads();
    if constexpr (MIXED) {
      T mx = 0, my = 0;
      if (lane >= P && lane < kStripW - P) {
#pragma unroll
        for (int u = 0; u < W; ++u) {
          mx += cm[u] * gxr[lane - P + u];
          my += cm[u] * gyr[lane - P + u];
        }
      }
      wMx[t] = mx;
      wMy[t] = my;
    }
    const int o = r - 2 * P;
    if ((FAST || o >= y0) && writer) {
      const int cs = (t + W - P) % W;   // ring slot of Psi row o
      const T px = s_g[cs][0][lane], py = s_g[cs][1][lane];
      T kx, ky;
      if constexpr (!MIXED) {
        // Psi of the other degree on row o: y-pass over the window rows o - Q .. o + Q
        T qx = 0, qy = 0;
#pragma unroll
        for (int v = 0; v < WQ; ++v) {
          qx += cmq[v] * wQd[v];
          qy += cdq[v] * wQm[v];
        }
        kx = ky = pg_k_iso(mu, nu, pg_r_other_degree<RE>(mu, nu, px, py, qx, qy), px, py, kmi, cabs, csq, eps);
      } else {
        const T rx = ar * mu * (yrot(wMx, cm, t) - px);
        const T ry = ar * nu * (yrot(wMy, cm, t) - py);
        if constexpr (RE == 3) {
          kx = ky = pg_k_iso(mu, nu, pg_r_mixed(rx, ry), px, py, kmi, cabs, csq, eps);
        } else {
          kx = pg_k(kmx, amu, rx, px, cabs, csq, eps);
          ky = pg_k(kmy, anu, ry, py, cabs, csq, eps);
        }
      }
      const size_t ro = base + size_t(o) * n;
      if (a.kx_out) {
        at(a.kx_out + ro, bo) = kx;
        at(a.ky_out + ro, bo) = ky;
      }
      if (a.kx_out_f) {
        at(a.kx_out_f + ro, bof) = float(kx);
        at(a.ky_out_f + ro, bof) = float(ky);
      }
    }
  };
  const int flo = y0 + 2 * P, fhi = min(n - 1, rend);
  const int f0 = rbeg + W * ((max(flo - rbeg, 0) + W - 1) / W);
  int r0 = rbeg;
  for (; r0 < rend && r0 < f0; r0 += W) {
#pragma unroll
    for (int t = 0; t < W; ++t) {
      if (r0 + t >= rend) break;
      step(r0 + t, t, std::false_type{});
    }
  }
  for (; r0 + W <= fhi; r0 += W) {
#pragma unroll
    for (int t = 0; t < W; ++t) step(r0 + t, t, std::true_type{});
  }
  for (; r0 < rend; r0 += W) {
#pragma unroll
    for (int t = 0; t < W; ++t) {
      if (r0 + t >= rend) break;
      step(r0 + t, t, std::false_type{});
    }
  }
}

// Fused non-linear form: the diffusivities are formed in the same pass and never stored.
// A wavefront owns 64 columns, lane l at column xs - 2P + l, and writes the 64 - 4P columns
// xs .. xs + 63 - 4P; rows stream through a four-stage pipeline (row r loaded at step r):
//   A  Psi_x, Psi_y of row r - P          (x-pass on the psi row, y-pass over registers)
//   B  R_x, R_y and k_x, k_y of row r - 2P (x-pass on the Psi row, y-pass over registers)
//   C  x-passes of psi, k psi, k for row r - 3P (the k halo copies the nearest interior row and
//      column)
//   D  output row r - 4P (y-passes over registers)
// psi, Psi and k rows live in LDS rings deep enough for every later stage that reads them (the
// centre values of psi and k at row r - 4P included; up to P = 2 those of Psi at row r - 4P are kept
// in registers from stage B); the y-pass windows rotate with the unrolled step.
// slot of the row `off` rows above the row in slot s (0 <= off < depth)
__device__ __forceinline__ int ring_back(int s, int off, int depth) { return s >= off ? s - off : s - off + depth; }
__device__ __forceinline__ int ring_next(int s, int depth) { return s + 1 == depth ? 0 : s + 1; }

// ACC: a.acc64 is given (mode 1), its values are prefetched with the other per-cell data.
// RE: the diffusivity, as in k_pg_diffusivity (0 anisotropic; 3 isotropic with the mixed mass; 1 / 2
// isotropic from the advection estimates of degrees P and P - 1 / P + 1, the other degree x-passed
// in stage A into shifted windows that reach back to row r - 2P - Q when stage B forms k of row
// r - 2P).
template <int P, int RE, typename T, bool ACC>
__global__ __launch_bounds__(kStripW, P == 2 ? (sizeof(T) == 4 ? (ACC ? 3 : 4) : 2) : 1) void k_pg_fused(PGArgs<T> a) {
  if (idle(a.L.dims.active)) return;
  static_assert(RE == 0 || RE == 3 || (RE == 1 && P >= 2) || (RE == 2 && P + 1 <= kMaxP),
                "residual estimate degree");
  constexpr bool MIXED = RE == 0 || RE == 3;   // R from the mixed mass (anisotropic or isotropic k)
  constexpr int W = 2 * P + 1;
  constexpr int PQ = RE == 1 ? P - 1 : (RE == 2 ? P + 1 : 0);   // the other degree
  constexpr int WQ = 2 * PQ + 1;
  constexpr int KQ = MIXED ? 1 : 2 * P + PQ + 1;
  constexpr int RW = kStripW + 2 * P;   // psi row with a P-column halo
  // Rings (slots numbered from the strip's first row).  Up to P = 2 (PS2) the psi ring (rows
  // r - 4P .. r) is two unrolled passes deep (4P + 1 <= 2W) and the interior loop runs pairs of
  // passes, so its slots are static; at P >= 3 that unroll costs occupancy and the ring (4P + 1
  // rows) takes run-time slots.  With GS (up to P = 2, and at P = 3 in float32) the Psi ring holds
  // rows r - 2P .. r - P in W static slots (slot t: the row formed at step t), the Psi of row
  // r - 4P that stage D needs being kept in registers from stage B; otherwise (float64 at P = 3,
  // P = 4: those registers would cost occupancy) it holds rows r - 4P .. r - P in run-time slots.
  constexpr bool PS2 = P <= 2;
  constexpr bool GS = P <= 2 || (P == 3 && sizeof(T) == 4);
  constexpr int PR = PS2 ? 2 * W : 4 * P + 1;
  constexpr int GR = GS ? W : 3 * P + 1;
  constexpr int KR = 2 * P + 1;         // k rows kept (r - 4P .. r - 2P)
  constexpr int OW = kStripW - 4 * P;   // columns written per strip
  // x and y components side by side, so that both are addressed from one base; Psi and k rows
  // carry P unused entries on either side, so that every lane's taps stay inside the array
  // (lanes whose results are not used read those entries instead of branching around the taps)
  constexpr int GW = kStripW + 2 * P;
  __shared__ T s_psi[PR][RW];
  __shared__ T s_g[GR][2][GW];   // Psi_x, Psi_y of lane l at index P + l
  __shared__ T s_k[KR][2][GW];   // k_x, k_y (columns outside the domain: the k halo copy)
  const int n = a.L.dims.n;
  const int lane = threadIdx.x;
  const StripBlock sb = strip_block(unsigned(a.ntx));
  const int xs = (sb.strip % a.ntx) * OW, y0 = (sb.strip / a.ntx) * a.strip_h;
  const int c0 = xs - 2 * P;            // column of lane 0
  const int dir = sb.dir, g = sb.g;
  const size_t ncell = size_t(n) * n;
  const size_t base = (size_t(g) * a.L.dims.nd + dir) * ncell;
  const T mu = a.L.mu[dir], nu = a.L.nu[dir];
  const T h = T(a.L.dims.h);
  const T* __restrict__ psi = a.psi + base;
  T cm[W], cd[W], ck[W];
#pragma unroll
  for (int t = 0; t < W; ++t) {
    cm[t] = a.st.m[t];
    cd[t] = a.st.d[t];
    ck[t] = a.st.k[t];
    if constexpr (P <= 2) {
      // up to p = 2: keep the taps in vector registers (in scalar registers they crowd out the
      // loop's buffer resources and addresses, which then spill into vector lanes)
      asm volatile("" : "+v"(cm[t]));
      asm volatile("" : "+v"(cd[t]));
      asm volatile("" : "+v"(ck[t]));
    }
  }
  T cmq[WQ] = {}, cdq[WQ] = {};
  if constexpr (!MIXED) {
#pragma unroll
    for (int t = 0; t < WQ; ++t) {
      cmq[t] = a.st.mr[t];
      cdq[t] = a.st.dr[t];
    }
  }
  T wXd[W] = {}, wXm[W] = {}, wMx[W] = {}, wMy[W] = {};
  // Psi of the lane's own column, row r - 2P, read again by stage D 2P steps later
  T wDx[GS ? W : 1] = {}, wDy[GS ? W : 1] = {};
  T wA1x[W] = {}, wA2x[W] = {}, wA3x[W] = {}, wA1y[W] = {}, wA2y[W] = {}, wA3y[W] = {};
  // shifted windows (newest row last) of the other degree's x-passes
  T wQd[KQ] = {}, wQm[KQ] = {};
  // psi row loads: lane l -> column c0 - P + l; lanes < 2P also column c0 - P + 64 + l
  const int lc0 = c0 - P + lane, lc1 = lc0 + kStripW;
  const int cc0 = clampi(lc0, 0, n - 1), cc1 = clampi(lc1, 0, n - 1);
  const bool zx0 = (lc0 < 0 && (a.bc_vac & 1) && mu > T(0)) || (lc0 >= n && (a.bc_vac & 2) && mu < T(0));
  const bool zx1 = (lc1 < 0 && (a.bc_vac & 1) && mu > T(0)) || (lc1 >= n && (a.bc_vac & 2) && mu < T(0));
  const int col = c0 + lane;
  const bool writer = lane >= 2 * P && lane < kStripW - 2 * P && col < n;
  // strips that reach past the domain copy k of the nearest interior column into those columns
  const bool edge_strip = c0 < 0 || c0 + kStripW > n;
  const int kcl = clampi(col, 0, n - 1) - c0;   // lane of the nearest interior column (own lane inside)
  const int hidx = lane < 2 * P ? kStripW + lane : lane;   // halo lanes also write the P columns past 64
  const int yend = min(y0 + a.strip_h, n);
  const T eps = a.eps_k, ar = a.alpha_r;
  const T cabs = a.akabs * h, csq = a.aksq * h, amu = tabs(mu), anu = tabs(nu);
  const T kmx = h * amu, kmy = h * anu, kmi = pg_kmax_iso(mu, nu, h);
  const T diag = a.beta * (tabs(mu) / h + tabs(nu) / h);
  double acc = 0.0;
  // loads are unconditional, from clamped addresses (halo rule and unused values applied at the
  // use), so that no join waits for a load in flight
  T p0, p1, fe0, fe1, fe2, frh, fs;
  double fy = 0.0;
  const double* __restrict__ yp = ACC ? a.acc64 + base : nullptr;
  const unsigned b64 = unsigned(clampi(col, 0, n - 1)) * 8u;
  const bool has_rhs = a.rhs != nullptr, p1mom = a.nmomE > 1;
  const T rsg = a.rhs_sign;
  const T* __restrict__ Eg = a.E + size_t(g) * a.nmomE * ncell;
  const T* __restrict__ sigg = a.L.sigma_t + size_t(g) * ncell;
  const T* __restrict__ rhsp = has_rhs ? a.rhs + base : Eg;
  const unsigned b0 = unsigned(cc0) * sizeof(T), b1 = unsigned(cc1) * sizeof(T);
  const unsigned bc = unsigned(clampi(col, 0, n - 1)) * sizeof(T);
  const unsigned bo = unsigned(col) * sizeof(T), bof = unsigned(col) * sizeof(float);
  // planes are below 2^29 bytes (n <= 8192): loads take the column as a vector byte offset and the
  // row as a scalar one.  The per-cell planes E0, E1, E2 are consecutive, one resource covers them.
  const unsigned pb = unsigned(ncell * sizeof(T));
  const __amdgpu_buffer_rsrc_t r_psi = plane_rsrc(psi, pb), r_sig = plane_rsrc(sigg, pb),
                               r_rh = plane_rsrc(rhsp, pb), r_e = plane_rsrc(Eg, p1mom ? 3 * pb : pb),
                               r_y = plane_rsrc(yp, unsigned(ncell * 8));
  const unsigned e1o = p1mom ? pb : 0u, e2o = p1mom ? 2 * pb : 0u;
  // the float32 residual and sweep write their one output plane (and the sweep with the float64
  // update its float64 plane) through buffer stores; the float64 kernel keeps plain stores (its
  // scalar registers are short)
  constexpr bool BST = sizeof(T) == 4;
  const __amdgpu_buffer_rsrc_t w_out = plane_rsrc(BST ? a.out + base : nullptr, pb),
                               w_acc = plane_rsrc(BST && ACC ? a.acc64 + base : nullptr, unsigned(ncell * 8));
  // FAST: rows r and r - 4P need no clamping
  auto load_row = [&](int r, auto fast) {
    constexpr bool FAST = decltype(fast)::value;
    const unsigned ro = unsigned(FAST ? r : clampi(r, 0, n - 1)) * unsigned(n) * unsigned(sizeof(T));
    p0 = bload<T>(r_psi, b0, ro);
    p1 = bload<T>(r_psi, b1, ro);
    const unsigned cr = unsigned(FAST ? r - 4 * P : clampi(r - 4 * P, y0, yend - 1)) * unsigned(n);   // rows of this strip only
    const unsigned co = cr * unsigned(sizeof(T));
    fe0 = bload<T>(r_e, bc, co);
    fe1 = bload<T>(r_e, bc, co + e1o);
    fe2 = bload<T>(r_e, bc, co + e2o);
    frh = bload<T>(r_rh, bc, co);
    fs = bload<T>(r_sig, bc, co);
    if (ACC) fy = bload<double>(r_y, b64, cr * 8u);
  };
  const int rbeg = y0 - 3 * P, rend = yend + 4 * P;
  load_row(rbeg, std::false_type{});
  // The k ring is as deep as the unrolled pass (KR = W): the k row formed at step t sits in slot t.
  static_assert(KR == W && (GR == W || !GS), "k (and with GS Psi) ring depths equal the unroll");
  // One row step (t: its place in the unrolled pass; ps, gsl: the psi slot of row r and the Psi slot
  // of row r - P).  FAST: a row of the strip's interior, where rows r + 1, r - 2P, r - 3P and r - 4P
  // lie inside the domain and the strip (no clamping, no halo rows, the output row written): the
  // bounds checks drop out of the compiled step.
  auto step = [&](const int r, const int t, const int ps, const int gsl, auto fast) __attribute__((always_inline)) {
    constexpr bool FAST = decltype(fast)::value;
    T* const prow = s_psi[ps];
    const bool zy = !FAST && ((r < 0 && (a.bc_vac & 4) && nu > T(0)) || (r >= n && (a.bc_vac & 8) && nu < T(0)));
    const T v0 = (zy || zx0) ? T(0) : p0, v1 = (zy || zx1) ? T(0) : p1;
    prow[lane] = v0;
    prow[hidx] = lane < 2 * P ? v1 : v0;   // other lanes rewrite their own value
    const T e0 = fe0, e1 = fe1, e2 = fe2, rh = frh, sig = fs;
    const double y64 = fy;
    load_row(r + 1, fast);   // past the last row this reloads a clamped row, unused
    __syncthreads();
    // A: Psi of row r - P
    T* const gxr = &s_g[gsl][0][P];
    T* const gyr = &s_g[gsl][1][P];
    {
      const T xd = xanti<P>(prow + lane, cd);
      T xm = 0;
#pragma unroll
      for (int u = 0; u < W; ++u) xm += cm[u] * prow[lane + u];
      wXd[t] = xd;
      wXm[t] = xm;
      gxr[lane] = yrot(wXd, cm, t);
      gyr[lane] = yanti(wXm, cd, t);
      if constexpr (!MIXED) {
        // taps lq - 1 .. lq + 2P + 1 (degree P + 1) stay inside the row; lq = lane on every lane
        // whose k is read (P .. 63 - P)
        const int lq = RE == 2 ? clampi(lane, 1, kStripW - 2) : lane;
        T qd = 0, qm = 0;
#pragma unroll
        for (int u = 0; u < WQ; ++u) {
          const T v = prow[lq + P - PQ + u];
          qd += cdq[u] * v;
          qm += cmq[u] * v;
        }
        push(wQd, qd);
        push(wQm, qm);
      }
    }
    // the other-degree estimates read Psi of their own lane only: no wait for its neighbours
    if constexpr (MIXED) __syncthreads();
    // B: k of row r - 2P
    {
      if constexpr (MIXED) {
        T mx = 0, my = 0;
#pragma unroll
        for (int u = 0; u < W; ++u) {
          mx += cm[u] * gxr[lane - P + u];
          my += cm[u] * gyr[lane - P + u];
        }
        wMx[t] = mx;
        wMy[t] = my;
      }
      const int rk = r - 2 * P;
      if (FAST || (rk >= 0 && rk < n)) {
        const int gs = ring_back(gsl, P, GR);
        const T px = s_g[gs][0][P + lane], py = s_g[gs][1][P + lane];
        if constexpr (GS) {
          wDx[t] = px;
          wDy[t] = py;
        }
        T* const k0r = &s_k[t][0][P];
        T* const k1r = &s_k[t][1][P];
        if constexpr (!MIXED) {
          // Psi of the other degree on row rk: y-pass over the window rows rk - Q .. rk + Q
          T qx = 0, qy = 0;
#pragma unroll
          for (int v = 0; v < WQ; ++v) {
            qx += cmq[v] * wQd[v];
            qy += cdq[v] * wQm[v];
          }
          const T kk = pg_k_iso(mu, nu, pg_r_other_degree<RE>(mu, nu, px, py, qx, qy), px, py, kmi, cabs, csq, eps);
          k0r[lane] = kk;
          k1r[lane] = kk;
        } else if constexpr (RE == 3) {
          const T rx = ar * mu * (yrot(wMx, cm, t) - px);
          const T ry = ar * nu * (yrot(wMy, cm, t) - py);
          const T kk = pg_k_iso(mu, nu, pg_r_mixed(rx, ry), px, py, kmi, cabs, csq, eps);
          k0r[lane] = kk;
          k1r[lane] = kk;
        } else {
          const T rx = ar * mu * (yrot(wMx, cm, t) - px);
          const T ry = ar * nu * (yrot(wMy, cm, t) - py);
          k0r[lane] = pg_k(kmx, amu, rx, px, cabs, csq, eps);
          k1r[lane] = pg_k(kmy, anu, ry, py, cabs, csq, eps);
        }
        if (edge_strip) {
          // columns outside the domain take k of the nearest interior column
          __syncthreads();
          const T ox = k0r[kcl], oy = k1r[kcl];
          __syncthreads();
          k0r[lane] = ox;
          k1r[lane] = oy;
        }
      }
    }
    __syncthreads();
    // C: x-passes of row s = r - 3P (k of the clamped row and columns)
    {
      const int srow = r - 3 * P;
      const T* const spr = s_psi[ring_back(ps, 3 * P, PR)];
      // k of row srow (formed P steps ago), or of the nearest interior row (formed at step row + 2P)
      int ks = (t + W - P) % W;
      if (!FAST && (srow < 0 || srow >= n)) ks = int(unsigned(clampi(srow, 0, n - 1) + 2 * P - rbeg) % unsigned(W));
      const T* const kxr = &s_k[ks][0][P];
      const T* const kyr = &s_k[ks][1][P];
      T a1x = 0, a2x = 0, a3x = 0, a1y = 0, a2y = 0, a3y = 0;
#pragma unroll
      for (int u = 0; u < W; ++u) {
        const T v = spr[lane + u];
        const T kv = kxr[lane - P + u], qv = kyr[lane - P + u];
        a1x += ck[u] * v;
        a2x += ck[u] * (kv * v);
        a3x += ck[u] * kv;
        a1y += cm[u] * v;
        a2y += cm[u] * (qv * v);
        a3y += cm[u] * qv;
      }
      wA1x[t] = a1x;
      wA2x[t] = a2x;
      wA3x[t] = a3x;
      wA1y[t] = a1y;
      wA2y[t] = a2y;
      wA3y[t] = a3y;
    }
    // D: output row r - 4P
    const int o = r - 4 * P;
    if ((FAST || o >= y0) && writer) {
      const int ks = (t + W - 2 * P) % W;
      // with GS, Psi of this row as read by stage B 2P steps ago, made opaque here so that no
      // product stage B formed from it (the isotropic bound's nu Psi_y) is reused in this residual,
      // which then contracts as in the two-pass kernel, bit for bit
      T px, py;
      if constexpr (GS) {
        px = wDx[ks % (GS ? W : 1)];
        py = wDy[ks % (GS ? W : 1)];
        asm volatile("" : "+v"(px), "+v"(py));
      } else {
        const int gs = ring_back(gsl, 3 * P, GR);
        px = s_g[gs][0][P + lane];
        py = s_g[gs][1][P + lane];
      }
      const T psc = s_psi[ring_back(ps, 4 * P, PR)][lane + P];
      const T kxc = s_k[ks][0][P + lane], kyc = s_k[ks][1][P + lane];
      const T dx = ykdiff(wA1x, wA2x, wA3x, cm, t, kxc, psc);
      const T dy = ykdiff(wA1y, wA2y, wA3y, ck, t, kyc, psc);
      const unsigned orow = unsigned(o) * unsigned(n);
      T q = e0;
      if (p1mom) q = emission_p1(q, e1, e2, mu, nu);
      if (has_rhs) q = tfma(rsg, rh, q);
      const T rho = q - mu * px - nu * py - dx - dy - sig * psc;
      if constexpr (BST) {
        // float32: the one output `out` (a float32 launch with out_f or psi_f is refused)
        if (a.mode == 0) {
          bstore(a.sign * rho, w_out, bo, orow * 4u);
        } else {
          const T un = psc + qdiv(rho, diag + a.beta * sig);
          bstore(un, w_out, bo, orow * 4u);
          if constexpr (ACC) bstore(y64 + (double(un) - double(float(y64))), w_acc, unsigned(col) * 8u, orow * 8u);
        }
      } else {
        const size_t ro = base + size_t(orow);
        if (a.psi_f) at(a.psi_f + ro, bof) = float(psc);
        if (a.mode == 0) {
          const T val = a.sign * rho;
          if (a.out) at(a.out + ro, bo) = val;
          if (a.out_f) at(a.out_f + ro, bof) = float(val);
          if constexpr (sizeof(T) == 8) acc += double(val) * double(val);
        } else {
          const T un = psc + qdiv(rho, diag + a.beta * sig);
          at(a.out + ro, bo) = un;
          if (ACC) at(a.acc64 + ro, unsigned(col) * 8u) = y64 + (double(un) - double(float(y64)));
        }
      }
    }
    __syncthreads();   // the next step overwrites ring slots read above
  };
  // the interior rows r in [flo, fhi) run the FAST step in whole interior passes (FP rows: two
  // unrolled passes up to P = 2, psi slot t of the pair; else one) aligned to rbeg; the head and
  // tail passes take the psi slot at run time
  constexpr int FP = PS2 ? 2 * W : W;
  const int flo = y0 + 4 * P, fhi = min(n - 1, yend + 4 * P - 1);
  const int f0 = rbeg + FP * ((max(flo - rbeg, 0) + FP - 1) / FP);
  int r0 = rbeg, half = 0, sp = 0, sg = 0;   // sp, sg: run-time slots (without PS2, GS)
  for (; r0 < rend && r0 < f0; r0 += W, half ^= W) {
#pragma unroll
    for (int t = 0; t < W; ++t) {
      if (r0 + t >= rend) break;
      step(r0 + t, t, PS2 ? half + t : sp, GS ? t : sg, std::false_type{});
      if constexpr (!PS2) sp = ring_next(sp, PR);
      if constexpr (!GS) sg = ring_next(sg, GR);
    }
  }
  for (; r0 + FP <= fhi; r0 += FP) {
#pragma unroll
    for (int t = 0; t < FP; ++t) {
      step(r0 + t, t % W, PS2 ? t : sp, GS ? t % W : sg, std::true_type{});
      if constexpr (!PS2) sp = ring_next(sp, PR);
      if constexpr (!GS) sg = ring_next(sg, GR);
    }
  }
  for (; r0 < rend; r0 += W, half ^= W) {
#pragma unroll
    for (int t = 0; t < W; ++t) {
      if (r0 + t >= rend) break;
      step(r0 + t, t, PS2 ? half + t : sp, GS ? t : sg, std::false_type{});
      if constexpr (!PS2) sp = ring_next(sp, PR);
      if constexpr (!GS) sg = ring_next(sg, GR);
    }
  }
  // norms are float64 only (a float32 launch with partial sums is refused by launch_pg)
  if (sizeof(T) == 8 && a.partial) {
    __shared__ double red[kStripW];
    red[lane] = acc;
    __syncthreads();
    for (int st = kStripW / 2; st > 0; st >>= 1) {
      if (lane < st) red[lane] += red[lane + st];
      __syncthreads();
    }
    if (lane == 0) {
      const size_t b = blockIdx.x + size_t(gridDim.x) * (blockIdx.y + size_t(gridDim.y) * blockIdx.z);
      a.partial[b] = red[0] * double(a.L.w[dir]) * a.L.dims.h * a.L.dims.h;
    }
  }
}

// ---------------------------------------------------------------------------------------------
// finest upwind operator (eq. discretised_hfm): rho = q - A_up psi - sigma_t psi
// mode 0: out = sign * rho (to out and / or out_f), with one float64 partial sum of
// w_n h^2 (sign rho)^2 per block when partial is given; mode 1: out = psi + rho / d (a Jacobi sweep).
// Threads are laid out as in the correction sweep below: 64 columns x row groups of R rows,
// each thread walking its rows in the ordinate's downwind y order with every load issued up front
// from clamped addresses, so psi is read once for the centre and once, from cache, as x neighbour.
// A block takes K consecutive ordinates of one face (same signs, so the same walk and upwind
// column): the per-cell emission and sigma_t of its rows are loaded once for all K.
constexpr int kCorrRows = 8;
constexpr int kFullBlock = 256;
// rows per thread of the finest upwind operator: fewer in float64, whose values take two
// registers (eight rows held 212 registers per thread with four ordinates per block: two waves)
template <typename T> constexpr int full_rows() { return sizeof(T) == 8 ? 4 : 8; }
template <typename T, int K>
__device__ __forceinline__ void b_upwind_full(const VBlk& vb, LevelData<T> L, int bc_vac,
                                                            const T* __restrict__ psi,
                                                            const T* __restrict__ E, int nmomE,
                                                            T* __restrict__ out, float* __restrict__ out_f,
                                                            int mode, T sign, const T* __restrict__ rhs,
                                                            double* __restrict__ partial) {
  if (idle(L.dims.active)) return;
  constexpr int R = full_rows<T>();
  const int n = L.dims.n, nd = L.dims.nd;
  const int ntx = (n + 63) >> 6;
  const int tx = int(vb.x) % ntx, ty = int(vb.x) / ntx;
  const int i = tx * 64 + int(threadIdx.x & 63);
  const int jb = (ty * (kFullBlock / 64) + int(threadIdx.x >> 6)) * R;
  const int d0 = int(vb.y) * K, g = vb.z;
  const size_t ncell = size_t(n) * n;
  double acc = 0.0;   // sum over the block's ordinates of w_n (sign rho)^2
  if (i < n && jb < n) {
    const T h = T(L.dims.h);
    const T mu0 = L.mu[d0], nu0 = L.nu[d0];   // signs shared by the K ordinates
    const int je = min(jb + R, n);
    const int iu = mu0 > T(0) ? i - 1 : i + 1;
    const bool x_in = iu >= 0 && iu < n;
    const int iuc = clampi(iu, 0, n - 1);
    const bool xvac = mu0 > T(0) ? (bc_vac & 1) : (bc_vac & 2);
    const bool yvac = nu0 > T(0) ? (bc_vac & 4) : (bc_vac & 8);
    const T* __restrict__ sg = L.sigma_t + size_t(g) * ncell;
    const T* __restrict__ E0 = E + size_t(g) * nmomE * ncell;
    const bool down = nu0 > T(0);
    const int j0 = down ? jb : je - 1;
    const int ju = down ? j0 - 1 : j0 + 1;
    const bool y_in = ju >= 0 && ju < n;
    const int rows = je - jb;
    // per-cell values, once for the K ordinates
    T q0[R], q1[R], q2[R], vs[R];
#pragma unroll
    for (int t = 0; t < R; ++t) {
      const int j = down ? min(j0 + t, je - 1) : max(j0 - t, jb);
      const size_t row = size_t(j) * n;
      q0[t] = E0[row + i];
      vs[t] = sg[row + i];
      q1[t] = q2[t] = T(0);
    }
    if (nmomE > 1) {
#pragma unroll
      for (int t = 0; t < R; ++t) {
        const int j = down ? min(j0 + t, je - 1) : max(j0 - t, jb);
        const size_t row = size_t(j) * n;
        q1[t] = E0[ncell + row + i];
        q2[t] = E0[2 * ncell + row + i];
      }
    }
#pragma unroll 1
    for (int k = 0; k < K; ++k) {   // not unrolled: one ordinate's rows in registers at a time
      const int dir = d0 + k;
      const size_t plane = (size_t(g) * nd + dir) * ncell;
      const T mu = L.mu[dir], nu = L.nu[dir];
      const T amu = tabs(mu) / h, anu = tabs(nu) / h;
      const T* __restrict__ pp = psi + plane;
      const T* __restrict__ rp = rhs ? rhs + plane : pp;
      T vc[R], vx[R], vr[R];
#pragma unroll
      for (int t = 0; t < R; ++t) {
        const int j = down ? min(j0 + t, je - 1) : max(j0 - t, jb);
        const size_t row = size_t(j) * n;
        vc[t] = pp[row + i];
        vx[t] = pp[row + iuc];
        vr[t] = rp[row + i];
      }
      T prev = pp[size_t(clampi(ju, 0, n - 1)) * n + i];   // the upwind row, used only inside the domain
      double acck = 0.0;
#pragma unroll
      for (int t = 0; t < R; ++t) {
        if (t >= rows) break;
        const size_t cell = size_t(down ? j0 + t : j0 - t) * n + i;
        const T pc = vc[t];
        const T px = x_in ? vx[t] : (xvac ? T(0) : pc);
        const T py = (t > 0 || y_in) ? prev : (yvac ? T(0) : pc);
        T q = q0[t];
        if (nmomE > 1) q = emission_p1(q, q1[t], q2[t], mu, nu);
        if (rhs) q += vr[t];
        const T sig = vs[t];
        const T rho = q - amu * (pc - px) - anu * (pc - py) - sig * pc;
        if (mode == 0) {
          const T val = sign * rho;
          if (out) out[plane + cell] = val;
          if (out_f) out_f[plane + cell] = float(val);
          acck += double(val) * double(val);
        } else {
          const T dd = amu + anu + sig;
          out[plane + cell] = pc + qdivr(rho, dd, qrcp(dd));
        }
        prev = pc;
      }
      acc += double(L.w[dir]) * acck;
    }
  }
  if (partial) {
    // block sum in a fixed order (deterministic), one partial per block
    __shared__ double red[kFullBlock];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int st = kFullBlock / 2; st > 0; st >>= 1) {
      if (int(threadIdx.x) < st) red[threadIdx.x] += red[threadIdx.x + st];
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      const size_t b = vb.x + size_t(vb.gx) * (vb.y + size_t(vb.gy) * vb.z);
      partial[b] = red[0] * L.dims.h * L.dims.h;
    }
  }
}
template <typename T, int K>
__global__ __launch_bounds__(kFullBlock) void k_upwind_full(LevelData<T> L, int bc_vac, const T* __restrict__ psi, const T* __restrict__ E, int nmomE, T* __restrict__ out, float* __restrict__ out_f, int mode, T sign, const T* __restrict__ rhs, double* __restrict__ partial) {
  b_upwind_full<T, K>(hw_blk(), L, bc_vac, psi, E, nmomE, out, out_f, mode, sign, rhs, partial);
}

// correction sweep on one level: e_new = e + (rhs - A_up e - sigma_t e) / d
// XMODE 0: e read from xin (same level); 1: e = UpSamp of the next coarser level's xin; 2: e = 0.
// A block is 64 columns x (blockDim / 64) row groups; each thread owns one column of kCorrRows
// rows and walks them in the ordinate's downwind y order, so the upwind y neighbour is the value
// it read one row before (every e value is loaded once for the centre and once, from cache, as an
// x neighbour).  With acc the new value is added to acc instead of being written to xout.
template <typename T, int XMODE, bool SCAT>
__device__ __forceinline__ void b_upwind_corr(const VBlk& vb, LevelData<T> L, int bc_vac,
                                                         const T* __restrict__ xin, int ndc,
                                                         const T* __restrict__ rhs,
                                                         T* __restrict__ xout, T* __restrict__ acc,
                                                         const T* __restrict__ E, int nmomE) {
  if (idle(L.dims.active)) return;
  const int n = L.dims.n, nd = L.dims.nd;
  const int ntx = (n + 63) >> 6;
  const int tx = int(vb.x) % ntx, ty = int(vb.x) / ntx;
  const int i = tx * 64 + int(threadIdx.x & 63);
  const int jb = (ty * int(vb.bd >> 6) + int(threadIdx.x >> 6)) * kCorrRows;
  if (i >= n || jb >= n) return;
  const int je = min(jb + kCorrRows, n);
  const int dir = vb.y, g = vb.z;
  const size_t ncell = size_t(n) * n;
  const size_t plane = (size_t(g) * nd + dir) * ncell;
  const T mu = L.mu[dir], nu = L.nu[dir], h = T(L.dims.h);
  const int iu = mu > T(0) ? i - 1 : i + 1;
  const bool xin_dom = iu >= 0 && iu < n;
  const int iuc = clampi(iu, 0, n - 1);
  const bool xvac = mu > T(0) ? (bc_vac & 1) : (bc_vac & 2);
  const bool yvac = nu > T(0) ? (bc_vac & 4) : (bc_vac & 8);
  const T amu = tabs(mu) / h, anu = tabs(nu) / h;
  const T* __restrict__ sigma = L.sigma_t + size_t(g) * ncell;
  // coarse source of XMODE 1: the parent ordinate's plane on the grid of half the size
  const int nc = n >> 1;
  const T* __restrict__ src = xin;
  if (XMODE == 1)
    src = xin + (size_t(g) * ndc + parent_dir_dev(dir, L.dims.na)) * (size_t(nc) * nc);
  auto value = [&](int jj, int ii) -> T {
    if (XMODE == 0) return xin[plane + size_t(jj) * n + ii];
    if (XMODE == 1) return src[size_t(jj >> 1) * nc + (ii >> 1)];
    return T(0);
  };
  const bool down = nu > T(0);          // upwind row j - 1: walk with increasing j
  const int j0 = down ? jb : je - 1;
  const int ju0 = down ? j0 - 1 : j0 + 1;
  const bool prev_in = ju0 >= 0 && ju0 < n;
  // every load of the thread's rows first (rows past the strip end clamped to its last row, so
  // all loads are in bounds and independent), then the sweep itself
  T ec[kCorrRows], ex[kCorrRows], rh[kCorrRows], sg[kCorrRows], av[kCorrRows], q[kCorrRows];
  // SCAT: the scattering of the correction, E[g][m][cell] (emission of e, no source), as a source
  const T* __restrict__ Eg = SCAT ? E + size_t(g) * nmomE * ncell : nullptr;
#pragma unroll
  for (int t = 0; t < kCorrRows; ++t) {
    const int j = down ? min(j0 + t, je - 1) : max(j0 - t, jb);
    const size_t cell = size_t(j) * n + i;
    ec[t] = value(j, i);
    ex[t] = value(j, iuc);
    rh[t] = rhs[plane + cell];
    sg[t] = sigma[cell];
    av[t] = acc ? acc[plane + cell] : T(0);
    if (SCAT) {
      T qv = Eg[cell];
      if (nmomE > 1) qv += mu * Eg[ncell + cell] + nu * Eg[2 * ncell + cell];
      q[t] = qv;
    }
  }
  T eprev = value(clampi(ju0, 0, n - 1), i);   // used only if that row is inside the domain
  const int rows = je - jb;
#pragma unroll
  for (int t = 0; t < kCorrRows; ++t) {
    if (t >= rows) break;
    const int j = down ? j0 + t : j0 - t;
    const size_t cell = size_t(j) * n + i;
    const T c = ec[t];
    const T x = xin_dom ? ex[t] : (xvac ? T(0) : c);
    const T y = (t > 0 || prev_in) ? eprev : (yvac ? T(0) : c);
    const T sig = sg[t];
    const T r = (SCAT ? rh[t] + q[t] : rh[t]) - amu * (c - x) - anu * (c - y) - sig * c;
    const T dd = amu + anu + sig;
    const T enew = c + qdivr(r, dd, qrcp(dd));
    if (acc) acc[plane + cell] = av[t] + enew;
    else xout[plane + cell] = enew;
    eprev = c;
  }
}
template <typename T, int XMODE, bool SCAT>
__global__ __launch_bounds__(1024) void k_upwind_corr(LevelData<T> L, int bc_vac, const T* __restrict__ xin, int ndc, const T* __restrict__ rhs, T* __restrict__ xout, T* __restrict__ acc, const T* __restrict__ E, int nmomE) {
  b_upwind_corr<T, XMODE, SCAT>(hw_blk(), L, bc_vac, xin, ndc, rhs, xout, acc, E, nmomE);
}

// Two correction sweeps in one pass: e1 = S(e0), e2 = S(e1), S the sweep above without the
// scattering term.  Besides e1 on its own column, each thread forms e1 on the upwind x neighbour
// column (from loads that share cache lines with its own) and, for its first row, on the upwind
// row, so that no intermediate value crosses threads and e1 never goes to memory.  The arithmetic
// of every value is that of the single sweep.  R rows per thread.
template <typename T, int XMODE, int R, int K>
__device__ __forceinline__ void b_upwind_corr2(const VBlk& vb, LevelData<T> L, int bc_vac,
                                                          const T* __restrict__ xin, int ndc,
                                                          const T* __restrict__ rhs,
                                                          T* __restrict__ xout, T* __restrict__ acc) {
  if (idle(L.dims.active)) return;
  const int n = L.dims.n, nd = L.dims.nd;
  const int ntx = (n + 63) >> 6;
  const int tx = int(vb.x) % ntx, ty = int(vb.x) / ntx;
  const int i = tx * 64 + int(threadIdx.x & 63);
  const int jb = (ty * int(vb.bd >> 6) + int(threadIdx.x >> 6)) * R;
  if (i >= n || jb >= n) return;
  const int je = min(jb + R, n);
  const int d0 = int(vb.y) * K, g = vb.z;
  const size_t ncell = size_t(n) * n;
  const T h = T(L.dims.h);
  const T mu0 = L.mu[d0], nu0 = L.nu[d0];   // signs shared by the K ordinates of the block
  const int sx = mu0 > T(0) ? 1 : -1;
  const int iu = i - sx, iuu = i - 2 * sx;
  const bool x1 = iu >= 0 && iu < n, x2 = iuu >= 0 && iuu < n;
  const int iuc = clampi(iu, 0, n - 1), iuuc = clampi(iuu, 0, n - 1);
  const bool xvac = mu0 > T(0) ? (bc_vac & 1) : (bc_vac & 2);
  const bool yvac = nu0 > T(0) ? (bc_vac & 4) : (bc_vac & 8);
  const T* __restrict__ sigma = L.sigma_t + size_t(g) * ncell;
  const int nc = n >> 1;
  const bool down = nu0 > T(0);
  const int j0 = down ? jb : je - 1;
  const int ju0 = down ? j0 - 1 : j0 + 1, juu0 = down ? j0 - 2 : j0 + 2;
  const bool y1 = ju0 >= 0 && ju0 < n, y2 = juu0 >= 0 && juu0 < n;
  const int juc = clampi(ju0, 0, n - 1), juuc = clampi(juu0, 0, n - 1);
  const int rows = je - jb;
  // sigma_t of the rows (own and upwind column) and of the upwind row, once for the K ordinates
  // (in-plane offsets are 32-bit: n <= 32768)
  T sc[R], sxv[R];
#pragma unroll
  for (int t = 0; t < R; ++t) {
    const int j = down ? min(j0 + t, je - 1) : max(j0 - t, jb);
    const unsigned row = unsigned(j) * unsigned(n);
    sc[t] = sigma[row + i];
    sxv[t] = sigma[row + iuc];
  }
  const T hs = sigma[unsigned(juc) * unsigned(n) + i];
#pragma unroll 1
  for (int k = 0; k < K; ++k) {   // not unrolled: one ordinate's rows in registers at a time
    const int dir = d0 + k;
    const size_t plane = (size_t(g) * nd + dir) * ncell;
    const T mu = L.mu[dir], nu = L.nu[dir];
    const T amu = tabs(mu) / h, anu = tabs(nu) / h;
    const T* __restrict__ rp = rhs + plane;
    const T* __restrict__ xp = XMODE == 0 ? xin + plane : xin;
    T* __restrict__ op = acc ? acc + plane : xout + plane;
    const T* __restrict__ src = xin;
    if (XMODE == 1)
      src = xin + (size_t(g) * ndc + parent_dir_dev(dir, L.dims.na)) * (size_t(nc) * nc);
    auto value = [&](int jj, int ii) -> T {
      if (XMODE == 0) return xp[unsigned(jj) * unsigned(n) + ii];
      if (XMODE == 1) return src[size_t(jj >> 1) * nc + (ii >> 1)];
      return T(0);
    };
    auto sweep = [&](T c, T x, T y, T r, T sig, T d, T rd) -> T {
      const T rr = r - amu * (c - x) - anu * (c - y) - sig * c;
      return c + qdivr(rr, d, rd);
    };
    T ec[R], ex[R], exx[R], rc[R], rx[R], av[R];
#pragma unroll
    for (int t = 0; t < R; ++t) {
      const int j = down ? min(j0 + t, je - 1) : max(j0 - t, jb);
      const unsigned row = unsigned(j) * unsigned(n);
      ec[t] = value(j, i);
      ex[t] = value(j, iuc);
      exx[t] = value(j, iuuc);
      rc[t] = rp[row + i];
      rx[t] = rp[row + iuc];
      av[t] = acc ? op[row + i] : T(0);
    }
    // the upwind row (its values are used only when it lies inside the domain)
    const T hc = value(juc, i), hx = value(juc, iuc), hh = value(juuc, i);
    const T hr = rp[unsigned(juc) * unsigned(n) + i];
    const T dh = amu + anu + hs;
    T e1prev = sweep(hc, x1 ? hx : (xvac ? T(0) : hc), y2 ? hh : (yvac ? T(0) : hc), hr, hs, dh, qrcp(dh));
    T e0c_prev = hc, e0x_prev = hx;
#pragma unroll
    for (int t = 0; t < R; ++t) {
      if (t >= rows) break;
      const int j = down ? j0 + t : j0 - t;
      const bool yin = t > 0 || y1;
      const T c = ec[t], cx = ex[t];
      // one reciprocal per cell: the two sweeps at (i, j) share it
      const T dc = amu + anu + sc[t], dx = amu + anu + sxv[t];
      const T rdc = qrcp(dc), rdx = qrcp(dx);
      const T e1c = sweep(c, x1 ? cx : (xvac ? T(0) : c), yin ? e0c_prev : (yvac ? T(0) : c), rc[t], sc[t], dc, rdc);
      const T e1x = sweep(cx, x2 ? exx[t] : (xvac ? T(0) : cx), yin ? e0x_prev : (yvac ? T(0) : cx), rx[t], sxv[t],
                          dx, rdx);
      const T e2 = sweep(e1c, x1 ? e1x : (xvac ? T(0) : e1c), yin ? e1prev : (yvac ? T(0) : e1c), rc[t], sc[t], dc,
                         rdc);
      const unsigned cell = unsigned(j) * unsigned(n) + i;
      op[cell] = acc ? av[t] + e2 : e2;
      e0c_prev = c;
      e0x_prev = cx;
      e1prev = e1c;
    }
  }
}
template <typename T, int XMODE, int R, int K>
__global__ __launch_bounds__(K == 1 ? 1024 : 256) void k_upwind_corr2(LevelData<T> L, int bc_vac, const T* __restrict__ xin, int ndc, const T* __restrict__ rhs, T* __restrict__ xout, T* __restrict__ acc) {
  b_upwind_corr2<T, XMODE, R, K>(hw_blk(), L, bc_vac, xin, ndc, rhs, xout, acc);
}

// restriction: coarse = sum_{child ordinates, 2x2 cells} w_n rho h^2 / (w_N H^2)
template <typename T>
__device__ __forceinline__ void b_restrict(const VBlk& vb, LevelData<T> Lf, LevelData<T> Lc,
                                                      const T* __restrict__ fine,
                                                      T* __restrict__ coarse) {
  if (idle(Lf.dims.active)) return;
  const int nc = Lc.dims.n, ndc = Lc.dims.nd, nf = Lf.dims.n, naf = Lf.dims.na;
  const size_t nccell = size_t(nc) * nc, nfcell = size_t(nf) * nf;
  const int cell = int(vb.x) * kBlock + int(threadIdx.x);
  if (cell >= int(nccell)) return;
  const int N = vb.y, g = vb.z;
  const size_t idx = (size_t(g) * ndc + N) * nccell + cell;
  const int J = cell / nc, I = cell - J * nc;
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
__global__ __launch_bounds__(kBlock) void k_restrict(LevelData<T> Lf, LevelData<T> Lc, const T* __restrict__ fine, T* __restrict__ coarse) {
  b_restrict<T>(hw_blk(), Lf, Lc, fine, coarse);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_prolong(LevelData<T> Lf, int ndc,
                                                     const T* __restrict__ coarse,
                                                     T* __restrict__ fine) {
  const int n = Lf.dims.n, nd = Lf.dims.nd;
  const size_t ncell = size_t(n) * n;
  const int cell = int(blockIdx.x) * kBlock + int(threadIdx.x);
  if (cell >= int(ncell)) return;
  const int dir = blockIdx.y, g = blockIdx.z;
  const size_t idx = (size_t(g) * nd + dir) * ncell + cell;
  const int j = cell / n, i = cell - j * n;
  const int nc = n >> 1;
  fine[idx] = coarse[(size_t(g) * ndc + parent_dir_dev(dir, Lf.dims.na)) *
                         (size_t(nc) * nc) + size_t(j >> 1) * nc + (i >> 1)];
}

// weighted squared norm, two deterministic passes
constexpr int kNormBlocks = 1024;

template <typename T>
__global__ __launch_bounds__(kBlock) void k_wnorm2_partial(LevelData<T> L, const T* __restrict__ v,
                                                            double* __restrict__ partial) {
  if (idle(L.dims.active)) return;
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

__device__ __forceinline__ void b_sum_partials(const VBlk& vb, const double* __restrict__ partial, int np,
                                                          double* __restrict__ out, const int* active) {
  if (idle(active)) return;
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
__global__ __launch_bounds__(kBlock) void k_sum_partials(const double* __restrict__ partial, int np, double* __restrict__ out, const int* active) {
  b_sum_partials(hw_blk(), partial, np, out, active);
}

// first stage of a long sum: block b adds the b-th of kSumBlocks contiguous chunks (fixed order)
constexpr int kSumBlocks = 256;
__device__ __forceinline__ void b_sum_chunks(const VBlk& vb, const double* __restrict__ partial, int np,
                                                        double* __restrict__ stage, const int* active) {
  if (idle(active)) return;
  __shared__ double red[kBlock];
  const int chunk = (np + kSumBlocks - 1) / kSumBlocks;
  const int beg = int(vb.x) * chunk, end = min(beg + chunk, np);
  double acc = 0.0;
  for (int i = beg + int(threadIdx.x); i < end; i += kBlock) acc += partial[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) stage[vb.x] = red[0];
}
__global__ __launch_bounds__(kBlock) void k_sum_chunks(const double* __restrict__ partial, int np, double* __restrict__ stage, const int* active) {
  b_sum_chunks(hw_blk(), partial, np, stage, active);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_axpy(T* __restrict__ y, const T* __restrict__ x, T a,
                                                  size_t n, const int* active) {
  if (idle(active)) return;
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
                                                 size_t n, const int* active) {
  if (idle(active)) return;
  const size_t i = size_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i < n) out[i] = float(in[i]);
}
__global__ __launch_bounds__(kBlock) void k_f2d(const float* __restrict__ in, double* __restrict__ out,
                                                 size_t n) {
  const size_t i = size_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i < n) out[i] = double(in[i]);
}
__device__ __forceinline__ void b_add_f2d(const VBlk& vb, double* __restrict__ y, const float* __restrict__ x,
                                                     size_t n, const int* active) {
  if (idle(active)) return;
  const size_t i = size_t(vb.x) * kBlock + threadIdx.x;
  if (i < n) y[i] += double(x[i]);
}
__global__ __launch_bounds__(kBlock) void k_add_f2d(double* __restrict__ y, const float* __restrict__ x, size_t n, const int* active) {
  b_add_f2d(hw_blk(), y, x, n, active);
}

// y += u - fl32(y): the full-approximation update, with the float32 start value re-derived from y
__global__ __launch_bounds__(kBlock) void k_add_diff_f2d(double* __restrict__ y, const float* __restrict__ u,
                                                          size_t n, const int* active) {
  if (idle(active)) return;
  const size_t i = size_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i < n) {
    const double yi = y[i];
    y[i] = yi + (double(u[i]) - double(float(yi)));
  }
}

__global__ void k_update_active(const double* __restrict__ norm2, double bnorm, double rtol,
                                double* __restrict__ rel, int* __restrict__ active, double* __restrict__ steps) {
  if (threadIdx.x != 0 || *active == 0) return;
  const double r = sqrt(norm2[0]) / bnorm;
  rel[0] = r;
  const int on = (r > rtol || r != r) ? 1 : 0;
  *active = on;
  if (on && steps) steps[0] += 1.0;
}

__global__ void k_set_int(int* p, int v) {
  if (threadIdx.x == 0) *p = v;
}

template <typename T>
__device__ __forceinline__ void b_copy(const VBlk& vb, T* __restrict__ dst, const T* __restrict__ src, size_t n,
                                                  const int* active) {
  if (idle(active)) return;
  const size_t i = size_t(vb.x) * kBlock + threadIdx.x;
  if (i < n) dst[i] = src[i];
}
template <typename T>
__global__ __launch_bounds__(kBlock) void k_copy(T* __restrict__ dst, const T* __restrict__ src, size_t n, const int* active) {
  b_copy<T>(hw_blk(), dst, src, n, active);
}

inline unsigned nblocks(size_t total) { return unsigned((total + kBlock - 1) / kBlock); }

}  // namespace

// ---------------------------------------------------------------------------------------------
// Recording for the persistent batched solve.  While a tape is open on the calling thread, the
// launchers of the upwind solve path append one operation (kind, template choice, grid and
// arguments) to it instead of launching, and every other launcher fails with
// hipErrorNotSupported.  Recorded arguments carry no activity flag: the persistent kernel skips
// the operations of a converged problem itself.  Sweeps are recorded at 256 threads per block
// (the block shape changes no arithmetic).
enum PKind : int { P_MOM, P_MOM_MFMA, P_EMIS, P_UPF, P_CORR, P_CORR2, P_RESTRICT, P_SUMCH, P_SUMP, P_ACTIVE,
                   P_COPY, P_ADDF2D };

template <typename T> struct AMom { LevelData<T> L; const T* psi; T* phi; int nmom; };
template <typename T> struct AEmis { LevelDims d; const T* phi; const T* ss; int nl; const T* src; T* E; int coarse; };
template <typename T> struct AUpf {
  LevelData<T> L; int bc_vac; const T* psi; const T* E; int nmomE; T* out; float* out_f; int mode; T sign;
  const T* rhs; double* partial;
};
template <typename T> struct ACorr { LevelData<T> L; int bc_vac; const T* xin; int ndc; const T* rhs; T* xout; T* acc; };
template <typename T> struct ARestrict { LevelData<T> Lf, Lc; const T* fine; T* coarse; };
struct ASum { const double* partial; int np; double* out; };
struct AActive { const double* norm2; double bnorm, rtol; double* rel; int* active; double* steps; };
template <typename T> struct ACopy { T* dst; const T* src; size_t n; };
struct AAddF2D { double* y; const float* x; size_t n; };

constexpr int kOpArgBytes = 176;
struct alignas(16) POp {
  int kind, fp64, xmode, kb;       // kb: ordinates per block of the upwind operator / paired sweep
  unsigned gx, gy, gz, tiles;      // the operation's grid; a tile is one block of it
  unsigned chunk, items;           // tiles per work item, work items
  unsigned long long before;       // work items of the problem's step ahead of this operation
  unsigned char arg[kOpArgBytes];  // one of the argument structs above
};

}  // namespace ctf

struct ctf::PersistTape {
  std::vector<POp> ops;
  int* active = nullptr;  // the problem's activity flag (argument of its update operation)
  bool bad = false;       // a launcher that cannot be recorded was called
};

namespace ctf {

namespace {
thread_local PersistTape* g_tape = nullptr;

template <typename A>
hipError_t tape_add(int kind, int fp64, int xmode, int kb, dim3 grid, const A& a) {
  static_assert(sizeof(A) <= kOpArgBytes, "operation arguments too large");
  static_assert(std::is_trivially_copyable<A>::value, "operation arguments must be plain data");
  POp op{};
  op.kind = kind;
  op.fp64 = fp64;
  op.xmode = xmode;
  op.kb = kb;
  op.gx = grid.x;
  op.gy = grid.y;
  op.gz = grid.z;
  op.tiles = grid.x * grid.y * grid.z;
  std::memcpy(op.arg, &a, sizeof(A));
  g_tape->ops.push_back(op);
  return hipSuccess;
}

hipError_t tape_refuse() {
  g_tape->bad = true;
  return hipErrorNotSupported;
}

template <typename T>
LevelData<T> no_flag(LevelData<T> L) {
  L.dims.active = nullptr;
  return L;
}
}  // namespace

PersistTape* tape_open() {
  g_tape = new PersistTape();
  return g_tape;
}
void tape_close() { g_tape = nullptr; }
void tape_free(PersistTape* t) { delete t; }
bool tape_usable(const PersistTape* t) { return t && !t->bad && t->active && !t->ops.empty(); }

// ---------------------------------------------------------------------------------------------
template <typename T>
hipError_t launch_moments(const LevelData<T>& L, const T* psi, T* phi, int nmom, hipStream_t s) {
  const int ncell = L.dims.n * L.dims.n;
  const dim3 grid((ncell + kMomCells - 1) / kMomCells, L.dims.G);
  if (g_tape) return tape_add(P_MOM, sizeof(T) == 8, 0, 0, grid, AMom<T>{no_flag(L), psi, phi, nmom});
  hipLaunchKernelGGL(k_moments<T>, grid, dim3(kBlock), 0, s, L, psi, phi, nmom);
  return hipGetLastError();
}

hipError_t launch_moments_mfma(const LevelData<float>& L, const float* psi, float* phi, int nmom,
                               hipStream_t s) {
  const int ncell = L.dims.n * L.dims.n;
  const dim3 grid((ncell + 63) / 64, L.dims.G);
  if (g_tape) return tape_add(P_MOM_MFMA, 0, 0, 0, grid, AMom<float>{no_flag(L), psi, phi, nmom});
  hipLaunchKernelGGL(k_moments_mfma, grid, dim3(kBlock), 0, s, L, psi, phi, nmom);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_emission(const LevelDims& d, const T* phi, const T* ss, int nl, const T* src,
                           T* E, hipStream_t s, int phi_coarse) {
  const size_t ncell = size_t(d.n) * d.n;
  const dim3 grid(nblocks(ncell), d.G);
  if (g_tape) {
    LevelDims dn = d;
    dn.active = nullptr;
    return tape_add(P_EMIS, sizeof(T) == 8, 0, 0, grid, AEmis<T>{dn, phi, ss, nl, src, E, phi_coarse});
  }
  hipLaunchKernelGGL(k_emission<T>, grid, dim3(kBlock), 0, s, d, phi, ss, nl, src, E, phi_coarse);
  return hipGetLastError();
}

// Kernel template code of the diffusivity: 0 anisotropic (eq. ano-k, mixed-mass R_x, R_y); the
// isotropic form with R from the mixed mass (3), the degree P - 1 estimate (1) or the degree
// P + 1 estimate (2).
int pg_re(const PGParams& pp) { return pp.isotropic ? (pp.r_estimate ? pp.r_estimate : 3) : 0; }

template <typename T>
PGArgs<T> pg_args(const LevelData<T>& L, const Stencils<T>& st, const PGParams& pp, const PGLaunch<T>& o) {
  PGArgs<T> a{};
  a.L = L;
  a.st = st;
  a.alpha_r = T(pp.alpha_r);
  a.eps_k = T(pp.eps_k);
  a.akabs = T(pp.alpha_kabs);
  a.aksq = T(pp.alpha_ksq);
  a.beta = T(pp.beta);
  a.bc_vac = pp.bc_vac;
  a.psi = o.psi;
  a.E = o.E;
  a.nmomE = o.nmomE;
  a.rhs = o.rhs;
  a.rhs_sign = o.rhs_sign;
  a.mode = o.mode;
  a.sign = o.sign;
  a.strip_h = o.strip_h;
  a.psi_f = o.psi_f;
  a.acc64 = o.acc64;
  return a;
}

template <typename T>
hipError_t launch_pg_diffusivity(int p, const LevelData<T>& L, const Stencils<T>& st, const PGParams& pp,
                                 const PGLaunch<T>& o, hipStream_t s) {
  if (g_tape) return tape_refuse();
  if (!o.kx_out || !o.ky_out) return hipErrorInvalidValue;
  PGArgs<T> a = pg_args(L, st, pp, o);
  a.kx_out = o.kx_out;
  a.ky_out = o.ky_out;
  a.kx_out_f = o.kx_out_f;
  a.ky_out_f = o.ky_out_f;
  const int n = L.dims.n;
  const int ow = kStripW - 2 * p;
  a.ntx = (n + ow - 1) / ow;
  const dim3 grid(a.ntx * ((n + a.strip_h - 1) / a.strip_h), L.dims.nd, L.dims.G);
  if (pp.r_estimate && !pp.isotropic) return hipErrorInvalidValue;
  switch (p * 4 + pg_re(pp)) {
    case 4: hipLaunchKernelGGL((k_pg_diffusivity<1, 0, T>), grid, dim3(kStripW), 0, s, a); break;
    case 8: hipLaunchKernelGGL((k_pg_diffusivity<2, 0, T>), grid, dim3(kStripW), 0, s, a); break;
    case 12: hipLaunchKernelGGL((k_pg_diffusivity<3, 0, T>), grid, dim3(kStripW), 0, s, a); break;
    case 16: hipLaunchKernelGGL((k_pg_diffusivity<4, 0, T>), grid, dim3(kStripW), 0, s, a); break;
    case 7: hipLaunchKernelGGL((k_pg_diffusivity<1, 3, T>), grid, dim3(kStripW), 0, s, a); break;
    case 11: hipLaunchKernelGGL((k_pg_diffusivity<2, 3, T>), grid, dim3(kStripW), 0, s, a); break;
    case 15: hipLaunchKernelGGL((k_pg_diffusivity<3, 3, T>), grid, dim3(kStripW), 0, s, a); break;
    case 19: hipLaunchKernelGGL((k_pg_diffusivity<4, 3, T>), grid, dim3(kStripW), 0, s, a); break;
    case 9: hipLaunchKernelGGL((k_pg_diffusivity<2, 1, T>), grid, dim3(kStripW), 0, s, a); break;
    case 13: hipLaunchKernelGGL((k_pg_diffusivity<3, 1, T>), grid, dim3(kStripW), 0, s, a); break;
    case 17: hipLaunchKernelGGL((k_pg_diffusivity<4, 1, T>), grid, dim3(kStripW), 0, s, a); break;
    case 6: hipLaunchKernelGGL((k_pg_diffusivity<1, 2, T>), grid, dim3(kStripW), 0, s, a); break;
    case 10: hipLaunchKernelGGL((k_pg_diffusivity<2, 2, T>), grid, dim3(kStripW), 0, s, a); break;
    case 14: hipLaunchKernelGGL((k_pg_diffusivity<3, 2, T>), grid, dim3(kStripW), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_pg(int p, const LevelData<T>& L, const Stencils<T>& st, const PGParams& pp,
                     const PGLaunch<T>& o, hipStream_t s) {
  if (g_tape) return tape_refuse();
  if (sizeof(T) == 4 && o.partial) return hipErrorInvalidValue;   // the float32 kernels form no norms
  // the float32 kernels write their one output plane `out`
  if (sizeof(T) == 4 && (!o.out || o.out_f || o.psi_f)) return hipErrorInvalidValue;
  PGArgs<T> a = pg_args(L, st, pp, o);
  const int n = L.dims.n;
  if (!o.kx_in && !o.kx_out && !o.kx_out_f) {
    // fused: the diffusivities of psi are formed on the fly
    if (pp.r_estimate && !pp.isotropic) return hipErrorInvalidValue;
    a.out = o.out;
    a.out_f = o.out_f;
    a.partial = o.partial;
    const int ow = kStripW - 4 * p;
    a.ntx = (n + ow - 1) / ow;
    const dim3 grid(a.ntx * ((n + a.strip_h - 1) / a.strip_h), L.dims.nd, L.dims.G);
    if (o.npartial) *o.npartial = int(grid.x * grid.y * grid.z);
    if (a.acc64 && a.mode != 1) return hipErrorInvalidValue;
#define CTF_FUSED(PP, RE) \
  if (acc) hipLaunchKernelGGL((k_pg_fused<PP, RE, T, true>), grid, dim3(kStripW), 0, s, a); \
  else hipLaunchKernelGGL((k_pg_fused<PP, RE, T, false>), grid, dim3(kStripW), 0, s, a)
    const bool acc = a.acc64 != nullptr;
    switch (p * 4 + pg_re(pp)) {
      case 4: CTF_FUSED(1, 0); break;
      case 8: CTF_FUSED(2, 0); break;
      case 12: CTF_FUSED(3, 0); break;
      case 16: CTF_FUSED(4, 0); break;
      case 7: CTF_FUSED(1, 3); break;
      case 11: CTF_FUSED(2, 3); break;
      case 15: CTF_FUSED(3, 3); break;
      case 19: CTF_FUSED(4, 3); break;
      case 9: CTF_FUSED(2, 1); break;
      case 13: CTF_FUSED(3, 1); break;
      case 17: CTF_FUSED(4, 1); break;
      case 6: CTF_FUSED(1, 2); break;
      case 10: CTF_FUSED(2, 2); break;
      case 14: CTF_FUSED(3, 2); break;
      default: return hipErrorInvalidValue;
    }
#undef CTF_FUSED
    return hipGetLastError();
  }
  if (!o.kx_in) {
    // diffusivities of psi first (into kx_out / ky_out, and their float copies if asked)
    const hipError_t e = launch_pg_diffusivity(p, L, st, pp, o, s);
    if (e != hipSuccess) return e;
    a.kx_in = o.kx_out;
    a.ky_in = o.ky_out;
  } else {
    a.kx_in = o.kx_in;
    a.ky_in = o.ky_in;
  }
  a.out = o.out;
  a.out_f = o.out_f;
  a.partial = o.partial;
  a.ntx = (n + kStripW - 1) / kStripW;
  const dim3 grid(a.ntx * ((n + a.strip_h - 1) / a.strip_h), L.dims.nd, L.dims.G);
  if (o.npartial) *o.npartial = int(grid.x * grid.y * grid.z);
  if (a.acc64 && a.mode != 1) return hipErrorInvalidValue;
#define CTF_STREAM(PP, A) hipLaunchKernelGGL((k_pg_stream<PP, T, A>), grid, dim3(kStripW), 0, s, a)
  const bool acc = a.acc64 != nullptr;
  switch (p) {
    case 1: if (acc) CTF_STREAM(1, true); else CTF_STREAM(1, false); break;
    case 2: if (acc) CTF_STREAM(2, true); else CTF_STREAM(2, false); break;
    case 3: if (acc) CTF_STREAM(3, true); else CTF_STREAM(3, false); break;
    case 4: if (acc) CTF_STREAM(4, true); else CTF_STREAM(4, false); break;
    default: return hipErrorInvalidValue;
  }
#undef CTF_STREAM
  return hipGetLastError();
}

size_t pg_partials(const LevelDims& d, int strip_h) {
  // the fused kernel's strips are the narrowest (64 - 4P columns, P <= 3)
  const int ow = kStripW - 4 * kMaxP;
  const size_t strips = size_t((d.n + ow - 1) / ow) * ((d.n + strip_h - 1) / strip_h);
  return strips * d.nd * d.G;
}

size_t upwind_full_blocks(const LevelDims& d) {   // the larger count of the two precisions
  const int rows_per_block = (kFullBlock / 64) * full_rows<double>();
  return size_t((d.n + 63) / 64) * ((d.n + rows_per_block - 1) / rows_per_block) * d.nd * d.G;
}

template <typename T>
hipError_t launch_upwind_full(const LevelData<T>& L, int bc_vac, const T* psi, const T* E, int nmomE,
                              T* out, int mode, T sign, const T* rhs, hipStream_t s, float* out_f,
                              double* partial, size_t partial_cap, int* npartial) {
  const int n = L.dims.n;
  const int rows_per_block = (kFullBlock / 64) * full_rows<T>();
  // ordinates per block: four when a face holds a multiple of four (n_dir = 8 or 4 faces of na^2)
  const int per_face = L.dims.na * L.dims.na;
  const int kb = per_face % 4 == 0 ? 4 : 1;
  const dim3 grid(unsigned((n + 63) / 64) * unsigned((n + rows_per_block - 1) / rows_per_block),
                  unsigned(L.dims.nd / kb), L.dims.G);
  const size_t blocks = size_t(grid.x) * grid.y * grid.z;
  if (partial && blocks > partial_cap) return hipErrorInvalidValue;
  if (mode == 0 && !out && !out_f) return hipErrorInvalidValue;
  if (L.dims.nd % per_face) return hipErrorInvalidValue;
  if (npartial) *npartial = int(blocks);
  if (g_tape)
    return tape_add(P_UPF, sizeof(T) == 8, 0, kb, grid,
                    AUpf<T>{no_flag(L), bc_vac, psi, E, nmomE, out, out_f, mode, sign, rhs, partial});
  if (kb == 4)
    hipLaunchKernelGGL((k_upwind_full<T, 4>), grid, dim3(kFullBlock), 0, s, L, bc_vac, psi, E, nmomE, out, out_f,
                       mode, sign, rhs, partial);
  else
    hipLaunchKernelGGL((k_upwind_full<T, 1>), grid, dim3(kFullBlock), 0, s, L, bc_vac, psi, E, nmomE, out, out_f,
                       mode, sign, rhs, partial);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_upwind_correction(const LevelData<T>& L, int bc_vac, const T* x_in, int xmode,
                                    int ndc, const T* rhs, T* x_out, T* psi_acc, hipStream_t s, int block,
                                    const T* E, int nmomE) {
  if (g_tape) {
    if (E) return tape_refuse();   // the scattering-coupled sweep is not recorded
    block = kBlock;
  }
  if (block < 64 || block > 1024 || block % 64) return hipErrorInvalidValue;
  const int n = L.dims.n;
  const int rows_per_block = (block / 64) * kCorrRows;
  const unsigned nb = unsigned((n + 63) / 64) * unsigned((n + rows_per_block - 1) / rows_per_block);
  const dim3 grid(nb, L.dims.nd, L.dims.G), blk(block);
  if (g_tape)
    return tape_add(P_CORR, sizeof(T) == 8, xmode, 1, grid,
                    ACorr<T>{no_flag(L), bc_vac, x_in, ndc, rhs, x_out, psi_acc});
#define CTF_CORR(X, S) hipLaunchKernelGGL((k_upwind_corr<T, X, S>), grid, blk, 0, s, L, bc_vac, x_in, ndc, rhs, \
                                          x_out, psi_acc, E, nmomE)
  if (E) {
    if (xmode == 0) CTF_CORR(0, true);
    else if (xmode == 1) CTF_CORR(1, true);
    else CTF_CORR(2, true);
  } else {
    if (xmode == 0) CTF_CORR(0, false);
    else if (xmode == 1) CTF_CORR(1, false);
    else CTF_CORR(2, false);
  }
#undef CTF_CORR
  return hipGetLastError();
}

// rows per thread of the two-sweep kernel (fewer for float64, whose values take two registers)
template <typename T> constexpr int corr2_rows() { return sizeof(T) == 8 ? 4 : 8; }

template <typename T>
hipError_t launch_upwind_correction2(const LevelData<T>& L, int bc_vac, const T* x_in, int xmode, int ndc,
                                     const T* rhs, T* x_out, T* psi_acc, hipStream_t s, int block) {
  if (g_tape) block = kBlock;
  if (block < 64 || block > 1024 || block % 64) return hipErrorInvalidValue;
  constexpr int R = corr2_rows<T>();
  const int n = L.dims.n;
  // float64: four ordinates per block when a face holds a multiple of four (sigma_t loaded once for
  // them; measured 7% faster at 1024^2 x 512).  float32 keeps one: the blocked form's registers
  // halve its occupancy, which cost more than the saved loads (measured 26% slower).
  const int per_face = L.dims.na * L.dims.na;
  if (L.dims.nd % per_face) return hipErrorInvalidValue;
  const int kb = (sizeof(T) == 8 && per_face % 4 == 0) ? 4 : 1;
  if (kb == 4) block = min(block, 256);   // the blocked form keeps more per thread: at most 256 threads
  const int rows_pb = (block / 64) * R;
  const unsigned nb = unsigned((n + 63) / 64) * unsigned((n + rows_pb - 1) / rows_pb);
  const dim3 grid(nb, unsigned(L.dims.nd / kb), L.dims.G), blk(block);
  if (g_tape)
    return tape_add(P_CORR2, sizeof(T) == 8, xmode, kb, grid,
                    ACorr<T>{no_flag(L), bc_vac, x_in, ndc, rhs, x_out, psi_acc});
#define CTF_CORR2(X, KK) hipLaunchKernelGGL((k_upwind_corr2<T, X, R, KK>), grid, blk, 0, s, L, bc_vac, x_in, ndc, \
                                            rhs, x_out, psi_acc)
  if (kb == 4) {
    if (xmode == 0) CTF_CORR2(0, 4);
    else if (xmode == 1) CTF_CORR2(1, 4);
    else CTF_CORR2(2, 4);
  } else {
    if (xmode == 0) CTF_CORR2(0, 1);
    else if (xmode == 1) CTF_CORR2(1, 1);
    else CTF_CORR2(2, 1);
  }
#undef CTF_CORR2
  return hipGetLastError();
}

template <typename T>
hipError_t launch_restrict(const LevelData<T>& Lf, const LevelData<T>& Lc, const T* fine, T* coarse,
                           hipStream_t s) {
  const dim3 grid(nblocks(size_t(Lc.dims.n) * Lc.dims.n), Lc.dims.nd, Lc.dims.G);
  if (g_tape)
    return tape_add(P_RESTRICT, sizeof(T) == 8, 0, 0, grid, ARestrict<T>{no_flag(Lf), no_flag(Lc), fine, coarse});
  hipLaunchKernelGGL(k_restrict<T>, grid, dim3(kBlock), 0, s, Lf, Lc, fine, coarse);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_prolong(const LevelData<T>& Lf, int ndc, const T* coarse, T* fine, hipStream_t s) {
  if (g_tape) return tape_refuse();
  const dim3 grid(nblocks(size_t(Lf.dims.n) * Lf.dims.n), Lf.dims.nd, Lf.dims.G);
  hipLaunchKernelGGL(k_prolong<T>, grid, dim3(kBlock), 0, s, Lf, ndc, coarse, fine);
  return hipGetLastError();
}

int wnorm2_partials(const LevelDims&) { return kNormBlocks; }

template <typename T>
hipError_t launch_wnorm2(const LevelData<T>& L, const T* v, double* partial, int npartial,
                         double* out, hipStream_t s) {
  if (g_tape) return tape_refuse();
  hipLaunchKernelGGL(k_wnorm2_partial<T>, dim3(npartial), dim3(kBlock), 0, s, L, v, partial);
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kBlock), 0, s, partial, npartial, out, L.dims.active);
  return hipGetLastError();
}

int sum_partials_extra() { return kSumBlocks; }

hipError_t launch_sum_partials(double* partial, int np, double* out, hipStream_t s, const int* active) {
  if (g_tape) {
    if (np > 16 * kBlock) {
      (void)tape_add(P_SUMCH, 1, 0, 0, dim3(kSumBlocks), ASum{partial, np, partial + np});
      return tape_add(P_SUMP, 1, 0, 0, dim3(1), ASum{partial + np, kSumBlocks, out});
    }
    return tape_add(P_SUMP, 1, 0, 0, dim3(1), ASum{partial, np, out});
  }
  if (np > 16 * kBlock) {
    // two stages: kSumBlocks chunk sums after the np partials, then their sum
    double* stage = partial + np;
    hipLaunchKernelGGL(k_sum_chunks, dim3(kSumBlocks), dim3(kBlock), 0, s, partial, np, stage, active);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kBlock), 0, s, stage, kSumBlocks, out, active);
  } else {
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kBlock), 0, s, partial, np, out, active);
  }
  return hipGetLastError();
}

hipError_t launch_update_active(const double* norm2, double bnorm, double rtol, double* rel, int* active,
                                double* steps, hipStream_t s) {
  if (g_tape) {
    if (g_tape->active && g_tape->active != active) return tape_refuse();
    g_tape->active = active;
    return tape_add(P_ACTIVE, 1, 0, 0, dim3(1), AActive{norm2, bnorm, rtol, rel, active, steps});
  }
  hipLaunchKernelGGL(k_update_active, dim3(1), dim3(64), 0, s, norm2, bnorm, rtol, rel, active, steps);
  return hipGetLastError();
}

hipError_t launch_set_int(int* p, int v, hipStream_t s) {
  if (g_tape) return tape_refuse();
  hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, s, p, v);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_copy(T* dst, const T* src, size_t n, hipStream_t s, const int* active) {
  if (g_tape) return tape_add(P_COPY, sizeof(T) == 8, 0, 0, dim3(nblocks(n)), ACopy<T>{dst, src, n});
  hipLaunchKernelGGL(k_copy<T>, dim3(nblocks(n)), dim3(kBlock), 0, s, dst, src, n, active);
  return hipGetLastError();
}
template hipError_t launch_copy<double>(double*, const double*, size_t, hipStream_t, const int*);
template hipError_t launch_copy<float>(float*, const float*, size_t, hipStream_t, const int*);

template <typename T>
hipError_t launch_axpy(T* y, const T* x, T a, size_t n, hipStream_t s, const int* active) {
  if (g_tape) return tape_refuse();
  hipLaunchKernelGGL(k_axpy<T>, dim3(nblocks(n)), dim3(kBlock), 0, s, y, x, a, n, active);
  return hipGetLastError();
}

hipError_t launch_harmonic_coarsen(const double* fine, double* coarse, int G, int nc, hipStream_t s) {
  if (g_tape) return tape_refuse();
  hipLaunchKernelGGL(k_harmonic, dim3(nblocks(size_t(nc) * nc * G)), dim3(kBlock), 0, s, fine,
                     coarse, G, nc);
  return hipGetLastError();
}

hipError_t launch_convert_d2f(const double* in, float* out, size_t n, hipStream_t s, const int* active) {
  if (g_tape) return tape_refuse();
  hipLaunchKernelGGL(k_d2f, dim3(nblocks(n)), dim3(kBlock), 0, s, in, out, n, active);
  return hipGetLastError();
}
hipError_t launch_convert_f2d(const float* in, double* out, size_t n, hipStream_t s) {
  if (g_tape) return tape_refuse();
  hipLaunchKernelGGL(k_f2d, dim3(nblocks(n)), dim3(kBlock), 0, s, in, out, n);
  return hipGetLastError();
}
hipError_t launch_add_diff_f2d(double* y, const float* u, size_t n, hipStream_t s,
                               const int* active) {
  if (g_tape) return tape_refuse();
  hipLaunchKernelGGL(k_add_diff_f2d, dim3(nblocks(n)), dim3(kBlock), 0, s, y, u, n, active);
  return hipGetLastError();
}
hipError_t launch_add_f2d(double* y, const float* x, size_t n, hipStream_t s, const int* active) {
  if (g_tape) return tape_add(P_ADDF2D, 1, 0, 0, dim3(nblocks(n)), AAddF2D{y, x, n});
  hipLaunchKernelGGL(k_add_f2d, dim3(nblocks(n)), dim3(kBlock), 0, s, y, x, n, active);
  return hipGetLastError();
}

#define CTF_INSTANTIATE(T)                                                                          \
  template hipError_t launch_moments<T>(const LevelData<T>&, const T*, T*, int, hipStream_t);       \
  template hipError_t launch_emission<T>(const LevelDims&, const T*, const T*, int, const T*, T*,   \
                                         hipStream_t, int);                                         \
  template hipError_t launch_pg<T>(int, const LevelData<T>&, const Stencils<T>&, const PGParams&,   \
                                   const PGLaunch<T>&, hipStream_t);                                \
  template hipError_t launch_pg_diffusivity<T>(int, const LevelData<T>&, const Stencils<T>&,        \
                                               const PGParams&, const PGLaunch<T>&, hipStream_t);   \
  template hipError_t launch_upwind_full<T>(const LevelData<T>&, int, const T*, const T*, int, T*,  \
                                            int, T, const T*, hipStream_t, float*, double*, size_t,  \
                                            int*);                                                  \
  template hipError_t launch_upwind_correction<T>(const LevelData<T>&, int, const T*, int, int,     \
                                                  const T*, T*, T*, hipStream_t, int, const T*, int); \
  template hipError_t launch_upwind_correction2<T>(const LevelData<T>&, int, const T*, int, int,    \
                                                   const T*, T*, T*, hipStream_t, int);             \
  template hipError_t launch_restrict<T>(const LevelData<T>&, const LevelData<T>&, const T*, T*,    \
                                         hipStream_t);                                              \
  template hipError_t launch_prolong<T>(const LevelData<T>&, int, const T*, T*, hipStream_t);       \
  template hipError_t launch_wnorm2<T>(const LevelData<T>&, const T*, double*, int, double*,        \
                                       hipStream_t);                                                \
  template hipError_t launch_axpy<T>(T*, const T*, T, size_t, hipStream_t, const int*);

CTF_INSTANTIATE(double)
CTF_INSTANTIATE(float)

// ---------------------------------------------------------------------------------------------
// Persistent batched solve: one launch of k_persist runs up to max_steps solver steps of every
// problem from their tapes.  Work items (a chunk of tiles of one operation) are handed out by a
// ticket counter in a fixed order: round r (one step of every problem), then the operations in
// tape order (slot s), then the problems, then the chunks.  An item of problem j first waits until
// every item of j ahead of it has finished (done[j] counts j's finished items).  Tickets are taken
// in order and an item waits only on items of smaller tickets, so the smallest unfinished ticket
// can always run: with every block resident the launch cannot deadlock.  Items of a problem that
// its update operation found converged are skipped.  Every wait is bounded: past spin_limit polls
// the launch records an error and every block leaves.
namespace {

struct PSched {
  const unsigned* op_begin;              // [nprob] first operation of problem j
  const unsigned long long* step_items;  // [nprob] work items of one step of problem j
  int* const* active;                    // [nprob] activity flags
  const unsigned* item_slot;             // [round_items] slot k = s * nprob + j of each item of a round
  const unsigned long long* slot_first;  // [n_slots * nprob] first item of slot k within a round
  unsigned long long round_items, total_items;
  unsigned nprob, spin_limit;
  unsigned long long* ticket;
  unsigned long long* done;              // [nprob]
  int* n_active;
  int* error;
};

template <typename A>
__device__ __forceinline__ const A& oparg(const POp* o) {
  return *reinterpret_cast<const A*>(o->arg);
}
template <typename V>
__device__ __forceinline__ V ald(const V* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename V>
__device__ __forceinline__ void ast(V* p, V v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long aadd(unsigned long long* p, unsigned long long v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T>
__device__ __forceinline__ void run_typed(const POp* __restrict__ o, const VBlk& vb) {
  constexpr int R = corr2_rows<T>();
  switch (o->kind) {
    case P_MOM: {
      const auto& A = oparg<AMom<T>>(o);
      b_moments<T>(vb, A.L, A.psi, A.phi, A.nmom);
      break;
    }
    case P_EMIS: {
      const auto& A = oparg<AEmis<T>>(o);
      b_emission<T>(vb, A.d, A.phi, A.ss, A.nl, A.src, A.E, A.coarse);
      break;
    }
    case P_UPF: {
      const auto& A = oparg<AUpf<T>>(o);
      if (o->kb == 4)
        b_upwind_full<T, 4>(vb, A.L, A.bc_vac, A.psi, A.E, A.nmomE, A.out, A.out_f, A.mode, A.sign, A.rhs, A.partial);
      else
        b_upwind_full<T, 1>(vb, A.L, A.bc_vac, A.psi, A.E, A.nmomE, A.out, A.out_f, A.mode, A.sign, A.rhs, A.partial);
      break;
    }
    case P_CORR: {
      const auto& A = oparg<ACorr<T>>(o);
      if (o->xmode == 0)
        b_upwind_corr<T, 0, false>(vb, A.L, A.bc_vac, A.xin, A.ndc, A.rhs, A.xout, A.acc, nullptr, 1);
      else if (o->xmode == 1)
        b_upwind_corr<T, 1, false>(vb, A.L, A.bc_vac, A.xin, A.ndc, A.rhs, A.xout, A.acc, nullptr, 1);
      else
        b_upwind_corr<T, 2, false>(vb, A.L, A.bc_vac, A.xin, A.ndc, A.rhs, A.xout, A.acc, nullptr, 1);
      break;
    }
    case P_CORR2: {
      const auto& A = oparg<ACorr<T>>(o);
      if (sizeof(T) == 8 && o->kb == 4) {   // the blocked form is recorded for float64 only
        if (o->xmode == 0)
          b_upwind_corr2<T, 0, R, 4>(vb, A.L, A.bc_vac, A.xin, A.ndc, A.rhs, A.xout, A.acc);
        else if (o->xmode == 1)
          b_upwind_corr2<T, 1, R, 4>(vb, A.L, A.bc_vac, A.xin, A.ndc, A.rhs, A.xout, A.acc);
        else
          b_upwind_corr2<T, 2, R, 4>(vb, A.L, A.bc_vac, A.xin, A.ndc, A.rhs, A.xout, A.acc);
      } else {
        if (o->xmode == 0)
          b_upwind_corr2<T, 0, R, 1>(vb, A.L, A.bc_vac, A.xin, A.ndc, A.rhs, A.xout, A.acc);
        else if (o->xmode == 1)
          b_upwind_corr2<T, 1, R, 1>(vb, A.L, A.bc_vac, A.xin, A.ndc, A.rhs, A.xout, A.acc);
        else
          b_upwind_corr2<T, 2, R, 1>(vb, A.L, A.bc_vac, A.xin, A.ndc, A.rhs, A.xout, A.acc);
      }
      break;
    }
    case P_RESTRICT: {
      const auto& A = oparg<ARestrict<T>>(o);
      b_restrict<T>(vb, A.Lf, A.Lc, A.fine, A.coarse);
      break;
    }
    case P_COPY: {
      const auto& A = oparg<ACopy<T>>(o);
      b_copy<T>(vb, A.dst, A.src, A.n, nullptr);
      break;
    }
    default:
      break;
  }
}

__device__ __forceinline__ void run_op(const POp* __restrict__ o, const VBlk& vb) {
  switch (o->kind) {
    case P_MOM_MFMA: {
      const auto& A = oparg<AMom<float>>(o);
      b_moments_mfma(vb, A.L, A.psi, A.phi, A.nmom);
      return;
    }
    case P_SUMCH: {
      const auto& A = oparg<ASum>(o);
      b_sum_chunks(vb, A.partial, A.np, A.out, nullptr);
      return;
    }
    case P_SUMP: {
      const auto& A = oparg<ASum>(o);
      b_sum_partials(vb, A.partial, A.np, A.out, nullptr);
      return;
    }
    case P_ADDF2D: {
      const auto& A = oparg<AAddF2D>(o);
      b_add_f2d(vb, A.y, A.x, A.n, nullptr);
      return;
    }
    default:
      break;
  }
  if (o->fp64) run_typed<double>(o, vb);
  else run_typed<float>(o, vb);
}

// The update of the activity flag (one thread): rel = sqrt(norm2) / bnorm, active = rel > rtol,
// steps += 1 while active, as the stand-alone update kernel does.  Values other blocks wrote in
// this launch are read with atomic loads.
__device__ void run_active(const POp* __restrict__ o, int* n_active, int* error) {
  const auto& A = oparg<AActive>(o);
  if (ald(A.active) == 0) return;
  const double r = sqrt(ald(A.norm2)) / A.bnorm;
  ast(A.rel, r);
  const int on = (r > A.rtol || r != r) ? 1 : 0;
  ast(A.active, on);
  if (on) {
    if (A.steps) ast(A.steps, ald(A.steps) + 1.0);
  } else {
    __hip_atomic_fetch_add(n_active, -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (!(r <= 1.7976931348623157e308)) ast(error, int(kPersistNonFinite));
}

__global__ __launch_bounds__(kBlock, 2) void k_persist(const POp* __restrict__ ops, PSched S) {
  __shared__ int s_ctl;
  __shared__ unsigned s_j, s_op, s_item;
  unsigned long long t_next = 0;
  if (threadIdx.x == 0) t_next = aadd(S.ticket, 1ull);
  for (;;) {
    if (threadIdx.x == 0) {
      // ctl: 0 run the item, 1 skip it (problem converged), 2 leave, 3 the update ran here
      const unsigned long long t = t_next;
      int ctl = 0;
      unsigned j = 0, opi = 0, item = 0;
      if (t >= S.total_items || ald(S.error) != 0 || ald(S.n_active) == 0) {
        ctl = 2;
      } else {
        t_next = aadd(S.ticket, 1ull);   // the next ticket, fetched while this item runs
        const unsigned long long r = t / S.round_items, rem = t - r * S.round_items;
        const unsigned k = S.item_slot[rem];
        const unsigned slot = k / S.nprob;
        j = k - slot * S.nprob;
        item = unsigned(rem - S.slot_first[k]);
        opi = S.op_begin[j] + slot;
        const unsigned long long need = r * S.step_items[j] + ops[opi].before;
        const int* act = S.active[j];
        for (unsigned polls = 0;; ++polls) {
          if (ald(act) == 0) {
            ctl = 1;
            break;
          }
          if (ald(S.done + j) >= need) break;
          if (ald(S.error) != 0) {
            ctl = 2;
            break;
          }
          if (polls >= S.spin_limit) {
            ast(S.error, int(kPersistSpin));
            ctl = 2;
            break;
          }
          __builtin_amdgcn_s_sleep(2);
        }
        if (ctl == 0) {
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
          if (ops[opi].kind == P_ACTIVE) {
            run_active(ops + opi, S.n_active, S.error);
            ctl = 3;
          }
        }
      }
      s_ctl = ctl;
      s_j = j;
      s_op = opi;
      s_item = item;
    }
    __syncthreads();
    const int ctl = __builtin_amdgcn_readfirstlane(s_ctl);
    const unsigned j = __builtin_amdgcn_readfirstlane(s_j);
    const unsigned opi = __builtin_amdgcn_readfirstlane(s_op);
    const unsigned item = __builtin_amdgcn_readfirstlane(s_item);
    __syncthreads();
    if (ctl == 2) return;
    if (ctl == 0) {
      const POp* __restrict__ o = ops + opi;
      const unsigned gx = o->gx, gy = o->gy, gz = o->gz;
      const unsigned t0 = item * o->chunk, t1 = min(t0 + o->chunk, o->tiles);
      for (unsigned tile = t0; tile < t1; ++tile) {
        const VBlk vb{tile % gx, (tile / gx) % gy, tile / (gx * gy), gx, gy, gz, unsigned(kBlock)};
        run_op(o, vb);
        __syncthreads();   // the operations' LDS is reused by the next tile
      }
    }
    if (ctl == 0 || ctl == 3) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      __syncthreads();
      if (threadIdx.x == 0) aadd(S.done + j, 1ull);
    }
  }
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

hipError_t persist_grid(int* blocks) {
  int dev = 0, cus = 0, occ = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_persist, kBlock, 0);
  if (e != hipSuccess) return e;
  if (cus < 1 || occ < 1) return hipErrorInvalidConfiguration;
  *blocks = cus * occ;
  return hipSuccess;
}

namespace {
// The schedule of a batch: chunk sizes and item counts of every operation, the slot table and the
// workspace layout.  items_per_block: work items per resident block that one operation of the
// largest problem is split into.
struct PersistPlan {
  std::vector<POp> ops;
  std::vector<unsigned> op_begin;
  std::vector<unsigned long long> step_items, slot_first;
  std::vector<unsigned> item_slot;
  unsigned long long round_items = 0;
  size_t off_done = 0, off_active = 0, off_begin = 0, off_step = 0, off_ops = 0, off_first = 0, off_slot = 0,
         bytes = 0;
};

PersistPlan plan_persist(const PersistTape* const* tapes, int nprob, int blocks, int items_per_block) {
  PersistPlan pl;
  size_t n_slots = 0;
  const unsigned long long target = (unsigned long long)blocks * unsigned(std::max(1, items_per_block));
  for (int j = 0; j < nprob; ++j) {
    pl.op_begin.push_back(unsigned(pl.ops.size()));
    unsigned long long before = 0;
    for (POp op : tapes[j]->ops) {
      op.chunk = unsigned(std::max<unsigned long long>(1, (op.tiles + target - 1) / target));
      op.items = (op.tiles + op.chunk - 1) / op.chunk;
      op.before = before;
      before += op.items;
      pl.ops.push_back(op);
    }
    pl.step_items.push_back(before);
    n_slots = std::max(n_slots, tapes[j]->ops.size());
  }
  pl.slot_first.resize(n_slots * nprob);
  for (size_t sl = 0; sl < n_slots; ++sl)
    for (int j = 0; j < nprob; ++j) {
      const size_t k = sl * nprob + j;
      pl.slot_first[k] = pl.round_items;
      if (sl < tapes[j]->ops.size()) {
        const unsigned items = pl.ops[pl.op_begin[j] + sl].items;
        pl.item_slot.insert(pl.item_slot.end(), items, unsigned(k));
        pl.round_items += items;
      }
    }
  size_t off = 256;   // ticket, n_active, error
  pl.off_done = off;
  off = align256(off + sizeof(unsigned long long) * nprob);
  pl.off_active = off;
  off = align256(off + sizeof(int*) * nprob);
  pl.off_begin = off;
  off = align256(off + sizeof(unsigned) * nprob);
  pl.off_step = off;
  off = align256(off + sizeof(unsigned long long) * nprob);
  pl.off_ops = off;
  off = align256(off + sizeof(POp) * pl.ops.size());
  pl.off_first = off;
  off = align256(off + sizeof(unsigned long long) * pl.slot_first.size());
  pl.off_slot = off;
  off = align256(off + sizeof(unsigned) * pl.item_slot.size());
  pl.bytes = off;
  return pl;
}
}  // namespace

size_t persist_workspace_bytes(const PersistTape* const* tapes, int nprob, int blocks, int items_per_block) {
  return plan_persist(tapes, nprob, blocks, items_per_block).bytes;
}

hipError_t persist_solve(const PersistTape* const* tapes, int nprob, int max_steps, int blocks, int items_per_block,
                         unsigned spin_limit, void* ws, size_t ws_bytes, hipStream_t s, PersistResult* res) {
  const PersistPlan pl = plan_persist(tapes, nprob, blocks, items_per_block);
  if (!ws || ws_bytes < pl.bytes || (reinterpret_cast<uintptr_t>(ws) & 255)) return hipErrorInvalidValue;
  if (pl.round_items == 0 || max_steps < 1 || blocks < 1) return hipErrorInvalidValue;
  char* base = static_cast<char*>(ws);
  std::vector<char> img(pl.bytes, 0);
  int n_active = nprob;
  std::memcpy(img.data() + 8, &n_active, sizeof(int));
  std::vector<int*> act(nprob);
  for (int j = 0; j < nprob; ++j) act[j] = tapes[j]->active;
  std::memcpy(img.data() + pl.off_active, act.data(), sizeof(int*) * nprob);
  std::memcpy(img.data() + pl.off_begin, pl.op_begin.data(), sizeof(unsigned) * nprob);
  std::memcpy(img.data() + pl.off_step, pl.step_items.data(), sizeof(unsigned long long) * nprob);
  std::memcpy(img.data() + pl.off_ops, pl.ops.data(), sizeof(POp) * pl.ops.size());
  std::memcpy(img.data() + pl.off_first, pl.slot_first.data(), sizeof(unsigned long long) * pl.slot_first.size());
  std::memcpy(img.data() + pl.off_slot, pl.item_slot.data(), sizeof(unsigned) * pl.item_slot.size());
  hipError_t e = hipMemcpyAsync(base, img.data(), pl.bytes, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return e;
  PSched S;
  S.op_begin = reinterpret_cast<const unsigned*>(base + pl.off_begin);
  S.step_items = reinterpret_cast<const unsigned long long*>(base + pl.off_step);
  S.active = reinterpret_cast<int* const*>(base + pl.off_active);
  S.item_slot = reinterpret_cast<const unsigned*>(base + pl.off_slot);
  S.slot_first = reinterpret_cast<const unsigned long long*>(base + pl.off_first);
  S.round_items = pl.round_items;
  S.total_items = pl.round_items * (unsigned long long)max_steps;
  S.nprob = unsigned(nprob);
  S.spin_limit = spin_limit;
  S.ticket = reinterpret_cast<unsigned long long*>(base);
  S.n_active = reinterpret_cast<int*>(base + 8);
  S.error = reinterpret_cast<int*>(base + 12);
  S.done = reinterpret_cast<unsigned long long*>(base + pl.off_done);
  hipLaunchKernelGGL(k_persist, dim3(blocks), dim3(kBlock), 0, s, reinterpret_cast<const POp*>(base + pl.off_ops), S);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  char head[16];
  e = hipMemcpyAsync(head, base, sizeof(head), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  if (res) {
    std::memcpy(&res->tickets, head, 8);
    std::memcpy(&res->n_active, head + 8, 4);
    std::memcpy(&res->error, head + 12, 4);
    res->round_items = pl.round_items;
    res->blocks = blocks;
  }
  return hipSuccess;
}

}  // namespace ctf
