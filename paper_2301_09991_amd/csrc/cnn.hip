// Small convolutional network for the learned coarse-grid correction: forward (bf16 MFMA with
// float32 accumulation, or float32 vector arithmetic), backward (float32, weight gradients
// accumulated in float64 in a fixed order), mean-squared-error loss and Adam.
//
// Network: four 3x3 zero-padded convolutions, channels 3 -> 32 -> 32 -> 32 -> 1, ReLU after the
// first three.  Parameters: one flat float32 vector W1, b1, W2, b2, W3, b3, W4, b4 with
// W[c_out][c_in][ky][kx].  Activations: float32 [batch][channel][y][x]; in bf16 mode every stored
// activation is rounded to a bf16 value, so the MFMA operands are exact copies of it.
#include <hip/hip_runtime.h>

#include <mutex>

#include "internal.h"

namespace ctf {

namespace {

constexpr int kB = 256;
constexpr int kC[5] = {3, 32, 32, 32, 1};

typedef short v8s_t __attribute__((ext_vector_type(8)));
typedef __bf16 v8bf_t __attribute__((ext_vector_type(8)));
typedef float v4f_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ v8bf_t as_bf16x8(v8s_t v) { return __builtin_bit_cast(v8bf_t, v); }

__device__ __forceinline__ unsigned short to_bf16(float x) {
  unsigned int u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return static_cast<unsigned short>(u >> 16);
}
__device__ __forceinline__ float round_bf16(float x) {
  return __uint_as_float(static_cast<unsigned int>(to_bf16(x)) << 16);
}

// ---- forward, float32 vector form: one thread per output pixel, all output channels ----------
template <int CI, int CO>
__global__ __launch_bounds__(kB) void k_conv_fwd_f32(const float* __restrict__ in, const float* __restrict__ W,
                                                     const float* __restrict__ bias, float* __restrict__ out,
                                                     int B, int H, int Wd, int relu, int bf16) {
  __shared__ float sw[CO * CI * 9];
  for (int i = threadIdx.x; i < CO * CI * 9; i += kB) sw[i] = W[i];
  __syncthreads();
  const int hw = H * Wd;
  const int p = blockIdx.x * kB + threadIdx.x;
  if (p >= B * hw) return;
  const int b = p / hw, r = p - b * hw, y = r / Wd, x = r - y * Wd;
  float acc[CO];
#pragma unroll
  for (int co = 0; co < CO; ++co) acc[co] = bias[co];
  for (int ci = 0; ci < CI; ++ci) {
    const float* src = in + (size_t(b) * CI + ci) * hw;
#pragma unroll
    for (int v = 0; v < 3; ++v) {
      const int yy = y + v - 1;
#pragma unroll
      for (int u = 0; u < 3; ++u) {
        const int xx = x + u - 1;
        const float a = (yy >= 0 && yy < H && xx >= 0 && xx < Wd) ? src[yy * Wd + xx] : 0.f;
#pragma unroll
        for (int co = 0; co < CO; ++co) acc[co] += sw[(co * CI + ci) * 9 + v * 3 + u] * a;
      }
    }
  }
#pragma unroll
  for (int co = 0; co < CO; ++co) {
    float z = acc[co];
    if (relu) z = z > 0.f ? z : 0.f;
    if (bf16) z = round_bf16(z);
    out[(size_t(b) * CO + co) * hw + r] = z;
  }
}

// ---- forward on MFMA: implicit GEMM D[pixel][c_out] = sum_k A[pixel][k] Bw[k][c_out], with
// k = c_in * 9 + tap; one wave computes 16 consecutive pixels of a row for all output channels
// (NT tiles of 16 channels) with gfx950's v_mfma_f32_16x16x32_bf16 (K = 32 per instruction:
// 288 = 9 x 32 for the 32-channel layers, one zero-padded instruction for the 3-channel input).
template <int CI, int CO>
__global__ __launch_bounds__(64) void k_conv_fwd_mfma(const float* __restrict__ in, const float* __restrict__ W,
                                                      const float* __restrict__ bias, float* __restrict__ out,
                                                      int B, int H, int Wd, int relu) {
  constexpr int K = CI * 9;
  constexpr int NT = (CO + 15) / 16;
  const int lane = threadIdx.x;
  const int i = lane % 16, kq = lane / 16;
  const int nxt = (Wd + 15) / 16;
  const int b = blockIdx.x / (H * nxt), rem = blockIdx.x - b * H * nxt;
  const int y = rem / nxt, x0 = (rem - y * nxt) * 16;
  const int hw = H * Wd;
  v4f_t acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = v4f_t{0.f, 0.f, 0.f, 0.f};
  const float* src = in + size_t(b) * CI * hw;
  for (int k0 = 0; k0 < K; k0 += 32) {
    v8s_t a;
    v8s_t bw[NT];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int k = k0 + 8 * kq + j;
      float av = 0.f;
      int ci = 0, tap = 0;
      if (k < K) {
        ci = k / 9;
        tap = k - ci * 9;
        const int yy = y + tap / 3 - 1, xx = x0 + i + tap % 3 - 1;
        if (yy >= 0 && yy < H && xx >= 0 && xx < Wd) av = src[size_t(ci) * hw + yy * Wd + xx];
      }
      a[j] = static_cast<short>(to_bf16(av));
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const int co = 16 * t + i;
        const float wv = (k < K && co < CO) ? W[(co * CI + ci) * 9 + tap] : 0.f;
        bw[t][j] = static_cast<short>(to_bf16(wv));
      }
    }
#pragma unroll
    for (int t = 0; t < NT; ++t)
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(a), as_bf16x8(bw[t]), acc[t], 0, 0, 0);
  }
  // lane holds pixels 4*kq .. 4*kq+3 of output channel 16 t + i
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int co = 16 * t + i;
    if (co >= CO) continue;
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      const int x = x0 + 4 * kq + jj;
      if (x >= Wd) continue;
      float z = acc[t][jj] + bias[co];
      if (relu) z = z > 0.f ? z : 0.f;
      out[(size_t(b) * CO + co) * hw + y * Wd + x] = round_bf16(z);
    }
  }
}

// ---- loss: d = 2 (out - target) / count; partial sums of (out - target)^2 in float64 --------
__global__ __launch_bounds__(kB) void k_mse(const float* __restrict__ out, const float* __restrict__ tgt,
                                           float* __restrict__ d, double* __restrict__ partial, int count) {
  __shared__ double red[kB];
  double acc = 0.0;
  for (int i = blockIdx.x * kB + threadIdx.x; i < count; i += gridDim.x * kB) {
    const float e = out[i] - tgt[i];
    d[i] = 2.f * e / float(count);
    acc += double(e) * double(e);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = kB / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(kB) void k_finish_loss(const double* __restrict__ partial, int np, int count,
                                                   double* __restrict__ loss) {
  __shared__ double red[kB];
  double acc = 0.0;
  for (int i = threadIdx.x; i < np; i += kB) acc += partial[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = kB / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[0] = red[0] / count;
}

// dz = d * (h > 0) in place (ReLU backward through the stored post-activation)
__global__ __launch_bounds__(kB) void k_relu_bwd(float* __restrict__ d, const float* __restrict__ h, size_t n) {
  const size_t i = size_t(blockIdx.x) * kB + threadIdx.x;
  if (i < n && !(h[i] > 0.f)) d[i] = 0.f;
}

// ---- backward data: din[b][ci][y][x] = sum_{co, v, u} W[co][ci][v][u] dz[b][co][y-v+1][x-u+1] ----
template <int CI, int CO>
__global__ __launch_bounds__(kB) void k_conv_bwd_data(const float* __restrict__ dz, const float* __restrict__ W,
                                                      float* __restrict__ din, int B, int H, int Wd) {
  __shared__ float sw[CO * CI * 9];
  for (int i = threadIdx.x; i < CO * CI * 9; i += kB) sw[i] = W[i];
  __syncthreads();
  const int hw = H * Wd;
  const int p = blockIdx.x * kB + threadIdx.x;
  if (p >= B * hw) return;
  const int b = p / hw, r = p - b * hw, y = r / Wd, x = r - y * Wd;
  float acc[CI];
#pragma unroll
  for (int ci = 0; ci < CI; ++ci) acc[ci] = 0.f;
  for (int co = 0; co < CO; ++co) {
    const float* src = dz + (size_t(b) * CO + co) * hw;
#pragma unroll
    for (int v = 0; v < 3; ++v) {
      const int yy = y - v + 1;
#pragma unroll
      for (int u = 0; u < 3; ++u) {
        const int xx = x - u + 1;
        const float g = (yy >= 0 && yy < H && xx >= 0 && xx < Wd) ? src[yy * Wd + xx] : 0.f;
#pragma unroll
        for (int ci = 0; ci < CI; ++ci) acc[ci] += sw[(co * CI + ci) * 9 + v * 3 + u] * g;
      }
    }
  }
#pragma unroll
  for (int ci = 0; ci < CI; ++ci) din[(size_t(b) * CI + ci) * hw + r] = acc[ci];
}

// ---- backward weights: one block per (co, ci): 9 taps; the bias gradient rides on ci == 0 ------
// Each thread sums its pixels p, p + kB, ... in that order in float64.  The pixel loop runs four
// pixels per pass with every load issued first (eight: fewer waves, slower); taps outside the image and zero gradients (the
// ReLU's) contribute an exact zero product instead of being skipped, which leaves every partial
// sum unchanged, so the result is that of summing the nonzero terms alone.
template <int CI, int CO>
__global__ __launch_bounds__(kB) void k_conv_bwd_weight(const float* __restrict__ dz, const float* __restrict__ in,
                                                        float* __restrict__ gW, float* __restrict__ gb,
                                                        int B, int H, int Wd) {
  const int co = blockIdx.x / CI, ci = blockIdx.x - co * CI;
  const int hw = H * Wd, total = B * hw;
  double acc[10];
#pragma unroll
  for (int t = 0; t < 10; ++t) acc[t] = 0.0;
  // the gradient and the nine taps of pixel p (taps outside the image read as 0)
  auto load = [&](int p, float& g, float (&sv)[9]) {
    const int b = p / hw, r = p - b * hw, y = r / Wd, x = r - y * Wd;
    g = dz[(size_t(b) * CO + co) * hw + r];
    const float* src = in + (size_t(b) * CI + ci) * hw;
#pragma unroll
    for (int v = 0; v < 3; ++v) {
      const int yy = y + v - 1;
#pragma unroll
      for (int u = 0; u < 3; ++u) {
        const int xx = x + u - 1;
        const bool ok = yy >= 0 && yy < H && xx >= 0 && xx < Wd;
        sv[v * 3 + u] = src[ok ? yy * Wd + xx : r];
        if (!ok) sv[v * 3 + u] = 0.f;
      }
    }
  };
  auto add = [&](float g, const float (&sv)[9]) {
#pragma unroll
    for (int t = 0; t < 9; ++t) acc[t] += double(g) * double(sv[t]);
    acc[9] += double(g);
  };
  constexpr int U = 4;
  int p = threadIdx.x;
  for (; p + (U - 1) * kB < total; p += U * kB) {
    float g[U], sv[U][9];
#pragma unroll
    for (int k = 0; k < U; ++k) load(p + k * kB, g[k], sv[k]);
#pragma unroll
    for (int k = 0; k < U; ++k) add(g[k], sv[k]);
  }
  for (; p < total; p += kB) {
    float g, sv[9];
    load(p, g, sv);
    add(g, sv);
  }
  __shared__ double red[10][kB];
#pragma unroll
  for (int t = 0; t < 10; ++t) red[t][threadIdx.x] = acc[t];
  __syncthreads();
  for (int s = kB / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s)
#pragma unroll
      for (int t = 0; t < 10; ++t) red[t][threadIdx.x] += red[t][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x < 9) gW[(co * CI + ci) * 9 + threadIdx.x] = float(red[threadIdx.x][0]);
  if (threadIdx.x == 9 && ci == 0) gb[co] = float(red[9][0]);
}

__global__ __launch_bounds__(kB) void k_adam(float* __restrict__ th, float* __restrict__ m, float* __restrict__ v,
                                            const float* __restrict__ g, int n, float lr, float c1, float c2) {
  const int i = blockIdx.x * kB + threadIdx.x;
  if (i >= n) return;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  th[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

inline unsigned nb(size_t n) { return unsigned((n + kB - 1) / kB); }

size_t param_offset(int layer) {
  size_t off = 0;
  for (int l = 0; l < layer; ++l) off += size_t(kC[l + 1]) * kC[l] * 9 + kC[l + 1];
  return off;
}

template <int L>
hipError_t fwd_layer(const float* in, const float* theta, float* out, int B, int H, int W, int bf16,
                     hipStream_t s) {
  constexpr int CI = kC[L], CO = kC[L + 1];
  const float* Wt = theta + param_offset(L);
  const float* bias = Wt + size_t(CO) * CI * 9;
  const int relu = L < 3;
  if (bf16) {
    const int nxt = (W + 15) / 16;
    hipLaunchKernelGGL((k_conv_fwd_mfma<CI, CO>), dim3(B * H * nxt), dim3(64), 0, s, in, Wt, bias, out, B, H,
                       W, relu);
  } else {
    hipLaunchKernelGGL((k_conv_fwd_f32<CI, CO>), dim3(nb(size_t(B) * H * W)), dim3(kB), 0, s, in, Wt, bias,
                       out, B, H, W, relu, 0);
  }
  return hipGetLastError();
}

template <int L>
hipError_t bwd_layer(const float* dz, const float* in, const float* theta, float* gtheta, float* din, int B,
                     int H, int W, hipStream_t s) {
  constexpr int CI = kC[L], CO = kC[L + 1];
  const float* Wt = theta + param_offset(L);
  float* gW = gtheta + param_offset(L);
  float* gb = gW + size_t(CO) * CI * 9;
  hipLaunchKernelGGL((k_conv_bwd_weight<CI, CO>), dim3(CO * CI), dim3(kB), 0, s, dz, in, gW, gb, B, H, W);
  if (din)
    hipLaunchKernelGGL((k_conv_bwd_data<CI, CO>), dim3(nb(size_t(B) * H * W)), dim3(kB), 0, s, dz, Wt, din, B,
                       H, W);
  return hipGetLastError();
}

constexpr int kLossBlocks = 256;

}  // namespace

// ---- workspace: h1, h2, h3 (32 ch), out (1 ch), d_a, d_b (32 ch), loss partials ----------------
size_t cnn_workspace_bytes(int B, int H, int W) {
  const size_t px = size_t(B) * H * W;
  return (3 * 32 * px + px + 2 * 32 * px) * sizeof(float) + kLossBlocks * sizeof(double) + 4096;
}

int cnn_param_count() { return int(param_offset(4)); }

namespace {
struct CnnWs {
  float *h1, *h2, *h3, *out, *da, *db;
  double* partial;
};
CnnWs carve(void* ws, int B, int H, int W) {
  const size_t px = size_t(B) * H * W;
  char* p = static_cast<char*>(ws);
  p += (256 - (reinterpret_cast<uintptr_t>(p) & 255)) & 255;
  CnnWs c;
  c.h1 = reinterpret_cast<float*>(p);
  c.h2 = c.h1 + 32 * px;
  c.h3 = c.h2 + 32 * px;
  c.out = c.h3 + 32 * px;
  c.da = c.out + px;
  c.db = c.da + 32 * px;
  c.partial = reinterpret_cast<double*>(((reinterpret_cast<uintptr_t>(c.db + 32 * px)) + 255) & ~uintptr_t(255));
  return c;
}
}  // namespace

// Hidden activations of cnn_forward_noalloc: one array per GPU, held until the process ends.  In
// host code its name is only a stand-in; the device address comes from hipGetSymbolAddress.
static __device__ __align__(256) float scratch[3 * 32 * kCnnScratchPixels];

namespace {
// the four layers with the three hidden activations in h1, h2, h3 (32 channels each)
hipError_t forward_layers(const float* theta, const float* in, float* h1, float* h2, float* h3, float* out,
                          int B, int H, int W, int bf16, hipStream_t s) {
  hipError_t e;
  if ((e = fwd_layer<0>(in, theta, h1, B, H, W, bf16, s))) return e;
  if ((e = fwd_layer<1>(h1, theta, h2, B, H, W, bf16, s))) return e;
  if ((e = fwd_layer<2>(h2, theta, h3, B, H, W, bf16, s))) return e;
  return fwd_layer<3>(h3, theta, out, B, H, W, bf16, s);
}

constexpr int kMaxDevices = 64;
std::mutex scratch_mutex;
float* scratch_ptr[kMaxDevices] = {};

// the device address of this GPU's scratch array, looked up once per device
hipError_t scratch_address(float** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(scratch_mutex);
  if (!scratch_ptr[dev]) {
    void* p = nullptr;
    if ((e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch))) != hipSuccess) return e;
    scratch_ptr[dev] = static_cast<float*>(p);
  }
  *out = scratch_ptr[dev];
  return hipSuccess;
}
}  // namespace

hipError_t cnn_forward(const float* theta, const float* in, float* out, int B, int H, int W, int bf16,
                       void* ws, hipStream_t s) {
  CnnWs c = carve(ws, B, H, W);
  return forward_layers(theta, in, c.h1, c.h2, c.h3, out ? out : c.out, B, H, W, bf16, s);
}

hipError_t cnn_forward_noalloc(const float* theta, const float* in, float* out, int B, int H, int W, int bf16,
                               hipStream_t s) {
  float* sc = nullptr;
  hipError_t e = scratch_address(&sc);
  if (e != hipSuccess) return e;
  const size_t px = size_t(B) * H * W;
  return forward_layers(theta, in, sc, sc + 32 * px, sc + 64 * px, out, B, H, W, bf16, s);
}

hipError_t cnn_loss_grad(const float* theta, const float* in, const float* target, int B, int H, int W,
                         int bf16, float* grad, double* loss, void* ws, hipStream_t s) {
  CnnWs c = carve(ws, B, H, W);
  hipError_t e = cnn_forward(theta, in, c.out, B, H, W, bf16, ws, s);
  if (e) return e;
  const int count = B * H * W;
  hipLaunchKernelGGL(k_mse, dim3(kLossBlocks), dim3(kB), 0, s, c.out, target, c.da, c.partial, count);
  hipLaunchKernelGGL(k_finish_loss, dim3(1), dim3(kB), 0, s, c.partial, kLossBlocks, count, loss);
  const size_t px = size_t(B) * H * W;
  // layer 4 (no ReLU): dz = d
  if ((e = bwd_layer<3>(c.da, c.h3, theta, grad, c.db, B, H, W, s))) return e;
  hipLaunchKernelGGL(k_relu_bwd, dim3(nb(32 * px)), dim3(kB), 0, s, c.db, c.h3, 32 * px);
  if ((e = bwd_layer<2>(c.db, c.h2, theta, grad, c.da, B, H, W, s))) return e;
  hipLaunchKernelGGL(k_relu_bwd, dim3(nb(32 * px)), dim3(kB), 0, s, c.da, c.h2, 32 * px);
  if ((e = bwd_layer<1>(c.da, c.h1, theta, grad, c.db, B, H, W, s))) return e;
  hipLaunchKernelGGL(k_relu_bwd, dim3(nb(32 * px)), dim3(kB), 0, s, c.db, c.h1, 32 * px);
  if ((e = bwd_layer<0>(c.db, in, theta, grad, nullptr, B, H, W, s))) return e;
  return hipGetLastError();
}

// ---- coarse-grid correction helpers (one energy group) --------------------------------------
namespace {
template <typename T>
__global__ __launch_bounds__(kB) void k_scalar_residual(LevelData<T> L, const T* __restrict__ rho,
                                                        float* __restrict__ f0) {
  const int ncell = L.dims.n * L.dims.n;
  const int c = blockIdx.x * kB + threadIdx.x;
  if (c >= ncell) return;
  double acc = 0.0;
  for (int d = 0; d < L.dims.nd; ++d) acc += double(L.w[d]) * double(rho[size_t(d) * ncell + c]);
  f0[c] = float(acc);
}

// scale = RMS of f0 (fixed-order block reduction), f0 /= scale
__global__ __launch_bounds__(1024) void k_normalise(float* __restrict__ f0, int count, double* __restrict__ scale) {
  __shared__ double red[1024];
  double acc = 0.0;
  for (int i = threadIdx.x; i < count; i += 1024) acc += double(f0[i]) * double(f0[i]);
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  const double rms = sqrt(red[0] / count);
  const double sc = rms > 0.0 ? rms : 1.0;
  for (int i = threadIdx.x; i < count; i += 1024) f0[i] = float(double(f0[i]) / sc);
  if (threadIdx.x == 0) scale[0] = sc;
}

// psi[n][j][i] += scale * out~(j, i) / (4 pi) for every ordinate, out~ the bilinear interpolation
// of the coarse cell-centred field at the fine cell centre (constant beyond the outer centres)
template <typename T>
__global__ __launch_bounds__(kB) void k_apply_correction(T* __restrict__ psi, const float* __restrict__ out,
                                                         const double* __restrict__ scale, int n, int nd,
                                                         int shift) {
  const int ncell = n * n;
  const int c = blockIdx.x * kB + threadIdx.x;
  if (c >= ncell) return;
  const int j = c / n, i = c - j * n, nc = n >> shift;
  const double inv = 1.0 / double(1 << shift);
  const double ty = (j + 0.5) * inv - 0.5, tx = (i + 0.5) * inv - 0.5;
  const int J0 = int(floor(ty)), I0 = int(floor(tx));
  const double wy = ty - J0, wx = tx - I0;
  const int ja = min(max(J0, 0), nc - 1), jb = min(max(J0 + 1, 0), nc - 1);
  const int ia = min(max(I0, 0), nc - 1), ib = min(max(I0 + 1, 0), nc - 1);
  const double v = (1 - wy) * ((1 - wx) * out[ja * nc + ia] + wx * out[ja * nc + ib]) +
                   wy * ((1 - wx) * out[jb * nc + ia] + wx * out[jb * nc + ib]);
  const T add = T(scale[0] * v * 0.07957747154594767);
  for (int d = 0; d < nd; ++d) psi[size_t(d) * ncell + c] += add;
}

// target[J][I] = mean of phi_err over the 2^shift x 2^shift block / scale
__global__ __launch_bounds__(kB) void k_target(const double* __restrict__ phi_err, float* __restrict__ tgt,
                                               const double* __restrict__ scale, int n, int shift) {
  const int nc = n >> shift, b = 1 << shift;
  const int c = blockIdx.x * kB + threadIdx.x;
  if (c >= nc * nc) return;
  const int J = c / nc, I = c - J * nc;
  double acc = 0.0;
  for (int dj = 0; dj < b; ++dj)
    for (int di = 0; di < b; ++di) acc += phi_err[size_t(J * b + dj) * n + I * b + di];
  tgt[c] = float(acc / (b * b) / scale[0]);
}

// static features: f1 = H sigma_t (coarse), f2 = mean over the block of sigma_s / sigma_t (fine)
__global__ __launch_bounds__(kB) void k_static_features(const double* __restrict__ st_c, const double* __restrict__ ss_f,
                                                        const double* __restrict__ st_f, float* __restrict__ f1,
                                                        float* __restrict__ f2, int n, int shift, double H) {
  const int nc = n >> shift, b = 1 << shift;
  const int c = blockIdx.x * kB + threadIdx.x;
  if (c >= nc * nc) return;
  const int J = c / nc, I = c - J * nc;
  double acc = 0.0;
  for (int dj = 0; dj < b; ++dj)
    for (int di = 0; di < b; ++di) {
      const size_t k = size_t(J * b + dj) * n + I * b + di;
      acc += st_f[k] > 0.0 ? ss_f[k] / st_f[k] : 0.0;
    }
  f1[c] = float(H * st_c[c]);
  f2[c] = float(acc / (b * b));
}
}  // namespace

template <typename T>
hipError_t cnn_scalar_residual(const LevelData<T>& L, const T* rho, float* f0, double* scale, hipStream_t s) {
  const int ncell = L.dims.n * L.dims.n;
  hipLaunchKernelGGL(k_scalar_residual<T>, dim3(nb(ncell)), dim3(kB), 0, s, L, rho, f0);
  hipLaunchKernelGGL(k_normalise, dim3(1), dim3(1024), 0, s, f0, ncell, scale);
  return hipGetLastError();
}
template hipError_t cnn_scalar_residual<double>(const LevelData<double>&, const double*, float*, double*, hipStream_t);
template hipError_t cnn_scalar_residual<float>(const LevelData<float>&, const float*, float*, double*, hipStream_t);

template <typename T>
hipError_t cnn_apply_correction(T* psi, const float* out, const double* scale, int n, int nd, int shift,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_apply_correction<T>, dim3(nb(size_t(n) * n)), dim3(kB), 0, s, psi, out, scale, n, nd, shift);
  return hipGetLastError();
}
template hipError_t cnn_apply_correction<double>(double*, const float*, const double*, int, int, int, hipStream_t);
template hipError_t cnn_apply_correction<float>(float*, const float*, const double*, int, int, int, hipStream_t);

hipError_t cnn_target(const double* phi_err, float* tgt, const double* scale, int n, int shift, hipStream_t s) {
  const int nc = n >> shift;
  hipLaunchKernelGGL(k_target, dim3(nb(size_t(nc) * nc)), dim3(kB), 0, s, phi_err, tgt, scale, n, shift);
  return hipGetLastError();
}

hipError_t cnn_static_features(const double* st_c, const double* ss_f, const double* st_f, float* f1, float* f2,
                               int n, int shift, double H, hipStream_t s) {
  const int nc = n >> shift;
  hipLaunchKernelGGL(k_static_features, dim3(nb(size_t(nc) * nc)), dim3(kB), 0, s, st_c, ss_f, st_f, f1, f2, n,
                     shift, H);
  return hipGetLastError();
}

hipError_t cnn_adam(float* theta, float* m, float* v, const float* g, int n, int step, float lr, hipStream_t s) {
  const float c1 = 1.f - powf(0.9f, float(step)), c2 = 1.f - powf(0.999f, float(step));
  hipLaunchKernelGGL(k_adam, dim3(nb(n)), dim3(kB), 0, s, theta, m, v, g, n, lr, c1, c2);
  return hipGetLastError();
}

}  // namespace ctf
