// Internal declarations shared by the host driver (api.cpp, setup.cpp) and the HIP kernels
// (kernels.hip).  Nothing here crosses the C-ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/ctf.h"

namespace ctf {

constexpr int kMaxP = 4;
constexpr int kMaxLevels = 16;

// ---- host-side setup (setup.cpp) ---------------------------------------------------------------
struct Quadrature {
  int na = 0;
  int faces = 8;                       // 8, or 4 (the xi > 0 half)
  std::vector<double> mu, nu, xi, w;  // n_dir = faces * na^2 each, w sums to 4 pi
};

// Finest ordinates of the octahedral patch set (section "Discrete Ordinates"); faces = 4 keeps
// the faces with xi > 0 (the weights, normalised to 4 pi, are then twice the full set's).
Quadrature build_quadrature(int na, int faces = 8);
// Coarse ordinates: children patches added (section "Space-Angle Multigrid").
Quadrature coarsen_quadrature(const Quadrature& q);
// Parent ordinate of fine ordinate n on a face grid of na x na (identity once na == 1).
inline int parent_dir(int n, int na) {
  if (na == 1) return n;
  int f = n / (na * na), r = n % (na * na);
  int a = r / na, b = r % na, nc = na / 2;
  return f * nc * nc + (a / 2) * nc + (b / 2);
}
// 1D ConvFEM stencils (m, d, k), 2p+1 entries each (Appendix A construction).
void convfem_stencils(int p, double* m, double* d, double* k);

// ---- device kernel arguments -------------------------------------------------------------------
// Stencils are passed by value (tiny) so that every kernel reads them from its argument segment.
template <typename T>
struct Stencils {
  T m[2 * kMaxP + 1];
  T d[2 * kMaxP + 1];  // already divided by h
  T k[2 * kMaxP + 1];  // already divided by h^2
  T mr[2 * kMaxP + 1]; // m and d (divided by h) of the other degree of the low / high residual
  T dr[2 * kMaxP + 1]; // estimate (degree p - 1 or p + 1), zero otherwise
};

struct LevelDims {
  int n;        // nodes per side
  int nd;       // ordinates
  int na;
  int G;
  double h;
  const int* active;  // device flag: kernels of a converged problem return at once (may be null)
};

template <typename T>
struct LevelData {
  LevelDims dims;
  const T* mu;       // [nd]
  const T* nu;       // [nd]
  const T* w;        // [nd]
  const T* sigma_t;  // [G][n][n]
};

// bc bits: bit s set <=> side s (x-, x+, y-, y+) is vacuum
struct PGParams {
  double alpha_r, eps_k, alpha_kabs, alpha_ksq, beta;
  int bc_vac;
  int isotropic = 0;   // 1: the isotropic diffusivity (k_x = k_y) instead of the anisotropic pair
  int r_estimate = 0;  // its residual estimate: 0 mixed mass, 1 degree p - 1, 2 degree p + 1
};

// ---- kernel launchers (kernels.hip) ------------------------------------------------------------
// Every launcher queues work on `s` and returns hipGetLastError().
template <typename T>
hipError_t launch_moments(const LevelData<T>& L, const T* psi, T* phi, int nmom, hipStream_t s);

// The same contraction on bf16 MFMA (float32 accumulation), for float32 psi.
hipError_t launch_moments_mfma(const LevelData<float>& L, const float* psi, float* phi, int nmom,
                               hipStream_t s);

// E[g][m][cell]: q_n = E0 + mu_n E1 + nu_n E2 (E1, E2 only if nl == 2), divided by 4 pi;
// source == null: no external source.  phi_coarse: phi is on the grid of half the size and read at
// each cell's parent (the moments of an UpSamp'd correction).
template <typename T>
hipError_t launch_emission(const LevelDims& d, const T* phi, const T* sigma_s, int nl,
                           const T* source, T* E, hipStream_t s, int phi_coarse = 0);

// Finest ConvFEM Petrov-Galerkin operator.
//   mode 0: out = sign * rho (out and / or out_f; partial: per-block sum of w_n h^2 out^2)
//   mode 1: out = psi + rho / (beta d)
//   kx_in, ky_in != null: these diffusivities (frozen); else k is computed from psi: on the fly
//   (fused kernel) when no k output is requested, or first into kx_out, ky_out (plus float
//   copies in kx_out_f, ky_out_f if non-null)
//   rhs != null: a per-DOF term added to the emission (right-hand side of a correction equation)
template <typename T>
struct PGLaunch {
  const T* psi = nullptr;
  const T* E = nullptr;
  int nmomE = 1;
  const T* kx_in = nullptr;
  const T* ky_in = nullptr;
  T* out = nullptr;
  float* out_f = nullptr;
  double* partial = nullptr;
  T* kx_out = nullptr;
  T* ky_out = nullptr;
  float* kx_out_f = nullptr;
  float* ky_out_f = nullptr;
  const T* rhs = nullptr;
  T rhs_sign = T(1);  // the rhs enters as rhs_sign * rhs (+1 or -1)
  int mode = 0;
  T sign = T(1);
  int strip_h = 32;   // rows per wavefront strip (tunable)
  int* npartial = nullptr;  // receives the number of per-block partial sums written (mode 0)
  float* psi_f = nullptr;   // optional: psi rounded to float at the output cells
  double* acc64 = nullptr;  // mode 1, optional: acc64 += out - float(acc64) at the output cells
};
// Residual / sweep of the ConvFEM-PG operator.  With neither kx_in nor kx_out the non-linear
// diffusivities are formed inside the one pass; with kx_out (and no kx_in) they are formed by
// launch_pg_diffusivity first and read back; with kx_in they are taken as given.
template <typename T>
hipError_t launch_pg(int p, const LevelData<T>& L, const Stencils<T>& st, const PGParams& pp,
                     const PGLaunch<T>& o, hipStream_t s);
// The diffusivities of o.psi alone, into o.kx_out / o.ky_out (and o.kx_out_f / o.ky_out_f).
template <typename T>
hipError_t launch_pg_diffusivity(int p, const LevelData<T>& L, const Stencils<T>& st, const PGParams& pp,
                                 const PGLaunch<T>& o, hipStream_t s);
// number of per-block partial sums a mode-0 launch_pg writes with this strip height
size_t pg_partials(const LevelDims& d, int strip_h);

// Finest upwind operator: mode 0 out = sign * rho (to out and / or out_f; with partial, one float64
// partial sum of w_n h^2 (sign rho)^2 per block, their count in *npartial, at most partial_cap),
// mode 1 out = psi + rho / d.
template <typename T>
hipError_t launch_upwind_full(const LevelData<T>& L, int bc_vac, const T* psi, const T* E,
                              int nmomE, T* out, int mode, T sign, const T* rhs, hipStream_t s,
                              float* out_f = nullptr, double* partial = nullptr, size_t partial_cap = 0,
                              int* npartial = nullptr);
// number of per-block partial sums a mode-0 launch_upwind_full writes
size_t upwind_full_blocks(const LevelDims& d);

// Correction sweep e_new = e + (rhs - A_up e - sigma_t e) / d on one level.
//   xmode 0: e from x_in;  1: e = UpSamp(x_coarse) (x_in is the level+1 array, ndc its n_dir);
//   2: e = 0.   psi_acc != null: psi_acc += e_new instead of writing x_out.
//   E != null: the emission of the sweep's input e (no external source) is added to rhs, the
//   scattering-coupled sweep.
template <typename T>
hipError_t launch_upwind_correction(const LevelData<T>& L, int bc_vac, const T* x_in, int xmode,
                                    int ndc, const T* rhs, T* x_out, T* psi_acc, hipStream_t s,
                                    int block = 256, const T* E = nullptr, int nmomE = 1);
// Two such sweeps (without the scattering term) in one pass: the first from (x_in, xmode), the
// second from its result; the result as for one sweep.
template <typename T>
hipError_t launch_upwind_correction2(const LevelData<T>& L, int bc_vac, const T* x_in, int xmode,
                                     int ndc, const T* rhs, T* x_out, T* psi_acc, hipStream_t s,
                                     int block = 256);

template <typename T>
hipError_t launch_restrict(const LevelData<T>& Lf, const LevelData<T>& Lc, const T* fine,
                           T* coarse, hipStream_t s);

template <typename T>
hipError_t launch_prolong(const LevelData<T>& Lf, int ndc, const T* coarse, T* fine, hipStream_t s);

// partial[b] = sum over block b of w_n h^2 v^2, then out[0] = sum of partials (fixed order).
template <typename T>
hipError_t launch_wnorm2(const LevelData<T>& L, const T* v, double* partial, int npartial,
                         double* out, hipStream_t s);
int wnorm2_partials(const LevelDims& d);
// out[0] = sum of np partials in a fixed order (a function of np only).  The buffer needs room for
// sum_partials_extra() more doubles after the np partials (first-stage sums of long inputs).
hipError_t launch_sum_partials(double* partial, int np, double* out, hipStream_t s,
                               const int* active = nullptr);
int sum_partials_extra();
// if *active: rel[0] = sqrt(norm2[0]) / bnorm, *active = (rel > rtol), and steps[0] += 1 while
// still active (batched solves)
hipError_t launch_update_active(const double* norm2, double bnorm, double rtol, double* rel, int* active,
                                double* steps, hipStream_t s);
hipError_t launch_set_int(int* p, int v, hipStream_t s);
template <typename T>
hipError_t launch_copy(T* dst, const T* src, size_t n, hipStream_t s, const int* active = nullptr);

template <typename T>
hipError_t launch_axpy(T* y, const T* x, T a, size_t n, hipStream_t s, const int* active = nullptr);

hipError_t launch_harmonic_coarsen(const double* fine, double* coarse, int G, int nc, hipStream_t s);

// precision conversions
hipError_t launch_convert_d2f(const double* in, float* out, size_t n, hipStream_t s,
                              const int* active = nullptr);
hipError_t launch_convert_f2d(const float* in, double* out, size_t n, hipStream_t s);
// y(double) += x(float)
hipError_t launch_add_f2d(double* y, const float* x, size_t n, hipStream_t s, const int* active = nullptr);
// y(double) += u(float) - fl32(y): the full-approximation update
hipError_t launch_add_diff_f2d(double* y, const float* u, size_t n, hipStream_t s,
                               const int* active = nullptr);

// ---- persistent batched solve (kernels.hip) ------------------------------------------------------
// While a tape is open on the calling thread, the launchers of the upwind solve path (moments,
// emission, upwind operator, sweeps, restriction, norm sums, activity update, copies) append their
// work to it instead of launching; any other launcher fails with hipErrorNotSupported and marks
// the tape unusable.
struct PersistTape;
PersistTape* tape_open();
void tape_close();
void tape_free(PersistTape* t);
// recorded without a refused launch, with an activity update and at least one operation
bool tape_usable(const PersistTape* t);

enum PersistError : int { kPersistSpin = 1, kPersistNonFinite = 2 };
struct PersistResult {
  unsigned long long tickets = 0;      // work items handed out (including ones fetched at exit)
  unsigned long long round_items = 0;  // work items of one step of every problem
  int n_active = 0;                    // problems not converged when the launch ended
  int error = 0;                       // 0, kPersistSpin (a bounded wait ran out) or kPersistNonFinite
  int blocks = 0;
};
// resident blocks of the persistent kernel on the current device (its grid)
hipError_t persist_grid(int* blocks);
size_t persist_workspace_bytes(const PersistTape* const* tapes, int nprob, int blocks, int items_per_block);
// Runs up to max_steps steps of every taped problem in one launch on s and waits for it.  Each
// problem's flags must be set (active = 1) and its step counters cleared beforehand.
hipError_t persist_solve(const PersistTape* const* tapes, int nprob, int max_steps, int blocks, int items_per_block,
                         unsigned spin_limit, void* ws, size_t ws_bytes, hipStream_t s, PersistResult* res);

// ---- learned coarse-grid correction (cnn.hip) ---------------------------------------------------
int cnn_param_count();
size_t cnn_workspace_bytes(int B, int H, int W);
hipError_t cnn_forward(const float* theta, const float* in, float* out, int B, int H, int W, int bf16,
                       void* ws, hipStream_t s);
// the same network with its hidden activations in a file-scope device array instead of a workspace
// (batch * h * w <= kCnnScratchPixels; calls that overlap on one GPU share that array)
constexpr size_t kCnnScratchPixels = 32768;
hipError_t cnn_forward_noalloc(const float* theta, const float* in, float* out, int B, int H, int W, int bf16,
                               hipStream_t s);
hipError_t cnn_loss_grad(const float* theta, const float* in, const float* target, int B, int H, int W,
                         int bf16, float* grad, double* loss, void* ws, hipStream_t s);
hipError_t cnn_adam(float* theta, float* m, float* v, const float* g, int n, int step, float lr, hipStream_t s);
// f0 = sum_n w_n rho_n on one level (group 0), normalised by its RMS (stored in scale[0])
template <typename T>
hipError_t cnn_scalar_residual(const LevelData<T>& L, const T* rho, float* f0, double* scale, hipStream_t s);
// psi (finest, group 0) += scale * out(coarse cell) / (4 pi)
template <typename T>
hipError_t cnn_apply_correction(T* psi, const float* out, const double* scale, int n, int nd, int shift,
                                hipStream_t s);
hipError_t cnn_target(const double* phi_err, float* tgt, const double* scale, int n, int shift, hipStream_t s);
hipError_t cnn_static_features(const double* st_c, const double* ss_f, const double* st_f, float* f1, float* f2,
                               int n, int shift, double H, hipStream_t s);

}  // namespace ctf
