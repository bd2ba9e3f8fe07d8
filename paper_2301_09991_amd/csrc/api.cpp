// C-ABI of the solver (declared in include/ctf.h): problem setup, workspace layout and the
// sawtooth-cycle / refinement drivers that queue the HIP kernels of kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <fstream>
#include <map>
#include <sstream>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "internal.h"

using namespace ctf;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define CTF_HIP(call)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(CTF_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));         \
  } while (0)

bool is_pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }

int validate(const ctf_config* c) {
  if (!c) return fail(CTF_EINVAL, "null config");
  if (c->n < 2 || c->n > 8192) return fail(CTF_EINVAL, "n must be in [2, 8192]");
  if (!(c->length > 0.0)) return fail(CTF_EINVAL, "length must be > 0");
  if (c->discretisation != CTF_UPWIND && (c->p < 1 || c->p > kMaxP))
    return fail(CTF_EINVAL, "p must be 1..4");
  if (!is_pow2(c->na)) return fail(CTF_EINVAL, "na must be a power of two");
  if (c->ngroups < 1) return fail(CTF_EINVAL, "ngroups must be >= 1");
  if (c->scatter_order < 0 || c->scatter_order > 1) return fail(CTF_EINVAL, "scatter_order 0 or 1");
  if (c->discretisation < CTF_UPWIND || c->discretisation > CTF_CONVFEM_PG_FROZEN_K)
    return fail(CTF_EINVAL, "bad discretisation");
  for (int s = 0; s < 4; ++s)
    if (c->bc[s] != CTF_VACUUM && c->bc[s] != CTF_ZERO_GRADIENT) return fail(CTF_EINVAL, "bad bc");
  if (c->precision < CTF_FP64 || c->precision > CTF_FP32_IR_BF16_MOMENTS)
    return fail(CTF_EINVAL, "bad precision");
  if (c->n_jacobi < 1 || c->n_pg < 0) return fail(CTF_EINVAL, "n_jacobi >= 1 and n_pg >= 0");
  if (c->max_levels < 0 || c->max_levels > kMaxLevels) return fail(CTF_EINVAL, "bad max_levels");
  if (c->precision != CTF_FP64 && c->n_inner < 1) return fail(CTF_EINVAL, "n_inner >= 1");
  if (!(c->beta_pg > 0.0) || !(c->eps_k > 0.0)) return fail(CTF_EINVAL, "beta_pg, eps_k > 0");
  if (c->cnn_level >= 0 && !(c->cnn_max_growth > 0.0)) return fail(CTF_EINVAL, "cnn_max_growth > 0");
  if (c->cnn_level >= 0 && c->ngroups != 1)
    return fail(CTF_EUNSUPPORTED, "the learned correction supports one energy group");
  if (c->hemisphere != 0 && c->hemisphere != 1) return fail(CTF_EINVAL, "hemisphere 0 or 1");
  if (c->coupled_scatter != 0 && c->coupled_scatter != 1) return fail(CTF_EINVAL, "coupled_scatter 0 or 1");
  if (c->pg_isotropic != 0 && c->pg_isotropic != 1) return fail(CTF_EINVAL, "pg_isotropic 0 or 1");
  if (c->pg_r_estimate < CTF_R_MIXED_MASS || c->pg_r_estimate > CTF_R_HIGH)
    return fail(CTF_EINVAL, "pg_r_estimate must be CTF_R_MIXED_MASS, CTF_R_LOW or CTF_R_HIGH");
  if (c->pg_r_estimate != CTF_R_MIXED_MASS && c->discretisation != CTF_UPWIND) {
    if (!c->pg_isotropic) return fail(CTF_EINVAL, "the low / high residual estimates need pg_isotropic = 1");
    if (c->pg_r_estimate == CTF_R_LOW && c->p < 2) return fail(CTF_EINVAL, "the low residual estimate needs p >= 2");
    if (c->pg_r_estimate == CTF_R_HIGH && c->p + 1 > kMaxP)
      return fail(CTF_EUNSUPPORTED, "the high residual estimate needs p <= 3 (filters of degree p + 1)");
  }
  return CTF_OK;
}

int level_count(const ctf_config* c) {
  int L = 1, n = c->n;
  while (n % 2 == 0 && n > 2 && L < kMaxLevels && (c->max_levels == 0 || L < c->max_levels)) {
    n /= 2;
    ++L;
  }
  return L;
}

// bump allocator over the caller's workspace (256-byte aligned slices)
struct Carver {
  char* base;
  size_t off = 0;
  template <typename T>
  T* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

}  // namespace

struct ctf_problem {
  ctf_config cfg{};
  hipStream_t stream = nullptr;
  int L = 0;
  int nmom = 1;  // moments the emission needs: 1 (isotropic) or 3 (P1)
  LevelDims dims[kMaxLevels];
  Quadrature quad[kMaxLevels];
  // per level device data
  double* dirs_d[kMaxLevels];  // mu | nu | w
  float* dirs_f[kMaxLevels];
  double* sigt_d[kMaxLevels];
  float* sigt_f[kMaxLevels];
  double* rho[kMaxLevels];
  double* ea[kMaxLevels];
  double* eb[kMaxLevels];
  float* rho_f[kMaxLevels];
  float* ea_f[kMaxLevels];
  float* eb_f[kMaxLevels];
  // finest-level data
  double* sigma_s = nullptr;
  double* sigs_d[kMaxLevels] = {};   // sigma_s per level (level 0: sigma_s; coarser: 2 x 2 harmonic)
  float* sigs_f[kMaxLevels] = {};
  double* source = nullptr;
  float* sigma_s_f = nullptr;
  double* phi = nullptr;
  double* E = nullptr;
  float* phi_f = nullptr;
  float* E_f = nullptr;
  double* psi_tmp = nullptr;
  double* kx = nullptr;
  double* ky = nullptr;
  bool k_held = false;
  float* kx_f = nullptr;
  float* ky_f = nullptr;
  float* e_f = nullptr;    // float32 correction of a refinement step
  float* e_tmp_f = nullptr;
  float* r_f = nullptr;    // float32 right-hand side of the correction equation
  double* partial = nullptr;
  double* scal = nullptr;  // device scalars
  int npartial = 0;
  size_t partial_cap = 0;   // length of partial
  double bnorm = 0.0;
  Stencils<double> st_d{};
  Stencils<float> st_f{};
  PGParams pp{};
  int bc_vac = 0;
  int* active = nullptr;     // device flag read by every kernel (0: converged member of a batch)
  int strip_h = 128;         // launch shapes (defaults: fastest measured on the 256^2 p = 2 workload)
  int corr_block = 256;
  int pg_fused = 1;          // non-linear PG: diffusivities formed in the same pass (1) or stored (0)
  bool psi32_ready = false;  // e_f holds psi rounded to float (left by the outer residual)
  // learned coarse-grid correction
  int cnn_level = -1;
  bool cnn_on = false;
  bool cnn_ready = false;
  float* cnn_params = nullptr;
  float* cnn_feat = nullptr;   // [3][nc][nc]
  float* cnn_out = nullptr;    // [nc][nc]
  void* cnn_ws = nullptr;
  size_t cnn_ws_bytes = 0;
  double* cnn_scale = nullptr;
  double* cnn_backup = nullptr;  // psi before a step with the correction (restored on rejection)
  // in-library kernel timers: per kernel class, pairs of events recorded around each launch
  bool timing = false;
  int timing_cap = 0;
  unsigned timing_mask = ~0u;   // bit c set: class c is timed
  std::vector<hipEvent_t> ev[CTF_T_COUNT];
  int ev_used[CTF_T_COUNT] = {};
  int ev_dropped[CTF_T_COUNT] = {};

  ~ctf_problem() {
    for (auto& v : ev)
      for (hipEvent_t e : v) (void)hipEventDestroy(e);
  }

  size_t dof(int l) const { return size_t(dims[l].n) * dims[l].n * dims[l].nd * dims[l].G; }
  LevelData<double> ld(int l) const {
    const int nd = dims[l].nd;
    return LevelData<double>{dims[l], dirs_d[l], dirs_d[l] + nd, dirs_d[l] + 2 * nd, sigt_d[l]};
  }
  LevelData<float> lf(int l) const {
    const int nd = dims[l].nd;
    return LevelData<float>{dims[l], dirs_f[l], dirs_f[l] + nd, dirs_f[l] + 2 * nd, sigt_f[l]};
  }
  bool mixed() const { return cfg.precision != CTF_FP64; }
};

namespace {

// Records a start/stop event pair on the problem's stream around one kernel launch while the
// problem's timers are enabled.
struct Timed {
  ctf_problem* P;
  int cls, slot = -1;
  Timed(ctf_problem* p, int c) : P(p), cls(c) {
    if (!P->timing || !((P->timing_mask >> cls) & 1u)) return;
    if (P->ev_used[cls] >= P->timing_cap) {
      ++P->ev_dropped[cls];
      return;
    }
    slot = P->ev_used[cls]++;
    (void)hipEventRecord(P->ev[cls][2 * slot], P->stream);
  }
  ~Timed() {
    if (slot >= 0) (void)hipEventRecord(P->ev[cls][2 * slot + 1], P->stream);
  }
};

// Lay out every device array of the problem over the workspace (base == nullptr: sizing pass).
size_t layout(ctf_problem* P, char* base) {
  Carver c{base};
  const ctf_config& cfg = P->cfg;
  const int G = cfg.ngroups;
  const size_t nc0 = size_t(cfg.n) * cfg.n;
  const bool mixed = cfg.precision != CTF_FP64;
  for (int l = 0; l < P->L; ++l) {
    const size_t dof = P->dof(l);
    const size_t ncell = size_t(P->dims[l].n) * P->dims[l].n;
    P->dirs_d[l] = c.take<double>(3 * size_t(P->dims[l].nd));
    P->dirs_f[l] = c.take<float>(3 * size_t(P->dims[l].nd));
    P->sigt_d[l] = c.take<double>(G * ncell);
    P->sigt_f[l] = c.take<float>(G * ncell);
    P->rho[l] = c.take<double>(dof);
    P->ea[l] = c.take<double>(dof);
    P->eb[l] = c.take<double>(dof);
    if (mixed) {
      P->rho_f[l] = c.take<float>(dof);
      P->ea_f[l] = c.take<float>(dof);
      P->eb_f[l] = c.take<float>(dof);
    } else {
      P->rho_f[l] = P->ea_f[l] = P->eb_f[l] = nullptr;
    }
  }
  const int nl = cfg.scatter_order + 1;
  P->sigma_s = c.take<double>(size_t(nl) * G * G * nc0);
  P->source = c.take<double>(G * nc0);
  P->phi = c.take<double>(3 * G * nc0);
  P->E = c.take<double>(3 * G * nc0);
  P->psi_tmp = c.take<double>(P->dof(0));
  const bool need_k = cfg.discretisation != CTF_UPWIND;
  P->kx = need_k ? c.take<double>(P->dof(0)) : nullptr;
  P->ky = need_k ? c.take<double>(P->dof(0)) : nullptr;
  P->sigs_d[0] = P->sigma_s;
  for (int l = 1; l < P->L && cfg.coupled_scatter; ++l)
    P->sigs_d[l] = c.take<double>(size_t(nl) * G * G * size_t(P->dims[l].n) * P->dims[l].n);
  if (mixed) {
    P->sigma_s_f = c.take<float>(size_t(nl) * G * G * nc0);
    P->sigs_f[0] = P->sigma_s_f;
    for (int l = 1; l < P->L && cfg.coupled_scatter; ++l)
      P->sigs_f[l] = c.take<float>(size_t(nl) * G * G * size_t(P->dims[l].n) * P->dims[l].n);
    P->phi_f = c.take<float>(3 * G * nc0);
    P->E_f = c.take<float>(3 * G * nc0);
    P->kx_f = need_k ? c.take<float>(P->dof(0)) : nullptr;
    P->ky_f = need_k ? c.take<float>(P->dof(0)) : nullptr;
    P->e_f = c.take<float>(P->dof(0));
    P->e_tmp_f = c.take<float>(P->dof(0));
    P->r_f = c.take<float>(P->dof(0));
  }
  if (cfg.cnn_level >= 0 && cfg.cnn_level < P->L) {
    const int nc = P->dims[cfg.cnn_level].n;
    P->cnn_params = c.take<float>(cnn_param_count());
    P->cnn_feat = c.take<float>(3 * size_t(nc) * nc);
    P->cnn_out = c.take<float>(size_t(nc) * nc);
    P->cnn_ws_bytes = cnn_workspace_bytes(1, nc, nc);
    P->cnn_ws = c.take<char>(P->cnn_ws_bytes);
    P->cnn_scale = c.take<double>(4);
    P->cnn_backup = c.take<double>(P->dof(0));
  }
  P->npartial = wnorm2_partials(P->dims[0]);
  P->partial_cap = std::max<size_t>({size_t(P->npartial), pg_partials(P->dims[0], 8), upwind_full_blocks(P->dims[0])});
  P->partial = c.take<double>(P->partial_cap + sum_partials_extra());
  P->scal = c.take<double>(8);
  P->active = c.take<int>(64);
  for (int l = 0; l < P->L; ++l) P->dims[l].active = P->active;
  return c.off + 256;
}

void init_dims(ctf_problem* P) {
  const ctf_config& c = P->cfg;
  P->L = level_count(&c);
  int n = c.n, na = c.na;
  double h = c.length / c.n;
  for (int l = 0; l < P->L; ++l) {
    P->dims[l] = LevelDims{n, (c.hemisphere ? 4 : 8) * na * na, na, c.ngroups, h, nullptr};
    n /= 2;
    na = na > 1 ? na / 2 : 1;
    h *= 2.0;
  }
}

int check_level(const ctf_problem* P, int level) {
  if (!P) return fail(CTF_EINVAL, "null problem");
  if (level < 0 || level >= P->L) return fail(CTF_EINVAL, "level out of range");
  return CTF_OK;
}

// ---- building blocks -------------------------------------------------------------------------
// E <- emission of psi (source S if with_source, else none)
int emission64(ctf_problem* P, const double* psi, bool with_source) {
  const int nl = P->cfg.scatter_order + 1;
  {
    Timed t(P, CTF_T_MOMENTS);
    CTF_HIP(launch_moments<double>(P->ld(0), psi, P->phi, P->nmom, P->stream));
  }
  Timed t(P, CTF_T_EMISSION);
  CTF_HIP(launch_emission<double>(P->dims[0], P->phi, P->sigma_s, nl,
                                  with_source ? P->source : nullptr, P->E, P->stream));
  return CTF_OK;
}

// One PG launch with its timers: when the diffusivities are stored (kx_out without kx_in) their pass
// is timed as a class of its own, then the residual pass reads them back.
template <typename T>
int run_pg(ctf_problem* P, int cls, int cls_k, const LevelData<T>& L, const Stencils<T>& st, PGLaunch<T> o) {
  if (!o.kx_in && o.kx_out) {
    {
      Timed t(P, cls_k);
      CTF_HIP(launch_pg_diffusivity<T>(P->cfg.p, L, st, P->pp, o, P->stream));
    }
    o.kx_in = o.kx_out;
    o.ky_in = o.ky_out;
    o.kx_out = o.ky_out = nullptr;
    o.kx_out_f = o.ky_out_f = nullptr;
  }
  Timed t(P, cls);
  CTF_HIP(launch_pg<T>(P->cfg.p, L, st, P->pp, o, P->stream));
  return CTF_OK;
}

// Finest operator with the emission already in E.
//   mode 0: out = sign * rho(psi) (out and / or out_f), with the squared weighted norm summed into
//           P->scal[0] when want_norm; mode 1: out = psi + rho / (beta d).
//   k_float: also float copies of the diffusivities computed from psi (mixed precision);
//   psi_f: psi rounded to float (PG forms), or null.
int finest64(ctf_problem* P, const double* psi, double* out, int mode, double sign,
             float* out_f = nullptr, bool want_norm = false, bool k_float = false, float* psi_f = nullptr) {
  const ctf_config& c = P->cfg;
  if (c.discretisation == CTF_UPWIND) {
    if (psi_f) return fail(CTF_EUNSUPPORTED, "internal: float copy of psi from the upwind operator");
    double* partial = (mode == 0 && want_norm) ? P->partial : nullptr;
    int np = 0;
    {
      Timed t(P, CTF_T_UPWIND64);
      CTF_HIP(launch_upwind_full<double>(P->ld(0), P->bc_vac, psi, P->E, P->nmom, out, mode, sign,
                                         nullptr, P->stream, out_f, partial, P->partial_cap, &np));
    }
    if (partial) {
      Timed t(P, CTF_T_NORM);
      CTF_HIP(launch_sum_partials(P->partial, np, P->scal, P->stream, P->active));
    }
    return CTF_OK;
  }
  const bool frozen = c.discretisation == CTF_CONVFEM_PG_FROZEN_K;
  if (frozen && !P->k_held) return fail(CTF_EINVAL, "frozen-k discretisation needs ctf_freeze_k first");
  PGLaunch<double> o;
  o.psi = psi;
  o.E = P->E;
  o.nmomE = P->nmom;
  if (frozen) {
    o.kx_in = P->kx;
    o.ky_in = P->ky;
  } else if (k_float || !P->pg_fused) {
    o.kx_out = P->kx;
    o.ky_out = P->ky;
    if (k_float) {
      o.kx_out_f = P->kx_f;
      o.ky_out_f = P->ky_f;
    }
  }
  o.out = out;
  o.out_f = out_f;
  o.mode = mode;
  o.sign = sign;
  o.partial = (mode == 0 && want_norm) ? P->partial : nullptr;
  o.psi_f = psi_f;
  o.strip_h = P->strip_h;
  int np = 0;
  o.npartial = &np;
  int rc = run_pg<double>(P, CTF_T_PG64, CTF_T_PGK64, P->ld(0), P->st_d, o);
  if (rc) return rc;
  if (o.partial) {
    Timed t(P, CTF_T_NORM);
    CTF_HIP(launch_sum_partials(P->partial, np, P->scal, P->stream, P->active));
  }
  return CTF_OK;
}

// sqrt of the squared norm in P->scal[0] (synchronous)
int read_norm(ctf_problem* P, double* out_host) {
  double s2 = 0.0;
  CTF_HIP(hipMemcpyAsync(&s2, P->scal, sizeof(double), hipMemcpyDeviceToHost, P->stream));
  CTF_HIP(hipStreamSynchronize(P->stream));
  *out_host = std::sqrt(s2);
  if (!std::isfinite(*out_host)) return fail(CTF_ENONFINITE, "non-finite residual norm");
  return CTF_OK;
}

int wnorm64(ctf_problem* P, int level, const double* v, double* out_host) {
  {
    Timed t(P, CTF_T_NORM);
    CTF_HIP(launch_wnorm2<double>(P->ld(level), v, P->partial, P->npartial, P->scal, P->stream));
  }
  return read_norm(P, out_host);
}

// per-precision views of the problem's level data and moment / emission buffers
template <typename T> LevelData<T> level_data(const ctf_problem* P, int l);
template <> LevelData<double> level_data<double>(const ctf_problem* P, int l) { return P->ld(l); }
template <> LevelData<float> level_data<float>(const ctf_problem* P, int l) { return P->lf(l); }
template <typename T> T* phi_buffer(ctf_problem* P);
template <> double* phi_buffer<double>(ctf_problem* P) { return P->phi; }
template <> float* phi_buffer<float>(ctf_problem* P) { return P->phi_f; }
template <typename T> T* emission_buffer(ctf_problem* P);
template <> double* emission_buffer<double>(ctf_problem* P) { return P->E; }
template <> float* emission_buffer<float>(ctf_problem* P) { return P->E_f; }
template <typename T> const T* level_sigma_s(const ctf_problem* P, int l);
template <> const double* level_sigma_s<double>(const ctf_problem* P, int l) { return P->sigs_d[l]; }
template <> const float* level_sigma_s<float>(const ctf_problem* P, int l) { return P->sigs_f[l]; }

// n upwind correction sweeps on level l: the first from (xmode, xsrc), the buffer holding the
// result returned through result; acc != null: the last sweep adds into acc instead of writing a
// buffer (result is then not meaningful); final != null: the last sweep writes there.  With coupled_scatter every sweep adds the scattering of its input e (the
// emission of e on the level, no external source; for the first sweep from the coarser level the
// moments of UpSamp(e) are those of e on its own level, read at the parent cells).
template <typename T>
int correction_sweeps(ctf_problem* P, const LevelData<T>& L, int l, const T* xsrc, int xmode,
                      const T* rhs, int nsweeps, T* bufa, T* bufb, T* acc, const T** result,
                      T* final = nullptr) {
  const int ndc = (l + 1 < P->L) ? P->dims[l + 1].nd : 1;   // ordinates of the next coarser level
  const T* cur = xsrc;
  int mode = xmode;
  for (int s = 0, pass = 0; s < nsweeps; ++pass) {
    // without the scattering term, two sweeps run as one pass; passes alternate between the buffers
    const bool pair = !P->cfg.coupled_scatter && s + 1 < nsweeps;
    const bool last = s + (pair ? 2 : 1) == nsweeps;
    T* dst = (last && final) ? final : ((pass % 2 == 0) ? bufa : bufb);
    if (pair) {
      Timed t(P, l == 0 ? CTF_T_CORR0 : CTF_T_CORRC);
      CTF_HIP(launch_upwind_correction2<T>(L, P->bc_vac, cur, mode, ndc, rhs, dst, (last && acc) ? acc : nullptr,
                                           P->stream, P->corr_block));
      cur = dst;
      mode = 0;
      s += 2;
      continue;
    }
    const T* Esc = nullptr;
    if (P->cfg.coupled_scatter && mode != 2) {
      Timed t(P, CTF_T_CSCAT);
      const int nl = P->cfg.scatter_order + 1;
      T* phi = phi_buffer<T>(P);
      if (mode == 1)
        CTF_HIP(launch_moments<T>(level_data<T>(P, l + 1), cur, phi, P->nmom, P->stream));
      else
        CTF_HIP(launch_moments<T>(L, cur, phi, P->nmom, P->stream));
      CTF_HIP(launch_emission<T>(P->dims[l], phi, level_sigma_s<T>(P, l), nl, nullptr, emission_buffer<T>(P),
                                 P->stream, mode == 1 ? 1 : 0));
      Esc = emission_buffer<T>(P);
    }
    Timed t(P, l == 0 ? CTF_T_CORR0 : CTF_T_CORRC);
    CTF_HIP(launch_upwind_correction<T>(L, P->bc_vac, cur, mode, ndc, rhs, dst,
                                        (last && acc) ? acc : nullptr, P->stream, P->corr_block, Esc,
                                        P->nmom));
    cur = dst;
    mode = 0;
    ++s;
  }
  if (result) *result = cur;
  return CTF_OK;
}

// network input from the restricted residual on the correction level (cnn_feat[0], cnn_scale);
// with run_net, also the network output (cnn_out)
template <typename T>
int cnn_features_and_net(ctf_problem* P, const LevelData<T>& Lc, const T* rho_c, bool run_net) {
  Timed t(P, CTF_T_CNN);
  CTF_HIP(cnn_scalar_residual<T>(Lc, rho_c, P->cnn_feat, P->cnn_scale, P->stream));
  if (run_net) {
    const int nc = Lc.dims.n;
    CTF_HIP(cnn_forward(P->cnn_params, P->cnn_feat, P->cnn_out, 1, nc, nc, 1, P->cnn_ws, P->stream));
  }
  return CTF_OK;
}

// the part of the sawtooth cycle after rho_0 (in P->rho[0]) is known; use_cnn: apply the learned
// correction; features_only: compute the network input but do not apply the network
int cycle_rest64(ctf_problem* P, double* psi, bool use_cnn = false, bool features_only = false) {
  const ctf_config& c = P->cfg;
  const int L = P->L;
  for (int l = 1; l < L; ++l) {
    Timed t(P, CTF_T_RESTRICT);
    CTF_HIP(launch_restrict<double>(P->ld(l - 1), P->ld(l), P->rho[l - 1], P->rho[l], P->stream));
  }
  if (use_cnn || features_only) {
    int rc = cnn_features_and_net<double>(P, P->ld(P->cnn_level), P->rho[P->cnn_level], use_cnn);
    if (rc) return rc;
  }
  const double* e = nullptr;
  for (int l = L - 1; l >= 0; --l) {
    const int xmode = (l == L - 1) ? 2 : 1;
    int rc = correction_sweeps<double>(P, P->ld(l), l, e, xmode, P->rho[l], c.n_jacobi, P->ea[l],
                                       P->eb[l], l == 0 ? psi : nullptr, &e);
    if (rc) return rc;
  }
  if (use_cnn) {
    Timed t(P, CTF_T_CNN);
    CTF_HIP(cnn_apply_correction<double>(psi, P->cnn_out, P->cnn_scale, c.n, P->dims[0].nd, P->cnn_level,
                                         P->stream));
  }
  // finest smoothing on the full equations
  double* cur = psi;
  double* other = P->psi_tmp;
  for (int s = 0; s < c.n_pg; ++s) {
    int rc = emission64(P, cur, true);
    if (rc) return rc;
    rc = finest64(P, cur, other, 1, 1.0);
    if (rc) return rc;
    std::swap(cur, other);
  }
  if (cur != psi) CTF_HIP(launch_copy<double>(psi, cur, P->dof(0), P->stream, P->active));
  return CTF_OK;
}

// ---- mixed precision ------------------------------------------------------------------------------
// Linear discretisations (upwind, frozen k): float32 cycles on the correction equation A e = r,
// r the float64 residual rounded to float32 (P->r_f), e in P->e_f, starting from e = 0.
// Non-linear Petrov-Galerkin: full-approximation form.  With psi32 = psi64 rounded, the float32
// cycles solve A32(u) = b32, b32 = A32(psi32) + rho64, from u = psi32 (k recomputed from u in
// every float32 residual, as the float64 cycle does), and psi64 += u - psi32.  In both forms the
// float32 fixed point is the float64 one up to float32 rounding, which the float64 refinement
// removes.

// float32 finest operator on x (emission of x without source, per-DOF term r = rsign rhs, rhs = r_f
// unless given):
//   mode 0: out = sign (r + q(x) - L x);  mode 1: out = x + (r + q(x) - L x)/(beta d)
int inner_finest32(ctf_problem* P, const float* x, float* out, int mode, float sign = 1.0f,
                   const float* rhs = nullptr, float rsign = 1.0f, double* acc64 = nullptr) {
  const ctf_config& c = P->cfg;
  const int nl = c.scatter_order + 1;
  if (c.precision == CTF_FP32_IR_BF16_MOMENTS) {
    Timed t(P, CTF_T_MOMENTS_MFMA);
    CTF_HIP(launch_moments_mfma(P->lf(0), x, P->phi_f, P->nmom, P->stream));
  } else {
    Timed t(P, CTF_T_MOMENTS);
    CTF_HIP(launch_moments<float>(P->lf(0), x, P->phi_f, P->nmom, P->stream));
  }
  {
    Timed t(P, CTF_T_EMISSION);
    CTF_HIP(launch_emission<float>(P->dims[0], P->phi_f, P->sigma_s_f, nl, nullptr, P->E_f, P->stream));
  }
  if (c.discretisation == CTF_UPWIND) {
    if (rhs || rsign != 1.0f || acc64)
      return fail(CTF_EUNSUPPORTED, "internal: upwind float32 operator with another rhs or a float64 update");
    Timed t(P, CTF_T_UPWIND32);
    CTF_HIP(launch_upwind_full<float>(P->lf(0), P->bc_vac, x, P->E_f, P->nmom, out, mode, sign,
                                      P->r_f, P->stream));
    return CTF_OK;
  }
  PGLaunch<float> o;
  o.psi = x;
  o.E = P->E_f;
  o.nmomE = P->nmom;
  if (c.discretisation != CTF_CONVFEM_PG) {
    o.kx_in = P->kx_f;   // frozen k
    o.ky_in = P->ky_f;
  } else if (!P->pg_fused) {
    o.kx_out = P->kx_f;  // full-approximation form: k of x itself, stored then read
    o.ky_out = P->ky_f;
  }
  o.out = out;
  o.rhs = rhs ? rhs : P->r_f;
  o.rhs_sign = rsign;
  o.acc64 = acc64;
  o.mode = mode;
  o.sign = sign;
  o.strip_h = P->strip_h;
  return run_pg<float>(P, acc64 ? CTF_T_PG32U : CTF_T_PG32, CTF_T_PGK32, P->lf(0), P->st_f, o);
}

// one float32 sawtooth cycle on P->e_f; e_is_zero: the correction form's first cycle (e = 0);
// r0_given: P->rho_f[0] already holds the finest residual of e_f; psi64: the last finest sweep
// also applies the full-approximation update psi64 += u - float(psi64) with its result u
int inner_cycle32(ctf_problem* P, bool e_is_zero, bool use_cnn = false, bool r0_given = false,
                  double* psi64 = nullptr) {
  const ctf_config& c = P->cfg;
  const int L = P->L;
  // inner residual r - A e (just r while e = 0)
  const float* r0 = r0_given ? P->rho_f[0] : P->r_f;
  if (!e_is_zero && !r0_given) {
    int rc = inner_finest32(P, P->e_f, P->rho_f[0], 0);
    if (rc) return rc;
    r0 = P->rho_f[0];
  }
  for (int l = 1; l < L; ++l) {
    Timed t(P, CTF_T_RESTRICT);
    CTF_HIP(launch_restrict<float>(P->lf(l - 1), P->lf(l), l == 1 ? r0 : P->rho_f[l - 1], P->rho_f[l],
                                   P->stream));
  }
  if (use_cnn) {
    const int lc = P->cnn_level;
    int rc = cnn_features_and_net<float>(P, P->lf(lc), lc == 0 ? r0 : P->rho_f[lc], true);
    if (rc) return rc;
  }
  const float* e = nullptr;
  for (int l = L - 1; l >= 0; --l) {
    const int xmode = (l == L - 1) ? 2 : 1;
    const float* rhs = l == 0 ? r0 : P->rho_f[l];
    // e = 0 before the cycle: the finest correction is the new e itself (written to e_f);
    // otherwise the last finest sweep adds into e_f
    int rc = correction_sweeps<float>(P, P->lf(l), l, e, xmode, rhs, c.n_jacobi, P->ea_f[l],
                                      P->eb_f[l], (l == 0 && !e_is_zero) ? P->e_f : nullptr, &e,
                                      (l == 0 && e_is_zero) ? P->e_f : nullptr);
    if (rc) return rc;
  }
  if (use_cnn) {
    Timed t(P, CTF_T_CNN);
    CTF_HIP(cnn_apply_correction<float>(P->e_f, P->cnn_out, P->cnn_scale, c.n, P->dims[0].nd, P->cnn_level,
                                        P->stream));
  }
  float* cur = P->e_f;
  float* other = P->e_tmp_f;
  for (int s = 0; s < c.n_pg; ++s) {
    int rc = inner_finest32(P, cur, other, 1, 1.0f, nullptr, 1.0f, s == c.n_pg - 1 ? psi64 : nullptr);
    if (rc) return rc;
    std::swap(cur, other);
  }
  if (cur != P->e_f) CTF_HIP(launch_copy<float>(P->e_f, cur, P->dof(0), P->stream, P->active));
  return CTF_OK;
}

// Float64 residual of psi and its norm.  rho64 rounded to float32 goes to r_f (linear forms) or
// to rho_f[0] (full-approximation form, see refine_rest).  Returns ||rho||_W / ||b||_W through rel.
// the float64 residual and its squared norm (in P->scal[0]) without synchronising
int outer_residual_async(ctf_problem* P, const double* psi) {
  int rc = emission64(P, psi, true);
  if (rc) return rc;
  const int disc = P->cfg.discretisation;
  const size_t n = P->dof(0);
  if (disc == CTF_CONVFEM_PG) {
    // the same pass leaves psi rounded to float in e_f for refine_rest
    rc = finest64(P, psi, nullptr, 0, 1.0, P->rho_f[0], true, false, P->e_f);
    P->psi32_ready = rc == CTF_OK;
    return rc;
  }
  rc = finest64(P, psi, nullptr, 0, 1.0, P->r_f, true, false);
  if (rc) return rc;
  if (disc == CTF_CONVFEM_PG_FROZEN_K) {
    CTF_HIP(launch_convert_d2f(P->kx, P->kx_f, n, P->stream, P->active));
    CTF_HIP(launch_convert_d2f(P->ky, P->ky_f, n, P->stream, P->active));
  }
  return CTF_OK;
}

int outer_residual(ctf_problem* P, const double* psi, double* rel) {
  int rc = outer_residual_async(P, psi);
  if (rc) return rc;
  double nr = 0.0;
  rc = read_norm(P, &nr);
  if (rc) return rc;
  *rel = nr / P->bnorm;
  return CTF_OK;
}

// one refinement step after outer_residual: n_inner float32 cycles and the float64 update
int refine_rest(ctf_problem* P, double* psi, int max_inner, int* done, bool use_cnn = false) {
  const size_t n = P->dof(0);
  const bool fas = P->cfg.discretisation == CTF_CONVFEM_PG;
  if (fas) {
    // u = psi32 = psi64 rounded (left in e_f by the outer residual); b32 = A32(psi32) + rho64 into
    // r_f, with rho64 rounded in rho_f[0]: b32 = -(-rho64 + q(u) - L u)
    if (!P->psi32_ready) CTF_HIP(launch_convert_d2f(psi, P->e_f, n, P->stream, P->active));
    P->psi32_ready = false;
    int rc = inner_finest32(P, P->e_f, P->r_f, 0, -1.0f, P->rho_f[0], -1.0f);
    if (rc) return rc;
  }
  const int n_run = std::max(0, std::min(P->cfg.n_inner, max_inner));
  // full-approximation form: the last finest sweep of the last cycle applies psi += u - fl32(psi)
  const bool fused_update = fas && P->cfg.n_pg > 0;
  int it = 0;
  for (; it < n_run; ++it) {
    // The learned correction acts in the first float32 cycle of a refinement step only.  In the
    // full-approximation form the first cycle's residual b32 - A32(psi32) is rho64 up to float32
    // rounding, and rho64 rounded (in rho_f[0]) is taken for it.
    int rc = inner_cycle32(P, !fas && it == 0, use_cnn && it == 0, fas && it == 0,
                           fused_update && it + 1 == n_run ? psi : nullptr);
    if (rc) return rc;
  }
  if (it > 0) {
    if (fas) {
      if (!fused_update) CTF_HIP(launch_add_diff_f2d(psi, P->e_f, n, P->stream, P->active));   // psi += u - fl32(psi)
    } else {
      CTF_HIP(launch_add_f2d(psi, P->e_f, n, P->stream, P->active));
    }
  }
  if (done) *done = it;
  return CTF_OK;
}

// One solver step with no host synchronisation (graph-capturable): residual and its norm, the
// activity flag (0 once rel <= rtol; every later kernel of this problem then returns at once),
// then the rest of the cycle / refinement step.
int step_async(ctf_problem* P, double* psi, double rtol) {
  int rc;
  if (P->mixed()) {
    rc = outer_residual_async(P, psi);
  } else {
    rc = emission64(P, psi, true);
    if (!rc) rc = finest64(P, psi, P->rho[0], 0, 1.0, nullptr, true);
  }
  if (rc) return rc;
  CTF_HIP(launch_update_active(P->scal, P->bnorm, rtol, P->scal + 1, P->active, P->scal + 2, P->stream));
  return P->mixed() ? refine_rest(P, psi, P->cfg.n_inner, nullptr) : cycle_rest64(P, psi);
}

}  // namespace

// ================================================================================================
namespace {

// milliseconds per call of fn (events on the problem's stream; 1 warm-up, then reps calls)
template <typename F>
int time_ms(ctf_problem* P, F&& fn, int reps, double* ms) {
  hipEvent_t a, b;
  CTF_HIP(hipEventCreate(&a));
  CTF_HIP(hipEventCreate(&b));
  int rc = fn();
  if (!rc) {
    (void)hipEventRecord(a, P->stream);
    for (int r = 0; r < reps && !rc; ++r) rc = fn();
    (void)hipEventRecord(b, P->stream);
    (void)hipEventSynchronize(b);
    float t = 0.f;
    (void)hipEventElapsedTime(&t, a, b);
    *ms = double(t) / reps;
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return rc;
}

std::string tune_key(const ctf_problem* P) {
  std::ostringstream k;
  k << "p" << P->cfg.p << "_disc" << P->cfg.discretisation << "_prec" << P->cfg.precision << "_n" << P->cfg.n
    << "_nd" << P->dims[0].nd << "_g" << P->cfg.ngroups;
  return k.str();
}

// cache file: one JSON object, one entry per line: "key": {"strip_h": a, "corr_block": b, ...}
std::map<std::string, std::string> read_cache(const char* path) {
  std::map<std::string, std::string> m;
  std::ifstream in(path);
  std::string line;
  while (std::getline(in, line)) {
    const size_t q0 = line.find('"');
    if (q0 == std::string::npos) continue;
    const size_t q1 = line.find('"', q0 + 1);
    const size_t b0 = line.find('{', q1);
    const size_t b1 = line.rfind('}');
    if (q1 == std::string::npos || b0 == std::string::npos || b1 == std::string::npos || b1 < b0) continue;
    m[line.substr(q0 + 1, q1 - q0 - 1)] = line.substr(b0, b1 - b0 + 1);
  }
  return m;
}

int field(const std::string& obj, const char* name, double* v) {
  const std::string k = std::string("\"") + name + "\":";
  const size_t p = obj.find(k);
  if (p == std::string::npos) return 0;
  return std::sscanf(obj.c_str() + p + k.size(), "%lf", v) == 1;
}

}  // namespace

extern "C" {

void ctf_default_config(ctf_config* c) {
  if (!c) return;
  std::memset(c, 0, sizeof(*c));
  c->n = 32;
  c->length = 1.0;
  c->p = 1;
  c->na = 4;
  c->ngroups = 1;
  c->scatter_order = 0;
  c->discretisation = CTF_CONVFEM_PG;
  for (int s = 0; s < 4; ++s) c->bc[s] = CTF_VACUUM;
  c->precision = CTF_FP64;
  c->n_jacobi = 2;
  c->n_pg = 2;
  c->max_levels = 0;
  c->beta_pg = 3.0;
  c->alpha_r = 3.0;
  c->eps_k = 1e-3;
  c->n_inner = 4;   // measured fastest to 1e-6 on the 1024^2 x 512 workload (2: 1.044 s, 3: 0.981, 4: 0.956)
  c->cnn_level = -1;
  c->cnn_max_growth = 1.0;
  c->cnn_max_uses = 2;
  c->hemisphere = 0;
  c->coupled_scatter = 0;
  c->pg_isotropic = 0;
  c->pg_r_estimate = CTF_R_MIXED_MASS;
}

size_t ctf_workspace_bytes(const ctf_config* cfg) {
  if (validate(cfg) != CTF_OK) return 0;
  ctf_problem tmp;
  tmp.cfg = *cfg;
  init_dims(&tmp);
  return layout(&tmp, nullptr);
}

int ctf_create_problem(const ctf_config* cfg, const double* sigma_t, const double* sigma_s,
                       const double* source, void* workspace, size_t ws_bytes, void* stream,
                       ctf_problem** out) {
  int rc = validate(cfg);
  if (rc) return rc;
  if (!out || !sigma_t || !sigma_s || !source || !workspace)
    return fail(CTF_EINVAL, "null argument");
  ctf_problem* P = new ctf_problem();
  P->cfg = *cfg;
  P->stream = static_cast<hipStream_t>(stream);
  init_dims(P);
  const size_t need = layout(P, nullptr);
  if (ws_bytes < need) {
    delete P;
    return fail(CTF_ENOMEM, "workspace too small: need " + std::to_string(need) + " bytes");
  }
  // align the base to 256 bytes inside the caller's buffer
  char* base = static_cast<char*>(workspace);
  base += (256 - (reinterpret_cast<uintptr_t>(base) & 255)) & 255;
  layout(P, base);
  P->nmom = cfg->scatter_order ? 3 : 1;
  P->bc_vac = 0;
  for (int s = 0; s < 4; ++s)
    if (cfg->bc[s] == CTF_VACUUM) P->bc_vac |= 1 << s;
  const double h0 = cfg->length / cfg->n;
  const int p = cfg->discretisation == CTF_UPWIND ? 1 : cfg->p;
  {
    double m[2 * kMaxP + 1], d[2 * kMaxP + 1], k[2 * kMaxP + 1];
    convfem_stencils(p, m, d, k);
    for (int i = 0; i < 2 * kMaxP + 1; ++i) {
      const bool in = i < 2 * p + 1;
      P->st_d.m[i] = in ? m[i] : 0.0;
      P->st_d.d[i] = in ? d[i] / h0 : 0.0;
      P->st_d.k[i] = in ? k[i] / (h0 * h0) : 0.0;
      P->st_f.m[i] = float(P->st_d.m[i]);
      P->st_f.d[i] = float(P->st_d.d[i]);
      P->st_f.k[i] = float(P->st_d.k[i]);
    }
  }
  if (cfg->discretisation != CTF_UPWIND && cfg->pg_r_estimate != CTF_R_MIXED_MASS) {
    // the other degree of the low / high residual estimate
    const int q = cfg->pg_r_estimate == CTF_R_LOW ? p - 1 : p + 1;
    double m[2 * kMaxP + 1], d[2 * kMaxP + 1], k[2 * kMaxP + 1];
    convfem_stencils(q, m, d, k);
    for (int i = 0; i < 2 * kMaxP + 1; ++i) {
      const bool in = i < 2 * q + 1;
      P->st_d.mr[i] = in ? m[i] : 0.0;
      P->st_d.dr[i] = in ? d[i] / h0 : 0.0;
      P->st_f.mr[i] = float(P->st_d.mr[i]);
      P->st_f.dr[i] = float(P->st_d.dr[i]);
    }
  }
  P->pp.alpha_r = cfg->alpha_r;
  P->pp.eps_k = cfg->eps_k;
  P->pp.alpha_kabs = std::pow(2.0, p) / 16.0;
  P->pp.alpha_ksq = std::pow(2.0, p) / 2.0;
  P->pp.beta = cfg->beta_pg;
  P->pp.bc_vac = P->bc_vac;
  P->pp.isotropic = cfg->pg_isotropic;
  P->pp.r_estimate = cfg->discretisation == CTF_UPWIND ? 0 : cfg->pg_r_estimate;
  // default launch shape: the single-pass PG form up to p = 3 (at p = 3 on the 512^2 x 2048 x 4
  // workload with 256-row strips: float32 sweep 18.6 ms vs 11.7 + 8.1 ms stored-diffusivity, float64
  // residual 39.0 vs 22.4 + 17.4 ms), the stored-diffusivity form at p = 4 (not measured)
  P->pg_fused = cfg->p >= 4 ? 0 : 1;
  // strips of 256 rows instead of 128 once the PG launch still has at least eight rounds of the
  // chip's 4096 wavefront slots: fewer halo rows per output row (7p per strip), measured 2% faster
  // on the 1024^2 x 512 workload; smaller problems keep 128 rows to fill the chip.  Strips of 512
  // rows once that launch still has sixteen rounds (the 512^2 x 2048-ordinate x 4-group workload:
  // step 306 -> 302 ms; on 1024^2 x 512 ordinates, 4.75 rounds, 512 rows were 0.8% slower)
  {
    const long long ow = 64 - 4 * (cfg->p < 1 ? 1 : cfg->p);
    const long long planes = (cfg->hemisphere ? 4LL : 8LL) * cfg->na * cfg->na * cfg->ngroups;
    const long long ntx = (cfg->n + ow - 1) / ow;
    if (ntx * ((cfg->n + 255) / 256) * planes >= 8LL * 4096) P->strip_h = 256;
    if (ntx * ((cfg->n + 511) / 512) * planes >= 16LL * 4096) P->strip_h = 512;
  }

  hipStream_t s = P->stream;
  auto bail = [&](int code) {
    delete P;
    return code;
  };
  const int G = cfg->ngroups;
  const size_t nc0 = size_t(cfg->n) * cfg->n;
  const int nl = cfg->scatter_order + 1;
  // quadrature per level
  P->quad[0] = build_quadrature(cfg->na, cfg->hemisphere ? 4 : 8);
  for (int l = 1; l < P->L; ++l) P->quad[l] = coarsen_quadrature(P->quad[l - 1]);
  std::vector<std::vector<double>> hd(P->L);
  std::vector<std::vector<float>> hf(P->L);
  for (int l = 0; l < P->L; ++l) {
    const int nd = P->dims[l].nd;
    hd[l].resize(3 * nd);
    hf[l].resize(3 * nd);
    for (int n = 0; n < nd; ++n) {
      hd[l][n] = P->quad[l].mu[n];
      hd[l][nd + n] = P->quad[l].nu[n];
      hd[l][2 * nd + n] = P->quad[l].w[n];
    }
    for (int i = 0; i < 3 * nd; ++i) hf[l][i] = float(hd[l][i]);
    if (hipMemcpyAsync(P->dirs_d[l], hd[l].data(), 3 * nd * sizeof(double), hipMemcpyHostToDevice, s) ||
        hipMemcpyAsync(P->dirs_f[l], hf[l].data(), 3 * nd * sizeof(float), hipMemcpyHostToDevice, s))
      return bail(fail(CTF_EHIP, "copy of ordinates failed"));
  }
  if (hipMemcpyAsync(P->sigt_d[0], sigma_t, G * nc0 * sizeof(double), hipMemcpyDeviceToDevice, s) ||
      hipMemcpyAsync(P->sigma_s, sigma_s, nl * size_t(G) * G * nc0 * sizeof(double),
                     hipMemcpyDeviceToDevice, s) ||
      hipMemcpyAsync(P->source, source, G * nc0 * sizeof(double), hipMemcpyDeviceToDevice, s))
    return bail(fail(CTF_EHIP, "copy of materials failed"));
  for (int l = 1; l < P->L; ++l) {
    if (launch_harmonic_coarsen(P->sigt_d[l - 1], P->sigt_d[l], G, P->dims[l].n, s))
      return bail(fail(CTF_EHIP, "harmonic coarsening failed"));
    if (cfg->coupled_scatter && launch_harmonic_coarsen(P->sigs_d[l - 1], P->sigs_d[l], nl * G * G, P->dims[l].n, s))
      return bail(fail(CTF_EHIP, "harmonic coarsening failed"));
  }
  if (P->mixed()) {
    for (int l = 0; l < P->L; ++l)
      if (launch_convert_d2f(P->sigt_d[l], P->sigt_f[l], G * size_t(P->dims[l].n) * P->dims[l].n, s))
        return bail(fail(CTF_EHIP, "conversion failed"));
    if (launch_convert_d2f(P->sigma_s, P->sigma_s_f, nl * size_t(G) * G * nc0, s))
      return bail(fail(CTF_EHIP, "conversion failed"));
    for (int l = 1; l < P->L && cfg->coupled_scatter; ++l)
      if (launch_convert_d2f(P->sigs_d[l], P->sigs_f[l], nl * size_t(G) * G * P->dims[l].n * P->dims[l].n, s))
        return bail(fail(CTF_EHIP, "conversion failed"));
  }
  if (launch_set_int(P->active, 1, s)) return bail(fail(CTF_EHIP, "flag init failed"));
  if (cfg->cnn_level >= 0) {
    if (cfg->cnn_level >= P->L) return bail(fail(CTF_EINVAL, "cnn_level beyond the coarsest level"));
    const int lc = cfg->cnn_level, nc = P->dims[lc].n;
    P->cnn_level = lc;
    if (cnn_static_features(P->sigt_d[lc], P->sigma_s, P->sigt_d[0], P->cnn_feat + size_t(nc) * nc,
                            P->cnn_feat + 2 * size_t(nc) * nc, cfg->n, lc, P->dims[lc].h, s))
      return bail(fail(CTF_EHIP, "learned-correction features failed"));
  }
  // ||b||_W with b = S / (4 pi): sum_n w_n = 4 pi, so ||b||^2 = h^2 sum S^2 / (4 pi)
  std::vector<double> src(G * nc0);
  if (hipMemcpyAsync(src.data(), source, G * nc0 * sizeof(double), hipMemcpyDeviceToHost, s) ||
      hipStreamSynchronize(s))
    return bail(fail(CTF_EHIP, "source copy / sync failed"));
  double ss = 0.0;
  for (double v : src) ss += v * v;
  P->bnorm = std::sqrt(ss * h0 * h0 / (4.0 * M_PI));
  if (!(P->bnorm > 0.0)) P->bnorm = 1.0;  // no external source: report absolute norms
  *out = P;
  return CTF_OK;
}

void ctf_destroy_problem(ctf_problem* P) { delete P; }

int ctf_num_levels(const ctf_problem* P) { return P ? P->L : 0; }

int ctf_level_info(const ctf_problem* P, int level, ctf_level_desc* out) {
  int rc = check_level(P, level);
  if (rc) return rc;
  if (!out) return fail(CTF_EINVAL, "null out");
  out->n = P->dims[level].n;
  out->na = P->dims[level].na;
  out->n_dir = P->dims[level].nd;
  out->h = P->dims[level].h;
  out->dof = static_cast<long long>(P->dof(level));
  return CTF_OK;
}

int ctf_level_quadrature(const ctf_problem* P, int level, double* mu, double* nu, double* w) {
  int rc = check_level(P, level);
  if (rc) return rc;
  const Quadrature& q = P->quad[level];
  const size_t nd = q.w.size();
  if (mu) std::memcpy(mu, q.mu.data(), nd * sizeof(double));
  if (nu) std::memcpy(nu, q.nu.data(), nd * sizeof(double));
  if (w) std::memcpy(w, q.w.data(), nd * sizeof(double));
  return CTF_OK;
}

int ctf_convfem_stencils(int p, double* m, double* d, double* k) {
  if (p < 1 || p > kMaxP) return fail(CTF_EINVAL, "p must be 1..4");
  double mm[2 * kMaxP + 1], dd[2 * kMaxP + 1], kk[2 * kMaxP + 1];
  convfem_stencils(p, mm, dd, kk);
  for (int i = 0; i < 2 * p + 1; ++i) {
    if (m) m[i] = mm[i];
    if (d) d[i] = dd[i];
    if (k) k[i] = kk[i];
  }
  return CTF_OK;
}

int ctf_quadrature(int na, double* mu, double* nu, double* w) {
  if (!is_pow2(na)) return fail(CTF_EINVAL, "na must be a power of two");
  const Quadrature q = build_quadrature(na);
  const size_t nd = q.w.size();
  if (mu) std::memcpy(mu, q.mu.data(), nd * sizeof(double));
  if (nu) std::memcpy(nu, q.nu.data(), nd * sizeof(double));
  if (w) std::memcpy(w, q.w.data(), nd * sizeof(double));
  return CTF_OK;
}

int ctf_level_sigma_t(const ctf_problem* P, int level, double* out) {
  int rc = check_level(P, level);
  if (rc) return rc;
  const size_t cnt = size_t(P->dims[level].G) * P->dims[level].n * P->dims[level].n;
  CTF_HIP(hipMemcpyAsync(out, P->sigt_d[level], cnt * sizeof(double), hipMemcpyDeviceToDevice, P->stream));
  return CTF_OK;
}

int ctf_apply_operator(ctf_problem* P, const double* psi, double* out, int mode) {
  if (!P || !psi || !out) return fail(CTF_EINVAL, "null argument");
  if (mode != CTF_OP_APPLY && mode != CTF_OP_RESIDUAL) return fail(CTF_EINVAL, "bad mode");
  if (psi == out) return fail(CTF_EINVAL, "psi and out must not alias");
  int rc = emission64(P, psi, mode == CTF_OP_RESIDUAL);
  if (rc) return rc;
  return finest64(P, psi, out, 0, mode == CTF_OP_RESIDUAL ? 1.0 : -1.0);
}

int ctf_moments(ctf_problem* P, const double* psi, double* phi) {
  if (!P || !psi || !phi) return fail(CTF_EINVAL, "null argument");
  CTF_HIP(launch_moments<double>(P->ld(0), psi, phi, 3, P->stream));
  return CTF_OK;
}

int ctf_moments_f32(ctf_problem* P, const float* psi, float* phi, int use_mfma) {
  if (!P || !psi || !phi) return fail(CTF_EINVAL, "null argument");
  if (!P->mixed()) return fail(CTF_EINVAL, "float32 moments need a mixed-precision problem");
  if (use_mfma) {
    Timed t(P, CTF_T_MOMENTS_MFMA);
    CTF_HIP(launch_moments_mfma(P->lf(0), psi, phi, 3, P->stream));
  } else {
    Timed t(P, CTF_T_MOMENTS);
    CTF_HIP(launch_moments<float>(P->lf(0), psi, phi, 3, P->stream));
  }
  return CTF_OK;
}

int ctf_freeze_k(ctf_problem* P, const double* psi, double* kx, double* ky) {
  if (!P || !psi) return fail(CTF_EINVAL, "null argument");
  if (P->cfg.discretisation == CTF_UPWIND) return fail(CTF_EINVAL, "upwind has no diffusivities");
  int rc = emission64(P, psi, true);
  if (rc) return rc;
  PGLaunch<double> o;
  o.psi = psi;
  o.E = P->E;
  o.nmomE = P->nmom;
  o.kx_out = P->kx;
  o.ky_out = P->ky;
  o.strip_h = P->strip_h;
  {
    Timed t(P, CTF_T_PGK64);
    CTF_HIP(launch_pg_diffusivity<double>(P->cfg.p, P->ld(0), P->st_d, P->pp, o, P->stream));
  }
  P->k_held = true;
  const size_t bytes = P->dof(0) * sizeof(double);
  if (kx) CTF_HIP(hipMemcpyAsync(kx, P->kx, bytes, hipMemcpyDeviceToDevice, P->stream));
  if (ky) CTF_HIP(hipMemcpyAsync(ky, P->ky, bytes, hipMemcpyDeviceToDevice, P->stream));
  return CTF_OK;
}

int ctf_smooth(ctf_problem* P, int level, int kind, double* x, const double* rhs, int nsweeps) {
  int rc = check_level(P, level);
  if (rc) return rc;
  if (!x || nsweeps < 0) return fail(CTF_EINVAL, "bad argument");
  if (kind == CTF_SMOOTH_UPWIND) {
    if (!rhs) return fail(CTF_EINVAL, "upwind smoothing needs rhs");
    if (nsweeps == 0) return CTF_OK;
    const double* res = nullptr;
    rc = correction_sweeps<double>(P, P->ld(level), level, x, 0, rhs, nsweeps, P->ea[level],
                                   P->eb[level], nullptr, &res);
    if (rc) return rc;
    CTF_HIP(hipMemcpyAsync(x, res, P->dof(level) * sizeof(double), hipMemcpyDeviceToDevice, P->stream));
    return CTF_OK;
  }
  if (kind == CTF_SMOOTH_FINEST) {
    if (level != 0 || rhs) return fail(CTF_EINVAL, "finest smoothing: level 0 and rhs = NULL");
    double* cur = x;
    double* other = P->psi_tmp;
    for (int s = 0; s < nsweeps; ++s) {
      rc = emission64(P, cur, true);
      if (rc) return rc;
      rc = finest64(P, cur, other, 1, 1.0);
      if (rc) return rc;
      std::swap(cur, other);
    }
    if (cur != x)
      CTF_HIP(hipMemcpyAsync(x, cur, P->dof(0) * sizeof(double), hipMemcpyDeviceToDevice, P->stream));
    return CTF_OK;
  }
  return fail(CTF_EINVAL, "bad smoother kind");
}

int ctf_restrict(ctf_problem* P, int level, const double* fine, double* coarse) {
  int rc = check_level(P, level);
  if (rc) return rc;
  if (level + 1 >= P->L) return fail(CTF_EINVAL, "no coarser level");
  CTF_HIP(launch_restrict<double>(P->ld(level), P->ld(level + 1), fine, coarse, P->stream));
  return CTF_OK;
}

int ctf_prolong(ctf_problem* P, int level, const double* coarse, double* fine) {
  int rc = check_level(P, level);
  if (rc) return rc;
  if (level + 1 >= P->L) return fail(CTF_EINVAL, "no coarser level");
  CTF_HIP(launch_prolong<double>(P->ld(level), P->dims[level + 1].nd, coarse, fine, P->stream));
  return CTF_OK;
}

int ctf_norm(ctf_problem* P, const double* v, double* out) {
  if (!P || !v || !out) return fail(CTF_EINVAL, "null argument");
  return wnorm64(P, 0, v, out);
}

int ctf_mg_cycle(ctf_problem* P, double* psi, double* rel_res) {
  if (!P || !psi) return fail(CTF_EINVAL, "null argument");
  if (P->cfg.discretisation == CTF_CONVFEM_PG_FROZEN_K && !P->k_held)
    return fail(CTF_EINVAL, "frozen-k discretisation needs ctf_freeze_k first");
  if (P->mixed()) {
    // one refinement step: float64 residual, n_inner float32 cycles, float64 update
    double rel = 0.0;
    int rc = outer_residual(P, psi, &rel);
    if (rc) return rc;
    if (rel_res) *rel_res = rel;
    return refine_rest(P, psi, P->cfg.n_inner, nullptr);
  }
  int rc = emission64(P, psi, true);
  if (rc) return rc;
  rc = finest64(P, psi, P->rho[0], 0, 1.0, nullptr, rel_res != nullptr);
  if (rc) return rc;
  if (rel_res) {
    double nr = 0.0;
    rc = read_norm(P, &nr);
    if (rc) return rc;
    *rel_res = nr / P->bnorm;
  }
  return cycle_rest64(P, psi);
}

int ctf_solve(ctf_problem* P, double* psi, double rtol, int max_cycles, ctf_solve_info* info) {
  if (!P || !psi || max_cycles < 0) return fail(CTF_EINVAL, "bad argument");
  if (P->cfg.discretisation == CTF_CONVFEM_PG_FROZEN_K && !P->k_held)
    return fail(CTF_EINVAL, "frozen-k discretisation needs ctf_freeze_k first");
  const auto t0 = std::chrono::steady_clock::now();
  const size_t n = P->dof(0);
  CTF_HIP(launch_set_int(P->active, 1, P->stream));
  int cycles = 0, outer = 0, nhist = 0, applied = 0, rejected = 0;
  double rel = 0.0, prev = 0.0;
  bool last_used_cnn = false;
  int status = CTF_NOT_CONVERGED;
  for (;;) {
    int rc;
    if (P->mixed()) {
      rc = outer_residual(P, psi, &rel);
    } else {
      rc = emission64(P, psi, true);
      if (!rc) rc = finest64(P, psi, P->rho[0], 0, 1.0, nullptr, true);
      if (!rc) {
        double nr = 0.0;
        rc = read_norm(P, &nr);
        rel = nr / P->bnorm;
      }
    }
    // plain multigrid is the fallback and the arbiter: a step with the learned correction that
    // raised the residual (or made it non-finite) is undone and the correction switched off
    if (last_used_cnn && (rc == CTF_ENONFINITE || (rc == CTF_OK && rel > P->cfg.cnn_max_growth * prev))) {
      CTF_HIP(hipMemcpyAsync(psi, P->cnn_backup, n * sizeof(double), hipMemcpyDeviceToDevice, P->stream));
      P->cnn_on = false;
      rejected = 1;
      last_used_cnn = false;
      continue;
    }
    if (rc) return rc;
    if (info && info->history && nhist < info->history_len) info->history[nhist] = rel;
    ++nhist;
    if (rel <= rtol) {
      status = CTF_OK;
      break;
    }
    if (cycles >= max_cycles) break;
    const bool use_cnn = P->cnn_on && P->cnn_ready && applied < P->cfg.cnn_max_uses;
    if (use_cnn)
      CTF_HIP(hipMemcpyAsync(P->cnn_backup, psi, n * sizeof(double), hipMemcpyDeviceToDevice, P->stream));
    if (P->mixed()) {
      int done = 0;
      rc = refine_rest(P, psi, max_cycles - cycles, &done, use_cnn);
      if (rc) return rc;
      cycles += done;
      ++outer;
    } else {
      rc = cycle_rest64(P, psi, use_cnn);
      if (rc) return rc;
      ++cycles;
    }
    applied += use_cnn ? 1 : 0;
    last_used_cnn = use_cnn;
    prev = rel;
  }
  CTF_HIP(hipStreamSynchronize(P->stream));
  if (info) {
    info->cycles = cycles;
    info->outer_steps = outer;
    info->rel_residual = rel;
    info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    info->cnn_applied = applied;
    info->cnn_rejected = rejected;
  }
  return status;
}

int ctf_solve_batch(ctf_problem* const* probs, int nprob, double* const* psis, double rtol, int max_steps,
                    int steps_per_graph, ctf_solve_info* infos) {
  if (!probs || !psis || nprob < 1 || max_steps < 0 || steps_per_graph < 1)
    return fail(CTF_EINVAL, "bad argument");
  for (int i = 0; i < nprob; ++i) {
    if (!probs[i] || !psis[i]) return fail(CTF_EINVAL, "null problem or psi");
    if (probs[i]->cfg.discretisation == CTF_CONVFEM_PG_FROZEN_K && !probs[i]->k_held)
      return fail(CTF_EINVAL, "frozen-k discretisation needs ctf_freeze_k first");
    for (int j = 0; j < i; ++j)
      if (probs[j] == probs[i]) return fail(CTF_EINVAL, "a problem appears twice in the batch");
  }
  const auto t0 = std::chrono::steady_clock::now();
  hipStream_t s0 = nullptr;  // the capture origin: a stream of our own (the default stream cannot be captured)
  const int ns = std::min(nprob, 8);
  std::vector<hipStream_t> streams(ns, nullptr);
  std::vector<hipEvent_t> joins(ns, nullptr);
  hipEvent_t fork = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<hipStream_t> saved(nprob);
  std::vector<bool> timing(nprob);
  int rc = CTF_OK;
  auto cleanup = [&]() {
    for (int i = 0; i < nprob; ++i) {
      probs[i]->stream = saved[i] ? saved[i] : probs[i]->stream;
      // every problem leaves active again: the flag gates all of its kernels, also outside a batch
      (void)launch_set_int(probs[i]->active, 1, probs[i]->stream);
      (void)hipStreamSynchronize(probs[i]->stream);
    }
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (fork) (void)hipEventDestroy(fork);
    for (auto e : joins)
      if (e) (void)hipEventDestroy(e);
    for (auto st : streams)
      if (st) (void)hipStreamDestroy(st);
    if (s0) (void)hipStreamDestroy(s0);
  };
  // every problem restarts active, with its step counter at zero; all prior work finished
  for (int i = 0; i < nprob; ++i) {
    ctf_problem* P = probs[i];
    saved[i] = P->stream;
    if (launch_set_int(P->active, 1, P->stream) != hipSuccess ||
        hipMemsetAsync(P->scal, 0, 8 * sizeof(double), P->stream) != hipSuccess ||
        hipStreamSynchronize(P->stream) != hipSuccess) {
      cleanup();
      return fail(CTF_EHIP, "batch initialisation failed");
    }
    saved[i] = nullptr;
  }
  if (hipEventCreateWithFlags(&fork, hipEventDisableTiming) != hipSuccess ||
      hipStreamCreateWithFlags(&s0, hipStreamNonBlocking) != hipSuccess) {
    cleanup();
    return fail(CTF_EHIP, "event / stream creation failed");
  }
  for (int k = 0; k < ns; ++k)
    if (hipStreamCreateWithFlags(&streams[k], hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&joins[k], hipEventDisableTiming) != hipSuccess) {
      cleanup();
      return fail(CTF_EHIP, "stream creation failed");
    }
  // capture: steps_per_graph steps of every problem, problems spread over ns parallel branches
  if (hipStreamBeginCapture(s0, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    cleanup();
    return fail(CTF_EHIP, "stream capture failed to start");
  }
  bool cap_ok = hipEventRecord(fork, s0) == hipSuccess;
  for (int k = 0; k < ns && cap_ok; ++k) cap_ok = hipStreamWaitEvent(streams[k], fork, 0) == hipSuccess;
  for (int i = 0; i < nprob && cap_ok && rc == CTF_OK; ++i) {
    ctf_problem* P = probs[i];
    saved[i] = P->stream;
    timing[i] = P->timing;
    P->timing = false;
    P->stream = streams[i % ns];
    for (int r = 0; r < steps_per_graph && rc == CTF_OK; ++r) rc = step_async(P, psis[i], rtol);
    P->stream = saved[i];
    P->timing = timing[i];
    saved[i] = nullptr;
  }
  for (int k = 0; k < ns && cap_ok; ++k)
    cap_ok = hipEventRecord(joins[k], streams[k]) == hipSuccess &&
             hipStreamWaitEvent(s0, joins[k], 0) == hipSuccess;
  const hipError_t ec = hipStreamEndCapture(s0, &graph);
  if (rc != CTF_OK || !cap_ok || ec != hipSuccess) {
    cleanup();
    return rc != CTF_OK ? rc : fail(CTF_EHIP, "stream capture of the batched step failed");
  }
  if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
    cleanup();
    return fail(CTF_EHIP, "graph instantiation failed");
  }
  // replay until every problem is inactive (converged) or the step budget is spent
  std::vector<double> host(3 * size_t(nprob));
  std::vector<int> act(nprob, 1);
  int launched = 0;
  int status = CTF_NOT_CONVERGED;
  while (launched < max_steps) {
    if (hipGraphLaunch(exec, s0) != hipSuccess) {
      cleanup();
      return fail(CTF_EHIP, "graph launch failed");
    }
    launched += steps_per_graph;
    for (int i = 0; i < nprob; ++i)
      if (hipMemcpyAsync(&host[3 * i], probs[i]->scal, 3 * sizeof(double), hipMemcpyDeviceToHost, s0) != hipSuccess ||
          hipMemcpyAsync(&act[i], probs[i]->active, sizeof(int), hipMemcpyDeviceToHost, s0) != hipSuccess) {
        cleanup();
        return fail(CTF_EHIP, "status copy failed");
      }
    if (hipStreamSynchronize(s0) != hipSuccess) {
      cleanup();
      return fail(CTF_EHIP, "synchronisation failed");
    }
    bool any = false, bad = false;
    for (int i = 0; i < nprob; ++i) {
      any = any || act[i];
      bad = bad || !std::isfinite(host[3 * i + 1]);
    }
    if (bad) {
      cleanup();
      return fail(CTF_ENONFINITE, "non-finite residual norm in the batch");
    }
    if (!any) {
      status = CTF_OK;
      break;
    }
  }
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (infos) {
    for (int i = 0; i < nprob; ++i) {
      const int steps = int(host[3 * i + 2]);
      const bool mixed = probs[i]->mixed();
      infos[i].cycles = mixed ? steps * probs[i]->cfg.n_inner : steps;
      infos[i].outer_steps = mixed ? steps : 0;
      infos[i].rel_residual = host[3 * i + 1];
      infos[i].seconds = secs;
      infos[i].cnn_applied = 0;
      infos[i].cnn_rejected = 0;
    }
  }
  cleanup();
  return status;
}

namespace {
// One solver step of every problem recorded as a tape of operations (the launches step_async makes,
// not launched); the problems' timers are off while recording.
struct TapeSet {
  std::vector<PersistTape*> tapes;
  ~TapeSet() {
    for (PersistTape* t : tapes) tape_free(t);
  }
};

int record_steps(ctf_problem* const* probs, int nprob, double* const* psis, double rtol, TapeSet* ts) {
  for (int i = 0; i < nprob; ++i) {
    ctf_problem* P = probs[i];
    if (P->cfg.discretisation != CTF_UPWIND || P->cfg.coupled_scatter || P->cnn_on)
      return fail(CTF_EUNSUPPORTED, "the persistent batch runs the upwind discretisation without scattering-coupled "
                                    "sweeps or the learned correction");
    const bool timing = P->timing;
    P->timing = false;
    ts->tapes.push_back(tape_open());
    const int rc = step_async(P, psis ? psis[i] : nullptr, rtol);
    tape_close();
    P->timing = timing;
    if (rc != CTF_OK) return rc;
    if (!tape_usable(ts->tapes.back())) return fail(CTF_EUNSUPPORTED, "a step of this problem cannot be recorded");
  }
  return CTF_OK;
}

int persist_items_per_block(int v) { return v > 0 ? v : 1; }
constexpr unsigned kPersistSpinLimit = 1u << 21;   // polls (about 2 us each) of one bounded wait
}  // namespace

size_t ctf_solve_batch_persistent_bytes(ctf_problem* const* probs, int nprob, int items_per_block) {
  if (!probs || nprob < 1 || items_per_block < 0) return 0;
  for (int i = 0; i < nprob; ++i)
    if (!probs[i]) return 0;
  TapeSet ts;
  if (record_steps(probs, nprob, nullptr, 0.0, &ts) != CTF_OK) return 0;
  int blocks = 0;
  if (persist_grid(&blocks) != hipSuccess) return 0;
  return persist_workspace_bytes(ts.tapes.data(), nprob, blocks, persist_items_per_block(items_per_block));
}

int ctf_solve_batch_persistent(ctf_problem* const* probs, int nprob, double* const* psis, double rtol, int max_steps,
                               int items_per_block, void* workspace, size_t ws_bytes, ctf_solve_info* infos) {
  if (!probs || !psis || nprob < 1 || max_steps < 1 || items_per_block < 0) return fail(CTF_EINVAL, "bad argument");
  for (int i = 0; i < nprob; ++i) {
    if (!probs[i] || !psis[i]) return fail(CTF_EINVAL, "null problem or psi");
    for (int j = 0; j < i; ++j)
      if (probs[j] == probs[i]) return fail(CTF_EINVAL, "a problem appears twice in the batch");
  }
  const auto t0 = std::chrono::steady_clock::now();
  TapeSet ts;
  int rc = record_steps(probs, nprob, psis, rtol, &ts);
  if (rc != CTF_OK) return rc;
  int blocks = 0;
  CTF_HIP(persist_grid(&blocks));
  const int ipb = persist_items_per_block(items_per_block);
  const size_t need = persist_workspace_bytes(ts.tapes.data(), nprob, blocks, ipb);
  if (!workspace || ws_bytes < need) return fail(CTF_ENOMEM, "workspace too small for the persistent batch");
  if (reinterpret_cast<uintptr_t>(workspace) & 255) return fail(CTF_EINVAL, "workspace must be 256-byte aligned");
  // every problem restarts active with its step counter at zero; all prior work finished
  for (int i = 0; i < nprob; ++i) {
    ctf_problem* P = probs[i];
    CTF_HIP(launch_set_int(P->active, 1, P->stream));
    CTF_HIP(hipMemsetAsync(P->scal, 0, 8 * sizeof(double), P->stream));
    CTF_HIP(hipStreamSynchronize(P->stream));
  }
  PersistResult res;
  CTF_HIP(persist_solve(ts.tapes.data(), nprob, max_steps, blocks, ipb, kPersistSpinLimit, workspace, ws_bytes,
                        probs[0]->stream, &res));
  std::vector<double> host(3 * size_t(nprob));
  std::vector<int> act(nprob, 1);
  for (int i = 0; i < nprob; ++i) {
    CTF_HIP(hipMemcpyAsync(&host[3 * i], probs[i]->scal, 3 * sizeof(double), hipMemcpyDeviceToHost,
                           probs[0]->stream));
    CTF_HIP(hipMemcpyAsync(&act[i], probs[i]->active, sizeof(int), hipMemcpyDeviceToHost, probs[0]->stream));
  }
  CTF_HIP(hipStreamSynchronize(probs[0]->stream));
  // every problem leaves active again: the flag gates all of its kernels, also outside a batch
  for (int i = 0; i < nprob; ++i) CTF_HIP(launch_set_int(probs[i]->active, 1, probs[0]->stream));
  CTF_HIP(hipStreamSynchronize(probs[0]->stream));
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  bool any = false;
  for (int i = 0; i < nprob; ++i) {
    any = any || act[i];
    if (infos) {
      const int steps = int(host[3 * i + 2]);
      const bool mixed = probs[i]->mixed();
      infos[i].cycles = mixed ? steps * probs[i]->cfg.n_inner : steps;
      infos[i].outer_steps = mixed ? steps : 0;
      infos[i].rel_residual = host[3 * i + 1];
      infos[i].seconds = secs;
      infos[i].cnn_applied = 0;
      infos[i].cnn_rejected = 0;
    }
  }
  if (res.error == kPersistNonFinite) return fail(CTF_ENONFINITE, "non-finite residual norm in the batch");
  if (res.error == kPersistSpin)
    return fail(CTF_EHIP, "a bounded wait of the persistent batch ran out (were all its blocks resident?)");
  return any ? CTF_NOT_CONVERGED : CTF_OK;
}

int ctf_set_launch_shape(ctf_problem* P, int strip_h, int corr_block, int pg_fused) {
  if (!P) return fail(CTF_EINVAL, "null problem");
  if (strip_h < 8 || strip_h > 512 || corr_block < 64 || corr_block > 1024 || corr_block % 64 ||
      (pg_fused != 0 && pg_fused != 1))
    return fail(CTF_EINVAL, "strip_h in [8, 512], corr_block a multiple of 64 in [64, 1024], pg_fused 0/1");
  P->strip_h = strip_h;
  P->corr_block = corr_block;
  P->pg_fused = pg_fused;
  return CTF_OK;
}

int ctf_get_launch_shape(const ctf_problem* P, int* strip_h, int* corr_block, int* pg_fused) {
  if (!P) return fail(CTF_EINVAL, "null problem");
  if (strip_h) *strip_h = P->strip_h;
  if (corr_block) *corr_block = P->corr_block;
  if (pg_fused) *pg_fused = P->pg_fused;
  return CTF_OK;
}

int ctf_autotune(ctf_problem* P, const char* cache_path, int force, int* strip_h, int* corr_block,
                 int* pg_fused) {
  if (!P) return fail(CTF_EINVAL, "null problem");
  const std::string key = tune_key(P);
  std::map<std::string, std::string> cache;
  if (cache_path) cache = read_cache(cache_path);
  auto it = cache.find(key);
  double a = 0, b = 0;
  double f = 0;
  if (!force && it != cache.end() && field(it->second, "strip_h", &a) && field(it->second, "corr_block", &b)) {
    (void)field(it->second, "pg_fused", &f);
    int rc = ctf_set_launch_shape(P, int(a), int(b), int(f));
    if (rc) return rc;
  } else {
    const ctf_config& c = P->cfg;
    const size_t n = P->dof(0);
    // scratch inputs: zero fields (the timing does not depend on the values)
    CTF_HIP(hipMemsetAsync(P->ea[0], 0, n * sizeof(double), P->stream));
    CTF_HIP(hipMemsetAsync(P->eb[0], 0, n * sizeof(double), P->stream));
    if (P->mixed()) {
      CTF_HIP(hipMemsetAsync(P->ea_f[0], 0, n * sizeof(float), P->stream));
      CTF_HIP(hipMemsetAsync(P->r_f, 0, n * sizeof(float), P->stream));
      if (P->kx_f) {
        CTF_HIP(hipMemsetAsync(P->kx_f, 0, n * sizeof(float), P->stream));
        CTF_HIP(hipMemsetAsync(P->ky_f, 0, n * sizeof(float), P->stream));
      }
      CTF_HIP(hipMemsetAsync(P->E_f, 0, 3 * size_t(c.ngroups) * c.n * c.n * sizeof(float), P->stream));
    }
    int rc = emission64(P, P->ea[0], true);
    if (rc) return rc;
    const bool saved_timing = P->timing;
    P->timing = false;
    double best_pg = 1e30, best_corr = 1e30;
    int best_h = P->strip_h, best_b = P->corr_block;
    int best_f = P->pg_fused;
    if (c.discretisation != CTF_UPWIND) {
      for (int fz = 0; fz < (c.discretisation == CTF_CONVFEM_PG ? 2 : 1); ++fz)
      for (int h : {8, 16, 32, 64, 128, 256, 512}) {
        P->strip_h = h;
        P->pg_fused = fz;
        double ms = 0.0;
        if (P->mixed()) {
          PGLaunch<float> o;
          o.psi = P->ea_f[0];
          o.E = P->E_f;
          o.nmomE = P->nmom;
          if (c.discretisation == CTF_CONVFEM_PG_FROZEN_K) {
            o.kx_in = P->kx_f;
            o.ky_in = P->ky_f;
          } else if (!fz) {
            o.kx_out = P->kx_f;
            o.ky_out = P->ky_f;
          }
          o.out = P->eb_f[0];
          o.rhs = P->r_f;
          o.mode = 1;
          o.strip_h = h;
          rc = time_ms(P, [&]() -> int { return launch_pg<float>(c.p, P->lf(0), P->st_f, P->pp, o, P->stream)
                                                     ? CTF_EHIP : CTF_OK; }, 5, &ms);
        } else {
          rc = time_ms(P, [&]() { return finest64(P, P->ea[0], P->eb[0], 1, 1.0); }, 5, &ms);
        }
        if (rc) break;
        if (ms < best_pg) {
          best_pg = ms;
          best_h = h;
          best_f = fz;
        }
      }
    }
    for (int bsz : {64, 128, 256, 512, 1024}) {
      if (rc) break;
      P->corr_block = bsz;
      double ms = 0.0;
      if (P->mixed())
        rc = time_ms(P, [&]() -> int { return launch_upwind_correction<float>(P->lf(0), P->bc_vac, P->ea_f[0], 0, 1,
                                                  P->r_f, P->eb_f[0], nullptr, P->stream, bsz) ? CTF_EHIP : CTF_OK; }, 5, &ms);
      else
        rc = time_ms(P, [&]() -> int { return launch_upwind_correction<double>(P->ld(0), P->bc_vac, P->ea[0], 0, 1,
                                                  P->rho[0], P->eb[0], nullptr, P->stream, bsz) ? CTF_EHIP : CTF_OK; }, 5, &ms);
      if (!rc && ms < best_corr) {
        best_corr = ms;
        best_b = bsz;
      }
    }
    P->timing = saved_timing;
    P->strip_h = best_h;
    P->corr_block = best_b;
    P->pg_fused = best_f;
    if (rc) return rc;
    if (cache_path) {
      std::ostringstream e;
      e << "{\"strip_h\": " << best_h << ", \"corr_block\": " << best_b << ", \"pg_fused\": " << best_f
        << ", \"pg_ms\": "
        << (best_pg < 1e30 ? best_pg : 0.0) << ", \"corr_ms\": " << best_corr << "}";
      cache[key] = e.str();
      std::ofstream outf(cache_path, std::ios::trunc);
      if (!outf) return fail(CTF_EINVAL, std::string("cannot write autotune cache ") + cache_path);
      outf << "{\n";
      size_t i = 0;
      for (const auto& kv : cache) outf << "  \"" << kv.first << "\": " << kv.second << (++i < cache.size() ? ",\n" : "\n");
      outf << "}\n";
    }
  }
  if (strip_h) *strip_h = P->strip_h;
  if (corr_block) *corr_block = P->corr_block;
  if (pg_fused) *pg_fused = P->pg_fused;
  return CTF_OK;
}

int ctf_cnn_param_count(void) { return cnn_param_count(); }

size_t ctf_cnn_workspace_bytes(int batch, int h, int w) {
  if (batch < 1 || h < 1 || w < 1) return 0;
  return cnn_workspace_bytes(batch, h, w);
}

int ctf_cnn_forward(const float* params, const float* in, float* out, int batch, int h, int w, int bf16,
                    void* workspace, size_t ws_bytes, void* stream) {
  if (!params || !in || !out || !workspace || batch < 1 || h < 1 || w < 1)
    return fail(CTF_EINVAL, "bad argument");
  if (ws_bytes < cnn_workspace_bytes(batch, h, w)) return fail(CTF_ENOMEM, "network workspace too small");
  CTF_HIP(cnn_forward(params, in, out, batch, h, w, bf16, workspace, static_cast<hipStream_t>(stream)));
  return CTF_OK;
}

int ctf_cnn_forward_noalloc(const float* params, const float* in, float* out, int batch, int h, int w, int bf16,
                            void* stream) {
  if (!params || !in || !out || batch < 1 || h < 1 || w < 1) return fail(CTF_EINVAL, "bad argument");
  if (size_t(batch) * size_t(h) * size_t(w) > kCnnScratchPixels)
    return fail(CTF_EINVAL, "batch * h * w exceeds the no-allocation limit of " +
                                std::to_string(kCnnScratchPixels) + " pixels");
  CTF_HIP(cnn_forward_noalloc(params, in, out, batch, h, w, bf16, static_cast<hipStream_t>(stream)));
  return CTF_OK;
}

int ctf_cnn_loss_grad(const float* params, const float* in, const float* target, int batch, int h, int w,
                      int bf16, float* grad, double* loss, void* workspace, size_t ws_bytes, void* stream) {
  if (!params || !in || !target || !grad || !loss || !workspace || batch < 1 || h < 1 || w < 1)
    return fail(CTF_EINVAL, "bad argument");
  if (ws_bytes < cnn_workspace_bytes(batch, h, w)) return fail(CTF_ENOMEM, "network workspace too small");
  CTF_HIP(cnn_loss_grad(params, in, target, batch, h, w, bf16, grad, loss, workspace,
                        static_cast<hipStream_t>(stream)));
  return CTF_OK;
}

int ctf_cnn_adam(float* params, float* m, float* v, const float* grad, int n, int step, float lr, void* stream) {
  if (!params || !m || !v || !grad || n < 1 || step < 1) return fail(CTF_EINVAL, "bad argument");
  CTF_HIP(cnn_adam(params, m, v, grad, n, step, lr, static_cast<hipStream_t>(stream)));
  return CTF_OK;
}

int ctf_cnn_attach(ctf_problem* P, const float* params) {
  if (!P || !params) return fail(CTF_EINVAL, "null argument");
  if (P->cnn_level < 0) return fail(CTF_EINVAL, "problem created without cnn_level");
  CTF_HIP(hipMemcpyAsync(P->cnn_params, params, size_t(cnn_param_count()) * sizeof(float),
                         hipMemcpyDeviceToDevice, P->stream));
  P->cnn_ready = true;
  P->cnn_on = true;
  return CTF_OK;
}

int ctf_cnn_enable(ctf_problem* P, int on) {
  if (!P) return fail(CTF_EINVAL, "null argument");
  if (on && !P->cnn_ready) return fail(CTF_EINVAL, "no network attached");
  P->cnn_on = on != 0;
  return CTF_OK;
}

int ctf_cnn_sample(ctf_problem* P, double* psi, const double* psi_star, float* features, float* target,
                   double* scale) {
  if (!P || !psi || !psi_star || !features || !target || !scale) return fail(CTF_EINVAL, "null argument");
  if (P->cnn_level < 0) return fail(CTF_EINVAL, "problem created without cnn_level");
  if (P->mixed()) return fail(CTF_EINVAL, "training samples come from float64 cycles");
  int rc = emission64(P, psi, true);
  if (rc) return rc;
  rc = finest64(P, psi, P->rho[0], 0, 1.0);
  if (rc) return rc;
  rc = cycle_rest64(P, psi, false, true);
  if (rc) return rc;
  const int lc = P->cnn_level, nc = P->dims[lc].n;
  CTF_HIP(hipMemcpyAsync(features, P->cnn_feat, 3 * size_t(nc) * nc * sizeof(float), hipMemcpyDeviceToDevice,
                         P->stream));
  // angle-integrated error after the cycle, averaged onto the correction grid
  const size_t n = P->dof(0);
  CTF_HIP(hipMemcpyAsync(P->psi_tmp, psi_star, n * sizeof(double), hipMemcpyDeviceToDevice, P->stream));
  CTF_HIP(launch_axpy<double>(P->psi_tmp, psi, -1.0, n, P->stream));
  CTF_HIP(launch_moments<double>(P->ld(0), P->psi_tmp, P->phi, 1, P->stream));
  CTF_HIP(cnn_target(P->phi, target, P->cnn_scale, P->cfg.n, lc, P->stream));
  CTF_HIP(hipMemcpyAsync(scale, P->cnn_scale, sizeof(double), hipMemcpyDeviceToHost, P->stream));
  CTF_HIP(hipStreamSynchronize(P->stream));
  return CTF_OK;
}

int ctf_timing_enable(ctf_problem* P, int on, int capacity, unsigned class_mask) {
  if (!P || capacity < 0) return fail(CTF_EINVAL, "bad argument");
  P->timing_mask = class_mask ? class_mask : ~0u;
  CTF_HIP(hipStreamSynchronize(P->stream));
  P->timing = false;
  for (int c = 0; c < CTF_T_COUNT; ++c) {
    P->ev_used[c] = 0;
    P->ev_dropped[c] = 0;
  }
  if (!on) return CTF_OK;
  for (int c = 0; c < CTF_T_COUNT; ++c) {
    while (static_cast<int>(P->ev[c].size()) < 2 * capacity) {
      hipEvent_t e;
      CTF_HIP(hipEventCreate(&e));
      P->ev[c].push_back(e);
    }
  }
  P->timing_cap = capacity;
  P->timing = true;
  return CTF_OK;
}

int ctf_timing_read(ctf_problem* P, int cls, double* total_ms, int* launches, int* dropped) {
  if (!P || cls < 0 || cls >= CTF_T_COUNT) return fail(CTF_EINVAL, "bad argument");
  CTF_HIP(hipStreamSynchronize(P->stream));
  double tot = 0.0;
  for (int s = 0; s < P->ev_used[cls]; ++s) {
    float ms = 0.0f;
    CTF_HIP(hipEventElapsedTime(&ms, P->ev[cls][2 * s], P->ev[cls][2 * s + 1]));
    tot += ms;
  }
  if (total_ms) *total_ms = tot;
  if (launches) *launches = P->ev_used[cls];
  if (dropped) *dropped = P->ev_dropped[cls];
  return CTF_OK;
}

const char* ctf_last_error(void) { return g_err.c_str(); }

}  // extern "C"
