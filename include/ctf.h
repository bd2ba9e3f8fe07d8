/*
 * ctf.h -- C-ABI of the MI355X (gfx950) ConvFEM space-angle multigrid transport library.
 *
 * Method: arXiv 2301.09991 (Phillips, Heaney, Chen, Buchan, Pain), "Solving the Discretised
 * Boltzmann Transport Equations using Neural Networks".  The library solves the fixed-source,
 * multigroup, discrete-ordinates transport equations (section "Boltzmann Transport Equation",
 * fission term absent) on an N x N structured grid of the square [0, L]^2 with the octahedral
 * 8 * na^2 ordinate set (section "Discrete Ordinates"), discretised either by first-order upwind
 * control volumes (eq. discretised_hfm) or by ConvFEM filters of degree p with the anisotropic
 * non-linear Petrov-Galerkin dissipation (eqs. Petrov, kxx, kyy, ano-k; Appendix A), and solved
 * by the sawtooth space-angle multigrid cycle (section "Space-Angle Multigrid").
 *
 * Conventions shared by every call
 *   - Angular-flux-shaped arrays are float64 [G][n_dir][N][N] (x fastest), with
 *     n_dir = 8 * na^2 and ordinate index n = f * na^2 + a * na + b, f the octant face
 *     (bit 0: mu < 0, bit 1: nu < 0, bit 2: xi < 0), a the patch row towards the pole and
 *     b the patch column.  Offsets are 64-bit (N^2 * n_dir * G may exceed 2^31).
 *   - rho = b - A(psi) is the residual, b_{g,n} = S_g / (4 pi).  A(psi) holds streaming,
 *     Petrov-Galerkin dissipation, removal sigma_t psi and minus the scattering emission
 *     (isotropic, plus linearly anisotropic when scatter_order = 1).
 *   - Norms are ||v||_W = sqrt(sum p_n h^2 v^2); residuals are reported relative to ||b||_W.
 *   - Every device pointer is owned by the caller; the library owns only the opaque host struct.
 *     All device memory is carved from one caller-allocated workspace (ctf_workspace_bytes).
 *   - Calls are asynchronous on the problem's HIP stream unless stated otherwise.  Calls on one
 *     problem are not thread-safe; different problems on different streams are independent.
 *   - Return codes: CTF_OK (0), CTF_NOT_CONVERGED (1) or a negative error; ctf_last_error()
 *     returns a thread-local message describing the last failure.
 */
#ifndef CTF_H
#define CTF_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  CTF_OK = 0,
  CTF_NOT_CONVERGED = 1,
  CTF_EINVAL = -1,       /* bad configuration, shape or argument */
  CTF_ENOMEM = -2,       /* workspace too small */
  CTF_EHIP = -3,         /* a HIP runtime call failed */
  CTF_ENONFINITE = -4,   /* NaN or Inf found in a residual norm */
  CTF_EUNSUPPORTED = -5  /* valid request the library does not implement */
};

/* discretisation */
enum { CTF_UPWIND = 0, CTF_CONVFEM_PG = 1, CTF_CONVFEM_PG_FROZEN_K = 2 };
/* boundary condition per side (x-, x+, y-, y+) */
enum { CTF_VACUUM = 0, CTF_ZERO_GRADIENT = 1 };
/* arithmetic of the cycle; the outer residual and norms are always float64 */
enum { CTF_FP64 = 0, CTF_FP32_IR = 1, CTF_FP32_IR_BF16_MOMENTS = 2 };
/* apply_operator modes */
enum { CTF_OP_APPLY = 0, CTF_OP_RESIDUAL = 1 };
/* smoother kinds */
enum { CTF_SMOOTH_UPWIND = 0, CTF_SMOOTH_FINEST = 1 };
/* residual estimate R of the isotropic PG diffusivity (ctf_config.pg_r_estimate) */
enum { CTF_R_MIXED_MASS = 0, CTF_R_LOW = 1, CTF_R_HIGH = 2 };

typedef struct ctf_config {
  int n;               /* nodes per side of the finest grid (N x N), 2 <= N <= 8192 (byte
                          offsets inside one ordinate plane, and inside the three emission
                          moment planes of a group, are 32-bit) */
  double length;       /* side L of the square domain; h = L / N */
  int p;               /* ConvFEM degree 1..4 (ignored by CTF_UPWIND) */
  int na;              /* ordinates per face side, a power of two: n_dir = 8 na^2 */
  int ngroups;         /* G >= 1 */
  int scatter_order;   /* 0 isotropic, 1 adds linearly anisotropic (P1) scattering */
  int discretisation;  /* CTF_UPWIND, CTF_CONVFEM_PG, CTF_CONVFEM_PG_FROZEN_K */
  int bc[4];           /* CTF_VACUUM or CTF_ZERO_GRADIENT for x-, x+, y-, y+ */
  int precision;       /* CTF_FP64, CTF_FP32_IR, CTF_FP32_IR_BF16_MOMENTS */
  int n_jacobi;        /* upwind Jacobi sweeps per level and cycle (>= 1) */
  int n_pg;            /* finest-level smoothing sweeps after the update (>= 0) */
  int max_levels;      /* 0: coarsen while N is even and > 2 */
  double beta_pg;      /* Jacobi diagonal factor of the finest PG sweeps (paper: 3) */
  double alpha_r;      /* factor of the anisotropic residual estimates (paper: 3) */
  double eps_k;        /* epsilon_k of the diffusivities (paper: 0.001) */
  int n_inner;         /* float32 cycles per float64 refinement step (precision != FP64) */
  int cnn_level;       /* level of the learned coarse-grid correction, -1 = none (one group only) */
  double cnn_max_growth; /* the correction is switched off once a cycle applying it multiplies the
                            residual by more than this (default 1: it must not grow) */
  int cnn_max_uses;      /* steps of a solve that may apply the correction (default 2) */
  int hemisphere;        /* 1: only the ordinates with xi > 0 (faces 0..3, n_dir = 4 na^2), weights
                            doubled (normalised to 4 pi over the half set).  The 2D equations see
                            only (mu, nu), and every ordinate has a mirror with xi < 0, equal
                            (mu, nu) and equal weight, so the flux is even in xi and the result on
                            the kept ordinates equals the full set's; half the work.  Default 0. */
  int coupled_scatter;   /* 1: every correction sweep on every level adds the scattering of the
                            correction (emission of e with the level's 2 x 2 harmonic sigma_s, no
                            external source), so the coarse levels correct the scattering modes too;
                            the discrete equations and their solution are unchanged.  An extension
                            (the paper's sweeps are transport-only).  Default 0. */
  int pg_isotropic;      /* 1: the isotropic non-linear PG diffusivity (section "Non-Linear
                            Petrov-Galerkin Dissipation": mixed-mass residual R, k = min(k_max, k_abs,
                            k_square), the same k in x and y) instead of the anisotropic pair of
                            eq. ano-k.  Default 0. */
  int pg_r_estimate;     /* residual estimate R of the isotropic diffusivity (same section), with
                            Psi_x = f(psi; w_x), Psi_y = f(psi; w_y) of degree p:
                            CTF_R_MIXED_MASS: R = alpha_r f(mu Psi_x + nu Psi_y; m_L^-1 m - I);
                            CTF_R_LOW: R = (mu Psi_x + nu Psi_y) minus the same with the filters of
                            degree p - 1 (needs p >= 2);
                            CTF_R_HIGH: R = the same with the filters of degree p + 1 minus
                            (mu Psi_x + nu Psi_y) (needs p <= 3).  No factor on the low and high
                            forms.  Other than CTF_R_MIXED_MASS needs pg_isotropic = 1.  Every
                            estimate runs in either launch shape (pg_fused), with the same bits.
                            Default CTF_R_MIXED_MASS. */
} ctf_config;

typedef struct ctf_problem ctf_problem;

typedef struct ctf_level_desc {
  int n;               /* nodes per side on this level */
  int na;              /* ordinates per face side */
  int n_dir;           /* 8 na^2 */
  double h;            /* node spacing */
  long long dof;       /* G * n_dir * n^2 */
} ctf_level_desc;

typedef struct ctf_solve_info {
  int cycles;              /* sawtooth cycles performed */
  int outer_steps;         /* float64 refinement steps (mixed precision) */
  double rel_residual;     /* final ||rho||_W / ||b||_W, evaluated in float64 */
  double seconds;          /* wall time of the call */
  double* history;         /* optional caller buffer of history_len doubles: residual per check */
  int history_len;
  int cnn_applied;         /* cycles that applied the learned correction */
  int cnn_rejected;        /* 1 if the learned correction raised the residual and was switched off */
} ctf_solve_info;

/* Fill cfg with the paper's defaults: p = 1, na = 4, vacuum boundaries, upwind sweeps n_j = 2,
 * n_pg = 2, beta_pg = 3, alpha_r = 3, eps_k = 1e-3, FP64, no learned correction; and this library's
 * n_inner = 4 float32 cycles per refinement step (the paper has no mixed precision). */
void ctf_default_config(ctf_config* cfg);

/* Bytes of device workspace a problem with this configuration needs (0 on invalid cfg; the
 * reason is in ctf_last_error()). */
size_t ctf_workspace_bytes(const ctf_config* cfg);

/* Create a problem: the fixed-source multigroup discrete-ordinates equations of section
 * "Boltzmann Transport Equation" (no fission term) on the grid of eq. discretised_hfm, with the
 * ordinates of section "Discrete Ordinates" and the level hierarchy of section "Space-Angle
 * Multigrid".
 *   sigma_t  device float64 [G][N][N]             total cross-section (> 0 or = 0 for void)
 *   sigma_s  device float64 [L_s+1][G][G][N][N]   scattering sigma_{s,l}(g_from -> g_to) stored
 *                                                 [l][g_to][g_from]; L_s = scatter_order
 *   source   device float64 [G][N][N]             isotropic external source S_g
 *   workspace / ws_bytes: caller-owned device memory of at least ctf_workspace_bytes(cfg);
 *   stream: the hipStream_t all work of this problem is queued on (NULL = default stream).
 * The three inputs are copied into the workspace (they may be freed after return); the call
 * builds the quadrature, the ConvFEM stencils and the level hierarchy (coarse sigma_t by the
 * harmonic mean of 2x2 children) and synchronises the stream once.
 * Errors: CTF_EINVAL (cfg), CTF_ENOMEM (workspace too small), CTF_EHIP. */
int ctf_create_problem(const ctf_config* cfg, const double* sigma_t, const double* sigma_s,
                       const double* source, void* workspace, size_t ws_bytes, void* stream,
                       ctf_problem** out);

/* Release the host-side problem (the workspace stays the caller's). NULL is ignored. */
void ctf_destroy_problem(ctf_problem* prob);

/* Number of multigrid levels, and one level's sizes. */
int ctf_num_levels(const ctf_problem* prob);
int ctf_level_info(const ctf_problem* prob, int level, ctf_level_desc* out);

/* Host copies of one level's ordinates: mu, nu, w (weights p_n, summing to 4 pi), each n_dir
 * doubles in caller-owned host memory (section "Discrete Ordinates"; coarse levels add the
 * child patches: p summed, direction p-weighted). */
int ctf_level_quadrature(const ctf_problem* prob, int level, double* mu, double* nu, double* w);

/* The 1D ConvFEM stencils of degree p over offsets -p..p (2p+1 doubles each, host memory):
 * normalised mass m, first derivative d (times 1/h) and negated second derivative k (times
 * 1/h^2), from the averaged assembled rows of the degree-p element (section "ConvFEM",
 * Appendix A: the 2D filters are their tensor products). */
int ctf_convfem_stencils(int p, double* m, double* d, double* k);

/* Host-only: the finest ordinates (mu, nu, w) of the 8 na^2 octahedral set, same as level 0 of
 * ctf_level_quadrature; caller-owned host arrays of 8 na^2 doubles. */
int ctf_quadrature(int na, double* mu, double* nu, double* w);

/* Device copy of level `level`'s total cross-section, float64 [G][n][n] (caller buffer). */
int ctf_level_sigma_t(const ctf_problem* prob, int level, double* out);

/* A(psi) (mode CTF_OP_APPLY, no external source) or rho = b - A(psi) (CTF_OP_RESIDUAL) on the
 * finest level (eq. Petrov, or eq. discretised_hfm for CTF_UPWIND).  psi and out: device
 * float64 [G][n_dir][N][N], must not alias.  CTF_CONVFEM_PG_FROZEN_K uses the diffusivities held
 * by the last ctf_freeze_k. */
int ctf_apply_operator(ctf_problem* prob, const double* psi, double* out, int mode);

/* Moments of psi: phi[g][m][j][i] = sum_n w_n Y_m(n) psi[g][n][j][i] with Y = (1, mu, nu)
 * (section "Discrete Ordinates": phi_g = sum p_n psi_n).  phi: device float64 [G][3][N][N]. */
int ctf_moments(ctf_problem* prob, const double* psi, double* phi);

/* Float32 moments of a float32 angular flux (mixed-precision problems only): phi device float32
 * [G][3][N][N].  use_mfma = 1 evaluates the contraction on bf16 MFMA with float32 accumulation
 * (psi rounded to bf16, weights kept as a bf16 hi + lo pair); 0 uses float32 vector arithmetic.
 * The inner cycles of CTF_FP32_IR_BF16_MOMENTS use the MFMA form. */
int ctf_moments_f32(ctf_problem* prob, const float* psi, float* phi, int use_mfma);

/* Compute and hold the PG diffusivities k_x, k_y of psi (eq. ano-k) for the frozen-k
 * discretisation; if kx / ky are non-NULL they also receive a device float64 copy
 * [G][n_dir][N][N]. */
int ctf_freeze_k(ctf_problem* prob, const double* psi, double* kx, double* ky);

/* nsweeps Jacobi sweeps (eq. matrix_full) in place on x.
 *   CTF_SMOOTH_UPWIND: on level `level`, x <- x + (rhs - A_up x - sigma_t x)/d with the upwind
 *     diagonal d = |mu|/h + |nu|/h + sigma_t (beta = 1); x, rhs sized for that level.
 *   CTF_SMOOTH_FINEST: level 0 only, rhs must be NULL: psi <- psi + rho(psi)/(beta d) with the
 *     finest discretisation's residual (beta = beta_pg for ConvFEM, 1 for upwind). */
int ctf_smooth(ctf_problem* prob, int level, int kind, double* x, const double* rhs, int nsweeps);

/* Restriction from level `level` to level+1 (section "Space-Angle Multigrid": weight by p_n h^2,
 * sum the 2x2 cells and 2x2 child ordinates, divide by the coarse p_N H^2). */
int ctf_restrict(ctf_problem* prob, int level, const double* fine, double* coarse);

/* UpSamp from level+1 to level: every fine value copies its parent cell and ordinate. */
int ctf_prolong(ctf_problem* prob, int level, const double* coarse, double* fine);

/* One sawtooth cycle (section "Space-Angle Multigrid" and its sawtooth-cycle figure): the finest
 * residual restricted to every level, Jacobi sweeps from zero on the coarsest level, UpSamp and
 * sweeps level by level up to the finest, psi += e, then n_pg finest sweeps (eq. matrix_full with
 * beta_pg for ConvFEM).  In place on psi (device float64 [G][n_dir][N][N]); with precision !=
 * CTF_FP64 one call is one refinement step (as in ctf_solve).  If rel_res is non-NULL the call
 * synchronises and stores ||rho(psi_in)||_W / ||b||_W of the input psi. */
int ctf_mg_cycle(ctf_problem* prob, double* psi, double* rel_res);

/* Cycle until ||rho||_W / ||b||_W <= rtol (checked before every cycle) or max_cycles cycles;
 * in place from the given psi (warm start).  With precision != CTF_FP64 every outer step
 * evaluates rho in float64, runs n_inner float32 cycles and updates psi in float64: for the
 * non-linear PG the cycles act on the full-approximation problem A32(u) = A32(fl32(psi)) + rho
 * (diffusivities re-formed from u in every float32 evaluation), for the linear discretisations on
 * the correction equation A e = rho.  Synchronous.
 * Returns CTF_OK, CTF_NOT_CONVERGED, or an error (CTF_ENONFINITE on a NaN/Inf residual). */
int ctf_solve(ctf_problem* prob, double* psi, double rtol, int max_cycles, ctf_solve_info* info);

/* Solve nprob independent problems together (synchronous).  A solver step of every problem is
 * captured once into one HIP graph (steps_per_graph steps per problem; problems spread over up to 8
 * parallel branches); the graph is replayed until every problem has converged or max_steps steps
 * were launched.  Convergence is decided on the device: each problem holds a flag that its step
 * clears once ||rho||_W / ||b||_W <= rtol, after which all of that problem's kernels return at
 * once, so converged problems drop out without host involvement; the host reads the flags only
 * between replays.  psis[i] is problem i's angular flux (in place, warm start); infos (nprob
 * entries, optional) receive per-problem cycles, outer steps, final residual and the call's wall
 * time.  The problems must be distinct; their own streams must be idle.  Every problem's flag is set
 * again before the call returns, so the problems stay usable.  Returns CTF_OK when all converged,
 * CTF_NOT_CONVERGED otherwise. */
int ctf_solve_batch(ctf_problem* const* probs, int nprob, double* const* psis, double rtol,
                    int max_steps, int steps_per_graph, ctf_solve_info* infos);

/* The same solve in ONE launch of a persistent kernel (upwind discretisation, any precision; no
 * scattering-coupled sweeps, no learned correction; CTF_EUNSUPPORTED otherwise).  A solver step of
 * every problem is recorded once as a list of operations; the launch keeps one wave of resident
 * blocks that take work items (a chunk of tiles of one operation of one problem) from a device
 * ticket counter in a fixed order (step, operation, problem, chunk), each item first waiting until
 * the items of its problem ahead of it have finished.  A problem's update of its convergence flag
 * runs on the device, and once converged its remaining items are skipped; the launch ends when
 * every problem has converged or after max_steps steps of each.  Every wait is bounded (about 4 s):
 * if one runs out, the launch ends and CTF_EHIP is returned.  Iterates, norms and step counts are
 * those of ctf_solve_batch, bit for bit (the same per-element arithmetic and reduction orders).
 * items_per_block (0: default 1): the largest operation of the batch is split into about that many
 * work items per resident block (1 was the fastest measured; every item costs a device-wide
 * release and acquire of memory).  workspace: device memory of ctf_solve_batch_persistent_bytes()
 * bytes, 256-byte aligned, owned by the caller (the schedule and the counters; overwritten).  Runs
 * on the first problem's stream and returns when the launch has finished; the problems' own
 * streams must be idle.  Every problem's flag is set again before the call returns.  Returns CTF_OK
 * when all converged, CTF_NOT_CONVERGED otherwise. */
int ctf_solve_batch_persistent(ctf_problem* const* probs, int nprob, double* const* psis, double rtol,
                               int max_steps, int items_per_block, void* workspace, size_t ws_bytes,
                               ctf_solve_info* infos);
/* Workspace bytes of ctf_solve_batch_persistent for these problems on the current device (0 on a
 * bad argument, an unsupported problem or no device). */
size_t ctf_solve_batch_persistent_bytes(ctf_problem* const* probs, int nprob, int items_per_block);

/* Launch shape of the finest-level kernels: rows per wavefront strip of the ConvFEM/PG kernels
 * (8..512), the block size of the upwind correction sweeps (multiple of 64, <= 1024), and for
 * the non-linear PG whether the diffusivities are formed in the residual's own pass (pg_fused = 1)
 * or in a pass of their own whose result the residual pass reads (0).  Results do not depend on
 * the shape.  Defaults: strip_h 128 (256 once a
 * PG launch has at least eight rounds of 4096 wavefront slots, 512 once it has sixteen with
 * 512-row strips), corr_block 256, pg_fused 1 for p <= 3 and 0 for p = 4. */
int ctf_set_launch_shape(ctf_problem* prob, int strip_h, int corr_block, int pg_fused);
int ctf_get_launch_shape(const ctf_problem* prob, int* strip_h, int* corr_block, int* pg_fused);

/* Autotuner: time the candidate launch shapes of the finest-level kernels on this problem's own
 * buffers (strip heights 8..512 and fused / two-pass for ConvFEM/PG, sweep blocks 64..1024),
 * keep the fastest, and
 * record them in the JSON file cache_path under a key of (p, discretisation, precision, n, n_dir,
 * groups).  A problem whose key is already cached takes the cached shape without timing unless
 * force is set.  cache_path may be NULL (no file).  Synchronous; overwrites the problem's scratch
 * buffers (not psi).  The chosen shape is returned through strip_h / corr_block (may be NULL). */
int ctf_autotune(ctf_problem* prob, const char* cache_path, int force, int* strip_h, int* corr_block,
                 int* pg_fused);

/* ||v||_W of a finest-level array (synchronous). */
int ctf_norm(ctf_problem* prob, const double* v, double* out);

/* ---- learned coarse-grid correction ---------------------------------------------------------
 * Not in the paper (its filters are fixed); this project's own extension.  A four-layer 3x3
 * convolutional network (channels 3 -> 32 -> 32 -> 32 -> 1, ReLU after the first three, zero
 * padding) maps three fields on the grid of level cnn_level -- the angle-integrated restricted
 * residual sum_n w_n rho_n divided by its RMS s, H sigma_t, and the mean scattering ratio -- to the
 * angle-integrated error left by a plain sawtooth cycle, in units of s.  In a cycle with the
 * correction, psi (or the float32 correction) gains s * net / (4 pi) in every ordinate,
 * interpolated bilinearly from the cell centres of that level to the finest cell centres, after the
 * finest correction sweeps and before the finest smoothing.  In
 * ctf_solve plain multigrid stays the arbiter: a step with the correction that multiplies the
 * residual by more than cnn_max_growth (or makes it non-finite) is undone and the correction is
 * switched off for the rest of the solve; at most cnn_max_uses steps apply it (in a float32
 * refinement step, only its first cycle).
 * Parameters: float32 device vector of ctf_cnn_param_count() values, W1 b1 W2 b2 W3 b3 W4 b4 with
 * W[c_out][c_in][ky][kx].  Activations: float32 [batch][channel][y][x]. */
int ctf_cnn_param_count(void);
/* Device workspace for ctf_cnn_forward / ctf_cnn_loss_grad at this batch and size. */
size_t ctf_cnn_workspace_bytes(int batch, int h, int w);
/* out[batch][1][h][w] = net(in[batch][3][h][w]).  bf16 = 1: activations rounded to bf16 and
 * the convolutions on bf16 MFMA with float32 accumulation; 0: float32 vector arithmetic. */
int ctf_cnn_forward(const float* params, const float* in, float* out, int batch, int h, int w, int bf16,
                    void* workspace, size_t ws_bytes, void* stream);
/* The same forward pass for callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid allocation): no workspace argument, and the call
 * makes no allocation of any kind.  The three hidden activations live in a file-scope device array
 * of 3 * 32 * 32768 float32 values (12 MiB) that each GPU the library runs on holds until the
 * process ends, so batch * h * w must not exceed 32768 (else CTF_EINVAL, nothing launched).
 * Every call on one GPU uses that GPU's one array: calls that overlap on one GPU (different
 * streams, or host threads) race and must be ordered by the caller.  Nothing in the array needs
 * clearing between calls; each layer writes all of its output.  Results equal ctf_cnn_forward's
 * bit for bit (the same kernels). */
int ctf_cnn_forward_noalloc(const float* params, const float* in, float* out, int batch, int h, int w,
                            int bf16, void* stream);
/* Mean-squared-error loss of net(in) against target[batch][1][h][w] (loss: device float64 scalar)
 * and its gradient grad (device float32, ctf_cnn_param_count() values). */
int ctf_cnn_loss_grad(const float* params, const float* in, const float* target, int batch, int h,
                      int w, int bf16, float* grad, double* loss, void* workspace, size_t ws_bytes,
                      void* stream);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) at step >= 1 on params with moments m, v. */
int ctf_cnn_adam(float* params, float* m, float* v, const float* grad, int n, int step, float lr,
                 void* stream);
/* Copy the network parameters into a problem created with cnn_level >= 0 and switch it on. */
int ctf_cnn_attach(ctf_problem* prob, const float* params);
/* Switch an attached network on (1) or off (0). */
int ctf_cnn_enable(ctf_problem* prob, int on);
/* Training sample (float64 problems): one plain sawtooth cycle in place on psi; features receives
 * the network input of the cycle's starting residual (device float32 [3][n_c][n_c] on the grid of
 * cnn_level), target the angle-integrated error psi_star - psi after the cycle averaged onto that
 * grid and divided by the feature scale s, and *scale (host) receives s. */
int ctf_cnn_sample(ctf_problem* prob, double* psi, const double* psi_star, float* features,
                   float* target, double* scale);

/* In-library kernel timers (HIP events recorded on the problem's stream around each launch of a
 * kernel class).  ctf_timing_enable(prob, 1, cap, mask) synchronises, clears the counters and
 * records at most cap launches per class from then on, for the classes whose bit (1u << class) is
 * set in mask (0: every class; each recorded launch adds two event records to the stream, so
 * timing only the classes of interest keeps the overhead small); (prob, 0, 0, 0) stops recording.
 * ctf_timing_read synchronises and returns the summed event time (ms) of the recorded launches
 * of one class, their count, and how many launches were not recorded for lack of capacity. */
enum {
  CTF_T_PG64 = 0,      /* finest ConvFEM/PG residual or sweep, float64 */
  CTF_T_PG32,          /* same, float32 (refinement inner cycles) */
  CTF_T_UPWIND64,      /* finest upwind residual or sweep, float64 */
  CTF_T_UPWIND32,
  CTF_T_CORR0,         /* upwind correction sweeps on the finest level */
  CTF_T_CORRC,         /* upwind correction sweeps on coarse levels */
  CTF_T_RESTRICT,
  CTF_T_MOMENTS,
  CTF_T_EMISSION,
  CTF_T_NORM,
  CTF_T_MOMENTS_MFMA,  /* bf16 MFMA moment contraction */
  CTF_T_CNN,           /* learned correction: features, network, application */
  CTF_T_PGK64,         /* stored non-linear PG diffusivities (their own pass), float64 */
  CTF_T_PGK32,         /* same, float32 */
  CTF_T_CSCAT,         /* moments + emission of the corrections (coupled_scatter) */
  CTF_T_PG32U,         /* the last float32 PG sweep of a refinement step, which also applies the
                          float64 full-approximation update */
  CTF_T_COUNT
};
int ctf_timing_enable(ctf_problem* prob, int on, int capacity, unsigned class_mask);
int ctf_timing_read(ctf_problem* prob, int cls, double* total_ms, int* launches, int* dropped);

/* Thread-local description of the last error ("" if none). */
const char* ctf_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* CTF_H */
