"""Throughput benchmark of the ConvFEM space-angle multigrid solver on one MI355X.

Headline workload (the learned-correction workload, on which the metric's comparison is quoted):
1024 x 1024 nodes on a 32 x 32 square, biquadratic ConvFEM (p = 2) with the non-linear anisotropic
Petrov-Galerkin dissipation, 512 ordinates (octahedral, 8 x 8 patches per face = 16 polar x 32
azimuthal), one energy group, isotropic scattering with c uniform in [0.8, 0.99], coefficients
piecewise constant on 32 x 32-cell patches, unit source on the central 8 x 8 square.  The mixed-
precision (1024^2 x 512 x 2 groups) and MFMA (512^2, p = 3, 2048 ordinates, 4 groups, P1) workloads
are timed the same way and reported beside it.  All inputs are seeded synthetic arrays
(workloads.make_inputs).

One step = one refinement step of the mixed-precision solver: float64 residual (with the
diffusivities of the current psi) + float64 norm, n_inner float32 sawtooth cycles on the
full-approximation problem (the library's default, 4), and the float64 update.  value = finest DOF x float32 cycles / second.
Inputs are resident in HBM before the timed region starts.

Prints ONE JSON line (see the repository's measurement notes for the roofline fields).
"""
import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "space-angle DOF-updates/s; time-to-1e-6 residual, learned+mixed vs plain FP64 MG"
HBM_PEAK_GBS = 8000.0
FP32_VALU_TFLOPS = 157.3
FP64_VALU_TFLOPS = 78.6


# Algorithmic flops per finest DOF of one evaluation of the ConvFEM/PG residual or sweep (separable
# tensor-product filters, W = 2p + 1 taps): the scope table's figures, by element degree.
PG_FLOPS_PER_DOF = {1: 150, 2: 220, 3: 290}


def implementation_flops(kernel, p, fused=True):
    """Flops per DOF the PG kernels of this library issue (two per multiply-add, divisions and
    minima counted as one), stage by stage.  Fused kernel: A, Psi_x and Psi_y (2 x-sums, 2 y-passes);
    B, the mixed-mass R_x and R_y (2 + 2); C, the x-sums of the k-Diff terms (6 sums, plus the 2
    products k psi per tap); D, their y-passes (6); 57 for k, the emission and the epilogue:
    42 W + 57.  The two-pass form evaluates A and B in the diffusivity pass (16 W + 34) and again
    the gradients in the stream pass (32 W + 23)."""
    W = 2 * p + 1
    if kernel in ("pg32", "pg64", "pg32_update"):
        return 42 * W + 57 if fused else 32 * W + 23
    if kernel in ("pgk32", "pgk64"):
        return 16 * W + 34
    return algorithmic_cost(kernel, p, fused)[1]


def algorithmic_cost(kernel, p, fused=False):
    """Algorithmic bytes and flops per finest DOF of one launch of a kernel class.

    Bytes: the arrays every DOF must read or write once (per-cell data shared by all ordinates --
    sigma_t, emission moments -- is amortised to ~0): for the PG residual and sweeps 2b (read psi,
    write the residual or the new psi), b = 4 in float32 and 8 in float64.  Flops: PG_FLOPS_PER_DOF
    for the PG kernels, two per multiply-add elsewhere."""
    if kernel in ("pg32", "pg32_update"):
        return 8, PG_FLOPS_PER_DOF[p]
    if kernel == "pg64":
        return 16, PG_FLOPS_PER_DOF[p]
    if kernel == "pgk32":              # read x; write k_x, k_y
        return 12, 16 * (2 * p + 1) + 34
    if kernel == "pgk64":
        return 24, 16 * (2 * p + 1) + 34
    if kernel in ("corr0", "upwind32"):
        return 12, 12                   # read e, rhs; write e (last sweep: read-modify-write)
    if kernel == "upwind64":
        return 24, 12
    if kernel in ("moments", "moments_mfma"):
        return 4, 6
    raise KeyError(kernel)


def implementation_bytes(kernel, p, fused=True):
    """Bytes per DOF the PG kernels move by design: the full-approximation sweeps also read their
    right-hand side; the float64 residual also writes psi rounded to float32; the last float32
    sweep reads and writes psi64; the two-pass form reads k_x, k_y back."""
    extra = {"pg32": 4 if fused else 12, "pg32_update": 20 if fused else 28, "pg64": 4 if fused else 20}
    return algorithmic_cost(kernel, p, fused)[0] + extra.get(kernel, 0)


def kernel_symbol(kernel, p, fused):
    """The one HIP kernel a timer class launches (as rocprofv3 names it, template arguments in
    angle brackets) and a file-name form of it."""
    t = "double" if kernel.endswith("64") else "float"
    name = {"pg32": "k_pg_fused" if fused else "k_pg_stream", "pg64": "k_pg_fused" if fused else "k_pg_stream",
            "pgk32": "k_pg_diffusivity", "pgk64": "k_pg_diffusivity"}.get(kernel)
    if name is None:
        return kernel, kernel
    # the second template argument of both kernels is the residual estimate (0, the mixed mass); the
    # fused kernel's last one selects the form with the float64 update (its own timer class)
    args = {"k_pg_fused": "%d, 0, %s, false", "k_pg_diffusivity": "%d, 0, %s"}.get(name, "%d, %s") % (p, t)
    return "%s<%s>" % (name, args), "%s_p%d_%s" % (name, p, "f64" if t == "double" else "f32")


def read_traffic(kernel_symbol, workload):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3 counter summary of
    that kernel on that workload, if it was taken on the kernel source as it is now (else None)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic_%s_%s.txt" % (kernel_symbol, workload))
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    src = os.path.join(ROOT, "paper_2301_09991_amd", "csrc", "kernels.hip")
    digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if vals.get("kernels.hip sha256") != digest:
        return None
    try:
        return float(vals["scaled bytes per launch"])
    except (KeyError, ValueError):
        return None


def _host_cpu():
    """(CPU model string, logical CPUs visible to this process)."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, len(os.sched_getaffinity(0))


_POOL = {}


def _pool_residual(block):
    """PG residual of one block of ordinates (pool worker; the arrays come from the parent by fork):
    the worker forms the moments of the whole flux and the emission of its own ordinates."""
    from oracle.transport import emission_from_moments, moments, pg_residual
    g = _POOL
    sel = slice(*block)
    quad = {"mu": g["quad"]["mu"][sel], "nu": g["quad"]["nu"][sel]}
    q = emission_from_moments(moments(g["psi"], g["quad"]), quad, g["ss"], g["src"])
    return pg_residual(g["psi"][:, sel], q, g["st"], quad, g["h"], g["h"], g["p"], g["bc"])


def cpu_baseline_worker(workers):
    """Time the float64 oracle (test infrastructure, run here only as the CPU baseline) on the
    learned-correction workload's recipe at N = 64 (same p, ordinates, group, L = 32), from a
    psi after one cycle from zero: the finest PG residual (apply_operator), one finest upwind
    correction sweep, one sawtooth cycle, single-threaded; the same residual split over ordinate
    blocks in a process pool of ``workers`` (moments in the parent, then one block of ordinates per
    task; the per-ordinate stencil work is independent once the emission is known); and the plain
    float64 solve of the small workload (32 x 32, 128 ordinates, upwind) to 1e-8."""
    import multiprocessing as mp
    import numpy as np
    from oracle import multigrid as omg
    from workloads import WORKLOADS, make_inputs, scaled
    out = {}
    w = scaled(WORKLOADS["c4_learned"], 64)
    st, ss, src = make_inputs(w)
    prob = omg.Problem(w.N, w.L, w.p, w.na, st, ss, src, disc=omg.PG)
    psi = omg.sawtooth_cycle(prob, np.zeros(prob.shape()))
    out["dof"] = w.dof

    def timed(fn):
        t = time.perf_counter()
        fn()
        return time.perf_counter() - t
    out["apply_operator_s"] = timed(lambda: omg.finest_residual(prob, psi))
    rho = omg.finest_residual(prob, psi)
    out["upwind_sweep_s"] = timed(lambda: omg.upwind_jacobi(prob, 0, np.zeros_like(psi), rho, 1))
    out["mg_cycle_s"] = timed(lambda: omg.sawtooth_cycle(prob, psi))
    # all cores: ordinate blocks of one face quarter each
    nd = psi.shape[1]
    nblk = max(workers, 1)
    edges = np.linspace(0, nd, min(nblk * 2, nd) + 1).astype(int)
    blocks = [(int(a), int(b)) for a, b in zip(edges[:-1], edges[1:]) if b > a]
    _POOL.update(quad=prob.quad, psi=psi, st=prob.sigma_t, ss=prob.sigma_s, src=prob.source, h=prob.h,
                 p=prob.p, bc=prob.bc)
    ctx = mp.get_context("fork")
    with ctx.Pool(workers) as pool:
        pool.map(_pool_residual, blocks[:workers])      # start-up of the workers, not timed
        t = time.perf_counter()
        parts = pool.map(_pool_residual, blocks)
        res = np.concatenate(parts, axis=1)
        out["apply_operator_pool_s"] = time.perf_counter() - t
    ref = omg.finest_residual(prob, psi)
    out["pool_matches_serial"] = bool(np.allclose(res, ref, rtol=1e-12, atol=1e-14 * np.abs(ref).max()))
    out["workers"] = workers
    w0 = WORKLOADS["c0_plain_fp64"]
    st0, ss0, src0 = make_inputs(w0)
    p0 = omg.Problem(w0.N, w0.L, w0.p, w0.na, st0, ss0, src0, disc=omg.UPWIND)
    t = time.perf_counter()
    _, hist, ok = omg.solve(p0, rtol=1e-8, max_cycles=400)
    out["c0_upwind_solve_s"] = time.perf_counter() - t
    out["c0_upwind_solve_cycles"] = len(hist) - 1
    out["c0_upwind_solve_converged"] = ok
    out["c0_dof"] = w0.dof
    print(json.dumps(out))


def cpu_baseline():
    """The float64 oracle timed on this host's cores (single thread, and a process pool of at most
    16 workers for the residual), in a subprocess so that the thread limits hold."""
    model, ncpu = _host_cpu()
    workers = max(1, min(16, ncpu))
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    out = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-baseline-worker", str(workers)],
                         env=env, capture_output=True, text=True, timeout=900)
    if out.returncode != 0:
        return {"error": out.stderr[-500:]}
    r = json.loads(out.stdout.strip().splitlines()[-1])
    dof = r["dof"]
    return {"value": dof / r["mg_cycle_s"], "unit": "DOF-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"one float64 oracle sawtooth cycle (numpy, one thread) of the learned-correction recipe "
                      f"at N=64 ({dof} DOF, p=2, 512 ordinates, 1 group, L=32), {r['mg_cycle_s']:.1f} s",
            "host": {"cpu_model": model, "logical_cpus": ncpu},
            "items": {
                "apply_operator": {"dof_per_s": dof / r["apply_operator_s"], "cores": 1,
                                   "seconds": r["apply_operator_s"]},
                "apply_operator_all_cores": {"dof_per_s": dof / r["apply_operator_pool_s"],
                                             "cores": r["workers"], "seconds": r["apply_operator_pool_s"],
                                             "matches_serial": r["pool_matches_serial"]},
                "upwind_sweep": {"dof_per_s": dof / r["upwind_sweep_s"], "cores": 1,
                                 "seconds": r["upwind_sweep_s"]},
                "mg_cycle": {"dof_per_s": dof / r["mg_cycle_s"], "cores": 1, "seconds": r["mg_cycle_s"]},
                "c0_plain_fp64_upwind_solve_1e-8": {"seconds": r["c0_upwind_solve_s"],
                                                    "cycles": r["c0_upwind_solve_cycles"],
                                                    "converged": r["c0_upwind_solve_converged"],
                                                    "dof": r["c0_dof"], "cores": 1}}}


def time_to_tolerance(log):
    """Learned-correction workload (1024 x 1024 nodes, L = 32, p = 2, 512 ordinates, one group,
    c in [0.8, 0.99]), upwind discretisation: wall time of ctf_solve from psi = 0 to a float64
    relative residual of 1e-6 for plain float64 multigrid, float32 cycles + float64 refinement,
    and the same with the learned coarse-grid correction, trained here on residual/error pairs
    from 200 seeded solves at 128 x 128 (same L, so the correction level's 32 x 32 grid has the
    same cell size H = 1 as the evaluation problem's)."""
    import torch
    from paper_2301_09991_amd import ctf, learned
    from workloads import WORKLOADS, Workload, make_inputs
    w = WORKLOADS["c4_learned"]
    t0 = time.perf_counter()

    def tw(N, seed, patch):
        return Workload(f"train{seed}", N, w.L, w.p, 2, 1, patch, "iso", "box_quarter_phys", w.c_range, seed)
    train = [(tw(128, 4000 + k, 4), 2) for k in range(200)]
    F, T = learned.generate_samples(train, make_inputs)
    log(f"training samples from {len(train)} solves at 128x128 in {time.perf_counter() - t0:.1f} s")
    theta, hist = learned.train(F, T, epochs=150, batch=16, lr=2e-3, seed=0)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    log(f"learned correction trained in {train_s:.1f} s ({F.shape[0]} samples, loss {hist[0]:.3g} -> {hist[-1]:.3g})")
    inputs = make_inputs(w)
    level = 5  # 32 x 32 correction grid, H = 1 (the training cell size)
    out = {"workload": f"{w.name}: {w.N}x{w.N} nodes, L={w.L}, p={w.p}, {w.n_dir} ordinates, 1 group, "
                       f"c in {list(w.c_range)}, upwind discretisation, rtol 1e-6",
           "discretisation": "upwind",
           "substitute": "the workload is specified with biquadratic ConvFEM + PG; the non-linear PG cycle "
                         "does not contract on these optically thin cells (sigma_t h in [0.016, 0.0625]), so "
                         "the times to 1e-6 are measured with the upwind discretisation",
           "dof": w.dof, "train_seconds": train_s, "train_samples": int(F.shape[0]),
           "train_loss_first_last": [hist[0], hist[-1]]}
    # the last two rows solve the same problem on the xi > 0 half of the ordinates (doubled weights;
    # the 2D flux is even in xi): a separate optimisation, reported beside the others and not part
    # of any DOF count
    # "coupled" rows: correction sweeps that include the scattering of the correction (an
    # extension), also reported beside the others
    for name, prec, use, half, coupled in (
            ("plain_fp64", ctf.FP64, False, False, False), ("mixed", ctf.FP32_IR, False, False, False),
            ("learned_mixed", ctf.FP32_IR, True, False, False),
            ("plain_fp64_half_set", ctf.FP64, False, True, False),
            ("learned_mixed_half_set", ctf.FP32_IR, True, True, False),
            ("coupled_fp64", ctf.FP64, False, False, True), ("coupled_mixed", ctf.FP32_IR, False, False, True)):
        prob = learned.make_problem(w, inputs, level, precision=prec, hemisphere=half, coupled=coupled)
        if use:
            prob.cnn_attach(theta)
        psi = prob.zeros()
        torch.cuda.synchronize()
        info = prob.solve(psi, 1e-6, 2000)
        out[name] = {"seconds": info["seconds"], "cycles": info["cycles"], "converged": info["converged"],
                     "rel_residual": info["rel_residual"], "cnn_applied": info["cnn_applied"],
                     "cnn_rejected": info["cnn_rejected"]}
        log(f"time-to-1e-6 {name}: {info['seconds']:.3f} s, {info['cycles']} cycles")
        del prob, psi
        torch.cuda.empty_cache()
    out["speedup_learned_mixed_vs_plain_fp64"] = out["plain_fp64"]["seconds"] / out["learned_mixed"]["seconds"]
    out["speedup_mixed_vs_plain_fp64"] = out["plain_fp64"]["seconds"] / out["mixed"]["seconds"]
    out["speedup_learned_mixed_half_set_vs_plain_fp64"] = (out["plain_fp64"]["seconds"]
                                                           / out["learned_mixed_half_set"]["seconds"])
    return out


def duct_study(log):
    """The paper's straight-duct study (28 x 36 cm, void duct, no scattering) as a self-convergence
    study: upwind discretisation (the non-linear PG iteration does not converge with the void
    duct), 128 ordinates at dx = 0.8, 0.4, 0.2, 0.1 cm and 512 at dx = 0.1; relative L2 errors of
    the scalar flux over the 28 x 36 cm domain against the dx = 0.1 solution averaged onto each
    grid (spatial, 128 ordinates) and between 128 and 512 ordinates at dx = 0.1 (angular); the
    flux along the duct centre line x = 14 cm; and the paper's PG procedure (100 cycles from zero)
    at dx = 0.8 and 0.4 for p = 1, 2, 3: the residual left and the centre-line flux."""
    import numpy as np
    import torch
    from paper_2301_09991_amd import ctf
    from workloads import DUCT_PAD, duct_inputs

    def run(dx, na, disc=ctf.UPWIND, p=1, rtol=1e-10, cycles=3000):
        N, L, st, ss, src = duct_inputs(dx)
        cfg = ctf.default_config(n=N, length=L, p=p, na=na, ngroups=1, scatter_order=0, discretisation=disc)
        prob = ctf.Problem(cfg, st, ss, src)
        psi = prob.zeros()
        info = prob.solve(psi, rtol, cycles)
        phi = torch.empty((1, 3, N, N), dtype=torch.float64, device="cuda")
        prob.moments(psi, phi)
        return info, phi[0, 0].cpu().numpy()

    out = {"solves": {}}
    flux = {}
    for dx, na in ((0.8, 4), (0.4, 4), (0.2, 4), (0.1, 4), (0.1, 8)):
        info, phi = run(dx, na)
        flux[(dx, na)] = phi
        out["solves"][f"dx{dx}_na{na}"] = {"cycles": info["cycles"], "converged": info["converged"],
                                           "seconds": info["seconds"]}
        log(f"duct dx={dx} na={na}: {info['cycles']} cycles, {info['seconds']:.3f} s")
    def rel_err(dx, na, ref):
        f = int(round(dx / 0.1))
        n = ref.shape[0] // f
        refc = ref.reshape(n, f, n, f).mean(axis=(1, 3))
        pad = int(round(DUCT_PAD / dx))
        d = (flux[(dx, na)] - refc)[:, pad:n - pad]
        return float(np.sqrt((d ** 2).sum() / (refc[:, pad:n - pad] ** 2).sum()))

    # spatial: 128-ordinate solutions against the 128-ordinate dx = 0.1 one; angular: 128 against
    # 512 ordinates at dx = 0.1
    errs = {f"dx{dx}": rel_err(dx, 4, flux[(0.1, 4)]) for dx in (0.8, 0.4, 0.2)}
    out["spatial_rel_l2_error_vs_dx0.1"] = errs
    out["angular_rel_l2_error_128_vs_512_at_dx0.1"] = rel_err(0.1, 4, flux[(0.1, 8)])
    e = [errs[f"dx{dx}"] for dx in (0.8, 0.4, 0.2)]
    out["observed_order"] = [float(np.log2(e[0] / e[1])), float(np.log2(e[1] / e[2]))]
    # the flux along the duct centre line (x = 14 cm in the 28 cm frame) at dx = 0.2, every 1 cm
    phi = flux[(0.2, 4)]
    col = int(round((14.0 + DUCT_PAD) / 0.2))
    out["centre_line_phi_dx0.2"] = [float(0.5 * (phi[j, col - 1] + phi[j, col])) for j in range(2, 180, 5)]
    # the paper's PG procedure: a fixed 100 sawtooth cycles from zero at dx = 0.8 and 0.4 (128
    # ordinates), p = 1, 2, 3; the residual left, and the centre-line flux against the upwind
    # dx = 0.1 reference averaged onto the same cells (relative L2 along the line; the PG iteration
    # does not converge here, so these are the iterates, not discrete solutions)
    ref = flux[(0.1, 4)]
    pg = {}
    for dx in (0.8, 0.4):
        f = int(round(dx / 0.1))
        n = ref.shape[0] // f
        refc = ref.reshape(n, f, n, f).mean(axis=(1, 3))
        c = int(round((14.0 + DUCT_PAD) / dx))
        ref_line = 0.5 * (refc[:, c - 1] + refc[:, c])
        for p in (1, 2, 3):
            info, phi = run(dx, 4, ctf.CONVFEM_PG, p, rtol=1e-10, cycles=100)
            line = 0.5 * (phi[:, c - 1] + phi[:, c])
            d = line - ref_line
            pg[f"dx{dx}_p{p}"] = {"cycles": info["cycles"], "rel_residual": info["rel_residual"],
                                  "centre_line_rel_l2_vs_upwind_dx0.1": float(np.sqrt((d ** 2).sum() / (ref_line ** 2).sum())),
                                  "centre_line_phi_every_1p6cm": [float(v) for v in line[::max(1, int(round(1.6 / dx)))]]}
            log(f"duct PG dx={dx} p={p}: residual {info['rel_residual']:.3g} after {info['cycles']} cycles")
    out["pg_after_100_cycles"] = pg
    log(f"duct errors {errs}, orders {out['observed_order']}")
    return out


def batched(log):
    """The batched workload: 64 problems with sizes drawn from {64, ..., 384}^2, p = 2, 512
    ordinates, one group, upwind discretisation, float32 cycles + float64 refinement to 1e-6, all
    solved by replays of one captured HIP graph (launch shapes autotuned per size), then again from
    zero in one launch of the persistent work-queue kernel."""
    import tempfile
    import torch
    from paper_2301_09991_amd import ctf
    from workloads import batch_workloads, make_inputs
    ws = batch_workloads()
    probs, psis, shapes = [], [], {}
    with tempfile.TemporaryDirectory() as d:
        cache = os.path.join(d, "autotune.json")
        for w in ws:
            st, ss, src = make_inputs(w)
            cfg = ctf.default_config(n=w.N, length=w.L, p=w.p, na=w.na, ngroups=1, discretisation=ctf.UPWIND,
                                     precision=ctf.FP32_IR)
            p = ctf.Problem(cfg, st, ss, src)
            shapes[w.N] = p.autotune(cache)
            probs.append(p)
            psis.append(p.zeros())
    torch.cuda.synchronize()
    dof = sum(w.dof for w in ws)
    t0 = time.perf_counter()
    ok, infos = ctf.solve_batch(probs, psis, 1e-6, 400, 2)
    dt = time.perf_counter() - t0
    cyc = [i["cycles"] for i in infos]
    log(f"batched: {len(ws)} problems, {dof} DOF, converged={ok}, {dt:.3f} s")
    # the same solves again from zero in one launch of the persistent work-queue kernel
    for x in psis:
        x.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ok_p, infos_p = ctf.solve_batch_persistent(probs, psis, 1e-6, 400)
    dt_p = time.perf_counter() - t0
    cyc_p = [i["cycles"] for i in infos_p]
    log(f"batched, persistent launch: converged={ok_p}, {dt_p:.3f} s")
    persistent = {"converged": ok_p, "seconds": dt_p, "cycles_equal_to_graph_form": cyc_p == cyc,
                  "dof_updates_per_s": sum(w.dof * c for w, c in zip(ws, cyc_p)) / dt_p,
                  "max_rel_residual": max(i["rel_residual"] for i in infos_p),
                  "graph_over_persistent_time": dt / dt_p}
    return {"problems": len(ws), "dof": dof, "converged": ok, "seconds": dt, "persistent_launch": persistent,
            "discretisation": "upwind",
            "substitute": "the batched workload is specified with biquadratic ConvFEM + PG; the non-linear "
                          "PG cycle does not contract on these optically thin media, so the solves to 1e-6 "
                          "run the upwind discretisation (same ordinates, levels and precision)",
            "dof_updates_per_s": sum(w.dof * c for w, c in zip(ws, cyc)) / dt,
            "cycles_min_max": [min(cyc), max(cyc)],
            "max_rel_residual": max(i["rel_residual"] for i in infos),
            "launch_shapes_by_n": {str(k): list(v) for k, v in sorted(shapes.items())}}


def step_throughput(wname, steps, warmup, launch_shape=None, log=None):
    """Time `steps` refinement steps of one workload (after `warmup` untimed ones) and return the
    measurements: whole-step wall time, every kernel class from an untimed diagnostic pass, and the
    dominant class timed with HIP events on the problem's stream inside the timed region."""
    import torch
    from paper_2301_09991_amd import ctf
    from workloads import WORKLOADS, make_inputs
    w = WORKLOADS[wname]
    st, ss, src = make_inputs(w)
    precision = ctf.FP32_IR_BF16_MOMENTS if w.scatter == "p1" else ctf.FP32_IR
    cfg = ctf.default_config(n=w.N, length=w.L, p=w.p, na=w.na, ngroups=w.G,
                             scatter_order=ss.shape[0] - 1, discretisation=ctf.CONVFEM_PG,
                             precision=precision)   # the library's default n_inner
    prob = ctf.Problem(cfg, st, ss, src)
    del st, ss, src
    if launch_shape:
        prob.set_launch_shape(*[int(v) for v in launch_shape.split(",")])
    psi = prob.zeros()
    torch.cuda.synchronize()
    if log:
        log(f"workload {w.name}: N={w.N} p={w.p} n_dir={w.n_dir} G={w.G} DOF={w.dof}")
    for _ in range(warmup):
        prob.mg_cycle(psi)
    torch.cuda.synchronize()
    # diagnostic pass (not timed): every kernel class timed, to find the dominant one and report the
    # breakdown; event records between launches cost time, so the timed region below records
    # events around the dominant class only
    n_diag = max(1, min(5, steps))
    prob.timing_enable(True, capacity=64 * n_diag)
    for _ in range(n_diag):
        prob.mg_cycle(psi)
    diag = prob.timing_read()
    prob.timing_enable(False)
    kernels = {}
    for name, (ms, n, dropped) in diag.items():
        if n:
            kernels[name] = {"avg_ms": ms / n, "launches_per_step": n / n_diag, "total_ms_per_step": ms / n_diag,
                             "dropped": dropped}
    dom = max(kernels, key=lambda k: kernels[k]["total_ms_per_step"])
    prob.timing_enable(True, capacity=64 * max(steps, 1), classes=[dom])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        prob.mg_cycle(psi)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    timed = prob.timing_read()[dom]
    prob.timing_enable(False)
    fused = bool(prob.launch_shape()[2])
    shape = dict(zip(("strip_h", "corr_block", "pg_fused"), prob.launch_shape()))
    del prob, psi
    torch.cuda.empty_cache()
    cycles = steps * cfg.n_inner
    avg_s = timed[0] / timed[1] * 1e-3
    bytes_per, flops_per = algorithmic_cost(dom, w.p, fused)
    gbs = w.dof * bytes_per / avg_s / 1e9
    tflops = w.dof * flops_per / avg_s / 1e12
    valu_peak = FP32_VALU_TFLOPS if dom.endswith("32") else FP64_VALU_TFLOPS
    hbm_time, alu_time = bytes_per / HBM_PEAK_GBS, flops_per / (valu_peak * 1e3)
    if hbm_time >= alu_time:
        roof = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS}
    else:
        roof = {"bound": "alu", "achieved": tflops, "peak": valu_peak, "unit": "TFLOP/s",
                "frac": tflops / valu_peak}
    sym, sym_file = kernel_symbol(dom, w.p, fused)
    impl_f = implementation_flops(dom, w.p, fused)
    impl_b = implementation_bytes(dom, w.p, fused)
    roof.update({"traffic": read_traffic(sym_file, w.name), "kernel": dom, "kernel_symbol": sym,
                 "algorithmic_bytes_per_dof": bytes_per, "algorithmic_flops_per_dof": flops_per,
                 "dof_per_launch": w.dof, "avg_launch_ms": avg_s * 1e3, "launches_timed": timed[1],
                 "hbm_gbs_at_algorithmic_bytes": gbs,
                 "implementation_flops_per_dof": impl_f,
                 "implementation_tflops": w.dof * impl_f / avg_s / 1e12,
                 "implementation_bytes_per_dof": impl_b})
    if roof["bound"] == "alu":
        # packed FP32 instructions are not used (build flags), so the vector rate this code can reach
        # is half the published FP32 figure; FP64 vector math has no packed form
        roof["frac_of_unpacked_vector_peak"] = tflops / (valu_peak / 2 if dom.endswith("32") else valu_peak)
    if log:
        log(f"{w.name}: {steps} steps in {dt:.3f} s ({1e3 * dt / steps:.3f} ms/step), dominant {sym} "
            f"{avg_s * 1e3:.3f} ms")
    return {"workload": w, "value": w.dof * cycles / dt, "ms_per_step": 1e3 * dt / steps, "dt": dt,
            "cycles_per_step": cfg.n_inner, "roofline": roof, "kernels": kernels, "n_diag": n_diag,
            "launch_shape": shape}


def describe(w, n_inner):
    scat = {"iso": "isotropic scattering", "downscatter": "downscatter", "p1": "P1 scattering"}[w.scatter]
    mom = ", bf16-MFMA moments in the float32 cycles" if w.scatter == "p1" else ""
    return (f"{w.name}: {w.N}x{w.N} nodes, L={w.L:g}, p={w.p} ConvFEM + non-linear PG, {w.n_dir} ordinates, "
            f"{w.G} group(s) {scat}, c in {list(w.c_range)}{mom}; step = f64 residual + {n_inner} f32 "
            f"sawtooth cycles + f64 update")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default="c4_learned")
    ap.add_argument("--also", default="c1_mixed,c2_mfma_p1",
                    help="other workloads whose step throughput is reported beside the headline ('' for none)")
    ap.add_argument("--also-steps", type=int, default=5)
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the time-to-tolerance, batched and straight-duct measurements")
    ap.add_argument("--duct-study", action="store_true",
                    help="run the straight-duct study (about a second) also with --no-extras")
    ap.add_argument("--launch-shape", default=None,
                    help="strip_h,corr_block,pg_fused for the timed problem (default: the library's)")
    ap.add_argument("--calibration-copy-mib", type=int, default=0,
                    help="before the workload, run an elementwise copy kernel (torch.neg) of this many "
                         "MiB three times, as the reference for hardware byte counters")
    ap.add_argument("--cpu-baseline-worker", type=int, default=0, help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.cpu_baseline_worker:
        cpu_baseline_worker(args.cpu_baseline_worker)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this solver runs on one GPU; multi-GPU runs are not part of it",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    log = lambda m: print(f"[bench] {m}", file=sys.stderr, flush=True)

    if args.calibration_copy_mib > 0:
        nel = args.calibration_copy_mib * (1 << 20) // 4
        a = torch.ones(nel, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            torch.neg(a, out=b)
        torch.cuda.synchronize()
        log(f"calibration copy: {nel * 4} bytes read and {nel * 4} written per launch")
        del a, b
    r = step_throughput(args.workload, args.steps, args.warmup, args.launch_shape, log)
    w = r["workload"]
    line = {
        "metric": METRIC, "value": r["value"], "unit": "DOF-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": r["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": describe(w, r["cycles_per_step"]), "dof": w.dof, "cycles_per_step": r["cycles_per_step"],
                   "outer_precision": "f64", "launch_shape": r["launch_shape"]},
        "roofline": r["roofline"],
        "kernels": r["kernels"],
        "kernels_from": f"diagnostic pass of {r['n_diag']} steps before the timed region, every class timed",
    }
    also = {}
    for name in [a for a in args.also.split(",") if a]:
        x = step_throughput(name, args.also_steps, 2, None, log)
        also[name] = {"workload": describe(x["workload"], x["cycles_per_step"]), "dof": x["workload"].dof, "value": x["value"],
                      "unit": "DOF-updates/s", "ms_per_step": x["ms_per_step"], "steps": args.also_steps,
                      "roofline": x["roofline"],
                      "kernels": {k: {"avg_ms": v["avg_ms"], "launches_per_step": v["launches_per_step"]}
                                  for k, v in x["kernels"].items()}}
        torch.cuda.empty_cache()
    if also:
        line["other_workloads"] = also
    if not args.no_extras:
        line["time_to_tol"] = time_to_tolerance(log)
        torch.cuda.empty_cache()
        line["batched"] = batched(log)
    if args.duct_study or not args.no_extras:
        line["duct_study"] = duct_study(log)
    if not args.no_cpu_baseline:
        log("timing the oracle on the host cores")
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line))


if __name__ == "__main__":
    main()
