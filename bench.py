"""Throughput benchmark of the ConvFEM space-angle multigrid solver on one MI355X.

Workload (the mixed-precision workload): 256 x 256 nodes on the unit square, biquadratic ConvFEM
(p = 2) with the non-linear anisotropic Petrov-Galerkin dissipation, 512 ordinates (octahedral,
8 x 8 patches per face = 16 polar x 32 azimuthal), 2 energy groups with downscatter-only
scattering, coefficients piecewise constant on 16 x 16-cell patches, Gaussian source (sigma 0.1).
All inputs are seeded synthetic arrays (workloads.make_inputs).

One step = one refinement step of the solver: float64 residual (with the diffusivities of the
current psi) + float64 norm, n_inner = 2 float32 sawtooth cycles on the correction equation, and
the float64 update.  value = finest DOF x float32 cycles / second.  Inputs are resident in HBM
before the timed region starts.

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


def algorithmic_cost(kernel, p, fused=False):
    """Algorithmic bytes and flops per finest DOF of one launch of a kernel class.

    Bytes: arrays every DOF must read or write once (per-cell data shared by all ordinates --
    sigma_t, emission moments -- is amortised to ~0).  Flops: two per multiply-add of the
    separable (tensor-product) evaluation with W = 2p + 1 taps, divisions and minima counted as one.
    """
    W = 2 * p + 1
    stream = 16 * W + 16 * W + 23      # 7 x-pass sums (+2 products per tap), 8 y-passes, epilogue
    kdiff = 16 * W + 34                 # Psi_x, Psi_y (x + y passes), R (x + y passes), k_x, k_y
    if kernel == "pg32":               # refinement inner cycles, full-approximation form
        return (12, stream + kdiff) if fused else (20, stream)   # read x, rhs (+ k_x, k_y); write out
    if kernel == "pg32_update":        # the same, plus psi64 += u - fl32(psi64): read and write psi64
        return (28, stream + kdiff + 3) if fused else (36, stream + 3)
    if kernel == "pgk32":              # read x; write k_x, k_y
        return 12, kdiff
    if kernel == "pg64":               # outer residual: read psi (+ k_x, k_y); write float32 residual and psi
        return (16, stream + kdiff) if fused else (32, stream)
    if kernel == "pgk64":
        return 24, kdiff
    if kernel in ("corr0", "upwind32"):
        return 12, 12                   # read e, rhs; write e (last sweep: read-modify-write)
    if kernel == "upwind64":
        return 24, 12
    if kernel in ("moments", "moments_mfma"):
        return 4, 6
    raise KeyError(kernel)


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


def read_traffic(kernel_symbol):
    """HBM bytes per DOF of the dominant kernel from the committed rocprofv3 counter summary, if it
    was taken on the kernel source as it is now (else None)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic_%s.txt" % kernel_symbol)
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


def cpu_baseline(seconds_hint=20.0):
    """Time the FP64 oracle (single thread) on a bounded sample: one sawtooth cycle of the same
    workload recipe at N = 64 (same p, ordinates, groups), in a subprocess."""
    code = r"""
import json, os, sys, time
sys.path.insert(0, %r)
from oracle import multigrid as omg
from workloads import WORKLOADS, make_inputs, scaled
w = scaled(WORKLOADS["c1_mixed"], 64)
st, ss, src = make_inputs(w)
prob = omg.Problem(w.N, w.L, w.p, w.na, st, ss, src, disc=omg.PG)
import numpy as np
psi = np.zeros(prob.shape())
t = time.time(); cycles = 0
while True:
    psi = omg.sawtooth_cycle(prob, psi); cycles += 1
    if time.time() - t > %f or cycles >= 3:
        break
dt = time.time() - t
print(json.dumps({"dof": w.dof, "cycles": cycles, "seconds": dt}))
""" % (ROOT, seconds_hint)
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                         timeout=600)
    if out.returncode != 0:
        return {"error": out.stderr[-500:]}
    r = json.loads(out.stdout.strip().splitlines()[-1])
    return {"value": r["dof"] * r["cycles"] / r["seconds"], "unit": "DOF-updates/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{r['cycles']} float64 oracle sawtooth cycle(s) of the same recipe at N=64 "
                      f"({r['dof']} DOF, p=2, 512 ordinates, 2 groups), numpy single thread, "
                      f"{r['seconds']:.1f} s"}


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
    flux along the duct centre line x = 14 cm; and the PG residual after the paper's 100 cycles at
    dx = 0.4 for p = 1, 2, 3."""
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
    pg = {}
    for p in (1, 2, 3):
        info, _ = run(0.4, 4, ctf.CONVFEM_PG, p, rtol=1e-10, cycles=100)
        pg[f"p{p}"] = {"cycles": info["cycles"], "rel_residual": info["rel_residual"]}
    out["pg_after_100_cycles_dx0.4"] = pg
    log(f"duct errors {errs}, orders {out['observed_order']}")
    return out


def batched(log):
    """The batched workload: 64 problems with sizes drawn from {64, ..., 384}^2, p = 2, 512
    ordinates, one group, upwind discretisation, float32 cycles + float64 refinement to 1e-6, all
    solved by replays of one captured HIP graph; launch shapes autotuned per size."""
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
    return {"problems": len(ws), "dof": dof, "converged": ok, "seconds": dt,
            "dof_updates_per_s": sum(w.dof * c for w, c in zip(ws, cyc)) / dt,
            "cycles_min_max": [min(cyc), max(cyc)],
            "max_rel_residual": max(i["rel_residual"] for i in infos),
            "launch_shapes_by_n": {str(k): list(v) for k, v in sorted(shapes.items())}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default="c1_mixed")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the time-to-tolerance and batched measurements")
    ap.add_argument("--duct-study", action="store_true",
                    help="also run the straight-duct self-convergence study (reported in the JSON line)")
    ap.add_argument("--launch-shape", default=None,
                    help="strip_h,corr_block,pg_fused for the timed problem (default: the library's)")
    ap.add_argument("--calibration-copy-mib", type=int, default=0,
                    help="before the workload, run an elementwise copy kernel (torch.neg) of this many "
                         "MiB three times, as the reference for hardware byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this solver runs on one GPU; multi-GPU runs are not part of it",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2301_09991_amd import ctf
    from workloads import WORKLOADS, make_inputs

    if args.calibration_copy_mib > 0:
        nel = args.calibration_copy_mib * (1 << 20) // 4
        a = torch.ones(nel, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            torch.neg(a, out=b)
        torch.cuda.synchronize()
        print(f"[bench] calibration copy: {nel * 4} bytes read and {nel * 4} written per launch",
              file=sys.stderr, flush=True)
        del a, b
    w = WORKLOADS[args.workload]
    st, ss, src = make_inputs(w)
    cfg = ctf.default_config(n=w.N, length=w.L, p=w.p, na=w.na, ngroups=w.G,
                             scatter_order=ss.shape[0] - 1, discretisation=ctf.CONVFEM_PG,
                             precision=ctf.FP32_IR, n_inner=2)
    prob = ctf.Problem(cfg, st, ss, src)
    del st, ss, src
    if args.launch_shape:
        prob.set_launch_shape(*[int(v) for v in args.launch_shape.split(",")])
    psi = prob.zeros()
    torch.cuda.synchronize()
    print(f"[bench] workload {w.name}: N={w.N} p={w.p} n_dir={w.n_dir} G={w.G} DOF={w.dof}",
          file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        prob.mg_cycle(psi)
    torch.cuda.synchronize()
    # diagnostic pass (not timed): every kernel class timed, to find the dominant one and report the
    # breakdown; event records between launches cost time, so the timed region below records
    # events around the dominant class only
    n_diag = max(1, min(5, args.steps))
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
    prob.timing_enable(True, capacity=64 * max(args.steps, 1), classes=[dom])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        prob.mg_cycle(psi)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    timed = prob.timing_read()[dom]
    prob.timing_enable(False)
    ms_per_step = 1e3 * dt / args.steps
    cycles = args.steps * cfg.n_inner
    value = w.dof * cycles / dt
    print(f"[bench] {args.steps} steps in {dt:.3f} s ({ms_per_step:.3f} ms/step)", file=sys.stderr,
          flush=True)

    avg_s = timed[0] / timed[1] * 1e-3
    fused = bool(prob.launch_shape()[2])
    bytes_per, flops_per = algorithmic_cost(dom, w.p, fused)
    gbs = w.dof * bytes_per / avg_s / 1e9
    tflops = w.dof * flops_per / avg_s / 1e12
    valu_peak = FP32_VALU_TFLOPS if dom.endswith("32") else FP64_VALU_TFLOPS
    hbm_time, alu_time = bytes_per / HBM_PEAK_GBS, flops_per / (valu_peak * 1e3)
    if hbm_time >= alu_time:
        roof = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": gbs / HBM_PEAK_GBS}
    else:
        roof = {"bound": "alu", "achieved": tflops, "peak": valu_peak, "unit": "TFLOP/s",
                "frac": tflops / valu_peak}
    sym, sym_file = kernel_symbol(dom, w.p, fused)
    traffic = read_traffic(sym_file)
    roof.update({"traffic": traffic, "kernel": dom, "kernel_symbol": sym,
                 "algorithmic_bytes_per_dof": bytes_per,
                 "algorithmic_flops_per_dof": flops_per, "dof_per_launch": w.dof,
                 "avg_launch_ms": avg_s * 1e3, "launches_timed": timed[1]})

    line = {
        "metric": METRIC, "value": value, "unit": "DOF-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {w.N}x{w.N} nodes, p={w.p} ConvFEM + non-linear PG, "
                               f"{w.n_dir} ordinates, {w.G} groups downscatter; step = f64 residual"
                               f" + {cfg.n_inner} f32 sawtooth cycles + f64 update",
                   "dof": w.dof, "cycles_per_step": cfg.n_inner, "outer_precision": "f64",
                   "launch_shape": dict(zip(("strip_h", "corr_block", "pg_fused"), prob.launch_shape()))},
        "roofline": roof,
        "kernels": kernels,
        "kernels_from": f"diagnostic pass of {n_diag} steps before the timed region, every class timed",
    }
    del prob, psi
    torch.cuda.empty_cache()
    log = lambda m: print(f"[bench] {m}", file=sys.stderr, flush=True)
    if not args.no_extras:
        line["time_to_tol"] = time_to_tolerance(log)
        torch.cuda.empty_cache()
        line["batched"] = batched(log)
    if args.duct_study:
        line["duct_study"] = duct_study(log)
    if not args.no_cpu_baseline:
        log("timing the oracle on the host cores")
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line))


if __name__ == "__main__":
    main()
