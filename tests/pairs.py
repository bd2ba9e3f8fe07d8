"""Build the same problem twice: once in the CPU oracle, once in the HIP library (GPU tests)."""
import numpy as np

from oracle import multigrid as omg
from oracle.transport import VACUUM, ZERO_GRADIENT
from workloads import Workload, make_inputs

DISC = {"upwind": (omg.UPWIND, 0), "pg": (omg.PG, 1), "pg_frozen": (omg.PG_FROZEN, 2)}
BCS = {"vac": (VACUUM,) * 4,
       "mixed": (VACUUM, ZERO_GRADIENT, ZERO_GRADIENT, VACUUM),
       "zg": (ZERO_GRADIENT,) * 4}


def workload(N=40, na=2, G=1, scatter="iso", p=2, L=1.0, patch=8, seed=11, source="gaussian",
             c_range=(0.3, 0.9)):
    return Workload(f"test_N{N}", N, L, p, na, G, patch, scatter, source, c_range, seed)


def make_pair(w, disc="pg", bc="vac", precision=0, n_jacobi=2, n_pg=2, n_inner=2, max_levels=0,
              hemisphere=False, coupled=False, isotropic=False, r_estimate="mixed"):
    from paper_2301_09991_amd import ctf
    st, ss, src = make_inputs(w)
    od, cd = DISC[disc]
    bcs = BCS[bc]
    oprob = omg.Problem(w.N, w.L, w.p, w.na, st, ss, src, bc=bcs, disc=od, n_jacobi=n_jacobi,
                        n_pg=n_pg, max_levels=max_levels, coupled=coupled, isotropic=isotropic,
                        r_estimate=r_estimate)
    cfg = ctf.default_config(n=w.N, length=w.L, p=w.p, na=w.na, ngroups=w.G,
                             scatter_order=ss.shape[0] - 1, discretisation=cd,
                             bc=[0 if b == VACUUM else 1 for b in bcs], precision=precision,
                             n_jacobi=n_jacobi, n_pg=n_pg, n_inner=n_inner, max_levels=max_levels,
                             hemisphere=int(hemisphere), coupled_scatter=int(coupled),
                             pg_isotropic=int(isotropic),
                             pg_r_estimate={"mixed": 0, "low": 1, "high": 2}[r_estimate])
    gprob = ctf.Problem(cfg, st, ss, src)
    return oprob, gprob


def to_dev(x):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def to_host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel_w(a, b, quad, h):
    """||a - b||_W / ||b||_W."""
    d = np.einsum("gnji,n->", (a - b) ** 2, quad["p"])
    r = np.einsum("gnji,n->", b ** 2, quad["p"])
    return float(np.sqrt(d / r))
