"""Training driver of the learned coarse-grid correction (orchestration only: every sample, loss,
gradient and Adam step is computed by the HIP library; PyTorch holds the device buffers).

Samples come from the solver itself: for each seeded training problem the float64 cycle is run to
a tight residual (psi*), then restarted from zero; at chosen cycles k the library records the
network input of the cycle's starting residual and the angle-integrated error psi* - psi left
after that plain cycle (both on the grid of the correction level, the error in units of the
input's scale).  The network is trained on these pairs by mean-squared error with Adam.
"""
import numpy as np

from . import ctf

SAMPLE_CYCLES = (1, 2, 4, 8, 16, 32)


def init_params(seed, device="cuda"):
    """Seeded He-uniform weights (bound sqrt(6 / fan_in)), zero biases, flat float32 vector."""
    import torch
    rng = np.random.Generator(np.random.PCG64(seed))
    chans = (3, 32, 32, 32, 1)
    parts = []
    for ci, co in zip(chans[:-1], chans[1:]):
        bound = np.sqrt(6.0 / (ci * 9))
        parts.append(rng.uniform(-bound, bound, size=co * ci * 9))
        parts.append(np.zeros(co))
    theta = np.concatenate(parts).astype(np.float32)
    assert theta.size == ctf.cnn_param_count()
    return torch.as_tensor(theta, device=device)


def make_problem(w, inputs, cnn_level, precision=ctf.FP64, disc=ctf.UPWIND, n_inner=4, max_growth=1.0,
                 max_uses=2, hemisphere=False, coupled=False):
    st, ss, src = inputs
    cfg = ctf.default_config(n=w.N, length=w.L, p=w.p, na=w.na, ngroups=w.G,
                             scatter_order=ss.shape[0] - 1, discretisation=disc,
                             precision=precision, n_inner=n_inner, cnn_level=cnn_level,
                             cnn_max_growth=max_growth, cnn_max_uses=max_uses, hemisphere=int(hemisphere),
                             coupled_scatter=int(coupled))
    return ctf.Problem(cfg, st, ss, src)


def generate_samples(workloads, make_inputs, cnn_level=0, cycles=SAMPLE_CYCLES, star_rtol=1e-9,
                     max_cycles=4000, disc=ctf.UPWIND):
    """Features [S, 3, nc, nc] and targets [S, 1, nc, nc] (float32 device tensors).

    workloads: a list of workloads sampled at ``cnn_level``, or of (workload, level) pairs; all
    must give the same correction grid nc = N / 2^level."""
    import torch
    feats, tgts = [], []
    kmax = max(cycles)
    # the reference solutions psi* of a group of problems in one batched solve (the iterates of
    # individual solves, bit for bit), then the sampling cycles problem by problem
    group = 64
    for g0 in range(0, len(workloads), group):
        probs, stars = [], []
        for item in workloads[g0:g0 + group]:
            w, lvl = item if isinstance(item, tuple) else (item, cnn_level)
            probs.append(make_problem(w, make_inputs(w), lvl, disc=disc))
            stars.append(probs[-1].zeros())
        ctf.solve_batch(probs, stars, star_rtol, max_cycles, 4)
        for prob, star in zip(probs, stars):
            nc = prob.cnn_grid()
            psi = prob.zeros()
            for k in range(1, kmax + 1):
                if k in cycles:
                    f = torch.empty((3, nc, nc), dtype=torch.float32, device="cuda")
                    t = torch.empty((1, nc, nc), dtype=torch.float32, device="cuda")
                    prob.cnn_sample(psi, star, f, t)
                    feats.append(f)
                    tgts.append(t)
                else:
                    prob.mg_cycle(psi)
        del probs, stars
    return torch.stack(feats), torch.stack(tgts)


def train(features, targets, epochs=60, batch=16, lr=1e-3, seed=0, bf16=True, log=None):
    """Adam on the mean-squared error; returns (params, per-epoch mean training loss)."""
    import torch
    S, _, h, w = features.shape
    net = ctf.Cnn(batch, h, w)
    theta = init_params(seed)
    m = torch.zeros_like(theta)
    v = torch.zeros_like(theta)
    grad = torch.zeros_like(theta)
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    history, step = [], 0
    for ep in range(epochs):
        # the epoch's order goes to the device once and its losses are summed there: one host
        # synchronisation per epoch
        perm = torch.as_tensor(rng.permutation(S), device=theta.device)
        loss_sum = torch.zeros(1, dtype=torch.float64, device=theta.device)
        nb = 0
        for b0 in range(0, S - batch + 1, batch):
            idx = perm[b0:b0 + batch]
            x = features.index_select(0, idx).contiguous()
            t = targets.index_select(0, idx).contiguous()
            loss_sum += net.loss_grad(theta, x, t, grad, bf16=bf16)
            nb += 1
            step += 1
            net.adam(theta, m, v, grad, step, lr)
        history.append(float(loss_sum.item()) / nb if nb else float("nan"))
        if log:
            log(f"epoch {ep}: loss {history[-1]:.4e}")
    return theta, history


def evaluate_loss(theta, features, targets, bf16=True):
    import torch
    S, _, h, w = features.shape
    net = ctf.Cnn(S, h, w)
    grad = torch.zeros_like(theta)
    return net.loss_grad(theta, features.contiguous(), targets.contiguous(), grad, bf16=bf16).item()
