"""Seeded synthetic inputs (materials, sources, problem sizes) for the fixed-source workloads.

This module holds input construction only: no part of the transport method's arithmetic.  Both the
HIP library's tests/benchmark and the CPU oracle take their inputs from here.

Random numbers come from numpy's PCG64 generator.  Coefficients are piecewise constant on square
patches of cells; per group the draws are, in order: sigma_t (uniform in [0.5, 2]), the
scattering ratio c, and for linearly anisotropic scattering the mean cosine gbar in [0, 0.6].
"""
from dataclasses import dataclass, field
import numpy as np


@dataclass
class Workload:
    name: str
    N: int            # nodes per side
    L: float          # domain side
    p: int            # ConvFEM element degree (1..3)
    na: int           # ordinates per face side: 8 * na^2 ordinates
    G: int            # energy groups
    patch: int        # cells per coefficient patch side
    scatter: str      # "iso", "downscatter", "p1"
    source: str       # "box_center8", "gaussian", "box_quarter", "box_quarter_phys"
    c_range: tuple = (0.3, 0.9)
    seed: int = 0
    rtol: float = 1e-8
    extra: dict = field(default_factory=dict)

    @property
    def n_dir(self):
        return 8 * self.na * self.na

    @property
    def dof(self):
        return self.N * self.N * self.n_dir * self.G


# The five fixed-source workloads (sizes, element degrees, angular grids, groups and coefficient
# statistics); "polar x azimuth" grids of 2na x 4na ordinates over the sphere are the octahedral
# 8 * na^2 sets.
WORKLOADS = {
    "c0_plain_fp64": Workload("c0_plain_fp64", 32, 1.0, 1, 4, 1, 4, "iso", "box_center8", seed=0, rtol=1e-8),
    "c1_mixed": Workload("c1_mixed", 256, 1.0, 2, 8, 2, 16, "downscatter", "gaussian", seed=1, rtol=1e-10),
    "c2_mfma_p1": Workload("c2_mfma_p1", 512, 1.0, 3, 16, 4, 32, "p1", "gaussian", seed=2, rtol=1e-6),
    "c4_learned": Workload("c4_learned", 1024, 32.0, 2, 8, 1, 32, "iso", "box_quarter_phys",
                           c_range=(0.8, 0.99), seed=4, rtol=1e-6),
}

BATCH_SIZES = (64, 96, 128, 192, 256, 384)


def scaled(w, N, patch=None, seed=None, na=None, G=None, name=None):
    """The same workload recipe on a smaller grid (tests): same p, statistics, source shape."""
    return Workload(name or (w.name + f"_N{N}"), N, w.L, w.p, w.na if na is None else na,
                    w.G if G is None else G, patch or max(1, w.patch * N // w.N), w.scatter, w.source,
                    w.c_range, w.seed if seed is None else seed, w.rtol, dict(w.extra))


def batch_workloads(n=64, size_seed=3, base_seed=3000):
    """The batched set: n independent problems, N drawn uniformly from BATCH_SIZES."""
    rng = np.random.Generator(np.random.PCG64(size_seed))
    sizes = rng.choice(np.array(BATCH_SIZES), size=n)
    return [Workload(f"c3_batch_{k}", int(N), 1.0, 2, 8, 1, 4, "iso", "box_quarter",
                     seed=base_seed + k, rtol=1e-6) for k, N in enumerate(sizes)]


def _patch_field(rng, N, patch, lo, hi):
    npatch = -(-N // patch)
    vals = rng.uniform(lo, hi, size=(npatch, npatch))
    return np.repeat(np.repeat(vals, patch, axis=0), patch, axis=1)[:N, :N]


def make_inputs(w):
    """sigma_t[G,N,N], sigma_s[l, g_to, g_from, N, N], source[G,N,N] (all float64)."""
    rng = np.random.Generator(np.random.PCG64(w.seed))
    N, G = w.N, w.G
    st = np.zeros((G, N, N))
    cc = np.zeros((G, N, N))
    gb = np.zeros((G, N, N))
    for g in range(G):
        st[g] = _patch_field(rng, N, w.patch, 0.5, 2.0)
        cc[g] = _patch_field(rng, N, w.patch, *w.c_range)
        if w.scatter == "p1":
            gb[g] = _patch_field(rng, N, w.patch, 0.0, 0.6)
    nl = 2 if w.scatter == "p1" else 1
    ss = np.zeros((nl, G, G, N, N))
    if w.scatter == "iso":
        for g in range(G):
            ss[0, g, g] = cc[g] * st[g]
    elif w.scatter in ("downscatter", "p1"):
        for g in range(G):
            if g + 1 < G:
                ss[0, g, g] = 0.5 * cc[g] * st[g]
                ss[0, g + 1, g] = 0.5 * cc[g] * st[g]
            else:
                ss[0, g, g] = cc[g] * st[g]
        if w.scatter == "p1":
            for g in range(G):
                for gt in range(G):
                    ss[1, gt, g] = gb[g] * ss[0, gt, g]
    else:
        raise ValueError(w.scatter)
    src = np.zeros((G, N, N))
    h = w.L / N
    xc = (np.arange(N) + 0.5) * h
    if w.source == "box_center8":
        lo = N // 2 - N // 8
        src[0, lo:lo + N // 4, lo:lo + N // 4] = 1.0
    elif w.source == "box_quarter":
        lo = (N - N // 4) // 2
        src[0, lo:lo + N // 4, lo:lo + N // 4] = 1.0
    elif w.source == "box_quarter_phys":
        a, b = 0.5 * w.L - w.L / 8, 0.5 * w.L + w.L / 8
        inside = (xc >= a) & (xc < b)
        src[0] = np.outer(inside, inside).astype(float)
    elif w.source == "gaussian":
        X, Y = np.meshgrid(xc, xc, indexing="xy")
        c = 0.5 * w.L
        src[0] = np.exp(-((X - c) ** 2 + (Y - c) ** 2) / (2 * 0.1**2))
    else:
        raise ValueError(w.source)
    return st, ss, src


def random_field(shape, seed, lo=-1.0, hi=1.0):
    """Seeded uniform random array (test vectors such as psi for operator parity)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(lo, hi, size=shape)


# ------------------------------------------------------------------------------------------------
# Straight-duct problem (the paper's mono-energetic fixed-source duct study; its table of
# regions): a 28 cm (x) by 36 cm (y) domain.  Region 1, the 6 x 6 cm source in the centre
# (x in [11, 17], y in [15, 21]): S = 1, sigma_a = 0.5; region 2, absorber on both sides of the
# duct column (x < 11 or x > 17): sigma_a = 0.5; region 3, the duct above and below the source
# (x in [11, 17]): void.  No scattering.  The solver's domains are square, so the 28 cm width is
# centred in a 36 cm square and the 4 cm on either side are void: with no scattering there, a
# particle that leaves the 28 cm domain never returns, as at a vacuum boundary.  Each cell takes
# the area average of sigma and S over it, so that every resolution (the region edges fall inside
# cells at dx = 0.8 and 0.4) carries the same total source and absorber.
DUCT_WIDTH, DUCT_HEIGHT = 28.0, 36.0
DUCT_PAD = (DUCT_HEIGHT - DUCT_WIDTH) / 2.0


def _overlap(a0, a1, b0, b1):
    return np.clip(np.minimum(a1, b1) - np.maximum(a0, b0), 0.0, None)


def duct_inputs(dx):
    """(N, L, sigma_t[1, N, N], sigma_s[1, 1, 1, N, N], source[1, N, N]) at node spacing dx."""
    L = DUCT_HEIGHT
    N = int(round(L / dx))
    if abs(N * dx - L) > 1e-9 * L:
        raise ValueError("dx must divide 36 cm")
    e0 = np.arange(N) * dx
    x0, x1 = e0 - DUCT_PAD, e0 + dx - DUCT_PAD    # cell edges in the 28 cm frame
    y0, y1 = e0, e0 + dx
    fx_abs = (_overlap(x0, x1, 0.0, 11.0) + _overlap(x0, x1, 17.0, DUCT_WIDTH)) / dx
    fx_col = _overlap(x0, x1, 11.0, 17.0) / dx
    fy_src = _overlap(y0, y1, 15.0, 21.0) / dx
    f_src = fy_src[:, None] * fx_col[None, :]
    f_abs = np.ones((N, 1)) * fx_abs[None, :]
    sigma = 0.5 * (f_abs + f_src)
    return N, L, sigma[None].copy(), np.zeros((1, 1, 1, N, N)), f_src[None].copy()
