"""ctypes binding of the C-ABI in include/ctf.h (argument marshalling only).

Device memory and streams come from PyTorch-ROCm tensors; every step of the solver runs in the HIP
library ``libctf.so`` built in this directory.  Loading fails loudly when the library is missing:
there is no fallback implementation.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libctf.so")

CTF_OK, CTF_NOT_CONVERGED = 0, 1
CTF_EINVAL, CTF_ENOMEM, CTF_EHIP, CTF_ENONFINITE, CTF_EUNSUPPORTED = -1, -2, -3, -4, -5
UPWIND, CONVFEM_PG, CONVFEM_PG_FROZEN_K = 0, 1, 2
VACUUM, ZERO_GRADIENT = 0, 1
FP64, FP32_IR, FP32_IR_BF16_MOMENTS = 0, 1, 2
OP_APPLY, OP_RESIDUAL = 0, 1
SMOOTH_UPWIND, SMOOTH_FINEST = 0, 1
R_MIXED_MASS, R_LOW, R_HIGH = 0, 1, 2

EXPORTED = [
    "ctf_default_config", "ctf_workspace_bytes", "ctf_create_problem", "ctf_destroy_problem",
    "ctf_num_levels", "ctf_level_info", "ctf_level_quadrature", "ctf_convfem_stencils",
    "ctf_level_sigma_t", "ctf_apply_operator", "ctf_moments", "ctf_freeze_k", "ctf_smooth",
    "ctf_restrict", "ctf_prolong", "ctf_mg_cycle", "ctf_solve", "ctf_norm", "ctf_last_error",
    "ctf_quadrature", "ctf_timing_enable", "ctf_timing_read", "ctf_moments_f32",
    "ctf_cnn_param_count", "ctf_cnn_workspace_bytes", "ctf_cnn_forward", "ctf_cnn_loss_grad",
    "ctf_cnn_adam", "ctf_cnn_attach", "ctf_cnn_enable", "ctf_cnn_sample",
    "ctf_solve_batch", "ctf_set_launch_shape", "ctf_get_launch_shape", "ctf_autotune",
    "ctf_cnn_forward_noalloc", "ctf_solve_batch_persistent", "ctf_solve_batch_persistent_bytes",
]
TIMER_CLASSES = ["pg64", "pg32", "upwind64", "upwind32", "corr0", "corrc", "restrict", "moments",
                 "emission", "norm", "moments_mfma", "cnn", "pgk64", "pgk32", "corr_scatter",
                 "pg32_update"]


class Config(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int), ("length", ctypes.c_double), ("p", ctypes.c_int), ("na", ctypes.c_int),
        ("ngroups", ctypes.c_int), ("scatter_order", ctypes.c_int), ("discretisation", ctypes.c_int),
        ("bc", ctypes.c_int * 4), ("precision", ctypes.c_int), ("n_jacobi", ctypes.c_int),
        ("n_pg", ctypes.c_int), ("max_levels", ctypes.c_int), ("beta_pg", ctypes.c_double),
        ("alpha_r", ctypes.c_double), ("eps_k", ctypes.c_double), ("n_inner", ctypes.c_int),
        ("cnn_level", ctypes.c_int), ("cnn_max_growth", ctypes.c_double), ("cnn_max_uses", ctypes.c_int),
        ("hemisphere", ctypes.c_int), ("coupled_scatter", ctypes.c_int), ("pg_isotropic", ctypes.c_int),
        ("pg_r_estimate", ctypes.c_int),
    ]


class LevelDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("na", ctypes.c_int), ("n_dir", ctypes.c_int),
                ("h", ctypes.c_double), ("dof", ctypes.c_longlong)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("cycles", ctypes.c_int), ("outer_steps", ctypes.c_int),
                ("rel_residual", ctypes.c_double), ("seconds", ctypes.c_double),
                ("history", ctypes.POINTER(ctypes.c_double)), ("history_len", ctypes.c_int),
                ("cnn_applied", ctypes.c_int), ("cnn_rejected", ctypes.c_int)]


_lib = None


def load():
    """Load libctf.so (built by paper_2301_09991_amd/build.py); raise if it is absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library {LIB_PATH} is not built: run paper_2301_09991_amd/build.py")
    # PyTorch first: libctf.so then binds to the HIP runtime PyTorch loaded (same soname), so
    # device pointers and streams handed over from torch tensors are valid in the library.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    P, I, D, S = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    cfgp = ctypes.POINTER(Config)
    sig = {
        "ctf_default_config": (None, [cfgp]),
        "ctf_workspace_bytes": (S, [cfgp]),
        "ctf_create_problem": (I, [cfgp, P, P, P, P, S, P, ctypes.POINTER(P)]),
        "ctf_destroy_problem": (None, [P]),
        "ctf_num_levels": (I, [P]),
        "ctf_level_info": (I, [P, I, ctypes.POINTER(LevelDesc)]),
        "ctf_level_quadrature": (I, [P, I, P, P, P]),
        "ctf_convfem_stencils": (I, [I, P, P, P]),
        "ctf_quadrature": (I, [I, P, P, P]),
        "ctf_level_sigma_t": (I, [P, I, P]),
        "ctf_apply_operator": (I, [P, P, P, I]),
        "ctf_moments": (I, [P, P, P]),
        "ctf_moments_f32": (I, [P, P, P, I]),
        "ctf_cnn_param_count": (I, []),
        "ctf_cnn_workspace_bytes": (S, [I, I, I]),
        "ctf_cnn_forward": (I, [P, P, P, I, I, I, I, P, S, P]),
        "ctf_cnn_loss_grad": (I, [P, P, P, I, I, I, I, P, P, P, S, P]),
        "ctf_cnn_forward_noalloc": (I, [P, P, P, I, I, I, I, P]),
        "ctf_cnn_adam": (I, [P, P, P, P, I, I, ctypes.c_float, P]),
        "ctf_cnn_attach": (I, [P, P]),
        "ctf_cnn_enable": (I, [P, I]),
        "ctf_cnn_sample": (I, [P, P, P, P, P, ctypes.POINTER(D)]),
        "ctf_solve_batch": (I, [ctypes.POINTER(P), I, ctypes.POINTER(P), D, I, I, ctypes.POINTER(SolveInfo)]),
        "ctf_solve_batch_persistent": (I, [ctypes.POINTER(P), I, ctypes.POINTER(P), D, I, I, P, S,
                                           ctypes.POINTER(SolveInfo)]),
        "ctf_solve_batch_persistent_bytes": (S, [ctypes.POINTER(P), I, I]),
        "ctf_set_launch_shape": (I, [P, I, I, I]),
        "ctf_get_launch_shape": (I, [P, ctypes.POINTER(I), ctypes.POINTER(I), ctypes.POINTER(I)]),
        "ctf_autotune": (I, [P, ctypes.c_char_p, I, ctypes.POINTER(I), ctypes.POINTER(I), ctypes.POINTER(I)]),
        "ctf_freeze_k": (I, [P, P, P, P]),
        "ctf_smooth": (I, [P, I, I, P, P, I]),
        "ctf_restrict": (I, [P, I, P, P]),
        "ctf_prolong": (I, [P, I, P, P]),
        "ctf_mg_cycle": (I, [P, P, ctypes.POINTER(D)]),
        "ctf_solve": (I, [P, P, D, I, ctypes.POINTER(SolveInfo)]),
        "ctf_norm": (I, [P, P, ctypes.POINTER(D)]),
        "ctf_last_error": (ctypes.c_char_p, []),
        "ctf_timing_enable": (I, [P, I, I, ctypes.c_uint]),
        "ctf_timing_read": (I, [P, I, ctypes.POINTER(D), ctypes.POINTER(I), ctypes.POINTER(I)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class CtfError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"ctf error {code}: {msg}")
        self.code = code


def _check(rc, allow_not_converged=False):
    if rc == CTF_OK or (allow_not_converged and rc == CTF_NOT_CONVERGED):
        return rc
    raise CtfError(rc, load().ctf_last_error().decode())


def default_config(**kw):
    cfg = Config()
    load().ctf_default_config(ctypes.byref(cfg))
    for k, v in kw.items():
        if k == "bc":
            for s in range(4):
                cfg.bc[s] = int(v[s])
        else:
            setattr(cfg, k, v)
    return cfg


def workspace_bytes(cfg):
    nb = load().ctf_workspace_bytes(ctypes.byref(cfg))
    if nb == 0:
        raise CtfError(CTF_EINVAL, load().ctf_last_error().decode())
    return nb


def convfem_stencils(p):
    import numpy as np
    m, d, k = (np.zeros(2 * p + 1) for _ in range(3))
    _check(load().ctf_convfem_stencils(p, m.ctypes.data, d.ctypes.data, k.ctypes.data))
    return m, d, k


def quadrature(na):
    """Finest-level ordinates (mu, nu, w) of the octahedral set with 8 na^2 ordinates."""
    import numpy as np
    nd = 8 * na * na
    mu, nu, w = np.zeros(nd), np.zeros(nd), np.zeros(nd)
    _check(load().ctf_quadrature(na, mu.ctypes.data, nu.ctypes.data, w.ctypes.data))
    return mu, nu, w


def solve_batch(problems, psis, rtol, max_steps, steps_per_graph=1):
    """Solve several problems with one captured HIP graph (ctf_solve_batch)."""
    n = len(problems)
    lib = load()
    hs = (ctypes.c_void_p * n)(*[p.handle.value for p in problems])
    ps = (ctypes.c_void_p * n)(*[t.data_ptr() for t in psis])
    infos = (SolveInfo * n)()
    rc = _check(lib.ctf_solve_batch(hs, n, ps, rtol, max_steps, steps_per_graph, infos),
                allow_not_converged=True)
    return rc == CTF_OK, [{"cycles": i.cycles, "outer_steps": i.outer_steps, "rel_residual": i.rel_residual,
                           "seconds": i.seconds} for i in infos]


def solve_batch_persistent(problems, psis, rtol, max_steps, items_per_block=0):
    """Solve several problems in one launch of the persistent kernel (ctf_solve_batch_persistent);
    the schedule's workspace is a torch allocation on the problems' device."""
    import torch
    n = len(problems)
    lib = load()
    hs = (ctypes.c_void_p * n)(*[p.handle.value for p in problems])
    ps = (ctypes.c_void_p * n)(*[t.data_ptr() for t in psis])
    nb = lib.ctf_solve_batch_persistent_bytes(hs, n, items_per_block)
    if nb == 0:
        raise CtfError(CTF_EINVAL, lib.ctf_last_error().decode())
    ws = torch.empty(nb, dtype=torch.uint8, device=psis[0].device)
    infos = (SolveInfo * n)()
    rc = _check(lib.ctf_solve_batch_persistent(hs, n, ps, rtol, max_steps, items_per_block,
                                               ctypes.c_void_p(ws.data_ptr()), nb, infos),
                allow_not_converged=True)
    return rc == CTF_OK, [{"cycles": i.cycles, "outer_steps": i.outer_steps, "rel_residual": i.rel_residual,
                           "seconds": i.seconds} for i in infos]


def cnn_param_count():
    return load().ctf_cnn_param_count()


# largest batch * h * w of cnn_forward_noalloc
CNN_NOALLOC_MAX_PIXELS = 32768


def cnn_forward_noalloc(params, x, out, bf16=True, stream=None):
    """net(x) into out without any workspace or allocation (x: float32 [batch][3][h][w])."""
    import torch
    b, _, h, w = x.shape
    s = stream if stream is not None else torch.cuda.current_stream(x.device)
    _check(load().ctf_cnn_forward_noalloc(_ptr(params), _ptr(x), _ptr(out), b, h, w, int(bf16),
                                          ctypes.c_void_p(s.cuda_stream)))
    return out


class Cnn:
    """Network kernels on caller-owned float32 device tensors (workspace sized per batch)."""

    def __init__(self, batch, h, w, device="cuda", stream=None):
        import torch
        self.torch = torch
        self.lib = load()
        self.batch, self.h, self.w = batch, h, w
        self.stream = stream if stream is not None else torch.cuda.current_stream(torch.device(device))
        nb = self.lib.ctf_cnn_workspace_bytes(batch, h, w)
        self.ws = torch.empty(nb, dtype=torch.uint8, device=device)
        self.loss = torch.zeros(1, dtype=torch.float64, device=device)

    def _s(self):
        return ctypes.c_void_p(self.stream.cuda_stream)

    def forward(self, params, x, out, bf16=True):
        b = x.shape[0]
        _check(self.lib.ctf_cnn_forward(_ptr(params), _ptr(x), _ptr(out), b, self.h, self.w, int(bf16),
                                        _ptr(self.ws), self.ws.numel(), self._s()))
        return out

    def loss_grad(self, params, x, target, grad, bf16=True):
        b = x.shape[0]
        _check(self.lib.ctf_cnn_loss_grad(_ptr(params), _ptr(x), _ptr(target), b, self.h, self.w, int(bf16),
                                          _ptr(grad), _ptr(self.loss), _ptr(self.ws), self.ws.numel(),
                                          self._s()))
        return self.loss

    def adam(self, params, m, v, grad, step, lr):
        _check(self.lib.ctf_cnn_adam(_ptr(params), _ptr(m), _ptr(v), _ptr(grad), params.numel(), step,
                                     ctypes.c_float(lr), self._s()))


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class Problem:
    """A problem on the HIP library: the workspace is a torch uint8 tensor on the device, inputs are
    float64 device tensors; every call forwards to the C-ABI of the same name."""

    def __init__(self, cfg, sigma_t, sigma_s, source, device="cuda", stream=None):
        import torch
        self.torch = torch
        self.cfg = cfg
        self.lib = load()
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        nb = workspace_bytes(cfg)
        self.workspace = torch.empty(nb + 256, dtype=torch.uint8, device=self.device)
        st = torch.as_tensor(sigma_t, dtype=torch.float64, device=self.device).contiguous()
        ss = torch.as_tensor(sigma_s, dtype=torch.float64, device=self.device).contiguous()
        src = torch.as_tensor(source, dtype=torch.float64, device=self.device).contiguous()
        G, N = cfg.ngroups, cfg.n
        if tuple(st.shape) != (G, N, N) or tuple(src.shape) != (G, N, N) or \
                tuple(ss.shape) != (cfg.scatter_order + 1, G, G, N, N):
            raise CtfError(CTF_EINVAL, "material / source shapes do not match the configuration")
        h = ctypes.c_void_p()
        _check(self.lib.ctf_create_problem(ctypes.byref(cfg), _ptr(st), _ptr(ss), _ptr(src),
                                           _ptr(self.workspace), nb + 256,
                                           ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self.handle = h
        self.levels = [self.level_info(l) for l in range(self.lib.ctf_num_levels(h))]

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            self.lib.ctf_destroy_problem(h)
            self.handle = None

    # -- sizes and setup data
    def level_info(self, level):
        d = LevelDesc()
        _check(self.lib.ctf_level_info(self.handle, level, ctypes.byref(d)))
        return d

    def shape(self, level=0):
        d = self.levels[level]
        return (self.cfg.ngroups, d.n_dir, d.n, d.n)

    def empty(self, level=0):
        return self.torch.empty(self.shape(level), dtype=self.torch.float64, device=self.device)

    def zeros(self, level=0):
        return self.torch.zeros(self.shape(level), dtype=self.torch.float64, device=self.device)

    def level_quadrature(self, level):
        import numpy as np
        nd = self.levels[level].n_dir
        mu, nu, w = np.zeros(nd), np.zeros(nd), np.zeros(nd)
        _check(self.lib.ctf_level_quadrature(self.handle, level, mu.ctypes.data, nu.ctypes.data,
                                             w.ctypes.data))
        return mu, nu, w

    def level_sigma_t(self, level):
        d = self.levels[level]
        out = self.torch.empty((self.cfg.ngroups, d.n, d.n), dtype=self.torch.float64, device=self.device)
        _check(self.lib.ctf_level_sigma_t(self.handle, level, _ptr(out)))
        return out

    # -- the hot path
    def apply_operator(self, psi, out, mode=OP_RESIDUAL):
        _check(self.lib.ctf_apply_operator(self.handle, _ptr(psi), _ptr(out), mode))
        return out

    def moments(self, psi, phi):
        _check(self.lib.ctf_moments(self.handle, _ptr(psi), _ptr(phi)))
        return phi

    def moments_f32(self, psi32, phi32, use_mfma=True):
        _check(self.lib.ctf_moments_f32(self.handle, _ptr(psi32), _ptr(phi32), int(use_mfma)))
        return phi32

    def freeze_k(self, psi, kx=None, ky=None):
        _check(self.lib.ctf_freeze_k(self.handle, _ptr(psi), _ptr(kx), _ptr(ky)))

    def smooth(self, level, kind, x, rhs, nsweeps):
        _check(self.lib.ctf_smooth(self.handle, level, kind, _ptr(x), _ptr(rhs), nsweeps))
        return x

    def restrict(self, level, fine, coarse):
        _check(self.lib.ctf_restrict(self.handle, level, _ptr(fine), _ptr(coarse)))
        return coarse

    def prolong(self, level, coarse, fine):
        _check(self.lib.ctf_prolong(self.handle, level, _ptr(coarse), _ptr(fine)))
        return fine

    def mg_cycle(self, psi, want_residual=False):
        r = ctypes.c_double(0.0)
        _check(self.lib.ctf_mg_cycle(self.handle, _ptr(psi), ctypes.byref(r) if want_residual else None))
        return r.value if want_residual else None

    def solve(self, psi, rtol, max_cycles, history_len=0):
        import numpy as np
        info = SolveInfo()
        hist = np.zeros(max(history_len, 1))
        if history_len:
            info.history = hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            info.history_len = history_len
        rc = _check(self.lib.ctf_solve(self.handle, _ptr(psi), rtol, max_cycles, ctypes.byref(info)),
                    allow_not_converged=True)
        checks = (info.outer_steps if self.cfg.precision != FP64 else info.cycles) + 1
        n = min(history_len, checks) if history_len else 0
        return {"converged": rc == CTF_OK, "cycles": info.cycles, "outer_steps": info.outer_steps,
                "rel_residual": info.rel_residual, "seconds": info.seconds,
                "history": hist[:n].copy() if history_len else None,
                "cnn_applied": info.cnn_applied, "cnn_rejected": info.cnn_rejected}

    def timing_enable(self, on=True, capacity=4096, classes=None):
        """Record HIP events around the launches of the named kernel classes (default: all)."""
        mask = 0
        for name in classes or ():
            mask |= 1 << TIMER_CLASSES.index(name)
        _check(self.lib.ctf_timing_enable(self.handle, int(on), capacity if on else 0, mask))

    def timing_read(self):
        """{class: (total_ms, launches, dropped)} of the recorded kernel launches."""
        out = {}
        for c, name in enumerate(TIMER_CLASSES):
            ms, n, dr = ctypes.c_double(), ctypes.c_int(), ctypes.c_int()
            _check(self.lib.ctf_timing_read(self.handle, c, ctypes.byref(ms), ctypes.byref(n),
                                            ctypes.byref(dr)))
            out[name] = (ms.value, n.value, dr.value)
        return out

    # -- launch shapes
    def set_launch_shape(self, strip_h, corr_block, pg_fused=0):
        _check(self.lib.ctf_set_launch_shape(self.handle, strip_h, corr_block, int(pg_fused)))

    def launch_shape(self):
        a, b, f = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(self.lib.ctf_get_launch_shape(self.handle, ctypes.byref(a), ctypes.byref(b), ctypes.byref(f)))
        return a.value, b.value, f.value

    def autotune(self, cache_path=None, force=False):
        a, b, f = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        path = cache_path.encode() if cache_path else None
        _check(self.lib.ctf_autotune(self.handle, path, int(force), ctypes.byref(a), ctypes.byref(b),
                                     ctypes.byref(f)))
        return a.value, b.value, f.value

    # -- learned coarse-grid correction
    def cnn_attach(self, params):
        _check(self.lib.ctf_cnn_attach(self.handle, _ptr(params)))

    def cnn_enable(self, on):
        _check(self.lib.ctf_cnn_enable(self.handle, int(on)))

    def cnn_grid(self):
        return self.levels[self.cfg.cnn_level].n

    def cnn_sample(self, psi, psi_star, features, target):
        sc = ctypes.c_double(0.0)
        _check(self.lib.ctf_cnn_sample(self.handle, _ptr(psi), _ptr(psi_star), _ptr(features), _ptr(target),
                                       ctypes.byref(sc)))
        return sc.value

    def norm(self, v):
        r = ctypes.c_double(0.0)
        _check(self.lib.ctf_norm(self.handle, _ptr(v), ctypes.byref(r)))
        return r.value
