"""The C-ABI library: it loads, exports every symbol include/ctf.h declares, and its host-only
setup (ordinates, ConvFEM stencils, configuration checks) agrees with the oracle.  CPU only: no
call here touches a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2301_09991_amd import ctf
from oracle import convfem, quadrature as qd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "ctf.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ctf_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(ctf.LIB_PATH)
    names = _declared()
    assert len(names) >= 20
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(ctf.EXPORTED) == names


@pytest.mark.parametrize("na", [1, 2, 4, 8, 16])
def test_host_quadrature_matches_oracle(na):
    mu, nu, w = ctf.quadrature(na)
    q = qd.quadrature(na)
    assert np.abs(mu - q["mu"]).max() < 1e-13
    assert np.abs(nu - q["nu"]).max() < 1e-13
    assert np.abs(w - q["p"]).max() < 1e-13


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_host_stencils_match_oracle(p):
    m, d, k = ctf.convfem_stencils(p)
    mo, do, ko = convfem.stencils_1d_float(p)
    assert np.abs(m - mo).max() < 1e-14
    assert np.abs(d - do).max() < 1e-14
    assert np.abs(k - ko).max() < 1e-13


def test_config_validation():
    with pytest.raises(ctf.CtfError):
        ctf.workspace_bytes(ctf.default_config(na=3))
    with pytest.raises(ctf.CtfError):
        ctf.workspace_bytes(ctf.default_config(p=5))
    with pytest.raises(ctf.CtfError):
        ctf.workspace_bytes(ctf.default_config(n=1))
    with pytest.raises(ctf.CtfError):
        ctf.workspace_bytes(ctf.default_config(n=32770))
    # planes stay below 2^29 bytes in float64 (the strip kernels address a plane with 32-bit offsets)
    with pytest.raises(ctf.CtfError):
        ctf.workspace_bytes(ctf.default_config(n=8194))
    assert ctf.workspace_bytes(ctf.default_config(n=8192, na=1)) > 8 * 8192 * 8192 * 8
    with pytest.raises(ctf.CtfError):
        ctf.workspace_bytes(ctf.default_config(n_jacobi=0))
    with pytest.raises(ctf.CtfError):
        ctf.convfem_stencils(0)
    # residual estimates: low needs p >= 2, high p <= 3, both the isotropic diffusivity
    pg = dict(discretisation=ctf.CONVFEM_PG, pg_isotropic=1)
    for bad in (dict(pg, p=1, pg_r_estimate=ctf.R_LOW), dict(pg, p=4, pg_r_estimate=ctf.R_HIGH),
                dict(pg, p=2, pg_r_estimate=3), dict(pg, p=2, pg_isotropic=0, pg_r_estimate=ctf.R_LOW)):
        with pytest.raises(ctf.CtfError):
            ctf.workspace_bytes(ctf.default_config(**bad))
    for good in (dict(pg, p=2, pg_r_estimate=ctf.R_LOW), dict(pg, p=4, pg_r_estimate=ctf.R_LOW),
                 dict(pg, p=1, pg_r_estimate=ctf.R_HIGH), dict(pg, p=3, pg_r_estimate=ctf.R_HIGH)):
        assert ctf.workspace_bytes(ctf.default_config(**good)) > 0
    small = ctf.workspace_bytes(ctf.default_config(n=32))
    big = ctf.workspace_bytes(ctf.default_config(n=64))
    assert 3.5 * small < big < 4.5 * small
    mixed = ctf.workspace_bytes(ctf.default_config(n=64, precision=ctf.FP32_IR))
    assert mixed > big


def test_default_config_is_the_papers():
    c = ctf.default_config()
    assert c.beta_pg == 3.0 and c.alpha_r == 3.0 and c.eps_k == 1e-3
    assert c.n_jacobi == 2 and c.bc[:] == [ctf.VACUUM] * 4


def test_null_and_empty_arguments_are_refused():
    """Every entry point checks its arguments before it touches a device: null handles and
    buffers, empty batches and negative counts return CTF_EINVAL with a message."""
    lib = ctf.load()
    null = ctypes.c_void_p(0)
    info = ctf.SolveInfo()
    one = (ctypes.c_void_p * 1)(0)
    calls = [
        lambda: lib.ctf_apply_operator(null, null, null, ctf.OP_RESIDUAL),
        lambda: lib.ctf_mg_cycle(null, null, None),
        lambda: lib.ctf_solve(null, null, 1e-6, 10, ctypes.byref(info)),
        lambda: lib.ctf_smooth(null, 0, 0, null, null, 1),
        lambda: lib.ctf_moments(null, null, null),
        lambda: lib.ctf_restrict(null, 0, null, null),
        lambda: lib.ctf_solve_batch(one, 0, one, 1e-6, 10, 1, None),
        lambda: lib.ctf_solve_batch(None, 1, one, 1e-6, 10, 1, None),
        lambda: lib.ctf_solve_batch_persistent(one, 0, one, 1e-6, 10, 0, null, 0, None),
        lambda: lib.ctf_set_launch_shape(null, 128, 256, 1),
    ]
    for call in calls:
        assert call() == ctf.CTF_EINVAL
        assert lib.ctf_last_error().decode()
    assert lib.ctf_solve_batch_persistent_bytes(one, 0, 0) == 0
