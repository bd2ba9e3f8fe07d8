"""The library's host setup code (setup.cpp: ordinates, coarse ordinates, ConvFEM stencils) built
with g++ under AddressSanitizer and UndefinedBehaviorSanitizer, run, and checked against the
oracle: any memory error or undefined behaviour aborts the run; the values must match to 1e-13."""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

from oracle import convfem, quadrature as qd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def output():
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "setup_check")
        cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
               "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-D__HIP_PLATFORM_AMD__",
               "-I/opt/rocm/include", os.path.join(ROOT, "tests", "host", "setup_check.cpp"),
               os.path.join(ROOT, "paper_2301_09991_amd", "csrc", "setup.cpp"), "-o", exe]
        subprocess.run(cmd, check=True, capture_output=True, timeout=300)
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1:verify_asan_link_order=0")
        run = subprocess.run([exe], capture_output=True, text=True, timeout=120, env=env)
        assert run.returncode == 0, run.stderr[-2000:]
        assert "runtime error" not in run.stderr, run.stderr[-2000:]
        return run.stdout.splitlines()


def _blocks(lines):
    out, i = [], 0
    while i < len(lines):
        head = lines[i].split()
        if head[0] == "Q":
            na, faces, coarse, nd = map(int, head[1:])
            vals = np.array([[float(v) for v in lines[i + 1 + k].split()] for k in range(nd)])
            out.append(("Q", (na, faces, coarse), vals))
            i += 1 + nd
        else:
            p = int(head[1])
            vals = np.array([[float(v) for v in lines[i + 1 + k].split()] for k in range(2 * p + 1)])
            out.append(("S", p, vals))
            i += 2 * p + 2
    return out


def test_host_setup_under_sanitizers_matches_oracle(output):
    blocks = _blocks(output)
    assert len(blocks) == 3 * 2 * 2 + 4   # na 1, 2, 4 x full / half x fine / coarse; p = 1..4
    for kind, key, vals in blocks:
        if kind == "Q":
            na, faces, coarse = key
            q = qd.quadrature(na)
            if coarse:
                q = qd.coarsen(q)
            nd = len(vals)
            mu, nu, p = q["mu"][:nd], q["nu"][:nd], q["p"][:nd] * (2.0 if faces == 4 else 1.0)
            assert np.abs(vals[:, 0] - mu).max() < 1e-13
            assert np.abs(vals[:, 1] - nu).max() < 1e-13
            assert np.abs(vals[:, 2] - p).max() < 1e-13
        else:
            m, d, k = convfem.stencils_1d_float(key)
            assert np.abs(vals[:, 0] - m).max() < 1e-14
            assert np.abs(vals[:, 1] - d).max() < 1e-14
            assert np.abs(vals[:, 2] - k).max() < 1e-14
