"""Host-side logic of bench.py (no GPU): the algorithmic cost model, the kernel names it looks up
in the rocprofv3 summaries, and the rule that a committed traffic measurement is reported only
while the kernel source it was taken on is unchanged."""
import hashlib
import os

import pytest

import bench


def test_algorithmic_cost_model():
    # p = 2: W = 5 taps; fused residual reads u, rhs and writes out (12 B) with 32W + 23 + 16W + 34 flops
    b, f = bench.algorithmic_cost("pg32", 2, fused=True)
    assert (b, f) == (12, 32 * 5 + 23 + 16 * 5 + 34) == (12, 297)
    assert bench.algorithmic_cost("pg32", 2, fused=False) == (20, 32 * 5 + 23)
    assert bench.algorithmic_cost("pg32_update", 2, fused=True)[0] == 12 + 16   # psi64 read and written
    assert bench.algorithmic_cost("pg64", 2, fused=True)[0] == 8 + 4 + 4   # psi read; residual and fl32(psi) written
    assert bench.algorithmic_cost("moments", 2) == (4, 6)
    with pytest.raises(KeyError):
        bench.algorithmic_cost("no_such_class", 2)


def test_kernel_symbols_match_the_profiler_names():
    assert bench.kernel_symbol("pg32", 2, True) == ("k_pg_fused<2, 0, float, false>", "k_pg_fused_p2_f32")
    assert bench.kernel_symbol("pg64", 3, True) == ("k_pg_fused<3, 0, double, false>", "k_pg_fused_p3_f64")
    assert bench.kernel_symbol("pg32", 2, False) == ("k_pg_stream<2, float>", "k_pg_stream_p2_f32")
    assert bench.kernel_symbol("pgk64", 3, False) == ("k_pg_diffusivity<3, 0, double>", "k_pg_diffusivity_p3_f64")
    assert bench.kernel_symbol("corr0", 2, True) == ("corr0", "corr0")


def test_traffic_is_reported_only_for_the_measured_source(tmp_path, monkeypatch):
    src = tmp_path / "paper_2301_09991_amd" / "csrc"
    src.mkdir(parents=True)
    (tmp_path / "profiles").mkdir()
    kern = src / "kernels.hip"
    kern.write_text("// kernel source as measured\n")
    digest = hashlib.sha256(kern.read_bytes()).hexdigest()
    (tmp_path / "profiles" / "traffic_k_x.txt").write_text(
        "# comment: 1\nscaled bytes per launch: 123456\nkernels.hip sha256: %s\n" % digest)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.read_traffic("k_x") == 123456.0
    kern.write_text("// kernel source changed since\n")
    assert bench.read_traffic("k_x") is None
    assert bench.read_traffic("k_missing") is None


def test_committed_traffic_summary_is_well_formed():
    path = os.path.join(os.path.dirname(bench.__file__), "profiles", "traffic_k_pg_fused_p2_f32.txt")
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    assert vals["kernel"] == "k_pg_fused<2, 0, float, false>"
    scaled, alg = float(vals["scaled bytes per launch"]), float(vals["algorithmic bytes per launch"])
    assert alg == 12 * 256 * 256 * 512 * 2
    assert 1.0 <= scaled / alg < 1.5   # measured HBM bytes cannot undercut the arrays the kernel must move


def test_more_than_one_gpu_is_refused_with_a_message():
    """bench.py --gpus N with N > 1 exits (status 2) with a message, before touching a GPU."""
    import json
    import subprocess
    import sys
    root = os.path.dirname(bench.__file__)
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]
