"""Host-side logic of bench.py (no GPU): the algorithmic cost model, the kernel names it looks up
in the rocprofv3 summaries, and the rule that a committed traffic measurement is reported only
while the kernel source it was taken on is unchanged."""
import hashlib
import os

import pytest

import bench


def test_algorithmic_cost_model():
    # the PG residual / sweep: 2b bytes (read psi, write the result) and the scope table's flop count
    assert bench.algorithmic_cost("pg32", 2, fused=True) == (8, 220)
    assert bench.algorithmic_cost("pg32", 1) == (8, 150)
    assert bench.algorithmic_cost("pg64", 3, fused=True) == (16, 290)
    assert bench.algorithmic_cost("pg32_update", 2) == (8, 220)
    assert bench.algorithmic_cost("moments", 2) == (4, 6)
    with pytest.raises(KeyError):
        bench.algorithmic_cost("no_such_class", 2)


def test_implementation_cost_model():
    # fused kernel stage by stage at p = 2 (W = 5 taps): A 2 x-sums + 2 y-passes, B 2 + 2, C 6 x-sums
    # plus 2 products per tap, D 6 y-passes, each pass one multiply-add (2 flops) per tap: 42 W;
    # k, emission and epilogue 57
    W = 5
    assert bench.implementation_flops("pg32", 2, fused=True) == 2 * W * (4 + 4 + 6 + 6) + 2 * W + 57 == 267
    assert bench.implementation_flops("pg32", 2, fused=False) == 32 * W + 23
    assert bench.implementation_flops("pgk32", 2) == 16 * W + 34
    # full-approximation sweeps also read their right-hand side; the float64 residual also writes
    # fl32(psi); the last float32 sweep reads and writes psi64
    assert bench.implementation_bytes("pg32", 2) == 12
    assert bench.implementation_bytes("pg64", 2) == 20
    assert bench.implementation_bytes("pg32_update", 2) == 28


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
    (tmp_path / "profiles" / "traffic_k_x_wl.txt").write_text(
        "# comment: 1\nscaled bytes per launch: 123456\nkernels.hip sha256: %s\n" % digest)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.read_traffic("k_x", "wl") == 123456.0
    assert bench.read_traffic("k_x", "other") is None
    kern.write_text("// kernel source changed since\n")
    assert bench.read_traffic("k_x", "wl") is None
    assert bench.read_traffic("k_missing", "wl") is None


@pytest.mark.parametrize("fname,dof", [("traffic_k_pg_fused_p2_f32_c1_mixed.txt", 256 * 256 * 512 * 2),
                                       ("traffic_k_pg_fused_p2_f32_c4_learned.txt", 1024 * 1024 * 512)])
def test_committed_traffic_summary_is_well_formed(fname, dof):
    path = os.path.join(os.path.dirname(bench.__file__), "profiles", fname)
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    assert vals["kernel"] == "k_pg_fused<2, 0, float, false>"
    fetch = float(vals["FETCH_SIZE KiB per dispatch"]) * 1024 * float(vals["FETCH scale"])
    write = float(vals["WRITE_SIZE KiB per dispatch"]) * 1024 * float(vals["WRITE scale"])
    assert abs(fetch + write - float(vals["scaled bytes per launch"])) < 1e-4 * (fetch + write)
    scaled = float(vals["scaled bytes per launch"])
    # the kernel reads x and its right-hand side and writes its output, 4 bytes each per DOF
    assert 1.0 <= scaled / (12 * dof) < 3.0


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
