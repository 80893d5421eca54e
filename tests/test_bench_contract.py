"""bench.py's output contract: one GPU only; the oracle baseline record;
the committed HBM and SQ counter records still match the kernel sources
they were taken on (else the bench would report traffic and the VALU issue
fraction as null); and, on the GPU,
one JSON line carrying every field of the contract."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_records_match_the_kernel_sources():
    for precs, rec, src in ((("fp64", "mixed"), bench.TRAFFIC_FILE, bench.KERNEL_SRC),
                            (("mixed", "fp64"), bench.TRAFFIC3_FILE, bench.KERNEL3_SRC)):
        for prec in precs:
            t = bench.measured_traffic(prec, rec, src)
            assert t is not None and t > 0, (rec, prec)


def test_issue_record_matches_the_kernel_source():
    """The committed SQ counter record (VALU instructions per launch of the
    headline particle kernel) was taken on the current kernel source."""
    for prec in ("fp64", "mixed"):
        v = bench.measured_valu(prec)
        assert v is not None and v > 0, prec


def test_traffic_is_null_for_another_source(tmp_path):
    other = tmp_path / "k.hip"
    other.write_text("// not the kernel the counters were taken on\n")
    assert bench.measured_traffic("mixed", bench.TRAFFIC_FILE, str(other)) is None


def test_counter_records_apply_only_at_their_launch_shape():
    """The committed counter records state the tile, scan width and exit
    mode they were taken at; a leg run at another shape gets no traffic or
    VALU figure."""
    for precs, rec in ((("fp64", "mixed"), bench.TRAFFIC_FILE), (("fp64", "mixed"), bench.PAIR_TRAFFIC_FILE)):
        for prec in precs:
            leg = json.load(open(rec))[prec]
            t, s = leg["tile"], leg["scan"]
            assert bench.measured_traffic(prec, rec, tile=t, scan=s) == leg["hbm_bytes_per_launch"]
            other = 512 if t != 512 else 768
            assert bench.measured_traffic(prec, rec, tile=other, scan=s) is None
            assert bench.measured_traffic(prec, rec, tile=t, scan=64 if s != 64 else 8) is None
    leg = json.load(open(bench.TRAFFIC_FILE))["mixed"]
    assert bench.measured_traffic("mixed", bench.TRAFFIC_FILE, tile=leg["tile"], scan=leg["scan"],
                                  defer=1 - leg["defer_exits"]) is None
    leg = json.load(open(bench.ISSUE_FILE))["fp64"]
    assert bench.measured_valu("fp64", tile=leg["tile"], scan=leg["scan"]) == leg["valu_per_launch"]
    assert bench.measured_valu("fp64", tile=leg["tile"] - 256, scan=leg["scan"]) is None


def test_cpu_baseline_record(oracle_lib):
    from paper_1707_04333_amd import inputs as I
    w = I.large_run(n_side=40, n_particles=5000, precision="fp64")
    cb = bench.cpu_baseline(w, "hc", steps=2)
    assert cb["kind"] == "oracle" and cb["unit"] == "particle-steps/s"
    assert cb["cores"] == bench.oracle_threads() >= 1
    for k in ("cpu_model", "os_cpu_count", "affinity_cpus", "OMP_NUM_THREADS"):
        assert k in cb["host"], k
    assert cb["value"] > 0 and "all 5000 particles" in cb["sample"] and "2 FP64 steps" in cb["sample"]


@pytest.mark.gpu
def test_bench_json_line():
    r = subprocess.run([sys.executable, "bench.py", "--workload", "pair", "--pairs", "50000",
                        "--steps", "20", "--warmup", "5", "--no-batched", "--no-autotune",
                        "--no-cpu", "--no-mixed"], cwd=ROOT, capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = r.stdout.strip().splitlines()
    assert len(lines) == 1
    out = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
              "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config",
              "roofline"):
        assert k in out, k
    assert out["n_gpus"] == 1 and out["steps"] == 20 and out["warmup"] == 5
    assert out["config"]["workload"] == "pair_plasma_bernstein" and out["value"] > 0
    assert out["dtype"] == "f64" and out["sorts_in_timed_steps"] >= 1
    rl = out["roofline"]
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in rl, k
    assert rl["bound"] == "hbm" and rl["unit"] == "GB/s" and rl["peak"] == 8000.0
    assert rl["traffic"] is None  # the counters were taken on the default size only
    assert abs(rl["frac"] - rl["achieved"] / rl["peak"]) < 1e-12
