"""Host-side checks of bench.py that need no GPU: the single-GPU guard and the recorded HBM
traffic of the trailing update."""
import hashlib
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    # the guard runs before torch or the HIP library is imported, so this touches no device
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_records_belong_to_the_current_trailing_update_sources():
    """bench.py reports roofline.traffic only while the kernel's source file matches the one
    its counters were taken on; every committed record must be for the committed source."""
    import bench
    assert bench.TRAFFIC
    for (precision, workload, tiling), rec in bench.TRAFFIC.items():
        with open(bench.gemm_source(precision, tiling), "rb") as f:
            digest = hashlib.sha256(f.read()).hexdigest()
        assert rec["sha256"] == digest, ("the source of %s tiling %d changed after its FETCH_SIZE / WRITE_SIZE "
                                         "counters were taken: re-take them and update the record"
                                         % (precision, tiling))
        # measured HBM bytes cannot fall below the algorithmic minimum
        assert rec["bytes_per_launch"] / rec["alg_bytes_per_launch"] >= 1.0
    # wasted re-reads show up as a large ratio: the library's default split-mode tiling (19,
    # tiles in bands of eight rows) must stay close to the algorithmic bytes
    rec = bench.TRAFFIC[("split", "fcc4000", 19)]
    assert rec["bytes_per_launch"] / rec["alg_bytes_per_launch"] < 1.3
