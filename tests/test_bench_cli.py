"""bench.py's command line on the CPU: it measures one GPU only, so a request
for several exits with status 2 and says why, before touching a device."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_several_gpus_are_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def test_several_ranks_are_refused():
    env = dict(os.environ, WORLD_SIZE="2")
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr


def test_committed_counters_match_the_sources():
    """The committed counter summaries were taken at the current kernel and
    BVH-builder sources, so the bench line carries measured VALU work and HBM
    traffic; after a change to those sources the profiles must be taken again
    (until then the bench reports them as null)."""
    sys.path.insert(0, ROOT)
    import bench
    for workload in ("apartment", "apartment_disney", "office_floor"):
        for kernel in ("colour", "grad_forward", "adjoint_replay"):
            c = bench.measured_counters(kernel, workload)
            assert {"valu_insts_per_launch", "lane_util", "hbm_bytes_per_launch"} <= set(c), (
                "profiles/ holds no counters of %s (%s) for kernel sources %s" % (
                    kernel, workload, bench.kernel_source_hash()))
            assert 0.0 < c["lane_util"] <= 1.0 and c["valu_insts_per_launch"] > 0 and c["hbm_bytes_per_launch"] > 0
