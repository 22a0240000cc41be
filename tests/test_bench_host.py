"""Host logic of bench.py (CPU only): the one-GPU guard and the use of the
committed HBM-traffic record."""
import argparse
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, cwd=ROOT, timeout=120)
    assert res.returncode == 2
    assert "one GPU" in res.stderr


def test_traffic_record_applies_to_its_workload_only():
    sys.path.insert(0, ROOT)
    import bench
    base = dict(nel=32, p=3, scheme="compact", eta_ip=0.0, integrator="rk4")
    rec_ok = bench.measured_traffic(argparse.Namespace(**base), "fp32")
    # a record taken on other kernel sources is not used (traffic reported as
    # null); one taken on the current sources is at least the algorithmic
    # 80 B per solution point of the 32^3 p = 3 workload
    with open(os.path.join(ROOT, "profiles", "rhs_traffic_tgv32p3.json")) as f:
        stale = bench.sources_sha256() != json.load(f)["sources_sha256"]
    assert (rec_ok is None) if stale else (rec_ok is not None and 1.68e8 < rec_ok < 2e9)
    for change in (dict(nel=64), dict(p=5), dict(scheme="br1"), dict(eta_ip=0.1), dict(integrator="ssprk54")):
        args = argparse.Namespace(**{**base, **change})
        assert bench.measured_traffic(args, "fp32") is None, change


def test_closure_record_shows_the_gain():
    """The committed 64^3 -> 16^3 closure record(s): on each held-out seed
    the corrected coarse run's KE and enstrophy errors are below the plain
    coarse run's, and the corrected run is faster than the fine run."""
    sys.path.insert(0, ROOT)
    import bench
    recs = bench.closure_record()
    assert recs, "no closure record under profiles/"
    for r in recs:
        assert r["test_seed"] >= 8 and r["target"] == "interval"
        assert r["ke_err"]["closure"] < r["ke_err"]["plain"]
        assert r["ens_err"]["closure"] < r["ens_err"]["plain"]
        assert r["wall_s"]["closure"] < r["wall_s"]["fine"] / 10
