"""Host-side checks of bench.py: the one-GPU contract and the traffic-summary lookup."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    """The benchmark measures one GPU; --gpus N > 1 (or a multi-rank launch) exits with status 2
    and says why, before touching a GPU."""
    for args, env in ((["--gpus", "2"], {}), (["--gpus", "8"], {}), ([], {"WORLD_SIZE": "2"})):
        r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + args,
                           env=dict(os.environ, **env), capture_output=True, text=True,
                           timeout=120)
        assert r.returncode == 2
        assert "one GPU only" in r.stderr
        assert r.stdout == ""


def test_traffic_summary_is_used_only_for_its_own_configuration():
    """The committed HBM-traffic summary is keyed to the kernel sources, box size and launch
    options: the default configuration finds it while the kernel sources are those it was
    measured on, any other configuration gets None."""
    import re

    sys.path.insert(0, ROOT)
    import bench

    if not os.path.exists(bench.TRAFFIC_SUMMARY):
        assert bench.measured_traffic(256, 32, 1, 1) is None
        return
    with open(bench.TRAFFIC_SUMMARY) as f:
        recorded = re.search(r"kernel_source_sha256: (\w+)", f.read()).group(1)
    t = bench.measured_traffic(256, 32, 1, 1)  # the default: runs of 32 tiles per XCD
    if recorded == bench.kernel_source_hash():
        assert t is not None and 1.0e9 < t < 4.0e9
    else:
        assert t is None
    for other in ((128, 32, 1, 1), (256, 8, 1, 1), (256, 0, 1, 1), (256, 32, 0, 1), (256, 32, 1, 0),
                  (256, 32, 1, 1, 0)):
        assert bench.measured_traffic(*other) is None
