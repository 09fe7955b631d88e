"""Host logic of bench.py that needs no GPU: the time-to-threshold rule, the
counter summaries it reads for the roofline's traffic, and the one-GPU
guard."""
import glob
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_time_to_threshold_takes_the_first_iteration_that_stays_within():
    eref = np.array([-1.0, -0.5])
    hist_e = np.array([[-0.9, -0.4], [-1.0 + 1e-9, -0.5], [-1.0 + 2e-8, -0.5], [-1.0, -0.5 - 5e-9],
                       [-1.0, -0.5]])
    hist_t = np.array([10.0, 20.0, 30.0, 40.0, 50.0])
    t, i = bench.time_to_threshold(hist_e, hist_t, eref)
    # iteration 1 is within 1e-8 but iteration 2 leaves it again
    assert i == 3 and t == 0.04
    t, i = bench.time_to_threshold(hist_e[:3], hist_t[:3], eref)
    assert i == -1 and np.isnan(t)


def test_every_counter_summary_parses_to_its_stated_traffic():
    files = sorted(glob.glob(os.path.join(ROOT, "profiles", "*_pmc.txt")))
    assert len(files) >= 4
    for f in files:
        b = bench.read_traffic(f)
        assert b is not None and b > 1e9, f
        txt = open(f).read()
        stated = float(txt.split("Scaled traffic per launch:")[1].split("GB")[0])
        assert abs(b / 1e9 - stated) < 0.006, f
        assert "rocprofv3 --pmc FETCH_SIZE" in txt and "rocprofv3 --pmc WRITE_SIZE" in txt, f
    assert bench.read_traffic(os.path.join(ROOT, "profiles", "no_such_kernel_pmc.txt")) is None


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
