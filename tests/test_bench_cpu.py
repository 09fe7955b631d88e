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
    assert len(files) >= 1
    for f in files:
        b = bench.parse_traffic(f)
        assert b is not None and b > 1e8, f
        txt = open(f).read()
        stated = float(txt.split("Scaled traffic per launch:")[1].split("GB")[0])
        assert abs(b / 1e9 - stated) < 0.006, f
        assert "rocprofv3 --pmc FETCH_SIZE" in txt and "rocprofv3 --pmc WRITE_SIZE" in txt, f
    assert bench.read_traffic(os.path.join(ROOT, "profiles", "no_such_kernel_pmc.txt")) is None


def test_counter_traffic_is_dropped_once_the_kernel_changed(tmp_path):
    src = "paper_2405_10197_amd/csrc/sigma_kernels.hip"
    body = ("FETCH_SIZE_KiB: 1000\nWRITE_SIZE_KiB: 500\nfetch_scale: 2.0\nwrite_scale: 1.0\n"
            "kernel_sources: %s\nkernel_sources_sha256: %s\n")
    cur = tmp_path / "cur_pmc.txt"
    cur.write_text(body % (src, bench.sources_sha256([src])))
    assert bench.read_traffic(str(cur)) == 1024.0 * (1000 * 2.0 + 500 * 1.0)
    old = tmp_path / "old_pmc.txt"
    old.write_text(body % (src, "0" * 64))
    assert bench.read_traffic(str(old)) is None
    bare = tmp_path / "bare_pmc.txt"
    bare.write_text(body.split("kernel_sources")[0])
    assert bench.read_traffic(str(bare)) is None and bench.parse_traffic(str(bare)) is not None


def test_oracle_work_per_sigma():
    # CAS(12,12): 853,776 determinants x 1819 connected determinants each
    assert bench.elements_per_sigma(12, 6, 6) == 853776 * 1819
    assert bench.elements_per_sigma(16, 8, 8) == 12870 ** 2 * (1 + 2 * 64 + 2 * 784 + 64 * 64)
    # brute force on a tiny space: pairs of determinants differing by at most
    # two substitutions with the spin counts kept
    import itertools
    n, na, nb = 5, 2, 2
    dets = [(a, b) for a in itertools.combinations(range(n), na) for b in itertools.combinations(range(n), nb)]
    cnt = 0
    for (a1, b1) in dets:
        for (a2, b2) in dets:
            if len(set(a1) - set(a2)) + len(set(b1) - set(b2)) <= 2:
                cnt += 1
    assert bench.elements_per_sigma(n, na, nb) == cnt


def test_cpu_leg_reports_its_tiers():
    out = bench.cpu_leg(0.5)
    assert out["cores"] >= 1 and set(out["tiers"]) == {"T0_cas6", "T0_cas8", "T2_cas12"}
    t2 = out["tiers"]["T2_cas12"]
    assert t2["rows_done"] > 0 and out["t_sigma12"] > 0


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
