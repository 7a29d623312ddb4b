"""Host-side parts of bench.py's JSON line: the kernel each class of the
roofline names for each operator layout the library reports, the rule that
committed HBM counters count only while the kernel sources they were taken
on are unchanged, and the refusal of more than one GPU."""
import json
import os
import subprocess
import sys
from types import SimpleNamespace

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_kernel_names_follow_the_reported_layouts():
    kron = SimpleNamespace(residual_layout=2, transfer_layout=2, resid_rows=4)
    k = bench.kernel_map(kron, 2, 5)
    assert k["residual"] == ("kron_resid<double, 2, false, 11, 4>", "bytes_spmv")
    assert k["restrict"][0] == "kron_xgrid<double, 2, false, 8>"
    assert k["prolong"][0] == "kron_xgrid<double, 2, true, 8>"
    assert k["upper"] == ("trisolve_upper<double>", "bytes_trisolve_u")
    stencil = SimpleNamespace(residual_layout=1, transfer_layout=1, resid_rows=1)
    s = bench.kernel_map(stencil, 3, 3)
    assert s["residual"][0] == "stencil_resid<double, 3, false, 7, 1>"
    assert s["restrict"][0] == "xgrid_spmv<double, 3, false>"
    csr = SimpleNamespace(residual_layout=0, transfer_layout=0, resid_rows=0)
    c = bench.kernel_map(csr, 2, 6)
    assert c["residual"][0] == "csr_kernel<double, G, 0>"
    assert c["restrict"][0] == "csr_kernel<double, G, 2>" and c["prolong"][0] == "csr_kernel<double, G, 3>"


def test_committed_counters_name_the_kernels_of_their_workloads():
    d = json.load(open(os.path.join(ROOT, "profiles", "traffic_counters.json")))
    assert d["calibration"]["fetch_factor"] > 1.0 and d["calibration"]["write_factor"] > 0.5
    for wl, (dim, deg) in {"2d-unit-square-p5-h1/1024": (2, 5), "3d-unit-cube-p3-h1/64": (3, 3)}.items():
        ks = d["workloads"][wl]["kernels"]
        for cls in ("residual", "lower", "upper", "restrict", "prolong"):
            k = ks[cls]
            assert k["kernel"].startswith("pmg::")
            assert k["bytes_per_launch"] > 0 and k["algorithmic_bytes"] > 0
            # real traffic is never below the bytes the operation must move
            assert k["bytes_per_launch"] >= 0.99 * k["algorithmic_bytes"], (wl, cls)
        assert ks["upper"]["kernel"] == "pmg::trisolve_upper<double>"


def test_traffic_only_for_the_sources_the_counters_were_taken_on(monkeypatch):
    d = json.load(open(os.path.join(ROOT, "profiles", "traffic_counters.json")))
    wl = "2d-unit-square-p5-h1/1024"
    monkeypatch.setattr(bench, "_kernel_source_hash", lambda: d["kernel_source_hash"])
    assert bench._traffic("upper", wl) == d["workloads"][wl]["kernels"]["upper"]["bytes_per_launch"]
    assert bench._traffic("upper", "no-such-workload") is None
    monkeypatch.setattr(bench, "_kernel_source_hash", lambda: "0" * 16)
    assert bench._traffic("upper", wl) is None


@pytest.mark.parametrize("env,argv", [({}, ["--gpus", "2"]), ({"WORLD_SIZE": "4"}, [])])
def test_more_than_one_gpu_is_refused(env, argv):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + argv, capture_output=True, text=True,
                       env={**os.environ, **env}, timeout=300)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""
