"""Host-side checks of bench.py: the one-GPU rule, the CPU-baseline record, the
workload table and the traffic record read from the committed profile."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_cpu_baseline_record():
    import bench
    rec = bench.cpu_baseline("cfg1", 2, 1)
    assert set(rec) == {"value", "unit", "cores", "kind", "sample"}
    assert rec["kind"] == "oracle" and rec["unit"] == "qpwf-steps/s"
    assert rec["value"] > 0 and rec["cores"] >= 1
    assert "2 of the workload's qpwfs" in rec["sample"]


@pytest.mark.parametrize("name, shape, ncomp, prec", [
    ("cfg1", (8, 8, 8), 2, 0), ("cfg2", (32, 32, 32), 2, 0), ("cfg2_fp32", (32, 32, 32), 2, 1),
    ("cfg3", (48, 48, 48), 2, 1), ("cfg4", (64, 64, 64), 4, 2), ("cfg4_fp32", (64, 64, 64), 4, 1)])
def test_workload_table(name, shape, ncomp, prec):
    import bench
    w = bench.make_workload(name, M=4)
    lat = w.lattice
    assert (lat.nx, lat.ny, lat.nz) == shape
    assert w.functional.ncomp == ncomp and w.functional.precision == prec and w.M == 4


def test_traffic_record_from_profile():
    """The bench reads per-qpwf HBM bytes of the FP64 32^3 ABM kernels (the plane kernel
    with the z-term inside) from the committed PMC summary, or None when the kernel
    sources changed since the counters were taken."""
    import bench
    rec = bench.measured_traffic()
    path = os.path.join(ROOT, "profiles", bench.TRAFFIC_FILES["cfg2"])
    line = [l for l in open(path) if l.startswith("TRAFFIC_JSON")][0]
    stored = json.loads(line.split(" ", 1)[1])
    # one 32^3 FP64 two-component state array per qpwf is 1 MiB: 9 of them in phase 1,
    # 5 in phase 2 (plus the density partial sums and the column reads that miss L2)
    mib = 1 << 20
    assert 9 * mib <= stored["abm1_bytes_per_qpwf"] < 9.6 * mib
    assert 5 * mib <= stored["abm2_bytes_per_qpwf"] < 5.4 * mib
    assert "kz_bytes_per_qpwf" not in stored     # no z-axis kernel in the ABM step
    assert rec is None or rec == stored


def test_every_traffic_file_holds_a_record():
    """Each form's PMC summary named in bench.TRAFFIC_FILES exists, gives its rocprofv3
    commands and one TRAFFIC_JSON line with per-qpwf bytes for every kernel it covers."""
    import bench
    for key, name in bench.TRAFFIC_FILES.items():
        path = os.path.join(ROOT, "profiles", name)
        text = open(path).read()
        assert "rocprofv3 --pmc FETCH_SIZE" in text and "rocprofv3 --pmc WRITE_SIZE" in text, name
        lines = [l for l in text.splitlines() if l.startswith("TRAFFIC_JSON ")]
        assert len(lines) == 1, name
        rec = json.loads(lines[0].split(" ", 1)[1])
        assert len(rec["source_hash"]) == 16
        vals = [v for k, v in rec.items() if k != "source_hash"]
        assert vals and all(v > 0 for v in vals), name
