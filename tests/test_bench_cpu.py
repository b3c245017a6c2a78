"""bench.py's host-side contract, without a GPU: one GPU only (N > 1 exits
with a message before touching the device), and the traffic figures it
reports come from the committed counter summary of the current kernel
sources (null otherwise)."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


@pytest.mark.parametrize("n", [2, 8])
def test_more_than_one_gpu_exits_with_a_message(n):
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)],
                         capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert res.returncode == 2
    assert "one GPU" in res.stderr and res.stdout == ""


def test_traffic_lookup_follows_the_kernel_sources(tmp_path, monkeypatch):
    import bench
    F = 8 * 512 * 512 * 16
    with open(os.path.join(ROOT, "profiles", "cg_dir_traffic_n4_512.json")) as f:
        t = json.load(f)
    assert set(t["bytes_per_launch_by_cw"]) == {"4", "8", "16"}
    if t["kernel_source_sha256_16"] == bench.kernel_source_hash():
        for cw in (4, 8, 16):
            b = bench.measured_traffic(F, cw)
            # at least the algorithmic 4.5F per launch (odd k 3F, even k 6F:
            # x is updated every other iteration), at most that plus the halo
            assert 4.5 * F <= b <= 1.4 * 4.5 * F
            par = t["by_parity"][str(cw)]
            assert 3 * F <= par["odd_k"] <= 1.4 * 3 * F
            assert 6 * F <= par["even_k"] <= 1.4 * 6 * F
    # a summary taken on other sources is not reported
    stale = dict(t, kernel_source_sha256_16="0" * 16)
    p = tmp_path / "traffic.json"
    p.write_text(json.dumps(stale))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(p))
    assert bench.measured_traffic(F, 8) is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.json"))
    assert bench.measured_traffic(F, 8) is None
