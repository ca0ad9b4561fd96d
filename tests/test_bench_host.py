"""Host-side checks of bench.py's contract: one GPU only (a request for more
exits with a message and a nonzero status before touching a GPU), and the
counter-traffic helpers."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr and r.stdout.strip() == ""


def test_short_kernel_names():
    assert bench._short_kernel("void ttx::k_moved<float, false, 64, 64, 4, 4, false>(ttx::TileArgs<float, float>)") == \
        "k_moved<float, false, 64, 64, 4, 4, false>"
    assert bench._short_kernel("ttx_jit_moved_float_b_64x64_20ec9384") == "ttx_jit_moved_float_b_64x64_20ec9384"


def test_traffic_table_is_keyed_by_the_current_sources():
    """profiles/traffic_counters.json holds the hash of the kernel sources it
    was measured with; bench.py reports counter traffic only while they match."""
    import pytest
    with open(os.path.join(ROOT, "profiles", "traffic_counters.json")) as f:
        tr = json.load(f)
    if tr["source_hash"] != bench.kernel_source_hash():
        pytest.skip("counters predate the current kernel sources (bench.py reports traffic as null)")
    assert 1.9 < tr["scale"]["FETCH_SIZE"] < 2.1 and 0.95 < tr["scale"]["WRITE_SIZE"] < 1.05
    for name, k in tr["kernels"].items():
        assert abs(k["traffic_bytes"] - k["fetch_bytes"] - k["write_bytes"]) <= 1, name   # each rounded
