"""Host-side checks of bench.py (no GPU): the one-GPU contract and the JSON
fields it derives without running a kernel."""
import importlib.util
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_peaks_and_chamfer_roofline_constants():
    b = _bench()
    assert b.FP32_PEAK == 157.3e12 and b.FP64_PEAK == 78.6e12
    # FP32 lane operations per second: 256 CUs x 128 lanes x 2.4 GHz
    assert abs(b.ALU_LANES - 256 * 128 * 2.4e9) / b.ALU_LANES < 1e-3
    assert b.CHAMFER_OPS_PER_PAIR == 5


def test_traffic_summary_parses():
    b = _bench()
    v = b.traffic_from_profile()
    # None only when the FP32 pass sources changed since the counters were taken
    assert v is None or 1e8 < v < 1e10


def test_method_flop_counts():
    """The roofline counts the method's own work: 30 FLOP per placement and 8 per
    crank rotation, whatever the precision and its bookkeeping."""
    b = _bench()
    assert b.FLOP_DYAD == 30 and b.FLOP_TIP == 8
