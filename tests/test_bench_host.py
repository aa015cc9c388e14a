"""Host-side logic of bench.py (no GPU): the one-GPU contract and the stored
HBM-traffic figures of the dominant kernel."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, HERE)

import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    res = subprocess.run([sys.executable, os.path.join(HERE, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120)
    assert res.returncode != 0
    assert "one GPU" in res.stderr


def test_stored_sweep_traffic_is_calibrated_and_above_the_algorithmic_bytes():
    """The counters are stored with a hash of the kernel sources: either they
    match the sources (then the calibrated bytes of both sweep kinds lie
    between their algorithmic bytes and 1.5 times that), or the bench
    reports null."""
    t = bench.TRAFFIC
    assert t["cal_fetch"] > 0 and t["cal_write"] > 0
    # FETCH_SIZE counts about half the bytes a copy reads, WRITE_SIZE all it writes
    kib = bench.CAL_BYTES / 1024.0
    assert 0.4 < t["cal_fetch"] / kib < 0.6
    assert 0.9 < t["cal_write"] / kib < 1.1
    got = bench.sweep_traffic_bytes()
    if got is None:
        return
    # algorithmic bytes of one FP32 sweep at 512^2, k = 4: packed maps, face-block
    # inverse triangles, three trace vectors; the r.z sweep also reads r (FP64)
    nel, nface, nlam = 512 * 512, 2 * 512 * 511, 2 * 512 * 511 * 5
    alg = (nel * 210 + nface * 15 + 3 * nlam) * 4
    assert alg <= got["plain"] <= 1.5 * alg
    assert alg + 8 * nlam <= got["rz"] <= 1.5 * (alg + 8 * nlam)
