"""Host-side pieces of bench.py (no GPU): the one-GPU guard, the committed traffic
records it reports, and its reading of the finite-difference fixture."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, "tests", "golden"))

import bench  # noqa: E402
import c4_reference as REF  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_records_match_the_current_sources():
    """Every record the benchmark reports was taken on the kernels' current sources, and its
    measured bytes are within 2% of the algorithmic bytes of one launch."""
    for rec, key, bpn, nodes in [("collide_traffic_re5200_1536x128x384.json", "c3:f32", 152, 1536 * 128 * 384),
                                 ("collide_traffic_re5200_1536x256x384.json", "c5:f32", 152, 1536 * 256 * 384),
                                 ("collide_traffic_re1000_768x64x192.json", "c2:f32", 152, 768 * 64 * 192),
                                 ("collide_traffic_re1000_768x64x192.json", "c2:f16dev", 76, 768 * 64 * 192),
                                 ("adjoint_traffic_256x64x64.json", "c4:adjoint", 228, 256 * 64 * 64),
                                 ("adjoint_traffic_512x64x128.json", "c5a:adjoint:f16ref", 190, 512 * 64 * 128),
                                 ("adjoint_traffic_512x64x128.json", "c5a:adjoint:f16dev", 190, 512 * 64 * 128)]:
        t = bench.measured_traffic(rec, key)
        assert t is not None, (rec, key)
        assert abs(t / (bpn * nodes) - 1) < 0.02, (rec, key, t / (bpn * nodes))
    assert bench.measured_traffic("collide_traffic_re5200_1536x128x384.json", "no-such-leg") is None


def test_fd_fixture_reading_matches_the_reference_script():
    names, fd, L0 = bench.read_fd_fixture()
    n2, fd2, L02 = REF.read_fd()
    assert names == n2 and np.array_equal(fd, fd2) and L0 == L02
    assert names == ["s%d" % b for b in REF.FD_BINS] + ["cs"]
