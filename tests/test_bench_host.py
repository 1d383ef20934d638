"""Host-side logic of bench.py (CPU only): the one-GPU contract and the
algorithmic byte counts the roofline uses."""
import os
import subprocess
import sys
from types import SimpleNamespace

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_algorithmic_bytes_per_unit():
    """Ax: 7 reads + 1 write per local point in FP64 (Sec. 1), 32 B in FP32;
    FDM: input and output E-vectors, S and the eigenvalues per element, and
    the stored RAS weight E-vector at p <= 3 (computed from p = 4 on);
    gather-scatter: a read and a write per shared member."""
    p, E = 7, 32768
    L = SimpleNamespace(p=p, E=E, nmembers=9699328, nshared=4312737)
    n = E * (p + 1) ** 3
    assert bench.algorithmic_bytes("ax64", L) == 64 * n
    assert bench.algorithmic_bytes("ax32", L) == 32 * n
    assert bench.algorithmic_bytes("fdm", L) == E * (2 * 512 * 4 + 3 * 100 * 4 + 3 * 10 * 4)
    L3 = SimpleNamespace(p=3, E=E)
    assert bench.algorithmic_bytes("fdm", L3) == E * (3 * 64 * 4 + 3 * 36 * 4 + 3 * 6 * 4)
    assert bench.algorithmic_bytes("gs32", L) == 8 * 9699328
    assert bench.algorithmic_bytes("gs64", L) == 16 * 9699328
    assert bench.fdm_flops(L) == E * (12 * 10 ** 4 + 10 ** 3)
