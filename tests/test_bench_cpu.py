"""bench.py's contract pieces that run without a GPU: more than one GPU is
refused with a message and exit status 2, before any device is touched; the
algorithmic byte counts follow the kernels' compulsory traffic."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout == ""


def test_algorithmic_bytes():
    import bench

    n, nnz, r = 1000, 8000, 16
    # CSR (row_ptr + int32 index + value), diagonal, X read once, product written
    assert bench.spmm_bytes(n, nnz, r, "bf16") == (n + 1) * 4 + nnz * 8 + n * 4 + n * r * 2 + n * r * 4
    assert bench.spmm_bytes(n, nnz, r, "f64") == (n + 1) * 4 + nnz * 12 + n * 8 + n * r * 8 + n * r * 8
    # objective/gradient: CSR, diagonal, R read, G written, y, b read and A(RR^T) written
    assert bench.objgrad_bytes(n, nnz, r, "f32") == (n + 1) * 4 + nnz * 8 + n * 4 + 2 * n * r * 4 + 3 * n * 8
