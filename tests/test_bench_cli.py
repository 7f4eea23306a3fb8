"""bench.py's command line, checked without a GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_algorithmic_byte_model():
    sys.path.insert(0, ROOT)
    import bench
    n, nnz, w = 2_097_152, 55_742_968, 27
    # CRS: values + columns + row pointers + x + y
    assert bench.spmv_bytes("crs", n, nnz, w, 8, 8) == 12 * nnz + 4 * (n + 1) + 16 * n == 710_858_660
    # ELL-Row counts the padded slots
    assert bench.spmv_bytes("ell_row", n, nnz, w, 8, 8) == 12 * n * w + 16 * n == 713_031_680
    assert bench.transform_bytes("ell_row", n, nnz, w, 8) == 12 * nnz + 4 * (n + 1) + 12 * n * w
    assert bench.spmv_bytes("coo_row", n, nnz, w, 2, 4) == 10 * nnz + 8 * n
