"""Host-side contracts (CPU only): the binding refuses to run without the HIP library
(there is no CPU fallback), and the benchmark measures one GPU only."""
import os
import subprocess
import sys

import pytest

from paper_2401_08586_amd import nnps

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_binding_raises_without_the_library(monkeypatch, tmp_path):
    monkeypatch.setattr(nnps, "LIB_PATH", str(tmp_path / "libnnps.so"))
    monkeypatch.setattr(nnps, "_lib", None)
    with pytest.raises(ImportError):
        nnps.load()


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
