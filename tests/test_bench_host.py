"""bench.py's host-side contract, on the CPU: a request for several GPUs
exits with a message (the library measures one GPU), and the counter
summaries it reads parse and name the kernel and workload they describe."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_several_gpus_refused():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert out.returncode != 0
    assert "one GPU" in (out.stdout + out.stderr)


def test_counter_summaries_parse():
    for name, kernel, workload in (
            ("k_ipp_slab_uniform1024_lds.json", "k_ipp_slab<2, false, false>", "uniform1024"),
            ("k_ipp_slab_uniform1024_traffic.json", "k_ipp_slab<2, false, false>", "uniform1024"),
            ("k_ipp_slab3d_expansion3d_valu.json", "k_ipp_slab_persistent<3, false, true, false>",
             "expansion3d")):
        with open(os.path.join(ROOT, "profiles", name)) as fh:
            d = json.load(fh)
        assert d["kernel"] == kernel and d["workload"] == workload
        assert len(d["kernel_source_sha"]) == 16
