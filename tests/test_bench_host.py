"""Host logic of bench.py that needs no GPU: the one-GPU guard, the stored HBM-traffic ratio (reported only for
the kernel and workload it was measured on, and only while that kernel's sources are unchanged), and the
library profile names it maps to source files."""
import importlib.util
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_host_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def test_profile_names_map_to_their_sources():
    b = _bench()
    assert b._base_name("k_brick<k_bl_adjoint_step>1") == "k_brick<k_bl_adjoint_step>"
    assert b._base_name("k_axis0[4F0P]") == "k_axis0"
    for name, (_, files) in b.KERNEL_SOURCES.items():
        for f in files:
            assert os.path.exists(os.path.join(ROOT, "paper_2006_06823_amd", "csrc", f)), (name, f)


def test_stored_traffic_only_for_its_kernel_workload_and_sources(tmp_path):
    b = _bench()
    kernel = "k_brick<k_bl_adjoint_step>1"
    digest = b._source_digest(b.KERNEL_SOURCES["k_brick<k_bl_adjoint_step>"][1])
    table = {"workload": [128, 128, 128, 32, 32, 32, 1], "fetch_scale": 2.0, "write_scale": 1.0,
             "kernels": {kernel: {"traffic_over_algorithmic": 1.25, "source_digest": digest}}}
    path = tmp_path / "traffic.json"
    path.write_text(json.dumps(table))
    b.TRAFFIC_FILE = str(path)
    N, K = (128, 128, 128), (32, 32, 32)
    t, note = b.stored_traffic(kernel, N, K, 1, 1000.0)
    assert t == 1250 and "stored ratio 1.25" in note
    assert b.stored_traffic(kernel, N, K, 3, 1000.0)[0] is None            # another variant
    assert b.stored_traffic(kernel, (96, 96, 96), K, 1, 1000.0)[0] is None  # another grid
    assert b.stored_traffic("k_brick<k_interp>1", N, K, 1, 1000.0)[0] is None  # another kernel
    table["kernels"][kernel]["source_digest"] = "0" * 16                  # sources changed since
    path.write_text(json.dumps(table))
    t, note = b.stored_traffic(kernel, N, K, 1, 1000.0)
    assert t is None and "changed" in note
    b.TRAFFIC_FILE = str(tmp_path / "missing.json")
    assert b.stored_traffic(kernel, N, K, 1, 1000.0)[0] is None

