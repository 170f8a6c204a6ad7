"""Host-side pieces of bench.py: the traffic table's lookup (every committed
figure is reachable while the kernels are built as they were measured:
source, device header and compile flags; unknown kernels read as None) and
the refusal of more than one GPU."""
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_traffic_lookup():
    b = _bench()
    sha = b.traffic_key()
    for cfg, table in b.TRAFFIC.items():
        for name, val in table.items():
            if name == "sha256":
                continue
            assert name in b.KERNELS, name
            got = b.kernel_traffic(cfg, name)
            if table["sha256"] == sha:
                assert got == val and isinstance(got, int) and got > 0, (cfg, name)
            else:
                assert got is None
    assert b.kernel_traffic("thick256_fp64", "no_such_kernel") is None
    assert b.kernel_traffic("no_such_config", "k_resid") is None


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr) or "1 GPU" in (r.stdout + r.stderr)
