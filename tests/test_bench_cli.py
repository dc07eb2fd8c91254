"""bench.py's command line on a host without a GPU: the one-GPU rule and the
side-measurement filters are checked before any device is touched."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=120)


def test_more_than_one_gpu_is_refused():
    r = _bench("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_unknown_side_measurement_is_refused():
    for flag, val in (("--extras", "bogus"), ("--learned-patterns", "lognormal,bogus"),
                      ("--learned-calls", "bogus"), ("--kv-patterns", "bogus"),
                      ("--seg-workloads", "bogus")):
        r = _bench(flag, val)
        assert r.returncode == 2, (flag, r.stderr)
        assert "unknown name" in r.stderr
