"""Host-side checks of bench.py's command line (no GPU needed)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], cwd=ROOT,
                          capture_output=True, text=True, timeout=120)


def test_bench_refuses_more_than_one_gpu():
    """A product is one dependent chain of swaps: the benchmark measures one
    GPU and says so, before touching any device, when asked for more."""
    for n in ("2", "8"):
        p = _bench("--gpus", n)
        assert p.returncode == 2
        assert "one GPU" in p.stderr and p.stdout == ""


def test_bench_options_parse():
    p = _bench("--help")
    assert p.returncode == 0
    for opt in ("--steps", "--warmup", "--sweep", "--upper-precisions", "--svd-mode", "--no-rsvd"):
        assert opt in p.stdout
