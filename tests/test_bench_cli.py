"""bench.py's command line, checked without a GPU: the one-GPU contract."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], cwd=ROOT,
                          capture_output=True, text=True, timeout=120)


def test_more_than_one_gpu_is_refused_with_a_message():
    for n in ("2", "8"):
        r = _bench("--gpus", n, "--steps", "1", "--warmup", "0")
        assert r.returncode == 2
        assert "one GPU only" in r.stderr
        assert r.stdout == ""


def test_help_lists_the_contract_flags():
    r = _bench("--help")
    assert r.returncode == 0
    for flag in ("--gpus", "--steps", "--warmup", "--render-streams", "--no-clip"):
        assert flag in r.stdout


def test_render_streams_take_one_or_two():
    """--render-streams: the step's render launches in flight at once (1 or 2);
    anything else is refused by the parser before the GPU is touched."""
    r = _bench("--help")
    assert "--render-streams" in r.stdout
    for bad in ("0", "3"):
        r = _bench("--render-streams", bad, "--steps", "1")
        assert r.returncode == 2 and "--render-streams" in r.stderr and r.stdout == ""
