"""Host-side behaviour of bench.py that needs no GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    for argv, env in ((["--gpus", "2"], {}), ([], {"WORLD_SIZE": "4"})):
        p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + argv, cwd=ROOT,
                           env=dict(os.environ, **env), capture_output=True, text=True, timeout=120)
        assert p.returncode == 2, (argv, p.returncode, p.stderr[-400:])
        assert "one GPU" in p.stderr
        assert p.stdout == ""
