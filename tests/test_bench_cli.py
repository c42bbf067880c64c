"""Host-side behaviour of bench.py that needs no GPU: it measures one device
and says so when asked for more, and it reports the digest of the kernel
sources that its committed traffic profiles are keyed by."""
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench(*args, env=None):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          cwd=ROOT, env=env, timeout=120)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = _bench("--gpus", "2")
    assert r.returncode != 0
    assert "one GPU" in r.stderr and r.stdout == ""


def test_world_size_above_one_is_refused():
    env = dict(os.environ, WORLD_SIZE="2")
    r = _bench(env=env)
    assert r.returncode != 0 and "one GPU" in r.stderr


def test_traffic_profiles_match_the_kernel_sources():
    r = _bench("--kernel-digest")
    assert r.returncode == 0
    digest = r.stdout.strip()
    assert re.fullmatch(r"[0-9a-f]{16}", digest)
    prof = os.path.join(ROOT, "profiles")
    keyed = [f for f in os.listdir(prof) if f.endswith("_hbm_traffic.md")]
    assert keyed
    for f in keyed:
        text = open(os.path.join(prof, f)).read()
        assert f"- kernel_digest: {digest}" in text, f
