"""Host-side pieces of the benchmark (no GPU): the one-GPU guard and the source
digest that ties a counter profile to the kernel it was taken on."""
import os
import re
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_digest_covers_existing_definitions():
    kry = open(os.path.join(ROOT, "paper_2101_03777_amd", "csrc", "krylov.hip")).read()
    for key in bench.KERNEL_PARTS:
        block = bench._block(kry, key)
        assert block.startswith(key)
        assert block.count("{") == block.count("}") and block.endswith("}")
    d = bench.source_digest()
    assert re.fullmatch(r"[0-9a-f]{16}", d)
    assert d == bench.source_digest()


def test_block_extraction():
    text = "int f() { if (x) { y(); } return 1; }\nint g() { return 2; }"
    assert bench._block(text, "int f(") == "int f() { if (x) { y(); } return 1; }"
    assert bench._block(text, "int g(") == "int g() { return 2; }"
