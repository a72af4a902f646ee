"""Host-side parts of bench.py (no GPU): the source hash that ties the committed counter
summaries to the kernels ignores comments and blank lines but not code, every mode and
kernel kind has an algorithmic operation count, and a request for more than one GPU is
refused with a message before anything touches a device."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_code_only_ignores_comments_not_code():
    a = "// header\nint f(int x) {  // one\n  return x + 1;\n}\n"
    b = "/* another\n   header */\nint f(int x) {\n\n  // a new line of comment\n  return x + 1;  // two\n}\n"
    c = "// header\nint f(int x) {  // one\n  return x + 2;\n}\n"
    assert bench._code_only(a) == bench._code_only(b)
    assert bench._code_only(a) != bench._code_only(c)


def test_source_hash_is_stable_and_covers_the_kernel_sources():
    h = bench.source_hash()
    assert len(h) == 16 and h == bench.source_hash()
    for name in bench.KERNEL_SOURCES:
        assert os.path.exists(os.path.join(ROOT, "paper_1010_2641_amd", "csrc", name))


def test_every_kernel_has_an_operation_count():
    for mode in ("ph64", "f32", "grid"):
        for dom in ("fwd", "bwd"):
            for fkind in ("complex", "unit"):
                assert bench.ALG_SLOTS[(mode, dom, fkind)] > 0


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""
