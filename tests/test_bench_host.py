"""Host-side pieces of bench.py: the source hash that ties the committed
traffic counters to the step kernel ignores comments but not code, and the
one-GPU guard."""
import os

import bench


def test_code_tokens_drop_comments_keep_code():
    src = 'int a = 1; // note with an apostrophe\'s\n/* block\n comment */ int b = "//kept"; char q = \'/\';\n'
    assert bench.code_tokens(src) == 'int a = 1; int b = "//kept"; char q = \'/\';'


def test_comment_edit_keeps_hash_code_edit_changes_it():
    base = "x = a + b; // sum\n"
    assert bench.code_tokens(base) == bench.code_tokens("x = a + b;   /* the sum */\n")
    assert bench.code_tokens(base) != bench.code_tokens("x = a - b; // sum\n")


def test_fused_kernel_hash_is_stable():
    assert bench.fused_kernel_hash() == bench.fused_kernel_hash()
    assert len(bench.fused_kernel_hash()) == 16


def test_more_than_one_gpu_is_refused():
    """The library runs on one GPU: --gpus N > 1 prints a JSON error and exits 2
    before touching a device."""
    import json
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    out = json.loads(r.stdout.strip().splitlines()[-1])
    assert out["n_gpus"] == 2 and "one GPU" in out["error"]
