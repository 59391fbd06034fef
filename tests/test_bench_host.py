"""Host-side pieces of bench.py: the source hash that ties the committed
traffic counters to the step kernel ignores comments but not code."""
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
