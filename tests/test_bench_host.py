"""Host logic of bench.py: the hash that gates the committed HBM counters follows the code of
the step kernel, not its comments or layout."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_code_text_drops_comments_and_keeps_literals():
    src = ('int x = 1;   // a comment\n/* a block\n comment */ asm volatile("" : "+v"(x));\n'
           "char q = '\"'; const char *s = \"a // b /* c */\";")
    assert bench.code_text(src) == ('int x = 1; asm volatile("" : "+v"(x)); char q = \'"\'; '
                                    'const char *s = "a // b /* c */";')
    assert bench.code_text("a  //x\n b") == bench.code_text("a\n\n  b /* y */")
    assert bench.code_text("a + b") != bench.code_text("a - b")


def test_kernel_source_hash_is_stable():
    h = bench.kernel_source_hash()
    assert len(h) == 16 and h == bench.kernel_source_hash()
