"""Host logic of bench.py that decides whether committed counter summaries
still describe the kernels: the kernel-source fingerprint ignores comments and
layout, and only those."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_strip_comments_keeps_code_and_literals():
    src = 'a = "x // y /* z */"; // gone\nb = \'/\';  /* also\n gone */ c = a /b;\n'
    assert bench.strip_comments(src) == 'a = "x // y /* z */"; b = \'/\'; c = a /b;'
    assert bench.strip_comments('s = "q\\"//"; // c') == 's = "q\\"//";'


def test_fingerprint_ignores_comments_not_code():
    base = "int f(int x) { return x * 2; }\n"
    assert bench.strip_comments("// header\n" + base) == bench.strip_comments(base)
    assert bench.strip_comments(base.replace("  ", " ") + "/* note */") == bench.strip_comments(base)
    assert bench.strip_comments(base.replace("* 2", "* 3")) != bench.strip_comments(base)
