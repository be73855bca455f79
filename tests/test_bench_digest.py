"""The digest that ties stored counters to the engine's code ignores comments
and blank lines and changes with any code token."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _digest_of(tmp_path, text):
    p = tmp_path / "k.hip"
    p.write_text(text)
    return bench.code_digest(str(p))


def test_comments_and_blank_lines_do_not_count(tmp_path):
    base = "int f(int x) {\n  return x + 1;\n}\n"
    noted = "// adds one\nint f(int x) {  \n\n  return x + 1;   // the sum\n  /* block\n comment */\n}\n"
    assert _digest_of(tmp_path, base) == _digest_of(tmp_path, noted)


def test_code_changes_count(tmp_path):
    assert _digest_of(tmp_path, "int f(int x) { return x + 1; }\n") != \
        _digest_of(tmp_path, "int f(int x) { return x + 2; }\n")

