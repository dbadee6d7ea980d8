"""Host-side helpers of the benchmark: the code hash that ties a stored
traffic figure to the kernel it was taken on, and the algorithmic byte
count of a lookup batch (checked against counts worked by hand)."""
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


def test_code_tokens_drop_comments_and_layout():
    a = "int x = 1; // one\n/* block\n comment */ int  y=2;\n"
    b = "int x = 1;\n\n\tint y=2; /* other */"
    assert bench.code_tokens(a) == bench.code_tokens(b) == "int x = 1; int y=2;"


def test_code_tokens_keep_literals():
    src = 'const char* s = "a // b /* c */";  char q = \'"\'; char e = \'\\\'\'; // tail'
    t = bench.code_tokens(src)
    assert '"a // b /* c */"' in t and "'\"'" in t and "'\\''" in t and "tail" not in t


def test_code_tokens_see_code_changes():
    assert bench.code_tokens("a = b + 1;") != bench.code_tokens("a = b + 2;")
    assert bench.code_tokens("x = 1; // y = 2;") != bench.code_tokens("x = 1; y = 2;")


def test_lookup_sources_hash_ignores_comment_edits(tmp_path, monkeypatch):
    csrc = tmp_path / "paper_2604_21117_amd" / "csrc"
    csrc.mkdir(parents=True)
    for f in ("common.h", "traverse.h", "lookup.hip", "kernels.h"):
        (csrc / f).write_text(f"// {f}\nint {f.split('.')[0]}_v = 1;\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h0 = bench.lookup_sources_hash()
    (csrc / "lookup.hip").write_text("/* reworded */\nint   lookup_v = 1;  // note\n")
    assert bench.lookup_sources_hash() == h0
    (csrc / "lookup.hip").write_text("int lookup_v = 2;\n")
    assert bench.lookup_sources_hash() != h0
    # the same text moved from one file to the next is a different build
    (csrc / "lookup.hip").write_text("int lookup_v = 1; int kernels_v = 1;\n")
    (csrc / "kernels.h").write_text("\n")
    assert bench.lookup_sources_hash() != h0


def test_algorithmic_bytes_by_hand():
    # 16^3 keys at 16 a leaf: 256 leaves under 16 parents under one root
    keys = np.arange(4096, dtype=np.uint64) * 3
    # one query per leaf: every node of the tree once
    q = keys[::16]
    ab = bench.algorithmic_bytes(keys, q, height=3, hits=len(q))
    assert ab["distinct_nodes_per_level"] == [1, 16, 256]
    assert ab["bytes"] == (1 + 16) * 128 + 256 * 128 + 256 * (8 + 8 + 1) + 256 * 8
    # all queries in one leaf: one path
    q = keys[32:48]
    ab = bench.algorithmic_bytes(keys, q, height=3, hits=8)
    assert ab["distinct_nodes_per_level"] == [1, 1, 1]
    assert ab["bytes"] == 3 * 128 + 16 * 17 + 8 * 8
    # an absent key above the largest ends in the last leaf
    q = np.array([keys[-1] + 1], dtype=np.uint64)
    assert bench.algorithmic_bytes(keys, q, height=3, hits=0)["distinct_nodes_per_level"] == [1, 1, 1]
