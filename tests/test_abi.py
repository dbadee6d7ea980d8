"""The C-ABI library loads and exports every function declared in
include/gtree.h (no GPU needed: nothing is called that touches a device)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not h.endswith(".h"):
            continue
        src = open(os.path.join(ROOT, "include", h)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        src = re.sub(r"//[^\n]*", "", src)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                             src, flags=re.M):
            if m.group(1) not in ("if", "while", "for", "return", "sizeof"):
                names.append(m.group(1))
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for f in ("tree_build", "tree_lookup_batch", "tree_insert_batch", "tree_delete_batch", "tree_range_batch",
              "tree_lookup_levelwise", "gt_set_sort_spin_limit"):
        assert f in names


def test_library_exports_every_declared_symbol():
    import paper_2604_21117_amd as g
    lib = ctypes.CDLL(g.LIB_PATH)
    missing = [f for f in declared_functions() if not hasattr(lib, f)]
    assert not missing, missing


def test_host_side_errors_without_device():
    import paper_2604_21117_amd as g
    p = g.make_params(8)
    assert g.tree_arena_bytes(p, 1 << 16, 0) > 0
    bad = g.make_params(5)
    assert g.tree_arena_bytes(bad, 10, 0) == 0
    # a null handle is rejected before anything is enqueued
    assert g.lib().tree_lookup_batch(None, None, 4, None, None, None) == g.GT_ERR_INVALID
    assert g.lib().tree_destroy(None) == g.GT_ERR_INVALID
    assert g.status_str(g.GT_ERR_CAPACITY) == "capacity exceeded"
    assert g.lib().tree_delete_batch(None, None, 4, None, None) == g.GT_ERR_INVALID


def test_sort_spin_limit_hook_is_host_only():
    """The testing hook sets a host value read at launch: it returns the
    previous limit (the default 2^20) and touches no device."""
    import paper_2604_21117_amd as g
    old = g.set_sort_spin_limit(5)
    try:
        assert old == 1 << 20
        assert g.set_sort_spin_limit(0) == 5
    finally:
        assert g.set_sort_spin_limit(old) == 0
    assert g.set_sort_spin_limit(old) == old
