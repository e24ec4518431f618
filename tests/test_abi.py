"""The C-ABI library loads without a GPU and exports every declared function."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        txt = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(gothic_[a-z_]+)\s*\(", txt))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    import paper_1610_07279_amd as g
    lib = ctypes.CDLL(g.LIB_PATH)
    names = _declared()
    assert len(names) >= 12
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_defaults_and_cpu_only_errors():
    import paper_1610_07279_amd as g
    p = g.default_params()
    assert (p.key_kind, p.n_leaf, p.multipole, p.group_size, p.list_depth, p.compensated,
            p.check, p.timing, p.node_capacity) == (0, 16, 1, 32, 384, 1, 1, 0, 0)
    assert p.r_crit == -0.0625
    # a NULL context is rejected before any device call
    rc = g.lib.gothic_tree_forces(None, 10, None, ctypes.c_float(0.1), ctypes.c_float(0.5),
                                  None, None, None)
    assert rc == g.EINVAL
    assert b"NULL" in g.lib.gothic_last_error()
    assert g.lib.gothic_destroy(None) == g.OK


def test_oracle_does_not_enter_the_package():
    # the product path never imports or links the oracle
    for f in glob.glob(os.path.join(ROOT, "paper_1610_07279_amd", "**", "*"), recursive=True):
        if f.endswith((".py", ".hip", ".h", ".cpp")):
            txt = open(f).read()
            assert "import oracle" not in txt and "liboracle" not in txt and "orc_" not in txt, f
