"""CPU checks of the C ABI: the library loads, exports every entry point that
include/*.h declares, and rejects bad arguments on the host (no GPU needed)."""
import ctypes
import glob
import os
import re

import pytest

import svgen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DECL = re.compile(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(sv_\w+)\s*\(", re.M)


def declared_symbols():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(DECL.findall(text))
    return sorted(names)


@pytest.fixture(scope="module")
def b():
    from paper_2402_15281_amd import _binding
    return _binding


def test_every_declared_symbol_is_exported(b):
    names = declared_symbols()
    assert "sv_check_motions" in names and "sv_fk" in names
    for n in names:
        assert hasattr(b.lib, n), f"{n} declared in include/ but not exported by libsv.so"


def test_host_side_validation(b):
    arm = svgen.make_arm(1)
    r = b.make_robot(arm)
    assert b.lib.sv_status_string(-3) == b"workspace missing or too small"
    bad = b.make_robot(arm)
    bad.dof = 0
    assert b.lib.sv_fk(ctypes.byref(bad), None, 0, None, 0, None) == -1
    assert b"dof" in b.lib.sv_last_error()
    assert b.lib.sv_fk(ctypes.byref(r), None, -1, None, 0, None) == -2
    assert b.lib.sv_fk(ctypes.byref(r), None, 5, None, 0, None) == -1
    m = b.sv_motions(0, 0, 4, None, None, None)                        # T = 0
    c = b.sv_cloud(0, None, None, None)
    n = ctypes.c_size_t(0)
    assert b.lib.sv_workspace_size(1, ctypes.byref(r), None, 0, ctypes.byref(m), ctypes.byref(c), ctypes.byref(n)) == -1
    m = b.sv_motions(1, 16, 4, None, None, None)                       # spline without pointers
    assert b.lib.sv_workspace_size(1, ctypes.byref(r), None, 0, ctypes.byref(m), ctypes.byref(c), ctypes.byref(n)) == -1
    m = b.sv_motions(0, 16, 4, 1, 1, None)
    assert b.lib.sv_workspace_size(1, ctypes.byref(r), None, 0, ctypes.byref(m), ctypes.byref(c), ctypes.byref(n)) == 0
    assert n.value >= 4 * 7 * 16 * 32                                   # at least the FP32 capsule table


def test_oracle_and_library_share_no_code():
    """The HIP sources never include oracle files and the oracle never includes
    library sources; neither Python side imports the other."""
    for src in glob.glob(os.path.join(ROOT, "paper_2402_15281_amd", "**", "*.*"), recursive=True):
        if src.endswith((".hip", ".h", ".py", ".cpp")):
            assert "oracle" not in open(src).read().replace("oracle is the oracle", ""), src
    for src in glob.glob(os.path.join(ROOT, "oracle", "*.*")):
        if src.endswith((".c", ".py", ".h")):
            t = open(src).read()
            assert "paper_2402_15281_amd" not in t and "sv_internal" not in t, src


def test_network_validation_on_host(b):
    arm = svgen.make_arm(1)
    r = b.make_robot(arm)
    m = b.sv_motions(0, 16, 4, 1, 1, None)
    c = b.sv_cloud(100, 1, 1, 1)
    n = ctypes.c_size_t(0)
    net = b.sv_mlp(15, 512, 8, 1)
    assert b.lib.sv_workspace_size(2, None, ctypes.byref(net), 1, ctypes.byref(m), ctypes.byref(c), ctypes.byref(n)) == 0
    assert n.value == 7 * 512 * 512 * 2
    assert b.lib.sv_workspace_size(2, None, ctypes.byref(net), 0, ctypes.byref(m), ctypes.byref(c), ctypes.byref(n)) == 0
    assert n.value == 0
    assert b.lib.sv_workspace_size(1, ctypes.byref(r), ctypes.byref(net), 1, ctypes.byref(m), ctypes.byref(c),
                                   ctypes.byref(n)) == 0
    assert n.value >= 4 * 100 * 4 + 7 * 512 * 512 * 2
    bad = b.sv_mlp(15, 96, 8, 1)                     # BF16 needs 128/256/512
    assert b.lib.sv_workspace_size(2, None, ctypes.byref(bad), 1, ctypes.byref(m), ctypes.byref(c),
                                   ctypes.byref(n)) == -4
    bad = b.sv_mlp(17, 512, 8, 1)                    # in_dim does not match dof 6
    assert b.lib.sv_workspace_size(1, ctypes.byref(r), ctypes.byref(bad), 1, ctypes.byref(m), ctypes.byref(c),
                                   ctypes.byref(n)) == -2
    spline = b.sv_motions(1, 16, 4, 1, 1, 1)
    res = b.sv_results(None, None, None, None)
    assert b.lib.sv_check_motions(ctypes.byref(r), ctypes.byref(net), 2, 0.01, 0.03, ctypes.byref(spline),
                                  ctypes.byref(c), ctypes.byref(res), None, 0, None) == -4
    assert b.lib.sv_check_motions(ctypes.byref(r), None, 2, 0.01, 0.03, ctypes.byref(m),
                                  ctypes.byref(c), ctypes.byref(res), None, 0, None) == -1
