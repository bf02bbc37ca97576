"""The built library loads on the host and exports every entry point that
include/afq.h declares (no compute call: no GPU is needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "afq.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(afq_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared()
    for need in ("afq_init_hamiltonian", "afq_init_trial", "afq_propagate_batch",
                 "afq_local_energy_batch"):
        assert need in names


def test_library_exports_every_declared_symbol():
    path = os.path.join(ROOT, "paper_2403_02542_amd", "libafq.so")
    if not os.path.exists(path):
        pytest.fail("libafq.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, f"declared but not exported: {missing}"
    from paper_2403_02542_amd import afq
    assert sorted(afq.EXPORTED) == declared()
