"""The C-ABI library loads and exports every entry point of include/mps.h
(no compute calls: this runs without a GPU)."""
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "mps.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|size_t|const char\*)\s+(mps_\w+)\s*\(", text, re.M)))


def test_header_declares_core_calls():
    names = _declared()
    for n in ("mps_plan_create", "mps_estimate", "mps_estimate_batch", "mps_assign", "mps_fft",
              "mps_server_create", "mps_submit", "mps_wait", "mps_strerror"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2005_06170_amd import _lib
    L = _lib.lib()
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing
