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


def test_python_constants_match_the_header():
    from paper_2005_06170_amd import _lib
    text = open(os.path.join(ROOT, "include", "mps.h")).read()
    defs = dict(re.findall(r"^#define\s+(MPS_\w+)\s+(.+?)\s*(?:/\*.*)?$", text, re.M))
    for name in ("STATIC_MAX_GRID", "STATIC_MAX_PARTICLES", "SCATTER_MIN_GRID", "SCATTER_GATHER_MAX_MEAN",
                 "SCATTER_HALO_MAX_MEAN", "SCATTER_GATHER64_MAX_MEAN"):
        assert getattr(_lib, name) == eval(defs["MPS_" + name]), name
