"""CPU-side checks of the C-ABI library: it loads, and it exports every entry
point that the headers under include/ declare.  No compute calls (no GPU here)."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
INCLUDE = os.path.join(ROOT, "include")


def declared_functions():
    names = set()
    for h in sorted(os.listdir(INCLUDE)):
        if h.endswith(".h"):
            text = re.sub(r"/\*.*?\*/", "", open(os.path.join(INCLUDE, h)).read(), flags=re.S)
            names |= set(re.findall(r"\b((?:sim|rt)_[a-z_]+)\s*\(", text))
    return sorted(n for n in names if not n.endswith("_fn"))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("sim_create", "sim_load_demand", "sim_step", "sim_stats", "sim_set_control", "rt_create", "rt_plan",
              "rt_weights_from_stats"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_1807_01148_amd as P
    lib_path = P.LIB_PATH
    if not os.path.exists(lib_path):
        pytest.fail("libtrafficsim.so is not built")
    out = subprocess.check_output(["nm", "-D", "--defined-only", lib_path]).decode()
    exported = set(re.findall(r" T ((?:sim|rt)_\w+)", out))
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing
    lib = P.library()
    for n in declared_functions():
        assert hasattr(lib, n)
    assert set(P.EXPORTED) <= exported


def test_library_is_built_for_gfx950():
    import paper_1807_01148_amd as P
    # the HIP fat binary names its code objects by target
    data = open(P.LIB_PATH, "rb").read()
    assert b"gfx950" in data


def test_strerror_codes():
    import paper_1807_01148_amd as P
    lib = P.library()
    assert lib.sim_strerror(0) == b"ok"
    assert lib.sim_strerror(P.SIM_EROUTE) == b"invalid route"
    assert lib.sim_strerror(12345) == b"unknown error"


def test_check_classes_match_the_header():
    import paper_1807_01148_amd as P
    text = open(os.path.join(INCLUDE, "trafficsim.h")).read()
    body = re.search(r"enum sim_check_class \{(.*?)\};", text, flags=re.S).group(1)
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    names = re.findall(r"SIM_CHECK_([A-Z]+)", body)
    assert names[-1] == "CLASSES"
    assert tuple(n.lower() for n in names[:-1]) == P.CHECK_CLASSES
