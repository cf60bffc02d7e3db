"""Host-side checks of the C ABI library (no GPU needed): it loads, exports every function
include/rbstep.h declares, and rejects invalid models before touching the device."""
import os
import re

import pytest

from workloads import robots

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "rbstep.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rb_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def rb():
    import paper_2601_22074_amd as pkg
    pkg.lib()
    return pkg


def test_header_matches_exports(rb):
    from paper_2601_22074_amd import rbstep
    names = _declared()
    assert names == sorted(rbstep.EXPORTED)
    L = rb.lib()
    for n in names:
        assert hasattr(L, n), n


def _create_error(m):
    from paper_2601_22074_amd import rbstep
    import ctypes as C
    d, keep = rbstep.marshal_desc(m)
    h = C.c_void_p()
    rc = rbstep.lib().rb_model_create(C.byref(d), C.byref(h))
    return rc, rbstep.lib().rb_last_error().decode()


@pytest.mark.parametrize("case", ["parent", "mass", "triangle", "quat", "free_not_root", "two_joints", "pair",
                                  "moving_pair", "actuator_free"])
def test_invalid_models_rejected(rb, case):
    m = robots.quadruped()
    if case == "parent":
        m["bodies"][3]["parent"] = 5
    elif case == "mass":
        m["bodies"][2]["mass"] = 0.0
    elif case == "triangle":
        m["bodies"][2]["inertia"] = [1.0, 0.1, 0.1]
    elif case == "quat":
        m["bodies"][2]["quat"] = [1.0, 0.1, 0.0, 0.0]
    elif case == "free_not_root":
        m["joints"][1]["type"] = "free"
    elif case == "two_joints":
        m["joints"].insert(2, dict(m["joints"][1]))
    elif case == "pair":
        m["geoms"][0]["type"] = "sphere"; m["geoms"][0]["size"] = [0.1, 0, 0]
    elif case == "moving_pair":
        m["geoms"][1]["conaffinity"] = 1          # torso box would collide with the feet
    elif case == "actuator_free":
        m["actuators"][0]["joint"] = 0
    rc, msg = _create_error(m)
    assert rc == -1, (rc, msg)
    assert msg
