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
                                  "moving_pair", "actuator_free", "free_range", "inverted_range", "free_damping",
                                  "negative_damping", "condim", "nan_pos", "inf_size", "negative_spin",
                                  "generic_rows"])
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
        m["geoms"][0]["body"] = 1                 # a plane on a moving body
    elif case == "moving_pair":
        # the torso box would collide with the feet: two moving bodies, which take pyramidal cones
        m["geoms"][1]["conaffinity"] = 1
        m["opt"]["cone"] = "elliptic"
    elif case == "actuator_free":
        m["actuators"][0]["joint"] = 0
    elif case == "free_range":
        m["joints"][0]["range"] = [-1.0, 1.0]
    elif case == "inverted_range":
        m["joints"][2]["range"] = [0.5, -0.5]
    elif case == "free_damping":
        m["joints"][0]["damping"] = 1.0
    elif case == "negative_damping":
        m["joints"][2]["damping"] = -1.0
    elif case == "condim":
        m["geoms"][1]["condim"] = 5
    elif case == "negative_spin":
        m["geoms"][1].update(condim=4, friction_spin=-0.1)
    elif case == "generic_rows":
        # condim 6 on the torso box (8 contacts) and the four feet: 6 x 12 = 72 rows > 64
        for g in m["geoms"]:
            g["condim"] = 6
    elif case == "nan_pos":
        m["bodies"][2]["pos"][0] = float("nan")
    elif case == "inf_size":
        m["geoms"][1]["size"][0] = float("inf")
    rc, msg = _create_error(m)
    assert rc == -1, (rc, msg)
    assert msg


def _create_json_error(text):
    from paper_2601_22074_amd import rbstep
    import ctypes as C
    h = C.c_void_p()
    rc = rbstep.lib().rb_model_create_json(text.encode(), C.byref(h))
    return rc, rbstep.lib().rb_last_error().decode()


@pytest.mark.parametrize("case", ["parent", "mass", "triangle", "quat", "free_not_root", "two_joints", "pair",
                                  "moving_pair", "actuator_free", "free_range", "inverted_range", "free_damping",
                                  "negative_damping", "condim", "nan_pos", "inf_size", "negative_spin",
                                  "generic_rows"])
def test_json_models_validated_like_descriptions(rb, case):
    """The JSON entry point hands the same description to the same validation: every invalid
    model above is rejected with the message the struct entry point gives."""
    import json
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
        m["geoms"][0]["body"] = 1                 # a plane on a moving body
    elif case == "moving_pair":
        # the torso box would collide with the feet: two moving bodies, which take pyramidal cones
        m["geoms"][1]["conaffinity"] = 1
        m["opt"]["cone"] = "elliptic"
    elif case == "actuator_free":
        m["actuators"][0]["joint"] = 0
    elif case == "free_range":
        m["joints"][0]["range"] = [-1.0, 1.0]
    elif case == "inverted_range":
        m["joints"][2]["range"] = [0.5, -0.5]
    elif case == "free_damping":
        m["joints"][0]["damping"] = 1.0
    elif case == "negative_damping":
        m["joints"][2]["damping"] = -1.0
    elif case == "condim":
        m["geoms"][1]["condim"] = 5
    elif case == "negative_spin":
        m["geoms"][1].update(condim=4, friction_spin=-0.1)
    elif case == "generic_rows":
        # condim 6 on the torso box (8 contacts) and the four feet: 6 x 12 = 72 rows > 64
        for g in m["geoms"]:
            g["condim"] = 6
    elif case == "nan_pos":
        m["bodies"][2]["pos"][0] = float("nan")
    elif case == "inf_size":
        m["geoms"][1]["size"][0] = float("inf")
    rc_d, msg_d = _create_error(m)
    rc_j, msg_j = _create_json_error(json.dumps(m))
    if case in ("nan_pos", "inf_size"):
        # JSON has no NaN or infinity: the parser already refuses the text
        assert rc_j == -1 and "model JSON" in msg_j, msg_j
        return
    assert (rc_j, msg_j) == (rc_d, msg_d)


@pytest.mark.parametrize("mutate,needle", [
    (lambda s: s[:-1], "offset"),                                        # truncated
    (lambda s: s + " x", "trailing"),
    (lambda s: s.replace('"mass": 6.0', '"mass": "6.0"', 1), "body 1: \"mass\" is not a number"),
    (lambda s: s.replace('"iquat": [1.0, 0.0, 0.0, 0.0]', '"iquat": [1.0, 0.0, 0.0]', 1), "\"iquat\" is not an array of 4"),
    (lambda s: s.replace('"type": "hinge"', '"type": "slide"', 1), "unknown type \"slide\""),
    (lambda s: s.replace('"type": "capsule"', '"type": "mesh"', 1), "unknown type \"mesh\""),
    (lambda s: s.replace('"contype": 1', '"contype": 1.5', 1), "not an integer"),
    (lambda s: s.replace('"solimp"', '"solimp_"', 1), "opt: missing \"solimp\""),
    (lambda s: s.replace('"joints"', '"joint_list"', 1), "model: missing \"joints\""),
    (lambda s: "[" + s + "]", "not an object"),
    (lambda s: "", "offset 0"),
    (lambda s: s.replace('"mass": 6.0', '"mass": -inf', 1), "non-finite number"),
    (lambda s: s.replace('"armature": 0.01}', '"armature": 0.01, "range": [0.1]}', 1), "\"range\" is not an array of 2"),
])
def test_malformed_json_rejected(rb, mutate, needle):
    import json
    text = json.dumps(robots.quadruped())
    bad = mutate(text)
    assert bad != text
    rc, msg = _create_json_error(bad)
    assert rc == -1, (rc, msg)
    assert needle in msg, msg


@pytest.mark.parametrize("name", ["chain3", "quadruped", "humanoid", "arm_box", "chain3_lim", "quadruped_lim",
                                  "humanoid_lim", "quadruped_terrain", "humanoid_terrain", "chain3_damp",
                                  "humanoid_damp", "quadruped_slip", "quadruped_elliptic4", "humanoid_elliptic4",
                                  "quadruped_elliptic6"])
def test_model_files_match_generators(name):
    """workloads/models/<name>.json holds exactly what the generator builds (float values
    round-trip through JSON unchanged)."""
    import json
    with open(os.path.join(ROOT, "workloads", "models", name + ".json")) as f:
        assert json.load(f) == json.loads(json.dumps(robots.by_name(name)))


def test_size_limits_rejected(rb):
    """Models past the kernel's static bounds are refused before any device call: more than
    128 collision pairs (the humanoid on a 3x3 tile grid has 220), more than 64 dofs."""
    rc, msg = _create_error(robots.humanoid_terrain(n=3))
    assert rc == -1 and "128 collision pairs" in msg, msg
    rc, msg = _create_error(robots.chain(65, "chain65"))
    assert rc == -1 and "64 dofs" in msg, msg
    # contact ids carry geom indices in 8-bit fields: more than 256 geoms are refused even when
    # they make no collision pair
    m = robots.chain3()
    for i in range(260):
        m["geoms"].append(dict(m["geoms"][1], contype=0, conaffinity=0))
    rc, msg = _create_error(m)
    assert rc == -1 and "256 geoms" in msg, msg


def test_every_declaration_cites_its_passage():
    """Each function of include/rbstep.h carries a comment that cites the paper passage that
    defines the operation (or states that no passage does); the allocation-free step names the
    callers it is for instead."""
    src = open(os.path.join(ROOT, "include", "rbstep.h")).read()
    names = _declared()
    for n in names:
        m = re.search(r"^[A-Za-z_][\w\s\*]*\b" + n + r"\s*\(", src, flags=re.M)
        assert m, n
        head = src[:m.start()]
        comment_end = head.rstrip().endswith("*/")
        assert comment_end, f"{n}: no comment right before the declaration"
        comment = re.sub(r"\s*\n\s*\*?\s*", " ", head[head.rstrip().rfind("/*"):])
        if n == "rb_step_noalloc":
            # no passage defines it: its comment names the callers it is for
            assert "callers that cannot allocate" in comment, n
            continue
        assert "Cites:" in comment and ("section" in comment or "no passage" in comment or "as rb_" in comment), n


def test_contacts_capacity_checked():
    """Contact buffers whose slots per world differ from the batch's capacity are refused before
    any launch (the kernel writes world w's contacts at w * capacity)."""
    from paper_2601_22074_amd import rbstep
    c = rbstep.Contacts(4, 8, device="cpu")
    c._struct(4, 8)
    with pytest.raises(ValueError):
        c._struct(4, 16)
    with pytest.raises(ValueError):
        c._struct(5, 8)


def test_c_caller_builds(tmp_path):
    """include/rbstep.h is a C99 header: a C caller (tests/c_abi_step.c) compiles with -Wall
    -Wextra -Werror and links against the library and the HIP runtime (it runs in the GPU
    tests)."""
    from c_abi_build import build_c_caller
    exe = build_c_caller(str(tmp_path / "c_abi_step"))
    assert os.path.exists(exe)
