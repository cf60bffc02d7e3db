"""The autotuner's decision key (host logic, CPU): models of equal sizes but different
features get different keys; the same plan gets the same key."""
from types import SimpleNamespace

from paper_2601_22074_amd import autotune
from workloads import robots


def _batch(desc, ncap=64, lds=9728):
    return SimpleNamespace(model=SimpleNamespace(desc=desc, lds_bytes=lds), ncap=ncap)


def test_same_plan_same_key():
    a = [_batch(robots.humanoid()), _batch(robots.quadruped())]
    b = [_batch(robots.humanoid()), _batch(robots.quadruped())]
    assert autotune.signature(a, [8192, 4096]) == autotune.signature(b, [8192, 4096])


def test_features_and_counts_change_the_key():
    base = autotune.signature([_batch(robots.humanoid())], [8192])
    assert autotune.signature([_batch(robots.humanoid_damp())], [8192]) != base
    assert autotune.signature([_batch(robots.humanoid_lim())], [8192]) != base
    assert autotune.signature([_batch(robots.humanoid())], [4096]) != base
    assert autotune.signature([_batch(robots.humanoid(), ncap=32)], [8192]) != base


def test_candidates_cover_every_dimension():
    """The candidate schedules: the separate plain launches, and fused launches over every
    dispatch order with every world launched at once, persistent grids of 1x and 2x the resident
    capacity where they are smaller than the work list, the occupancy settings (automatic, 3,
    capped at 2) and 1, 2 or 4 worlds per workgroup; each a (kind, order, grid, occupancy,
    worlds per workgroup) tuple, with no duplicates."""
    from paper_2601_22074_amd import rbstep
    c = autotune.candidates(7680, 2048)
    assert c[0] == ("separate", None, None, None, None)
    fused = [x for x in c if x[0] == "fused"]
    assert len(set(fused)) == len(fused) and all(len(x) == 5 for x in c)
    orders = {rbstep.ORDER_HEAVY_FIRST, rbstep.ORDER_INTERLEAVE, rbstep.ORDER_BATCH}
    assert {x[1] for x in fused} == orders
    assert {x[2] for x in fused} == {0, 2048, 4096}
    assert {x[3] for x in fused} == {0, 3, 2}
    assert {x[4] for x in fused} == {1, 2, 4}
    # a work list smaller than the resident capacity has no persistent grid
    assert {x[2] for x in autotune.candidates(1000, 2048) if x[0] == "fused"} == {0}
