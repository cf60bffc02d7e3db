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
