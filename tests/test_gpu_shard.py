"""Splitting a Wigner ensemble by sample (the runs are independent, Sec. 2.2)
on one GPU: contexts over disjoint sample ranges, numbered in the whole
ensemble through spin1_init_wigner_shard, reproduce one context over the
whole ensemble bit for bit (fields, per-sample shell means, observables)."""
import numpy as np
import pytest

from oracle import spin1 as O

pytestmark = pytest.mark.gpu

P = dict(c0=1.0, c1=-0.1, q=0.09)


def run(lib, groups, dtype, seed, first=None, steps=7, dt=0.02):
    sim = lib.Sim(groups, P, dtype=dtype)
    sim.init_wigner(seed, first)
    init = sim.fields()
    sim.step(steps, dt)
    out = {"init": init, "fields": sim.fields(),
           "bins": [sim.structure_factor_samples(g) for g in range(len(groups))],
           "obs": [sim.observables(g) for g in range(len(groups))]}
    sim.close()
    return out


def split(groups, cut):
    """Two shards of every group: samples [0, cut[i]) and [cut[i], S_i)."""
    a = [(d, n, dx, c) for (d, n, dx, s), c in zip(groups, cut)]
    b = [(d, n, dx, s - c) for (d, n, dx, s), c in zip(groups, cut)]
    return a, [0] * len(groups), b, list(cut)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("groups,cut", [
    ([(2, (64, 32), 0.5, 8)], [3]),
    ([(1, (256,), 0.5, 12), (2, (32, 32), 0.5, 6), (2, (64, 64), 0.5, 4)], [5, 2, 3]),
])
def test_shards_reproduce_the_full_ensemble(lib, dtype, groups, cut):
    full = run(lib, groups, dtype, 1207)
    ga, fa, gb, fb = split(groups, cut)
    a = run(lib, ga, dtype, 1207, fa)
    b = run(lib, gb, dtype, 1207, fb)
    for i, c in enumerate(cut):
        for key in ("init", "fields", "bins", "obs"):
            whole = full[key][i]
            assert np.array_equal(whole[:c], a[key][i]), (key, i)
            assert np.array_equal(whole[c:], b[key][i]), (key, i)


def test_shard_init_matches_oracle_sample_range(lib):
    """The shard's samples are the oracle's samples first .. first + S - 1."""
    grid = (2, (32, 16), 0.5, 3)
    og = O.Grid(2, (32, 16), 0.5, 3)
    op = O.Params(1.0, -0.1, 0.09)
    for group_count, first in ((1, 5), (2, 40)):
        groups = [grid] * group_count
        sim = lib.Sim(groups, P, dtype="c128")
        sim.init_wigner(2024, [first] * group_count)
        got = sim.fields()
        sim.close()
        for g in range(group_count):
            ref = O.init_wigner(2024, og, op, group=g, samples=range(first, first + 3))
            assert np.max(np.abs(got[g] - ref)) <= 1e-15 * np.max(np.abs(ref))


def test_shard_offset_validation(lib):
    sim = lib.Sim([(1, (64,), 0.5, 2)], P, dtype="c64")
    with pytest.raises(lib.Spin1Error) as ei:
        sim.init_wigner(1, [-1])
    assert ei.value.code == lib.EINVAL
    assert "first_sample" in str(ei.value)
    # nothing was bound by the failed call
    with pytest.raises(lib.Spin1Error) as ei:
        sim.step(1, 0.01)
    assert ei.value.code == lib.ESTATE
    sim.close()
