"""Host checks of the seeded input generator: the seed schedule never reuses a seed.

The warm-start network is trained on config-4 pairs, evaluated on held-out config-5
pairs, and benchmarked on config-1 (and mixed-size config-3) pairs; a shared seed
would put evaluation pairs into the training set.
"""

import numpy as np
import pytest

from paper_1009_6039_amd import workloads as W


def seeds(config, count):
    return {W.seed_for(config, q) for q in range(count)}


def test_training_heldout_and_benchmark_seeds_are_disjoint():
    train = seeds(4, 20000)        # the network's 20k training pairs
    held = seeds(5, 1000)          # held-out evaluation pairs
    bench = seeds(1, 1024)         # benchmark / parity pairs
    mixed = seeds(3, 1024)         # mixed-size batch
    other = seeds(0, 16) | seeds(2, 16)
    assert len(train) == 20000 and len(held) == 1000 and len(bench) == 1024
    sets = [train, held, bench, mixed, other]
    for a in range(len(sets)):
        for b in range(a + 1, len(sets)):
            assert not (sets[a] & sets[b]), (a, b)


def test_seed_schedule_is_injective_across_the_index_boundary():
    pairs = [(c, q) for c in (0, 1, 4, 5, 99) for q in (0, 1, 998, 999, 1000, 1001, 4999, 10 ** 7 - 1)]
    got = [W.seed_for(c, q) for c, q in pairs]
    assert len(set(got)) == len(got)
    # the first thousand pairs of a config keep the plain schedule
    assert W.seed_for(1, 7) == W.SEED_BASE + 1007
    # config c, index >= 1000 never meets config c + 1, index < 1000 (the old collision)
    assert W.seed_for(4, 1000 + 3) != W.seed_for(5, 3)


@pytest.mark.parametrize("bad", [(-1, 0), (100, 0), (0, -1), (0, 10 ** 7)])
def test_seed_schedule_rejects_out_of_range_arguments(bad):
    with pytest.raises(ValueError):
        W.seed_for(*bad)


def test_same_seed_same_pair():
    a = W.blobs(32, W.seed_for(1, 3))
    b = W.blobs(32, W.seed_for(1, 3))
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_e1_example_mass_is_that_of_g():
    # f = g(T(x)) det DT(x) with T = x + grad u* a diffeomorphism of the torus: by change of
    # variables int f = int g = 1 (the trapezoid rule is spectrally exact for these smooth
    # periodic integrands)
    for kw in ({}, dict(alpha=0.5, rho=2), dict(gamma=2, k=200.0)):
        f, g, u = W.e1_example(64, **kw)
        assert abs(np.mean(f) - 1.0) < 1e-12 and abs(np.mean(g) - 1.0) < 1e-12
        assert np.all(f > 0)


def test_e1_family_members_are_valid_and_seeded():
    # positive densities of equal mass, a convex potential, different members per seed
    a = W.e1_family(64, W.seed_for(6, 0))
    b = W.e1_family(64, W.seed_for(6, 0))
    c = W.e1_family(64, W.seed_for(6, 1))
    assert all(np.array_equal(x, y) for x, y in zip(a, b))
    assert not np.array_equal(a[0], c[0])
    for f, g, u in (a, c):
        assert f.min() > 0 and g.min() > 0
        assert abs(f.mean() - g.mean()) < 1e-3 * g.mean()
