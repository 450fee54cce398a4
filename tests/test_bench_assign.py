"""Host logic of the benchmark's serving stream: the assignment of keys to servers (no GPU)."""
import itertools

import numpy as np
import pytest

from bench import assign_keys


def brute_size(sizes, weights, shards):
    """Smallest achievable largest load over every split of the sorted keys into contiguous intervals."""
    order = np.argsort(sizes, kind="stable")
    cost = (np.asarray(weights) * np.asarray(sizes))[order]
    n = len(sizes)
    best = np.inf
    for cuts in itertools.combinations(range(1, n), shards - 1):
        edges = (0,) + cuts + (n,)
        best = min(best, max(cost[edges[j]:edges[j + 1]].sum() for j in range(shards)))
    return best


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("shards", [1, 2, 3, 4])
def test_size_intervals_are_contiguous_and_minimise_the_largest_load(seed, shards):
    gen = np.random.default_rng(seed)
    n = 11
    sizes = np.exp(gen.uniform(0, 6, size=n))
    w = gen.dirichlet(np.ones(n))
    owner = assign_keys(sizes, w, shards, "size")
    assert sorted(set(owner)) == list(range(shards))          # every server gets a key
    # server j holds an interval of step times, below server j + 1's
    for j in range(shards - 1):
        assert sizes[owner == j].max() <= sizes[owner == j + 1].min()
    loads = [float((w * sizes)[owner == j].sum()) for j in range(shards)]
    assert max(loads) == pytest.approx(brute_size(sizes, w, shards), rel=1e-12)


def test_load_assignment_balances_and_covers_every_key():
    gen = np.random.default_rng(7)
    sizes = np.exp(gen.uniform(0, 6, size=40))
    w = gen.dirichlet(np.ones(40))
    owner = assign_keys(sizes, w, 3, "load")
    cost = w * sizes
    loads = np.array([cost[owner == j].sum() for j in range(3)])
    # greedy largest-first: no server exceeds the mean by more than the largest single key
    assert loads.max() - loads.mean() <= cost.max() + 1e-15
    assert set(owner) == {0, 1, 2}


def test_bad_arguments_are_refused():
    with pytest.raises(ValueError):
        assign_keys([1.0, 2.0], [0.5, 0.5], 3)
    with pytest.raises(ValueError):
        assign_keys([1.0, 2.0], [0.5, 0.5], 2, "random")
