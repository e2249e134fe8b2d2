"""The matching the GPU computes by local-minimum rounds equals the oracle's
sequential greedy matching in ascending priority key, for every priority
order of small random proposal graphs (CPU only).

The oracle claims proposals one by one in key order (the paper's CPU
semantics, Sec. 2.5).  The GPU instead repeats rounds over all live
proposals: each posts its key at both of its sites, a proposal holding the
minimum at both sites is claimed, and live proposals that touch a claimed
site die (Blelloch, Fineman, Shun, SPAA 2012).  The rounds are written out
here from that description and run against the oracle's `match` with the
keys of each permutation injected in place of its Philox keys.
"""

import itertools

import numpy as np

from oracle import OracleSystem


def _rounds(props, key):
    """Local-minimum rounds over the proposals props (site -> partner)."""
    live = dict(props)
    claimed, pairs = set(), []
    while live:
        best = {}
        for i, j in live.items():
            for v in (i, j):
                best[v] = min(best.get(v, key[i]), key[i])
        won = [i for i, j in live.items() if best[i] == key[i] and best[j] == key[i]]
        assert won, "every round claims at least the smallest live key"
        for i in won:
            j = live[i]
            claimed.update((i, j))
            pairs.append((i, j))
        live = {i: j for i, j in live.items() if i not in claimed and j not in claimed}
    return sorted(pairs)


def _oracle_match(props, key):
    o = OracleSystem(2, 1, 10.0, 1)     # only its matching is used
    o.match_keys = lambda a, s, ps: np.array([key[p] for p in ps], dtype=np.uint64)
    return sorted(o.match(0, 1, props))


def test_rounds_equal_greedy_for_every_priority_order():
    rng = np.random.default_rng(7)
    graphs = 0
    for _ in range(60):
        n_sites = int(rng.integers(3, 9))
        n_prop = int(rng.integers(2, min(6, n_sites) + 1))
        proposers = rng.choice(n_sites, n_prop, replace=False).tolist()
        props = {}
        for i in proposers:
            j = int(rng.integers(0, n_sites - 1))
            props[i] = j if j < i else j + 1          # any other site
        for perm in itertools.permutations(range(n_prop)):
            key = {p: (perm[k] << 32) | p for k, p in enumerate(sorted(props))}
            assert _rounds(props, key) == _oracle_match(props, key), (props, key)
        graphs += 1
    assert graphs == 60


def test_mutual_proposals_and_chains():
    """Hand-made cases: two sites proposing to each other form one pair; a
    chain a -> b -> c -> d matches by keys (smallest first)."""
    props = {0: 1, 1: 0}
    key = {0: (5 << 32) | 0, 1: (3 << 32) | 1}
    assert _rounds(props, key) == _oracle_match(props, key) == [(1, 0)]
    props = {0: 1, 1: 2, 2: 3}
    key = {0: (2 << 32) | 0, 1: (1 << 32) | 1, 2: (3 << 32) | 2}
    # 1-2 is claimed first (key 1); 0-1 and 2-3 touch it and die
    assert _rounds(props, key) == _oracle_match(props, key) == [(1, 2)]
    key = {0: (1 << 32) | 0, 1: (3 << 32) | 1, 2: (2 << 32) | 2}
    # 0-1 first, then 2-3; 1-2 touches 1
    assert _rounds(props, key) == _oracle_match(props, key) == [(0, 1), (2, 3)]
