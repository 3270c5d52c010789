"""Pins of the oracle's DBSCAN clustering of detections (Sec. 2.3): hand
examples (chains, the MinPts edge, inclusive extents per dimension, a
border point reached from two clusters), scikit-learn's DBSCAN with the
Chebyshev metric on exactly scaled coordinates (same core points, noise and
partition), a pure-Python density-reachability search on small random
sets, and the empty input."""
import numpy as np
import pytest

import oracle


def _core(s, d, q, te, de, se, mp):
    return np.array([len(n) >= mp for n in oracle.cluster_neighbours(s, d, q, te, de, se)])


def test_two_blobs_and_noise():
    lab, k = oracle.cluster([0, 1, 2, 10, 11, 12, 50], [0, 0, 0, 5, 5, 5, 9], [7, 7, 7, 8, 8, 8, 9], 2, 1, 1.0, 3)
    assert k == 2 and list(lab) == [0, 0, 0, 1, 1, 1, -1]


def test_chain_and_border_ends():
    t = np.arange(0, 22, 2)
    lab, k = oracle.cluster(t, np.zeros_like(t), np.full(t.shape, 7.0), 2, 0, 1.0, 3)
    assert k == 1 and np.all(lab == 0)
    assert list(_core(t, np.zeros_like(t), np.full(t.shape, 7.0), 2, 0, 1.0, 3)) == [False] + [True] * 9 + [False]
    lab, k = oracle.cluster(t, np.zeros_like(t), np.full(t.shape, 7.0), 1, 0, 1.0, 2)
    assert k == 0 and np.all(lab == -1)


def test_min_pts_counts_the_point_itself():
    s, d, q = [0, 1, 2], [0, 0, 0], [7.0, 7.0, 7.0]
    assert oracle.cluster(s, d, q, 5, 0, 1.0, 3)[1] == 1     # 3 points within reach: core
    assert oracle.cluster(s, d, q, 5, 0, 1.0, 4)[1] == 0     # one short: noise


@pytest.mark.parametrize("dim", ["t", "dm", "snr"])
def test_extents_are_inclusive(dim):
    te, de, se = 3, 2, 0.5
    base = dict(t=[0, 0], dm=[0, 0], snr=[6.0, 6.0])
    at = dict(base)
    past = dict(base)
    at[dim] = [base[dim][0], base[dim][0] + dict(t=te, dm=de, snr=se)[dim]]
    past[dim] = [base[dim][0], base[dim][0] + dict(t=te + 1, dm=de + 1, snr=se + 0.25)[dim]]
    assert oracle.cluster(at["t"], at["dm"], at["snr"], te, de, se, 2)[1] == 1
    assert oracle.cluster(past["t"], past["dm"], past["snr"], te, de, se, 2)[1] == 0


def test_border_reached_from_two_clusters():
    # cluster A: t = 0..2 (indices 0-2), border b at t = 5 (index 3), cluster B: t = 8..10 (indices 4-6);
    # b reaches index 2 (t = 2) and index 4 (t = 8): it joins A, its lowest-indexed core neighbour's cluster
    s = [0, 1, 2, 5, 8, 9, 10]
    lab, k = oracle.cluster(s, [0] * 7, [7.0] * 7, 3, 0, 1.0, 4)
    assert k == 2 and list(lab) == [0, 0, 0, 0, 1, 1, 1]
    # the same points listed with B first: b now joins B
    s2 = [8, 9, 10, 5, 0, 1, 2]
    lab2, _ = oracle.cluster(s2, [0] * 7, [7.0] * 7, 3, 0, 1.0, 4)
    assert list(lab2) == [0, 0, 0, 0, 1, 1, 1]


def _random_points(n, seed):
    rng = np.random.default_rng(seed)
    s = rng.integers(0, 400, n).astype(np.int64)
    d = rng.integers(0, 40, n).astype(np.int32)
    q = (rng.integers(24, 48, n) * 0.25).astype(np.float32)
    # a few dense streaks, as a dispersed pulse leaves over neighbouring DMs
    for c in range(3):
        m = rng.integers(10, 30)
        i = rng.choice(n, m, replace=False)
        s[i] = rng.integers(0, 400) + rng.integers(-3, 4, m)
        d[i] = rng.integers(0, 40) + rng.integers(-2, 3, m)
    return s, d, q


@pytest.mark.parametrize("seed,mp", [(1, 3), (2, 4), (3, 5)])
def test_matches_sklearn_dbscan(seed, mp):
    from sklearn.cluster import DBSCAN
    te, de, se = 4, 2, 0.5          # powers of two: the scaled coordinates are exact
    s, d, q = _random_points(600, seed)
    lab, k = oracle.cluster(s, d, q, te, de, se, mp)
    X = np.stack([s / te, d / de, q.astype(np.float64) / se], axis=1)
    sk = DBSCAN(eps=1.0, min_samples=mp, metric="chebyshev").fit(X)
    core = np.zeros(len(s), bool)
    core[sk.core_sample_indices_] = True
    assert np.array_equal(core, _core(s, d, q, te, de, se, mp))
    assert np.array_equal(sk.labels_ == -1, lab == -1)
    assert k == len(set(sk.labels_[core]))
    # the same partition of the core points
    pairs = set(zip(lab[core], sk.labels_[core]))
    assert len(pairs) == k == len({a for a, _ in pairs}) == len({b for _, b in pairs})
    # numbering: clusters in order of their lowest core index
    firsts = [int(np.flatnonzero(core & (lab == c))[0]) for c in range(k)]
    assert firsts == sorted(firsts)


@pytest.mark.parametrize("seed", [4, 5, 6])
def test_matches_density_reachability_search(seed):
    """Pure-Python DBSCAN by definition: neighbourhoods by a double loop,
    clusters by expanding density-reachability from each unvisited core
    point, border points to their lowest-indexed core neighbour's cluster."""
    te, de, se, mp = 3, 1, 0.75, 3
    s, d, q = _random_points(150, seed)
    n = len(s)
    nb = [[j for j in range(n) if abs(int(s[i]) - int(s[j])) <= te and abs(int(d[i]) - int(d[j])) <= de
           and abs(float(np.float32(q[i]) - np.float32(q[j]))) <= se] for i in range(n)]
    core = [len(x) >= mp for x in nb]
    lab = [-1] * n
    k = 0
    for i in range(n):
        if core[i] and lab[i] < 0:
            lab[i] = k
            stack = [i]
            while stack:
                p = stack.pop()
                for j in nb[p]:
                    if core[j] and lab[j] < 0:
                        lab[j] = k
                        stack.append(j)
            k += 1
    for i in range(n):
        if not core[i]:
            cn = [j for j in nb[i] if core[j]]
            lab[i] = lab[min(cn)] if cn else -1
    got, kk = oracle.cluster(s, d, q, te, de, se, mp)
    assert kk == k and list(got) == lab


def test_empty_input():
    lab, k = oracle.cluster(np.zeros(0, np.int64), np.zeros(0, np.int32), np.zeros(0, np.float32), 2, 1, 1.0, 3)
    assert k == 0 and lab.shape == (0,)
