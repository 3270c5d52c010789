"""Pins of the oracle's FDBSCAN (Sec. 2.3): representative points of a core
point's neighbourhood (two per dimension) seed the expansion.  Hand examples
where it equals DBSCAN (a blob, a chain walked by its end points), where it
loses a point and where it splits a cluster (a point reachable only through
a core point that is never a representative), and properties against the
exact DBSCAN on random sets: core points are never noise, every DBSCAN noise
point stays noise, and the core points of one FDBSCAN cluster lie in one
DBSCAN cluster."""
import numpy as np
import pytest

import oracle


def test_blobs_equal_dbscan():
    s, d, q = [0, 1, 2, 10, 11, 12, 50], [0, 0, 0, 5, 5, 5, 9], [7, 7, 7, 8, 8, 8, 9]
    lab, k, nq = oracle.fdbscan(s, d, q, 2, 1, 1.0, 3)
    ref, kr = oracle.cluster(s, d, q, 2, 1, 1.0, 3)
    assert k == kr == 2 and np.array_equal(lab, ref)
    assert nq <= len(s)


def test_chain_walked_by_its_end_points():
    """Along a chain the +t and -t representatives are the next links, so the
    expansion reaches every point, as DBSCAN does."""
    t = np.arange(0, 22, 2)
    z = np.zeros_like(t)
    q = np.full(t.shape, 7.0)
    lab, k, _ = oracle.fdbscan(t, z, q, 2, 0, 1.0, 3)
    ref, kr = oracle.cluster(t, z, q, 2, 0, 1.0, 3)
    assert k == kr == 1 and np.array_equal(lab, ref)


# A core point A at the origin with six points on the border of its box, one
# per direction of each dimension (t, DM, SNR extents 2, 2, 2), and an
# interior core point B = (1, 1, 1).  X = (3, 3, 1) lies within B's box only:
# B is never a representative (no dimension has it farthest), so FDBSCAN
# never queries B and never reaches X.
_BOX = [(0, 0, 0), (2, 0, 0), (-2, 0, 0), (0, 2, 0), (0, -2, 0), (0, 0, 2), (0, 0, -2), (1, 1, 1), (3, 3, 1)]


def _pts(p):
    a = np.array(p, dtype=np.float64)
    return (a[:, 0] + 10).astype(np.int64), (a[:, 1] + 10).astype(np.int64), (a[:, 2] + 7).astype(np.float32)


def test_point_reachable_only_through_an_interior_core_point_is_lost():
    s, d, q = _pts(_BOX)
    ref, kr = oracle.cluster(s, d, q, 2, 2, 2.0, 4)
    lab, k, _ = oracle.fdbscan(s, d, q, 2, 2, 2.0, 4)
    assert kr == 1 and np.all(ref == 0)            # DBSCAN: X is a border point of B
    assert k == 1 and list(lab) == [0] * 8 + [-1]  # FDBSCAN: X is lost


def test_cluster_reached_through_an_interior_core_point_is_split():
    # X gets two more neighbours of its own and becomes a core point: DBSCAN
    # joins it to A's cluster through B, FDBSCAN starts a second cluster at X
    # (B keeps the first cluster's label)
    s, d, q = _pts(_BOX + [(4, 4, 1), (5, 5, 1)])
    ref, kr = oracle.cluster(s, d, q, 2, 2, 2.0, 4)
    lab, k, _ = oracle.fdbscan(s, d, q, 2, 2, 2.0, 4)
    assert kr == 1 and np.all(ref == 0)
    assert k == 2 and list(lab) == [0] * 8 + [1, 1, 1]


def test_no_representative_where_nothing_lies_off_the_origin():
    # all points share DM and SNR: only the time representatives exist, and a
    # lone pair below MinPts is noise in both
    s, d, q = [0, 1, 2, 3, 40, 41], [5] * 6, [7.0] * 6
    lab, k, nq = oracle.fdbscan(s, d, q, 1, 3, 1.0, 3)
    ref, kr = oracle.cluster(s, d, q, 1, 3, 1.0, 3)
    assert k == kr == 1 and np.array_equal(lab, ref) and list(lab) == [0, 0, 0, 0, -1, -1]


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_properties_against_exact_dbscan(seed):
    rng = np.random.default_rng(seed)
    n = 400
    s = rng.integers(0, 300, n)
    d = rng.integers(0, 40, n)
    q = rng.uniform(3, 9, n).astype(np.float32)
    order = np.lexsort((s, d))
    s, d, q = s[order], d[order], q[order]
    te, de, se, mp = 6, 3, 2.0, 4
    ref, kr = oracle.cluster(s, d, q, te, de, se, mp)
    lab, k, nq = oracle.fdbscan(s, d, q, te, de, se, mp)
    core = np.array([len(x) >= mp for x in oracle.cluster_neighbours(s, d, q, te, de, se)])
    assert core.any() and kr > 1
    assert np.all(lab[core] >= 0)                   # core points are never noise
    assert np.all(lab[ref < 0] < 0)                 # DBSCAN noise stays noise
    for c in range(k):                              # one FDBSCAN cluster's core points: one DBSCAN cluster
        assert len(set(ref[(lab == c) & core].tolist())) <= 1
    assert k >= kr and nq <= n


def test_empty():
    lab, k, nq = oracle.fdbscan([], [], [], 2, 1, 1.0, 3)
    assert lab.shape == (0,) and k == 0 and nq == 0


def test_fdbscan_agrees_with_dbscan_on_the_benchmark_list():
    """The clustering workload's detection list (640 DMs x 59434 samples,
    3-sigma background plus five pulse bow-ties; T_t = 16, DM_t = 4,
    SNR_t = 2, MinPts = 5): FDBSCAN finds the same 27 clusters as the exact
    DBSCAN, splits none and loses one border point of 2753."""
    from paper_1307_5700_amd import synth
    s, d, q = synth.detections(640, 59434, seed=1)
    ref, kr = oracle.cluster(s, d, q, 16, 4, 2.0, 5)
    lab, k, nq = oracle.fdbscan(s, d, q, 16, 4, 2.0, 5)
    assert k == kr == 27
    assert int((ref >= 0).sum()) == 2753
    lost = (ref >= 0) & (lab < 0)
    assert int(lost.sum()) == 1 and np.array_equal(lab[~lost], ref[~lost])
    assert nq < len(s)
