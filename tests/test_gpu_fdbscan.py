"""FDBSCAN (Sec. 2.3, expansion from representative points) on the GPU
against the oracle's sequential FDBSCAN: labels, cluster count and number
of region queries exact, on the hand examples where FDBSCAN equals DBSCAN,
loses a border point or splits a cluster, on random point sets over several
extents and MinPts, on the empty list, and on the 640-DM x 59434-sample
detection list the cluster bench times (where it loses one border point of
the exact DBSCAN's 2753)."""
import numpy as np
import pytest
import torch

import oracle
from paper_1307_5700_amd import synth

from gpu_util import api

pytestmark = pytest.mark.gpu


def _records(s, d, q):
    A = api()
    order = np.lexsort((s, d))
    rec = np.zeros(len(s), A.CANDIDATE_DTYPE)
    rec["dm_index"] = np.asarray(d)[order]
    rec["sample"] = np.asarray(s)[order]
    rec["snr"] = np.asarray(q, np.float32)[order]
    return rec


def _gpu(rec, ndms, te, de, se, mp):
    A = api()
    buf = torch.from_numpy(rec.view(np.uint8).copy()).cuda() if len(rec) else torch.zeros(1, dtype=torch.uint8,
                                                                                          device="cuda")
    labels, nc, nq = A.fdbscan_candidates(buf, len(rec), ndms, te, de, se, mp)
    torch.cuda.synchronize()
    return labels.cpu().numpy(), int(nc.item()), int(nq.item())


def _check(rec, ndms, te, de, se, mp):
    got, k, nq = _gpu(rec, ndms, te, de, se, mp)
    want, kw, nqw = oracle.fdbscan(rec["sample"], rec["dm_index"], rec["snr"], te, de, se, mp)
    assert k == kw
    assert nq == nqw
    assert np.array_equal(got, want)
    return got, k


# a core point A at the origin with six points on the border of its box, an
# interior core point B = (1, 1, 1) and X = (3, 3, 1) within B's box only
_BOX = [(0, 0, 0), (2, 0, 0), (-2, 0, 0), (0, 2, 0), (0, -2, 0), (0, 0, 2), (0, 0, -2), (1, 1, 1), (3, 3, 1)]


def _box(p):
    a = np.array(p, dtype=np.float64)
    return _records((a[:, 0] + 10).astype(np.int64), (a[:, 1] + 10).astype(np.int64),
                    (a[:, 2] + 7).astype(np.float32))


def test_blobs_equal_dbscan():
    rec = _records([0, 1, 2, 10, 11, 12, 50], [0, 0, 0, 5, 5, 5, 9], [7, 7, 7, 8, 8, 8, 9])
    got, k = _check(rec, 10, 2, 1, 1.0, 3)
    assert k == 2


def test_chain_walked_by_its_end_points():
    t = np.arange(0, 22, 2)
    got, k = _check(_records(t, np.zeros_like(t), np.full(t.shape, 7.0)), 1, 2, 0, 1.0, 3)
    assert k == 1 and np.all(got == 0)


def test_point_reachable_only_through_an_interior_core_point_is_lost():
    rec = _box(_BOX)
    got, k = _check(rec, 16, 2, 2, 2.0, 4)
    assert k == 1 and (got < 0).sum() == 1


def test_cluster_reached_through_an_interior_core_point_is_split():
    got, k = _check(_box(_BOX + [(4, 4, 1), (5, 5, 1)]), 16, 2, 2, 2.0, 4)
    assert k == 2


def test_no_representative_where_nothing_lies_off_the_origin():
    got, k = _check(_records([0, 1, 2, 3, 40, 41], [5] * 6, [7.0] * 6), 6, 1, 3, 1.0, 3)
    assert k == 1


@pytest.mark.parametrize("te,de,se,mp", [(6, 3, 2.0, 4), (4, 2, 0.5, 3), (10, 3, 2.0, 5), (0, 0, 0.0, 1),
                                         (50, 10, 1.0, 12)])
@pytest.mark.parametrize("seed", [0, 1])
def test_random_sets_match_oracle(te, de, se, mp, seed):
    rng = np.random.default_rng(seed)
    n = 1500
    s = rng.integers(0, 600, n)
    d = rng.integers(0, 40, n)
    q = (rng.integers(12, 36, n) * 0.25).astype(np.float32)
    _check(_records(s, d, q), 40, te, de, se, mp)


def test_empty():
    A = api()
    got, k, nq = _gpu(np.zeros(0, A.CANDIDATE_DTYPE), 8, 2, 1, 1.0, 3)
    assert got.shape == (0,) and k == 0 and nq == 0


def test_benchmark_detection_list():
    s, d, q = synth.detections(640, 59434, seed=1)
    rec = _records(s, d, q)
    got, k = _check(rec, 640, 16, 4, 2.0, 5)
    exact, ke = oracle.cluster(rec["sample"], rec["dm_index"], rec["snr"], 16, 4, 2.0, 5)
    assert k == ke == 27
    lost = (exact >= 0) & (got < 0)
    assert int(lost.sum()) == 1 and np.array_equal(got[~lost], exact[~lost])
