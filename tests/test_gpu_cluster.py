"""DBSCAN clustering of detections (Sec. 2.3) on the GPU against the
oracle: labels and cluster counts bit-exact (the result is a function of
the input alone), on random point sets over several extents and MinPts,
chains and dense blobs that stress the union-find, degenerate extents, the
empty list, and the 640-DM x 59434-sample detection list the cluster bench
times."""
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
    labels, nc = A.cluster_candidates(buf, len(rec), ndms, te, de, se, mp)
    torch.cuda.synchronize()
    return labels.cpu().numpy(), int(nc.item())


def _check(rec, ndms, te, de, se, mp):
    got, k = _gpu(rec, ndms, te, de, se, mp)
    want, kw = oracle.cluster(rec["sample"], rec["dm_index"], rec["snr"], te, de, se, mp)
    assert k == kw
    assert np.array_equal(got, want)
    return k


def _random(n, seed, ns=400, nd=40):
    rng = np.random.default_rng(seed)
    key = rng.choice(ns * nd, size=n, replace=False)
    d, s = key // ns, key % ns
    q = (rng.integers(24, 48, n) * 0.25).astype(np.float32)
    return _records(s, d, q)


@pytest.mark.parametrize("te,de,se,mp", [(4, 2, 0.5, 3), (3, 1, 0.75, 4), (10, 3, 2.0, 5), (0, 0, 0.0, 1),
                                         (2, 0, 100.0, 2), (50, 10, 1.0, 12)])
@pytest.mark.parametrize("seed", [1, 2])
def test_random_sets_match_oracle(te, de, se, mp, seed):
    _check(_random(3000, seed), 40, te, de, se, mp)


def test_long_chain_is_one_cluster():
    n = 20000
    rec = _records(np.arange(n), np.zeros(n, np.int32), np.full(n, 5.0, np.float32))
    assert _check(rec, 1, 1, 0, 0.0, 3) == 1


def test_dense_blob_and_zigzag():
    rng = np.random.default_rng(7)
    key = rng.choice(64 * 64, size=3000, replace=False)
    rec = _records(key % 64, key // 64, rng.uniform(3, 4, 3000).astype(np.float32))
    assert _check(rec, 64, 2, 2, 1.0, 4) >= 1
    # a zigzag over DM rows: links only through alternating rows
    s = np.arange(5000)
    _check(_records(s, (s % 2) * 3, np.full(5000, 6.0, np.float32)), 4, 1, 3, 0.0, 2)


def test_empty_and_single():
    assert _gpu(_records(np.zeros(0, np.int64), np.zeros(0, np.int32), np.zeros(0, np.float32)),
                10, 1, 1, 1.0, 1)[1] == 0
    assert _check(_records([5], [3], [7.0]), 10, 1, 1, 1.0, 1) == 1
    assert _check(_records([5], [3], [7.0]), 10, 1, 1, 1.0, 2) == 0


def test_bench_detection_list():
    """The bench input: a 640-DM x 59434-sample detection list (background
    at the density of a 3-sigma pass and five pulse bow-ties)."""
    s, d, q = synth.detections(640, 59434, seed=1)
    rec = _records(s, d, q)
    assert len(rec) > 50000
    assert _check(rec, 640, 16, 4, 2.0, 5) > 5
