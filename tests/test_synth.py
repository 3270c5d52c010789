"""The seeded input generator: determinism, chunked rendering and storage."""
import numpy as np

import oracle
from paper_1307_5700_amd import synth


def test_deterministic_and_seed_sensitive():
    b = synth.plain_single_beam()
    s = oracle.delay_table(**b.plan_kwargs())
    x1, x2 = synth.render(b, s), synth.render(b, s)
    assert np.array_equal(x1, x2)
    b.seed = 99
    assert not np.array_equal(synth.render(b, s), x1)


def test_chunks_agree_with_whole():
    b = synth.paper_beam(dtype="u8", nsamps=16384)
    s = oracle.delay_table(**b.plan_kwargs())
    whole = synth.render(b, s)
    part = synth.render(b, s, nsamps=5000, sample0=7000)
    assert np.array_equal(part, whole[:, 7000:12000])


def test_storage_recipes():
    v = np.array([[-9.0, -0.03, 0.0, 0.03125, 7.9, 20.0]], dtype=np.float32)
    assert list(synth.quantise(v, "u8")[0]) == [0, 128, 128, 128, 254, 255]
    h = synth.quantise(v, "f16")
    assert h.dtype == np.float16 and np.array_equal(h.astype(np.float32), v.astype(np.float16).astype(np.float32))
    assert synth.quantise(v, "f32").dtype == np.float32


def test_workload_shapes():
    assert synth.paper_beam().nchans == 1024 and synth.paper_beam().ndms == 640
    beams = synth.batch_beams()
    assert len(beams) == 8 and {b.dtype for b in beams} == {"u8"}
    assert sorted({b.nchans for b in beams}) == [512, 768, 1024, 1536, 2048]
    for b in beams:
        s = oracle.delay_table(**b.plan_kwargs())
        assert s.max() < b.nsamps
        for p in b.pulses:
            assert p.t0 + p.width <= b.nsamps - s.max()
