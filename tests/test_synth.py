"""Seeded generator: determinism, shapes and the structure of the workloads."""
import numpy as np

from paper_2401_12890_amd import synth


def test_deterministic_and_seeded():
    a = synth.generate("c1")
    b = synth.generate("c1")
    assert a.m.tobytes() == b.m.tobytes() and a.K.tobytes() == b.K.tobytes()
    c = synth.generate("c1", seed=11)
    assert not np.array_equal(a.m, c.m)


def test_shapes_and_dictionary_structure():
    p = synth.generate("c1")
    assert p.K.shape == (30, 100) and p.m.shape == (1024, 30) and p.grid == (32, 32, 1)
    # b = 0 rows depend only on TE/T2; the first spectral axis is major in q
    K = p.K
    assert np.allclose(K[0].reshape(10, 10), K[0].reshape(10, 10)[0][None, :])
    assert np.all(K > 0) and np.all(K <= 1)
    # spectral blobs sum to one; fields are >= 0.05
    assert np.allclose(p.meta["blobs"].sum(axis=1), 1.0)
    assert p.meta["fields"].min() >= 0.05


def test_crop_and_fingerprinting_dictionary():
    p = synth.generate("c2", grid=(6, 5, 4))
    assert p.K.shape == (60, 1600) and p.m.shape == (120, 60)
    q = synth.generate("c3", grid=(4, 4, 2))
    assert q.K.shape == (1000, 1024) and q.m.shape == (32, 1000)
    assert np.isfinite(q.K).all() and (q.K < 0).any() and (q.K > 0).any()
