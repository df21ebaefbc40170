import hashlib

import numpy as np

from paper_2007_01088_amd.synth import make_inputs, perturb_t2, sample_triples


def _h(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def test_deterministic_and_symmetric():
    a = make_inputs(4, 20, 60)
    b = make_inputs(4, 20, 60)
    for key in ("eps", "L", "t1", "t2"):
        assert _h(a[key]) == _h(b[key])
    assert _h(make_inputs(4, 20, 60, tag=1)["t2"]) != _h(a["t2"])
    L, t2, eps = a["L"], a["t2"], a["eps"]
    assert np.array_equal(L, L.transpose(0, 2, 1))
    assert np.array_equal(t2, t2.transpose(1, 0, 3, 2))
    assert np.all(eps[:4] < -0.49) and np.all(eps[:4] >= -2.0)
    assert np.all(eps[4:] > 0.19) and np.all(eps[4:] <= 3.0)
    assert np.all(np.diff(eps[:4]) >= 0) and np.all(np.diff(eps[4:]) >= 0)
    assert 0.04 < L.std() < 0.06 and 0.007 < t2.std() < 0.013


def test_perturb_and_sample():
    a = make_inputs(5, 8, 10)
    p = perturb_t2(a["t2"], seed=3)
    assert np.array_equal(p, p.transpose(1, 0, 3, 2))
    assert 0 < np.abs(p - a["t2"]).max() < 1e-3
    s = sample_triples(6, 10, seed=1)
    assert s.shape == (10, 3) and s.dtype == np.int32
    assert np.all(s[:, 0] >= s[:, 1]) and np.all(s[:, 1] >= s[:, 2])
    assert not np.any((s[:, 0] == s[:, 1]) & (s[:, 1] == s[:, 2]))
    assert len({tuple(t) for t in s}) == 10


def test_left_inputs_deterministic_and_symmetric():
    from paper_2007_01088_amd.synth import make_left_inputs
    a = make_left_inputs(4, 9)
    b = make_left_inputs(4, 9)
    assert a["omega"] == b["omega"] and 0.2 <= a["omega"] <= 0.6
    for key in ("l1", "l2"):
        assert _h(a[key]) == _h(b[key])
    assert _h(make_left_inputs(4, 9, tag=1)["l2"]) != _h(a["l2"])
    assert np.array_equal(a["l2"], a["l2"].transpose(1, 0, 3, 2))
    # omega stays below every triples excitation of make_inputs' orbital energies
    eps = make_inputs(4, 9, 12)["eps"]
    assert a["omega"] < 3 * eps[4:].min() - 3 * eps[:4].max()
