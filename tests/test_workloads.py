"""The seeded generators are deterministic and have the configured shapes."""
import math

import numpy as np

import workloads as W


def test_grids_and_manufactured_problem():
    u = W.manufactured_u(5, 2)
    assert u.shape == (33, 33) and u[0].max() == 0 and u[:, -1].max() == 0
    f = W.manufactured_f(5, 2)
    assert np.allclose(f, 2 * math.pi ** 2 * u)
    assert W.manufactured_u(3, 3).shape == (9, 9, 9)


def test_initial_guess_is_seeded():
    a = W.initial_guess(5, 2, 0)
    b = W.initial_guess(5, 2, 0)
    assert (a == b).all() and a[0].max() == 0 and np.abs(a).max() <= 1


def test_batch_trace_shape():
    t = W.batch_trace()
    assert len(t) == 4096
    assert {s.side for s in t} == {33, 65, 129, 257}
    dof = sum((s.side - 2) ** 2 for s in t)
    assert 80e6 < dof < 95e6
    assert t[0].modes.k.shape == (8, 2) and (t[0].modes.k >= 1).all() and (t[0].modes.k <= 8).all()
    assert W.batch_trace()[17].modes.a.tolist() == t[17].modes.a.tolist()


def test_serving_trace():
    t = W.serving_trace(2000)
    assert all(r.t_arrival > 0 for r in t)
    assert all(b.t_arrival > a.t_arrival for a, b in zip(t, t[1:]))
    for r in t:
        assert r.w in (8, 16, 24, 32)
        j = r.level
        assert r.side == (1 << j) + 1
        assert (6 <= j <= 10) if r.ndim == 2 else (5 <= j <= 7)
    rate = len(t) / t[-1].t_arrival
    assert 1700 < rate < 2300
