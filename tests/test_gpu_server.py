"""The request server: mixed 2D/3D requests of several sizes and widths run
concurrently in slots; every result equals, bit for bit, the same solve run
alone, whatever the slot count and however tight the memory budget (which
forces hierarchies to be evicted and re-created)."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import paper_2307_00124_amd as P
import workloads as W

pytestmark = pytest.mark.gpu


def requests(count, seed=9):
    g = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        ndim = 2 if g.random() < 0.5 else 3
        side = int(g.choice([9, 17, 33, 65] if ndim == 2 else [5, 9, 17]))
        w = int(g.choice([8, 16, 24, 32]))
        out.append((ndim, side, w, W.draw_sine_modes(g, ndim)))
    return out


def make(req):
    ndim, side, w, modes = req
    L = int(round(np.log2(side - 1)))
    prm = P.batch_params(ndim, L, w)
    rhs = [torch.from_numpy(np.ascontiguousarray(W.sine_f(j, modes))).cuda()
           for j in range(1, L + 1)]
    x = torch.zeros((side,) * ndim, dtype=torch.float64, device="cuda")
    return prm, rhs, x


def alone(prm, rhs):
    H = P.Hierarchy(prm)
    for j, f in enumerate(rhs, 1):
        H.set_rhs(j, f)
    H.fmg()
    return P.bfp_vec_to_f64(H.get_vec(prm.L, 0))


def run_server(S, items):
    torch.cuda.synchronize()   # inputs ready before the server's streams read them
    tickets = [S.submit(prm, rhs, x) for prm, rhs, x in items]
    pending = dict(enumerate(tickets))
    for _ in range(2_000_000):
        for i in list(pending):
            r = S.poll(pending[i])
            if r is not None:
                assert r[0] == 0
                del pending[i]
        if not pending:
            break
    assert not pending, "requests did not finish"
    torch.cuda.synchronize()


@pytest.mark.parametrize("slots,tight", [(4, False), (1, False), (3, True)])
def test_server_results_equal_solo(slots, tight):
    reqs = requests(16)
    items = [make(r) for r in reqs]
    # a tight budget holds about two of the largest hierarchies, so most
    # requests evict an idle hierarchy and create their own
    biggest = max(P.lib.mg_hierarchy_bytes(P.C.byref(prm)) for prm, _, _ in items)
    budget = 2 * biggest + 4096 if tight else 512 << 20
    S = P.Server(budget, max_slots=slots)
    run_server(S, items)
    for (prm, rhs, x), r in zip(items, reqs):
        ref = alone(prm, rhs)
        assert torch.equal(x, ref), r[:3]
    q, running, resident = S.stats()
    assert q == 0 and running == 0 and resident <= budget


def test_server_errors():
    S = P.Server(1 << 20, max_slots=2, max_queue=2)
    prm, rhs, x = make((2, 257, 16, W.draw_sine_modes(np.random.default_rng(1), 2)))
    t = S.submit(prm, rhs, x)           # needs more than the 1 MiB budget
    with pytest.raises(P.BFPError) as e:
        S.poll(t)
    assert e.value.code == P.abi.BFP_ENOMEM
    with pytest.raises(P.BFPError):
        S.poll(12345)


def test_graph_replays_match_eager_with_eager_work_between():
    """A resident hierarchy's captured solve replayed several times, with
    eager library work and synchronizations in between, matches the eager
    solve every time."""
    reqs = requests(3, seed=4)
    items = [make(r) for r in reqs]
    refs = [alone(prm, rhs) for prm, rhs, _ in items]
    S = P.Server(256 << 20, max_slots=1)
    for rep in range(4):
        for k, (prm, rhs, x) in enumerate(items):
            x.zero_()
            torch.cuda.synchronize()   # the server's streams do not wait on torch's
            run_server(S, [(prm, rhs, x)])
            assert torch.equal(x, refs[k]), (rep, k)
            # eager work between replays: a solve of another request
            assert torch.equal(alone(*items[(k + 1) % 3][:2]), refs[(k + 1) % 3])
            torch.cuda.synchronize()


def test_server_large_requests_equal_solo():
    """The request sizes of the serving trace's upper end (513^2, 1025^2,
    65^3, 129^3), whose coarse levels the server runs in its executor up to
    its larger point limit: each result equals the solve run alone."""
    g = np.random.default_rng(31)
    reqs = [(2, 513, 16), (2, 1025, 16), (3, 65, 16), (3, 129, 16), (2, 1025, 32), (3, 129, 8)]
    reqs = [(nd, side, w, W.draw_sine_modes(g, nd)) for nd, side, w in reqs]
    items = [make(r) for r in reqs]
    S = P.Server(4 << 30, max_slots=3, exec_max_points=70000)
    run_server(S, items)
    for (prm, rhs, x), r in zip(items, reqs):
        assert torch.equal(x, alone(prm, rhs)), r[:3]
