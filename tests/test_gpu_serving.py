"""The serving loop: interleaved walk queries and update batches give, for every request, the
result of issuing the same requests one by one (each query sees exactly the batches submitted
before it), whatever the overlap on the device.  Checked against direct calls on a second device
graph and against the oracle."""
import random

import numpy as np
import pytest
import torch

import oracle as O
import synth

pytestmark = pytest.mark.gpu


def B():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2504_10233_amd as B_
    return B_


def make_requests(n, m_live, rng, count=48):
    reqs = []
    for i in range(count):
        if rng.random() < 0.2:
            k = rng.randrange(1, 300)
            ins = [(rng.randrange(n), rng.randrange(n), rng.randrange(1, 1 << 16)) for _ in range(k // 2)]
            dels = [rng.choice(m_live) for _ in range(k - k // 2)]
            reqs.append(("update", ins, dels))
        else:
            nw = int(10 ** rng.uniform(0, 3.3))
            reqs.append(("walk", [rng.randrange(n) for _ in range(nw)], rng.randrange(5, 81),
                         rng.getrandbits(63), rng.getrandbits(40)))
    return reqs


def arrays(ins, dels):
    a = np.array([x[0] for x in ins], np.int64); b = np.array([x[1] for x in ins], np.int64)
    c = np.array([x[2] for x in ins], np.int64)
    d = np.array([x[0] for x in dels], np.int64); e = np.array([x[1] for x in dels], np.int64)
    return a, b, c, d, e


@pytest.mark.parametrize("inflight,budget,batch", [(4, 0, 8), (1, 0, 1), (8, 1, 32), (2, 0, 32), (1, 0, 32)])
def test_serving_results_equal_sequential(inflight, budget, batch):
    b = B()
    c = synth.config_c1()
    n = c["n"]
    src, dst, w = c["src"].numpy(), c["dst"].numpy(), c["w"].numpy()
    rng = random.Random(inflight * 7 + budget)
    live = list(zip(src.tolist(), dst.tolist()))
    reqs = make_requests(n, live, rng)
    g1 = b.Graph(n, torch.from_numpy(src), torch.from_numpy(dst), torch.from_numpy(w))
    srv = b.Server(g1, max_inflight=inflight, hbm_budget_bytes=budget, max_batch=batch)
    tickets = []
    for r in reqs:
        if r[0] == "walk":
            tickets.append(srv.submit_walk(np.array(r[1]), r[2], r[3], r[4]))
        else:
            tickets.append(srv.submit_update(*arrays(r[1], r[2])))
    results = [srv.wait(t) for t in tickets]
    srv.close()
    # the same requests one by one, on a second device graph and on the oracle
    g2 = b.Graph(n, torch.from_numpy(src), torch.from_numpy(dst), torch.from_numpy(w))
    og = O.Graph(n, src, dst, w)
    epoch = 0
    for r, (paths, info) in zip(reqs, results):
        assert info["status"] == 0 and info["epoch"] == epoch and info["latency_us"] > 0
        if r[0] == "walk":
            starts = np.array(r[1])
            p2, s2 = g2.walk(starts, r[2], r[3], base=r[4])
            op, os_ = og.deepwalk(starts, r[2], r[3], base=r[4])
            assert np.array_equal(paths, op)
            assert np.array_equal(p2.cpu().numpy().view(np.uint32), op)
            assert info["steps"] == os_ == int(s2.item())
        else:
            a = arrays(r[1], r[2])
            s2 = g2.update(*[torch.from_numpy(x) for x in a])
            so = og.update(*a)
            assert info["updates_applied"] == so["inserted"] + so["deleted"] == s2["inserted"] + s2["deleted"]
            assert info["updates_not_found"] == so["not_found"]
            epoch += 1
    assert np.array_equal(g1.export(), og.dump())
    assert np.array_equal(g2.export(), og.dump())
    assert np.array_equal(g1.export_index(), og.index_dump())
    assert np.array_equal(g2.export_index(), og.index_dump())


def test_serving_concurrent_queries_overlap_and_finish():
    b = B()
    c = synth.config_c1()
    g = b.Graph(c["n"], c["src"], c["dst"], c["w"])
    srv = b.Server(g, max_inflight=6)
    starts = np.arange(1000)
    ts = [srv.submit_walk(starts, 80, 100 + i, base=i * 1000) for i in range(24)]
    outs = [srv.wait(t) for t in ts]
    srv.close()
    og = O.Graph(c["n"], c["src"].numpy(), c["dst"].numpy(), c["w"].numpy())
    for i, (paths, info) in enumerate(outs):
        op, _ = og.deepwalk(starts, 80, 100 + i, base=i * 1000)
        assert np.array_equal(paths, op)
