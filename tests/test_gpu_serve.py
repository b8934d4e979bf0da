"""The serving loop: resident factors under a memory budget, continuous
batching of refinement steps across requests of different operators and
right-hand side counts.  Each result must be the same bits alone and in the
mix, reach the residual target, and the budget must force evictions."""
import numpy as np
import pytest

import workloads as W
from oracle import direct

pytestmark = pytest.mark.gpu


def _op(acr, st):
    return acr.Operator.from_arrays(st.nx, st.ny, *st.arrays())


def _problems():
    return [(W.poisson(128), 32, 1e-8), (W.varkappa(128), 32, 1e-8), (W.convdiff(96, 40), 24, 1e-7),
            (W.varkappa(256), 64, 1e-6), (W.poisson(64, 33), 16, 1e-8)]


def test_serve_alone_equals_in_mix(gpu):
    import torch
    probs = _problems()
    srv = gpu.Server(memory_budget=8 << 30, tol=1e-10, maxit=40)
    ids = [srv.add_operator(_op(gpu, st), leaf, eps, "mixed") for st, leaf, eps in probs]
    rng = np.random.default_rng(W.seed_for(5, 1))
    # the request under test, alone (its operator factored first, nothing else running)
    st0 = probs[3][0]
    b0 = torch.from_numpy(W.rhs(st0.n, 5, seed=W.seed_for(5, 2))).cuda()
    x_alone, its_a, rel_a, _ = srv.wait(srv.submit(ids[3], b0))
    # the same request in a mix of 40 requests over every operator, 1..12 right-hand sides
    rids, refs = [], []
    for k in range(40):
        if k == 17:
            rids.append(srv.submit(ids[3], b0))
            refs.append(("test", None))
            continue
        o = int(rng.integers(0, len(probs)))
        st = probs[o][0]
        b = torch.from_numpy(W.rhs(st.n, int(rng.integers(1, 13)), seed=W.seed_for(5, 100 + k))).cuda()
        rids.append(srv.submit(ids[o], b))
        refs.append((o, b))
    for rid, (o, b) in zip(rids, refs):
        x, its, rel, lat = srv.wait(rid)
        assert rel <= 1e-10
        if o == "test":
            assert np.array_equal(x.cpu().numpy(), x_alone.cpu().numpy()), "result differs in the mix"
            assert its == its_a
        else:
            st = probs[o][0]
            assert direct.residual(st, x.cpu().numpy(), b.cpu().numpy()) <= 1e-10
    s = srv.stats()
    print("serve stats:", {k: round(v, 3) if isinstance(v, float) else v for k, v in s.items()})
    assert s["requests"] == 41 and s["steps"] > 0
    srv.close()


def test_serve_memory_budget_evicts(gpu):
    import torch
    probs = _problems()
    # budget below the sum of the factors: every operator fits alone, not all together
    srv = gpu.Server(memory_budget=40 << 20, tol=1e-10, maxit=40)
    ids = [srv.add_operator(_op(gpu, st), leaf, eps, "mixed") for st, leaf, eps in probs]
    rids = []
    for rep in range(3):
        for o, (st, leaf, eps) in enumerate(probs):
            b = torch.from_numpy(W.rhs(st.n, 2, seed=W.seed_for(5, 300 + 10 * rep + o))).cuda()
            rids.append((o, b, srv.submit(ids[o], b)))
    for o, b, rid in rids:
        x, its, rel, lat = srv.wait(rid)
        assert direct.residual(probs[o][0], x.cpu().numpy(), b.cpu().numpy()) <= 1e-10
    s = srv.stats()
    print("budget stats:", s)
    assert s["evictions"] > 0
    assert s["peak_resident_bytes"] <= (40 << 20) or s["factorizations"] >= len(probs)
    srv.close()


def test_serve_not_converged_and_errors(gpu):
    import torch
    st = W.varkappa(64)
    srv = gpu.Server(memory_budget=1 << 30, tol=1e-30, maxit=2)
    oid = srv.add_operator(_op(gpu, st), 16, 1e-6, "mixed")
    b = torch.from_numpy(W.rhs(st.n, 1)).cuda()
    rid = srv.submit(oid, b)
    with pytest.raises(gpu.ACRError) as ei:
        srv.wait(rid)
    assert ei.value.name == "ACR_ERR_NOT_CONVERGED"
    with pytest.raises(gpu.ACRError) as ei:
        srv.submit(7, b)
    assert ei.value.name == "ACR_ERR_INVALID_ARG"
    srv.close()
