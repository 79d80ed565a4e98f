"""The serving engine (kkt_server_*) through the C ABI: requests of several patterns that
arrive together run concurrently on worker streams, replicas are created within the device
byte budget and evicted when other patterns need room, and every result is bitwise the
same as the same request served alone (one worker, one request at a time), with backward
error <= 1e-10 recomputed on the host by the oracle's residual."""
import numpy as np
import pytest

import kktgen
import oracle
import paper_2302_08656_amd as K
from test_gpu_parity import cuda

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def workload():
    specs = [kktgen.small(200, config_id=170, steps=4), kktgen.small(500, config_id=171, steps=4),
             kktgen.small(2000, config_id=172, steps=4)]
    seqs = [kktgen.make_sequence(s) for s in specs]
    rng = np.random.default_rng(np.random.SeedSequence([0, 170, 7, 0]))
    reqs = [(int(p), int(t), int(r)) for p, t, r in zip(rng.integers(0, 3, 24), rng.integers(0, 4, 24),
                                                         rng.integers(1, 4, 24))]
    return seqs, reqs


def serve(seqs, reqs, fp, inflight, budget, together):
    sv = K.KKTServer(hbm_budget=budget, max_inflight=inflight, max_nrhs=4)
    pids = [sv.add_pattern(q.n, q.rowptr, q.colind, q.values(0), factor_precision=fp) for q in seqs]
    vals = [[cuda(q.values(t)) for t in range(q.steps)] for q in seqs]
    outs, res = [], []
    tickets = []
    for p, t, r in reqs:
        q = seqs[p]
        b = cuda(np.stack([q.rhs(t, nrhs=r)[j] for j in range(r)]) if r > 1 else q.rhs(t))
        x = torch.empty_like(b)
        tk = sv.submit(pids[p], vals[p][t], b, x)
        if together:
            tickets.append((tk, x))
        else:
            res.append(sv.wait(tk))
            outs.append(x.cpu().numpy())
    for tk, x in tickets:
        res.append(sv.wait(tk))
        outs.append(x.cpu().numpy())
    st = sv.stats()
    sv.close()
    return outs, res, st


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_same_alone_and_in_the_mix(prec):
    print(f"[gpu] serving mix {prec}", flush=True)
    fp = K.FP32 if prec == "fp32" else K.FP64
    seqs, reqs = workload()
    # room for about two replicas of the largest pattern: the mix must evict
    budget = 60 << 20
    mix, res_m, st_m = serve(seqs, reqs, fp, 4, budget, True)
    alone, res_a, st_a = serve(seqs, reqs, fp, 1, budget, False)
    print(f"[gpu]   mix: {st_m}", flush=True)
    assert st_m["completed"] == len(reqs) and st_m["peak_bytes"] <= budget
    assert st_m["replicas_created"] > len(seqs) and st_m["evictions"] > 0
    for i, ((p, t, r), xm, xa, rm, ra) in enumerate(zip(reqs, mix, alone, res_m, res_a)):
        assert np.array_equal(xm, xa), (i, p, t, r)
        assert rm[0] == K.OK and ra[0] == K.OK, (i, rm, ra)
        q = seqs[p]
        X = xm.reshape(r, q.n)
        B = np.stack([q.rhs(t, nrhs=r)[j] for j in range(r)]) if r > 1 else q.rhs(t)[None]
        for j in range(r):
            _, berr = oracle.residual(q.n, q.rowptr, q.colind, q.values(t), X[j], B[j])
            assert berr <= 1e-10, (i, j, berr)
        assert [(f.iters, f.status) for f in rm[1]] == [(f.iters, f.status) for f in ra[1]]


def test_budget_and_argument_errors():
    print("[gpu] serving errors", flush=True)
    q = kktgen.make_sequence(kktgen.small(200, config_id=170, steps=2))
    sv = K.KKTServer(hbm_budget=1 << 20, max_inflight=2)
    with pytest.raises(K.KKTError) as e:             # one replica exceeds the budget
        sv.add_pattern(q.n, q.rowptr, q.colind, q.values(0))
    assert e.value.code == K.ERR_NOMEM
    sv.close()
    sv = K.KKTServer(max_inflight=2, max_nrhs=2)
    p = sv.add_pattern(q.n, q.rowptr, q.colind, q.values(0))
    b = cuda(np.stack([q.rhs(1)] * 3))
    with pytest.raises(K.KKTError) as e:             # more right-hand sides than max_nrhs
        sv.submit(p, cuda(q.values(1)), b, torch.empty_like(b))
    assert e.value.code == K.ERR_ARG
    sv.close()
