"""The allocation-free binding (kkt_bind_scratch: the workspace is the library's static
device array) against the ordinary binding (kkt_bind: a caller workspace), through the C
ABI.  The two run the same kernels on the same inputs, so the factors, scale factors, the
plain solve and the refined solution must be bitwise equal.  Two calls in a row, the second
on a smaller system, which reuses the array that the first left behind."""
import numpy as np
import pytest

import kktgen
import paper_2302_08656_amd as K

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def unit(sk, q, t):
    v, b = cuda(q.values(t)), cuda(q.rhs(t))
    sk.refactor(v)
    x0 = sk.solve(b).cpu().numpy()
    x, info = sk.refine(b)
    lu, r, c = sk.export_factors()
    return lu, r, c, x0, x.cpu().numpy(), info[0]


def test_scratch_bind_matches_workspace_bind():
    prev = None
    # a 2,000-bus grid (25 MiB of workspace), then a 200-bus grid (2.6 MiB)
    for buses, cid in ((2000, 147), (200, 145)):
        print(f"[gpu] scratch binding, {buses}-bus grid", flush=True)
        q = kktgen.make_sequence(kktgen.small(buses, config_id=cid, steps=3))
        v0 = q.values(0)
        ref = K.KKTSolver(q.n, q.rowptr, q.colind, v0).bind(0)
        scr = K.KKTSolver(q.n, q.rowptr, q.colind, v0)
        assert scr.workspace_bytes(1) <= K.SCRATCH_BYTES
        torch.cuda.synchronize()
        before = torch.cuda.memory_allocated()
        scr.bind_scratch(0)
        assert torch.cuda.memory_allocated() == before
        if prev is not None:
            # the previous holder of the array lost its binding
            with pytest.raises(K.KKTError) as e:
                prev.refactor(cuda(q0.values(0)))
            assert e.value.code == K.ERR_STATE
        for t in (1, 2):
            a, b = unit(ref, q, t), unit(scr, q, t)
            for k, (ga, gb) in enumerate(zip(a[:5], b[:5])):
                assert np.array_equal(ga, gb), (buses, t, k)
            assert (a[5].iters, a[5].status, a[5].berr, a[5].perturbed_pivots) == \
                (b[5].iters, b[5].status, b[5].berr, b[5].perturbed_pivots)
            assert b[5].status == K.OK and b[5].berr <= 1e-10
        ref.close()
        prev, q0 = scr, q
    prev.close()
