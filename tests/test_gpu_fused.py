"""kkt_refactor_refine (refactorization with the forward substitution beside it) against
kkt_refactor followed by kkt_refine, through the C ABI.

Both run the same kernels on the same items with the same arithmetic; the fused call only
changes when the forward items run (each once the columns it reads are factored and the
unknowns it reads are solved), so factors, x and info must be equal bit for bit.  The
separate calls are pinned to the oracle by the parity tests; the full-size case here also
recomputes the backward error with the oracle's residual.
"""
import numpy as np
import pytest

import kktgen
import oracle
import paper_2302_08656_amd as K

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def pair(q, **kw):
    v0 = q.values(0)
    sep = K.KKTSolver(q.n, q.rowptr, q.colind, v0, **kw).bind()
    fus = K.KKTSolver(q.n, q.rowptr, q.colind, v0, **kw).bind()
    return sep, fus


def same_step(q, t, sep, fus, alias=False):
    v = q.values(t)
    b = q.rhs(t)
    vd = cuda(v)
    sep.refactor(vd)
    xs, info_s = sep.refine(cuda(b))
    bd = cuda(b)
    xf, info_f = fus.refactor_refine(vd, bd, bd if alias else None)
    assert np.array_equal(xs.cpu().numpy(), xf.cpu().numpy()), t
    assert info_s[0] == info_f, (t, info_s[0], info_f)
    lu_s, r_s, c_s = sep.export_factors()
    lu_f, r_f, c_f = fus.export_factors()
    assert np.array_equal(lu_s, lu_f) and np.array_equal(r_s, r_f) and np.array_equal(c_s, c_f)
    return v, b, xf, info_f


CASES = [
    ("grid200", kktgen.config(0), {}),
    ("grid300_widening", kktgen.small(300, config_id=140, steps=3), {}),
    ("grid2000", kktgen.small(2000, config_id=147, steps=2), {}),
    ("grid2000_level_solves", kktgen.small(2000, config_id=147, steps=2), {"persistent_solve": 0}),
    ("grid2000_tickets", kktgen.small(2000, config_id=147, steps=2), {"persistent_solve": 2}),
    ("grid2000_tau1e-3", kktgen.small(2000, config_id=147, steps=2), {"tau": 1e-3}),
    ("grid3000_fp32", kktgen.small(3000, config_id=149, steps=2), {"factor_precision": K.FP32}),
    ("grid2000_chains", kktgen.small(2000, config_id=150, steps=2), {"fuse_chains": 1}),
]


@pytest.mark.parametrize("name,spec,kw", CASES, ids=[c[0] for c in CASES])
def test_fused_equals_refactor_then_refine(name, spec, kw):
    print(f"[gpu] fused refactor+refine {name}", flush=True)
    q = kktgen.make_sequence(spec)
    kw = {("pivot_tau" if k == "tau" else k): v for k, v in kw.items()}
    fc = kw.pop("fuse_chains", None)
    sep, fus = pair(q, **kw)
    if fc:
        for sk in (sep, fus):
            t = sk.tuning()
            sk.set_tuning(t["panel_max"], t["small_rows"], t["group"], t["wide256"], fc, t["tiny_rows"])
            sk.bind()
    for t in range(q.steps):
        v, b, x, info = same_step(q, t, sep, fus)
        assert info.status == K.OK
        _, berr = oracle.residual(q.n, q.rowptr, q.colind, v, x.cpu().numpy(), b)
        assert berr <= 1e-10, (t, berr)


def test_fused_replays_aliasing_rebind_and_fallbacks():
    print("[gpu] fused: replays, aliasing, rebind, profiler fallback", flush=True)
    q = kktgen.make_sequence(kktgen.small(2500, config_id=152, steps=4))
    sep, fus = pair(q)
    for t in range(4):                     # eager work of the other handle between replays
        same_step(q, t, sep, fus, alias=(t == 2))
    fus.profile(True)                      # one by one while profiling
    same_step(q, 1, sep, fus)
    fus.profile(False)
    fus.bind()                             # a new workspace drops the recording
    same_step(q, 3, sep, fus)
    same_step(q, 0, sep, fus)
    # refine again on the factors of the last calls (both of value set 0)
    b = cuda(q.rhs(0, nrhs=2))
    xa, ia = sep.refine(b)
    xb, ib = fus.refine(b)
    assert np.array_equal(xa.cpu().numpy(), xb.cpu().numpy()) and ia == ib
    # no graphs at all: the two calls one after the other
    nog = K.KKTSolver(q.n, q.rowptr, q.colind, q.values(0), graph_refactor=0).bind()
    same_step(q, 2, sep, nog)


def test_fused_nonfinite_reported():
    print("[gpu] fused: non-finite values", flush=True)
    q = kktgen.make_sequence(kktgen.small(2000, config_id=145))
    sep, fus = pair(q)
    v = q.values(1)
    v[q.nnz // 2] = np.nan
    with pytest.raises(K.KKTError) as e:
        fus.refactor_refine(cuda(v), cuda(q.rhs(1)))
    assert e.value.code == K.ERR_NONFINITE
    same_step(q, 1, sep, fus)              # recovers with finite values


def test_fused_full_size_grid70k():
    """The 70k-bus grid: fused equals separate bit for bit, backward error <= 1e-10 by the
    oracle's residual."""
    print("[gpu] fused full size grid70k", flush=True)
    q = kktgen.make_sequence(kktgen.config(2))
    sep, fus = pair(q)
    for t in (0, 1, 49):
        print(f"[gpu]   step {t}", flush=True)
        v, b, x, info = same_step(q, t, sep, fus)
        _, berr = oracle.residual(q.n, q.rowptr, q.colind, v, x.cpu().numpy(), b)
        assert info.status == K.OK and berr <= 1e-10, (t, berr, info)


def test_fused_on_scratch_binding():
    """A handle bound to the library's static array launches the fused levels one by one
    (no graph); results equal the separate calls on an ordinary binding."""
    print("[gpu] fused on the static scratch binding", flush=True)
    q = kktgen.make_sequence(kktgen.small(1500, config_id=153, steps=3))
    sep = K.KKTSolver(q.n, q.rowptr, q.colind, q.values(0)).bind()
    scr = K.KKTSolver(q.n, q.rowptr, q.colind, q.values(0)).bind_scratch(0)
    for t in range(3):
        same_step(q, t, sep, scr, alias=(t == 1))


def test_profiler_counts_every_level_launch():
    """The launch profiler brackets runs of level launches with one event pair but still
    counts each launch: per unit, the refactorization classes add up to the level count."""
    print("[gpu] launch profiler counts", flush=True)
    q = kktgen.make_sequence(kktgen.small(3000, config_id=149, steps=2))
    sk = K.KKTSolver(q.n, q.rowptr, q.colind, q.values(0)).bind()
    vd, bd = cuda(q.values(1)), cuda(q.rhs(1))
    for fused in (True, False):
        sk.profile(True)
        if fused:
            sk.refactor_refine(vd, bd)
        else:
            sk.refactor(vd)
            sk.refine(bd)
        pr = sk.profile_read()
        sk.profile(False)
        levels = sum(pr[c][0] for c in ("refactor_large", "refactor_medium", "refactor_w256", "refactor_small"))
        assert levels == sk.stats["gpu_levels_f"], (fused, pr)
        assert all(pr[c][1] > 0 for c in pr if pr[c][0] > 0), pr
