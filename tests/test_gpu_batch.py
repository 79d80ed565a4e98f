"""Batched refactorization (kkt_batch_*) and the schedule autotuner (kkt_autotune,
kkt_set_tuning) through the C ABI.

A batch runs, for each handle, exactly the blocks of that handle's own launches (only their
place in the merged launch differs), so each batched result must be bitwise equal to the
same system refactored alone; the autotuned and hand-set schedules change launch shapes and
rounding order only, so their factors are checked against the oracle under the entrywise
factor bound and their refined solutions under the backward-error target."""
import numpy as np
import pytest
import scipy.sparse as sp

import kktgen
import oracle
import paper_2302_08656_amd as K
from test_gpu_parity import check_factor_parity, cuda

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def mixed_specs():
    # three patterns (one repeated with another value set), sizes 150 to 1,200 buses
    return [kktgen.small(150, config_id=160, steps=3), kktgen.small(600, config_id=161, steps=3),
            kktgen.small(1200, config_id=162, steps=3), kktgen.small(600, config_id=161, steps=3)]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batch_bitwise_equal_to_alone(prec):
    print(f"[gpu] batch vs alone {prec}", flush=True)
    fp = K.FP32 if prec == "fp32" else K.FP64
    seqs = [kktgen.make_sequence(s) for s in mixed_specs()]
    alone = [K.KKTSolver(q.n, q.rowptr, q.colind, q.values(0), factor_precision=fp).bind() for q in seqs]
    inb = [K.KKTSolver(q.n, q.rowptr, q.colind, q.values(0), factor_precision=fp).bind() for q in seqs]
    batch = K.KKTBatch(inb)
    for t in range(3):
        # the repeated pattern takes another value set in the batch (step t + 1 mod 3)
        ts = [t, t, t, (t + 1) % 3]
        vals = [cuda(q.values(tt)) for q, tt in zip(seqs, ts)]
        rhs = [cuda(q.rhs(tt)) for q, tt in zip(seqs, ts)]
        batch.refactor(vals)
        xs, infos = batch.refine(rhs)
        for i, (q, sk) in enumerate(zip(seqs, alone)):
            sk.refactor(vals[i])
            x, info = sk.refine(rhs[i])
            fa, ra, ca = sk.export_factors()
            fb, rb, cb = inb[i].export_factors()
            assert np.array_equal(fa, fb) and np.array_equal(ra, rb) and np.array_equal(ca, cb), (t, i)
            assert np.array_equal(x.cpu().numpy(), xs[i].cpu().numpy()), (t, i)
            assert inb[i].refactor_status() == sk.refactor_status()
            assert (info[0].iters, info[0].status) == (infos[i].iters, infos[i].status)
            if prec == "fp64":
                _, berr = oracle.residual(q.n, q.rowptr, q.colind, q.values(ts[i]), xs[i].cpu().numpy(),
                                          q.rhs(ts[i]))
                assert infos[i].status == K.OK and berr <= 1e-10
    batch.close()


def test_batch_rejects_bad_input():
    print("[gpu] batch errors", flush=True)
    q = kktgen.make_sequence(kktgen.config(0))
    a = K.KKTSolver(q.n, q.rowptr, q.colind, q.values(0)).bind()
    f = K.KKTSolver(q.n, q.rowptr, q.colind, q.values(0), factor_precision=K.FP32).bind()
    u = K.KKTSolver(q.n, q.rowptr, q.colind, q.values(0))
    for group, code in (([a, a], K.ERR_ARG), ([a, f], K.ERR_ARG), ([a, u], K.ERR_STATE)):
        with pytest.raises(K.KKTError) as e:
            K.KKTBatch(group)
        assert e.value.code == code
    b = K.KKTBatch([a])
    a.bind()                                  # a new workspace: the batch is stale
    with pytest.raises(K.KKTError) as e:
        b.refactor([cuda(q.values(1))])
    assert e.value.code == K.ERR_STATE
    b.close()


TUNING_FIELDS = ("panel_max", "small_rows", "group", "wide256", "fuse_chains", "tiny_rows")


@pytest.mark.parametrize("tuning", [(16, 32, 16, 1, 1, 16), (8, 64, 32, 0, 1, 0), (32, 0, 8, 1, 0, 16),
                                    (32, 64, 32, 0, 0, 0), (32, 64, 32, 1, 1, 8)])
def test_set_tuning_parity(tuning):
    print(f"[gpu] tuned schedule {tuning}", flush=True)
    q = kktgen.make_sequence(kktgen.small(2000, config_id=147, steps=2))
    v0 = q.values(0)
    so = oracle.Symbolic(q.n, q.rowptr, q.colind, v0)
    sk = K.KKTSolver(q.n, q.rowptr, q.colind, v0)
    sk.set_tuning(*tuning)
    assert sk.tuning() == dict(zip(TUNING_FIELDS, tuning))
    sk.bind()
    for t in range(q.steps):
        v, b = q.values(t), q.rhs(t)
        sk.refactor(cuda(v))
        st, np_g = sk.refactor_status()
        lu_g, r_g, c_g = sk.export_factors()
        lu_o, r_o, c_o, np_o, _ = so.refactor(v)
        assert np.array_equal(r_g, r_o) and np_g == np_o
        At = sp.diags(r_o) @ q.scipy(t) @ sp.diags(c_o)
        check_factor_parity(so, lu_g, lu_o, np_o, oracle.EPS * abs(At).sum(axis=1).max())
        x, info = sk.refine(cuda(b))
        _, berr = oracle.residual(q.n, q.rowptr, q.colind, v, x.cpu().numpy(), b)
        assert info[0].status == K.OK and berr <= 1e-10


@pytest.mark.parametrize("spec", [kktgen.small(2000, config_id=147, steps=2), kktgen.config(1)],
                         ids=["grid2000", "grid25k"])
def test_tiny_items_bitwise(spec):
    # narrow items on 4-lane groups (tiny_rows 16, the default) or all on 16 lanes (0): the
    # same operations in the same order, so the factors agree bit for bit
    print(f"[gpu] tiny items on/off {spec.name}", flush=True)
    q = kktgen.make_sequence(spec)
    on = K.KKTSolver(q.n, q.rowptr, q.colind, q.values(0))
    off = K.KKTSolver(q.n, q.rowptr, q.colind, q.values(0))
    t = off.tuning()
    assert t["tiny_rows"] == 16
    off.set_tuning(t["panel_max"], t["small_rows"], t["group"], t["wide256"], t["fuse_chains"], 0)
    on.bind()
    off.bind()
    for step in (0, q.steps - 1):
        v = cuda(q.values(step))
        on.refactor(v)
        off.refactor(v)
        assert on.refactor_status() == off.refactor_status()
        lu_on, r_on, c_on = on.export_factors()
        lu_off, r_off, c_off = off.export_factors()
        assert np.array_equal(lu_on.view(np.uint64), lu_off.view(np.uint64)), step
        assert np.array_equal(r_on, r_off) and np.array_equal(c_on, c_off)
        b = cuda(q.rhs(step))
        x_on, _ = on.refine(b)
        x_off, _ = off.refine(b)
        assert torch.equal(x_on, x_off), step
    on.close()
    off.close()


def test_autotune_picks_a_valid_schedule():
    print("[gpu] autotune", flush=True)
    q = kktgen.make_sequence(kktgen.small(2000, config_id=147, steps=2))
    sk = K.KKTSolver(q.n, q.rowptr, q.colind, q.values(0)).bind()
    v = cuda(q.values(1))
    choice, ms = sk.autotune(v, reps=2)
    assert ms > 0 and choice["panel_max"] in (8, 16, 32) and choice == sk.tuning()
    with pytest.raises(K.KKTError) as e:           # unbound by the tuner
        sk.refactor(v)
    assert e.value.code == K.ERR_STATE
    sk.bind()
    sk.refactor(v)
    x, info = sk.refine(cuda(q.rhs(1)))
    _, berr = oracle.residual(q.n, q.rowptr, q.colind, q.values(1), x.cpu().numpy(), q.rhs(1))
    assert info[0].status == K.OK and berr <= 1e-10
