"""Mixed precision on the GPU (factor_precision = FP32) against the FP64 oracle, through the
C ABI.

The FP32 path rounds the scaled values A~ = R A C to FP32 once (|dA| <= u32 |A~|), factors
them in FP32 with the same pivot order and pattern, and the oracle factors A~ in FP64 with
the same tiny-pivot factor (2^-26).  Each factorization satisfies the entrywise LU bound for
its own arithmetic, so

    |L^U^ - L U| <= g32 |L^||U^| + g64 |L||U| + u32 |A~| + eta      (off the diagonal)

with g = (m + 2) u, m the longest column, and eta = (m + 2) 2^-126 for FP32 underflow; on
the diagonal a pivot replaced by either side adds at most eps ||A~||_inf each, and the two
sides may replace different pivots (they compute them in different precisions), so the
diagonal may exceed the bound by up to twice that (eps the tiny-pivot factor).  The triangular solves read the FP32
factors into FP64 sums, so one solve application is checked against the FP64 componentwise
solve bound with the widened factors.  Refinement (FP64 residuals, orthogonalisation and
update) must reach a backward error <= 1e-10 on the original A, recomputed on the host.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import kktgen
import oracle
import paper_2302_08656_amd as K
from test_gpu_parity import berr_close, check_solve_componentwise, cuda, factors

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

U64 = np.finfo(np.float64).eps / 2
U32 = np.finfo(np.float32).eps / 2
EPS32 = 2.0 ** -26   # the FP32 path's default tiny-pivot factor


def setup32(q, **kw):
    v0 = q.values(0)
    so = oracle.Symbolic(q.n, q.rowptr, q.colind, v0)
    sk = K.KKTSolver(q.n, q.rowptr, q.colind, v0, factor_precision=K.FP32, **kw).bind()
    return so, sk


def check_factor_bound32(so, A_t, lu_g, lu_o, thresh):
    """A_t: the scaled matrix R A C (scipy, permuted back by the caller's P, Q below)."""
    n = so.n
    Lg, Ug = factors(n, so.colptr, so.rowidx, lu_g)
    Lo, Uo = factors(n, so.colptr, so.rowidx, lu_o)
    m = int(np.diff(so.colptr).max())
    g32, g64 = (m + 2) * U32, (m + 2) * U64
    eta = (m + 2) * 2.0 ** -126
    PAQ = abs(A_t[so.P][:, so.Q])
    D = abs(Lg @ Ug - Lo @ Uo)
    B = g32 * (abs(Lg) @ abs(Ug)) + g64 * (abs(Lo) @ abs(Uo)) + U32 * PAQ
    E = (D - B).tocsr()
    E.data -= eta
    E.data[E.data < 0] = 0
    E.eliminate_zeros()
    excess = E.diagonal()
    off = E - sp.diags(excess)
    off.eliminate_zeros()
    assert off.nnz == 0 or off.max() == 0, f"off-diagonal excess {off.max():.3e}"
    assert np.all(excess <= 2 * thresh * (1 + 1e-6)), f"diagonal excess {excess.max():.3e}"
    # the FP32 factors are genuinely FP32 values (widened exactly by the export)
    assert np.array_equal(lu_g, lu_g.astype(np.float32).astype(np.float64))


CASES32 = [
    ("grid200", kktgen.config(0), {}),
    ("grid300_widening", kktgen.small(300, config_id=140, steps=4), {}),
    ("grid2000_vector_fma", kktgen.small(2000, config_id=147, steps=2), {"dense_mfma": 0}),
    ("grid2000_mfma", kktgen.small(2000, config_id=147, steps=2), {}),
    ("grid2000_level_solves", kktgen.small(2000, config_id=147, steps=2), {"persistent_solve": 0}),
    ("grid2000_tau1e-3", kktgen.small(2000, config_id=147, steps=2), {"pivot_tau": 1e-3}),
]


@pytest.mark.parametrize("name,spec,kw", CASES32, ids=[c[0] for c in CASES32])
def test_fp32_refactor_and_refine(name, spec, kw):
    print(f"[gpu] fp32 {name}", flush=True)
    q = kktgen.make_sequence(spec)
    v0 = q.values(0)
    so = oracle.Symbolic(q.n, q.rowptr, q.colind, v0, **({"tau": kw["pivot_tau"]} if "pivot_tau" in kw else {}))
    sk = K.KKTSolver(q.n, q.rowptr, q.colind, v0, factor_precision=K.FP32, **kw).bind()
    for t in range(q.steps):
        v, b = q.values(t), q.rhs(t)
        vd = cuda(v)
        sk.refactor(vd)
        st, np_g = sk.refactor_status()
        lu_g, r_g, c_g = sk.export_factors()
        lu_o, r_o, c_o, np_o, _ = so.refactor(v, eps=EPS32)
        assert np.array_equal(r_g, r_o) and np.array_equal(c_g, c_o)
        At = sp.diags(r_o) @ q.scipy(t) @ sp.diags(c_o)
        thresh = EPS32 * abs(At).sum(axis=1).max()
        check_factor_bound32(so, At.tocsr(), lu_g, lu_o, thresh)
        check_solve_componentwise(so, lu_g, r_g, c_g, b, sk.solve(cuda(b)).cpu().numpy())
        x, info = sk.refine(cuda(b))
        _, berr = oracle.residual(q.n, q.rowptr, q.colind, v, x.cpu().numpy(), b)
        print(f"[gpu]   step {t}: perturbed gpu {np_g} oracle {np_o}; fgmres {info[0].iters} berr {berr:.2e}",
              flush=True)
        assert info[0].status == K.OK and berr <= 1e-10 and berr_close(q, info[0].berr, berr), (t, berr, info)


def test_fp32_deterministic_and_options():
    print("[gpu] fp32 determinism", flush=True)
    q = kktgen.make_sequence(kktgen.small(300, config_id=140, steps=2))
    so, sk = setup32(q)
    assert sk.opts["factor_precision"] == K.FP32 and sk.opts["tiny_pivot_fp32"] == EPS32
    # the FP32 factor halves the factor storage of the workspace
    sk64 = K.KKTSolver(q.n, q.rowptr, q.colind, q.values(0))
    assert sk64.workspace_bytes(1) - sk.workspace_bytes(1) >= 2 * 4 * sk.nnz_lu - 4096
    vd = cuda(q.values(1))
    out = []
    for _ in range(2):
        sk.refactor(vd)
        lu, _, _ = sk.export_factors()
        x, _ = sk.refine(cuda(q.rhs(1)))
        out.append((lu, x.cpu().numpy()))
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


@pytest.mark.parametrize("cid,steps", [(1, (0, 1, 15, 29)), (2, (0, 1, 25, 49))], ids=["grid25k", "grid70k"])
def test_fp32_full_size(cid, steps):
    """Sampled full-size steps: FP32 factors within the bound against the FP64 oracle, one
    solve within its componentwise bound, refinement to 1e-10 (any step short of it is
    named)."""
    print(f"[gpu] fp32 full size config {cid}", flush=True)
    q = kktgen.make_sequence(kktgen.config(cid))
    so, sk = setup32(q)
    short = []
    for t in steps:
        v, b = q.values(t), q.rhs(t)
        vd = cuda(v)
        sk.refactor(vd)
        st, np_g = sk.refactor_status()
        lu_g, r_g, c_g = sk.export_factors()
        lu_o, r_o, c_o, np_o, _ = so.refactor(v, eps=EPS32)
        assert np.array_equal(r_g, r_o) and np.array_equal(c_g, c_o)
        At = sp.diags(r_o) @ q.scipy(t) @ sp.diags(c_o)
        check_factor_bound32(so, At.tocsr(), lu_g, lu_o, EPS32 * abs(At).sum(axis=1).max())
        check_solve_componentwise(so, lu_g, r_g, c_g, b, sk.solve(cuda(b)).cpu().numpy())
        x, info = sk.refine(cuda(b))
        _, berr = oracle.residual(q.n, q.rowptr, q.colind, v, x.cpu().numpy(), b)
        print(f"[gpu]   step {t}: perturbed gpu {np_g} oracle {np_o}; fgmres {info[0].iters} berr {berr:.2e} "
              f"status {info[0].status}", flush=True)
        if not (info[0].status == K.OK and berr <= 1e-10):
            short.append((t, info[0].iters, berr, info[0].status))
    assert not short, f"steps short of 1e-10: {short}"
