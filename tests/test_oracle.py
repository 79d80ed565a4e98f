"""Pins of the CPU oracle against facts that do not come from the oracle itself:
textbook LU and library routines, brute-force replays of the symbolic definitions,
closed forms, rounding-error bounds, the paper's printed grid sizes and a hand-computed
backward error."""
import math
import os

import numpy as np
import pytest
import scipy.linalg

import kktgen
import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
U = np.finfo(np.float64).eps / 2


def dense_to_csr(M, force_diag=True):
    n = M.shape[0]
    pat = M != 0
    if force_diag:
        pat = pat | np.eye(n, dtype=bool)
    rowptr = np.zeros(n + 1, np.int64)
    cols, vals = [], []
    for i in range(n):
        c = np.flatnonzero(pat[i])
        cols.append(c)
        vals.append(M[i, c])
        rowptr[i + 1] = rowptr[i] + len(c)
    return rowptr, np.concatenate(cols).astype(np.int32), np.concatenate(vals).astype(np.float64)


def random_sparse_sym_pattern(n, density, rng):
    M = rng.random((n, n)) < density
    M = M | M.T | np.eye(n, dtype=bool)
    return M


def kkt_small(buses=12, cid=101, schedule="widening", steps=4):
    return kktgen.make_sequence(kktgen.small(buses, config_id=cid, steps=steps, schedule=schedule))


# --------------------------------------------------------------------- generator (T0)

def test_generator_closed_form_sizes_and_symmetry():
    for spec in (kktgen.config(0), kktgen.small(300, config_id=7), kktgen.small(50, config_id=8, flows=1)):
        q = kktgen.make_sequence(spec)
        n, nnz = kktgen.closed_form_sizes(spec.buses, len(q.gen_bus), len(q.branches),
                                          spec.flows_per_branch)
        assert (q.n, q.nnz) == (n, nnz)
        A = q.scipy(0)
        assert abs(A - A.T).max() == 0.0
        assert np.all(A.diagonal() != 0)
        assert len(q.branches) == round(spec.avg_degree * spec.buses / 2)
        # simple graph: no duplicate branches, no self loops
        assert len(np.unique(q.branches, axis=0)) == len(q.branches)
        assert np.all(q.branches[:, 0] < q.branches[:, 1])


def test_generator_seeded_reproducible():
    a = kktgen.make_sequence(kktgen.small(80, config_id=9))
    b = kktgen.make_sequence(kktgen.small(80, config_id=9))
    assert np.array_equal(a.colind, b.colind) and np.array_equal(a.rowptr, b.rowptr)
    assert np.array_equal(a.values(2), b.values(2))
    assert np.array_equal(a.rhs(1), b.rhs(1))
    c = kktgen.make_sequence(kktgen.small(80, config_id=10))
    assert not np.array_equal(a.values(0)[: c.nnz], c.values(0)[: a.nnz]) or a.nnz != c.nnz


def test_generator_widening_diagonal_range():
    q = kktgen.make_sequence(kktgen.small(200, config_id=11, steps=5))
    d_first = q.values(0)[q._dslot]
    d_last = q.values(4)[q._dslot]
    assert np.abs(d_first).max() < 1e2 * 1.5 + 50     # e_0 = 2 plus H diagonal
    assert np.abs(d_last).max() > 1e9                   # e_T = 10


def test_generator_matches_paper_grid_sizes():
    """Table I prints N and nnz of the TAMU grids; with zero flow-limit rows the
    generator's closed form at the same bus/generator/branch counts is within 4%."""
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "table1_grid_sizes.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 2
    for name, B, G, Br, N, nnz in rows:
        n_c, nnz_c = kktgen.closed_form_sizes(int(B), int(G), int(Br), 0)
        assert abs(n_c - int(N)) / int(N) < 0.04, name
        assert abs(nnz_c - int(nnz)) / int(nnz) < 0.04, name


# --------------------------------------------------------------------- O0 validation

def test_validate_rejects_bad_patterns():
    rp, ci, _ = dense_to_csr(np.eye(3) + np.diag([1, 1], 1))
    assert oracle.validate(3, rp, ci) == oracle.OK
    bad = ci.copy()
    bad[0], bad[1] = bad[1], bad[0]                        # unsorted row
    assert oracle.validate(3, rp, bad) == oracle.ERR_PATTERN
    dup = ci.copy()
    dup[1] = dup[0]                                        # duplicate
    assert oracle.validate(3, rp, dup) == oracle.ERR_PATTERN
    oob = ci.copy()
    oob[-1] = 3                                            # out of range
    assert oracle.validate(3, rp, oob) == oracle.ERR_PATTERN
    nodiag_rp = np.array([0, 1, 2, 3], np.int64)
    nodiag_ci = np.array([1, 0, 2], np.int32)              # rows 0, 1 lack their diagonal
    assert oracle.validate(3, nodiag_rp, nodiag_ci) == oracle.ERR_PATTERN


def test_analyze_error_paths():
    M = np.array([[2.0, 1.0], [1.0, 3.0]])
    rp, ci, v = dense_to_csr(M)
    v2 = v.copy()
    v2[1] = np.nan
    with pytest.raises(oracle.OracleError) as e:
        oracle.Symbolic(2, rp, ci, v2)
    assert e.value.code == oracle.ERR_NONFINITE
    Z = np.array([[1.0, 0.0, 0.0], [0.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    rp, ci, v = dense_to_csr(Z)                            # zero row/column 1
    with pytest.raises(oracle.OracleError) as e:
        oracle.Symbolic(3, rp, ci, v)
    assert e.value.code == oracle.ERR_SINGULAR


# --------------------------------------------------------------------- O1 minimum degree

def brute_min_degree_replay(n, pattern_sym, order):
    """Replays an elimination order with explicit elimination graphs and asserts each pick
    is argmin (degree, index), the degree being recomputed by graph search."""
    alive = set(range(n))
    adj = {v: set(np.flatnonzero(pattern_sym[v])) - {v} for v in range(n)}
    eliminated = set()

    def degree(v):
        # uneliminated vertices reachable from v through eliminated vertices
        seen, stack, out = {v}, [v], set()
        while stack:
            u = stack.pop()
            for w in adj[u]:
                if w in seen:
                    continue
                seen.add(w)
                if w in eliminated:
                    stack.append(w)
                else:
                    out.add(w)
        return len(out)

    for v in order:
        degs = {u: degree(u) for u in alive}
        best = min(alive, key=lambda u: (degs[u], u))
        assert v == best, (v, best, degs[v], degs[best])
        alive.remove(v)
        eliminated.add(v)


@pytest.mark.parametrize("seed,n,dens", [(1, 30, 0.1), (2, 60, 0.05), (3, 120, 0.03)])
def test_min_degree_brute_force_replay(seed, n, dens):
    rng = np.random.default_rng(seed)
    pat = random_sparse_sym_pattern(n, dens, rng)
    rp, ci, _ = dense_to_csr(pat.astype(float))
    order = oracle.min_degree(n, rp, ci)
    assert sorted(order) == list(range(n))
    brute_min_degree_replay(n, pat, order)


def test_min_degree_replay_kkt():
    q = kkt_small(10, cid=102)
    pat = q.scipy(0).toarray() != 0
    order = oracle.min_degree(q.n, q.rowptr, q.colind)
    brute_min_degree_replay(q.n, pat, order)


def test_min_degree_unsymmetric_pattern_uses_a_plus_at():
    rng = np.random.default_rng(4)
    n = 40
    M = (rng.random((n, n)) < 0.06) | np.eye(n, dtype=bool)
    rp, ci, _ = dense_to_csr(M.astype(float))
    order = oracle.min_degree(n, rp, ci)
    brute_min_degree_replay(n, M | M.T, order)


# --------------------------------------------------------------------- O2 equilibration

def test_equilibration_is_exact_power_of_two_scaling():
    q = kkt_small(20, cid=103)
    v = q.values(2)
    r, c = oracle.equilibrate(q.n, q.rowptr, q.colind, v)
    for s in (r, c):
        m, e = np.frexp(s)
        assert np.all(m == 0.5)                             # exact powers of two
    A = q.scipy(2).tocsr()
    RA = np.abs(A.multiply(r[:, None])).max(axis=1).toarray().ravel()
    assert np.all((RA >= 1) & (RA < 2))                     # row maxima after row scaling
    At = (A.multiply(r[:, None])).multiply(c[None, :]).tocsc()
    CM = np.abs(At).max(axis=0).toarray().ravel()
    assert np.all((CM >= 1) & (CM < 2))                     # column maxima of R A C
    # scaling then unscaling reproduces A bitwise (no rounding)
    B = At.multiply(1 / r[:, None]).multiply(1 / c[None, :]).tocsr()
    B.sort_indices()
    assert np.array_equal(B.data, A.data)


# --------------------------------------------------------------------- O3 pivots / factors

def test_partial_pivoting_special_case_matches_lapack():
    """tau = 1, Q = identity, no scaling: threshold pivoting is partial pivoting."""
    rng = np.random.default_rng(5)
    for n in (5, 17, 40):
        M = rng.standard_normal((n, n))
        rp, ci, v = dense_to_csr(M)
        s = oracle.Symbolic(n, rp, ci, v, tau=1.0, scale=False, fixed_q=np.arange(n))
        lu, piv = scipy.linalg.lu_factor(M)
        perm = np.arange(n)
        for k in range(n):
            perm[[k, piv[k]]] = perm[[piv[k], k]]
        assert np.array_equal(s.P, perm)
        L, Uu = s.dense_factors(s.lu_k1)
        assert np.allclose(np.tril(lu, -1) + np.eye(n), L, rtol=0, atol=1e-12 * n)
        assert np.allclose(np.triu(lu), Uu, rtol=0, atol=1e-12 * n * np.abs(M).max())


def doolittle(A):
    """Textbook right-looking Gaussian elimination without pivoting."""
    n = A.shape[0]
    A = A.copy()
    for k in range(n):
        A[k + 1:, k] /= A[k, k]
        A[k + 1:, k + 1:] -= np.outer(A[k + 1:, k], A[k, k + 1:])
    return np.tril(A, -1) + np.eye(n), np.triu(A)




@pytest.mark.parametrize("cid", [104, 105])
def test_factors_match_dense_doolittle_and_error_bound(cid):
    q = kkt_small(6, cid=cid)
    v = q.values(0)
    s = oracle.Symbolic(q.n, q.rowptr, q.colind, v)
    A = q.scipy(0).toarray()
    lu, r, c, npert, rc = s.refactor(v)
    At = (r[:, None] * A) * c[None, :]
    PAQ = At[np.ix_(s.P, s.Q)]
    L, Uu = s.dense_factors(lu)
    if npert == 0:
        Ld, Ud = doolittle(PAQ)
        scale = np.abs(Ld) @ np.abs(Ud)
        assert np.all(np.abs(L - Ld) <= 1e-8 * (np.abs(Ld) + 1e-300) + 1e-10)
        assert np.all(np.abs(L @ Uu - Ld @ Ud) <= 64 * q.n * U * scale + 1e-300)
    n = q.n
    E = PAQ - L @ Uu
    # the perturbed pivots change the diagonal only, by at most eps*||A~||
    anorm = np.abs(At).sum(axis=1).max()
    off = E - np.diag(np.diag(E))
    bound = 4 * n * U * (np.abs(L) @ np.abs(Uu))
    assert np.all(np.abs(off) <= bound + 1e-300)
    assert np.all(np.abs(np.diag(E)) <= oracle.EPS * anorm + np.diag(bound) + 1e-300)


def test_refactor_of_analysed_values_reproduces_analysis_factors():
    q = kktgen.make_sequence(kktgen.config(0))
    v = q.values(0)
    s = oracle.Symbolic(q.n, q.rowptr, q.colind, v, tau=1e-3)     # off-diagonal pivots too
    lu, r, c, npert, rc = s.refactor(v, eps=0.0)
    assert np.array_equal(lu, s.lu_k1)


def test_threshold_pivot_invariant():
    q = kktgen.make_sequence(kktgen.small(60, config_id=106))
    v = q.values(0)
    tau = 1e-3
    s = oracle.Symbolic(q.n, q.rowptr, q.colind, v, tau=tau)
    # recompute each column's candidates densely and check |u_kk| >= tau * max|candidate|
    A = q.scipy(0).toarray()
    r, c = oracle.equilibrate(q.n, q.rowptr, q.colind, v)
    At = (r[:, None] * A) * c[None, :]
    PAQ = At[np.ix_(s.P, s.Q)]
    L, Uu = s.dense_factors(s.lu_k1)
    # Schur complement column k before elimination: candidates are rows >= k of column k of
    # (PAQ - L[:, :k] U[:k, :]); pivot is row k
    for k in range(0, q.n, 7):
        colk = PAQ[k:, k] - L[k:, :k] @ Uu[:k, k]
        m = np.abs(colk).max()
        assert abs(colk[0]) >= tau * m * (1 - 1e-9)


def pivot_rule_replay(At, P, Q, tau):
    """Replays the analysis pivot sequence by dense right-looking elimination of A~(:, Q)
    (rows kept in original index) and checks every step's choice against the rule:
    the diagonal row Q[k] is taken exactly when it is a non-pivotal row with a nonzero value
    and |x_diag| >= tau * max|x_candidates|; otherwise the largest candidate, lowest row on
    ties.  Steps whose decision lies within rounding of the threshold or of a tie are not
    asserted.  Returns (asserted steps, steps where the diagonal won without being the
    largest candidate, steps that took an off-diagonal row)."""
    n = At.shape[0]
    M = At[:, Q].copy()
    pivotal = np.zeros(n, dtype=bool)
    rows = np.arange(n)
    checked = diag_not_max = offdiag = 0
    for k in range(n):
        cand = ~pivotal
        x = np.where(cand, M[:, k], 0.0)
        ax = np.abs(x)
        m = ax.max()
        assert m > 0.0, k
        d = Q[k]
        diag_ok = bool(cand[d] and x[d] != 0.0 and ax[d] >= tau * m)
        near_thr = cand[d] and x[d] != 0.0 and abs(ax[d] - tau * m) <= 1e-11 * m
        win = np.flatnonzero(cand & (ax >= m * (1 - 1e-9)))
        exact_tie = np.all(ax[win] == m)
        if not near_thr:
            if diag_ok:
                assert P[k] == d, (k, P[k], d)
                diag_not_max += int(ax[d] < m)
            else:
                assert P[k] != d or not cand[d] or x[d] == 0.0, k
                if len(win) == 1 or exact_tie:
                    assert P[k] == win.min(), (k, P[k], win)
                else:
                    assert P[k] in win, (k, P[k], win)
                offdiag += int(P[k] != d)
            checked += 1
        piv = P[k]
        assert cand[piv], k
        el = cand & (rows != piv)
        M[el, k + 1:] -= np.outer(M[el, k] / M[piv, k], M[piv, k + 1:])
        pivotal[piv] = True
    return checked, diag_not_max, offdiag


@pytest.mark.parametrize("tau", [0.0, 1e-3, 0.1])
def test_pivot_rule_dense_replay_kkt(tau):
    """The diagonal preference of the analysis pivot rule, replayed densely on a KKT grid.
    At tau = 0 every nonzero diagonal is kept, also where another candidate is larger, so
    an oracle that always took the largest candidate fails here."""
    q = kktgen.make_sequence(kktgen.small(14, config_id=109, steps=1, schedule="fixed"))
    v = q.values(0)
    s = oracle.Symbolic(q.n, q.rowptr, q.colind, v, tau=tau)
    r, c = oracle.equilibrate(q.n, q.rowptr, q.colind, v)
    At = (r[:, None] * q.scipy(0).toarray()) * c[None, :]
    checked, diag_not_max, offdiag = pivot_rule_replay(At, s.P, s.Q, tau)
    assert checked >= q.n - 2
    assert diag_not_max > 0
    if tau == 0.0:
        assert np.array_equal(s.P, s.Q)


@pytest.mark.parametrize("seed,tau", [(0, 0.0), (1, 1e-3), (2, 0.1), (3, 0.1), (4, 0.5)])
def test_pivot_rule_dense_replay_random_unsymmetric(seed, tau):
    rng = np.random.default_rng(300 + seed)
    n = 48
    M = (rng.random((n, n)) < 0.12) * rng.standard_normal((n, n))
    M[np.arange(n), np.arange(n)] = rng.standard_normal(n) * (rng.random(n) < 0.8)
    rp, ci, v = dense_to_csr(M, force_diag=True)
    try:
        s = oracle.Symbolic(n, rp, ci, v, tau=tau)
    except oracle.OracleError:
        pytest.skip("structurally singular draw")
    r, c = oracle.equilibrate(n, rp, ci, v)
    A = np.zeros((n, n))
    A[np.repeat(np.arange(n), np.diff(rp)), ci] = v
    At = (r[:, None] * A) * c[None, :]
    checked, diag_not_max, offdiag = pivot_rule_replay(At, s.P, s.Q, tau)
    assert checked >= n - 2
    if tau <= 0.1:
        assert diag_not_max > 0
    if tau > 0.0:
        assert offdiag > 0


def test_pivot_rule_hand_built_3x3():
    """Q = I, no scaling; column 0 holds (0.5, 2, 0) or (0.5, 2, -2) or (0, 2, -2)."""
    def piv0(col0, tau):
        M = np.array([[col0[0], 1.0, 0.0], [col0[1], 1.0, 1.0], [col0[2], 1.0, 3.0]])
        rp, ci, v = dense_to_csr(M)
        s = oracle.Symbolic(3, rp, ci, v, tau=tau, scale=False, fixed_q=np.arange(3))
        return int(s.P[0])
    # diagonal between tau*max and max: kept although row 1 is larger
    assert piv0((0.5, 2.0, 0.0), 0.1) == 0
    assert piv0((0.5, 2.0, 0.0), 0.25) == 0          # exactly tau * max: kept
    assert piv0((0.5, 2.0, 0.0), 0.0) == 0
    # diagonal below tau*max: the largest candidate
    assert piv0((0.5, 2.0, 0.0), 0.5) == 1
    # tie in magnitude: the lowest row
    assert piv0((0.5, 2.0, -2.0), 0.5) == 1
    assert piv0((0.5, -2.0, 2.0), 0.5) == 1
    # zero diagonal is never kept, even at tau = 0
    assert piv0((0.0, 2.0, -2.0), 0.0) == 1
    assert piv0((0.0, -1.0, 3.0), 0.0) == 2


def test_closed_form_2x2_saddle():
    a, b, cc = 3.0, 2.0, 0.5
    M = np.array([[a, b], [b, -cc]])
    rp, ci, v = dense_to_csr(M)
    s = oracle.Symbolic(2, rp, ci, v, scale=False, fixed_p=[0, 1], fixed_q=[0, 1])
    lu, r, c, npert, rc = s.refactor(v, eps=0.0)
    L, Uu = s.dense_factors(lu)
    assert L[1, 0] == b / a
    assert Uu[1, 1] == -cc - (b / a) * b


def test_closed_form_kkt_schur_complement():
    """H = 0: [[D, J^T], [J, -dc I]] eliminated primal-first leaves -dc I - J D^-1 J^T."""
    rng = np.random.default_rng(7)
    npv, m = 8, 5
    D = np.diag(10 ** rng.uniform(-1, 1, npv))
    J = rng.standard_normal((m, npv)) * (rng.random((m, npv)) < 0.5)
    dc = 1e-3
    K = np.block([[D, J.T], [J, -dc * np.eye(m)]])
    rp, ci, v = dense_to_csr(K)
    n = npv + m
    s = oracle.Symbolic(n, rp, ci, v, scale=False, fixed_p=np.arange(n), fixed_q=np.arange(n))
    lu, r, c, npert, rc = s.refactor(v, eps=0.0)
    L, Uu = s.dense_factors(lu)
    S = -dc * np.eye(m) - J @ np.linalg.solve(D, J.T)
    S_fact = L[npv:, npv:] @ Uu[npv:, npv:]
    assert np.allclose(S_fact, S, rtol=1e-12, atol=1e-12)


def test_tiny_pivot_perturbation_closed_form():
    a, b = 2.0, 3.0
    M = np.array([[a, b], [b, b * b / a]])            # u22 = 0 exactly
    rp, ci, v = dense_to_csr(M)
    s = oracle.Symbolic(2, rp, ci, v, scale=False, fixed_p=[0, 1], fixed_q=[0, 1])
    lu, r, c, npert, rc = s.refactor(v)
    assert npert == 1 and rc == oracle.WARN_PERTURBED
    anorm = max(abs(a) + abs(b), abs(b) + b * b / a)
    L, Uu = s.dense_factors(lu)
    assert Uu[1, 1] == oracle.EPS * anorm               # +0 perturbs to the positive side
    v_neg = v.copy()
    v_neg[-1] = b * b / a * (1 - 2 ** -40)              # tiny negative pivot after the update
    lu2, _, _, npert2, _ = s.refactor(v_neg)
    L2, U2 = s.dense_factors(lu2)
    assert npert2 == 1 and U2[1, 1] < 0


# --------------------------------------------------------------------- O4 symbolic

def symbolic_dense_elimination(pat):
    """Boolean Gaussian elimination (no cancellation): pattern of L+U of a matrix."""
    P = pat.copy()
    n = P.shape[0]
    for k in range(n):
        rows = np.flatnonzero(P[k + 1:, k]) + k + 1
        cols = np.flatnonzero(P[k, k + 1:]) + k + 1
        P[np.ix_(rows, cols)] = True
    return P


def canonical_pattern(s):
    n = s.n
    M = np.zeros((n, n), bool)
    for k in range(n):
        M[s.rowidx[s.colptr[k]:s.colptr[k + 1]], k] = True
    return M


@pytest.mark.parametrize("tau", [0.0, 1e-3, 0.5])
def test_fill_pattern_and_products_brute_force(tau):
    q = kkt_small(12, cid=107)
    v = q.values(0)
    s = oracle.Symbolic(q.n, q.rowptr, q.colind, v, tau=tau, sn_max=5)
    n = q.n
    A = q.scipy(0).toarray() != 0
    PAQ = A[np.ix_(s.P, s.Q)]
    F = symbolic_dense_elimination(PAQ)
    M = canonical_pattern(s)
    assert np.array_equal(M, F)
    # canonical order within a column: rows ascending (U rows, diagonal, L rows)
    for k in range(n):
        rows = s.rowidx[s.colptr[k]:s.colptr[k + 1]]
        assert np.all(np.diff(rows) > 0) and k in rows
    # etree
    for j in range(n):
        below = np.flatnonzero(M[j + 1:, j]) + j + 1
        assert s.parent[j] == (below[0] if len(below) else -1)
    # levels by exhaustive recursion on the definitions
    import functools
    import sys
    sys.setrecursionlimit(10000)

    @functools.lru_cache(None)
    def lf(k):
        deps = [j for j in range(k) if M[j, k]]
        return 1 + max(lf(j) for j in deps) if deps else 0

    @functools.lru_cache(None)
    def ll(i):
        deps = [j for j in range(i) if M[i, j]]
        return 1 + max(ll(j) for j in deps) if deps else 0

    @functools.lru_cache(None)
    def lu_(i):
        deps = [j for j in range(i + 1, n) if M[i, j]]
        return 1 + max(lu_(j) for j in deps) if deps else 0

    assert [lf(k) for k in range(n)] == list(s.lev_f)
    assert [ll(k) for k in range(n)] == list(s.lev_l)
    assert [lu_(k) for k in range(n)] == list(s.lev_u)
    # supernodes by definition
    starts = [0]
    width = 1
    for j in range(1, n):
        ok = (width < 5 and M[j, j - 1] and M[j - 1, j]
              and np.array_equal(M[j + 1:, j - 1], M[j + 1:, j])
              and np.array_equal(M[j - 1, j + 1:], M[j, j + 1:]))
        if ok:
            width += 1
        else:
            starts.append(j)
            width = 1
    starts.append(n)
    assert list(s.sn_start) == starts
    # scatter map by dictionary lookup
    pinv = np.empty(n, int)
    pinv[s.P] = np.arange(n)
    qinv = np.empty(n, int)
    qinv[s.Q] = np.arange(n)
    slot = {}
    for k in range(n):
        for p in range(s.colptr[k], s.colptr[k + 1]):
            slot[(s.rowidx[p], k)] = p
    for i in range(n):
        for p in range(q.rowptr[i], q.rowptr[i + 1]):
            assert s.map[p] == slot[(pinv[i], qinv[q.colind[p]])]


def test_no_fill_closed_forms():
    n = 30
    rng = np.random.default_rng(8)
    # diagonal: L = I, U = A~
    Dm = np.diag(rng.uniform(1, 2, n))
    rp, ci, v = dense_to_csr(Dm)
    s = oracle.Symbolic(n, rp, ci, v)
    assert s.nnz_lu == n
    lu, r, c, _, _ = s.refactor(v)
    assert np.array_equal(lu, (r[s.P] * np.diag(Dm)[s.P]) * c[s.Q])
    # tridiagonal and arrow (hub last after ordering): no fill
    T = np.diag(np.full(n, 4.0)) + np.diag(np.full(n - 1, -1.0), 1) + np.diag(np.full(n - 1, -1.0), -1)
    rp, ci, v = dense_to_csr(T)
    assert oracle.Symbolic(n, rp, ci, v).nnz_lu == len(ci)
    Aw = np.diag(np.full(n, float(n)))
    Aw[0, :] = 1.0
    Aw[:, 0] = 1.0
    Aw[0, 0] = float(n)
    rp, ci, v = dense_to_csr(Aw)
    s = oracle.Symbolic(n, rp, ci, v)
    assert s.nnz_lu == len(ci) and 0 in s.Q[-2:]             # the hub goes with the last leaf
    s_bad = oracle.Symbolic(n, rp, ci, v, fixed_q=np.arange(n), fixed_p=np.arange(n))
    assert s_bad.nnz_lu == n * n                             # hub first fills everything


# --------------------------------------------------------------------- O6 / O7 / O8

def test_solve_matches_numpy_on_well_conditioned():
    rng = np.random.default_rng(9)
    n = 50
    M = rng.standard_normal((n, n)) * (rng.random((n, n)) < 0.15) + np.diag(rng.uniform(3, 5, n))
    rp, ci, v = dense_to_csr(M)
    s = oracle.Symbolic(n, rp, ci, v)
    lu, r, c, _, _ = s.refactor(v)
    b = rng.standard_normal(n)
    x = s.solve(lu, r, c, b)
    xr = np.linalg.solve(M, b)
    assert np.allclose(x, xr, rtol=0, atol=np.linalg.cond(M) * 1e-14 * np.abs(xr).max())


def test_backward_error_hand_computed():
    d = {}
    for line in open(os.path.join(HERE, "golden", "berr_3x3.txt")):
        if line.strip() and not line.startswith("#"):
            k, *vals = line.split()
            d[k] = np.array([float(t) for t in vals])
    A = d["A"].reshape(3, 3)
    rp, ci, v = dense_to_csr(A, force_diag=False)
    res, be = oracle.residual(3, rp, ci, v, d["x"], d["b"])
    assert np.array_equal(res, d["r"])
    assert be == d["berr"][0]


def test_fgmres_converges_with_inexact_preconditioner():
    """Flexible GMRES must reach the tolerance for the matrix it is given, even when the
    preconditioner factors a different matrix; its answer then matches numpy."""
    q = kkt_small(15, cid=108, schedule="fixed", steps=3)
    v0 = q.values(0)
    s = oracle.Symbolic(q.n, q.rowptr, q.colind, v0)
    lu, r, c, _, _ = s.refactor(v0)
    v1 = q.values(1)                                        # a different system
    b = q.rhs(1)
    x, it, be, rc = s.fgmres(v1, lu, r, c, b, restart=10, max_it=200, tol=1e-12)
    assert rc == oracle.OK and be <= 1e-12 and it > 0
    _, be_chk = oracle.residual(q.n, q.rowptr, q.colind, v1, x, b)
    assert be_chk <= 1e-12
    A1 = q.scipy(1).toarray()
    assert np.linalg.norm(A1 @ x - b, np.inf) <= 1e-12 * (np.abs(A1).sum(1).max() * np.abs(x).max() + np.abs(b).max())
    # exact preconditioner: x0 is already accurate, no Arnoldi step needed
    lu1, r1, c1, np1, _ = s.refactor(v1)
    x, it, be, rc = s.fgmres(v1, lu1, r1, c1, b, tol=1e-10)
    if np1 == 0:
        assert it == 0 and be <= 1e-10


def test_fgmres_reports_not_converged():
    q = kkt_small(15, cid=109, schedule="fixed", steps=2)
    v0 = q.values(0)
    s = oracle.Symbolic(q.n, q.rowptr, q.colind, v0)
    lu, r, c, _, _ = s.refactor(v0)
    x, it, be, rc = s.fgmres(q.values(1), lu, r, c, q.rhs(1), restart=2, max_it=1, tol=1e-30)
    assert rc == oracle.WARN_NOT_CONVERGED and it == 1 and be > 1e-30


def test_sequence_reaches_target_backward_error_200bus():
    q = kktgen.make_sequence(kktgen.config(0))
    s = oracle.Symbolic(q.n, q.rowptr, q.colind, q.values(0))
    for t in range(q.steps):
        v = q.values(t)
        lu, r, c, _, _ = s.refactor(v)
        x, it, be, rc = s.fgmres(v, lu, r, c, q.rhs(t))
        assert rc == oracle.OK and be <= 1e-10


@pytest.mark.slow
def test_sequence_reaches_target_backward_error_2000bus():
    q = kktgen.make_sequence(kktgen.small(2000, config_id=110, steps=6))
    s = oracle.Symbolic(q.n, q.rowptr, q.colind, q.values(0))
    for t in range(q.steps):
        v = q.values(t)
        lu, r, c, _, _ = s.refactor(v)
        x, it, be, rc = s.fgmres(v, lu, r, c, q.rhs(t))
        assert rc == oracle.OK and be <= 1e-10


# ------------------------------------------------------------------ O9 approximate solves

def _sym3_identity():
    """3x3 full pattern with P = Q = I and no scaling; returns (Symbolic, canonical lu) for
    the hand-worked factors of tests/golden/approx_sweeps_3x3.txt."""
    L = np.array([[1.0, 0, 0], [2, 1, 0], [-1, 3, 1]])
    U = np.array([[2.0, 1, -1], [0, 4, 2], [0, 0, 0.5]])
    A = L @ U
    rowptr = np.array([0, 3, 6, 9])
    colind = np.tile(np.arange(3, dtype=np.int32), 3)
    ident = np.arange(3, dtype=np.int32)
    so = oracle.Symbolic(3, rowptr, colind, A.ravel(), scale=False, fixed_p=ident, fixed_q=ident)
    lu = np.empty(so.nnz_lu)
    for k in range(3):
        for p in range(so.colptr[k], so.colptr[k + 1]):
            i = so.rowidx[p]
            lu[p] = L[i, k] if i > k else U[i, k]
    return so, lu


def test_approx_sweeps_hand_example():
    so, lu = _sym3_identity()
    one = np.ones(3)
    b = np.array([1.0, 2.0, 3.0])
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "approx_sweeps_3x3.txt")) if l.strip() and l[0] != "#"]
    assert len(rows) == 5
    for kind, chunk, sweeps, *xs in rows:
        x = so.approx_solve(lu, one, one, b, int(sweeps), int(kind), int(chunk))
        assert np.array_equal(x, np.array([float(v) for v in xs])), (kind, chunk, sweeps, x)


def _well_conditioned_factors(so, seed):
    """Random factor values on the analysed pattern with a dominant U diagonal, so that the
    triangular systems are well conditioned."""
    rng = np.random.default_rng(seed)
    cols = np.repeat(np.arange(so.n), np.diff(so.colptr))
    lu = rng.uniform(-0.3, 0.3, so.nnz_lu)
    diag = so.rowidx == cols
    lu[diag] = rng.uniform(2.0, 3.0, int(diag.sum())) * rng.choice([-1.0, 1.0], int(diag.sum()))
    return lu


def test_approx_sweeps_closed_forms():
    """One Jacobi sweep is x = Q C D^-1 P R b; enough Jacobi sweeps (more than the level
    depth: the strictly triangular parts are nilpotent) and one block Gauss-Seidel sweep
    with a single chunk are the exact triangular solves; block Gauss-Seidel with chunks of
    one row is Jacobi, bit for bit."""
    q = kktgen.make_sequence(kktgen.config(0))
    so = oracle.Symbolic(q.n, q.rowptr, q.colind, q.values(0))
    lu = _well_conditioned_factors(so, 5)
    _, r, c, _, _ = so.refactor(q.values(1))
    b = q.rhs(1)
    Lm, Um = so.dense_factors(lu)
    bt = r[so.P] * b[so.P]
    exact_t = scipy.linalg.solve_triangular(Um, scipy.linalg.solve_triangular(Lm, bt, lower=True, unit_diagonal=True))
    exact = np.empty(so.n)
    exact[so.Q] = c[so.Q] * exact_t
    one = np.empty(so.n)
    one[so.Q] = c[so.Q] * (bt / np.diag(Um))
    assert np.allclose(so.approx_solve(lu, r, c, b, 1, 0), one, rtol=4e-16, atol=0)
    depth = max(so.lev_l.max(), so.lev_u.max()) + 1
    xj = so.approx_solve(lu, r, c, b, depth, 0)
    assert np.allclose(xj, exact, rtol=1e-11, atol=1e-11 * abs(exact).max())
    xg = so.approx_solve(lu, r, c, b, 1, 1, chunk=so.n)
    assert np.allclose(xg, exact, rtol=1e-11, atol=1e-11 * abs(exact).max())
    for sweeps in (1, 3):
        assert np.array_equal(so.approx_solve(lu, r, c, b, sweeps, 1, chunk=1), so.approx_solve(lu, r, c, b, sweeps, 0))
    # three Jacobi sweeps, fewer than the depth, are not exact
    assert depth > 3 and abs(so.approx_solve(lu, r, c, b, 3, 0) - exact).max() > 1e-6
    with pytest.raises(oracle.OracleError):
        so.approx_solve(lu, r, c, b, 0, 0)
