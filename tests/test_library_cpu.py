"""Host-side checks of the HIP library through its C ABI (no GPU needed): every declared
symbol is exported, the analysis is bit-exact with the oracle, and the host-detected error
and call-order paths return the documented codes."""
import ctypes
import os
import re

import numpy as np
import pytest

import kktgen
import oracle
import paper_2302_08656_amd as K

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SYMBOLIC_KEYS = ("P", "Q", "colptr", "rowidx", "parent", "lev_f", "lev_l", "lev_u", "sn_start", "map")


def declared_functions():
    names = []
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            text = open(os.path.join(ROOT, "include", h)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names += re.findall(r"\b(kkt_\w+)\s*\(", text)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(K.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 13
    for name in names:
        assert hasattr(lib, name), name
    assert set(K.EXPORTS) <= set(names)


def test_default_options():
    o = K.default_opts()
    assert o["pivot_tau"] == oracle.TAU
    assert o["tiny_pivot"] == oracle.EPS
    assert o["sn_max_width"] == oracle.SN_MAX
    assert o["berr_tol"] == 1e-10 and o["gmres_restart"] == 30 and o["max_iters"] == 100
    assert o["graph_refactor"] == 1 and o["approx_sweeps"] == 0


def compare_symbolic(n, rowptr, colind, values, **kw):
    so = oracle.Symbolic(n, rowptr, colind, values, **{k: v for k, v in kw.items() if k in
                                                       ("tau", "sn_max", "scale", "fixed_p", "fixed_q")})
    lib_kw = {}
    for k, v in kw.items():
        lib_kw[{"tau": "pivot_tau", "sn_max": "sn_max_width", "scale": "equilibrate"}.get(k, k)] = v
    if "equilibrate" in lib_kw:
        lib_kw["equilibrate"] = int(lib_kw["equilibrate"])
    sk = K.KKTSolver(n, rowptr, colind, values, **lib_kw)
    e = sk.export_symbolic()
    for key in SYMBOLIC_KEYS:
        assert np.array_equal(e[key], getattr(so, key)), key
    return sk, so


@pytest.mark.parametrize("spec,tau", [
    (kktgen.config(0), 0.0),
    (kktgen.config(0), 1e-3),
    (kktgen.small(400, config_id=130), 0.0),
    (kktgen.small(400, config_id=131), 1e-3),
    (kktgen.small(80, config_id=132, schedule="fixed", flows=1), 0.5),
])
def test_symbolic_bit_exact_with_oracle(spec, tau):
    q = kktgen.make_sequence(spec)
    compare_symbolic(q.n, q.rowptr, q.colind, q.values(0), tau=tau)


def test_symbolic_bit_exact_options():
    q = kktgen.make_sequence(kktgen.small(100, config_id=133))
    v = q.values(0)
    compare_symbolic(q.n, q.rowptr, q.colind, v, sn_max=3)
    compare_symbolic(q.n, q.rowptr, q.colind, v, scale=False, tau=1e-2)
    rng = np.random.default_rng(0)
    perm = rng.permutation(q.n).astype(np.int32)
    compare_symbolic(q.n, q.rowptr, q.colind, v, fixed_q=perm)
    sk, so = compare_symbolic(q.n, q.rowptr, q.colind, v, fixed_q=perm, fixed_p=perm)


@pytest.mark.parametrize("seed", range(6))
def test_symbolic_bit_exact_random_unsymmetric(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(20, 120))
    M = (rng.random((n, n)) < 0.05) * rng.standard_normal((n, n))
    M[np.arange(n), np.arange(n)] = rng.standard_normal(n) * (rng.random(n) < 0.7)
    pat = (M != 0) | np.eye(n, dtype=bool)
    rowptr = np.concatenate([[0], np.cumsum(pat.sum(1))]).astype(np.int64)
    colind = np.concatenate([np.flatnonzero(pat[i]) for i in range(n)]).astype(np.int32)
    vals = np.concatenate([M[i, pat[i]] for i in range(n)])
    try:
        oracle.Symbolic(n, rowptr, colind, vals, tau=0.1)
    except oracle.OracleError as e:
        with pytest.raises(K.KKTError) as ke:
            K.KKTSolver(n, rowptr, colind, vals, pivot_tau=0.1)
        assert ke.value.code == e.code
        return
    compare_symbolic(n, rowptr, colind, vals, tau=0.1)


@pytest.mark.slow
@pytest.mark.parametrize("cid", [1, 2], ids=["grid25k", "grid70k"])
def test_symbolic_bit_exact_full_size_grids(cid):
    q = kktgen.make_sequence(kktgen.config(cid))
    sk, so = compare_symbolic(q.n, q.rowptr, q.colind, q.values(0))
    # the default static diagonal pivoting keeps every diagonal on these grids
    assert np.array_equal(so.P, so.Q)


def test_analyze_errors_match_oracle():
    M = np.array([[1.0, 0.0, 0.0], [0.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    rowptr = np.array([0, 1, 2, 3], np.int64)
    colind = np.array([0, 1, 2], np.int32)
    vals = np.array([1.0, 0.0, 1.0])
    with pytest.raises(K.KKTError) as e:
        K.KKTSolver(3, rowptr, colind, vals)
    assert e.value.code == K.ERR_SINGULAR
    with pytest.raises(K.KKTError) as e:
        K.KKTSolver(3, rowptr, colind, np.array([1.0, np.inf, 1.0]))
    assert e.value.code == K.ERR_NONFINITE
    with pytest.raises(K.KKTError) as e:
        K.KKTSolver(3, rowptr, np.array([0, 2, 1], np.int32), vals)
    assert e.value.code == K.ERR_PATTERN
    with pytest.raises(K.KKTError) as e:
        K.KKTSolver(3, rowptr, colind, vals, gmres_restart=0)
    assert e.value.code == K.ERR_ARG
    with pytest.raises(K.KKTError) as e:
        K.KKTSolver(3, rowptr, colind, vals, fixed_p=np.arange(3))
    assert e.value.code == K.ERR_ARG
    for bad in (-1, 1025):
        with pytest.raises(K.KKTError) as e:
            K.KKTSolver(3, rowptr, colind, vals, approx_sweeps=bad)
        assert e.value.code == K.ERR_ARG
    diag = K.KKTSolver(3, np.arange(4), np.arange(3, dtype=np.int32), np.array([1.0, 2.0, 3.0]), approx_sweeps=1024)
    assert diag.opts["approx_sweeps"] == 1024


def test_call_order_errors_without_device():
    q = kktgen.make_sequence(kktgen.small(20, config_id=134))
    sk = K.KKTSolver(q.n, q.rowptr, q.colind, q.values(0))
    L = K._lib()
    dummy = ctypes.c_void_p(256)
    # refactor before bind, solve and refine before refactor: state errors, no device work
    assert L.kkt_refactor(sk._h, dummy, None) == K.ERR_STATE
    assert L.kkt_solve(sk._h, dummy, dummy, 1, q.n, None) == K.ERR_STATE
    assert L.kkt_refine(sk._h, dummy, dummy, 1, q.n, None, None) == K.ERR_STATE
    assert L.kkt_refactor_status(sk._h, None, None) == K.ERR_STATE
    assert L.kkt_solve(sk._h, dummy, dummy, 0, q.n, None) == K.ERR_ARG
    assert L.kkt_bind(sk._h, ctypes.c_void_p(257), 1 << 30, 1, None) == K.ERR_ARG
    assert L.kkt_bind(sk._h, dummy, 16, 1, None) == K.ERR_NOMEM
    assert sk.workspace_bytes(1) > 8 * (sk.nnz_lu * 2)


def test_tiny_rows_tuning_host_checks():
    """tiny_rows (4-lane narrow items) defaults to 16, accepts 0..16 and only reorders items
    within a level: the workspace size does not change with it."""
    q = kktgen.make_sequence(kktgen.small(300, config_id=140, steps=1))
    sk = K.KKTSolver(q.n, q.rowptr, q.colind, q.values(0))
    t = sk.tuning()
    assert t["tiny_rows"] == 16
    base = (t["panel_max"], t["small_rows"], t["group"], t["wide256"], t["fuse_chains"])
    ws = sk.workspace_bytes(1)
    for bad in (-1, 17):
        with pytest.raises(K.KKTError) as e:
            sk.set_tuning(*base, bad)
        assert e.value.code == K.ERR_ARG
    for ok in (0, 8, 16):
        sk.set_tuning(*base, ok)
        assert sk.tuning()["tiny_rows"] == ok
        assert sk.workspace_bytes(1) == ws


def test_scratch_bind_host_checks():
    """kkt_bind_scratch rejects bad arguments and systems whose workspace exceeds the static
    array before it touches a device; the binding's size constant matches the header's."""
    hdr = open(os.path.join(ROOT, "include", "kkt.h")).read()
    m = re.search(r"#define KKT_SCRATCH_BYTES \(\(size_t\)(\d+) << (\d+)\)", hdr)
    assert m and int(m.group(1)) << int(m.group(2)) == K.SCRATCH_BYTES
    L = K._lib()
    q = kktgen.make_sequence(kktgen.small(20, config_id=134))
    sk = K.KKTSolver(q.n, q.rowptr, q.colind, q.values(0))
    assert L.kkt_bind_scratch(sk._h, 0, None) == K.ERR_ARG
    assert L.kkt_bind_scratch(None, 1, None) == K.ERR_ARG
    big = kktgen.make_sequence(kktgen.small(6000, config_id=134, steps=1))
    sb = K.KKTSolver(big.n, big.rowptr, big.colind, big.values(0))
    assert sb.workspace_bytes(1) > K.SCRATCH_BYTES
    assert L.kkt_bind_scratch(sb._h, 1, None) == K.ERR_NOMEM
    # still unbound: no state changed
    assert L.kkt_refactor(sb._h, ctypes.c_void_p(256), None) == K.ERR_STATE


def test_precision_and_sweep_options():
    """The FP32 factor option and the sweep kind: defaults, rejected values, the smaller
    workspace of FP32 factors, and the call-order errors of kkt_solve_approx."""
    o = K.default_opts()
    assert o["factor_precision"] == K.FP64 and o["tiny_pivot_fp32"] == 2.0 ** -26 and o["approx_kind"] == 0
    q = kktgen.make_sequence(kktgen.small(30, config_id=134))
    for kw in ({"factor_precision": 2}, {"factor_precision": -1}, {"approx_kind": 2}, {"tiny_pivot_fp32": -1.0}):
        with pytest.raises(K.KKTError) as e:
            K.KKTSolver(q.n, q.rowptr, q.colind, q.values(0), **kw)
        assert e.value.code == K.ERR_ARG, kw
    s64 = K.KKTSolver(q.n, q.rowptr, q.colind, q.values(0))
    s32 = K.KKTSolver(q.n, q.rowptr, q.colind, q.values(0), factor_precision=K.FP32)
    assert s32.opts["factor_precision"] == K.FP32
    # the factor and its row-ordered copy shrink from 8 to 4 bytes per entry
    assert s64.workspace_bytes(1) - s32.workspace_bytes(1) >= 8 * s64.nnz_lu - 2 * 256
    L = K._lib()
    dummy = ctypes.c_void_p(256)
    sa = K.KKTSolver(q.n, q.rowptr, q.colind, q.values(0), approx_sweeps=2, approx_kind=1)
    assert L.kkt_solve_approx(sa._h, dummy, dummy, 1, q.n, None) == K.ERR_STATE
    assert L.kkt_solve_approx(s64._h, dummy, dummy, 1, q.n, None) == K.ERR_ARG   # no sweeps configured
    assert L.kkt_solve_approx(sa._h, dummy, dummy, 0, q.n, None) == K.ERR_ARG
