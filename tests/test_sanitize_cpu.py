"""The host analysis and the GPU schedule builder built alone with AddressSanitizer and
UndefinedBehaviorSanitizer (g++, no HIP) and run on grids, random unsymmetric patterns and
error cases; any report aborts the driver.  The sizes it prints must equal the library's."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import kktgen
import paper_2302_08656_amd as K

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2302_08656_amd", "csrc")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    out = str(tmp_path_factory.mktemp("asan") / "kkt_host_asan")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           os.path.join(ROOT, "tests", "sanitize_driver.cpp"),
           os.path.join(CSRC, "kkt_symbolic.cpp"), os.path.join(CSRC, "kkt_schedule.cpp"), "-o", out]
    subprocess.run(cmd, check=True)
    return out


def run(driver, tmp_path, n, rowptr, colind, vals, tau=0.0):
    path = str(tmp_path / "m.bin")
    with open(path, "wb") as f:
        f.write(np.int32(n).tobytes() + np.int64(len(colind)).tobytes() + np.float64(tau).tobytes())
        f.write(np.ascontiguousarray(rowptr, np.int64).tobytes())
        f.write(np.ascontiguousarray(colind, np.int32).tobytes())
        f.write(np.ascontiguousarray(vals, np.float64).tobytes())
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    p = subprocess.run([driver, path], capture_output=True, text=True, env=env, timeout=600)
    assert p.returncode == 0, p.stderr[-4000:]
    assert "ERROR" not in p.stderr and "runtime error" not in p.stderr, p.stderr[-4000:]
    return [int(x) for x in p.stdout.split()]


@pytest.mark.parametrize("spec,tau", [(kktgen.config(0), 0.0), (kktgen.config(0), 1e-3),
                                      (kktgen.small(2000, config_id=147, steps=1), 0.0),
                                      (kktgen.small(60, config_id=141, steps=1, schedule="fixed"), 0.5)],
                         ids=["grid200", "grid200_tau1e-3", "grid2000", "grid60_tau0.5"])
def test_sanitized_analysis_on_grids(driver, tmp_path, spec, tau):
    q = kktgen.make_sequence(spec)
    v = q.values(0)
    rc, n, nnz_lu, npan, nit, nl, nu = run(driver, tmp_path, q.n, q.rowptr, q.colind, v, tau)
    sk = K.KKTSolver(q.n, q.rowptr, q.colind, v, pivot_tau=tau)
    assert rc == 0 and n == q.n and nnz_lu == sk.nnz_lu
    assert nit > 0 and nl > 0 and nu > 0
    sk.close()


@pytest.mark.parametrize("seed", range(4))
def test_sanitized_analysis_random_and_errors(driver, tmp_path, seed):
    rng = np.random.default_rng(700 + seed)
    n = int(rng.integers(30, 150))
    M = (rng.random((n, n)) < 0.04) * rng.standard_normal((n, n))
    M[np.arange(n), np.arange(n)] = rng.standard_normal(n) * (rng.random(n) < 0.7)
    pat = (M != 0) | np.eye(n, dtype=bool)
    rowptr = np.concatenate([[0], np.cumsum(pat.sum(1))]).astype(np.int64)
    colind = np.concatenate([np.flatnonzero(pat[i]) for i in range(n)]).astype(np.int32)
    vals = np.concatenate([M[i, pat[i]] for i in range(n)])
    rc = run(driver, tmp_path, n, rowptr, colind, vals, 0.1)[0]
    try:
        sk = K.KKTSolver(n, rowptr, colind, vals, pivot_tau=0.1)
        assert rc == 0
        sk.close()
    except K.KKTError as e:
        assert rc == e.code
    # error paths: unsorted row, missing diagonal, non-finite value
    bad = colind.copy()
    r0 = int(np.flatnonzero(np.diff(rowptr) >= 2)[0])
    bad[rowptr[r0]], bad[rowptr[r0] + 1] = bad[rowptr[r0] + 1], bad[rowptr[r0]]
    assert run(driver, tmp_path, n, rowptr, bad, vals)[0] == K.ERR_PATTERN
    v2 = vals.copy()
    v2[-1] = np.inf
    assert run(driver, tmp_path, n, rowptr, colind, v2)[0] == K.ERR_NONFINITE
