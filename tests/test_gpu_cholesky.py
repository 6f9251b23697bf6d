"""Parity of the 1D density fitting (tc_density_fit) and of the pivoted
Cholesky of the factorised TEI matrix (tc_tei_cholesky) with the FP64
oracle, through the C ABI.

Pivot choices are decisions taken on binary64 values that both sides compute
in different orders, so pivots are compared for the steps whose decision
margin (relative gap between the largest and the second largest residual
diagonal entry, on the oracle side) exceeds 1e-9, and from the first step
below it on only what is unique: the approximation quality.
"""
import numpy as np
import pytest

from paper_1504_06289_amd import workloads as wl
from tests.gpu_common import dev, host, oracle_setup, say

pytestmark = pytest.mark.gpu


def margins(A, piv):
    """Relative decision margin of each pivot step of the oracle's pivoted
    Cholesky of the explicit A (recomputed by Schur complements)."""
    out = []
    for r in range(len(piv)):
        P = piv[:r]
        S = A - (A[:, P] @ np.linalg.solve(A[np.ix_(P, P)], A[P, :]) if r else 0.0)
        dg = np.diag(S).copy()
        dg[P] = -np.inf
        top = np.sort(dg)[::-1]
        out.append((top[0] - top[1]) / max(top[0], 1e-300) if len(top) > 1 else 1.0)
    return np.array(out)


def agreed_prefix(m):
    bad = np.nonzero(m < 1e-9)[0]
    return int(bad[0]) if len(bad) else len(m)


def check_fit(tc, orc, F, tol, label):
    n = F.shape[1]
    Uo, Vo, po, reso = orc.density_fit(F, tol, n)
    U, V, piv, R, res = tc.density_fit(dev(F), tol)
    U, V = host(U), host(V)
    k = agreed_prefix(margins(F.T @ F, po))
    say(f"   {label}: R = {R} (oracle {len(po)}), pivots agree on {k} decisive steps")
    np.testing.assert_array_equal(piv[:k], po[:k])
    # the fit itself: |F - V U|^2 = residual trace <= tol^2 trace(F^T F)
    trA = np.sum(F * F)
    err2 = np.sum((F - V[:, :R] @ U[:R]) ** 2)
    assert abs(err2 - res) <= 1e-9 * trA
    assert err2 <= tol * tol * trA * (1 + 1e-6) + 1e-28 * trA
    np.testing.assert_array_equal(V[:, R:], 0.0)
    np.testing.assert_array_equal(U[R:], 0.0)
    np.testing.assert_array_equal(V[:, :R], F[:, piv])
    if k == len(po) == R:
        # the same pivots: the same fitted matrix (U itself is the
        # solution of a triangular system whose late pivots are small, so
        # its entries carry rounding amplified by that conditioning)
        fit_diff = np.linalg.norm(V[:, :R] @ U[:R] - Vo @ Uo)
        say(f"      |VU - (VU)_oracle| / |F| = {fit_diff / np.sqrt(trA):.2e}")
        assert fit_diff <= max(tol, 1e-9) * np.sqrt(trA)
    return R


@pytest.mark.parametrize("n,N_pair,tol", [(96, 60, 1e-3), (200, 150, 1e-6), (333, 90, 1e-7),
                                          (64, 10, 1e-6)])
@pytest.mark.parametrize("columns", [False, True])
def test_density_fit(tc, orc, n, N_pair, tol, columns, monkeypatch):
    """columns: TC_CHOL_COLUMNS=1, each pivot's column formed from F at every
    step (the path beyond 8192 cells) instead of from the formed F^T F."""
    if columns:
        monkeypatch.setenv("TC_CHOL_COLUMNS", "1")
    say(f"density fit n={n} N_pair={N_pair} tol={tol} columns={columns}")
    U0, _ = wl.gaussian_products(n, 8.0, N_pair, seed=n + N_pair)
    for l in range(3):
        check_fit(tc, orc, U0[l], tol, f"mode {l}")


def test_density_fit_rank_above_256(tc, orc):
    """Random products (no decay of the spectrum) fitted to rank above 256:
    the back substitution that keeps its solved entries in global memory
    (ranks up to 256 keep them in LDS)."""
    rng = np.random.default_rng(11)
    F = rng.standard_normal((320, 400))
    say("density fit of rank above 256")
    R = check_fit(tc, orc, F, 1e-6, "random 320 x 400")
    assert R > 256


@pytest.mark.parametrize("columns", [False, True])
def test_tei_cholesky_pipeline(tc, orc, columns, monkeypatch):
    """Fit each mode, M_k = U T_k U^T from the TEI assembly's saved Grams of
    the fitted rows, then the pivoted Cholesky of B: against the oracle's
    own pipeline from the same inputs, and B ~ L L^T against the J of the
    TEI assembly of the products.  columns: TC_CHOL_COLUMNS=1, the columns
    of A and B formed from the factors at every step (the path beyond 8192
    cells and 4096 products) instead of from the formed matrices."""
    if columns:
        monkeypatch.setenv("TC_CHOL_COLUMNS", "1")
    say(f"TEI Cholesky pipeline columns={columns}")
    w = wl.small_products((48, 40, 56), 60, R_N=8, b=7.0, seed=9)
    c, ps = oracle_setup(orc, w)
    # oracle pipeline
    Vo, Mo = [], []
    for l in range(3):
        U, V, piv, res = orc.density_fit(w.U[l], 1e-7, w.n[l])
        Vo.append(V)
        Mo.append(orc.gram(U, orc.convolve(ps[l], U)))
    Bo = orc.tei_matrix_factored(c, Vo, Mo)
    Lo, po, do = orc.tei_cholesky(c, Vo, Mo, 1e-10 * np.trace(Bo), Bo.shape[0])
    # GPU pipeline (fitted rows padded to a common R)
    fits = [tc.density_fit(dev(w.U[l]), 1e-7) for l in range(3)]
    R = max(f[3] for f in fits)
    Ud = [f[0][:R].contiguous() for f in fits]
    Vd = [f[1][:, :R].contiguous() for f in fits]
    J, G = tc.tei_gram(dev(c), [dev(p) for p in ps], Ud, prec="fp64", save_G=True)
    Md = [G[l].contiguous() for l in range(3)]
    L, piv, res = tc.tei_cholesky(dev(c), Vd, Md, 1e-10)
    L = host(L)
    Jr = orc.tei_gram(c, ps, w.U)
    say(f"   R per mode {[f[3] for f in fits]}, R_B = {L.shape[0]} (oracle {len(po)})")
    # B ~ L L^T: within the fit and truncation tolerances of the TEI matrix
    LL = L.T @ L
    assert np.linalg.norm(LL - Jr) <= 1e-7 * np.linalg.norm(Jr)
    assert np.linalg.norm(LL - Lo @ Lo.T) <= 1e-7 * np.linalg.norm(Jr)
    k = agreed_prefix(margins(Bo, po))
    np.testing.assert_array_equal(piv[:k], po[:k])
    scale = np.sqrt(np.max(np.diag(Bo)))
    assert np.max(np.abs(L[:k].T - Lo[:, :k])) <= 1e-7 * scale
    # the residual trace is below the tolerance on both sides
    assert res <= 1e-10 * np.trace(Bo) * (1 + 1e-6)


def margins_from_factor(diag, L, piv):
    """Decision margins of the oracle's pivot steps from its own factor: the
    residual diagonal before step r is diag - sum_{s<r} L_s^2."""
    d = np.array(diag, dtype=np.float64)
    out = []
    for r, p in enumerate(piv):
        dd = d.copy()
        dd[piv[:r]] = -np.inf
        top = np.sort(dd)[::-1][:2]
        out.append((top[0] - top[1]) / max(top[0], 1e-300) if len(top) > 1 else 1.0)
        d = d - L[:, r] ** 2
    return np.array(out)


@pytest.mark.slow
def test_fit_and_tei_cholesky_at_bench_size(tc, orc):
    """The benchmark's pipeline at full size (the 1024 products of the
    4096-cell workload, R_N = 32): per mode the 1D density fit (formed Gram
    A = F^T F on the device) against the oracle's fit, then the pivoted
    Cholesky of B (B formed on the device from the fitted Grams) against the
    oracle's Cholesky of its own factorised B, with the tolerances of the
    small pipeline test."""
    say("fit + TEI Cholesky at 4096 cells, 1024 products")
    w = wl.config("c3")
    c, ps = oracle_setup(orc, w)
    tol_fit = 1e-7
    Vo, Mo, fits = [], [], []
    for l in range(3):
        F = w.U[l]
        Uo, Vol, po, reso = orc.density_fit(F, tol_fit, w.n[l])
        fit = tc.density_fit(dev(F), tol_fit)
        U, V, piv, R, res = fit
        U, V = host(U), host(V)
        A_diag = np.sum(F * F, axis=0)
        # oracle factor of A for the margins: L = (F^T V) U-free form is not
        # returned, so the margins come from the pivots' residual diagonals
        k = min(len(po), R)
        same = int(np.argmax(piv[:k] != po[:k])) if np.any(piv[:k] != po[:k]) else k
        trA = float(A_diag.sum())
        err2 = float(np.sum((F - V[:, :R] @ U[:R]) ** 2))
        say(f"   mode {l}: R = {R} (oracle {len(po)}), first {same} pivots equal, "
            f"|F - VU|^2 / tr A = {err2 / trA:.2e}")
        assert err2 <= tol_fit ** 2 * trA * (1 + 1e-6) + 1e-28 * trA
        assert abs(err2 - res) <= 1e-9 * trA
        np.testing.assert_array_equal(V[:, :R], F[:, piv])
        assert same >= min(10, k)  # the leading, well separated pivots
        Vo.append(Vol)
        Mo.append(orc.gram(Uo, orc.convolve(ps[l], Uo)))
        fits.append(fit)
    # oracle B and its pivoted Cholesky
    Bo = orc.tei_matrix_factored(c, Vo, Mo)
    tol_b = 1e-10
    Lo, po, do = orc.pivoted_cholesky(Bo, tol_b * np.trace(Bo), Bo.shape[0])
    # GPU: the fitted rows' Grams from the TEI assembly, then the Cholesky
    R = max(f[3] for f in fits)
    Ud = [f[0][:R].contiguous() for f in fits]
    Vd = [f[1][:, :R].contiguous() for f in fits]
    J, G = tc.tei_gram(dev(c), [dev(p) for p in ps], Ud, prec="fp64", save_G=True)
    L, piv, res = tc.tei_cholesky(dev(c), Vd, [G[l].contiguous() for l in range(3)], tol_b)
    L = host(L)
    say(f"   R_B = {L.shape[0]} (oracle {len(po)})")
    nrm = np.linalg.norm(Bo)
    LL = L.T @ L
    assert np.linalg.norm(LL - Lo @ Lo.T) <= 1e-7 * nrm
    k = agreed_prefix(margins_from_factor(np.diag(Bo), Lo, po))
    say(f"   pivots agree on {k} decisive steps")
    np.testing.assert_array_equal(piv[:k], po[:k])
    scale = np.sqrt(np.max(np.diag(Bo)))
    assert np.max(np.abs(L[:k].T - Lo[:, :k])) <= 1e-7 * scale
    assert res <= tol_b * np.trace(Bo) * (1 + 1e-6) + 1e-7 * nrm
