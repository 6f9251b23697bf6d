"""Pins of the FP64 oracle against mathematics and the paper (CPU only).

Each test ties one oracle function to something other than itself: a
library routine for a special case, a closed form, an identity, an
invariant, or brute force on a small grid.  Together they are chosen so that
a plausible mistake anywhere in the oracle (a dropped term, a wrong sign or
index, a transposed operand, a missing h^3) fails at least one of them.
"""
import math
import os

import mpmath as mp
import numpy as np
import pytest

from paper_1504_06289_amd import workloads as wl
from tests.metrics import e_J

SQRTPI = math.sqrt(math.pi)


def accurate_rule(h, t_lo=1e-9, hu=0.25):
    """A fine sinc rule: nodes from t_lo (lower truncation error about
    1.13 t_lo r) to 2e4/h (the origin-cell error falls like (t_hi h)^-2) with
    step hu (discretisation error ~exp(-pi^2/hu))."""
    lo, hi = math.log(t_lo), math.log(2e4 / h)
    R_N = int(math.ceil((hi - lo) / hu)) + 1
    return R_N, lo, hu


# --------------------------------------------------------------------------
# Quadrature building blocks
# --------------------------------------------------------------------------
def test_gauss_legendre_matches_library(orc):
    x, w = orc.gauss_legendre(20)
    xr, wr = np.polynomial.legendre.leggauss(20)
    order = np.argsort(x)
    np.testing.assert_allclose(x[order], xr, rtol=0, atol=1e-15)
    np.testing.assert_allclose(w[order], wr, rtol=1e-13)
    # exact for polynomials of degree <= 39
    for k in range(20):
        assert abs(np.sum(w * x ** (2 * k)) - 2.0 / (2 * k + 1)) < 1e-14


def _cell_integral_mp(t, h, m):
    """(sqrt(pi)/2t)(erfc(alpha) - erfc(beta)) in 60-digit arithmetic (the
    complementary form keeps full relative precision in the far tail)."""
    m = abs(m)
    with mp.workdps(60):
        t, h = mp.mpf(t), mp.mpf(h)
        alpha = t * (m - mp.mpf(1) / 2) * h
        beta = t * (m + mp.mpf(1) / 2) * h
        return mp.sqrt(mp.pi) / (2 * t) * (mp.erfc(alpha) - mp.erfc(beta))


@pytest.mark.parametrize("t", [6.5e-6, 1e-3, 0.37, 2.0, 17.0, 183.0, 533.0])
@pytest.mark.parametrize("h", [0.15625, 0.0195, 0.005859375])
def test_cell_integral_vs_mpmath(orc, t, h):
    """Appendix 3, vector b(t_k): every evaluation branch (erf at the
    origin, erf / erfc differences, the flat-cell Gauss-Legendre form) against
    high-precision arithmetic."""
    for m in [0, 1, -1, 2, 3, 7, 31, 100, 1023, 4095]:
        ref = _cell_integral_mp(t, h, m)
        got = orc.cell_integral(t, h, m)
        if abs(ref) < 1e-300:      # below the smallest normal double
            assert abs(got) < 1e-300
            continue
        rel = abs((got - ref) / ref)
        # the value at the given doubles is conditioned like exp(-x^2) at
        # x = t(|m|+1/2)h: rounding the argument alone moves it by ~2x^2 ulp
        x = t * (abs(m) + 0.5) * h
        assert rel < 3e-15 + 4.5e-16 * 2 * x * x, (t, h, m, got, float(ref), float(rel))


@pytest.mark.parametrize("name", ["c1", "c3"])
def test_kernel_telescoping_and_symmetry(orc, name):
    """The cells tile [-(n-1/2)h, (n-1/2)h]: the sum over all lags is a single
    erf (an identity independent of the per-cell evaluation)."""
    w = wl.config(name) if name == "c1" else None
    if w is None:
        n, b, R_N = 4096, 12.0, 32
        u0, hu = wl.sinc_params(R_N, n, b)
    else:
        n, b, R_N, u0, hu = w.n[0], w.b, w.R_N, w.u0, w.hu
    h = 2 * b / n
    t, a, c, p = orc.newton_kernel(n, h, R_N, u0, hu)
    assert p.shape == (R_N, 2 * n - 1)
    np.testing.assert_array_equal(p, p[:, ::-1])            # p[-m] = p[m]
    np.testing.assert_allclose(c, a * h ** 3, rtol=1e-15)
    for k in range(R_N):
        tot = math.fsum(p[k])
        ref = SQRTPI / t[k] * math.erf(t[k] * (n - 0.5) * h)
        assert abs(tot - ref) / ref < 2e-14, (k, tot, ref)
        # bell shape: maximal at lag 0, non-increasing in |m|
        assert np.all(np.diff(p[k, n - 1:]) <= 0)


def test_sinc_rule_reproduces_inverse_distance(orc):
    """r * sum_k a_k exp(-t_k^2 r^2) -> 1 (eq. sinc_Newt) with the fitted
    parameters, and the error falls fast when the node density is raised
    over the same node range (the exponential sinc convergence)."""
    h, b = 20.0 / 128, 10.0
    r = np.logspace(np.log10(h / 2), np.log10(2 * np.sqrt(3) * b), 3000)

    def err(R_N, u0, hu):
        t, a = orc.sinc_rule(R_N, u0, hu)
        s = (a[None, :] * np.exp(-np.outer(r * r, t * t))).sum(1)
        return np.max(np.abs(r * s - 1))

    u0, hu = wl.sinc_params(20, 128, 10.0)
    assert err(20, u0, hu) < 1e-2
    # refine: same node range [lo, hi], more nodes, wider coverage
    lo, hi = math.log(1e-10), math.log(1e3)
    errs = []
    for R_N in (30, 45, 60, 90, 120):
        errs.append(err(R_N, lo, (hi - lo) / (R_N - 1)))
    assert errs[-1] < 3e-8, errs
    assert all(errs[i + 1] < errs[i] for i in range(len(errs) - 1))
    # the weights are the rule's: a_k = (2/sqrt(pi)) hu t_k
    t, a = orc.sinc_rule(5, -1.0, 0.25)
    np.testing.assert_allclose(t, np.exp(-1.0 + 0.25 * np.arange(5)), rtol=1e-15)
    np.testing.assert_allclose(a, 2 / SQRTPI * 0.25 * t, rtol=1e-15)


# --------------------------------------------------------------------------
# The 3D kernel against exact cell integrals of 1/|y|
# --------------------------------------------------------------------------
def _prism(x1, x2, y1, y2, z1, z2):
    """Exact integral of 1/|y| over a box (potential of a uniform prism)."""
    def F(x, y, z):
        r = mp.sqrt(x * x + y * y + z * z)
        s = mp.mpf(0)
        for c, v in ((y * z, x + r), (x * z, y + r), (x * y, z + r)):
            if c != 0:
                s += c * mp.log(v)
        for q, num, den in ((x, y * z, x * r), (y, x * z, y * r), (z, x * y, z * r)):
            if q != 0:
                s -= q * q / 2 * mp.atan(num / den)
        return s

    tot = mp.mpf(0)
    for x, sx in ((x2, 1), (x1, -1)):
        for y, sy in ((y2, 1), (y1, -1)):
            for z, sz in ((z2, 1), (z1, -1)):
                tot += sx * sy * sz * F(mp.mpf(x), mp.mpf(y), mp.mpf(z))
    return tot


def test_prism_formula_against_cubature():
    from scipy.integrate import tplquad
    with mp.workdps(30):
        got = float(_prism(0.5, 1.5, -0.5, 0.5, -0.5, 1.5))
    ref, err = tplquad(lambda z, y, x: 1 / math.sqrt(x * x + y * y + z * z),
                       0.5, 1.5, -0.5, 0.5, -0.5, 1.5, epsabs=1e-14, epsrel=1e-13)
    assert abs(got - ref) / ref < 1e-12
    with mp.workdps(30):
        assert abs(_prism(-.5, .5, -.5, .5, -.5, .5)
                   - (3 * mp.log(2 + mp.sqrt(3)) - mp.pi / 2)) < 1e-25


def test_origin_cell_identity(orc):
    """sum_k a_k p_k[0]^3 -> h^2 (3 ln(2+sqrt3) - pi/2) = integral of 1/|y|
    over the cell at the origin."""
    const = 3 * math.log(2 + math.sqrt(3)) - math.pi / 2
    assert abs(const - 2.3800773639795535) < 1e-15
    for h in (0.15625, 0.0195, 0.004):
        R_N, lo, hu = accurate_rule(h)
        t, a, c, p = orc.newton_kernel(8, h, R_N, lo, hu)
        val = math.fsum(a * p[:, 7] ** 3)
        assert abs(val / (h * h) - const) / const < 2e-7, (h, val / h / h)


def test_lag_kernel_vs_exact_prism(orc):
    """sum_k a_k prod_l p_k[m_l] against the exact cell integral of 1/|y| at
    a spread of lag vectors: pins the Galerkin kernel (with h^3 scaling)
    up to the sinc-quadrature error."""
    n, h = 64, 0.1
    R_N, lo, hu = accurate_rule(h)
    t, a, c, p = orc.newton_kernel(n, h, R_N, lo, hu)
    for m in [(0, 0, 0), (1, 0, 0), (1, 1, 1), (3, 2, 0), (10, 5, 7), (40, 0, 3), (-7, 2, -1),
              (63, 63, 63)]:
        val = math.fsum(a * p[:, m[0] + n - 1] * p[:, m[1] + n - 1] * p[:, m[2] + n - 1])
        with mp.workdps(40):
            ref = _prism(*[x for mm in m for x in ((mm - 0.5) * h, (mm + 0.5) * h)])
        assert abs(val - ref) / ref < 2e-7, (m, val, float(ref))
    # the fitted 20-term rule of the 128-cell workload: within its fit error
    w = wl.config("c1")
    h = 2 * w.b / 128
    t, a, c, p = orc.newton_kernel(128, h, w.R_N, w.u0, w.hu)
    for m in [(0, 0, 0), (2, 1, 0), (30, 20, 10), (100, 0, 0)]:
        val = math.fsum(a * p[:, m[0] + 127] * p[:, m[1] + 127] * p[:, m[2] + 127])
        with mp.workdps(40):
            ref = _prism(*[x for mm in m for x in ((mm - 0.5) * h, (mm + 0.5) * h)])
        assert abs(val - ref) / ref < 5e-3


# --------------------------------------------------------------------------
# Separable algebra: Toeplitz products, Grams, Hadamard sum
# --------------------------------------------------------------------------
def test_convolve_and_gram_against_dense_algebra(orc):
    """W_k = T_k U with T_k[a, b] = p_k[a-b], G_k = U^T W_k: an explicit dense
    Toeplitz matrix built with scipy and a matmul (library special case)."""
    from scipy.linalg import toeplitz
    rng = np.random.default_rng(3)
    n, R_f, R_N = 37, 5, 3
    p = rng.standard_normal((R_N, 2 * n - 1))
    p = 0.5 * (p + p[:, ::-1])
    U = rng.standard_normal((R_f, n))
    W = orc.convolve(p, U)
    G = orc.gram(U, W)
    for k in range(R_N):
        col = p[k, n - 1:]           # T[a, 0] = p[a]
        row = p[k, n - 1::-1]        # T[0, b] = p[-b]
        T = toeplitz(col, row)
        np.testing.assert_allclose(W[k], (T @ U.T).T, rtol=1e-13, atol=1e-13)
        np.testing.assert_allclose(G[k], U @ T @ U.T, rtol=1e-12, atol=1e-12)
    # asymmetric p pins the lag direction: W[a] = sum_b p[a-b] u[b]
    q = rng.standard_normal((1, 2 * n - 1))
    Wq = orc.convolve(q, U)
    Tq = toeplitz(q[0, n - 1:], q[0, n - 1::-1])
    np.testing.assert_allclose(Wq[0], (Tq @ U.T).T, rtol=1e-13, atol=1e-13)
    # plain (uncompensated) loops agree to rounding
    np.testing.assert_allclose(orc.convolve(p, U, compensated=False), W, rtol=1e-12, atol=1e-12)


def test_tei_gram_matches_bruteforce_3d(orc):
    """The factorised J against direct summation over the full 3D grid with
    the assembled 3D kernel: pins lag direction, mode pairing and h^3."""
    n, b, R_N = 14, 6.0, 10
    h = 2 * b / n
    u0, hu = wl.sinc_params(R_N, n, b)
    U, meta = wl.gaussian_products(n, b, 3, seed=11, alpha=(0.1, 3.0))
    t, a, c, p = orc.newton_kernel(n, h, R_N, u0, hu)
    J = orc.tei_gram(c, [p, p, p], U)
    Jb = orc.bruteforce_J(h, a, p, U)
    assert e_J(J, Jb) < 1e-13
    # symmetric up to rounding
    assert np.max(np.abs(J - J.T)) <= 1e-14 * np.max(np.abs(J))


def _boys_ssss(a1, A1, a2, A2):
    """(ss|ss) for unnormalised s Gaussians: 2 pi^{5/2}/(pq sqrt(p+q)) F0(T)."""
    with mp.workdps(40):
        p, q = mp.mpf(a1), mp.mpf(a2)
        R2 = sum((mp.mpf(x) - mp.mpf(y)) ** 2 for x, y in zip(A1, A2))
        T = p * q / (p + q) * R2
        F0 = mp.mpf(1) if T == 0 else mp.sqrt(mp.pi / T) * mp.erf(mp.sqrt(T)) / 2
        return 2 * mp.pi ** mp.mpf(2.5) / (p * q * mp.sqrt(p + q)) * F0


@pytest.mark.slow
def test_tei_gram_boys_closed_form_h2(orc):
    """J -> the Gaussian-Gaussian Coulomb integral (Boys function) with an
    O(h^2) discretisation error (the accuracy of the collocated grid
    representation), once the quadrature error is negligible."""
    b = 10.0
    alphas = np.array([0.6, 1.3, 0.8, 2.0])
    centres = np.array([[0.3, -0.4, 0.1], [-1.1, 0.7, 0.5], [1.4, 1.0, -0.8], [0.0, 0.2, 0.0]])
    ref = np.array([[float(_boys_ssss(alphas[i], centres[i], alphas[j], centres[j]))
                     for j in range(4)] for i in range(4)])
    errs = []
    Js = {}
    for n in (64, 128, 256, 512):
        h = 2 * b / n
        R_N, lo, hu = accurate_rule(h)
        t, a, c, p = orc.newton_kernel(n, h, R_N, lo, hu)
        U, _ = wl.s_gaussians(n, b, 4, alphas=alphas, centres=centres)
        J = orc.tei_gram(c, [p, p, p], U)
        Js[n] = J
        errs.append(np.max(np.abs(J - ref) / np.abs(ref)))
    ratios = [errs[i] / errs[i + 1] for i in range(3)]
    assert errs[-1] < 2e-4
    for r in ratios[1:]:
        assert 3.5 < r < 4.6, (errs, ratios)
    rich = (4 * Js[512] - Js[256]) / 3
    assert np.max(np.abs(rich - ref) / np.abs(ref)) < 2e-6, errs


def test_coulomb_of_product_density_is_J_times_d(orc):
    """A density expanded in the product functions themselves (V = U, weights
    d) gives Jd = J d with the J of the TEI assembly: the Hartree-potential
    route and the factorised TEI matrix compute the same integrals."""
    w = wl.small_products((40, 33, 47), 21, R_N=9, b=7.0, seed=6)
    ps, c = [], None
    for l in range(3):
        t, a, cc, p = orc.newton_kernel(w.n[l], w.h[l], w.R_N, w.u0, w.hu)
        ps.append(p)
    c = a * w.h[0] * w.h[1] * w.h[2]
    d = np.random.default_rng(3).standard_normal(w.R_f)
    Jd = orc.coulomb(c, ps, w.U, w.U, d)
    J = orc.tei_gram(c, ps, w.U)
    bound = 1e-13 * (np.abs(J) @ np.abs(d))
    assert np.all(np.abs(Jd - J @ d) <= bound)
    # a density of a subset of the products: the matching columns of J
    sel = [2, 5, 11]
    Jd2 = orc.coulomb(c, ps, w.U, [u[sel] for u in w.U], d[sel])
    assert np.all(np.abs(Jd2 - J[:, sel] @ d[sel]) <= 1e-13 * (np.abs(J[:, sel]) @ np.abs(d[sel])))


@pytest.mark.slow
def test_coulomb_boys_closed_form_h2(orc):
    """An s-Gaussian density against s-Gaussian functions: the Coulomb
    entries converge to the Boys closed form at O(h^2)."""
    b = 10.0
    alphas = np.array([0.6, 1.3, 0.8])
    centres = np.array([[0.3, -0.4, 0.1], [-1.1, 0.7, 0.5], [1.4, 1.0, -0.8]])
    dal = np.array([0.9, 1.7])
    dcen = np.array([[0.2, 0.1, -0.3], [-0.5, 0.8, 0.4]])
    d = np.array([1.5, -0.7])
    ref = np.array([sum(d[m] * float(_boys_ssss(alphas[i], centres[i], dal[m], dcen[m]))
                        for m in range(2)) for i in range(3)])
    errs, Js = [], {}
    for n in (64, 128, 256, 512):
        h = 2 * b / n
        R_N, lo, hu = accurate_rule(h)
        t, a, c, p = orc.newton_kernel(n, h, R_N, lo, hu)
        U, _ = wl.s_gaussians(n, b, 3, alphas=alphas, centres=centres)
        V, _ = wl.s_gaussians(n, b, 2, alphas=dal, centres=dcen)
        Jd = orc.coulomb(c, [p, p, p], U, V, d)
        Js[n] = Jd
        errs.append(np.max(np.abs(Jd - ref) / np.abs(ref)))
    ratios = [errs[i] / errs[i + 1] for i in range(3)]
    assert errs[-1] < 2e-4
    for r in ratios[1:]:
        assert 3.5 < r < 4.6, (errs, ratios)
    rich = (4 * Js[512] - Js[256]) / 3
    assert np.max(np.abs(rich - ref) / np.abs(ref)) < 2e-6, errs


def test_pivoted_cholesky_is_greedy_schur_complement(orc):
    """Pivoted Cholesky against its definition: after r steps the residual
    A - L L^T is the Schur complement of A on the pivots (zero rows and
    columns there), the next pivot is its largest diagonal entry, L is
    triangular in pivot order, and a rank-r matrix is recovered exactly."""
    rng = np.random.default_rng(1)
    X = rng.standard_normal((40, 9))
    A = X @ X.T
    L, piv, d = orc.pivoted_cholesky(A, 1e-10 * np.trace(A), 40)
    assert len(piv) == 9 and len(set(piv.tolist())) == 9
    assert np.max(np.abs(A - L @ L.T)) <= 1e-12 * np.max(np.abs(A))
    for r in range(9):
        assert np.all(L[piv[r], r + 1:] == 0.0)
    # truncated: explicit Schur complement on the first pivots
    L4, piv4, d4 = orc.pivoted_cholesky(A, 0.0, 4)
    P = piv4
    S = A - A[:, P] @ np.linalg.solve(A[np.ix_(P, P)], A[P, :])
    np.testing.assert_allclose(A - L4 @ L4.T, S, atol=1e-10 * np.max(np.abs(A)))
    np.testing.assert_allclose(d4, np.diag(S), atol=1e-10 * np.max(np.abs(A)))
    for r in range(4):   # each pivot maximises the residual diagonal of its step
        Pr = P[:r]
        Sr = A - (A[:, Pr] @ np.linalg.solve(A[np.ix_(Pr, Pr)], A[Pr, :]) if r else 0.0)
        assert P[r] == int(np.argmax(np.diag(Sr)))


def test_density_fit_error_identity_and_interpolation(orc):
    """F ~ V U with V = F[:, P] and U = A_PP^-1 A_P: interpolates at the
    pivot points (U[:, P] = I), and |F - V U|_F^2 equals the residual trace
    of the pivoted Cholesky of A = F^T F, which the tolerance bounds."""
    n = 96
    U0, _ = wl.gaussian_products(n, 8.0, 60, seed=4)
    for F in U0:
        for tol in (1e-3, 1e-6):
            U, V, piv, res = orc.density_fit(F, tol, n)
            R = len(piv)
            assert 0 < R < n
            np.testing.assert_array_equal(V, F[:, piv])
            np.testing.assert_allclose(U[:, piv], np.eye(R), atol=1e-9)
            err2 = np.sum((F - V @ U) ** 2)
            trA = np.sum(F * F)
            assert abs(err2 - res) <= 1e-9 * trA
            assert err2 <= tol * tol * trA * (1 + 1e-6)


def test_factored_tei_matrix_with_fitted_modes_is_J(orc):
    """With each mode's side matrix fitted to 1e-10 and M_k = U T_k U^T from
    the convolution and Gram of the fitted rows, the factorised
    B = sum_k c_k o_l V M_k V^T reproduces J of the TEI assembly."""
    w = wl.small_products((48, 40, 56), 30, R_N=8, b=7.0, seed=9)
    ps = []
    for l in range(3):
        t, a, cc, p = orc.newton_kernel(w.n[l], w.h[l], w.R_N, w.u0, w.hu)
        ps.append(p)
    c = a * w.h[0] * w.h[1] * w.h[2]
    J = orc.tei_gram(c, ps, w.U)
    for tol in (1e-6, 1e-10):
        V3, M3 = [], []
        for l in range(3):
            U, V, piv, res = orc.density_fit(w.U[l], tol, w.n[l])
            V3.append(V)
            M3.append(orc.gram(U, orc.convolve(ps[l], U)))
        B = orc.tei_matrix_factored(c, V3, M3)
        # the fit error of each side matrix is tol relative (Frobenius)
        assert np.linalg.norm(B - J) <= max(10 * tol, 1e-11) * np.linalg.norm(J)
    # and the pivoted Cholesky of B: residual diagonal bounds every entry
    L, piv, d = orc.tei_cholesky(c, V3, M3, 1e-8 * np.trace(B), B.shape[0])
    S = B - L @ L.T
    assert np.all(np.abs(S) <= np.sqrt(np.outer(np.abs(np.diag(S)), np.abs(np.diag(S)))) +
                  1e-12 * np.max(np.abs(B)))
    assert d.sum() <= 1e-8 * np.trace(B)
    assert len(piv) < B.shape[0]


def test_lattice_sum_is_the_separable_lattice_loop(orc):
    """The assembled vectors of each direction reproduce, through the rank-R
    product, the kernel summed over every lattice point one by one (the sum
    over a Cartesian lattice of products is the product of the sums)."""
    n0, L3 = 5, (3, 4, 2)
    b = 2.0
    h = b / n0
    R_N, lo, hu = 14, math.log(0.05), 0.45
    p3, hs = [], []
    for l in range(3):
        n = n0 * L3[l]
        t, a, c, p = orc.newton_kernel(n, h, R_N, lo, hu)
        p3.append(p)
        hs.append(h)
    c = a * h ** 3
    A3 = [orc.lattice_sum(p3[l], n0, L3[l]) for l in range(3)]
    rng = np.random.default_rng(2)
    pts = [tuple(int(rng.integers(0, n0 * L3[l])) for l in range(3)) for _ in range(12)]
    w = c / h ** 6
    V = np.array([np.sum(w * A3[0][:, i] * A3[1][:, j] * A3[2][:, k]) for (i, j, k) in pts])
    Vd = orc.lattice_potential_direct(c, p3, hs, n0, L3, pts)
    assert np.max(np.abs(V - Vd) / np.abs(Vd)) <= 1e-13
    # the entry-wise form (used to sample the full-size lattice sum) through
    # the same identity: its entries rebuild the point potentials
    Ve = []
    for (i, j, k) in pts:
        cols = []
        for l, x in enumerate((i, j, k)):
            v, sc = orc.lattice_sum_entries(p3[l], n0, L3[l], [(q, x) for q in range(R_N)])
            assert np.all(np.abs(v) <= sc)
            cols.append(v)
        Ve.append(np.sum(w * cols[0] * cols[1] * cols[2]))
    assert np.max(np.abs(np.array(Ve) - Vd) / np.abs(Vd)) <= 1e-13


@pytest.mark.slow
def test_lattice_potential_and_energy_against_coulomb_sums(orc):
    """The lattice-summed kernel against the Coulomb sum sum_j 1/|x - x_j| at
    grid points at least b/2 from every charge, and the pair energy
    Z^2/2 sum_{k != j} K(x_k - x_j) against the exact Coulomb lattice energy
    (O(h^4) here: the cell average of a harmonic function has no h^2 term),
    with Richardson extrapolation."""
    b, L3, Z = 2.0, (3, 3, 2), 1.0
    Eex = orc.coulomb_lattice_energy_exact(b, L3, Z)
    errs, Es = [], {}
    for n0 in (4, 8, 16):
        h = b / n0
        R_N, lo, hu = accurate_rule(h)
        p3 = []
        for l in range(3):
            t, a, c, p = orc.newton_kernel(n0 * L3[l], h, R_N, lo, hu)
            p3.append(p)
        c = a * h ** 3
        E = orc.lattice_energy_direct(c, p3, [h, h, h], n0, L3, Z)
        Es[n0] = E
        errs.append(abs(E - Eex) / Eex)
        if n0 == 8:
            # potential at a few grid points away from the charges
            grid = [(np.arange(n0 * Ll) + 0.5) * h for Ll in L3]
            charges = np.stack(np.meshgrid(*[(np.arange(Ll) * n0 + n0 // 2 + 0.5) * h
                                             for Ll in L3], indexing="ij"), -1).reshape(-1, 3)
            rng = np.random.default_rng(4)
            pts = []
            while len(pts) < 4:
                cand = tuple(int(rng.integers(0, n0 * Ll)) for Ll in L3)
                x = np.array([grid[0][cand[0]], grid[1][cand[1]], grid[2][cand[2]]])
                if np.sqrt(np.sum((charges - x) ** 2, axis=1)).min() >= b / 2:
                    pts.append(cand)
            Vd = orc.lattice_potential_direct(c, p3, [h, h, h], n0, L3, pts)
            for (i, j, k), v in zip(pts, Vd):
                x = np.array([grid[0][i], grid[1][j], grid[2][k]])
                dist = np.sqrt(np.sum((charges - x) ** 2, axis=1))
                assert abs(v - np.sum(1.0 / dist)) <= 5e-3 * np.sum(1.0 / dist)
    # the cell average of the harmonic 1/|x| has no h^2 term away from the
    # origin, so the pair energy converges at O(h^4)
    ratios = [errs[i] / errs[i + 1] for i in range(2)]
    assert errs[-1] < 1e-6
    for r in ratios:
        assert 12.0 < r < 20.0, (errs, ratios)
    rich = (16 * Es[16] - Es[8]) / 15
    assert abs(rich - Eex) / Eex < errs[-1] / 5, (errs, rich, Eex)


def test_J_symmetric_psd_products(orc):
    """J = J^T, J_ii > 0 and J is positive semi-definite up to rounding (each
    T_k is positive definite, Schur products of PSD matrices are PSD and
    c_k > 0)."""
    w = wl.small_products(96, 24, R_N=12, b=8.0, seed=5)
    h = w.h[0]
    t, a, c, p = orc.newton_kernel(w.n[0], h, w.R_N, w.u0, w.hu)
    assert np.all(c > 0)
    J = orc.tei_gram(c, [p, p, p], w.U)
    assert np.max(np.abs(J - J.T)) <= 1e-15 * np.max(np.abs(J))
    assert np.all(np.diag(J) > 0)
    lam = np.linalg.eigvalsh(0.5 * (J + J.T))
    assert lam[0] >= -1e-13 * lam[-1]
    # Cauchy-Schwarz bound that the normalised metric relies on
    d = np.sqrt(np.diag(J))
    assert np.all(np.abs(J) <= np.outer(d, d) * (1 + 1e-12))


def test_tei_gram_columns_match_full(orc):
    w = wl.small_products((40, 33, 47), 9, R_N=7, b=7.0, seed=2)
    ps, c = [], None
    for l in range(3):
        t, a, cc, p = orc.newton_kernel(w.n[l], w.h[l], w.R_N, w.u0, w.hu)
        ps.append(p)
    c = a * w.h[0] * w.h[1] * w.h[2]
    J, G = orc.tei_gram(c, ps, w.U, return_G=True)
    cols = [0, 4, 8]
    Jc = orc.tei_gram_columns(c, ps, w.U, cols)
    np.testing.assert_allclose(Jc, J[:, cols].T, rtol=1e-14, atol=0)
    # G symmetric per mode and term
    np.testing.assert_allclose(G, np.swapaxes(G, 2, 3), rtol=1e-13, atol=1e-300)


# --------------------------------------------------------------------------
# Potential factors (tc_convolve): the Hartree potential of one Gaussian
# --------------------------------------------------------------------------
def test_potential_factors_give_gaussian_potential(orc):
    """V(x) = sum_k a_k prod_l W^l_k[x_l] (eq. conv with the canonical kernel)
    approximates the potential of exp(-alpha|x-A|^2), which is
    (pi/alpha)^{3/2} erf(sqrt(alpha)|x-A|)/|x-A|."""
    n, b = 256, 10.0
    h = 2 * b / n
    R_N, lo, hu = accurate_rule(h)
    t, a, c, p = orc.newton_kernel(n, h, R_N, lo, hu)
    alpha, A = np.array([0.9]), np.array([[0.2, -0.3, 0.45]])
    U, _ = wl.s_gaussians(n, b, 1, alphas=alpha, centres=A)
    Ws = [orc.convolve(p, U[l]) for l in range(3)]
    x = wl.grid(n, b)
    worst = 0.0
    for idx in [(128, 128, 128), (100, 140, 129), (60, 200, 130), (10, 128, 240)]:
        V = math.fsum(a[k] * Ws[0][k, 0, idx[0]] * Ws[1][k, 0, idx[1]] * Ws[2][k, 0, idx[2]]
                      for k in range(R_N))
        r = math.sqrt(sum((x[idx[l]] - A[0, l]) ** 2 for l in range(3)))
        ref = (math.pi / alpha[0]) ** 1.5 * math.erf(math.sqrt(alpha[0]) * r) / r
        worst = max(worst, abs(V - ref) / ref)
    assert worst < 2e-3


# --------------------------------------------------------------------------
# Adjoint
# --------------------------------------------------------------------------
def test_backward_matches_central_differences(orc):
    """f = w^T J w is quadratic in every single entry of U^l, so the central
    difference is exact up to rounding of the compensated forward."""
    w = wl.small_products((24, 19, 28), 6, R_N=6, b=6.0, seed=9)
    ps = []
    for l in range(3):
        t, a, cc, p = orc.newton_kernel(w.n[l], w.h[l], w.R_N, w.u0, w.hu)
        ps.append(p)
    c = a * w.h[0] * w.h[1] * w.h[2]
    rng = np.random.default_rng(4)
    wv = rng.standard_normal(w.R_f)
    dU = orc.tei_gram_backward(c, ps, w.U, np.outer(wv, wv))

    def f(U3):
        return float(wv @ orc.tei_gram(c, ps, U3) @ wv)

    for l in range(3):
        for (i, a_) in [(0, 3), (2, w.n[l] // 2), (5, w.n[l] - 1), (3, 7)]:
            delta = 1e-3 * max(abs(w.U[l][i, a_]), 1e-3)
            Up = [u.copy() for u in w.U]
            Um = [u.copy() for u in w.U]
            Up[l][i, a_] += delta
            Um[l][i, a_] -= delta
            fd = (f(Up) - f(Um)) / (2 * delta)
            scale = np.max(np.abs(dU[l]))
            assert abs(fd - dU[l][i, a_]) <= 1e-9 * scale, (l, i, a_, fd, dU[l][i, a_])
    # a non-symmetric Jbar is symmetrised by the adjoint
    Jb = rng.standard_normal((w.R_f, w.R_f))
    d1 = orc.tei_gram_backward(c, ps, w.U, Jb)
    d2 = orc.tei_gram_backward(c, ps, w.U, 0.5 * (Jb + Jb.T))
    for l in range(3):
        np.testing.assert_allclose(d1[l], d2[l], rtol=1e-13, atol=1e-13 * np.abs(d2[l]).max())


def _boys_ssss_grad(a1, A1, a2, A2):
    """Analytic derivatives of (ss|ss) = K F0(T), K = 2 pi^{5/2}/(p q sqrt(p+q)),
    T = p q/(p+q) |A1-A2|^2, with respect to the first Gaussian's centre A1
    (3 components) and exponent p = a1, using F0'(T) = -F1(T) and
    F1(T) = (F0(T) - e^-T)/(2T)  (F1(0) = 1/3).  Returns (dA1 [3], dp)."""
    with mp.workdps(40):
        p, q = mp.mpf(a1), mp.mpf(a2)
        D = [mp.mpf(x) - mp.mpf(y) for x, y in zip(A1, A2)]
        R2 = sum(d * d for d in D)
        rho = p * q / (p + q)
        T = rho * R2
        if T == 0:
            F0, F1 = mp.mpf(1), mp.mpf(1) / 3
        else:
            F0 = mp.sqrt(mp.pi / T) * mp.erf(mp.sqrt(T)) / 2
            F1 = (F0 - mp.exp(-T)) / (2 * T)
        K = 2 * mp.pi ** mp.mpf(2.5) / (p * q * mp.sqrt(p + q))
        # dT/dA1 = 2 rho (A1 - A2);  dT/dp = q^2/(p+q)^2 |A1-A2|^2
        dA = [float(K * (-F1) * 2 * rho * d) for d in D]
        dK_dp = -K / p - K / (2 * (p + q))
        dp = dK_dp * F0 + K * (-F1) * (q * q / (p + q) ** 2) * R2
        return np.array(dA), float(dp)


@pytest.mark.slow
def test_backward_boys_gradient_h2(orc):
    """The adjoint, chained through the grid functions, reproduces the
    analytic centre and exponent derivatives of the Boys closed form.
    For f = w^T J w of s Gaussians U^l[i][a] = exp(-alpha_i (x_a - A_il)^2):
      df/dA_il   = sum_a dU^l[i][a] 2 alpha_i (x_a - A_il) U^l[i][a],
      df/dalpha_i = -sum_l sum_a dU^l[i][a] (x_a - A_il)^2 U^l[i][a],
    against 2 w_i sum_{j != i} w_j dJ_ij/dA_i (dJ_ii/dA_i = 0) and
    2 w_i sum_{j != i} w_j dJ_ij/dalpha_i + w_i^2 dJ_ii/dalpha_i, where
    J_ii = 2 pi^{5/2} (2 alpha_i)^{-1/2} alpha_i^{-2} gives
    dJ_ii/dalpha_i = -(5/2) J_ii/alpha_i.  The grid error is O(h^2)
    (ratio ~4 per halving of h) and Richardson extrapolation removes it down
    to the quadrature floor, as for J itself."""
    b = 10.0
    alphas = np.array([0.6, 1.3, 0.8, 2.0])
    centres = np.array([[0.3, -0.4, 0.1], [-1.1, 0.7, 0.5], [1.4, 1.0, -0.8], [0.0, 0.2, 0.0]])
    w = np.array([0.7, -1.2, 0.4, 0.9])
    F = len(alphas)
    gA = np.zeros((F, 3))
    ga = np.zeros(F)
    for i in range(F):
        for j in range(F):
            if j == i:
                Jii = float(_boys_ssss(alphas[i], centres[i], alphas[i], centres[i]))
                ga[i] += w[i] * w[i] * (-2.5 * Jii / alphas[i])
                continue
            dA, dp = _boys_ssss_grad(alphas[i], centres[i], alphas[j], centres[j])
            gA[i] += 2 * w[i] * w[j] * dA
            ga[i] += 2 * w[i] * w[j] * dp
    ref = np.concatenate([gA.ravel(), ga])
    scale = np.abs(ref).max()
    got = {}
    errs = []
    for n in (64, 128, 256, 512):
        h = 2 * b / n
        R_N, lo, hu = accurate_rule(h)
        t, a, c, p = orc.newton_kernel(n, h, R_N, lo, hu)
        U, _ = wl.s_gaussians(n, b, F, alphas=alphas, centres=centres)
        dU = orc.tei_gram_backward(c, [p, p, p], U, np.outer(w, w))
        x = wl.grid(n, b)
        dA = np.zeros((F, 3))
        dal = np.zeros(F)
        for l in range(3):
            dx = x[None, :] - centres[:, l, None]                  # [F][n]
            dA[:, l] = np.sum(dU[l] * 2 * alphas[:, None] * dx * U[l], axis=1)
            dal -= np.sum(dU[l] * dx * dx * U[l], axis=1)
        g = np.concatenate([dA.ravel(), dal])
        got[n] = g
        errs.append(np.abs(g - ref).max() / scale)
    ratios = [errs[i] / errs[i + 1] for i in range(3)]
    # measured: 1.4e-3, 3.6e-4, 8.9e-5, 2.2e-5 (ratios 4.0); Richardson 1.4e-8
    assert errs[-1] < 4e-5, errs
    for r in ratios:
        assert 3.8 < r < 4.2, (errs, ratios)
    rich = (4 * got[512] - got[256]) / 3
    assert np.abs(rich - ref).max() / scale < 2e-7, (errs, np.abs(rich - ref).max() / scale)
    # a sign or factor slip in the chain (e.g. dropping the factor 2 of the
    # symmetric adjoint) would move the result by O(1), far beyond these bounds


# --------------------------------------------------------------------------
# Input recipe against values printed in the paper
# --------------------------------------------------------------------------
def test_grid_reproduces_printed_mesh_sizes():
    """The cell-centred grid h = 2b/n on [-b, b] gives the mesh sizes that
    Section 3.2 prints for its H2O grids in the box [-20,20]^3, to the digits
    printed (fixture tests/golden/tei_mesh_sizes.txt)."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "tei_mesh_sizes.txt")
    rows = [line.split() for line in open(path) if line.strip() and not line.startswith("#")]
    assert len(rows) == 4
    for n, printed, digits in rows:
        n, printed, digits = int(n), float(printed), int(digits)
        x = wl.grid(n, 20.0)
        h = x[1] - x[0]
        assert math.isclose(h, 40.0 / n, rel_tol=1e-12)
        assert x[0] == pytest.approx(-20.0 + h / 2, abs=1e-12)
        assert float(f"{h:.{digits}g}") == printed

def _lattice_table():
    path = os.path.join(os.path.dirname(__file__), "golden", "lattice_energy_table.txt")
    rows = []
    for line in open(path):
        if line.strip() and not line.startswith("#"):
            L, E, digits, reading = line.split()
            rows.append((int(L), float(E), int(digits), reading))
    return rows


def printed_value_holds(E, printed, digits, reading):
    """E agrees with a value printed to `digits` significant digits, to within
    one unit of the last printed digit."""
    if reading != "digit":
        raise ValueError(reading)
    ulp = 10.0 ** (math.floor(math.log10(abs(printed))) - digits + 1)
    return abs(E - printed) < ulp


@pytest.mark.slow
def test_exact_lattice_energy_against_printed_table(orc):
    """The exact Coulomb energy 1/2 sum_{k != j} 1/|x_k - x_j| of the 24^3
    hydrogen lattice of Section 5.2 (Z = 1, spacing 2 bohr), pair by pair,
    against the energy printed there (fixture
    tests/golden/lattice_energy_table.txt; the tensor values printed agree
    with direct summation to 2e-8).  The larger lattices are checked on the
    GPU path, whose energy is O(L) per term."""
    rows = {r[0]: r for r in _lattice_table()}
    for L in (24,):
        _, printed, digits, reading = rows[L]
        E = orc.coulomb_lattice_energy_exact(2.0, (L, L, L), 1.0)
        assert printed_value_holds(E, printed, digits, reading), (L, E, printed)


def test_lattice_energy_by_lags_is_the_pair_sum(orc):
    """Grouping the pairs of a lattice by lag changes only the order of the
    sum: brute force over all ordered pairs on small rectangular lattices."""
    for b, L3, Z in [(2.0, (1, 1, 1), 1.0), (1.5, (2, 3, 4), 2.0), (0.7, (5, 1, 3), -1.0),
                     (2.0, (6, 7, 5), 1.0)]:
        El = orc.coulomb_lattice_energy_lags(b, L3, Z)
        Ep = orc.coulomb_lattice_energy_exact(b, L3, Z)
        assert abs(El - Ep) <= 1e-13 * max(abs(Ep), 1.0), (L3, El, Ep)


def test_nuclear_matrix_is_the_grid_sum(orc):
    """The separable nuclear-potential matrix against the potential formed on
    the whole 3D grid and integrated cell by cell (tiny grids, unequal modes,
    nuclei on the boundary cells too)."""
    rng = np.random.default_rng(5)
    n3, b = (9, 7, 8), 3.0
    h3 = [2 * b / nl for nl in n3]
    R_N = 6
    p3 = []
    for l in range(3):
        t, a, c, p = orc.newton_kernel(n3[l], h3[l], R_N, -2.0, 0.6)
        p3.append(p)
    c = a * h3[0] * h3[1] * h3[2]
    U3 = [rng.standard_normal((5, nl)) for nl in n3]
    Z = np.array([1.0, 8.0, 2.5])
    pos = [(0, 6, 3), (4, 3, 7), (8, 0, 0)]
    V = orc.nuclear(c, p3, h3, U3, Z, pos)
    Vb = orc.nuclear_bruteforce(c, p3, h3, U3, Z, pos)
    assert np.max(np.abs(V - Vb)) <= 1e-12 * np.max(np.abs(Vb))
    assert np.max(np.abs(V - V.T)) <= 1e-14 * np.max(np.abs(V))
    # the entry-wise form (used to sample the full-size matrix) against the
    # same grid sum, with its scale bounding every entry
    pairs = [(k, m) for k in range(5) for m in range(5)]
    Ve, sc = orc.nuclear_entries(c, p3, h3, U3, Z, pos, pairs)
    Vbe = np.array([Vb[k, m] for k, m in pairs])
    assert np.max(np.abs(Ve - Vbe)) <= 1e-12 * np.max(np.abs(Vb))
    assert np.all(np.abs(Ve) <= sc * (1 + 1e-12))


def _nuclear_ss(a1, A1, a2, A2, C):
    """Nuclear attraction of two unnormalised s Gaussians with a unit charge
    at C: -(2 pi / p) exp(-a1 a2/p |A1 - A2|^2) F0(p |P - C|^2)."""
    with mp.workdps(40):
        a1, a2 = mp.mpf(a1), mp.mpf(a2)
        p = a1 + a2
        AB2 = sum((mp.mpf(x) - mp.mpf(y)) ** 2 for x, y in zip(A1, A2))
        P = [(a1 * mp.mpf(x) + a2 * mp.mpf(y)) / p for x, y in zip(A1, A2)]
        T = p * sum((Pi - mp.mpf(ci)) ** 2 for Pi, ci in zip(P, C))
        F0 = mp.mpf(1) if T == 0 else mp.sqrt(mp.pi / T) * mp.erf(mp.sqrt(T)) / 2
        return -2 * mp.pi / p * mp.exp(-a1 * a2 / p * AB2) * F0


@pytest.mark.slow
def test_nuclear_matrix_boys_closed_form_h2(orc):
    """s Gaussians against two nuclei at cell centres: the matrix converges to
    the closed-form nuclear attraction integrals at O(h^2) (the cell average of
    1/|x| is integrated exactly, the smooth factor by the midpoint rule)."""
    b = 10.0
    alphas = np.array([0.6, 1.3, 0.8])
    centres = np.array([[0.3, -0.4, 0.1], [-1.1, 0.7, 0.5], [1.4, 1.0, -0.8]])
    Z = np.array([1.0, 3.0])
    targets = np.array([[0.37, -0.52, 0.21], [-0.8, 0.6, -0.3]])
    errs = []
    for n in (64, 128, 256, 512):
        h = 2 * b / n
        R_N, lo, hu = accurate_rule(h)
        t, a, c, p = orc.newton_kernel(n, h, R_N, lo, hu)
        U, _ = wl.s_gaussians(n, b, 3, alphas=alphas, centres=centres)
        pos = [tuple(int(np.floor((x + b) / h)) for x in tg) for tg in targets]
        C = [[-b + (i + 0.5) * h for i in ps] for ps in pos]
        ref = np.array([[float(sum(Z[g] * _nuclear_ss(alphas[i], centres[i], alphas[j],
                                                       centres[j], C[g]) for g in range(2)))
                         for j in range(3)] for i in range(3)])
        V = orc.nuclear(c, [p, p, p], [h, h, h], U, Z, pos)
        errs.append(np.max(np.abs(V - ref) / np.abs(ref)))
    ratios = [errs[i] / errs[i + 1] for i in range(3)]
    assert errs[-1] < 2e-4, errs
    for r in ratios[1:]:
        assert 3.5 < r < 4.6, (errs, ratios)


def test_canonical_to_tucker_recovers_low_multilinear_rank(orc):
    """A canonical tensor of rank 40 whose side matrices span r_l-dimensional
    subspaces has multilinear rank (r1, r2, r3): the transform with those ranks
    reproduces the full tensor, with orthonormal bases, for any sweep count;
    with ranks equal to n_l it is exact as well."""
    rng = np.random.default_rng(7)
    n3, r3, R = (11, 9, 13), (3, 4, 5), 40
    A3 = [rng.standard_normal((R, r3[l])) @ rng.standard_normal((r3[l], n3[l])) for l in range(3)]
    c = rng.uniform(0.5, 2.0, R)
    T = orc.canonical_full(c, A3)
    for m_max in (0, 1, 3):
        Z3, beta, sv = orc.canonical_to_tucker(c, A3, r3, m_max)
        for l in range(3):
            np.testing.assert_allclose(Z3[l] @ Z3[l].T, np.eye(r3[l]), atol=1e-13)
        assert np.max(np.abs(orc.tucker_full(Z3, beta) - T)) <= 1e-12 * np.max(np.abs(T))
    Z3, beta, sv = orc.canonical_to_tucker(c, A3, n3, 1)
    assert np.max(np.abs(orc.tucker_full(Z3, beta) - T)) <= 1e-12 * np.max(np.abs(T))
    # the epsilon truncation finds the multilinear rank from larger maximal ranks
    Z3, beta, sv = orc.canonical_to_tucker(c, A3, (7, 8, 9), 2, eps=1e-10)
    assert [int(np.sum(np.linalg.norm(z, axis=1) > 0.5)) for z in Z3] == list(r3)
    assert np.max(np.abs(orc.tucker_full(Z3, beta) - T)) <= 1e-12 * np.max(np.abs(T))


def test_canonical_to_tucker_sweep_is_the_unfolding_svd(orc):
    """One alternating step against the full tensor: after a sweep, Z^3 spans
    the dominant left singular vectors of the mode-3 unfolding of the full
    tensor projected onto Z^1, Z^2 (formed in 3D), and the core is the full
    tensor projected onto all three bases."""
    rng = np.random.default_rng(8)
    n3, R, r3 = (10, 12, 8), 30, (4, 3, 5)
    A3 = [rng.standard_normal((R, n3[l])) for l in range(3)]
    c = rng.standard_normal(R)
    T = orc.canonical_full(c, A3)
    Z3, beta, sv = orc.canonical_to_tucker(c, A3, r3, 1)
    # the bases of modes 1, 2 at the time mode 3 was updated are the final ones
    P = np.einsum("abc,ia,jb->ijc", T, Z3[0], Z3[1]).reshape(-1, n3[2])   # [(i j)][c]
    u, s, vt = np.linalg.svd(P.T, full_matrices=False)
    Pz = Z3[2].T @ Z3[2]
    Pu = u[:, :r3[2]] @ u[:, :r3[2]].T
    assert np.max(np.abs(Pz - Pu)) <= 1e-12
    np.testing.assert_allclose(sv[2][:r3[2]], s[:r3[2]], rtol=1e-12)
    beta_ref = np.einsum("abc,ia,jb,mc->ijm", T, Z3[0], Z3[1], Z3[2])
    assert np.max(np.abs(beta - beta_ref)) <= 1e-12 * np.max(np.abs(beta_ref))
    # the sweep does not increase the error of the first (RHOSVD) step
    Z0, b0, _ = orc.canonical_to_tucker(c, A3, r3, 0)
    e0 = np.linalg.norm(orc.tucker_full(Z0, b0) - T)
    e1 = np.linalg.norm(orc.tucker_full(Z3, beta) - T)
    assert e1 <= e0 * (1 + 1e-12)
    # the core of orthonormal bases holds the projected norm
    assert abs(np.linalg.norm(beta) - np.linalg.norm(beta_ref)) <= 1e-12 * np.linalg.norm(beta_ref)


def test_tucker_ranks_threshold_and_clamp(orc):
    """The epsilon truncation rule on given spectra: the count of singular
    values at least eps times the largest, kept between 1 and the maximal
    rank, then clamped to the product of the other two modes' ranks."""
    sv = [np.array([1.0, 0.5, 0.1, 0.01, 1e-5]),
          np.array([2.0, 1e-3, 1e-4, 1e-6, 1e-9]),
          np.array([3.0, 2.9, 2.8, 2.7, 2.6])]
    assert orc.tucker_ranks(sv, (5, 5, 5), 0.0) == [5, 5, 5]
    assert orc.tucker_ranks(sv, (5, 5, 5), 0.05) == [3, 1, 3]   # mode 3: min(5, 3 * 1)
    assert orc.tucker_ranks(sv, (2, 5, 5), 0.05) == [2, 1, 2]   # mode 3: min(5, 2 * 1)
    assert orc.tucker_ranks(sv, (5, 5, 5), 1e-4) == [4, 2, 5]   # 1e-4 * 2 excludes 1e-4
    assert orc.tucker_ranks(sv, (5, 5, 5), 0.99) == [1, 1, 1]   # at least one vector each
