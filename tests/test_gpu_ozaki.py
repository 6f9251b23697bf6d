"""Parity of the int8 error-free-splitting path (TC_OZAKI_I8) with the FP64
oracle, through the C ABI.

Error model: every operand row is split into four int8 slices that keep 28
bits relative to the row maximum, and the ten leading slice products are
accumulated exactly.  A contraction x^T y then differs from the exact one by
at most about 2^-26 (max|x| |y|_1 + max|y| |x|_1); these tests use that bound
for W = T U and for the Grams, and the target 1e-7 for the normalised error
of J and for the relative error of the adjoint.
"""

import numpy as np
import pytest

from paper_1504_06289_amd import workloads as wl
from tests.gpu_common import (algorithm, block_columns, column_errors, dev, host, oracle_columns,
                              oracle_setup, say, shapes_of)
from tests.metrics import e_J, rel_fro

pytestmark = pytest.mark.gpu


ALGOS = ["direct", "fft"]
PREC = "ozaki8"
TOL_J = 1e-7


def split_bound_W(p, U):
    """2^-26 (max|p_k| |u_j|_1 + max|u_j| |p_k|_1) per (k, j)."""
    pm = np.abs(p).max(axis=1)
    p1 = np.abs(p).sum(axis=1)
    um = np.abs(U).max(axis=1)
    u1 = np.abs(U).sum(axis=1)
    return 2.0 ** -26 * (pm[:, None] * u1[None, :] + um[None, :] * p1[:, None])


@pytest.mark.parametrize("n,R_f,R_N", [(1, 1, 1), (5, 3, 2), (64, 64, 3), (100, 7, 4),
                                       (257, 130, 5), (1000, 65, 3)])
def test_convolve_ozaki(tc, orc, n, R_f, R_N):
    """The direct int8 route (the FFT route computes W in binary64 and is
    covered by the FP64 parity tests)."""
    say(f"ozaki convolve n={n} R_f={R_f} R_N={R_N}")
    b = 6.0
    h = 2 * b / n
    u0, hu = wl.sinc_params(R_N, n, b)
    U, _ = wl.gaussian_products(n, b, R_f, seed=n + R_f)
    t, a, c, p = orc.newton_kernel(n, h, R_N, u0, hu)
    with algorithm(tc, "direct", [(n, R_f, R_N)], PREC):
        W = host(tc.convolve(dev(p), dev(U[0]), prec=PREC))
    Wr = orc.convolve(p, U[0])
    bound = split_bound_W(p, U[0])                    # [R_N][R_f]
    err = np.abs(W - Wr).max(axis=2)
    assert np.all(err <= bound + 1e-300), float((err / (bound + 1e-300)).max())


def test_convolve_ozaki_asymmetric(tc, orc):
    say("ozaki convolve asymmetric")
    rng = np.random.default_rng(1)
    n, R_f, R_N = 200, 19, 3
    p = rng.standard_normal((R_N, 2 * n - 1))
    U = rng.standard_normal((R_f, n))
    with algorithm(tc, "direct", [(n, R_f, R_N)], PREC):
        W = host(tc.convolve(dev(p), dev(U), prec=PREC))
    Wr = orc.convolve(p, U)
    assert np.all(np.abs(W - Wr).max(axis=2) <= split_bound_W(p, U))


SMALL = [((1, 1, 1), 1, 1), ((8, 8, 8), 2, 3), ((64, 64, 64), 16, 5), ((100, 100, 100), 33, 7),
         ((40, 33, 47), 9, 4), ((257, 257, 257), 70, 12), ((130, 64, 200), 65, 6),
         ((300, 300, 300), 129, 8)]


@pytest.mark.parametrize("algo", ALGOS)
@pytest.mark.parametrize("n,R_f,R_N", SMALL)
def test_tei_gram_ozaki_small(tc, orc, n, R_f, R_N, algo):
    say(f"ozaki tei_gram n={n} R_f={R_f} R_N={R_N} {algo}")
    w = wl.small_products(n, R_f, R_N=R_N, b=6.0, seed=sum(n) + R_f)
    c, ps = oracle_setup(orc, w)
    with algorithm(tc, algo, shapes_of(w), PREC):
        J, G = tc.tei_gram(dev(c), [dev(p) for p in ps], [dev(u) for u in w.U], prec=PREC,
                           save_G=True)
    Jr, Gr = orc.tei_gram(c, ps, w.U, return_G=True)
    J, G = host(J), host(G)
    err = e_J(J, Jr)
    say(f"   e_J = {err:.2e}")
    assert err <= TOL_J
    np.testing.assert_array_equal(J, J.T)
    # Grams: |dG_ij| <= 2^-26 (max|u_i| |W_j|_1 + max|W_j| |u_i|_1) + W error
    for l in range(3):
        Wr = orc.convolve(ps[l], w.U[l])
        U = w.U[l]
        um, u1 = np.abs(U).max(1), np.abs(U).sum(1)
        wm, w1 = np.abs(Wr).max(2), np.abs(Wr).sum(2)          # [R_N][R_f]
        bW = split_bound_W(ps[l], U)                            # W error per (k, j)
        bound = (2.0 ** -26 * (um[None, :, None] * w1[:, None, :] + wm[:, None, :] * u1[None, :, None])
                 + u1[None, :, None] * bW[:, None, :])
        assert np.all(np.abs(G[l] - Gr[l]) <= bound + 1e-300)


@pytest.mark.parametrize("algo", ALGOS)
@pytest.mark.parametrize("name", ["c1", "c2", "c5", "c3"])
def test_tei_gram_ozaki_sampled_full_size(tc, orc, name, algo):
    """Full-size workloads against oracle columns: both ends and two seeded
    columns in every block of 128 (18 columns at R_f = 1024), so that every
    column block of the 128 x 128 Gram tiles (and of the XCD chunks of work
    items) is visited."""
    say(f"ozaki tei_gram sampled {name} {algo}")
    w = wl.config(name)
    c, ps = oracle_setup(orc, w)
    # one grid spacing in all directions: one kernel tensor for the three
    # modes, as a caller passes it (the modes then share its spectra)
    assert all(np.array_equal(ps[0], q) for q in ps)
    pd = dev(ps[0])
    with algorithm(tc, algo, shapes_of(w), PREC):
        J = host(tc.tei_gram(dev(c), [pd, pd, pd], [dev(u) for u in w.U], prec=PREC))
    S = block_columns(w.R_f, seed=123)
    Jc = oracle_columns(orc, name, c, ps, w.U, S)
    err, err_cols = column_errors(J, Jc, S)
    say(f"   {len(S)} columns: e_J(block) = {err:.2e}, columns = {err_cols:.2e}")
    assert err <= TOL_J and err_cols <= TOL_J
    np.testing.assert_array_equal(J, J.T)


@pytest.mark.parametrize("algo", ALGOS)
def test_tei_gram_ozaki_shared_kernel_tensor(tc, orc, algo):
    """The three modes given one kernel tensor (whose spectra, term classes
    and S_k the modes then share) give bitwise the J of three separate copies,
    with the modes concurrent and with kernel timing on (modes in turn)."""
    say(f"ozaki shared kernel tensor {algo}")
    w = wl.small_products(300, 100, R_N=24, b=8.0, seed=11)
    c, ps = oracle_setup(orc, w)
    Us = [dev(u) for u in w.U]
    pd = dev(ps[0])
    with algorithm(tc, algo, shapes_of(w), PREC):
        J_sep = host(tc.tei_gram(dev(c), [dev(p) for p in ps], Us, prec=PREC))
        J_one = host(tc.tei_gram(dev(c), [pd, pd, pd], Us, prec=PREC))
        tc.profile_enable(True)
        try:
            J_ser = host(tc.tei_gram(dev(c), [pd, pd, pd], Us, prec=PREC))
        finally:
            tc.profile_enable(False)
            tc.profile_read()
    np.testing.assert_array_equal(J_one, J_sep)
    np.testing.assert_array_equal(J_ser, J_sep)
    assert e_J(J_one, orc.tei_gram(c, ps, w.U)) <= TOL_J
    if algo == "fft":
        cls = tc.term_classes(pd)
        say(f"   classes: {cls.tolist()}")
        assert (cls == -2).any() and (cls != -2).any()


def test_tei_gram_ozaki_deterministic(tc, orc):
    say("ozaki determinism")
    w = wl.small_products(300, 100, R_N=9, b=6.0, seed=4)
    c, ps = oracle_setup(orc, w)
    args = (dev(c), [dev(p) for p in ps], [dev(u) for u in w.U])
    np.testing.assert_array_equal(host(tc.tei_gram(*args, prec=PREC)),
                                  host(tc.tei_gram(*args, prec=PREC)))


@pytest.mark.parametrize("algo", ALGOS)
@pytest.mark.parametrize("n,R_f,R_N", [((24, 19, 28), 6, 6), ((100, 100, 100), 40, 5),
                                       ((70, 130, 300), 67, 4)])
def test_backward_ozaki(tc, orc, n, R_f, R_N, algo):
    say(f"ozaki backward n={n} R_f={R_f} R_N={R_N} {algo}")
    w = wl.small_products(n, R_f, R_N=R_N, b=6.0, seed=R_f)
    c, ps = oracle_setup(orc, w)
    rng = np.random.default_rng(5)
    wv = rng.standard_normal(R_f)
    Jb = np.outer(wv, wv)
    dUr = orc.tei_gram_backward(c, ps, w.U, Jb)
    with algorithm(tc, algo, shapes_of(w), PREC):
        dU = tc.tei_gram_backward(dev(c), [dev(p) for p in ps], [dev(u) for u in w.U], dev(Jb),
                                  prec=PREC)
    for l in range(3):
        err = rel_fro(host(dU[l]), dUr[l])
        say(f"   mode {l}: rel err {err:.2e}")
        assert err <= TOL_J


def test_autograd_ozaki(tc, orc):
    say("ozaki autograd")
    w = wl.small_products(90, 20, R_N=6, b=6.0, seed=3)
    c, ps = oracle_setup(orc, w)
    wv = np.random.default_rng(8).standard_normal(w.R_f)
    Us = [dev(u).requires_grad_(True) for u in w.U]
    J = tc.TeiGram.apply(dev(c), dev(ps[0]), dev(ps[1]), dev(ps[2]), *Us, PREC)
    wt = dev(wv)
    (wt @ J @ wt).backward()
    dUr = orc.tei_gram_backward(c, ps, w.U, np.outer(wv, wv))
    for l in range(3):
        assert rel_fro(host(Us[l].grad), dUr[l]) <= TOL_J


def test_term_classes_c3(tc, orc):
    """The term classes of the 4096-cell kernel (R_N = 32) against the
    criteria recomputed on the host: minimal band for narrow terms, and the
    polynomial-fit residual for smooth and general ones (decisions within a
    small margin of a threshold are not checked)."""
    say("term classes c3")
    w = wl.config("c3")
    t, c, p = tc.newton_kernel(w.n[0], w.h[0], w.R_N, w.u0, w.hu)
    cls = tc.term_classes(p)
    P = host(p)
    n = w.n[0]
    say(f"   classes: {cls.tolist()}")
    lag = np.arange(-(n - 1), n) / (n - 1.0)
    Qv, _ = np.linalg.qr(np.polynomial.chebyshev.chebvander(lag, 31))
    for k in range(w.R_N):
        a = np.abs(P[k])
        tot = a.sum()
        thr = 2.0 ** -60 * tot
        # the outer entries summed directly (tot minus the centre would cancel)
        tail = lambda B: a[:n - 1 - B].sum() + a[n + B:].sum()
        if cls[k] >= 0:
            B = int(cls[k])
            assert B <= 16
            assert tail(B) <= thr * (1 + 1e-9) + 1e-300
            if B > 0:
                assert tail(B - 1) > thr * (1 - 1e-9)
            continue
        assert tail(16) > thr * (1 - 1e-9)       # not narrow
        res = np.abs(P[k] - Qv @ (Qv.T @ P[k])).max() / a.max()
        if cls[k] == -2:
            assert res <= 4 * 2.0 ** -44, (k, res)
        else:
            assert res > 2.0 ** -44 / 4, (k, res)
    # this kernel: 7 narrow (t_k >= 85), 15 smooth (t_k <= 0.08), 10 general
    assert (cls >= 0).sum() == 7 and (cls == -2).sum() == 15


def test_smooth_term_grams_binary64_accuracy(tc, orc):
    """The Grams of smooth terms come from the rank-32 polynomial projection
    in binary64: within 2 (2n-1) 2^-44 max|p_k| |u_i| |u_j| of the oracle
    (much tighter than the int8 bound the other terms meet)."""
    say("smooth-term Grams")
    w = wl.small_products((512, 512, 512), 48, R_N=12, b=8.0, seed=11)
    c, ps = oracle_setup(orc, w)
    with algorithm(tc, "fft", shapes_of(w), PREC):
        J, G = tc.tei_gram(dev(c), [dev(p) for p in ps], [dev(u) for u in w.U], prec=PREC,
                           save_G=True)
    Jr, Gr = orc.tei_gram(c, ps, w.U, return_G=True)
    G = host(G)
    assert e_J(host(J), Jr) <= TOL_J
    nsmooth = 0
    for l in range(3):
        cls = tc.term_classes(dev(ps[l]))
        un = np.linalg.norm(w.U[l], axis=1)
        n = w.n[l]
        for k in np.nonzero(cls == -2)[0]:
            nsmooth += 1
            bound = 2 * (2 * n - 1) * 2.0 ** -44 * np.abs(ps[l][k]).max() * np.outer(un, un)
            assert np.all(np.abs(G[l][k] - Gr[l][k]) <= bound + 1e-300), (l, k)
            np.testing.assert_array_equal(G[l][k], G[l][k].T)
    say(f"   smooth terms checked: {nsmooth}")
    assert nsmooth > 0
