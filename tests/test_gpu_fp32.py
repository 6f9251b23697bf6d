"""Parity of the binary32 matrix-core path (TC_FP32) with the FP64 oracle,
through the C ABI.

Error model (u = 2^-24): rounding both operands to binary32 costs 2u per
product, and a binary32 partial sum over a chunk of 64 products at most 64u of
the sum of absolute values; the chunk sums are added in binary64.  So a
contraction x^T y is off by at most 70u |x|^T |y|.  For the direct route the
Gram reads a W that carries this error already, so
  |dW| <= 70u |T||U|,        |dG| <= 141u |U|^T |T| |U|;
the FFT route computes W in binary64 (its own norm-based error bound, as on
the FP64 path) and then only the Gram term remains.
Binary32 also has a narrow exponent range: an operand, product or partial sum
below the smallest normal number m = 2^-126 may be flushed to zero.  The
library scales every operand row by 2^-e (max|x| < 2^e <= 2 max|x|) before
rounding, so a flush costs at most
  2m (max|y| |x|_1 + max|x| |y|_1 + 6K max|x| max|y|)
in a contraction of length K, far below the rounding term.  The
normalised error e_J of this path is measured and reported; it is expected
above the 1e-7 target of the mixed-precision path (that is why the int8
splitting path exists), and the tests cap it at 1e-5.
"""
import numpy as np
import pytest

from paper_1504_06289_amd import workloads as wl
from tests.gpu_common import algorithm, dev, host, oracle_setup, say, shapes_of
from tests.metrics import e_J, rel_fro

pytestmark = pytest.mark.gpu

ALGOS = ["direct", "fft"]
PREC = "fp32"
U32 = 2.0 ** -24
M32 = 2.0 ** -126
CAP_J = 1e-5


def flush_bound(X, Y, K):
    """2m (max|y| |x|_1 + max|x| |y|_1 + 6K max|x| max|y|) for rows x of X, y of Y."""
    xm, x1 = np.abs(X).max(1), np.abs(X).sum(1)
    ym, y1 = np.abs(Y).max(1), np.abs(Y).sum(1)
    return 2 * M32 * (ym[None, :] * x1[:, None] + xm[:, None] * y1[None, :]
                      + 6 * K * xm[:, None] * ym[None, :])


def abs_gram_bound(orc, p, U):
    """|U|^T |T_k| |U| for every k: [R_N][R_f][R_f]."""
    A = np.abs(U)
    TA = orc.convolve(np.abs(p), A)                       # [R_N][R_f][n]
    return np.einsum("ia,kja->kij", A, TA)


@pytest.mark.parametrize("n,R_f,R_N", [(1, 1, 1), (5, 3, 2), (64, 64, 3), (100, 7, 4),
                                       (257, 130, 5), (1000, 65, 3)])
def test_convolve_fp32(tc, orc, n, R_f, R_N):
    say(f"fp32 convolve n={n} R_f={R_f} R_N={R_N}")
    b = 6.0
    h = 2 * b / n
    u0, hu = wl.sinc_params(R_N, n, b)
    U, _ = wl.gaussian_products(n, b, R_f, seed=n + R_f)
    t, a, c, p = orc.newton_kernel(n, h, R_N, u0, hu)
    with algorithm(tc, "direct", [(n, R_f, R_N)], PREC):
        W = host(tc.convolve(dev(p), dev(U[0]), prec=PREC))
    Wr = orc.convolve(p, U[0])
    under = flush_bound(p, U[0], n)[:, :, None]
    bound = 70 * U32 * orc.convolve(np.abs(p), np.abs(U[0])) + under
    assert np.all(np.abs(W - Wr) <= bound + 1e-300)
    # the binary32 rounding is really there (the result is not the binary64 one)
    if n >= 64:
        assert np.abs(W - Wr).max() > 1e-3 * U32 * np.abs(Wr).max()


SMALL = [((1, 1, 1), 1, 1), ((8, 8, 8), 2, 3), ((64, 64, 64), 16, 5), ((100, 100, 100), 33, 7),
         ((40, 33, 47), 9, 4), ((257, 257, 257), 70, 12), ((130, 64, 200), 65, 6)]


@pytest.mark.parametrize("algo", ALGOS)
@pytest.mark.parametrize("n,R_f,R_N", SMALL)
def test_tei_gram_fp32_small(tc, orc, n, R_f, R_N, algo):
    say(f"fp32 tei_gram n={n} R_f={R_f} R_N={R_N} {algo}")
    w = wl.small_products(n, R_f, R_N=R_N, b=6.0, seed=sum(n) + R_f)
    c, ps = oracle_setup(orc, w)
    with algorithm(tc, algo, shapes_of(w), PREC):
        J, G = tc.tei_gram(dev(c), [dev(p) for p in ps], [dev(u) for u in w.U], prec=PREC,
                           save_G=True)
    Jr, Gr = orc.tei_gram(c, ps, w.U, return_G=True)
    J, G = host(J), host(G)
    err = e_J(J, Jr)
    say(f"   e_J = {err:.2e}")
    assert err <= CAP_J
    np.testing.assert_array_equal(J, J.T)
    for l in range(3):
        B = abs_gram_bound(orc, ps[l], w.U[l])
        Wr = orc.convolve(ps[l], w.U[l])                          # [R_N][R_f][n]
        u1 = np.abs(w.U[l]).sum(1)
        wunder = flush_bound(ps[l], w.U[l], n[l])                 # [R_N][R_f], W flushes
        under = np.stack([flush_bound(w.U[l], Wr[k], n[l]) for k in range(R_N)])
        under = under + u1[None, :, None] * wunder[:, None, :]    # [R_N][R_f][R_f]
        bound = 141 * U32 * B + 2 * under
        if algo == "fft":
            # binary64 FFT convolution error, norm-based (as for the FP64 path)
            un = np.linalg.norm(w.U[l], axis=1)
            pn = np.linalg.norm(ps[l], axis=1)
            bound = bound + 1e-13 * pn[:, None, None] * un[None, :, None] * un[None, None, :]
        assert np.all(np.abs(G[l] - Gr[l]) <= bound)


@pytest.mark.parametrize("algo", ALGOS)
@pytest.mark.parametrize("name,ncols", [("c2", 12), ("c3", 4)])
def test_tei_gram_fp32_sampled_full_size(tc, orc, name, ncols, algo):
    say(f"fp32 tei_gram sampled {name} {algo}")
    w = wl.config(name)
    c, ps = oracle_setup(orc, w)
    with algorithm(tc, algo, shapes_of(w), PREC):
        J = host(tc.tei_gram(dev(c), [dev(p) for p in ps], [dev(u) for u in w.U], prec=PREC))
    rng = np.random.default_rng(321)
    S = np.sort(rng.choice(w.R_f, size=min(ncols, w.R_f), replace=False))
    Jc = orc.tei_gram_columns(c, ps, w.U, S)
    d = np.diag(Jc[:, S])
    dg = np.sqrt(np.abs(np.diag(J)))
    err = np.max(np.abs(J[:, S] - Jc.T) / np.outer(dg, np.sqrt(d)))
    say(f"   e_J(columns) = {err:.2e}")
    assert err <= CAP_J
    np.testing.assert_array_equal(J, J.T)


@pytest.mark.parametrize("algo", ALGOS)
def test_backward_fp32(tc, orc, algo):
    say(f"fp32 backward {algo}")
    w = wl.small_products((100, 100, 100), 40, R_N=5, b=6.0, seed=40)
    c, ps = oracle_setup(orc, w)
    wv = np.random.default_rng(5).standard_normal(w.R_f)
    Jb = np.outer(wv, wv)
    dUr = orc.tei_gram_backward(c, ps, w.U, Jb)
    with algorithm(tc, algo, shapes_of(w), PREC):
        dU = tc.tei_gram_backward(dev(c), [dev(p) for p in ps], [dev(u) for u in w.U], dev(Jb),
                                  prec=PREC)
    for l in range(3):
        err = rel_fro(host(dU[l]), dUr[l])
        say(f"   mode {l}: rel err {err:.2e}")
        assert err <= CAP_J
