"""The FFT route beyond 4096 cells (four-step binary64 transforms of length
N = 16384 .. 131072, two real rows per complex sequence) against the FP64
oracle through the C ABI:
  * W = T U per entry, with the FFT's rounding bound
    |dW| <= 1e-14 |p_k|_2 |u_j|_2 log2(N) (spread over the row), including an
    asymmetric kernel (lag direction), odd R_f (an unpaired last row) and
    n = 65536 (N = 131072, the largest length);
  * J at 8192 and 16384 cells on sampled columns (every block of 64 or 128
    columns), binary64 (1e-12) and the int8 split (1e-7, the wide ragged Gram
    at R_f = 330), and an instance whose modes take both FFT routes;
  * the autotuner timing both algorithms at 8192 cells.
"""

import numpy as np
import pytest

from paper_1504_06289_amd import workloads as wl
from tests.gpu_common import (algorithm, block_columns, column_errors, dev, host, oracle_columns,
                              oracle_setup, say, shapes_of)
from tests.metrics import e_J

pytestmark = pytest.mark.gpu


def fft_scale(p, U, n):
    N = 1
    while N < 2 * n - 1:
        N *= 2
    return (np.linalg.norm(p, axis=1)[:, None] * np.linalg.norm(U, axis=1)[None, :]
            * np.log2(N))[:, :, None]


@pytest.mark.parametrize("n,R_f,R_N", [(4097, 3, 2), (8192, 5, 3), (12000, 4, 2), (16384, 2, 2),
                                       (65536, 1, 1)])
def test_convolve_large_fft(tc, orc, n, R_f, R_N):
    say(f"large FFT convolve n={n} R_f={R_f} R_N={R_N}")
    b = 10.0
    h = 2 * b / n
    u0, hu = wl.sinc_params(R_N, n, b)
    U, _ = wl.gaussian_products(n, b, R_f, seed=n + R_f)
    t, a, c, pr = orc.newton_kernel(n, h, R_N, u0, hu)
    with algorithm(tc, "fft", [(n, R_f, R_N)], "fp64"):
        assert tc.tune_get(n, R_f, R_N, "fp64") == "fft"
        W = host(tc.convolve(dev(pr), dev(U[0])))
    Wr = orc.convolve(pr, U[0])
    err = np.abs(W - Wr) / (fft_scale(pr, U[0], n) + 1e-300)
    say(f"   max |dW| / (|p|_2 |u|_2 log2 N) = {err.max():.2e}")
    assert err.max() <= 1e-14


def test_convolve_large_fft_asymmetric(tc, orc):
    rng = np.random.default_rng(3)
    n, R_f, R_N = 5000, 7, 2
    p = rng.standard_normal((R_N, 2 * n - 1))
    U = rng.standard_normal((R_f, n))
    with algorithm(tc, "fft", [(n, R_f, R_N)], "fp64"):
        W = host(tc.convolve(dev(p), dev(U)))
    Wr = orc.convolve(p, U)
    err = np.abs(W - Wr) / fft_scale(p, U, n)
    say(f"   asymmetric: {err.max():.2e}")
    assert err.max() <= 1e-14


@pytest.mark.parametrize("prec,n,R_f", [("fp64", 8192, 96), ("fp64", 16384, 70),
                                        ("ozaki8", 8192, 330), ("ozaki8", 16384, 96)])
def test_tei_gram_large_fft_sampled(tc, orc, prec, n, R_f):
    say(f"large FFT tei_gram {prec} n={n} R_f={R_f}")
    w = wl.small_products(n, R_f, R_N=30, b=10.0, seed=n + R_f)
    c, ps = oracle_setup(orc, w)
    pd = dev(ps[0])
    with algorithm(tc, "fft", shapes_of(w), prec):
        J = host(tc.tei_gram(dev(c), [pd, pd, pd], [dev(u) for u in w.U], prec=prec))
    S = block_columns(w.R_f, seed=9, per_block=1, block=64)
    Jc = oracle_columns(orc, f"large{n}_{R_f}", c, ps, w.U, S)
    e_blk, e_cols = column_errors(J, Jc, S)
    say(f"   {len(S)} columns: block {e_blk:.2e}, columns {e_cols:.2e}")
    tol = 1e-12 if prec == "fp64" else 1e-7
    assert e_blk <= tol and e_cols <= tol
    np.testing.assert_array_equal(J, J.T)


@pytest.mark.parametrize("prec", ["fp64", "ozaki8"])
def test_tei_gram_both_fft_routes_in_one_instance(tc, orc, prec):
    """Modes of 8192, 300 and 5000 cells: the four-step route, the LDS route
    (with the int8 term classes for ozaki8) and the four-step route again."""
    ns = (8192, 300, 5000)
    w = wl.small_products(ns, 40, R_N=8, b=8.0, seed=17)
    c, ps = oracle_setup(orc, w)
    with algorithm(tc, "fft", shapes_of(w), prec):
        J = host(tc.tei_gram(dev(c), [dev(p) for p in ps], [dev(u) for u in w.U], prec=prec))
    err = e_J(J, orc.tei_gram(c, ps, w.U))
    say(f"   {prec}: e_J {err:.2e}")
    assert err <= (1e-12 if prec == "fp64" else 1e-7)


def test_autotune_times_both_routes_at_8192(tc, orc):
    w = wl.small_products(8192, 64, R_N=12, b=10.0, seed=5)
    c, ps = oracle_setup(orc, w)
    try:
        ms = tc.autotune(dev(c), [dev(p) for p in ps], [dev(u) for u in w.U], prec="ozaki8")
        d, f = ms[0]
        say(f"   8192 cells, R_f=64, R_N=12, ozaki8: direct {d:.3f} ms, fft {f:.3f} ms")
        assert d > 0 and f > 0
        assert tc.tune_get(8192, 64, 12, "ozaki8") == ("fft" if f < d else "direct")
    finally:
        tc.tune_set(8192, 64, 12, "ozaki8", "auto")
