"""Parity of the HIP library (through the C ABI) with the FP64 CPU oracle.

Every GPU result is compared element by element with the oracle on the same
seeded inputs, at sizes spanning several tiles with ragged tails, plus the
degenerate sizes.  Tolerances (FP64 path):
  * kernel vectors p: relative 1e-14 plus the conditioning of exp(-x^2) at
    x = t(|m|+1/2)h (rounding the argument moves the value by ~2x^2 ulp);
  * W = T U: |dW| <= 1e-13 (|T| |U|)  (a rounding-error bound of the product);
  * J: normalised error max |dJ_ij| / sqrt(J_ii J_jj) <= 1e-12;
  * adjoint: relative Frobenius error <= 1e-12 per mode.
"""

import numpy as np
import pytest
import torch

from paper_1504_06289_amd import workloads as wl
from tests.gpu_common import (algorithm, block_columns, column_errors, dev, host, oracle_columns,
                              oracle_setup, say, shapes_of)
from tests.metrics import e_J, rel_fro

pytestmark = pytest.mark.gpu


ALGOS = ["direct", "fft"]


def kernel_tol(t, h, n):
    m = np.abs(np.arange(-(n - 1), n))
    x = np.outer(t, (m + 0.5) * h)
    return 1e-14 + 9e-16 * 2 * x * x


# --------------------------------------------------------------------------
@pytest.mark.parametrize("R_N,n,b", [(20, 128, 10.0), (30, 1024, 10.0), (32, 4096, 12.0),
                                     (7, 1, 3.0), (3, 2, 1.0), (150, 300, 10.0)])
def test_newton_kernel_parity(tc, orc, R_N, n, b):
    say(f"newton_kernel R_N={R_N} n={n} b={b}")
    h = 2 * b / n
    u0, hu = wl.sinc_params(R_N, n, b)
    t, c, p = tc.newton_kernel(n, h, R_N, u0, hu)
    tr, ar, cr, pr = orc.newton_kernel(n, h, R_N, u0, hu)
    np.testing.assert_allclose(t, tr, rtol=2e-16, atol=0)
    np.testing.assert_allclose(c, cr, rtol=4e-16, atol=0)
    pg = host(p)
    tiny = (np.abs(pr) < 1e-300) & (np.abs(pg) < 1e-300)
    rel = np.abs(pg - pr) / np.where(tiny, 1.0, np.abs(pr))
    rel[tiny] = 0.0
    assert np.all(rel <= kernel_tol(tr, h, n)), float(rel.max())
    np.testing.assert_array_equal(pg, pg[:, ::-1])


# --------------------------------------------------------------------------
@pytest.mark.parametrize("algo", ALGOS)
@pytest.mark.parametrize("n,R_f,R_N", [(1, 1, 1), (5, 3, 2), (64, 64, 3), (100, 7, 4),
                                       (257, 130, 5), (1024, 33, 2), (4096, 9, 2)])
def test_convolve_parity(tc, orc, n, R_f, R_N, algo):
    say(f"convolve n={n} R_f={R_f} R_N={R_N} {algo}")
    b = 6.0
    h = 2 * b / n
    u0, hu = wl.sinc_params(R_N, n, b)
    U, _ = wl.gaussian_products(n, b, R_f, seed=n + R_f)
    t, a, c, pr = orc.newton_kernel(n, h, R_N, u0, hu)
    with algorithm(tc, algo, [(n, R_f, R_N)], "fp64"):
        W = host(tc.convolve(dev(pr), dev(U[0])))
    Wr = orc.convolve(pr, U[0])
    if algo == "direct":
        bound = orc.convolve(np.abs(pr), np.abs(U[0]))
        assert np.all(np.abs(W - Wr) <= 1e-13 * bound + 1e-300)
    else:
        # FFT rounding is spread over the row: |dW| <= 1e-14 |p|_2 |u|_2 log2(N) per row
        scale = (np.linalg.norm(pr, axis=1)[:, None] * np.linalg.norm(U[0], axis=1)[None, :]
                 * np.log2(2 * n + 2))[:, :, None]
        assert np.all(np.abs(W - Wr) <= 1e-14 * scale + 1e-300)


@pytest.mark.parametrize("algo", ALGOS)
def test_convolve_asymmetric_kernel_lag_direction(tc, orc, algo):
    """A non-symmetric p pins the lag direction W[a] = sum_b p[a-b] u[b]."""
    say(f"convolve asymmetric p {algo}")
    rng = np.random.default_rng(1)
    n, R_f, R_N = 77, 19, 3
    p = rng.standard_normal((R_N, 2 * n - 1))
    U = rng.standard_normal((R_f, n))
    with algorithm(tc, algo, [(n, R_f, R_N)], "fp64"):
        W = host(tc.convolve(dev(p), dev(U)))
    Wr = orc.convolve(p, U)
    bound = orc.convolve(np.abs(p), np.abs(U))
    assert np.all(np.abs(W - Wr) <= 1e-13 * bound * (1 if algo == "direct" else 30))


# --------------------------------------------------------------------------


SMALL = [((1, 1, 1), 1, 1), ((8, 8, 8), 2, 3), ((64, 64, 64), 16, 5), ((100, 100, 100), 33, 7),
         ((40, 33, 47), 9, 4), ((257, 257, 257), 70, 12), ((130, 64, 200), 65, 6)]


@pytest.mark.parametrize("algo", ALGOS)
@pytest.mark.parametrize("n,R_f,R_N", SMALL)
def test_tei_gram_parity_small(tc, orc, n, R_f, R_N, algo):
    say(f"tei_gram n={n} R_f={R_f} R_N={R_N} {algo}")
    w = wl.small_products(n, R_f, R_N=R_N, b=6.0, seed=sum(n) + R_f)
    c, ps = oracle_setup(orc, w)
    with algorithm(tc, algo, shapes_of(w), "fp64"):
        J, G = tc.tei_gram(dev(c), [dev(p) for p in ps], [dev(u) for u in w.U], save_G=True)
    Jr, Gr = orc.tei_gram(c, ps, w.U, return_G=True)
    J, G = host(J), host(G)
    err = e_J(J, Jr)
    say(f"   e_J = {err:.2e}")
    assert err <= 1e-12
    np.testing.assert_array_equal(J, J.T)
    # each Gram entry within a rounding-error bound of the product U^T T U:
    # |dG| <= 1e-13 |U|^T |T| |U| (p-type columns make G_ii much smaller than
    # that bound for the wide kernel terms, so a G_ii-relative bound is wrong)
    for l in range(3):
        if algo == "direct":
            absG = orc.gram(np.abs(w.U[l]), orc.convolve(np.abs(ps[l]), np.abs(w.U[l])))
            assert np.all(np.abs(G[l] - Gr[l]) <= 1e-13 * absG + 1e-300)
        else:
            un = np.linalg.norm(w.U[l], axis=1)
            pn = np.linalg.norm(ps[l], axis=1)
            scale = pn[:, None, None] * un[None, :, None] * un[None, None, :]
            assert np.all(np.abs(G[l] - Gr[l]) <= 1e-13 * scale + 1e-300)


def test_tei_gram_single_cell(tc, orc):
    """n = 1 in every mode: each Gram is the single product u p[0] u."""
    say("tei_gram single cell")
    U, _ = wl.s_gaussians(1, 2.0, 3, alphas=[0.5, 1.0, 2.0], centres=np.zeros((3, 3)))
    R_N = 5
    t, a, cc, p = orc.newton_kernel(1, 4.0, R_N, -2.0, 0.7)
    c = a * 4.0 ** 3
    J = host(tc.tei_gram(dev(c), [dev(p)] * 3, [dev(u) for u in U]))
    Jr = orc.tei_gram(c, [p] * 3, U)
    assert e_J(J, Jr) <= 1e-14


def test_tei_gram_parity_c1(tc, orc):
    """The 128-cell, 8-function s-Gaussian workload, with its potential factors."""
    say("tei_gram c1")
    w = wl.config("c1")
    c, ps = oracle_setup(orc, w)
    t, cg, pg = tc.newton_kernel(w.n[0], w.h[0], w.R_N, w.u0, w.hu)
    J = host(tc.tei_gram(torch.from_numpy(cg).cuda(), [pg, pg, pg], [dev(u) for u in w.U]))
    Jr = orc.tei_gram(c, ps, w.U)
    assert e_J(J, Jr) <= 1e-12
    for l in range(3):
        W = host(tc.convolve(pg, dev(w.U[l])))
        Wr = orc.convolve(ps[l], w.U[l])
        bound = orc.convolve(np.abs(ps[l]), np.abs(w.U[l]))
        assert np.all(np.abs(W - Wr) <= 1e-13 * bound + 1e-300)


@pytest.mark.parametrize("algo", ALGOS)
@pytest.mark.parametrize("name", ["c2", "c5", "c3"])
def test_tei_gram_parity_sampled_full_size(tc, orc, name, algo):
    """Full-size workloads: the GPU J (whole matrix) against oracle columns:
    both ends and two seeded columns in every block of 128 (18 columns at
    R_f = 1024), so that every column block of the Gram tiles is visited;
    the S x S block is compared with the normalised metric using oracle
    diagonals only."""
    say(f"tei_gram sampled {name} {algo}")
    w = wl.config(name)
    c, ps = oracle_setup(orc, w)
    with algorithm(tc, algo, shapes_of(w), "fp64"):
        J = host(tc.tei_gram(dev(c), [dev(p) for p in ps], [dev(u) for u in w.U]))
    S = block_columns(w.R_f, seed=123)
    Jc = oracle_columns(orc, name, c, ps, w.U, S)     # [len(S)][R_f]
    err, err_cols = column_errors(J, Jc, S)
    say(f"   {len(S)} columns: e_J(block) = {err:.2e}, columns = {err_cols:.2e}")
    assert err <= 1e-12, err
    assert err_cols <= 1e-12, err_cols
    # structure at full size
    np.testing.assert_array_equal(J, J.T)
    assert np.all(np.diag(J) > 0)


@pytest.mark.parametrize("algo", ALGOS)
def test_tei_gram_deterministic(tc, orc, algo):
    say(f"tei_gram determinism {algo}")
    w = wl.small_products(300, 100, R_N=9, b=6.0, seed=4)
    c, ps = oracle_setup(orc, w)
    args = (dev(c), [dev(p) for p in ps], [dev(u) for u in w.U])
    with algorithm(tc, algo, shapes_of(w), "fp64"):
        J1 = host(tc.tei_gram(*args))
        J2 = host(tc.tei_gram(*args))
    np.testing.assert_array_equal(J1, J2)


def test_tei_gram_batched_matches_single(tc, orc):
    say("tei_gram batched vs single")
    insts = []
    for i, (n, R_f, R_N) in enumerate([(64, 10, 4), (130, 37, 6), (33, 5, 3)]):
        w = wl.small_products(n, R_f, R_N=R_N, b=6.0, seed=i)
        c, ps = oracle_setup(orc, w)
        insts.append((dev(c), [dev(p) for p in ps], [dev(u) for u in w.U]))
    Js = [host(J) for J in tc.tei_gram_batched(insts)]
    for (c, ps, Us), Jb in zip(insts, Js):
        np.testing.assert_array_equal(Jb, host(tc.tei_gram(c, ps, Us)))


# --------------------------------------------------------------------------
@pytest.mark.parametrize("algo", ALGOS)
@pytest.mark.parametrize("n,R_f,R_N", [((24, 19, 28), 6, 6), ((100, 100, 100), 40, 5),
                                       ((70, 130, 300), 67, 4),
                                       # the adjoint contraction split into 3 K ranges
                                       ((200, 150, 96), 130, 12)])
def test_backward_parity(tc, orc, n, R_f, R_N, algo):
    say(f"backward n={n} R_f={R_f} R_N={R_N} {algo}")
    w = wl.small_products(n, R_f, R_N=R_N, b=6.0, seed=R_f)
    c, ps = oracle_setup(orc, w)
    rng = np.random.default_rng(5)
    Jb = rng.standard_normal((R_f, R_f))
    dUr = orc.tei_gram_backward(c, ps, w.U, Jb)
    cd, pd, Ud = dev(c), [dev(p) for p in ps], [dev(u) for u in w.U]
    with algorithm(tc, algo, shapes_of(w), "fp64"):
        dU = tc.tei_gram_backward(cd, pd, Ud, dev(Jb))
        for l in range(3):
            assert rel_fro(host(dU[l]), dUr[l]) <= 1e-12
        # with saved Grams
        J, G = tc.tei_gram(cd, pd, Ud, save_G=True)
        dU2 = tc.tei_gram_backward(cd, pd, Ud, dev(Jb), G=G)
        for l in range(3):
            assert rel_fro(host(dU2[l]), dUr[l]) <= 1e-12


def test_autograd_function(tc, orc):
    say("autograd TeiGram")
    w = wl.small_products(90, 20, R_N=6, b=6.0, seed=3)
    c, ps = oracle_setup(orc, w)
    rng = np.random.default_rng(8)
    wv = rng.standard_normal(w.R_f)
    Us = [dev(u).requires_grad_(True) for u in w.U]
    J = tc.TeiGram.apply(dev(c), dev(ps[0]), dev(ps[1]), dev(ps[2]), *Us)
    wt = dev(wv)
    f = wt @ J @ wt
    f.backward()
    dUr = orc.tei_gram_backward(c, ps, w.U, np.outer(wv, wv))
    for l in range(3):
        assert rel_fro(host(Us[l].grad), dUr[l]) <= 1e-12


def test_autotune_records_a_choice(tc, orc):
    say("autotune")
    w = wl.small_products(512, 64, R_N=8, b=6.0, seed=12)
    c, ps = oracle_setup(orc, w)
    ms = tc.autotune(dev(c), [dev(p) for p in ps], [dev(u) for u in w.U], prec="fp64")
    say(f"   ms (direct, fft) per mode: {ms}")
    for l in range(3):
        d, f = ms[l]
        assert d > 0 and f > 0
        assert tc.tune_get(512, 64, 8, "fp64") == ("fft" if f < d else "direct")
    tc.tune_set(512, 64, 8, "fp64", "auto")


def test_autotune_batched_then_batch_matches_oracle(tc, orc):
    """The batched autotuner records one choice per distinct mode shape; the
    batch run afterwards (with those choices) still matches the oracle."""
    say("autotune batched")
    ws = [wl.small_products((300, 300, 300), 40, R_N=6, b=6.0, seed=1),
          wl.small_products((130, 64, 200), 20, R_N=6, b=6.0, seed=2),
          wl.small_products((300, 300, 300), 40, R_N=6, b=6.0, seed=3)]
    batch, refs = [], []
    for w in ws:
        c, ps = oracle_setup(orc, w)
        batch.append((dev(c), [dev(p) for p in ps], [dev(u) for u in w.U]))
        refs.append(orc.tei_gram(c, ps, w.U))
    shapes = sorted({(nl, w.R_f, w.R_N) for w in ws for nl in w.n})
    try:
        ms = tc.autotune_batched(batch, prec="ozaki8")
        assert ms.shape == (3, 3, 2) and np.all(ms > 0)
        np.testing.assert_array_equal(ms[0], ms[2])  # the same shapes, timed once
        for i, w in enumerate(ws):
            for l in range(3):
                d, f = ms[i, l]
                assert tc.tune_get(w.n[l], w.R_f, w.R_N, "ozaki8") == ("fft" if f < d else "direct")
        Js = tc.tei_gram_batched(batch, prec="ozaki8")
        for J, Jr in zip(Js, refs):
            assert e_J(host(J), Jr) <= 1e-7
    finally:
        for sh in shapes:
            tc.tune_set(*sh, "ozaki8", "auto")


@pytest.mark.parametrize("count", [1, 3])
@pytest.mark.parametrize("prec", ["fp64", "ozaki8"])
def test_graph_replays_match_eager(tc, orc, prec, count):
    """A batch captured in a HIP graph (one instance: its modes on parallel
    branches; three: the instances on parallel branches): every replay (with
    eager work and synchronisations in between) reproduces the eager result
    bitwise, and the eager result matches the oracle."""
    say(f"graph replay {prec} count={count}")
    insts, refs = [], []
    shapes = [((300, 257, 130), 40, 6), (130, 70, 5), (64, 9, 4)][:count]
    for i, (n, R_f, R_N) in enumerate(shapes):
        w = wl.small_products(n, R_f, R_N=R_N, b=6.0, seed=40 + i)
        c, ps = oracle_setup(orc, w)
        insts.append((dev(c), [dev(p) for p in ps], [dev(u) for u in w.U]))
        refs.append(orc.tei_gram(c, ps, w.U))
    eager = [host(J) for J in tc.tei_gram_batched(insts, prec=prec)]
    for Je, Jr in zip(eager, refs):
        assert e_J(Je, Jr) <= (1e-12 if prec == "fp64" else 1e-7)
    g = tc.TeiGramGraph(insts, prec=prec)
    for rep in range(4):
        Js = [host(J) for J in g.replay()]
        for Jg, Je in zip(Js, eager):
            np.testing.assert_array_equal(Jg, Je)
        # unrelated eager work between replays
        junk = torch.randn(1 << 20, device="cuda", dtype=torch.float64)
        (junk * 2.0).sum().item()
        torch.cuda.synchronize()
