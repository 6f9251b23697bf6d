"""Parity at the benchmark configurations that the per-size tests do not
reach, through the C ABI against the FP64 oracle:

  * the adjoint of f = w^T J w at 2048 cells, R_f = 512, R_N = 30 (w ~ N(0,1)),
    against the oracle's full adjoint, on both precisions and both Toeplitz
    routes, through the autograd function (forward with saved Grams, which
    at R_f >= 256 are written by the wide int8 Gram with mirrored output, and
    an adjoint contraction split into several K ranges) and without saved
    Grams;
  * a recorded 8-instance subset of the 64-instance batched workload (every
    n in {512, 1024, 2048, 4096}, ragged R_f of the 128-wide int8 Gram tiles,
    the smallest R_f), as one batched call and as graph replays, against
    oracle columns per instance;
  * modes that reuse an earlier mode's kernel part ([pa, pb, pa]) on the int8
    FFT route, alone and in a batch.

Tolerances: FP64 route 1e-12 (normalised J error, relative Frobenius error
of each mode's gradient), int8 split route 1e-7.  The worst relative error of
a single gradient column is reported as well and held to ten times these:
a column of dU^l = 2 sum_k W_k D_k is a sum over (k, j) whose terms partly
cancel, so its relative error exceeds that of the whole mode (measured on
the int8 direct route: 8e-10 per mode, 1.9e-7 for the worst column).
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
TOL = {"fp64": 1e-12, "ozaki8": 1e-7}


# --------------------------------------------------------------------------
# adjoint at 2048 cells, R_f = 512
# --------------------------------------------------------------------------
@pytest.fixture(scope="module")
def c5_ref(orc):
    w = wl.config("c5")
    c, ps = oracle_setup(orc, w)
    wv = w.meta["w"]
    Jb = np.outer(wv, wv)
    say("oracle adjoint c5 (full) ...")
    dUr = orc.tei_gram_backward(c, ps, w.U, Jb)
    S = block_columns(w.R_f, seed=77)
    Jc = oracle_columns(orc, "c5", c, ps, w.U, S)
    return w, c, ps, Jb, dUr, S, Jc


def grad_errors(dU, dUr):
    """Relative Frobenius error per mode and the worst relative column error."""
    fro = [rel_fro(dU[l], dUr[l]) for l in range(3)]
    col = max(float(np.max(np.linalg.norm(dU[l] - dUr[l], axis=1) /
                           np.linalg.norm(dUr[l], axis=1))) for l in range(3))
    return max(fro), col


@pytest.mark.parametrize("algo", ALGOS)
@pytest.mark.parametrize("prec", ["fp64", "ozaki8"])
def test_adjoint_c5_full_size(tc, c5_ref, prec, algo):
    w, c, ps, Jb, dUr, S, Jc = c5_ref
    say(f"adjoint c5 {prec} {algo}")
    assert all(np.array_equal(ps[0], q) for q in ps)
    cd, pd = dev(c), dev(ps[0])
    wv = dev(w.meta["w"])
    tol = TOL[prec]
    with algorithm(tc, algo, shapes_of(w), prec):
        # autograd: the forward keeps the Grams (both triangles), the backward
        # contracts them with the recomputed W
        Us = [dev(u).requires_grad_(True) for u in w.U]
        J = tc.TeiGram.apply(cd, pd, pd, pd, *Us, prec)
        (wv @ J @ wv).backward()
        dU = [host(u.grad) for u in Us]
        fro, col = grad_errors(dU, dUr)
        e_blk, e_cols = column_errors(host(J), Jc, S)
        say(f"   autograd: grad fro {fro:.2e} worst column {col:.2e}; "
            f"J {len(S)} columns {e_cols:.2e}")
        assert fro <= tol and col <= 10 * tol, (fro, col)
        assert e_blk <= tol and e_cols <= tol, (e_blk, e_cols)
        # no saved Grams: the backward recomputes them
        dU2 = [host(x) for x in tc.tei_gram_backward(cd, [pd, pd, pd], [dev(u) for u in w.U],
                                                     dev(Jb), prec=prec)]
        fro2, col2 = grad_errors(dU2, dUr)
        say(f"   recomputed Grams: grad fro {fro2:.2e} worst column {col2:.2e}")
        assert fro2 <= tol and col2 <= 10 * tol, (fro2, col2)


# --------------------------------------------------------------------------
# batched workload: a recorded 8-instance subset
# --------------------------------------------------------------------------
# instance -> (n, R_f): 0 (4096, 338), 1 (1024, 278), 3 (4096, 73),
# 4 (2048, 485), 11 (512, 93), 14 (512, 431), 34 (512, 33), 51 (1024, 485);
# 338, 485 pad to 384 and 512: ragged 128-wide int8 Gram tiles
C4_SUBSET = [0, 1, 3, 4, 11, 14, 34, 51]


@pytest.fixture(scope="module")
def c4_subset(orc):
    insts = wl.batched_instances(64, seed=0)
    chosen = [insts[i] for i in C4_SUBSET]
    assert sorted({w.n[0] for w in chosen}) == [512, 1024, 2048, 4096]
    refs = []
    for i, w in zip(C4_SUBSET, chosen):
        c, ps = oracle_setup(orc, w)
        S = block_columns(w.R_f, seed=1000 + i, per_block=1)
        say(f"oracle columns c4[{i}] n={w.n[0]} R_f={w.R_f}: {len(S)} columns")
        refs.append((c, ps, S, oracle_columns(orc, f"c4[{i}]", c, ps, w.U, S)))
    return chosen, refs


def _batch(chosen, refs):
    kern = {}
    batch = []
    for w, (c, ps, S, Jc) in zip(chosen, refs):
        if w.n[0] not in kern:
            kern[w.n[0]] = (dev(c), dev(ps[0]))
        cd, pd = kern[w.n[0]]
        batch.append((cd, [pd, pd, pd], [dev(u) for u in w.U]))
    return batch


def _check_batch(Js, chosen, refs, tol, tag):
    worst = 0.0
    for i, (J, w, (c, ps, S, Jc)) in enumerate(zip(Js, chosen, refs)):
        Jh = host(J)
        e_blk, e_cols = column_errors(Jh, Jc, S)
        worst = max(worst, e_blk, e_cols)
        assert e_blk <= tol and e_cols <= tol, (tag, C4_SUBSET[i], e_blk, e_cols)
        np.testing.assert_array_equal(Jh, Jh.T)
    say(f"   {tag}: worst normalised column error {worst:.2e}")


_EAGER = {}


@pytest.mark.parametrize("prec,route", [("fp64", "auto"), ("ozaki8", "fork_join"),
                                        ("ozaki8", "queue"), ("ozaki8", "queue_t64"),
                                        ("ozaki8", "queue_k2"), ("ozaki8", "queue_t64_k2"),
                                        ("ozaki8", "auto")])
def test_batched_c4_subset(tc, c4_subset, prec, route):
    """The 8-instance subset on every batch route: eager against the oracle
    columns, graph replays bitwise equal to the eager batch.  Every
    work-queue route gives bitwise the fork-join J: the int8 products
    accumulate exactly whatever the tile, and the binary64 recombination of a
    tile's int32 sums spans at most 53 bits, so it is exact, also for each of
    two K parts and for their sum.
    "auto": the autotuner picks the Toeplitz algorithm per mode shape and
    (int8) the batch route, as the benchmark runs the batch."""
    chosen, refs = c4_subset
    batch = _batch(chosen, refs)
    tol = TOL[prec]
    shapes = sorted({(w.n[0], w.R_f, w.R_N) for w in chosen})
    try:
        if route == "auto":
            tc.autotune_batched(batch, prec=prec)
        else:
            tc.batch_tune_set(batch, prec, route)
        used = tc.batch_tune_get(batch, prec)
        say(f"batched c4 subset {prec}: route {route} -> {used}")
        eager = tc.tei_gram_batched(batch, prec=prec)
        _check_batch(eager, chosen, refs, tol, f"eager ({used})")
        eager_h = [host(J) for J in eager]
        if route != "auto":
            _EAGER[(prec, route)] = eager_h
            ref = _EAGER.get((prec, "fork_join"))
            if ref is not None and route != "fork_join":
                for Jq, Jf in zip(eager_h, ref):
                    np.testing.assert_array_equal(Jq, Jf)
                say("   bitwise equal to the fork-join batch")
        g = tc.TeiGramGraph(batch, prec=prec)
        for rep in range(3):
            Js = g.replay()
            for Jg, Je in zip(Js, eager_h):
                np.testing.assert_array_equal(host(Jg), Je)
            junk = torch.randn(1 << 20, device="cuda", dtype=torch.float64)
            (junk * 2.0).sum().item()
            torch.cuda.synchronize()
        say("   graph replays bitwise equal to the eager batch")
    finally:
        for sh in shapes:
            tc.tune_set(*sh, prec, "auto")
        tc.batch_tune_set(batch, prec, "auto")


@pytest.mark.parametrize("route", ["queue", "queue_t64", "queue_k2", "queue_t64_k2"])
def test_queue_batch_saved_grams(tc, orc, route):
    """Saved Grams (both triangles, as the adjoint reads them) from the work
    queue, bitwise those of the fork-join route, with smooth, narrow and
    general terms (FFT route), the direct route and ragged R_f."""
    specs = [(300, 100, 24), (257, 300, 12), (64, 9, 4), (130, 70, 5)]
    batch, ws_ = [], []
    for i, (n, R_f, R_N) in enumerate(specs):
        w = wl.small_products(n, R_f, R_N=R_N, b=8.0, seed=70 + i)
        c, ps = oracle_setup(orc, w)
        batch.append((dev(c), [dev(p) for p in ps], [dev(u) for u in w.U]))
        ws_.append((w, c, ps))
    try:
        # a batch that keeps its Grams has its own entry in the tuning table
        tc.batch_tune_set(batch, "ozaki8", "fork_join", save_G=True)
        assert tc.batch_tune_get(batch, "ozaki8", save_G=True) == "fork_join"
        Jf, Gf = tc.tei_gram_batched(batch, prec="ozaki8", save_G=True)
        Gf = [host(G) for G in Gf]
        Jf = [host(J) for J in Jf]
        tc.batch_tune_set(batch, "ozaki8", route, save_G=True)
        Jq, Gq = tc.tei_gram_batched(batch, prec="ozaki8", save_G=True)
    finally:
        tc.batch_tune_set(batch, "ozaki8", "auto", save_G=True)
    for (w, c, ps), J1, G1, J2, G2 in zip(ws_, Jf, Gf, Jq, Gq):
        J2, G2 = host(J2), host(G2)
        np.testing.assert_array_equal(G2, np.swapaxes(G2, -1, -2))
        np.testing.assert_array_equal(G2, G1)
        np.testing.assert_array_equal(J2, J1)
        assert e_J(J2, orc.tei_gram(c, ps, w.U)) <= 1e-7


# --------------------------------------------------------------------------
# modes borrowing an earlier mode's kernel part
# --------------------------------------------------------------------------
@pytest.mark.parametrize("ns", [(256, 256, 256), (256, 200, 256)])
def test_modes_reusing_kernel_part(tc, orc, ns):
    """Kernel vectors [pa, pb, pa] (pb: another grid spacing, and in the
    second case another n): the third mode may reuse only the first mode's
    kernel part, which the second mode must not overwrite, both for a lone
    instance (one scratch region per mode) and in a batch (one region shared
    by the modes in turn)."""
    say(f"kernel part reuse {ns}")
    R_f, R_N = 70, 12
    w = wl.small_products(ns, R_f, R_N=R_N, b=6.0, seed=5)
    ua, ub = wl.sinc_params(R_N, ns[0], 6.0)
    ha, hb = 12.0 / ns[0], 9.0 / ns[1]
    t, a, _, pa = orc.newton_kernel(ns[0], ha, R_N, ua, ub)
    _, _, _, pb = orc.newton_kernel(ns[1], hb, R_N, ua, ub)
    c = a * ha * hb * ha
    ps = [pa, pb, pa]
    Jr = orc.tei_gram(c, ps, w.U)
    w2 = wl.small_products(ns, 33, R_N=R_N, b=6.0, seed=6)
    Jr2 = orc.tei_gram(c, ps, w2.U)
    cd, pad, pbd = dev(c), dev(pa), dev(pb)
    shapes = sorted({(nl, R_f, R_N) for nl in ns} | {(nl, 33, R_N) for nl in ns})
    for prec in ("ozaki8", "fp64"):
        with algorithm(tc, "fft", shapes, prec):
            J1 = host(tc.tei_gram(cd, [pad, pbd, pad], [dev(u) for u in w.U], prec=prec))
            Jb = tc.tei_gram_batched([(cd, [pad, pbd, pad], [dev(u) for u in w.U]),
                                      (cd, [pad, pbd, pad], [dev(u) for u in w2.U])], prec=prec)
            e1, eb, eb2 = e_J(J1, Jr), e_J(host(Jb[0]), Jr), e_J(host(Jb[1]), Jr2)
        say(f"   {prec}: lone {e1:.2e}, batch {eb:.2e} / {eb2:.2e}")
        assert max(e1, eb, eb2) <= TOL[prec], (prec, e1, eb, eb2)
