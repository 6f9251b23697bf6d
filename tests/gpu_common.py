"""Helpers shared by the GPU parity tests (device transfer, forcing the
Toeplitz algorithm, oracle set-up of the kernel vectors)."""
import contextlib
import sys

import numpy as np
import torch


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def host(x):
    torch.cuda.synchronize()
    return x.detach().cpu().numpy()


@contextlib.contextmanager
def algorithm(tc, algo, shapes, prec):
    """Force the Toeplitz algorithm for the given (n, R_f, R_N) mode shapes."""
    keys = sorted(set(shapes))
    for key in keys:
        if algo == "fft" and key[0] > 65536:
            continue
        tc.tune_set(*key, prec, algo)
    try:
        yield
    finally:
        for key in keys:
            tc.tune_set(*key, prec, "auto")


def shapes_of(w):
    return [(nl, w.R_f, w.R_N) for nl in w.n]


def oracle_setup(orc, w):
    """Oracle kernel vectors of the three modes and the weights c_k = a_k h1 h2 h3."""
    ps = []
    for l in range(3):
        t, a, cc, p = orc.newton_kernel(w.n[l], w.h[l], w.R_N, w.u0, w.hu)
        ps.append(p)
    c = a * w.h[0] * w.h[1] * w.h[2]
    return c, ps


def block_columns(R_f, seed, per_block=2, block=128):
    """Sampled columns of J for full-size checks: both ends and `per_block`
    seeded columns in every block of `block` columns (the Gram kernels tile
    J in blocks of 64 or 128, so every tile column is visited)."""
    rng = np.random.default_rng(seed)
    cols = {0, R_f - 1}
    for b0 in range(0, R_f, block):
        b1 = min(R_f, b0 + block)
        k = min(per_block, b1 - b0)
        cols.update(int(x) for x in rng.choice(np.arange(b0, b1), size=k, replace=False))
    return np.array(sorted(cols), dtype=np.int64)


_COLUMN_CACHE = {}


def oracle_columns(orc, key, c, ps, U, cols):
    """Oracle columns J[:, cols] ([len(cols)][R_f]), cached per (key, cols) so
    that tests of several routes on one workload share one oracle run."""
    k = (key, tuple(int(x) for x in cols))
    if k not in _COLUMN_CACHE:
        _COLUMN_CACHE[k] = orc.tei_gram_columns(c, ps, U, cols)
    return _COLUMN_CACHE[k]


def column_errors(J, Jc, S):
    """Normalised errors of the sampled columns S of J against the oracle
    columns Jc ([len(S)][R_f]): the S x S block with oracle diagonals only,
    and the whole columns scaled by the GPU diagonal for rows outside S."""
    block = Jc[:, S]
    d = np.diag(block)
    err_block = float(np.max(np.abs(J[np.ix_(S, S)] - block.T) / np.sqrt(np.outer(d, d))))
    dg = np.sqrt(np.abs(np.diag(J)))
    err_cols = float(np.max(np.abs(J[:, S] - Jc.T) / np.outer(dg, np.sqrt(d))))
    return err_block, err_cols
