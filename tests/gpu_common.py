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
        if algo == "fft" and key[0] > 4096:
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
