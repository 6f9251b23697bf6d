"""Parity of the nuclear potential matrix (tc_nuclear, Section 3.3) with the
FP64 oracle, through the C ABI.

Bound: every 1D matrix entry sum_x U[i][x] U[j][x] s[x] is a binary64
contraction of n products (MFMA partial sums: error below n u sum|U_i U_j s|),
and V sums M R_N products of three of them.  The tests assert, per entry,
  |dV_ij| <= 1e-12 sum_a |Z_a| sum_q |c_q|/vol prod_l sum_x |U^l_i U^l_j s^l_aq|
(the absolute condition scale of the entry) and report the largest ratio."""
import numpy as np
import pytest

from paper_1504_06289_amd import workloads as wl
from tests.gpu_common import dev, host, oracle_setup, say

pytestmark = pytest.mark.gpu


def scale(c, ps, h3, U3, Z, pos):
    vol = h3[0] * h3[1] * h3[2]
    S = np.zeros((U3[0].shape[0],) * 2)
    for a in range(len(Z)):
        for q in range(len(c)):
            prod = np.full_like(S, abs(Z[a] * c[q]) / vol)
            for l in range(3):
                n = U3[l].shape[1]
                s = np.abs(ps[l][q, np.arange(n) - pos[a][l] + n - 1])
                A = np.abs(U3[l])
                prod = prod * ((A * s[None, :]) @ A.T)
            S += prod
    return S


def worst(V, Vr, sc):
    """Largest |dV| / scale; entries of zero scale (functions that do not
    overlap anywhere) must agree exactly."""
    d = np.abs(V - Vr)
    assert np.all(d[sc == 0] == 0)
    return float(np.max(d[sc > 0] / sc[sc > 0]))


def run(tc, c, ps, U3, h3, Z, pos):
    return host(tc.nuclear(dev(c), [dev(p) for p in ps], [dev(u) for u in U3], h3, Z, pos))


@pytest.mark.parametrize("n,R_f,R_N,M", [((1, 1, 1), 1, 1, 1), ((40, 33, 47), 21, 9, 2),
                                         ((130, 64, 200), 70, 6, 3),
                                         ((257, 257, 257), 65, 12, 5),
                                         ((300, 100, 512), 130, 8, 1),
                                         ((96, 96, 96), 200, 20, 70)])
def test_nuclear_small(tc, orc, n, R_f, R_N, M):
    say(f"nuclear n={n} R_f={R_f} R_N={R_N} M={M}")
    w = wl.small_products(n, R_f, R_N=R_N, b=7.0, seed=R_f + M)
    c, ps = oracle_setup(orc, w)
    rng = np.random.default_rng(M)
    Z = rng.uniform(1.0, 8.0, M).round()
    pos = [[int(rng.integers(0, nl)) for nl in w.n] for _ in range(M)]
    pos[0] = [0, w.n[1] - 1, w.n[2] // 2]   # boundary cells
    V = run(tc, c, ps, w.U, w.h, Z, pos)
    Vr = orc.nuclear(c, ps, w.h, w.U, Z, pos)
    ratio = worst(V, Vr, scale(c, ps, w.h, w.U, Z, pos))
    say(f"   max |dV| / scale = {ratio:.2e}")
    assert ratio <= 1e-12
    assert np.array_equal(V, V.T)


def test_nuclear_determinism_and_device_kernel(tc, orc):
    """Kernel vectors from tc_newton_kernel, charges of both signs (a point
    charge difference), bitwise repeatable."""
    w = wl.small_products((120, 90, 77), 50, R_N=14, b=6.0, seed=11)
    t, c, p = tc.newton_kernel(w.n[0], w.h[0], w.R_N, w.u0, w.hu)
    c = c / w.h[0] ** 3 * (w.h[0] * w.h[1] * w.h[2])   # a_q h1 h2 h3
    ps = []
    for l in range(3):
        ps.append(tc.newton_kernel(w.n[l], w.h[l], w.R_N, w.u0, w.hu)[2])
    Z = np.array([6.0, -1.0, 1.0])
    pos = [[10, 20, 30], [60, 45, 38], [119, 0, 76]]
    U3 = [dev(u) for u in w.U]
    V1 = host(tc.nuclear(dev(c), ps, U3, w.h, Z, pos))
    V2 = host(tc.nuclear(dev(c), ps, U3, w.h, Z, pos))
    assert np.array_equal(V1, V2)
    c_o, ps_o = oracle_setup(orc, w)
    Vr = orc.nuclear(c_o, ps_o, w.h, w.U, Z, pos)
    sc = scale(c_o, ps_o, w.h, w.U, Z, pos)
    # kernel vectors within 1e-12 relative of the oracle's
    assert worst(V1, Vr, sc) <= 5e-12


def test_nuclear_largest_pair_count(tc, orc):
    """2047 nuclei x 32 terms = 65504 (nucleus, term) pairs, the most the grid
    of the diagonal Gram takes (the ABI limit is 65535), in 32 argument
    chunks."""
    w = wl.small_products((64, 48, 40), 8, R_N=32, b=5.0, seed=9)
    c, ps = oracle_setup(orc, w)
    rng = np.random.default_rng(2047)
    M = 2047
    Z = rng.uniform(0.5, 3.0, M)
    pos = [[int(rng.integers(0, nl)) for nl in w.n] for _ in range(M)]
    say(f"nuclear M={M} pairs={M * 32}")
    V = run(tc, c, ps, w.U, w.h, Z, pos)
    Vr = orc.nuclear(c, ps, w.h, w.U, Z, pos)
    ratio = worst(V, Vr, scale(c, ps, w.h, w.U, Z, pos))
    say(f"   max |dV| / scale = {ratio:.2e}")
    assert ratio <= 1e-12


def test_nuclear_full_size_sampled(tc, orc):
    """The bench configuration (the 4096-cell products, 1024 functions, 32
    kernel terms, three nuclei in a water-like geometry): 24 sampled entries
    against the oracle's entry-by-entry evaluation of the definition."""
    w = wl.config("c3")
    c, ps = oracle_setup(orc, w)
    geom = np.array([[0.0, 0.0, 0.0], [1.43, 1.11, 0.0], [-1.43, 1.11, 0.0]])
    Z = np.array([8.0, 1.0, 1.0])
    pos = [[int((x + w.b) / w.h[l]) for l, x in enumerate(g)] for g in geom]
    say(f"nuclear full size: n={w.n} R_f={w.R_f} R_N={w.R_N}")
    V = run(tc, c, ps, w.U, w.h, Z, pos)
    rng = np.random.default_rng(12)
    pairs = []
    for s_ in range(24):
        i = int(rng.integers(0, w.R_f))
        pairs.append((i, i if s_ % 3 == 0 else int(rng.integers(0, w.R_f))))
    ref, sc = orc.nuclear_entries(c, ps, w.h, w.U, Z, pos, pairs)
    worst_ratio, overlapping = 0.0, 0
    for (i, j), r, s_ in zip(pairs, ref, sc):
        if s_ == 0.0:  # the two functions do not overlap in some mode
            assert V[i, j] == 0.0
            continue
        overlapping += 1
        worst_ratio = max(worst_ratio, abs(V[i, j] - r) / s_)
    say(f"   max |dV| / scale over {overlapping} overlapping samples = {worst_ratio:.2e}")
    assert overlapping >= 8
    assert worst_ratio <= 1e-12
