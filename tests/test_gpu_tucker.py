"""Parity of the canonical-to-Tucker transform (tc_canonical_to_tucker,
Appendix part 1) with the oracle, through the C ABI, binary64.

The oracle takes every dominant subspace from a full SVD; the GPU from
orthogonal iteration and a Rayleigh-Ritz step.  Both fix each basis
vector's sign the same way, so where the leading singular values are apart
(relative gaps down to 3e-5 here) the bases agree entry by entry: a singular
vector moves by about u sigma_1^2 / (sigma_i^2 - sigma_{i+1}^2).  The tests
assert |dZ| <= 1e-9 per entry, |dbeta| <= 1e-9 max|beta|, the singular values
to 1e-10 relative, and orthonormal rows."""
import numpy as np
import pytest

from paper_1504_06289_amd import workloads as wl
from tests.gpu_common import dev, host, say

pytestmark = pytest.mark.gpu


def compare(tc, orc, c, A3, ranks, m_max, its=20, eps=0.0):
    Zg, bg, svg, rg = tc.canonical_to_tucker(dev(c), [dev(a) for a in A3], ranks, m_max, its,
                                             eps)
    Zg = [host(z) for z in Zg]
    bg = host(bg)
    Zo, bo, svo = orc.canonical_to_tucker(c, A3, ranks, m_max, eps)
    if eps > 0:
        # step (A)'s singular values, not too close to the threshold
        sA = [np.linalg.svd(A3[l].T, compute_uv=False) for l in range(3)]
        ro = orc.tucker_ranks(sA, ranks, eps)
        say(f"   ranks: GPU {rg}, oracle {ro}")
        assert rg == ro
        for l in range(3):
            rat = np.maximum(sA[l][:ranks[l]] / sA[l][0], 1e-300)
            assert np.min(np.abs(np.log(rat / eps))) > 0.05
    for l in range(3):
        s = svo[l]
        r = rg[l] if eps > 0 else ranks[l]
        gaps = (s[:r] - s[1:r + 1]) / s[0] if len(s) > r else (s[:r - 1] - s[1:r]) / s[0]
        dz = np.max(np.abs(Zg[l] - Zo[l]))
        orth = np.max(np.abs(Zg[l][:r] @ Zg[l][:r].T - np.eye(r)))
        assert np.all(Zg[l][r:] == 0.0)
        dsv = np.max(np.abs(svg[l][:r] - s[:r]) / s[0])
        say(f"   mode {l}: min gap {gaps.min():.1e}  |dZ| {dz:.1e}  orth {orth:.1e}  "
            f"dsv {dsv:.1e}")
        assert orth <= 1e-13
        assert dsv <= 1e-10
        assert dz <= 1e-9
    db = np.max(np.abs(bg - bo)) / np.max(np.abs(bo))
    say(f"   |dbeta| / max|beta| = {db:.1e}")
    assert db <= 1e-9
    return Zg, bg


@pytest.mark.parametrize("n,R,ranks,m_max", [((128, 96, 80), 60, (8, 6, 7), 2),
                                              ((256, 256, 256), 200, (16, 16, 16), 2),
                                              ((300, 200, 100), 150, (12, 10, 9), 1),
                                              ((200, 150, 120), 90, (10, 10, 10), 0),
                                              ((20, 12, 30), 40, (6, 5, 7), 2),
                                              ((512, 512, 512), 400, (24, 20, 22), 1),
                                              ((48, 40, 36), 400, (8, 8, 8), 1)])
def test_c2t_density(tc, orc, n, R, ranks, m_max):
    """A density in canonical format (Gaussian-product factors, weights in
    [0.1, 1]): the rank reduction the transform is there for."""
    say(f"c2t density n={n} R={R} ranks={ranks} m_max={m_max}")
    V, d = wl.density(n, 7.0, R, seed=R)
    compare(tc, orc, d, V, ranks, m_max)


def test_c2t_exact_low_multilinear_rank(tc, orc):
    """Side matrices spanning r_l-dimensional subspaces: the Tucker form
    reproduces the tensor (checked on the full 3D grid)."""
    rng = np.random.default_rng(3)
    n3, r3, R = (40, 33, 27), (5, 4, 6), 70
    A3 = [rng.standard_normal((R, r3[l])) @ rng.standard_normal((r3[l], n3[l])) for l in range(3)]
    c = rng.uniform(0.5, 2.0, R)
    say("c2t exact multilinear rank")
    Zg, bg = compare(tc, orc, c, A3, r3, 2)
    T = orc.canonical_full(c, A3)
    assert np.max(np.abs(orc.tucker_full(Zg, bg) - T)) <= 1e-11 * np.max(np.abs(T))


def test_c2t_subspace_of_64_rows(tc, orc):
    """Ranks of 32 make the iterated subspace k = 64 rows in every mode: the
    largest orthonormalisation block (four Cholesky panels, the 64-row
    substitution) on full-rank side matrices with a decaying spectrum; phase
    (A) takes the Gram form (m = 200), the sweeps iterate on X (m = 1024)."""
    rng = np.random.default_rng(8)
    n3, R, r3 = (80, 76, 72), 200, (32, 32, 32)
    A3 = [rng.standard_normal((R, n3[l])) * np.exp(-0.05 * np.arange(n3[l]))[None, :]
          for l in range(3)]
    c = rng.uniform(0.5, 2.0, R)
    say("c2t k = 64")
    compare(tc, orc, c, A3, r3, 1)


def test_c2t_few_terms_and_determinism(tc, orc):
    """Fewer terms than the iterated subspace (R < k: the subspace is filled
    with pseudo-random rows) and bitwise repeatable results."""
    V, d = wl.density((90, 70, 60), 6.0, 10, seed=2)
    say("c2t R=10 < k")
    compare(tc, orc, d, V, (4, 4, 4), 1)
    A = [dev(v) for v in V]
    Z1, b1, _, _ = tc.canonical_to_tucker(dev(d), A, (4, 4, 4), 1)
    Z2, b2, _, _ = tc.canonical_to_tucker(dev(d), A, (4, 4, 4), 1)
    assert np.array_equal(host(b1), host(b2))
    assert all(np.array_equal(host(x), host(y)) for x, y in zip(Z1, Z2))


def test_c2t_epsilon_truncation(tc, orc):
    """The epsilon truncation of step (A): the true ranks of a tensor of low
    multilinear rank from larger maximal ranks (full tensor reproduced), and
    a density truncated at 0.29 of the largest singular value, against the
    oracle's ranks, bases and core."""
    rng = np.random.default_rng(4)
    n3, r3, R = (40, 33, 27), (5, 4, 6), 70
    A3 = [rng.standard_normal((R, r3[l])) @ rng.standard_normal((r3[l], n3[l])) for l in range(3)]
    c = rng.uniform(0.5, 2.0, R)
    say("c2t eps exact")
    Zg, bg = compare(tc, orc, c, A3, (9, 8, 10), 1, eps=1e-9)
    T = orc.canonical_full(c, A3)
    assert np.max(np.abs(orc.tucker_full(Zg, bg) - T)) <= 1e-11 * np.max(np.abs(T))
    V, d = wl.density((160, 120, 100), 7.0, 80, seed=6)
    say("c2t eps density")
    compare(tc, orc, d, V, (16, 16, 16), 1, eps=0.29)


@pytest.mark.parametrize("n3,R,ranks,m_max", [((1, 2, 3), 5, (1, 1, 1), 2),
                                              ((1, 1, 1), 1, (1, 1, 1), 1),
                                              ((7, 3, 9), 2, (2, 2, 2), 1)])
def test_c2t_degenerate_sizes(tc, orc, n3, R, ranks, m_max):
    """One cell in a mode (a subspace of k = n rows), a single term, and fewer
    terms than the ranks' images: the full tensor is reproduced whenever the
    ranks reach the multilinear rank."""
    rng = np.random.default_rng(sum(n3) + R)
    A3 = [rng.standard_normal((R, nl)) for nl in n3]
    c = rng.uniform(0.5, 1.5, R)
    say(f"c2t degenerate n={n3} R={R} ranks={ranks}")
    Zg, bg, _, rg = tc.canonical_to_tucker(dev(c), [dev(a) for a in A3], ranks, m_max)
    Zg = [host(z) for z in Zg]
    bg = host(bg)
    for l in range(3):
        np.testing.assert_allclose(Zg[l] @ Zg[l].T, np.eye(ranks[l]), atol=1e-13)
    T = orc.canonical_full(c, A3)
    Zo, bo, _ = orc.canonical_to_tucker(c, A3, ranks, m_max)
    To = orc.tucker_full(Zo, bo)
    Tg = orc.tucker_full(Zg, bg)
    assert np.max(np.abs(Tg - To)) <= 1e-12 * max(np.max(np.abs(T)), 1e-300)
