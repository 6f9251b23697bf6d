"""ctypes front end of the FP64 CPU oracle (oracle/tc_oracle.c).

TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the benchmark's
CPU-baseline leg import this module.  The product library never does, and
this module imports nothing from the product package.

Arrays are numpy float64, C-contiguous, in the layouts of tc_oracle.h:
U [R_f][n], p [R_N][2n-1], W [R_N][R_f][n], G [R_N][R_f][R_f], J [R_f][R_f].
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tc_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# IEEE semantics are required by the error-free transformations in the
# compensated sums: no contraction into FMAs, no fast-math.  x86-64-v3 gives a
# hardware FMA for the TwoProduct step on any AVX2 host.
CFLAGS = ["-O2", "-std=c11", "-march=x86-64-v3", "-ffp-contract=off",
          "-fno-fast-math", "-fopenmp", "-fPIC", "-shared"]


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (every call recompiles when force)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm", "-lpthread"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        d = ctypes.c_double
        pd = ctypes.POINTER(ctypes.c_double)
        ppd = ctypes.POINTER(pd)
        pi = ctypes.POINTER(ctypes.c_int)
        L.oracle_sinc_rule.argtypes = [ctypes.c_int, d, d, pd, pd]
        L.oracle_cell_integral.argtypes = [d, d, ctypes.c_long]
        L.oracle_cell_integral.restype = d
        L.oracle_newton_kernel.argtypes = [ctypes.c_int, d, ctypes.c_int, d, d, pd, pd, pd, pd]
        L.oracle_convolve.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, pd, pd, pd,
                                      ctypes.c_int]
        L.oracle_gram.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, pd, pd, pd,
                                  ctypes.c_int]
        L.oracle_tei_gram.argtypes = [pi, ctypes.c_int, ctypes.c_int, pd, ppd, ppd, pd, pd,
                                      ctypes.c_int]
        L.oracle_tei_gram_columns.argtypes = [pi, ctypes.c_int, ctypes.c_int, pd, ppd, ppd,
                                              ctypes.c_int, pi, pd, ctypes.c_int]
        L.oracle_tei_gram_backward.argtypes = [pi, ctypes.c_int, ctypes.c_int, pd, ppd, ppd,
                                               pd, ppd]
        L.oracle_coulomb.argtypes = [pi, ctypes.c_int, ctypes.c_int, ctypes.c_int, pd, ppd,
                                     ppd, ppd, pd, pd, ctypes.c_int]
        L.oracle_bruteforce_J.argtypes = [ctypes.c_int, d, ctypes.c_int, ctypes.c_int, pd, pd,
                                          ppd, pd]
        L.oracle_gauss_legendre.argtypes = [ctypes.c_int, pd, pd]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _pp(arrs):
    ptrs = (ctypes.POINTER(ctypes.c_double) * len(arrs))(*[_p(a) for a in arrs])
    return ptrs


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def sinc_rule(R_N: int, u0: float, hu: float):
    t = np.empty(R_N)
    a = np.empty(R_N)
    lib().oracle_sinc_rule(R_N, u0, hu, _p(t), _p(a))
    return t, a


def cell_integral(t: float, h: float, m: int) -> float:
    return lib().oracle_cell_integral(t, h, m)


def newton_kernel(n: int, h: float, R_N: int, u0: float, hu: float):
    """Returns (t, a, c, p) with c_k = a_k h^3 and p [R_N][2n-1]."""
    t, a, c = np.empty(R_N), np.empty(R_N), np.empty(R_N)
    p = np.empty((R_N, 2 * n - 1))
    lib().oracle_newton_kernel(n, h, R_N, u0, hu, _p(t), _p(a), _p(c), _p(p))
    return t, a, c, p


def convolve(p: np.ndarray, U: np.ndarray, compensated: bool = True) -> np.ndarray:
    p, U = _f64(p), _f64(U)
    R_N, L = p.shape
    R_f, n = U.shape
    assert L == 2 * n - 1
    W = np.empty((R_N, R_f, n))
    lib().oracle_convolve(n, R_f, R_N, _p(p), _p(U), _p(W), int(compensated))
    return W


def gram(U: np.ndarray, W: np.ndarray, compensated: bool = True) -> np.ndarray:
    U, W = _f64(U), _f64(W)
    R_f, n = U.shape
    R_N = W.shape[0]
    G = np.empty((R_N, R_f, R_f))
    lib().oracle_gram(n, R_f, R_N, _p(U), _p(W), _p(G), int(compensated))
    return G


def tei_gram(c, p3, U3, return_G: bool = False, compensated: bool = True):
    """J = sum_k c_k G1_k o G2_k o G3_k.  p3, U3: sequences of 3 arrays."""
    c = _f64(c)
    p3 = [_f64(x) for x in p3]
    U3 = [_f64(x) for x in U3]
    R_f = U3[0].shape[0]
    R_N = c.shape[0]
    n = (ctypes.c_int * 3)(*[u.shape[1] for u in U3])
    J = np.empty((R_f, R_f))
    G = np.empty((3, R_N, R_f, R_f)) if return_G else None
    lib().oracle_tei_gram(n, R_f, R_N, _p(c), _pp(p3), _pp(U3), _p(J),
                          _p(G) if G is not None else None, int(compensated))
    return (J, G) if return_G else J


def tei_gram_columns(c, p3, U3, cols, compensated: bool = True) -> np.ndarray:
    """Returns J[:, cols] as an array of shape [len(cols)][R_f] (row q = column cols[q])."""
    c = _f64(c)
    p3 = [_f64(x) for x in p3]
    U3 = [_f64(x) for x in U3]
    R_f = U3[0].shape[0]
    R_N = c.shape[0]
    n = (ctypes.c_int * 3)(*[u.shape[1] for u in U3])
    cols = np.ascontiguousarray(cols, dtype=np.int32)
    out = np.empty((len(cols), R_f))
    lib().oracle_tei_gram_columns(n, R_f, R_N, _p(c), _pp(p3), _pp(U3), len(cols),
                                  cols.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                  _p(out), int(compensated))
    return out


def coulomb(c, p3, U3, V3, d, compensated: bool = True) -> np.ndarray:
    """Jd[i] = sum_q c_q sum_m d_m prod_l <U^l[i], (T^l_q V^l)[m]>: the Coulomb
    entries of the product functions (rows of U^l) against the density
    sum_m d_m v^1_m x v^2_m x v^3_m (rows of V^l), Section 3.1."""
    c, d = _f64(c), _f64(d)
    p3 = [_f64(x) for x in p3]
    U3 = [_f64(x) for x in U3]
    V3 = [_f64(x) for x in V3]
    R_f, R_rho, R_N = U3[0].shape[0], V3[0].shape[0], c.shape[0]
    for l in range(3):
        assert U3[l].shape[1] == V3[l].shape[1] and V3[l].shape[0] == R_rho
    n = (ctypes.c_int * 3)(*[u.shape[1] for u in U3])
    Jd = np.empty(R_f)
    lib().oracle_coulomb(n, R_f, R_rho, R_N, _p(c), _pp(p3), _pp(U3), _pp(V3), _p(d),
                         _p(Jd), int(compensated))
    return Jd


def tei_gram_backward(c, p3, U3, Jbar):
    c = _f64(c)
    p3 = [_f64(x) for x in p3]
    U3 = [_f64(x) for x in U3]
    Jbar = _f64(Jbar)
    R_f = U3[0].shape[0]
    R_N = c.shape[0]
    n = (ctypes.c_int * 3)(*[u.shape[1] for u in U3])
    dU = [np.empty_like(u) for u in U3]
    lib().oracle_tei_gram_backward(n, R_f, R_N, _p(c), _pp(p3), _pp(U3), _p(Jbar), _pp(dU))
    return dU


def bruteforce_J(h: float, a, p, U3) -> np.ndarray:
    a, p = _f64(a), _f64(p)
    U3 = [_f64(x) for x in U3]
    R_f, n = U3[0].shape
    R_N = a.shape[0]
    J = np.empty((R_f, R_f))
    lib().oracle_bruteforce_J(n, h, R_f, R_N, _p(a), _p(p), _pp(U3), _p(J))
    return J


def gauss_legendre(npts: int):
    x, w = np.empty(npts), np.empty(npts)
    lib().oracle_gauss_legendre(npts, _p(x), _p(w))
    return x, w


# --------------------------------------------------------------------------
# 1D density fitting and the factorised TEI matrix (Section 3.2): plain NumPy
# on explicit matrices, for small sizes.
# --------------------------------------------------------------------------
def pivoted_cholesky(A: np.ndarray, tol: float, R_max: int):
    """Pivoted (diagonally pivoted, rank-revealing) Cholesky of a symmetric
    positive semi-definite A: at each step the pivot is the largest residual
    diagonal entry; the step is taken while the residual trace exceeds tol
    (and fewer than R_max columns exist).  Returns (L [N][R], pivots [R],
    residual diagonal [N]) with A ~ L L^T, the residual diagonal of A - L L^T
    and L[pivots[r], s] = 0 for s > r."""
    A = np.asarray(A, dtype=np.float64)
    N = A.shape[0]
    d = np.diag(A).copy()
    L = np.zeros((N, 0))
    piv = []
    while len(piv) < R_max and d.sum() > tol:
        p = int(np.argmax(d))
        if d[p] <= 0.0:
            break
        col = A[:, p] - L @ L[p, :]
        l = col / np.sqrt(d[p])
        l[piv] = 0.0   # the residual vanishes on the earlier pivots
        L = np.column_stack([L, l])
        d = d - l * l
        d[p] = 0.0
        piv.append(p)
    return L, np.array(piv, dtype=np.int64), d


def density_fit(F: np.ndarray, tol: float, R_max: int):
    """1D density fitting of one mode's side matrix F [N_pair][n] (rows: pair
    products on the grid): pivoted Cholesky of A = F^T F over the grid points
    (truncated when the residual trace is at most tol^2 trace(A)), then
    F ~ V U with V = F[:, P] (the products at the R pivot points) and
    U = A[P, P]^-1 A[P, :] (R x n), i.e. U = L[P, :]^-T L^T.
    Returns (U [R][n], V [N_pair][R], pivots [R], residual trace)."""
    F = np.asarray(F, dtype=np.float64)
    A = F.T @ F
    L, piv, d = pivoted_cholesky(A, tol * tol * np.trace(A), R_max)
    R = len(piv)
    if R == 0:
        return np.zeros((0, F.shape[1])), np.zeros((F.shape[0], 0)), piv, float(d.sum())
    LP = L[piv, :]                                   # lower triangular in pivot order
    U = np.linalg.solve(LP.T, L.T)                   # L[P,:]^-T L^T
    V = F[:, piv]
    return U, V, piv, float(d.sum())


def tei_matrix_factored(c, V3, M3) -> np.ndarray:
    """B = sum_k c_k  o_l  V^l M^l_k V^l^T  (Section 3.2, the factorised TEI
    matrix over the pair products; V^l [N_pair][R_l], M^l [R_N][R_l][R_l])."""
    c = np.asarray(c, dtype=np.float64)
    B = 0.0
    for k in range(c.shape[0]):
        term = c[k]
        for l in range(3):
            term = term * (V3[l] @ M3[l][k] @ V3[l].T)
        B = B + term
    return B


def tei_cholesky(c, V3, M3, tol: float, R_max: int):
    """Pivoted Cholesky of the factorised B (Section 3.2): B ~ L L^T, the
    steps taken while the residual trace exceeds tol.
    Returns (L [N_pair][R_B], pivots [R_B], residual diagonal)."""
    return pivoted_cholesky(tei_matrix_factored(c, V3, M3), tol, R_max)


# --------------------------------------------------------------------------
# Assembled lattice sums of the Newton kernel (Section 5.1, eq. CoulombLatTensCan)
# and the lattice interaction energy (Section 5.2, eq. EnergyLattice).  The
# lattice has L_l unit cells of n0 grid cells per direction (n_l = n0 L_l); the charge of unit cell j sits in
# grid cell j n0 + n0 // 2 (the cell at the unit cell's centre).
# --------------------------------------------------------------------------
def lattice_sum(p: np.ndarray, n0: int, L: int) -> np.ndarray:
    """Assembled vectors of one direction: A[q][i] = sum_j p_q[i - (j n0 + n0//2)],
    i < n = n0 L, the kernel vector p [R][2n-1] indexed by lag (lag m at m + n - 1):
    the sum over the lattice of the shifted and windowed kernel vectors."""
    p = np.asarray(p, dtype=np.float64)
    n = n0 * L
    R = p.shape[0]
    assert p.shape[1] == 2 * n - 1
    A = np.zeros((R, n))
    i = np.arange(n)
    for j in range(L):
        A += p[:, i - (j * n0 + n0 // 2) + n - 1]
    return A


def lattice_sum_entries(p: np.ndarray, n0: int, L: int, samples):
    """Entries A[q][i] of lattice_sum for the listed (q, i) pairs, each an
    exactly rounded sum (math.fsum) over the L unit cells, with the sum of
    the magnitudes of its terms (the scale of a rounding bound)."""
    import math
    p = np.asarray(p, dtype=np.float64)
    n = n0 * L
    assert p.shape[1] == 2 * n - 1
    vals, scales = [], []
    for q, i in samples:
        terms = [p[q, i - (j * n0 + n0 // 2) + n - 1] for j in range(L)]
        vals.append(math.fsum(terms))
        scales.append(math.fsum(abs(x) for x in terms))
    return np.array(vals), np.array(scales)


def lattice_potential_direct(c, p3, h3, n0, L3, points) -> np.ndarray:
    """The separable kernel summed over the lattice, point by point: for grid
    points (i1, i2, i3), V = sum_j sum_q (c_q / (h1 h2 h3)^2) prod_l p^l_q[i_l - x_jl]
    (x_j the charge cells), i.e. sum_j K(x_i - x_j) with K the kernel's
    approximation of 1/|x| (its cell integrals divided by the cell volume)."""
    c = np.asarray(c, dtype=np.float64)
    w = c / (h3[0] * h3[1] * h3[2]) ** 2
    out = []
    for (i1, i2, i3) in points:
        idx = (i1, i2, i3)
        s = 0.0
        for j1 in range(L3[0]):
            for j2 in range(L3[1]):
                for j3 in range(L3[2]):
                    js = (j1, j2, j3)
                    prod = w.copy()
                    for l in range(3):
                        n = n0 * L3[l]
                        prod = prod * p3[l][:, idx[l] - (js[l] * n0 + n0 // 2) + n - 1]
                    s += prod.sum()
        out.append(s)
    return np.array(out)


def lattice_energy_direct(c, p3, h3, n0, L3, Z: float) -> float:
    """E = Z^2/2 sum_{k != j} K(x_k - x_j) over the charge cells, pair by pair,
    with the separable kernel K of lattice_potential_direct."""
    c = np.asarray(c, dtype=np.float64)
    w = c / (h3[0] * h3[1] * h3[2]) ** 2
    pts = [(j1, j2, j3) for j1 in range(L3[0]) for j2 in range(L3[1]) for j3 in range(L3[2])]
    E = 0.0
    for a in pts:
        for b in pts:
            if a == b:
                continue
            prod = w.copy()
            for l in range(3):
                n = n0 * L3[l]
                prod = prod * p3[l][:, (a[l] - b[l]) * n0 + n - 1]
            E += prod.sum()
    return 0.5 * Z * Z * E


def coulomb_lattice_energy_lags(b: float, L3, Z: float) -> float:
    """The same energy grouped by lattice lag: the lag d occurs in
    prod_l (L_l - |d_l|) ordered pairs, so
    E = Z^2/2 sum_{d != 0} prod_l (L_l - |d_l|) / (b |d|), O(L^3) terms."""
    j = [np.arange(-(Ll - 1), Ll) for Ll in L3]
    m = [(Ll - np.abs(jl)).astype(np.float64) for Ll, jl in zip(L3, j)]
    E = 0.0
    for a in range(len(j[0])):
        d2 = (j[0][a] ** 2 + j[1][:, None] ** 2 + j[2][None, :] ** 2).astype(np.float64)
        mult = m[0][a] * m[1][:, None] * m[2][None, :]
        if j[0][a] == 0:
            d2[L3[1] - 1, L3[2] - 1] = np.inf   # the zero lag: no pair
        E += np.sum(mult / (b * np.sqrt(d2)))
    return 0.5 * Z * Z * E


def coulomb_lattice_energy_exact(b: float, L3, Z: float) -> float:
    """E = Z^2/2 sum_{k != j} 1/|x_k - x_j| for charges on the lattice b Z^3."""
    g = np.stack(np.meshgrid(*[np.arange(Ll) for Ll in L3], indexing="ij"), -1).reshape(-1, 3)
    E = 0.0
    for a in range(len(g)):
        d = np.sqrt(np.sum(((g - g[a]) * b) ** 2, axis=1))
        d[a] = np.inf
        E += np.sum(1.0 / d)
    return 0.5 * Z * Z * E


# --------------------------------------------------------------------------
# Nuclear potential operator (Section 3.3): the master kernel shifted to each
# nucleus, summed with the charges, and its Galerkin matrix in the basis of
# rank-1 products.  Nuclei sit at grid-cell centres (the windowing shifts by
# whole cells): pos[alpha][l] is the cell of nucleus alpha along mode l.
# --------------------------------------------------------------------------
def nuclear(c, p3, h3, U3, Z, pos) -> np.ndarray:
    """V[k][m] = -sum_alpha Z_alpha sum_q (c_q / (h1 h2 h3))
                 prod_l sum_a U^l[k][a] U^l[m][a] p^l_q[a - pos_alpha,l],
    i.e. vol sum_x g_k(x) g_m(x) V_c(x) over the grid cells x, with
    V_c(x) = -sum_alpha Z_alpha K(x - x_alpha) and K the kernel's
    approximation of 1/|x| (c_q/(h1 h2 h3)^2 prod_l p^l_q)."""
    c = _f64(c)
    U3 = [_f64(u) for u in U3]
    p3 = [_f64(p) for p in p3]
    vol = float(h3[0] * h3[1] * h3[2])
    R_f = U3[0].shape[0]
    V = np.zeros((R_f, R_f))
    for alpha in range(len(Z)):
        for q in range(c.shape[0]):
            prod = np.ones((R_f, R_f))
            for l in range(3):
                n = U3[l].shape[1]
                s = p3[l][q, np.arange(n) - int(pos[alpha][l]) + n - 1]
                prod = prod * ((U3[l] * s[None, :]) @ U3[l].T)
            V -= Z[alpha] * c[q] / vol * prod
    return V


def nuclear_entries(c, p3, h3, U3, Z, pos, pairs):
    """Entries V[k][m] of nuclear for the listed (k, m) pairs, each formed
    from its own definition: for every nucleus and kernel term the product
    over the modes of sum_a U^l[k][a] U^l[m][a] p^l_q[a - pos_alpha,l].
    Also returns, per entry, the same sum over absolute values (the scale of
    a rounding bound; zero when the two functions do not overlap)."""
    c = _f64(c)
    U3 = [_f64(u) for u in U3]
    p3 = [_f64(p) for p in p3]
    vol = float(h3[0] * h3[1] * h3[2])
    vals, scales = [], []
    for k, m in pairs:
        v, sc = 0.0, 0.0
        for alpha in range(len(Z)):
            for q in range(c.shape[0]):
                prod = Z[alpha] * c[q] / vol
                aprod = abs(Z[alpha] * c[q]) / vol
                for l in range(3):
                    n = U3[l].shape[1]
                    s = p3[l][q, np.arange(n) - int(pos[alpha][l]) + n - 1]
                    prod *= float(np.dot(U3[l][k] * U3[l][m], s))
                    aprod *= float(np.dot(np.abs(U3[l][k] * U3[l][m]), np.abs(s)))
                v -= prod
                sc += aprod
        vals.append(v)
        scales.append(sc)
    return np.array(vals), np.array(scales)


def nuclear_bruteforce(c, p3, h3, U3, Z, pos) -> np.ndarray:
    """The same matrix on the full 3D grid (tiny grids only): the potential
    V_c on every cell, then vol sum_x g_k(x) g_m(x) V_c(x)."""
    c = _f64(c)
    n = [u.shape[1] for u in U3]
    vol = float(h3[0] * h3[1] * h3[2])
    Vc = np.zeros(n)
    for alpha in range(len(Z)):
        for q in range(c.shape[0]):
            f = [p3[l][q, np.arange(n[l]) - int(pos[alpha][l]) + n[l] - 1] for l in range(3)]
            Vc -= Z[alpha] * c[q] / vol ** 2 * np.einsum("a,b,c->abc", f[0], f[1], f[2])
    R_f = U3[0].shape[0]
    V = np.zeros((R_f, R_f))
    for k in range(R_f):
        gk = np.einsum("a,b,c->abc", U3[0][k], U3[1][k], U3[2][k])
        for m in range(R_f):
            gm = np.einsum("a,b,c->abc", U3[0][m], U3[1][m], U3[2][m])
            V[k, m] = vol * np.sum(gk * gm * Vc)
    return V


# --------------------------------------------------------------------------
# Canonical-to-Tucker transform (Appendix, part 1): the SVD of each side
# matrix gives a first mode basis, the side matrices are projected onto it,
# alternating sweeps replace each mode's basis by the dominant left singular
# vectors of the partially projected image, and the core is the fully
# projected tensor.  Side matrices are stored as A^l [R][n_l] (row k = the
# mode-l vector of term k), bases as Z^l [r_l][n_l] (orthonormal rows).
# --------------------------------------------------------------------------
def _sign_rows(Z: np.ndarray) -> np.ndarray:
    """Fix the sign of each basis vector: its entry of largest magnitude (the
    first such) is positive."""
    Z = Z.copy()
    for i in range(Z.shape[0]):
        if Z[i, np.argmax(np.abs(Z[i]))] < 0:
            Z[i] = -Z[i]
    return Z


def _leading_left(Mt: np.ndarray, r: int):
    """The r dominant left singular vectors of the n x m matrix Mt^T (Mt is
    [m][n]) as rows [r][n], and the singular values."""
    Zf, s, _ = np.linalg.svd(Mt.T, full_matrices=False)
    Z = np.zeros((r, Mt.shape[1]))
    k = min(r, Zf.shape[1])
    Z[:k] = Zf[:, :k].T
    return _sign_rows(Z), s


def tucker_ranks(sv3, ranks, eps: float):
    """The epsilon truncation of step (A): per mode the number of singular
    values of the side matrix at least eps times the largest (at least 1, at
    most ranks[l]), then each clamped to the product of the other two so that
    the alternating sweeps stay defined.  eps <= 0 keeps the given ranks."""
    if eps <= 0:
        return list(ranks)
    r = [max(1, min(int(ranks[l]), int(np.sum(sv3[l] >= eps * sv3[l][0])))) for l in range(3)]
    for l in range(3):
        m1, m2 = [x for x in range(3) if x != l]
        r[l] = min(r[l], r[m1] * r[m2])
    return r


def canonical_to_tucker(c, A3, ranks, m_max: int, eps: float = 0.0):
    """Returns (Z3 [r_l][n_l] each, beta [r1][r2][r3], sv3: singular values of
    the last SVD of each mode).  With eps > 0 the ranks are the epsilon
    truncation of step (A) (tucker_ranks) and the outputs keep the shapes of
    `ranks`, zero beyond the chosen ranks."""
    c = _f64(c)
    A3 = [_f64(a) for a in A3]
    # (A) dominant subspace of each side matrix; (B) projection
    Z3, sv3 = [], []
    for l in range(3):
        Z, s = _leading_left(A3[l], ranks[l])
        Z3.append(Z)
        sv3.append(s)
    rk = tucker_ranks(sv3, ranks, eps)
    for l in range(3):
        Z3[l][rk[l]:] = 0.0
    Ut = [Z3[l] @ A3[l].T for l in range(3)]            # [r_l][R]
    # (C, D) alternating sweeps over the modes
    for _ in range(m_max):
        for l in range(3):
            m1, m2 = [x for x in range(3) if x != l]
            # partially projected image, mode l in physical space:
            # M[a][(i, j)] = sum_k c_k A^l[k][a] Ut^m1[i][k] Ut^m2[j][k]
            K = (c[None, None, :] * Ut[m1][:, None, :] * Ut[m2][None, :, :]).reshape(-1, c.shape[0])
            Mt = K @ A3[l]                                # [r_m1 r_m2][n_l] = M^T
            Z3[l], sv3[l] = _leading_left(Mt, ranks[l])
            Z3[l][rk[l]:] = 0.0
            Ut[l] = Z3[l] @ A3[l].T
    # (E) core
    beta = np.einsum("k,ik,jk,mk->ijm", c, Ut[0], Ut[1], Ut[2])
    return Z3, beta, sv3


def tucker_full(Z3, beta) -> np.ndarray:
    """The full tensor of a Tucker representation (small grids only)."""
    return np.einsum("ijm,ia,jb,mc->abc", beta, Z3[0], Z3[1], Z3[2])


def canonical_full(c, A3) -> np.ndarray:
    """The full tensor of a canonical representation (small grids only)."""
    return np.einsum("k,ka,kb,kc->abc", _f64(c), A3[0], A3[1], A3[2])
