"""Python binding of the tc C ABI (include/tc.h): argument marshalling only.

Every step of the computation runs in the HIP library; PyTorch supplies the
device memory (float64 CUDA/HIP tensors) and the current stream.  Names
follow the C ABI.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib
from ._lib import ALGORITHMS, PRECISIONS, TcDensity, TcInstance, check


def _stream(device: torch.device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _prec(prec) -> int:
    if isinstance(prec, int):
        return prec
    try:
        return PRECISIONS[prec]
    except KeyError:
        raise ValueError(f"unknown precision {prec!r}; expected one of {list(PRECISIONS)}")


def _dev_f64(x: torch.Tensor, name: str) -> torch.Tensor:
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if x.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    if not x.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return x


def _ptr(x: Optional[torch.Tensor]):
    return ctypes.c_void_p(x.data_ptr()) if x is not None else ctypes.c_void_p(0)


def _workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def newton_kernel(n: int, h: float, R_N: int, u0: float, hu: float, device="cuda"):
    """Canonical Newton kernel: returns (t [R_N] numpy, c [R_N] numpy with
    c_k = a_k h^3, p [R_N][2n-1] float64 device tensor)."""
    device = torch.device(device)
    t = np.empty(R_N)
    c = np.empty(R_N)
    p = torch.empty((R_N, 2 * n - 1), dtype=torch.float64, device=device)
    pd = ctypes.POINTER(ctypes.c_double)
    check(_lib.lib().tc_newton_kernel(int(n), float(h), int(R_N), float(u0), float(hu),
                                      t.ctypes.data_as(pd), c.ctypes.data_as(pd), _ptr(p),
                                      _stream(device)), "tc_newton_kernel")
    return t, c, p


def convolve(p: torch.Tensor, U: torch.Tensor, prec="fp64",
             out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Potential factors W[k][j][a] = sum_b p[k][a-b+n-1] U[j][b]."""
    _dev_f64(p, "p")
    _dev_f64(U, "U")
    R_N, L = p.shape
    R_f, n = U.shape
    if L != 2 * n - 1:
        raise ValueError("p must have 2n-1 columns")
    W = out if out is not None else torch.empty((R_N, R_f, n), dtype=torch.float64,
                                                device=U.device)
    _dev_f64(W, "out")
    inst = TcInstance()
    inst.n[0], inst.R_f, inst.R_N = n, R_f, R_N
    ws_bytes = _lib.lib().tc_workspace_bytes(_lib.TC_OP_CONVOLVE, ctypes.byref(inst), 1,
                                             _prec(prec))
    ws = _workspace(ws_bytes, U.device) if ws_bytes else None
    check(_lib.lib().tc_convolve(n, R_f, R_N, _ptr(p), _ptr(U), _ptr(W), _prec(prec), _ptr(ws),
                                 ws_bytes, _stream(U.device)), "tc_convolve")
    return W


def coulomb(c: torch.Tensor, p3: Sequence[torch.Tensor], U3: Sequence[torch.Tensor],
            V3: Sequence[torch.Tensor], d: torch.Tensor, prec="fp64",
            out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """tc_coulomb: Jd[i] = sum_q c_q sum_m d_m prod_l <U^l[i], (T^l_q V^l)[m]>, the
    Coulomb entries of the product functions (rows of U^l) against the density
    sum_m d_m v^1_m x v^2_m x v^3_m (rows of V^l)."""
    _dev_f64(c, "c")
    _dev_f64(d, "d")
    R_f, R_rho, R_N = U3[0].shape[0], V3[0].shape[0], c.shape[0]
    dev = c.device
    Jd = out if out is not None else torch.empty(R_f, dtype=torch.float64, device=dev)
    _dev_f64(Jd, "out")
    D = TcDensity()
    D.R_f, D.R_rho, D.R_N = R_f, R_rho, R_N
    D.c, D.d, D.Jd = c.data_ptr(), d.data_ptr(), Jd.data_ptr()
    for l in range(3):
        for x, name in ((p3[l], "p"), (U3[l], "U"), (V3[l], "V")):
            _dev_f64(x, f"{name}[{l}]")
        D.n[l] = U3[l].shape[1]
        D.p[l], D.U[l], D.V[l] = p3[l].data_ptr(), U3[l].data_ptr(), V3[l].data_ptr()
    L = _lib.lib()
    ws_bytes = L.tc_coulomb_workspace_bytes(ctypes.byref(D), _prec(prec))
    if ws_bytes == ctypes.c_size_t(-1).value:
        raise ValueError("tc_coulomb: sizes out of range")
    ws = _workspace(ws_bytes, dev)
    check(L.tc_coulomb(ctypes.byref(D), _prec(prec), _ptr(ws), ws_bytes, _stream(dev)),
          "tc_coulomb")
    return Jd


def canonical_to_tucker(c: torch.Tensor, A3: Sequence[torch.Tensor], ranks: Sequence[int],
                        m_max: int = 2, its: int = 20, eps: float = 0.0):
    """tc_canonical_to_tucker: Tucker form of sum_k c_k a^1_k x a^2_k x a^3_k
    (A3[l] [R][n_l]).  Returns (Z3: [r_l][n_l] orthonormal rows, beta
    [r1][r2][r3], sv: numpy singular values of the last step of each mode,
    the ranks used: `ranks`, or with eps > 0 the epsilon truncation, rows and
    core entries beyond them zero)."""
    _dev_f64(c, "c")
    R = c.shape[0]
    dev = c.device
    n = [int(A3[l].shape[1]) for l in range(3)]
    for l in range(3):
        _dev_f64(A3[l], f"A[{l}]")
        if A3[l].shape[0] != R:
            raise ValueError(f"A[{l}] must be [R][n_{l}]")
    r = [int(x) for x in ranks]
    Z3 = [torch.empty((r[l], n[l]), dtype=torch.float64, device=dev) for l in range(3)]
    beta = torch.empty((r[0], r[1], r[2]), dtype=torch.float64, device=dev)
    sv = torch.empty(sum(r), dtype=torch.float64, device=dev)
    ni = (ctypes.c_int * 3)(*n)
    ri = (ctypes.c_int * 3)(*r)
    L = _lib.lib()
    ws_bytes = L.tc_canonical_to_tucker_workspace_bytes(ni, R, ri)
    if ws_bytes == ctypes.c_size_t(-1).value:
        raise ValueError("tc_canonical_to_tucker: sizes or ranks out of range")
    ws = _workspace(ws_bytes, dev)
    av = (ctypes.c_void_p * 3)(*[x.data_ptr() for x in A3])
    zv = (ctypes.c_void_p * 3)(*[x.data_ptr() for x in Z3])
    ro = (ctypes.c_int * 3)(0, 0, 0)
    check(L.tc_canonical_to_tucker(ni, R, _ptr(c), av, ri, int(m_max), int(its), float(eps), zv,
                                   _ptr(beta), _ptr(sv), ro, _ptr(ws), ws_bytes, _stream(dev)),
          "tc_canonical_to_tucker")
    s = sv.cpu().numpy()
    return Z3, beta, [s[:r[0]], s[r[0]:r[0] + r[1]], s[r[0] + r[1]:]], [int(x) for x in ro]


def nuclear(c: torch.Tensor, p3: Sequence[torch.Tensor], U3: Sequence[torch.Tensor],
            h: Sequence[float], Z, pos) -> torch.Tensor:
    """tc_nuclear: V[i][j] = -sum_a Z_a sum_q (c_q/(h1 h2 h3)) prod_l
    sum_x U^l[i][x] U^l[j][x] p^l_q[x - pos[a][l]], the nuclear potential
    matrix of the product functions (Z [M] charges, pos [M][3] grid cells)."""
    _dev_f64(c, "c")
    R_f, R_N = U3[0].shape[0], c.shape[0]
    dev = c.device
    Zh = np.ascontiguousarray(Z, dtype=np.float64).reshape(-1)
    ph = np.ascontiguousarray(pos, dtype=np.int32).reshape(-1, 3)
    if ph.shape[0] != Zh.shape[0]:
        raise ValueError("pos must be [M][3] with M = len(Z)")
    V = torch.empty((R_f, R_f), dtype=torch.float64, device=dev)
    P = _lib.TcNuclear()
    P.R_f, P.R_N, P.M = R_f, R_N, Zh.shape[0]
    P.c, P.V = c.data_ptr(), V.data_ptr()
    P.Z, P.pos = Zh.ctypes.data, ph.ctypes.data
    for l in range(3):
        _dev_f64(p3[l], f"p[{l}]")
        _dev_f64(U3[l], f"U[{l}]")
        P.n[l] = U3[l].shape[1]
        P.h[l] = float(h[l])
        P.p[l], P.U[l] = p3[l].data_ptr(), U3[l].data_ptr()
    L = _lib.lib()
    ws_bytes = L.tc_nuclear_workspace_bytes(ctypes.byref(P))
    if ws_bytes == ctypes.c_size_t(-1).value:
        raise ValueError("tc_nuclear: sizes, charges or cells out of range")
    ws = _workspace(ws_bytes, dev)
    check(L.tc_nuclear(ctypes.byref(P), _ptr(ws), ws_bytes, _stream(dev)), "tc_nuclear")
    return V


def density_fit(F: torch.Tensor, tol: float, R_max: Optional[int] = None):
    """tc_density_fit: F [N_pair][n] ~ V U through the pivoted Cholesky of
    F^T F.  Returns (U [R_max][n], V [N_pair][R_max], pivots numpy [R],
    R, residual trace); rows of U and columns of V beyond R are zero."""
    _dev_f64(F, "F")
    N_pair, n = F.shape
    R_max = n if R_max is None else int(R_max)
    dev = F.device
    U = torch.empty((R_max, n), dtype=torch.float64, device=dev)
    V = torch.empty((N_pair, R_max), dtype=torch.float64, device=dev)
    piv = np.zeros(R_max, dtype=np.int32)
    R = ctypes.c_int(0)
    res = ctypes.c_double(0.0)
    L = _lib.lib()
    ws_bytes = L.tc_density_fit_workspace_bytes(n, N_pair, R_max)
    if ws_bytes == ctypes.c_size_t(-1).value:
        raise ValueError("tc_density_fit: sizes out of range")
    ws = _workspace(ws_bytes, dev)
    check(L.tc_density_fit(n, N_pair, _ptr(F), float(tol), R_max, _ptr(U), _ptr(V),
                           piv.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), ctypes.byref(R),
                           ctypes.byref(res), _ptr(ws), ws_bytes, _stream(dev)),
          "tc_density_fit")
    return U, V, piv[:R.value].astype(np.int64), R.value, res.value


def tei_cholesky(c: torch.Tensor, V3: Sequence[torch.Tensor], M3: Sequence[torch.Tensor],
                 tol: float, R_max: Optional[int] = None):
    """tc_tei_cholesky: B = sum_k c_k o_l V^l M^l_k V^l^T ~ L L^T.  V3: three
    [N_pair][R] tensors, M3: three [R_N][R][R] tensors.  Returns (L [R_B][N_pair]
    (row r = column r of the factor), pivots numpy [R_B], residual trace)."""
    _dev_f64(c, "c")
    N_pair, R = V3[0].shape
    R_N = c.shape[0]
    for l in range(3):
        _dev_f64(V3[l], f"V[{l}]")
        _dev_f64(M3[l], f"M[{l}]")
        if tuple(V3[l].shape) != (N_pair, R) or tuple(M3[l].shape) != (R_N, R, R):
            raise ValueError("V and M shapes must agree across modes")
    R_max = N_pair if R_max is None else int(R_max)
    dev = c.device
    Lout = torch.empty((R_max, N_pair), dtype=torch.float64, device=dev)
    piv = np.zeros(R_max, dtype=np.int32)
    RB = ctypes.c_int(0)
    res = ctypes.c_double(0.0)
    vp3 = (ctypes.c_void_p * 3)(*[x.data_ptr() for x in V3])
    mp3 = (ctypes.c_void_p * 3)(*[x.data_ptr() for x in M3])
    L = _lib.lib()
    ws_bytes = L.tc_tei_cholesky_workspace_bytes(N_pair, R, R_N, R_max)
    if ws_bytes == ctypes.c_size_t(-1).value:
        raise ValueError("tc_tei_cholesky: sizes out of range")
    ws = _workspace(ws_bytes, dev)
    check(L.tc_tei_cholesky(N_pair, R, R_N, _ptr(c), vp3, mp3, float(tol), R_max, _ptr(Lout),
                            piv.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), ctypes.byref(RB),
                            ctypes.byref(res), _ptr(ws), ws_bytes, _stream(dev)),
          "tc_tei_cholesky")
    return Lout[:RB.value], piv[:RB.value].astype(np.int64), res.value


def lattice_sum(p3: Sequence[torch.Tensor], n0: int, L: Sequence[int]):
    """tc_lattice_sum: assembled vectors A^l [R_N][n0 L[l]] of the kernel
    summed over the lattice (p3: the kernel vectors of the three directions,
    each [R_N][2 n0 L[l] - 1])."""
    R_N = p3[0].shape[0]
    dev = p3[0].device
    A3 = []
    for l in range(3):
        _dev_f64(p3[l], f"p[{l}]")
        n = int(n0) * int(L[l])
        if tuple(p3[l].shape) != (R_N, 2 * n - 1):
            raise ValueError(f"p[{l}] must be [R_N][2 n0 L[{l}] - 1]")
        A3.append(torch.empty((R_N, n), dtype=torch.float64, device=dev))
    Li = (ctypes.c_int * 3)(*[int(x) for x in L])
    pv = (ctypes.c_void_p * 3)(*[x.data_ptr() for x in p3])
    av = (ctypes.c_void_p * 3)(*[x.data_ptr() for x in A3])
    check(_lib.lib().tc_lattice_sum(int(n0), Li, R_N, pv, av, _stream(dev)), "tc_lattice_sum")
    return A3


def lattice_energy(c: torch.Tensor, p3: Sequence[torch.Tensor], h: Sequence[float], n0: int,
                   L: Sequence[int], Z: float = 1.0) -> float:
    """tc_lattice_energy: Z^2/2 sum_{k != j} K(x_k - x_j) over the lattice."""
    _dev_f64(c, "c")
    R_N = c.shape[0]
    dev = c.device
    for l in range(3):
        _dev_f64(p3[l], f"p[{l}]")
    Li = (ctypes.c_int * 3)(*[int(x) for x in L])
    hd = (ctypes.c_double * 3)(*[float(x) for x in h])
    pv = (ctypes.c_void_p * 3)(*[x.data_ptr() for x in p3])
    E = ctypes.c_double(0.0)
    ws_bytes = 8 * (R_N + 1)
    ws = _workspace(ws_bytes, dev)
    check(_lib.lib().tc_lattice_energy(int(n0), Li, R_N, _ptr(c), hd, pv, float(Z),
                                       ctypes.byref(E), _ptr(ws), ws_bytes, _stream(dev)),
          "tc_lattice_energy")
    return E.value


def term_classes(p: torch.Tensor) -> np.ndarray:
    """tc_term_classes: per kernel term, B >= 0 (narrow, band B), -2 (smooth,
    low-rank Gram) or -1 (general), as the int8 FFT route treats it."""
    _dev_f64(p, "p")
    R_N, L = p.shape
    n = (L + 1) // 2
    cls = torch.empty(R_N, dtype=torch.int32, device=p.device)
    check(_lib.lib().tc_term_classes(n, R_N, _ptr(p), _ptr(cls), _stream(p.device)),
          "tc_term_classes")
    return cls.cpu().numpy()


def make_instance(c: torch.Tensor, p3: Sequence[torch.Tensor], U3: Sequence[torch.Tensor],
                  J: torch.Tensor, G: Optional[torch.Tensor] = None) -> TcInstance:
    _dev_f64(c, "c")
    inst = TcInstance()
    R_f = U3[0].shape[0]
    inst.R_f = R_f
    inst.R_N = c.shape[0]
    for l in range(3):
        _dev_f64(p3[l], f"p[{l}]")
        _dev_f64(U3[l], f"U[{l}]")
        if U3[l].shape[0] != R_f:
            raise ValueError("all modes must have R_f columns")
        inst.n[l] = U3[l].shape[1]
        if p3[l].shape != (inst.R_N, 2 * inst.n[l] - 1):
            raise ValueError(f"p[{l}] must be [R_N][2n-1]")
        inst.p[l] = p3[l].data_ptr()
        inst.U[l] = U3[l].data_ptr()
    _dev_f64(J, "J")
    inst.c = c.data_ptr()
    inst.J = J.data_ptr()
    inst.G_saved = G.data_ptr() if G is not None else None
    return inst


def tei_gram(c: torch.Tensor, p3, U3, prec="fp64", save_G: bool = False):
    """J = sum_k c_k G1_k o G2_k o G3_k.  Returns J, or (J, G) with
    G [3][R_N][R_f][R_f] when save_G."""
    dev = U3[0].device
    R_f = U3[0].shape[0]
    R_N = c.shape[0]
    J = torch.empty((R_f, R_f), dtype=torch.float64, device=dev)
    G = torch.empty((3, R_N, R_f, R_f), dtype=torch.float64, device=dev) if save_G else None
    inst = make_instance(c, p3, U3, J, G)
    _run_gram([inst], prec, dev)
    return (J, G) if save_G else J


def tei_gram_batched(instances, prec="fp64", save_G: bool = False):
    """instances: sequence of (c, p3, U3).  Returns the list of J (and Gs)."""
    dev = instances[0][2][0].device
    Js, Gs, arr = [], [], (TcInstance * len(instances))()
    for i, (c, p3, U3) in enumerate(instances):
        R_f = U3[0].shape[0]
        J = torch.empty((R_f, R_f), dtype=torch.float64, device=dev)
        G = (torch.empty((3, c.shape[0], R_f, R_f), dtype=torch.float64, device=dev)
             if save_G else None)
        arr[i] = make_instance(c, p3, U3, J, G)
        Js.append(J)
        Gs.append(G)
    _run_gram(arr, prec, dev)
    return (Js, Gs) if save_G else Js


def tei_gram_noalloc(instances, prec="fp64"):
    """tc_tei_gram_noalloc: as tei_gram_batched (sequence of (c, p3, U3)), with
    the library's static device scratch in place of a workspace.  The output
    J tensors are the caller's (allocated here, outside the call)."""
    dev = instances[0][2][0].device
    Js, arr = [], (TcInstance * len(instances))()
    for i, (c, p3, U3) in enumerate(instances):
        R_f = U3[0].shape[0]
        J = torch.empty((R_f, R_f), dtype=torch.float64, device=dev)
        arr[i] = make_instance(c, p3, U3, J, None)
        Js.append(J)
    check(_lib.lib().tc_tei_gram_noalloc(arr, len(instances), _prec(prec), _stream(dev)),
          "tc_tei_gram_noalloc")
    return Js


def _run_gram(insts, prec, dev):
    if isinstance(insts, list):
        arr = (TcInstance * len(insts))(*insts)
    else:
        arr = insts
    count = len(arr)
    L = _lib.lib()
    ws_bytes = L.tc_workspace_bytes(_lib.TC_OP_TEI_GRAM, arr, count, _prec(prec))
    if ws_bytes == ctypes.c_size_t(-1).value:
        raise ValueError("invalid problem sizes")
    ws = _workspace(ws_bytes, dev) if ws_bytes else None
    check(L.tc_tei_gram(arr, count, _prec(prec), _ptr(ws), ws_bytes, _stream(dev)),
          "tc_tei_gram")


def tei_gram_backward(c: torch.Tensor, p3, U3, Jbar: torch.Tensor,
                      G: Optional[torch.Tensor] = None, prec="fp64"):
    """dU^l = 2 sum_k T_k U^l D^l_k for f = <Jbar, J>.  Returns [dU1, dU2, dU3]."""
    dev = U3[0].device
    R_f = U3[0].shape[0]
    _dev_f64(Jbar, "Jbar")
    if Jbar.shape != (R_f, R_f):
        raise ValueError("Jbar must be [R_f][R_f]")
    dummyJ = torch.empty((1, 1), dtype=torch.float64, device=dev)
    inst = make_instance(c, p3, U3, dummyJ, G)
    dU = [torch.empty_like(U3[l]) for l in range(3)]
    arr = (TcInstance * 1)(inst)
    jb = (ctypes.c_void_p * 1)(Jbar.data_ptr())
    du = (ctypes.c_void_p * 3)(*[d.data_ptr() for d in dU])
    L = _lib.lib()
    ws_bytes = L.tc_workspace_bytes(_lib.TC_OP_TEI_GRAM_BACKWARD, arr, 1, _prec(prec))
    ws = _workspace(ws_bytes, dev)
    check(L.tc_tei_gram_backward(arr, 1, jb, du, _prec(prec), _ptr(ws), ws_bytes, _stream(dev)),
          "tc_tei_gram_backward")
    return dU


class TeiGram(torch.autograd.Function):
    """J = TeiGram.apply(c, p1, p2, p3, U1, U2, U3, prec): differentiable in
    U1..U3 through the hand-written adjoint (tc_tei_gram_backward)."""

    @staticmethod
    def forward(ctx, c, p1, p2, p3, U1, U2, U3, prec="fp64"):
        J, G = tei_gram(c, (p1, p2, p3), (U1, U2, U3), prec=prec, save_G=True)
        ctx.save_for_backward(c, p1, p2, p3, U1, U2, U3, G)
        ctx.prec = prec
        return J

    @staticmethod
    def backward(ctx, Jbar):
        c, p1, p2, p3, U1, U2, U3, G = ctx.saved_tensors
        dU = tei_gram_backward(c, (p1, p2, p3), (U1, U2, U3), Jbar.contiguous(), G=G,
                               prec=ctx.prec)
        return None, None, None, None, dU[0], dU[1], dU[2], None


def _algo(algo) -> int:
    if isinstance(algo, int):
        return algo
    try:
        return ALGORITHMS[algo]
    except KeyError:
        raise ValueError(f"unknown algorithm {algo!r}; expected one of {list(ALGORITHMS)}")


def tune_set(n: int, R_f: int, R_N: int, prec, algo) -> None:
    """Pin the Toeplitz algorithm ("direct", "fft" or "auto" to clear) used for
    modes of n cells with R_f functions and R_N terms at precision prec."""
    check(_lib.lib().tc_tune_set(n, R_f, R_N, _prec(prec), _algo(algo)), "tc_tune_set")


def tune_get(n: int, R_f: int, R_N: int, prec) -> str:
    a = _lib.lib().tc_tune_get(n, R_f, R_N, _prec(prec))
    return {v: k for k, v in ALGORITHMS.items()}[a]


def _batch_array(instances, save_G=False):
    """Descriptors of a batch for the tuning table, which keys a batch by its
    sizes and by whether its Grams are kept (only the presence of G matters)."""
    dev = instances[0][2][0].device
    arr = (TcInstance * len(instances))()
    dummy = torch.empty((1, 1), dtype=torch.float64, device=dev)
    for i, (c, p3, U3) in enumerate(instances):
        arr[i] = make_instance(c, p3, U3, dummy, dummy if save_G else None)
    return arr


def batch_tune_set(instances, prec, route, save_G: bool = False) -> None:
    """Pin how tc_tei_gram runs this batch (sequence of (c, p3, U3); save_G as
    for tei_gram_batched): "fork_join", "queue", "queue_t64", "queue_k2",
    "queue_t64_k2", or "auto" to clear."""
    arr = _batch_array(instances, save_G)
    check(_lib.lib().tc_batch_tune_set(arr, len(instances), _prec(prec),
                                       _lib.BATCH_ROUTES[route]), "tc_batch_tune_set")


def batch_tune_get(instances, prec, save_G: bool = False) -> str:
    arr = _batch_array(instances, save_G)
    r = _lib.lib().tc_batch_tune_get(arr, len(instances), _prec(prec))
    return {v: k for k, v in _lib.BATCH_ROUTES.items()}[r]


def autotune(c: torch.Tensor, p3, U3, prec="fp64"):
    """Time both Toeplitz algorithms on this problem's modes (tc_autotune),
    record the faster per mode shape, and return {mode: (ms_direct, ms_fft)}."""
    dev = U3[0].device
    R_f = U3[0].shape[0]
    J = torch.empty((R_f, R_f), dtype=torch.float64, device=dev)
    inst = make_instance(c, p3, U3, J, None)
    arr = (TcInstance * 1)(inst)
    L = _lib.lib()
    ws_bytes = L.tc_workspace_bytes(_lib.TC_OP_AUTOTUNE, arr, 1, _prec(prec))
    ws = _workspace(ws_bytes, dev)
    ms = np.zeros(6)
    check(L.tc_autotune(arr, 1, _prec(prec), _ptr(ws), ws_bytes, _stream(dev),
                        ms.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), "tc_autotune")
    return {l: (float(ms[2 * l]), float(ms[2 * l + 1])) for l in range(3)}


def autotune_batched(instances, prec="fp64"):
    """tc_autotune over a batch (sequence of (c, p3, U3)): every distinct mode
    shape is timed once with both algorithms and the faster is recorded.
    Returns an array [count][3][2] of (ms_direct, ms_fft) per instance and mode."""
    dev = instances[0][2][0].device
    arr = (TcInstance * len(instances))()
    Js = []
    for i, (c, p3, U3) in enumerate(instances):
        R_f = U3[0].shape[0]
        J = torch.empty((R_f, R_f), dtype=torch.float64, device=dev)
        arr[i] = make_instance(c, p3, U3, J, None)
        Js.append(J)
    L = _lib.lib()
    ws_bytes = L.tc_workspace_bytes(_lib.TC_OP_AUTOTUNE, arr, len(instances), _prec(prec))
    ws = _workspace(ws_bytes, dev)
    ms = np.zeros(6 * len(instances))
    check(L.tc_autotune(arr, len(instances), _prec(prec), _ptr(ws), ws_bytes, _stream(dev),
                        ms.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), "tc_autotune")
    return ms.reshape(len(instances), 3, 2)


def profile_enable(on: bool = True) -> None:
    """Bracket every kernel launch of the library with HIP events."""
    check(_lib.lib().tc_profile_enable(1 if on else 0), "tc_profile_enable")


def profile_read(max_kernels: int = 64) -> dict:
    """Synchronise the recorded events and return {kernel: (total_ms, launches)}
    accumulated since the previous read."""
    names = (ctypes.c_char * 64 * max_kernels)()
    ms = np.zeros(max_kernels)
    calls = np.zeros(max_kernels, dtype=np.int64)
    nk = _lib.lib().tc_profile_read(max_kernels, names, ms.ctypes.data_as(
        ctypes.POINTER(ctypes.c_double)), calls.ctypes.data_as(ctypes.POINTER(ctypes.c_long)))
    if nk < 0:
        raise RuntimeError("tc_profile_read: event query failed")
    return {names[i].value.decode(): (float(ms[i]), int(calls[i])) for i in range(min(nk, max_kernels))}


class TeiGramGraph:
    """A batch of TEI problems captured once into a HIP graph and replayed.

    instances: sequence of (c, p3, U3) device tensors (as for tei_gram_batched).
    The outputs J (one [R_f][R_f] tensor per instance) and the workspace are
    allocated once; replay() re-runs every kernel of tc_tei_gram(count) with
    one graph launch, reading the current contents of the input tensors.
    The tuning table is consulted at capture time (the captured kernels are
    fixed).  Kernel timing (profile_enable) must be off while capturing.
    """

    def __init__(self, instances, prec="fp64"):
        self.dev = instances[0][2][0].device
        self.prec = prec
        self.Js = []
        self.arr = (TcInstance * len(instances))()
        for i, (c, p3, U3) in enumerate(instances):
            R_f = U3[0].shape[0]
            J = torch.empty((R_f, R_f), dtype=torch.float64, device=self.dev)
            self.arr[i] = make_instance(c, p3, U3, J, None)
            self.Js.append(J)
        self._keep = instances  # the graph reads these buffers
        L = _lib.lib()
        self.ws_bytes = L.tc_workspace_bytes(_lib.TC_OP_TEI_GRAM, self.arr, len(instances),
                                             _prec(prec))
        if self.ws_bytes == ctypes.c_size_t(-1).value:
            raise ValueError("invalid problem sizes")
        self.ws = _workspace(self.ws_bytes, self.dev)
        side = torch.cuda.Stream(self.dev)
        side.wait_stream(torch.cuda.current_stream(self.dev))
        with torch.cuda.stream(side):
            self._launch()  # eager warm-up on the side stream
        torch.cuda.current_stream(self.dev).wait_stream(side)
        torch.cuda.synchronize(self.dev)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self._launch()

    def _launch(self):
        check(_lib.lib().tc_tei_gram(self.arr, len(self.arr), _prec(self.prec), _ptr(self.ws),
                                     self.ws_bytes, _stream(self.dev)), "tc_tei_gram")

    def replay(self):
        self.graph.replay()
        return self.Js
