"""Seeded synthetic workloads: grid-sampled Gaussian basis products.

The paper's molecules and basis sets are not available, so these generators
stand in for them with the same structure: separable (rank-1) functions
sampled at the cell centres of an n-cell grid per mode (Section 3.1, eq.
disc_GTO) and their pairwise products (the product side matrices of Section
3.2), with exponents spanning the ranges of common Gaussian basis sets.

This module is shared by the GPU library's tests/benchmark and by the
oracle's tests as *data*: it holds no step of the method (no kernel
vectors, convolutions, Grams or contractions), only the inputs.

Grid (cell-centred reading): box [-b, b] per mode, h = 2b/n, centres
x_a = -b + (a + 1/2) h, a = 0..n-1.
Side matrix layout: U[l] has shape [R_f][n], column j of the paper's
n x R_f matrix U^(l) stored as the contiguous row U[l][j].
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

# Sinc-rule parameters (u0, hu) per (R_N, n, b): the minimax relative fit of
# the rank-R_N projected kernel against the exact cell integrals of 1/|y|
# over a sample of lags (origin cell included), made by oracle/sinc_fit.py.
# They are input parameters of both sides; parity never depends on them.
SINC_PARAMS = {
    (20, 128, 10.0): (-9.611457, 0.731688),     # rel. error 4.2e-3
    (30, 512, 10.0): (-10.685519, 0.591411),    # rel. error 1.1e-3
    (30, 1024, 10.0): (-11.151208, 0.628423),   # rel. error 1.3e-3
    (30, 2048, 10.0): (-10.547035, 0.628740),   # rel. error 1.5e-3
    (30, 4096, 10.0): (-10.893526, 0.658542),   # rel. error 1.9e-3
    (32, 4096, 12.0): (-11.407495, 0.634190),   # rel. error 1.4e-3
}


def sinc_params(R_N: int, n: int, b: float):
    key = (R_N, n, float(b))
    if key in SINC_PARAMS:
        return SINC_PARAMS[key]
    # generic fallback: node range spans 1/(10 r_max) .. 10/r_min
    h = 2.0 * b / n
    t_lo = 0.1 / (2.0 * np.sqrt(3.0) * b)
    t_hi = 20.0 / h
    hu = (np.log(t_hi) - np.log(t_lo)) / max(R_N - 1, 1)
    return float(np.log(t_lo)), float(hu)


def grid(n: int, b: float) -> np.ndarray:
    h = 2.0 * b / n
    return -b + (np.arange(n) + 0.5) * h


@dataclass
class Workload:
    name: str
    n: tuple            # cells per mode
    b: float            # half-width of the box [-b, b]^3
    R_N: int
    R_f: int
    u0: float
    hu: float
    U: list             # 3 arrays [R_f][n_l], float64
    seed: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def h(self):
        return tuple(2.0 * self.b / nl for nl in self.n)

    def flops(self) -> float:
        """Algorithmic flops of the Toeplitz-Gram method:
        sum over modes and terms of 2 n^2 R_f (W = T U) + 2 n R_f^2 (G = U^T W)."""
        return float(sum(self.R_N * (2.0 * nl * nl * self.R_f + 2.0 * nl * self.R_f ** 2)
                         for nl in self.n))


def _log_uniform(rng, lo, hi, size=None):
    return np.exp(rng.uniform(np.log(lo), np.log(hi), size=size))


def s_gaussians(n: int, b: float, R_f: int, seed: int = 0, alpha=(0.1, 50.0),
                centre=3.0, alphas=None, centres=None):
    """R_f single s-type Gaussians exp(-alpha |x - A|^2) sampled per mode."""
    rng = np.random.default_rng(seed)
    if alphas is None:
        alphas = _log_uniform(rng, alpha[0], alpha[1], size=R_f)
    if centres is None:
        centres = rng.uniform(-centre, centre, size=(R_f, 3))
    alphas = np.asarray(alphas, dtype=np.float64)
    centres = np.asarray(centres, dtype=np.float64)
    x = grid(n, b)
    U = [np.ascontiguousarray(np.exp(-alphas[:, None] * (x[None, :] - centres[:, l, None]) ** 2))
         for l in range(3)]
    return U, {"alpha": alphas, "centre": centres}


def gaussian_products(n, b: float, R_f: int, seed: int = 0, alpha=(0.05, 500.0),
                      centre=3.0, screen=1e-8):
    """R_f products phi_mu phi_nu of primitive s or p Gaussians.

    Primitive: type s with probability 1/2, p_x / p_y / p_z with 1/6 each;
    exponent log-uniform in `alpha`; centre uniform in [-centre, centre]^3.
    Pairs whose Gaussian-product prefactor exp(-ab/(a+b)|A-B|^2) falls below
    `screen` are redrawn (standard integral screening).  Mode-l factor:
    (x-A_l)^{la_l} (x-B_l)^{lb_l} exp(-a (x-A_l)^2 - b (x-B_l)^2).
    n may be an int or a 3-tuple (cells per mode)."""
    ns = (n, n, n) if np.isscalar(n) else tuple(n)
    rng = np.random.default_rng(seed)
    params = []
    while len(params) < R_f:
        a, bb = _log_uniform(rng, alpha[0], alpha[1], size=2)
        A = rng.uniform(-centre, centre, size=3)
        B = rng.uniform(-centre, centre, size=3)
        ta, tb = rng.random(2)
        la = np.zeros(3, dtype=int)
        lb = np.zeros(3, dtype=int)
        if ta >= 0.5:
            la[min(int((ta - 0.5) * 6.0), 2)] = 1
        if tb >= 0.5:
            lb[min(int((tb - 0.5) * 6.0), 2)] = 1
        if np.exp(-a * bb / (a + bb) * np.sum((A - B) ** 2)) < screen:
            continue
        params.append((a, A, la, bb, B, lb))
    U = []
    for l in range(3):
        x = grid(ns[l], b)
        cols = np.empty((R_f, ns[l]))
        for j, (a, A, la, bb, B, lb) in enumerate(params):
            cols[j] = ((x - A[l]) ** la[l] * (x - B[l]) ** lb[l]
                       * np.exp(-a * (x - A[l]) ** 2 - bb * (x - B[l]) ** 2))
        U.append(np.ascontiguousarray(cols))
    return U, {"pairs": params}


# ---------------------------------------------------------------------------
# The benchmark configurations
# ---------------------------------------------------------------------------
def config(name: str, seed: int = 0) -> Workload:
    if name == "c1":
        n, b, R_N, R_f = 128, 10.0, 20, 8
        U, meta = s_gaussians(n, b, R_f, seed=seed)
    elif name == "c2":
        n, b, R_N, R_f = 1024, 10.0, 30, 256
        U, meta = gaussian_products(n, b, R_f, seed=seed)
    elif name == "c3":
        n, b, R_N, R_f = 4096, 12.0, 32, 1024
        U, meta = gaussian_products(n, b, R_f, seed=seed)
    elif name == "c5":
        n, b, R_N, R_f = 2048, 10.0, 30, 512
        U, meta = gaussian_products(n, b, R_f, seed=seed)
        meta["w"] = np.random.default_rng(seed + 7919).standard_normal(R_f)
    else:
        raise ValueError(f"unknown workload {name!r}")
    u0, hu = sinc_params(R_N, n, b)
    return Workload(name, (n, n, n), b, R_N, R_f, u0, hu, U, seed, meta)


def batched_instances(count: int = 64, seed: int = 0):
    """The batched workload: `count` independent instances with
    n uniform in {512, 1024, 2048, 4096}, R_f uniform in [32, 512], R_N = 30,
    b = 10, instance i seeded with seed + i."""
    out = []
    for i in range(count):
        rng = np.random.default_rng(seed + i)
        n = int(rng.choice([512, 1024, 2048, 4096]))
        R_f = int(rng.integers(32, 513))
        U, meta = gaussian_products(n, 10.0, R_f, seed=seed + 1000003 + i)
        u0, hu = sinc_params(30, n, 10.0)
        out.append(Workload(f"c4[{i}]", (n, n, n), 10.0, 30, R_f, u0, hu, U, seed + i, meta))
    return out


def small_products(n: int, R_f: int, R_N: int = 12, b: float = 8.0, seed: int = 0):
    """A small product workload for parity tests (several tiles + ragged tails)."""
    U, meta = gaussian_products(n, b, R_f, seed=seed)
    u0, hu = sinc_params(R_N, n if np.isscalar(n) else n[0], b)
    ns = (n, n, n) if np.isscalar(n) else tuple(n)
    return Workload(f"small_{ns}_{R_f}_{R_N}", ns, b, R_N, R_f, u0, hu, U, seed, meta)


def density(n, b: float, R_rho: int, seed: int = 0):
    """A density in canonical format for the Coulomb entries: R_rho terms
    d_m v^1_m x v^2_m x v^3_m whose factors are Gaussian products from the
    same generator as the functions (a rank-reduced density is again a short
    sum of separable terms), with weights d_m uniform in [0.1, 1].  Returns
    (V: three arrays [R_rho][n_l], d [R_rho])."""
    V, _ = gaussian_products(n, b, R_rho, seed=seed + 424242)
    d = np.random.default_rng(seed + 99991).uniform(0.1, 1.0, size=R_rho)
    return V, d
