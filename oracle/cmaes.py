"""FP64 CMA-ES oracle (test infrastructure only).

Follows the paper's evolutionary optimisation (Sec. III-A.1, Eq. cmaes_update:
weighted recombination of the elite candidates, rank-one and rank-mu
covariance terms, adapted step size sigma) and, where the paper is silent
(step-size rule, evolution paths, h_sigma, default constants), Hansen's
tutorial "The CMA Evolution Strategy: A Tutorial" (arXiv:1604.00772).
Block-diagonal covariance for the bi-manual case follows Sec. III-B.

Random numbers: Philox4x32-10 (Salmon et al., SC'11) counter-based generator,
key = seed, counter = (group j, candidate k, generation g, 0); each 4x32-bit
output gives two Box-Muller pairs for dimensions 4j..4j+3.

Sampling square root: y = L z with L the (lower) Cholesky factor of C, which
gives y ~ N(0, C) exactly as the tutorial's y = B D z does (any A with
A A^T = C does).  The eigendecomposition C = B D^2 B^T still provides
C^(-1/2) = B D^(-1) B^T for the conjugate evolution path; each update takes it
from the covariance the candidates were drawn with.
"""
from __future__ import annotations

import math

import numpy as np

# ---------------------------------------------------------------- Philox4x32-10

_M0, _M1 = 0xD2511F53, 0xCD9E8D57
_W0, _W1 = 0x9E3779B9, 0xBB67AE85
_MASK = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """ctr: [..., 4] integers, key: (k0, k1) -> [..., 4] uint32 (vectorised)."""
    ctr = np.asarray(ctr, dtype=np.uint64)
    c0, c1, c2, c3 = (ctr[..., i].copy() for i in range(4))
    k0 = np.uint64(int(key[0]) & _MASK)
    k1 = np.uint64(int(key[1]) & _MASK)
    m0, m1, mask = np.uint64(_M0), np.uint64(_M1), np.uint64(_MASK)
    for r in range(10):
        if r > 0:
            k0 = np.uint64((int(k0) + _W0) & _MASK)
            k1 = np.uint64((int(k1) + _W1) & _MASK)
        p0 = m0 * c0
        p1 = m1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & mask
        hi1, lo1 = p1 >> np.uint64(32), p1 & mask
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return np.stack([c0, c1, c2, c3], -1).astype(np.uint32)


def normals(seed: int, gen: int, lam: int, n: int) -> np.ndarray:
    """Standard normal draws Z[lam, n] for generation `gen`."""
    groups = (n + 3) // 4
    k, j = np.meshgrid(np.arange(lam), np.arange(groups), indexing="ij")
    ctr = np.stack([j, k, np.full_like(k, gen), np.zeros_like(k)], -1)
    x = philox4x32_10(ctr, (seed & _MASK, (seed >> 32) & _MASK)).astype(np.float64)
    u = (x + 0.5) * 2.0 ** -32                       # in (0, 1)
    z = np.empty((lam, groups, 4))
    for p in range(2):
        r = np.sqrt(-2.0 * np.log(u[..., 2 * p]))
        t = 2.0 * math.pi * u[..., 2 * p + 1]
        z[..., 2 * p] = r * np.cos(t)
        z[..., 2 * p + 1] = r * np.sin(t)
    return z.reshape(lam, groups * 4)[:, :n]


# ---------------------------------------------------------------- CMA-ES

def default_constants(n: int, lam: int, c_m_scale=1.0, c_mu_scale=1.0, c1_scale=1.0) -> dict:
    mu = lam // 2
    w = math.log((lam + 1) / 2.0) - np.log(np.arange(1, mu + 1))
    w = w / w.sum()
    mu_eff = 1.0 / np.sum(w ** 2)
    c_sigma = (mu_eff + 2.0) / (n + mu_eff + 5.0)
    d_sigma = 1.0 + 2.0 * max(0.0, math.sqrt((mu_eff - 1.0) / (n + 1.0)) - 1.0) + c_sigma
    c_c = (4.0 + mu_eff / n) / (n + 4.0 + 2.0 * mu_eff / n)
    c1 = 2.0 / ((n + 1.3) ** 2 + mu_eff)
    c_mu = min(1.0 - c1, 2.0 * (mu_eff - 2.0 + 1.0 / mu_eff) / ((n + 2.0) ** 2 + mu_eff))
    c1 = c1 * c1_scale
    c_mu = min(c_mu * c_mu_scale, 1.0 - c1)
    chi_n = math.sqrt(n) * (1.0 - 1.0 / (4.0 * n) + 1.0 / (21.0 * n * n))
    return dict(mu=mu, weights=w, mu_eff=mu_eff, c_sigma=c_sigma, d_sigma=d_sigma, c_c=c_c,
                c1=c1, c_mu=c_mu, c_m=float(c_m_scale), chi_n=chi_n)


def cholesky_floored(C: np.ndarray, n_blocks: int = 1):
    """Lower Cholesky factor L of each diagonal block of C (L L^T = C), by the
    row-by-row (Cholesky-Banachiewicz) recurrences written out: for column j,
    s = C_jj - sum_{k<j} L_jk^2, L_jj = sqrt(s), L_ij = (C_ij - sum_{k<j} L_ik
    L_jk) / L_jj for i > j.  A pivot s that is not above the floor
    1e-20 * max_i C_ii (the analogue of the eigenvalue floor; rounding can
    make a numerically singular C lose definiteness) is replaced by the floor.
    Returns (L, floored)."""
    n = C.shape[0]
    nb = n // n_blocks
    dmax = float(np.max(np.diag(C)))
    floor = 1e-20 * dmax if dmax > 0.0 else 0.0
    if not floor > 0.0:
        floor = np.finfo(np.float64).tiny
    L = np.zeros((n, n))
    floored = False
    for b in range(n_blocks):
        o = b * nb
        for j in range(nb):
            s = C[o + j, o + j] - sum(L[o + j, o + k] ** 2 for k in range(j))
            if not s > floor:
                s, floored = floor, True
            L[o + j, o + j] = math.sqrt(s)
            for i in range(j + 1, nb):
                t = C[o + i, o + j] - sum(L[o + i, o + k] * L[o + j, o + k] for k in range(j))
                L[o + i, o + j] = t / L[o + j, o + j]
    return L, floored


class CMAES:
    """State (m, sigma, C, L, p_sigma, p_c, g) in the normalised space, with
    B, D the eigendecomposition of the covariance the last update whitened
    with; physical candidates are theta = offset + scale * x."""

    def __init__(self, n, lam, mean0, sigma0, offset, scale, seed, c_m_scale=1.0, c_mu_scale=1.0,
                 c1_scale=1.0, n_blocks=1):
        self.n, self.lam, self.seed = int(n), int(lam), int(seed)
        self.n_blocks = int(n_blocks)
        assert self.n % self.n_blocks == 0
        self.k = default_constants(n, lam, c_m_scale, c_mu_scale, c1_scale)
        self.m = np.array(mean0, dtype=np.float64).copy()
        self.sigma = float(sigma0)
        self.offset = np.array(offset, dtype=np.float64).copy()
        self.scale = np.array(scale, dtype=np.float64).copy()
        self.C = np.eye(n)
        self.L = np.eye(n)
        self.B = np.eye(n)
        self.D = np.ones(n)
        self.p_sigma = np.zeros(n)
        self.p_c = np.zeros(n)
        self.g = 0
        self.Z = None
        self.Y = None
        self.eig_floored = False
        self.chol_floored = False

    def set_covariance(self, C):
        """Replace C (symmetric positive definite) and its sampling factor."""
        self.C = np.array(C, dtype=np.float64).copy()
        self.L, self.chol_floored = cholesky_floored(self.C, self.n_blocks)

    # sample: z ~ N(0, I), y = L z (y ~ N(0, C)), x = m + sigma y   (tutorial eqs. 38-40)
    def sample(self):
        self.Z = normals(self.seed, self.g, self.lam, self.n)
        self.Y = self.Z @ self.L.T
        X = self.m[None, :] + self.sigma * self.Y
        theta = self.offset[None, :] + self.scale[None, :] * X
        return theta

    def block_mask(self) -> np.ndarray:
        nb = self.n // self.n_blocks
        mask = np.zeros((self.n, self.n), dtype=bool)
        for b in range(self.n_blocks):
            mask[b * nb:(b + 1) * nb, b * nb:(b + 1) * nb] = True
        return mask

    @staticmethod
    def ranking(loss) -> np.ndarray:
        """Order of candidates by (loss, index) ascending; NaN counts as +inf."""
        key = np.where(np.isnan(loss), np.inf, np.asarray(loss, dtype=np.float64))
        return np.lexsort((np.arange(len(key)), key))

    def update(self, loss):
        k, n = self.k, self.n
        self._decompose()                   # B, D of the covariance the candidates came from
        order = self.ranking(loss)
        ysel = self.Y[order[:k["mu"]]]
        w = k["weights"]
        y_w = w @ ysel
        self.m = self.m + k["c_m"] * self.sigma * y_w
        c_inv_sqrt = (self.B / self.D[None, :]) @ self.B.T
        cs = k["c_sigma"]
        self.p_sigma = (1.0 - cs) * self.p_sigma + math.sqrt(cs * (2.0 - cs) * k["mu_eff"]) * (c_inv_sqrt @ y_w)
        ps_norm = float(np.linalg.norm(self.p_sigma))
        h_sigma = 1.0 if ps_norm / math.sqrt(1.0 - (1.0 - cs) ** (2 * (self.g + 1))) < \
            (1.4 + 2.0 / (n + 1.0)) * k["chi_n"] else 0.0
        cc = k["c_c"]
        self.p_c = (1.0 - cc) * self.p_c + h_sigma * math.sqrt(cc * (2.0 - cc) * k["mu_eff"]) * y_w
        delta = (1.0 - h_sigma) * cc * (2.0 - cc)
        c1, cmu = k["c1"], k["c_mu"]
        rank_mu = (ysel * w[:, None]).T @ ysel
        C = (1.0 - c1 - cmu * w.sum()) * self.C + c1 * (np.outer(self.p_c, self.p_c) + delta * self.C) \
            + cmu * rank_mu
        self.sigma = self.sigma * math.exp((cs / k["d_sigma"]) * (ps_norm / k["chi_n"] - 1.0))
        self.g += 1
        self.h_sigma = h_sigma
        C = 0.5 * (C + C.T)
        if self.n_blocks > 1:
            C = np.where(self.block_mask(), C, 0.0)
        self.set_covariance(C)
        return order

    def _decompose(self):
        """B, D: eigendecomposition of each diagonal block of C (numpy's eigh),
        eigenvalues floored at 1e-20 times the largest."""
        nb = self.n // self.n_blocks
        B = np.zeros((self.n, self.n))
        ev = np.zeros(self.n)
        for b in range(self.n_blocks):
            s = slice(b * nb, (b + 1) * nb)
            e, V = np.linalg.eigh(self.C[s, s])
            ev[s] = e
            B[s, s] = V
        floor = 1e-20 * max(float(ev.max()), 0.0)
        self.eig_floored = bool(np.any(ev < floor))
        ev = np.maximum(ev, floor)
        self.B = B
        self.D = np.sqrt(ev)

    def physical_mean(self) -> np.ndarray:
        return self.offset + self.scale * self.m
