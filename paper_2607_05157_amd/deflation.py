"""Deflation of the trace estimator with low modes of Q = Gamma5 D (Sec. 2,
eq. defl-split), on top of libwdt.

Every vector operation runs in the library (block solves, the operator,
gamma5, the block products X^dag Y and Y = beta Y + X W, contractions); this
module only does the small dense algebra on k x k or m x m matrices
(Cholesky, Hermitian eigenproblems) on the host.

- low_modes: the k eigenpairs of Q with the smallest |lambda| by subspace
  iteration on Q^-1 = D^-1 Gamma5 (one batched solve of the whole block per
  step), Cholesky orthonormalisation applied twice, and Rayleigh-Ritz: first
  with Q^2 = (Q Z)^dag (Q Z) to pick the k-dimensional subspace of smallest
  |lambda| (Q is indefinite, so Ritz values of Q alone can be spurious near
  zero, mixtures of +lambda and -lambda modes), then with Q inside it.
- Deflation.deflate: eta' = eta - Gamma5 V_k V_k^dag Gamma5 eta for a batch of
  sources (two block products).
- Deflation.exact_part: the low-mode part tr(B D^-1 Gamma5 Pi Gamma5) =
  sum_i (Gamma5 v_i)^dag B D^-1 Gamma5 v_i for the insertion B = spin on
  slice t, by one batched solve of the k vectors Gamma5 v_i (exact for any
  orthonormal V_k, so modes that are not fully converged cost variance
  reduction, not bias); exact_part_eig is the closed form
  sum_i v_i^dag Gamma5 B v_i / lambda_i, equal to it for exact eigenvectors.
With these, tr(B D^-1) = exact_part + E[eta^dag B D^-1 eta'].
"""
import numpy as np

from . import wdt

GAMMA5 = np.diag([1.0, 1.0, -1.0, -1.0]).astype(np.complex128)


def _torch():
    import torch
    return torch


def _apply_q(gauge, lat, m0, x, out, n):
    """out = Gamma5 D x (FP64)."""
    wdt.apply_D(gauge, m0, x, out, n, wdt.FP64)
    wdt.gamma5(lat, out, out, n)
    return out


def _orthonormalise(lat, Z, m, tmp):
    """Z <- Z L^-dag with Z^dag Z = L L^dag, twice (Cholesky QR 2)."""
    for _ in range(2):
        G = wdt.block_dot(lat, Z, m, Z, m)
        G = 0.5 * (G + G.conj().T)
        L = np.linalg.cholesky(G)
        Linv_h = np.linalg.inv(L).conj().T
        wdt.block_combine(lat, Z, m, Linv_h, tmp, m, beta=0.0)
        Z.copy_(tmp)
    return Z


def low_modes(gauge, lat, m0, k, extra=16, max_iter=60, tol=1e-8, solve_tol=1e-11,
              prec=wdt.FP16, seed=0, log=None):
    """k eigenpairs (lambda, V_k) of Q = Gamma5 D with the smallest |lambda|.

    Block of m = k + extra vectors (m <= 64): start from seeded Rademacher
    vectors; each step solves D Z = Gamma5 X for the whole block (Z = Q^-1 X),
    orthonormalises Z, and takes the Ritz pairs of Q on span(Z).  Stops when
    the k wanted pairs have ||Q v - lambda v|| <= tol |lambda|.  Returns
    (lam[k], V device batch [V][12][k], info)."""
    torch = _torch()
    m = k + extra
    if not (1 <= k and m <= 64):
        raise ValueError("need 1 <= k and k + extra <= 64")
    X = lat.new_batch(m)
    wdt.sources(lat, wdt.source_descs([seed * 1000 + i for i in range(m)]), X)
    Z = lat.new_batch(m)
    W = lat.new_batch(m)
    tmp = lat.new_batch(m)
    _orthonormalise(lat, X, m, tmp)
    info = dict(iterations=0, solves=0, residuals=None)
    lam = None
    for it in range(1, max_iter + 1):
        wdt.gamma5(lat, X, tmp, m)
        Z.zero_()
        wdt.solve(gauge, m0, tmp, Z, m, tol=solve_tol, prec=prec, max_iter=20000, max_outer=80)
        info["solves"] += m
        _orthonormalise(lat, Z, m, tmp)
        _apply_q(gauge, lat, m0, Z, W, m)
        H = wdt.block_dot(lat, Z, m, W, m)           # Z^dag Q Z
        H = 0.5 * (H + H.conj().T)
        H2 = wdt.block_dot(lat, W, m, W, m)          # Z^dag Q^2 Z
        H2 = 0.5 * (H2 + H2.conj().T)
        _, S2 = np.linalg.eigh(H2)                   # ascending: smallest |lambda| first
        Sk = S2[:, :k]
        theta, T = np.linalg.eigh(Sk.conj().T @ H @ Sk)
        order = np.argsort(np.abs(theta), kind="stable")
        theta, T = theta[order], T[:, order]
        C = np.concatenate([Sk @ T, S2[:, k:]], axis=1)   # unitary m x m
        wdt.block_combine(lat, Z, m, C, X, m, beta=0.0)          # new block, wanted first
        wdt.block_combine(lat, W, m, C, tmp, m, beta=0.0)        # Q applied to it
        dth = np.zeros((m, m), dtype=complex)
        dth[np.arange(k), np.arange(k)] = -theta
        wdt.block_combine(lat, X, m, dth, tmp, m, beta=1.0)      # residuals of the k wanted
        res = np.sqrt(wdt.contract(lat, None, tmp, m, mode=wdt.CONTRACT_NORM2).sum(axis=1))
        lam = theta
        info["iterations"] = it
        info["residuals"] = res[:k] / np.abs(theta)
        if log:
            log(f"low modes: step {it}, max relative residual {info['residuals'].max():.3e}")
        if np.all(info["residuals"] <= tol):
            break
    Vk = lat.new_batch(k)
    wdt.block_combine(lat, X, m, np.eye(m)[:, :k], Vk, k, beta=0.0)
    del Z, W, tmp, X
    torch.cuda.empty_cache()
    return lam, Vk, info


class Deflation:
    """The projector of eq. defl-split on k low modes of Q and its two uses:
    deflating a batch of sources and the exact part of a trace."""

    def __init__(self, lat, lam, Vk):
        self.lat, self.lam, self.V = lat, np.asarray(lam), Vk
        self.k = len(self.lam)
        self.g5V = lat.new_batch(self.k)
        wdt.gamma5(lat, Vk, self.g5V, self.k)

    def deflate(self, b, n):
        """b <- b - Gamma5 V_k V_k^dag Gamma5 b, in place (n <= 64 RHS)."""
        C = wdt.block_dot(self.lat, self.g5V, self.k, b, n)      # (Gamma5 V)^dag b
        wdt.block_combine(self.lat, self.g5V, self.k, -C, b, n, beta=1.0)
        return b

    def exact_part(self, gauge, m0, t=None, spin=None, tol=1e-10, prec=wdt.FP16):
        """sum_i (Gamma5 v_i)^dag B D^-1 (Gamma5 v_i), B = spin on slice t (None:
        the whole lattice; spin None: the identity), by one batched solve."""
        y = self.lat.new_batch(self.k)
        wdt.solve(gauge, m0, self.g5V, y, self.k, tol=tol, prec=prec, max_iter=20000,
                  max_outer=80)
        per = wdt.contract(self.lat, self.g5V, y, self.k, spin=spin)   # [k, Lt]
        vals = per.sum(axis=1) if t is None else per[:, t]
        return complex(np.sum(vals))

    def exact_part_eig(self, t=None, spin=None):
        """sum_i v_i^dag Gamma5 B v_i / lambda_i (exact eigenvectors only)."""
        S = np.eye(4) if spin is None else np.asarray(spin)
        per = wdt.contract(self.lat, self.V, self.V, self.k, spin=GAMMA5 @ S)   # [k, Lt]
        vals = per.sum(axis=1) if t is None else per[:, t]
        return complex(np.sum(vals / self.lam))
