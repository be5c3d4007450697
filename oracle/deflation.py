"""Deflated trace estimation with low modes of Q = Gamma5 D (Sec. 2, eq.
defl-split).  Test infrastructure: only tests/, the smoke check and the
bench's CPU leg use the oracle.

Q = Gamma5 D is Hermitian (gamma5-hermiticity of D).  V_k holds the k
eigenvectors of Q whose eigenvalues lambda_i are smallest in magnitude, and
Pi = V_k V_k^dag is the orthogonal projector of eq. defl-split.  Since
D^-1 = Q^-1 Gamma5 and Q^-1 Pi = sum_i v_i v_i^dag / lambda_i, for any
insertion B (a spin matrix on one time slice, or the identity):

  tr(B D^-1) = tr(B D^-1 Gamma5 Pi Gamma5)                      low-mode part
             + tr(B D^-1 (I - Gamma5 Pi Gamma5))                  stochastic part

for ANY V_k with orthonormal columns; the low-mode part is computed exactly
with k solves, sum_i (Gamma5 v_i)^dag B D^-1 (Gamma5 v_i) (the paper's "exact
computation involving k linear solves").  For exact eigenvectors it reduces
to sum_i v_i^dag Gamma5 B v_i / lambda_i, since then B D^-1 Gamma5 Pi Gamma5 =
B Q^-1 Pi Gamma5.
The stochastic part is sampled with deflated sources
eta' = eta - Gamma5 V_k V_k^dag Gamma5 eta, one sample being
eta^dag B D^-1 eta'.  With B = 1 and eigenvectors the low-mode part is
tr(Pi D^-1) of the paper's split; the projector acts on the source side (as
Gamma5 Pi Gamma5) so that the contraction is unchanged and the eigenvector
closed form holds for every B.
D^-1 (I - Gamma5 Pi Gamma5) = Q^-1 (I - Pi) Gamma5 has spectral norm
1 / |lambda_{k+1}|: the low modes that dominate the variance (Sec. 2, first
paragraph) are gone from the sampled part.
"""
import numpy as np

from .estimator import sample_dot, slice_mask
from .gamma import GAMMA5, spin_colour


def gamma5_full(V):
    """Gamma5 on the whole lattice (n = 12 V), as a diagonal vector."""
    return np.tile(np.diag(spin_colour(GAMMA5)).real, V)


def q_matrix(D):
    """Q = Gamma5 D for a dense D (rows scaled by the diagonal Gamma5)."""
    V = D.shape[0] // 12
    return gamma5_full(V)[:, None] * D


def low_modes(Q, k):
    """(lambda[:k], V_k): eigenpairs of the Hermitian Q with the smallest
    |lambda| (numpy's Hermitian eigensolver, then ordered by magnitude)."""
    lam, vec = np.linalg.eigh(Q)
    order = np.argsort(np.abs(lam), kind="stable")
    return lam[order[:k]], vec[:, order[:k]]


def exact_part(lam, Vk, dims, t=None, spin=None):
    """sum_i v_i^dag Gamma5 B v_i / lambda_i with B = spin (x) 1_colour on slice
    t (t = None: the whole lattice)."""
    S = np.eye(4) if spin is None else np.asarray(spin)
    tot = 0j
    for i in range(len(lam)):
        v = Vk[:, i].reshape(-1, 12)
        tot += sample_dot(v, v, dims, t, GAMMA5 @ S) / lam[i]
    return tot


def exact_part_solves(Dinv, Vk, dims, t=None, spin=None):
    """sum_i (Gamma5 v_i)^dag B D^-1 (Gamma5 v_i), B = spin on slice t: the
    low-mode part for any orthonormal V_k."""
    g5 = gamma5_full(Vk.shape[0] // 12)
    tot = 0j
    for i in range(Vk.shape[1]):
        w = g5 * Vk[:, i]
        tot += sample_dot(w.reshape(-1, 12), (Dinv @ w).reshape(-1, 12), dims, t, spin)
    return tot


def deflate_source(eta, Vk):
    """eta - Gamma5 V_k V_k^dag Gamma5 eta (eta: vector or [n, N] block)."""
    g5 = gamma5_full(Vk.shape[0] // 12)
    eta = np.asarray(eta)
    if eta.ndim == 1:
        return eta - g5 * (Vk @ (Vk.conj().T @ (g5 * eta)))
    return eta - g5[:, None] * (Vk @ (Vk.conj().T @ (g5[:, None] * eta)))


def deflated_sample(Dinv, Vk, eta, dims, t=None, spin=None):
    """One sample eta^dag B D^-1 eta' of the stochastic part (B on slice t)."""
    x = Dinv @ deflate_source(eta, Vk)
    return sample_dot(np.asarray(eta).reshape(-1, 12), x.reshape(-1, 12), dims, t, spin)


def deflated_operator(Dinv, Vk):
    """D^-1 (I - Gamma5 Pi Gamma5) as a dense matrix."""
    n = Dinv.shape[0]
    g5 = gamma5_full(n // 12)
    P = (g5[:, None] * Vk) @ (Vk.conj().T * g5[None, :])
    return Dinv @ (np.eye(n) - P)


def stochastic_trace(Dinv, Vk, dims, t=None, spin=None):
    """tr(B D^-1 (I - Gamma5 Pi Gamma5)) with B = spin on slice t (dense)."""
    A = deflated_operator(Dinv, Vk)
    B = spin_colour(np.eye(4) if spin is None else spin)
    V = Dinv.shape[0] // 12
    if t is None:
        rows = np.ones(12 * V, dtype=bool)
    else:
        rows = slice_mask(dims, t)
    tot = 0j
    for s in np.nonzero(rows.reshape(V, 12)[:, 0])[0]:
        tot += np.trace(B @ A[12 * s:12 * s + 12, 12 * s:12 * s + 12])
    return tot
