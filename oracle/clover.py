"""The clover (Sheikholeslami-Wohlert) term of the Wilson-Dirac operator, for
real ensembles generated with it.  Test infrastructure: only tests/, the
smoke check and the bench's CPU leg use the oracle.

The paper fixes no operator beyond "Wilson-Dirac"; the clover term is read
in its standard form, added to the site's own term:

    (D_sw psi)(x) = (D psi)(x) - (c_sw / 2) sum_{mu < nu} sigma_{mu nu} F_{mu nu}(x) psi(x),

sigma_{mu nu} = (i/2) [gamma_mu, gamma_nu] (spin) and F_{mu nu}(x) the
clover-leaf field strength (colour): with Q_{mu nu}(x) the sum of the four
plaquettes in the (mu, nu) plane that start and end at x, all traversed in
the same sense, F = (Q - Q^dag) / (8i).  F is used as it stands, without
removing its colour trace (for SU(3) links that trace is Im tr Q / 4, not
zero).  The sign is the one that cancels the O(a) Wilson shift at tree level
for c_sw = 1.  The fermion boundary factor of the hops is not part of the
gauge loops.
"""
import numpy as np

from .dirac import dense_D
from .gamma import GAMMA
from .geometry import neighbour, volume


def sigma(mu, nu):
    """sigma_{mu nu} = (i/2) [gamma_mu, gamma_nu] (4 x 4)."""
    return 0.5j * (GAMMA[mu] @ GAMMA[nu] - GAMMA[nu] @ GAMMA[mu])


def _dag(M):
    return np.conj(np.swapaxes(M, -1, -2))


def field_strength(U, dims):
    """F[V, mu, nu, 3, 3]: (Q_{mu nu} - Q_{mu nu}^dag) / (8i) from the four
    plaquettes around each site."""
    U = np.asarray(U, dtype=np.complex128)
    V = volume(dims)
    F = np.zeros((V, 4, 4, 3, 3), dtype=np.complex128)
    idx = np.arange(V)
    step = lambda s, mu, d: neighbour(dims, mu, d, +1)[0][s]
    for mu in range(4):
        for nu in range(4):
            if mu == nu:
                continue
            xp_mu = step(idx, mu, +1)
            xp_nu = step(idx, nu, +1)
            xm_mu = step(idx, mu, -1)
            xm_nu = step(idx, nu, -1)
            # the four leaves, each a closed loop from x back to x
            l1 = U[idx, mu] @ U[xp_mu, nu] @ _dag(U[xp_nu, mu]) @ _dag(U[idx, nu])
            l2 = (U[idx, nu] @ _dag(U[step(xp_nu, mu, -1), mu]) @ _dag(U[xm_mu, nu])
                  @ U[xm_mu, mu])
            xmm = step(xm_mu, nu, -1)
            l3 = _dag(U[xm_mu, mu]) @ _dag(U[xmm, nu]) @ U[xmm, mu] @ U[xm_nu, nu]
            l4 = _dag(U[xm_nu, nu]) @ U[xm_nu, mu] @ U[step(xm_nu, mu, +1), nu] @ _dag(U[idx, mu])
            Q = l1 + l2 + l3 + l4
            F[:, mu, nu] = (Q - _dag(Q)) / 8j
    return F


def clover_blocks(U, dims, csw):
    """[V, 12, 12]: -(csw/2) sum_{mu<nu} sigma_{mu nu} (x) F_{mu nu}(x)
    (spin-colour index 3*spin + colour)."""
    F = field_strength(U, dims)
    V = volume(dims)
    C = np.zeros((V, 12, 12), dtype=np.complex128)
    for mu in range(4):
        for nu in range(mu + 1, 4):
            C += np.einsum("st,xab->xsatb", sigma(mu, nu), F[:, mu, nu]).reshape(V, 12, 12)
    return -0.5 * csw * C


def dense_D_clover(U, m0, dims, csw, bc_t=-1):
    """The Wilson operator plus the clover term as a dense matrix."""
    D = dense_D(U, m0, dims, bc_t)
    C = clover_blocks(U, dims, csw)
    for s in range(volume(dims)):
        D[12 * s:12 * s + 12, 12 * s:12 * s + 12] += C[s]
    return D


def apply_clover(U, dims, csw, psi):
    """The clover term alone applied to psi [V, 12, N]."""
    C = clover_blocks(U, dims, csw)
    return np.einsum("xij,xjn->xin", C, np.asarray(psi))
