"""Derivatives of f = eta^dag D^-1 eta (the per-sample Hutchinson term of
Sec. 1) with respect to the bare mass m0 and the gauge links.

With x = D^-1 eta and y = D^-dag eta (= gamma5 D^-1 gamma5 eta by the
Hermiticity of Gamma5 D, Sec. 2), d f = -y^dag (dD) x.  D depends on m0 through
(4 + m0) 1, and on each link entry U_mu(x)_ab holomorphically through the
forward hop and anti-holomorphically through the backward hop (which uses
U_mu(x)^dag), treating the 9 complex entries as free (no group projection):

    df/dm0              = -y^dag x
    df/dU_mu(x)_ab      = A_mu(x)_ab =  1/2 phi sum_{s,s'} conj(y(x)_{s a})
                                          (1 - gamma_mu)_{s s'} x(x + mu)_{s' b}
    df/dconj(U_mu(x)_ab) = B_mu(x)_ab = 1/2 phi sum_{s,s'} conj(y(x + mu)_{s b})
                                          (1 + gamma_mu)_{s s'} x(x)_{s' a}

phi is the time-boundary factor of the hop x -> x + mu.  For a grad_output g
of f (the convention of torch complex autograd, where the gradient stored for
a complex leaf z is dL/dconj(z)):

    grad_U  = sum_k  g_k conj(A_k) + conj(g_k) B_k
    grad_m0 = sum_k  Re( g_k conj(df_k/dm0) )      (m0 is a real leaf)

g = 1 gives the gradient of Re f (d/dRe U + i d/dIm U), g = 1j that of Im f.
"""
import numpy as np

from .gamma import GAMMA, ID4
from .geometry import neighbour


def force_terms(x, y, dims, bc_t=-1):
    """A, B of shape [V, 4, 3, 3] for one pair (x, y) of [V, 12] solutions."""
    x = np.asarray(x).reshape(-1, 4, 3)
    y = np.asarray(y).reshape(-1, 4, 3)
    V = x.shape[0]
    A = np.zeros((V, 4, 3, 3), dtype=np.complex128)
    B = np.zeros((V, 4, 3, 3), dtype=np.complex128)
    for mu in range(4):
        fwd, ph = neighbour(dims, mu, +1, bc_t)
        Pm = ID4 - GAMMA[mu]
        Pp = ID4 + GAMMA[mu]
        A[:, mu] = 0.5 * ph[:, None, None] * np.einsum(
            "xsa,st,xtb->xab", np.conj(y), Pm, x[fwd])
        B[:, mu] = 0.5 * ph[:, None, None] * np.einsum(
            "xsb,st,xta->xab", np.conj(y[fwd]), Pp, x)
    return A, B


def dm0(x, y):
    """df/dm0 = -y^dag x for one sample."""
    return -np.vdot(np.ravel(y), np.ravel(x))


def grad_links(xs, ys, g, dims, bc_t=-1):
    """grad_U = sum_k g_k conj(A_k) + conj(g_k) B_k  (torch convention)."""
    tot = None
    for x, y, gk in zip(xs, ys, g):
        A, B = force_terms(x, y, dims, bc_t)
        term = gk * np.conj(A) + np.conj(gk) * B
        tot = term if tot is None else tot + term
    return tot


def grad_m0(xs, ys, g):
    """Gradient for the real leaf m0: sum_k Re(g_k conj(df_k/dm0))."""
    return float(sum(np.real(gk * np.conj(dm0(x, y))) for x, y, gk in zip(xs, ys, g)))
