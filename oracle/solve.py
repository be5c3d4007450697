"""Linear solves D x = eta (Sec. 1: each sample needs one solve with D as the
system matrix).  Two plain solvers:

- `dense_solve`: LU factorisation of the dense D (scipy lu_factor/lu_solve);
  "exact" up to rounding, used on tiny lattices.
- `bicgstab`: the textbook (van der Vorst 1992) BiCGStab on a sparse D, one
  right-hand side at a time, stopped on the true relative residual.
"""
import numpy as np
import scipy.linalg as sla


def dense_solve(D, B):
    """X = D^-1 B for a dense D and B of shape [n] or [n, k]."""
    lu = sla.lu_factor(D)
    return sla.lu_solve(lu, B)


def dense_inverse(D):
    return dense_solve(D, np.eye(D.shape[0], dtype=np.complex128))


def bicgstab(A, b, tol=1e-12, max_iter=10000):
    """Textbook BiCGStab with r0_hat = r0 = b (x0 = 0); returns (x, iterations)."""
    b = np.asarray(b, dtype=np.complex128)
    x = np.zeros_like(b)
    r = b.copy()
    rhat = r.copy()
    bnorm = np.linalg.norm(b)
    if bnorm == 0:
        return x, 0
    rho = alpha = omega = 1.0 + 0j
    v = np.zeros_like(b)
    p = np.zeros_like(b)
    for it in range(1, max_iter + 1):
        rho_new = np.vdot(rhat, r)
        beta = (rho_new / rho) * (alpha / omega)
        rho = rho_new
        p = r + beta * (p - omega * v)
        v = A @ p
        alpha = rho / np.vdot(rhat, v)
        s = r - alpha * v
        t = A @ s
        omega = np.vdot(t, s) / np.vdot(t, t)
        x = x + alpha * p + omega * s
        r = s - omega * t
        if np.linalg.norm(b - A @ x) <= tol * bnorm:
            return x, it
    return x, max_iter
