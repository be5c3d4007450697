"""Dirac matrices in the DeGrand-Rossi basis, mu = 1..4 = x, y, z, t.

The paper's D carries 4 spin components per site (Sec. 1) without fixing a
basis; the DeGrand-Rossi basis is the one chosen here.  gamma5 =
g1 g2 g3 g4 = diag(1, 1, -1, -1) in this basis (checked by the tests, not
assumed).  Spin-colour component index: 3*spin + colour.
"""
import numpy as np

_i = 1j
GAMMA = np.array([
    [[0, 0, 0, _i], [0, 0, _i, 0], [0, -_i, 0, 0], [-_i, 0, 0, 0]],   # gamma_x
    [[0, 0, 0, -1], [0, 0, 1, 0], [0, 1, 0, 0], [-1, 0, 0, 0]],       # gamma_y
    [[0, 0, _i, 0], [0, 0, 0, -_i], [-_i, 0, 0, 0], [0, _i, 0, 0]],   # gamma_z
    [[0, 0, 1, 0], [0, 0, 0, 1], [1, 0, 0, 0], [0, 1, 0, 0]],         # gamma_t
], dtype=np.complex128)

GAMMA5 = GAMMA[0] @ GAMMA[1] @ GAMMA[2] @ GAMMA[3]
ID4 = np.eye(4, dtype=np.complex128)


def spin_colour(spin_matrix):
    """Lift a 4x4 spin matrix to the 12x12 spin-colour space (index 3*s + c)."""
    return np.kron(np.asarray(spin_matrix, dtype=np.complex128), np.eye(3))
