"""Natural auxiliary functions (NAF) of one LIS domain (FP64, CPU).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py); never used by the product.

Follows Sec. "Natural auxiliary functions" (eq. naf_w): for each spin the
matrix W_s[X][Y] = sum over orbital pairs p <= q of J_s[X][p][q] J_s[Y][p][q]
is built from the three-index integrals J_s of the LIS orbitals (all of
them, occupied first, then virtual); the spin average W = (W_a + W_b)/2 is
diagonalised, and the eigenvectors whose eigenvalues exceed eps are kept as
the NAFs shared by both spins.  The three-index factors in the NAF basis are
B^Q_pq = sum_X U[X][Q] J[X][p][q], returned in order of decreasing
eigenvalue and sliced into the occupied-occupied, occupied-virtual and
virtual-virtual blocks of each spin.  numpy's eigh is the library primitive
of the diagonalisation.
"""
from __future__ import annotations

import numpy as np


def w_matrix(J):
    """W_s = sum_{p <= q} J[:, p, q] J[:, p, q]^T for one spin, J [nx][n][n]."""
    nx, n, _ = J.shape
    iu, ju = np.triu_indices(n)
    P = J[:, iu, ju]                      # [nx][pairs]
    return P @ P.T


def naf(Ja, Jb, eps):
    """Returns (lam, U, m, B): all eigenvalues of W in decreasing order, the
    matching eigenvectors (columns), the number kept (lam > eps) and, per
    spin, B [m][n][n] = U[:, :m]^T J."""
    W = 0.5 * (w_matrix(Ja) + w_matrix(Jb))
    lam, U = np.linalg.eigh(W)
    order = np.argsort(-lam, kind="stable")
    lam, U = lam[order], U[:, order]
    m = int(np.sum(lam > eps))
    Uk = U[:, :m]
    B = [np.einsum("xQ,xpq->Qpq", Uk, J, optimize=True) for J in (Ja, Jb)]
    return lam, U, m, B


def split(B, no):
    """(Boo, Bov, Bvv) of one spin from B [m][n][n] with the occupied first."""
    return (np.ascontiguousarray(B[:, :no, :no]), np.ascontiguousarray(B[:, :no, no:]),
            np.ascontiguousarray(B[:, no:, no:]))
