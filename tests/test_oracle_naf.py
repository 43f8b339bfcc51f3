"""Pins of the NAF oracle (oracle.naf) against facts that do not come from
it: orthogonal invariance of the four-index integrals when nothing is
discarded, the discarded weight equal to the discarded eigenvalues
(Eckart-Young), the trace of W in closed form, the closed-shell limit that
the paper's factor 1/2 is there for, and the rank of exactly low-rank input."""
import numpy as np
import pytest

import synth
from oracle import naf


def _pairs(J):
    n = J.shape[1]
    iu, ju = np.triu_indices(n)
    return J[:, iu, ju]


@pytest.mark.parametrize("no_a,nv_a,no_b,nv_b,nx", [(3, 5, 2, 6, 20), (4, 6, 4, 6, 30), (2, 3, 1, 4, 7)])
def test_no_truncation_reproduces_four_index_integrals(no_a, nv_a, no_b, nv_b, nx):
    Ja, Jb = synth.make_naf_input(no_a, nv_a, no_b, nv_b, nx, seed=5)
    lam, U, m, B = naf.naf(Ja, Jb, eps=-np.inf)
    assert m == nx
    assert np.allclose(U.T @ U, np.eye(nx), atol=1e-12)
    for J, Bs in zip((Ja, Jb), B):
        n = J.shape[1]
        g_ref = J.reshape(nx, n * n).T @ J.reshape(nx, n * n)     # (pq|rs)
        g = Bs.reshape(nx, n * n).T @ Bs.reshape(nx, n * n)
        assert np.max(np.abs(g - g_ref)) <= 1e-12 * np.max(np.abs(g_ref))
    # mixed-spin integrals (pq|RS) need the shared basis
    na, nb = Ja.shape[1], Jb.shape[1]
    mix_ref = Ja.reshape(nx, na * na).T @ Jb.reshape(nx, nb * nb)
    mix = B[0].reshape(nx, na * na).T @ B[1].reshape(nx, nb * nb)
    assert np.max(np.abs(mix - mix_ref)) <= 1e-12 * np.max(np.abs(mix_ref))


def test_trace_and_discarded_weight():
    """tr W = (|P_a|^2 + |P_b|^2)/2 over the pair-packed integrals, and the
    spin-averaged residual of the truncated projection equals the sum of the
    discarded eigenvalues."""
    Ja, Jb = synth.make_naf_input(4, 7, 3, 8, 40, seed=9, decay=8.0)
    lam, U, m, B = naf.naf(Ja, Jb, eps=1e-2)
    Pa, Pb = _pairs(Ja), _pairs(Jb)
    tr = 0.5 * (np.sum(Pa * Pa) + np.sum(Pb * Pb))
    assert abs(np.sum(lam) - tr) <= 1e-12 * tr
    assert 0 < m < 40
    Uk = U[:, :m]
    res = 0.0
    for P in (Pa, Pb):
        R = P - Uk @ (Uk.T @ P)
        res += 0.5 * np.sum(R * R)
    assert abs(res - np.sum(lam[m:])) <= 1e-10 * tr
    assert np.all(lam[:m] > 1e-2) and np.all(lam[m:] <= 1e-2)
    assert np.all(np.diff(lam) <= 0)


def test_closed_shell_limit():
    """Identical spins: the NAFs are those of one spin's W (the factor 1/2)."""
    Ja, _ = synth.make_naf_input(4, 6, 4, 6, 25, seed=3)
    lam, U, m, B = naf.naf(Ja, Ja.copy(), eps=1e-3)
    lam1 = np.sort(np.linalg.eigvalsh(naf.w_matrix(Ja)))[::-1]
    assert np.allclose(lam, lam1, rtol=1e-12, atol=1e-12 * lam1[0])
    assert np.array_equal(B[0], B[1])


def test_exact_low_rank_input():
    """J built from r auxiliary directions gives r nonzero eigenvalues."""
    rng = np.random.default_rng(4)
    n, nx, r = 7, 30, 11
    C = rng.normal(size=(nx, r))
    Z = rng.normal(size=(r, n, n))
    Z = Z + Z.transpose(0, 2, 1)
    J = np.einsum("xr,rpq->xpq", C, Z)
    lam, U, m, B = naf.naf(J, J.copy(), eps=1e-6)
    assert m == r
    assert np.max(np.abs(lam[r:])) <= 1e-10 * lam[0]


def test_planted_missing_diagonal_pairs_is_caught(monkeypatch):
    """Summing p < q only (dropping the diagonal pairs) breaks the trace pin."""
    Ja, Jb = synth.make_naf_input(3, 5, 3, 5, 20, seed=2)

    def bad(J):
        n = J.shape[1]
        iu, ju = np.triu_indices(n, 1)
        P = J[:, iu, ju]
        return P @ P.T
    monkeypatch.setattr(naf, "w_matrix", bad)
    lam, U, m, B = naf.naf(Ja, Jb, eps=-np.inf)
    tr = 0.5 * (np.sum(_pairs(Ja) ** 2) + np.sum(_pairs(Jb) ** 2))
    assert abs(np.sum(lam) - tr) > 1e-6 * tr
