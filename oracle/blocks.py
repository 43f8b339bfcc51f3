"""Spin-blocked (T) energy, one unique occupied triplet at a time (FP64).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py); never used by the product.

Follows the paper's eq. cim_pt_energy: the total (T) energy of a LIS is the
sum over the spin cases aaa, aab, abb, bbb of t*W terms, with W = t*D
(semicanonical orbitals, so the triples amplitudes are uncoupled).  The
spin-orbital working equations behind the paper's t and W are the standard
ones it cites (connected W, disconnected V with the singles term and, for an
RO reference whose Fock matrix is not block diagonal, the f_ov term; see
Sec. "Local MP2 energy in the extended domains", eq. off_diagonal_fock).
Written per spin case (all integrals real, (pq|rs) = sum_Q B^Q_pq B^Q_rs):

aaa (i<j<k, a<b<c):
  W = P(i/jk)P(a/bc)[ sum_e t^{ae}_{jk}<ei||bc> - sum_m t^{bc}_{im}<ma||jk> ]
  V = P(i/jk)P(a/bc)[ t^a_i <jk||bc> + f_ia t^{bc}_{jk} ]
aab (i<j alpha, K beta; a<b alpha, C beta):
  W = P(ij)P(ab) sum_E t^{aE}_{iK}(jb|EC) - P(ij) sum_e t^{eC}_{iK}<je||ab>
      + P(ab) sum_e t^{ae}_{ij}(be|KC) - P(ij)P(ab) sum_M t^{aC}_{iM}(bj|MK)
      - P(ij) sum_m t^{ab}_{im}(jm|CK) - P(ab) sum_m t^{bC}_{mK}<am||ij>
  V = P(ij)P(ab)[ t^a_i (jb|KC) + f_ia t^{bC}_{jK} ] + t^C_K <ij||ab> + f_KC t^{ab}_{ij}
abb: the same as aab with the roles of alpha and beta exchanged.
D = e_i + e_j + e_k - e_a - e_b - e_c;  E_case = sum W (W + V) / D over the
unique index ranges above, i.e. 1/6 (same-spin) or 1/2 (mixed) of the sum
over the full virtual cube.  Parts: E4 = W*W/D, E_ST = W*V_t1/D,
E_DT = W*V_f/D.

Items are (block, p, q, r): block 0 aaa (i,j,k), 1 aab (i,j,K),
2 abb (I,J,k), 3 bbb (I,J,K), with p<q(<r) for the same-spin indices.
"""
from __future__ import annotations

from functools import lru_cache

import numpy as np

BLOCK_NAMES = ("aaa", "aab", "abb", "bbb")


def enumerate_items(noa: int, nob: int) -> np.ndarray:
    """All unique occupied triplets, in block order then lexicographic."""
    rows = []
    rows += [(0, i, j, k) for i in range(noa) for j in range(i + 1, noa) for k in range(j + 1, noa)]
    rows += [(1, i, j, k) for i in range(noa) for j in range(i + 1, noa) for k in range(nob)]
    rows += [(2, i, j, k) for i in range(nob) for j in range(i + 1, nob) for k in range(noa)]
    rows += [(3, i, j, k) for i in range(nob) for j in range(i + 1, nob) for k in range(j + 1, nob)]
    return np.asarray(rows, dtype=np.int64).reshape(-1, 4)


class _Spin:
    """Per-spin data of one domain (index 0 = alpha, 1 = beta)."""

    def __init__(self, dom, s):
        a = "a" if s == 0 else "b"
        self.t1 = getattr(dom, "t1" + a)
        self.t2 = getattr(dom, "t2" + a + a)
        self.f = getattr(dom, "fov_" + a)
        self.eo = getattr(dom, "eo_" + a)
        self.ev = getattr(dom, "ev_" + a)
        self.Boo = getattr(dom, "Boo_" + a)
        self.Bov = getattr(dom, "Bov_" + a)
        self.Bvv = getattr(dom, "Bvv_" + a)


class _Integrals:
    """Four-index integrals built from the DF factors on demand."""

    def __init__(self, dom, cache_slabs=True):
        self.sp = (_Spin(dom, 0), _Spin(dom, 1))
        if cache_slabs:
            self.ovvv = lru_cache(maxsize=16)(self._ovvv)
            self.ovoo = lru_cache(maxsize=64)(self._ovoo)
        else:
            self.ovvv = self._ovvv
            self.ovoo = self._ovoo

    def _ovvv(self, x, y, i):
        """(i a|b c), i,a of spin x, b,c of spin y, as [a][b][c]."""
        bx = self.sp[x].Bov[:, i, :]                      # [Q][a]
        by = self.sp[y].Bvv                               # [Q][b][c]
        nq, nb, nc = by.shape
        return (bx.T @ by.reshape(nq, nb * nc)).reshape(bx.shape[1], nb, nc)

    def _ovoo(self, x, y, i):
        """(i a|m n), i,a of spin x, m,n of spin y, as [a][m][n]."""
        bx = self.sp[x].Bov[:, i, :]
        by = self.sp[y].Boo
        nq, nm, nn = by.shape
        return (bx.T @ by.reshape(nq, nm * nn)).reshape(bx.shape[1], nm, nn)

    def ovov(self, x, y, i, j):
        """(i a|j b), i,a of spin x, j,b of spin y, as [a][b]."""
        return self.sp[x].Bov[:, i, :].T @ self.sp[y].Bov[:, j, :]


def _P_a_bc(z):
    """P(a/bc) z(abc) = z(abc) - z(bac) - z(cba) over the virtual axes."""
    return z - z.transpose(1, 0, 2) - z.transpose(2, 1, 0)


def same_spin_cubes(ints, s, i, j, k):
    """W, V_t1, V_f and D of the same-spin triple (i, j, k) of spin s over the
    full virtual cube [a][b][c], for any order of i, j, k (W and V are
    antisymmetric in the occupied indices, so a repeated index gives zero)."""
    sp = ints.sp[s]
    t1, t2, f = sp.t1, sp.t2, sp.f
    nv = t1.shape[1]

    def vvvo(p):
        """<e p||b c> = (eb|pc) - (ec|pb) as [e][b][c]."""
        g = ints.ovvv(s, s, p).transpose(1, 2, 0)          # (pc|eb) -> [e][b][c]
        return g - g.transpose(0, 2, 1)

    def ooov(q, r):
        """<m a||q r> = (mq|ar) - (mr|aq) as [m][a]."""
        return ints.ovoo(s, s, r)[:, :, q].T - ints.ovoo(s, s, q)[:, :, r].T

    def conn(p, q, r):
        x = (t2[q, r] @ vvvo(p).reshape(nv, nv * nv)).reshape(nv, nv, nv)
        y = np.einsum("mbc,ma->abc", t2[p], ooov(q, r), optimize=True)
        return x - y

    def oovv(q, r):
        """<q r||b c> = (qb|rc) - (qc|rb) as [b][c]."""
        g = ints.ovov(s, s, q, r)
        return g - g.T

    def disc(p, q, r):
        vt = np.einsum("a,bc->abc", t1[p], oovv(q, r))
        vf = np.einsum("a,bc->abc", f[p], t2[q, r])
        return vt, vf

    z = conn(i, j, k) - conn(j, i, k) - conn(k, j, i)
    w = _P_a_bc(z)
    vt_i, vf_i = disc(i, j, k)
    vt_j, vf_j = disc(j, i, k)
    vt_k, vf_k = disc(k, j, i)
    vt = _P_a_bc(vt_i - vt_j - vt_k)
    vf = _P_a_bc(vf_i - vf_j - vf_k)
    ev = sp.ev
    d = (sp.eo[i] + sp.eo[j] + sp.eo[k]) - ev[:, None, None] - ev[None, :, None] - ev[None, None, :]
    return w, vt, vf, d


def _item_same_spin(ints, s, i, j, k):
    w, vt, vf, d = same_spin_cubes(ints, s, i, j, k)
    wd = w / d
    return np.array([np.sum(wd * w), np.sum(wd * vt), np.sum(wd * vf)]) / 6.0


def mixed_cubes(ints, dom, s, i, j, K):
    """W, V_t1, V_f and D of the mixed triple with the same-spin pair (i, j)
    of spin s and the odd index K of spin 1-s, over the full virtual cube
    [a][b][C], for either order of i, j (antisymmetric in them)."""
    t = 1 - s
    ss, st = ints.sp[s], ints.sp[t]

    if s == 0:
        def tm(p, q):       # t^{aC}_{pq}: p,a of spin s; q,C of spin t -> [a][C]
            return dom.t2ab[p, q]

        def tm_q(p):        # [q][a][C]
            return dom.t2ab[p]

        def tm_p(q):        # [p][a][C]
            return dom.t2ab[:, q]
    else:
        def tm(p, q):
            return dom.t2ab[q, p].T

        def tm_q(p):
            return dom.t2ab[:, p].transpose(0, 2, 1)

        def tm_p(q):
            return dom.t2ab[q].transpose(0, 2, 1)

    def PAB(x):
        return x - x.transpose(1, 0, 2)

    def asym_vvv(p):
        """<p e||a b> = (pa|eb) - (pb|ea) as [e][a][b]."""
        g = ints.ovvv(s, s, p)                             # [a][e][b]
        return g.transpose(1, 0, 2) - g.transpose(1, 2, 0)

    def amij():
        """<a m||i j> = (ai|mj) - (aj|mi) as [a][m]."""
        return ints.ovoo(s, s, i)[:, :, j] - ints.ovoo(s, s, j)[:, :, i]

    # P(ij)P(ab) sum_E t^{aE}_{iK}(jb|EC)
    def t1_(p, q):
        return np.einsum("aE,bEC->abC", tm(p, K), ints.ovvv(s, t, q), optimize=True)
    term1 = PAB(t1_(i, j) - t1_(j, i))

    # -P(ij) sum_e t^{eC}_{iK}<je||ab>
    def t2_(p, q):
        return np.einsum("eC,eab->abC", tm(p, K), asym_vvv(q), optimize=True)
    term2 = -(t2_(i, j) - t2_(j, i))

    # P(ab) sum_e t^{ae}_{ij}(be|KC);  (KC|be) = ovvv(t,s,K)[C][b][e]
    term3 = PAB(np.einsum("ae,Cbe->abC", ss.t2[i, j], ints.ovvv(t, s, K), optimize=True))

    # -P(ij)P(ab) sum_M t^{aC}_{iM}(bj|MK);  (jb|MK) = ovoo(s,t,j)[b][M][K]
    def t4_(p, q):
        return np.einsum("MaC,bM->abC", tm_q(p), ints.ovoo(s, t, q)[:, :, K], optimize=True)
    term4 = -PAB(t4_(i, j) - t4_(j, i))

    # -P(ij) sum_m t^{ab}_{im}(jm|CK);  (KC|jm) = ovoo(t,s,K)[C][j][m]
    def t5_(p, q):
        return np.einsum("mab,Cm->abC", ss.t2[p], ints.ovoo(t, s, K)[:, q, :], optimize=True)
    term5 = -(t5_(i, j) - t5_(j, i))

    # -P(ab) sum_m t^{bC}_{mK}<am||ij>
    term6 = -PAB(np.einsum("mbC,am->abC", tm_p(K), amij(), optimize=True))

    w = term1 + term2 + term3 + term4 + term5 + term6

    # V = P(ij)P(ab)[t^a_i (jb|KC) + f_ia t^{bC}_{jK}] + t^C_K <ij||ab> + f_KC t^{ab}_{ij}
    def vt_(p, q):
        return np.einsum("a,bC->abC", ss.t1[p], ints.ovov(s, t, q, K))

    def vf_(p, q):
        return np.einsum("a,bC->abC", ss.f[p], tm(q, K))
    g = ints.ovov(s, s, i, j)
    oovv = g - g.T
    vt = PAB(vt_(i, j) - vt_(j, i)) + np.einsum("C,ab->abC", st.t1[K], oovv)
    vf = PAB(vf_(i, j) - vf_(j, i)) + np.einsum("C,ab->abC", st.f[K], ss.t2[i, j])

    d = ((ss.eo[i] + ss.eo[j] + st.eo[K]) - ss.ev[:, None, None] - ss.ev[None, :, None]
         - st.ev[None, None, :])
    return w, vt, vf, d


def _item_mixed(ints, dom, s, i, j, K):
    """Mixed block with the same-spin pair of spin s and the odd index of spin 1-s."""
    w, vt, vf, d = mixed_cubes(ints, dom, s, i, j, K)
    wd = w / d
    return np.array([np.sum(wd * w), np.sum(wd * vt), np.sum(wd * vf)]) / 2.0


def item_parts(ints, dom, item):
    """[E4, E_ST, E_DT] of one item (block, p, q, r)."""
    b, p, q, r = (int(x) for x in item)
    if b == 0:
        return _item_same_spin(ints, 0, p, q, r)
    if b == 3:
        return _item_same_spin(ints, 1, p, q, r)
    if b == 1:
        return _item_mixed(ints, dom, 0, p, q, r)
    if b == 2:
        return _item_mixed(ints, dom, 1, p, q, r)
    raise ValueError(f"bad block {b}")


def energy(dom, items=None, return_items=False, cache_slabs=True):
    """E(T) of a domain (or of a subset of its items).

    Returns a dict: 'E' (float), 'parts' [4][3] (block x {E4, E_ST, E_DT}),
    and, if return_items, 'items' [n][3] in the order of `items`.
    """
    if items is None:
        items = enumerate_items(dom.noa, dom.nob)
    items = np.asarray(items).reshape(-1, 4)
    ints = _Integrals(dom, cache_slabs=cache_slabs)
    per = np.zeros((len(items), 3))
    # group by block so the slab cache sees related items together
    for n, it in enumerate(items):
        per[n] = item_parts(ints, dom, it)
    parts = np.zeros((4, 3))
    for b in range(4):
        sel = items[:, 0] == b
        if np.any(sel):
            parts[b] = per[sel].sum(axis=0)
    out = {"E": float(parts.sum()), "parts": parts}
    if return_items:
        out["items"] = per
    return out
