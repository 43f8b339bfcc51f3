"""Host checks of the algebra behind the spin-adapted closed-shell GPU path
(ltriples_energy_rhf), against the oracle's closed-shell formula
(oracle/rhf.py, the spin-adapted form over spatial orbitals).

The GPU path rests on two rewritings that are not in the paper and are
checked here in plain NumPy on small domains, independently of any kernel:

1. W^{abc}_{ijk} (the sum over the six joint permutations of (ia), (jb),
   (kc) of one connected term) equals
   F(i,j,k)[a][bc] + F(j,i,k)[b][ac] + F(k,i,j)[c][ab] with
   F(p,q,r)[x][yz] = sum_e tau^{xe}_{pq}(rz|ye) + sum_e tau^{xe}_{pr}(qy|ze)
                   - sum_m (px|mr) tau^{yz}_{qm} - sum_m (px|mq) tau^{yz}_{mr}.
2. The energy summed over the orderings of each occupied triple i <= j <= k
   is (m/3) sum over ordered (a,b,c) of Y^{abc} V^{abc} / D, with
   Y = 4W^{abc} + W^{bca} + W^{cab} - 2(W^{acb} + W^{bac} + W^{cba}) and m the
   number of distinct orderings of (i,j,k); summed over unique virtual tile
   triples with all six orderings of each (a,b,c) at weight 1/(tile
   permutations that fix the tile), every ordered (a,b,c) counts once.
"""
import itertools

import numpy as np
import pytest

import synth
from oracle import rhf

PERMS = list(itertools.permutations(range(3)))


def _ints(dom):
    no, nv, nq = dom.noa, dom.nva, dom.naux
    Bov, Boo, Bvv = dom.Bov_a, dom.Boo_a, dom.Bvv_a
    kc_be = (Bov.reshape(nq, -1).T @ Bvv.reshape(nq, -1)).reshape(no, nv, nv, nv)
    kc_mj = (Bov.reshape(nq, -1).T @ Boo.reshape(nq, -1)).reshape(no, nv, no, no)
    ia_jb = (Bov.reshape(nq, -1).T @ Bov.reshape(nq, -1)).reshape(no, nv, no, nv)
    return kc_be, kc_mj, ia_jb


def _F(dom, kc_be, kc_mj, p, q, r):
    """F(p,q,r) as [x][y][z], written from its definition term by term."""
    tau = dom.t2ab
    t1 = np.einsum("xe,zye->xyz", tau[p, q], kc_be[r])          # tau^{xe}_{pq} (rz|ye)
    t2 = np.einsum("xe,yze->xyz", tau[p, r], kc_be[q])          # tau^{xe}_{pr} (qy|ze)
    t3 = np.einsum("xm,myz->xyz", kc_mj[p][:, :, r], tau[q])    # (px|mr) tau^{yz}_{qm}
    t4 = np.einsum("xm,myz->xyz", kc_mj[p][:, :, q], tau[:, r])  # (px|mq) tau^{yz}_{mr}
    return t1 + t2 - t3 - t4


def _W_definition(dom, kc_be, kc_mj, occ):
    """W from its definition: the six joint permutations of one term."""
    tau = dom.t2ab
    out = np.zeros((dom.nva,) * 3)
    for p in PERMS:
        i, j, k = (occ[x] for x in p)
        x = np.einsum("ae,cbe->abc", tau[i, j], kc_be[k]) - np.einsum("mab,cm->abc", tau[i], kc_mj[k][:, :, j])
        out += np.einsum("".join("abc"[s] for s in p) + "->abc", x)
    return out


@pytest.mark.parametrize("shape", [(3, 6, 14), (4, 5, 11)])
def test_w_as_three_contractions(shape):
    dom = synth.make_rhf_domain(*shape, seed=17)
    kc_be, kc_mj, _ = _ints(dom)
    no = dom.noa
    for occ in itertools.product(range(no), repeat=3):
        i, j, k = occ
        w = (_F(dom, kc_be, kc_mj, i, j, k) + _F(dom, kc_be, kc_mj, j, i, k).transpose(1, 0, 2)
             + _F(dom, kc_be, kc_mj, k, i, j).transpose(1, 2, 0))
        ref = _W_definition(dom, kc_be, kc_mj, occ)
        assert np.allclose(w, ref, rtol=0, atol=1e-14 * max(1.0, np.abs(ref).max())), occ


@pytest.mark.parametrize("shape,tile", [((4, 7, 20), 3), ((3, 5, 12), 2), ((2, 6, 14), 4)])
def test_symmetric_form_over_unique_tiles_equals_the_formula(shape, tile):
    dom = synth.make_rhf_domain(*shape, seed=29, sigma_f=3e-2, sigma_t1=3e-2)
    kc_be, kc_mj, ia_jb = _ints(dom)
    no, nv = dom.noa, dom.nva
    tau, t1, f, eo, ev = dom.t2ab, dom.t1a, dom.fov_a, dom.eo_a, dom.ev_a
    nt = -(-nv // tile)
    E = np.zeros(3)
    for i in range(no):
        for j in range(i, no):
            for k in range(j, no):
                if i == k:
                    continue                      # all equal: no contribution
                m = len(set(itertools.permutations((i, j, k))))
                w = (_F(dom, kc_be, kc_mj, i, j, k) + _F(dom, kc_be, kc_mj, j, i, k).transpose(1, 0, 2)
                     + _F(dom, kc_be, kc_mj, k, i, j).transpose(1, 2, 0))
                vt = (np.einsum("a,bc->abc", t1[i], ia_jb[j, :, k, :]) + np.einsum("b,ac->abc", t1[j], ia_jb[i, :, k, :])
                      + np.einsum("c,ab->abc", t1[k], ia_jb[i, :, j, :]))
                vf = (np.einsum("a,bc->abc", f[i], tau[j, k]) + np.einsum("b,ac->abc", f[j], tau[i, k])
                      + np.einsum("c,ab->abc", f[k], tau[i, j]))
                for TA in range(nt):
                    for TB in range(TA, nt):
                        for TC in range(TB, nt):
                            T = (TA, TB, TC)
                            mult = sum(1 for p in PERMS if tuple(T[s] for s in p) == T)
                            for a in range(TA * tile, min(nv, TA * tile + tile)):
                                for b in range(TB * tile, min(nv, TB * tile + tile)):
                                    for c in range(TC * tile, min(nv, TC * tile + tile)):
                                        t = (a, b, c)
                                        pos = [tuple(t[p[s]] for s in range(3)) for p in PERMS]
                                        ww = np.array([w[x] for x in pos])    # abc, acb, bac, bca, cab, cba
                                        se, so = ww[0] + ww[3] + ww[4], ww[1] + ww[2] + ww[5]
                                        y = 3.0 * ww + np.array([se - 2 * so, so - 2 * se, so - 2 * se,
                                                                 se - 2 * so, se - 2 * so, so - 2 * se])
                                        d = eo[i] + eo[j] + eo[k] - ev[a] - ev[b] - ev[c]
                                        g = (m / 3.0) / mult / d
                                        E += g * np.array([y @ ww, y @ np.array([vt[x] for x in pos]),
                                                           y @ np.array([vf[x] for x in pos])])
    ref = rhf.energy(dom)
    want = np.array([ref["E4"], ref["E_ST"], ref["E_DT"]])
    assert np.allclose(E, want, rtol=1e-12, atol=0), (E, want)
