"""Brute-force spin-orbital (T) energy (FP64), for tiny domains only.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py); never used by the product.

The master formula (the paper's eq. cim_pt_energy summed over the central
index, with the standard connected/disconnected (T) numerators it cites):

  W^{abc}_{ijk} = P(i/jk)P(a/bc)[ sum_e t^{ae}_{jk}<ei||bc> - sum_m t^{bc}_{im}<ma||jk> ]
  V^{abc}_{ijk} = P(i/jk)P(a/bc)[ t^a_i <jk||bc> + f_ia t^{bc}_{jk} ]
  E(T) = 1/36 sum_{ijk} sum_{abc} W (W + V) / D

is evaluated literally over ALL ordered occupied triples (repeated indices
included) and the full spin-orbital virtual cube.  Spin orbitals are the
alpha orbitals followed by the beta orbitals; a spin-orbital quantity is the
spin-blocked input where the spins match and zero otherwise.  Here
P(i/jk) g(ijk) = g(ijk) - g(jik) - g(kji), <pq||rs> = (pr|qs) - (ps|qr).
"""
from __future__ import annotations

import numpy as np


def _spin_orbital_arrays(dom):
    oa, ob, va, vb = dom.noa, dom.nob, dom.nva, dom.nvb
    no, nv = oa + ob, va + vb
    t1 = np.zeros((no, nv))
    t1[:oa, :va] = dom.t1a
    t1[oa:, va:] = dom.t1b
    f = np.zeros((no, nv))
    f[:oa, :va] = dom.fov_a
    f[oa:, va:] = dom.fov_b
    t2 = np.zeros((no, no, nv, nv))
    t2[:oa, :oa, :va, :va] = dom.t2aa
    t2[oa:, oa:, va:, va:] = dom.t2bb
    ab = dom.t2ab                          # t^{aB}_{iJ} at [i][J][a][B]
    t2[:oa, oa:, :va, va:] = ab
    t2[:oa, oa:, va:, :va] = -ab.transpose(0, 1, 3, 2)
    t2[oa:, :oa, :va, va:] = -ab.transpose(1, 0, 2, 3)
    t2[oa:, :oa, va:, :va] = ab.transpose(1, 0, 3, 2)
    eo = np.concatenate([dom.eo_a, dom.eo_b])
    ev = np.concatenate([dom.ev_a, dom.ev_b])
    # spin-orbital DF factors over [occ | vir], zero between spins
    nq = dom.naux
    n = no + nv
    B = np.zeros((nq, n, n))
    oo = [slice(0, oa), slice(oa, no)]
    vv = [slice(no, no + va), slice(no + va, n)]
    for s, (Boo, Bov, Bvv) in enumerate(((dom.Boo_a, dom.Bov_a, dom.Bvv_a),
                                          (dom.Boo_b, dom.Bov_b, dom.Bvv_b))):
        B[:, oo[s], oo[s]] = Boo
        B[:, oo[s], vv[s]] = Bov
        B[:, vv[s], oo[s]] = Bov.transpose(0, 2, 1)
        B[:, vv[s], vv[s]] = Bvv
    return no, nv, t1, f, t2, eo, ev, B


def _chem(B, p, q, r, s):
    """(pq|rs) = sum_Q B^Q_pq B^Q_rs for index slices."""
    x = B[:, p, q]
    y = B[:, r, s]
    nq = B.shape[0]
    return (x.reshape(nq, -1).T @ y.reshape(nq, -1)).reshape(x.shape[1:] + y.shape[1:])


def energy(dom):
    """Returns {'E', 'E4', 'E_ST', 'E_DT'} by brute force over ordered triples."""
    no, nv, t1, f, t2, eo, ev, B = _spin_orbital_arrays(dom)
    O = slice(0, no)
    Vs = slice(no, no + nv)
    # <ei||bc> = (eb|ic) - (ec|ib)       as [e][i][b][c]
    eb_ic = _chem(B, Vs, Vs, O, Vs)                   # [e][b][i][c]
    vovv = eb_ic.transpose(0, 2, 1, 3) - eb_ic.transpose(0, 2, 3, 1)
    # <ma||jk> = (mj|ak) - (mk|aj)       as [m][a][j][k]
    mj_ak = _chem(B, O, O, Vs, O)                     # [m][j][a][k]
    ovoo = mj_ak.transpose(0, 2, 1, 3) - mj_ak.transpose(0, 2, 3, 1)
    # <jk||bc> = (jb|kc) - (jc|kb)       as [j][k][b][c]
    jb_kc = _chem(B, O, Vs, O, Vs)                    # [j][b][k][c]
    oovv = jb_kc.transpose(0, 2, 1, 3) - jb_kc.transpose(0, 2, 3, 1)

    def P_abc(z):
        return z - z.transpose(1, 0, 2) - z.transpose(2, 1, 0)

    def conn(i, j, k):
        x = (t2[j, k] @ vovv[:, i].reshape(nv, nv * nv)).reshape(nv, nv, nv)
        y = np.einsum("mbc,ma->abc", t2[i], ovoo[:, :, j, k])
        return x - y

    def disc(i, j, k):
        return (np.einsum("a,bc->abc", t1[i], oovv[j, k]),
                np.einsum("a,bc->abc", f[i], t2[j, k]))

    e4 = est = edt = 0.0
    dv = ev[:, None, None] + ev[None, :, None] + ev[None, None, :]
    for i in range(no):
        for j in range(no):
            for k in range(no):
                w = P_abc(conn(i, j, k) - conn(j, i, k) - conn(k, j, i))
                a1, a2 = disc(i, j, k)
                b1, b2 = disc(j, i, k)
                c1, c2 = disc(k, j, i)
                vt = P_abc(a1 - b1 - c1)
                vf = P_abc(a2 - b2 - c2)
                d = (eo[i] + eo[j] + eo[k]) - dv
                wd = w / d
                e4 += np.sum(wd * w)
                est += np.sum(wd * vt)
                edt += np.sum(wd * vf)
    e4, est, edt = e4 / 36.0, est / 36.0, edt / 36.0
    return {"E": e4 + est + edt, "E4": e4, "E_ST": est, "E_DT": edt}
