"""Closed-shell (T) energy for alpha == beta inputs (FP64).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py); never used by the product.

The paper states that its open-shell method reduces exactly to the
closed-shell one for closed-shell systems (Sec. "Summary and conclusions";
also the LNO and NAF constructions, Secs. "Local natural orbitals" and
"Natural auxiliary functions", which become spin independent).  This module
is the independent closed-shell side of that check, written in the
spin-adapted (Rendell-Lee-Komornicki type) form over spatial orbitals with
amplitudes tau^{ab}_{ij} = tau^{ba}_{ji}:

  W^{abc}_{ijk} = Perm[ sum_e tau^{ae}_{ij}(ck|be) - sum_m tau^{ab}_{im}(ck|mj) ]
  (Perm: sum over the 6 simultaneous permutations of the pairs (ia),(jb),(kc))
  V^{abc}_{ijk} = W + t^a_i(jb|kc) + t^b_j(ia|kc) + t^c_k(ia|jb)
                    + f_ia tau^{bc}_{jk} + f_jb tau^{ac}_{ik} + f_kc tau^{ab}_{ij}
  E = 1/3 sum_{ijk} sum_{abc} (4W^{abc} + W^{bca} + W^{cab})(V^{abc} - V^{cba}) / D^{abc}_{ijk}

Both sums run over all ordered indices.  The parts are split the same way
as the open-shell code: E4 from the W part of V, E_ST from the t1 terms,
E_DT from the f_ov terms.  The spatial tau is read from the mixed-spin input
block (t2ab) and all other quantities from the alpha inputs.
"""
from __future__ import annotations

import itertools

import numpy as np


def energy(dom):
    no, nv = dom.noa, dom.nva
    tau = dom.t2ab                         # [i][j][a][b]
    t1 = dom.t1a
    f = dom.fov_a
    eo, ev = dom.eo_a, dom.ev_a
    nq = dom.naux
    Bov, Boo, Bvv = dom.Bov_a, dom.Boo_a, dom.Bvv_a
    # (ck|be) = (kc|be) as [k][c][b][e];  (ck|mj) = (kc|mj) as [k][c][m][j];  (ia|jb) as [i][a][j][b]
    kc_be = (Bov.reshape(nq, -1).T @ Bvv.reshape(nq, -1)).reshape(no, nv, nv, nv)
    kc_mj = (Bov.reshape(nq, -1).T @ Boo.reshape(nq, -1)).reshape(no, nv, no, no)
    ia_jb = (Bov.reshape(nq, -1).T @ Bov.reshape(nq, -1)).reshape(no, nv, no, nv)

    def X(i, j, k):
        # sum_e tau^{ae}_{ij}(ck|be) -> [a][b][c];  sum_m tau^{ab}_{im}(ck|mj) -> [a][b][c]
        x = np.einsum("ae,cbe->abc", tau[i, j], kc_be[k], optimize=True)
        y = np.einsum("mab,cm->abc", tau[i], kc_mj[k][:, :, j], optimize=True)
        return x - y

    perms = list(itertools.permutations(range(3)))
    letters = "abc"

    def W_of(occ):
        w = np.zeros((nv, nv, nv))
        for p in perms:
            sub = "".join(letters[x] for x in p)
            w += np.einsum(sub + "->abc", X(*(occ[x] for x in p)))
        return w

    def disc(i, j, k):
        vt = (np.einsum("a,bc->abc", t1[i], ia_jb[j, :, k, :])
              + np.einsum("b,ac->abc", t1[j], ia_jb[i, :, k, :])
              + np.einsum("c,ab->abc", t1[k], ia_jb[i, :, j, :]))
        vf = (np.einsum("a,bc->abc", f[i], tau[j, k])
              + np.einsum("b,ac->abc", f[j], tau[i, k])
              + np.einsum("c,ab->abc", f[k], tau[i, j]))
        return vt, vf

    dv = ev[:, None, None] + ev[None, :, None] + ev[None, None, :]
    e4 = est = edt = 0.0
    for i in range(no):
        for j in range(no):
            for k in range(no):
                w = W_of((i, j, k))
                vt, vf = disc(i, j, k)
                z = 4.0 * w + w.transpose(1, 2, 0) + w.transpose(2, 0, 1)
                d = (eo[i] + eo[j] + eo[k]) - dv
                zd = z / d
                e4 += np.sum(zd * (w - w.transpose(2, 1, 0)))
                est += np.sum(zd * (vt - vt.transpose(2, 1, 0)))
                edt += np.sum(zd * (vf - vf.transpose(2, 1, 0)))
    e4, est, edt = e4 / 3.0, est / 3.0, edt / 3.0
    return {"E": e4 + est + edt, "E4": e4, "E_ST": est, "E_DT": edt}
