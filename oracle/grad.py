"""Gradient of the spin-blocked (T) energy with respect to the amplitudes, the
density-fitting factors and, on request, the Fock quantities: the
occupied-virtual block f_ov and the semicanonical orbital energies (FP64, CPU).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py); never used by the product.

The energy is written once more, item by item, in PyTorch float64 CPU ops
(the same working equations as oracle.blocks: connected W, disconnected V
with the singles and f_ov terms, exact denominators, unique virtual ranges),
with every four-index integral formed from the DF factors inside the item,
and differentiated by reverse-mode automatic differentiation.  The energy of
this transcription is checked against oracle.blocks, and its gradient
against exact finite-difference stencils of oracle.blocks and of the
brute-force spin-orbital energy (E is a quadratic polynomial in (T1, T2) and
a quartic one in B, so a 3-point resp. 5-point central stencil is exact up
to rounding; f_ov enters only V, linearly, so E is linear in it; the
orbital energies enter only D, and E is homogeneous of degree -1 in them
and invariant under a common shift).

Convention for inputs that carry a symmetry (the projected gradient): the
returned dE/dt2aa and dE/dt2bb are antisymmetrised in (i,j) and (a,b), dE/dBoo
and dE/dBvv are symmetrised in their two orbital indices; t1, t2ab and Bov
carry no constraint.  A finite difference that moves all symmetry images of
one element together therefore sees 4x (t2, off-diagonal), 2x (Boo/Bvv,
off-diagonal) or 1x the returned element.
"""
from __future__ import annotations

import numpy as np
import torch

FIELDS = ("t1a", "t1b", "t2aa", "t2bb", "t2ab", "Boo_a", "Bov_a", "Bvv_a", "Boo_b", "Bov_b", "Bvv_b")
FOCK_FIELDS = ("fov_a", "fov_b", "eo_a", "ev_a", "eo_b", "ev_b")


def _mixed_amp(X, s):
    """t^{xY}_{pQ} with p,x of spin s and Q,Y of the other spin, as [p][Q][x][Y]."""
    t2ab = X["t2ab"]
    return t2ab if s == 0 else t2ab.permute(1, 0, 3, 2)


class _Item:
    def __init__(self, X, C):
        self.X, self.C = X, C

    def sp(self, s):
        a = "ab"[s]
        X, C = self.X, self.C
        return dict(t1=X["t1" + a], t2=X["t2" + a + a], Boo=X["Boo_" + a], Bov=X["Bov_" + a], Bvv=X["Bvv_" + a],
                    f=C["fov_" + a], eo=C["eo_" + a], ev=C["ev_" + a])

    # (p x|y z) etc. built from the DF factors: (pq|rs) = sum_Q B^Q_pq B^Q_rs
    @staticmethod
    def ov_vv(x, y, p):
        """(p a|b c), p,a of spin-data x, b,c of y: [a][b][c]"""
        return torch.einsum("Qa,Qbc->abc", x["Bov"][:, p, :], y["Bvv"])

    @staticmethod
    def ov_oo(x, y, p):
        """(p a|m n): [a][m][n]"""
        return torch.einsum("Qa,Qmn->amn", x["Bov"][:, p, :], y["Boo"])

    @staticmethod
    def ov_ov(x, y, p, q):
        """(p a|q b): [a][b]"""
        return x["Bov"][:, p, :].T @ y["Bov"][:, q, :]

    def same(self, s, i, j, k):
        S = self.sp(s)
        t1, t2, f = S["t1"], S["t2"], S["f"]
        nv = t1.shape[1]

        def anti_vvv(p):
            # <e p||b c> = (eb|pc) - (ec|pb), as [e][b][c]; (pc|eb) = ov_vv(p)[c][e][b]
            g = self.ov_vv(S, S, p).permute(1, 2, 0)
            return g - g.transpose(1, 2)

        def anti_oov(q, r):
            # <m a||q r> = (mq|ar) - (mr|aq) = (ra|mq) - (qa|mr), as [m][a]
            return self.ov_oo(S, S, r)[:, :, q].T - self.ov_oo(S, S, q)[:, :, r].T

        def connected(p, q, r):
            # sum_e t^{ae}_{qr} <ep||bc> - sum_m t^{bc}_{pm} <ma||qr>
            x = (t2[q, r] @ anti_vvv(p).reshape(nv, nv * nv)).reshape(nv, nv, nv)
            y = torch.einsum("mbc,ma->abc", t2[p], anti_oov(q, r))
            return x - y

        def oovv(q, r):
            g = self.ov_ov(S, S, q, r)          # (qb|rc)
            return g - g.T                      # <qr||bc>

        def disconnected(p, q, r):
            return (torch.einsum("a,bc->abc", t1[p], oovv(q, r)),
                    torch.einsum("a,bc->abc", f[p], t2[q, r]))

        def P_abc(z):
            return z - z.permute(1, 0, 2) - z.permute(2, 1, 0)

        w = P_abc(connected(i, j, k) - connected(j, i, k) - connected(k, j, i))
        d1, d2, d3 = disconnected(i, j, k), disconnected(j, i, k), disconnected(k, j, i)
        vt = P_abc(d1[0] - d2[0] - d3[0])
        vf = P_abc(d1[1] - d2[1] - d3[1])
        ev = S["ev"]
        d = (S["eo"][i] + S["eo"][j] + S["eo"][k]) - ev[:, None, None] - ev[None, :, None] - ev[None, None, :]
        # the full virtual cube counts every unique a<b<c six times
        return torch.sum(w * (w + vt + vf) / d) / 6.0

    def mixed(self, s, i, j, K):
        t = 1 - s
        Ss, St = self.sp(s), self.sp(t)
        tm = _mixed_amp(self.X, s)            # [p][Q][x][Y]

        def Pab(x):
            return x - x.permute(1, 0, 2)

        def anti_vvv(p):
            # <p e||a b> = (pa|eb) - (pb|ea) as [e][a][b]; ov_vv(p)[a][e][b] = (pa|eb)
            g = self.ov_vv(Ss, Ss, p)
            return g.permute(1, 0, 2) - g.permute(1, 2, 0)

        def anti_amij():
            # <a m||i j> = (ai|mj) - (aj|mi) as [a][m]
            return self.ov_oo(Ss, Ss, i)[:, :, j] - self.ov_oo(Ss, Ss, j)[:, :, i]

        ovvv_st = lambda p: self.ov_vv(Ss, St, p)     # (pb|EC)  [b][E][C]
        ovvv_ts = lambda p: self.ov_vv(St, Ss, p)     # (KC|be)  [C][b][e]
        ovoo_st = lambda p: self.ov_oo(Ss, St, p)     # (jb|MN)  [b][M][N]
        ovoo_ts = lambda p: self.ov_oo(St, Ss, p)     # (KC|mn)  [C][m][n]

        def w1(p, q):      # sum_E t^{aE}_{pK} (qb|EC)
            return torch.einsum("aE,bEC->abC", tm[p, K], ovvv_st(q))

        def w2(p, q):      # sum_e t^{eC}_{pK} <qe||ab>
            return torch.einsum("eC,eab->abC", tm[p, K], anti_vvv(q))

        def w4(p, q):      # sum_M t^{aC}_{pM} (qb|MK)
            return torch.einsum("MaC,bM->abC", tm[p], ovoo_st(q)[:, :, K])

        def w5(p, q):      # sum_m t^{ab}_{pm} (KC|qm)
            return torch.einsum("mab,Cm->abC", Ss["t2"][p], ovoo_ts(K)[:, q, :])

        w = (Pab(w1(i, j) - w1(j, i)) - (w2(i, j) - w2(j, i))
             + Pab(torch.einsum("ae,Cbe->abC", Ss["t2"][i, j], ovvv_ts(K)))
             - Pab(w4(i, j) - w4(j, i)) - (w5(i, j) - w5(j, i))
             - Pab(torch.einsum("mbC,am->abC", tm[:, K], anti_amij())))

        def vt_(p, q):     # t^a_p (qb|KC)
            return torch.einsum("a,bC->abC", Ss["t1"][p], self.ov_ov(Ss, St, q, K))

        def vf_(p, q):     # f_pa t^{bC}_{qK}
            return torch.einsum("a,bC->abC", Ss["f"][p], tm[q, K])

        g = self.ov_ov(Ss, Ss, i, j)
        vt = Pab(vt_(i, j) - vt_(j, i)) + torch.einsum("C,ab->abC", St["t1"][K], g - g.T)
        vf = Pab(vf_(i, j) - vf_(j, i)) + torch.einsum("C,ab->abC", St["f"][K], Ss["t2"][i, j])
        d = ((Ss["eo"][i] + Ss["eo"][j] + St["eo"][K]) - Ss["ev"][:, None, None] - Ss["ev"][None, :, None]
             - St["ev"][None, None, :])
        # the full (a,b) square counts every unique a<b twice
        return torch.sum(w * (w + vt + vf) / d) / 2.0

    def energy(self, item):
        b, p, q, r = (int(x) for x in item)
        if b == 0:
            return self.same(0, p, q, r)
        if b == 3:
            return self.same(1, p, q, r)
        return self.mixed(0 if b == 1 else 1, p, q, r)


def project(grads):
    """Projection onto the constrained inputs' symmetric subspaces."""
    out = dict(grads)
    for k in ("t2aa", "t2bb"):
        g = grads[k]
        out[k] = (g - g.transpose(1, 0, 2, 3) - g.transpose(0, 1, 3, 2) + g.transpose(1, 0, 3, 2)) / 4.0
    for k in ("Boo_a", "Bvv_a", "Boo_b", "Bvv_b"):
        g = grads[k]
        out[k] = (g + g.transpose(0, 2, 1)) / 2.0
    return out


def energy_and_grad(dom, items=None, gbar=1.0, threads=None, fock=False):
    """E(T) of the domain (or of an item subset) and gbar * dE/dx for every
    field in FIELDS (projected convention), as float64 numpy arrays; with
    `fock`, also for the fields of FOCK_FIELDS (no constraints)."""
    from oracle.blocks import enumerate_items
    if threads:
        torch.set_num_threads(int(threads))
    if items is None:
        items = enumerate_items(dom.noa, dom.nob)
    items = np.asarray(items).reshape(-1, 4)
    X = {k: torch.tensor(np.asarray(getattr(dom, k)), dtype=torch.float64, requires_grad=True) for k in FIELDS}
    C = {k: torch.tensor(np.asarray(getattr(dom, k)), dtype=torch.float64,
                         requires_grad=bool(fock) and k in FOCK_FIELDS)
         for k in ("fov_a", "fov_b", "eo_a", "ev_a", "eo_b", "ev_b")}
    it = _Item(X, C)
    E = 0.0
    for row in items:
        e = it.energy(row)
        (gbar * e).backward()
        E += float(e.detach())
    grads = {k: (X[k].grad.numpy().copy() if X[k].grad is not None else np.zeros(X[k].shape))
             for k in FIELDS}
    grads = project(grads)
    if fock:
        for k in FOCK_FIELDS:
            grads[k] = C[k].grad.numpy().copy() if C[k].grad is not None else np.zeros(C[k].shape)
    return E, grads


RHF_FIELDS = ("t1", "tau", "Boo", "Bov", "Bvv", "eo", "ev", "fov")


def _rhf_energy_torch(X):
    """The closed-shell formula of oracle.rhf, transcribed in torch float64
    (same steps and order): all ordered occupied triples, full virtual
    cubes."""
    import itertools
    t1, tau, f = X["t1"], X["tau"], X["fov"]
    eo, ev = X["eo"], X["ev"]
    Boo, Bov, Bvv = X["Boo"], X["Bov"], X["Bvv"]
    no, nv = t1.shape
    nq = Bov.shape[0]
    kc_be = (Bov.reshape(nq, -1).T @ Bvv.reshape(nq, -1)).reshape(no, nv, nv, nv)
    kc_mj = (Bov.reshape(nq, -1).T @ Boo.reshape(nq, -1)).reshape(no, nv, no, no)
    ia_jb = (Bov.reshape(nq, -1).T @ Bov.reshape(nq, -1)).reshape(no, nv, no, nv)

    def Xt(i, j, k):
        x = torch.einsum("ae,cbe->abc", tau[i, j], kc_be[k])
        y = torch.einsum("mab,cm->abc", tau[i], kc_mj[k][:, :, j])
        return x - y

    perms = list(itertools.permutations(range(3)))
    letters = "abc"
    dv = ev[:, None, None] + ev[None, :, None] + ev[None, None, :]
    E = 0.0
    for i in range(no):
        for j in range(no):
            for k in range(no):
                occ = (i, j, k)
                w = 0.0
                for p in perms:
                    sub = "".join(letters[x] for x in p)
                    w = w + torch.einsum(sub + "->abc", Xt(*(occ[x] for x in p)))
                vt = (torch.einsum("a,bc->abc", t1[i], ia_jb[j, :, k, :])
                      + torch.einsum("b,ac->abc", t1[j], ia_jb[i, :, k, :])
                      + torch.einsum("c,ab->abc", t1[k], ia_jb[i, :, j, :]))
                vf = (torch.einsum("a,bc->abc", f[i], tau[j, k])
                      + torch.einsum("b,ac->abc", f[j], tau[i, k])
                      + torch.einsum("c,ab->abc", f[k], tau[i, j]))
                v = w + vt + vf
                z = 4.0 * w + w.permute(1, 2, 0) + w.permute(2, 0, 1)
                d = (eo[i] + eo[j] + eo[k]) - dv
                E = E + torch.sum(z * (v - v.permute(2, 1, 0)) / d)
    return E / 3.0


def rhf_energy_and_grad(arrays, gbar=1.0, threads=None):
    """Closed-shell E(T) of spatial-orbital arrays (keys RHF_FIELDS) and
    gbar * dE/dx for each, by reverse mode over the closed-shell formula.
    Convention: dE/dtau is projected onto the symmetry tau^{ab}_{ij} =
    tau^{ba}_{ji}, dE/dBoo and dE/dBvv are symmetrised in their orbital
    indices; the others carry no constraint."""
    if threads:
        torch.set_num_threads(int(threads))
    X = {k: torch.tensor(np.asarray(arrays[k]), dtype=torch.float64, requires_grad=True) for k in RHF_FIELDS}
    E = _rhf_energy_torch(X)
    (gbar * E).backward()
    g = {k: (X[k].grad.numpy().copy() if X[k].grad is not None else np.zeros(X[k].shape)) for k in RHF_FIELDS}
    g["tau"] = 0.5 * (g["tau"] + g["tau"].transpose(1, 0, 3, 2))
    for k in ("Boo", "Bvv"):
        g[k] = 0.5 * (g[k] + g[k].transpose(0, 2, 1))
    return float(E.detach()), g
