"""(T) share of one central LMO with a Laplace-factorised denominator.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py); never used by the product.

Follows the paper's eq. local_pt (Sec. "Correlation energy calculation in
the LIS"): the contribution of central LMO I is one third of a sum, over the
quadrature points q of eq. laplace_transform, of products of triples
amplitudes and W in which I is one of the three occupied indices and the
other two run over j < k (or over all j, K when they have different spins),
the virtual indices over their unique ranges, with the Laplace energy
factors absorbed into the amplitudes.  The central LMO is a unit vector c
over the occupied LIS orbitals of its spin (the LIS basis contains it,
Sec. "Local natural orbitals"); the (semicanonical) orbitals carry the
orbital energies.

Written out for central spin sigma (D < 0 as everywhere in this package,
W, V of the master formula, so 1/D = -int_0^inf exp(D s) ds):

  exp(D s) factorises over the six orbitals, so with the point s_q, weight
  w_q and c~_i = c_i exp(s_q e_i / 2) the central-rotated quantities are
    W_c = sum_i c~_i W_{i..},  X_c = sum_i c~_i (W + V)_{i..}
  and
    dE_c = -(1/3) sum_q w_q sum_{items with the central slot}
                      sum_{unique virtuals} W_c X_c exp(s_q D')
  with D' the sum of the other two occupied minus the three virtual orbital
  energies.  The items, for sigma = alpha: (c, j, k) with j < k alpha; (c, j)
  with any alpha j and any beta K (mixed, central in the same-spin pair);
  (J, K, c) with J < K beta (mixed, central as the odd index); the mirror for
  sigma = beta.  The parts E4, E_ST, E_DT split X_c into W_c, V_t1 and V_f.

Reading (the paper defers the definitions to its LaplaceT reference):
the exact-denominator mode is the limit of infinitely many points of the
form above: exp(s e_i / 2) exp(s e_i' / 2) exp(s D') integrates to
-2 / (D_i + D_i') with D_i = e_i + D', so
    dE_c = (1/3) sum sum_{i,i'} c_i c_i' W_{i..} (W + V)_{i'..} 2 / (D_i + D_i')
which for c = e_i is one third of the per-item energies of the items that
contain i, and summed over an orthonormal basis of both spins' occupied
spaces is E(T).
"""
from __future__ import annotations

import numpy as np

from .blocks import _Integrals, mixed_cubes, same_spin_cubes


def _groups(dom, spin):
    """(kind, label, other indices) for every item group of the central spin:
    kind 'same' -> (j, k), j < k of the central spin; 'pair' -> (j, K), the
    central index in the same-spin pair; 'odd' -> (J, K), J < K of the other
    spin, the central index as the odd one."""
    o = (dom.noa, dom.nob)
    s, t = spin, 1 - spin
    out = []
    for j in range(o[s]):
        for k in range(j + 1, o[s]):
            out.append(("same", j, k))
    for j in range(o[s]):
        for K in range(o[t]):
            out.append(("pair", j, K))
    for J in range(o[t]):
        for K in range(J + 1, o[t]):
            out.append(("odd", J, K))
    return out


# block index of each group kind, per central spin (0 aaa, 1 aab, 2 abb, 3 bbb)
_BLOCK = {0: {"same": 0, "pair": 1, "odd": 2}, 1: {"same": 3, "pair": 2, "odd": 1}}


def _cubes(ints, dom, spin, kind, i, p, q):
    """(W, V_t1, V_f, D) with the central slot at orbital i of the central spin."""
    s, t = spin, 1 - spin
    if kind == "same":
        return same_spin_cubes(ints, s, i, p, q)            # triple (i, j, k), i first
    if kind == "pair":
        return mixed_cubes(ints, dom, s, i, p, q)           # pair (i, j) of spin s, odd K
    return mixed_cubes(ints, dom, t, p, q, i)               # pair (J, K) of spin t, odd i


def _central_factor(s, e):
    """exp(s e / 2): the central orbital's half of the exp(D s) factor."""
    return np.exp(0.5 * s * e)


def central_share(dom, spin: int, c, quad=None):
    """Share of the central LMO c (vector over the occupied orbitals of
    `spin`, 0 alpha, 1 beta).  `quad` = (s, w): Laplace points and weights;
    None = the exact-denominator limit.  Returns {'E': float, 'parts': [4][3]}
    (block x {E4, E_ST, E_DT})."""
    c = np.asarray(c, dtype=np.float64)
    o = (dom.noa, dom.nob)
    if c.shape != (o[spin],):
        raise ValueError("c must have one entry per occupied orbital of its spin")
    ints = _Integrals(dom)
    eo = (dom.eo_a, dom.eo_b)[spin]
    support = [i for i in range(o[spin]) if c[i] != 0.0]
    parts = np.zeros((4, 3))
    for kind, p, q in _groups(dom, spin):
        cubes = {i: _cubes(ints, dom, spin, kind, i, p, q) for i in support}
        wt = 1.0 / 6.0 if kind == "same" else 0.5             # unique virtual ranges
        b = _BLOCK[spin][kind]
        if quad is None:
            acc = np.zeros(3)
            for i in support:
                wi = cubes[i][0]
                for i2 in support:
                    w2, vt2, vf2, d2 = cubes[i2]
                    k2 = 2.0 / (cubes[i][3] + d2)
                    cc = c[i] * c[i2]
                    acc += cc * np.array([np.sum(wi * w2 * k2), np.sum(wi * vt2 * k2), np.sum(wi * vf2 * k2)])
            parts[b] += acc * wt / 3.0
            continue
        s_q, w_q = (np.asarray(x, dtype=np.float64) for x in quad)
        # D' = D - e_i (the same for every i of the central slot)
        i0 = support[0]
        dprime = cubes[i0][3] - eo[i0]
        for sq, wq in zip(s_q, w_q):
            ct = {i: c[i] * _central_factor(sq, eo[i]) for i in support}
            Wc = sum(ct[i] * cubes[i][0] for i in support)
            Vt = sum(ct[i] * cubes[i][1] for i in support)
            Vf = sum(ct[i] * cubes[i][2] for i in support)
            g = -wq * np.exp(sq * dprime)
            parts[b] += np.array([np.sum(Wc * Wc * g), np.sum(Wc * Vt * g), np.sum(Wc * Vf * g)]) * wt / 3.0
    return {"E": float(parts.sum()), "parts": parts}


def laplace_energy(dom, quad, items=None):
    """E(T) of the whole domain (or an item list) with 1/D replaced by the
    quadrature -sum_q w_q exp(s_q D) element by element (no rotation): the
    quantity the central shares of an orthonormal basis of both spins add up
    to.  Returns {'E', 'parts', 'items'}."""
    from .blocks import enumerate_items
    s_q, w_q = (np.asarray(x, dtype=np.float64) for x in quad)
    if items is None:
        items = enumerate_items(dom.noa, dom.nob)
    items = np.asarray(items).reshape(-1, 4)
    ints = _Integrals(dom)
    per = np.zeros((len(items), 3))
    for n, (b, p, q, r) in enumerate(items):
        if b in (0, 3):
            w, vt, vf, d = same_spin_cubes(ints, 0 if b == 0 else 1, p, q, r)
            wt = 1.0 / 6.0
        else:
            w, vt, vf, d = mixed_cubes(ints, dom, 0 if b == 1 else 1, p, q, r)
            wt = 0.5
        g = -sum(wq * np.exp(sq * d) for sq, wq in zip(s_q, w_q))
        per[n] = np.array([np.sum(w * w * g), np.sum(w * vt * g), np.sum(w * vf * g)]) * wt
    parts = np.zeros((4, 3))
    for b in range(4):
        sel = items[:, 0] == b
        if np.any(sel):
            parts[b] = per[sel].sum(axis=0)
    return {"E": float(parts.sum()), "parts": parts, "items": per}
