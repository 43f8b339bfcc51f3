"""Pins of the FP64 CPU oracle against facts that do not come from the oracle.

Each pin is chosen so that a plausible mistake in the oracle (a dropped term,
a wrong sign or index, a transposed operand) fails at least one of them; the
mutation tests at the end plant such mistakes in the oracle (on the CPU) and
check that a pin catches them.
"""
import numpy as np
import pytest

import synth
from oracle import blocks, rhf, spinorb

TINY_SHAPES = [
    (3, 2, 6, 7, 24),
    (4, 2, 5, 7, 20),
    (3, 0, 4, 5, 16),
    (1, 2, 3, 3, 8),
    (2, 3, 4, 6, 12),
]


def _rel(a, b):
    return abs(a - b) / max(abs(a), abs(b), 1e-300)


def _dom(shape, seed=7, **kw):
    return synth.make_domain(*shape, seed=seed, **kw)


@pytest.mark.parametrize("shape", TINY_SHAPES)
def test_spin_orbital_brute_force_equals_blocks(shape):
    """P1: the spin-blocked loops equal the literal 1/36 spin-orbital sum."""
    dom = _dom(shape, sigma_f=3e-2, sigma_t1=3e-2)
    so = spinorb.energy(dom)
    bl = blocks.energy(dom)
    p = bl["parts"].sum(axis=0)
    assert _rel(so["E"], bl["E"]) < 1e-12
    assert _rel(so["E4"], p[0]) < 1e-12
    assert _rel(so["E_ST"], p[1]) < 1e-11
    assert _rel(so["E_DT"], p[2]) < 1e-11
    assert abs(so["E_ST"]) > 0 or dom.noa + dom.nob < 3


def test_spin_orbital_brute_force_config0():
    """P1 on the small FP64 domain of the workload set (5,4,30,31,120)."""
    dom = synth.config_domain("tiny")
    so = spinorb.energy(dom)
    bl = blocks.energy(dom)
    p = bl["parts"].sum(axis=0)
    assert _rel(so["E"], bl["E"]) < 1e-12
    for n, key in enumerate(("E4", "E_ST", "E_DT")):
        assert _rel(so[key], p[n]) < 1e-10


@pytest.mark.parametrize("no,nv,naux", [(3, 6, 20), (4, 5, 16)])
def test_closed_shell_reduction(no, nv, naux):
    """P2: alpha == beta inputs give the closed-shell (T) formula."""
    dom = synth.make_rhf_domain(no, nv, naux, seed=11, sigma_f=3e-2, sigma_t1=3e-2)
    bl = blocks.energy(dom)
    cs = rhf.energy(dom)
    so = spinorb.energy(dom)
    parts = bl["parts"]
    assert np.allclose(parts[0], parts[3], rtol=1e-12, atol=0)
    assert np.allclose(parts[1], parts[2], rtol=1e-12, atol=0)
    assert _rel(bl["E"], cs["E"]) < 1e-12
    assert _rel(so["E"], cs["E"]) < 1e-12
    tot = parts.sum(axis=0)
    for n, key in enumerate(("E4", "E_ST", "E_DT")):
        assert _rel(tot[n], cs[key]) < 1e-11


def _permute(dom, spin, occ_perm=None, vir_perm=None):
    """Relabel orbitals of one spin consistently in every input."""
    s = "a" if spin == 0 else "b"
    no = dom.noa if spin == 0 else dom.nob
    nv = dom.nva if spin == 0 else dom.nvb
    po = np.arange(no) if occ_perm is None else occ_perm
    pv = np.arange(nv) if vir_perm is None else vir_perm
    kw = {}
    kw["t1" + s] = getattr(dom, "t1" + s)[np.ix_(po, pv)]
    t2 = getattr(dom, "t2" + s + s)
    kw["t2" + s + s] = t2[np.ix_(po, po, pv, pv)]
    if spin == 0:
        kw["t2ab"] = dom.t2ab[po][:, :, pv]
    else:
        kw["t2ab"] = dom.t2ab[:, po][:, :, :, pv]
    kw["Boo_" + s] = getattr(dom, "Boo_" + s)[:, po][:, :, po]
    kw["Bov_" + s] = getattr(dom, "Bov_" + s)[:, po][:, :, pv]
    kw["Bvv_" + s] = getattr(dom, "Bvv_" + s)[:, pv][:, :, pv]
    kw["eo_" + s] = getattr(dom, "eo_" + s)[po]
    kw["ev_" + s] = getattr(dom, "ev_" + s)[pv]
    kw["fov_" + s] = getattr(dom, "fov_" + s)[np.ix_(po, pv)]
    return dom.replace(**{k: np.ascontiguousarray(v) for k, v in kw.items()})


@pytest.mark.parametrize("spin", [0, 1])
def test_relabelling_invariance(spin):
    """P3: a consistent relabelling of one spin's orbitals leaves E unchanged."""
    dom = _dom((4, 3, 6, 7, 20), sigma_f=3e-2, sigma_t1=3e-2)
    rng = np.random.default_rng(5)
    no = dom.noa if spin == 0 else dom.nob
    nv = dom.nva if spin == 0 else dom.nvb
    ref = blocks.energy(dom)
    per = _permute(dom, spin, rng.permutation(no), rng.permutation(nv))
    got = blocks.energy(per)
    assert _rel(ref["E"], got["E"]) < 1e-12
    assert np.allclose(ref["parts"], got["parts"], rtol=1e-10, atol=1e-14 * abs(ref["E"]))


def _phase(dom, spin, kind, p):
    """Flip the sign of orbital p (occupied or virtual) of one spin in all inputs."""
    s = "a" if spin == 0 else "b"
    d = {k: v.copy() for k, v in dom.arrays().items()}
    if kind == "occ":
        d["t1" + s][p] *= -1
        d["t2" + s + s][p] *= -1
        d["t2" + s + s][:, p] *= -1
        if spin == 0:
            d["t2ab"][p] *= -1
        else:
            d["t2ab"][:, p] *= -1
        d["Boo_" + s][:, p] *= -1
        d["Boo_" + s][:, :, p] *= -1
        d["Bov_" + s][:, p] *= -1
        d["fov_" + s][p] *= -1
    else:
        d["t1" + s][:, p] *= -1
        d["t2" + s + s][:, :, p] *= -1
        d["t2" + s + s][:, :, :, p] *= -1
        if spin == 0:
            d["t2ab"][:, :, p] *= -1
        else:
            d["t2ab"][:, :, :, p] *= -1
        d["Bov_" + s][:, :, p] *= -1
        d["Bvv_" + s][:, p] *= -1
        d["Bvv_" + s][:, :, p] *= -1
        d["fov_" + s][:, p] *= -1
    return dom.replace(**d)


@pytest.mark.parametrize("spin,kind,p", [(0, "occ", 1), (1, "occ", 0), (0, "vir", 2), (1, "vir", 4)])
def test_phase_invariance(spin, kind, p):
    """P4: flipping an orbital's sign everywhere leaves E unchanged."""
    dom = _dom((4, 3, 6, 7, 20), sigma_f=3e-2, sigma_t1=3e-2)
    ref = blocks.energy(dom)
    got = blocks.energy(_phase(dom, spin, kind, p))
    assert _rel(ref["E"], got["E"]) < 1e-12
    assert np.allclose(ref["parts"], got["parts"], rtol=1e-10, atol=1e-14 * abs(ref["E"]))


def test_spin_flip():
    """P5: exchanging alpha and beta data keeps E and swaps the block parts."""
    dom = _dom((4, 3, 6, 8, 20), sigma_f=3e-2, sigma_t1=3e-2)
    ref = blocks.energy(dom)
    got = blocks.energy(synth.flip_spin(dom))
    assert _rel(ref["E"], got["E"]) < 1e-12
    assert np.allclose(ref["parts"], got["parts"][::-1], rtol=1e-10, atol=0)


def test_homogeneity_exact():
    """P6: E(2T1, 2T2) = 4E bitwise; E4, E_ST ~ mu^4 and E_DT ~ mu^2 under B -> mu B."""
    dom = _dom((4, 3, 6, 7, 20), sigma_f=3e-2, sigma_t1=3e-2)
    ref = blocks.energy(dom)
    t2 = blocks.energy(dom.scaled(lam_t=2.0))
    assert np.array_equal(t2["parts"], 4.0 * ref["parts"])
    b2 = blocks.energy(dom.scaled(mu_b=2.0))
    assert np.array_equal(b2["parts"][:, 0], 16.0 * ref["parts"][:, 0])
    assert np.array_equal(b2["parts"][:, 1], 16.0 * ref["parts"][:, 1])
    assert np.array_equal(b2["parts"][:, 2], 4.0 * ref["parts"][:, 2])


def test_special_cases():
    """P7: T2 = 0, T1 = 0, f_ov = 0, sign of E4, odd parts."""
    dom = _dom((4, 3, 6, 7, 20), sigma_f=3e-2, sigma_t1=3e-2)
    ref = blocks.energy(dom)
    z2 = blocks.energy(dom.replace(t2aa=0 * dom.t2aa, t2bb=0 * dom.t2bb, t2ab=0 * dom.t2ab))
    assert z2["E"] == 0.0
    z1 = blocks.energy(dom.replace(t1a=0 * dom.t1a, t1b=0 * dom.t1b))
    assert np.all(z1["parts"][:, 1] == 0.0)
    assert np.allclose(z1["parts"][:, [0, 2]], ref["parts"][:, [0, 2]], rtol=1e-13, atol=0)
    zf = blocks.energy(dom.scaled(nu_f=0.0))
    assert np.all(zf["parts"][:, 2] == 0.0)
    assert np.all(ref["parts"][:, 0] <= 0.0)
    neg1 = blocks.energy(dom.replace(t1a=-dom.t1a, t1b=-dom.t1b))
    assert np.allclose(neg1["parts"][:, 1], -ref["parts"][:, 1], rtol=1e-12, atol=0)
    negf = blocks.energy(dom.scaled(nu_f=-1.0))
    assert np.allclose(negf["parts"][:, 2], -ref["parts"][:, 2], rtol=1e-12, atol=0)


def test_edge_shapes():
    """P8: nob = 0 leaves only aaa; fewer than 3 occupied gives E = 0; nv = 0 gives 0."""
    dom = _dom((4, 0, 5, 6, 16))
    r = blocks.energy(dom)
    assert np.all(r["parts"][1:] == 0.0) and r["parts"][0, 0] < 0
    so = spinorb.energy(dom)
    assert _rel(so["E"], r["E"]) < 1e-12
    assert blocks.energy(_dom((1, 1, 4, 4, 8)))["E"] == 0.0
    assert blocks.energy(_dom((2, 0, 4, 4, 8)))["E"] == 0.0
    assert blocks.energy(_dom((3, 2, 0, 2, 8)))["parts"][:3].sum() == 0.0


def test_item_additivity():
    """P10: E over disjoint item lists adds up."""
    dom = _dom((4, 3, 6, 7, 20), sigma_f=3e-2, sigma_t1=3e-2)
    items = blocks.enumerate_items(dom.noa, dom.nob)
    rng = np.random.default_rng(3)
    mask = rng.random(len(items)) < 0.5
    e1 = blocks.energy(dom, items[mask])["E"]
    e2 = blocks.energy(dom, items[~mask])["E"]
    assert _rel(e1 + e2, blocks.energy(dom)["E"]) < 1e-13


# ----- planted mistakes: each must be caught by a pin above ---------------------

def _p1_gap(dom):
    so = spinorb.energy(dom)
    bl = blocks.energy(dom)
    return max(_rel(so["E"], bl["E"]), _rel(so["E_ST"], bl["parts"][:, 1].sum()),
               _rel(so["E_DT"], bl["parts"][:, 2].sum()))


def test_planted_mistake_dropped_permutation(monkeypatch):
    dom = _dom((3, 2, 6, 7, 24), sigma_f=3e-2, sigma_t1=3e-2)
    monkeypatch.setattr(blocks, "_P_a_bc", lambda z: z - z.transpose(1, 0, 2))
    assert _p1_gap(dom) > 1e-6


def test_planted_mistake_sign_of_mixed_slab(monkeypatch):
    dom = _dom((3, 2, 6, 7, 24), sigma_f=3e-2, sigma_t1=3e-2)
    orig = blocks._Integrals._ovvv

    def bad(self, x, y, i):
        g = orig(self, x, y, i)
        return -g if (x, y) == (0, 1) else g
    monkeypatch.setattr(blocks._Integrals, "_ovvv", bad)
    assert _p1_gap(dom) > 1e-6


def test_planted_mistake_disconnected_transpose(monkeypatch):
    dom = _dom((3, 2, 6, 7, 24), sigma_f=3e-2, sigma_t1=3e-2)
    orig = blocks._Integrals.ovov

    def bad(self, x, y, i, j):
        g = orig(self, x, y, i, j)
        return g if x == y else g[::-1]
    monkeypatch.setattr(blocks._Integrals, "ovov", bad)
    assert _p1_gap(dom) > 1e-6


def test_planted_mistake_closed_shell_formula(monkeypatch):
    """A wrong weight in the closed-shell formula breaks the P2 reduction."""
    dom = synth.make_rhf_domain(3, 6, 20, seed=11, sigma_f=3e-2, sigma_t1=3e-2)
    good = rhf.energy(dom)["E"]
    bl = blocks.energy(dom)["E"]
    assert _rel(good, bl) < 1e-12
    src_energy = rhf.energy

    def bad(d):
        d2 = d.replace(t2ab=np.ascontiguousarray(d.t2ab.transpose(0, 1, 3, 2)))
        return src_energy(d2)
    assert _rel(bad(dom)["E"], bl) > 1e-6
