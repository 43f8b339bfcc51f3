"""Pins of the oracle's central-LMO share (oracle/central.py) and of its
Laplace quadrature (oracle/laplace.py), on the CPU.

What fixes them independently of their own code:
  * exact denominators and c = e_i: one third of the per-item energies of
    oracle/blocks over the items that contain orbital i (eq. local_pt's 1/3
    with the items of eq. cim_pt_energy), both spins, parts per block;
  * the shares of any orthonormal basis of both spins' occupied spaces add up
    to E(T) (exact mode) resp. to the element-wise Laplace energy (Laplace
    mode), per block: the rotation of the central index and its half of the
    exp(D s) factor are then right;
  * the Laplace share with c = e_i lies within the quadrature's error bound
    of the exact one, and the Laplace energy approaches E(T) as the number of
    points grows;
  * planted mistakes (the central factor dropped, a sign of V_t1 in the mixed
    pair group) make a pin fail.
"""
import numpy as np
import pytest

import synth
from oracle import blocks, central, laplace

ALPHA_SLOTS = {0: (1, 2, 3), 1: (1, 2), 2: (3,), 3: ()}
BETA_SLOTS = {0: (), 1: (3,), 2: (1, 2), 3: (1, 2, 3)}
SHAPES = [(4, 3, 12, 13, 30), (3, 1, 9, 10, 20), (2, 3, 8, 7, 16)]
_Q = {}


def _quad(n, dom):
    """Oracle quadrature for the domain's |D| range, cached per (n, range)."""
    ev = np.concatenate([dom.ev_a, dom.ev_b])
    eo = np.concatenate([dom.eo_a, dom.eo_b])
    dmin = 3 * ev.min() - 3 * eo.max()
    dmax = 3 * ev.max() - 3 * eo.min()
    key = (n, round(dmin, 12), round(dmax, 12))
    if key not in _Q:
        s, w, err = laplace.quadrature(n, dmin, dmax)
        _Q[key] = (s, w, err, dmin)
    return _Q[key]


def _items_with(items, spin, i):
    sl = ALPHA_SLOTS if spin == 0 else BETA_SLOTS
    return [n for n, r in enumerate(items) if any(r[s] == i for s in sl[int(r[0])])]


@pytest.mark.parametrize("shape", SHAPES)
def test_unit_vector_is_a_third_of_its_items(shape):
    dom = synth.make_domain(*shape, seed=11)
    items = blocks.enumerate_items(dom.noa, dom.nob)
    ref = blocks.energy(dom, return_items=True)
    for spin in (0, 1):
        o = (dom.noa, dom.nob)[spin]
        for i in range(o):
            c = np.zeros(o)
            c[i] = 1.0
            got = central.central_share(dom, spin, c)
            sel = _items_with(items, spin, i)
            want = np.zeros((4, 3))
            for n in sel:
                want[items[n][0]] += ref["items"][n] / 3.0
            np.testing.assert_allclose(got["parts"], want, rtol=1e-12, atol=1e-300)


@pytest.mark.parametrize("shape", SHAPES[:2])
def test_orthonormal_basis_adds_up_to_the_energy(shape):
    dom = synth.make_domain(*shape, seed=12)
    ref = blocks.energy(dom)
    rng = np.random.default_rng(3)
    tot = np.zeros((4, 3))
    for spin in (0, 1):
        o = (dom.noa, dom.nob)[spin]
        if o == 0:
            continue
        U, _ = np.linalg.qr(rng.normal(size=(o, o)))
        for k in range(o):
            tot += central.central_share(dom, spin, U[:, k])["parts"]
    np.testing.assert_allclose(tot, ref["parts"], rtol=1e-11, atol=1e-16)


def _laplace_basis_sum(dom, quad, seed):
    rng = np.random.default_rng(seed)
    tot = np.zeros((4, 3))
    for spin in (0, 1):
        o = (dom.noa, dom.nob)[spin]
        if o == 0:
            continue
        U, _ = np.linalg.qr(rng.normal(size=(o, o)))
        for k in range(o):
            tot += central.central_share(dom, spin, U[:, k], quad)["parts"]
    return tot


def test_laplace_basis_sum_is_the_elementwise_laplace_energy():
    dom = synth.make_domain(*SHAPES[0], seed=13)
    s, w, _, _ = _quad(3, dom)
    want = central.laplace_energy(dom, (s, w))["parts"]
    np.testing.assert_allclose(_laplace_basis_sum(dom, (s, w), 4), want, rtol=1e-11, atol=1e-16)
    # arbitrary positive points and weights: the identity does not depend on the quadrature
    rng = np.random.default_rng(8)
    quad = (rng.uniform(0.05, 1.5, 3), rng.uniform(0.1, 1.0, 3))
    want = central.laplace_energy(dom, quad)["parts"]
    np.testing.assert_allclose(_laplace_basis_sum(dom, quad, 5), want, rtol=1e-11, atol=1e-16)


def test_laplace_share_within_the_quadrature_bound():
    """|dE_i(Laplace) - dE_i(exact)| <= (1/3) sum |W (W + V)| * max|1/|D| - L(|D|)|
    over the items containing i, and the Laplace energy approaches E(T) as
    the number of points grows."""
    from oracle.blocks import _Integrals, mixed_cubes, same_spin_cubes
    dom = synth.make_domain(*SHAPES[0], seed=14)
    items = blocks.enumerate_items(dom.noa, dom.nob)
    ints = _Integrals(dom)
    mag = np.zeros(len(items))
    for n, (b, p, q, r) in enumerate(items):
        if b in (0, 3):
            w, vt, vf, _ = same_spin_cubes(ints, 0 if b == 0 else 1, p, q, r)
            mag[n] = np.sum(np.abs(w * (w + vt + vf))) / 6.0
        else:
            w, vt, vf, _ = mixed_cubes(ints, dom, 0 if b == 1 else 1, p, q, r)
            mag[n] = np.sum(np.abs(w * (w + vt + vf))) / 2.0
    E = blocks.energy(dom)["E"]
    errs = []
    for nq in (1, 2, 3, 4):
        s, w, emax, _ = _quad(nq, dom)
        for spin, i in ((0, 1), (1, 2)):
            o = (dom.noa, dom.nob)[spin]
            c = np.zeros(o)
            c[i] = 1.0
            lap = central.central_share(dom, spin, c, (s, w))["E"]
            ex = central.central_share(dom, spin, c)["E"]
            bound = mag[_items_with(items, spin, i)].sum() / 3.0 * emax
            assert abs(lap - ex) <= bound * (1 + 1e-9) + 1e-15, (nq, spin, i, lap, ex, bound)
        errs.append(abs(central.laplace_energy(dom, (s, w))["E"] - E))
    assert all(b < a for a, b in zip(errs, errs[1:])), errs
    assert errs[-1] < 1e-3 * abs(E)


def test_phase_of_the_central_vector():
    dom = synth.make_domain(*SHAPES[1], seed=15)
    rng = np.random.default_rng(6)
    c = rng.normal(size=dom.noa)
    c /= np.linalg.norm(c)
    quad = (np.array([0.3, 0.9]), np.array([0.5, 0.4]))
    for q in (None, quad):
        a = central.central_share(dom, 0, c, q)["parts"]
        b = central.central_share(dom, 0, -c, q)["parts"]
        np.testing.assert_allclose(a, b, rtol=1e-13, atol=1e-300)


def test_planted_mistakes_are_caught(monkeypatch):
    dom = synth.make_domain(*SHAPES[0], seed=16)
    quad = (np.array([0.2, 0.7, 1.4]), np.array([0.3, 0.5, 0.2]))
    want = central.laplace_energy(dom, quad)["parts"]
    # the central orbital's half of exp(D s) dropped: the basis sum misses exp(s e_i)
    monkeypatch.setattr(central, "_central_factor", lambda s, e: 1.0)
    got = _laplace_basis_sum(dom, quad, 4)
    assert not np.allclose(got, want, rtol=1e-6, atol=0)
    monkeypatch.undo()
    # the sign of V_t1 flipped in the mixed group with the central index in the pair
    orig = central._cubes

    def bad(ints, dom_, spin, kind, i, p, q):
        w, vt, vf, d = orig(ints, dom_, spin, kind, i, p, q)
        return (w, -vt, vf, d) if kind == "pair" else (w, vt, vf, d)
    monkeypatch.setattr(central, "_cubes", bad)
    items = blocks.enumerate_items(dom.noa, dom.nob)
    ref = blocks.energy(dom, return_items=True)
    c = np.zeros(dom.noa)
    c[0] = 1.0
    got = central.central_share(dom, 0, c)["parts"]
    sel = _items_with(items, 0, 0)
    want = np.zeros((4, 3))
    for n in sel:
        want[items[n][0]] += ref["items"][n] / 3.0
    assert not np.allclose(got, want, rtol=1e-6, atol=0)


def test_quadrature_error_decreases_and_equioscillates():
    """The exponential sums of the oracle quadrature on [1, 11]: the maximum
    error falls with every added point; where the Remez exchange converged
    (n <= 3 here) the error equioscillates at 2n + 1 points of [1, R] with
    equal magnitude (the characterisation of the best approximation)."""
    R = 11.0
    x = np.geomspace(1.0, R, 100001)
    prev = np.inf
    for n in (1, 2, 3, 4):
        a, w, emax = laplace.minimax(n, R)
        e = laplace._err(x, w, a)
        assert np.max(np.abs(e)) <= emax * (1 + 1e-6)
        assert emax < prev
        prev = emax
        if n <= 3:
            xs = laplace._extremal_set(w, a, R, n)
            assert xs is not None
            ev = laplace._err(xs, w, a)
            assert np.all(np.sign(ev[1:]) == -np.sign(ev[:-1]))
            assert np.ptp(np.abs(ev)) <= 1e-7 * np.max(np.abs(ev))
    # scaled to [xmin, xmax]
    s, wq, err = laplace.quadrature(3, 0.7, 7.7)
    y = np.geomspace(0.7, 7.7, 20001)
    approx = np.exp(-np.outer(y, s)) @ wq
    assert np.max(np.abs(1.0 / y - approx)) <= err * (1 + 1e-6)
