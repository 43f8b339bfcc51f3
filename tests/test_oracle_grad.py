"""Pins of the oracle gradient (oracle.grad) against facts that do not come
from it: exact finite-difference stencils of the independently pinned
NumPy energy (oracle.blocks) and of the brute-force spin-orbital energy
(oracle.spinorb), and the symmetry-image convention of the projected
gradient.  E is quadratic in (T1, T2) and quartic in B, so the 3-point
central stencil is exact in T and the 5-point one exact in B, up to rounding.
"""
import numpy as np
import pytest

import synth
from oracle import blocks, grad, spinorb

T_FIELDS = ("t1a", "t1b", "t2aa", "t2bb", "t2ab")
B_FIELDS = ("Boo_a", "Bov_a", "Bvv_a", "Boo_b", "Bov_b", "Bvv_b")
SHAPES = [(3, 2, 5, 6, 14), (4, 3, 6, 5, 12), (3, 0, 4, 5, 10), (2, 2, 4, 4, 9)]
FOV_FIELDS = ("fov_a", "fov_b")


def _dom(shape, seed=5):
    # larger f_ov and T1 than the workload recipe so that every term of the
    # gradient is well above rounding
    return synth.make_domain(*shape, seed=seed, sigma_f=3e-2, sigma_t1=3e-2)


def _direction(dom, field, rng):
    """A random direction in the constrained subspace of `field`."""
    x = getattr(dom, field)
    d = rng.normal(0.0, 1.0, size=x.shape) * (np.std(x) + 1e-3)
    if field in ("t2aa", "t2bb"):
        d = d - d.transpose(1, 0, 2, 3)
        d = d - d.transpose(0, 1, 3, 2)
    if field.startswith("Boo") or field.startswith("Bvv"):
        d = d + d.transpose(0, 2, 1)
    return d


def _E(dom, field, d, h, fn):
    return fn(dom.replace(**{field: getattr(dom, field) + h * d}))


def _stencil(dom, field, d, fn):
    """Exact derivative along d: 3-point for T, 5-point for B."""
    h = 0.5
    if field in T_FIELDS:
        return (_E(dom, field, d, h, fn) - _E(dom, field, d, -h, fn)) / (2 * h)
    return (-_E(dom, field, d, 2 * h, fn) + 8 * _E(dom, field, d, h, fn)
            - 8 * _E(dom, field, d, -h, fn) + _E(dom, field, d, -2 * h, fn)) / (12 * h)


def _blocks_E(dom):
    return blocks.energy(dom)["E"]


@pytest.mark.parametrize("shape", SHAPES)
def test_transcription_energy_equals_blocks(shape):
    dom = _dom(shape)
    E, _ = grad.energy_and_grad(dom)
    ref = blocks.energy(dom)["E"]
    assert abs(E - ref) <= 1e-12 * abs(ref)


@pytest.mark.parametrize("shape", SHAPES)
def test_directional_derivatives_exact_stencil(shape):
    """<g, d> equals the exact stencil of the NumPy energy for every input."""
    dom = _dom(shape)
    _, g = grad.energy_and_grad(dom)
    rng = np.random.default_rng(17)
    for field in T_FIELDS + B_FIELDS:
        if getattr(dom, field).size == 0:
            continue
        d = _direction(dom, field, rng)
        fd = _stencil(dom, field, d, _blocks_E)
        an = float(np.sum(g[field] * d))
        scale = max(abs(fd), 1e-9 * abs(_blocks_E(dom)))
        assert abs(an - fd) <= 1e-8 * scale, (field, an, fd)


def test_directional_derivatives_against_spin_orbital_brute_force():
    """Same check against the literal 1/36 spin-orbital sum."""
    dom = _dom((3, 2, 4, 5, 10), seed=9)
    _, g = grad.energy_and_grad(dom)
    rng = np.random.default_rng(3)
    fn = lambda x: spinorb.energy(x)["E"]
    for field in ("t1b", "t2aa", "t2ab", "Bov_a", "Bvv_b", "Boo_a"):
        d = _direction(dom, field, rng)
        fd = _stencil(dom, field, d, fn)
        an = float(np.sum(g[field] * d))
        assert abs(an - fd) <= 1e-8 * max(abs(fd), 1e-12), (field, an, fd)


def _images_fd(dom, field, idx, imgs, h=1e-2):
    x = getattr(dom, field)
    d = np.zeros_like(x)
    for sgn, ix in imgs(idx):
        d[ix] = sgn
    return (_E(dom, field, d, h, _blocks_E) - _E(dom, field, d, -h, _blocks_E)) / (2 * h)


def test_projected_convention_symmetry_images():
    """Moving all signed images of one t2aa element gives 4x the returned
    element, of one off-diagonal Bvv element 2x, of a diagonal one 1x."""
    dom = _dom((4, 2, 5, 6, 12))
    _, g = grad.energy_and_grad(dom)
    t2img = lambda ix: [(1, ix), (-1, (ix[1], ix[0], ix[2], ix[3])), (-1, (ix[0], ix[1], ix[3], ix[2])),
                        (1, (ix[1], ix[0], ix[3], ix[2]))]
    ix = (0, 2, 1, 4)
    assert abs(_images_fd(dom, "t2aa", ix, t2img) - 4 * g["t2aa"][ix]) <= 1e-9 * abs(4 * g["t2aa"][ix])
    symimg = lambda ix: [(1, ix), (1, (ix[0], ix[2], ix[1]))]
    ix = (3, 1, 4)
    assert abs(_images_fd(dom, "Bvv_b", ix, symimg) - 2 * g["Bvv_b"][ix]) <= 1e-8 * abs(2 * g["Bvv_b"][ix])
    diag = lambda ix: [(1, ix)]
    ix = (2, 3, 3)
    assert abs(_images_fd(dom, "Boo_a", ix, diag) - g["Boo_a"][ix]) <= 1e-8 * abs(g["Boo_a"][ix])
    # the projected gradients carry the symmetry of their inputs
    for k, perm, sgn in (("t2aa", (1, 0, 2, 3), -1), ("t2bb", (0, 1, 3, 2), -1), ("Bvv_a", (0, 2, 1), 1),
                         ("Boo_b", (0, 2, 1), 1)):
        assert np.max(np.abs(g[k] - sgn * g[k].transpose(*perm))) <= 1e-14 * np.max(np.abs(g[k]))


def test_gbar_scales_and_items_add():
    dom = _dom((4, 3, 5, 6, 12))
    items = blocks.enumerate_items(dom.noa, dom.nob)
    _, g = grad.energy_and_grad(dom)
    _, g2 = grad.energy_and_grad(dom, gbar=-2.0)
    _, ga = grad.energy_and_grad(dom, items=items[::2])
    _, gb = grad.energy_and_grad(dom, items=items[1::2])
    for k in grad.FIELDS:
        assert np.allclose(g2[k], -2.0 * g[k], rtol=1e-14, atol=0)
        assert np.allclose(ga[k] + gb[k], g[k], rtol=1e-12, atol=1e-18)


def test_planted_unprojected_gradient_is_caught(monkeypatch):
    """Without the projection the image convention pin fails."""
    monkeypatch.setattr(grad, "project", lambda g: g)
    dom = _dom((4, 2, 5, 6, 12))
    _, g = grad.energy_and_grad(dom)
    t2img = lambda ix: [(1, ix), (-1, (ix[1], ix[0], ix[2], ix[3])), (-1, (ix[0], ix[1], ix[3], ix[2])),
                        (1, (ix[1], ix[0], ix[3], ix[2]))]
    ix = (0, 2, 1, 4)
    fd = _images_fd(dom, "t2aa", ix, t2img)
    assert abs(fd - 4 * g["t2aa"][ix]) > 1e-6 * abs(fd)


def test_planted_sign_error_in_transcription_is_caught(monkeypatch):
    """A sign flip of one mixed-block singles term changes the gradient along
    t1b, and the exact stencil of the NumPy energy sees it."""
    dom = _dom((3, 2, 5, 6, 12))
    orig = grad._Item.mixed

    def bad(self, s, i, j, K):
        t1 = self.X["t1" + "ab"[1 - s]]
        self.X["t1" + "ab"[1 - s]] = -t1
        try:
            return orig(self, s, i, j, K)
        finally:
            self.X["t1" + "ab"[1 - s]] = t1
    monkeypatch.setattr(grad._Item, "mixed", bad)
    _, g = grad.energy_and_grad(dom)
    rng = np.random.default_rng(1)
    d = _direction(dom, "t1b", rng)
    fd = _stencil(dom, "t1b", d, _blocks_E)
    assert abs(float(np.sum(g["t1b"] * d)) - fd) > 1e-6 * abs(fd)


@pytest.mark.parametrize("shape", SHAPES)
def test_fock_gradient_exact_stencil(shape):
    """f_ov enters only the disconnected V, linearly, so E is linear in f_ov
    and the central difference of the NumPy energy is exact for any step:
    along random directions and on single entries."""
    dom = _dom(shape)
    E0, g = grad.energy_and_grad(dom, fock=True)
    _, g0 = grad.energy_and_grad(dom)
    for k in grad.FIELDS:              # the Fock request changes nothing else
        assert np.array_equal(g[k], g0[k])
    rng = np.random.default_rng(23)
    for field in FOV_FIELDS:
        x = getattr(dom, field)
        if x.size == 0:
            continue
        d = rng.normal(0.0, 1.0, size=x.shape)
        h = 2.0
        fd = (_E(dom, field, d, h, _blocks_E) - _E(dom, field, d, -h, _blocks_E)) / (2 * h)
        an = float(np.sum(g[field] * d))
        assert abs(an - fd) <= 1e-8 * max(abs(fd), 1e-9 * abs(E0)), (field, an, fd)
        # linearity: the one-sided difference agrees as well
        fw = (_E(dom, field, d, h, _blocks_E) - _blocks_E(dom)) / h
        assert abs(an - fw) <= 1e-8 * max(abs(fw), 1e-9 * abs(E0)), (field, an, fw)
        for ix in ((0, 0), (x.shape[0] - 1, x.shape[1] - 1)):
            e = np.zeros_like(x)
            e[ix] = 1.0
            fd1 = (_E(dom, field, e, 1.0, _blocks_E) - _E(dom, field, e, -1.0, _blocks_E)) / 2.0
            assert abs(g[field][ix] - fd1) <= 1e-8 * max(abs(fd1), 1e-12 * abs(E0)), (field, ix)


def test_fock_gradient_against_spin_orbital_brute_force():
    dom = _dom((3, 2, 4, 5, 10), seed=9)
    _, g = grad.energy_and_grad(dom, fock=True)
    rng = np.random.default_rng(8)
    fn = lambda x: spinorb.energy(x)["E"]
    for field in FOV_FIELDS:
        d = rng.normal(0.0, 1.0, size=getattr(dom, field).shape)
        fd = (_E(dom, field, d, 1.0, fn) - _E(dom, field, d, -1.0, fn)) / 2.0
        an = float(np.sum(g[field] * d))
        assert abs(an - fd) <= 1e-8 * max(abs(fd), 1e-12), (field, an, fd)


def test_fock_gradient_vanishes_without_connected_triples():
    """dE/df_ov is sum W dV/df / D: with T2 = 0 and no integrals W vanishes
    and so must the gradient, whatever T1 and f_ov are."""
    dom = _dom((3, 2, 5, 6, 12))
    z = {k: np.zeros_like(getattr(dom, k)) for k in ("t2aa", "t2bb", "t2ab")}
    _, g = grad.energy_and_grad(dom.replace(**z), fock=True)
    for k in FOV_FIELDS:
        assert np.max(np.abs(g[k])) == 0.0
    _, g = grad.energy_and_grad(dom, fock=True)
    assert all(np.max(np.abs(g[k])) > 0 for k in FOV_FIELDS)


def test_planted_fock_sign_error_is_caught(monkeypatch):
    """A sign flip of f_ov inside the mixed blocks only is caught by the exact
    stencil along f_ov of the other spin's block structure."""
    dom = _dom((3, 2, 5, 6, 12))
    orig = grad._Item.mixed

    def bad(self, s, i, j, K):
        f = self.C["fov_" + "ab"[1 - s]]
        self.C["fov_" + "ab"[1 - s]] = -f
        try:
            return orig(self, s, i, j, K)
        finally:
            self.C["fov_" + "ab"[1 - s]] = f
    monkeypatch.setattr(grad._Item, "mixed", bad)
    _, g = grad.energy_and_grad(dom, fock=True)
    rng = np.random.default_rng(2)
    d = rng.normal(0.0, 1.0, size=dom.fov_b.shape)
    fd = (_E(dom, "fov_b", d, 1.0, _blocks_E) - _E(dom, "fov_b", d, -1.0, _blocks_E)) / 2.0
    assert abs(float(np.sum(g["fov_b"] * d)) - fd) > 1e-6 * abs(fd)


EPS_FIELDS = ("eo_a", "ev_a", "eo_b", "ev_b")


@pytest.mark.parametrize("shape", SHAPES)
def test_orbital_energy_gradient_identities(shape):
    """D is occupied minus virtual orbital energies, so E does not change
    when every orbital energy moves by the same amount (the gradient sums to
    zero over both spins), and E is homogeneous of degree -1 in them
    (sum e dE/de = -E)."""
    dom = _dom(shape)
    E, g = grad.energy_and_grad(dom, fock=True)
    tot = sum(float(np.sum(g[k])) for k in EPS_FIELDS)
    mag = sum(float(np.sum(np.abs(g[k]))) for k in EPS_FIELDS)
    assert mag > 0
    assert abs(tot) <= 1e-12 * mag, (tot, mag)
    euler = sum(float(np.sum(np.asarray(getattr(dom, k)) * g[k])) for k in EPS_FIELDS)
    assert abs(euler + E) <= 1e-12 * abs(E), (euler, E)


@pytest.mark.parametrize("shape", SHAPES)
def test_orbital_energy_gradient_five_point_stencil(shape):
    """Against the 5-point central difference of the NumPy energy, along
    random directions and on single entries (E is smooth in the orbital
    energies; with steps of 1e-3 against gaps of order one the stencil error
    is far below the bar)."""
    dom = _dom(shape)
    E0, g = grad.energy_and_grad(dom, fock=True)
    rng = np.random.default_rng(31)
    h = 1e-3

    def five(field, d):
        return (-_E(dom, field, d, 2 * h, _blocks_E) + 8 * _E(dom, field, d, h, _blocks_E)
                - 8 * _E(dom, field, d, -h, _blocks_E) + _E(dom, field, d, -2 * h, _blocks_E)) / (12 * h)
    for field in EPS_FIELDS:
        x = np.asarray(getattr(dom, field))
        if x.size == 0:
            continue
        d = rng.normal(0.0, 1.0, size=x.shape)
        fd = five(field, d)
        an = float(np.sum(g[field] * d))
        assert abs(an - fd) <= 1e-7 * max(abs(fd), 1e-9 * abs(E0)), (field, an, fd)
        for ix in (0, x.shape[0] - 1):
            e = np.zeros_like(x)
            e[ix] = 1.0
            fd1 = five(field, e)
            assert abs(g[field][ix] - fd1) <= 1e-7 * max(abs(fd1), 1e-9 * abs(E0)), (field, ix, fd1)


def test_orbital_energy_gradient_against_spin_orbital_brute_force():
    dom = _dom((3, 2, 4, 5, 10), seed=9)
    _, g = grad.energy_and_grad(dom, fock=True)
    rng = np.random.default_rng(12)
    fn = lambda x: spinorb.energy(x)["E"]
    h = 1e-3
    for field in EPS_FIELDS:
        d = rng.normal(0.0, 1.0, size=np.asarray(getattr(dom, field)).shape)
        fd = (-_E(dom, field, d, 2 * h, fn) + 8 * _E(dom, field, d, h, fn)
              - 8 * _E(dom, field, d, -h, fn) + _E(dom, field, d, -2 * h, fn)) / (12 * h)
        an = float(np.sum(g[field] * d))
        assert abs(an - fd) <= 1e-7 * max(abs(fd), 1e-12), (field, an, fd)


def test_planted_denominator_error_breaks_shift_invariance(monkeypatch):
    """A mixed-block denominator that drops the third occupied energy is no
    longer shift invariant, and the identity pin sees it."""
    dom = _dom((3, 2, 5, 6, 12))
    orig = grad._Item.mixed

    def bad(self, s, i, j, K):
        t = 1 - s
        eo = self.C["eo_" + "ab"[t]]
        self.C["eo_" + "ab"[t]] = eo * 0.0
        try:
            return orig(self, s, i, j, K)
        finally:
            self.C["eo_" + "ab"[t]] = eo
    monkeypatch.setattr(grad._Item, "mixed", bad)
    _, g = grad.energy_and_grad(dom, fock=True)
    tot = sum(float(np.sum(g[k])) for k in EPS_FIELDS)
    mag = sum(float(np.sum(np.abs(g[k]))) for k in EPS_FIELDS)
    assert abs(tot) > 1e-6 * mag


def _rhf_arrays(shape, seed=13):
    dom = synth.make_rhf_domain(*shape, seed=seed, sigma_f=3e-2, sigma_t1=3e-2)
    return dom, synth.rhf_arrays(dom)


def _rhf_dir(arr, k, rng):
    x = np.asarray(arr[k])
    d = rng.normal(0.0, 1.0, size=x.shape) * (np.std(x) + 1e-3)
    if k == "tau":
        d = d + d.transpose(1, 0, 3, 2)
    if k in ("Boo", "Bvv"):
        d = d + d.transpose(0, 2, 1)
    return d


@pytest.mark.parametrize("shape", [(3, 5, 12), (4, 4, 10), (2, 5, 9)])
def test_rhf_gradient_against_closed_shell_formula(shape):
    """The torch transcription's energy equals oracle.rhf, and <g, d> equals
    the 5-point central difference of oracle.rhf along random directions in
    every input's constrained space (exact for the polynomial inputs, to the
    stencil error for the orbital energies)."""
    from oracle import rhf
    dom, arr = _rhf_arrays(shape)
    E, g = grad.rhf_energy_and_grad(arr)
    E0 = rhf.energy(dom)["E"]
    assert abs(E - E0) <= 1e-12 * abs(E0)
    rng = np.random.default_rng(41)

    def erhf(k, d, h):
        a = dict(arr)
        a[k] = np.asarray(arr[k]) + h * d
        # oracle.rhf reads the alpha arrays of a spin-blocked domain
        key = {"t1": "t1a", "tau": "t2ab", "Boo": "Boo_a", "Bov": "Bov_a", "Bvv": "Bvv_a", "eo": "eo_a",
               "ev": "ev_a", "fov": "fov_a"}[k]
        return rhf.energy(dom.replace(**{key: a[k]}))["E"]
    for k in grad.RHF_FIELDS:
        d = _rhf_dir(arr, k, rng)
        h = 1e-3 if k in ("eo", "ev") else 0.5
        fd = (-erhf(k, d, 2 * h) + 8 * erhf(k, d, h) - 8 * erhf(k, d, -h) + erhf(k, d, -2 * h)) / (12 * h)
        an = float(np.sum(g[k] * d))
        assert abs(an - fd) <= 1e-7 * max(abs(fd), 1e-9 * abs(E0)), (k, an, fd)


def test_rhf_gradient_symmetry_and_identities():
    dom, arr = _rhf_arrays((3, 5, 12))
    E, g = grad.rhf_energy_and_grad(arr)
    assert np.max(np.abs(g["tau"] - g["tau"].transpose(1, 0, 3, 2))) <= 1e-15 * np.max(np.abs(g["tau"]))
    # common shift of the orbital energies, degree -1 homogeneity
    tot = float(np.sum(g["eo"]) + np.sum(g["ev"]))
    assert abs(tot) <= 1e-12 * float(np.sum(np.abs(g["eo"])) + np.sum(np.abs(g["ev"])))
    euler = float(np.sum(arr["eo"] * g["eo"]) + np.sum(arr["ev"] * g["ev"]))
    assert abs(euler + E) <= 1e-12 * abs(E)
