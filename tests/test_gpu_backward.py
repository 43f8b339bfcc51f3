"""GPU parity of the adjoint pass (ltriples_backward) through the C ABI.

Reference: the oracle gradient (reverse-mode derivative of the spin-blocked
FP64 energy, pinned by exact finite-difference stencils).  Bar per gradient
tensor: max|g_gpu - g_ref| <= tol * max|g_ref| with tol 1e-10 (FP64) and 1e-5
(FP32, and BF16X3: the forward contraction recomputed in split BF16 products,
whose W carries about 1e-6 of relative error, with FP32 reverse GEMMs).  At the full gradient workload (20,18,160,162,640) the check is the
oracle gradient of a sampled item subset, and the exact directional
derivative of the GPU's own FP64 energy (E is quadratic in T1, T2 and
linear in f_ov).
"""
import numpy as np
import pytest

import paper_2311_10048_amd as lt
import synth
from oracle import grad as ograd
from tests.gpu_util import to_device

pytestmark = pytest.mark.gpu

TOL = {lt.LT_FP64: 1e-10, lt.LT_FP32: 1e-5, lt.LT_BF16X3: 1e-5}
ALL_GRAD = lt.GRAD_FIELDS + lt.FOCK_GRAD_FIELDS

SHAPES = {
    "tiny": (5, 4, 30, 31, 120),
    "ragged": (4, 3, 21, 22, 40),
    "no_beta_occ": (4, 0, 21, 22, 40),
    "one_beta": (3, 1, 17, 18, 30),
    "wide": (3, 3, 70, 67, 64),
    "no_beta_vir": (4, 3, 20, 0, 30),
    "no_alpha_vir": (3, 3, 0, 5, 20),
    "no_alpha_occ": (0, 4, 21, 22, 40),
    "one_alpha_two_beta": (1, 2, 15, 16, 30),
}


def _dom(shape, seed=synth.BASE_SEED + 41):
    # larger T1 and f_ov than the workload recipe so that their gradient
    # terms stand well above the FP64 rounding of the others
    return synth.make_domain(*shape, seed=seed, sigma_f=3e-2, sigma_t1=3e-2)


def _gpu_grad(dom, prec, tensors=None, **kw):
    import torch
    t = tensors if tensors is not None else to_device(dom)
    g = lt.ltriples_backward(t, dom.dims, prec, **kw)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in g.items()}


def _compare(g, ref, tol, label=""):
    for k in ALL_GRAD:
        if k not in ref:
            continue
        r = ref[k]
        if r.size == 0:
            continue
        scale = np.max(np.abs(r))
        err = np.max(np.abs(g[k] - r))
        assert err <= tol * max(scale, 1e-300), (label, k, err, scale)


@pytest.mark.parametrize("prec", [lt.LT_FP64, lt.LT_FP32, lt.LT_BF16X3])
@pytest.mark.parametrize("name", list(SHAPES))
def test_backward_parity_shapes(name, prec):
    dom = _dom(SHAPES[name])
    print(f"[backward] {name} {SHAPES[name]} prec={prec}", flush=True)
    _, ref = ograd.energy_and_grad(dom, fock=True)
    g = _gpu_grad(dom, prec)
    _compare(g, ref, TOL[prec], name)


def test_backward_small_batches_and_gbar():
    """Batches of 3 items give the same gradient (to rounding: the batch
    partition orders the accumulation); gbar scales it."""
    import torch
    dom = _dom(SHAPES["ragged"])
    t = to_device(dom)
    g1 = _gpu_grad(dom, lt.LT_FP64, tensors=t)
    g3 = _gpu_grad(dom, lt.LT_FP64, tensors=t, batch_items=3)
    _compare(g3, g1, 1e-13, "batch3")
    gb = torch.full((1,), -2.5, dtype=torch.float64, device="cuda")
    g2 = _gpu_grad(dom, lt.LT_FP64, tensors=t, gbar=gb)
    _compare(g2, {k: -2.5 * v for k, v in g1.items()}, 1e-14, "gbar")


def test_backward_chunked_builds_bitwise_equal():
    """The adjoint with its forward operand builds in 1 MiB chunks gives
    exactly the default gradient."""
    dom = _dom(SHAPES["wide"])
    t = to_device(dom)
    g0 = _gpu_grad(dom, lt.LT_FP64, tensors=t)
    g1 = _gpu_grad(dom, lt.LT_FP64, tensors=t, build_chunk_mib=1)
    for k in ALL_GRAD:
        assert np.array_equal(g0[k], g1[k]), k


def test_backward_bf16x3_chunks_and_batches():
    """The BF16X3 adjoint keeps the FP32 operands beside their split copies
    and splits chunked operand builds in place: with 1 MiB build chunks
    (several chunks per operand on this shape) it gives exactly the default
    gradient; with batches of 3 items it agrees to rounding (the batching
    orders the reverse sums), and both stay at the FP32 bar."""
    dom = _dom(SHAPES["wide"])
    t = to_device(dom)
    g0 = _gpu_grad(dom, lt.LT_BF16X3, tensors=t)
    g1 = _gpu_grad(dom, lt.LT_BF16X3, tensors=t, build_chunk_mib=1)
    for k in ALL_GRAD:
        assert np.array_equal(g0[k], g1[k]), k
    g3 = _gpu_grad(dom, lt.LT_BF16X3, tensors=t, batch_items=3)
    _compare(g3, g0, 1e-6, "bf16x3 batch3")
    _, ref = ograd.energy_and_grad(dom, fock=True)
    _compare(g1, ref, TOL[lt.LT_BF16X3], "bf16x3 chunks")


def test_backward_workspace_garbage_never_read():
    import torch
    dom = _dom(SHAPES["wide"])
    t = to_device(dom)
    d = lt.make_domain(dom.dims, t)
    need = lt.ltriples_backward_workspace_size(d, lt.LT_FP64)
    outs = []
    for fill in (0.0, float("nan")):
        ws = torch.full((need // 8 + 1,), fill, dtype=torch.float64, device="cuda").view(torch.uint8)
        outs.append(_gpu_grad(dom, lt.LT_FP64, tensors=t, workspace=ws))
    for k in ALL_GRAD:
        assert np.array_equal(outs[0][k], outs[1][k]), k


_GRAD_REF = {}


def _grad_workload_ref():
    """The gradient workload, a sampled item list and the oracle gradient of
    E(items) (computed once for the tests below)."""
    if not _GRAD_REF:
        dom = synth.config_domain("grad")
        items = synth.sample_items(dom.noa, dom.nob, 1, seed=77)
        _, ref = ograd.energy_and_grad(dom, items=items, fock=True)
        _GRAD_REF.update(dom=dom, items=items, ref=ref)
    return _GRAD_REF["dom"], _GRAD_REF["items"], _GRAD_REF["ref"]


@pytest.mark.parametrize("prec", [lt.LT_FP64, lt.LT_FP32, lt.LT_BF16X3])
def test_backward_sampled_items_gradient_workload(prec):
    """Full-size gradient workload, restricted to a sampled item list: the
    gradient of E(items) against the oracle's gradient of the same items, at
    the FP64 (1e-10) and FP32 (1e-5) bars."""
    dom, items, ref = _grad_workload_ref()
    print(f"[backward] grad workload {dom.dims}, {len(items)} sampled items, prec={prec}", flush=True)
    g = _gpu_grad(dom, prec, items=items)
    _compare(g, ref, TOL[prec], "grad-sampled")


def test_backward_central_differences_gradient_workload():
    """The gradient workload (20,18,160,162,640): 50 random entries over T1,
    T2 and the DF factors of both spins, central differences with h = 1e-5
    of the FP64 GPU energy of a sampled item list (milliseconds per energy)
    against ltriples_backward of the same items.  The amplitude entries are
    drawn among the occupied orbitals the items contain (other entries have
    zero derivative).  Bar: |FD - g| <= 1e-5 |g| + 100 eps |E| / h (E is
    quadratic in T, so the difference is exact up to rounding; quartic in B,
    with a truncation error of relative size (h / 0.05)^2).  Each difference
    moves every symmetry image of the entry (4x for t2aa/t2bb, 2x for
    off-diagonal Boo/Bvv)."""
    import torch
    dom, items, _ = _grad_workload_ref()
    t = to_device(dom)
    d = lt.make_domain(dom.dims, t)
    o, _ = lt.make_options(items=items)
    ws = torch.empty(max(lt.ltriples_workspace_size(d, lt.LT_FP64, o),
                         lt.ltriples_backward_workspace_size(d, lt.LT_FP64, o)), dtype=torch.uint8, device="cuda")
    g = _gpu_grad(dom, lt.LT_FP64, tensors=t, items=items, workspace=ws)
    e0, _ = lt.ltriples_energy(t, dom.dims, lt.LT_FP64, items=items, workspace=ws)
    torch.cuda.synchronize()
    E0 = float(e0.item())
    # occupied orbitals of each spin in the items: (0, i, j, k) aaa, (1, i, j, K) aab,
    # (2, I, J, k) abb, (3, I, J, K) bbb
    alpha_slots = {0: (1, 2, 3), 1: (1, 2), 2: (3,), 3: ()}
    beta_slots = {0: (), 1: (3,), 2: (1, 2), 3: (1, 2, 3)}
    it = np.asarray(items)
    occ = {"a": sorted({int(r[c]) for r in it for c in alpha_slots[int(r[0])]}),
           "b": sorted({int(r[c]) for r in it for c in beta_slots[int(r[0])]})}
    rng = np.random.default_rng(3003)
    h, eps = 1e-5, np.finfo(np.float64).eps
    plan = ["t1a"] * 4 + ["t1b"] * 4 + ["t2aa"] * 7 + ["t2bb"] * 7 + ["t2ab"] * 7 + \
           ["Boo_a", "Bov_a", "Bvv_a", "Boo_b", "Bov_b", "Bvv_b"] * 3 + ["Bov_a", "Bvv_b", "Bvv_a"]
    assert len(plan) == 50
    print(f"[backward] central differences on {len(plan)} entries of {dom.dims}", flush=True)
    for k in plan:
        x = getattr(dom, k)
        if k in ("t1a", "t1b"):
            idx = (int(rng.choice(occ[k[-1]])), int(rng.integers(0, x.shape[1])))
        elif k in ("t2aa", "t2bb"):
            o_ = occ[k[-1]]
            i = int(rng.choice(o_))
            j = int(rng.integers(0, x.shape[0]))
            while j == i:
                j = int(rng.integers(0, x.shape[0]))
            a, b = (int(y) for y in rng.choice(x.shape[2], size=2, replace=False))
            idx = (i, j, a, b)
        elif k == "t2ab":
            idx = (int(rng.choice(occ["a"])), int(rng.choice(occ["b"])), int(rng.integers(0, x.shape[2])),
                   int(rng.integers(0, x.shape[3])))
        else:
            idx = tuple(int(rng.integers(0, m)) for m in x.shape)
        images, mult = [(idx, 1.0)], 1.0
        if k in ("t2aa", "t2bb"):
            i, j, a, b = idx
            images = [((i, j, a, b), 1.0), ((j, i, a, b), -1.0), ((i, j, b, a), -1.0), ((j, i, b, a), 1.0)]
            mult = 4.0
        elif k in ("Boo_a", "Boo_b", "Bvv_a", "Bvv_b") and idx[1] != idx[2]:
            q, p_, r = idx
            images, mult = [((q, p_, r), 1.0), ((q, r, p_), 1.0)], 2.0
        es = []
        for sgn in (1.0, -1.0):
            tp = dict(t)
            y = t[k].clone()
            for im, w in images:
                y[im] += sgn * w * h
            tp[k] = y
            e, _ = lt.ltriples_energy(tp, dom.dims, lt.LT_FP64, items=items, workspace=ws)
            torch.cuda.synchronize()
            es.append(float(e.item()))
        fd = (es[0] - es[1]) / (2 * h)
        want = mult * g[k][idx]
        assert abs(fd - want) <= 1e-5 * abs(want) + 100 * eps * abs(E0) / h, (k, idx, fd, want, E0)


def test_backward_directional_derivative_gradient_workload():
    """Whole gradient workload: <dE/dT, d> equals the exact central difference
    of the GPU FP64 energy along d (E is quadratic in T1, T2); FP32 adjoint
    agrees with FP64 to 1e-5."""
    import torch
    dom = synth.config_domain("grad")
    print(f"[backward] grad workload {dom.dims}, all items", flush=True)
    t = to_device(dom)
    g64 = lt.ltriples_backward(t, dom.dims, lt.LT_FP64)
    g32 = lt.ltriples_backward(t, dom.dims, lt.LT_FP32)
    torch.cuda.synchronize()
    for k in ALL_GRAD:
        a, b = g64[k], g32[k]
        assert float((a - b).abs().max()) <= 1e-5 * float(a.abs().max()), k
    rng = np.random.default_rng(5)
    dirs = {}
    for k in ("t1a", "t2aa", "t2ab", "t1b", "t2bb"):
        x = getattr(dom, k)
        d = rng.normal(0.0, 1.0, size=x.shape) * np.std(x)
        if k in ("t2aa", "t2bb"):
            d = d - d.transpose(1, 0, 2, 3)
            d = d - d.transpose(0, 1, 3, 2)
        dirs[k] = torch.from_numpy(d).cuda()
    h = 0.25
    tp = dict(t); tm = dict(t)
    for k, d in dirs.items():
        tp[k] = t[k] + h * d
        tm[k] = t[k] - h * d
    ep, _ = lt.ltriples_energy(tp, dom.dims, lt.LT_FP64)
    em, _ = lt.ltriples_energy(tm, dom.dims, lt.LT_FP64)
    e0, _ = lt.ltriples_energy(t, dom.dims, lt.LT_FP64)
    torch.cuda.synchronize()
    fd = (float(ep.item()) - float(em.item())) / (2 * h)
    an = sum(float((g64[k] * d).sum()) for k, d in dirs.items())
    assert abs(an - fd) <= 1e-9 * max(abs(fd), 1e-12 * abs(float(e0.item()))), (an, fd)
    # f_ov alone: E is linear in it, so the central difference is exact
    fdirs = {k: torch.from_numpy(rng.normal(0.0, 1.0, size=getattr(dom, k).shape)).cuda()
             for k in ("fov_a", "fov_b")}
    h = 1.0
    tp = dict(t); tm = dict(t)
    for k, d in fdirs.items():
        tp[k] = t[k] + h * d
        tm[k] = t[k] - h * d
    ep, _ = lt.ltriples_energy(tp, dom.dims, lt.LT_FP64)
    em, _ = lt.ltriples_energy(tm, dom.dims, lt.LT_FP64)
    torch.cuda.synchronize()
    fd = (float(ep.item()) - float(em.item())) / (2 * h)
    an = sum(float((g64[k] * d).sum()) for k, d in fdirs.items())
    assert abs(an - fd) <= 1e-9 * max(abs(fd), 1e-12 * abs(float(e0.item()))), ("fov", an, fd)
    # orbital energies: a common shift leaves every D unchanged (the gradient
    # sums to zero) and E is homogeneous of degree -1 in them
    eps = ("eo_a", "ev_a", "eo_b", "ev_b")
    tot = sum(float(g64[k].sum()) for k in eps)
    mag = sum(float(g64[k].abs().sum()) for k in eps)
    assert abs(tot) <= 1e-10 * mag, (tot, mag)
    euler = sum(float((t[k] * g64[k]).sum()) for k in eps)
    E0 = float(e0.item())
    assert abs(euler + E0) <= 1e-10 * abs(E0), (euler, E0)


def test_backward_central_differences_random_entries():
    """51 random entries of the FP64 GPU gradient, spread over all seventeen
    gradient inputs (f_ov and the orbital energies included), against
    central differences (h = 1e-5) of the FP64 GPU energy.  Each difference moves all symmetry images of the entry, so it
    sees 4x (t2aa, t2bb) or 2x (off-diagonal Boo, Bvv) the returned projected
    element."""
    import torch
    dom = _dom(SHAPES["ragged"])
    t = to_device(dom)
    g = _gpu_grad(dom, lt.LT_FP64, tensors=t)
    rng = np.random.default_rng(2024)
    h = 1e-5
    fields = [k for k in ALL_GRAD if getattr(dom, k).size > 0]
    for n in range(51):
        k = fields[n % len(fields)]
        x = getattr(dom, k)
        idx = tuple(int(rng.integers(0, m)) for m in x.shape)
        images, mult = [(idx, 1.0)], 1.0
        if k in ("t2aa", "t2bb"):
            i, j, a, b = idx
            if i == j or a == b:        # zero by antisymmetry: pick another entry
                i, j, a, b = 0, 1, 0, 1
            idx = (i, j, a, b)
            images = [((i, j, a, b), 1.0), ((j, i, a, b), -1.0), ((i, j, b, a), -1.0), ((j, i, b, a), 1.0)]
            mult = 4.0
        elif k in ("Boo_a", "Boo_b", "Bvv_a", "Bvv_b"):
            q, p, r = idx
            if p != r:
                images, mult = [((q, p, r), 1.0), ((q, r, p), 1.0)], 2.0
        es = []
        for sgn in (1.0, -1.0):
            tp = dict(t)
            y = t[k].clone()
            for im, w in images:
                y[im] += sgn * w * h
            tp[k] = y
            e, _ = lt.ltriples_energy(tp, dom.dims, lt.LT_FP64)
            torch.cuda.synchronize()
            es.append(float(e.item()))
        fd = (es[0] - es[1]) / (2 * h)
        want = mult * g[k][idx]
        scale = np.max(np.abs(g[k]))
        assert abs(fd - want) <= 1e-6 * scale + 1e-6 * abs(want), (k, idx, fd, want, scale)


def test_autograd_function_matches_backward():
    import torch
    dom = _dom(SHAPES["tiny"])
    t = to_device(dom)
    leaves = {k: (v.clone().requires_grad_(k in ALL_GRAD)) for k, v in t.items()}
    E = lt.triples_energy(leaves, dom.dims, "fp64")
    E.backward()
    g = lt.ltriples_backward(t, dom.dims, lt.LT_FP64)
    torch.cuda.synchronize()
    for k in ALL_GRAD:
        assert torch.equal(leaves[k].grad, g[k]), k
    e_ref, _ = lt.ltriples_energy(t, dom.dims, lt.LT_FP64)
    assert float(E.detach()) == float(e_ref.item())
    # a BF16X3 forward is differentiated by the FP32 adjoint unless FP64 or
    # the BF16X3 adjoint is asked for
    g32 = lt.ltriples_backward(t, dom.dims, lt.LT_FP32)
    gbf = lt.ltriples_backward(t, dom.dims, lt.LT_BF16X3)
    for bp, ref in ((None, g32), ("fp64", g), ("bf16x3", gbf)):
        lv = {k: (v.clone().requires_grad_(k in ALL_GRAD)) for k, v in t.items()}
        E = lt.triples_energy(lv, dom.dims, "bf16x3", backward_precision=bp)
        E.backward()
        torch.cuda.synchronize()
        for k in ALL_GRAD:
            assert torch.equal(lv[k].grad, ref[k]), (bp, k)


def test_backward_tall_shape_identities():
    """v > 384 (several row tiles in every reverse GEMM and contraction):
    <dE/dT, d> equals the exact central difference of the FP64 GPU energy
    (E is quadratic in T1, T2), the f_ov gradient the exact difference along
    f_ov (E is linear in it), the orbital-energy gradient satisfies the shift
    and homogeneity identities, and FP32 agrees with FP64 to 1e-5."""
    import torch
    dom = _dom((3, 1, 400, 401, 48))
    print(f"[backward] tall {dom.dims}", flush=True)
    t = to_device(dom)
    g64 = lt.ltriples_backward(t, dom.dims, lt.LT_FP64)
    g32 = lt.ltriples_backward(t, dom.dims, lt.LT_FP32)
    e0, _ = lt.ltriples_energy(t, dom.dims, lt.LT_FP64)
    torch.cuda.synchronize()
    E0 = float(e0.item())
    for k in ALL_GRAD:
        a, b = g64[k], g32[k]
        if a.numel():
            assert float((a - b).abs().max()) <= 1e-5 * float(a.abs().max()), k
    rng = np.random.default_rng(9)

    def fd(dirs, h):
        tp = dict(t); tm = dict(t)
        for k, d in dirs.items():
            tp[k] = t[k] + h * d
            tm[k] = t[k] - h * d
        ep, _ = lt.ltriples_energy(tp, dom.dims, lt.LT_FP64)
        em, _ = lt.ltriples_energy(tm, dom.dims, lt.LT_FP64)
        torch.cuda.synchronize()
        return (float(ep.item()) - float(em.item())) / (2 * h)
    dirs = {}
    for k in ("t1a", "t1b", "t2aa", "t2ab"):
        x = getattr(dom, k)
        d = rng.normal(0.0, 1.0, size=x.shape) * np.std(x)
        if k == "t2aa":
            d = d - d.transpose(1, 0, 2, 3)
            d = d - d.transpose(0, 1, 3, 2)
        dirs[k] = torch.from_numpy(d).cuda()
    an = sum(float((g64[k] * d).sum()) for k, d in dirs.items())
    num = fd(dirs, 0.25)
    assert abs(an - num) <= 1e-9 * max(abs(num), 1e-12 * abs(E0)), (an, num)
    fdirs = {k: torch.from_numpy(rng.normal(0.0, 1.0, size=getattr(dom, k).shape)).cuda()
             for k in ("fov_a", "fov_b")}
    an = sum(float((g64[k] * d).sum()) for k, d in fdirs.items())
    num = fd(fdirs, 1.0)
    assert abs(an - num) <= 1e-9 * max(abs(num), 1e-12 * abs(E0)), ("fov", an, num)
    eps = ("eo_a", "ev_a", "eo_b", "ev_b")
    tot = sum(float(g64[k].sum()) for k in eps)
    mag = sum(float(g64[k].abs().sum()) for k in eps)
    assert abs(tot) <= 1e-10 * mag, (tot, mag)
    euler = sum(float((t[k] * g64[k]).sum()) for k in eps)
    assert abs(euler + E0) <= 1e-10 * abs(E0), (euler, E0)
