"""Per-item W dumps (ltriples_debug_w) on the small domain (5,4,30,31,120)
against the oracle's W cubes: the connected triples amplitude of the master
formula (eq. cim_pt_energy) element by element, before V and the denominator
enter, for every triplet of every spin block.

W is what the contraction kernels produce; the dump forms it from their
outputs exactly as the energy epilogues read them, so a wrong sign, index or
operand in any contraction term shows here even where it would cancel in E.
Bars, relative to the largest |W| of the item's cube: FP64 1e-12; FP32 1e-5
(about 2v + 2o = 70 terms summed in FP32, each rounding 2^-24); BF16x3 1e-4
(each product keeps about 16 bits of its operands, 2^-16, plus the FP32
accumulation).  The item energy returned with the dump is checked against the
oracle's at the energy bars.
"""
import numpy as np
import pytest

import paper_2311_10048_amd as lt
import synth
from oracle import blocks
from tests.gpu_util import to_device

pytestmark = pytest.mark.gpu

TOL_W = {lt.LT_FP64: 1e-12, lt.LT_FP32: 1e-5, lt.LT_BF16X3: 1e-4}
TOL_E = {lt.LT_FP64: 1e-11, lt.LT_FP32: 1e-8, lt.LT_BF16X3: 1e-6}
_REF = {}


def _reference(dom):
    """Oracle W cube and item energy of every triplet of the domain."""
    if id(dom) in _REF:
        return _REF[id(dom)]
    ints = blocks._Integrals(dom)
    items = [it for lst in synth._block_lists(dom.noa, dom.nob) for it in lst]
    ref = blocks.energy(dom, items=np.asarray(items), return_items=True)["items"]
    out = []
    for n, (b, p, q, r) in enumerate(items):
        if b in (0, 3):
            w = blocks.same_spin_cubes(ints, 0 if b == 0 else 1, p, q, r)[0]
        else:
            w = blocks.mixed_cubes(ints, dom, 0 if b == 1 else 1, p, q, r)[0]
        out.append(((b, p, q, r), w, float(ref[n].sum())))
    _REF[id(dom)] = out
    return out


@pytest.fixture(scope="module")
def tiny():
    dom = synth.config_domain("tiny")
    return dom, to_device(dom)


@pytest.mark.parametrize("prec", [lt.LT_FP64, lt.LT_FP32, lt.LT_BF16X3])
def test_w_dump_every_item_matches_the_oracle(tiny, prec):
    import torch
    dom, t = tiny
    print(f"[wdump] tiny {dom.dims} prec={prec}", flush=True)
    worst = 0.0
    for item, w_ref, e_ref in _reference(dom):
        w, e = lt.ltriples_debug_w(t, dom.dims, item, prec)
        torch.cuda.synchronize()
        w = w.cpu().numpy()
        assert w.shape == w_ref.shape, (item, w.shape, w_ref.shape)
        scale = float(np.max(np.abs(w_ref)))
        assert scale > 0.0, item
        err = float(np.max(np.abs(w - w_ref))) / scale
        worst = max(worst, err)
        assert err <= TOL_W[prec], (item, err)
        assert abs(float(e.item()) - e_ref) <= TOL_E[prec] * max(1.0, abs(e_ref)), (item, float(e.item()), e_ref)
    print(f"[wdump] prec={prec}: worst max|dW|/max|W| = {worst:.3e}", flush=True)


def test_w_dump_is_antisymmetric_and_zero_on_repeated_indices(tiny):
    """Properties of the dump itself (FP64): exact antisymmetry under a swap
    of two virtual indices of equal spin, zeros where they coincide."""
    import torch
    dom, t = tiny
    w, _ = lt.ltriples_debug_w(t, dom.dims, (0, 0, 2, 4), lt.LT_FP64)
    x, _ = lt.ltriples_debug_w(t, dom.dims, (2, 1, 3, 0), lt.LT_FP64)
    torch.cuda.synchronize()
    w, x = w.cpu().numpy(), x.cpu().numpy()
    assert np.array_equal(w, -w.transpose(1, 0, 2)) and np.array_equal(w, -w.transpose(0, 2, 1))
    assert np.array_equal(w, w.transpose(1, 2, 0))
    assert np.array_equal(x, -x.transpose(1, 0, 2))
    v = dom.nva
    idx = np.arange(v)
    assert not np.any(w[idx, idx, :]) and not np.any(w[:, idx, idx]) and not np.any(x[idx, idx, :])


def test_w_dump_rejects_bad_items(tiny):
    dom, t = tiny
    for item in ((0, 0, 0, 1), (1, 0, 1, dom.nob), (4, 0, 1, 2)):
        with pytest.raises((lt.LtError, ValueError)):
            lt.ltriples_debug_w(t, dom.dims, item, lt.LT_FP64)
