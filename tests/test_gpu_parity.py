"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle.

Tolerances, relative to max(1 Eh, |E|) (the absolute bars of 1e-8 / 1e-6 Eh
after rescaling E to at most 1 Eh, since E scales exactly with the square of
the amplitudes): FP64 1e-11 on E and every per-block part, FP32 1e-8, BF16x3
1e-6; per-item values at the same bars.  The parts E_ST / E_DT are compared
against their own magnitudes.
"""
import numpy as np
import pytest

import paper_2311_10048_amd as lt
import synth
from oracle import blocks
from tests.gpu_util import gpu_energy, rel, to_device

pytestmark = pytest.mark.gpu

TOL_E = {lt.LT_FP64: 1e-11, lt.LT_FP32: 1e-8, lt.LT_BF16X3: 1e-6}
TOL_PART = {lt.LT_FP64: 1e-10, lt.LT_FP32: 1e-4, lt.LT_BF16X3: 1e-3}

SHAPES = {
    "tiny": synth.SHAPES["tiny"],          # (5,4,30,31,120)
    "ragged": (6, 5, 45, 47, 96),          # several tiles, ragged tails everywhere
    "no_beta_occ": (4, 0, 21, 22, 40),     # only the aaa block
    "one_beta": (3, 1, 17, 18, 30),        # aaa, aab
    "wide": (3, 3, 70, 67, 64),            # v > 64: several GEMM and epilogue tiles
    "tall": (3, 1, 400, 401, 48),          # v > 384: several row tiles per contraction (aaa, aab)
    "no_beta_vir": (4, 3, 20, 0, 30),      # empty beta virtual space: mixed blocks have no C
    "no_alpha_vir": (3, 3, 0, 5, 20),      # empty alpha virtual space: only bbb contributes
    "no_alpha_occ": (0, 4, 21, 22, 40),    # only the bbb block
    "one_alpha_two_beta": (1, 2, 15, 16, 30),   # only the abb block, one item
}
_REF = {}   # oracle results per shape, shared by the three precisions


def _check(dom, prec, ref=None, items=None):
    ref = ref if ref is not None else blocks.energy(dom, items=items, return_items=items is not None)
    E, parts, e_items = gpu_energy(dom, prec, items=items)
    scale = max(1.0, abs(ref["E"]))
    assert abs(E - ref["E"]) / scale <= TOL_E[prec], (E, ref["E"])
    for b in range(4):
        r4, rs, rd = ref["parts"][b]
        g4, gs, gd = parts[b]
        assert abs(g4 - r4) <= TOL_E[prec] * max(1.0, abs(r4)) * 10, (b, g4, r4)
        if rs != 0:
            assert abs(gs - rs) <= TOL_PART[prec] * abs(rs) + 1e-300, (b, gs, rs)
        if rd != 0:
            assert abs(gd - rd) <= TOL_PART[prec] * abs(rd) + 1e-300, (b, gd, rd)
    if items is not None:
        for n in range(len(items)):
            ri, gi = ref["items"][n], e_items[n]
            s = max(1.0, abs(ri[0]))
            assert abs(gi[0] - ri[0]) <= 10 * TOL_E[prec] * s, (n, gi, ri)
    return E, ref["E"]


@pytest.mark.parametrize("prec", [lt.LT_FP64, lt.LT_FP32, lt.LT_BF16X3])
@pytest.mark.parametrize("name", list(SHAPES))
def test_parity_shapes(name, prec):
    dom = synth.make_domain(*SHAPES[name], seed=synth.BASE_SEED + 17)
    print(f"[parity] {name} {SHAPES[name]} prec={prec}", flush=True)
    if name not in _REF:
        _REF[name] = blocks.energy(dom)
    _check(dom, prec, ref=_REF[name])


@pytest.mark.parametrize("prec", [lt.LT_FP64, lt.LT_FP32, lt.LT_BF16X3])
def test_workspace_garbage_never_read(prec):
    """A NaN-filled workspace gives the same result: no never-written word of
    the workspace (row padding included) reaches the energy.  The two spins
    have different padded row lengths here (70 -> 72, 67 -> 68)."""
    dom = synth.make_domain(*SHAPES["wide"], seed=synth.BASE_SEED + 17)
    E0, p0, _ = gpu_energy(dom, prec, ws_fill=0.0)
    E1, p1, _ = gpu_energy(dom, prec, ws_fill=float("nan"))
    assert E0 == E1 and np.array_equal(p0, p1)


@pytest.mark.parametrize("prec", [lt.LT_FP64, lt.LT_FP32, lt.LT_BF16X3])
@pytest.mark.parametrize("name", ["wide", "tall"])
def test_chunked_operand_builds_bitwise_equal(name, prec):
    """Operand builds in 1 MiB chunks of their occupied index (several chunks
    of <ei||bc>, (jb|EC), (be|KC) and the (ov|ov) rows on these shapes) give
    exactly the default result."""
    dom = synth.make_domain(*SHAPES[name], seed=synth.BASE_SEED + 17)
    print(f"[chunks] {name} {SHAPES[name]} prec={prec}", flush=True)
    E0, p0, _ = gpu_energy(dom, prec)
    E1, p1, _ = gpu_energy(dom, prec, build_chunk_mib=1)
    assert E0 == E1 and np.array_equal(p0, p1)


def test_parity_config0_items_fp64():
    """Per-item values of every triplet of the small domain, in caller order."""
    dom = synth.config_domain("tiny")
    items = blocks.enumerate_items(dom.noa, dom.nob)[::-1].copy()
    _check(dom, lt.LT_FP64, items=items)


def test_fewer_than_three_occupied_is_zero():
    dom = synth.make_domain(1, 1, 8, 9, 20, seed=3)
    E, parts, _ = gpu_energy(dom, lt.LT_FP64)
    assert E == 0.0 and np.all(parts == 0.0)


def test_small_batches_bitwise_equal():
    """Batch size does not change a single bit of the result."""
    dom = synth.make_domain(*SHAPES["ragged"], seed=5)
    E1, p1, _ = gpu_energy(dom, lt.LT_FP32)
    E2, p2, _ = gpu_energy(dom, lt.LT_FP32, batch_items=3)
    assert E1 == E2 and np.array_equal(p1, p2)


def test_denominator_check():
    dom = synth.make_domain(3, 2, 6, 7, 16, seed=3)
    bad = dom.replace(eo_a=dom.eo_a + 2.0)
    with pytest.raises(lt.LtError) as ei:
        gpu_energy(bad, lt.LT_FP64)
    assert ei.value.code == lt.LT_EDENOM


@pytest.mark.parametrize("case", ["tiny_gap", "huge_energy"])
def test_denominator_range_check(case):
    """Energies that would put some |D| outside [3e-100, 6e100] are rejected
    before any kernel runs (the epilogues' reciprocal assumes that range)."""
    dom = synth.make_domain(3, 2, 6, 7, 16, seed=3)
    if case == "tiny_gap":
        # occupied energies below the virtual ones, but only 2e-101 apart
        sc = 1e-101
        bad = dom.replace(eo_a=-sc * (1.0 + np.arange(dom.eo_a.size)), eo_b=-sc * (1.0 + np.arange(dom.eo_b.size)),
                          ev_a=sc * (1.0 + np.arange(dom.ev_a.size)), ev_b=sc * (1.0 + np.arange(dom.ev_b.size)))
    else:
        bad = dom.replace(ev_b=dom.ev_b + 1e101)
    with pytest.raises(lt.LtError) as ei:
        gpu_energy(bad, lt.LT_FP64)
    assert ei.value.code == lt.LT_EDENOM


def test_plain_bf16_ablation_runs():
    """Single-product BF16 (ablation): finite and within 1e-3 of the oracle
    on the ragged shape; reported, not a precision claim."""
    dom = synth.make_domain(*SHAPES["ragged"], seed=synth.BASE_SEED + 17)
    ref = blocks.energy(dom)
    E, parts, _ = gpu_energy(dom, lt.LT_BF16)
    assert np.isfinite(E)
    assert abs(E - ref["E"]) / abs(ref["E"]) < 1e-3


@pytest.mark.parametrize("prec", [lt.LT_BF16X3, lt.LT_FP32, lt.LT_FP64])
@pytest.mark.parametrize("name", ["ragged", "wide", "tall"])
def test_autotune_changes_no_bit(name, prec):
    """Tile-shape tuning picks among configurations that sum every output in
    the same order: the energies, parts and per-item values are bitwise
    those of the default configurations, on the tuning call and after it."""
    import torch
    dom = synth.make_domain(*SHAPES[name], seed=synth.BASE_SEED + 17)
    t = to_device(dom)
    items = synth.sample_items(dom.noa, dom.nob, 3, seed=5)
    lt.ltriples_autotune_reset()
    outs = []
    for tune in (False, True, False):
        ei = torch.zeros(len(items), 3, dtype=torch.float64, device="cuda")
        e, p = lt.ltriples_energy(t, dom.dims, prec, autotune=tune)
        lt.ltriples_energy(t, dom.dims, prec, items=items, e_items=ei, autotune=tune)
        torch.cuda.synchronize()
        outs.append((e.cpu().numpy(), p.cpu().numpy(), ei.cpu().numpy()))
    lt.ltriples_autotune_reset()
    for o in outs[1:]:
        for a, b in zip(outs[0], o):
            assert np.array_equal(a, b)


@pytest.mark.parametrize("prec", [lt.LT_FP64, lt.LT_BF16X3])
def test_item_order_changes_no_bit(prec):
    """The same item set in a shuffled order gives bitwise the same energy
    and parts, and each item's value at its caller position."""
    dom = synth.make_domain(*SHAPES["ragged"], seed=synth.BASE_SEED + 17)
    items = np.asarray(synth.sample_items(dom.noa, dom.nob, 6, seed=3)).reshape(-1, 4)
    perm = np.random.default_rng(4).permutation(len(items))
    t = to_device(dom)
    E1, p1, e1 = gpu_energy(dom, prec, items=items, tensors=t)
    E2, p2, e2 = gpu_energy(dom, prec, items=items[perm], tensors=t)
    assert E1 == E2 and np.array_equal(p1, p2)
    assert np.array_equal(e1[perm], e2)


def test_workspace_too_small_and_nonfinite_energies():
    """LT_EWORKSPACE for a caller workspace one byte short, LT_ENONFINITE
    for a NaN orbital energy; both before any work is enqueued."""
    import torch
    dom = synth.config_domain("tiny")
    t = to_device(dom)
    d = lt.make_domain(dom.dims, t)
    need = lt.ltriples_workspace_size(d, lt.LT_FP32)
    ws = torch.empty(need - 1, dtype=torch.uint8, device="cuda")
    with pytest.raises(lt.LtError) as ei:
        lt.ltriples_energy(t, dom.dims, lt.LT_FP32, workspace=ws)
    assert ei.value.code == lt.LT_EWORKSPACE
    t2 = dict(t)
    t2["eo_b"] = t["eo_b"].clone()
    t2["eo_b"][1] = float("nan")
    with pytest.raises(lt.LtError) as ei:
        lt.ltriples_energy(t2, dom.dims, lt.LT_FP32)
    assert ei.value.code == lt.LT_ENONFINITE
    e, _ = lt.ltriples_energy(t, dom.dims, lt.LT_FP32)      # the library is still usable
    torch.cuda.synchronize()
    assert np.isfinite(float(e.item()))
