"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle.

Tolerances, relative to max(1 Eh, |E|) (the absolute bars of 1e-8 / 1e-6 Eh
after rescaling E to at most 1 Eh, since E scales exactly with the square of
the amplitudes): FP64 1e-11, FP32 1e-8, BF16x3 1e-6, on E and on every
block's E4.  The parts E_ST / E_DT are compared against their own magnitudes
(FP64 1e-10, FP32 1e-4, BF16x3 1e-3).  Per-item values: FP64 every part of
every item relative to its own magnitude (E4 1e-11, E_ST and E_DT 1e-10);
FP32 and BF16x3 each item's energy at the E bar of max(1, |E_item|) and its
E_ST / E_DT parts at the part bars relative to the larger of their own
magnitude and the root mean square of that part over the block's items (a
single item's E_ST or E_DT can cancel to far below its terms, and the
rounding of the reduced-precision W scales with the terms).
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
        assert abs(g4 - r4) <= TOL_E[prec] * max(1.0, abs(r4)), (b, g4, r4)
        if rs != 0:
            assert abs(gs - rs) <= TOL_PART[prec] * abs(rs) + 1e-300, (b, gs, rs)
        if rd != 0:
            assert abs(gd - rd) <= TOL_PART[prec] * abs(rd) + 1e-300, (b, gd, rd)
    if items is not None:
        check_items(ref["items"], e_items, prec, np.asarray(items)[:, 0])
    return E, ref["E"]


def check_items(ref_items, got_items, prec, blocks_of=None):
    """Per-item parity at the bars of the module docstring; `blocks_of`
    gives each item's block (for the reduced-precision part scales)."""
    rms = np.zeros((4, 3))
    blk = np.zeros(len(ref_items), dtype=int) if blocks_of is None else np.asarray(blocks_of)
    for b in range(4):
        sel = ref_items[blk == b]
        if len(sel):
            rms[b] = np.sqrt(np.mean(sel ** 2, axis=0))
    for n in range(len(ref_items)):
        ri, gi = ref_items[n], got_items[n]
        if prec == lt.LT_FP64:
            assert abs(gi[0] - ri[0]) <= 1e-11 * abs(ri[0]) + 1e-300, (n, 0, gi, ri)
            for k in (1, 2):
                assert abs(gi[k] - ri[k]) <= 1e-10 * abs(ri[k]) + 1e-300, (n, k, gi, ri)
        else:
            e_r, e_g = ri.sum(), gi.sum()
            assert abs(e_g - e_r) <= TOL_E[prec] * max(1.0, abs(e_r)), (n, gi, ri)
            for k in (1, 2):
                scale = max(abs(ri[k]), rms[blk[n], k])
                assert abs(gi[k] - ri[k]) <= TOL_PART[prec] * scale, (n, k, gi, ri, scale)


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


@pytest.mark.parametrize("prec", [lt.LT_FP64, lt.LT_FP32, lt.LT_BF16X3])
def test_parity_config0_items(prec):
    """Per-item values {E4, E_ST, E_DT} of every triplet of the small domain,
    in caller order (reversed), at the per-item bars."""
    dom = synth.config_domain("tiny")
    items = blocks.enumerate_items(dom.noa, dom.nob)[::-1].copy()
    _check(dom, prec, items=items)


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


@pytest.mark.parametrize("prec", [lt.LT_BF16X3, lt.LT_FP32, lt.LT_FP64])
def test_forced_tiles_change_no_bit(prec):
    """options.tile_override forces one configuration of the precision's
    table per output layout; every configuration sums each output element in
    the same order, so energies, parts and per-item values are bitwise those
    of the automatic choice."""
    import torch
    dom = synth.make_domain(*SHAPES["ragged"], seed=synth.BASE_SEED + 17)
    t = to_device(dom)
    items = synth.sample_items(dom.noa, dom.nob, 3, seed=5)
    outs = []
    for force in ((0, 0, 0), (1, 2, 3), (4, 5, 6), (8, 7, 8)):
        ei = torch.zeros(len(items), 3, dtype=torch.float64, device="cuda")
        e, p = lt.ltriples_energy(t, dom.dims, prec, items=items, e_items=ei, tile_override=force)
        torch.cuda.synchronize()
        outs.append((e.cpu().numpy(), p.cpu().numpy(), ei.cpu().numpy()))
    for o in outs[1:]:
        for a, b in zip(outs[0], o):
            assert np.array_equal(a, b)


def test_check_finite_scans_every_input():
    """With options.check_finite a NaN or an infinity anywhere in the inputs
    gives LT_ENONFINITE (found on the device before any other work); clean
    inputs give the usual result, bitwise."""
    import torch
    dom = synth.config_domain("tiny")
    t = to_device(dom)
    e0, p0 = lt.ltriples_energy(t, dom.dims, lt.LT_FP64)
    e1, p1 = lt.ltriples_energy(t, dom.dims, lt.LT_FP64, check_finite=True)
    torch.cuda.synchronize()
    assert float(e0.item()) == float(e1.item()) and torch.equal(p0, p1)
    for k, val in (("t2ab", float("nan")), ("Bvv_b", float("inf")), ("fov_a", float("-inf")), ("t1b", float("nan"))):
        bad = dict(t)
        bad[k] = t[k].clone()
        bad[k].view(-1)[bad[k].numel() // 2] = val
        with pytest.raises(lt.LtError) as ei:
            lt.ltriples_energy(bad, dom.dims, lt.LT_FP32, check_finite=True)
        assert ei.value.code == lt.LT_ENONFINITE, k
        # without the scan such a value flows through (only the orbital energies are always checked)
        e, _ = lt.ltriples_energy(bad, dom.dims, lt.LT_FP32)
        torch.cuda.synchronize()
        assert not np.isfinite(float(e.item())), k


def test_tune_cache_file_round_trip(tmp_path):
    """LTRIPLES_TUNE_CACHE: a process that tunes writes its choices to the
    file, and a fresh process reads them back and uses them without tuning
    (same result bits either way)."""
    import json
    import os
    import subprocess
    import sys
    cache = tmp_path / "tune.json"
    code = (
        "import sys, torch, numpy as np\n"
        "sys.path.insert(0, %r)\n"
        "import paper_2311_10048_amd as lt, synth\n"
        "from tests.gpu_util import to_device\n"
        "dom = synth.make_domain(6, 5, 45, 47, 96, seed=3)\n"
        "t = to_device(dom)\n"
        "e, p = lt.ltriples_energy(t, dom.dims, lt.LT_BF16X3, autotune=%s)\n"
        "torch.cuda.synchronize()\n"
        "print(repr(float(e.item())))\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, LTRIPLES_TUNE_CACHE=str(cache), LTRIPLES_LOG="1")
    r1 = subprocess.run([sys.executable, "-c", code % (root, "True")], capture_output=True, text=True, env=env,
                        timeout=300)
    assert r1.returncode == 0, r1.stderr[-3000:]
    data = json.loads(cache.read_text())
    assert data["entries"] and all(e["family"] == "bf16" for e in data["entries"])
    r2 = subprocess.run([sys.executable, "-c", code % (root, "True")], capture_output=True, text=True, env=env,
                        timeout=300)
    assert r2.returncode == 0, r2.stderr[-3000:]
    assert "tuned BF16 contraction" in r1.stderr
    assert "tuned BF16 contraction" not in r2.stderr     # every class came from the file
    assert r1.stdout.strip().splitlines()[-1] == r2.stdout.strip().splitlines()[-1]


def test_library_owned_workspace_and_stream_order():
    """ws == NULL: the library allocates the workspace stream-ordered on the
    call's stream and frees it on return (also on an error return); the
    result is bitwise that of a caller workspace.  The orbital energies are
    read in the order of the caller's stream: energies written there just
    before the call (on a side stream that the default stream does not wait
    for) are the ones checked."""
    import ctypes
    import torch
    dom = synth.config_domain("tiny")
    t = to_device(dom)
    lib = lt.load_library()
    d = lt.make_domain(dom.dims, t)
    e_ref, p_ref = lt.ltriples_energy(t, dom.dims, lt.LT_FP64)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    e = torch.empty(1, dtype=torch.float64, device="cuda")
    p = torch.empty(4, 3, dtype=torch.float64, device="cuda")
    for _ in range(3):
        with torch.cuda.stream(s):
            assert lib.ltriples_energy(ctypes.byref(d), lt.LT_FP64, None, e.data_ptr(), p.data_ptr(), None, 0,
                                       s.cuda_stream) == lt.LT_OK
        s.synchronize()
        assert torch.equal(e, e_ref) and torch.equal(p, p_ref)
    # energies made invalid on the side stream right before the call: the check sees them
    eo = t["eo_a"].clone()
    t2 = dict(t)
    t2["eo_a"] = eo
    d2 = lt.make_domain(dom.dims, t2)
    with torch.cuda.stream(s):
        torch.cuda._sleep(20_000_000)                  # keep the side stream busy
        eo.add_(10.0)                                 # occupied energies above the virtual ones
        code = lib.ltriples_energy(ctypes.byref(d2), lt.LT_FP64, None, e.data_ptr(), p.data_ptr(), None, 0,
                                   s.cuda_stream)
    s.synchronize()
    assert code == lt.LT_EDENOM, (code, lt.ltriples_last_error())
    # a failing call with a library workspace leaves the library usable
    with torch.cuda.stream(s):
        assert lib.ltriples_energy(ctypes.byref(d), lt.LT_FP64, None, e.data_ptr(), p.data_ptr(), None, 0,
                                   s.cuda_stream) == lt.LT_OK
    s.synchronize()
    assert torch.equal(e, e_ref)
