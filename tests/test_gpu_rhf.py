"""GPU parity of the closed-shell entry points (ltriples_energy_rhf, the
spin-adapted path, and ltriples_energy_rhf_spin_block) through the C ABI.

Reference: the oracle's independent closed-shell (T) formula over spatial
orbitals (oracle.rhf, pinned on the CPU against the spin-orbital brute force
and the spin-block energy with identical alpha and beta data).  Bars as the
open-shell parity tests, relative to max(1 Eh, |E|): FP64 1e-11, FP32 1e-8,
BF16x3 1e-6 on E; the parts E_ST and E_DT against their own magnitude
(1e-10, 1e-4, 1e-3).  The call must also agree with the open-shell call on
the same alpha == beta data.
"""
import numpy as np
import pytest

import paper_2311_10048_amd as lt
import synth
from oracle import rhf
from tests.gpu_util import to_device

pytestmark = pytest.mark.gpu

TOL_E = {lt.LT_FP64: 1e-11, lt.LT_FP32: 1e-8, lt.LT_BF16X3: 1e-6}
TOL_PART = {lt.LT_FP64: 1e-10, lt.LT_FP32: 1e-4, lt.LT_BF16X3: 1e-3}

SHAPES = {
    "small": (4, 21, 40),      # one epilogue tile plus a ragged one
    "ragged": (6, 45, 96),     # several tiles, ragged tails
    "two_occ": (2, 17, 30),    # no aaa items, aab only
    "wide": (3, 70, 64),       # v > 64: several GEMM tiles
}
_REF = {}


def _rhf_dev(dom):
    import torch
    return {k: torch.from_numpy(np.ascontiguousarray(v)).cuda() for k, v in synth.rhf_arrays(dom).items()}


def _dom(shape):
    # T1 and f_ov larger than the workload recipe so that E_ST and E_DT are
    # well above the rounding of E4
    return synth.make_rhf_domain(*shape, seed=synth.BASE_SEED + 23, sigma_f=3e-2, sigma_t1=3e-2)


def _gpu(dom, prec, **kw):
    import torch
    e, parts = lt.ltriples_energy_rhf(_rhf_dev(dom), (dom.noa, dom.nva, dom.naux), prec, **kw)
    torch.cuda.synchronize()
    return float(e.item()), parts.cpu().numpy()


@pytest.mark.parametrize("prec", [lt.LT_FP64, lt.LT_FP32, lt.LT_BF16X3])
@pytest.mark.parametrize("name", list(SHAPES))
def test_rhf_parity_shapes(name, prec):
    dom = _dom(SHAPES[name])
    print(f"[rhf] {name} {SHAPES[name]} prec={prec}", flush=True)
    if name not in _REF:
        _REF[name] = rhf.energy(dom)
    ref = _REF[name]
    E, parts = _gpu(dom, prec)
    scale = max(1.0, abs(ref["E"]))
    assert abs(E - ref["E"]) <= TOL_E[prec] * scale, (E, ref["E"])
    assert abs(parts[0] - ref["E4"]) <= 10 * TOL_E[prec] * max(1.0, abs(ref["E4"])), (parts[0], ref["E4"])
    for x, key in ((1, "E_ST"), (2, "E_DT")):
        assert abs(parts[x] - ref[key]) <= TOL_PART[prec] * abs(ref[key]) + 1e-300, (key, parts[x], ref[key])


def test_rhf_matches_open_shell_call_on_identical_spins():
    """E = 2 E_aaa + 2 E_aab: the open-shell call on the alpha == beta data
    returns the same energy (its bbb and abb blocks equal aaa and aab)."""
    import torch
    dom = _dom(SHAPES["ragged"])
    E, parts = _gpu(dom, lt.LT_FP64)
    e2, p2 = lt.ltriples_energy(to_device(dom), dom.dims, lt.LT_FP64)
    torch.cuda.synchronize()
    p2 = p2.cpu().numpy()
    assert abs(E - float(e2.item())) <= 1e-13 * abs(E)
    assert np.allclose(p2[0], p2[3], rtol=1e-13, atol=0) and np.allclose(p2[1], p2[2], rtol=1e-13, atol=0)
    assert np.allclose(parts, p2.sum(axis=0), rtol=1e-12, atol=0)


def test_rhf_degenerate_shapes_give_zero():
    """One doubly occupied orbital has no triples; no virtuals or no
    occupied orbitals give nothing either."""
    import torch
    for shape in ((1, 10, 20), (3, 0, 10), (0, 5, 10)):
        dom = synth.make_rhf_domain(*shape, seed=3)
        e, parts = lt.ltriples_energy_rhf(_rhf_dev(dom), shape, lt.LT_FP64)
        torch.cuda.synchronize()
        assert float(e.item()) == 0.0 and not parts.cpu().numpy().any(), shape


def test_rhf_batching_and_chunks_bitwise():
    """Small batches and 1 MiB build chunks give the same bits as the
    defaults (fixed reduction order)."""
    dom = _dom(SHAPES["wide"])
    E0, p0 = _gpu(dom, lt.LT_FP32)
    E1, p1 = _gpu(dom, lt.LT_FP32, build_chunk_mib=1)
    assert E0 == E1 and np.array_equal(p0, p1)
    E2, p2 = _gpu(dom, lt.LT_FP32, batch_items=2)
    assert abs(E2 - E0) <= 1e-12 * abs(E0)


def test_spin_adapted_matches_spin_block_path():
    """The two closed-shell GPU paths (spin-adapted contractions over
    spatial orbitals; spin-block reuse with identical spins) on the same
    data, FP64: E and every part within 1e-12 relative of each other."""
    for name in ("ragged", "two_occ"):
        dom = _dom(SHAPES[name])
        E0, p0 = _gpu(dom, lt.LT_FP64)
        E1, p1 = _gpu(dom, lt.LT_FP64, method="spin_block")
        assert abs(E0 - E1) <= 1e-12 * abs(E1), (name, E0, E1)
        assert np.allclose(p0, p1, rtol=1e-11, atol=0), (name, p0, p1)


def test_rhf_forced_tiles_and_autotune_change_no_bit():
    """Forced contraction tiles (tile_override[0]) and the autotuner change
    no bit of the spin-adapted energy (every tile sums the same segments in
    the same order)."""
    dom = _dom(SHAPES["wide"])
    for prec in (lt.LT_FP32, lt.LT_BF16X3, lt.LT_FP64):
        E0, p0 = _gpu(dom, prec)
        for kw in ({"tile_override": (1, 0, 0)}, {"tile_override": (3, 0, 0)}, {"autotune": True}):
            E1, p1 = _gpu(dom, prec, **kw)
            assert E0 == E1 and np.array_equal(p0, p1), (prec, kw)


def test_rhf_check_finite_rejects_nan():
    import torch
    dom = _dom(SHAPES["small"])
    t = _rhf_dev(dom)
    t["tau"][1, 2, 3, 4] = float("nan")
    with pytest.raises(lt.LtError) as ei:
        lt.ltriples_energy_rhf(t, (dom.noa, dom.nva, dom.naux), lt.LT_FP64, check_finite=True)
    assert ei.value.code == lt.LT_ENONFINITE
    torch.cuda.synchronize()


def test_rhf_lno_sized_domain_two_paths():
    """The closed-shell LNO-sized workload (40,300,1200): the spin-adapted
    BF16X3 energy against the spin-block BF16X3 path at the BF16x3 bar, and
    the FP32 spin-adapted energy against both at the same bar (the oracle
    would need hours at this size; the FP64 paths are held to it above)."""
    import torch
    torch.cuda.empty_cache()
    dom = synth.rhf_config_domain("rhf")
    t = _rhf_dev(dom)
    dims = (dom.noa, dom.nva, dom.naux)
    print(f"[rhf] lno-sized {dims}", flush=True)
    res = {}
    for key, prec, method in (("sa", lt.LT_BF16X3, "spin_adapted"), ("sb", lt.LT_BF16X3, "spin_block"),
                              ("sa32", lt.LT_FP32, "spin_adapted")):
        e, p = lt.ltriples_energy_rhf(t, dims, prec, method=method)
        torch.cuda.synchronize()
        res[key] = (float(e.item()), p.cpu().numpy())
        torch.cuda.empty_cache()
        print(f"[rhf] {key} done", flush=True)
    E = res["sb"][0]
    for key in ("sa", "sa32"):
        assert abs(res[key][0] - E) <= TOL_E[lt.LT_BF16X3] * max(1.0, abs(E)), (key, res[key][0], E)
    del t
    torch.cuda.empty_cache()


# ---- adjoint ------------------------------------------------------------------------------
from oracle import grad as ograd  # noqa: E402

GTOL = {lt.LT_FP64: 1e-10, lt.LT_FP32: 1e-5, lt.LT_BF16X3: 1e-5}


@pytest.mark.parametrize("prec", [lt.LT_FP64, lt.LT_FP32, lt.LT_BF16X3])
@pytest.mark.parametrize("shape", [(3, 17, 30), (4, 21, 40), (2, 13, 20)])
def test_rhf_backward_parity(shape, prec):
    """Every closed-shell gradient against the oracle's reverse mode over
    the closed-shell formula: max|dg| <= tol * max|g_ref| per input."""
    import torch
    dom = _dom(shape)
    print(f"[rhf-bwd] {shape} prec={prec}", flush=True)
    _, ref = ograd.rhf_energy_and_grad(synth.rhf_arrays(dom))
    g = lt.ltriples_backward_rhf(_rhf_dev(dom), (dom.noa, dom.nva, dom.naux), prec)
    torch.cuda.synchronize()
    for k in lt.RHF_FIELDS:
        r = ref[k]
        if r.size == 0:
            continue
        err = float(np.max(np.abs(g[k].cpu().numpy() - r)))
        assert err <= GTOL[prec] * max(float(np.max(np.abs(r))), 1e-300), (k, err, float(np.max(np.abs(r))))


def test_rhf_backward_gbar_and_partial_outputs():
    import torch
    dom = _dom((3, 17, 30))
    t = _rhf_dev(dom)
    dims = (dom.noa, dom.nva, dom.naux)
    g1 = lt.ltriples_backward_rhf(t, dims, lt.LT_FP64)
    gb = torch.full((1,), -1.5, dtype=torch.float64, device="cuda")
    only = {"tau": torch.empty_like(t["tau"]), "ev": torch.empty_like(t["ev"])}
    g2 = lt.ltriples_backward_rhf(t, dims, lt.LT_FP64, gbar=gb, out=only)
    torch.cuda.synchronize()
    for k in ("tau", "ev"):
        err = float((g2[k] + 1.5 * g1[k]).abs().max())
        assert err <= 1e-13 * float(g1[k].abs().max()), (k, err)


def test_rhf_rejects_bad_denominators():
    """An occupied energy above a virtual one is rejected before any work,
    by the energy and by the adjoint."""
    import torch
    dom = _dom((3, 17, 30))
    t = _rhf_dev(dom)
    t["ev"] = t["ev"].clone()
    t["ev"][0] = float(t["eo"].max().item()) + 0.0   # gap of zero
    dims = (dom.noa, dom.nva, dom.naux)
    with pytest.raises(lt.LtError) as ei:
        lt.ltriples_energy_rhf(t, dims, lt.LT_FP64)
    assert ei.value.code == lt.LT_EDENOM
    with pytest.raises(lt.LtError) as ei:
        lt.ltriples_backward_rhf(t, dims, lt.LT_FP64)
    assert ei.value.code == lt.LT_EDENOM
    torch.cuda.synchronize()
