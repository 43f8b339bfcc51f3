"""The no-allocation entry point (ltriples_energy_noalloc) through the C ABI
against ltriples_energy on the same inputs: two calls in a row on one GPU,
the second on a smaller domain, each bitwise equal to the allocating entry
point (same kernels; the refitted batches and build chunks change no bit).
The fixed per-device array keeps the previous call's contents, so the
second, smaller call also checks that nothing stale reaches a result."""
import numpy as np
import pytest

import paper_2311_10048_amd as lt
import synth
from tests.gpu_util import to_device

pytestmark = pytest.mark.gpu

# (first, second) domains of each pair; the first is the larger one
PAIRS = {
    lt.LT_FP64: ((6, 5, 45, 47, 96), (5, 4, 30, 31, 120)),
    lt.LT_FP32: ((10, 9, 80, 81, 320), (6, 5, 45, 47, 96)),     # the first needs smaller batches to fit
    lt.LT_BF16X3: ((10, 9, 80, 81, 320), (5, 4, 30, 31, 120)),
}


def _reference(t, dims, prec, items=None):
    import torch
    n_it = None if items is None else len(items)
    ei = None if n_it is None else torch.full((n_it, 3), float("nan"), dtype=torch.float64, device="cuda")
    e, p = lt.ltriples_energy(t, dims, prec, items=items, e_items=ei)
    torch.cuda.synchronize()
    return e.cpu().numpy(), p.cpu().numpy(), None if ei is None else ei.cpu().numpy()


def _noalloc(t, dims, prec, items=None):
    import torch
    n_it = None if items is None else len(items)
    ei = None if n_it is None else torch.full((n_it, 3), float("nan"), dtype=torch.float64, device="cuda")
    out = (torch.full((1,), float("nan"), dtype=torch.float64, device="cuda"),
           torch.full((4, 3), float("nan"), dtype=torch.float64, device="cuda"))
    e, p = lt.ltriples_energy_noalloc(t, dims, prec, items=items, e_items=ei, out=out)
    torch.cuda.synchronize()
    return e.cpu().numpy(), p.cpu().numpy(), None if ei is None else ei.cpu().numpy()


@pytest.mark.parametrize("prec", [lt.LT_FP64, lt.LT_FP32, lt.LT_BF16X3])
def test_noalloc_matches_energy_two_calls(prec):
    import torch
    big, small = PAIRS[prec]
    print(f"[noalloc] prec={prec} first {big}, then {small}", flush=True)
    dom1 = synth.make_domain(*big, seed=synth.BASE_SEED + 31)
    dom2 = synth.make_domain(*small, seed=synth.BASE_SEED + 32)
    t1, t2 = to_device(dom1), to_device(dom2)
    items2 = synth.sample_items(dom2.noa, dom2.nob, 2, seed=7)
    ref1 = _reference(t1, dom1.dims, prec)
    ref2 = _reference(t2, dom2.dims, prec, items=items2)
    got1 = _noalloc(t1, dom1.dims, prec)
    got2 = _noalloc(t2, dom2.dims, prec, items=items2)
    for ref, got in ((ref1, got1), (ref2, got2)):
        assert np.isfinite(got[0]).all() and np.isfinite(got[1]).all()
        assert np.array_equal(ref[0], got[0]), (ref[0], got[0])
        assert np.array_equal(ref[1], got[1])
    assert np.array_equal(ref2[2], got2[2])
    # the library's array holds the last call's contents; a repeat of the
    # first call after the second still gives the same bits
    again = _noalloc(t1, dom1.dims, prec)
    assert np.array_equal(ref1[0], again[0]) and np.array_equal(ref1[1], again[1])
    del t1, t2
    torch.cuda.empty_cache()


def test_noalloc_refuses_stats_autotune_and_oversized_domains():
    """Arguments that would need an allocation, and domains that do not fit
    the fixed array even in single-item batches, are refused before any work
    is enqueued; the entry point stays usable afterwards."""
    import torch
    dom = synth.config_domain("tiny")
    t = to_device(dom)
    with pytest.raises(lt.LtError) as ei:
        lt.ltriples_energy_noalloc(t, dom.dims, lt.LT_FP64, tile_override=(0, 0, 9))
    assert ei.value.code == lt.LT_EINVAL
    lib = lt.load_library()
    d = lt.make_domain(dom.dims, t)
    e = torch.empty(1, dtype=torch.float64, device="cuda")
    o, _ = lt.make_options(autotune=True)
    assert lib.ltriples_energy_noalloc(lt.ctypes.byref(d), lt.LT_FP64, lt.ctypes.byref(o), e.data_ptr(), None,
                                       None) == lt.LT_EINVAL
    big = synth.SHAPES["grad"]
    sizes = lt.domain_sizes(big)
    tb = {f: torch.zeros(max(sizes[f], 1), dtype=torch.float64, device="cuda") for f in lt.ARRAY_FIELDS}
    db = lt.make_domain(big, tb)
    assert lib.ltriples_energy_noalloc(lt.ctypes.byref(db), lt.LT_BF16X3, None, e.data_ptr(), None,
                                       None) == lt.LT_EWORKSPACE
    del tb
    assert "no-allocation" in lt.ltriples_last_error()
    got = _noalloc(t, dom.dims, lt.LT_FP64)
    ref = _reference(t, dom.dims, lt.LT_FP64)
    assert np.array_equal(ref[0], got[0]) and np.array_equal(ref[1], got[1])
