"""Forward parity at the full LNO-sized domain (40,38,300,302,1200) in the
launch configuration the benchmark times: the whole domain in BF16X3 with the
default batching.  The oracle cannot run the whole domain in seconds, so the
check is (a) the per-triplet energies of a stratified sample against the FP64
CPU oracle, (b) the same sample through the FP64 GPU path, and (c) properties
that hold at any size: every triplet's energy is written, and E and the
per-block parts equal the sums of the per-triplet energies."""
import math

import numpy as np
import pytest

import paper_2311_10048_amd as lt
import synth
from oracle import blocks
from tests.gpu_util import to_device

pytestmark = pytest.mark.gpu

TOL_ITEM = {lt.LT_BF16X3: 1e-6, lt.LT_FP64: 1e-11}


def test_lno_whole_domain_bf16x3_sampled_items():
    import torch
    torch.cuda.empty_cache()          # blocks cached by earlier tests
    dom = synth.config_domain("lno")
    print(f"[full] lno {dom.dims}: whole domain, BF16X3", flush=True)
    t = to_device(dom)
    d = lt.make_domain(dom.dims, t)
    _, n_all = lt.ltriples_flops(d, None)
    e_items = torch.full((n_all, 3), float("nan"), dtype=torch.float64, device="cuda")
    E, parts = lt.ltriples_energy(t, dom.dims, lt.LT_BF16X3, e_items=e_items)
    torch.cuda.synchronize()
    E, parts, ei = float(E.item()), parts.cpu().numpy(), e_items.cpu().numpy()

    # (c) every triplet written; E and the parts are the sums of the per-triplet energies
    assert np.isfinite(ei).all()
    lists = synth._block_lists(dom.noa, dom.nob)
    sizes = [len(x) for x in lists]
    assert sum(sizes) == n_all
    first = np.cumsum([0] + sizes)
    for b in range(4):
        blk = ei[first[b]:first[b + 1]]
        for k in range(3):
            ref = math.fsum(blk[:, k])
            assert abs(parts[b][k] - ref) <= 1e-12 * max(abs(ref), 1e-300) + 1e-18, (b, k, parts[b][k], ref)
    tot = math.fsum(ei.ravel())
    assert abs(E - tot) <= 1e-12 * abs(tot), (E, tot)

    # (a) stratified sample against the FP64 CPU oracle, (b) and through the FP64 GPU path
    items = synth.sample_items(dom.noa, dom.nob, 2, seed=4242)
    pos = {r: n for n, r in enumerate(r for lst in lists for r in lst)}
    idx = np.asarray([pos[tuple(int(x) for x in r)] for r in items])
    print(f"[full] oracle on {len(items)} sampled triplets", flush=True)
    ref = blocks.energy(dom, items=items, return_items=True)["items"]
    e64 = torch.full((len(items), 3), float("nan"), dtype=torch.float64, device="cuda")
    lt.ltriples_energy(t, dom.dims, lt.LT_FP64, items=items, e_items=e64)
    torch.cuda.synchronize()
    e64 = e64.cpu().numpy()
    for n in range(len(items)):
        r = ref[n].sum()
        s = max(1.0, abs(r))
        assert abs(ei[idx[n]].sum() - r) <= TOL_ITEM[lt.LT_BF16X3] * s, (items[n], ei[idx[n]], ref[n])
        assert abs(e64[n].sum() - r) <= TOL_ITEM[lt.LT_FP64] * s, (items[n], e64[n], ref[n])


def test_large_domain_bf16x3_on_one_gpu_sampled_items():
    """The largest domain (60,58,500,502,2000) in BF16X3 on one GPU (chunked
    operand builds keep workspace and inputs within its memory), on a
    stratified sample of 8 triplets per spin block (32 in all, spread over
    the occupied ranges).  Every sampled triplet against the FP32 GPU path
    (a different contraction kernel, itself held to the oracle at 1e-8 on the
    smaller shapes) at the BF16x3 bar, and 2 per block against the FP64 CPU
    oracle (the oracle needs about ten seconds per triplet at this size).
    Contractions here have M = 500 or 502, i.e. two row tiles."""
    import torch
    torch.cuda.empty_cache()          # blocks cached by earlier tests
    dom = synth.config_domain("large")
    items = synth.sample_items(dom.noa, dom.nob, 8, seed=5151)
    print(f"[full] large {dom.dims}: BF16X3, {len(items)} sampled triplets", flush=True)
    t = to_device(dom)
    res = {}
    for prec in (lt.LT_BF16X3, lt.LT_FP32):
        ei = torch.full((len(items), 3), float("nan"), dtype=torch.float64, device="cuda")
        E, parts = lt.ltriples_energy(t, dom.dims, prec, items=items, e_items=ei)
        torch.cuda.synchronize()
        res[prec] = (float(E.item()), ei.cpu().numpy())
        del ei
        torch.cuda.empty_cache()
        print(f"[full] large prec={prec} done", flush=True)
    del t
    torch.cuda.empty_cache()
    E, ei = res[lt.LT_BF16X3]
    e32 = res[lt.LT_FP32][1]
    assert np.isfinite(ei).all() and np.isfinite(e32).all()
    assert abs(E - math.fsum(ei.ravel())) <= 1e-12 * abs(E)
    for n in range(len(items)):
        r = e32[n].sum()
        assert abs(ei[n].sum() - r) <= TOL_ITEM[lt.LT_BF16X3] * max(1.0, abs(r)), (items[n], ei[n], e32[n])
    # the oracle on the first two sampled triplets of each block
    blk = np.asarray(items)[:, 0]
    sel = np.concatenate([np.flatnonzero(blk == b)[:2] for b in range(4)])
    print(f"[full] oracle on {len(sel)} of the sampled triplets", flush=True)
    ref = blocks.energy(dom, items=np.asarray(items)[sel], return_items=True)["items"]
    for m, n in enumerate(sel):
        r = ref[m].sum()
        assert abs(ei[n].sum() - r) <= TOL_ITEM[lt.LT_BF16X3] * max(1.0, abs(r)), (items[n], ei[n], ref[m])
