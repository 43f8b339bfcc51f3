"""Launch groups of ltriples_energy_batched (options.group_budget): domains
packed, longest first, into groups whose contraction launches take one item
batch of every domain of the group.

A domain's batches, epilogues and reductions do not depend on the launch it
shares, so every energy and part must be bitwise those of the ungrouped call
and of the single-domain call, in every precision, for every budget (one
group, groups split by bytes, groups split by the 16-domain cap, a budget
below every domain), eager and replayed from a captured graph."""
import numpy as np
import pytest

import paper_2311_10048_amd as lt
import synth
from oracle import blocks
from tests.gpu_util import to_device

pytestmark = pytest.mark.gpu

TOL_E = {lt.LT_FP64: 1e-11, lt.LT_FP32: 1e-8, lt.LT_BF16X3: 1e-6}

# uneven domains, degenerate ones included: a single beta orbital, fewer than
# three occupied orbitals (zero energy), an empty beta virtual space, only the
# bbb block
SHAPES = [(5, 4, 30, 31, 120), (3, 1, 17, 18, 30), (6, 5, 45, 47, 96), (2, 0, 9, 10, 12), (4, 4, 26, 22, 50),
          (4, 3, 20, 0, 30), (0, 4, 21, 22, 40), (6, 4, 38, 40, 80)]


def _doms(shapes, seed0):
    return [synth.make_domain(*s, seed=synth.BASE_SEED + seed0 + n) for n, s in enumerate(shapes)]


def _run(tens, dims, prec, budget, **kw):
    import torch
    e, p = lt.ltriples_energy_batched(tens, dims, prec, group_budget=budget, **kw)
    torch.cuda.synchronize()
    return e.cpu().numpy(), p.cpu().numpy()


@pytest.mark.parametrize("prec", [lt.LT_BF16X3, lt.LT_BF16, lt.LT_FP32, lt.LT_FP64])
def test_groups_bitwise_equal_ungrouped_and_single(prec):
    import torch
    doms = _doms(SHAPES, 400)
    tens = [to_device(d) for d in doms]
    dims = [d.dims for d in doms]
    print(f"[groups] prec={prec} shapes={SHAPES}", flush=True)
    e0, p0 = _run(tens, dims, prec, 0)
    # region sizes decide the packing: one group, a split by bytes, one domain per group
    sizes = sorted(lt.ltriples_workspace_size(lt.make_domain(d, t), prec) for d, t in zip(dims, tens))
    for budget in (1 << 50, sizes[-1] + sizes[-2] // 2, 1):
        e, p = _run(tens, dims, prec, budget)
        print(f"[groups] prec={prec} budget={budget}", flush=True)
        assert np.array_equal(e, e0), (budget, e, e0)
        assert np.array_equal(p, p0), budget
    for n in range(len(doms)):
        e1, p1 = lt.ltriples_energy(tens[n], dims[n], prec)
        torch.cuda.synchronize()
        assert e0[n] == float(e1.item()), (n, e0[n], float(e1.item()))
        assert np.array_equal(p0[n], p1.cpu().numpy()), n
    if prec in TOL_E:
        for n, d in enumerate(doms):
            ref = blocks.energy(d)["E"]
            assert abs(e0[n] - ref) <= TOL_E[prec] * max(1.0, abs(ref)), (n, e0[n], ref)
    assert e0[3] == 0.0


def test_groups_beyond_sixteen_domains_and_graph_replays():
    """21 small domains (two groups by the 16-domain cap) in BF16X3: bitwise
    the ungrouped result, eager and on three graph replays with the inputs
    changed in place between them."""
    import torch
    lt.ltriples_graph_reset()
    rng = np.random.default_rng(5)
    shapes = []
    for _ in range(21):
        no = int(rng.integers(3, 7))
        nv = int(rng.integers(12, 40))
        shapes.append((no, no - 1, nv, nv + 1, 3 * nv))
    doms = _doms(shapes, 500)
    tens = [to_device(d) for d in doms]
    dims = [d.dims for d in doms]
    prec = lt.LT_BF16X3
    budget = 1 << 50
    opts, _ = lt.make_options(group_budget=budget)
    ws = torch.empty(lt.ltriples_workspace_size_batched(dims, tens, prec, opts), dtype=torch.uint8, device="cuda")
    out = (torch.empty(len(doms), dtype=torch.float64, device="cuda"),
           torch.empty(len(doms), 4, 3, dtype=torch.float64, device="cuda"))
    base_t1 = [t["t1a"].clone() for t in tens]
    for rep in range(3):
        for n, t in enumerate(tens):
            t["t1a"].copy_(base_t1[n] * (1.0 + 0.25 * rep))
        out[0].fill_(float("nan"))
        print(f"[groups] 21 domains, graph replay {rep}", flush=True)
        lt.ltriples_energy_batched(tens, dims, prec, graph=True, workspace=ws, out=out, group_budget=budget)
        torch.cuda.synchronize()
        got_e, got_p = out[0].cpu().numpy().copy(), out[1].cpu().numpy().copy()
        e0, p0 = _run(tens, dims, prec, 0)
        eg, pg = _run(tens, dims, prec, budget)
        assert np.array_equal(eg, e0) and np.array_equal(pg, p0), rep
        assert np.array_equal(got_e, e0) and np.array_equal(got_p, p0), rep
    lt.ltriples_graph_reset()


def test_groups_on_small_domains_of_the_batch_set():
    """The eight smallest domains (by flop count) of the 64-domain set in one
    BF16X3 group: bitwise the ungrouped call, and within 1e-6 of the FP64
    ungrouped call."""
    shapes = synth.batch_shapes()
    F = []
    for n, s in enumerate(shapes):
        d = lt.make_domain(s, {f: (1 << 40) for f in lt.ARRAY_FIELDS})   # sizes only, never dereferenced
        F.append((lt.ltriples_flops(d)[0], n))
    F.sort()
    pick = [n for _, n in F[:8]]
    doms = [synth.batch_domain(n, shapes) for n in pick]
    dims = [d.dims for d in doms]
    print(f"[groups] set domains {pick}: {dims}", flush=True)
    tens = [to_device(d) for d in doms]
    e0, p0 = _run(tens, dims, lt.LT_BF16X3, 0)
    eg, pg = _run(tens, dims, lt.LT_BF16X3, 1 << 50)
    assert np.array_equal(eg, e0) and np.array_equal(pg, p0)
    e64, _ = _run(tens, dims, lt.LT_FP64, 1 << 50)
    for n in range(len(doms)):
        assert abs(eg[n] - e64[n]) <= TOL_E[lt.LT_BF16X3] * max(1.0, abs(e64[n])), (pick[n], eg[n], e64[n])
