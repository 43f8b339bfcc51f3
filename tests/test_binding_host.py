"""Host-side checks of the Python binding's argument checks (no GPU): every
tensor handed to the kernels must be contiguous float64, large enough for
the declared dimensions and resident on the GPU, and the synthetic domains
of every GPU test shape meet the size rule exactly."""
import numpy as np
import pytest
import torch

import paper_2311_10048_amd as lt
import synth
from tests import test_gpu_backward, test_gpu_naf, test_gpu_parity, test_gpu_rhf

OPEN_SHAPES = sorted(set(test_gpu_parity.SHAPES.values()) | set(test_gpu_backward.SHAPES.values()))
RHF_SHAPES = sorted(set(test_gpu_rhf.SHAPES.values()))


@pytest.mark.parametrize("shape", OPEN_SHAPES)
def test_open_shell_test_domains_have_the_declared_sizes(shape):
    dom = synth.make_domain(*shape, seed=1)
    need = lt.domain_sizes(dom.dims)
    assert set(dom.arrays()) == set(lt.ARRAY_FIELDS)
    for k, v in dom.arrays().items():
        assert v.size == need[k], k
        lt.check_array(k, torch.from_numpy(np.ascontiguousarray(v)), need[k], device=False)


@pytest.mark.parametrize("shape", RHF_SHAPES)
def test_closed_shell_test_domains_have_the_declared_sizes(shape):
    dom = synth.make_rhf_domain(*shape, seed=1)
    need = lt.rhf_sizes(shape)
    arrs = synth.rhf_arrays(dom)
    assert set(arrs) == set(lt.RHF_FIELDS)
    for k, v in arrs.items():
        assert v.size == need[k], k


@pytest.mark.parametrize("shape", sorted({s for s, _d, _e in test_gpu_naf.CASES.values()}))
def test_naf_test_inputs_have_the_declared_sizes(shape):
    Ja, Jb = synth.make_naf_input(*shape, seed=1, decay=10.0)
    na, nb = shape[0] + shape[1], shape[2] + shape[3]
    assert Ja.size == shape[4] * na * na and Jb.size == shape[4] * nb * nb


def test_check_array_rejects_what_the_kernels_cannot_use():
    t = torch.zeros(12, dtype=torch.float64)
    lt.check_array("x", t, 12, device=False)
    lt.check_array("x", t, 10, device=False)                 # a larger buffer is fine
    with pytest.raises(ValueError, match="elements"):
        lt.check_array("x", t, 13, device=False)
    with pytest.raises(ValueError, match="float64"):
        lt.check_array("x", t.float(), 12, device=False)
    with pytest.raises(ValueError, match="contiguous"):
        lt.check_array("x", t.reshape(3, 4).t(), 12, device=False)
    with pytest.raises(ValueError, match="GPU tensor"):
        lt.check_array("x", t, 12)
    lt.check_array("x", torch.zeros(0, dtype=torch.float64), 0)   # empty arrays may live anywhere
    lt.check_array("x", 0x1000, 12)                               # raw addresses pass through


def test_make_domain_rejects_host_and_undersized_tensors():
    dims = (3, 2, 5, 6, 8)
    need = lt.domain_sizes(dims)
    host = {k: torch.zeros(need[k], dtype=torch.float64) for k in lt.ARRAY_FIELDS}
    with pytest.raises(ValueError, match="GPU tensor"):
        lt.make_domain(dims, host)
    addrs = {k: 0x1000 * (n + 1) for n, k in enumerate(lt.ARRAY_FIELDS)}
    addrs["t2ab"] = torch.zeros(need["t2ab"] - 1, dtype=torch.float64)
    with pytest.raises(ValueError, match="t2ab has"):
        lt.make_domain(dims, addrs)
    rd = (3, 5, 8)
    rneed = lt.rhf_sizes(rd)
    with pytest.raises(ValueError, match="GPU tensor"):
        lt.make_rhf_domain(rd, {k: torch.zeros(rneed[k], dtype=torch.float64) for k in lt.RHF_FIELDS})
    with pytest.raises(ValueError, match="GPU tensor"):
        lt.make_naf_input((2, 3, 2, 3, 4), torch.zeros(4 * 25, dtype=torch.float64), 0x1000)


def test_energy_rejects_short_or_host_item_outputs():
    """e_items receives three doubles per item: a shorter or host tensor is
    refused before anything is enqueued (the domain arrays here are fake
    device addresses that are never dereferenced)."""
    try:
        lt.load_library()
    except Exception as ex:             # the library is built by the build step
        pytest.skip(f"library not built: {ex}")
    dims = (4, 3, 10, 11, 20)
    addrs = {k: 0x1000 * (n + 1) for n, k in enumerate(lt.ARRAY_FIELDS)}
    items = [[0, 0, 1, 2], [1, 0, 1, 2]]
    with pytest.raises(ValueError, match="e_items has 5 elements"):
        lt.ltriples_energy(addrs, dims, lt.LT_FP64, items=items, e_items=torch.zeros(5, dtype=torch.float64))
    with pytest.raises(ValueError, match="GPU tensor"):
        lt.ltriples_energy(addrs, dims, lt.LT_FP64, items=items, e_items=torch.zeros(2, 3, dtype=torch.float64))


def test_arrays_without_any_tensor_get_a_clear_error():
    try:
        lt.load_library()
    except Exception as ex:
        pytest.skip(f"library not built: {ex}")
    addrs = {k: 0x1000 * (n + 1) for n, k in enumerate(lt.ARRAY_FIELDS)}
    with pytest.raises(ValueError, match="no torch tensor"):
        lt.ltriples_energy(addrs, (4, 3, 10, 11, 20), lt.LT_FP64)


def test_gradient_outputs_for_arrays_passed_as_none():
    """An empty input may be passed as None; its gradient output is then a
    flat tensor of the (zero) element count instead of a failure."""
    t = {"t1a": torch.zeros(2, 5, dtype=torch.float64), "t1b": None}
    g = lt._grad_like(t, "t1a", 10, torch.device("cpu"))
    assert g.shape == (2, 5)
    g = lt._grad_like(t, "t1b", 0, torch.device("cpu"))
    assert g.shape == (0,) and g.dtype == torch.float64


def test_autograd_backward_precision_is_fp64_fp32_or_bf16x3():
    """The adjoint runs in FP64, FP32 or BF16X3 (split-product recompute, FP32
    reverse GEMMs): asking the differentiable energy for the plain-BF16
    ablation as its backward is refused before anything runs."""
    dims = (5, 4, 30, 31, 120)
    with pytest.raises(ValueError):
        lt.triples_energy({k: None for k in lt.ARRAY_FIELDS}, dims, "bf16x3", backward_precision="bf16")
