"""Host-only checks of the C ABI: the library loads, exports every declared
symbol, validates arguments with the documented error codes, and counts
flops by the documented formula.  No GPU is needed (no compute calls)."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2311_10048_amd as lt
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ltriples.h")


def _lib():
    if not os.path.exists(lt.LIB_PATH):
        pytest.skip("libltriples.so not built")
    return lt.load_library()


def _declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|size_t|const char\*)\s+(ltriples_\w+)\s*\(", src, re.M)))


def test_exports_every_declared_symbol():
    lib = _lib()
    names = _declared()
    assert "ltriples_energy" in names and len(names) >= 6
    for n in names:
        assert hasattr(lib, n), n
    assert lt.ltriples_version().startswith("ltriples")


def _fake_domain(dims, null=()):
    # fake, never-dereferenced device addresses: validation only checks for NULL
    t = {n: (0 if n in null else 0x1000 * (k + 1)) for k, n in enumerate(lt.ARRAY_FIELDS)}
    return lt.make_domain(dims, t)


def test_validate_ok_and_errors():
    _lib()
    d = _fake_domain((4, 3, 10, 11, 20))
    assert lt.ltriples_validate(d, lt.LT_FP64) == lt.LT_OK
    assert lt.ltriples_validate(d, lt.LT_FP32) == lt.LT_OK
    assert lt.ltriples_validate(d, 17) == lt.LT_EPREC
    assert lt.ltriples_validate(_fake_domain((4, -1, 10, 11, 20)), lt.LT_FP64) == lt.LT_EINVAL
    assert lt.ltriples_validate(_fake_domain((4, 3, 10, 11, 20), null=("t2ab",)), lt.LT_FP64) == lt.LT_EINVAL
    assert "t2ab" in lt.ltriples_last_error()
    assert lt.ltriples_validate(_fake_domain((4, 3, 10, 11, 0)), lt.LT_FP64) == lt.LT_ESHAPE
    # size limits: per dimension, and 2^37 FP64 input elements in all (checked
    # before any product of dimensions is formed)
    assert lt.ltriples_validate(_fake_domain((4097, 3, 10, 11, 20)), lt.LT_FP64) == lt.LT_ESHAPE
    assert lt.ltriples_validate(_fake_domain((4, 3, 46341, 11, 20)), lt.LT_FP64) == lt.LT_ESHAPE
    assert lt.ltriples_validate(_fake_domain((3, 3, 30, 30, 2**31 - 1)), lt.LT_FP64) == lt.LT_ESHAPE
    assert lt.ltriples_validate(_fake_domain((40, 38, 20000, 20000, 1200)), lt.LT_FP64) == lt.LT_ESHAPE
    assert "inputs too large" in lt.ltriples_last_error()
    assert lt.ltriples_validate(_fake_domain((60, 58, 500, 502, 2000)), lt.LT_FP64) == lt.LT_OK
    # NULL allowed for empty arrays
    assert lt.ltriples_validate(_fake_domain((4, 0, 10, 11, 20), null=("t1b", "t2bb", "t2ab", "Boo_b",
                                                                       "Bov_b", "eo_b", "fov_b")),
                                lt.LT_FP64) == lt.LT_OK


@pytest.mark.parametrize("item,code", [
    ((0, 0, 1, 2), lt.LT_OK), ((0, 1, 0, 2), lt.LT_ESHAPE), ((0, 0, 1, 4), lt.LT_ESHAPE),
    ((1, 0, 1, 2), lt.LT_OK), ((1, 0, 1, 3), lt.LT_ESHAPE), ((2, 0, 2, 3), lt.LT_OK),
    ((2, 0, 3, 0), lt.LT_ESHAPE), ((3, 0, 1, 2), lt.LT_OK), ((4, 0, 1, 2), lt.LT_ESHAPE),
])
def test_validate_items(item, code):
    _lib()
    d = _fake_domain((4, 3, 10, 11, 20))
    o, keep = lt.make_options(items=[item])
    assert lt.ltriples_validate(d, lt.LT_FP64, o) == code


def _flops_formula(oa, ob, va, vb):
    c = lambda n, k: float(np.prod([n - i for i in range(k)]) / np.prod(range(1, k + 1))) if n >= k else 0.0
    return (c(oa, 3) * (6 * va**4 + 6 * va**3 * oa) + c(ob, 3) * (6 * vb**4 + 6 * vb**3 * ob)
            + c(oa, 2) * ob * (4 * va**2 * vb**2 + 6 * va**3 * vb + 4 * va**2 * vb * ob + 6 * va**2 * vb * oa)
            + oa * c(ob, 2) * (4 * va**2 * vb**2 + 6 * vb**3 * va + 4 * vb**2 * va * oa + 6 * vb**2 * va * ob))


@pytest.mark.parametrize("name", ["tiny", "lno", "grad", "large"])
def test_flops_and_item_counts(name):
    _lib()
    oa, ob, va, vb, q = synth.SHAPES[name]
    f, n = lt.ltriples_flops(_fake_domain((oa, ob, va, vb, q)))
    assert abs(f - _flops_formula(oa, ob, va, vb)) <= 1e-12 * f
    assert n == oa * (oa - 1) * (oa - 2) // 6 + oa * (oa - 1) // 2 * ob + ob * (ob - 1) // 2 * oa \
        + ob * (ob - 1) * (ob - 2) // 6


def test_workspace_size_grows_with_precision():
    _lib()
    d = _fake_domain((5, 4, 30, 31, 120))
    w64 = lt.ltriples_workspace_size(d, lt.LT_FP64)
    w32 = lt.ltriples_workspace_size(d, lt.LT_FP32)
    assert w64 > w32 > 0


def test_energy_rejects_bad_args_without_gpu_work():
    lib = _lib()
    d = _fake_domain((4, 3, 10, 11, 20))
    code = lib.ltriples_energy(ctypes.byref(d), 9, None, None, None, None, 0, None)
    assert code == lt.LT_EPREC
    code = lib.ltriples_energy(ctypes.byref(d), lt.LT_FP64, None, None, None, None, 0, None)
    assert code == lt.LT_EINVAL


def _fake_array(dims_list):
    arr = (lt.Domain * len(dims_list))()
    for n, dims in enumerate(dims_list):
        arr[n] = _fake_domain(dims)
    return arr


def test_batched_workspace_is_shared_big_part_plus_small_parts():
    lib = _lib()
    dims = [(5, 4, 30, 31, 120), (6, 5, 45, 47, 96), (3, 0, 12, 13, 20)]
    singles = [lt.ltriples_workspace_size(_fake_domain(x), lt.LT_FP32) for x in dims]
    n = ctypes.c_size_t(0)
    assert lib.ltriples_workspace_size_batched(_fake_array(dims), 3, lt.LT_FP32, None, ctypes.byref(n)) == lt.LT_OK
    # one shared region of the largest domain's size, plus small per-domain tables
    assert max(singles) <= n.value < sum(singles)
    n1 = ctypes.c_size_t(0)
    assert lib.ltriples_workspace_size_batched(_fake_array(dims[1:2]), 1, lt.LT_FP32, None,
                                               ctypes.byref(n1)) == lt.LT_OK
    assert n1.value >= singles[1]


def test_batched_workspace_with_launch_groups():
    """options.group_budget: one group holds every domain's region side by
    side (about the sum of the single-domain workspaces); a budget below
    every domain gives one domain per group, sharing one region as without
    groups; a budget between packs the largest domain alone."""
    lib = _lib()
    dims = [(5, 4, 30, 31, 120), (6, 5, 45, 47, 96), (3, 0, 12, 13, 20), (4, 4, 26, 22, 50)]
    singles = [lt.ltriples_workspace_size(_fake_domain(x), lt.LT_BF16X3) for x in dims]

    def size(budget):
        o, _ = lt.make_options(group_budget=budget)
        n = ctypes.c_size_t(0)
        assert lib.ltriples_workspace_size_batched(_fake_array(dims), len(dims), lt.LT_BF16X3, ctypes.byref(o),
                                                   ctypes.byref(n)) == lt.LT_OK
        return n.value

    plain, one, every = size(0), size(1 << 50), size(1)
    assert every == plain
    slack = 2 * 256 * len(dims)   # region alignment
    assert abs(one - sum(singles)) <= slack, (one, sum(singles))
    # the largest domain (index 1) alone, the other three together in a
    # region no larger than its own: the same size as without groups
    assert sum(singles) - singles[1] < singles[1]
    between = size(max(singles))
    assert plain <= between < one
    assert abs(between - plain) <= slack, (between, plain)


def test_batched_rejects_item_lists_and_bad_domains():
    lib = _lib()
    dims = [(5, 4, 30, 31, 120), (4, 3, 10, 11, 20)]
    o, keep = lt.make_options(items=[(0, 0, 1, 2)])
    n = ctypes.c_size_t(0)
    assert lib.ltriples_workspace_size_batched(_fake_array(dims), 2, lt.LT_FP64, ctypes.byref(o),
                                               ctypes.byref(n)) == lt.LT_EINVAL
    bad = _fake_array(dims + [(4, 3, 10, 11, 0)])
    assert lib.ltriples_workspace_size_batched(bad, 3, lt.LT_FP64, None, ctypes.byref(n)) == lt.LT_ESHAPE
    assert "domain 2" in lt.ltriples_last_error()
    assert lib.ltriples_energy_batched(_fake_array(dims), 2, 9, None, None, None, None, 0, None) == lt.LT_EINVAL
    assert lib.ltriples_energy_batched(_fake_array(dims), 2, 9, None, 0x1000, None, None, 0, None) == lt.LT_EPREC
    assert lib.ltriples_energy_batched(None, 0, lt.LT_FP64, None, None, None, None, 0, None) == lt.LT_OK
    assert lib.ltriples_graph_reset() == lt.LT_OK


BWD_SHAPES = [(5, 4, 30, 31, 120), (6, 5, 45, 47, 96), (4, 0, 21, 22, 40), (3, 1, 17, 18, 30), (3, 3, 70, 67, 64),
              (2, 2, 9, 7, 12), (1, 2, 5, 6, 8), (0, 3, 5, 6, 8), (4, 4, 1, 2, 3), (20, 18, 160, 162, 640)]


@pytest.mark.parametrize("prec", [lt.LT_FP64, lt.LT_FP32, lt.LT_BF16X3])
@pytest.mark.parametrize("shape", BWD_SHAPES)
def test_backward_plan_descriptors_in_bounds(shape, prec):
    """Every range the adjoint's reverse-contraction descriptors address lies
    inside its buffer and the targets of one launch are disjoint (checked on
    the host before any kernel runs)."""
    lib = _lib()
    d = _fake_domain(shape)
    code = lib.ltriples_plan_check(ctypes.byref(d), prec, None, 1)
    assert code == lt.LT_OK, lt.ltriples_last_error()
    for bi in (1, 3):
        o, keep = lt.make_options(batch_items=bi)
        code = lib.ltriples_plan_check(ctypes.byref(d), prec, ctypes.byref(o), 1)
        assert code == lt.LT_OK, lt.ltriples_last_error()


def test_backward_plan_item_subsets_and_errors():
    lib = _lib()
    d = _fake_domain((6, 5, 20, 23, 40))
    items = synth.sample_items(6, 5, 3, seed=4)
    o, keep = lt.make_options(items=items, batch_items=2)
    assert lib.ltriples_plan_check(ctypes.byref(d), lt.LT_FP32, ctypes.byref(o), 1) == lt.LT_OK, \
        lt.ltriples_last_error()
    assert lib.ltriples_plan_check(ctypes.byref(d), lt.LT_BF16X3, None, 1) == lt.LT_OK
    assert lib.ltriples_plan_check(ctypes.byref(d), lt.LT_BF16, None, 1) == lt.LT_EPREC
    # the BF16X3 adjoint keeps the FP32 operands beside their split copies
    assert lt.ltriples_backward_workspace_size(d, lt.LT_BF16X3) > lt.ltriples_backward_workspace_size(d, lt.LT_FP32)
    n = ctypes.c_size_t(0)
    assert lib.ltriples_backward_workspace_size(ctypes.byref(d), lt.LT_FP64, None, ctypes.byref(n)) == lt.LT_OK
    assert n.value > lt.ltriples_workspace_size(d, lt.LT_FP64)
    assert lib.ltriples_backward(ctypes.byref(d), lt.LT_FP64, None, None, None, None, 0, None) == lt.LT_EINVAL


def test_build_chunks_fit_the_large_domain_on_one_gpu():
    """Chunked operand builds keep the BF16x3 workspace of the largest
    domain (60,58,500,502,2000) plus its FP64 inputs under one MI355X's
    288 GiB, and smaller chunks only shrink the workspace."""
    dims = synth.SHAPES["large"]
    d = _fake_domain(dims)
    no, nb, va, vb, q = dims
    inputs = 8 * (no * va + nb * vb + no * no * va * va + nb * nb * vb * vb + no * nb * va * vb
                  + q * (no * no + no * va + va * va + nb * nb + nb * vb + vb * vb)
                  + 2 * (no + va + nb + vb) + no * va + nb * vb)
    w = {p: lt.ltriples_workspace_size(d, p) for p in (lt.LT_FP32, lt.LT_BF16X3)}
    assert w[lt.LT_BF16X3] + inputs < 0.95 * 288 * 2 ** 30, (w, inputs)
    o, _ = lt.make_options(build_chunk_mib=64)
    for p in (lt.LT_FP64, lt.LT_FP32, lt.LT_BF16X3):
        small = lt.ltriples_workspace_size(d, p, o)
        assert small <= lt.ltriples_workspace_size(d, p), p


@pytest.mark.parametrize("prec", [lt.LT_FP64, lt.LT_FP32, lt.LT_BF16X3])
def test_backward_plan_in_bounds_with_small_build_chunks(prec):
    d = _fake_domain((6, 5, 45, 47, 96))
    o, _ = lt.make_options(build_chunk_mib=1)
    lib = lt.load_library()
    assert lib.ltriples_plan_check(ctypes.byref(d), prec, ctypes.byref(o), 1) == lt.LT_OK


def _fake_rhf(dims, null=()):
    t = {n: (0 if n in null else 0x1000 * (k + 1)) for k, n in enumerate(lt.RHF_FIELDS)}
    return lt.make_rhf_domain(dims, t)


@pytest.mark.parametrize("no,nv,naux", [(4, 10, 20), (40, 300, 1200), (2, 5, 8), (1, 5, 8)])
def test_rhf_flops_items_and_workspace(no, nv, naux):
    """The spin-adapted closed-shell call runs the unordered occupied
    triples i <= j <= k that are not all equal, three contractions of
    nv x nv^2 outputs over 2 (nv + no) rows each; the spin-block entry
    point runs the aaa and aab items of the alpha == beta domain, half the
    open-shell count, and needs more workspace on the LNO-sized domain."""
    _lib()
    d = _fake_rhf((no, nv, naux))
    f, n = lt.ltriples_rhf_flops(d)
    n_sa = (no * (no + 1) * (no + 2) // 6 - no) if no > 1 else 0
    assert n == n_sa
    assert abs(f - n_sa * 12.0 * nv**3 * (nv + no)) <= 1e-12 * max(f, 1.0)
    c = lambda m, k: float(np.prod([m - i for i in range(k)]) / np.prod(range(1, k + 1))) if m >= k else 0.0
    f_sb = c(no, 3) * (6 * nv**4 + 6 * nv**3 * no) \
        + c(no, 2) * no * (4 * nv**4 + 6 * nv**4 + 4 * nv**3 * no + 6 * nv**3 * no)
    fo, _ = lt.ltriples_flops(_fake_domain((no, no, nv, nv, naux)))
    if fo > 0:
        assert abs(f_sb / fo - 0.5) < 1e-12
    if no == 40:
        assert f < 0.4 * f_sb                 # the spin-adapted form's saving on the LNO-sized domain
    for prec in (lt.LT_FP64, lt.LT_FP32, lt.LT_BF16X3):
        w = lt.ltriples_rhf_workspace_size(d, prec)
        assert w >= 8 * no * no * nv * nv
        assert lt.ltriples_rhf_spin_block_workspace_size(d, prec) >= 8 * no * no * nv * nv
    if no == 40:
        # at the same batch budget the spin-adapted form needs less memory (one
        # v^3 cube per contraction item instead of pair-packed spin-block outputs);
        # its default budget is twice the spin-block form's
        o8, _ = lt.make_options(workspace_budget=8 << 30)
        assert lt.ltriples_rhf_workspace_size(d, lt.LT_BF16X3, o8) < lt.ltriples_rhf_spin_block_workspace_size(
            d, lt.LT_BF16X3, o8)
        o16, _ = lt.make_options(workspace_budget=16 << 30)
        assert lt.ltriples_rhf_workspace_size(d, lt.LT_BF16X3) == lt.ltriples_rhf_workspace_size(
            d, lt.LT_BF16X3, o16)


def test_rhf_rejects_bad_args():
    lib = _lib()
    assert lib.ltriples_rhf_workspace_size(None, lt.LT_FP64, None, ctypes.byref(ctypes.c_size_t())) == lt.LT_EINVAL
    n = ctypes.c_size_t()
    d = _fake_rhf((4, -1, 20))
    assert lib.ltriples_rhf_workspace_size(ctypes.byref(d), lt.LT_FP64, None, ctypes.byref(n)) == lt.LT_EINVAL
    d = _fake_rhf((4, 10, 20), null=("tau",))
    assert lib.ltriples_rhf_workspace_size(ctypes.byref(d), lt.LT_FP64, None, ctypes.byref(n)) == lt.LT_EINVAL
    assert "tau" in lt.ltriples_last_error()
    d = _fake_rhf((4, 10, 20))
    assert lib.ltriples_rhf_workspace_size(ctypes.byref(d), 11, None, ctypes.byref(n)) == lt.LT_EPREC
    o, keep = lt.make_options(items=[(0, 0, 1, 2)])
    assert lib.ltriples_rhf_workspace_size(ctypes.byref(d), lt.LT_FP64, ctypes.byref(o),
                                           ctypes.byref(n)) == lt.LT_EINVAL
    assert "closed-shell" in lt.ltriples_last_error()
    assert lib.ltriples_energy_rhf(ctypes.byref(d), lt.LT_FP64, None, None, None, None, 0, None) == lt.LT_EINVAL


def test_naf_workspace_and_errors():
    lib = _lib()
    x = lt.make_naf_input((3, 5, 2, 6, 20), 0x1000, 0x2000)
    w = lt.ltriples_naf_workspace_size(x)
    na = nb = 8
    # pair-packed integrals, W, eigenvectors, the kept vectors and one spin's factors
    assert w >= 8 * (20 * na * (na + 1) // 2 + 2 * 20 * 20 + 20 * na * na)
    n = ctypes.c_size_t()
    bad = lt.make_naf_input((3, 5, 2, 6, 20), 0, 0x2000)
    assert lib.ltriples_naf_workspace_size(ctypes.byref(bad), ctypes.byref(n)) == lt.LT_EINVAL
    assert "Ja" in lt.ltriples_last_error()
    bad = lt.make_naf_input((3, -5, 2, 6, 20), 0x1000, 0x2000)
    assert lib.ltriples_naf_workspace_size(ctypes.byref(bad), ctypes.byref(n)) == lt.LT_EINVAL
    out = lt.NafOutput()
    m = ctypes.c_int32()
    assert lib.ltriples_naf(ctypes.byref(x), 1e-2, None, ctypes.byref(m), None, 0, None) == lt.LT_EINVAL
    assert lib.ltriples_naf(ctypes.byref(x), float("nan"), ctypes.byref(out), ctypes.byref(m), None, 0,
                            None) == lt.LT_EINVAL


def test_rhf_backward_workspace_and_errors():
    lib = _lib()
    d = _fake_rhf((4, 10, 20))
    n = ctypes.c_size_t()
    assert lib.ltriples_backward_rhf_workspace_size(ctypes.byref(d), lt.LT_FP64, None, ctypes.byref(n)) == lt.LT_OK
    assert n.value > 4 * 8 * 4 * 4 * 10 * 10
    assert lib.ltriples_backward_rhf_workspace_size(ctypes.byref(d), lt.LT_BF16X3, None,
                                                    ctypes.byref(n)) == lt.LT_OK
    assert lib.ltriples_backward_rhf_workspace_size(ctypes.byref(d), lt.LT_BF16, None,
                                                    ctypes.byref(n)) == lt.LT_EPREC
    g = lt.RhfGrad()
    assert lib.ltriples_backward_rhf(ctypes.byref(d), lt.LT_FP64, None, None, ctypes.byref(g), None, 0,
                                     None) == lt.LT_EINVAL


def test_ctypes_layouts_match_the_header(tmp_path):
    """The binding's ctypes structures have the C sizes and field offsets of
    the header's structs (compiled with the host C compiler)."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {
        "ltriples_domain": (lt.Domain, ["noa", "t1a", "fov_b"]),
        "ltriples_options": (lt.Options, ["workspace_budget", "items", "e_items", "stats", "graph",
                                          "build_chunk_mib", "autotune", "deterministic", "check_finite",
                                          "tile_override"]),
        "ltriples_stats": (lt.Stats, ["n_items"]),
        "ltriples_domain_grad": (lt.DomainGrad, ["t1a", "fov_b", "eo_a", "ev_b"]),
        "ltriples_rhf_domain": (lt.RhfDomain, ["no", "t1", "fov"]),
        "ltriples_rhf_grad": (lt.RhfGrad, ["t1", "fov"]),
        "ltriples_naf_input": (lt.NafInput, ["nx", "Ja", "Jb"]),
        "ltriples_naf_output": (lt.NafOutput, ["Boo_a", "eigenvalues"]),
    }
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "ltriples.h"', "int main(void) {"]
    for name, (_, fields) in structs.items():
        lines.append(f'  printf("{name} %zu\\n", sizeof({name}));')
        for f in fields:
            lines.append(f'  printf("{name}.{f} %zu\\n", offsetof({name}, {f}));')
    lines.append("  return 0;\n}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = dict(line.rsplit(" ", 1) for line in subprocess.run([str(exe)], capture_output=True, text=True,
                                                                check=True).stdout.split("\n") if line)
    for name, (cls, fields) in structs.items():
        assert int(out[name]) == ctypes.sizeof(cls), name
        for f in fields:
            assert int(out[f"{name}.{f}"]) == getattr(cls, f).offset, (name, f)


def test_option_fields_validated():
    """tile_override takes 0 (automatic) or a configuration 1..8 per output
    layout; check_finite is 0 or 1; deterministic is accepted with any value
    (every call is deterministic)."""
    _lib()
    d = _fake_domain((4, 3, 10, 11, 20))
    o, _ = lt.make_options(tile_override=(8, 1, 0), check_finite=True)
    assert lt.ltriples_validate(d, lt.LT_BF16X3, o) == lt.LT_OK
    o.deterministic = 0
    assert lt.ltriples_validate(d, lt.LT_FP64, o) == lt.LT_OK
    for bad in ((9, 0, 0), (0, -1, 0), (0, 0, 100)):
        o, _ = lt.make_options(tile_override=bad)
        assert lt.ltriples_validate(d, lt.LT_FP32, o) == lt.LT_EINVAL
        assert "tile_override" in lt.ltriples_last_error()
    o, _ = lt.make_options()
    o.check_finite = 3
    assert lt.ltriples_validate(d, lt.LT_FP32, o) == lt.LT_EINVAL
    lib = lt.load_library()
    n = ctypes.c_size_t(0)
    o, _ = lt.make_options(tile_override=(0, 0, 9))
    assert lib.ltriples_workspace_size_batched(_fake_array([(4, 3, 10, 11, 20)]), 1, lt.LT_FP32, ctypes.byref(o),
                                               ctypes.byref(n)) == lt.LT_EINVAL


def test_workspace_budget_bounds_the_batch_scratch():
    """The per-batch scratch follows options.workspace_budget: a smaller
    budget gives a smaller workspace for the same domain."""
    _lib()
    d = _fake_domain((10, 9, 80, 81, 320))
    big = lt.ltriples_workspace_size(d, lt.LT_FP32, lt.make_options()[0])
    small = lt.ltriples_workspace_size(d, lt.LT_FP32, lt.make_options(workspace_budget=64 << 20)[0])
    assert small < big


def test_central_share_sizing_and_argument_checks():
    """ltriples_central_workspace_size: the extended domain (one more
    occupied orbital per quadrature point) needs a little more workspace
    than the domain itself; bad central arguments give LT_EINVAL, a central
    spin without occupied orbitals LT_ESHAPE, all host-only."""
    _lib()
    d = _fake_domain((5, 4, 30, 31, 120))
    base = lt.ltriples_workspace_size(d, lt.LT_BF16X3)
    for spin in (0, 1):
        cen, keep = lt.make_central(spin, 0x5000, [0.2, 0.7, 1.9], [0.3, 0.4, 0.6])
        w = lt.ltriples_central_workspace_size(d, cen, lt.LT_BF16X3)
        assert base < w < 3 * base
    lib = lt.load_library()
    n = ctypes.c_size_t(0)
    for spin, c, s, w, code in ((3, 0x5000, [0.5], [1.0], lt.LT_EINVAL), (0, 0, [0.5], [1.0], lt.LT_EINVAL),
                                (0, 0x5000, [0.0], [1.0], lt.LT_EINVAL), (1, 0x5000, [0.5] * 65, [1.0] * 65,
                                                                          lt.LT_EINVAL)):
        cen, keep = lt.make_central(spin, c, s, w)
        assert lib.ltriples_central_workspace_size(ctypes.byref(d), ctypes.byref(cen), lt.LT_FP64, None,
                                                   ctypes.byref(n)) == code, (spin, c, s, w)
    cen, keep = lt.make_central(0, 0x5000, [0.5], [1.0])
    o, _ = lt.make_options(items=[(0, 0, 1, 2)])
    assert lib.ltriples_central_workspace_size(ctypes.byref(d), ctypes.byref(cen), lt.LT_FP64, ctypes.byref(o),
                                               ctypes.byref(n)) == lt.LT_EINVAL
    d0 = _fake_domain((0, 4, 30, 31, 120), null=("t1a", "t2aa", "t2ab", "Boo_a", "Bov_a", "eo_a", "fov_a"))
    assert lib.ltriples_central_workspace_size(ctypes.byref(d0), ctypes.byref(cen), lt.LT_FP64, None,
                                               ctypes.byref(n)) == lt.LT_ESHAPE


def test_debug_w_argument_checks():
    """ltriples_debug_w: a NULL item or output gives LT_EINVAL and an item
    outside the domain (or not in canonical order) LT_ESHAPE, all before any
    device work."""
    lib = _lib()
    d = _fake_domain((5, 4, 30, 31, 120))
    it = (ctypes.c_int32 * 4)(0, 0, 1, 2)
    assert lib.ltriples_debug_w(ctypes.byref(d), lt.LT_FP64, None, 0x6000, 0x7000, None, 0, None) == lt.LT_EINVAL
    assert lib.ltriples_debug_w(ctypes.byref(d), lt.LT_FP64, it, None, 0x7000, None, 0, None) == lt.LT_EINVAL
    for bad in ((0, 0, 0, 1), (1, 0, 1, 4), (2, 1, 0, 0), (3, 0, 1, 4), (5, 0, 1, 2)):
        b = (ctypes.c_int32 * 4)(*bad)
        assert lib.ltriples_debug_w(ctypes.byref(d), lt.LT_FP64, b, 0x6000, 0x7000, None, 0,
                                    None) == lt.LT_ESHAPE, bad
