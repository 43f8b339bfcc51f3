"""ltriples: perturbative-triples energy E(T) of one LNO domain on MI355X.

Thin Python binding over the C ABI in ``include/ltriples.h`` (libltriples.so,
HIP for gfx950).  Only argument marshalling happens here: every step of the
(T) path runs in the library's kernels.  PyTorch provides device memory and
the current stream; the library is required, there is no fallback.

    import paper_2311_10048_amd as lt
    e, parts = lt.ltriples_energy(tensors, lt.LT_FP32)

``tensors`` maps the field names of ``ltriples_domain`` (t1a, t1b, t2aa,
t2bb, t2ab, Boo_a, Bov_a, Bvv_a, Boo_b, Bov_b, Bvv_b, eo_a, ev_a, eo_b, ev_b,
fov_a, fov_b) to contiguous float64 tensors on the current HIP device, in the
layouts documented in the header.
"""
from __future__ import annotations

import ctypes
import os
from typing import Mapping, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libltriples.so")

LT_OK = 0
LT_EINVAL = -1
LT_ESHAPE = -2
LT_EDENOM = -3
LT_EPREC = -4
LT_EWORKSPACE = -5
LT_EHIP = -6
LT_ENONFINITE = -7

LT_FP64 = 0
LT_FP32 = 1
LT_BF16X3 = 2
LT_BF16 = 3
PRECISIONS = {"fp64": LT_FP64, "fp32": LT_FP32, "bf16x3": LT_BF16X3, "bf16": LT_BF16}

ARRAY_FIELDS = ("t1a", "t1b", "t2aa", "t2bb", "t2ab", "Boo_a", "Bov_a", "Bvv_a",
                "Boo_b", "Bov_b", "Bvv_b", "eo_a", "ev_a", "eo_b", "ev_b", "fov_a", "fov_b")

_dp = ctypes.POINTER(ctypes.c_double)


class Domain(ctypes.Structure):
    _fields_ = ([(n, ctypes.c_int32) for n in ("noa", "nob", "nva", "nvb", "naux")]
                + [(n, ctypes.c_void_p) for n in ARRAY_FIELDS])


RHF_FIELDS = ("t1", "tau", "Boo", "Bov", "Bvv", "eo", "ev", "fov")
NAF_OUT_FIELDS = ("Boo_a", "Bov_a", "Bvv_a", "Boo_b", "Bov_b", "Bvv_b", "eigenvalues")


class NafInput(ctypes.Structure):
    _fields_ = ([(n, ctypes.c_int32) for n in ("no_a", "nv_a", "no_b", "nv_b", "nx")]
                + [("Ja", ctypes.c_void_p), ("Jb", ctypes.c_void_p)])


class NafOutput(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in NAF_OUT_FIELDS]


class RhfDomain(ctypes.Structure):
    _fields_ = ([(n, ctypes.c_int32) for n in ("no", "nv", "naux")]
                + [(n, ctypes.c_void_p) for n in RHF_FIELDS])


class RhfGrad(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in RHF_FIELDS]


class Central(ctypes.Structure):
    _fields_ = [("spin", ctypes.c_int32), ("c", ctypes.c_void_p), ("nq", ctypes.c_int32),
                ("s", ctypes.POINTER(ctypes.c_double)), ("w", ctypes.POINTER(ctypes.c_double))]


class Stats(ctypes.Structure):
    _fields_ = [("total_ms", ctypes.c_double),
                ("setup_ms", ctypes.c_double),
                ("triples_gemm_ms", ctypes.c_double),
                ("epilogue_ms", ctypes.c_double),
                ("triples_gemm_launches", ctypes.c_int64),
                ("triples_gemm_flops", ctypes.c_double),
                ("algorithmic_flops", ctypes.c_double),
                ("n_items", ctypes.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class Options(ctypes.Structure):
    _fields_ = [("workspace_budget", ctypes.c_size_t),
                ("items", ctypes.c_void_p),
                ("n_items", ctypes.c_int32),
                ("e_items", ctypes.c_void_p),
                ("batch_items", ctypes.c_int32),
                ("stats", ctypes.POINTER(Stats)),
                ("graph", ctypes.c_int32),
                ("build_chunk_mib", ctypes.c_int32),
                ("autotune", ctypes.c_int32),
                ("deterministic", ctypes.c_int32),
                ("check_finite", ctypes.c_int32),
                ("tile_override", ctypes.c_int32 * 3),
                ("group_budget", ctypes.c_size_t)]


GRAD_FIELDS = ("t1a", "t1b", "t2aa", "t2bb", "t2ab", "Boo_a", "Bov_a", "Bvv_a", "Boo_b", "Bov_b", "Bvv_b")
FOCK_GRAD_FIELDS = ("fov_a", "fov_b", "eo_a", "ev_a", "eo_b", "ev_b")


class DomainGrad(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in GRAD_FIELDS + FOCK_GRAD_FIELDS]


class LtError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"ltriples error {code}: {msg}")
        self.code = code


_lib = None


def load_library(path: Optional[str] = None):
    """Load libltriples.so (raises if it has not been built)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"{p} not found: build it with `python -m paper_2311_10048_amd.build`")
    # torch ships its own copy of the HIP runtime under the same soname; loaded
    # first, it also serves this library, so device pointers and streams from
    # torch are valid here.  Loading this library first would bring in the
    # system copy as a second runtime beside torch's.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(p)
    Dp, Op = ctypes.POINTER(Domain), ctypes.POINTER(Options)
    lib.ltriples_validate.argtypes = [Dp, ctypes.c_int32, Op]
    lib.ltriples_workspace_size.argtypes = [Dp, ctypes.c_int32, Op, ctypes.POINTER(ctypes.c_size_t)]
    lib.ltriples_flops.argtypes = [Dp, Op, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
    lib.ltriples_energy.argtypes = [Dp, ctypes.c_int32, Op, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
    lib.ltriples_energy_noalloc.argtypes = [Dp, ctypes.c_int32, Op, ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.c_void_p]
    lib.ltriples_debug_w.argtypes = [Dp, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
    lib.ltriples_noalloc_capacity.argtypes = []
    lib.ltriples_noalloc_capacity.restype = ctypes.c_size_t
    Cp = ctypes.POINTER(Central)
    lib.ltriples_central_workspace_size.argtypes = [Dp, Cp, ctypes.c_int32, Op, ctypes.POINTER(ctypes.c_size_t)]
    lib.ltriples_energy_central.argtypes = [Dp, Cp, ctypes.c_int32, Op, ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
    lib.ltriples_workspace_size_batched.argtypes = [Dp, ctypes.c_int32, ctypes.c_int32, Op,
                                                    ctypes.POINTER(ctypes.c_size_t)]
    lib.ltriples_energy_batched.argtypes = [Dp, ctypes.c_int32, ctypes.c_int32, Op, ctypes.c_void_p,
                                            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
    lib.ltriples_graph_reset.argtypes = []
    lib.ltriples_autotune_reset.argtypes = []
    lib.ltriples_plan_check.argtypes = [Dp, ctypes.c_int32, Op, ctypes.c_int32]
    Gp = ctypes.POINTER(DomainGrad)
    lib.ltriples_backward_workspace_size.argtypes = [Dp, ctypes.c_int32, Op, ctypes.POINTER(ctypes.c_size_t)]
    lib.ltriples_backward.argtypes = [Dp, ctypes.c_int32, Op, ctypes.c_void_p, Gp, ctypes.c_void_p,
                                      ctypes.c_size_t, ctypes.c_void_p]
    Rp = ctypes.POINTER(RhfDomain)
    lib.ltriples_rhf_workspace_size.argtypes = [Rp, ctypes.c_int32, Op, ctypes.POINTER(ctypes.c_size_t)]
    lib.ltriples_rhf_spin_block_workspace_size.argtypes = [Rp, ctypes.c_int32, Op, ctypes.POINTER(ctypes.c_size_t)]
    lib.ltriples_energy_rhf_spin_block.argtypes = [Rp, ctypes.c_int32, Op, ctypes.c_void_p, ctypes.c_void_p,
                                                   ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
    lib.ltriples_rhf_flops.argtypes = [Rp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
    lib.ltriples_energy_rhf.argtypes = [Rp, ctypes.c_int32, Op, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
    lib.ltriples_backward_rhf_workspace_size.argtypes = [Rp, ctypes.c_int32, Op, ctypes.POINTER(ctypes.c_size_t)]
    lib.ltriples_backward_rhf.argtypes = [Rp, ctypes.c_int32, Op, ctypes.c_void_p, ctypes.POINTER(RhfGrad),
                                          ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
    Np = ctypes.POINTER(NafInput)
    lib.ltriples_naf_workspace_size.argtypes = [Np, ctypes.POINTER(ctypes.c_size_t)]
    lib.ltriples_naf.argtypes = [Np, ctypes.c_double, ctypes.POINTER(NafOutput), ctypes.POINTER(ctypes.c_int32),
                                 ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
    lib.ltriples_last_error.restype = ctypes.c_char_p
    lib.ltriples_version.restype = ctypes.c_char_p
    for f in ("ltriples_validate", "ltriples_workspace_size", "ltriples_flops", "ltriples_energy",
              "ltriples_energy_noalloc", "ltriples_debug_w",
              "ltriples_workspace_size_batched", "ltriples_energy_batched", "ltriples_graph_reset",
              "ltriples_backward_workspace_size", "ltriples_backward", "ltriples_plan_check",
              "ltriples_rhf_workspace_size", "ltriples_rhf_flops", "ltriples_energy_rhf",
              "ltriples_rhf_spin_block_workspace_size", "ltriples_energy_rhf_spin_block",
              "ltriples_backward_rhf_workspace_size", "ltriples_backward_rhf",
              "ltriples_naf_workspace_size", "ltriples_naf", "ltriples_autotune_reset",
              "ltriples_central_workspace_size", "ltriples_energy_central"):
        getattr(lib, f).restype = ctypes.c_int
    if path is None:
        _lib = lib
    return lib


def ltriples_last_error() -> str:
    return load_library().ltriples_last_error().decode()


def ltriples_version() -> str:
    return load_library().ltriples_version().decode()


def _check(code: int):
    if code != LT_OK:
        raise LtError(code, ltriples_last_error())


def domain_sizes(dims) -> dict:
    """Element count of every ltriples_domain array for (noa, nob, nva, nvb, naux)."""
    oa, ob, va, vb, q = (int(x) for x in dims)
    return {"t1a": oa * va, "t1b": ob * vb, "t2aa": oa * oa * va * va, "t2bb": ob * ob * vb * vb,
            "t2ab": oa * ob * va * vb, "Boo_a": q * oa * oa, "Bov_a": q * oa * va, "Bvv_a": q * va * va,
            "Boo_b": q * ob * ob, "Bov_b": q * ob * vb, "Bvv_b": q * vb * vb, "eo_a": oa, "ev_a": va,
            "eo_b": ob, "ev_b": vb, "fov_a": oa * va, "fov_b": ob * vb}


def rhf_sizes(dims) -> dict:
    """Element count of every ltriples_rhf_domain array for (no, nv, naux)."""
    o, v, q = (int(x) for x in dims)
    return {"t1": o * v, "tau": o * o * v * v, "Boo": q * o * o, "Bov": q * o * v, "Bvv": q * v * v,
            "eo": o, "ev": v, "fov": o * v}


def check_array(name: str, t, need: int, device: bool = True) -> None:
    """The kernels read (or write) `need` float64 elements through this
    tensor's pointer: it must be contiguous float64 with at least that many
    elements and, with `device`, live in GPU memory.  Raw integer addresses
    are passed through unchecked."""
    if t is None or isinstance(t, int) or not hasattr(t, "is_contiguous"):
        return
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if str(t.dtype) != "torch.float64":
        raise ValueError(f"{name} must be float64")
    if t.numel() < need:
        raise ValueError(f"{name} has {t.numel()} elements; the dimensions need {need}")
    if device and need > 0 and t.device.type != "cuda":
        raise ValueError(f"{name} must be a GPU tensor (got one on {t.device})")


def _ptr(x) -> int:
    if x is None:
        return 0
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    raise TypeError(f"cannot take a device pointer of {type(x)}")


def _device_of(tensors: Mapping[str, object]):
    """The device of the first torch tensor among the arguments."""
    for t in tensors.values():
        if hasattr(t, "device"):
            return t.device
    raise ValueError("no torch tensor among the arrays: pass device tensors (raw addresses only to the "
                     "ctypes-level calls)")


def _grad_like(tensors: Mapping[str, object], k: str, n: int, dev):
    """Output for the gradient of input k: shaped like the input, or a flat
    tensor of its element count when the input was passed as None."""
    import torch
    t = tensors.get(k)
    if hasattr(t, "shape"):
        return torch.empty_like(t)
    return torch.empty(n, dtype=torch.float64, device=dev)


def make_domain(dims, tensors: Optional[Mapping[str, object]] = None) -> Domain:
    """ltriples_domain from (noa, nob, nva, nvb, naux) and device tensors
    (or raw device addresses) keyed by field name; missing arrays are NULL."""
    d = Domain()
    d.noa, d.nob, d.nva, d.nvb, d.naux = (int(x) for x in dims)
    tensors = tensors or {}
    need = domain_sizes(dims)
    for n in ARRAY_FIELDS:
        t = tensors.get(n)
        check_array(n, t, need[n])
        setattr(d, n, _ptr(t))
    return d


def make_options(items=None, e_items=None, workspace_budget: int = 0, batch_items: int = 0,
                 stats: Optional[Stats] = None, build_chunk_mib: int = 0, autotune: bool = False,
                 check_finite: bool = False, tile_override=None, deterministic: bool = True,
                 group_budget: int = 0):
    """ltriples_options; `items` is a host int32 array [n][4] (kept alive by
    the returned tuple's second element); `tile_override` is None or three
    configuration numbers (0 = automatic) for the S, G and Y layouts;
    `group_budget` (bytes, batched calls only) enables launch groups."""
    o = Options()
    o.workspace_budget = int(workspace_budget)
    o.group_budget = int(group_budget)
    o.deterministic = 1 if deterministic else 0
    o.check_finite = 1 if check_finite else 0
    if tile_override is not None:
        for k, v in enumerate(tile_override):
            o.tile_override[k] = int(v)
    o.batch_items = int(batch_items)
    o.build_chunk_mib = int(build_chunk_mib)
    o.autotune = 1 if autotune else 0
    if stats is not None:
        o.stats = ctypes.pointer(stats)
    keep = None
    if items is not None:
        keep = np.ascontiguousarray(np.asarray(items, dtype=np.int32).reshape(-1, 4))
        o.items = keep.ctypes.data
        o.n_items = keep.shape[0]
    o.e_items = _ptr(e_items)
    return o, keep


def ltriples_validate(dom: Domain, precision: int, options: Optional[Options] = None) -> int:
    lib = load_library()
    return lib.ltriples_validate(ctypes.byref(dom), int(precision),
                                 ctypes.byref(options) if options is not None else None)


def ltriples_workspace_size(dom: Domain, precision: int, options: Optional[Options] = None) -> int:
    lib = load_library()
    n = ctypes.c_size_t(0)
    _check(lib.ltriples_workspace_size(ctypes.byref(dom), int(precision),
                                       ctypes.byref(options) if options is not None else None,
                                       ctypes.byref(n)))
    return n.value


def ltriples_flops(dom: Domain, options: Optional[Options] = None):
    """(algorithmic W-contraction flops, number of items) of the item list."""
    lib = load_library()
    f = ctypes.c_double(0)
    n = ctypes.c_int64(0)
    _check(lib.ltriples_flops(ctypes.byref(dom), ctypes.byref(options) if options is not None else None,
                              ctypes.byref(f), ctypes.byref(n)))
    return f.value, n.value


def ltriples_energy(tensors: Mapping[str, object], dims, precision: int = LT_FP32, items=None,
                    e_items=None, workspace_budget: int = 0, batch_items: int = 0, workspace=None,
                    stream=None, stats: Optional[Stats] = None, build_chunk_mib: int = 0,
                    autotune: bool = False, check_finite: bool = False, tile_override=None):
    """E(T) of one domain on the current HIP device.

    Returns (e, parts): a float64 device tensor of shape [1] and one of shape
    [4, 3] (blocks aaa, aab, abb, bbb x {E4, E_ST, E_DT}).  `workspace`, if
    given, is a uint8 device tensor at least ltriples_workspace_size() long;
    otherwise one is allocated through torch.  The call is asynchronous on
    `stream` (default: torch's current stream) except for one small
    synchronous read of the orbital energies.  Passing a ``Stats`` object
    makes the call time its phases with HIP events and wait for the stream.
    """
    import torch
    if isinstance(precision, str):
        precision = PRECISIONS[precision]
    dom = make_domain(dims, tensors)
    opts, keep = make_options(items, e_items, workspace_budget, batch_items, stats, build_chunk_mib, autotune,
                              check_finite, tile_override)
    if e_items is not None and not isinstance(e_items, int):
        try:
            n_it = ltriples_flops(dom, opts)[1]
        except LtError:
            n_it = None          # the energy call below reports the same error
        if n_it is not None:
            check_array("e_items", e_items, 3 * n_it)
    dev = _device_of(tensors)
    need = ltriples_workspace_size(dom, precision, opts)
    if workspace is None:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    e = torch.empty(1, dtype=torch.float64, device=dev)
    parts = torch.empty(4, 3, dtype=torch.float64, device=dev)
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    lib = load_library()
    code = lib.ltriples_energy(ctypes.byref(dom), int(precision), ctypes.byref(opts),
                               e.data_ptr(), parts.data_ptr(), workspace.data_ptr(),
                               workspace.numel(), st.cuda_stream)
    _check(code)
    del keep
    return e, parts


def ltriples_debug_w(tensors: Mapping[str, object], dims, item, precision: int = LT_FP64, stream=None):
    """Debug dump of one triplet's W over its full virtual cube, as the GPU
    path forms it (see ltriples_debug_w in include/ltriples.h).

    `item` = (block, p, q, r).  Returns (w, e): a float64 device tensor of
    shape [v_s, v_s, v_s] (same spin) or [v_s, v_s, v_t] (mixed: a, b of the
    pair's spin s, C of the odd index's spin t), and the item's energy as a
    float64 device tensor of shape [1].  Waits for nothing beyond what
    ltriples_energy waits for."""
    import torch
    if isinstance(precision, str):
        precision = PRECISIONS[precision]
    it = np.ascontiguousarray(np.asarray(item, dtype=np.int32).reshape(4))
    blk = int(it[0])
    if blk not in (0, 1, 2, 3):
        raise ValueError("item block must be 0..3")
    dom = make_domain(dims, tensors)
    nv = (int(dims[2]), int(dims[3]))
    s = 0 if blk in (0, 1) else 1
    shape = (nv[s], nv[s], nv[s]) if blk in (0, 3) else (nv[s], nv[s], nv[1 - s])
    dev = _device_of(tensors)
    w = torch.empty(shape, dtype=torch.float64, device=dev)
    e = torch.empty(1, dtype=torch.float64, device=dev)
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    lib = load_library()
    code = lib.ltriples_debug_w(ctypes.byref(dom), int(precision), it.ctypes.data, w.data_ptr(), e.data_ptr(),
                                None, 0, st.cuda_stream)
    _check(code)
    return w, e


def ltriples_noalloc_capacity() -> int:
    """Bytes of the fixed per-device workspace of ltriples_energy_noalloc."""
    return int(load_library().ltriples_noalloc_capacity())


def ltriples_energy_noalloc(tensors: Mapping[str, object], dims, precision: int = LT_FP32, items=None,
                            e_items=None, out=None, stream=None, workspace_budget: int = 0, batch_items: int = 0,
                            build_chunk_mib: int = 0, check_finite: bool = False, tile_override=None):
    """E(T) of one domain through the no-allocation entry point: the library
    uses its fixed per-device workspace and allocates nothing.  `out` may
    supply the (e [1], parts [4, 3]) float64 device tensors (otherwise they
    are allocated here, by torch, before the call).  Returns (e, parts)."""
    import torch
    if isinstance(precision, str):
        precision = PRECISIONS[precision]
    dom = make_domain(dims, tensors)
    opts, keep = make_options(items, e_items, workspace_budget, batch_items, None, build_chunk_mib, False,
                              check_finite, tile_override)
    if e_items is not None and not isinstance(e_items, int):
        try:
            n_it = ltriples_flops(dom, opts)[1]
        except LtError:
            n_it = None
        if n_it is not None:
            check_array("e_items", e_items, 3 * n_it)
    dev = _device_of(tensors)
    if out is None:
        out = (torch.empty(1, dtype=torch.float64, device=dev), torch.empty(4, 3, dtype=torch.float64, device=dev))
    e, parts = out
    check_array("e", e, 1)
    check_array("parts", parts, 12)
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    _check(load_library().ltriples_energy_noalloc(ctypes.byref(dom), int(precision), ctypes.byref(opts),
                                                  e.data_ptr(), parts.data_ptr(), st.cuda_stream))
    del keep
    return e, parts


def make_central(spin: int, c, s, w):
    """ltriples_central from the central orbital's spin, its coefficients
    (device tensor, or a raw address) and the quadrature points and weights
    (host sequences; kept alive by the returned tuple's second element)."""
    x = Central()
    x.spin = int(spin)
    x.c = _ptr(c)
    sv = np.ascontiguousarray(np.asarray(s, dtype=np.float64).ravel())
    wv = np.ascontiguousarray(np.asarray(w, dtype=np.float64).ravel())
    if sv.size != wv.size:
        raise ValueError("quadrature points and weights differ in length")
    x.nq = int(sv.size)
    x.s = sv.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    x.w = wv.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    return x, (sv, wv)


def ltriples_central_workspace_size(dom: Domain, central: Central, precision: int,
                                    options: Optional[Options] = None) -> int:
    lib = load_library()
    n = ctypes.c_size_t(0)
    _check(lib.ltriples_central_workspace_size(ctypes.byref(dom), ctypes.byref(central), int(precision),
                                               ctypes.byref(options) if options is not None else None,
                                               ctypes.byref(n)))
    return n.value


def ltriples_energy_central(tensors: Mapping[str, object], dims, spin: int, c, s, w, precision: int = LT_FP32,
                            workspace_budget: int = 0, batch_items: int = 0, workspace=None, stream=None,
                            stats: Optional[Stats] = None, build_chunk_mib: int = 0, autotune: bool = False,
                            check_finite: bool = False, tile_override=None):
    """(T) share of the central orbital `c` (device float64 tensor over the
    occupied orbitals of `spin`) with the Laplace points `s` and weights `w`
    (host sequences).  Returns (e [1], parts [4, 3]) as float64 device
    tensors."""
    import torch
    if isinstance(precision, str):
        precision = PRECISIONS[precision]
    dom = make_domain(dims, tensors)
    nocc = int(dims[0]) if int(spin) == 0 else int(dims[1])
    check_array("c", c, nocc)
    cen, keep_q = make_central(spin, c, s, w)
    opts, keep = make_options(None, None, workspace_budget, batch_items, stats, build_chunk_mib, autotune,
                              check_finite, tile_override)
    dev = _device_of(tensors)
    need = ltriples_central_workspace_size(dom, cen, precision, opts)
    if workspace is None:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    e = torch.empty(1, dtype=torch.float64, device=dev)
    parts = torch.empty(4, 3, dtype=torch.float64, device=dev)
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    _check(load_library().ltriples_energy_central(ctypes.byref(dom), ctypes.byref(cen), int(precision),
                                                  ctypes.byref(opts), e.data_ptr(), parts.data_ptr(),
                                                  workspace.data_ptr(), workspace.numel(), st.cuda_stream))
    del keep, keep_q
    return e, parts


def make_rhf_domain(dims, tensors: Optional[Mapping[str, object]] = None) -> RhfDomain:
    """ltriples_rhf_domain from (no, nv, naux) and device tensors keyed by
    RHF_FIELDS; missing arrays are NULL."""
    d = RhfDomain()
    d.no, d.nv, d.naux = (int(x) for x in dims)
    tensors = tensors or {}
    need = rhf_sizes(dims)
    for n in RHF_FIELDS:
        t = tensors.get(n)
        check_array(n, t, need[n])
        setattr(d, n, _ptr(t))
    return d


def ltriples_rhf_workspace_size(dom: RhfDomain, precision: int, options: Optional[Options] = None) -> int:
    lib = load_library()
    n = ctypes.c_size_t(0)
    _check(lib.ltriples_rhf_workspace_size(ctypes.byref(dom), int(precision),
                                           ctypes.byref(options) if options is not None else None,
                                           ctypes.byref(n)))
    return n.value


def ltriples_rhf_flops(dom: RhfDomain):
    """(W-contraction flops executed by ltriples_energy_rhf, number of items)."""
    lib = load_library()
    f = ctypes.c_double(0)
    n = ctypes.c_int64(0)
    _check(lib.ltriples_rhf_flops(ctypes.byref(dom), ctypes.byref(f), ctypes.byref(n)))
    return f.value, n.value


def ltriples_rhf_spin_block_workspace_size(dom: RhfDomain, precision: int,
                                           options: Optional[Options] = None) -> int:
    lib = load_library()
    n = ctypes.c_size_t(0)
    _check(lib.ltriples_rhf_spin_block_workspace_size(ctypes.byref(dom), int(precision),
                                                      ctypes.byref(options) if options is not None else None,
                                                      ctypes.byref(n)))
    return n.value


def ltriples_energy_rhf(tensors: Mapping[str, object], dims, precision: int = LT_FP32, workspace_budget: int = 0,
                        batch_items: int = 0, workspace=None, stream=None, stats: Optional[Stats] = None,
                        build_chunk_mib: int = 0, method: str = "spin_adapted", autotune: bool = False,
                        check_finite: bool = False, tile_override=None):
    """Closed-shell E(T) of one domain given in spatial orbitals (RHF_FIELDS,
    dims (no, nv, naux)).  Returns (e, parts): float64 device tensors of
    shapes [1] and [3] ({E4, E_ST, E_DT}).  `method`: "spin_adapted"
    (ltriples_energy_rhf) or "spin_block" (ltriples_energy_rhf_spin_block)."""
    import torch
    if isinstance(precision, str):
        precision = PRECISIONS[precision]
    if method not in ("spin_adapted", "spin_block"):
        raise ValueError("method must be 'spin_adapted' or 'spin_block'")
    dom = make_rhf_domain(dims, tensors)
    opts, keep = make_options(None, None, workspace_budget, batch_items, stats, build_chunk_mib, autotune,
                              check_finite, tile_override)
    dev = _device_of(tensors)
    sa = method == "spin_adapted"
    need = (ltriples_rhf_workspace_size if sa else ltriples_rhf_spin_block_workspace_size)(dom, precision, opts)
    if workspace is None:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    e = torch.empty(1, dtype=torch.float64, device=dev)
    parts = torch.empty(3, dtype=torch.float64, device=dev)
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    lib = load_library()
    fn = lib.ltriples_energy_rhf if sa else lib.ltriples_energy_rhf_spin_block
    _check(fn(ctypes.byref(dom), int(precision), ctypes.byref(opts), e.data_ptr(), parts.data_ptr(),
              workspace.data_ptr(), workspace.numel(), st.cuda_stream))
    del keep
    return e, parts


def ltriples_backward_rhf(tensors: Mapping[str, object], dims, precision: int = LT_FP64, gbar=None,
                          workspace_budget: int = 0, batch_items: int = 0, workspace=None, out=None, stream=None,
                          build_chunk_mib: int = 0):
    """gbar * dE/dx of the closed-shell energy for x in RHF_FIELDS (dE/dtau
    projected onto its symmetry, dE/dBoo and dE/dBvv symmetrised).  Returns
    a dict of float64 device tensors; `out` may supply them (missing keys
    are not computed)."""
    import torch
    if isinstance(precision, str):
        precision = PRECISIONS[precision]
    dom = make_rhf_domain(dims, tensors)
    opts, keep = make_options(None, None, workspace_budget, batch_items, None, build_chunk_mib)
    dev = _device_of(tensors)
    if gbar is None:
        gbar = torch.ones(1, dtype=torch.float64, device=dev)
    if gbar.dtype != torch.float64 or gbar.numel() != 1 or not gbar.is_contiguous():
        raise ValueError("gbar must be one contiguous float64 element")
    if out is None:
        out = {k: _grad_like(tensors, k, n_k, dev) for k, n_k in rhf_sizes(dims).items()}
    g = RhfGrad()
    need_g = rhf_sizes(dims)
    for k in RHF_FIELDS:
        check_array(f"out[{k!r}]", out.get(k), need_g[k])
        setattr(g, k, _ptr(out.get(k)))
    lib = load_library()
    n = ctypes.c_size_t(0)
    _check(lib.ltriples_backward_rhf_workspace_size(ctypes.byref(dom), int(precision), ctypes.byref(opts),
                                                    ctypes.byref(n)))
    if workspace is None:
        workspace = torch.empty(max(n.value, 1), dtype=torch.uint8, device=dev)
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    _check(lib.ltriples_backward_rhf(ctypes.byref(dom), int(precision), ctypes.byref(opts), gbar.data_ptr(),
                                     ctypes.byref(g), workspace.data_ptr(), workspace.numel(), st.cuda_stream))
    del keep
    return out


def make_naf_input(dims, Ja=None, Jb=None) -> NafInput:
    """ltriples_naf_input from (no_a, nv_a, no_b, nv_b, nx) and the two
    three-index integral tensors [nx][n_s][n_s] (device)."""
    x = NafInput()
    x.no_a, x.nv_a, x.no_b, x.nv_b, x.nx = (int(v) for v in dims)
    na, nb = x.no_a + x.nv_a, x.no_b + x.nv_b
    for name, t, n in (("Ja", Ja, na), ("Jb", Jb, nb)):
        check_array(name, t, x.nx * n * n)
        setattr(x, name, _ptr(t))
    return x


def ltriples_naf_workspace_size(inp: NafInput) -> int:
    lib = load_library()
    n = ctypes.c_size_t(0)
    _check(lib.ltriples_naf_workspace_size(ctypes.byref(inp), ctypes.byref(n)))
    return n.value


def ltriples_naf(Ja, Jb, dims, eps: float, workspace=None, stream=None):
    """Natural auxiliary functions of one LIS: returns (naux, dict) with the
    compressed factors Boo_a ... Bvv_b ([naux][..][..]) and all eigenvalues
    of W in decreasing order, as float64 device tensors."""
    import torch
    no_a, nv_a, no_b, nv_b, nx = (int(v) for v in dims)
    inp = make_naf_input(dims, Ja, Jb)
    dev = Ja.device
    need = ltriples_naf_workspace_size(inp)
    if workspace is None:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    shapes = {"Boo_a": (no_a, no_a), "Bov_a": (no_a, nv_a), "Bvv_a": (nv_a, nv_a),
              "Boo_b": (no_b, no_b), "Bov_b": (no_b, nv_b), "Bvv_b": (nv_b, nv_b)}
    outs = {k: torch.empty((nx,) + sh, dtype=torch.float64, device=dev) for k, sh in shapes.items()}
    outs["eigenvalues"] = torch.empty(nx, dtype=torch.float64, device=dev)
    o = NafOutput()
    for k in NAF_OUT_FIELDS:
        setattr(o, k, _ptr(outs[k]) if outs[k].numel() else 0)
    naux = ctypes.c_int32(0)
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    lib = load_library()
    _check(lib.ltriples_naf(ctypes.byref(inp), float(eps), ctypes.byref(o), ctypes.byref(naux),
                            workspace.data_ptr(), workspace.numel(), st.cuda_stream))
    m = naux.value
    res = {k: v[:m].contiguous() for k, v in outs.items() if k != "eigenvalues"}
    res["eigenvalues"] = outs["eigenvalues"]
    return m, res


def _domain_array(dims_list, tensors_list):
    arr = (Domain * len(dims_list))()
    for n, (dims, t) in enumerate(zip(dims_list, tensors_list)):
        arr[n] = make_domain(dims, t)
    return arr


def ltriples_workspace_size_batched(dims_list, tensors_list, precision: int, options: Optional[Options] = None) -> int:
    lib = load_library()
    arr = _domain_array(dims_list, tensors_list)
    n = ctypes.c_size_t(0)
    _check(lib.ltriples_workspace_size_batched(arr, len(dims_list), int(precision),
                                               ctypes.byref(options) if options is not None else None,
                                               ctypes.byref(n)))
    return n.value


def ltriples_energy_batched(tensors_list, dims_list, precision: int = LT_FP32, graph: bool = False,
                            workspace_budget: int = 0, batch_items: int = 0, workspace=None, out=None,
                            stream=None, build_chunk_mib: int = 0, autotune: bool = False,
                            check_finite: bool = False, tile_override=None, group_budget: int = 0):
    """E(T) of several domains in one call.  Returns (e [ndom], parts [ndom,4,3]).
    With graph=True the launch sequence is captured into a hipGraph on the
    first call and replayed on later calls with the same shapes, pointers,
    workspace and output tensors (pass `workspace` and `out` to reuse them).
    group_budget > 0 (bytes) packs the domains, longest first, into launch
    groups whose contraction launches take items of all their domains
    (options.group_budget); results are bitwise unchanged."""
    import torch
    if isinstance(precision, str):
        precision = PRECISIONS[precision]
    ndom = len(dims_list)
    opts, _ = make_options(workspace_budget=workspace_budget, batch_items=batch_items, build_chunk_mib=build_chunk_mib,
                           autotune=autotune, check_finite=check_finite, tile_override=tile_override,
                           group_budget=group_budget)
    opts.graph = 1 if graph else 0
    arr = _domain_array(dims_list, tensors_list)
    dev = _device_of(tensors_list[0])
    lib = load_library()
    n = ctypes.c_size_t(0)
    _check(lib.ltriples_workspace_size_batched(arr, ndom, int(precision), ctypes.byref(opts), ctypes.byref(n)))
    if workspace is None:
        workspace = torch.empty(max(n.value, 1), dtype=torch.uint8, device=dev)
    if out is None:
        out = (torch.empty(ndom, dtype=torch.float64, device=dev),
               torch.empty(ndom, 4, 3, dtype=torch.float64, device=dev))
    e, parts = out
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    _check(lib.ltriples_energy_batched(arr, ndom, int(precision), ctypes.byref(opts), e.data_ptr(),
                                       parts.data_ptr(), workspace.data_ptr(), workspace.numel(),
                                       st.cuda_stream))
    return e, parts


def ltriples_autotune_reset():
    _check(load_library().ltriples_autotune_reset())


def ltriples_graph_reset():
    _check(load_library().ltriples_graph_reset())


def ltriples_backward_workspace_size(dom: Domain, precision: int, options: Optional[Options] = None) -> int:
    lib = load_library()
    n = ctypes.c_size_t(0)
    _check(lib.ltriples_backward_workspace_size(ctypes.byref(dom), int(precision),
                                                ctypes.byref(options) if options is not None else None,
                                                ctypes.byref(n)))
    return n.value


def ltriples_backward(tensors: Mapping[str, object], dims, precision: int = LT_FP64, gbar=None, items=None,
                      workspace_budget: int = 0, batch_items: int = 0, workspace=None, out=None, stream=None,
                      stats: Optional[Stats] = None, build_chunk_mib: int = 0, check_finite: bool = False):
    """gbar * dE/dx for x in GRAD_FIELDS (projected convention for t2aa, t2bb,
    Boo, Bvv) and FOCK_GRAD_FIELDS (f_ov and the orbital energies).  Returns a dict of float64 device
    tensors shaped like the inputs.  `gbar` is a float64 device tensor with
    one element (default 1); `out` may supply the output tensors (a dict keyed
    like the result; missing keys are not computed)."""
    import torch
    if isinstance(precision, str):
        precision = PRECISIONS[precision]
    dom = make_domain(dims, tensors)
    opts, keep = make_options(items, None, workspace_budget, batch_items, stats, build_chunk_mib,
                              check_finite=check_finite)
    dev = _device_of(tensors)
    if gbar is None:
        gbar = torch.ones(1, dtype=torch.float64, device=dev)
    if gbar.dtype != torch.float64 or gbar.numel() != 1 or not gbar.is_contiguous():
        raise ValueError("gbar must be one contiguous float64 element")
    if out is None:
        sizes = domain_sizes(dims)
        out = {k: _grad_like(tensors, k, sizes[k], dev) for k in GRAD_FIELDS + FOCK_GRAD_FIELDS}
    g = DomainGrad()
    need_g = domain_sizes(dims)
    for k in GRAD_FIELDS + FOCK_GRAD_FIELDS:
        check_array(f"out[{k!r}]", out.get(k), need_g[k])
        setattr(g, k, _ptr(out.get(k)))
    need = ltriples_backward_workspace_size(dom, precision, opts)
    if workspace is None:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    _check(load_library().ltriples_backward(ctypes.byref(dom), int(precision), ctypes.byref(opts), gbar.data_ptr(),
                                            ctypes.byref(g), workspace.data_ptr(), workspace.numel(),
                                            st.cuda_stream))
    del keep
    return out


def _autograd_function():
    import torch

    class TriplesEnergy(torch.autograd.Function):
        """E(T) as a differentiable function of T1, T2, the DF factors, f_ov
        and the orbital energies."""

        @staticmethod
        def forward(ctx, precision, bprec, dims, *arrays):
            tens = dict(zip(ARRAY_FIELDS, arrays))
            e, _ = ltriples_energy(tens, dims, precision)
            ctx.bprec, ctx.dims = bprec, dims
            ctx.save_for_backward(*arrays)
            return e.reshape(())

        @staticmethod
        def backward(ctx, gE):
            tens = dict(zip(ARRAY_FIELDS, ctx.saved_tensors))
            gbar = gE.detach().to(torch.float64).reshape(1).contiguous()
            g = ltriples_backward(tens, ctx.dims, ctx.bprec, gbar=gbar)
            return (None, None, None) + tuple(g.get(k) if ctx.needs_input_grad[3 + n] else None
                                              for n, k in enumerate(ARRAY_FIELDS))

    return TriplesEnergy


_TE = None


def triples_energy(tensors: Mapping[str, object], dims, precision="fp64", backward_precision=None):
    """Differentiable E(T) (0-d float64 tensor).  Gradients flow to T1, T2,
    the DF factors, f_ov and the orbital energies through ltriples_backward,
    which runs in FP64, FP32 or BF16X3 (the forward contraction recomputed in
    split BF16 products, FP32 reverse GEMMs): `backward_precision` picks one
    ("fp64", "fp32" or "bf16x3"); by default FP64 for an FP64 forward and
    FP32 for every reduced-precision forward (FP32, BF16X3, BF16)."""
    global _TE
    if _TE is None:
        _TE = _autograd_function()
    if isinstance(precision, str):
        precision = PRECISIONS[precision]
    if backward_precision is None:
        bprec = LT_FP64 if precision == LT_FP64 else LT_FP32
    else:
        bprec = PRECISIONS[backward_precision] if isinstance(backward_precision, str) else int(backward_precision)
        if bprec not in (LT_FP64, LT_FP32, LT_BF16X3):
            raise ValueError("backward_precision must be fp64, fp32 or bf16x3")
    return _TE.apply(int(precision), int(bprec), tuple(int(x) for x in dims), *(tensors[k] for k in ARRAY_FIELDS))
