"""Helpers shared by the GPU tests: move a synthetic domain to the device and
call the library through its Python binding."""
import numpy as np

import paper_2311_10048_amd as lt
import synth


def to_device(dom: synth.Domain, device="cuda"):
    import torch
    return {k: torch.from_numpy(np.ascontiguousarray(v)).to(device) for k, v in dom.arrays().items()}


def gpu_energy(dom: synth.Domain, precision, items=None, tensors=None, ws_fill=None, **kw):
    """(E, parts [4][3], e_items [n][3] or None) as numpy, computed on the GPU.
    ws_fill: pre-fill the workspace with this float64 value (e.g. NaN) to
    catch reads of memory the library never wrote."""
    import torch
    t = tensors if tensors is not None else to_device(dom)
    if ws_fill is not None:
        d = lt.make_domain(dom.dims, t)
        o, keep = lt.make_options(items=items)
        need = lt.ltriples_workspace_size(d, precision, o)
        ws = torch.full((need // 8 + 1,), float(ws_fill), dtype=torch.float64, device="cuda")
        kw["workspace"] = ws.view(torch.uint8)
    e_items = None
    if items is not None:
        items = np.asarray(items, dtype=np.int32).reshape(-1, 4)
        e_items = torch.full((items.shape[0], 3), float("nan"), dtype=torch.float64, device="cuda")
    e, parts = lt.ltriples_energy(t, dom.dims, precision, items=items, e_items=e_items, **kw)
    torch.cuda.synchronize()
    return (float(e.item()), parts.cpu().numpy(),
            None if e_items is None else e_items.cpu().numpy())


def rel(a, b):
    return abs(a - b) / max(abs(a), abs(b), 1e-300)
