"""Seeded synthetic open-shell domains for the (T) energy path.

This module only draws random inputs; it contains none of the (T) arithmetic.
Both the CPU oracle (``oracle/``) and the GPU path's tests and benchmark take
their inputs from here, so the two sides always see bit-identical data.

Shapes follow the paper's statement of the problem for one local interacting
subspace (LIS): semicanonical alpha/beta occupied and virtual orbitals
(Sec. "Theoretical background", orbital-notation table), spin-blocked CCSD
amplitudes (eq. cim_ccsd_energy), and density-fitted three-index factors in a
natural-auxiliary-function basis shared by both spins (Sec. "Natural
auxiliary functions").  SOMOs count as alpha occupied and beta virtual
(Sec. "PAO construction"), so n_occ_b = n_occ_a - n_somo and
n_vir_b = n_vir_a + n_somo.

Readings of the synthetic recipe:
  * N(0, s) means standard deviation s (numpy ``normal(0, s)``).
  * B^Q_pq per spin: X ~ N(0, s) over the full (occ+vir) range, then
    B = (X + X^T)/sqrt(2), sliced into oo/ov/vv.  alpha and beta are drawn
    independently but share the auxiliary index Q.
  * Same-spin T2: X ~ N(0, s), t = (X - X_ji - X_ba + X_ji,ba)/2, which is
    antisymmetric in (i,j) and in (a,b) with element std s.  The alpha-beta
    block t2ab[i][J][a][B] has no symmetry.
  * Occupied energies U[-1.5,-0.3] Eh, virtual U[0.1,3.0] Eh, each sorted.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

BASE_SEED = 231110048

# (noa, nob, nva, nvb, naux) of the fixed single-domain workloads
SHAPES = {
    "tiny": (5, 4, 30, 31, 120),        # small FP64 domain
    "lno": (40, 38, 300, 302, 1200),     # one LNO-sized domain
    "grad": (20, 18, 160, 162, 640),     # differentiation domain
    "large": (60, 58, 500, 502, 2000),   # large delocalised-SOMO domain
}
# (no, nv, naux) of the closed-shell (SOMO-free) workload: an LNO-sized domain
RHF_SHAPES = {"rhf": (40, 300, 1200)}
# seed offsets of the workloads above, and of the batched set
CONFIG_INDEX = {"tiny": 0, "lno": 1, "batch": 2, "grad": 3, "large": 4, "rhf": 5}


@dataclasses.dataclass
class Domain:
    """One LIS domain, all arrays float64 and C-contiguous.

    Layouts (row-major):
      t1a [noa][nva], t1b [nob][nvb]
      t2aa [noa][noa][nva][nva], t2bb [nob][nob][nvb][nvb]
      t2ab [noa][nob][nva][nvb]   (t^{aB}_{iJ} at [i][J][a][B])
      Boo_x [naux][no_x][no_x], Bov_x [naux][no_x][nv_x], Bvv_x [naux][nv_x][nv_x]
      eo_x [no_x], ev_x [nv_x], fov_x [no_x][nv_x]
    """
    noa: int
    nob: int
    nva: int
    nvb: int
    naux: int
    t1a: np.ndarray
    t1b: np.ndarray
    t2aa: np.ndarray
    t2bb: np.ndarray
    t2ab: np.ndarray
    Boo_a: np.ndarray
    Bov_a: np.ndarray
    Bvv_a: np.ndarray
    Boo_b: np.ndarray
    Bov_b: np.ndarray
    Bvv_b: np.ndarray
    eo_a: np.ndarray
    ev_a: np.ndarray
    eo_b: np.ndarray
    ev_b: np.ndarray
    fov_a: np.ndarray
    fov_b: np.ndarray

    ARRAYS = ("t1a", "t1b", "t2aa", "t2bb", "t2ab", "Boo_a", "Bov_a", "Bvv_a",
              "Boo_b", "Bov_b", "Bvv_b", "eo_a", "ev_a", "eo_b", "ev_b",
              "fov_a", "fov_b")

    @property
    def dims(self):
        return (self.noa, self.nob, self.nva, self.nvb, self.naux)

    def arrays(self):
        return {k: getattr(self, k) for k in self.ARRAYS}

    def replace(self, **kw) -> "Domain":
        return dataclasses.replace(self, **kw)

    def scaled(self, lam_t: float = 1.0, mu_b: float = 1.0, nu_f: float = 1.0,
               lam_t1: Optional[float] = None) -> "Domain":
        """Copy with T2 (and T1) scaled by lam_t, B by mu_b, f_ov by nu_f."""
        l1 = lam_t if lam_t1 is None else lam_t1
        return self.replace(
            t1a=self.t1a * l1, t1b=self.t1b * l1,
            t2aa=self.t2aa * lam_t, t2bb=self.t2bb * lam_t, t2ab=self.t2ab * lam_t,
            Boo_a=self.Boo_a * mu_b, Bov_a=self.Bov_a * mu_b, Bvv_a=self.Bvv_a * mu_b,
            Boo_b=self.Boo_b * mu_b, Bov_b=self.Bov_b * mu_b, Bvv_b=self.Bvv_b * mu_b,
            fov_a=self.fov_a * nu_f, fov_b=self.fov_b * nu_f)


def _antisym(x: np.ndarray) -> np.ndarray:
    """(X - X_ji - X_ba + X_ji,ba)/2 over axes (0,1) and (2,3)."""
    return 0.5 * (x - x.transpose(1, 0, 2, 3) - x.transpose(0, 1, 3, 2)
                  + x.transpose(1, 0, 3, 2))


def _df_factor(rng, naux, no, nv, sigma):
    n = no + nv
    x = rng.normal(0.0, sigma, size=(naux, n, n))
    b = (x + x.transpose(0, 2, 1)) * (1.0 / np.sqrt(2.0))
    del x
    boo = np.ascontiguousarray(b[:, :no, :no])
    bov = np.ascontiguousarray(b[:, :no, no:])
    bvv = np.ascontiguousarray(b[:, no:, no:])
    return boo, bov, bvv


def make_domain(noa: int, nob: int, nva: int, nvb: int, naux: int, seed: int,
                sigma_b: float = 0.05, sigma_t1: float = 1e-3,
                sigma_t2: float = 1e-2, sigma_f: float = 1e-3,
                eocc=(-1.5, -0.3), evir=(0.1, 3.0)) -> Domain:
    """Draw one domain in the fixed order: energies, f_ov, T1, T2, B."""
    for v, name in ((noa, "noa"), (nob, "nob"), (nva, "nva"), (nvb, "nvb"), (naux, "naux")):
        if v < 0:
            raise ValueError(f"{name} must be >= 0")
    rng = np.random.Generator(np.random.PCG64(seed))
    eo_a = np.sort(rng.uniform(eocc[0], eocc[1], size=noa))
    ev_a = np.sort(rng.uniform(evir[0], evir[1], size=nva))
    eo_b = np.sort(rng.uniform(eocc[0], eocc[1], size=nob))
    ev_b = np.sort(rng.uniform(evir[0], evir[1], size=nvb))
    fov_a = rng.normal(0.0, sigma_f, size=(noa, nva))
    fov_b = rng.normal(0.0, sigma_f, size=(nob, nvb))
    t1a = rng.normal(0.0, sigma_t1, size=(noa, nva))
    t1b = rng.normal(0.0, sigma_t1, size=(nob, nvb))
    t2aa = _antisym(rng.normal(0.0, sigma_t2, size=(noa, noa, nva, nva)))
    t2bb = _antisym(rng.normal(0.0, sigma_t2, size=(nob, nob, nvb, nvb)))
    t2ab = rng.normal(0.0, sigma_t2, size=(noa, nob, nva, nvb))
    Boo_a, Bov_a, Bvv_a = _df_factor(rng, naux, noa, nva, sigma_b)
    Boo_b, Bov_b, Bvv_b = _df_factor(rng, naux, nob, nvb, sigma_b)
    c = np.ascontiguousarray
    return Domain(noa, nob, nva, nvb, naux, c(t1a), c(t1b), c(t2aa), c(t2bb), c(t2ab),
                  Boo_a, Bov_a, Bvv_a, Boo_b, Bov_b, Bvv_b,
                  eo_a, ev_a, eo_b, ev_b, c(fov_a), c(fov_b))


def make_rhf_domain(no: int, nv: int, naux: int, seed: int, sigma_b: float = 0.05,
                    sigma_t1: float = 1e-3, sigma_t2: float = 1e-2,
                    sigma_f: float = 1e-3) -> Domain:
    """Closed-shell-consistent domain: alpha and beta data identical.

    Spatial doubles tau^{ab}_{ij} = tau^{ba}_{ji}; t2ab = tau and
    t2aa = t2bb = tau^{ab}_{ij} - tau^{ba}_{ij}.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    eo = np.sort(rng.uniform(-1.5, -0.3, size=no))
    ev = np.sort(rng.uniform(0.1, 3.0, size=nv))
    fov = rng.normal(0.0, sigma_f, size=(no, nv))
    t1 = rng.normal(0.0, sigma_t1, size=(no, nv))
    x = rng.normal(0.0, sigma_t2, size=(no, no, nv, nv))
    tau = (x + x.transpose(1, 0, 3, 2)) * (1.0 / np.sqrt(2.0))
    tss = tau - tau.transpose(0, 1, 3, 2)
    boo, bov, bvv = _df_factor(rng, naux, no, nv, sigma_b)
    c = np.ascontiguousarray
    return Domain(no, no, nv, nv, naux, c(t1), c(t1.copy()), c(tss), c(tss.copy()), c(tau),
                  boo, bov, bvv, boo.copy(), bov.copy(), bvv.copy(),
                  eo, ev, eo.copy(), ev.copy(), c(fov), c(fov.copy()))


RHF_ARRAYS = ("t1", "tau", "Boo", "Bov", "Bvv", "eo", "ev", "fov")


def rhf_arrays(dom: Domain) -> dict:
    """Spatial-orbital arrays of a closed-shell-consistent domain (the alpha
    data; tau is the mixed-spin block)."""
    return {"t1": dom.t1a, "tau": dom.t2ab, "Boo": dom.Boo_a, "Bov": dom.Bov_a, "Bvv": dom.Bvv_a,
            "eo": dom.eo_a, "ev": dom.ev_a, "fov": dom.fov_a}


def rhf_config_domain(name: str) -> Domain:
    no, nv, naux = RHF_SHAPES[name]
    return make_rhf_domain(no, nv, naux, BASE_SEED + 1000 * CONFIG_INDEX[name])


def make_naf_input(no_a: int, nv_a: int, no_b: int, nv_b: int, nx: int, seed: int, sigma: float = 0.05,
                   decay: Optional[float] = None, rotate: bool = True):
    """Three-index integrals J_s [nx][n_s][n_s] (n_s = no_s + nv_s, occupied
    first) of both spins in one auxiliary basis: Z_s ~ N(0, sigma) symmetric
    in the orbital pair, scaled along the auxiliary index by exp(-Y/decay)
    (no scaling without decay) and, with rotate, mixed by one random
    orthogonal matrix shared by the spins."""
    rng = np.random.Generator(np.random.PCG64(seed))
    d = np.ones(nx) if decay is None else np.exp(-np.arange(nx) / float(decay))
    Q = np.linalg.qr(rng.normal(size=(nx, nx)))[0] if (rotate and nx > 0) else None
    out = []
    for no, nv in ((no_a, nv_a), (no_b, nv_b)):
        n = no + nv
        x = rng.normal(0.0, sigma, size=(nx, n, n))
        z = (x + x.transpose(0, 2, 1)) * (1.0 / np.sqrt(2.0))
        del x
        z *= d[:, None, None]
        if Q is not None:
            z = (Q @ z.reshape(nx, n * n)).reshape(nx, n, n)
        out.append(np.ascontiguousarray(z))
    return out[0], out[1]


def config_domain(name: str) -> Domain:
    """The fixed single-domain workloads by name (see SHAPES)."""
    noa, nob, nva, nvb, naux = SHAPES[name]
    return make_domain(noa, nob, nva, nvb, naux, BASE_SEED + 1000 * CONFIG_INDEX[name])


def batch_shapes(ndom: int = 64, seed: Optional[int] = None):
    """Shapes of the uneven batched set: noa ~ U{10..40}, nob = noa - U{1,2},
    nva ~ U{80..320}, nvb = nva + (noa - nob), naux = 4*nva.  Drawn from a
    stream of its own so the shapes do not depend on the value draws."""
    s = BASE_SEED + 1000 * CONFIG_INDEX["batch"] if seed is None else seed
    rng = np.random.Generator(np.random.PCG64(s + 999_999))
    out = []
    for _ in range(ndom):
        noa = int(rng.integers(10, 40, endpoint=True))
        nob = noa - int(rng.integers(1, 2, endpoint=True))
        nva = int(rng.integers(80, 320, endpoint=True))
        nvb = nva + (noa - nob)
        out.append((noa, nob, nva, nvb, 4 * nva))
    return out


def batch_domain(d: int, shapes=None) -> Domain:
    """Domain d of the batched set (values seeded per domain)."""
    shapes = batch_shapes() if shapes is None else shapes
    noa, nob, nva, nvb, naux = shapes[d]
    return make_domain(noa, nob, nva, nvb, naux, BASE_SEED + 1000 * CONFIG_INDEX["batch"] + d)


def flip_spin(dom: Domain) -> Domain:
    """Swap alpha and beta data; t2ab -> [J][i][B][a]."""
    c = np.ascontiguousarray
    return Domain(dom.nob, dom.noa, dom.nvb, dom.nva, dom.naux,
                  dom.t1b, dom.t1a, dom.t2bb, dom.t2aa, c(dom.t2ab.transpose(1, 0, 3, 2)),
                  dom.Boo_b, dom.Bov_b, dom.Bvv_b, dom.Boo_a, dom.Bov_a, dom.Bvv_a,
                  dom.eo_b, dom.ev_b, dom.eo_a, dom.ev_a, dom.fov_b, dom.fov_a)


def _block_lists(noa: int, nob: int):
    aaa = [(0, i, j, k) for i in range(noa) for j in range(i + 1, noa) for k in range(j + 1, noa)]
    aab = [(1, i, j, k) for i in range(noa) for j in range(i + 1, noa) for k in range(nob)]
    abb = [(2, i, j, k) for i in range(nob) for j in range(i + 1, nob) for k in range(noa)]
    bbb = [(3, i, j, k) for i in range(nob) for j in range(i + 1, nob) for k in range(j + 1, nob)]
    return aaa, aab, abb, bbb


def first_items(noa: int, nob: int, per_block: int):
    """The first `per_block` occupied triplets of each spin block in the
    natural enumeration order (the order in which a whole-domain call visits
    and batches them), same row format as sample_items."""
    rows = []
    for cands in _block_lists(noa, nob):
        rows += cands[:per_block]
    return np.asarray(rows, dtype=np.int32).reshape(-1, 4)


def sample_items(noa: int, nob: int, per_block: int, seed: int):
    """Seeded sample of unique occupied triplets, `per_block` per spin block.

    Returns an int32 array [n][4] of (block, p, q, r): block 0 = aaa (i<j<k),
    1 = aab (i<j alpha, K beta), 2 = abb (k alpha, I<J beta; stored as
    (2, I, J, k)), 3 = bbb (I<J<K).  This is an index selection only.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    rows = []

    def pick(cands):
        if len(cands) == 0:
            return []
        sel = rng.choice(len(cands), size=min(per_block, len(cands)), replace=False)
        return [cands[s] for s in sorted(sel)]

    for cands in _block_lists(noa, nob):
        rows += pick(cands)
    return np.asarray(rows, dtype=np.int32).reshape(-1, 4)


def central_inputs(no: int, nq: int, seed: int):
    """Inputs of a central-orbital share: a seeded unit vector over `no`
    occupied orbitals, and nq positive quadrature points and weights (seeded
    draws; the share is defined for any of them).  Draws only."""
    rng = np.random.Generator(np.random.PCG64(seed))
    c = rng.normal(size=no)
    c /= np.linalg.norm(c)
    s = np.sort(rng.uniform(0.05, 2.0, size=nq))
    w = rng.uniform(0.1, 1.0, size=nq)
    return c, s, w
