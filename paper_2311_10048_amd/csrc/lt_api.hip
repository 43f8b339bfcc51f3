// C ABI of ltriples: validation, planning, workspace layout and the launch
// sequence of the (T) energy of one domain.
//
// Launch sequence (all on the caller's stream):
//  1. convert/copy the DF factors into k-major, padded operand layouts;
//  2. FP64 builds of the small integral classes (ov|oo) and (ov|ov) and the
//     operands derived from them (<ma||jk>, (aj|MK), (jm|CK), <qr||yz>);
//  3. amplitude operands (transposed, pair-packed, spin-permuted copies);
//  4. the (ov|vv) slabs <ei||bc> (pair packed), (jb|EC), (be|KC) built by
//     MFMA GEMMs over the auxiliary index;
//  5. per spin block, batches of occupied triplets: contraction GEMMs into
//     batch buffers, then the FP64 energy epilogue and per-item reduction;
//  6. per-block parts and the total, summed in a fixed order.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <map>
#include <mutex>
#include <vector>

#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include "lt_internal.h"
#include "ltriples.h"

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIPCHK(...)                                                                  \
  do {                                                                               \
    hipError_t e_ = (__VA_ARGS__);                                                   \
    if (e_ != hipSuccess)                                                            \
      return fail(LT_EHIP, "HIP error %s at %s:%d", hipGetErrorString(e_), __FILE__, \
                  __LINE__);                                                         \
  } while (0)

inline int64_t ld4(int64_t n) { return (n + 3) & ~int64_t(3); }
inline int64_t npair(int64_t n) { return n * (n - 1) / 2; }
inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline size_t align256(size_t n) { return (n + 255) & ~size_t(255); }

// o: occupied orbitals per spin (they index the amplitudes, factors and
// items); oi: the first oi of them are the ones the contractions sum over.
// oi = o, except for a central-orbital share, whose rotated central
// orbitals are appended after the LIS orbitals and only ever appear as an
// item's own (external) index.
struct Dims {
  int64_t o[2], v[2], Q, oi[2];
};

Dims dims_of(const ltriples_domain* d) {
  Dims x;
  x.o[0] = d->noa; x.o[1] = d->nob; x.v[0] = d->nva; x.v[1] = d->nvb; x.Q = d->naux;
  x.oi[0] = x.o[0]; x.oi[1] = x.o[1];
  return x;
}

// block b -> (sigma, is_mixed): 0 aaa, 1 aab (sigma=a), 2 abb (sigma=b), 3 bbb
inline int blk_sigma(int b) { return (b == 0 || b == 1) ? 0 : 1; }
inline bool blk_mixed(int b) { return b == 1 || b == 2; }

int check_items(const Dims& D, const ltriples_options* o) {
  if (!o || !o->items) return LT_OK;
  if (o->n_items < 0) return fail(LT_EINVAL, "n_items < 0");
  for (int32_t n = 0; n < o->n_items; ++n) {
    const int32_t* it = o->items + 4 * n;
    const int b = it[0];
    if (b < 0 || b > 3) return fail(LT_ESHAPE, "item %d: bad block %d", n, b);
    const int s = blk_sigma(b);
    const int64_t os = D.o[s], ot = D.o[1 - s];
    if (blk_mixed(b)) {
      if (!(0 <= it[1] && it[1] < it[2] && it[2] < os && 0 <= it[3] && it[3] < ot))
        return fail(LT_ESHAPE, "item %d: bad indices (%d,%d,%d,%d)", n, b, it[1], it[2], it[3]);
    } else {
      if (!(0 <= it[1] && it[1] < it[2] && it[2] < it[3] && it[3] < os))
        return fail(LT_ESHAPE, "item %d: bad indices (%d,%d,%d,%d)", n, b, it[1], it[2], it[3]);
    }
  }
  return LT_OK;
}

int validate_options(const ltriples_options* o) {
  if (!o) return LT_OK;
  for (int k = 0; k < 3; ++k)
    if (o->tile_override[k] < 0 || o->tile_override[k] > 8)
      return fail(LT_EINVAL, "tile_override[%d] = %d outside 0..8", k, o->tile_override[k]);
  if (o->check_finite != 0 && o->check_finite != 1) return fail(LT_EINVAL, "check_finite must be 0 or 1");
  return LT_OK;
}

int validate(const ltriples_domain* d, int32_t prec, const ltriples_options* o) {
  if (!d) return fail(LT_EINVAL, "domain is NULL");
  if (d->noa < 0 || d->nob < 0 || d->nva < 0 || d->nvb < 0 || d->naux < 0)
    return fail(LT_EINVAL, "negative dimension");
  if (prec != LT_FP64 && prec != LT_FP32 && prec != LT_BF16X3 && prec != LT_BF16)
    return fail(LT_EPREC, "unsupported precision %d", prec);
  const int64_t oa = d->noa, ob = d->nob, va = d->nva, vb = d->nvb, Q = d->naux;
  // per-dimension limits first, so that the element counts below cannot overflow
  if (va > 46340 || vb > 46340 || oa > 4096 || ob > 4096 || Q > (int64_t(1) << 24))
    return fail(LT_ESHAPE, "dimension too large");
  struct P { const double* p; int64_t n; const char* name; } ps[] = {
      {d->t1a, oa * va, "t1a"}, {d->t1b, ob * vb, "t1b"},
      {d->t2aa, oa * oa * va * va, "t2aa"}, {d->t2bb, ob * ob * vb * vb, "t2bb"},
      {d->t2ab, oa * ob * va * vb, "t2ab"},
      {d->Boo_a, Q * oa * oa, "Boo_a"}, {d->Bov_a, Q * oa * va, "Bov_a"}, {d->Bvv_a, Q * va * va, "Bvv_a"},
      {d->Boo_b, Q * ob * ob, "Boo_b"}, {d->Bov_b, Q * ob * vb, "Bov_b"}, {d->Bvv_b, Q * vb * vb, "Bvv_b"},
      {d->eo_a, oa, "eo_a"}, {d->ev_a, va, "ev_a"}, {d->eo_b, ob, "eo_b"}, {d->ev_b, vb, "ev_b"},
      {d->fov_a, oa * va, "fov_a"}, {d->fov_b, ob * vb, "fov_b"}};
  for (auto& x : ps)
    if (x.n > 0 && !x.p) return fail(LT_EINVAL, "%s is NULL", x.name);
  if ((va > 0 || vb > 0) && (oa + ob) >= 3 && Q == 0)
    return fail(LT_ESHAPE, "naux = 0");
  // FP64 inputs beyond 1 TiB cannot be resident on one device; the bound also
  // keeps every workspace size the planner derives far from size_t overflow
  int64_t total = 0;
  for (auto& x : ps) total += x.n;   // each term below 2^56 under the limits above
  if (total > (int64_t(1) << 37))
    return fail(LT_ESHAPE, "inputs too large (%lld FP64 elements, limit 2^37)", (long long)total);
  if (o && o->items && o->n_items > 0) {
    const int r = check_items(dims_of(d), o);
    if (r) return r;
  }
  if (o && o->items == nullptr && o->n_items != 0)
    return fail(LT_EINVAL, "n_items given without items");
  return validate_options(o);
}

// Items grouped by block: trip (p,q,r) and the caller-order index.
struct ItemLists {
  std::vector<int32_t> trip[4];
  std::vector<int32_t> dst[4];
  int64_t total = 0;
};

void build_items(const Dims& D, const ltriples_options* o, ItemLists& L) {
  if (o && o->items) {
    // each block's items in canonical (p, q, r) order, whatever the caller's
    // order: batches, launch order and every reduction order then depend on
    // the item set only (per-item values still go to the caller's positions)
    std::vector<std::array<int32_t, 4>> blk[4];
    for (int32_t n = 0; n < o->n_items; ++n) {
      const int32_t* it = o->items + 4 * n;
      blk[it[0]].push_back({it[1], it[2], it[3], n});
    }
    for (int b = 0; b < 4; ++b) {
      std::stable_sort(blk[b].begin(), blk[b].end(), [](const std::array<int32_t, 4>& x,
                                                          const std::array<int32_t, 4>& y) {
        return x[0] != y[0] ? x[0] < y[0] : x[1] != y[1] ? x[1] < y[1] : x[2] < y[2];
      });
      for (auto& x : blk[b]) {
        L.trip[b].insert(L.trip[b].end(), {x[0], x[1], x[2]});
        L.dst[b].push_back(x[3]);
      }
    }
    L.total = o->n_items;
    return;
  }
  int32_t n = 0;
  const int32_t oa = (int32_t)D.o[0], ob = (int32_t)D.o[1];
  for (int32_t i = 0; i < oa; ++i)
    for (int32_t j = i + 1; j < oa; ++j)
      for (int32_t k = j + 1; k < oa; ++k) { L.trip[0].insert(L.trip[0].end(), {i, j, k}); L.dst[0].push_back(n++); }
  for (int32_t i = 0; i < oa; ++i)
    for (int32_t j = i + 1; j < oa; ++j)
      for (int32_t k = 0; k < ob; ++k) { L.trip[1].insert(L.trip[1].end(), {i, j, k}); L.dst[1].push_back(n++); }
  for (int32_t i = 0; i < ob; ++i)
    for (int32_t j = i + 1; j < ob; ++j)
      for (int32_t k = 0; k < oa; ++k) { L.trip[2].insert(L.trip[2].end(), {i, j, k}); L.dst[2].push_back(n++); }
  for (int32_t i = 0; i < ob; ++i)
    for (int32_t j = i + 1; j < ob; ++j)
      for (int32_t k = j + 1; k < ob; ++k) { L.trip[3].insert(L.trip[3].end(), {i, j, k}); L.dst[3].push_back(n++); }
  L.total = n;
}

int64_t count_all_items(const Dims& D) {
  const int64_t oa = D.o[0], ob = D.o[1];
  return oa * (oa - 1) * (oa - 2) / 6 + oa * (oa - 1) / 2 * ob + ob * (ob - 1) / 2 * oa +
         ob * (ob - 1) * (ob - 2) / 6;
}

// the occupied contraction lengths are the summed orbitals (oi)
double item_flops(const Dims& D, int b) {
  const int s = blk_sigma(b), t = 1 - s;
  const double o = (double)D.oi[s], v = (double)D.v[s], ot = (double)D.oi[t], vt = (double)D.v[t];
  if (!blk_mixed(b)) return 6 * v * v * v * v + 6 * v * v * v * o;
  return 4 * v * v * vt * vt + 6 * v * v * v * vt + 4 * v * v * vt * ot + 6 * v * v * vt * o;
}

// ---------------------------------------------------------------------------
// Workspace plan
// ---------------------------------------------------------------------------
struct Buf { size_t off = 0, bytes = 0; };

struct Plan {
  int prec = 0;
  size_t ts = 8;          // compute element size
  Dims D;
  int64_t n_blk[4] = {0, 0, 0, 0};
  bool need_as[2] = {false, false};     // As, Tp, T2T, GamT, U of spin s
  bool need_mix[2] = {false, false};    // mixed block with pair spin s
  bool any_mix = false;
  int64_t ldv[2], ldvv[2], ldnp[2], ldcb[2], ldov[2], ldoo[2];
  // persistent
  Buf BvvP[2], BovR[2], BovP64[2], BooP64[2];
  Buf As[2], Tp[2], T2T[2], GamT[2], U[2];
  Buf LmixT[2], Mst[2], Mts[2], Tmix[2], ZpT[2], TmT[2], OOT[2];
  Buf OVab, e_items, trip, dst, order, firstcnt, flag, segtab;
  // adjoint pass: extra operands, mirrors (gradients of the prepared
  // operands, same layouts), FP64 four-index integral gradients, descriptors
  bool bwd = false;
  Buf T1p[2], Fp[2], Up[2], OVc[2], BvvP64[2];
  Buf dT2T[2], dTp[2], dAs[2], dGamT[2], dUp[2], dT1p[2], dFp[2];
  Buf dLmixT[2], dMst[2], dMts[2], dTmix[2], dZpT[2], dTmT[2], dOOT[2], dOVc[2];
  Buf dOVVV[2][2], dOVOO[2][2], dOVOV[3];   // ovov: aa, bb, ab
  Buf rblk, rseg, dfblk, dfseg, rred, dfred, rpart;
  // BF16 modes: hi/lo octet copies of the contraction operands
  int bf = 0;                     // 0: none, 3: split products, 1: plain bf16
  // BF16X3 adjoint: the FP32 operands stay resident for the reverse GEMMs
  // beside their octet copies (the forward keeps only the octets)
  bool keep32 = false;
  enum { T2T8, As8, GamT8, Tp8, LmixT8, Mst8, Mts8, Tmix8, Tmx28, ZpT8, TmT8, OOT8, NT8 };
  Buf O8h[2][NT8], O8l[2][NT8];
  // operand builds split along their leading occupied index: blocks per
  // chunk of <ei||bc> (and its (eb|ic) intermediate), (jb|EC), (be|KC) and
  // of the same-spin (ov|ov) rows behind <qr||yz>
  int64_t cAs[2] = {1, 1}, cMst[2] = {1, 1}, cMts[2] = {1, 1}, cOV[2] = {1, 1};
  Buf stage;                      // BF16 modes: staging of one FP32 operand tensor (or chunk)
  // scratch
  Buf scratch;
  size_t sc_OO[2][2], sc_OV;      // offsets within scratch (phase 1a)
  int64_t nb[4];                  // items per batch
  size_t per_item[4];             // batch bytes per item (T outputs)
  size_t o1[4], o2[4];            // aligned per-item bytes of the two output layouts
  size_t part_off[4];             // partials offset within scratch (phase 2)
  int64_t ntile[4];
  int64_t bwg[4];                 // backward epilogue tiles per item
  int64_t ld_ri[4];               // orbital-energy adjoint: per-item index sums
  size_t big = 0, small = 0, small_base = 0, total = 0;
  // central-orbital share: device table [nq][2] of (point, signed weight)
  // and the spin of the central orbital (-1: an ordinary energy)
  const double* lap = nullptr;
  int lap_spin = -1;
  // debug dump (a call with a single item): that item's W cube, FP64
  double* dump_w = nullptr;
};

// `oi` (optional): the summed occupied orbitals per spin, when they are fewer
// than the domain's (a central-orbital share); default all of them.
void plan_domain(const ltriples_domain* d, int32_t prec, const ltriples_options* o,
                 const ItemLists& L, Plan& P, bool bwd = false, const int64_t* oi = nullptr) {
  P.prec = prec;
  P.bwd = bwd;
  P.ts = prec == LT_FP64 ? 8 : 4;   // BF16 modes prepare FP32 operands, then split them
  P.D = dims_of(d);
  if (oi) { P.D.oi[0] = oi[0]; P.D.oi[1] = oi[1]; }
  const Dims& D = P.D;
  for (int b = 0; b < 4; ++b) P.n_blk[b] = (int64_t)L.dst[b].size();
  for (int b = 0; b < 4; ++b)
    if (P.n_blk[b] > 0) {
      P.need_as[blk_sigma(b)] = true;
      if (blk_mixed(b)) { P.need_mix[blk_sigma(b)] = true; P.any_mix = true; }
    }
  for (int s = 0; s < 2; ++s) {
    P.ldv[s] = ld4(D.v[s]);
    P.ldvv[s] = ld4(D.v[s] * D.v[s]);
    P.ldnp[s] = ld4(npair(D.v[s]));
    P.ldcb[s] = ld4(D.v[s] * D.v[1 - s]);
    P.ldov[s] = ld4(D.o[s] * D.v[s]);
    P.ldoo[s] = ld4(D.o[s] * D.o[s]);
  }
  size_t off = 0;
  P.bf = prec == LT_BF16X3 ? 3 : (prec == LT_BF16 ? 1 : 0);
  P.keep32 = bwd && P.bf;
  // BF16 energies keep only the split (octet) copies of the contraction
  // operands: every FP32 operand tensor is built in one shared staging
  // buffer and split before the next one is built.  The BF16X3 adjoint keeps
  // both (the reverse GEMMs read the FP32 operands).
  std::vector<std::pair<Buf*, size_t>> staged;
  auto take = [&](Buf& b, size_t bytes) { b.off = off; b.bytes = bytes; off = align256(off + bytes); };
  auto take_op = [&](Buf& b, size_t bytes, size_t stage_bytes = 0) {
    if (!P.bf || P.keep32) { take(b, bytes); return; }
    b.bytes = bytes;
    staged.push_back({&b, stage_bytes ? stage_bytes : bytes});
  };
  const size_t ts = P.ts;
  const int64_t Q = D.Q;
  // chunks of the big operand builds: at most build_chunk_mib MiB each
  const size_t cap = (size_t)((o && o->build_chunk_mib > 0) ? o->build_chunk_mib : 2048) << 20;
  auto per_chunk = [&](int64_t nblk, size_t blk_bytes) -> int64_t {
    return std::max<int64_t>(1, std::min<int64_t>(nblk, (int64_t)(cap / std::max<size_t>(blk_bytes, 1))));
  };
  for (int s = 0; s < 2; ++s) {
    const int t = 1 - s;
    const int64_t os = D.o[s], vs = D.v[s], ot = D.o[t], vt = D.v[t];
    P.cAs[s] = per_chunk(os, ts * (size_t)(vs * vs * P.ldv[s]));   // (eb|ic) rows of one i
    P.cMst[s] = per_chunk(os, ts * (size_t)(vt * P.ldcb[s]));
    P.cMts[s] = per_chunk(ot, ts * (size_t)(vs * P.ldcb[s]));
    P.cOV[s] = per_chunk(os, 8 * (size_t)(vs * os * vs));          // (ov|ov) rows of one q
  }
  for (int s = 0; s < 2; ++s) {
    const bool need_df = P.need_as[s] || P.any_mix;
    const int64_t os = D.o[s], vs = D.v[s];
    if (need_df) {
      take(P.BvvP[s], ts * Q * P.ldvv[s]);
      take(P.BovR[s], ts * os * Q * P.ldv[s]);
      take(P.BovP64[s], 8 * Q * P.ldov[s]);
      take(P.BooP64[s], 8 * Q * P.ldoo[s]);
    }
    if (P.need_as[s]) {
      take_op(P.As[s], ts * os * vs * P.ldnp[s], ts * P.cAs[s] * vs * P.ldnp[s]);
      take_op(P.Tp[s], ts * os * os * P.ldnp[s]);
      take_op(P.T2T[s], ts * os * os * vs * P.ldv[s]);
      take_op(P.GamT[s], ts * os * os * os * P.ldv[s]);
      take(P.U[s], 8 * os * os * vs * P.ldv[s]);
    }
    if (P.need_mix[s]) {
      const int t = 1 - s;
      const int64_t ot = D.o[t], vt = D.v[t];
      take_op(P.LmixT[s], ts * os * ot * vt * P.ldv[s]);
      take_op(P.Mst[s], ts * os * vt * P.ldcb[s], ts * P.cMst[s] * vt * P.ldcb[s]);
      take_op(P.Mts[s], ts * ot * vs * P.ldcb[s], ts * P.cMts[s] * vs * P.ldcb[s]);
      take_op(P.Tmix[s], ts * os * ot * P.ldcb[s]);
      take_op(P.ZpT[s], ts * os * ot * ot * P.ldv[s]);
      take_op(P.TmT[s], ts * os * ot * vs * P.ldv[t]);
      take_op(P.OOT[s], ts * ot * os * os * P.ldv[t]);
    }
  }
  if (!staged.empty()) {
    size_t mx = 0;
    for (auto& b : staged) mx = std::max(mx, b.second);
    take(P.stage, mx);
    for (auto& b : staged) b.first->off = P.stage.off;
  }
  if (P.any_mix) take(P.OVab, 8 * D.o[0] * D.v[0] * D.o[1] * D.v[1]);
  if (bwd) {
    for (int s = 0; s < 2; ++s) {
      const int t = 1 - s;
      const int64_t os = D.o[s], vs = D.v[s], ot = D.o[t], vt = D.v[t];
      const bool need_df = P.need_as[s] || P.any_mix;
      if (need_df) take(P.BvvP64[s], 8 * Q * P.ldvv[s]);
      if (need_df) { take(P.T1p[s], ts * os * P.ldv[s]); take(P.Fp[s], ts * os * P.ldv[s]); }
      if (need_df) { take(P.dT1p[s], ts * os * P.ldv[s]); take(P.dFp[s], ts * os * P.ldv[s]); }
      if (P.need_as[s]) {
        take(P.Up[s], ts * os * os * P.ldnp[s]);
        take(P.dAs[s], P.As[s].bytes); take(P.dTp[s], P.Tp[s].bytes); take(P.dT2T[s], P.T2T[s].bytes);
        take(P.dGamT[s], P.GamT[s].bytes); take(P.dUp[s], P.Up[s].bytes);
      }
      if (P.need_mix[s]) {
        take(P.OVc[s], ts * os * ot * P.ldcb[s]);
        take(P.dLmixT[s], P.LmixT[s].bytes); take(P.dMst[s], P.Mst[s].bytes); take(P.dMts[s], P.Mts[s].bytes);
        take(P.dTmix[s], P.Tmix[s].bytes); take(P.dZpT[s], P.ZpT[s].bytes); take(P.dTmT[s], P.TmT[s].bytes);
        take(P.dOOT[s], P.OOT[s].bytes); take(P.dOVc[s], P.OVc[s].bytes);
      }
      (void)vt;
    }
    for (int x = 0; x < 2; ++x)
      for (int y = 0; y < 2; ++y) {
        const bool need = x == y ? P.need_as[x] : (P.need_mix[x] || P.need_mix[y]);
        if (!need) continue;
        take(P.dOVVV[x][y], 8 * D.o[x] * D.v[x] * P.ldvv[y]);
        take(P.dOVOO[x][y], 8 * D.o[x] * D.v[x] * P.ldoo[y]);
      }
    for (int s = 0; s < 2; ++s)
      if (P.need_as[s]) take(P.dOVOV[s], 8 * D.o[s] * D.v[s] * P.ldov[s]);
    if (P.any_mix) take(P.dOVOV[2], 8 * D.o[0] * D.v[0] * P.ldov[1]);
  }
  if (P.bf) {
    auto k16 = [](int64_t k) { return (k + 15) & ~int64_t(15); };
    auto take8 = [&](int s, int t, int64_t nblk, int64_t K, int64_t ld) {
      const size_t bytes = 2 * (size_t)(nblk * k16(K) * ld) + 2 * 8 * 512;
      take(P.O8h[s][t], bytes);
      take(P.O8l[s][t], bytes);
    };
    for (int s = 0; s < 2; ++s) {
      const int t = 1 - s;
      const int64_t os = D.o[s], vs = D.v[s], ot = D.o[t], vt = D.v[t];
      const int64_t ois = D.oi[s], oit = D.oi[t];   // occupied contraction rows
      if (P.need_as[s]) {
        take8(s, Plan::T2T8, os * os, vs, P.ldv[s]);
        take8(s, Plan::As8, os, vs, P.ldnp[s]);
        take8(s, Plan::GamT8, os * os, ois, P.ldv[s]);
        take8(s, Plan::Tp8, os, ois, P.ldnp[s]);
      }
      if (P.need_mix[s]) {
        take8(s, Plan::LmixT8, os * ot, vt, P.ldv[s]);
        take8(s, Plan::Mst8, os, vt, P.ldcb[s]);
        take8(s, Plan::Mts8, ot, vs, P.ldcb[s]);
        take8(s, Plan::Tmix8, os, oit, P.ldcb[s]);
        take8(s, Plan::Tmx28, ot, ois, P.ldcb[s]);
        take8(s, Plan::ZpT8, os * ot, oit, P.ldv[s]);
        take8(s, Plan::TmT8, os * ot, vs, P.ldv[t]);
        take8(s, Plan::OOT8, ot * os, ois, P.ldv[t]);
      }
    }
  }

  // scratch, phase 1a: (ov|oo) classes and same-spin (ov|ov)
  size_t s1a = 0;
  for (int x = 0; x < 2; ++x)
    for (int y = 0; y < 2; ++y) {
      const bool need = (x == y) ? P.need_as[x] : P.any_mix;
      P.sc_OO[x][y] = s1a;
      if (need) s1a = align256(s1a + 8 * (size_t)(D.o[x] * D.v[x] * D.o[y] * D.o[y]));
    }
  {
    P.sc_OV = s1a;                 // one chunk of (ov|ov) rows, both spins in turn
    size_t ov = 0;
    for (int s = 0; s < 2; ++s)
      if (P.need_as[s]) ov = std::max(ov, 8 * (size_t)(P.cOV[s] * D.v[s] * D.o[s] * D.v[s]));
    s1a = align256(s1a + ov);
  }
  // phase 1b: (eb|ic) of one chunk of i before pair packing
  size_t s1b = 0;
  for (int s = 0; s < 2; ++s)
    if (P.need_as[s]) s1b = std::max(s1b, ts * (size_t)(P.cAs[s] * D.v[s] * D.v[s] * P.ldv[s]));
  // phase 2: batch buffers + partials.  Default budget: 8 GiB for the energy
  // (16 GiB measured slower on the LNO-sized domain, 20.39 against 20.18 s);
  // 32 GiB for the adjoint, whose reverse GEMMs gain from long concatenated
  // contractions (gradient workload (20,18,160,162,640): FP32 4.40 s with
  // 8 GiB, 4.07 s with 16, 3.93 s with 32; FP64 7.82, 7.08, 6.62 s)
  const size_t budget = (o && o->workspace_budget) ? o->workspace_budget : (size_t(bwd ? 32 : 8) << 30);
  size_t s2 = 0;
  for (int b = 0; b < 4; ++b) {
    P.nb[b] = 0; P.per_item[b] = 0; P.ntile[b] = 0; P.part_off[b] = 0; P.bwg[b] = 0; P.ld_ri[b] = 0;
    if (P.n_blk[b] == 0) continue;
    const int s = blk_sigma(b), t = 1 - s;
    const int64_t vs = D.v[s], vt = D.v[t];
    size_t outb;
    int64_t nt;
    if (!blk_mixed(b)) {
      outb = ts * (size_t)(vs * P.ldnp[s]);
      const int64_t n = cdiv(vs, lt::ET);
      nt = n * (n + 1) / 2;            // one partial per (a-tile <= b-tile) pair
    } else {
      outb = ts * (size_t)(vs * P.ldcb[s] + vt * P.ldnp[s]);
      const int64_t ns = cdiv(vs, lt::ET);
      nt = ns * (ns + 1) / 2;          // one partial per (a-tile <= b-tile) pair
    }
    P.ntile[b] = nt;
    P.o1[b] = align256(ts * (size_t)(blk_mixed(b) ? vs * P.ldcb[s] : vs * P.ldnp[s]));
    P.o2[b] = blk_mixed(b) ? align256(ts * (size_t)(vt * P.ldnp[s])) : 0;
    if (bwd) {
      const int64_t ns = cdiv(vs, lt::ET), nv = cdiv(vt, lt::ET);
      P.bwg[b] = blk_mixed(b) ? ns * (ns + 1) / 2 * nv : ns * (ns + 1) * (ns + 2) / 6;
      P.ld_ri[b] = ld4(vs + (blk_mixed(b) ? vt : 0) + 1);
    }
    // backward: three output copies, then the orbital-energy tile sums and
    // per-item index sums (after all batch outputs, see run_bwd)
    const size_t per = (bwd ? 3 : 1) * (P.o1[b] + P.o2[b]) + align256(8 * 3 * (size_t)std::max<int64_t>(nt, 1)) +
                       (bwd ? 512 * (size_t)P.bwg[b] + 8 * (size_t)P.ld_ri[b] : 0);
    P.per_item[b] = outb;
    int64_t nb = (o && o->batch_items > 0) ? o->batch_items : (int64_t)std::max<size_t>(1, budget / per);
    nb = std::min<int64_t>(nb, P.n_blk[b]);
    nb = std::min<int64_t>(nb, 65535);
    P.nb[b] = nb;
    const size_t need = (size_t)nb * per + 1024;
    s2 = std::max(s2, need);
  }
  const size_t sc = std::max(std::max(s1a, s1b), s2);
  take(P.scratch, std::max<size_t>(sc, 256));
  P.big = off;
  // per-domain small buffers (item lists, per-item energies), addressed
  // relative to small_base so that a batch of domains can share the big part
  off = 0;
  take(P.e_items, 8 * 3 * std::max<int64_t>(L.total, 1));
  take(P.trip, 4 * 3 * std::max<int64_t>(L.total, 1));
  take(P.dst, 4 * std::max<int64_t>(L.total, 1));
  take(P.order, 4 * std::max<int64_t>(L.total, 1));
  take(P.firstcnt, 4 * 8);
  take(P.flag, 4);
  if (P.bf) take(P.segtab, 2 * 6 * sizeof(lt::Seg8) * (size_t)std::max<int64_t>(L.total, 1));
  P.small = off;
  P.small_base = P.big;
  P.total = P.big + P.small;
}

// The BF16 contraction addresses a tensor's lo half through 32-bit octet
// offsets from its hi half.
int check_plan(const Plan& P) {
  if (!P.bf) return LT_OK;
  for (int s = 0; s < 2; ++s)
    for (int t8 = 0; t8 < Plan::NT8; ++t8)
      if (P.O8h[s][t8].bytes && P.O8l[s][t8].off - P.O8h[s][t8].off >= (size_t(1) << 36))
        return fail(LT_ESHAPE, "BF16 operand tensor too large (over 64 GiB per half)");
  return LT_OK;
}

void log_plan(const Plan& P) {
  if (!getenv("LTRIPLES_LOG")) return;
  fprintf(stderr, "[ltriples] plan prec=%d total=%zu bytes\n", P.prec, P.total);
  const char* sp = "ab";
  auto pr = [&](const char* n, int s, const Buf& b) {
    if (b.bytes) fprintf(stderr, "[ltriples] buf %s_%c off=%zu bytes=%zu\n", n, sp[s], b.off, b.bytes);
  };
  for (int s = 0; s < 2; ++s) {
    pr("BvvP", s, P.BvvP[s]); pr("BovR", s, P.BovR[s]); pr("BovP64", s, P.BovP64[s]); pr("BooP64", s, P.BooP64[s]);
    pr("As", s, P.As[s]); pr("Tp", s, P.Tp[s]); pr("T2T", s, P.T2T[s]); pr("GamT", s, P.GamT[s]); pr("U", s, P.U[s]);
    pr("LmixT", s, P.LmixT[s]); pr("Mst", s, P.Mst[s]); pr("Mts", s, P.Mts[s]); pr("Tmix", s, P.Tmix[s]);
    pr("ZpT", s, P.ZpT[s]); pr("TmT", s, P.TmT[s]); pr("OOT", s, P.OOT[s]);
  }
  pr("OVab", 0, P.OVab);
  pr("scratch", 0, P.scratch);
  for (int b = 0; b < 4; ++b)
    if (P.n_blk[b])
      fprintf(stderr, "[ltriples] block %d items=%lld batch=%lld tiles=%lld\n", b, (long long)P.n_blk[b],
              (long long)P.nb[b], (long long)P.ntile[b]);
}

template <typename T> T* at(void* ws, const Buf& b) { return (T*)((char*)ws + b.off); }
template <typename T> T* at_small(void* ws, const Plan& P, const Buf& b) {
  return (T*)((char*)ws + P.small_base + b.off);
}

// HIP-event timing of the call's phases (only when the caller asks for stats)
struct Timing {
  bool on = false;
  hipStream_t st = nullptr;
  std::vector<hipEvent_t> evs;
  hipEvent_t start = nullptr, setup_end = nullptr, end = nullptr;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> gemm, epi;
  double gemm_flops = 0;
  hipEvent_t mark() {
    if (!on) return nullptr;
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    (void)hipEventRecord(e, st);
    evs.push_back(e);
    return e;
  }
  ~Timing() { for (auto e : evs) (void)hipEventDestroy(e); }
  static double ms(hipEvent_t a, hipEvent_t b) {
    float x = 0.f;
    if (a && b) (void)hipEventElapsedTime(&x, a, b);
    return (double)x;
  }
};

// ---------------------------------------------------------------------------
// Launch sequence
// ---------------------------------------------------------------------------
// Block-ordered item arrays of a domain (host side).
struct HostItems {
  std::vector<int32_t> trip, dst;
  int32_t fc[8];
};

void host_items(const ItemLists& L, HostItems& H) {
  for (int b = 0; b < 4; ++b) {
    H.fc[b] = (int32_t)H.dst.size();
    H.fc[4 + b] = (int32_t)L.dst[b].size();
    H.trip.insert(H.trip.end(), L.trip[b].begin(), L.trip[b].end());
    H.dst.insert(H.dst.end(), L.dst[b].begin(), L.dst[b].end());
  }
}

// Copies the item arrays to the domain's small buffers and waits for the
// copies (host vectors are released afterwards).  Not capturable.
int upload_items(const Plan& P, const ItemLists& L, void* ws, hipStream_t st) {
  HostItems H;
  host_items(L, H);
  if (!H.trip.empty()) {
    HIPCHK(hipMemcpyAsync(at_small<int32_t>(ws, P, P.trip), H.trip.data(), H.trip.size() * 4,
                          hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(at_small<int32_t>(ws, P, P.dst), H.dst.data(), H.dst.size() * 4,
                          hipMemcpyHostToDevice, st));
  }
  HIPCHK(hipMemcpyAsync(at_small<int32_t>(ws, P, P.firstcnt), H.fc, sizeof(H.fc), hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  return LT_OK;
}

// Operand preparation (steps 1-4 of the launch sequence): kernels only.
template <typename T>
int prep(const ltriples_domain* d, const Plan& P, void* ws, hipStream_t st) {
  const Dims& D = P.D;
  const int64_t Q = D.Q;
  const double* Bvv[2] = {d->Bvv_a, d->Bvv_b};
  const double* Bov[2] = {d->Bov_a, d->Bov_b};
  const double* Boo[2] = {d->Boo_a, d->Boo_b};
  const double* T2ss[2] = {d->t2aa, d->t2bb};
  char* scr = (char*)ws + P.scratch.off;
  // BF16 modes: split one freshly built FP32 operand tensor into its hi/lo
  // octet copies (the FP32 tensors share one staging buffer)
  auto split_op = [&](int s, int t8) -> hipError_t {
    if (!P.bf) return hipSuccess;
    const int t = 1 - s;
    const int64_t os = D.o[s], vs = D.v[s], ot = D.o[t], vt = D.v[t], ois = D.oi[s], oit = D.oi[t];
    const int64_t lv = P.ldv[s], lvt = P.ldv[t], lp = P.ldnp[s], lc = P.ldcb[s], np = npair(vs);
    auto sp = [&](int64_t nblk, int64_t K, int64_t ld, int64_t ncol, const Buf& in, int64_t ibs,
                  int64_t iks) -> hipError_t {
      return lt::launch_split8(at<lt::bf16_t>(ws, P.O8h[s][t8]), at<lt::bf16_t>(ws, P.O8l[s][t8]), nblk,
                               (int32_t)K, ld, (int32_t)ncol, at<float>(ws, in), ibs, iks, st);
    };
    switch (t8) {
      case Plan::T2T8: return sp(os * os, vs, lv, vs, P.T2T[s], vs * lv, lv);
      case Plan::As8: return sp(os, vs, lp, np, P.As[s], vs * lp, lp);
      case Plan::GamT8: return sp(os * os, ois, lv, vs, P.GamT[s], os * lv, lv);
      case Plan::Tp8: return sp(os, ois, lp, np, P.Tp[s], os * lp, lp);
      case Plan::LmixT8: return sp(os * ot, vt, lv, vs, P.LmixT[s], vt * lv, lv);
      case Plan::Mst8: return sp(os, vt, lc, vt * vs, P.Mst[s], vt * lc, lc);
      case Plan::Mts8: return sp(ot, vs, lc, vt * vs, P.Mts[s], vs * lc, lc);
      case Plan::Tmix8: return sp(os, oit, lc, vt * vs, P.Tmix[s], ot * lc, lc);
      case Plan::Tmx28: return sp(ot, ois, lc, vt * vs, P.Tmix[s], lc, ot * lc);
      case Plan::ZpT8: return sp(os * ot, oit, lv, vs, P.ZpT[s], ot * lv, lv);
      case Plan::TmT8: return sp(os * ot, vs, lvt, vt, P.TmT[s], vs * lvt, lvt);
      default: return sp(ot * os, ois, lvt, vt, P.OOT[s], os * lvt, lvt);
    }
  };
  // BF16 modes: split blocks [b0, b0 + n) of a chunked operand, built in the
  // staging buffer (or, for the BF16X3 adjoint, in place), into their octet
  // copies
  auto split_chunk = [&](int s, int t8, int64_t b0, int64_t n) -> hipError_t {
    if (!P.bf) return hipSuccess;
    const int t = 1 - s;
    const int64_t vs = D.v[s], vt = D.v[t], lp = P.ldnp[s], lc = P.ldcb[s];
    int64_t K, ld, ncol, ibs, iks;
    const Buf* full;
    if (t8 == Plan::As8) { K = vs; ld = lp; ncol = npair(vs); ibs = vs * lp; iks = lp; full = &P.As[s]; }
    else if (t8 == Plan::Mst8) { K = vt; ld = lc; ncol = vt * vs; ibs = vt * lc; iks = lc; full = &P.Mst[s]; }
    else { K = vs; ld = lc; ncol = vt * vs; ibs = vs * lc; iks = lc; full = &P.Mts[s]; }   // Mts8
    const int64_t blk = ((K + 15) / 16) * 16 * ld;                       // elements per octet block
    const float* src = P.keep32 ? at<float>(ws, *full) + b0 * ibs : at<float>(ws, P.stage);
    return lt::launch_split8(at<lt::bf16_t>(ws, P.O8h[s][t8]) + b0 * blk, at<lt::bf16_t>(ws, P.O8l[s][t8]) + b0 * blk,
                             n, (int32_t)K, ld, (int32_t)ncol, src, ibs, iks, st);
  };
  // --- 1. DF factor layouts --------------------------------------------------
  for (int s = 0; s < 2; ++s) {
    if (!P.BvvP[s].bytes) continue;
    const int64_t os = D.o[s], vs = D.v[s];
    HIPCHK(lt::launch_copy4d<double, T>(at<T>(ws, P.BvvP[s]), 0, 0, P.ldvv[s], 1, 1, Q, vs * vs,
                                        Bvv[s], 0, 0, vs * vs, 1, nullptr, 0, 0, 0, 0, st));
    HIPCHK(lt::launch_copy4d<double, T>(at<T>(ws, P.BovR[s]), 0, Q * P.ldv[s], P.ldv[s], 1, os, Q, vs,
                                        Bov[s], 0, vs, os * vs, 1, nullptr, 0, 0, 0, 0, st));
    HIPCHK(lt::launch_copy4d<double, double>(at<double>(ws, P.BovP64[s]), 0, 0, P.ldov[s], 1, 1, Q, os * vs,
                                             Bov[s], 0, 0, os * vs, 1, nullptr, 0, 0, 0, 0, st));
    HIPCHK(lt::launch_copy4d<double, double>(at<double>(ws, P.BooP64[s]), 0, 0, P.ldoo[s], 1, 1, Q, os * os,
                                             Boo[s], 0, 0, os * os, 1, nullptr, 0, 0, 0, 0, st));
  }

  auto gemm64 = [&](int64_t M, int64_t N, const double* Lp, int64_t lks, const double* Rp, int64_t rks,
                    double* out, int64_t ldo) -> hipError_t {
    lt::GemmArgs<double> g{};
    g.M = (int32_t)M; g.N = (int32_t)N; g.nbatch = 1; g.mode = 0;
    g.out = out; g.s_mr = ldo; g.s_nr = 1;
    g.L = Lp; g.lks = lks; g.R = Rp; g.rks = rks; g.K = (int32_t)Q;
    return lt::launch_gemm<double>(g, st);
  };

  // --- 2. (ov|oo), (ov|ov) in FP64 and derived operands -----------------------
  double* OO[2][2];
  for (int x = 0; x < 2; ++x)
    for (int y = 0; y < 2; ++y) {
      OO[x][y] = (double*)(scr + P.sc_OO[x][y]);
      const bool need = (x == y) ? P.need_as[x] : P.any_mix;
      if (!need) continue;
      // OO_xy[k][a][m][j] = (ka|mj)
      HIPCHK(gemm64(D.o[x] * D.v[x], D.o[y] * D.o[y], at<double>(ws, P.BovP64[x]), P.ldov[x],
                    at<double>(ws, P.BooP64[y]), P.ldoo[y], OO[x][y], D.o[y] * D.o[y]));
    }
  for (int s = 0; s < 2; ++s) {
    if (!P.need_as[s]) continue;
    const int64_t o = D.o[s], v = D.v[s], lv = P.ldv[s];
    double* OV = (double*)(scr + P.sc_OV);
    // (ov|ov) rows (q, y) of a chunk of q, then U[q][r][y][z] = OV[q][y][r][z] - OV[q][z][r][y]
    for (int64_t q0 = 0; q0 < o; q0 += P.cOV[s]) {
      const int64_t n = std::min<int64_t>(P.cOV[s], o - q0);
      HIPCHK(gemm64(n * v, o * v, at<double>(ws, P.BovP64[s]) + q0 * v, P.ldov[s], at<double>(ws, P.BovP64[s]),
                    P.ldov[s], OV, o * v));
      HIPCHK(lt::launch_copy4d<double, double>(at<double>(ws, P.U[s]) + q0 * o * v * lv, o * v * lv, v * lv, lv,
                                               n, o, v, v, OV, v * o * v, v, o * v, 1, OV, v * o * v, v, 1, o * v,
                                               st));
    }
    // GamT[j][k][m][a] = OO[k][a][m][j] - OO[j][a][m][k]
    const double* oo = OO[s][s];
    HIPCHK(lt::launch_copy4d<double, T>(at<T>(ws, P.GamT[s]), o * o * lv, o * lv, lv, o, o, o, v,
                                        oo, 1, v * o * o, o, o * o, oo, v * o * o, 1, o, o * o, st));
    HIPCHK(split_op(s, Plan::GamT8));
  }
  if (P.any_mix) {
    const int64_t oa = D.o[0], va = D.v[0], ob = D.o[1], vb = D.v[1];
    HIPCHK(gemm64(oa * va, ob * vb, at<double>(ws, P.BovP64[0]), P.ldov[0], at<double>(ws, P.BovP64[1]),
                  P.ldov[1], at<double>(ws, P.OVab), ob * vb));
  }
  for (int s = 0; s < 2; ++s) {
    if (!P.need_mix[s]) continue;
    const int t = 1 - s;
    const int64_t os = D.o[s], vs = D.v[s], ot = D.o[t], vt = D.v[t];
    // ZpT[j][K][M][a] = OO_st[j][a][M][K]
    HIPCHK(lt::launch_copy4d<double, T>(at<T>(ws, P.ZpT[s]), ot * ot * P.ldv[s], ot * P.ldv[s], P.ldv[s],
                                        os, ot, ot, vs, OO[s][t], vs * ot * ot, 1, ot, ot * ot,
                                        nullptr, 0, 0, 0, 0, st));
    HIPCHK(split_op(s, Plan::ZpT8));
    // OOT[K][j][m][C] = OO_ts[K][C][j][m]
    HIPCHK(lt::launch_copy4d<double, T>(at<T>(ws, P.OOT[s]), os * os * P.ldv[t], os * P.ldv[t], P.ldv[t],
                                        ot, os, os, vt, OO[t][s], vt * os * os, os, 1, os * os,
                                        nullptr, 0, 0, 0, 0, st));
    HIPCHK(split_op(s, Plan::OOT8));
  }

  // --- 3. amplitude operands ----------------------------------------------------
  const int64_t oa = D.o[0], ob = D.o[1], va = D.v[0], vb = D.v[1];
  for (int s = 0; s < 2; ++s) {
    if (!P.need_as[s]) continue;
    const int64_t o = D.o[s], v = D.v[s], lv = P.ldv[s];
    // T2T[i][j][e][a] = t2[i][j][a][e]
    HIPCHK(lt::launch_copy4d<double, T>(at<T>(ws, P.T2T[s]), o * v * lv, v * lv, lv, o, o, v, v,
                                        T2ss[s], o * v * v, v * v, 1, v, nullptr, 0, 0, 0, 0, st));
    HIPCHK(split_op(s, Plan::T2T8));
    // Tp[i][m][p(a<b)] = t2[i][m][a][b]
    HIPCHK(lt::launch_pack_pairs<double, T>(at<T>(ws, P.Tp[s]), P.ldnp[s], o * o, (int32_t)v, T2ss[s],
                                            v * v, v, 1, false, st));
    HIPCHK(split_op(s, Plan::Tp8));
  }
  // mixed amplitude t^{xY}_{pQ} (p,x of pair spin; Q,Y of odd spin): strides (p, Q, x, Y)
  int64_t mstr[2][4] = {{ob * va * vb, va * vb, vb, 1}, {va * vb, ob * va * vb, 1, vb}};
  for (int s = 0; s < 2; ++s) {
    if (!P.need_mix[s]) continue;
    const int t = 1 - s;
    const int64_t os = D.o[s], vs = D.v[s], ot = D.o[t], vt = D.v[t];
    const int64_t* m = mstr[s];
    // LmixT[i][K][E][a] = t^{aE}_{iK}
    HIPCHK(lt::launch_copy4d<double, T>(at<T>(ws, P.LmixT[s]), ot * vt * P.ldv[s], vt * P.ldv[s], P.ldv[s],
                                        os, ot, vt, vs, d->t2ab, m[0], m[1], m[3], m[2], nullptr, 0, 0, 0, 0, st));
    HIPCHK(split_op(s, Plan::LmixT8));
    // Tmix[i][K][C*vs+b] = t^{bC}_{iK}
    HIPCHK(lt::launch_copy4d<double, T>(at<T>(ws, P.Tmix[s]), ot * P.ldcb[s], P.ldcb[s], vs,
                                        os, ot, vt, vs, d->t2ab, m[0], m[1], m[3], m[2], nullptr, 0, 0, 0, 0, st));
    HIPCHK(split_op(s, Plan::Tmix8));
    HIPCHK(split_op(s, Plan::Tmx28));
    // TmT[i][K][e][C] = t^{eC}_{iK}
    HIPCHK(lt::launch_copy4d<double, T>(at<T>(ws, P.TmT[s]), ot * vs * P.ldv[t], vs * P.ldv[t], P.ldv[t],
                                        os, ot, vs, vt, d->t2ab, m[0], m[1], m[2], m[3], nullptr, 0, 0, 0, 0, st));
    HIPCHK(split_op(s, Plan::TmT8));
  }

  // --- 4. (ov|vv) slabs ------------------------------------------------------------
  auto gemmT = [&](int64_t M, int64_t N, int64_t nbatch, const T* Lp, int64_t lks, int64_t lbs, const T* Rp,
                   int64_t rks, int64_t rbs, T* out, int64_t obs, int64_t s_mq, int64_t s_mr, int32_t mdiv,
                   int64_t s_nq, int64_t s_nr, int32_t ndiv) -> hipError_t {
    lt::GemmArgs<T> g{};
    g.M = (int32_t)M; g.N = (int32_t)N; g.nbatch = (int32_t)nbatch; g.mode = 0;
    g.out = out; g.obs = obs; g.s_mq = s_mq; g.s_mr = s_mr; g.mdiv = mdiv; g.s_nq = s_nq; g.s_nr = s_nr; g.ndiv = ndiv;
    g.L = Lp; g.lks = lks; g.lbs = lbs; g.R = Rp; g.rks = rks; g.rbs = rbs; g.K = (int32_t)Q;
    return lt::launch_gemm<T>(g, st);
  };
  for (int s = 0; s < 2; ++s) {
    if (!P.need_as[s]) continue;
    const int64_t o = D.o[s], v = D.v[s], lv = P.ldv[s];
    T* Kx = (T*)scr;
    for (int64_t i0 = 0; i0 < o; i0 += P.cAs[s]) {
      const int64_t n = std::min<int64_t>(P.cAs[s], o - i0);
      // Kx[i][(e,b)][c] = (eb|ic) for i in [i0, i0 + n)
      HIPCHK(gemmT(v * v, v, n, at<T>(ws, P.BvvP[s]), P.ldvv[s], 0, at<T>(ws, P.BovR[s]) + i0 * Q * lv, lv,
                   Q * lv, Kx, v * v * lv, 0, lv, 0, 0, 1, 0));
      // As[i][e][p(b<c)] = Kx[i][e][b][c] - Kx[i][e][c][b] (BF16 modes: into staging, then split)
      T* dst = P.bf && !P.keep32 ? at<T>(ws, P.stage) : at<T>(ws, P.As[s]) + i0 * v * P.ldnp[s];
      HIPCHK(lt::launch_pack_pairs<T, T>(dst, P.ldnp[s], n * v, (int32_t)v, Kx, v * lv, lv, 1, true, st));
      HIPCHK(split_chunk(s, Plan::As8, i0, n));
    }
  }
  for (int s = 0; s < 2; ++s) {
    if (!P.need_mix[s]) continue;
    const int t = 1 - s;
    const int64_t os = D.o[s], vs = D.v[s], ot = D.o[t], vt = D.v[t], lc = P.ldcb[s];
    // Mst[j][E][C*vs+b] = (jb|EC): rows (E,C), cols b; chunks of j
    for (int64_t j0 = 0; j0 < os; j0 += P.cMst[s]) {
      const int64_t n = std::min<int64_t>(P.cMst[s], os - j0);
      T* dst = P.bf && !P.keep32 ? at<T>(ws, P.stage) : at<T>(ws, P.Mst[s]) + j0 * vt * lc;
      HIPCHK(gemmT(vt * vt, vs, n, at<T>(ws, P.BvvP[t]), P.ldvv[t], 0, at<T>(ws, P.BovR[s]) + j0 * Q * P.ldv[s],
                   P.ldv[s], Q * P.ldv[s], dst, vt * lc, lc, vs, (int32_t)vt, 0, 1, 0));
      HIPCHK(split_chunk(s, Plan::Mst8, j0, n));
    }
    // Mts[K][e][C*vs+b] = (be|KC): rows C, cols (e,b); chunks of K
    for (int64_t k0 = 0; k0 < ot; k0 += P.cMts[s]) {
      const int64_t n = std::min<int64_t>(P.cMts[s], ot - k0);
      T* dst = P.bf && !P.keep32 ? at<T>(ws, P.stage) : at<T>(ws, P.Mts[s]) + k0 * vs * lc;
      HIPCHK(gemmT(vt, vs * vs, n, at<T>(ws, P.BovR[t]) + k0 * Q * P.ldv[t], P.ldv[t], Q * P.ldv[t],
                   at<T>(ws, P.BvvP[s]), P.ldvv[s], 0, dst, vs * lc, 0, vs, 0, lc, 1, (int32_t)vs));
      HIPCHK(split_chunk(s, Plan::Mts8, k0, n));
    }
  }

  if (P.bwd) {
    // adjoint pass: FP64 padded Bvv for the DF back-contraction; t1, f_ov rows;
    // <qr||bc> pair-packed; (jb|KC) in the mixed output layout
    const double* T1[2] = {d->t1a, d->t1b};
    const double* Fov[2] = {d->fov_a, d->fov_b};
    const int64_t va = D.v[0], ob = D.o[1], vb = D.v[1];
    const int64_t so[4] = {va * ob * vb, ob * vb, vb, 1};     // OVab strides (occ_a, vir_a, occ_b, vir_b)
    for (int s = 0; s < 2; ++s) {
      const int t = 1 - s;
      const int64_t os = D.o[s], vs = D.v[s], ot = D.o[t], vt = D.v[t], lv = P.ldv[s], lc = P.ldcb[s];
      if (P.BvvP64[s].bytes)
        HIPCHK(lt::launch_copy4d<double, double>(at<double>(ws, P.BvvP64[s]), 0, 0, P.ldvv[s], 1, 1, Q, vs * vs,
                                                 Bvv[s], 0, 0, vs * vs, 1, nullptr, 0, 0, 0, 0, st));
      if (P.T1p[s].bytes) {
        HIPCHK(lt::launch_copy4d<double, T>(at<T>(ws, P.T1p[s]), 0, 0, lv, 1, 1, os, vs, T1[s], 0, 0, vs, 1,
                                            nullptr, 0, 0, 0, 0, st));
        HIPCHK(lt::launch_copy4d<double, T>(at<T>(ws, P.Fp[s]), 0, 0, lv, 1, 1, os, vs, Fov[s], 0, 0, vs, 1,
                                            nullptr, 0, 0, 0, 0, st));
      }
      if (P.Up[s].bytes)   // Up[q][r][p(b<c)] = <qr||bc>
        HIPCHK(lt::launch_pack_pairs<double, T>(at<T>(ws, P.Up[s]), P.ldnp[s], os * os, (int32_t)vs,
                                                at<double>(ws, P.U[s]), vs * lv, lv, 1, false, st));
      if (P.OVc[s].bytes) {  // OVc[j][K][C*vs+b] = (jb|KC)
        const int64_t sj = s == 0 ? so[0] : so[2], sb = s == 0 ? so[1] : so[3];
        const int64_t sK = s == 0 ? so[2] : so[0], sC = s == 0 ? so[3] : so[1];
        HIPCHK(lt::launch_copy4d<double, T>(at<T>(ws, P.OVc[s]), ot * lc, lc, vs, os, ot, vt, vs,
                                            at<double>(ws, P.OVab), sj, sK, sC, sb, nullptr, 0, 0, 0, 0, st));
      }
    }
  }
  return LT_OK;
}

// Enqueues the whole (T) path of one domain on `st` (kernels only; safe to
// capture into a graph).
// One domain of a launch group: its plan, items, outputs and workspace base
// (the domain's big region starts at ws; its small region at ws + P.small_base).
struct GroupDom {
  const ltriples_domain* d;
  const Plan* P;
  const ItemLists* L;
  double* e_out;
  double* parts;
  void* ws;
};

// The forward launch sequence of a group of domains (steps 1-6).  Each
// domain's operands are prepared in its own region; then, for every spin
// block and every batch index r, one contraction launch per output layout
// takes the r-th item batch of every domain of the group (BF16X3 and BF16;
// FP32/FP64 launch per domain), followed by each domain's epilogue and
// per-item reduction.  A domain's batches, epilogues and reductions are
// exactly those of a call on that domain alone, so every result bit is too.
// Domains are taken in the given order (the batched entry point passes them
// longest first).
template <typename T>
int run_group(const GroupDom* G, int ng, const ltriples_options* o, hipStream_t st, Timing& tm) {
  struct Dom {
    int32_t fc[8];
    int32_t *d_trip, *d_dst, *d_fc;
    double* e_items;
    bool active;
    char* scr;
    lt::ItemOps<T> ops;
    lt::Seg8 *tab0, *tab1;
  };
  std::vector<Dom> S((size_t)ng);
  tm.start = tm.mark();
  // --- item arrays (already uploaded by upload_items), empty domains, operands
  for (int x = 0; x < ng; ++x) {
    const GroupDom& g = G[x];
    const Plan& P = *g.P;
    const ItemLists& L = *g.L;
    Dom& m = S[x];
    for (int b = 0, n = 0; b < 4; ++b) {
      m.fc[b] = n;
      m.fc[4 + b] = (int32_t)L.dst[b].size();
      n += m.fc[4 + b];
    }
    m.d_trip = at_small<int32_t>(g.ws, P, P.trip);
    m.d_dst = at_small<int32_t>(g.ws, P, P.dst);
    m.d_fc = at_small<int32_t>(g.ws, P, P.firstcnt);
    m.e_items = (o && o->e_items) ? o->e_items : at_small<double>(g.ws, P, P.e_items);
    m.scr = (char*)g.ws + P.scratch.off;
    if (o && o->e_items && L.total > 0) HIPCHK(lt::launch_zero(o->e_items, 3 * L.total, st));
    HIPCHK(lt::launch_zero(at_small<double>(g.ws, P, P.e_items), 3 * std::max<int64_t>(L.total, 1), st));
    m.active = !(L.total == 0 || (P.D.v[0] == 0 && P.D.v[1] == 0));
    if (!m.active) {
      HIPCHK(lt::launch_zero(g.e_out, 1, st));
      if (g.parts) HIPCHK(lt::launch_zero(g.parts, 12, st));
    }
  }
  for (int x = 0; x < ng; ++x)
    if (S[x].active) {
      const int r = prep<T>(G[x].d, *G[x].P, G[x].ws, st);
      if (r) return r;
    }
  tm.setup_end = tm.mark();
  bool any = false;
  for (int x = 0; x < ng; ++x) any = any || S[x].active;
  if (!any) {
    tm.end = tm.setup_end;
    return LT_OK;
  }
  const bool bf = G[0].P->bf != 0;   // one precision per call
  // --- 5. triplet batches --------------------------------------------------------------
  for (int b = 0; b < 4; ++b) {
    const int s = blk_sigma(b), t = 1 - s;
    const bool mixed = blk_mixed(b);
    int64_t nbatches = 0;   // batches of the domain with the most
    for (int x = 0; x < ng; ++x) {
      Dom& m = S[x];
      const Plan& P = *G[x].P;
      const Dims& D = P.D;
      void* ws = G[x].ws;
      if (!m.active || P.n_blk[b] == 0) continue;
      nbatches = std::max(nbatches, cdiv(P.n_blk[b], P.nb[b]));
      lt::ItemOps<T>& ops = m.ops;
      ops = lt::ItemOps<T>{};
      ops.o_s = (int32_t)D.o[s]; ops.v_s = (int32_t)D.v[s]; ops.o_t = (int32_t)D.o[t]; ops.v_t = (int32_t)D.v[t];
      ops.oi_s = (int32_t)D.oi[s]; ops.oi_t = (int32_t)D.oi[t];
      ops.ld_vs = P.ldv[s]; ops.ld_vt = P.ldv[t]; ops.ld_np = P.ldnp[s]; ops.ld_cb = P.ldcb[s];
      ops.T2T = at<T>(ws, P.T2T[s]); ops.Tp = at<T>(ws, P.Tp[s]); ops.As = at<T>(ws, P.As[s]);
      ops.GamT = at<T>(ws, P.GamT[s]);
      if (mixed) {
        ops.LmixT = at<T>(ws, P.LmixT[s]); ops.Mst = at<T>(ws, P.Mst[s]); ops.Mts = at<T>(ws, P.Mts[s]);
        ops.Tmix = at<T>(ws, P.Tmix[s]); ops.ZpT = at<T>(ws, P.ZpT[s]); ops.TmT = at<T>(ws, P.TmT[s]);
        ops.OOT = at<T>(ws, P.OOT[s]);
      }
      // BF16 modes: segment descriptors of every item of the block, per output
      // layout (S or G in the first half of the table, Y in the second)
      m.tab0 = m.tab1 = nullptr;
      if (P.bf) {
        lt::ItemOps8 o8{};
        o8.o_s = ops.o_s; o8.v_s = ops.v_s; o8.o_t = ops.o_t; o8.v_t = ops.v_t;
        o8.oi_s = ops.oi_s; o8.oi_t = ops.oi_t;
        o8.ld_vs = ops.ld_vs; o8.ld_vt = ops.ld_vt; o8.ld_np = ops.ld_np; o8.ld_cb = ops.ld_cb;
        auto H = [&](int t8) { return P.O8h[s][t8].bytes ? at<lt::bf16_t>(ws, P.O8h[s][t8]) : nullptr; };
        auto Lo = [&](int t8) { return P.O8l[s][t8].bytes ? at<lt::bf16_t>(ws, P.O8l[s][t8]) : nullptr; };
        o8.T2Th = H(Plan::T2T8); o8.T2Tl = Lo(Plan::T2T8); o8.Ash = H(Plan::As8); o8.Asl = Lo(Plan::As8);
        o8.GamTh = H(Plan::GamT8); o8.GamTl = Lo(Plan::GamT8); o8.Tph = H(Plan::Tp8); o8.Tpl = Lo(Plan::Tp8);
        o8.LmixTh = H(Plan::LmixT8); o8.LmixTl = Lo(Plan::LmixT8); o8.Msth = H(Plan::Mst8); o8.Mstl = Lo(Plan::Mst8);
        o8.Mtsh = H(Plan::Mts8); o8.Mtsl = Lo(Plan::Mts8); o8.Tmixh = H(Plan::Tmix8); o8.Tmixl = Lo(Plan::Tmix8);
        o8.Tmx2h = H(Plan::Tmx28); o8.Tmx2l = Lo(Plan::Tmx28); o8.ZpTh = H(Plan::ZpT8); o8.ZpTl = Lo(Plan::ZpT8);
        o8.TmTh = H(Plan::TmT8); o8.TmTl = Lo(Plan::TmT8); o8.OOTh = H(Plan::OOT8); o8.OOTl = Lo(Plan::OOT8);
        m.tab0 = at_small<lt::Seg8>(ws, P, P.segtab);
        m.tab1 = m.tab0 + 6 * std::max<int64_t>(G[x].L->total, 1);
        const int64_t nblk = P.n_blk[b];
        o8.items = m.d_trip + 3 * m.fc[b];
        o8.kind = mixed ? 1 : 0;
        HIPCHK(lt::launch_seg8_table(o8, (int32_t)nblk, m.tab0 + 6 * (int64_t)m.fc[b], st));
        if (mixed) {
          o8.kind = 2;
          HIPCHK(lt::launch_seg8_table(o8, (int32_t)nblk, m.tab1 + 6 * (int64_t)m.fc[b], st));
        }
      }
    }
    // output layouts of the block: S (same spin), or G then Y (mixed)
    const int kinds[2] = {mixed ? 1 : 0, 2};
    const int nkind = mixed ? 2 : 1;
    for (int64_t r = 0; r < nbatches; ++r) {
      // the r-th batch of domain x: items [first, first + n) of block b
      auto batch_of = [&](int x, int64_t& first, int64_t& n) {
        const Plan& P = *G[x].P;
        first = r * P.nb[b];
        n = (S[x].active && P.n_blk[b] > first) ? std::min<int64_t>(P.nb[b], P.n_blk[b] - first) : 0;
        return n > 0;
      };
      for (int kx = 0; kx < nkind; ++kx) {
        const int kind = kinds[kx];
        // one domain's contraction arguments for batch r and this layout
        auto args = [&](int x, int64_t first, int64_t n, lt::GemmArgs<T>& g) {
          const Plan& P = *G[x].P;
          const Dims& D = P.D;
          const int64_t vs = D.v[s], vt = D.v[t], os = D.o[s], ot = D.o[t];
          Dom& m = S[x];
          g = lt::GemmArgs<T>{};
          g.nbatch = (int32_t)n; g.mode = 1; g.s_nr = 1;
          g.ops = m.ops;
          g.ops.items = m.d_trip + 3 * (m.fc[b] + first);
          g.ops.kind = kind;
          if (kind == 0) {
            g.M = (int32_t)vs; g.N = (int32_t)npair(vs); g.out = (T*)m.scr; g.obs = (int64_t)(P.o1[b] / P.ts);
            g.s_mr = P.ldnp[s];
            return 2.0 * (double)g.M * (double)g.N * (double)(3 * vs + 3 * os) * (double)n;
          }
          if (kind == 1) {
            g.M = (int32_t)vs; g.N = (int32_t)(vt * vs); g.out = (T*)m.scr; g.obs = (int64_t)(P.o1[b] / P.ts);
            g.s_mr = P.ldcb[s];
            return 2.0 * (double)g.M * (double)g.N * (double)(2 * vt + vs + os + 2 * ot) * (double)n;
          }
          g.M = (int32_t)vt; g.N = (int32_t)npair(vs); g.out = (T*)(m.scr + (size_t)P.nb[b] * P.o1[b]);
          g.obs = (int64_t)(P.o2[b] / P.ts); g.s_mr = P.ldnp[s];
          return 2.0 * (double)g.M * (double)g.N * (double)(2 * vs + 2 * os) * (double)n;
        };
        const int force = o ? o->tile_override[kind] - 1 : -1;   // 0 = automatic
        const bool tune = o && o->autotune;
        // an empty output (a virtual space of size zero) has nothing to compute;
        // the tile selection divides by the row-tile count
        auto empty = [](const lt::GemmArgs<T>& g) { return g.M <= 0 || g.N <= 0 || g.nbatch <= 0; };
        // BF16 descriptor of one domain's batch
        auto chunk = [&](int x, const lt::GemmArgs<T>& g) {
          const int64_t first_item = (g.ops.items - S[x].d_trip) / 3;   // index in the block-ordered item list
          return lt::Chunk16{g.M, g.N, g.nbatch, (float*)g.out, g.obs, g.s_mr,
                             (kind == 2 ? S[x].tab1 : S[x].tab0) + 6 * first_item};
        };
        std::vector<int> xs;
        std::vector<lt::GemmArgs<T>> gs;
        for (int x = 0; x < ng; ++x) {
          int64_t first, n;
          if (!batch_of(x, first, n)) continue;
          lt::GemmArgs<T> g;
          tm.gemm_flops += args(x, first, n, g);
          if (empty(g)) continue;
          xs.push_back(x);
          gs.push_back(g);
        }
        hipEvent_t a = tm.mark();
        if (!bf) {
          for (auto& g : gs) HIPCHK(lt::launch_gemm<T>(g, st, tune, force));
        } else if (gs.size() == 1) {
          const lt::Chunk16 c = chunk(xs[0], gs[0]);
          lt::GemmArgs16 h{};
          h.M = c.M; h.N = c.N; h.nbatch = c.nbatch; h.nprod = G[xs[0]].P->bf;
          h.out = c.out; h.obs = c.obs; h.ldo = c.ldo; h.kind = kind; h.tab = c.tab;
          HIPCHK(lt::launch_gemm_bf16(h, st, tune, force));
        } else {
          // one launch per tile-selection class (32-row blocks of M, log2 N),
          // so that every domain's items run in the tile shape a launch of
          // its own would take (a shared larger tile pads the smaller
          // domains' rows: measured up to 1.5x slower); classes in the order
          // of their first domain
          auto cls = [](const lt::GemmArgs<T>& g) {
            int nlog = 0;
            while ((1 << (nlog + 1)) <= g.N) ++nlog;
            return std::make_pair((g.M + 31) / 32, nlog);
          };
          std::vector<bool> done(gs.size(), false);
          for (size_t c0 = 0; c0 < gs.size(); ++c0) {
            if (done[c0]) continue;
            lt::GemmArgs16 h{};
            h.nprod = G[xs[c0]].P->bf; h.kind = kind;
            for (size_t c = c0; c < gs.size() && h.nchunk < lt::kMaxChunk16; ++c) {
              if (done[c] || cls(gs[c]) != cls(gs[c0])) continue;
              const lt::Chunk16 ch = chunk(xs[c], gs[c]);
              h.ch[h.nchunk++] = ch;
              h.M = std::max(h.M, ch.M); h.N = std::max(h.N, ch.N); h.nbatch += ch.nbatch;
              done[c] = true;
            }
            if (h.nchunk == 1) {   // alone in its class: the plain launch
              const lt::Chunk16 c = h.ch[0];
              h = lt::GemmArgs16{};
              h.M = c.M; h.N = c.N; h.nbatch = c.nbatch; h.nprod = G[xs[c0]].P->bf;
              h.out = c.out; h.obs = c.obs; h.ldo = c.ldo; h.kind = kind; h.tab = c.tab;
            }
            HIPCHK(lt::launch_gemm_bf16(h, st, tune, force));
          }
        }
        if (!gs.empty()) tm.gemm.push_back({a, tm.mark()});
      }
      // epilogues and per-item reductions, domain by domain
      for (int x = 0; x < ng; ++x) {
        int64_t first, n;
        if (!batch_of(x, first, n)) continue;
        const GroupDom& gd = G[x];
        const ltriples_domain* d = gd.d;
        const Plan& P = *gd.P;
        const Dims& D = P.D;
        Dom& m = S[x];
        const int64_t os = D.o[s], vs = D.v[s], ot = D.o[t], vt = D.v[t];
        const int64_t va = D.v[0], ob = D.o[1], vb = D.v[1];
        const double* T2ss[2] = {d->t2aa, d->t2bb};
        const double* T1[2] = {d->t1a, d->t1b};
        const double* Fov[2] = {d->fov_a, d->fov_b};
        const double* EO[2] = {d->eo_a, d->eo_b};
        const double* EV[2] = {d->ev_a, d->ev_b};
        const size_t o1 = P.o1[b], o2 = P.o2[b];
        const int64_t nb = P.nb[b], nt = P.ntile[b];
        T* out1 = (T*)m.scr;
        T* out2 = (T*)(m.scr + (size_t)nb * o1);
        double* part = (double*)(m.scr + (size_t)nb * (o1 + o2));
        const int32_t* items = m.d_trip + 3 * (m.fc[b] + first);
        hipEvent_t ea = nullptr;
        if (!mixed) {
          if (P.dump_w) HIPCHK(lt::launch_dump_w_same<T>(out1, P.ldnp[s], (int32_t)vs, P.dump_w, st));
          ea = tm.mark();
          lt::EpiSame<T> e{};
          e.o = (int32_t)os; e.v = (int32_t)vs; e.ld_np = P.ldnp[s];
          e.S = out1; e.s_item = (int64_t)(o1 / P.ts); e.items = items;
          e.nt = (int32_t)cdiv(vs, lt::ET); e.ntri = (int32_t)nt;
          e.eo = EO[s]; e.ev = EV[s]; e.t1 = T1[s]; e.f = Fov[s]; e.t2 = T2ss[s];
          e.U = at<double>(gd.ws, P.U[s]); e.ld_v = P.ldv[s]; e.part = part;
          if (P.lap) { e.lap = P.lap; e.lap_o0 = (int32_t)D.oi[s]; e.lap_slot = 2; }   // (j, k, central)
          HIPCHK(lt::launch_epi_same<T>(e, (int32_t)n, st));
        } else {
          if (P.dump_w)
            HIPCHK(lt::launch_dump_w_mixed<T>(out1, P.ldcb[s], out2, P.ldnp[s], (int32_t)vs, (int32_t)vt, P.dump_w,
                                              st));
          ea = tm.mark();
          lt::EpiMixed<T> e{};
          e.o_s = (int32_t)os; e.v_s = (int32_t)vs; e.o_t = (int32_t)ot; e.v_t = (int32_t)vt;
          e.ld_np = P.ldnp[s]; e.ld_cb = P.ldcb[s];
          e.G = out1; e.g_item = (int64_t)(o1 / P.ts); e.Y = out2; e.y_item = (int64_t)(o2 / P.ts);
          e.items = items;
          e.nts = (int32_t)cdiv(vs, lt::ET); e.ntt = (int32_t)cdiv(vt, lt::ET); e.ntiles = (int32_t)nt;
          e.eo_s = EO[s]; e.ev_s = EV[s]; e.eo_t = EO[t]; e.ev_t = EV[t];
          e.t1_s = T1[s]; e.t1_t = T1[t]; e.f_s = Fov[s]; e.f_t = Fov[t]; e.t2ss = T2ss[s];
          e.U = at<double>(gd.ws, P.U[s]); e.ld_vs = P.ldv[s];
          // OVab[i_a][a_a][J_b][B_b]
          const int64_t so[4] = {va * ob * vb, ob * vb, vb, 1};   // (occ_a, vir_a, occ_b, vir_b)
          e.ov = at<double>(gd.ws, P.OVab);
          if (s == 0) { e.ov_o = so[0]; e.ov_v = so[1]; e.ov_O = so[2]; e.ov_V = so[3]; }
          else { e.ov_o = so[2]; e.ov_v = so[3]; e.ov_O = so[0]; e.ov_V = so[1]; }
          const int64_t mstr[2][4] = {{ob * va * vb, va * vb, vb, 1}, {va * vb, ob * va * vb, 1, vb}};
          e.tm = d->t2ab; e.tm_o = mstr[s][0]; e.tm_v = mstr[s][2]; e.tm_O = mstr[s][1]; e.tm_V = mstr[s][3];
          e.part = part;
          if (P.lap) {   // central orbital in the same-spin pair (i, central, K) or the odd slot (I, J, central)
            e.lap = P.lap;
            e.lap_slot = s == P.lap_spin ? 1 : 2;
            e.lap_o0 = (int32_t)D.oi[P.lap_spin];
          }
          HIPCHK(lt::launch_epi_mixed<T>(e, (int32_t)n, st));
        }
        HIPCHK(lt::launch_reduce_items(part, (int32_t)n, (int32_t)nt, m.d_dst + m.fc[b] + first, m.e_items, st));
        tm.epi.push_back({ea, tm.mark()});
      }
    }
  }

  // --- 6. totals ----------------------------------------------------------------------
  for (int x = 0; x < ng; ++x)
    if (S[x].active)
      HIPCHK(lt::launch_reduce_final(S[x].e_items, S[x].d_dst, S[x].d_fc, S[x].d_fc + 4, G[x].parts, G[x].e_out, st));
  tm.end = tm.mark();
  return LT_OK;
}

template <typename T>
int run(const ltriples_domain* d, const Plan& P, const ItemLists& L, const ltriples_options* o,
        double* e_out, double* parts, void* ws, hipStream_t st, Timing& tm) {
  const GroupDom g{d, &P, &L, e_out, parts, ws};
  return run_group<T>(&g, 1, o, st, tm);
}

// Every occupied energy below every virtual energy by at least 1e-100 and
// every energy finite and at most 1e100 in magnitude, so every denominator
// D = e_i + e_j + e_k - e_a - e_b - e_c lies in [-6e100, -3e-100] (the range
// the epilogues' reciprocal assumes).  Reads the orbital energies back to the
// host with copies ordered on the caller's stream (after whatever the caller
// enqueued there to produce them), then waits for that stream.
int check_denominators(const ltriples_domain* d, hipStream_t st) {
  const Dims D = dims_of(d);
  double omax = -INFINITY, vmin = INFINITY;
  std::vector<double> ho[2], hv[2];
  for (int s = 0; s < 2; ++s) {
    const double* eo = s ? d->eo_b : d->eo_a;
    const double* ev = s ? d->ev_b : d->ev_a;
    ho[s].resize(D.o[s]);
    hv[s].resize(D.v[s]);
    if (D.o[s]) HIPCHK(hipMemcpyAsync(ho[s].data(), eo, 8 * D.o[s], hipMemcpyDeviceToHost, st));
    if (D.v[s]) HIPCHK(hipMemcpyAsync(hv[s].data(), ev, 8 * D.v[s], hipMemcpyDeviceToHost, st));
  }
  HIPCHK(hipStreamSynchronize(st));
  for (int s = 0; s < 2; ++s) {
    for (double x : ho[s]) {
      if (!std::isfinite(x)) return fail(LT_ENONFINITE, "non-finite occupied energy");
      if (std::fabs(x) > 1e100) return fail(LT_EDENOM, "occupied energy %.6g above 1e100 in magnitude", x);
      omax = std::max(omax, x);
    }
    for (double x : hv[s]) {
      if (!std::isfinite(x)) return fail(LT_ENONFINITE, "non-finite virtual energy");
      if (std::fabs(x) > 1e100) return fail(LT_EDENOM, "virtual energy %.6g above 1e100 in magnitude", x);
      vmin = std::min(vmin, x);
    }
  }
  if (omax >= vmin) return fail(LT_EDENOM, "max occupied energy %.6g >= min virtual energy %.6g", omax, vmin);
  if (vmin - omax < 1e-100)
    return fail(LT_EDENOM, "occupied-virtual gap %.6g below 1e-100", vmin - omax);
  return LT_OK;
}

// Workspace of a call made with ws == NULL: allocated stream-ordered on the
// call's stream and released the same way on every return path (success or
// error), so it neither leaks nor makes the call wait for the stream.
struct OwnedWs {
  void* p = nullptr;
  hipStream_t st = nullptr;
  OwnedWs() = default;
  OwnedWs(const OwnedWs&) = delete;
  OwnedWs& operator=(const OwnedWs&) = delete;
  ~OwnedWs() {
    if (p) (void)hipFreeAsync(p, st);
  }
};

// The caller's workspace (checked against `need`), or a stream-ordered one.
int get_ws(void*& ws, size_t ws_bytes, size_t need, hipStream_t st, OwnedWs& own) {
  if (ws != nullptr) {
    if (ws_bytes < need) return fail(LT_EWORKSPACE, "workspace %zu bytes < required %zu", ws_bytes, need);
    return LT_OK;
  }
  HIPCHK(hipMallocAsync(&own.p, std::max<size_t>(need, 256), st));
  own.st = st;
  ws = own.p;
  return LT_OK;
}

// Opt-in scan of every input array of a domain for NaN and infinity, on the
// device, with the flag in the domain's small buffers; waits for the stream.
int scan_finite(const ltriples_domain* d, const Plan& P, void* ws, hipStream_t st) {
  const Dims D = dims_of(d);
  const int64_t oa = D.o[0], ob = D.o[1], va = D.v[0], vb = D.v[1], Q = D.Q;
  lt::FiniteScan a{};
  const struct { const double* p; int64_t n; } ps[] = {
      {d->t1a, oa * va}, {d->t1b, ob * vb}, {d->t2aa, oa * oa * va * va}, {d->t2bb, ob * ob * vb * vb},
      {d->t2ab, oa * ob * va * vb}, {d->Boo_a, Q * oa * oa}, {d->Bov_a, Q * oa * va}, {d->Bvv_a, Q * va * va},
      {d->Boo_b, Q * ob * ob}, {d->Bov_b, Q * ob * vb}, {d->Bvv_b, Q * vb * vb}, {d->eo_a, oa}, {d->ev_a, va},
      {d->eo_b, ob}, {d->ev_b, vb}, {d->fov_a, oa * va}, {d->fov_b, ob * vb}};
  for (const auto& x : ps)
    if (x.n > 0) { a.p[a.narr] = x.p; a.n[a.narr] = x.n; ++a.narr; }
  int32_t* flag = at_small<int32_t>(ws, P, P.flag);
  HIPCHK(lt::launch_zero32(flag, 1, st));
  HIPCHK(lt::launch_scan_finite(a, flag, st));
  int32_t h = 0;
  HIPCHK(hipMemcpyAsync(&h, flag, 4, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (h) return fail(LT_ENONFINITE, "NaN or infinity in the inputs (options.check_finite)");
  return LT_OK;
}

// ---------------------------------------------------------------------------
// Adjoint pass (backward).  Per batch of items: the forward contraction is
// recomputed (W is never stored), the backward epilogue writes the adjoints of
// the contraction outputs, and reverse GEMMs accumulate the gradients of every
// prepared operand into mirror buffers of the same layout.  The mirrors are
// then mapped back to the amplitudes and to FP64 four-index integral
// gradients, which the DF back-contraction turns into gradients of the DF
// factors; the gradients of symmetric inputs are projected last.
// ---------------------------------------------------------------------------
template <typename T> struct RevBuilder {
  struct Tgt { lt::RBlk<T> blk; std::vector<lt::RSeg<T>> segs; };
  struct Group { bool tb = false; std::map<uintptr_t, Tgt> tg; };
  struct Launch {
    bool tb; int64_t blk0, nblk; int32_t max_rows, max_cols; double flops;
    int64_t red0, nred; int32_t max_red;
  };
  // Long contractions are split at segment boundaries into chunks of about
  // kChunk elements that write partial sums into `part` (capacity part_cap
  // elements, reused by every launch); a fixed-order reduce adds them.  Many
  // reverse launches have only a few hundred targets of 64 rows, too few for
  // 256 CUs, so the split is fine: on the gradient domain (20,18,160,162,640)
  // chunks of 512 rather than 8192 took the FP32 adjoint from 4.82 to 4.40 s
  // and the FP64 one from 8.67 to 7.79 s.
  static constexpr int64_t kChunk = 512;
  T* part = nullptr;
  int64_t part_cap = 0, part_max = 0;
  std::vector<lt::RBlk<T>> blks;
  std::vector<lt::RSeg<T>> segs;
  std::vector<lt::RRed<T>> reds;
  std::vector<Launch> launches;
  std::vector<Group> groups;
  void begin(int n) { groups.assign(n, Group{}); }
  void add(int gi, bool tb, T* out, int64_t ldo, int64_t rows, int64_t cols, const lt::RSeg<T>& sg) {
    if (!out || rows <= 0 || cols <= 0 || sg.K <= 0) return;
    Group& g = groups[gi];
    g.tb = tb;
    Tgt& t = g.tg[(uintptr_t)out];
    if (t.segs.empty()) t.blk = lt::RBlk<T>{out, ldo, (int32_t)rows, (int32_t)cols, 0, 0, 0, 0};
    t.segs.push_back(sg);
  }
  // emits one launch per non-empty group, targets in address order
  void flush() {
    for (Group& g : groups) {
      if (g.tg.empty()) continue;
      // chunks per target, halved together until the partials fit
      std::vector<int64_t> nch;
      for (auto& kv : g.tg) {
        int64_t K = 0;
        for (auto& x : kv.second.segs) K += x.K;
        nch.push_back(std::min<int64_t>((int64_t)kv.second.segs.size(), std::max<int64_t>(1, cdiv(K, kChunk))));
      }
      for (;;) {
        int64_t need = 0;
        size_t q = 0;
        for (auto& kv : g.tg) {
          if (nch[q] > 1) need += nch[q] * kv.second.blk.rows * (int64_t)kv.second.blk.cols;
          ++q;
        }
        if (need <= part_cap) break;
        bool any = false;
        for (auto& c : nch)
          if (c > 1) { c = c / 2; any = true; }
        if (!any) break;
      }
      Launch l{g.tb, (int64_t)blks.size(), 0, 0, 0, 0.0, (int64_t)reds.size(), 0, 0};
      int64_t poff = 0;
      size_t q = 0;
      for (auto& kv : g.tg) {
        const lt::RBlk<T> tb = kv.second.blk;
        const auto& sv = kv.second.segs;
        int64_t K = 0;
        for (auto& x : sv) K += x.K;
        for (auto& x : sv) l.flops += 2.0 * tb.rows * (double)tb.cols * x.K;
        l.max_rows = std::max(l.max_rows, tb.rows);
        l.max_cols = std::max(l.max_cols, tb.cols);
        const int64_t c = nch[q++];
        if (c <= 1) {
          lt::RBlk<T> b = tb;
          b.beg = (int32_t)segs.size();
          segs.insert(segs.end(), sv.begin(), sv.end());
          b.end = (int32_t)segs.size();
          blks.push_back(b);
          ++l.nblk;
          continue;
        }
        // contiguous segment ranges of about K/c contraction elements each
        const int64_t elems = (int64_t)tb.rows * tb.cols;
        int64_t made = 0, acc = 0;
        size_t si = 0;
        while (si < sv.size()) {
          lt::RBlk<T> b = tb;
          b.out = part + poff + made * elems;
          b.ldo = tb.cols;
          b.store = 1;
          b.beg = (int32_t)segs.size();
          const int64_t goal = (made + 1) * K / c;
          do { acc += sv[si].K; segs.push_back(sv[si]); ++si; } while (si < sv.size() && acc < goal);
          b.end = (int32_t)segs.size();
          blks.push_back(b);
          ++l.nblk;
          ++made;
        }
        reds.push_back(lt::RRed<T>{tb.out, tb.ldo, part + poff, tb.rows, tb.cols, (int32_t)made, 0});
        ++l.nred;
        l.max_red = std::max<int32_t>(l.max_red, (int32_t)elems);
        poff += made * elems;
      }
      part_max = std::max(part_max, poff);
      launches.push_back(l);
    }
    groups.clear();
  }
};

// One forward contraction segment of an item: X = sign * L^T R over K rows,
// with the mirrors (gradient buffers) of both operands and the reverse groups.
template <typename T> struct FSeg {
  const T* L; T* dL; int64_t lks;
  const T* R; T* dR; int64_t rks;
  int64_t K; float sign; int gR, gL;
};

template <typename T>
void add_rev(RevBuilder<T>& rb, const FSeg<T>& f, const T* dX, int64_t ldX, int64_t M, int64_t N) {
  if (f.gR >= 0) rb.add(f.gR, false, f.dR, f.rks, f.K, N, lt::RSeg<T>{f.L, f.lks, dX, ldX, (int32_t)M, f.sign});
  if (f.gL >= 0) rb.add(f.gL, true, f.dL, f.lks, f.K, M, lt::RSeg<T>{f.R, f.rks, dX, ldX, (int32_t)N, f.sign});
}

// Descriptor lists of every batch (in launch order) for workspace base `ws`.
template <typename T>
void build_rev(const Plan& P, const ItemLists& L, char* ws, RevBuilder<T>& rb,
               std::vector<std::pair<size_t, size_t>>& batch_launch) {
  const Dims& D = P.D;
  char* scr = ws + P.scratch.off;
  auto A = [&](const Buf& b) { return (T*)(ws + b.off); };
  for (int b = 0; b < 4; ++b) {
    const int64_t nblk = P.n_blk[b];
    if (nblk == 0) continue;
    const int s = blk_sigma(b), t = 1 - s;
    const bool mixed = blk_mixed(b);
    const int64_t os = D.o[s], vs = D.v[s], ot = D.o[t], vt = D.v[t];
    const int64_t lv = P.ldv[s], lvt = P.ldv[t], lp = P.ldnp[s], lc = P.ldcb[s], np = npair(vs);
    const int64_t nb = P.nb[b];
    const size_t o1 = P.o1[b], o2 = P.o2[b];
    const int64_t s1 = (int64_t)(o1 / P.ts), s2 = (int64_t)(o2 / P.ts);
    T *T2T = A(P.T2T[s]), *dT2T = A(P.dT2T[s]), *As = A(P.As[s]), *dAs = A(P.dAs[s]);
    T *Gam = A(P.GamT[s]), *dGam = A(P.dGamT[s]), *Tp = A(P.Tp[s]), *dTp = A(P.dTp[s]);
    T *Up = A(P.Up[s]), *dUp = A(P.dUp[s]), *T1p = A(P.T1p[s]), *dT1p = A(P.dT1p[s]), *Fp = A(P.Fp[s]);
    T* dFp = A(P.dFp[s]);
    for (int64_t first = 0; first < nblk; first += nb) {
      const int64_t n = std::min<int64_t>(nb, nblk - first);
      const size_t l0 = rb.launches.size();
      const int32_t* tr = L.trip[b].data() + 3 * first;
      if (!mixed) {
        T* dS = (T*)(scr + (size_t)nb * o1);
        T* dSV = (T*)(scr + 2 * (size_t)nb * o1);
        rb.begin(6);
        for (int64_t m = 0; m < n; ++m) {
          const int64_t i = tr[3 * m], j = tr[3 * m + 1], k = tr[3 * m + 2];
          const int64_t pm[3][3] = {{i, j, k}, {j, i, k}, {k, j, i}};
          const float sg[3] = {1.f, -1.f, -1.f};
          const T* dSm = dS + m * s1;
          const T* dSVm = dSV + m * s1;
          for (int u = 0; u < 3; ++u) {
            const int64_t p = pm[u][0], q = pm[u][1], r = pm[u][2];
            const int64_t ot2 = (q * os + r) * vs * lv, og = (q * os + r) * os * lv;
            // sum_e t^{ae}_{qr} <ep||bc>
            add_rev(rb, FSeg<T>{T2T + ot2, dT2T + ot2, lv, As + p * vs * lp, dAs + p * vs * lp, lp, vs, sg[u], 0, 2},
                    dSm, lp, vs, np);
            // - sum_m <ma||qr> t^{bc}_{pm}
            add_rev(rb, FSeg<T>{Gam + og, dGam + og, lv, Tp + p * os * lp, dTp + p * os * lp, lp, os, -sg[u], 1, 3},
                    dSm, lp, vs, np);
            // singles and f_ov terms: t1[p] x <qr||bc>, f[p] x t^{bc}_{qr}
            const int64_t orow = (q * os + r) * lp;
            add_rev(rb, FSeg<T>{T1p + p * lv, dT1p + p * lv, lv, Up + orow, dUp + orow, lp, 1, sg[u], 4, 5},
                    dSVm, lp, vs, np);
            add_rev(rb, FSeg<T>{Fp + p * lv, dFp + p * lv, lv, Tp + orow, dTp + orow, lp, 1, sg[u], 4, 5},
                    dSVm, lp, vs, np);
          }
        }
        rb.flush();
      } else {
        T *LmT = A(P.LmixT[s]), *dLmT = A(P.dLmixT[s]), *Mst = A(P.Mst[s]), *dMst = A(P.dMst[s]);
        T *Mts = A(P.Mts[s]), *dMts = A(P.dMts[s]), *Tmix = A(P.Tmix[s]), *dTmix = A(P.dTmix[s]);
        T *ZpT = A(P.ZpT[s]), *dZpT = A(P.dZpT[s]), *TmT = A(P.TmT[s]), *dTmT = A(P.dTmT[s]);
        T *OOT = A(P.OOT[s]), *dOOT = A(P.dOOT[s]), *OVc = A(P.OVc[s]), *dOVc = A(P.dOVc[s]);
        T *T1t = A(P.T1p[t]), *dT1t = A(P.dT1p[t]), *Ft = A(P.Fp[t]), *dFt = A(P.dFp[t]);
        const size_t q1 = (size_t)nb * (o1 + o2);
        T* dG = (T*)(scr + q1);
        T* dY = (T*)(scr + q1 + (size_t)nb * o1);
        T* dGV = (T*)(scr + 2 * q1);
        T* dYV = (T*)(scr + 2 * q1 + (size_t)nb * o1);
        rb.begin(14);
        for (int64_t m = 0; m < n; ++m) {
          const int64_t i = tr[3 * m], j = tr[3 * m + 1], K = tr[3 * m + 2];
          const T* dGm = dG + m * s1;
          const T* dYm = dY + m * s2;
          const T* dGVm = dGV + m * s1;
          const T* dYVm = dYV + m * s2;
          const int64_t M1 = vs, N1 = vt * vs, M2 = vt, N2 = np;
          auto lm = [&](int64_t p) { return (p * ot + K) * vt * lv; };
          auto zp = [&](int64_t p) { return (p * ot + K) * ot * lv; };
          auto tm = [&](int64_t p) { return (p * ot + K) * vs * lvt; };
          auto oo = [&](int64_t p) { return (K * os + p) * os * lvt; };
          const int64_t oij2 = (i * os + j) * vs * lv, oijg = (i * os + j) * os * lv;
          // G[a][C*vs+b]
          add_rev(rb, FSeg<T>{LmT + lm(i), dLmT + lm(i), lv, Mst + j * vt * lc, dMst + j * vt * lc, lc, vt, 1.f, 0, 6},
                  dGm, lc, M1, N1);
          add_rev(rb, FSeg<T>{LmT + lm(j), dLmT + lm(j), lv, Mst + i * vt * lc, dMst + i * vt * lc, lc, vt, -1.f, 0, 6},
                  dGm, lc, M1, N1);
          add_rev(rb, FSeg<T>{T2T + oij2, dT2T + oij2, lv, Mts + K * vs * lc, dMts + K * vs * lc, lc, vs, 1.f, 1, 7},
                  dGm, lc, M1, N1);
          add_rev(rb, FSeg<T>{Gam + oijg, dGam + oijg, lv, Tmix + K * lc, dTmix + K * lc, ot * lc, os, 1.f, 2, 8},
                  dGm, lc, M1, N1);
          add_rev(rb, FSeg<T>{ZpT + zp(j), dZpT + zp(j), lv, Tmix + i * ot * lc, dTmix + i * ot * lc, lc, ot, 1.f, 3, 9},
                  dGm, lc, M1, N1);
          add_rev(rb, FSeg<T>{ZpT + zp(i), dZpT + zp(i), lv, Tmix + j * ot * lc, dTmix + j * ot * lc, lc, ot, -1.f, 3, 9},
                  dGm, lc, M1, N1);
          // Y[C][p(a<b)]
          add_rev(rb, FSeg<T>{TmT + tm(i), dTmT + tm(i), lvt, As + j * vs * lp, dAs + j * vs * lp, lp, vs, 1.f, 4, 10},
                  dYm, lp, M2, N2);
          add_rev(rb, FSeg<T>{TmT + tm(j), dTmT + tm(j), lvt, As + i * vs * lp, dAs + i * vs * lp, lp, vs, -1.f, 4, 10},
                  dYm, lp, M2, N2);
          add_rev(rb, FSeg<T>{OOT + oo(j), dOOT + oo(j), lvt, Tp + i * os * lp, dTp + i * os * lp, lp, os, -1.f, 5, 11},
                  dYm, lp, M2, N2);
          add_rev(rb, FSeg<T>{OOT + oo(i), dOOT + oo(i), lvt, Tp + j * os * lp, dTp + j * os * lp, lp, os, 1.f, 5, 11},
                  dYm, lp, M2, N2);
          // singles and f_ov terms of the P(ij)P(ab) part: t1[p] x (qb|KC), f[p] x t^{bC}_{qK}
          const int64_t pq[2][2] = {{i, j}, {j, i}};
          const float sg[2] = {1.f, -1.f};
          for (int u = 0; u < 2; ++u) {
            const int64_t p = pq[u][0], q = pq[u][1], orow = (q * ot + K) * lc;
            add_rev(rb, FSeg<T>{T1p + p * lv, dT1p + p * lv, lv, OVc + orow, dOVc + orow, lc, 1, sg[u], 12, 13},
                    dGVm, lc, M1, N1);
            add_rev(rb, FSeg<T>{Fp + p * lv, dFp + p * lv, lv, Tmix + orow, dTmix + orow, lc, 1, sg[u], 12, 13},
                    dGVm, lc, M1, N1);
          }
          // t1[K][C] <ij||ab>, f[K][C] t^{ab}_{ij}
          const int64_t orow = (i * os + j) * lp;
          add_rev(rb, FSeg<T>{T1t + K * lvt, dT1t + K * lvt, lvt, Up + orow, dUp + orow, lp, 1, 1.f, 12, 13},
                  dYVm, lp, M2, N2);
          add_rev(rb, FSeg<T>{Ft + K * lvt, dFt + K * lvt, lvt, Tp + orow, dTp + orow, lp, 1, 1.f, 12, 13},
                  dYVm, lp, M2, N2);
        }
        rb.flush();
      }
      batch_launch.push_back({l0, rb.launches.size()});
    }
  }
}

// DF back-contraction descriptors (FP64): gradients of the four-index
// integral classes -> gradients of Bov, Bvv, Boo (caller's buffers).
void build_df_rev(const Plan& P, char* ws, const ltriples_domain_grad* g, RevBuilder<double>& rb) {
  const Dims& D = P.D;
  const int64_t Q = D.Q;
  auto A = [&](const Buf& b) { return b.bytes ? (double*)(ws + b.off) : nullptr; };
  double* gBov[2] = {g->Bov_a, g->Bov_b};
  double* gBvv[2] = {g->Bvv_a, g->Bvv_b};
  double* gBoo[2] = {g->Boo_a, g->Boo_b};
  rb.begin(2);
  for (int x = 0; x < 2; ++x) {
    const int64_t nov = D.o[x] * D.v[x];
    for (int y = 0; y < 2; ++y) {
      if (double* Z = A(P.dOVVV[x][y])) {
        rb.add(0, true, gBov[x], nov, Q, nov,
               lt::RSeg<double>{A(P.BvvP64[y]), P.ldvv[y], Z, P.ldvv[y], (int32_t)(D.v[y] * D.v[y]), 1.f});
        rb.add(1, false, gBvv[y], D.v[y] * D.v[y], Q, D.v[y] * D.v[y],
               lt::RSeg<double>{A(P.BovP64[x]), P.ldov[x], Z, P.ldvv[y], (int32_t)nov, 1.f});
      }
      if (double* Z = A(P.dOVOO[x][y])) {
        rb.add(0, true, gBov[x], nov, Q, nov,
               lt::RSeg<double>{A(P.BooP64[y]), P.ldoo[y], Z, P.ldoo[y], (int32_t)(D.o[y] * D.o[y]), 1.f});
        rb.add(1, false, gBoo[y], D.o[y] * D.o[y], Q, D.o[y] * D.o[y],
               lt::RSeg<double>{A(P.BovP64[x]), P.ldov[x], Z, P.ldoo[y], (int32_t)nov, 1.f});
      }
    }
  }
  // (ia|jb) classes: aa, bb, ab
  const int xy[3][2] = {{0, 0}, {1, 1}, {0, 1}};
  for (int c = 0; c < 3; ++c) {
    double* Z = A(P.dOVOV[c]);
    if (!Z) continue;
    const int x = xy[c][0], y = xy[c][1];
    const int64_t nx = D.o[x] * D.v[x], ny = D.o[y] * D.v[y];
    rb.add(0, true, gBov[x], nx, Q, nx, lt::RSeg<double>{A(P.BovP64[y]), P.ldov[y], Z, P.ldov[y], (int32_t)ny, 1.f});
    rb.add(1, false, gBov[y], ny, Q, ny, lt::RSeg<double>{A(P.BovP64[x]), P.ldov[x], Z, P.ldov[y], (int32_t)nx, 1.f});
  }
  rb.flush();
}

const ltriples_domain_grad kNoGrad{};
char* const kFakeBase = (char*)(uintptr_t)(1ull << 40);

constexpr size_t kPartBytes = size_t(2048) << 20;  // split-contraction partials (cap; plans take what they need)

int plan_backward(const ltriples_domain* d, int32_t prec, const ltriples_options* o, const ItemLists& L,
                  Plan& P) {
  plan_domain(d, prec, o, L, P, true);
  size_t nblk = 0, nseg = 0, nred = 0, dblk = 0, dseg = 0, dred = 0, part = 0;
  std::vector<std::pair<size_t, size_t>> bl;
  if (prec == LT_FP64) {
    RevBuilder<double> rb;
    rb.part = (double*)kFakeBase; rb.part_cap = kPartBytes / 8;
    build_rev<double>(P, L, kFakeBase, rb, bl);
    nblk = rb.blks.size(); nseg = rb.segs.size(); nred = rb.reds.size(); part = 8 * rb.part_max;
  } else {
    RevBuilder<float> rb;
    rb.part = (float*)kFakeBase; rb.part_cap = kPartBytes / 4;
    build_rev<float>(P, L, kFakeBase, rb, bl);
    nblk = rb.blks.size(); nseg = rb.segs.size(); nred = rb.reds.size(); part = 4 * rb.part_max;
  }
  {
    ltriples_domain_grad all;
    double* fake = (double*)kFakeBase;
    all.t1a = all.t1b = all.t2aa = all.t2bb = all.t2ab = fake;
    all.Boo_a = fake + 1; all.Bov_a = fake + 2; all.Bvv_a = fake + 3;
    all.Boo_b = fake + 4; all.Bov_b = fake + 5; all.Bvv_b = fake + 6;
    RevBuilder<double> rb;
    rb.part = (double*)kFakeBase; rb.part_cap = kPartBytes / 8;
    build_df_rev(P, kFakeBase, &all, rb);
    dblk = rb.blks.size(); dseg = rb.segs.size(); dred = rb.reds.size();
    part = std::max(part, (size_t)(8 * rb.part_max));
  }
  size_t off = P.small;
  auto take = [&](Buf& b, size_t bytes) { b.off = off; b.bytes = bytes; off = align256(off + bytes); };
  take(P.rblk, sizeof(lt::RBlk<double>) * std::max<size_t>(nblk, 1));
  take(P.rseg, sizeof(lt::RSeg<double>) * std::max<size_t>(nseg, 1));
  take(P.rred, sizeof(lt::RRed<double>) * std::max<size_t>(nred, 1));
  take(P.dfblk, sizeof(lt::RBlk<double>) * std::max<size_t>(dblk, 1));
  take(P.dfseg, sizeof(lt::RSeg<double>) * std::max<size_t>(dseg, 1));
  take(P.dfred, sizeof(lt::RRed<double>) * std::max<size_t>(dred, 1));
  take(P.rpart, std::max<size_t>(part, 256));
  P.small = off;
  P.total = P.big + P.small;
  return LT_OK;
}

template <typename T>
void log_rev(const RevBuilder<T>& rb) {
  if (!getenv("LTRIPLES_LOG")) return;
  for (size_t l = 0; l < rb.launches.size(); ++l) {
    const auto& L = rb.launches[l];
    int64_t nseg = 0, kmax = 0;
    for (int64_t b = L.blk0; b < L.blk0 + L.nblk; ++b) {
      const auto& B = rb.blks[b];
      nseg += B.end - B.beg;
      int64_t k = 0;
      for (int32_t s = B.beg; s < B.end; ++s) k += rb.segs[s].K;
      kmax = std::max(kmax, k);
    }
    fprintf(stderr, "[ltriples] rev launch %zu tb=%d blocks=%lld rows<=%d cols<=%d segs=%lld maxK=%lld flops=%.3e\n", l,
            (int)L.tb, (long long)L.nblk, L.max_rows, L.max_cols, (long long)nseg, (long long)kmax, L.flops);
  }
}

template <typename T>
int launch_rev_list(const RevBuilder<T>& rb, size_t l0, size_t l1, const lt::RBlk<T>* dblk,
                    const lt::RSeg<T>* dseg, const lt::RRed<T>* dred, hipStream_t st) {
  for (size_t l = l0; l < l1; ++l) {
    const auto& L = rb.launches[l];
    lt::RArgs<T> g{};
    g.nblk = (int32_t)L.nblk; g.max_rows = L.max_rows; g.max_cols = L.max_cols;
    g.blks = dblk + L.blk0; g.segs = dseg;
    HIPCHK(lt::launch_rgemm<T>(g, L.tb, st));
    for (int64_t r = 0; r < L.nred; r += 65535)
      HIPCHK(lt::launch_rreduce<T>(dred + L.red0 + r, (int32_t)std::min<int64_t>(65535, L.nred - r), L.max_red, st));
  }
  return LT_OK;
}

template <typename T>
int run_bwd(const ltriples_domain* d, const Plan& P, const ItemLists& L, const ltriples_options* o,
            const double* gbar, const ltriples_domain_grad* gr, void* ws, hipStream_t st, Timing& tm,
            double* rev_flops) {
  const Dims& D = P.D;
  const int64_t Q = D.Q, oa = D.o[0], ob = D.o[1], va = D.v[0], vb = D.v[1];
  const double* T1[2] = {d->t1a, d->t1b};
  const double* Fov[2] = {d->fov_a, d->fov_b};
  const double* EO[2] = {d->eo_a, d->eo_b};
  const double* EV[2] = {d->ev_a, d->ev_b};
  const double* T2ss[2] = {d->t2aa, d->t2bb};
  char* scr = (char*)ws + P.scratch.off;
  tm.start = tm.mark();
  // outputs and accumulators start at zero
  struct Z { double* p; int64_t n; } outs[] = {
      {gr->t1a, oa * va}, {gr->t1b, ob * vb}, {gr->t2aa, oa * oa * va * va}, {gr->t2bb, ob * ob * vb * vb},
      {gr->t2ab, oa * ob * va * vb}, {gr->Boo_a, Q * oa * oa}, {gr->Bov_a, Q * oa * va}, {gr->Bvv_a, Q * va * va},
      {gr->Boo_b, Q * ob * ob}, {gr->Bov_b, Q * ob * vb}, {gr->Bvv_b, Q * vb * vb},
      {gr->fov_a, oa * va}, {gr->fov_b, ob * vb}, {gr->eo_a, oa}, {gr->ev_a, va}, {gr->eo_b, ob},
      {gr->ev_b, vb}};
  for (auto& z : outs)
    if (z.p) HIPCHK(lt::launch_zero(z.p, z.n, st));
  if (L.total == 0 || (va == 0 && vb == 0)) {
    tm.setup_end = tm.mark();
    tm.end = tm.setup_end;
    return LT_OK;
  }
  {
    const Buf* zb[] = {&P.dT2T[0], &P.dT2T[1], &P.dTp[0], &P.dTp[1], &P.dAs[0], &P.dAs[1], &P.dGamT[0],
                       &P.dGamT[1], &P.dUp[0], &P.dUp[1], &P.dT1p[0], &P.dT1p[1], &P.dFp[0], &P.dFp[1],
                       &P.dLmixT[0], &P.dLmixT[1],
                       &P.dMst[0], &P.dMst[1], &P.dMts[0], &P.dMts[1], &P.dTmix[0], &P.dTmix[1], &P.dZpT[0],
                       &P.dZpT[1], &P.dTmT[0], &P.dTmT[1], &P.dOOT[0], &P.dOOT[1], &P.dOVc[0], &P.dOVc[1],
                       &P.dOVVV[0][0], &P.dOVVV[0][1], &P.dOVVV[1][0], &P.dOVVV[1][1], &P.dOVOO[0][0],
                       &P.dOVOO[0][1], &P.dOVOO[1][0], &P.dOVOO[1][1], &P.dOVOV[0], &P.dOVOV[1], &P.dOVOV[2]};
    for (const Buf* b : zb)
      if (b->bytes) HIPCHK(lt::launch_zero32((char*)ws + b->off, (int64_t)(b->bytes / 4), st));
  }
  {
    const int r = prep<T>(d, P, ws, st);
    if (r) return r;
  }
  tm.setup_end = tm.mark();

  // descriptor lists (host), uploaded once
  RevBuilder<T> rb;
  std::vector<std::pair<size_t, size_t>> bl;
  rb.part = at_small<T>(ws, P, P.rpart); rb.part_cap = kPartBytes / sizeof(T);
  build_rev<T>(P, L, (char*)ws, rb, bl);
  RevBuilder<double> df;
  df.part = at_small<double>(ws, P, P.rpart); df.part_cap = kPartBytes / 8;
  build_df_rev(P, (char*)ws, gr, df);
  auto* d_blk = at_small<lt::RBlk<T>>(ws, P, P.rblk);
  auto* d_seg = at_small<lt::RSeg<T>>(ws, P, P.rseg);
  auto* d_red = at_small<lt::RRed<T>>(ws, P, P.rred);
  auto* d_dfblk = at_small<lt::RBlk<double>>(ws, P, P.dfblk);
  auto* d_dfseg = at_small<lt::RSeg<double>>(ws, P, P.dfseg);
  auto* d_dfred = at_small<lt::RRed<double>>(ws, P, P.dfred);
  if (rb.blks.size() * sizeof(rb.blks[0]) > P.rblk.bytes || rb.segs.size() * sizeof(rb.segs[0]) > P.rseg.bytes ||
      rb.reds.size() * sizeof(lt::RRed<T>) > P.rred.bytes || df.blks.size() * sizeof(df.blks[0]) > P.dfblk.bytes ||
      df.segs.size() * sizeof(df.segs[0]) > P.dfseg.bytes || df.reds.size() * sizeof(df.reds[0]) > P.dfred.bytes ||
      (size_t)rb.part_max * sizeof(T) > P.rpart.bytes || (size_t)df.part_max * 8 > P.rpart.bytes)
    return fail(LT_EWORKSPACE, "descriptor lists exceed their plan");
  auto up = [&](void* dst, const void* src, size_t bytes) -> hipError_t {
    return bytes ? hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st) : hipSuccess;
  };
  HIPCHK(up(d_blk, rb.blks.data(), rb.blks.size() * sizeof(rb.blks[0])));
  HIPCHK(up(d_seg, rb.segs.data(), rb.segs.size() * sizeof(rb.segs[0])));
  HIPCHK(up(d_red, rb.reds.data(), rb.reds.size() * sizeof(lt::RRed<T>)));
  HIPCHK(up(d_dfblk, df.blks.data(), df.blks.size() * sizeof(df.blks[0])));
  HIPCHK(up(d_dfseg, df.segs.data(), df.segs.size() * sizeof(df.segs[0])));
  HIPCHK(up(d_dfred, df.reds.data(), df.reds.size() * sizeof(df.reds[0])));
  HIPCHK(hipStreamSynchronize(st));   // host descriptor vectors go out of scope below
  double rf = 0;
  for (auto& l : rb.launches) rf += l.flops;
  *rev_flops = rf;

  int32_t* d_trip = at_small<int32_t>(ws, P, P.trip);
  int32_t fc[4];
  for (int b = 0, n = 0; b < 4; ++b) { fc[b] = n; n += (int32_t)L.dst[b].size(); }
  const int64_t mstr[2][4] = {{ob * va * vb, va * vb, vb, 1}, {va * vb, ob * va * vb, 1, vb}};
  double* gEO[2] = {gr->eo_a, gr->eo_b};
  double* gEV[2] = {gr->ev_a, gr->ev_b};
  const bool want_eps = gEO[0] || gEO[1] || gEV[0] || gEV[1];
  size_t bi = 0;
  for (int b = 0; b < 4; ++b) {
    const int64_t nblk = P.n_blk[b];
    if (nblk == 0) continue;
    const int s = blk_sigma(b), t = 1 - s;
    const bool mixed = blk_mixed(b);
    const int64_t os = D.o[s], vs = D.v[s], ot = D.o[t], vt = D.v[t];
    lt::ItemOps<T> ops{};
    ops.o_s = (int32_t)os; ops.v_s = (int32_t)vs; ops.o_t = (int32_t)ot; ops.v_t = (int32_t)vt;
    ops.oi_s = (int32_t)os; ops.oi_t = (int32_t)ot;   // the adjoint sums over every orbital
    ops.ld_vs = P.ldv[s]; ops.ld_vt = P.ldv[t]; ops.ld_np = P.ldnp[s]; ops.ld_cb = P.ldcb[s];
    ops.T2T = at<T>(ws, P.T2T[s]); ops.Tp = at<T>(ws, P.Tp[s]); ops.As = at<T>(ws, P.As[s]);
    ops.GamT = at<T>(ws, P.GamT[s]);
    if (mixed) {
      ops.LmixT = at<T>(ws, P.LmixT[s]); ops.Mst = at<T>(ws, P.Mst[s]); ops.Mts = at<T>(ws, P.Mts[s]);
      ops.Tmix = at<T>(ws, P.Tmix[s]); ops.ZpT = at<T>(ws, P.ZpT[s]); ops.TmT = at<T>(ws, P.TmT[s]);
      ops.OOT = at<T>(ws, P.OOT[s]);
    }
    // BF16X3 adjoint: the forward contraction is recomputed on the split
    // operands, from segment descriptors of every item of the block (S or G
    // in the first half of the table, Y in the second); the reverse GEMMs
    // below stay FP32
    lt::Seg8 *tab0 = nullptr, *tab1 = nullptr;
    if (P.bf) {
      lt::ItemOps8 o8{};
      o8.o_s = ops.o_s; o8.v_s = ops.v_s; o8.o_t = ops.o_t; o8.v_t = ops.v_t;
      o8.oi_s = ops.oi_s; o8.oi_t = ops.oi_t;
      o8.ld_vs = ops.ld_vs; o8.ld_vt = ops.ld_vt; o8.ld_np = ops.ld_np; o8.ld_cb = ops.ld_cb;
      auto H = [&](int t8) { return P.O8h[s][t8].bytes ? at<lt::bf16_t>(ws, P.O8h[s][t8]) : nullptr; };
      auto Lo = [&](int t8) { return P.O8l[s][t8].bytes ? at<lt::bf16_t>(ws, P.O8l[s][t8]) : nullptr; };
      o8.T2Th = H(Plan::T2T8); o8.T2Tl = Lo(Plan::T2T8); o8.Ash = H(Plan::As8); o8.Asl = Lo(Plan::As8);
      o8.GamTh = H(Plan::GamT8); o8.GamTl = Lo(Plan::GamT8); o8.Tph = H(Plan::Tp8); o8.Tpl = Lo(Plan::Tp8);
      o8.LmixTh = H(Plan::LmixT8); o8.LmixTl = Lo(Plan::LmixT8); o8.Msth = H(Plan::Mst8); o8.Mstl = Lo(Plan::Mst8);
      o8.Mtsh = H(Plan::Mts8); o8.Mtsl = Lo(Plan::Mts8); o8.Tmixh = H(Plan::Tmix8); o8.Tmixl = Lo(Plan::Tmix8);
      o8.Tmx2h = H(Plan::Tmx28); o8.Tmx2l = Lo(Plan::Tmx28); o8.ZpTh = H(Plan::ZpT8); o8.ZpTl = Lo(Plan::ZpT8);
      o8.TmTh = H(Plan::TmT8); o8.TmTl = Lo(Plan::TmT8); o8.OOTh = H(Plan::OOT8); o8.OOTl = Lo(Plan::OOT8);
      tab0 = at_small<lt::Seg8>(ws, P, P.segtab);
      tab1 = tab0 + 6 * std::max<int64_t>(L.total, 1);
      o8.items = d_trip + 3 * fc[b];
      o8.kind = mixed ? 1 : 0;
      HIPCHK(lt::launch_seg8_table(o8, (int32_t)nblk, tab0 + 6 * (int64_t)fc[b], st));
      if (mixed) {
        o8.kind = 2;
        HIPCHK(lt::launch_seg8_table(o8, (int32_t)nblk, tab1 + 6 * (int64_t)fc[b], st));
      }
    }
    auto contract = [&](const lt::GemmArgs<T>& g) -> hipError_t {
      if (!P.bf) return lt::launch_gemm<T>(g, st);
      if (g.M <= 0 || g.N <= 0 || g.nbatch <= 0) return hipSuccess;
      lt::GemmArgs16 h{};
      h.M = g.M; h.N = g.N; h.nbatch = g.nbatch; h.nprod = P.bf;
      h.out = (float*)(void*)g.out; h.obs = g.obs; h.ldo = g.s_mr; h.kind = g.ops.kind;
      h.tab = (g.ops.kind == 2 ? tab1 : tab0) + 6 * ((g.ops.items - d_trip) / 3);
      return lt::launch_gemm_bf16(h, st);
    };
    const int64_t nb = P.nb[b];
    const size_t o1 = P.o1[b], o2 = P.o2[b];
    const int64_t nt = P.ntile[b];
    // orbital-energy adjoint buffers behind the three output copies
    const size_t ep_off = 3 * (size_t)nb * (o1 + o2), ri_off = ep_off + 512 * (size_t)nb * P.bwg[b];
    if (want_eps && ri_off + 8 * (size_t)nb * P.ld_ri[b] > P.scratch.bytes)
      return fail(LT_EWORKSPACE, "orbital-energy adjoint buffers exceed the batch scratch");
    lt::EpsReduce er{};
    er.mixed = mixed ? 1 : 0; er.nwg = (int32_t)P.bwg[b];
    er.nt_s = (int32_t)cdiv(vs, lt::ET); er.nt_t = (int32_t)cdiv(vt, lt::ET);
    er.o_s = (int32_t)os; er.v_s = (int32_t)vs; er.o_t = (int32_t)ot; er.v_t = (int32_t)vt;
    er.ep = (double*)(scr + ep_off); er.ri = (double*)(scr + ri_off); er.ld_ri = P.ld_ri[b];
    er.eo_s = gEO[s]; er.ev_s = gEV[s]; er.eo_t = mixed ? gEO[t] : nullptr; er.ev_t = mixed ? gEV[t] : nullptr;
    for (int64_t first = 0; first < nblk; first += nb, ++bi) {
      const int64_t n = std::min<int64_t>(nb, nblk - first);
      const int32_t* items = d_trip + 3 * (fc[b] + first);
      ops.items = items;
      lt::GemmArgs<T> g{};
      g.nbatch = (int32_t)n; g.mode = 1; g.s_nr = 1;
      hipEvent_t a0 = tm.mark();
      if (!mixed) {
        T* S = (T*)scr;
        ops.kind = 0;
        g.M = (int32_t)vs; g.N = (int32_t)npair(vs); g.out = S; g.obs = (int64_t)(o1 / P.ts); g.s_mr = P.ldnp[s];
        g.ops = ops;
        HIPCHK(contract(g));
        tm.gemm_flops += 2.0 * (double)g.M * (double)g.N * (double)(3 * vs + 3 * os) * (double)n;
        hipEvent_t a1 = tm.mark();
        tm.gemm.push_back({a0, a1});
        lt::BwdSame<T> e{};
        e.e.o = (int32_t)os; e.e.v = (int32_t)vs; e.e.ld_np = P.ldnp[s];
        e.e.S = S; e.e.s_item = (int64_t)(o1 / P.ts); e.e.items = items;
        {
          const int64_t nt1 = cdiv(vs, lt::ET);
          e.e.nt = (int32_t)nt1;
          e.e.ntri = (int32_t)(nt1 * (nt1 + 1) * (nt1 + 2) / 6);   // backward grid: a <= b <= c tiles
        }
        e.e.eo = EO[s]; e.e.ev = EV[s]; e.e.t1 = T1[s]; e.e.f = Fov[s]; e.e.t2 = T2ss[s];
        e.e.U = at<double>(ws, P.U[s]); e.e.ld_v = P.ldv[s];
        e.gbar = gbar;
        e.dS = (T*)(scr + (size_t)nb * o1);
        e.dSV = (T*)(scr + 2 * (size_t)nb * o1);
        if (want_eps) e.ep = (double*)(scr + ep_off);
        if (e.e.ntri != P.bwg[b]) return fail(LT_ESHAPE, "backward epilogue grid does not match its plan");
        HIPCHK(lt::launch_bwd_same<T>(e, (int32_t)n, st));
        tm.epi.push_back({a1, tm.mark()});
      } else {
        T* G = (T*)scr;
        T* Y = (T*)(scr + (size_t)nb * o1);
        ops.kind = 1;
        g.M = (int32_t)vs; g.N = (int32_t)(vt * vs); g.out = G; g.obs = (int64_t)(o1 / P.ts); g.s_mr = P.ldcb[s];
        g.ops = ops;
        HIPCHK(contract(g));
        tm.gemm_flops += 2.0 * (double)g.M * (double)g.N * (double)(2 * vt + vs + os + 2 * ot) * (double)n;
        ops.kind = 2;
        g.M = (int32_t)vt; g.N = (int32_t)npair(vs); g.out = Y; g.obs = (int64_t)(o2 / P.ts); g.s_mr = P.ldnp[s];
        g.ops = ops;
        HIPCHK(contract(g));
        tm.gemm_flops += 2.0 * (double)g.M * (double)g.N * (double)(2 * vs + 2 * os) * (double)n;
        hipEvent_t a1 = tm.mark();
        tm.gemm.push_back({a0, a1});
        lt::BwdMixed<T> e{};
        lt::EpiMixed<T>& x = e.e;
        x.o_s = (int32_t)os; x.v_s = (int32_t)vs; x.o_t = (int32_t)ot; x.v_t = (int32_t)vt;
        x.ld_np = P.ldnp[s]; x.ld_cb = P.ldcb[s];
        x.G = G; x.g_item = (int64_t)(o1 / P.ts); x.Y = Y; x.y_item = (int64_t)(o2 / P.ts);
        x.items = items;
        x.nts = (int32_t)cdiv(vs, lt::ET); x.ntt = (int32_t)cdiv(vt, lt::ET);
        x.ntiles = x.nts * (x.nts + 1) / 2 * x.ntt;
        x.eo_s = EO[s]; x.ev_s = EV[s]; x.eo_t = EO[t]; x.ev_t = EV[t];
        x.t1_s = T1[s]; x.t1_t = T1[t]; x.f_s = Fov[s]; x.f_t = Fov[t]; x.t2ss = T2ss[s];
        x.U = at<double>(ws, P.U[s]); x.ld_vs = P.ldv[s];
        const int64_t so[4] = {va * ob * vb, ob * vb, vb, 1};
        x.ov = at<double>(ws, P.OVab);
        if (s == 0) { x.ov_o = so[0]; x.ov_v = so[1]; x.ov_O = so[2]; x.ov_V = so[3]; }
        else { x.ov_o = so[2]; x.ov_v = so[3]; x.ov_O = so[0]; x.ov_V = so[1]; }
        x.tm = d->t2ab; x.tm_o = mstr[s][0]; x.tm_v = mstr[s][2]; x.tm_O = mstr[s][1]; x.tm_V = mstr[s][3];
        e.gbar = gbar;
        const size_t q1 = (size_t)nb * (o1 + o2);
        e.dG = (T*)(scr + q1);
        e.dY = (T*)(scr + q1 + (size_t)nb * o1);
        e.dGV = (T*)(scr + 2 * q1);
        e.dYV = (T*)(scr + 2 * q1 + (size_t)nb * o1);
        if (want_eps) e.ep = (double*)(scr + ep_off);
        if (x.ntiles != P.bwg[b]) return fail(LT_ESHAPE, "backward epilogue grid does not match its plan");
        HIPCHK(lt::launch_bwd_mixed<T>(e, (int32_t)n, st));
        tm.epi.push_back({a1, tm.mark()});
      }
      if (want_eps) {
        er.nitems = (int32_t)n; er.items = items;
        HIPCHK(lt::launch_eps_reduce(er, st));
      }
      hipEvent_t r0 = tm.mark();
      {
        const int r = launch_rev_list<T>(rb, bl[bi].first, bl[bi].second, d_blk, d_seg, d_red, st);
        if (r) return r;
      }
      tm.gemm.push_back({r0, tm.mark()});
    }
  }

  // --- mirrors -> amplitude gradients and FP64 integral gradients ---------------------
  auto Tb = [&](const Buf& b) { return at<T>(ws, b); };
  auto Db = [&](const Buf& b) { return at<double>(ws, b); };
  double* gT1[2] = {gr->t1a, gr->t1b};
  double* gF[2] = {gr->fov_a, gr->fov_b};
  double* gT2[2] = {gr->t2aa, gr->t2bb};
  for (int s = 0; s < 2; ++s) {
    const int t = 1 - s;
    const int64_t o = D.o[s], v = D.v[s], lv = P.ldv[s], lp = P.ldnp[s];
    if (P.dT1p[s].bytes && gT1[s]) {
      const int64_t dd[4] = {1, 1, o, v}, os_[4] = {0, 0, v, 1}, is_[4] = {0, 0, lv, 1};
      HIPCHK(lt::launch_perm_acc<T>(gT1[s], dd, os_, Tb(P.dT1p[s]), is_, 1.0, st));
    }
    if (P.dFp[s].bytes && gF[s]) {
      const int64_t dd[4] = {1, 1, o, v}, os_[4] = {0, 0, v, 1}, is_[4] = {0, 0, lv, 1};
      HIPCHK(lt::launch_perm_acc<T>(gF[s], dd, os_, Tb(P.dFp[s]), is_, 1.0, st));
    }
    if (P.need_as[s]) {
      if (gT2[s]) {
        // T2T[i][j][e][a] = t2[i][j][a][e]
        const int64_t dd[4] = {o, o, v, v}, os_[4] = {o * v * v, v * v, 1, v}, is_[4] = {o * v * lv, v * lv, lv, 1};
        HIPCHK(lt::launch_perm_acc<T>(gT2[s], dd, os_, Tb(P.dT2T[s]), is_, 1.0, st));
        // Tp[i][m][p(a<b)] = t2[i][m][a][b]
        HIPCHK(lt::launch_unpack_acc<T>(gT2[s], o, o, (int32_t)v, o * v * v, v * v, v, 1, Tb(P.dTp[s]), o * lp, lp,
                                        1.0, 0.0, st));
      }
      const int64_t lvv = P.ldvv[s], loo = P.ldoo[s], lov = P.ldov[s];
      // As[i][e][p(b<c)] = (ic|eb) - (ib|ec)  ->  d(ix|ey) at [i][x][e*v+y]
      HIPCHK(lt::launch_unpack_acc<T>(Db(P.dOVVV[s][s]), o, v, (int32_t)v, v * lvv, v, lvv, 1, Tb(P.dAs[s]), v * lp,
                                      lp, -1.0, 1.0, st));
      // GamT[j][k][m][a] = (ak|mj) - (aj|mk)  ->  d(ka|mj) at [k][a][m*o+j]
      {
        const int64_t dd[4] = {o, o, o, v}, is_[4] = {o * o * lv, o * lv, lv, 1};
        const int64_t o1_[4] = {1, v * loo, o, loo}, o2_[4] = {v * loo, 1, o, loo};
        HIPCHK(lt::launch_perm_acc<T>(Db(P.dOVOO[s][s]), dd, o1_, Tb(P.dGamT[s]), is_, 1.0, st));
        HIPCHK(lt::launch_perm_acc<T>(Db(P.dOVOO[s][s]), dd, o2_, Tb(P.dGamT[s]), is_, -1.0, st));
      }
      // Up[q][r][p(b<c)] = (qb|rc) - (qc|rb)  ->  d(qx|ry) at [q][x][r*v+y]
      HIPCHK(lt::launch_unpack_acc<T>(Db(P.dOVOV[s]), o, o, (int32_t)v, v * lov, v, lov, 1, Tb(P.dUp[s]), o * lp, lp,
                                      1.0, -1.0, st));
    }
    if (P.need_mix[s]) {
      const int64_t os = o, vs = v, ot = D.o[t], vt = D.v[t], lvt = P.ldv[t], lc = P.ldcb[s];
      const int64_t* m = mstr[s];
      if (gr->t2ab) {
        // LmixT[i][K][E][a] = t^{aE}_{iK}; Tmix[i][K][C*vs+b] = t^{bC}_{iK}; TmT[i][K][e][C] = t^{eC}_{iK}
        const int64_t d1[4] = {os, ot, vt, vs}, i1[4] = {ot * vt * lv, vt * lv, lv, 1}, q1[4] = {m[0], m[1], m[3], m[2]};
        HIPCHK(lt::launch_perm_acc<T>(gr->t2ab, d1, q1, Tb(P.dLmixT[s]), i1, 1.0, st));
        const int64_t d2[4] = {os, ot, vt, vs}, i2[4] = {ot * lc, lc, vs, 1}, q2[4] = {m[0], m[1], m[3], m[2]};
        HIPCHK(lt::launch_perm_acc<T>(gr->t2ab, d2, q2, Tb(P.dTmix[s]), i2, 1.0, st));
        const int64_t d3[4] = {os, ot, vs, vt}, i3[4] = {ot * vs * lvt, vs * lvt, lvt, 1}, q3[4] = {m[0], m[1], m[2], m[3]};
        HIPCHK(lt::launch_perm_acc<T>(gr->t2ab, d3, q3, Tb(P.dTmT[s]), i3, 1.0, st));
      }
      // Mst[j][E][C*vs+b] = (jb|EC) -> [j][b][E*vt+C] of (ov|vv)_{st}
      {
        const int64_t l = P.ldvv[t];
        const int64_t dd[4] = {os, vt, vt, vs}, is_[4] = {vt * lc, lc, vs, 1}, oo_[4] = {vs * l, vt, 1, l};
        HIPCHK(lt::launch_perm_acc<T>(Db(P.dOVVV[s][t]), dd, oo_, Tb(P.dMst[s]), is_, 1.0, st));
      }
      // Mts[K][e][C*vs+b] = (KC|be) -> [K][C][b*vs+e] of (ov|vv)_{ts}
      {
        const int64_t l = P.ldvv[s];
        const int64_t dd[4] = {ot, vs, vt, vs}, is_[4] = {vs * lc, lc, vs, 1}, oo_[4] = {vt * l, 1, l, vs};
        HIPCHK(lt::launch_perm_acc<T>(Db(P.dOVVV[t][s]), dd, oo_, Tb(P.dMts[s]), is_, 1.0, st));
      }
      // ZpT[j][K][M][a] = (ja|MK) -> [j][a][M*ot+K] of (ov|oo)_{st}
      {
        const int64_t l = P.ldoo[t];
        const int64_t dd[4] = {os, ot, ot, vs}, is_[4] = {ot * ot * lv, ot * lv, lv, 1}, oo_[4] = {vs * l, 1, ot, l};
        HIPCHK(lt::launch_perm_acc<T>(Db(P.dOVOO[s][t]), dd, oo_, Tb(P.dZpT[s]), is_, 1.0, st));
      }
      // OOT[K][j][m][C] = (KC|jm) -> [K][C][j*os+m] of (ov|oo)_{ts}
      {
        const int64_t l = P.ldoo[s];
        const int64_t dd[4] = {ot, os, os, vt}, is_[4] = {os * os * lvt, os * lvt, lvt, 1}, oo_[4] = {vt * l, os, 1, l};
        HIPCHK(lt::launch_perm_acc<T>(Db(P.dOVOO[t][s]), dd, oo_, Tb(P.dOOT[s]), is_, 1.0, st));
      }
      // OVc[j][K][C*vs+b] = (jb|KC) -> (ov|ov)_{ab}
      {
        const int64_t l = P.ldov[1];
        const int64_t dd[4] = {os, ot, vt, vs}, is_[4] = {ot * lc, lc, vs, 1};
        const int64_t oa_[4] = {va * l, vb, 1, l};    // s = alpha: [j][b][K*vb+C]
        const int64_t ob_[4] = {vb, va * l, l, 1};    // s = beta:  [K][C][j*vb+b]
        HIPCHK(lt::launch_perm_acc<T>(Db(P.dOVOV[2]), dd, s == 0 ? oa_ : ob_, Tb(P.dOVc[s]), is_, 1.0, st));
      }
    }
  }
  // --- DF back-contraction -------------------------------------------------------------
  {
    const int r = launch_rev_list<double>(df, 0, df.launches.size(), d_dfblk, d_dfseg, d_dfred, st);
    if (r) return r;
  }
  // --- projections of the constrained inputs -------------------------------------------
  if (gr->t2aa) HIPCHK(lt::launch_antisym4(gr->t2aa, oa, va, st));
  if (gr->t2bb) HIPCHK(lt::launch_antisym4(gr->t2bb, ob, vb, st));
  if (gr->Boo_a) HIPCHK(lt::launch_sym3(gr->Boo_a, Q, oa, st));
  if (gr->Bvv_a) HIPCHK(lt::launch_sym3(gr->Bvv_a, Q, va, st));
  if (gr->Boo_b) HIPCHK(lt::launch_sym3(gr->Boo_b, Q, ob, st));
  if (gr->Bvv_b) HIPCHK(lt::launch_sym3(gr->Bvv_b, Q, vb, st));
  tm.end = tm.mark();
  (void)o;
  return LT_OK;
}

// Scratch of ltriples_energy_noalloc: the whole workspace of such a call
// (operand layouts, integral slabs, per-batch intermediates, item tables).
// One copy per device, placed when the library's code object is loaded on
// it and held until the process ends.  Host code never uses the symbol's
// name as an address: each device's copy is found once with
// hipGetSymbolAddress (noalloc_scratch) and that pointer is passed on.
constexpr size_t kNoAllocBytes = size_t(256) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;   // per device index

// This device's copy of `scratch` (looked up on the first call on it).
int noalloc_scratch(void** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr)
      return fail(LT_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return LT_OK;
}

// Shared body of ltriples_energy and ltriples_energy_noalloc.  With
// `noalloc` the workspace is this device's `scratch`: the plan is refitted to
// it with smaller item batches and build chunks when needed (results are
// bitwise the same for any batching and chunking), and nothing is allocated
// (options.stats and options.autotune, which create HIP events, are refused).
int energy_call(const ltriples_domain* d, int32_t precision, const ltriples_options* o, double* e_out,
                double* parts, void* ws, size_t ws_bytes, hipStream_t st, bool noalloc, double* dump_w = nullptr) {
  int r = validate(d, precision, o);
  if (r) return r;
  if (!e_out) return fail(LT_EINVAL, "e_out is NULL");
  if (noalloc && o && (o->stats || o->autotune))
    return fail(LT_EINVAL, "the no-allocation entry point takes no stats and no autotuning");
  const Dims D = dims_of(d);
  ltriples_options oo = o ? *o : ltriples_options{};
  ItemLists L;
  build_items(D, &oo, L);
  Plan P;
  plan_domain(d, precision, &oo, L, P);
  P.dump_w = dump_w;
  if (noalloc) {
    static const int64_t budgets_mib[] = {128, 64, 32, 16, 8, 4, 2, 1};
    for (int k = 0; P.total > kNoAllocBytes && k < (int)(sizeof(budgets_mib) / sizeof(budgets_mib[0])); ++k) {
      oo.workspace_budget = (size_t)budgets_mib[k] << 20;
      oo.build_chunk_mib = (int32_t)std::min<int64_t>(16, budgets_mib[k]);
      P = Plan{};
      plan_domain(d, precision, &oo, L, P);
    }
    if (P.total > kNoAllocBytes)
      return fail(LT_EWORKSPACE, "domain needs %zu bytes of workspace even in single-item batches; the "
                  "no-allocation entry point has %zu", P.total, kNoAllocBytes);
  }
  r = check_denominators(d, st);
  if (r) return r;
  log_plan(P);
  r = check_plan(P);
  if (r) return r;
  if (noalloc) {
    r = noalloc_scratch(&ws);
    if (r) return r;
    ws_bytes = kNoAllocBytes;
  }
  OwnedWs own;
  r = get_ws(ws, ws_bytes, P.total, st, own);
  if (r) return r;
  r = upload_items(P, L, ws, st);
  if (r) return r;
  if (oo.check_finite) {
    r = scan_finite(d, P, ws, st);
    if (r) return r;
  }
  Timing tm;
  tm.on = oo.stats != nullptr;
  tm.st = st;
  if (precision == LT_FP64) r = run<double>(d, P, L, &oo, e_out, parts, ws, st, tm);
  else r = run<float>(d, P, L, &oo, e_out, parts, ws, st, tm);   // FP32, BF16X3, BF16
  if (r == LT_OK && tm.on) {
    HIPCHK(hipStreamSynchronize(st));
    ltriples_stats* S = oo.stats;
    *S = ltriples_stats{};
    S->total_ms = Timing::ms(tm.start, tm.end);
    S->setup_ms = Timing::ms(tm.start, tm.setup_end);
    for (auto& x : tm.gemm) S->triples_gemm_ms += Timing::ms(x.first, x.second);
    for (auto& x : tm.epi) S->epilogue_ms += Timing::ms(x.first, x.second);
    S->triples_gemm_launches = (int64_t)tm.gemm.size();
    S->triples_gemm_flops = tm.gemm_flops;
    double f = 0;
    for (int b = 0; b < 4; ++b) f += (double)P.n_blk[b] * item_flops(D, b);
    S->algorithmic_flops = f;
    S->n_items = L.total;
  }
  return r;
}

}  // namespace

extern "C" {

int ltriples_validate(const ltriples_domain* d, int32_t precision, const ltriples_options* o) {
  g_err.clear();
  return validate(d, precision, o);
}

int ltriples_workspace_size(const ltriples_domain* d, int32_t precision, const ltriples_options* o,
                            size_t* bytes) {
  g_err.clear();
  if (!bytes) return fail(LT_EINVAL, "bytes is NULL");
  const int r = validate(d, precision, o);
  if (r) return r;
  ItemLists L;
  build_items(dims_of(d), o, L);
  Plan P;
  plan_domain(d, precision, o, L, P);
  log_plan(P);
  *bytes = P.total;
  return LT_OK;
}

int ltriples_flops(const ltriples_domain* d, const ltriples_options* o, double* flops, int64_t* n_items_out) {
  g_err.clear();
  if (!d || !flops) return fail(LT_EINVAL, "NULL argument");
  const Dims D = dims_of(d);
  if (o && o->items) {
    const int r = check_items(D, o);
    if (r) return r;
    double f = 0;
    for (int32_t n = 0; n < o->n_items; ++n) f += item_flops(D, o->items[4 * n]);
    *flops = f;
    if (n_items_out) *n_items_out = o->n_items;
    return LT_OK;
  }
  const int64_t oa = D.o[0], ob = D.o[1];
  const int64_t cnt[4] = {oa * (oa - 1) * (oa - 2) / 6, oa * (oa - 1) / 2 * ob, ob * (ob - 1) / 2 * oa,
                          ob * (ob - 1) * (ob - 2) / 6};
  double f = 0;
  for (int b = 0; b < 4; ++b) f += (double)cnt[b] * item_flops(D, b);
  *flops = f;
  if (n_items_out) *n_items_out = count_all_items(D);
  return LT_OK;
}

int ltriples_energy(const ltriples_domain* d, int32_t precision, const ltriples_options* o, double* e_out,
                    double* parts, void* ws, size_t ws_bytes, void* stream) {
  g_err.clear();
  return energy_call(d, precision, o, e_out, parts, ws, ws_bytes, (hipStream_t)stream, false);
}

int ltriples_energy_noalloc(const ltriples_domain* d, int32_t precision, const ltriples_options* o,
                            double* e_out, double* parts, void* stream) {
  g_err.clear();
  return energy_call(d, precision, o, e_out, parts, nullptr, 0, (hipStream_t)stream, true);
}

size_t ltriples_noalloc_capacity(void) { return kNoAllocBytes; }

int ltriples_debug_w(const ltriples_domain* d, int32_t precision, const int32_t* item, double* w,
                     double* e_out, void* ws, size_t ws_bytes, void* stream) {
  g_err.clear();
  if (!item) return fail(LT_EINVAL, "item is NULL");
  if (!w) return fail(LT_EINVAL, "w is NULL");
  ltriples_options o{};
  o.items = item;
  o.n_items = 1;
  return energy_call(d, precision, &o, e_out, nullptr, ws, ws_bytes, (hipStream_t)stream, false, w);
}

// ---------------------------------------------------------------------------
// Adjoint entry points
// ---------------------------------------------------------------------------
}  // extern "C"

static int validate_bwd(const ltriples_domain* d, int32_t precision, const ltriples_options* o) {
  int r = validate(d, precision, o);
  if (r) return r;
  if (precision != LT_FP64 && precision != LT_FP32 && precision != LT_BF16X3)
    return fail(LT_EPREC, "the adjoint pass supports FP64, FP32 and BF16X3 only");
  if (o && o->e_items) return fail(LT_EINVAL, "per-item outputs are a forward option");
  return LT_OK;
}

// ---------------------------------------------------------------------------
// Host-only plan self-check of the adjoint descriptors
// ---------------------------------------------------------------------------
namespace {

struct Range { uintptr_t lo, hi; const char* name; };

template <typename T>
int check_rev(const RevBuilder<T>& rb, const std::vector<Range>& bufs, uintptr_t grad_lo, uintptr_t grad_hi,
              bool element_check) {
  const size_t ts = sizeof(T);
  auto inside = [&](uintptr_t a, uintptr_t b) -> const Range* {
    for (const Range& r : bufs)
      if (a >= r.lo && b <= r.hi) return &r;
    if (a >= grad_lo && b <= grad_hi) return &bufs[0];   // caller outputs (checked per field below)
    return nullptr;
  };
  auto r4 = [](int64_t k) { return (k + 3) & ~int64_t(3); };
  for (size_t li = 0; li < rb.launches.size(); ++li) {
    const auto& L = rb.launches[li];
    std::vector<uintptr_t> elems;
    for (int64_t bi = L.blk0; bi < L.blk0 + L.nblk; ++bi) {
      const lt::RBlk<T>& b = rb.blks[bi];
      const uintptr_t o = (uintptr_t)b.out;
      if (b.rows <= 0 || b.cols <= 0 || b.ldo < b.cols) return fail(LT_ESHAPE, "launch %zu block %lld: bad shape", li, (long long)bi);
      if (!inside(o, o + ((b.rows - 1) * b.ldo + b.cols) * ts))
        return fail(LT_EWORKSPACE, "launch %zu block %lld: output outside its buffer", li, (long long)bi);
      if (element_check)
        for (int r = 0; r < b.rows; ++r)
          for (int c = 0; c < b.cols; ++c) elems.push_back(o + (r * b.ldo + c) * ts);
      for (int32_t si = b.beg; si < b.end; ++si) {
        const lt::RSeg<T>& sg = rb.segs[si];
        const uintptr_t a = (uintptr_t)sg.A, bb = (uintptr_t)sg.B;
        if (sg.K <= 0) continue;
        if ((a % 16) || (bb % 16) || (sg.lda % 4) || (sg.ldb % 4))
          return fail(LT_ESHAPE, "launch %zu segment %d: misaligned operand", li, si);
        if (sg.lda < sg.K && b.rows > 1) return fail(LT_ESHAPE, "launch %zu segment %d: lda < K", li, si);
        if (!inside(a, a + ((b.rows - 1) * sg.lda + r4(sg.K)) * ts))
          return fail(LT_EWORKSPACE, "launch %zu segment %d: A outside its buffer", li, si);
        const uintptr_t bend = L.tb ? bb + ((b.cols - 1) * sg.ldb + r4(sg.K)) * ts
                                    : bb + ((sg.K - 1) * sg.ldb + r4(b.cols)) * ts;
        if (!L.tb && sg.ldb < r4(b.cols)) return fail(LT_ESHAPE, "launch %zu segment %d: ldb < cols", li, si);
        if (!inside(bb, bend)) return fail(LT_EWORKSPACE, "launch %zu segment %d: B outside its buffer", li, si);
      }
    }
    if (element_check) {
      std::sort(elems.begin(), elems.end());
      if (std::adjacent_find(elems.begin(), elems.end()) != elems.end())
        return fail(LT_ESHAPE, "launch %zu: output blocks overlap", li);
    }
  }
  return LT_OK;
}

template <typename T>
int check_red(const RevBuilder<T>& rb, const std::vector<Range>& outs, const Range& part) {
  const size_t ts = sizeof(T);
  for (size_t i = 0; i < rb.reds.size(); ++i) {
    const lt::RRed<T>& r = rb.reds[i];
    const uintptr_t o = (uintptr_t)r.out, p = (uintptr_t)r.part;
    bool ok = false;
    for (const Range& x : outs)
      if (o >= x.lo && o + ((r.rows - 1) * r.ldo + r.cols) * ts <= x.hi) ok = true;
    if (!ok) return fail(LT_EWORKSPACE, "reduce %zu: target outside its buffer", i);
    if (!(p >= part.lo && p + (size_t)r.nchunk * r.rows * r.cols * ts <= part.hi))
      return fail(LT_EWORKSPACE, "reduce %zu: partials outside their buffer", i);
  }
  return LT_OK;
}

template <typename T>
int plan_check_bwd(const Plan& P, const ItemLists& L, bool element_check) {
  char* base = kFakeBase;
  std::vector<Range> bufs;
  // every planned buffer of the big and small regions
  const Buf* all[] = {&P.BvvP[0], &P.BvvP[1], &P.BovR[0], &P.BovR[1], &P.BovP64[0], &P.BovP64[1], &P.BooP64[0],
                      &P.BooP64[1], &P.As[0], &P.As[1], &P.Tp[0], &P.Tp[1], &P.T2T[0], &P.T2T[1], &P.GamT[0],
                      &P.GamT[1], &P.U[0], &P.U[1], &P.LmixT[0], &P.LmixT[1], &P.Mst[0], &P.Mst[1], &P.Mts[0],
                      &P.Mts[1], &P.Tmix[0], &P.Tmix[1], &P.ZpT[0], &P.ZpT[1], &P.TmT[0], &P.TmT[1], &P.OOT[0],
                      &P.OOT[1], &P.OVab, &P.T1p[0], &P.T1p[1], &P.Fp[0], &P.Fp[1], &P.Up[0], &P.Up[1],
                      &P.OVc[0], &P.OVc[1], &P.BvvP64[0], &P.BvvP64[1], &P.dT2T[0], &P.dT2T[1], &P.dTp[0],
                      &P.dTp[1], &P.dAs[0], &P.dAs[1], &P.dGamT[0], &P.dGamT[1], &P.dUp[0], &P.dUp[1],
                      &P.dT1p[0], &P.dT1p[1], &P.dFp[0], &P.dFp[1], &P.dLmixT[0], &P.dLmixT[1], &P.dMst[0],
                      &P.dMst[1], &P.dMts[0],
                      &P.dMts[1], &P.dTmix[0], &P.dTmix[1], &P.dZpT[0], &P.dZpT[1], &P.dTmT[0], &P.dTmT[1],
                      &P.dOOT[0], &P.dOOT[1], &P.dOVc[0], &P.dOVc[1], &P.dOVVV[0][0], &P.dOVVV[0][1],
                      &P.dOVVV[1][0], &P.dOVVV[1][1], &P.dOVOO[0][0], &P.dOVOO[0][1], &P.dOVOO[1][0],
                      &P.dOVOO[1][1], &P.dOVOV[0], &P.dOVOV[1], &P.dOVOV[2], &P.scratch};
  for (const Buf* b : all)
    if (b->bytes) bufs.push_back({(uintptr_t)(base + b->off), (uintptr_t)(base + b->off + b->bytes), ""});
  if (bufs.empty()) return LT_OK;
  for (size_t i = 0; i < bufs.size(); ++i)
    if (bufs[i].hi > (uintptr_t)(base + P.big)) return fail(LT_EWORKSPACE, "buffer beyond the planned region");
  char* pbase = base + P.small_base + P.rpart.off;
  const Range part{(uintptr_t)pbase, (uintptr_t)(pbase + P.rpart.bytes), "part"};
  if (part.hi > (uintptr_t)(base + P.total)) return fail(LT_EWORKSPACE, "partials beyond the workspace");
  const std::vector<Range> mirrors = bufs;
  bufs.push_back(part);
  RevBuilder<T> rb;
  std::vector<std::pair<size_t, size_t>> bl;
  rb.part = (T*)pbase; rb.part_cap = kPartBytes / sizeof(T);
  build_rev<T>(P, L, base, rb, bl);
  log_rev(rb);
  int r = check_rev<T>(rb, bufs, 0, 0, element_check);
  if (r) return r;
  r = check_red<T>(rb, mirrors, part);
  if (r) return r;
  // DF back-contraction: caller outputs as disjoint fake regions
  const Dims& D = P.D;
  const int64_t Q = D.Q;
  ltriples_domain_grad g{};
  uintptr_t gb = (uintptr_t)(base + P.total + 4096);
  const int64_t sizes[6] = {Q * D.o[0] * D.o[0], Q * D.o[0] * D.v[0], Q * D.v[0] * D.v[0],
                            Q * D.o[1] * D.o[1], Q * D.o[1] * D.v[1], Q * D.v[1] * D.v[1]};
  double** f[6] = {&g.Boo_a, &g.Bov_a, &g.Bvv_a, &g.Boo_b, &g.Bov_b, &g.Bvv_b};
  std::vector<Range> gr = bufs;
  for (int k = 0; k < 6; ++k) {
    *f[k] = (double*)gb;
    gr.push_back({gb, gb + 8 * (uintptr_t)sizes[k], ""});
    gb = align256(gb + 8 * (uintptr_t)sizes[k] + 4096);
  }
  RevBuilder<double> df;
  df.part = (double*)pbase; df.part_cap = kPartBytes / 8;
  build_df_rev(P, base, &g, df);
  std::vector<Range> gp = gr;
  gp.push_back(part);
  r = check_rev<double>(df, gp, 0, 0, element_check);
  if (r) return r;
  return check_red<double>(df, gr, part);
}

}  // namespace

extern "C" int ltriples_plan_check(const ltriples_domain* d, int32_t precision, const ltriples_options* o,
                                   int32_t backward) {
  g_err.clear();
  int r = backward ? validate_bwd(d, precision, o) : validate(d, precision, o);
  if (r) return r;
  if (!backward) return LT_OK;
  ItemLists L;
  build_items(dims_of(d), o, L);
  Plan P;
  plan_backward(d, precision, o, L, P);
  const bool el = P.total < (size_t(1) << 28);
  return precision == LT_FP64 ? plan_check_bwd<double>(P, L, el) : plan_check_bwd<float>(P, L, el);
}


extern "C" {

int ltriples_backward_workspace_size(const ltriples_domain* d, int32_t precision, const ltriples_options* o,
                                     size_t* bytes) {
  g_err.clear();
  if (!bytes) return fail(LT_EINVAL, "bytes is NULL");
  const int r = validate_bwd(d, precision, o);
  if (r) return r;
  ItemLists L;
  build_items(dims_of(d), o, L);
  Plan P;
  plan_backward(d, precision, o, L, P);
  *bytes = P.total;
  return LT_OK;
}

int ltriples_backward(const ltriples_domain* d, int32_t precision, const ltriples_options* o, const double* gbar,
                      const ltriples_domain_grad* grad, void* ws, size_t ws_bytes, void* stream) {
  g_err.clear();
  int r = validate_bwd(d, precision, o);
  if (r) return r;
  if (!gbar) return fail(LT_EINVAL, "gbar is NULL");
  if (!grad) return fail(LT_EINVAL, "grad is NULL");
  hipStream_t st = (hipStream_t)stream;
  const Dims D = dims_of(d);
  r = check_denominators(d, st);
  if (r) return r;
  ItemLists L;
  build_items(D, o, L);
  Plan P;
  plan_backward(d, precision, o, L, P);
  log_plan(P);
  OwnedWs own;
  r = get_ws(ws, ws_bytes, P.total, st, own);
  if (r) return r;
  r = upload_items(P, L, ws, st);
  if (r == LT_OK && o && o->check_finite) r = scan_finite(d, P, ws, st);
  if (r == LT_OK) {
    Timing tm;
    tm.on = o && o->stats;
    tm.st = st;
    double rev_flops = 0;
    if (precision == LT_FP64) r = run_bwd<double>(d, P, L, o, gbar, grad, ws, st, tm, &rev_flops);
    else r = run_bwd<float>(d, P, L, o, gbar, grad, ws, st, tm, &rev_flops);
    if (r == LT_OK && tm.on) {
      HIPCHK(hipStreamSynchronize(st));
      ltriples_stats* S = o->stats;
      *S = ltriples_stats{};
      S->total_ms = Timing::ms(tm.start, tm.end);
      S->setup_ms = Timing::ms(tm.start, tm.setup_end);
      for (auto& x : tm.gemm) S->triples_gemm_ms += Timing::ms(x.first, x.second);
      for (auto& x : tm.epi) S->epilogue_ms += Timing::ms(x.first, x.second);
      S->triples_gemm_launches = (int64_t)tm.gemm.size();
      S->triples_gemm_flops = tm.gemm_flops + rev_flops;
      double f = 0;
      for (int b = 0; b < 4; ++b) f += (double)P.n_blk[b] * item_flops(D, b);
      S->algorithmic_flops = 3.0 * f;
      S->n_items = L.total;
    }
  }
  return r;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batched domains.  The domains run one after another on the stream and share
// the big part of the workspace (operands, slabs, scratch); each keeps its own
// small buffers.  With options.graph = 1 the whole launch sequence is captured
// into a hipGraph on the first call and replayed on later calls whose shapes,
// pointers and options match (the graph reads the inputs at replay time).
// ---------------------------------------------------------------------------
namespace {

struct BatchPlan {
  std::vector<ItemLists> L;
  std::vector<Plan> P;
  std::vector<size_t> base;                 // start of each domain's big region in the workspace
  std::vector<std::vector<int32_t>> groups; // launch groups, each longest first
  size_t total = 0;
};

int plan_batch(const ltriples_domain* ds, int32_t ndom, int32_t precision, const ltriples_options* o,
               BatchPlan& B) {
  if (ndom < 0) return fail(LT_EINVAL, "ndom < 0");
  if (ndom > 0 && !ds) return fail(LT_EINVAL, "domains is NULL");
  if (o && (o->items || o->n_items || o->e_items))
    return fail(LT_EINVAL, "item lists and per-item outputs are single-domain options");
  {
    const int r = validate_options(o);
    if (r) return r;
  }
  for (int32_t d = 0; d < ndom; ++d) {
    const int r = validate(&ds[d], precision, nullptr);
    if (r) return fail(r, "domain %d: %s", d, g_err.c_str());
  }
  B.L.resize(ndom);
  B.P.resize(ndom);
  std::vector<double> cost(ndom, 0.0);
  for (int32_t d = 0; d < ndom; ++d) {
    build_items(dims_of(&ds[d]), nullptr, B.L[d]);
    plan_domain(&ds[d], precision, o, B.L[d], B.P[d]);
    const int r = check_plan(B.P[d]);
    if (r) return r;
    for (int b = 0; b < 4; ++b) cost[d] += (double)B.P[d].n_blk[b] * item_flops(B.P[d].D, b);
  }
  // Launch groups.  Without a group budget every domain runs alone and all
  // share one big region.  With one, the domains in descending order of
  // their triples flops (longest processing time first; ties by index) are
  // packed greedily into groups of consecutive domains, at most
  // kMaxChunk16, whose big regions together stay within the budget (a
  // domain larger than the budget forms a group of its own); the domains of
  // a group get big regions of their own, one after another.
  const size_t gbudget = o ? o->group_budget : 0;
  std::vector<int32_t> order(ndom);
  for (int32_t d = 0; d < ndom; ++d) order[d] = d;
  B.groups.clear();
  if (gbudget == 0) {
    for (int32_t d = 0; d < ndom; ++d) B.groups.push_back({d});
  } else {
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return cost[a] > cost[b]; });
    size_t used = 0;
    for (int32_t d : order) {
      const size_t need = align256(B.P[d].big);
      if (B.groups.empty() || B.groups.back().size() >= (size_t)lt::kMaxChunk16 || used + need > gbudget) {
        B.groups.push_back({});
        used = 0;
      }
      B.groups.back().push_back(d);
      used += need;
    }
  }
  B.base.assign(ndom, 0);
  size_t big = 0;
  for (const auto& g : B.groups) {
    size_t off = 0;
    for (int32_t d : g) {
      B.base[d] = off;
      off += align256(B.P[d].big);
    }
    big = std::max(big, off);
  }
  size_t off = align256(big);
  for (int32_t d = 0; d < ndom; ++d) {
    B.P[d].small_base = off - B.base[d];   // relative to the domain's own base
    off = align256(off + B.P[d].small);
  }
  B.total = std::max<size_t>(off, 256);
  return LT_OK;
}

struct GraphEntry {
  std::vector<uint64_t> key;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};
std::mutex g_graph_mu;
std::vector<GraphEntry> g_graphs;
constexpr size_t kMaxGraphs = 16;

std::vector<uint64_t> batch_key(const ltriples_domain* ds, int32_t ndom, int32_t precision,
                                const ltriples_options* o, const void* e_out, const void* parts,
                                const void* ws, size_t ws_bytes, int device) {
  // every option that changes the plan (buffer offsets, batches, chunks) or
  // the recorded launches (forced tiles) is part of the key
  std::vector<uint64_t> k = {(uint64_t)device, (uint64_t)precision, (uint64_t)ndom, (uint64_t)(uintptr_t)e_out,
                             (uint64_t)(uintptr_t)parts, (uint64_t)(uintptr_t)ws, (uint64_t)ws_bytes,
                             (uint64_t)(o ? o->workspace_budget : 0), (uint64_t)(o ? o->batch_items : 0),
                             (uint64_t)(o ? o->build_chunk_mib : 0), (uint64_t)(o ? o->group_budget : 0)};
  for (int t = 0; t < 3; ++t) k.push_back((uint64_t)(o ? o->tile_override[t] : 0));
  for (int32_t d = 0; d < ndom; ++d) {
    const ltriples_domain& x = ds[d];
    k.insert(k.end(), {(uint64_t)x.noa, (uint64_t)x.nob, (uint64_t)x.nva, (uint64_t)x.nvb, (uint64_t)x.naux});
    const void* ptrs[] = {x.t1a, x.t1b, x.t2aa, x.t2bb, x.t2ab, x.Boo_a, x.Bov_a, x.Bvv_a, x.Boo_b,
                          x.Bov_b, x.Bvv_b, x.eo_a, x.ev_a, x.eo_b, x.ev_b, x.fov_a, x.fov_b};
    for (const void* p : ptrs) k.push_back((uint64_t)(uintptr_t)p);
  }
  return k;
}

int enqueue_batch(const ltriples_domain* ds, int32_t ndom, int32_t precision, const ltriples_options* o,
                  const BatchPlan& B, double* e_out, double* parts, void* ws, hipStream_t st) {
  // every run-time option of the call (autotuning, forced tiles, budgets);
  // item lists, per-item outputs and stats are single-domain options
  ltriples_options oo = o ? *o : ltriples_options{};
  oo.items = nullptr; oo.n_items = 0; oo.e_items = nullptr; oo.stats = nullptr;
  (void)ndom;
  for (const auto& grp : B.groups) {
    std::vector<GroupDom> G;
    for (int32_t d : grp)
      G.push_back({&ds[d], &B.P[d], &B.L[d], e_out + d, parts ? parts + 12 * d : nullptr, (char*)ws + B.base[d]});
    Timing tm;  // off
    const int r = precision == LT_FP64 ? run_group<double>(G.data(), (int)G.size(), &oo, st, tm)
                                       : run_group<float>(G.data(), (int)G.size(), &oo, st, tm);
    if (r) return r;
  }
  return LT_OK;
}

}  // namespace

extern "C" {

int ltriples_workspace_size_batched(const ltriples_domain* ds, int32_t ndom, int32_t precision,
                                    const ltriples_options* o, size_t* bytes) {
  g_err.clear();
  if (!bytes) return fail(LT_EINVAL, "bytes is NULL");
  BatchPlan B;
  const int r = plan_batch(ds, ndom, precision, o, B);
  if (r) return r;
  *bytes = B.total;
  return LT_OK;
}

int ltriples_energy_batched(const ltriples_domain* ds, int32_t ndom, int32_t precision, const ltriples_options* o,
                            double* e_out, double* parts, void* ws, size_t ws_bytes, void* stream) {
  g_err.clear();
  if (!e_out && ndom > 0) return fail(LT_EINVAL, "e_out is NULL");
  BatchPlan B;
  int r = plan_batch(ds, ndom, precision, o, B);
  if (r) return r;
  if (ndom == 0) return LT_OK;
  hipStream_t st = (hipStream_t)stream;
  for (int32_t d = 0; d < ndom; ++d) {
    r = check_denominators(&ds[d], st);
    if (r) return fail(r, "domain %d: %s", d, g_err.c_str());
  }
  const bool use_graph = o && o->graph && ws != nullptr;
  OwnedWs own;
  r = get_ws(ws, ws_bytes, B.total, st, own);
  if (r) return r;
  // item tables go to each domain's small region on every call (also before a
  // replay: the caller may have used the workspace for other calls meanwhile)
  for (int32_t d = 0; d < ndom; ++d) {
    void* wsd = (char*)ws + B.base[d];
    r = upload_items(B.P[d], B.L[d], wsd, st);
    if (r) return r;
    if (o && o->check_finite) {
      r = scan_finite(&ds[d], B.P[d], wsd, st);
      if (r) return fail(r, "domain %d: %s", d, g_err.c_str());
    }
  }
  int device = 0;
  HIPCHK(hipGetDevice(&device));
  std::vector<uint64_t> key;
  if (use_graph) {
    key = batch_key(ds, ndom, precision, o, e_out, parts, ws, ws_bytes, device);
    std::lock_guard<std::mutex> lk(g_graph_mu);
    for (auto& g : g_graphs)
      if (g.key == key) {
        HIPCHK(hipGraphLaunch(g.exec, st));
        return LT_OK;
      }
  }
  if (!use_graph) return enqueue_batch(ds, ndom, precision, o, B, e_out, parts, ws, st);
  // capture on a private stream (the caller's may be the legacy default stream)
  hipStream_t cs = nullptr;
  HIPCHK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  hipGraph_t graph = nullptr;
  hipError_t ce = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (ce != hipSuccess) {
    (void)hipStreamDestroy(cs);
    return fail(LT_EHIP, "hipStreamBeginCapture: %s", hipGetErrorString(ce));
  }
  r = enqueue_batch(ds, ndom, precision, o, B, e_out, parts, ws, cs);
  ce = hipStreamEndCapture(cs, &graph);
  (void)hipStreamDestroy(cs);
  if (r) {
    if (graph) (void)hipGraphDestroy(graph);
    return r;
  }
  if (ce != hipSuccess) return fail(LT_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(ce));
  hipGraphExec_t exec = nullptr;
  ce = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (ce != hipSuccess) {
    (void)hipGraphDestroy(graph);
    return fail(LT_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(ce));
  }
  HIPCHK(hipGraphLaunch(exec, st));
  std::lock_guard<std::mutex> lk(g_graph_mu);
  if (g_graphs.size() >= kMaxGraphs) {
    (void)hipGraphExecDestroy(g_graphs.front().exec);
    (void)hipGraphDestroy(g_graphs.front().graph);
    g_graphs.erase(g_graphs.begin());
  }
  g_graphs.push_back({key, graph, exec});
  return LT_OK;
}

int ltriples_graph_reset(void) {
  g_err.clear();
  std::lock_guard<std::mutex> lk(g_graph_mu);
  for (auto& g : g_graphs) {
    (void)hipGraphExecDestroy(g.exec);
    (void)hipGraphDestroy(g.graph);
  }
  g_graphs.clear();
  return LT_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Central-orbital share (eq. local_pt with the quadrature of eq.
// laplace_transform).  For each point q the central orbital, scaled by its
// half of the point's exp(D s) factor, c~_q[i] = c[i] exp(s_q e_i / 2), is
// appended to the occupied orbitals of its spin: every input with an
// occupied index of that spin gets the rows sum_i c~_q[i] X[i] (both indices
// of Boo and of the same-spin amplitudes), with orbital energy 0.  The items
// are the triplets of that extended domain holding one appended orbital; the
// contractions sum only over the LIS orbitals (the appended ones are never an
// internal index), and the epilogue weighs each element by
// -(w_q / 3) exp(s_q D'), D' the denominator without the central energy.
// ---------------------------------------------------------------------------
namespace {

struct CentralSetup {
  ltriples_domain d{};     // the extended domain (head buffers or the caller's arrays)
  int spin = 0, nq = 0;
  int64_t o = 0;           // LIS occupied orbitals of the central spin
  ltriples_options opt{};
  std::vector<int32_t> items;
  std::vector<double> lap; // [nq][2]: (s_q, -w_q / 3)
  // head of the workspace: Laplace table, coefficients, extended inputs, scratch
  size_t o_lap = 0, o_coef = 0, o_t1 = 0, o_fov = 0, o_eo = 0, o_Boo = 0, o_Bov = 0, o_t2 = 0, o_t2ab = 0,
         o_tmp = 0, head = 0;
};

int central_setup(const ltriples_domain* d, const ltriples_central* c, int32_t precision,
                  const ltriples_options* o, CentralSetup& S) {
  int r = validate(d, precision, o);
  if (r) return r;
  if (!c) return fail(LT_EINVAL, "central is NULL");
  if (c->spin != 0 && c->spin != 1) return fail(LT_EINVAL, "central spin %d (0 alpha, 1 beta)", c->spin);
  if (c->nq < 1 || c->nq > 64) return fail(LT_EINVAL, "nq = %d outside 1..64", c->nq);
  if (!c->s || !c->w) return fail(LT_EINVAL, "quadrature points or weights are NULL");
  for (int q = 0; q < c->nq; ++q)
    if (!(std::isfinite(c->s[q]) && c->s[q] > 0.0 && std::isfinite(c->w[q])))
      return fail(LT_EINVAL, "quadrature point %d: need a finite t > 0 and a finite weight", q);
  if (o && (o->items || o->n_items || o->e_items || o->graph))
    return fail(LT_EINVAL, "item lists, per-item outputs and graphs are not central-share options");
  const Dims D0 = dims_of(d);
  S.spin = c->spin;
  S.nq = c->nq;
  S.o = D0.o[S.spin];
  if (S.o < 1) return fail(LT_ESHAPE, "no occupied orbital of the central spin");
  if (!c->c) return fail(LT_EINVAL, "central orbital coefficients are NULL");
  if (S.o + S.nq > 4096) return fail(LT_ESHAPE, "too many occupied orbitals with the quadrature points");
  const int sp = S.spin, tp = 1 - sp;
  const int64_t no = S.o, oe = no + S.nq, ot = D0.o[tp], v = D0.v[sp], vt = D0.v[tp], Q = D0.Q;
  // head layout (FP64)
  size_t off = 0;
  auto take = [&](int64_t n) { const size_t x = off; off = align256(off + 8 * (size_t)std::max<int64_t>(n, 1)); return x; };
  S.o_lap = take(2 * S.nq);
  S.o_coef = take(S.nq * no);
  S.o_t1 = take(oe * v);
  S.o_fov = take(oe * v);
  S.o_eo = take(oe);
  S.o_Boo = take(Q * oe * oe);
  S.o_Bov = take(Q * oe * v);
  S.o_t2 = take(oe * oe * v * v);
  S.o_t2ab = take(oe * ot * v * vt);
  S.o_tmp = take(std::max(oe * no * v * v, Q * oe * no));   // first pass of the two-index extensions
  S.head = off;
  S.lap.resize(2 * (size_t)S.nq);
  for (int q = 0; q < S.nq; ++q) {
    S.lap[2 * q] = c->s[q];
    S.lap[2 * q + 1] = -c->w[q] / 3.0;   // 1/D -> -sum_q w_q exp(s_q D); one third per eq. local_pt
  }
  // the extended domain (placeholder addresses below the head until the workspace is known)
  ltriples_domain& x = S.d;
  x = *d;
  int32_t* nocc[2] = {&x.noa, &x.nob};
  *nocc[sp] = (int32_t)oe;
  // items with exactly one appended orbital, ordered by block
  const int32_t oo = (int32_t)no, ott = (int32_t)ot;
  const int b_same = sp == 0 ? 0 : 3, b_pair = sp == 0 ? 1 : 2, b_odd = sp == 0 ? 2 : 1;
  for (int32_t q = 0; q < S.nq; ++q) {
    const int32_t cq = oo + q;
    for (int32_t j = 0; j < oo; ++j)
      for (int32_t k = j + 1; k < oo; ++k) S.items.insert(S.items.end(), {b_same, j, k, cq});
    for (int32_t i = 0; i < oo; ++i)
      for (int32_t K = 0; K < ott; ++K) S.items.insert(S.items.end(), {b_pair, i, cq, K});
    for (int32_t I = 0; I < ott; ++I)
      for (int32_t J = I + 1; J < ott; ++J) S.items.insert(S.items.end(), {b_odd, I, J, cq});
  }
  if (S.items.size() / 4 > (size_t)INT32_MAX) return fail(LT_ESHAPE, "too many items");
  if (o) S.opt = *o;
  S.opt.items = S.items.empty() ? nullptr : S.items.data();
  S.opt.n_items = (int32_t)(S.items.size() / 4);
  return LT_OK;
}

// Points the extended domain at the head buffers (and the caller's arrays of
// the other spin and of Bvv).
void central_bind(CentralSetup& S, const ltriples_domain* d, char* head) {
  ltriples_domain& x = S.d;
  x = *d;
  const int sp = S.spin;
  const int32_t oe = (int32_t)(S.o + S.nq);
  auto P = [&](size_t off) { return (const double*)(head + off); };
  if (sp == 0) {
    x.noa = oe;
    x.t1a = P(S.o_t1); x.fov_a = P(S.o_fov); x.eo_a = P(S.o_eo);
    x.Boo_a = P(S.o_Boo); x.Bov_a = P(S.o_Bov); x.t2aa = P(S.o_t2);
  } else {
    x.nob = oe;
    x.t1b = P(S.o_t1); x.fov_b = P(S.o_fov); x.eo_b = P(S.o_eo);
    x.Boo_b = P(S.o_Boo); x.Bov_b = P(S.o_Bov); x.t2bb = P(S.o_t2);
  }
  x.t2ab = P(S.o_t2ab);
}

// Enqueues the extended inputs into the head (kernels and one table copy).
int central_inputs(const CentralSetup& S, const ltriples_domain* d, const ltriples_central* c, char* head,
                   hipStream_t st) {
  const Dims D0 = dims_of(d);
  const int sp = S.spin, tp = 1 - sp;
  const int64_t o = S.o, oe = o + S.nq, ot = D0.o[tp], v = D0.v[sp], vt = D0.v[tp], Q = D0.Q;
  const int32_t oi = (int32_t)o, nq = S.nq;
  auto W = [&](size_t off) { return (double*)(head + off); };
  const double* t1 = sp ? d->t1b : d->t1a;
  const double* fov = sp ? d->fov_b : d->fov_a;
  const double* eo = sp ? d->eo_b : d->eo_a;
  const double* Boo = sp ? d->Boo_b : d->Boo_a;
  const double* Bov = sp ? d->Bov_b : d->Bov_a;
  const double* t2 = sp ? d->t2bb : d->t2aa;
  HIPCHK(hipMemcpyAsync(W(S.o_lap), S.lap.data(), 8 * S.lap.size(), hipMemcpyHostToDevice, st));
  HIPCHK(lt::launch_central_coef(W(S.o_coef), c->c, eo, W(S.o_lap), oi, nq, st));
  const double* coef = W(S.o_coef);
  HIPCHK(lt::launch_aug_axis(W(S.o_t1), t1, coef, 1, oi, nq, v, st));
  HIPCHK(lt::launch_aug_axis(W(S.o_fov), fov, coef, 1, oi, nq, v, st));
  // orbital energies: the LIS ones, then zeros (the central factor sits in the coefficients)
  HIPCHK(lt::launch_zero(W(S.o_eo), oe, st));
  HIPCHK(lt::launch_copy4d<double, double>(W(S.o_eo), 0, 0, 0, 1, 1, 1, o, eo, 0, 0, 0, 1, nullptr, 0, 0, 0, 0, st));
  // factors: Bov along its occupied index, Boo along both
  HIPCHK(lt::launch_aug_axis(W(S.o_Bov), Bov, coef, Q, oi, nq, v, st));
  HIPCHK(lt::launch_aug_axis(W(S.o_tmp), Boo, coef, Q, oi, nq, o, st));
  HIPCHK(lt::launch_aug_axis(W(S.o_Boo), W(S.o_tmp), coef, Q * oe, oi, nq, 1, st));
  // same-spin amplitudes along both occupied indices (the appended pair block,
  // never read, is not zero by construction but is antisymmetric like the rest)
  HIPCHK(lt::launch_aug_axis(W(S.o_tmp), t2, coef, 1, oi, nq, o * v * v, st));
  HIPCHK(lt::launch_aug_axis(W(S.o_t2), W(S.o_tmp), coef, oe, oi, nq, v * v, st));
  // mixed amplitudes along the central spin's occupied index: t2ab [oa][ob][va][vb]
  if (sp == 0) HIPCHK(lt::launch_aug_axis(W(S.o_t2ab), d->t2ab, coef, 1, oi, nq, ot * v * vt, st));
  else HIPCHK(lt::launch_aug_axis(W(S.o_t2ab), d->t2ab, coef, ot, oi, nq, vt * v, st));
  return LT_OK;
}

// Plan of the extended domain, with the LIS orbitals as the summed ones.
void central_plan(const CentralSetup& S, int32_t precision, ItemLists& L, Plan& P) {
  const Dims D = dims_of(&S.d);
  build_items(D, &S.opt, L);
  int64_t oi[2] = {D.o[0], D.o[1]};
  oi[S.spin] = S.o;
  plan_domain(&S.d, precision, &S.opt, L, P, false, oi);
}

}  // namespace

extern "C" {

int ltriples_central_workspace_size(const ltriples_domain* d, const ltriples_central* c, int32_t precision,
                                    const ltriples_options* o, size_t* bytes) {
  g_err.clear();
  if (!bytes) return fail(LT_EINVAL, "bytes is NULL");
  CentralSetup S;
  int r = central_setup(d, c, precision, o, S);
  if (r) return r;
  central_bind(S, d, kFakeBase);
  ItemLists L;
  Plan P;
  central_plan(S, precision, L, P);
  *bytes = S.head + P.total;
  return LT_OK;
}

int ltriples_energy_central(const ltriples_domain* d, const ltriples_central* c, int32_t precision,
                            const ltriples_options* o, double* e_out, double* parts, void* ws, size_t ws_bytes,
                            void* stream) {
  g_err.clear();
  CentralSetup S;
  int r = central_setup(d, c, precision, o, S);
  if (r) return r;
  if (!e_out) return fail(LT_EINVAL, "e_out is NULL");
  hipStream_t st = (hipStream_t)stream;
  central_bind(S, d, kFakeBase);
  ItemLists L;
  Plan P;
  central_plan(S, precision, L, P);
  r = check_plan(P);
  if (r) return r;
  const size_t need = S.head + P.total;
  r = check_denominators(d, st);
  if (r) return r;
  OwnedWs own;
  r = get_ws(ws, ws_bytes, need, st, own);
  if (r) return r;
  char* head = (char*)ws;
  void* inner = head + S.head;
  central_bind(S, d, head);
  log_plan(P);
  r = upload_items(P, L, inner, st);
  if (r) return r;
  if (S.opt.check_finite) {
    r = scan_finite(d, P, inner, st);
    if (r) return r;
    const double* cc = c->c;
    lt::FiniteScan a{};
    a.p[0] = cc; a.n[0] = S.o; a.narr = 1;
    int32_t* flag = at_small<int32_t>(inner, P, P.flag);
    HIPCHK(lt::launch_zero32(flag, 1, st));
    HIPCHK(lt::launch_scan_finite(a, flag, st));
    int32_t h = 0;
    HIPCHK(hipMemcpyAsync(&h, flag, 4, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (h) return fail(LT_ENONFINITE, "NaN or infinity in the central orbital (options.check_finite)");
  }
  r = central_inputs(S, d, c, head, st);
  if (r) return r;
  P.lap = (const double*)(head + S.o_lap);
  P.lap_spin = S.spin;
  Timing tm;
  tm.on = S.opt.stats != nullptr;
  tm.st = st;
  if (precision == LT_FP64) r = run<double>(&S.d, P, L, &S.opt, e_out, parts, inner, st, tm);
  else r = run<float>(&S.d, P, L, &S.opt, e_out, parts, inner, st, tm);
  if (r == LT_OK && tm.on) {
    HIPCHK(hipStreamSynchronize(st));
    ltriples_stats* St = S.opt.stats;
    *St = ltriples_stats{};
    St->total_ms = Timing::ms(tm.start, tm.end);
    St->setup_ms = Timing::ms(tm.start, tm.setup_end);
    for (auto& x : tm.gemm) St->triples_gemm_ms += Timing::ms(x.first, x.second);
    for (auto& x : tm.epi) St->epilogue_ms += Timing::ms(x.first, x.second);
    St->triples_gemm_launches = (int64_t)tm.gemm.size();
    St->triples_gemm_flops = tm.gemm_flops;
    double f = 0;
    for (int b = 0; b < 4; ++b) f += (double)P.n_blk[b] * item_flops(P.D, b);
    St->algorithmic_flops = f;
    St->n_items = L.total;
  }
  return r;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Closed-shell domains: the spin-block path with identical alpha and beta
// data, restricted to the aaa and aab blocks (the bbb and abb blocks equal
// them), E = 2 (E_aaa + E_aab).  The same-spin amplitudes are formed in the
// head of the workspace; the spin-block call gets the rest.
// ---------------------------------------------------------------------------
namespace {

struct RhfSetup {
  ltriples_domain d{};
  ltriples_options o{};
  std::vector<int32_t> items;
  size_t t2_bytes = 0, head = 0;
};

int rhf_setup(const ltriples_rhf_domain* r, const ltriples_options* o, RhfSetup& S) {
  if (!r) return fail(LT_EINVAL, "domain is NULL");
  if (r->no < 0 || r->nv < 0 || r->naux < 0) return fail(LT_EINVAL, "negative dimension");
  if (o && (o->items || o->n_items || o->e_items || o->graph))
    return fail(LT_EINVAL, "item lists, per-item outputs and graphs are not closed-shell options");
  const int64_t no = r->no, nv = r->nv, Q = r->naux;
  // the open-shell limits, before any product of dimensions is formed
  if (nv > 46340 || no > 4096 || Q > (int64_t(1) << 24)) return fail(LT_ESHAPE, "dimension too large");
  const struct { const double* p; int64_t n; const char* name; } ps[] = {
      {r->t1, no * nv, "t1"}, {r->tau, no * no * nv * nv, "tau"}, {r->Boo, Q * no * no, "Boo"},
      {r->Bov, Q * no * nv, "Bov"}, {r->Bvv, Q * nv * nv, "Bvv"}, {r->eo, no, "eo"}, {r->ev, nv, "ev"},
      {r->fov, no * nv, "fov"}};
  for (auto& x : ps)
    if (x.n > 0 && !x.p) return fail(LT_EINVAL, "%s is NULL", x.name);
  const int64_t n0 = no * (no - 1) * (no - 2) / 6, n1 = no * (no - 1) / 2 * no;
  if (n0 + n1 > (int64_t)INT32_MAX) return fail(LT_ESHAPE, "too many occupied triplets");
  ltriples_domain& d = S.d;
  d.noa = d.nob = r->no; d.nva = d.nvb = r->nv; d.naux = r->naux;
  d.t1a = d.t1b = r->t1;
  d.t2ab = r->tau;
  d.t2aa = d.t2bb = r->tau;   // placeholder for validation and planning; the workspace copy at run time
  d.Boo_a = d.Boo_b = r->Boo; d.Bov_a = d.Bov_b = r->Bov; d.Bvv_a = d.Bvv_b = r->Bvv;
  d.eo_a = d.eo_b = r->eo; d.ev_a = d.ev_b = r->ev;
  d.fov_a = d.fov_b = r->fov;
  S.items.reserve(4 * (size_t)(n0 + n1));
  for (int32_t i = 0; i < r->no; ++i)
    for (int32_t j = i + 1; j < r->no; ++j)
      for (int32_t k = j + 1; k < r->no; ++k) S.items.insert(S.items.end(), {0, i, j, k});
  for (int32_t i = 0; i < r->no; ++i)
    for (int32_t j = i + 1; j < r->no; ++j)
      for (int32_t K = 0; K < r->no; ++K) S.items.insert(S.items.end(), {1, i, j, K});
  if (o) S.o = *o;
  S.o.items = S.items.empty() ? nullptr : S.items.data();
  S.o.n_items = (int32_t)(S.items.size() / 4);
  S.t2_bytes = align256(8 * (size_t)(no * no * nv * nv));
  S.head = S.t2_bytes + 256;   // then 13 doubles: E and the four blocks' parts
  return LT_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Closed-shell domains, spin-adapted (the default of ltriples_energy_rhf).
// Over spatial orbitals with tau^{ab}_{ij} = tau^{ba}_{ji}, W^{abc}_{ijk} is
// the sum over the six joint permutations of (ia), (jb), (kc) of
//   sum_e tau^{ae}_{ij}(ck|be) - sum_m tau^{ab}_{im}(ck|mj).
// Grouped by the virtual index that the tau (or integral) factor carries,
// the twelve terms form one contraction per occupied triple (p,q,r):
//   F(p,q,r)[x][y*v+z] = sum_e tau^{xe}_{pq}(rz|ye) + sum_e tau^{xe}_{pr}(qy|ze)
//                      - sum_m (px|mr) tau^{yz}_{qm} - sum_m (px|mq) tau^{yz}_{mr},
// and W^{abc}_{ijk} = F(i,j,k)[a][bc] + F(j,i,k)[b][ac] + F(k,i,j)[c][ab].
// Each unordered occupied triple i <= j <= k (all equal excluded: its
// contribution vanishes) costs three contractions of v x v^2 outputs over
// 2(v + o) rows, written as three cubes; the epilogue (lt_epilogue.hip)
// forms W from them and sums the energy of all orderings of the triple over
// unique virtual tiles.
// ---------------------------------------------------------------------------
namespace {

enum { SA_T2T, SA_GCS, SA_TF, SA_TS, SA_RVC, SA_RVS, SA_NOP };

struct SaPlan {
  int prec = 0, bf = 0;
  size_t ts = 8;
  int64_t o = 0, v = 0, Q = 0, ldv = 0, ldvv = 0, ldov = 0, ldoo = 0;
  int64_t n_items = 0, nb = 0, nt = 0, ntiles = 0, cRV = 1;
  size_t cube = 0;                              // elements per contraction output cube
  Buf BvvP, BovR, BovP64, BooP64, OV64, op[SA_NOP], stage, O8h[SA_NOP], O8l[SA_NOP];
  Buf scratch;                                  // builds: (ov|oo); batches: cubes, then partials
  size_t part_off = 0;
  Buf items, fitems, dst, e_items, fc, parts, flag, segtab;
  size_t total = 0;
};

int64_t sa_items(int64_t o) { return o <= 1 ? 0 : o * (o + 1) * (o + 2) / 6 - o; }

void sa_plan(const ltriples_rhf_domain* r, int32_t prec, const ltriples_options* o, SaPlan& P) {
  P.prec = prec;
  P.ts = prec == LT_FP64 ? 8 : 4;
  P.bf = prec == LT_BF16X3 ? 3 : (prec == LT_BF16 ? 1 : 0);
  P.o = r->no; P.v = r->nv; P.Q = r->naux;
  const int64_t no = P.o, v = P.v, Q = P.Q;
  const size_t ts = P.ts;
  P.ldv = ld4(v); P.ldvv = ld4(v * v); P.ldov = ld4(no * v); P.ldoo = ld4(no * no);
  P.n_items = sa_items(no);
  P.nt = cdiv(v, lt::ET);
  P.ntiles = P.nt * (P.nt + 1) / 2;
  P.cube = (size_t)((v * v * v + 63) & ~int64_t(63));
  const size_t cap = (size_t)((o && o->build_chunk_mib > 0) ? o->build_chunk_mib : 2048) << 20;
  P.cRV = std::max<int64_t>(1, std::min<int64_t>(no, (int64_t)(cap / std::max<size_t>(ts * v * P.ldvv, 1))));
  size_t off = 0;
  auto take = [&](Buf& b, size_t bytes) { b.off = off; b.bytes = bytes; off = align256(off + bytes); };
  take(P.BvvP, ts * Q * P.ldvv);
  take(P.BovR, ts * no * Q * P.ldv);
  take(P.BovP64, 8 * Q * P.ldov);
  take(P.BooP64, 8 * Q * P.ldoo);
  take(P.OV64, 8 * no * v * no * v);
  // operand tensors (BF16 modes: built one by one in the staging buffer and split)
  const size_t opb[SA_NOP] = {ts * no * no * v * P.ldv, ts * no * no * no * P.ldv, ts * no * no * P.ldvv,
                              ts * no * no * P.ldvv, ts * no * v * P.ldvv, ts * no * v * P.ldvv};
  if (!P.bf) {
    for (int t = 0; t < SA_NOP; ++t) take(P.op[t], opb[t]);
  } else {
    size_t mx = ts * P.cRV * v * P.ldvv;
    for (int t = 0; t < SA_RVC; ++t) mx = std::max(mx, opb[t]);
    take(P.stage, mx);
    for (int t = 0; t < SA_NOP; ++t) { P.op[t].off = P.stage.off; P.op[t].bytes = opb[t]; }
    auto k16 = [](int64_t k) { return (k + 15) & ~int64_t(15); };
    const int64_t nblk[SA_NOP] = {no * no, no * no, no, no, no, no};
    const int64_t K[SA_NOP] = {v, no, no, no, v, v};
    const int64_t ld[SA_NOP] = {P.ldv, P.ldv, P.ldvv, P.ldvv, P.ldvv, P.ldvv};
    for (int t = 0; t < SA_NOP; ++t) {
      const size_t bytes = 2 * (size_t)(nblk[t] * k16(K[t]) * ld[t]) + 2 * 8 * 512;
      take(P.O8h[t], bytes);
      take(P.O8l[t], bytes);
    }
  }
  // batches: three cubes per item, then the per-tile partials.  Default
  // budget 16 GiB (52 triples per batch on the (40, 300, 1200) domain): on
  // that domain the step took 7.54 s with 8 GiB, 7.15 s with 16 and 7.13 s
  // with 32 (the epilogue fills the chip better with more triples per launch).
  const size_t budget = (o && o->workspace_budget) ? o->workspace_budget : (size_t(16) << 30);
  const size_t per = 3 * P.cube * ts + align256(24 * (size_t)std::max<int64_t>(P.ntiles, 1));
  int64_t nb = (o && o->batch_items > 0) ? o->batch_items : (int64_t)std::max<size_t>(1, budget / per);
  nb = std::min<int64_t>(nb, std::max<int64_t>(P.n_items, 1));
  nb = std::min<int64_t>(nb, 21845);   // three contraction items each
  P.nb = nb;
  P.part_off = align256(3 * P.cube * ts * (size_t)nb);
  const size_t s2 = P.part_off + 24 * (size_t)nb * (size_t)std::max<int64_t>(P.ntiles, 1);
  const size_t s1 = 8 * (size_t)(no * v * no * no);
  take(P.scratch, std::max<size_t>(std::max(s1, s2), 256));
  const size_t n = (size_t)std::max<int64_t>(P.n_items, 1);
  take(P.items, 12 * n);
  take(P.fitems, 36 * n);
  take(P.dst, 4 * n);
  take(P.e_items, 24 * n);
  take(P.fc, 64);
  take(P.parts, 16 * 8);
  take(P.flag, 256);
  if (P.bf) take(P.segtab, sizeof(lt::Seg8) * 6 * 3 * (size_t)nb);
  P.total = off;
}

template <typename T>
int sa_prep(const ltriples_rhf_domain* r, const SaPlan& P, void* ws, hipStream_t st) {
  const int64_t no = P.o, v = P.v, Q = P.Q, ldv = P.ldv, ldvv = P.ldvv;
  char* scr = (char*)ws + P.scratch.off;
  auto split = [&](int t, int64_t b0, int64_t nblk, int64_t K, int64_t ld, int64_t ncol, int64_t ibs,
                   int64_t iks) -> hipError_t {
    if (!P.bf) return hipSuccess;
    const int64_t blk = ((K + 15) / 16) * 16 * ld;
    return lt::launch_split8(at<lt::bf16_t>(ws, P.O8h[t]) + b0 * blk, at<lt::bf16_t>(ws, P.O8l[t]) + b0 * blk, nblk,
                             (int32_t)K, ld, (int32_t)ncol, at<float>(ws, P.stage), ibs, iks, st);
  };
  // DF factor layouts
  HIPCHK(lt::launch_copy4d<double, T>(at<T>(ws, P.BvvP), 0, 0, ldvv, 1, 1, Q, v * v, r->Bvv, 0, 0, v * v, 1,
                                      nullptr, 0, 0, 0, 0, st));
  HIPCHK(lt::launch_copy4d<double, T>(at<T>(ws, P.BovR), 0, Q * ldv, ldv, 1, no, Q, v, r->Bov, 0, v, no * v, 1,
                                      nullptr, 0, 0, 0, 0, st));
  HIPCHK(lt::launch_copy4d<double, double>(at<double>(ws, P.BovP64), 0, 0, P.ldov, 1, 1, Q, no * v, r->Bov, 0, 0,
                                           no * v, 1, nullptr, 0, 0, 0, 0, st));
  HIPCHK(lt::launch_copy4d<double, double>(at<double>(ws, P.BooP64), 0, 0, P.ldoo, 1, 1, Q, no * no, r->Boo, 0, 0,
                                           no * no, 1, nullptr, 0, 0, 0, 0, st));
  auto gemm64 = [&](int64_t M, int64_t N, const double* Lp, int64_t lks, const double* Rp, int64_t rks,
                    double* out, int64_t ldo) -> hipError_t {
    lt::GemmArgs<double> g{};
    g.M = (int32_t)M; g.N = (int32_t)N; g.nbatch = 1; g.mode = 0;
    g.out = out; g.s_mr = ldo; g.s_nr = 1;
    g.L = Lp; g.lks = lks; g.R = Rp; g.rks = rks; g.K = (int32_t)Q;
    return lt::launch_gemm<double>(g, st);
  };
  auto gemmT = [&](int64_t M, int64_t N, int64_t nbatch, const T* Lp, int64_t lks, int64_t lbs, const T* Rp,
                   int64_t rks, int64_t rbs, T* out, int64_t obs, int64_t s_mq, int64_t s_mr, int32_t mdiv,
                   int64_t s_nq, int64_t s_nr, int32_t ndiv) -> hipError_t {
    lt::GemmArgs<T> g{};
    g.M = (int32_t)M; g.N = (int32_t)N; g.nbatch = (int32_t)nbatch; g.mode = 0;
    g.out = out; g.obs = obs; g.s_mq = s_mq; g.s_mr = s_mr; g.mdiv = mdiv; g.s_nq = s_nq; g.s_nr = s_nr; g.ndiv = ndiv;
    g.L = Lp; g.lks = lks; g.lbs = lbs; g.R = Rp; g.rks = rks; g.rbs = rbs; g.K = (int32_t)Q;
    return lt::launch_gemm<T>(g, st);
  };
  // (ia|jb) as [o][v][o][v] for the epilogue; (ka|mj) as [k][a][m][j] for Gcs
  HIPCHK(gemm64(no * v, no * v, at<double>(ws, P.BovP64), P.ldov, at<double>(ws, P.BovP64), P.ldov,
                at<double>(ws, P.OV64), no * v));
  double* OO = (double*)scr;
  HIPCHK(gemm64(no * v, no * no, at<double>(ws, P.BovP64), P.ldov, at<double>(ws, P.BooP64), P.ldoo, OO, no * no));
  // Gcs[x][y][m][a] = (ya|mx) = OO[y][a][m][x]
  HIPCHK(lt::launch_copy4d<double, T>(at<T>(ws, P.op[SA_GCS]), no * no * ldv, no * ldv, ldv, no, no, no, v, OO, 1,
                                      v * no * no, no, no * no, nullptr, 0, 0, 0, 0, st));
  HIPCHK(split(SA_GCS, 0, no * no, no, ldv, v, no * ldv, ldv));
  // T2T[i][j][e][a] = tau[i][j][a][e]
  HIPCHK(lt::launch_copy4d<double, T>(at<T>(ws, P.op[SA_T2T]), no * v * ldv, v * ldv, ldv, no, no, v, v, r->tau,
                                      no * v * v, v * v, 1, v, nullptr, 0, 0, 0, 0, st));
  HIPCHK(split(SA_T2T, 0, no * no, v, ldv, v, v * ldv, ldv));
  // Tf[x][m][b*v+c] = tau[x][m][b][c];  Ts[x][m][b*v+c] = tau[m][x][b][c]
  HIPCHK(lt::launch_copy4d<double, T>(at<T>(ws, P.op[SA_TF]), no * ldvv, ldvv, v, no, no, v, v, r->tau, no * v * v,
                                      v * v, v, 1, nullptr, 0, 0, 0, 0, st));
  HIPCHK(split(SA_TF, 0, no, no, ldvv, v * v, no * ldvv, ldvv));
  HIPCHK(lt::launch_copy4d<double, T>(at<T>(ws, P.op[SA_TS]), no * ldvv, ldvv, v, no, no, v, v, r->tau, v * v,
                                      no * v * v, v, 1, nullptr, 0, 0, 0, 0, st));
  HIPCHK(split(SA_TS, 0, no, no, ldvv, v * v, no * ldvv, ldvv));
  // RVc[r][e][b*v+c] = (rc|be): rows (e,b), cols c; chunks of r
  for (int64_t r0 = 0; r0 < no; r0 += P.cRV) {
    const int64_t n = std::min<int64_t>(P.cRV, no - r0);
    T* dst = P.bf ? at<T>(ws, P.stage) : at<T>(ws, P.op[SA_RVC]) + r0 * v * ldvv;
    HIPCHK(gemmT(v * v, v, n, at<T>(ws, P.BvvP), ldvv, 0, at<T>(ws, P.BovR) + r0 * Q * ldv, ldv, Q * ldv, dst,
                 v * ldvv, ldvv, v, (int32_t)v, 0, 1, 0));
    HIPCHK(split(SA_RVC, r0, n, v, ldvv, v * v, v * ldvv, ldvv));
  }
  // RVs[q][e][b*v+c] = (qb|ce): rows b, cols (e,c); chunks of q
  for (int64_t q0 = 0; q0 < no; q0 += P.cRV) {
    const int64_t n = std::min<int64_t>(P.cRV, no - q0);
    T* dst = P.bf ? at<T>(ws, P.stage) : at<T>(ws, P.op[SA_RVS]) + q0 * v * ldvv;
    HIPCHK(gemmT(v, v * v, n, at<T>(ws, P.BovR) + q0 * Q * ldv, ldv, Q * ldv, at<T>(ws, P.BvvP), ldvv, 0, dst,
                 v * ldvv, 0, v, 0, ldvv, 1, (int32_t)v));
    HIPCHK(split(SA_RVS, q0, n, v, ldvv, v * v, v * ldvv, ldvv));
  }
  return LT_OK;
}

template <typename T>
int sa_run(const ltriples_rhf_domain* r, const SaPlan& P, const ltriples_options* o, double* e_out, double* parts,
           void* ws, hipStream_t st, Timing& tm) {
  const int64_t no = P.o, v = P.v;
  int32_t* d_items = at<int32_t>(ws, P.items);
  int32_t* d_fitems = at<int32_t>(ws, P.fitems);
  int32_t* d_dst = at<int32_t>(ws, P.dst);
  int32_t* d_fc = at<int32_t>(ws, P.fc);
  double* e_items = at<double>(ws, P.e_items);
  double* parts16 = at<double>(ws, P.parts);
  tm.start = tm.mark();
  if (P.n_items == 0 || v == 0) {
    HIPCHK(lt::launch_zero(e_out, 1, st));
    if (parts) HIPCHK(lt::launch_zero(parts, 3, st));
    tm.setup_end = tm.mark();
    tm.end = tm.setup_end;
    return LT_OK;
  }
  HIPCHK(lt::launch_zero(e_items, 3 * P.n_items, st));
  {
    const int rr = sa_prep<T>(r, P, ws, st);
    if (rr) return rr;
  }
  tm.setup_end = tm.mark();
  lt::ItemOps<T> ops{};
  ops.kind = 3;
  ops.o_s = ops.o_t = (int32_t)no; ops.v_s = ops.v_t = (int32_t)v; ops.oi_s = ops.oi_t = (int32_t)no;
  ops.ld_vs = ops.ld_vt = P.ldv; ops.ld_vv = P.ldvv;
  ops.T2T = at<T>(ws, P.op[SA_T2T]); ops.Gcs = at<T>(ws, P.op[SA_GCS]); ops.Tf = at<T>(ws, P.op[SA_TF]);
  ops.Ts = at<T>(ws, P.op[SA_TS]); ops.RVc = at<T>(ws, P.op[SA_RVC]); ops.RVs = at<T>(ws, P.op[SA_RVS]);
  lt::ItemOps8 o8{};
  if (P.bf) {
    o8.kind = 3;
    o8.o_s = o8.o_t = (int32_t)no; o8.v_s = o8.v_t = (int32_t)v; o8.oi_s = o8.oi_t = (int32_t)no;
    o8.ld_vs = o8.ld_vt = P.ldv; o8.ld_vv = P.ldvv;
    auto H = [&](int t) { return at<lt::bf16_t>(ws, P.O8h[t]); };
    auto Lo = [&](int t) { return at<lt::bf16_t>(ws, P.O8l[t]); };
    o8.T2Th = H(SA_T2T); o8.T2Tl = Lo(SA_T2T); o8.Gcsh = H(SA_GCS); o8.Gcsl = Lo(SA_GCS);
    o8.Tfh = H(SA_TF); o8.Tfl = Lo(SA_TF); o8.Tsh = H(SA_TS); o8.Tsl = Lo(SA_TS);
    o8.RVch = H(SA_RVC); o8.RVcl = Lo(SA_RVC); o8.RVsh = H(SA_RVS); o8.RVsl = Lo(SA_RVS);
  }
  const int force = o ? o->tile_override[0] - 1 : -1;
  const bool tune = o && o->autotune;
  char* scr = (char*)ws + P.scratch.off;
  T* cubes = (T*)scr;
  double* part = (double*)(scr + P.part_off);
  for (int64_t first = 0; first < P.n_items; first += P.nb) {
    const int64_t n = std::min<int64_t>(P.nb, P.n_items - first);
    const int32_t* fit = d_fitems + 9 * first;
    {
      hipEvent_t ea = tm.mark();
      if (!P.bf) {
        lt::GemmArgs<T> g{};
        g.M = (int32_t)v; g.N = (int32_t)(v * v); g.nbatch = (int32_t)(3 * n); g.mode = 1;
        g.out = cubes; g.obs = (int64_t)P.cube; g.s_mr = v * v; g.s_nr = 1;
        g.ops = ops;
        g.ops.items = fit;
        HIPCHK(lt::launch_gemm<T>(g, st, tune, force));
      } else {
        lt::Seg8* tab = at<lt::Seg8>(ws, P.segtab);
        lt::ItemOps8 t8 = o8;
        t8.items = fit;
        HIPCHK(lt::launch_seg8_table(t8, (int32_t)(3 * n), tab, st));
        lt::GemmArgs16 h{};
        h.M = (int32_t)v; h.N = (int32_t)(v * v); h.nbatch = (int32_t)(3 * n); h.nprod = P.bf;
        h.out = (float*)cubes; h.obs = (int64_t)P.cube; h.ldo = v * v; h.kind = 3; h.tab = tab;
        HIPCHK(lt::launch_gemm_bf16(h, st, tune, force));
      }
      tm.gemm.push_back({ea, tm.mark()});
      tm.gemm_flops += 2.0 * (double)v * (double)(v * v) * (double)(2 * v + 2 * no) * (double)(3 * n);
    }
    hipEvent_t eb = tm.mark();
    lt::EpiRhf<T> e{};
    e.o = (int32_t)no; e.v = (int32_t)v; e.nt = (int32_t)P.nt; e.ntiles = (int32_t)P.ntiles;
    e.W = cubes; e.w_item = 3 * (int64_t)P.cube; e.cube = (int64_t)P.cube; e.items = d_items + 3 * first;
    e.eo = r->eo; e.ev = r->ev; e.t1 = r->t1; e.f = r->fov; e.tau = r->tau; e.ov = at<double>(ws, P.OV64);
    e.part = part;
    HIPCHK(lt::launch_epi_rhf<T>(e, (int32_t)n, st));
    HIPCHK(lt::launch_reduce_items(part, (int32_t)n, (int32_t)P.ntiles, d_dst + first, e_items, st));
    tm.epi.push_back({eb, tm.mark()});
  }
  HIPCHK(lt::launch_reduce_final(e_items, d_dst, d_fc, d_fc + 4, parts16, e_out, st));
  if (parts)
    HIPCHK(lt::launch_copy4d<double, double>(parts, 0, 0, 0, 1, 1, 1, 3, parts16, 0, 0, 0, 1, nullptr, 0, 0, 0, 0, st));
  tm.end = tm.mark();
  return LT_OK;
}

// Host tables of the spin-adapted path: the items (i <= j <= k, not all
// equal), their three contraction triples, identity destinations and the
// single-block counts of the final reduction.
int sa_upload(const SaPlan& P, void* ws, hipStream_t st) {
  std::vector<int32_t> it, fit, dst;
  it.reserve(3 * (size_t)P.n_items);
  fit.reserve(9 * (size_t)P.n_items);
  for (int32_t i = 0; i < P.o; ++i)
    for (int32_t j = i; j < P.o; ++j)
      for (int32_t k = j; k < P.o; ++k) {
        if (i == k) continue;              // i == j == k
        it.insert(it.end(), {i, j, k});
        fit.insert(fit.end(), {i, j, k, j, i, k, k, i, j});
      }
  dst.resize((size_t)P.n_items);
  for (int64_t n = 0; n < P.n_items; ++n) dst[(size_t)n] = (int32_t)n;
  int32_t fc[8] = {0, 0, 0, 0, (int32_t)P.n_items, 0, 0, 0};
  if (P.n_items > 0) {
    HIPCHK(hipMemcpyAsync(at<int32_t>(ws, P.items), it.data(), 4 * it.size(), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(at<int32_t>(ws, P.fitems), fit.data(), 4 * fit.size(), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(at<int32_t>(ws, P.dst), dst.data(), 4 * dst.size(), hipMemcpyHostToDevice, st));
  }
  HIPCHK(hipMemcpyAsync(at<int32_t>(ws, P.fc), fc, sizeof(fc), hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  return LT_OK;
}

int sa_scan_finite(const ltriples_rhf_domain* r, const SaPlan& P, void* ws, hipStream_t st) {
  const int64_t no = r->no, nv = r->nv, Q = r->naux;
  lt::FiniteScan a{};
  const struct { const double* p; int64_t n; } ps[] = {
      {r->t1, no * nv}, {r->tau, no * no * nv * nv}, {r->Boo, Q * no * no}, {r->Bov, Q * no * nv},
      {r->Bvv, Q * nv * nv}, {r->eo, no}, {r->ev, nv}, {r->fov, no * nv}};
  for (const auto& x : ps)
    if (x.n > 0) { a.p[a.narr] = x.p; a.n[a.narr] = x.n; ++a.narr; }
  int32_t* flag = at<int32_t>(ws, P.flag);
  HIPCHK(lt::launch_zero32(flag, 1, st));
  HIPCHK(lt::launch_scan_finite(a, flag, st));
  int32_t h = 0;
  HIPCHK(hipMemcpyAsync(&h, flag, 4, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (h) return fail(LT_ENONFINITE, "NaN or infinity in the inputs (options.check_finite)");
  return LT_OK;
}

}  // namespace

extern "C" {

int ltriples_rhf_spin_block_workspace_size(const ltriples_rhf_domain* d, int32_t precision,
                                           const ltriples_options* o, size_t* bytes) {
  g_err.clear();
  if (!bytes) return fail(LT_EINVAL, "bytes is NULL");
  RhfSetup S;
  int r = rhf_setup(d, o, S);
  if (r) return r;
  size_t inner = 0;
  r = ltriples_workspace_size(&S.d, precision, &S.o, &inner);
  if (r) return r;
  *bytes = S.head + inner;
  return LT_OK;
}

int ltriples_rhf_workspace_size(const ltriples_rhf_domain* d, int32_t precision, const ltriples_options* o,
                                size_t* bytes) {
  g_err.clear();
  if (!bytes) return fail(LT_EINVAL, "bytes is NULL");
  RhfSetup S;
  int r = rhf_setup(d, o, S);
  if (r) return r;
  r = validate(&S.d, precision, nullptr);
  if (r) return r;
  r = validate_options(o);
  if (r) return r;
  SaPlan P;
  sa_plan(d, precision, o, P);
  *bytes = P.total;
  return LT_OK;
}

int ltriples_rhf_flops(const ltriples_rhf_domain* d, double* flops, int64_t* n_items_out) {
  g_err.clear();
  if (!flops) return fail(LT_EINVAL, "NULL argument");
  RhfSetup S;
  const int r = rhf_setup(d, nullptr, S);
  if (r) return r;
  const double no = (double)d->no, nv = (double)d->nv;
  const int64_t n = sa_items(d->no);
  *flops = (double)n * 3.0 * 2.0 * nv * nv * nv * (2.0 * nv + 2.0 * no);
  if (n_items_out) *n_items_out = n;
  return LT_OK;
}

int ltriples_energy_rhf(const ltriples_rhf_domain* rd, int32_t precision, const ltriples_options* o,
                        double* e_out, double* parts, void* ws, size_t ws_bytes, void* stream) {
  g_err.clear();
  RhfSetup S;
  int r = rhf_setup(rd, o, S);
  if (r) return r;
  if (!e_out) return fail(LT_EINVAL, "e_out is NULL");
  r = validate(&S.d, precision, nullptr);
  if (r) return r;
  r = validate_options(o);
  if (r) return r;
  SaPlan P;
  sa_plan(rd, precision, o, P);
  hipStream_t st = (hipStream_t)stream;
  r = check_denominators(&S.d, st);   // before anything is allocated or enqueued
  if (r) return r;
  OwnedWs own;
  r = get_ws(ws, ws_bytes, P.total, st, own);
  if (r) return r;
  r = sa_upload(P, ws, st);
  if (r) return r;
  if (o && o->check_finite) {
    r = sa_scan_finite(rd, P, ws, st);
    if (r) return r;
  }
  Timing tm;
  tm.on = o && o->stats;
  tm.st = st;
  if (precision == LT_FP64) r = sa_run<double>(rd, P, o, e_out, parts, ws, st, tm);
  else r = sa_run<float>(rd, P, o, e_out, parts, ws, st, tm);
  if (r == LT_OK && tm.on) {
    HIPCHK(hipStreamSynchronize(st));
    ltriples_stats* St = o->stats;
    *St = ltriples_stats{};
    St->total_ms = Timing::ms(tm.start, tm.end);
    St->setup_ms = Timing::ms(tm.start, tm.setup_end);
    for (auto& x : tm.gemm) St->triples_gemm_ms += Timing::ms(x.first, x.second);
    for (auto& x : tm.epi) St->epilogue_ms += Timing::ms(x.first, x.second);
    St->triples_gemm_launches = (int64_t)tm.gemm.size();
    St->triples_gemm_flops = tm.gemm_flops;
    St->algorithmic_flops = tm.gemm_flops;
    St->n_items = P.n_items;
  }
  return r;
}

int ltriples_energy_rhf_spin_block(const ltriples_rhf_domain* rd, int32_t precision, const ltriples_options* o,
                                   double* e_out, double* parts, void* ws, size_t ws_bytes, void* stream) {
  g_err.clear();
  RhfSetup S;
  int r = rhf_setup(rd, o, S);
  if (r) return r;
  if (!e_out) return fail(LT_EINVAL, "e_out is NULL");
  size_t inner = 0;
  r = ltriples_workspace_size(&S.d, precision, &S.o, &inner);
  if (r) return r;
  const size_t need = S.head + inner;
  hipStream_t st = (hipStream_t)stream;
  r = check_denominators(&S.d, st);   // before anything is allocated or enqueued
  if (r) return r;
  OwnedWs own;
  r = get_ws(ws, ws_bytes, need, st, own);
  if (r) return r;
  char* base = (char*)ws;
  double* t2 = (double*)base;
  double* tmp = (double*)(base + S.t2_bytes);
  const int64_t no = rd->no, nv = rd->nv;
  // t2aa[i][j][a][b] = tau[i][j][a][b] - tau[i][j][b][a]
  r = LT_OK;
  {
    const hipError_t e = lt::launch_copy4d<double, double>(t2, no * nv * nv, nv * nv, nv, no, no, nv, nv, rd->tau,
                                                           no * nv * nv, nv * nv, nv, 1, rd->tau, no * nv * nv,
                                                           nv * nv, 1, nv, st);
    if (e != hipSuccess) r = fail(LT_EHIP, "HIP error %s", hipGetErrorString(e));
  }
  if (r == LT_OK) {
    S.d.t2aa = S.d.t2bb = t2;
    r = ltriples_energy(&S.d, precision, &S.o, tmp, tmp + 1, base + S.head, need - S.head, stream);
  }
  if (r == LT_OK) {
    const hipError_t e = lt::launch_rhf_combine(tmp, e_out, parts, st);
    if (e != hipSuccess) r = fail(LT_EHIP, "HIP error %s", hipGetErrorString(e));
  }
  return r;
}

}  // extern "C"

namespace {

// Workspace of the closed-shell adjoint after the forward head: 2 gbar, then
// the beta-side and amplitude gradients of the spin-block adjoint.
struct RhfBwd {
  size_t g2, t1b, t2ab, t2aa, t2bb, Boo, Bov, Bvv, eo, ev, fov, end;
};

RhfBwd rhf_bwd_layout(const ltriples_rhf_domain* r, size_t head) {
  const size_t no = r->no, nv = r->nv, Q = r->naux;
  RhfBwd L{};
  size_t off = head;
  auto take = [&](size_t n) { const size_t o = off; off = align256(off + 8 * std::max<size_t>(n, 1)); return o; };
  L.g2 = take(1);
  L.t1b = take(no * nv);
  L.t2ab = take(no * no * nv * nv);
  L.t2aa = take(no * no * nv * nv);
  L.t2bb = take(no * no * nv * nv);
  L.Boo = take(Q * no * no);
  L.Bov = take(Q * no * nv);
  L.Bvv = take(Q * nv * nv);
  L.eo = take(no);
  L.ev = take(nv);
  L.fov = take(no * nv);
  L.end = off;
  return L;
}

}  // namespace

extern "C" {

int ltriples_backward_rhf_workspace_size(const ltriples_rhf_domain* d, int32_t precision, const ltriples_options* o,
                                         size_t* bytes) {
  g_err.clear();
  if (!bytes) return fail(LT_EINVAL, "bytes is NULL");
  RhfSetup S;
  int r = rhf_setup(d, o, S);
  if (r) return r;
  size_t inner = 0;
  r = ltriples_backward_workspace_size(&S.d, precision, &S.o, &inner);
  if (r) return r;
  *bytes = rhf_bwd_layout(d, S.head).end + inner;
  return LT_OK;
}

int ltriples_backward_rhf(const ltriples_rhf_domain* rd, int32_t precision, const ltriples_options* o,
                          const double* gbar, const ltriples_rhf_grad* grad, void* ws, size_t ws_bytes,
                          void* stream) {
  g_err.clear();
  RhfSetup S;
  int r = rhf_setup(rd, o, S);
  if (r) return r;
  if (!gbar) return fail(LT_EINVAL, "gbar is NULL");
  if (!grad) return fail(LT_EINVAL, "grad is NULL");
  size_t inner = 0;
  r = ltriples_backward_workspace_size(&S.d, precision, &S.o, &inner);
  if (r) return r;
  const RhfBwd Lb = rhf_bwd_layout(rd, S.head);
  const size_t need = Lb.end + inner;
  hipStream_t st = (hipStream_t)stream;
  r = check_denominators(&S.d, st);   // before anything is allocated or enqueued
  if (r) return r;
  OwnedWs own;
  r = get_ws(ws, ws_bytes, need, st, own);
  if (r) return r;
  char* base = (char*)ws;
  auto D = [&](size_t off) { return (double*)(base + off); };
  const int64_t no = rd->no, nv = rd->nv, Q = rd->naux;
  double* t2 = D(0);
  double* g2 = D(Lb.g2);
  auto run = [&]() -> int {
    // same-spin amplitudes tau^{ab}_{ij} - tau^{ba}_{ij}, and 2 gbar
    HIPCHK(lt::launch_copy4d<double, double>(t2, no * nv * nv, nv * nv, nv, no, no, nv, nv, rd->tau, no * nv * nv,
                                             nv * nv, nv, 1, rd->tau, no * nv * nv, nv * nv, 1, nv, st));
    HIPCHK(lt::launch_zero(g2, 1, st));
    {
      const int64_t d1[4] = {1, 1, 1, 1}, z[4] = {0, 0, 0, 0};
      HIPCHK(lt::launch_perm_acc<double>(g2, d1, z, gbar, z, 2.0, st));
    }
    S.d.t2aa = S.d.t2bb = t2;
    ltriples_domain_grad gi{};
    gi.t1a = grad->t1; gi.t1b = grad->t1 ? D(Lb.t1b) : nullptr;
    const bool wt = grad->tau != nullptr;
    gi.t2ab = wt ? D(Lb.t2ab) : nullptr; gi.t2aa = wt ? D(Lb.t2aa) : nullptr; gi.t2bb = wt ? D(Lb.t2bb) : nullptr;
    gi.Boo_a = grad->Boo; gi.Boo_b = grad->Boo ? D(Lb.Boo) : nullptr;
    gi.Bov_a = grad->Bov; gi.Bov_b = grad->Bov ? D(Lb.Bov) : nullptr;
    gi.Bvv_a = grad->Bvv; gi.Bvv_b = grad->Bvv ? D(Lb.Bvv) : nullptr;
    gi.eo_a = grad->eo; gi.eo_b = grad->eo ? D(Lb.eo) : nullptr;
    gi.ev_a = grad->ev; gi.ev_b = grad->ev ? D(Lb.ev) : nullptr;
    gi.fov_a = grad->fov; gi.fov_b = grad->fov ? D(Lb.fov) : nullptr;
    int rr = ltriples_backward(&S.d, precision, &S.o, g2, &gi, base + Lb.end, need - Lb.end, stream);
    if (rr) return rr;
    // alpha + beta for every shared input (flat copies)
    auto add_flat = [&](double* out, const double* in, int64_t n) -> int {
      if (!out || n <= 0) return LT_OK;
      const int64_t d1[4] = {1, 1, 1, n}, s1[4] = {0, 0, 0, 1};
      HIPCHK(lt::launch_perm_acc<double>(out, d1, s1, in, s1, 1.0, st));
      return LT_OK;
    };
    if ((rr = add_flat(grad->t1, gi.t1b, no * nv))) return rr;
    if ((rr = add_flat(grad->Boo, gi.Boo_b, Q * no * no))) return rr;
    if ((rr = add_flat(grad->Bov, gi.Bov_b, Q * no * nv))) return rr;
    if ((rr = add_flat(grad->Bvv, gi.Bvv_b, Q * nv * nv))) return rr;
    if ((rr = add_flat(grad->eo, gi.eo_b, no))) return rr;
    if ((rr = add_flat(grad->ev, gi.ev_b, nv))) return rr;
    if ((rr = add_flat(grad->fov, gi.fov_b, no * nv))) return rr;
    if (wt && no > 0 && nv > 0) {
      // dtau = (g_ab + g_ab^{ji,ba}) / 2 + 2 g_aa + 2 g_bb
      HIPCHK(lt::launch_zero(grad->tau, no * no * nv * nv, st));
      const int64_t dd[4] = {no, no, nv, nv}, sid[4] = {no * nv * nv, nv * nv, nv, 1};
      const int64_t swp[4] = {nv * nv, no * nv * nv, 1, nv};
      HIPCHK(lt::launch_perm_acc<double>(grad->tau, dd, sid, gi.t2ab, sid, 0.5, st));
      HIPCHK(lt::launch_perm_acc<double>(grad->tau, dd, sid, gi.t2ab, swp, 0.5, st));
      HIPCHK(lt::launch_perm_acc<double>(grad->tau, dd, sid, gi.t2aa, sid, 2.0, st));
      HIPCHK(lt::launch_perm_acc<double>(grad->tau, dd, sid, gi.t2bb, sid, 2.0, st));
    } else if (wt) {
      HIPCHK(lt::launch_zero(grad->tau, no * no * nv * nv, st));
    }
    return LT_OK;
  };
  return run();
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Natural auxiliary functions: pair-packed integrals -> W by GEMM (rocBLAS),
// eigenvectors by syevd (rocSOLVER), kept vectors in decreasing order, the
// compressed factors by GEMM and strided slices.
// ---------------------------------------------------------------------------
namespace {

struct NafPlan {
  int64_t n[2], o[2], nx, pmax, nmax;
  size_t oP, oW, oD, oE, oInfo, oUk, oB, total;
};

int naf_plan(const ltriples_naf_input* in, NafPlan& P) {
  if (!in) return fail(LT_EINVAL, "input is NULL");
  if (in->no_a < 0 || in->nv_a < 0 || in->no_b < 0 || in->nv_b < 0 || in->nx < 0)
    return fail(LT_EINVAL, "negative dimension");
  P.o[0] = in->no_a; P.o[1] = in->no_b;
  P.n[0] = (int64_t)in->no_a + in->nv_a; P.n[1] = (int64_t)in->no_b + in->nv_b;
  P.nx = in->nx;
  if (P.n[0] > 46340 || P.n[1] > 46340 || P.nx > 46340) return fail(LT_ESHAPE, "dimension too large");
  if (P.nx > 0 && P.n[0] > 0 && !in->Ja) return fail(LT_EINVAL, "Ja is NULL");
  if (P.nx > 0 && P.n[1] > 0 && !in->Jb) return fail(LT_EINVAL, "Jb is NULL");
  P.nmax = std::max(P.n[0], P.n[1]);
  P.pmax = P.nmax * (P.nmax + 1) / 2;
  size_t off = 0;
  auto take = [&](size_t bytes) { const size_t o = off; off = align256(off + std::max<size_t>(bytes, 1)); return o; };
  const size_t nx = (size_t)P.nx;
  P.oP = take(8 * nx * (size_t)P.pmax);
  P.oW = take(8 * nx * nx);
  P.oD = take(8 * nx);
  P.oE = take(8 * nx);
  P.oInfo = take(sizeof(rocblas_int));
  P.oUk = take(8 * nx * nx);
  P.oB = take(8 * nx * (size_t)(P.nmax * P.nmax));
  P.total = off;
  return LT_OK;
}

#define RBCHK(...)                                                                      \
  do {                                                                                  \
    rocblas_status s_ = (__VA_ARGS__);                                                  \
    if (s_ != rocblas_status_success) {                                                 \
      r = fail(LT_EHIP, "rocBLAS/rocSOLVER status %d at %s:%d", (int)s_, __FILE__, __LINE__); \
      goto done;                                                                        \
    }                                                                                   \
  } while (0)
#define HIPGO(...)                                                                      \
  do {                                                                                  \
    hipError_t e_ = (__VA_ARGS__);                                                      \
    if (e_ != hipSuccess) {                                                             \
      r = fail(LT_EHIP, "HIP error %s at %s:%d", hipGetErrorString(e_), __FILE__, __LINE__); \
      goto done;                                                                        \
    }                                                                                   \
  } while (0)

}  // namespace

extern "C" {

int ltriples_naf_workspace_size(const ltriples_naf_input* in, size_t* bytes) {
  g_err.clear();
  if (!bytes) return fail(LT_EINVAL, "bytes is NULL");
  NafPlan P;
  const int r = naf_plan(in, P);
  if (r) return r;
  *bytes = P.total;
  return LT_OK;
}

int ltriples_naf(const ltriples_naf_input* in, double eps, const ltriples_naf_output* out, int32_t* naux_out,
                 void* ws, size_t ws_bytes, void* stream) {
  g_err.clear();
  NafPlan P;
  int r = naf_plan(in, P);
  if (r) return r;
  if (!out || !naux_out) return fail(LT_EINVAL, "output is NULL");
  if (std::isnan(eps)) return fail(LT_EINVAL, "eps is NaN");
  hipStream_t st = (hipStream_t)stream;
  OwnedWs own;
  r = get_ws(ws, ws_bytes, P.total, st, own);
  if (r) return r;
  char* base = (char*)ws;
  double* Pk = (double*)(base + P.oP);
  double* W = (double*)(base + P.oW);
  double* D = (double*)(base + P.oD);
  double* E = (double*)(base + P.oE);
  rocblas_int* info = (rocblas_int*)(base + P.oInfo);
  double* Uk = (double*)(base + P.oUk);
  double* Bf = (double*)(base + P.oB);
  const double* J[2] = {in->Ja, in->Jb};
  double* outs[2][3] = {{out->Boo_a, out->Bov_a, out->Bvv_a}, {out->Boo_b, out->Bov_b, out->Bvv_b}};
  const int nx = (int)P.nx;
  rocblas_handle h = nullptr;
  std::vector<double> Dh(P.nx);
  rocblas_int info_h = 0;
  int64_t m = 0;
  *naux_out = 0;
  if (nx == 0) goto done;
  RBCHK(rocblas_create_handle(&h));
  RBCHK(rocblas_set_stream(h, st));
  RBCHK(rocblas_set_atomics_mode(h, rocblas_atomics_not_allowed));   // fixed summation order
  {
    // W = (W_a + W_b) / 2, W_s = P_s^T P_s over the pair-packed rows.  One
    // full-square GEMM per spin: with a contraction of ~n^2/2 pairs against
    // nx^2 outputs, the library's triangular SYRK splits into a few narrow
    // GEMMs that leave most of the GPU idle, while the square GEMM fills it
    // (twice the flops, several times faster).
    bool first = true;
    for (int s = 0; s < 2; ++s) {
      const int n = (int)P.n[s];
      if (n == 0) continue;
      const rocblas_int np = (rocblas_int)((int64_t)n * (n + 1) / 2);
      HIPGO(lt::launch_naf_pack(Pk, J[s], n, nx, st));
      const double alpha = 0.5, beta = first ? 0.0 : 1.0;
      RBCHK(rocblas_dgemm(h, rocblas_operation_transpose, rocblas_operation_none, nx, nx, np, &alpha, Pk, np, Pk, np,
                          &beta, W, nx));
      first = false;
    }
    if (first) HIPGO(lt::launch_zero(W, (int64_t)nx * nx, st));
  }
  RBCHK(rocsolver_dsyevd(h, rocblas_evect_original, rocblas_fill_upper, nx, W, nx, D, E, info));
  HIPGO(hipMemcpyAsync(Dh.data(), D, 8 * (size_t)nx, hipMemcpyDeviceToHost, st));
  HIPGO(hipMemcpyAsync(&info_h, info, sizeof(info_h), hipMemcpyDeviceToHost, st));
  HIPGO(hipStreamSynchronize(st));
  if (info_h != 0) {
    r = fail(LT_EHIP, "eigensolver did not converge (info %d)", (int)info_h);
    goto done;
  }
  for (int64_t k = 0; k < P.nx; ++k) m += Dh[k] > eps ? 1 : 0;
  // eigenvalues and kept vectors in decreasing order (syevd returns them increasing)
  if (out->eigenvalues)
    HIPGO(lt::launch_copy4d<double, double>(out->eigenvalues, 0, 0, 0, 1, 1, 1, nx, D + (nx - 1), 0, 0, 0, -1,
                                            nullptr, 0, 0, 0, 0, st));
  if (m > 0) {
    // Uk column Q (column-major, nx x m) = eigenvector nx - 1 - Q
    HIPGO(lt::launch_copy4d<double, double>(Uk, 0, 0, nx, 1, 1, m, nx, W + (int64_t)(nx - 1) * nx, 0, 0, -nx, 1,
                                            nullptr, 0, 0, 0, 0, st));
    for (int s = 0; s < 2; ++s) {
      const int64_t n = P.n[s], o = P.o[s], v = n - o;
      if (n == 0 || (!outs[s][0] && !outs[s][1] && !outs[s][2])) continue;
      // Bf[Q][pq] (column-major n^2 x m) = J_s (n^2 x nx) * Uk
      const double one = 1.0, zero = 0.0;
      RBCHK(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, (rocblas_int)(n * n), (rocblas_int)m,
                          nx, &one, J[s], (rocblas_int)(n * n), Uk, nx, &zero, Bf, (rocblas_int)(n * n)));
      if (outs[s][0])
        HIPGO(lt::launch_copy4d<double, double>(outs[s][0], 0, o * o, o, 1, m, o, o, Bf, 0, n * n, n, 1, nullptr, 0,
                                                0, 0, 0, st));
      if (outs[s][1])
        HIPGO(lt::launch_copy4d<double, double>(outs[s][1], 0, o * v, v, 1, m, o, v, Bf + o, 0, n * n, n, 1,
                                                nullptr, 0, 0, 0, 0, st));
      if (outs[s][2])
        HIPGO(lt::launch_copy4d<double, double>(outs[s][2], 0, v * v, v, 1, m, v, v, Bf + o * n + o, 0, n * n, n, 1,
                                                nullptr, 0, 0, 0, 0, st));
    }
  }
  *naux_out = (int32_t)m;
done:
  if (h) {
    const hipError_t e1 = hipStreamSynchronize(st);
    const rocblas_status e2 = rocblas_destroy_handle(h);
    if (r == LT_OK && (e1 != hipSuccess || e2 != rocblas_status_success))
      r = fail(LT_EHIP, "error at rocBLAS handle release");
  }
  return r;
}

int ltriples_autotune_reset(void) {
  g_err.clear();
  lt::reset_gemm_bf16_tuning();
  lt::reset_gemm_tuning();
  return LT_OK;
}

const char* ltriples_last_error(void) { return g_err.c_str(); }

const char* ltriples_version(void) { return "ltriples 0.1.0 (gfx950)"; }

}  // extern "C"
