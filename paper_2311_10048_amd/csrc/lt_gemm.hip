// Segmented, k-major MFMA GEMM for gfx950.
//
//   C[m][n] = sum_s sign_s sum_k Lt_s[k][m] R_s[k][n]
//
// Used for (a) the density-fitting builds of the (ov|vv), (ov|oo) and
// (ov|ov) integral classes (one segment, K = naux) and (b) the triples
// contractions of one occupied triplet, where the segments are the terms of
// the spin-block working equations that share an output layout (the
// occupied permutations P(i/jk) / P(ij) concatenated along K).
//
// Tiling: a work-group of 4 waves owns a BM x BN output tile, BM = MB row
// blocks of the MFMA shape (the whole virtual range of a triplet GEMM for
// MB <= 16), BN = 4 column blocks (one per wave).  K advances in chunks of
// 16 staged through double-buffered LDS; every global load is a 16-byte
// vector along a contiguous operand row.  Work-groups are renumbered so that
// consecutive logical tiles run on the same XCD (the dispatcher deals
// work-groups round-robin over the 8 XCDs), which keeps a triplet's small
// L operand and an R-operand tile shared by the row tiles in one L2.
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <vector>

#include "lt_internal.h"

namespace lt {

// Segment idx of the contraction of one occupied triplet (i, j, k); all
// arguments are wave-uniform, so the descriptor lives in scalar registers.
// Operand blocks are indexed over the o_s (o_t) orbitals; the contractions
// over occupied orbitals run over the first oi_s (oi_t) rows of a block.
template <typename T>
__device__ inline Seg<T> item_seg(const ItemOps<T>& s, int64_t i, int64_t j, int64_t k, int idx) {
  const int64_t o = s.o_s, v = s.v_s, ot = s.o_t, vt = s.v_t;
  const int64_t lv = s.ld_vs, lt_ = s.ld_vt, lp = s.ld_np, lc = s.ld_cb;
  if (s.kind == 0) {
    // S[a][p(b<c)] = P(i/jk)[sum_e t^{ae}_{jk}<ei||bc> - sum_m <ma||jk> t^{bc}_{im}]
    const int64_t tb = v * lv, ab = v * lp, gb = o * lv, pb = o * lp;
    switch (idx) {
      case 0: return {s.T2T + (j * o + k) * tb, lv, s.As + i * ab, lp, (int32_t)v, 1.f};
      case 1: return {s.T2T + (i * o + k) * tb, lv, s.As + j * ab, lp, (int32_t)v, -1.f};
      case 2: return {s.T2T + (j * o + i) * tb, lv, s.As + k * ab, lp, (int32_t)v, -1.f};
      case 3: return {s.GamT + (j * o + k) * gb, lv, s.Tp + i * pb, lp, s.oi_s, -1.f};
      case 4: return {s.GamT + (i * o + k) * gb, lv, s.Tp + j * pb, lp, s.oi_s, 1.f};
      default: return {s.GamT + (j * o + i) * gb, lv, s.Tp + k * pb, lp, s.oi_s, 1.f};
    }
  }
  if (s.kind == 3) {
    // closed shell, occupied triple (p,q,r) = (i,j,k) over spatial orbitals:
    // F[a][b*v+c] = sum_e tau^{ae}_{ij}(kc|be) + sum_e tau^{ae}_{ik}(jb|ce)
    //             - sum_m (ia|mk) tau^{bc}_{jm} - sum_m (ia|mj) tau^{bc}_{mk}
    const int64_t lvv = s.ld_vv;
    switch (idx) {
      case 0: return {s.T2T + (i * o + j) * v * lv, lv, s.RVc + k * v * lvv, lvv, (int32_t)v, 1.f};
      case 1: return {s.T2T + (i * o + k) * v * lv, lv, s.RVs + j * v * lvv, lvv, (int32_t)v, 1.f};
      case 2: return {s.Gcs + (k * o + i) * o * lv, lv, s.Tf + j * o * lvv, lvv, s.oi_s, -1.f};
      default: return {s.Gcs + (j * o + i) * o * lv, lv, s.Ts + k * o * lvv, lvv, s.oi_s, -1.f};
    }
  }
  if (s.kind == 1) {
    // G[a][C*v+b] = sum_E t^{aE}_{iK}(jb|EC) - sum_E t^{aE}_{jK}(ib|EC) + sum_e t^{ae}_{ij}(be|KC)
    //             - sum_m <am||ij> t^{bC}_{mK} + sum_M (aj|MK) t^{bC}_{iM} - sum_M (ai|MK) t^{bC}_{jM}
    switch (idx) {
      case 0: return {s.LmixT + (i * ot + k) * vt * lv, lv, s.Mst + j * vt * lc, lc, (int32_t)vt, 1.f};
      case 1: return {s.LmixT + (j * ot + k) * vt * lv, lv, s.Mst + i * vt * lc, lc, (int32_t)vt, -1.f};
      case 2: return {s.T2T + (i * o + j) * v * lv, lv, s.Mts + k * v * lc, lc, (int32_t)v, 1.f};
      case 3: return {s.GamT + (i * o + j) * o * lv, lv, s.Tmix + k * lc, ot * lc, s.oi_s, 1.f};
      case 4: return {s.ZpT + (j * ot + k) * ot * lv, lv, s.Tmix + i * ot * lc, lc, s.oi_t, 1.f};
      default: return {s.ZpT + (i * ot + k) * ot * lv, lv, s.Tmix + j * ot * lc, lc, s.oi_t, -1.f};
    }
  }
  // Y[C][p(a<b)] = -sum_e t^{eC}_{iK}<je||ab> + sum_e t^{eC}_{jK}<ie||ab>
  //              - sum_m (jm|CK) t^{ab}_{im} + sum_m (im|CK) t^{ab}_{jm}
  switch (idx) {
    case 0: return {s.TmT + (i * ot + k) * v * lt_, lt_, s.As + j * v * lp, lp, (int32_t)v, 1.f};
    case 1: return {s.TmT + (j * ot + k) * v * lt_, lt_, s.As + i * v * lp, lp, (int32_t)v, -1.f};
    case 2: return {s.OOT + (k * o + j) * o * lt_, lt_, s.Tp + i * o * lp, lp, s.oi_s, -1.f};
    default: return {s.OOT + (k * o + i) * o * lt_, lt_, s.Tp + j * o * lp, lp, s.oi_s, 1.f};
  }
}

template <typename T> struct Vec;
template <> struct Vec<float> { typedef float4 type; static constexpr int N = 4; };
template <> struct Vec<double> { typedef double2 type; static constexpr int N = 2; };

template <typename T>
__device__ inline typename Vec<T>::type vscale(typename Vec<T>::type v, float s) {
  if constexpr (Vec<T>::N == 4) { v.x *= s; v.y *= s; v.z *= s; v.w *= s; }
  else { v.x *= (double)s; v.y *= (double)s; }
  return v;
}

// Work-group tile: 4 waves in a WM x (4/WM) grid; each wave owns MBW x NBW
// MFMA blocks, so BM = WM*MBW*BR rows and BN = (4/WM)*NBW*BC columns.
template <typename T, int MBW, int NBW, int WM, int BK>
__device__ __forceinline__ void gemm_body(const GemmArgs<T>& g) {
  using F = MF<T>;
  using V = typename Vec<T>::type;
  constexpr int VN = Vec<T>::N;
  constexpr int BR = F::BR, BC = F::BC;
  constexpr int WN = 4 / WM;
  constexpr int BM = WM * MBW * BR;
  constexpr int BN = WN * NBW * BC;
  constexpr int AROW = BM / VN, BROW = BN / VN;       // vectors per staged row
  constexpr int AV = BK * AROW, BV = BK * BROW;
  constexpr int AVT = (AV + 255) / 256, BVT = (BV + 255) / 256;

  __shared__ __attribute__((aligned(16))) T As[2][BK][BM];
  __shared__ __attribute__((aligned(16))) T Bs[2][BK][BN];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;

  // logical tile id: consecutive ids share an XCD
  int b = blockIdx.x;
  {
    const int nblk = gridDim.x, x = b & 7, q = nblk >> 3, r = nblk & 7;
    b = (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + (b >> 3);
  }
  const int mtile = b % g.mt; b /= g.mt;
  const int ntile = b % g.nt; b /= g.nt;
  const int batch = b;
  const int m0 = mtile * BM, n0 = ntile * BN;

  int64_t ti = 0, tj = 0, tk = 0;
  int nseg = 1;
  if (g.mode == 1) {
    const int32_t* it = g.ops.items + 3 * batch;
    ti = it[0]; tj = it[1]; tk = it[2];
    nseg = g.ops.kind >= 2 ? 4 : 6;
  }
  auto seg = [&](int idx) -> Seg<T> {
    if (g.mode == 0)
      return {g.L + (int64_t)batch * g.lbs, g.lks, g.R + (int64_t)batch * g.rbs, g.rks, g.K, 1.f};
    return item_seg(g.ops, ti, tj, tk, idx);
  };

  typename F::acc_t acc[MBW][NBW];
#pragma unroll
  for (int mb = 0; mb < MBW; ++mb)
#pragma unroll
    for (int nb = 0; nb < NBW; ++nb)
#pragma unroll
      for (int r = 0; r < F::NACC; ++r) acc[mb][nb][r] = 0;

  V ra[AVT], rb[BVT];
  auto gload = [&](int s, int k0) {
    const Seg<T> sg = seg(s);
#pragma unroll
    for (int u = 0; u < AVT; ++u) {
      const int e = tid + u * 256;
      V v = {};
      if (e < AV) {
        const int kk = e / AROW, m = m0 + (e % AROW) * VN, k = k0 + kk;
        if (k < sg.K && m < g.M) v = vscale<T>(*(const V*)(sg.L + (int64_t)k * sg.lks + m), sg.sign);
      }
      ra[u] = v;
    }
#pragma unroll
    for (int u = 0; u < BVT; ++u) {
      const int e = tid + u * 256;
      V v = {};
      if (e < BV) {
        const int kk = e / BROW, n = n0 + (e % BROW) * VN, k = k0 + kk;
        if (k < sg.K && n < g.N) v = *(const V*)(sg.R + (int64_t)k * sg.rks + n);
      }
      rb[u] = v;
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int u = 0; u < AVT; ++u) {
      const int e = tid + u * 256;
      if (e < AV) *(V*)&As[buf][e / AROW][(e % AROW) * VN] = ra[u];
    }
#pragma unroll
    for (int u = 0; u < BVT; ++u) {
      const int e = tid + u * 256;
      if (e < BV) *(V*)&Bs[buf][e / BROW][(e % BROW) * VN] = rb[u];
    }
  };

  int s = 0, k0 = 0;
  while (s < nseg && seg(s).K <= 0) ++s;
  if (s < nseg) { gload(s, k0); sstore(0); }
  __syncthreads();
  int cur = 0;
  const int arow0 = wm * MBW * BR + F::a_row(lane);
  const int bcol0 = wn * NBW * BC + F::c_col(lane);
  while (s < nseg) {
    k0 += BK;
    while (s < nseg && k0 >= seg(s).K) { ++s; k0 = 0; }
    const bool more = s < nseg;
    if (more) gload(s, k0);
#pragma unroll
    for (int ks = 0; ks < BK; ks += F::KS) {
      const int kr = ks + F::a_k(lane);
      T bv[NBW];
#pragma unroll
      for (int nb = 0; nb < NBW; ++nb) bv[nb] = Bs[cur][kr][bcol0 + nb * BC];
#pragma unroll
      for (int mb = 0; mb < MBW; ++mb) {
        const T av = As[cur][kr][arow0 + mb * BR];
#pragma unroll
        for (int nb = 0; nb < NBW; ++nb) acc[mb][nb] = F::mma(av, bv[nb], acc[mb][nb]);
      }
    }
    if (more) sstore(cur ^ 1);
    __syncthreads();
    cur ^= 1;
  }

  // store
  T* out = g.out + (int64_t)batch * g.obs;
#pragma unroll
  for (int nb = 0; nb < NBW; ++nb) {
    const int n = n0 + bcol0 + nb * BC;
    if (n >= g.N) continue;
    const int64_t noff = g.ndiv ? (int64_t)(n / g.ndiv) * g.s_nq + (int64_t)(n % g.ndiv) * g.s_nr
                                : (int64_t)n * g.s_nr;
#pragma unroll
    for (int mb = 0; mb < MBW; ++mb)
#pragma unroll
      for (int r = 0; r < F::NACC; ++r) {
        const int m = m0 + wm * MBW * BR + mb * BR + F::c_row(lane, r);
        if (m < g.M) {
          const int64_t moff = g.mdiv ? (int64_t)(m / g.mdiv) * g.s_mq + (int64_t)(m % g.mdiv) * g.s_mr
                                      : (int64_t)m * g.s_mr;
          out[moff + noff] = acc[mb][nb][r];
        }
      }
  }
}

// Two entry points with distinct names so that profiles separate the
// integral builds from the triplet contractions.
template <typename T, int MBW, int NBW, int WM, int BK>
__global__ __launch_bounds__(256) void k_dfgemm(GemmArgs<T> g) { gemm_body<T, MBW, NBW, WM, BK>(g); }
template <typename T, int MBW, int NBW, int WM, int BK>
__global__ __launch_bounds__(256) void k_tgemm(GemmArgs<T> g) { gemm_body<T, MBW, NBW, WM, BK>(g); }

template <typename T, int MBW, int NBW, int WM, int BK>
hipError_t launch_cfg(GemmArgs<T> g, hipStream_t s) {
  constexpr int BM = WM * MBW * MF<T>::BR, BN = (4 / WM) * NBW * MF<T>::BC;
  g.mt = (g.M + BM - 1) / BM;
  g.nt = (g.N + BN - 1) / BN;
  const int64_t nblk = (int64_t)g.mt * g.nt * g.nbatch;
  if (nblk <= 0) return hipSuccess;
  if (nblk > 0x7fffffff) return hipErrorInvalidValue;
  if (g.mode == 1)
    hipLaunchKernelGGL((k_tgemm<T, MBW, NBW, WM, BK>), dim3((unsigned)nblk), dim3(256), 0, s, g);
  else
    hipLaunchKernelGGL((k_dfgemm<T, MBW, NBW, WM, BK>), dim3((unsigned)nblk), dim3(256), 0, s, g);
  return hipGetLastError();
}

#ifndef LT_GEMM_NO_DISPATCH
// Tile choice (measured on gfx950 at the triplet-contraction shapes): the
// whole M range in one work-group tile when it fits, 2 x 2 waves for
// M > 96; FP64 with K chunks of 8.  Large-M integral builds use 128-row tiles.
// Triplet contractions with more than 256 rows and at least 2^15 columns (the
// whole-domain shapes) take 64-row tiles instead: timed against the whole-M
// and 256-row tiles at M = 300 and 500 in FP32 and M = 300 in FP64, they cut
// the contraction time by 10-25 %.
// With tuning, the triplet contractions (mode 1) of each shape class may
// take another configuration from the candidates below; every configuration
// sums each output element in the same order, so results do not change.
namespace {

template <typename T> struct GCfg { int rows; hipError_t (*fn)(GemmArgs<T>, hipStream_t); };
const GCfg<float> kCfg32[] = {
    {32, launch_cfg<float, 1, 1, 1, 16>},  {64, launch_cfg<float, 2, 1, 1, 16>},
    {96, launch_cfg<float, 3, 1, 1, 16>},  {128, launch_cfg<float, 2, 2, 2, 16>},
    {192, launch_cfg<float, 3, 2, 2, 16>}, {256, launch_cfg<float, 4, 2, 2, 16>},
    {320, launch_cfg<float, 5, 2, 2, 16>}, {384, launch_cfg<float, 6, 2, 2, 16>}};
const GCfg<double> kCfg64[] = {
    {32, launch_cfg<double, 2, 1, 1, 8>},   {64, launch_cfg<double, 4, 1, 1, 8>},
    {128, launch_cfg<double, 4, 2, 2, 8>},  {192, launch_cfg<double, 6, 2, 2, 8>},
    {256, launch_cfg<double, 8, 2, 2, 8>},  {320, launch_cfg<double, 10, 2, 2, 8>},
    {384, launch_cfg<double, 12, 2, 2, 8>}, {512, launch_cfg<double, 16, 2, 2, 8>}};

int default32(int M) {
  const int need = (M + 31) / 32;
  if (need <= 1) return 0;
  if (need <= 2) return 1;
  if (need <= 3) return 2;
  if (need <= 4) return 3;
  if (need <= 6) return 4;
  if (need <= 8) return 5;
  if (need <= 10) return 6;
  if (need <= 12) return 7;
  if (need <= 16) return 5;   // two row tiles
  return 3;
}
int default64(int M) {
  const int need = (M + 15) / 16;
  if (need <= 2) return 0;
  if (need <= 4) return 1;
  if (need <= 8) return 2;
  if (need <= 12) return 3;
  if (need <= 16) return 4;
  if (need <= 20) return 5;
  if (need <= 24) return 6;
  if (need <= 32) return 7;
  return 2;
}

struct GKey {
  int dev, bytes, kind, rows32, nlog;
  bool operator<(const GKey& o) const {
    if (dev != o.dev) return dev < o.dev;
    if (bytes != o.bytes) return bytes < o.bytes;
    if (kind != o.kind) return kind < o.kind;
    if (rows32 != o.rows32) return rows32 < o.rows32;
    return nlog < o.nlog;
  }
};
std::mutex g_mu;
std::map<GKey, int> g_pick;

template <typename T, int NC>
hipError_t dispatch(const GCfg<T> (&cfg)[NC], int def, const GemmArgs<T>& g, hipStream_t s, bool tune, int force) {
  if (g.mode != 1) return cfg[def].fn(g, s);
  if (force >= 0 && force < NC) return cfg[force].fn(g, s);
  int nlog = 0;
  while ((1 << (nlog + 1)) <= g.N) ++nlog;
  int dev = 0;
  (void)hipGetDevice(&dev);
  const GKey key{dev, (int)sizeof(T), g.ops.kind, (g.M + 31) / 32, nlog};
  const char* fam = sizeof(T) == 8 ? "fp64" : "fp32";
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_pick.find(key);
  if (it != g_pick.end()) return cfg[it->second].fn(g, s);
  {
    const int c = tune_cache_get(fam, dev, (int)sizeof(T), g.ops.kind, (g.M + 31) / 32, nlog);
    if (c >= 0 && c < NC) {
      g_pick[key] = c;
      return cfg[c].fn(g, s);
    }
  }
  // candidates: the default, then every tile whose row padding stays within a quarter
  std::vector<int> cand{def};
  for (int i = 0; i < NC; ++i) {
    const int padded = (g.M + cfg[i].rows - 1) / cfg[i].rows * cfg[i].rows;
    if (i != def && 4 * padded <= 5 * g.M) cand.push_back(i);
  }
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (!tune || cand.size() < 2 || hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone)
    return cfg[def].fn(g, s);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t err = hipEventCreate(&e0);
  if (err == hipSuccess) err = hipEventCreate(&e1);
  int best = def;
  float best_ms = 0.f;
  for (size_t i = 0; i < cand.size() && err == hipSuccess; ++i) {
    err = cfg[cand[i]].fn(g, s);                      // warm run (same output bits)
    if (err == hipSuccess) err = hipEventRecord(e0, s);
    if (err == hipSuccess) err = cfg[cand[i]].fn(g, s);
    if (err == hipSuccess) err = hipEventRecord(e1, s);
    if (err == hipSuccess) err = hipEventSynchronize(e1);
    float ms = 0.f;
    if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
    if (err == hipSuccess && (i == 0 || ms < best_ms)) { best_ms = ms; best = cand[i]; }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (err != hipSuccess) return err;
  g_pick[key] = best;
  tune_cache_put(fam, dev, (int)sizeof(T), g.ops.kind, (g.M + 31) / 32, nlog, best);
  if (getenv("LTRIPLES_LOG"))
    fprintf(stderr, "[ltriples] tuned %s contraction (kind %d, M %d, N %d): tile rows %d (default %d)\n",
            sizeof(T) == 8 ? "FP64" : "FP32", g.ops.kind, g.M, g.N, cfg[best].rows, cfg[def].rows);
  return hipSuccess;
}

bool wide_contraction(const GemmArgs<float>& g) { return g.mode == 1 && g.M > 256 && g.N >= (1 << 15); }
bool wide_contraction(const GemmArgs<double>& g) { return g.mode == 1 && g.M > 256 && g.N >= (1 << 15); }

}  // namespace

template <> hipError_t launch_gemm<float>(const GemmArgs<float>& g, hipStream_t s, bool tune, int force) {
  return dispatch(kCfg32, wide_contraction(g) ? 1 : default32(g.M), g, s, tune, force);   // kCfg32[1]: 64 rows
}

template <> hipError_t launch_gemm<double>(const GemmArgs<double>& g, hipStream_t s, bool tune, int force) {
  return dispatch(kCfg64, wide_contraction(g) ? 1 : default64(g.M), g, s, tune, force);   // kCfg64[1]: 64 rows
}

void reset_gemm_tuning() {
  std::lock_guard<std::mutex> lk(g_mu);
  g_pick.clear();
}
#endif

}  // namespace lt
