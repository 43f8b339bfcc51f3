// Triplet contractions on the BF16 matrix cores with split-precision
// operands: every FP32 operand x is carried as hi = bf16(x) and
// lo = bf16(x - hi) (prepared once per call in octet layout), and each
// product is formed as hi*hi + hi*lo + lo*hi with FP32 accumulation
// (v_mfma_f32_32x32x16_bf16, three instructions per K step), or as the
// single hi*hi product for the plain-BF16 ablation.  The dropped lo*lo term
// and the rounding of lo leave a relative error of about 2^-16 per product.
//
// Tiling mirrors the FP32 kernel: 4 waves in a 2x2 grid, each owning
// MBW x NBW 32x32 blocks, the whole virtual range of the contraction in one
// work-group tile, K advancing by 16 (two octets) per double-buffered LDS
// stage; every global load is one 16-byte octet.
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <vector>

#include "lt_internal.h"

namespace lt {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ inline int64_t k16(int64_t k) { return (k + 15) & ~int64_t(15); }   // rows padded to 16

// Segment idx of the contraction of triplet (i, j, k); see item_seg in
// lt_gemm.hip for the equations (same terms, same order, same signs; kind 3
// is the closed-shell contraction over spatial orbitals).
// Blocks are indexed over the o_s (o_t) orbitals; occupied contraction rows
// (K) run over the first oi_s (oi_t), and the octet blocks of those operands
// hold exactly that many rows (padded to 16).
__device__ inline Seg8 item_seg8(const ItemOps8& s, int64_t i, int64_t j, int64_t k, int idx) {
  const int64_t o = s.o_s, v = s.v_s, ot = s.o_t, vt = s.v_t, oi = s.oi_s, oit = s.oi_t;
  const int64_t lv = s.ld_vs, lt_ = s.ld_vt, lp = s.ld_np, lc = s.ld_cb;
  const int64_t kv = k16(v), ko = k16(oi), kvt = k16(vt), kot = k16(oit);
  // block sizes (elements) of each octet tensor
  const int64_t bT2T = kv * lv, bAs = kv * lp, bGam = ko * lv, bTp = ko * lp;
  auto mk = [](const bf16_t* Lh, const bf16_t* Ll, int64_t lo, int64_t ll, const bf16_t* Rh, const bf16_t* Rl,
               int64_t ro, int64_t rl, int64_t K, float sg) -> Seg8 {
    return {Lh + lo, Ll + lo, ll * 8, Rh + ro, Rl + ro, rl * 8, (int32_t)K, sg};
  };
  if (s.kind == 0) {
    switch (idx) {
      case 0: return mk(s.T2Th, s.T2Tl, (j * o + k) * bT2T, lv, s.Ash, s.Asl, i * bAs, lp, v, 1.f);
      case 1: return mk(s.T2Th, s.T2Tl, (i * o + k) * bT2T, lv, s.Ash, s.Asl, j * bAs, lp, v, -1.f);
      case 2: return mk(s.T2Th, s.T2Tl, (j * o + i) * bT2T, lv, s.Ash, s.Asl, k * bAs, lp, v, -1.f);
      case 3: return mk(s.GamTh, s.GamTl, (j * o + k) * bGam, lv, s.Tph, s.Tpl, i * bTp, lp, oi, -1.f);
      case 4: return mk(s.GamTh, s.GamTl, (i * o + k) * bGam, lv, s.Tph, s.Tpl, j * bTp, lp, oi, 1.f);
      default: return mk(s.GamTh, s.GamTl, (j * o + i) * bGam, lv, s.Tph, s.Tpl, k * bTp, lp, oi, 1.f);
    }
  }
  if (s.kind == 3) {
    const int64_t lvv = s.ld_vv, bRV = kv * lvv, bTf = ko * lvv, bG = ko * lv;
    switch (idx) {
      case 0: return mk(s.T2Th, s.T2Tl, (i * o + j) * bT2T, lv, s.RVch, s.RVcl, k * bRV, lvv, v, 1.f);
      case 1: return mk(s.T2Th, s.T2Tl, (i * o + k) * bT2T, lv, s.RVsh, s.RVsl, j * bRV, lvv, v, 1.f);
      case 2: return mk(s.Gcsh, s.Gcsl, (k * o + i) * bG, lv, s.Tfh, s.Tfl, j * bTf, lvv, oi, -1.f);
      default: return mk(s.Gcsh, s.Gcsl, (j * o + i) * bG, lv, s.Tsh, s.Tsl, k * bTf, lvv, oi, -1.f);
    }
  }
  if (s.kind == 1) {
    const int64_t bLm = kvt * lv, bMst = kvt * lc, bMts = kv * lc, bTmx2 = ko * lc, bTmix = kot * lc,
                  bZp = kot * lv;
    switch (idx) {
      case 0: return mk(s.LmixTh, s.LmixTl, (i * ot + k) * bLm, lv, s.Msth, s.Mstl, j * bMst, lc, vt, 1.f);
      case 1: return mk(s.LmixTh, s.LmixTl, (j * ot + k) * bLm, lv, s.Msth, s.Mstl, i * bMst, lc, vt, -1.f);
      case 2: return mk(s.T2Th, s.T2Tl, (i * o + j) * bT2T, lv, s.Mtsh, s.Mtsl, k * bMts, lc, v, 1.f);
      case 3: return mk(s.GamTh, s.GamTl, (i * o + j) * bGam, lv, s.Tmx2h, s.Tmx2l, k * bTmx2, lc, oi, 1.f);
      case 4: return mk(s.ZpTh, s.ZpTl, (j * ot + k) * bZp, lv, s.Tmixh, s.Tmixl, i * bTmix, lc, oit, 1.f);
      default: return mk(s.ZpTh, s.ZpTl, (i * ot + k) * bZp, lv, s.Tmixh, s.Tmixl, j * bTmix, lc, oit, -1.f);
    }
  }
  const int64_t bTmT = kv * lt_, bOOT = ko * lt_;
  switch (idx) {
    case 0: return mk(s.TmTh, s.TmTl, (i * ot + k) * bTmT, lt_, s.Ash, s.Asl, j * bAs, lp, v, 1.f);
    case 1: return mk(s.TmTh, s.TmTl, (j * ot + k) * bTmT, lt_, s.Ash, s.Asl, i * bAs, lp, v, -1.f);
    case 2: return mk(s.OOTh, s.OOTl, (k * o + j) * bOOT, lt_, s.Tph, s.Tpl, i * bTp, lp, oi, -1.f);
    default: return mk(s.OOTh, s.OOTl, (k * o + i) * bOOT, lt_, s.Tph, s.Tpl, j * bTp, lp, oi, 1.f);
  }
}

__device__ inline bf16x8 as_bf16x8(uint4 u) { return __builtin_bit_cast(bf16x8, u); }

// Items per column-tile group: four work-groups per group in all (row tiles
// times items).  Measured on both domain sizes: for one row tile 4 items beat
// 8 by 3.5 % and 16 by 10 % (2 equal to 4); for two row tiles 2 items beat 4
// by 1 % and 8 by 20 %.
__host__ __device__ inline int items_per_group(int mt) { return mt >= 4 ? 1 : 4 / mt; }

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) const u32x4 guint4;   // global-memory octet

// Two work-groups per CU (two waves per SIMD): the compiler keeps the 160
// accumulators and the staged loads within 256 registers per lane, spilling
// a few address words; measured about 20% faster than one work-group per CU.

template <int MBW, int NBW, int WM, int NPROD>
__global__ __launch_bounds__(256, 2) void k_tgemm_bf16(GemmArgs16 g) {
  constexpr int BR = 32, BC = 32, BKQ = 2;      // 16 k per stage
  constexpr int WN = 4 / WM;
  constexpr int BM = WM * MBW * BR, BN = WN * NBW * BC;
  constexpr int AO = BKQ * BM, BO = BKQ * BN;   // octets per stage (each of hi, lo)
  constexpr int AVT = (2 * AO + 255) / 256, BVT = (2 * BO + 255) / 256;
  typedef float f32x16 __attribute__((ext_vector_type(16)));

  __shared__ uint4 As[2][2][BKQ][BM];   // [buf][hi/lo][q][m]
  __shared__ uint4 Bs[2][2][BKQ][BN];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  int b = blockIdx.x;
  {
    const int nblk = gridDim.x, x = b & 7, q = nblk >> 3, r = nblk & 7;
    b = (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + (b >> 3);
  }
  // the launch's items: one output shape, or chunks of several domains (the
  // chunk owning this work-group found by a search over their first
  // work-groups; all of it wave-uniform)
  int M = g.M, N = g.N, nbatch = g.nbatch, mt = g.mt, nt = g.nt;
  float* obase = g.out;
  int64_t obs = g.obs, ldo = g.ldo;
  const Seg8* tbase = g.tab;
  if (g.nchunk > 0) {
    int c = 0;
#pragma unroll
    for (int st = kMaxChunk16 / 2; st > 0; st >>= 1)
      if (c + st < g.nchunk && g.cblk[c + st] <= b) c += st;
    b -= g.cblk[c];
    M = g.ch[c].M; N = g.ch[c].N; nbatch = g.ch[c].nbatch;
    obase = g.ch[c].out; obs = g.ch[c].obs; ldo = g.ch[c].ldo; tbase = g.ch[c].tab;
    mt = (M + BM - 1) / BM; nt = (N + BN - 1) / BN;
  }
  // tile order: row tile, then GI consecutive items, then column tile, so the
  // work-groups in flight on one XCD share right-operand slices in its L2
  const int mtile = b % mt; b /= mt;
  const int GI = items_per_group(mt);
  const int ig = b % GI; b /= GI;
  const int ntile = b % nt; b /= nt;
  const int batch = b * GI + ig;
  if (batch >= nbatch) return;                   // whole work-group: before any barrier
  const int m0 = mtile * BM, n0 = ntile * BN;
  const Seg8* tab = tbase + (int64_t)batch * 6;   // read with wave-uniform (scalar) loads
  const int nseg = g.kind >= 2 ? 4 : 6;

  f32x16 acc[MBW][NBW];
#pragma unroll
  for (int mb = 0; mb < MBW; ++mb)
#pragma unroll
    for (int nb = 0; nb < NBW; ++nb)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[mb][nb][r] = 0.f;

  // Loads are unmasked: each octet tensor is zero-padded to 16 contraction
  // rows per block and carries slack past its last column, so whole-tile
  // loads stay in bounds, rows k >= K read zeros, and columns/rows past the
  // output shape only feed discarded outputs.  Each thread keeps 32-bit
  // offsets (in octets) from the segment's wave-uniform bases, set when the
  // segment changes and advanced by a constant per stage.
  // The lo array of every tensor lies after its hi array in the workspace
  // (less than 2^32 octets apart, checked by the planner), so a thread's
  // offset from the hi base covers both halves and no base is selected per
  // load.
  uint32_t oa[AVT], ob[BVT];
  guint4 *Lh = nullptr, *Rh = nullptr;
  uint32_t sa = 0, sb = 0, flip = 0;
  int K = 0;
  auto setseg = [&](int s) {
    const Seg8 sg = tab[s];
    K = sg.K;
    flip = sg.sign < 0.f ? 0x80008000u : 0u;
    sa = (uint32_t)(2 * sg.lq / 8); sb = (uint32_t)(2 * sg.rq / 8);
    Lh = (guint4*)sg.Lh; Rh = (guint4*)sg.Rh;
    const uint32_t dA = (uint32_t)((const uint4*)sg.Ll - (const uint4*)sg.Lh);
    const uint32_t dB = (uint32_t)((const uint4*)sg.Rl - (const uint4*)sg.Rh);
#pragma unroll
    for (int u = 0; u < AVT; ++u) {
      const int e = tid + u * 256, r = e % AO;
      oa[u] = (uint32_t)((r / BM) * (sg.lq / 8) + m0 + r % BM) + (e >= AO ? dA : 0u);
    }
#pragma unroll
    for (int u = 0; u < BVT; ++u) {
      const int e = tid + u * 256, r = e % BO;
      ob[u] = (uint32_t)((r / BN) * (sg.rq / 8) + n0 + r % BN) + (e >= BO ? dB : 0u);
    }
  };
  uint4 ra[AVT], rb[BVT];
  auto gload = [&]() {
#pragma unroll
    for (int u = 0; u < AVT; ++u) {
      const int e = tid + u * 256;
      if ((2 * AO) % 256 == 0 || e < 2 * AO) ra[u] = __builtin_bit_cast(uint4, Lh[oa[u]]);
      oa[u] += sa;
    }
#pragma unroll
    for (int u = 0; u < BVT; ++u) {
      const int e = tid + u * 256;
      if ((2 * BO) % 256 == 0 || e < 2 * BO) rb[u] = __builtin_bit_cast(uint4, Rh[ob[u]]);
      ob[u] += sb;
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int u = 0; u < AVT; ++u) {
      const int e = tid + u * 256;
      if ((2 * AO) % 256 == 0 || e < 2 * AO) {
        const int hl = e / AO, r = e % AO;
        uint4 v = ra[u];
        v.x ^= flip; v.y ^= flip; v.z ^= flip; v.w ^= flip;
        As[buf][hl][r / BM][r % BM] = v;
      }
    }
#pragma unroll
    for (int u = 0; u < BVT; ++u) {
      const int e = tid + u * 256;
      if ((2 * BO) % 256 == 0 || e < 2 * BO) {
        const int hl = e / BO, r = e % BO;
        Bs[buf][hl][r / BN][r % BN] = rb[u];
      }
    }
  };

  constexpr int BK = 8 * BKQ;
  int s = 0, k0 = 0;
  while (s < nseg && tab[s].K <= 0) ++s;
  if (s < nseg) { setseg(s); gload(); sstore(0); }
  __syncthreads();
  int cur = 0;
  const int arow = wm * MBW * BR + (lane & 31);
  const int bcol = wn * NBW * BC + (lane & 31);
  const int q = lane >> 5;
  while (s < nseg) {
    k0 += BK;
    if (k0 >= K) {
      ++s; k0 = 0;
      while (s < nseg && tab[s].K <= 0) ++s;
      if (s < nseg) setseg(s);
    }
    const bool more = s < nseg;
    if (more) gload();
    bf16x8 bh[NBW], bl[NBW];
#pragma unroll
    for (int nb = 0; nb < NBW; ++nb) {
      bh[nb] = as_bf16x8(Bs[cur][0][q][bcol + nb * BC]);
      if (NPROD == 3) bl[nb] = as_bf16x8(Bs[cur][1][q][bcol + nb * BC]);
    }
    // two row blocks at a time, product by product: between two MFMAs on the
    // same accumulator the pipe gets at least three independent ones (each
    // accumulator still sums lo*hi, hi*lo, hi*hi in that order)
#pragma unroll
    for (int m2 = 0; m2 < MBW; m2 += 2) {
      constexpr int P = 2;
      bf16x8 ah[P], al[P];
#pragma unroll
      for (int x = 0; x < P; ++x)
        if (m2 + x < MBW) {
          ah[x] = as_bf16x8(As[cur][0][q][arow + (m2 + x) * BR]);
          if (NPROD == 3) al[x] = as_bf16x8(As[cur][1][q][arow + (m2 + x) * BR]);
        }
      if (NPROD == 3) {
#pragma unroll
        for (int x = 0; x < P; ++x)
#pragma unroll
          for (int nb = 0; nb < NBW; ++nb)
            if (m2 + x < MBW)
              acc[m2 + x][nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[x], bh[nb], acc[m2 + x][nb], 0, 0, 0);
#pragma unroll
        for (int x = 0; x < P; ++x)
#pragma unroll
          for (int nb = 0; nb < NBW; ++nb)
            if (m2 + x < MBW)
              acc[m2 + x][nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[x], bl[nb], acc[m2 + x][nb], 0, 0, 0);
      }
#pragma unroll
      for (int x = 0; x < P; ++x)
#pragma unroll
        for (int nb = 0; nb < NBW; ++nb)
          if (m2 + x < MBW)
            acc[m2 + x][nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[x], bh[nb], acc[m2 + x][nb], 0, 0, 0);
    }
    if (more) sstore(cur ^ 1);
    __syncthreads();
    cur ^= 1;
  }

  float* out = obase + (int64_t)batch * obs;
#pragma unroll
  for (int nb = 0; nb < NBW; ++nb) {
    const int n = n0 + bcol + nb * BC;
    if (n >= N) continue;
#pragma unroll
    for (int mb = 0; mb < MBW; ++mb)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int m = m0 + wm * MBW * BR + mb * BR + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        if (m < M) out[(int64_t)m * ldo + n] = acc[mb][nb][r];
      }
  }
}

__global__ __launch_bounds__(256) void k_seg8_table(ItemOps8 ops, int32_t nitems, Seg8* tab) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)nitems * 6) return;
  const int64_t n = e / 6;
  const int sidx = (int)(e % 6);
  const int nseg = ops.kind >= 2 ? 4 : 6;
  const int32_t* it = ops.items + 3 * n;
  Seg8 sg{};
  if (sidx < nseg) sg = item_seg8(ops, it[0], it[1], it[2], sidx);
  else sg.K = 0;
  tab[e] = sg;
}

hipError_t launch_seg8_table(const ItemOps8& ops, int32_t nitems, Seg8* tab, hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  const int64_t n = (int64_t)nitems * 6;
  hipLaunchKernelGGL(k_seg8_table, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, ops, nitems, tab);
  return hipGetLastError();
}

template <int MBW, int NBW, int WM, int NPROD>
static hipError_t launch16(GemmArgs16 g, hipStream_t s) {
  constexpr int BM = WM * MBW * 32, BN = (4 / WM) * NBW * 32;
  auto groups = [](int64_t M, int64_t N, int64_t nb) {   // work-groups of one output shape
    const int64_t mt = (M + BM - 1) / BM, nt = (N + BN - 1) / BN, GI = items_per_group((int)mt);
    return mt * nt * ((nb + GI - 1) / GI) * GI;
  };
  g.mt = (g.M + BM - 1) / BM;
  g.nt = (g.N + BN - 1) / BN;
  int64_t nblk = 0;
  if (g.nchunk > 0) {
    if (g.nchunk > kMaxChunk16) return hipErrorInvalidValue;
    for (int c = 0; c < g.nchunk; ++c) {
      const Chunk16& h = g.ch[c];
      if (h.M <= 0 || h.N <= 0 || h.nbatch <= 0) return hipErrorInvalidValue;   // every chunk owns work-groups
      g.cblk[c] = (int32_t)nblk;
      nblk += groups(h.M, h.N, h.nbatch);
      if (nblk > 0x7fffffff) return hipErrorInvalidValue;
    }
    g.cblk[g.nchunk] = (int32_t)nblk;
  } else {
    nblk = groups(g.M, g.N, g.nbatch);
  }
  if (nblk <= 0) return hipSuccess;
  if (nblk > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_tgemm_bf16<MBW, NBW, WM, NPROD>), dim3((unsigned)nblk), dim3(256), 0, s, g);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Tile configurations and their selection.  Every configuration sums each
// output element over the same segments, k stages and products in the same
// order, so the choice changes no result bit, only the time.
// ---------------------------------------------------------------------------
namespace {

typedef hipError_t (*Fn16)(GemmArgs16, hipStream_t);
struct Cfg16 {
  int mbw, nbw, wm;
  Fn16 f1, f3;   // one product (plain BF16), three products (BF16x3)
};
const Cfg16 kCfg16[] = {
    {1, 1, 1, launch16<1, 1, 1, 1>, launch16<1, 1, 1, 3>}, {2, 1, 1, launch16<2, 1, 1, 1>, launch16<2, 1, 1, 3>},
    {3, 1, 1, launch16<3, 1, 1, 1>, launch16<3, 1, 1, 3>}, {2, 2, 2, launch16<2, 2, 2, 1>, launch16<2, 2, 2, 3>},
    {3, 2, 2, launch16<3, 2, 2, 1>, launch16<3, 2, 2, 3>}, {4, 2, 2, launch16<4, 2, 2, 1>, launch16<4, 2, 2, 3>},
    {5, 2, 2, launch16<5, 2, 2, 1>, launch16<5, 2, 2, 3>}, {6, 2, 2, launch16<6, 2, 2, 1>, launch16<6, 2, 2, 3>}};
constexpr int kNCfg = (int)(sizeof(kCfg16) / sizeof(kCfg16[0]));

int cfg_rows(int c) { return kCfg16[c].wm * kCfg16[c].mbw * 32; }

// The measured default for `need` 32-row blocks of output rows.
int default_cfg(int need) {
  if (need <= 1) return 0;
  if (need <= 2) return 1;
  if (need <= 3) return 2;
  if (need <= 4) return 3;
  if (need <= 6) return 4;
  if (need <= 8) return 5;
  if (need <= 10) return 6;
  if (need <= 12) return 7;
  return 5;   // several row tiles
}

// Candidates: the default first, then every configuration whose row tiles
// pad the rows by at most a quarter.
std::vector<int> candidates(int need) {
  std::vector<int> c{default_cfg(need)};
  const int rows = need * 32;
  for (int i = 0; i < kNCfg; ++i) {
    if (i == c[0]) continue;
    const int br = cfg_rows(i), padded = (rows + br - 1) / br * br;
    if (4 * padded <= 5 * rows) c.push_back(i);
  }
  return c;
}

struct TuneKey {
  int dev, nprod, kind, need, nlog;
  bool operator<(const TuneKey& o) const {
    if (dev != o.dev) return dev < o.dev;
    if (nprod != o.nprod) return nprod < o.nprod;
    if (kind != o.kind) return kind < o.kind;
    if (need != o.need) return need < o.need;
    return nlog < o.nlog;
  }
};
std::mutex g_tune_mu;
std::map<TuneKey, int> g_tuned;

hipError_t run_cfg(int c, const GemmArgs16& g, hipStream_t s) {
  return g.nprod == 3 ? kCfg16[c].f3(g, s) : kCfg16[c].f1(g, s);
}

}  // namespace

hipError_t launch_gemm_bf16(const GemmArgs16& g, hipStream_t s, bool tune, int force) {
  if (force >= 0 && force < kNCfg) return run_cfg(force, g, s);
  const int need = (g.M + 31) / 32;
  int nlog = 0;
  while ((1 << (nlog + 1)) <= g.N) ++nlog;
  int dev = 0;
  (void)hipGetDevice(&dev);
  const TuneKey key{dev, g.nprod, g.kind, need, nlog};
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tuned.find(key);
  if (it != g_tuned.end()) return run_cfg(it->second, g, s);
  {
    const int c = tune_cache_get("bf16", dev, g.nprod, g.kind, need, nlog);
    if (c >= 0 && c < kNCfg) {
      g_tuned[key] = c;
      return run_cfg(c, g, s);
    }
  }
  const std::vector<int> cand = candidates(need);
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (!tune || cand.size() < 2 || hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone)
    return run_cfg(cand[0], g, s);
  // time every candidate on this launch's own data (each run rewrites the
  // same output with the same bits): one warm run, one timed run
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t err = hipEventCreate(&e0);
  if (err == hipSuccess) err = hipEventCreate(&e1);
  int best = cand[0];
  float best_ms = 0.f;
  for (size_t i = 0; i < cand.size() && err == hipSuccess; ++i) {
    err = run_cfg(cand[i], g, s);
    if (err == hipSuccess) err = hipEventRecord(e0, s);
    if (err == hipSuccess) err = run_cfg(cand[i], g, s);
    if (err == hipSuccess) err = hipEventRecord(e1, s);
    if (err == hipSuccess) err = hipEventSynchronize(e1);
    float ms = 0.f;
    if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
    if (err == hipSuccess && (i == 0 || ms < best_ms)) { best_ms = ms; best = cand[i]; }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (err != hipSuccess) return err;
  g_tuned[key] = best;
  tune_cache_put("bf16", dev, g.nprod, g.kind, need, nlog, best);
  if (getenv("LTRIPLES_LOG"))
    fprintf(stderr, "[ltriples] tuned BF16 contraction (kind %d, M %d, N %d, %d products): tile %dx%d rows %d\n",
            g.kind, g.M, g.N, g.nprod, kCfg16[best].mbw, kCfg16[best].nbw, cfg_rows(best));
  return hipSuccess;   // the last candidate's run left the (identical) result in place
}

void reset_gemm_bf16_tuning() {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tuned.clear();
}

}  // namespace lt
