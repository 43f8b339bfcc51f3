// FP64 energy epilogue of the triples path.
//
// For one occupied triplet the contraction GEMMs leave, per output layout,
//   same spin:  S[a][p(b<c)]            W^{abc} = S[a][bc] - S[b][ac] + S[c][ab]   (a<b<c)
//   mixed:      G[a][C*v+b], Y[C][p(a<b)]  W^{abC} = G[a][Cb] - G[b][Ca] + Y[C][ab] (a<b)
// (the virtual permutation operator P(a/bc) resp. P(ab) applied by reading
// the intermediates at permuted indices).  A work-group takes a 16^3 tile of
// the unique virtual range, stages the permuted reads and the small FP64 V
// ingredients in LDS, forms W, V = V_t1 + V_f, D = e_i+e_j+e_k-e_a-e_b-e_c and
// accumulates W*W/D, W*V_t1/D, W*V_f/D in FP64, reduced over the wave by
// shuffles and over the work-group in LDS in a fixed order.  Each tile
// writes its own partial, so the later per-item sums are independent of
// scheduling.
#include <algorithm>

#include "lt_internal.h"

namespace lt {

__device__ inline double wave_sum(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

__device__ inline void block_write3(double e4, double est, double edt, double* dst) {
  __shared__ double red[4][3];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  e4 = wave_sum(e4); est = wave_sum(est); edt = wave_sum(edt);
  if (lane == 0) { red[wave][0] = e4; red[wave][1] = est; red[wave][2] = edt; }
  __syncthreads();
  if (threadIdx.x < 3) {
    const int q = threadIdx.x;
    dst[q] = ((red[0][q] + red[1][q]) + red[2][q]) + red[3][q];
  }
}

// tile triples A <= B <= C ordered by C, then B, then A
__device__ inline void tri_decode(int t, int& A, int& B, int& C) {
  int c = 0;
  while ((c + 1) * (c + 2) * (c + 3) / 6 <= t) ++c;
  t -= c * (c + 1) * (c + 2) / 6;
  int b = 0;
  while ((b + 1) * (b + 2) / 2 <= t) ++b;
  t -= b * (b + 1) / 2;
  A = t; B = b; C = c;
}

// Linear work-group id -> logical id such that consecutive logical ids run on
// one XCD (the dispatcher deals work-groups round-robin over the 8 XCDs).
// Neighbouring tiles read the two 64-byte halves of the same 128-byte lines,
// which then meet in that XCD's L2.
__device__ inline int xcd_logical(int w, int total) {
  const int x = w & 7, q = total >> 3, r = total & 7;
  return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + (w >> 3);
}

constexpr int SROW = ET * ET + 1;   // padded LDS row for [ta][tc*16+tb]

// 1/d by Newton-Raphson from the hardware reciprocal approximation: each step
// r <- r + r(1 - d r) squares the relative error, two steps reach FP64
// rounding (within an ulp or two of the correctly rounded quotient).  Valid
// for 1e-300 < |d| < 1e300; the host check on the orbital energies (gap of at
// least 1e-100, magnitudes at most 1e100) puts every denominator D in
// [-6e100, -3e-100], so no range test is needed per element.
__device__ inline double rcp64(double d) {
  double r = __builtin_amdgcn_rcp(d);
  double e = fma(-d, r, 1.0);
  r = fma(r, e, r);
  e = fma(-d, r, 1.0);
  return fma(r, e, r);
}

// With LAP (a central-orbital share) the staged virtual energies hold
// exp(-s ev) instead and the occupied part exp(s (e_i + e_j + e_k - ev_b)) times
// the point's weight, so each element's weight is a product, not a reciprocal.
template <typename T, bool LAP>
__global__ __launch_bounds__(256, 2) void k_epi_same(EpiSame<T> a) {
  // One work-group per (item, a-tile <= b-tile) walks the c-tiles from the
  // b-tile on; the operands of the next c-tile are loaded into registers while
  // the current one is computed, and the (a, b) and a-only operands are
  // staged once.  One FP64 partial per work-group.
  __shared__ T Sb[ET][SROW];        // S[b][p(a,c)]
  __shared__ T Sc[ET][SROW];        // S[c][p(a,b)]
  __shared__ double Uac[3][ET][ET + 1], Tac[3][ET][ET + 1];   // per c-tile
  __shared__ double Uba[3][ET][ET + 1], Tba[3][ET][ET + 1];   // once
  __shared__ double t1a[3][ET], fa[3][ET], eva[ET];
  __shared__ double t1cs[3][ET], fcs[3][ET], evcs[ET];         // per c-tile

  const int tid = threadIdx.x;
  const int L = xcd_logical(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);
  const int pi = L % gridDim.x;
  int TB = 0;
  while ((TB + 1) * (TB + 2) / 2 <= pi) ++TB;
  const int TA = pi - TB * (TB + 1) / 2;
  const int item = L / gridDim.x;
  const int32_t* it = a.items + 3 * item;
  const int occ[3] = {it[0], it[1], it[2]};
  const int v = a.v;
  double ls = 0.0, lw = 0.0;          // Laplace point and signed weight of this item
  if (LAP) {
    const int q = occ[a.lap_slot] - a.lap_o0;
    ls = a.lap[2 * q];
    lw = a.lap[2 * q + 1];
  }
  const int a0 = TA * ET, b0 = TB * ET;
  const T* S = a.S + (int64_t)item * a.s_item;
  const int64_t ldp = a.ld_np;
  // occupied pair (q, r), sign and t1 index of the three occupied permutations
  const int pq[3] = {occ[1], occ[0], occ[1]};
  const int pr[3] = {occ[2], occ[2], occ[0]};
  const double sg[3] = {1.0, -1.0, -1.0};
  const int64_t vv = (int64_t)v * v;
  int64_t ub[3], tb2[3];
#pragma unroll
  for (int pp = 0; pp < 3; ++pp) {
    ub[pp] = ((int64_t)pq[pp] * a.o + pr[pp]) * v * a.ld_v;
    tb2[pp] = ((int64_t)pq[pp] * a.o + pr[pp]) * vv;
  }

  // (a, b) and a-only operands
  for (int e = tid; e < 3 * ET * ET; e += 256) {
    const int pp = e / (ET * ET), r = e % (ET * ET), ta = r & 15, tx = r >> 4;
    const int aa = a0 + ta, bb = b0 + tx;
    const bool ba = aa < v && bb < v;
    Uba[pp][tx][ta] = ba ? a.U[ub[pp] + bb * a.ld_v + aa] : 0.0;
    Tba[pp][tx][ta] = ba ? a.t2[tb2[pp] + bb * v + aa] : 0.0;
  }
  if (tid < 3 * ET) {
    const int pp = tid / ET, ta = tid % ET, aa = a0 + ta;
    t1a[pp][ta] = aa < v ? a.t1[(int64_t)occ[pp] * v + aa] : 0.0;
    fa[pp][ta] = aa < v ? a.f[(int64_t)occ[pp] * v + aa] : 0.0;
  } else if (tid < 4 * ET) {
    const int ta = tid - 3 * ET, aa = a0 + ta;
    eva[ta] = aa < v ? (LAP ? exp(-ls * a.ev[aa]) : a.ev[aa]) : 0.0;
  }
  const int tb = tid & 15, tc = tid >> 4;
  const int b = b0 + tb;
  const bool brow = b < v;
  double t1b[3], fb[3];
#pragma unroll
  for (int pp = 0; pp < 3; ++pp) {
    t1b[pp] = brow ? sg[pp] * a.t1[(int64_t)occ[pp] * v + b] : 0.0;
    fb[pp] = brow ? sg[pp] * a.f[(int64_t)occ[pp] * v + b] : 0.0;
  }
  double dob = (a.eo[occ[0]] + a.eo[occ[1]] + a.eo[occ[2]]) - (brow ? a.ev[b] : 0.0);
  if (LAP) dob = lw * exp(ls * dob);
  const int na = min(ET, b - a0);

  // staging of one c-tile: elements tid + 256*u of the two permuted S blocks,
  // one element of each (a, c) block, one c-only value (threads 0..111), and
  // the thread's own (b, c) operands and direct-term run
  T rg[ET], ry[ET], rd[ET];
  double ruac[3], rtac[3], rUbc[3], rTbc[3], rcv;
  auto fetch = [&](int TCn) {
    const int c0 = TCn * ET;
#pragma unroll
    for (int u = 0; u < ET; ++u) {
      const int e = tid + 256 * u;
      const int ta = e & 15, tbb = (e >> 4) & 15, tcc = e >> 8;
      const int aa = a0 + ta, bb = b0 + tbb, cc = c0 + tcc;
      T x = 0, y = 0;
      if (cc < v && bb < v) {
        if (aa < cc) x = S[bb * ldp + (int64_t)cc * (cc - 1) / 2 + aa];
        if (aa < bb) y = S[cc * ldp + (int64_t)bb * (bb - 1) / 2 + aa];
      }
      rg[u] = x;
      ry[u] = y;
    }
    {
      const int ta = tid & 15, tx = tid >> 4, aa = a0 + ta, cc = c0 + tx;
      const bool ac = aa < v && cc < v;
#pragma unroll
      for (int pp = 0; pp < 3; ++pp) {
        ruac[pp] = ac ? a.U[ub[pp] + aa * a.ld_v + cc] : 0.0;
        rtac[pp] = ac ? a.t2[tb2[pp] + aa * v + cc] : 0.0;
      }
    }
    const int c = c0 + tc;
    const bool ok = brow && b < c && c < v;
#pragma unroll
    for (int pp = 0; pp < 3; ++pp) {
      rUbc[pp] = ok ? sg[pp] * a.U[ub[pp] + b * a.ld_v + c] : 0.0;
      rTbc[pp] = ok ? sg[pp] * a.t2[tb2[pp] + (int64_t)b * v + c] : 0.0;
    }
    {
      // c-only values: t1 (threads 0..47), f_ov (48..95), e_vir (96..111)
      const int x = tid & 15, cc = c0 + x, pp = (tid >> 4) % 3;
      rcv = 0.0;
      if (cc < v) {
        if (tid < 48) rcv = sg[pp] * a.t1[(int64_t)occ[pp] * v + cc];
        else if (tid < 96) rcv = sg[pp] * a.f[(int64_t)occ[pp] * v + cc];
        else if (tid < 112) rcv = LAP ? exp(-ls * a.ev[cc]) : a.ev[cc];
      }
    }
    const T* Srow = S + (int64_t)c * (c - 1) / 2 + b;
#pragma unroll
    for (int ta = 0; ta < ET; ++ta) rd[ta] = (ok && ta < na) ? Srow[(a0 + ta) * ldp] : (T)0;
  };

  double e4 = 0.0, est = 0.0, edt = 0.0;
  fetch(TB);
  for (int TC = TB; TC < a.nt; ++TC) {
    __syncthreads();                 // previous tile's LDS reads are done (first pass: nothing)
#pragma unroll
    for (int u = 0; u < ET; ++u) {
      const int e = tid + 256 * u;
      Sb[e & 15][(e >> 8) * ET + ((e >> 4) & 15)] = rg[u];
      Sc[e & 15][(e >> 8) * ET + ((e >> 4) & 15)] = ry[u];
    }
#pragma unroll
    for (int pp = 0; pp < 3; ++pp) {
      Uac[pp][tid & 15][tid >> 4] = ruac[pp];
      Tac[pp][tid & 15][tid >> 4] = rtac[pp];
    }
    if (tid < 48) t1cs[(tid >> 4) % 3][tid & 15] = rcv;
    else if (tid < 96) fcs[(tid >> 4) % 3][tid & 15] = rcv;
    else if (tid < 112) evcs[tid & 15] = rcv;
    double Ubc[3], Tbc[3];
#pragma unroll
    for (int pp = 0; pp < 3; ++pp) { Ubc[pp] = rUbc[pp]; Tbc[pp] = rTbc[pp]; }
    const int c = TC * ET + tc;
    const bool ok = brow && b < c && c < v;
    T sd[ET];
#pragma unroll
    for (int ta = 0; ta < ET; ++ta) sd[ta] = rd[ta];
    __syncthreads();
    double t1c[3], fc[3];
#pragma unroll
    for (int pp = 0; pp < 3; ++pp) { t1c[pp] = t1cs[pp][tc]; fc[pp] = fcs[pp][tc]; }
    const double dbc = LAP ? dob * evcs[tc] : dob - evcs[tc];
    if (TC + 1 < a.nt) fetch(TC + 1);   // next tile's loads in flight during this tile's work
    if (ok) {
      for (int ta = 0; ta < na; ++ta) {
        const double w = (double)sd[ta] - (double)Sb[ta][tc * ET + tb] + (double)Sc[ta][tc * ET + tb];
        double vt = 0.0, vf = 0.0;
#pragma unroll
        for (int pp = 0; pp < 3; ++pp) {
          vt += t1a[pp][ta] * Ubc[pp] - t1b[pp] * Uac[pp][ta][tc] - t1c[pp] * Uba[pp][tb][ta];
          vf += fa[pp][ta] * Tbc[pp] - fb[pp] * Tac[pp][ta][tc] - fc[pp] * Tba[pp][tb][ta];
        }
        const double wd = w * (LAP ? dbc * eva[ta] : rcp64(dbc - eva[ta]));
        e4 += wd * w;
        est += wd * vt;
        edt += wd * vf;
      }
    }
  }
  block_write3(e4, est, edt, a.part + ((int64_t)item * a.ntri + pi) * 3);
}

// Mixed blocks: one work-group per (item, a-tile <= b-tile) walks all C
// tiles; the operands of the next C tile are loaded into registers while the
// current one is computed (software pipelining), and the C-independent
// operands (t1, f_ov, e_vir of the a-tile, <ij||ab>, t^{ab}_{ij}) are staged
// once.  Thread (b, C) of a tile loops over the tile's a < b; each thread's
// FP64 partial sums run over all C tiles and one partial per work-group is
// written.
template <typename T, bool LAP>
__global__ __launch_bounds__(256) void k_epi_mixed(EpiMixed<T> a) {
  __shared__ T Gb[ET][SROW];        // G[b][C*v+a]
  __shared__ T Yl[ET][SROW];        // Y[C][p(a,b)]
  __shared__ double OVj[ET][ET + 1], OVi[ET][ET + 1], Tmj[ET][ET + 1], Tmi[ET][ET + 1];
  __shared__ double Uab[ET][ET + 1], T2ab[ET][ET + 1];
  __shared__ double t1ai[ET], t1aj[ET], fai[ET], faj[ET], eva[ET];

  const int tid = threadIdx.x;
  const int L = xcd_logical(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);
  const int pi = L % gridDim.x;
  int TB = 0;
  while ((TB + 1) * (TB + 2) / 2 <= pi) ++TB;
  const int TA = pi - TB * (TB + 1) / 2;
  const int item = L / gridDim.x;
  const int32_t* it = a.items + 3 * item;
  const int i = it[0], j = it[1], K = it[2];
  const int vs = a.v_s, vt = a.v_t;
  const int a0 = TA * ET, b0 = TB * ET;
  double ls = 0.0, lw = 0.0;          // Laplace point and signed weight (as k_epi_same)
  if (LAP) {
    const int q = it[a.lap_slot] - a.lap_o0;
    ls = a.lap[2 * q];
    lw = a.lap[2 * q + 1];
  }
  const T* G = a.G + (int64_t)item * a.g_item;
  const T* Y = a.Y + (int64_t)item * a.y_item;
  const int64_t lc = a.ld_cb, lp = a.ld_np;

  // C-independent operands
  {
    const int64_t ij = (int64_t)i * a.o_s + j;
    const int tx = tid & 15, ta = tid >> 4, aa = a0 + ta, bb = b0 + tx;
    const bool ab = aa < vs && bb < vs;
    Uab[tx][ta] = ab ? a.U[(ij * vs + aa) * a.ld_vs + bb] : 0.0;
    T2ab[tx][ta] = ab ? a.t2ss[(ij * vs + aa) * vs + bb] : 0.0;
  }
  if (tid < ET) {
    const int aa = a0 + tid;
    const bool ok = aa < vs;
    t1ai[tid] = ok ? a.t1_s[(int64_t)i * vs + aa] : 0.0;
    t1aj[tid] = ok ? a.t1_s[(int64_t)j * vs + aa] : 0.0;
    fai[tid] = ok ? a.f_s[(int64_t)i * vs + aa] : 0.0;
    faj[tid] = ok ? a.f_s[(int64_t)j * vs + aa] : 0.0;
    eva[tid] = ok ? (LAP ? exp(-ls * a.ev_s[aa]) : a.ev_s[aa]) : 0.0;
  }
  const int tb = tid & 15, tc = tid >> 4;
  const int b = b0 + tb;
  const bool brow = b < vs;
  const double t1bi = brow ? a.t1_s[(int64_t)i * vs + b] : 0.0, t1bj = brow ? a.t1_s[(int64_t)j * vs + b] : 0.0;
  const double fbi = brow ? a.f_s[(int64_t)i * vs + b] : 0.0, fbj = brow ? a.f_s[(int64_t)j * vs + b] : 0.0;
  double dob = (a.eo_s[i] + a.eo_s[j] + a.eo_t[K]) - (brow ? a.ev_s[b] : 0.0);
  if (LAP) dob = lw * exp(ls * dob);
  const int na = min(ET, b - a0);
  // staging of one C tile: thread tid stages elements tid + 256*u of the
  // permuted G block and of Y, one element of each small FP64 block, and its
  // own direct-term run
  const bool ovc = a.ov_V == 1, tmc = a.tm_V == 1;
  const int ov_ta = ovc ? tid >> 4 : tid & 15, ov_tx = ovc ? tid & 15 : tid >> 4;
  const int tm_ta = tmc ? tid >> 4 : tid & 15, tm_tx = tmc ? tid & 15 : tid >> 4;
  T rg[ET], ry[ET], rd[ET];
  double rovj, rovi, rtmj, rtmi, rOVjb, rOVib, rTmjb, rTmib, rt1C, rfC, revC;
  auto fetch = [&](int TCn) {
    const int c0 = TCn * ET;
#pragma unroll
    for (int u = 0; u < ET; ++u) {
      const int e = tid + 256 * u;
      const int ta = e & 15, tbb = (e >> 4) & 15, tcc = e >> 8;
      const int aa = a0 + ta, bb = b0 + tbb, cc = c0 + tcc;
      T x = 0, y = 0;
      if (aa < vs && bb < vs && cc < vt) {
        x = G[bb * lc + (int64_t)cc * vs + aa];
        if (aa < bb) y = Y[cc * lp + (int64_t)bb * (bb - 1) / 2 + aa];
      }
      rg[u] = x;
      ry[u] = y;
    }
    {
      const int aa = a0 + ov_ta, cc = c0 + ov_tx;
      const bool ac = aa < vs && cc < vt;
      rovj = ac ? a.ov[j * a.ov_o + aa * a.ov_v + K * a.ov_O + cc * a.ov_V] : 0.0;
      rovi = ac ? a.ov[i * a.ov_o + aa * a.ov_v + K * a.ov_O + cc * a.ov_V] : 0.0;
    }
    {
      const int aa = a0 + tm_ta, cc = c0 + tm_tx;
      const bool ac = aa < vs && cc < vt;
      rtmj = ac ? a.tm[j * a.tm_o + aa * a.tm_v + K * a.tm_O + cc * a.tm_V] : 0.0;
      rtmi = ac ? a.tm[i * a.tm_o + aa * a.tm_v + K * a.tm_O + cc * a.tm_V] : 0.0;
    }
    const int C = c0 + tc;
    const bool ok = brow && C < vt;
    rOVjb = ok ? a.ov[j * a.ov_o + b * a.ov_v + K * a.ov_O + C * a.ov_V] : 0.0;
    rOVib = ok ? a.ov[i * a.ov_o + b * a.ov_v + K * a.ov_O + C * a.ov_V] : 0.0;
    rTmjb = ok ? a.tm[j * a.tm_o + b * a.tm_v + K * a.tm_O + C * a.tm_V] : 0.0;
    rTmib = ok ? a.tm[i * a.tm_o + b * a.tm_v + K * a.tm_O + C * a.tm_V] : 0.0;
    rt1C = ok ? a.t1_t[(int64_t)K * vt + C] : 0.0;
    rfC = ok ? a.f_t[(int64_t)K * vt + C] : 0.0;
    revC = ok ? (LAP ? exp(-ls * a.ev_t[C]) : a.ev_t[C]) : 0.0;
    const T* Grow = G + (int64_t)C * vs + b;
#pragma unroll
    for (int ta = 0; ta < ET; ++ta) rd[ta] = (ok && ta < na) ? Grow[(a0 + ta) * lc] : (T)0;
  };

  double e4 = 0.0, est = 0.0, edt = 0.0;
  fetch(0);
  for (int TC = 0; TC < a.ntt; ++TC) {
    __syncthreads();                 // previous tile's LDS reads are done
#pragma unroll
    for (int u = 0; u < ET; ++u) {
      const int e = tid + 256 * u;
      Gb[e & 15][(e >> 8) * ET + ((e >> 4) & 15)] = rg[u];
      Yl[e & 15][(e >> 8) * ET + ((e >> 4) & 15)] = ry[u];
    }
    OVj[ov_ta][ov_tx] = rovj; OVi[ov_ta][ov_tx] = rovi;
    Tmj[tm_ta][tm_tx] = rtmj; Tmi[tm_ta][tm_tx] = rtmi;
    const double OVjb = rOVjb, OVib = rOVib, Tmjb = rTmjb, Tmib = rTmib, t1C = rt1C, fC = rfC;
    const double dbc = LAP ? dob * revC : dob - revC;
    const bool ok = brow && TC * ET + tc < vt;
    T gd[ET];
#pragma unroll
    for (int ta = 0; ta < ET; ++ta) gd[ta] = rd[ta];
    __syncthreads();
    if (TC + 1 < a.ntt) fetch(TC + 1);   // next tile's loads in flight during this tile's work
    if (ok) {
#pragma unroll
      for (int ta = 0; ta < ET; ++ta) {
        if (ta >= na) break;
        const double w = (double)gd[ta] - (double)Gb[ta][tc * ET + tb] + (double)Yl[ta][tc * ET + tb];
        const double vt1 = t1ai[ta] * OVjb - t1aj[ta] * OVib - t1bi * OVj[ta][tc] + t1bj * OVi[ta][tc]
                           + t1C * Uab[tb][ta];
        const double vfo = fai[ta] * Tmjb - faj[ta] * Tmib - fbi * Tmj[ta][tc] + fbj * Tmi[ta][tc]
                           + fC * T2ab[tb][ta];
        const double wd = w * (LAP ? dbc * eva[ta] : rcp64(dbc - eva[ta]));
        e4 += wd * w;
        est += wd * vt1;
        edt += wd * vfo;
      }
    }
  }
  block_write3(e4, est, edt, a.part + ((int64_t)item * a.ntiles + pi) * 3);
}

// ---------------------------------------------------------------------------
// Backward epilogues.  Same tiles and LDS staging as the forward ones; per
// unique virtual triple W, V, D are recomputed and the adjoints
// gbar (2W + V)/D and gbar W/D are scattered to the three (same spin) resp.
// three (mixed) output positions that W and V read, with the signs of the
// permutation operator.  Output positions that W never reads (an index
// repeated) are written with zeros by the tile that owns them, so every
// element of an item's output layout is written exactly once.
// ---------------------------------------------------------------------------
__device__ inline int64_t pidx(int x, int y) { return (int64_t)y * (y - 1) / 2 + x; }   // x < y

// Tile sums of q for the orbital-energy adjoint.  Thread (tb, tc) = (tid & 15,
// tid >> 4) holds qa[ta] for its elements and qbc = sum_ta qa[ta].  out gets
// the sums over the tile with the first index fixed (out[ta]), the second
// (out[16 + tb]), the third (out[32 + tc]) and the total (out[48]).  The
// first-index sums leave each wave by transpose-and-add: four exchanges
// halve the sixteen values per lane (lane l ends with index (l >> 2) & 15
// over sixteen lanes), two more add the remaining four lanes.  Every sum
// has a fixed order.  All 256 threads must call this; `lds` (336 doubles)
// may alias staging memory of the caller, which is not read afterwards.
__device__ inline void eps_tile_sums(const double (&qa)[ET], double qbc, double* out, double* lds) {
  double *red = lds, *qs = lds + 4 * ET, *rc = lds + 4 * ET + 256;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double y[8], z[4], u[2];
  {
    const bool hi = lane & 32;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const double keep = hi ? qa[k + 8] : qa[k], send = hi ? qa[k] : qa[k + 8];
      y[k] = keep + __shfl_xor(send, 32);
    }
  }
  {
    const bool hi = lane & 16;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const double keep = hi ? y[k + 4] : y[k], send = hi ? y[k] : y[k + 4];
      z[k] = keep + __shfl_xor(send, 16);
    }
  }
  {
    const bool hi = lane & 8;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const double keep = hi ? z[k + 2] : z[k], send = hi ? z[k] : z[k + 2];
      u[k] = keep + __shfl_xor(send, 8);
    }
  }
  double w;
  {
    const bool hi = lane & 4;
    const double keep = hi ? u[1] : u[0], send = hi ? u[0] : u[1];
    w = keep + __shfl_xor(send, 4);
  }
  w += __shfl_xor(w, 2);
  w += __shfl_xor(w, 1);
  __syncthreads();                     // every wave is done with the aliased staging
  if ((lane & 3) == 0) red[wave * ET + (lane >> 2)] = w;
  qs[tid] = qbc;
  __syncthreads();
  if (tid < ET) {
    out[tid] = ((red[tid] + red[ET + tid]) + red[2 * ET + tid]) + red[3 * ET + tid];
  } else if (tid < 2 * ET) {
    const int r = tid - ET;
    double acc = 0.0;
    for (int tc = 0; tc < ET; ++tc) acc += qs[r + ET * tc];
    out[ET + r] = acc;
  } else if (tid < 3 * ET) {
    const int r = tid - 2 * ET;
    double acc = 0.0;
    for (int tb = 0; tb < ET; ++tb) acc += qs[tb + ET * r];
    out[2 * ET + r] = acc;
    rc[r] = acc;
  }
  __syncthreads();
  if (tid == 0) {
    double acc = 0.0;
    for (int r = 0; r < ET; ++r) acc += rc[r];
    out[3 * ET] = acc;
  }
}

template <typename T, bool EPS>
__global__ __launch_bounds__(256) void k_bwd_same(BwdSame<T> A) {
  const EpiSame<T>& a = A.e;
  __shared__ T Sb[ET][SROW];
  __shared__ T Sc[ET][SROW];
  __shared__ double Uac[3][ET][ET + 1], Uba[3][ET][ET + 1], Tac[3][ET][ET + 1], Tba[3][ET][ET + 1];
  __shared__ double t1a[3][ET], fa[3][ET], eva[ET];

  const int tid = threadIdx.x;
  int TA, TB, TC;
  tri_decode(blockIdx.x, TA, TB, TC);
  const int item = blockIdx.y;
  const int32_t* it = a.items + 3 * item;
  const int occ[3] = {it[0], it[1], it[2]};
  const int v = a.v;
  const int a0 = TA * ET, b0 = TB * ET, c0 = TC * ET;
  const T* S = a.S + (int64_t)item * a.s_item;
  T* dS = A.dS + (int64_t)item * a.s_item;
  T* dSV = A.dSV + (int64_t)item * a.s_item;
  const int64_t ldp = a.ld_np;
  const int pq[3] = {occ[1], occ[0], occ[1]};
  const int pr[3] = {occ[2], occ[2], occ[0]};
  const double sg[3] = {1.0, -1.0, -1.0};
  const int64_t vv = (int64_t)v * v;

  for (int e = tid; e < ET * ET * ET; e += 256) {
    const int ta = e & 15, tb = (e >> 4) & 15, tc = e >> 8;
    const int aa = a0 + ta, bb = b0 + tb, cc = c0 + tc;
    T x = 0, y = 0;
    if (cc < v && bb < v) {
      if (aa < cc) x = S[bb * ldp + pidx(aa, cc)];
      if (aa < bb) y = S[cc * ldp + pidx(aa, bb)];
    }
    Sb[ta][tc * ET + tb] = x;
    Sc[ta][tc * ET + tb] = y;
  }
  for (int e = tid; e < 3 * ET * ET; e += 256) {
    const int pp = e / (ET * ET), r = e % (ET * ET), ta = r & 15, tx = r >> 4;
    const int aa = a0 + ta, cc = c0 + tx, bb = b0 + tx;
    const int64_t ub = ((int64_t)pq[pp] * a.o + pr[pp]) * v * a.ld_v;
    const int64_t tb_ = ((int64_t)pq[pp] * a.o + pr[pp]) * vv;
    const bool ac = aa < v && cc < v, ba = aa < v && bb < v;
    Uac[pp][ta][tx] = ac ? a.U[ub + aa * a.ld_v + cc] : 0.0;
    Tac[pp][ta][tx] = ac ? a.t2[tb_ + aa * v + cc] : 0.0;
    Uba[pp][tx][ta] = ba ? a.U[ub + bb * a.ld_v + aa] : 0.0;
    Tba[pp][tx][ta] = ba ? a.t2[tb_ + bb * v + aa] : 0.0;
  }
  if (tid < 3 * ET) {
    const int pp = tid / ET, ta = tid % ET, aa = a0 + ta;
    t1a[pp][ta] = aa < v ? a.t1[(int64_t)occ[pp] * v + aa] : 0.0;
    fa[pp][ta] = aa < v ? a.f[(int64_t)occ[pp] * v + aa] : 0.0;
  } else if (tid < 4 * ET) {
    const int ta = tid - 3 * ET, aa = a0 + ta;
    eva[ta] = aa < v ? a.ev[aa] : 0.0;
  }
  __syncthreads();

  const int tb = tid & 15, tc = tid >> 4;
  const int b = b0 + tb, c = c0 + tc;
  double qa[ET], qbc = 0.0;
  if constexpr (EPS) {
#pragma unroll
    for (int ta = 0; ta < ET; ++ta) qa[ta] = 0.0;
  }
  if (b < c && c < v) {
    const double g = A.gbar[0];
    double Ubc[3], Tbc[3], t1b[3], fb[3], t1c[3], fc[3];
#pragma unroll
    for (int pp = 0; pp < 3; ++pp) {
      const int64_t blk = (int64_t)pq[pp] * a.o + pr[pp];
      Ubc[pp] = sg[pp] * a.U[blk * v * a.ld_v + b * a.ld_v + c];
      Tbc[pp] = sg[pp] * a.t2[blk * vv + (int64_t)b * v + c];
      t1b[pp] = sg[pp] * a.t1[(int64_t)occ[pp] * v + b];
      fb[pp] = sg[pp] * a.f[(int64_t)occ[pp] * v + b];
      t1c[pp] = sg[pp] * a.t1[(int64_t)occ[pp] * v + c];
      fc[pp] = sg[pp] * a.f[(int64_t)occ[pp] * v + c];
    }
    const double dbc = (a.eo[occ[0]] + a.eo[occ[1]] + a.eo[occ[2]]) - a.ev[b] - a.ev[c];
    const int64_t pbc = pidx(b, c);
    const T* Srow = S + pbc;
    const int na = min(ET, b - a0);
    // one element (a0 + ta, b, c); returns q = gbar W (W + V) / D^2
    auto elem = [&](int ta) -> double {
      const int aa = a0 + ta;
      const double w = (double)Srow[aa * ldp] - (double)Sb[ta][tc * ET + tb] + (double)Sc[ta][tc * ET + tb];
      double vt = 0.0, vf = 0.0;
#pragma unroll
      for (int pp = 0; pp < 3; ++pp) {
        vt += t1a[pp][ta] * Ubc[pp] - t1b[pp] * Uac[pp][ta][tc] - t1c[pp] * Uba[pp][tb][ta];
        vf += fa[pp][ta] * Tbc[pp] - fb[pp] * Tac[pp][ta][tc] - fc[pp] * Tba[pp][tb][ta];
      }
      const double rd = rcp64(dbc - eva[ta]);
      const double wh = g * (2.0 * w + vt + vf) * rd, vh = g * w * rd;
      // W = S[a][bc] - S[b][ac] + S[c][ab]; V likewise from the singles/f_ov intermediate
      dS[aa * ldp + pbc] = (T)wh;
      dS[b * ldp + pidx(aa, c)] = (T)(-wh);
      dS[c * ldp + pidx(aa, b)] = (T)wh;
      dSV[aa * ldp + pbc] = (T)vh;
      dSV[b * ldp + pidx(aa, c)] = (T)(-vh);
      dSV[c * ldp + pidx(aa, b)] = (T)vh;
      return vh * (w + vt + vf) * rd;
    };
    if constexpr (EPS) {
#pragma unroll
      for (int ta = 0; ta < ET; ++ta)
        if (ta < na) {
          const double q = elem(ta);
          qa[ta] = q;
          qbc += q;
        }
    } else {
      for (int ta = 0; ta < na; ++ta) (void)elem(ta);
    }
    if (TA == TB) {
      dS[b * ldp + pbc] = (T)0; dS[c * ldp + pbc] = (T)0;
      dSV[b * ldp + pbc] = (T)0; dSV[c * ldp + pbc] = (T)0;
    }
  }
  if constexpr (EPS) {
    static_assert(sizeof(Sb) >= 336 * sizeof(double), "tile-sum scratch must fit the staging tile");
    eps_tile_sums(qa, qbc, A.ep + ((int64_t)item * gridDim.x + blockIdx.x) * 64, (double*)&Sb[0][0]);
  }
}

template <typename T, bool EPS>
__global__ __launch_bounds__(256) void k_bwd_mixed(BwdMixed<T> A) {
  const EpiMixed<T>& a = A.e;
  __shared__ T Gb[ET][SROW];
  __shared__ T Yl[ET][SROW];
  __shared__ double OVj[ET][ET + 1], OVi[ET][ET + 1], Tmj[ET][ET + 1], Tmi[ET][ET + 1];
  __shared__ double Uab[ET][ET + 1], T2ab[ET][ET + 1];
  __shared__ double t1ai[ET], t1aj[ET], fai[ET], faj[ET], eva[ET];

  const int tid = threadIdx.x;
  const int tile = blockIdx.x;
  const int TC = tile % a.ntt, pi = tile / a.ntt;
  int TB = 0;
  while ((TB + 1) * (TB + 2) / 2 <= pi) ++TB;
  const int TA = pi - TB * (TB + 1) / 2;
  const int item = blockIdx.y;
  const int32_t* it = a.items + 3 * item;
  const int i = it[0], j = it[1], K = it[2];
  const int vs = a.v_s, vt = a.v_t;
  const int a0 = TA * ET, b0 = TB * ET, c0 = TC * ET;
  const T* G = a.G + (int64_t)item * a.g_item;
  const T* Y = a.Y + (int64_t)item * a.y_item;
  T* dG = A.dG + (int64_t)item * a.g_item;
  T* dGV = A.dGV + (int64_t)item * a.g_item;
  T* dY = A.dY + (int64_t)item * a.y_item;
  T* dYV = A.dYV + (int64_t)item * a.y_item;
  const int64_t lc = a.ld_cb, lp = a.ld_np;

  for (int e = tid; e < ET * ET * ET; e += 256) {
    const int ta = e & 15, tb = (e >> 4) & 15, tc = e >> 8;
    const int aa = a0 + ta, bb = b0 + tb, cc = c0 + tc;
    T x = 0, y = 0;
    if (aa < vs && bb < vs && cc < vt) {
      x = G[bb * lc + (int64_t)cc * vs + aa];
      if (aa < bb) y = Y[cc * lp + pidx(aa, bb)];
    }
    Gb[ta][tc * ET + tb] = x;
    Yl[ta][tc * ET + tb] = y;
  }
  for (int e = tid; e < ET * ET; e += 256) {
    const int ta = e & 15, tx = e >> 4;
    const int aa = a0 + ta, cc = c0 + tx, bb = b0 + tx;
    const bool ac = aa < vs && cc < vt, ab = aa < vs && bb < vs;
    OVj[ta][tx] = ac ? a.ov[j * a.ov_o + aa * a.ov_v + K * a.ov_O + cc * a.ov_V] : 0.0;
    OVi[ta][tx] = ac ? a.ov[i * a.ov_o + aa * a.ov_v + K * a.ov_O + cc * a.ov_V] : 0.0;
    Tmj[ta][tx] = ac ? a.tm[j * a.tm_o + aa * a.tm_v + K * a.tm_O + cc * a.tm_V] : 0.0;
    Tmi[ta][tx] = ac ? a.tm[i * a.tm_o + aa * a.tm_v + K * a.tm_O + cc * a.tm_V] : 0.0;
    const int64_t ij = (int64_t)i * a.o_s + j;
    Uab[tx][ta] = ab ? a.U[(ij * vs + aa) * a.ld_vs + bb] : 0.0;
    T2ab[tx][ta] = ab ? a.t2ss[(ij * vs + aa) * vs + bb] : 0.0;
  }
  if (tid < ET) {
    const int aa = a0 + tid;
    const bool ok = aa < vs;
    t1ai[tid] = ok ? a.t1_s[(int64_t)i * vs + aa] : 0.0;
    t1aj[tid] = ok ? a.t1_s[(int64_t)j * vs + aa] : 0.0;
    fai[tid] = ok ? a.f_s[(int64_t)i * vs + aa] : 0.0;
    faj[tid] = ok ? a.f_s[(int64_t)j * vs + aa] : 0.0;
    eva[tid] = ok ? a.ev_s[aa] : 0.0;
  }
  __syncthreads();

  const int tb = tid & 15, tc = tid >> 4;
  const int b = b0 + tb, C = c0 + tc;
  double qa[ET], qbc = 0.0;
  if constexpr (EPS) {
#pragma unroll
    for (int ta = 0; ta < ET; ++ta) qa[ta] = 0.0;
  }
  if (b < vs && C < vt) {
    const double g = A.gbar[0];
    const double OVjb = a.ov[j * a.ov_o + b * a.ov_v + K * a.ov_O + C * a.ov_V];
    const double OVib = a.ov[i * a.ov_o + b * a.ov_v + K * a.ov_O + C * a.ov_V];
    const double Tmjb = a.tm[j * a.tm_o + b * a.tm_v + K * a.tm_O + C * a.tm_V];
    const double Tmib = a.tm[i * a.tm_o + b * a.tm_v + K * a.tm_O + C * a.tm_V];
    const double t1bi = a.t1_s[(int64_t)i * vs + b], t1bj = a.t1_s[(int64_t)j * vs + b];
    const double fbi = a.f_s[(int64_t)i * vs + b], fbj = a.f_s[(int64_t)j * vs + b];
    const double t1C = a.t1_t[(int64_t)K * vt + C], fC = a.f_t[(int64_t)K * vt + C];
    const double dbc = (a.eo_s[i] + a.eo_s[j] + a.eo_t[K]) - a.ev_s[b] - a.ev_t[C];
    const T* Grow = G + (int64_t)C * vs + b;
    const int64_t cb = (int64_t)C * vs;
    const int na = min(ET, b - a0);
    // one element (a0 + ta, b, C); returns q = gbar W (W + V) / D^2
    auto elem = [&](int ta) -> double {
      const int aa = a0 + ta;
      const double w = (double)Grow[aa * lc] - (double)Gb[ta][tc * ET + tb] + (double)Yl[ta][tc * ET + tb];
      const double vt1 = t1ai[ta] * OVjb - t1aj[ta] * OVib - t1bi * OVj[ta][tc] + t1bj * OVi[ta][tc]
                         + t1C * Uab[tb][ta];
      const double vfo = fai[ta] * Tmjb - faj[ta] * Tmib - fbi * Tmj[ta][tc] + fbj * Tmi[ta][tc]
                         + fC * T2ab[tb][ta];
      const double rd = rcp64(dbc - eva[ta]);
      const double wh = g * (2.0 * w + vt1 + vfo) * rd, vh = g * w * rd;
      // W = G[a][Cb] - G[b][Ca] + Y[C][ab]
      dG[aa * lc + cb + b] = (T)wh;
      dG[b * lc + cb + aa] = (T)(-wh);
      dY[C * lp + pidx(aa, b)] = (T)wh;
      dGV[aa * lc + cb + b] = (T)vh;
      dGV[b * lc + cb + aa] = (T)(-vh);
      dYV[C * lp + pidx(aa, b)] = (T)vh;
      return vh * (w + vt1 + vfo) * rd;
    };
    if constexpr (EPS) {
#pragma unroll
      for (int ta = 0; ta < ET; ++ta)
        if (ta < na) {
          const double q = elem(ta);
          qa[ta] = q;
          qbc += q;
        }
    } else {
      for (int ta = 0; ta < na; ++ta) (void)elem(ta);
    }
    if (TA == TB) {
      dG[b * lc + cb + b] = (T)0;
      dGV[b * lc + cb + b] = (T)0;
    }
  }
  if constexpr (EPS) {
    static_assert(sizeof(Gb) >= 336 * sizeof(double), "tile-sum scratch must fit the staging tile");
    eps_tile_sums(qa, qbc, A.ep + ((int64_t)item * gridDim.x + blockIdx.x) * 64, (double*)&Gb[0][0]);
  }
}

template <typename T>
hipError_t launch_bwd_same(const BwdSame<T>& a, int32_t nitems, hipStream_t s) {
  if (nitems <= 0 || a.e.ntri <= 0) return hipSuccess;
  if (a.ep) hipLaunchKernelGGL((k_bwd_same<T, true>), dim3(a.e.ntri, nitems), dim3(256), 0, s, a);
  else hipLaunchKernelGGL((k_bwd_same<T, false>), dim3(a.e.ntri, nitems), dim3(256), 0, s, a);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_bwd_mixed(const BwdMixed<T>& a, int32_t nitems, hipStream_t s) {
  if (nitems <= 0 || a.e.ntiles <= 0) return hipSuccess;
  if (a.ep) hipLaunchKernelGGL((k_bwd_mixed<T, true>), dim3(a.e.ntiles, nitems), dim3(256), 0, s, a);
  else hipLaunchKernelGGL((k_bwd_mixed<T, false>), dim3(a.e.ntiles, nitems), dim3(256), 0, s, a);
  return hipGetLastError();
}
template hipError_t launch_bwd_same<float>(const BwdSame<float>&, int32_t, hipStream_t);
template hipError_t launch_bwd_same<double>(const BwdSame<double>&, int32_t, hipStream_t);
template hipError_t launch_bwd_mixed<float>(const BwdMixed<float>&, int32_t, hipStream_t);
template hipError_t launch_bwd_mixed<double>(const BwdMixed<double>&, int32_t, hipStream_t);

// Per item: index sums of the tile sums (fixed loop order per index), and the
// item total.  Same spin: tile (A <= B <= C) is number C(C+1)(C+2)/6 +
// B(B+1)/2 + A; mixed: tile (A <= B, C) is number (B(B+1)/2 + A) nt_t + C.
__global__ __launch_bounds__(256) void k_eps_item(EpsReduce r) {
  __shared__ double sh[256];
  const int item = blockIdx.x, tid = threadIdx.x;
  const double* P = r.ep + (int64_t)item * r.nwg * 64;
  double* out = r.ri + (int64_t)item * r.ld_ri;
  auto wtri = [](int A, int B, int C) { return C * (C + 1) * (C + 2) / 6 + B * (B + 1) / 2 + A; };
  if (!r.mixed) {
    const int nt = r.nt_s;
    for (int x = tid; x < r.v_s; x += 256) {
      const int T = x / ET, q = x % ET;
      double acc = 0.0;
      for (int C = T; C < nt; ++C)                 // x first: T = A <= B <= C
        for (int B = T; B <= C; ++B) acc += P[(int64_t)wtri(T, B, C) * 64 + q];
      for (int C = T; C < nt; ++C)                 // x second: A <= T = B <= C
        for (int A = 0; A <= T; ++A) acc += P[(int64_t)wtri(A, T, C) * 64 + ET + q];
      for (int B = 0; B <= T; ++B)                 // x third: A <= B <= T = C
        for (int A = 0; A <= B; ++A) acc += P[(int64_t)wtri(A, B, T) * 64 + 2 * ET + q];
      out[x] = acc;
    }
  } else {
    const int ns = r.nt_s, ntt = r.nt_t, npr = ns * (ns + 1) / 2;
    for (int x = tid; x < r.v_s; x += 256) {
      const int T = x / ET, q = x % ET;
      double acc = 0.0;
      for (int B = T; B < ns; ++B)                 // x first: T = A <= B
        for (int C = 0; C < ntt; ++C) acc += P[((int64_t)(B * (B + 1) / 2 + T) * ntt + C) * 64 + q];
      for (int A = 0; A <= T; ++A)                 // x second: A <= T = B
        for (int C = 0; C < ntt; ++C) acc += P[((int64_t)(T * (T + 1) / 2 + A) * ntt + C) * 64 + ET + q];
      out[x] = acc;
    }
    for (int X = tid; X < r.v_t; X += 256) {
      const int T = X / ET, q = X % ET;
      double acc = 0.0;
      for (int pi = 0; pi < npr; ++pi) acc += P[((int64_t)pi * ntt + T) * 64 + 2 * ET + q];
      out[r.v_s + X] = acc;
    }
  }
  double acc = 0.0;
  for (int w = tid; w < r.nwg; w += 256) acc += P[(int64_t)w * 64 + 3 * ET];
  sh[tid] = acc;
  __syncthreads();
  if (tid == 0) {
    double t = 0.0;
    for (int k = 0; k < 256; ++k) t += sh[k];
    out[r.v_s + (r.mixed ? r.v_t : 0)] = t;
  }
}

// Over the batch's items, one thread per output index, items in order.
__global__ __launch_bounds__(64) void k_eps_batch(EpsReduce r) {
  const int x = blockIdx.x * 64 + threadIdx.x;
  const int vt = r.mixed ? r.v_t : 0, ot = r.mixed ? r.o_t : 0;
  const int tcol = r.v_s + vt;
  const double* ri = r.ri;
  const int64_t ld = r.ld_ri;
  if (x < r.v_s) {
    if (!r.ev_s) return;
    double acc = 0.0;
    for (int n = 0; n < r.nitems; ++n) acc += ri[n * ld + x];
    r.ev_s[x] += acc;
  } else if (x < r.v_s + vt) {
    const int X = x - r.v_s;
    if (!r.ev_t) return;
    double acc = 0.0;
    for (int n = 0; n < r.nitems; ++n) acc += ri[n * ld + r.v_s + X];
    r.ev_t[X] += acc;
  } else if (x < r.v_s + vt + r.o_s) {
    const int i = x - r.v_s - vt;
    if (!r.eo_s) return;
    double acc = 0.0;
    for (int n = 0; n < r.nitems; ++n) {
      const int32_t* it = r.items + 3 * n;
      if (it[0] == i || it[1] == i || (!r.mixed && it[2] == i)) acc += ri[n * ld + tcol];
    }
    r.eo_s[i] -= acc;
  } else if (x < r.v_s + vt + r.o_s + ot) {
    const int K = x - r.v_s - vt - r.o_s;
    if (!r.eo_t) return;
    double acc = 0.0;
    for (int n = 0; n < r.nitems; ++n)
      if (r.items[3 * n + 2] == K) acc += ri[n * ld + tcol];
    r.eo_t[K] -= acc;
  }
}

hipError_t launch_eps_reduce(const EpsReduce& r, hipStream_t s) {
  if (r.nitems <= 0 || r.nwg <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_eps_item, dim3(r.nitems), dim3(256), 0, s, r);
  const int n = r.v_s + r.o_s + (r.mixed ? r.v_t + r.o_t : 0);
  hipLaunchKernelGGL(k_eps_batch, dim3((n + 63) / 64), dim3(64), 0, s, r);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_epi_same(const EpiSame<T>& a, int32_t nitems, hipStream_t s) {
  if (nitems <= 0 || a.ntri <= 0) return hipSuccess;
  if (a.lap) hipLaunchKernelGGL((k_epi_same<T, true>), dim3(a.ntri, nitems), dim3(256), 0, s, a);
  else hipLaunchKernelGGL((k_epi_same<T, false>), dim3(a.ntri, nitems), dim3(256), 0, s, a);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_epi_mixed(const EpiMixed<T>& a, int32_t nitems, hipStream_t s) {
  if (nitems <= 0 || a.ntiles <= 0) return hipSuccess;
  // one work-group per (a-tile <= b-tile) pair; ntiles = that pair count
  if (a.lap) hipLaunchKernelGGL((k_epi_mixed<T, true>), dim3(a.ntiles, nitems), dim3(256), 0, s, a);
  else hipLaunchKernelGGL((k_epi_mixed<T, false>), dim3(a.ntiles, nitems), dim3(256), 0, s, a);
  return hipGetLastError();
}
template hipError_t launch_epi_same<float>(const EpiSame<float>&, int32_t, hipStream_t);
template hipError_t launch_epi_same<double>(const EpiSame<double>&, int32_t, hipStream_t);
template hipError_t launch_epi_mixed<float>(const EpiMixed<float>&, int32_t, hipStream_t);
template hipError_t launch_epi_mixed<double>(const EpiMixed<double>&, int32_t, hipStream_t);

// ---------------------------------------------------------------------------
// Closed-shell (spin-adapted) triples.  With spatial orbitals and
// tau^{ab}_{ij} = tau^{ba}_{ji}, W^{abc}_{ijk} is invariant under a joint
// permutation of the pairs (ia), (jb), (kc), and the energy of one occupied
// triple i <= j <= k (with all its distinct orderings) is
//   (m/3) sum over ordered (a,b,c) of Y^{abc} (W + V_t1 + V_f)^{abc} / D^{abc},
//   Y^{abc} = 4W^{abc} + W^{bca} + W^{cab} - 2W^{acb} - 2W^{bac} - 2W^{cba},
// m the number of distinct orderings of (i,j,k): the closed-shell energy
// expression summed over the orderings of the occupied triple and written
// as one symmetric form in the six orderings of (a,b,c).  A work-group takes
// the tiles a-tile <= b-tile <= c-tile and, for each (a,b,c) in them, adds
// all six orderings with weight 1/(number of tile permutations that map the
// tile onto itself), which counts every ordered (a,b,c) once with no test on
// repeated indices.
// ---------------------------------------------------------------------------

// One work-group per (item, a-tile <= b-tile) walks the c-tiles from the
// b-tile on; thread (b, c) = (tid >> 4, tid & 15) of a tile loops over the
// a-tile in two halves.  W is never stored: the three contraction cubes
// are read once each, at positions (a,b,c) and (b,a,c) directly (runs along
// c) and at the other four orderings through LDS, where each ordering's
// share of W is summed in two phases (runs along b, then along a); the
// (ia|jb), tau blocks with an a index are staged per half; the (b, c)
// values are the thread's.
// Pair q of the occupied triple: 0 (i,j), 1 (j,i), 2 (i,k), 3 (k,i),
// 4 (j,k), 5 (k,j); J_q[x][y] = (p x|p' y), Tq[x][y] = tau^{xy}_{p p'}.
template <typename T>
__global__ __launch_bounds__(256, 2) void k_epi_rhf(EpiRhf<T> a) {
  constexpr int HA = ET / 2, S1 = ET + 1;
  // staged parts of W at the six orderings of (a,b,c), [ta][tc][tb]
  __shared__ T Sabc[HA][ET][S1], Sacb[HA][ET][S1], Sbac[HA][ET][S1], Sbca[HA][ET][S1], Scab[HA][ET][S1],
      Scba[HA][ET][S1];
  __shared__ double Jab[6][HA][S1], Jac[6][HA][S1], Tab[6][HA][S1], Tac[6][HA][S1];
  __shared__ double t1a[3][HA], fa[3][HA], eva[HA];

  const int tid = threadIdx.x;
  const int L = xcd_logical(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);
  const int pi = L % gridDim.x;
  int TB = 0;
  while ((TB + 1) * (TB + 2) / 2 <= pi) ++TB;
  const int TA = pi - TB * (TB + 1) / 2;
  const int item = L / gridDim.x;
  const int32_t* it = a.items + 3 * item;
  const int occ[3] = {it[0], it[1], it[2]};
  const int v = a.v, o = a.o;
  const int64_t vv = (int64_t)v * v, ovv = (int64_t)o * v;
  const int pq[6][2] = {{occ[0], occ[1]}, {occ[1], occ[0]}, {occ[0], occ[2]},
                        {occ[2], occ[0]}, {occ[1], occ[2]}, {occ[2], occ[1]}};
  const T* A = a.W + (int64_t)item * a.w_item;   // F(i,j,k)[a][bc]
  const T* B = A + a.cube;                         // F(j,i,k)[b][ac]
  const T* C = A + 2 * a.cube;                     // F(k,i,j)[c][ab]
  const int a0 = TA * ET, b0 = TB * ET;
  const int tb = tid >> 4, tc = tid & 15;
  const int b = b0 + tb;
  const bool bok = b < v;
  double t1b[3], fb[3];
#pragma unroll
  for (int x = 0; x < 3; ++x) {
    t1b[x] = bok ? a.t1[(int64_t)occ[x] * v + b] : 0.0;
    fb[x] = bok ? a.f[(int64_t)occ[x] * v + b] : 0.0;
  }
  const double eijk = (a.eo[occ[0]] + a.eo[occ[1]]) + a.eo[occ[2]];
  const double evb = bok ? a.ev[b] : 0.0;

  double e4 = 0.0, est = 0.0, edt = 0.0;
  for (int TC = TB; TC < a.nt; ++TC) {
    const int c0 = TC * ET, c = c0 + tc;
    const bool ok = bok && c < v;
    // 1 / (permutations of the tile triple onto itself)
    const double wt = (TA == TB && TB == TC) ? 1.0 / 6.0 : ((TA == TB || TB == TC) ? 0.5 : 1.0);
    double Jbc[6], Tbc[6], t1c[3], fc[3];
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      Jbc[q] = ok ? a.ov[(int64_t)pq[q][0] * ovv * v + (int64_t)b * ovv + (int64_t)pq[q][1] * v + c] : 0.0;
      Tbc[q] = ok ? a.tau[((int64_t)pq[q][0] * o + pq[q][1]) * vv + (int64_t)b * v + c] : 0.0;
    }
#pragma unroll
    for (int x = 0; x < 3; ++x) {
      t1c[x] = ok ? a.t1[(int64_t)occ[x] * v + c] : 0.0;
      fc[x] = ok ? a.f[(int64_t)occ[x] * v + c] : 0.0;
    }
    const double dbc = eijk - evb - (ok ? a.ev[c] : 0.0);
    for (int h = 0; h < 2; ++h) {
      const int ah = a0 + h * HA;
      __syncthreads();               // the previous half's LDS reads are done
      // W^{xyz} = A[x][y][z] + B[y][x][z] + C[z][x][y].  Phase 1, runs along b:
      // positions [a][c][b] and [c][a][b] of the three cubes
#pragma unroll 2
      for (int u = 0; u < HA; ++u) {
        const int e = tid + 256 * u;
        const int x = e >> 8, y = (e >> 4) & 15, z = e & 15;
        const int aa = ah + x, cc = c0 + y, bb = b0 + z;
        T acb_a = 0, acb_b = 0, acb_c = 0, cab_a = 0, cab_b = 0, cab_c = 0;
        if (aa < v && cc < v && bb < v) {
          const int64_t p1 = aa * vv + (int64_t)cc * v + bb, p2 = cc * vv + (int64_t)aa * v + bb;
          acb_a = A[p1]; acb_b = B[p1]; acb_c = C[p1];
          cab_a = A[p2]; cab_b = B[p2]; cab_c = C[p2];
        }
        Sacb[x][y][z] = acb_a + cab_b;
        Scab[x][y][z] = acb_b + cab_a;
        Scba[x][y][z] = acb_c;
        Sabc[x][y][z] = cab_c;
      }
      for (int e = tid; e < 6 * HA * ET; e += 256) {
        const int q = e / (HA * ET), r = e % (HA * ET), x = r >> 4, z = r & 15;
        const int aa = ah + x, bb = b0 + z, cc = c0 + z;
        const int64_t p0 = pq[q][0], p1 = pq[q][1];
        const bool ab = aa < v && bb < v, ac = aa < v && cc < v;
        Jab[q][x][z] = ab ? a.ov[p0 * ovv * v + (int64_t)aa * ovv + p1 * v + bb] : 0.0;
        Jac[q][x][z] = ac ? a.ov[p0 * ovv * v + (int64_t)aa * ovv + p1 * v + cc] : 0.0;
        Tab[q][x][z] = ab ? a.tau[(p0 * o + p1) * vv + (int64_t)aa * v + bb] : 0.0;
        Tac[q][x][z] = ac ? a.tau[(p0 * o + p1) * vv + (int64_t)aa * v + cc] : 0.0;
      }
      if (tid < 3 * HA) {
        const int x = tid / HA, ta = tid % HA, aa = ah + ta;
        t1a[x][ta] = aa < v ? a.t1[(int64_t)occ[x] * v + aa] : 0.0;
        fa[x][ta] = aa < v ? a.f[(int64_t)occ[x] * v + aa] : 0.0;
      } else if (tid < 4 * HA) {
        const int ta = tid - 3 * HA, aa = ah + ta;
        eva[ta] = aa < v ? a.ev[aa] : 0.0;
      }
      __syncthreads();
      // phase 2, runs along a: positions [b][c][a] and [c][b][a]
#pragma unroll 2
      for (int u = 0; u < HA; ++u) {
        const int e = tid + 256 * u;
        const int z = e >> 7, y = (e >> 3) & 15, x = e & 7;
        const int aa = ah + x, cc = c0 + y, bb = b0 + z;
        T bca_a = 0, bca_b = 0, bca_c = 0, cba_a = 0, cba_b = 0, cba_c = 0;
        if (aa < v && cc < v && bb < v) {
          const int64_t p1 = bb * vv + (int64_t)cc * v + aa, p2 = cc * vv + (int64_t)bb * v + aa;
          bca_a = A[p1]; bca_b = B[p1]; bca_c = C[p1];
          cba_a = A[p2]; cba_b = B[p2]; cba_c = C[p2];
        }
        Sbca[x][y][z] = bca_a + cba_b;
        Sbac[x][y][z] = cba_c;
        Scab[x][y][z] += bca_c;
        Scba[x][y][z] += bca_b + cba_a;
      }
      __syncthreads();
      if (!ok) continue;
      const int na = min(HA, v - ah);
      for (int ta = 0; ta < na; ++ta) {
        const int aa = ah + ta;
        const int64_t pabc = aa * vv + (int64_t)b * v + c, pbac = b * vv + (int64_t)aa * v + c;
        const double w0 = ((double)A[pabc] + (double)B[pbac]) + (double)Sabc[ta][tc][tb];   // abc
        const double w2 = ((double)A[pbac] + (double)B[pabc]) + (double)Sbac[ta][tc][tb];   // bac
        const double w1 = (double)Sacb[ta][tc][tb] + (double)C[pbac];                       // acb
        const double w3 = (double)Sbca[ta][tc][tb] + (double)C[pabc];                       // bca
        const double w4 = (double)Scab[ta][tc][tb];                                         // cab
        const double w5 = (double)Scba[ta][tc][tb];                                         // cba
        const double se = (w0 + w3) + w4, so = (w1 + w2) + w5;
        const double ye = se - 2.0 * so, yo = so - 2.0 * se;
        const double y0 = 3.0 * w0 + ye, y3 = 3.0 * w3 + ye, y4 = 3.0 * w4 + ye;
        const double y1 = 3.0 * w1 + yo, y2 = 3.0 * w2 + yo, y5 = 3.0 * w5 + yo;
        const double ya = y0 * w0 + y1 * w1 + y2 * w2 + y3 * w3 + y4 * w4 + y5 * w5;
        // V_t1 and V_f of the six orderings (abc, acb, bac, bca, cab, cba)
        const double t0 = t1a[0][ta], t1_ = t1a[1][ta], t2_ = t1a[2][ta];
        const double vt0 = t0 * Jbc[4] + t1b[1] * Jac[2][ta][tc] + t1c[2] * Jab[0][ta][tb];
        const double vt1 = t0 * Jbc[5] + t1c[1] * Jab[2][ta][tb] + t1b[2] * Jac[0][ta][tc];
        const double vt2 = t1b[0] * Jac[4][ta][tc] + t1_ * Jbc[2] + t1c[2] * Jab[1][ta][tb];
        const double vt3 = t1b[0] * Jac[5][ta][tc] + t1c[1] * Jab[3][ta][tb] + t2_ * Jbc[0];
        const double vt4 = t1c[0] * Jab[4][ta][tb] + t1_ * Jbc[3] + t1b[2] * Jac[1][ta][tc];
        const double vt5 = t1c[0] * Jab[5][ta][tb] + t1b[1] * Jac[3][ta][tc] + t2_ * Jbc[1];
        const double f0 = fa[0][ta], f1 = fa[1][ta], f2 = fa[2][ta];
        const double vf0 = f0 * Tbc[4] + fb[1] * Tac[2][ta][tc] + fc[2] * Tab[0][ta][tb];
        const double vf1 = f0 * Tbc[5] + fc[1] * Tab[2][ta][tb] + fb[2] * Tac[0][ta][tc];
        const double vf2 = fb[0] * Tac[4][ta][tc] + f1 * Tbc[2] + fc[2] * Tab[1][ta][tb];
        const double vf3 = fb[0] * Tac[5][ta][tc] + fc[1] * Tab[3][ta][tb] + f2 * Tbc[0];
        const double vf4 = fc[0] * Tab[4][ta][tb] + f1 * Tbc[3] + fb[2] * Tac[1][ta][tc];
        const double vf5 = fc[0] * Tab[5][ta][tb] + fb[1] * Tac[3][ta][tc] + f2 * Tbc[1];
        const double yt = y0 * vt0 + y1 * vt1 + y2 * vt2 + y3 * vt3 + y4 * vt4 + y5 * vt5;
        const double yf = y0 * vf0 + y1 * vf1 + y2 * vf2 + y3 * vf3 + y4 * vf4 + y5 * vf5;
        const double g = wt * rcp64(dbc - eva[ta]);
        e4 += g * ya;
        est += g * yt;
        edt += g * yf;
      }
    }
  }
  // m / 3 with m the number of distinct orderings of (i, j, k)
  const double m = (occ[0] == occ[1] || occ[1] == occ[2]) ? 3.0 : 6.0;
  const double s = m / 3.0;
  block_write3(s * e4, s * est, s * edt, a.part + ((int64_t)item * a.ntiles + pi) * 3);
}

template <typename T>
hipError_t launch_epi_rhf(const EpiRhf<T>& a, int32_t nitems, hipStream_t s) {
  if (nitems <= 0 || a.ntiles <= 0) return hipSuccess;
  if (a.ntiles != a.nt * (a.nt + 1) / 2 || nitems > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_epi_rhf<T>), dim3(a.ntiles, nitems), dim3(256), 0, s, a);
  return hipGetLastError();
}
template hipError_t launch_epi_rhf<float>(const EpiRhf<float>&, int32_t, hipStream_t);
template hipError_t launch_epi_rhf<double>(const EpiRhf<double>&, int32_t, hipStream_t);

// ---------------------------------------------------------------------------
// Debug dumps of one item's W (the same formulas as the epilogues' first
// line, over the whole cube; the antisymmetry fills the other orderings and
// repeated virtual indices give zero)
// ---------------------------------------------------------------------------
__device__ inline int64_t pair_index(int lo, int hi) { return (int64_t)hi * (hi - 1) / 2 + lo; }   // lo < hi

template <typename T>
__global__ __launch_bounds__(256) void k_dump_w_same(const T* S, int64_t ldp, int32_t v, double* w) {
  const int64_t n = (int64_t)v * v * v, vv = (int64_t)v * v;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    int x = (int)(e / vv), y = (int)((e / v) % v), z = (int)(e % v);
    double sg = 1.0;
    if (x > y) { const int t = x; x = y; y = t; sg = -sg; }
    if (y > z) { const int t = y; y = z; z = t; sg = -sg; }
    if (x > y) { const int t = x; x = y; y = t; sg = -sg; }
    double val = 0.0;
    if (x < y && y < z)   // W^{xyz} = S[x][p(y,z)] - S[y][p(x,z)] + S[z][p(x,y)]
      val = ((double)S[x * ldp + pair_index(y, z)] - (double)S[y * ldp + pair_index(x, z)]) +
            (double)S[z * ldp + pair_index(x, y)];
    w[e] = sg * val;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_dump_w_mixed(const T* G, int64_t lc, const T* Y, int64_t lp, int32_t vs,
                                                      int32_t vt, double* w) {
  const int64_t n = (int64_t)vs * vs * vt, sv = (int64_t)vs * vt;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int a = (int)(e / sv), b = (int)((e / vt) % vs), C = (int)(e % vt);
    const int x = a < b ? a : b, y = a < b ? b : a;
    double val = 0.0;
    if (x < y)            // W^{xyC} = G[x][C v + y] - G[y][C v + x] + Y[C][p(x,y)]
      val = ((double)G[x * lc + (int64_t)C * vs + y] - (double)G[y * lc + (int64_t)C * vs + x]) +
            (double)Y[C * lp + pair_index(x, y)];
    w[e] = a < b ? val : -val;
  }
}

template <typename T>
hipError_t launch_dump_w_same(const T* S, int64_t ld_np, int32_t v, double* w, hipStream_t s) {
  const int64_t n = (int64_t)v * v * v;
  if (n <= 0) return hipSuccess;
  const int nb = (int)std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL((k_dump_w_same<T>), dim3(nb), dim3(256), 0, s, S, ld_np, v, w);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_dump_w_mixed(const T* G, int64_t ld_cb, const T* Y, int64_t ld_np, int32_t vs, int32_t vt,
                               double* w, hipStream_t s) {
  const int64_t n = (int64_t)vs * vs * vt;
  if (n <= 0) return hipSuccess;
  const int nb = (int)std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL((k_dump_w_mixed<T>), dim3(nb), dim3(256), 0, s, G, ld_cb, Y, ld_np, vs, vt, w);
  return hipGetLastError();
}
template hipError_t launch_dump_w_same<float>(const float*, int64_t, int32_t, double*, hipStream_t);
template hipError_t launch_dump_w_same<double>(const double*, int64_t, int32_t, double*, hipStream_t);
template hipError_t launch_dump_w_mixed<float>(const float*, int64_t, const float*, int64_t, int32_t, int32_t,
                                               double*, hipStream_t);
template hipError_t launch_dump_w_mixed<double>(const double*, int64_t, const double*, int64_t, int32_t, int32_t,
                                                double*, hipStream_t);

// ---------------------------------------------------------------------------
// Deterministic reductions
// ---------------------------------------------------------------------------
__device__ inline void tree3(double* sh, double& x0, double& x1, double& x2) {
  const int t = threadIdx.x;
  sh[t] = x0; sh[256 + t] = x1; sh[512 + t] = x2;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) {
      sh[t] += sh[t + w];
      sh[256 + t] += sh[256 + t + w];
      sh[512 + t] += sh[512 + t + w];
    }
    __syncthreads();
  }
  x0 = sh[0]; x1 = sh[256]; x2 = sh[512];
  __syncthreads();
}

__global__ __launch_bounds__(256) void k_reduce_items(const double* part, int32_t ntiles,
                                                      const int32_t* dst, double* e_items) {
  __shared__ double sh[768];
  const int item = blockIdx.x;
  const double* p = part + (int64_t)item * ntiles * 3;
  double x0 = 0, x1 = 0, x2 = 0;
  for (int t = threadIdx.x; t < ntiles; t += 256) { x0 += p[3 * t]; x1 += p[3 * t + 1]; x2 += p[3 * t + 2]; }
  tree3(sh, x0, x1, x2);
  if (threadIdx.x == 0) {
    double* d = e_items + 3 * (int64_t)dst[item];
    d[0] = x0; d[1] = x1; d[2] = x2;
  }
}

hipError_t launch_reduce_items(const double* part, int32_t nitems, int32_t ntiles,
                               const int32_t* dst, double* e_items, hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce_items, dim3(nitems), dim3(256), 0, s, part, ntiles, dst, e_items);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_reduce_final(const double* e_items, const int32_t* order,
                                                      const int32_t* first, const int32_t* count,
                                                      double* parts, double* e_out) {
  __shared__ double sh[768];
  double tot = 0.0;
  for (int blk = 0; blk < 4; ++blk) {
    double x0 = 0, x1 = 0, x2 = 0;
    for (int n = threadIdx.x; n < count[blk]; n += 256) {
      const double* e = e_items + 3 * (int64_t)order[first[blk] + n];
      x0 += e[0]; x1 += e[1]; x2 += e[2];
    }
    tree3(sh, x0, x1, x2);
    if (threadIdx.x == 0 && parts) { parts[3 * blk] = x0; parts[3 * blk + 1] = x1; parts[3 * blk + 2] = x2; }
    tot += (x0 + x1) + x2;
  }
  if (threadIdx.x == 0) e_out[0] = tot;
}

hipError_t launch_reduce_final(const double* e_items, const int32_t* order,
                               const int32_t* first, const int32_t* count,
                               double* parts, double* e_out, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(256), 0, s, e_items, order, first, count, parts, e_out);
  return hipGetLastError();
}

// Closed-shell result from the spin-block one with identical alpha and beta
// data: E = 2 (E_aaa + E_aab).  in[0] = E_aaa + E_aab, in[1 + 3 b + x] = part
// x of block b.
__global__ void k_rhf_combine(const double* in, double* e_out, double* parts) {
  if (threadIdx.x != 0) return;
  e_out[0] = 2.0 * in[0];
  if (parts)
    for (int x = 0; x < 3; ++x) parts[x] = 2.0 * (in[1 + x] + in[4 + x]);
}

hipError_t launch_rhf_combine(const double* in, double* e_out, double* parts, hipStream_t s) {
  hipLaunchKernelGGL(k_rhf_combine, dim3(1), dim3(64), 0, s, in, e_out, parts);
  return hipGetLastError();
}

}  // namespace lt
