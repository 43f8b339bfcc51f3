// Reverse (adjoint) GEMMs of the triplet contractions and of the DF integral
// builds, driven by descriptor lists built on the host.
//
// Every forward contraction X[m][n] = sign * sum_k L[k][m] R[k][n] of an item
// gives two reverse products with the adjoint dX of its output:
//   dR[k][n] += sign * sum_m L[k][m] dX[m][n]     (contraction over m)
//   dL[k][m] += sign * sum_n R[k][n] dX[m][n]     (contraction over n)
// In both the left operand is read with its contraction index contiguous
// (A(x, r) = A[r*lda + x]); the right one is dX in its own layout (row x
// contiguous in the output column) or read transposed.  Contributions of all
// items of a batch to one target block are concatenated along the contraction
// (one work-group tile owns its output elements: no atomics), and the sum is
// added to the target, so the result is deterministic for a fixed batching.
#include "lt_internal.h"

namespace lt {

template <typename T> struct RV;
template <> struct RV<float> { typedef float4 type; static constexpr int N = 4; };
template <> struct RV<double> { typedef double2 type; static constexpr int N = 2; };

template <typename T, int MBW, int NBW, int WM, int BK, bool TB>
__global__ __launch_bounds__(256) void k_rgemm(RArgs<T> g) {
  using F = MF<T>;
  using V = typename RV<T>::type;
  constexpr int VN = RV<T>::N;
  constexpr int BR = F::BR, BC = F::BC;
  constexpr int WN = 4 / WM;
  constexpr int BM = WM * MBW * BR;
  constexpr int BN = WN * NBW * BC;
  constexpr int KQ = BK / VN;                       // vectors along the contraction
  constexpr int KP = BK + 16 / (int)sizeof(T);      // padded LDS row of a contraction-contiguous tile
  constexpr int AV = BM * KQ;
  constexpr int BV = TB ? BN * KQ : BK * (BN / VN);
  constexpr int AVT = (AV + 255) / 256, BVT = (BV + 255) / 256;

  // A tiles (and B tiles read transposed) keep the contraction index
  // contiguous in LDS: one 16-byte store per loaded vector.
  __shared__ __attribute__((aligned(16))) T As[2][BM][KP];
  __shared__ __attribute__((aligned(16))) T Bs[2][TB ? BN : BK][TB ? KP : BN];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  int b = blockIdx.x;
  {
    const int nblk = gridDim.x, x = b & 7, q = nblk >> 3, r = nblk & 7;
    b = (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + (b >> 3);
  }
  const int mtile = b % g.mt; b /= g.mt;
  const int ntile = b % g.nt; b /= g.nt;
  const RBlk<T> bk = g.blks[b];
  const int m0 = mtile * BM, n0 = ntile * BN;
  if (m0 >= bk.rows || n0 >= bk.cols) return;       // whole work-group: before any barrier
  const RSeg<T>* segs = g.segs + bk.beg;
  const int nseg = bk.end - bk.beg;

  // FP32: the matrix-core accumulator `acc` covers at most one segment and
  // FOLD k-steps; it is then added into `tot` with compensated (Kahan)
  // summation, so long concatenated contractions lose about as much as one
  // short FP32 dot product instead of growing with their length.
  constexpr bool TWO = sizeof(T) == 4;
  constexpr int FOLD = 32;
  typename F::acc_t acc[MBW][NBW], tot[MBW][NBW], cmp[MBW][NBW];
#pragma unroll
  for (int mb = 0; mb < MBW; ++mb)
#pragma unroll
    for (int nb = 0; nb < NBW; ++nb)
#pragma unroll
      for (int r = 0; r < F::NACC; ++r) { acc[mb][nb][r] = 0; tot[mb][nb][r] = 0; cmp[mb][nb][r] = 0; }
  auto fold = [&]() {
    if constexpr (TWO) {
#pragma unroll
      for (int mb = 0; mb < MBW; ++mb)
#pragma unroll
        for (int nb = 0; nb < NBW; ++nb)
#pragma unroll
          for (int r = 0; r < F::NACC; ++r) {
            const T y = acc[mb][nb][r] - cmp[mb][nb][r];
            const T t = tot[mb][nb][r] + y;
            cmp[mb][nb][r] = (t - tot[mb][nb][r]) - y;
            tot[mb][nb][r] = t;
            acc[mb][nb][r] = 0;
          }
    }
  };

  V ra[AVT], rb[BVT];
  auto gload = [&](const RSeg<T>& sg, int k0) {
#pragma unroll
    for (int u = 0; u < AVT; ++u) {
      const int e = tid + u * 256;
      V v = {};
      if (e < AV) {
        const int m = e / KQ, x = k0 + (e % KQ) * VN, row = m0 + m;
        if (row < bk.rows && x < sg.K) {
          v = *(const V*)(sg.A + (int64_t)row * sg.lda + x);
          T* pv = (T*)&v;
#pragma unroll
          for (int t = 0; t < VN; ++t) pv[t] = (x + t < sg.K) ? pv[t] * (T)sg.sign : (T)0;
        }
      }
      ra[u] = v;
    }
#pragma unroll
    for (int u = 0; u < BVT; ++u) {
      const int e = tid + u * 256;
      V v = {};
      if (e < BV) {
        if constexpr (TB) {
          const int n = e / KQ, x = k0 + (e % KQ) * VN, col = n0 + n;
          if (col < bk.cols && x < sg.K) {
            v = *(const V*)(sg.B + (int64_t)col * sg.ldb + x);
            T* pv = (T*)&v;
#pragma unroll
            for (int t = 0; t < VN; ++t) if (x + t >= sg.K) pv[t] = (T)0;
          }
        } else {
          const int kk = e / (BN / VN), n = (e % (BN / VN)) * VN, x = k0 + kk, col = n0 + n;
          if (x < sg.K && col < bk.cols) v = *(const V*)(sg.B + (int64_t)x * sg.ldb + col);
        }
      }
      rb[u] = v;
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int u = 0; u < AVT; ++u) {
      const int e = tid + u * 256;
      if (e < AV) *(V*)&As[buf][e / KQ][(e % KQ) * VN] = ra[u];
    }
#pragma unroll
    for (int u = 0; u < BVT; ++u) {
      const int e = tid + u * 256;
      if (e < BV) {
        if constexpr (TB) *(V*)&Bs[buf][e / KQ][(e % KQ) * VN] = rb[u];
        else *(V*)&Bs[buf][e / (BN / VN)][(e % (BN / VN)) * VN] = rb[u];
      }
    }
  };

  int s = 0, k0 = 0;
  while (s < nseg && segs[s].K <= 0) ++s;
  RSeg<T> cs{};                  // descriptor of the segment being loaded (reloaded on change only)
  if (s < nseg) { cs = segs[s]; gload(cs, k0); sstore(0); }
  __syncthreads();
  int cur = 0;
  int seg_of[2] = {s, s};        // segment of the data staged in each LDS buffer
  int last = s, steps = 0;
  const int arow0 = wm * MBW * BR + F::a_row(lane);
  const int bcol0 = wn * NBW * BC + F::c_col(lane);
  while (s < nseg) {
    k0 += BK;
    while (s < nseg && k0 >= cs.K) {
      ++s; k0 = 0;
      if (s < nseg) cs = segs[s];
    }
    const bool more = s < nseg;
    if (more) gload(cs, k0);
    if (TWO && (seg_of[cur] != last || steps == FOLD)) { fold(); last = seg_of[cur]; steps = 0; }
    ++steps;
#pragma unroll
    for (int ks = 0; ks < BK; ks += F::KS) {
      const int kr = ks + F::a_k(lane);
      T bv[NBW];
#pragma unroll
      for (int nb = 0; nb < NBW; ++nb) {
        if constexpr (TB) bv[nb] = Bs[cur][bcol0 + nb * BC][kr];
        else bv[nb] = Bs[cur][kr][bcol0 + nb * BC];
      }
#pragma unroll
      for (int mb = 0; mb < MBW; ++mb) {
        const T av = As[cur][arow0 + mb * BR][kr];
#pragma unroll
        for (int nb = 0; nb < NBW; ++nb) acc[mb][nb] = F::mma(av, bv[nb], acc[mb][nb]);
      }
    }
    if (more) { sstore(cur ^ 1); seg_of[cur ^ 1] = s; }
    __syncthreads();
    cur ^= 1;
  }
  fold();

#pragma unroll
  for (int nb = 0; nb < NBW; ++nb) {
    const int n = n0 + bcol0 + nb * BC;
    if (n >= bk.cols) continue;
#pragma unroll
    for (int mb = 0; mb < MBW; ++mb)
#pragma unroll
      for (int r = 0; r < F::NACC; ++r) {
        const int m = m0 + wm * MBW * BR + mb * BR + F::c_row(lane, r);
        if (m < bk.rows) {
          T* o = bk.out + (int64_t)m * bk.ldo + n;
          const T x = TWO ? tot[mb][nb][r] : acc[mb][nb][r];
          *o = bk.store ? x : *o + x;
        }
      }
  }
}

template <typename T, int MBW, int NBW, int WM, int BK>
hipError_t rcfg(RArgs<T> g, bool tb, hipStream_t s) {
  constexpr int BM = WM * MBW * MF<T>::BR, BN = (4 / WM) * NBW * MF<T>::BC;
  g.mt = (g.max_rows + BM - 1) / BM;
  g.nt = (g.max_cols + BN - 1) / BN;
  const int64_t nwg = (int64_t)g.mt * g.nt * g.nblk;
  if (nwg <= 0) return hipSuccess;
  if (nwg > 0x7fffffff) return hipErrorInvalidValue;
  if (tb)
    hipLaunchKernelGGL((k_rgemm<T, MBW, NBW, WM, BK, true>), dim3((unsigned)nwg), dim3(256), 0, s, g);
  else
    hipLaunchKernelGGL((k_rgemm<T, MBW, NBW, WM, BK, false>), dim3((unsigned)nwg), dim3(256), 0, s, g);
  return hipGetLastError();
}

template <typename T>
__global__ __launch_bounds__(256) void k_rreduce(const RRed<T>* reds) {
  const RRed<T> r = reds[blockIdx.y];
  const int64_t n = (int64_t)r.rows * r.cols;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
    double sum = 0.0;
    for (int j = 0; j < r.nchunk; ++j) sum += (double)r.part[(int64_t)j * n + e];
    T* o = r.out + (e / r.cols) * r.ldo + e % r.cols;
    *o = (T)((double)*o + sum);
  }
}

template <typename T>
hipError_t launch_rreduce(const RRed<T>* reds, int32_t nred, int32_t max_elems, hipStream_t s) {
  if (nred <= 0 || max_elems <= 0) return hipSuccess;
  int64_t gx = (max_elems + 255) / 256;
  if (gx > 1024) gx = 1024;
  hipLaunchKernelGGL((k_rreduce<T>), dim3((unsigned)gx, (unsigned)nred), dim3(256), 0, s, reds);
  return hipGetLastError();
}
template hipError_t launch_rreduce<float>(const RRed<float>*, int32_t, int32_t, hipStream_t);
template hipError_t launch_rreduce<double>(const RRed<double>*, int32_t, int32_t, hipStream_t);

template <> hipError_t launch_rgemm<float>(RArgs<float> g, bool tb, hipStream_t s) {
  const int need = (g.max_rows + 31) / 32;
  // 64-row tiles above one 32-row block: 160 registers, three waves per SIMD.
  // Measured on the gradient workload (20,18,160,162,640): the whole FP32
  // adjoint 5.59 s with tiles covering all rows (one wave per SIMD: the
  // compensated sum keeps three accumulator sets) against 4.81 s; 32-row
  // tiles everywhere 4.80 s.
  if (need <= 1) return rcfg<float, 1, 1, 1, 16>(g, tb, s);
  return rcfg<float, 2, 1, 1, 16>(g, tb, s);
}

template <> hipError_t launch_rgemm<double>(RArgs<double> g, bool tb, hipStream_t s) {
  const int need = (g.max_rows + 15) / 16;
  // 64-row tiles above 32 rows (the FP64 adjoint on the gradient workload
  // 10.27 s with tiles of up to 160 rows, 8.65 s with these)
  if (need <= 2) return rcfg<double, 2, 1, 1, 8>(g, tb, s);
  return rcfg<double, 4, 1, 1, 8>(g, tb, s);
}

}  // namespace lt
