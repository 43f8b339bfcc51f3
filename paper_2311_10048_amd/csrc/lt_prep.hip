// Operand preparation: strided 4-D copies (permutation, precision change,
// optional antisymmetrisation by subtracting a second strided view) and
// pair packing (x<y) with optional antisymmetrisation.  These run once per
// call and are memory bound; they lay every contraction operand out k-major
// with padded, 16-byte aligned rows.
#include "lt_internal.h"

namespace lt {

template <typename Tin, typename Tout>
__global__ __launch_bounds__(256) void k_copy4d(Tout* out, int64_t os0, int64_t os1, int64_t os2,
                                                int64_t d0, int64_t d1, int64_t d2, int64_t d3,
                                                const Tin* in, int64_t s0, int64_t s1, int64_t s2, int64_t s3,
                                                const Tin* in2, int64_t u0, int64_t u1, int64_t u2, int64_t u3) {
  const int64_t total = d0 * d1 * d2 * d3;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    int64_t r = e;
    const int64_t x3 = r % d3; r /= d3;
    const int64_t x2 = r % d2; r /= d2;
    const int64_t x1 = r % d1; r /= d1;
    const int64_t x0 = r;
    double val = (double)in[x0 * s0 + x1 * s1 + x2 * s2 + x3 * s3];
    if (in2) val -= (double)in2[x0 * u0 + x1 * u1 + x2 * u2 + x3 * u3];
    out[x0 * os0 + x1 * os1 + x2 * os2 + x3] = (Tout)val;
  }
}

template <typename Tin, typename Tout>
hipError_t launch_copy4d(Tout* out, int64_t os0, int64_t os1, int64_t os2,
                         int64_t d0, int64_t d1, int64_t d2, int64_t d3,
                         const Tin* in, int64_t s0, int64_t s1, int64_t s2, int64_t s3,
                         const Tin* in2, int64_t u0, int64_t u1, int64_t u2, int64_t u3,
                         hipStream_t s) {
  const int64_t total = d0 * d1 * d2 * d3;
  if (total <= 0) return hipSuccess;
  int64_t nb = (total + 255) / 256;
  if (nb > 65536) nb = 65536;
  hipLaunchKernelGGL((k_copy4d<Tin, Tout>), dim3((unsigned)nb), dim3(256), 0, s, out, os0, os1, os2,
                     d0, d1, d2, d3, in, s0, s1, s2, s3, in2, u0, u1, u2, u3);
  return hipGetLastError();
}

// p = y(y-1)/2 + x, x < y
__device__ inline void pair_of(int64_t p, int32_t& x, int32_t& y) {
  int32_t yy = (int32_t)((1.0 + sqrt(1.0 + 8.0 * (double)p)) * 0.5);
  while ((int64_t)yy * (yy - 1) / 2 > p) --yy;
  while ((int64_t)(yy + 1) * yy / 2 <= p) ++yy;
  y = yy;
  x = (int32_t)(p - (int64_t)yy * (yy - 1) / 2);
}

template <typename Tin, typename Tout>
__global__ __launch_bounds__(256) void k_pack_pairs(Tout* out, int64_t ldo, int64_t rows, int32_t n,
                                                    const Tin* in, int64_t rs, int64_t xs, int64_t ys,
                                                    bool antisym) {
  const int64_t np = (int64_t)n * (n - 1) / 2;
  const int64_t total = rows * np;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / np, p = e % np;
    int32_t x, y;
    pair_of(p, x, y);
    const Tin* base = in + r * rs;
    double val = (double)base[x * xs + y * ys];
    if (antisym) val -= (double)base[y * xs + x * ys];
    out[r * ldo + p] = (Tout)val;
  }
}

template <typename Tin, typename Tout>
hipError_t launch_pack_pairs(Tout* out, int64_t ldo, int64_t rows, int32_t n,
                             const Tin* in, int64_t rs, int64_t xs, int64_t ys,
                             bool antisym, hipStream_t s) {
  const int64_t total = rows * ((int64_t)n * (n - 1) / 2);
  if (total <= 0) return hipSuccess;
  int64_t nb = (total + 255) / 256;
  if (nb > 65536) nb = 65536;
  hipLaunchKernelGGL((k_pack_pairs<Tin, Tout>), dim3((unsigned)nb), dim3(256), 0, s, out, ldo, rows, n,
                     in, rs, xs, ys, antisym);
  return hipGetLastError();
}

// Pair packing for the NAF metric: P[X][pair] = J[X][p][q] over p <= q,
// pairs ordered row by row (pair = p n - p (p - 1) / 2 + q - p).  One
// work-group per (p, X) row; reads and writes are contiguous in q.
__global__ __launch_bounds__(256) void k_naf_pack(double* P, const double* J, int32_t n, int64_t npairs) {
  const int p = blockIdx.x;
  const int64_t X = blockIdx.y;
  const int64_t off = (int64_t)p * n - (int64_t)p * (p - 1) / 2;
  const double* src = J + X * n * n + (int64_t)p * n;
  double* dst = P + X * npairs + off;
  for (int q = p + threadIdx.x; q < n; q += 256) dst[q - p] = src[q];
}

hipError_t launch_naf_pack(double* P, const double* J, int32_t n, int32_t nx, hipStream_t s) {
  if (n <= 0 || nx <= 0) return hipSuccess;
  const int64_t npairs = (int64_t)n * (n + 1) / 2;
  hipLaunchKernelGGL(k_naf_pack, dim3(n, nx), dim3(256), 0, s, P, J, n, npairs);
  return hipGetLastError();
}

template hipError_t launch_copy4d<double, double>(double*, int64_t, int64_t, int64_t, int64_t, int64_t,
                                                  int64_t, int64_t, const double*, int64_t, int64_t,
                                                  int64_t, int64_t, const double*, int64_t, int64_t,
                                                  int64_t, int64_t, hipStream_t);
template hipError_t launch_copy4d<double, float>(float*, int64_t, int64_t, int64_t, int64_t, int64_t,
                                                 int64_t, int64_t, const double*, int64_t, int64_t,
                                                 int64_t, int64_t, const double*, int64_t, int64_t,
                                                 int64_t, int64_t, hipStream_t);
template hipError_t launch_copy4d<float, float>(float*, int64_t, int64_t, int64_t, int64_t, int64_t,
                                                int64_t, int64_t, const float*, int64_t, int64_t,
                                                int64_t, int64_t, const float*, int64_t, int64_t,
                                                int64_t, int64_t, hipStream_t);
template hipError_t launch_pack_pairs<double, double>(double*, int64_t, int64_t, int32_t, const double*,
                                                      int64_t, int64_t, int64_t, bool, hipStream_t);
template hipError_t launch_pack_pairs<double, float>(float*, int64_t, int64_t, int32_t, const double*,
                                                     int64_t, int64_t, int64_t, bool, hipStream_t);
template hipError_t launch_pack_pairs<float, float>(float*, int64_t, int64_t, int32_t, const float*,
                                                    int64_t, int64_t, int64_t, bool, hipStream_t);

// Round-to-nearest-even FP32 -> BF16 (finite inputs; NaN stays NaN).
__device__ inline uint16_t bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline float bf16_to_f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// One thread per octet (block, q, column): 8 consecutive contraction rows of
// one column, split into hi = bf16(x) and lo = bf16(x - hi).
__global__ __launch_bounds__(256) void k_split8(bf16_t* hi, bf16_t* lo, int64_t nblk, int32_t K, int64_t ld,
                                                int32_t ncol, const float* in, int64_t ibs, int64_t iks) {
  const int64_t nq = ((K + 15) / 16) * 2;   // octets per block, rows padded to 16
  const int64_t total = nblk * nq * ld;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = e % ld, bq = e / ld, q = bq % nq, bb = bq / nq;
    uint16_t h[8], l[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int64_t k = 8 * q + t;
      float x = 0.f;
      if (k < K && c < ncol) x = in[bb * ibs + k * iks + c];
      h[t] = bf16_rne(x);
      l[t] = bf16_rne(x - bf16_to_f(h[t]));
    }
    uint4 vh, vl;
    vh.x = h[0] | ((uint32_t)h[1] << 16); vh.y = h[2] | ((uint32_t)h[3] << 16);
    vh.z = h[4] | ((uint32_t)h[5] << 16); vh.w = h[6] | ((uint32_t)h[7] << 16);
    vl.x = l[0] | ((uint32_t)l[1] << 16); vl.y = l[2] | ((uint32_t)l[3] << 16);
    vl.z = l[4] | ((uint32_t)l[5] << 16); vl.w = l[6] | ((uint32_t)l[7] << 16);
    *(uint4*)(hi + e * 8) = vh;
    *(uint4*)(lo + e * 8) = vl;
  }
}

hipError_t launch_split8(bf16_t* hi, bf16_t* lo, int64_t nblk, int32_t K, int64_t ld, int32_t ncol,
                         const float* in, int64_t ibs, int64_t iks, hipStream_t s) {
  const int64_t total = nblk * (((K + 15) / 16) * 2) * ld;
  if (total <= 0) return hipSuccess;
  int64_t nb = (total + 255) / 256;
  if (nb > 65536) nb = 65536;
  hipLaunchKernelGGL(k_split8, dim3((unsigned)nb), dim3(256), 0, s, hi, lo, nblk, K, ld, ncol, in, ibs, iks);
  return hipGetLastError();
}

__global__ void k_zero(double* p, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    p[e] = 0.0;
}

hipError_t launch_zero(double* p, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t nb = (n + 255) / 256;
  if (nb > 4096) nb = 4096;
  hipLaunchKernelGGL(k_zero, dim3((unsigned)nb), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_central_coef(double* coef, const double* c, const double* eo,
                                                      const double* lap, int32_t o, int32_t nq) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= o * nq) return;
  const int q = e / o, i = e % o;
  coef[e] = c[i] * exp(0.5 * lap[2 * q] * eo[i]);
}

hipError_t launch_central_coef(double* coef, const double* c, const double* eo, const double* lap, int32_t o,
                               int32_t nq, hipStream_t s) {
  const int n = o * nq;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_central_coef, dim3((n + 255) / 256), dim3(256), 0, s, coef, c, eo, lap, o, nq);
  return hipGetLastError();
}

// One thread per output element; the rotated rows (p >= o) sum over the o
// input rows with coalesced reads along the contiguous trailing index.
__global__ __launch_bounds__(256) void k_aug_axis(double* out, const double* in, const double* coef, int64_t pre,
                                                  int32_t o, int32_t nq, int64_t post) {
  const int64_t np = o + nq, total = pre * np * post;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t y = e % post, r = e / post;
    const int64_t p = r % np, x = r / np;
    const double* src = in + x * o * post + y;
    double acc;
    if (p < o) {
      acc = src[p * post];
    } else {
      const double* cq = coef + (p - o) * o;
      acc = 0.0;
      for (int i = 0; i < o; ++i) acc = fma(cq[i], src[(int64_t)i * post], acc);
    }
    out[e] = acc;
  }
}

hipError_t launch_aug_axis(double* out, const double* in, const double* coef, int64_t pre, int32_t o, int32_t nq,
                           int64_t post, hipStream_t s) {
  const int64_t total = pre * (int64_t)(o + nq) * post;
  if (total <= 0) return hipSuccess;
  int64_t nb = (total + 255) / 256;
  if (nb > 65536) nb = 65536;
  hipLaunchKernelGGL(k_aug_axis, dim3((unsigned)nb), dim3(256), 0, s, out, in, coef, pre, o, nq, post);
  return hipGetLastError();
}

// Grid-stride pass over each array in turn; any thread that meets a NaN or an
// infinity stores 1 to the flag (every writer stores the same value).
__global__ __launch_bounds__(256) void k_scan_finite(FiniteScan a, int32_t* flag) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  bool bad = false;
  for (int r = 0; r < a.narr; ++r) {
    const double* p = a.p[r];
    const int64_t n = a.n[r];
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride)
      bad |= !isfinite(p[e]);
  }
  if (bad) flag[0] = 1;
}

hipError_t launch_scan_finite(const FiniteScan& a, int32_t* flag, hipStream_t s) {
  if (a.narr <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scan_finite, dim3(2048), dim3(256), 0, s, a, flag);
  return hipGetLastError();
}

}  // namespace lt
