// Adjoint pass, memory-bound pieces: the transposes of the operand
// preparation (gradients of the prepared operands mapped back to the
// amplitudes and to the four-index integral classes, in FP64) and the
// projections of the gradients of symmetric inputs onto their symmetric
// subspaces.  Every map is a bijection or a gather, so each output element is
// written by one thread: no atomics, deterministic.
#include "lt_internal.h"

namespace lt {

template <typename Tin>
__global__ __launch_bounds__(256) void k_perm_acc(double* out, int64_t d0, int64_t d1, int64_t d2, int64_t d3,
                                                  int64_t o0, int64_t o1, int64_t o2, int64_t o3, const Tin* in,
                                                  int64_t i0, int64_t i1, int64_t i2, int64_t i3, double scale) {
  const int64_t total = d0 * d1 * d2 * d3;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    int64_t r = e;
    const int64_t x3 = r % d3; r /= d3;
    const int64_t x2 = r % d2; r /= d2;
    const int64_t x1 = r % d1;
    const int64_t x0 = r / d1;
    out[x0 * o0 + x1 * o1 + x2 * o2 + x3 * o3] += scale * (double)in[x0 * i0 + x1 * i1 + x2 * i2 + x3 * i3];
  }
}

template <typename Tin>
hipError_t launch_perm_acc(double* out, const int64_t d[4], const int64_t os[4], const Tin* in,
                           const int64_t is[4], double scale, hipStream_t s) {
  const int64_t total = d[0] * d[1] * d[2] * d[3];
  if (total <= 0) return hipSuccess;
  int64_t nb = (total + 255) / 256;
  if (nb > 65536) nb = 65536;
  hipLaunchKernelGGL((k_perm_acc<Tin>), dim3((unsigned)nb), dim3(256), 0, s, out, d[0], d[1], d[2], d[3], os[0],
                     os[1], os[2], os[3], in, is[0], is[1], is[2], is[3], scale);
  return hipGetLastError();
}

template <typename Tin>
__global__ __launch_bounds__(256) void k_unpack_acc(double* out, int64_t R0, int64_t R1, int32_t n, int64_t o0,
                                                    int64_t o1, int64_t ox, int64_t oy, const Tin* in, int64_t i0,
                                                    int64_t i1, double s_up, double s_lo) {
  const int64_t nn = (int64_t)n * n, total = R0 * R1 * nn;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / nn, q = e % nn;
    const int64_t r0 = r / R1, r1 = r % R1;
    const int32_t x = (int32_t)(q / n), y = (int32_t)(q % n);
    if (x == y) continue;
    const Tin* row = in + r0 * i0 + r1 * i1;
    const double val = x < y ? s_up * (double)row[(int64_t)y * (y - 1) / 2 + x]
                             : s_lo * (double)row[(int64_t)x * (x - 1) / 2 + y];
    out[r0 * o0 + r1 * o1 + x * ox + y * oy] += val;
  }
}

template <typename Tin>
hipError_t launch_unpack_acc(double* out, int64_t R0, int64_t R1, int32_t n, int64_t o0, int64_t o1,
                             int64_t ox, int64_t oy, const Tin* in, int64_t i0, int64_t i1, double s_up,
                             double s_lo, hipStream_t s) {
  const int64_t total = R0 * R1 * (int64_t)n * n;
  if (total <= 0) return hipSuccess;
  int64_t nb = (total + 255) / 256;
  if (nb > 65536) nb = 65536;
  hipLaunchKernelGGL((k_unpack_acc<Tin>), dim3((unsigned)nb), dim3(256), 0, s, out, R0, R1, n, o0, o1, ox, oy,
                     in, i0, i1, s_up, s_lo);
  return hipGetLastError();
}

// One thread per group {(i,j,a,b), (j,i,a,b), (i,j,b,a), (j,i,b,a)}, i<j, a<b;
// elements with i == j or a == b project to zero.
__global__ __launch_bounds__(256) void k_antisym4(double* t, int64_t o, int64_t v) {
  const int64_t total = o * o * v * v;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = e % v, a = (e / v) % v, j = (e / (v * v)) % o, i = e / (v * v * o);
    if (i == j || a == b) { t[e] = 0.0; continue; }
    if (i > j || a > b) continue;
    const int64_t eji = ((j * o + i) * v + a) * v + b, eba = ((i * o + j) * v + b) * v + a,
                  ejiba = ((j * o + i) * v + b) * v + a;
    const double g = 0.25 * ((t[e] - t[eji]) - (t[eba] - t[ejiba]));
    t[e] = g; t[eji] = -g; t[eba] = -g; t[ejiba] = g;
  }
}

__global__ __launch_bounds__(256) void k_sym3(double* b, int64_t Q, int64_t n) {
  const int64_t total = Q * n * n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t y = e % n, x = (e / n) % n, q = e / (n * n);
    if (x >= y) continue;
    const int64_t f = (q * n + y) * n + x;
    const double g = 0.5 * (b[e] + b[f]);
    b[e] = g; b[f] = g;
  }
}

hipError_t launch_antisym4(double* t, int64_t o, int64_t v, hipStream_t s) {
  const int64_t total = o * o * v * v;
  if (total <= 0) return hipSuccess;
  int64_t nb = (total + 255) / 256;
  if (nb > 65536) nb = 65536;
  hipLaunchKernelGGL(k_antisym4, dim3((unsigned)nb), dim3(256), 0, s, t, o, v);
  return hipGetLastError();
}

hipError_t launch_sym3(double* b, int64_t Q, int64_t n, hipStream_t s) {
  const int64_t total = Q * n * n;
  if (total <= 0) return hipSuccess;
  int64_t nb = (total + 255) / 256;
  if (nb > 65536) nb = 65536;
  hipLaunchKernelGGL(k_sym3, dim3((unsigned)nb), dim3(256), 0, s, b, Q, n);
  return hipGetLastError();
}

__global__ void k_zero32(uint32_t* p, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    p[e] = 0u;
}

hipError_t launch_zero32(void* p, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t nb = (n + 255) / 256;
  if (nb > 8192) nb = 8192;
  hipLaunchKernelGGL(k_zero32, dim3((unsigned)nb), dim3(256), 0, s, (uint32_t*)p, n);
  return hipGetLastError();
}

template hipError_t launch_perm_acc<float>(double*, const int64_t*, const int64_t*, const float*, const int64_t*,
                                           double, hipStream_t);
template hipError_t launch_perm_acc<double>(double*, const int64_t*, const int64_t*, const double*,
                                            const int64_t*, double, hipStream_t);
template hipError_t launch_unpack_acc<float>(double*, int64_t, int64_t, int32_t, int64_t, int64_t, int64_t,
                                             int64_t, const float*, int64_t, int64_t, double, double, hipStream_t);
template hipError_t launch_unpack_acc<double>(double*, int64_t, int64_t, int32_t, int64_t, int64_t, int64_t,
                                              int64_t, const double*, int64_t, int64_t, double, double,
                                              hipStream_t);

}  // namespace lt
