// Device kernels of the adjoint of the two-site energy (see backward.cpp).
#include <hip/hip_runtime.h>

#include "bsdmrg_internal.h"
#include "kernels.h"

namespace bsd {

// Partial inner product of a G sub-matrix and a T1 sub-matrix over a row range.
__global__ __launch_bounds__(256) void bwd_dot_kernel(const BwdDot* __restrict__ items,
                                                      const double* __restrict__ G,
                                                      const double* __restrict__ T1,
                                                      double* __restrict__ part) {
  __shared__ double sh[4];
  const BwdDot d = items[blockIdx.x];
  const int n = d.nrows * d.cols;
  double s = 0.0;
  for (int e = threadIdx.x; e < n; e += blockDim.x) {
    const int r = d.row0 + e / d.cols, c = e % d.cols;
    s += G[d.g_off + (int64_t)r * d.ld_g + c] * T1[d.t_off + (int64_t)r * d.ld_t + c];
  }
  for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

// out[idx[k]] (or out[k] without idx) = sum of the partial dots of key k, in order.
__global__ void bwd_coef_kernel(int n, const int32_t* __restrict__ ptr, const double* __restrict__ part,
                                const int64_t* __restrict__ idx, double* __restrict__ out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  double s = 0.0;
  for (int j = ptr[k]; j < ptr[k + 1]; ++j) s += part[j];
  out[idx ? idx[k] : k] = s;
}

// dW(e) = g * sum_j dWW(coef_j) * Wother(partner_j) over the CSR row of element e.
__global__ void bwd_wgrad_kernel(int64_t n, const int32_t* __restrict__ ptr, const int32_t* __restrict__ coef,
                                 const int64_t* __restrict__ partner, const double* __restrict__ dcoef,
                                 const double* __restrict__ Wother, double g, double* __restrict__ dW) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int j = ptr[e]; j < ptr[e + 1]; ++j) s += dcoef[coef[j]] * Wother[partner[j]];
    dW[e] = g * s;
  }
}

// out[e] = g[p] * (x[e] + y[e]) (y may be NULL; out may alias x), with p the
// problem that owns element e: base[p] <= e < base[p + 1].
__global__ void seg_scale_kernel(int64_t n, const int64_t* __restrict__ base, int np, const double* __restrict__ g,
                                 const double* x, const double* __restrict__ y, double* out) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    int lo = 0, hi = np - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (base[mid] <= e) lo = mid; else hi = mid - 1;
    }
    const double v = y ? x[e] + y[e] : x[e];
    out[e] = g[lo] * v;
  }
}

// One workgroup per site of a group: terms[base + b] = <x_b, y_b>, each
// thread summing a fixed stride, then the wave and workgroup sums in a fixed
// order (bit-identical on every call).
__global__ __launch_bounds__(256) void site_dot_kernel(SiteDotGroup g, int base, double* __restrict__ terms) {
  __shared__ double sh[4];
  const int b = blockIdx.x;
  const double* __restrict__ x = g.x[b];
  const double* __restrict__ y = g.y[b];
  const int64_t n = g.n[b];
  double s = 0.0;
  for (int64_t e = threadIdx.x; e < n; e += blockDim.x) s += x[e] * y[e];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) terms[base + b] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// terms[n] = terms[0] + terms[1] + ... + terms[n - 1], left to right.
__global__ void ordered_sum_kernel(int n, double* __restrict__ terms) {
  if (threadIdx.x != 0) return;
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += terms[i];
  terms[n] = s;
}

static unsigned grid_for(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 8192)); }

hipError_t launch_bwd_dots(const BwdDot* items, int n, const double* G, const double* T1, double* part,
                           hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(bwd_dot_kernel, dim3((unsigned)n), dim3(256), 0, s, items, G, T1, part);
  return hipGetLastError();
}
hipError_t launch_bwd_coef(int n, const int32_t* ptr, const double* part, const int64_t* idx, double* out,
                           hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(bwd_coef_kernel, dim3((n + 255) / 256), dim3(256), 0, s, n, ptr, part, idx, out);
  return hipGetLastError();
}
hipError_t launch_bwd_wgrad(int64_t n, const int32_t* ptr, const int32_t* coef, const int64_t* partner,
                            const double* dcoef, const double* Wother, double g, double* dW, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(bwd_wgrad_kernel, dim3(grid_for(n)), dim3(256), 0, s, n, ptr, coef, partner, dcoef, Wother, g,
                     dW);
  return hipGetLastError();
}
hipError_t launch_seg_scale(int64_t n, const int64_t* base, int np, const double* g, const double* x,
                            const double* y, double* out, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(seg_scale_kernel, dim3(grid_for(n)), dim3(256), 0, s, n, base, np, g, x, y, out);
  return hipGetLastError();
}
hipError_t launch_site_dots(const SiteDotGroup& g, int count, int base, double* terms, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(site_dot_kernel, dim3((unsigned)count), dim3(256), 0, s, g, base, terms);
  return hipGetLastError();
}
hipError_t launch_ordered_sum(int n, double* terms, hipStream_t s) {
  hipLaunchKernelGGL(ordered_sum_kernel, dim3(1), dim3(64), 0, s, n, terms);
  return hipGetLastError();
}
}  // namespace bsd
