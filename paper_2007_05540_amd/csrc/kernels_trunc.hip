// Device kernels of the truncated SVD split (Sec. II-C, Sec. IV-A): gather the
// blocks of theta into one column-major matrix per charge of the new bond,
// fix the sign gauge of every kept singular pair, scatter U, S, V^T into the
// MPS tensors A and B.
#include <hip/hip_runtime.h>

#include "bsdmrg_internal.h"
#include "kernels.h"

namespace bsd {

__global__ void copy_kernel(const CopyTask* __restrict__ tasks, const double* __restrict__ src,
                            double* __restrict__ dst, const double* __restrict__ fac) {
  const CopyTask t = tasks[blockIdx.x];
  const int n = t.rows * t.cols;
  for (int e = threadIdx.x; e < n; e += blockDim.x) {
    const int r = e / t.cols, c = e % t.cols;
    double v = src[t.src_off + (int64_t)r * t.src_rs + (int64_t)c * t.src_cs];
    if (t.fac_off >= 0) v *= fac[t.fac_off + (t.fac_on_rows ? r : c)];
    dst[t.dst_off + (int64_t)r * t.dst_rs + (int64_t)c * t.dst_cs] = v;
  }
}

// Sign gauge (see GaugeTask): one block per kept column.
__global__ void gauge_kernel(const GaugeTask* __restrict__ tasks, const double* __restrict__ U,
                             const double* __restrict__ S, double* __restrict__ sign,
                             double* __restrict__ sgn_s) {
  __shared__ double smax[256];
  __shared__ int sidx[256];
  const GaugeTask t = tasks[blockIdx.x];
  const double* u = U + t.u_off;
  double m = 0.0;
  for (int r = threadIdx.x; r < t.rows; r += blockDim.x) m = fmax(m, fabs(u[r]));
  smax[threadIdx.x] = m;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + o]);
    __syncthreads();
  }
  const double thr = smax[0] * (1.0 - 1e-10);
  int first = 1 << 30;
  for (int r = threadIdx.x; r < t.rows; r += blockDim.x)
    if (fabs(u[r]) >= thr) { first = r; break; }
  sidx[threadIdx.x] = first;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sidx[threadIdx.x] = min(sidx[threadIdx.x], sidx[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    // no qualifying row (a column without finite entries): keep the sign
    const double sg = (sidx[0] < t.rows && u[sidx[0]] < 0.0) ? -1.0 : 1.0;
    sign[blockIdx.x] = sg;
    sgn_s[blockIdx.x] = sg * S[t.s_idx];
  }
}

hipError_t launch_copy(const void* d_tasks, int n, const double* src, double* dst, const double* fac,
                       hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(copy_kernel, dim3((unsigned)n), dim3(256), 0, s, (const CopyTask*)d_tasks, src, dst, fac);
  return hipGetLastError();
}

hipError_t launch_gauge(const void* d_tasks, int n, const double* U, const double* S, double* sign,
                        double* sgn_s, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(gauge_kernel, dim3((unsigned)n), dim3(256), 0, s, (const GaugeTask*)d_tasks, U, S, sign,
                     sgn_s);
  return hipGetLastError();
}


}  // namespace bsd

namespace bsd {

// One-sided Jacobi SVD (Hestenes) of one matrix per workgroup.  X (m x n,
// column-major, n <= m) is orthogonalised column pair by column pair with
// plane rotations, V accumulates them; then sigma_j = ||x_j||, the left
// vectors are x_j / sigma_j and the right vectors the columns of V.  Pairs
// follow the round-robin (circle) order, so the n/2 rotations of a step are
// independent; each group of 16 lanes takes whole pairs.  The output is written in
// descending order of sigma in the layout of a LAPACK-style thin SVD of the
// original matrix M: U (rows x k, column-major, ld rows), S (k), Vt (k x
// cols, column-major, ld k), k = min(rows, cols); when M was wide, X holds
// M^T and the roles of the two vector sets swap.
constexpr int kSvdGroup = 16;   // lanes per column pair
__global__ __launch_bounds__(1024) void jacobi_svd_kernel(const SvdTask* __restrict__ tasks, double* __restrict__ work,
                                                         double* __restrict__ U, double* __restrict__ S,
                                                         double* __restrict__ Vt) {
  __shared__ int not_conv;
  __shared__ double fro[16];
  const SvdTask t = tasks[blockIdx.x];
  double* X = work + t.x_off;       // m x n, ld m
  double* V = work + t.v_off;       // n x n, ld n
  double* sig = work + t.sig_off;   // n
  int* perm = (int*)(work + t.perm_off);
  const int m = t.m, n = t.n;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int gl = threadIdx.x % kSvdGroup, grp = threadIdx.x / kSvdGroup, ngrp = blockDim.x / kSvdGroup;
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) V[e] = (e % n == e / n) ? 1.0 : 0.0;
  __syncthreads();
  const int ne = n + (n & 1), half = ne / 2;
  // a pair counts as orthogonal when |x_p . x_q| <= tol ||x_p|| ||x_q||; the
  // dot products carry rounding of about m eps, so tol follows m.  Columns
  // whose norm is below 1e-16 ||X||_F are rounding noise left by earlier
  // rotations: they are not rotated (their singular values are zero to
  // working precision), otherwise the noise columns would keep rotating
  // against each other and the sweeps would never stop.
  const double tol = fmax(1e-15, 4.0 * m * 2.220446049250313e-16);
  double f2 = 0.0;
  for (int64_t e = threadIdx.x; e < (int64_t)m * n; e += blockDim.x) f2 += X[e] * X[e];
  for (int o = 32; o > 0; o >>= 1) f2 += __shfl_xor(f2, o, 64);
  if (lane == 0) fro[wave] = f2;
  __syncthreads();
  double fro2 = 0.0;
  for (int w = 0; w < nw; ++w) fro2 += fro[w];
  const double negl = 1e-32 * fro2;
  for (int sweep = 0; sweep < 80 && ne > 1; ++sweep) {
    if (threadIdx.x == 0) not_conv = 0;
    __syncthreads();
    for (int step = 0; step < ne - 1; ++step) {
      // one pair per group of 16 lanes (4 pairs per wave in flight): the
      // per-pair chain of reductions and rotation arithmetic is short
      for (int k = grp; k < half; k += ngrp) {
        auto player = [&](int j) { return j == 0 ? 0 : 1 + ((j - 1 + step) % (ne - 1)); };
        const int a = player(k), b = player(ne - 1 - k);
        const int p = min(a, b), q = max(a, b);
        if (q >= n) continue;   // dummy column of an odd n
        double* xp = X + (int64_t)p * m;
        double* xq = X + (int64_t)q * m;
        double al = 0.0, be = 0.0, ga = 0.0;
        for (int r = gl; r < m; r += kSvdGroup) {
          const double u = xp[r], v = xq[r];
          al += u * u;
          be += v * v;
          ga += u * v;
        }
        for (int o = kSvdGroup / 2; o > 0; o >>= 1) {   // stays inside the group
          al += __shfl_xor(al, o, 64);
          be += __shfl_xor(be, o, 64);
          ga += __shfl_xor(ga, o, 64);
        }
        if (ga == 0.0 || al <= negl || be <= negl || fabs(ga) <= tol * sqrt(al * be)) continue;
        if (gl == 0) not_conv = 1;
        const double zeta = (be - al) / (2.0 * ga);
        const double tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / sqrt(1.0 + tt * tt), s = c * tt;
        for (int r = gl; r < m; r += kSvdGroup) {
          const double u = xp[r], v = xq[r];
          xp[r] = c * u - s * v;
          xq[r] = s * u + c * v;
        }
        double* vp = V + (int64_t)p * n;
        double* vq = V + (int64_t)q * n;
        for (int r = gl; r < n; r += kSvdGroup) {
          const double u = vp[r], v = vq[r];
          vp[r] = c * u - s * v;
          vq[r] = s * u + c * v;
        }
      }
      __syncthreads();
    }
    const int nc = not_conv;
    __syncthreads();
    if (!nc) break;
  }
  // singular values and their descending order (ties: lower index first)
  for (int j = wave; j < n; j += nw) {
    double s2 = 0.0;
    for (int r = lane; r < m; r += 64) s2 += X[(int64_t)j * m + r] * X[(int64_t)j * m + r];
    for (int o = 32; o > 0; o >>= 1) s2 += __shfl_xor(s2, o, 64);
    if (lane == 0) sig[j] = sqrt(s2);
  }
  __syncthreads();
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    int rank = 0;
    for (int i = 0; i < n; ++i) rank += (sig[i] > sig[j]) || (sig[i] == sig[j] && i < j);
    perm[rank] = j;
  }
  __syncthreads();
  double* Uo = U + t.u_off;     // rows x n (ld rows)
  double* Vo = Vt + t.vt_off;   // n x cols (ld n)
  for (int e = threadIdx.x; e < n; e += blockDim.x) S[t.s_off + e] = sig[perm[e]];
  // left vectors of X (length m) and right vectors (length n)
  for (int e = threadIdx.x; e < m * n; e += blockDim.x) {
    const int r = e % m, jj = e / m;
    const int j = perm[jj];
    const double sj = sig[j];
    const double xv = sj > 0.0 ? X[(int64_t)j * m + r] / sj : 0.0;
    if (!t.transposed) Uo[(int64_t)jj * t.rows + r] = xv;       // U(r, jj), rows = m
    else Vo[jj + (int64_t)r * n] = xv;                          // Vt(jj, r), cols = m
  }
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
    const int r = e % n, jj = e / n;
    const double vv = V[(int64_t)perm[jj] * n + r];
    if (!t.transposed) Vo[jj + (int64_t)r * n] = vv;            // Vt(jj, r), cols = n
    else Uo[(int64_t)jj * t.rows + r] = vv;                     // U(r, jj), rows = n
  }
}

hipError_t launch_jacobi_svd(const void* d_tasks, int n, double* work, double* U, double* S, double* Vt,
                             hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(jacobi_svd_kernel, dim3((unsigned)n), dim3(1024), 0, s, (const SvdTask*)d_tasks, work, U, S,
                     Vt);
  return hipGetLastError();
}

}  // namespace bsd
