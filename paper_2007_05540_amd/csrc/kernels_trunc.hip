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

// SVD of the charge matrices of a truncation: Householder QR with column
// pivoting, block one-sided Jacobi (Hestenes) on R^T, back-transformation.
//
// X (m x n, column-major, n <= m) is M or M^T.  QR with column pivoting
// X P = Q R (the column of largest remaining norm first) stops at the
// numerical rank r: once every remaining column has squared norm <= m eps^2
// ||X||_F^2 the rest of R is rounding noise and is dropped (a perturbation of
// the order of the rounding error of any SVD).  Pivoting puts the large
// columns first, so one-sided Jacobi on A = R^T (n x r) needs a few sweeps
// where Jacobi on X itself needs many on the graded, rank-deficient matrices
// a truncation sees.  Jacobi works on AV = [A; VJ] (VJ = I at the start):
// a rotation of two columns of A is applied to the same columns of VJ, so
// that A_end = A VJ.  The columns are cut into nb blocks of b; a sweep runs
// the nb - 1 round-robin steps of block pairs, every pair of a step in its
// own workgroup with the 2b columns in LDS: the first step of a sweep runs one
// inner cyclic sweep over all column pairs of the union, the later ones only
// the pairs across the two blocks (a pair counts as orthogonal when
// |a_p . a_q| <= tol ||a_p|| ||a_q||, tol following the rounding of an n-term
// dot product; columns at the rank threshold are left alone).  Sweeps stop
// when one makes no rotation.  Then sigma_j = ||a_j||, and with
// R = VJ S W^T (W = A_end S^-1):  X = (Q VJ) S (P W)^T.  The left vectors
// Q VJ come from applying the reflectors to the columns of VJ (one wave per
// column), the right ones from W with the pivots undone.  The output is in
// descending order of sigma in the layout of a LAPACK-style thin SVD of M:
// U (rows x k, column-major, ld rows), S (k), Vt (k x cols, column-major,
// ld k), k = min(rows, cols); singular values past the rank are 0 with zero
// vectors.  When M was wide, X holds M^T and the two vector sets swap.

// block-wide sum over 1024 threads (every thread gets the result)
__device__ __forceinline__ double svd_block_sum(double v, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < nw; ++w) s += red[w];
  return s;
}
// sum over an aligned group of gs lanes (gs a power of two <= 64)
// DPP move of a double (both halves through the same lane pattern).
template <int CTRL>
__device__ __forceinline__ double svd_dpp(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, true);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}
// Sum over a group of gs (a power of two <= 64) consecutive lanes starting at
// a multiple of gs, the same value on every lane of the group: register
// exchanges inside rows of 16 (pairs, quads, half rows, rows), then lane
// shuffles across rows.  Every lane of a group must be active.
__device__ __forceinline__ double svd_group_sum(double v, int gs) {
  if (gs >= 2) v += svd_dpp<0xB1>(v);    // quad_perm [1,0,3,2]
  if (gs >= 4) v += svd_dpp<0x4E>(v);    // quad_perm [2,3,0,1]
  if (gs >= 8) v += svd_dpp<0x141>(v);   // row_half_mirror
  if (gs >= 16) v += svd_dpp<0x140>(v);  // row_mirror
  if (gs >= 32) v += __shfl_xor(v, 16, 64);
  if (gs >= 64) v += __shfl_xor(v, 32, 64);
  return v;
}

// Pieces of the QR with column pivoting; every one runs on a workgroup of
// 1024 threads working on one matrix.  Aux layout: R diagonal (n),
// reflector factors (n), squared norms of the remaining columns (n), pivots
// (n ints), then the rank and the rank threshold.
struct QrView {
  int m, n;
  double *X, *AV, *rdiag, *beta, *cnorm, *rank_out;
  int* qperm;
  __device__ QrView(const SvdTask& t, double* work)
      : m(t.m), n(t.n), X(work + t.x_off), AV(work + t.av_off), rdiag(work + t.aux_off), beta(rdiag + t.n),
        cnorm(rdiag + 2 * t.n), rank_out(rdiag + 4 * t.n), qperm((int*)(rdiag + 3 * t.n)) {}
};

// ||X||_F^2, the rank threshold, column norms and pivots; false (S = NaN,
// rank -1) for a matrix with non-finite entries.
__device__ bool qr_init(const SvdTask& t, const QrView& q, double* S, double* red) {
  const int tid = threadIdx.x, nthr = blockDim.x;
  const double eps = 2.220446049250313e-16;
  double f2 = 0.0;
  for (int64_t e = tid; e < (int64_t)q.m * q.n; e += nthr) f2 += q.X[e] * q.X[e];
  const double fro2 = svd_block_sum(f2, red);
  if (!isfinite(fro2)) {   // uniform: reported to the caller as non-finite singular values
    for (int e = tid; e < q.n; e += nthr) S[t.s_off + e] = fro2 - fro2;
    if (tid == 0) q.rank_out[0] = -1.0;   // the later kernels skip this matrix
    return false;
  }
  int gs = 64;
  while (gs > 4 && gs * q.n > nthr) gs >>= 1;
  const int gl = tid % gs, grp = tid / gs, ngrp = nthr / gs;
  for (int j = grp; j < q.n; j += ngrp) {
    double c = 0.0;
    for (int i = gl; i < q.m; i += gs) c += q.X[(int64_t)j * q.m + i] * q.X[(int64_t)j * q.m + i];
    c = svd_group_sum(c, gs);
    if (gl == 0) {
      q.cnorm[j] = c;
      q.qperm[j] = j;
    }
  }
  if (tid == 0) q.rank_out[1] = (double)q.m * eps * eps * fro2;   // rank threshold (squared norm)
  __syncthreads();
  return true;
}

// Step k up to the reflector: pivot (largest remaining norm, the lowest
// column on ties), swap, H = I - beta v v^T with H x_k = alpha e_k.  false
// when every remaining column is at the rank threshold.
__device__ bool qr_head(const QrView& q, int k, double* red, int* redi) {
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int lane = tid & 63, wave = tid >> 6, nw = nthr >> 6;
  const double thr2 = q.rank_out[1];
  double bv = -1.0;
  int bi = q.n;
  for (int j = k + tid; j < q.n; j += nthr)
    if (q.cnorm[j] > bv) { bv = q.cnorm[j]; bi = j; }
  for (int o = 32; o > 0; o >>= 1) {
    const double ov = __shfl_xor(bv, o, 64);
    const int oi = __shfl_xor(bi, o, 64);
    if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
  }
  __syncthreads();
  if (lane == 0) { red[wave] = bv; redi[wave] = bi; }
  __syncthreads();
  bv = red[0];
  bi = redi[0];
  for (int w = 1; w < nw; ++w)
    if (red[w] > bv || (red[w] == bv && redi[w] < bi)) { bv = red[w]; bi = redi[w]; }
  if (!(bv > thr2)) return false;   // uniform: every thread computed the same bv
  const int p = bi, m = q.m;
  if (p != k) {
    for (int i = tid; i < m; i += nthr) {
      const double a = q.X[(int64_t)k * m + i];
      q.X[(int64_t)k * m + i] = q.X[(int64_t)p * m + i];
      q.X[(int64_t)p * m + i] = a;
    }
    if (tid == 0) {
      const double c = q.cnorm[k]; q.cnorm[k] = q.cnorm[p]; q.cnorm[p] = c;
      const int x = q.qperm[k]; q.qperm[k] = q.qperm[p]; q.qperm[p] = x;
    }
    __syncthreads();
  }
  double part = 0.0;
  for (int i = k + tid; i < m; i += nthr) part += q.X[(int64_t)k * m + i] * q.X[(int64_t)k * m + i];
  const double nrm2 = svd_block_sum(part, red);
  const double xkk = q.X[(int64_t)k * m + k];
  const double alpha = -copysign(sqrt(nrm2), xkk);
  const double v0 = xkk - alpha;
  const double vtv = (nrm2 - xkk * xkk) + v0 * v0;
  __syncthreads();   // every thread has read x_kk
  if (tid == 0) {
    q.X[(int64_t)k * m + k] = v0;
    q.rdiag[k] = alpha;
    q.beta[k] = vtv > 0.0 ? 2.0 / vtv : 0.0;
  }
  __syncthreads();
  return true;
}

// Reflector k applied to column j (> k) by a group of gs lanes, and the
// squared norm of the column's remaining part (rows > k).
__device__ __forceinline__ void qr_apply_col(const QrView& q, int k, int j, int gl, int gs) {
  const int m = q.m;
  const double* v = q.X + (int64_t)k * m;
  double* xj = q.X + (int64_t)j * m;
  double d = 0.0;
  for (int i = k + gl; i < m; i += gs) d += v[i] * xj[i];
  const double f = q.beta[k] * svd_group_sum(d, gs);
  double c = 0.0;
  for (int i = k + gl; i < m; i += gs) {
    const double y = xj[i] - f * v[i];
    xj[i] = y;
    if (i > k) c += y * y;
  }
  c = svd_group_sum(c, gs);
  if (gl == 0) q.cnorm[j] = c;
}

// AV: rows 0..n-1 of column i = row i of R; rows n..n+r-1 = identity.
__device__ void qr_build_av(const QrView& q, int r) {
  const int tid = threadIdx.x, nthr = blockDim.x, n = q.n, ld = 2 * q.n;
  for (int64_t e = tid; e < (int64_t)ld * r; e += nthr) {
    const int j = (int)(e % ld), i = (int)(e / ld);
    double val;
    if (j < n) val = j < i ? 0.0 : (j == i ? q.rdiag[i] : q.X[(int64_t)j * q.m + i]);
    else val = (j - n == i) ? 1.0 : 0.0;
    q.AV[e] = val;
  }
  if (tid == 0) q.rank_out[0] = (double)r;
}

// QR of one matrix per workgroup (matrices of the single-workgroup class).
__global__ __launch_bounds__(1024) void svd_qr_kernel(const SvdTask* __restrict__ tasks, double* __restrict__ work,
                                                     double* __restrict__ S) {
  __shared__ double red[16];
  __shared__ int redi[16];
  const SvdTask t = tasks[blockIdx.x];
  if (t.big_qr) return;   // multi-workgroup class
  const QrView q(t, work);
  if (!qr_init(t, q, S, red)) return;
  int gs = 64;
  while (gs > 4 && gs * q.n > (int)blockDim.x) gs >>= 1;
  const int gl = threadIdx.x % gs, grp = threadIdx.x / gs, ngrp = blockDim.x / gs;
  int r = 0;
  for (int k = 0; k < q.n; ++k) {
    if (!qr_head(q, k, red, redi)) break;
    for (int j = k + 1 + grp; j < q.n; j += ngrp) qr_apply_col(q, k, j, gl, gs);
    __syncthreads();
    r = k + 1;
  }
  qr_build_av(q, r);
}

// Multi-workgroup class (large matrices): one launch per phase and step; the
// rank is -2 while the factorisation runs.
__global__ __launch_bounds__(1024) void svd_qr_init_kernel(const int32_t* __restrict__ big,
                                                          const SvdTask* __restrict__ tasks,
                                                          double* __restrict__ work, double* __restrict__ S) {
  __shared__ double red[16];
  const SvdTask t = tasks[big[blockIdx.x]];
  const QrView q(t, work);
  if (qr_init(t, q, S, red) && threadIdx.x == 0) q.rank_out[0] = -2.0;
}
__global__ __launch_bounds__(1024) void svd_qr_head_kernel(const int32_t* __restrict__ big,
                                                          const SvdTask* __restrict__ tasks,
                                                          double* __restrict__ work, int k) {
  __shared__ double red[16];
  __shared__ int redi[16];
  const SvdTask t = tasks[big[blockIdx.x]];
  const QrView q(t, work);
  if (q.rank_out[0] != -2.0) return;   // finished (or non-finite)
  if (k >= q.n) {
    __syncthreads();
    if (threadIdx.x == 0) q.rank_out[0] = (double)q.n;
    return;
  }
  if (!qr_head(q, k, red, redi) && threadIdx.x == 0) q.rank_out[0] = (double)k;
}
// grid: (matrix, block of 16 columns); one wave per column
__global__ __launch_bounds__(1024) void svd_qr_apply_kernel(const SvdCols* __restrict__ cols,
                                                           const SvdTask* __restrict__ tasks,
                                                           double* __restrict__ work, int k) {
  const SvdCols cb = cols[blockIdx.x];
  const SvdTask t = tasks[cb.sec];
  const QrView q(t, work);
  if (q.rank_out[0] != -2.0) return;
  const int j = cb.col0 + (int)(threadIdx.x >> 6);
  if (j <= k || j >= q.n) return;   // wave-uniform; no barrier in this kernel
  qr_apply_col(q, k, j, threadIdx.x & 63, 64);
}
__global__ __launch_bounds__(1024) void svd_qr_finish_kernel(const int32_t* __restrict__ big,
                                                            const SvdTask* __restrict__ tasks,
                                                            double* __restrict__ work) {
  const SvdTask t = tasks[big[blockIdx.x]];
  const QrView q(t, work);
  const double rr = q.rank_out[0];
  if (rr == -1.0) return;   // non-finite
  const int r = rr == -2.0 ? q.n : (int)rr;
  __syncthreads();   // every thread has read the rank before it is rewritten
  qr_build_av(q, r);
}

// The rotation of a column pair with squared norms al, be and inner product
// ga, or false when the pair is left alone: |ga| <= tol sqrt(al be) (tested
// squared: no root), or a column at the rank threshold (squared norm <=
// thr2: rounding noise left by rotations, which would keep rotating against
// each other).  Rutishauser's formulas: zeta = (be - al) / (2 ga),
// t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)), c = 1 / sqrt(1 + t^2),
// s = c t; reciprocals and reciprocal roots from the hardware approximations
// refined by a Newton step (a few ulp, which the following sweeps absorb like
// any rounding of the rotation).
__device__ __forceinline__ bool svd_rotation(double al, double be, double ga, double thr2, double tol, double& cs,
                                             double& sn) {
  if (ga == 0.0 || al <= thr2 || be <= thr2 || ga * ga <= (tol * tol) * (al * be)) return false;
  auto rcp = [](double x) {
    double r = __builtin_amdgcn_rcp(x);
    return fma(r, fma(-x, r, 1.0), r);
  };
  auto rsq = [](double x) {
    double y = __builtin_amdgcn_rsq(x);
    return y * fma(-0.5 * x * y, y, 1.5);
  };
  const double zeta = (be - al) * rcp(2.0 * ga);
  const double az = fabs(zeta), sg = zeta >= 0.0 ? 1.0 : -1.0;
  const double z2 = fma(az, az, 1.0);
  // sqrt(1 + zeta^2) = (1 + zeta^2) rsq(1 + zeta^2); for |zeta| > 1e150 the
  // square overflows and t = 1 / (2 zeta) to working precision
  const double tt = az > 1e150 ? sg * 0.5 * rcp(az) : sg * rcp(az + z2 * rsq(z2));
  cs = rsq(fma(tt, tt, 1.0));
  sn = cs * tt;
  return true;
}

// One step of a block-Jacobi sweep: one workgroup (1024 threads) per block
// pair of a matrix, the pair's columns of AV held in LDS for one inner
// cyclic sweep.  rot[sec] is set to 1 when a rotation was applied; matrices
// with active[sec] == 0 have converged and are skipped.
constexpr int kSvdLds = 16384;   // doubles of LDS per workgroup (2 b (n + r) <= 4 b n)
__global__ __launch_bounds__(1024) void svd_bjac_kernel(const SvdPair* __restrict__ pairs,
                                                       const SvdTask* __restrict__ tasks, double* __restrict__ work,
                                                       const double* __restrict__ active, double* __restrict__ rot,
                                                       int step) {
  __shared__ double col[kSvdLds];
  __shared__ int rotated;
  const SvdPair pr = pairs[blockIdx.x];
  if (active[pr.sec] == 0.0) return;
  const SvdTask t = tasks[pr.sec];
  const int n = t.n, ld = 2 * n, b = t.b, nb = t.nb;
  if (step >= nb - 1) return;
  const double rr = work[t.aux_off + 4 * n];
  if (!(rr >= 2.0)) return;   // rank 0 or 1, or a non-finite matrix: nothing to rotate
  const int r = (int)rr;
  const double thr2 = work[t.aux_off + 4 * n + 1];
  auto player = [&](int j) { return j == 0 ? 0 : 1 + ((j - 1 + step) % (nb - 1)); };
  const int pa = player(pr.slot), pb = player(nb - 1 - pr.slot);
  const int I = min(pa, pb), J = max(pa, pb);
  const int vI = max(0, min(b, r - I * b)), vJ = max(0, min(b, r - J * b));
  const int nv = vI + vJ;
  if (nv <= 1) return;
  const int L = n + r;   // rows of AV in use
  double* AV = work + t.av_off;
  auto gcol = [&](int k) { return k < vI ? I * b + k : J * b + (k - vI); };
  const int tid = threadIdx.x, nthr = blockDim.x;
  // the pair's columns into LDS (nv * L <= kSvdLds: 32-bit index arithmetic),
  // eight loads of a thread in flight at a time
  const int ntot = nv * L;
  for (int e0 = tid; e0 < ntot; e0 += 8 * nthr) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * nthr;
      v[u] = 0.0;
      if (e < ntot) {
        const int k = e / L, i = e - k * L;
        v[u] = AV[(int64_t)gcol(k) * ld + i];
      }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (e0 + u * nthr < ntot) col[e0 + u * nthr] = v[u];
  }
  if (tid == 0) rotated = 0;
  __syncthreads();
  const double eps = 2.220446049250313e-16;
  const double tol = fmax(1e-15, 4.0 * n * eps);
  // Step 0 of a sweep runs a full cyclic sweep over all column pairs of the
  // union (this is where the pairs inside a block meet); the later steps
  // only rotate the vI x vJ pairs across the two blocks, in P = max(vI, vJ)
  // rounds of disjoint pairs (i, (i + t) mod P).
  const bool full = step == 0;
  const int ne = nv + (nv & 1);
  const int P = max(vI, vJ);
  const int hp = full ? ne / 2 : P;                  // pairs per round
  const int rounds = full ? ne - 1 : P;
  int gs = 64;
  while (gs * hp > nthr) gs >>= 1;
  const int gl = tid % gs, grp = tid / gs;
  double cs = 1.0, sn = 0.0;
  for (int st = 0; st < rounds; ++st) {
    int p = 0, q = nv;                                // q >= nv: no pair for this group
    if (grp < hp) {
      if (full) {
        auto pl = [&](int j) { return j == 0 ? 0 : 1 + ((j - 1 + st) % (ne - 1)); };
        const int a = pl(grp), c2 = pl(ne - 1 - grp);
        p = min(a, c2);
        q = max(a, c2);
      } else {
        const int i = grp, j = (grp + st) % P;
        if (i < vI && j < vJ) {
          p = i;
          q = vI + j;
        }
      }
    }
    if (q < nv) {
      double* ap = col + p * L;
      double* aq = col + q * L;
      double al = 0.0, be = 0.0, ga = 0.0;
      for (int i = gl; i < n; i += gs) {
        const double u = ap[i], w = aq[i];
        al += u * u;
        be += w * w;
        ga += u * w;
      }
      al = svd_group_sum(al, gs);
      be = svd_group_sum(be, gs);
      ga = svd_group_sum(ga, gs);
      if (svd_rotation(al, be, ga, thr2, tol, cs, sn)) {
        if (gl == 0) rotated = 1;
        for (int i = gl; i < L; i += gs) {
          const double u = ap[i], w = aq[i];
          ap[i] = cs * u - sn * w;
          aq[i] = sn * u + cs * w;
        }
      }
    }
    __syncthreads();
  }
  for (int e0 = tid; e0 < ntot; e0 += 8 * nthr) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = e0 + u * nthr < ntot ? col[e0 + u * nthr] : 0.0;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * nthr;
      if (e < ntot) {
        const int k = e / L, i = e - k * L;
        AV[(int64_t)gcol(k) * ld + i] = v[u];
      }
    }
  }
  if (tid == 0 && rotated) rot[pr.sec] = 1.0;
}

// Singular values, their order and the right vectors; one workgroup per matrix.
__global__ __launch_bounds__(1024) void svd_sort_kernel(const SvdTask* __restrict__ tasks, double* __restrict__ work,
                                                       double* __restrict__ U, double* __restrict__ S,
                                                       double* __restrict__ Vt) {
  const SvdTask t = tasks[blockIdx.x];
  const int n = t.n, ld = 2 * n;
  const double* aux = work + t.aux_off;
  const double rr = aux[4 * n];
  if (!(rr >= 0.0)) return;   // non-finite matrix: S holds NaN already
  const int r = (int)rr;
  const double* AV = work + t.av_off;
  const int* qperm = (const int*)(aux + 3 * n);   // after R diagonal, reflector factors, column norms
  double* sig = work + t.sig_off;
  int* perm = (int*)(work + t.perm_off);
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int lane = tid & 63, wave = tid >> 6, nw = nthr >> 6;
  for (int j = wave; j < r; j += nw) {
    double s2 = 0.0;
    for (int i = lane; i < n; i += 64) s2 += AV[(int64_t)j * ld + i] * AV[(int64_t)j * ld + i];
    for (int o = 32; o > 0; o >>= 1) s2 += __shfl_xor(s2, o, 64);
    if (lane == 0) sig[j] = sqrt(s2);
  }
  __syncthreads();
  for (int j = tid; j < r; j += nthr) {
    int rank = 0;
    for (int i = 0; i < r; ++i) rank += (sig[i] > sig[j]) || (sig[i] == sig[j] && i < j);
    perm[rank] = j;
  }
  __syncthreads();
  for (int e = tid; e < n; e += nthr) S[t.s_off + e] = e < r ? sig[perm[e]] : 0.0;
  double* Uo = U + t.u_off;     // rows x n (ld rows)
  double* Vo = Vt + t.vt_off;   // n x cols (ld n)
  // right vectors of X (length n): row qperm[i] of column jj = A(i, perm[jj]) / sigma
  for (int64_t e = tid; e < (int64_t)n * n; e += nthr) {
    const int i = (int)(e % n), jj = (int)(e / n);
    double vv = 0.0;
    if (jj < r) {
      const int j = perm[jj];
      const double sj = sig[j];
      vv = sj > 0.0 ? AV[(int64_t)j * ld + i] / sj : 0.0;
    }
    const int row = qperm[i];
    if (!t.transposed) Vo[jj + (int64_t)row * n] = vv;          // Vt(jj, row), cols = n
    else Uo[(int64_t)jj * t.rows + row] = vv;                   // U(row, jj), rows = n
  }
}

// Left vectors of X: column jj of Q [VJ(:, perm(jj)); 0], one wave per
// column (16 columns per workgroup), reflectors applied last to first.
__global__ __launch_bounds__(1024) void svd_left_kernel(const SvdCols* __restrict__ cols,
                                                       const SvdTask* __restrict__ tasks, double* __restrict__ work,
                                                       double* __restrict__ U, double* __restrict__ Vt) {
  const SvdCols cb = cols[blockIdx.x];
  const SvdTask t = tasks[cb.sec];
  const int m = t.m, n = t.n, ld = 2 * n;
  const double* aux = work + t.aux_off;
  const double rr = aux[4 * n];
  if (!(rr >= 0.0)) return;
  const int r = (int)rr;
  const double* X = work + t.x_off;
  const double* beta = aux + n;
  const double* AV = work + t.av_off;
  const int* perm = (const int*)(work + t.perm_off);
  double* Z = work + t.z_off;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int jj = cb.col0 + wave;
  if (jj >= n) return;   // wave-uniform; no block barrier below
  double* Uo = U + t.u_off;
  double* Vo = Vt + t.vt_off;
  if (jj >= r) {
    for (int i = lane; i < m; i += 64) {
      if (!t.transposed) Uo[(int64_t)jj * t.rows + i] = 0.0;
      else Vo[jj + (int64_t)i * n] = 0.0;
    }
    return;
  }
  double* z = Z + (int64_t)jj * m;
  const int j = perm[jj];
  for (int i = lane; i < m; i += 64) z[i] = i < r ? AV[(int64_t)j * ld + n + i] : 0.0;
  for (int k = r - 1; k >= 0; --k) {
    const double* v = X + (int64_t)k * m;
    double d = 0.0;
    for (int i = k + lane; i < m; i += 64) d += v[i] * z[i];
    for (int o = 32; o > 0; o >>= 1) d += __shfl_xor(d, o, 64);
    const double f = beta[k] * d;
    for (int i = k + lane; i < m; i += 64) z[i] -= f * v[i];
  }
  for (int i = lane; i < m; i += 64) {
    if (!t.transposed) Uo[(int64_t)jj * t.rows + i] = z[i];     // U(i, jj), rows = m
    else Vo[jj + (int64_t)i * n] = z[i];                        // Vt(jj, i), cols = m
  }
}

hipError_t launch_svd_qr(const void* d_tasks, int n, double* work, double* S, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(svd_qr_kernel, dim3((unsigned)n), dim3(1024), 0, s, (const SvdTask*)d_tasks, work, S);
  return hipGetLastError();
}
hipError_t launch_svd_qr_big(const void* d_big, int n_big, const void* d_cols, int n_cols, int n_max,
                             const void* d_tasks, double* work, double* S, hipStream_t s) {
  if (n_big == 0) return hipSuccess;
  hipLaunchKernelGGL(svd_qr_init_kernel, dim3((unsigned)n_big), dim3(1024), 0, s, (const int32_t*)d_big,
                     (const SvdTask*)d_tasks, work, S);
  for (int k = 0; k <= n_max; ++k) {
    hipLaunchKernelGGL(svd_qr_head_kernel, dim3((unsigned)n_big), dim3(1024), 0, s, (const int32_t*)d_big,
                       (const SvdTask*)d_tasks, work, k);
    if (k < n_max)
      hipLaunchKernelGGL(svd_qr_apply_kernel, dim3((unsigned)n_cols), dim3(1024), 0, s, (const SvdCols*)d_cols,
                         (const SvdTask*)d_tasks, work, k);
  }
  hipLaunchKernelGGL(svd_qr_finish_kernel, dim3((unsigned)n_big), dim3(1024), 0, s, (const int32_t*)d_big,
                     (const SvdTask*)d_tasks, work);
  return hipGetLastError();
}
hipError_t launch_svd_bjac(const void* d_pairs, int n_pairs, const void* d_tasks, double* work,
                           const double* active, double* rot, int step, hipStream_t s) {
  if (n_pairs == 0) return hipSuccess;
  hipLaunchKernelGGL(svd_bjac_kernel, dim3((unsigned)n_pairs), dim3(1024), 0, s, (const SvdPair*)d_pairs,
                     (const SvdTask*)d_tasks, work, active, rot, step);
  return hipGetLastError();
}
hipError_t launch_svd_finish(const void* d_tasks, int n, const void* d_cols, int n_cols, double* work, double* U,
                             double* S, double* Vt, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(svd_sort_kernel, dim3((unsigned)n), dim3(1024), 0, s, (const SvdTask*)d_tasks, work, U, S, Vt);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || n_cols == 0) return e;
  hipLaunchKernelGGL(svd_left_kernel, dim3((unsigned)n_cols), dim3(1024), 0, s, (const SvdCols*)d_cols,
                     (const SvdTask*)d_tasks, work, U, Vt);
  return hipGetLastError();
}

}  // namespace bsd
