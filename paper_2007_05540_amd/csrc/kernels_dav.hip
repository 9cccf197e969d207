// Device kernels of the Davidson routine (Alg. 1) for one or many independent
// problems.  Vectors span all problems of a plan; every reduction is split into
// fixed chunks that never straddle two problems and is finished in a fixed
// order, so results are bitwise reproducible.
#include <hip/hip_runtime.h>

#include "bsdmrg_internal.h"
#include "kernels.h"

namespace bsd {

constexpr int DT = 256;   // threads per block of the vector kernels
constexpr int PER = kChunk / DT;
constexpr int kMaxBasisD = 64;   // largest basis (J) of the multi-dot kernels

// Element i of a chunk-local array: a wave-uniform base plus a 32-bit byte
// offset (chunks hold kChunk elements), so loads and stores take a scalar base.
template <typename T>
__device__ __forceinline__ T ld_at(const T* base, unsigned i) {
  return *(const T*)((const char*)base + i * (unsigned)sizeof(T));
}
template <typename T>
__device__ __forceinline__ void st_at(T* base, unsigned i, T v) {
  *(T*)((char*)base + i * (unsigned)sizeof(T)) = v;
}

// Sum over the 64 lanes of a wave, the same value on every lane, in one
// fixed order: DPP exchanges inside each row of 16 lanes (pairs, quads, half
// rows, rows), then the four row sums read from lanes 0, 16, 32, 48 and
// added pairwise.  Register-only (no LDS crossbar); every lane must be active.
template <int CTRL>
__device__ __forceinline__ double mov_dpp_d(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, true);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double readlane_d(double v, int l) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane((int)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}
// old with lane l replaced by v (a per-lane select)
template <typename T>
__device__ __forceinline__ T writelane(T v, int l, T old) {
  return (int)(threadIdx.x & 63) == l ? v : old;
}
__device__ __forceinline__ double wave_total(double v) {
  v += mov_dpp_d<0xB1>(v);    // quad_perm [1,0,3,2]: lane ^ 1
  v += mov_dpp_d<0x4E>(v);    // quad_perm [2,3,0,1]: lane ^ 2
  v += mov_dpp_d<0x141>(v);   // row_half_mirror: the other quad of the half row
  v += mov_dpp_d<0x140>(v);   // row_mirror: the other half of the row
  return (readlane_d(v, 0) + readlane_d(v, 16)) + (readlane_d(v, 32) + readlane_d(v, 48));
}

// Sum over the threads of a block: wave sums, then the wave sums added in
// wave order by thread 0; the result is returned to every thread.
__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = wave_total(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) / 64;
    for (int w = 0; w < nw; ++w) r += sh[w];
    sh[8] = r;
  }
  __syncthreads();
  return sh[8];
}

__device__ __forceinline__ double wave_sum(double v) { return wave_total(v); }

// Ordering of LDS traffic between the lanes of one wave (code run by a
// single wave): LDS operations of a wave complete in order; the fence makes
// the compiler wait for them and keeps it from moving accesses across.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// out[j] = sum over the problem's chunks of part[j * nct + chunk] for j < J
// (thread-strided sums, then the deterministic block tree); result in LDS.
__device__ __forceinline__ void sum_partials(const double* __restrict__ part, int nct, const DavProb& pr,
                                             int J, double* out, double* sh) {
  for (int j = 0; j < J; ++j) {
    const double* col = part + (int64_t)j * nct + pr.chunk0;
    double v = 0.0;
    int c = threadIdx.x;
    for (; c + 7 * (int)blockDim.x < pr.nchunk; c += 8 * blockDim.x) {
      double t[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) t[u] = col[c + u * blockDim.x];
#pragma unroll
      for (int u = 0; u < 8; ++u) v += t[u];
    }
    for (; c < pr.nchunk; c += blockDim.x) v += col[c];
    v = block_sum(v, sh);
    if (threadIdx.x == 0) out[j] = v;
  }
  __syncthreads();
}

// red[p * ldr + j] = sum over problem p's chunks of part[j * nct + chunk]
// (grid: problems x J); one fixed reduction order.
__global__ __launch_bounds__(DT) void psum_kernel(const DavProb* __restrict__ probs, int nct, int J,
                                                  const double* __restrict__ part, int ldr,
                                                  double* __restrict__ red) {
  __shared__ double sh[16];
  const int p = blockIdx.x, j = blockIdx.y;
  const DavProb pr = probs[p];
  const double* col = part + (int64_t)j * nct + pr.chunk0;
  // the loads of a thread are issued together (they are independent), then
  // added in chunk order
  double v = 0.0;
  int c = threadIdx.x;
  for (; c + 7 * DT < pr.nchunk; c += 8 * DT) {
    double t[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) t[u] = col[c + u * DT];
#pragma unroll
    for (int u = 0; u < 8; ++u) v += t[u];
  }
  for (; c < pr.nchunk; c += DT) v += col[c];
  v = block_sum(v, sh);
  if (threadIdx.x == 0) red[(int64_t)p * ldr + j] = v;
}

// part[j * nct + ch] = sum_{e in chunk ch} X_j[e] y[e], j < J (wave sums
// per j, one barrier, the four wave sums added in order).
template <typename TX>
__global__ __launch_bounds__(DT) void dots_kernel(const Chunk* __restrict__ chunks, int nct, int J,
                                                  const TX* __restrict__ X, int64_t xstride,
                                                  const double* __restrict__ y, double* __restrict__ part,
                                                  int norm_col) {
  __shared__ double ws[kMaxBasisD + 1][4];
  const Chunk ch = chunks[blockIdx.x];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double yv[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = threadIdx.x + u * DT;
    yv[u] = e < ch.len ? ld_at(y + ch.start, e) : 0.0;
  }
#pragma unroll 4
  for (int j = 0; j < J; ++j) {
    const TX* Xj = X + j * xstride + ch.start;
    double s = 0.0;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = threadIdx.x + u * DT;
      if (e < ch.len) s += (double)ld_at(Xj, e) * yv[u];
    }
    s = wave_sum(s);
    if (lane == 0) ws[j][wave] = s;
  }
  // column J: ||y||^2 (the norm column read by the first Gram-Schmidt pass)
  if (norm_col) {
    double s = 0.0;
#pragma unroll
    for (int u = 0; u < PER; ++u) s += yv[u] * yv[u];
    s = wave_sum(s);
    if (lane == 0) ws[J][wave] = s;
  }
  __syncthreads();
  if ((int)threadIdx.x < J + (norm_col ? 1 : 0)) {
    const int j = threadIdx.x;
    part[(int64_t)j * nct + blockIdx.x] = ((ws[j][0] + ws[j][1]) + ws[j][2]) + ws[j][3];
  }
}

// y = x / ||x||_p with ||x||_p^2 = red[p * ldr].
__global__ __launch_bounds__(DT) void normalize_kernel(const Chunk* __restrict__ chunks, int ldr,
                                                       const double* __restrict__ red,
                                                       const double* __restrict__ x,
                                                       double* __restrict__ y) {
  const Chunk ch = chunks[blockIdx.x];
  const double inv = 1.0 / sqrt(red[(int64_t)ch.prob * ldr]);
  for (int e = threadIdx.x; e < ch.len; e += DT) y[ch.start + e] = x[ch.start + e] * inv;
}

constexpr int kMaxBasis = 64;
constexpr int GT = 64;   // one wave

// A[r][c] = Mp[r * B + c] for r, c < n (lane r loads row r; the loads of a
// group of G are issued before any of them is stored).
template <int G>
__device__ __forceinline__ void load_rows(double (*A)[kMaxBasis + 1], const double* __restrict__ Mp, int B, int n,
                                          int lane) {
  if (lane >= n) return;
  const double* row = Mp + (int64_t)lane * B;
  for (int c0 = 0; c0 < n; c0 += G) {
    double t[G];
#pragma unroll
    for (int u = 0; u < G; ++u) t[u] = c0 + u < n ? row[c0 + u] : 0.0;
#pragma unroll
    for (int u = 0; u < G; ++u)
      if (c0 + u < n) A[lane][c0 + u] = t[u];
  }
}

// Householder tridiagonalisation of the leading n x n block of A (n <= R,
// R = 16 or 32) held in registers: row r is split over LPR = 64 / R lanes
// (lanes r * LPR .. r * LPR + LPR - 1), lane r * LPR + q holding columns
// q * C .. q * C + C - 1 (C = R / LPR), so all 64 lanes share the products.
// Step k: the reflector v (zero in entries 0..k) from column k below the
// diagonal, p = A v (partial sums over a lane's columns, added across the
// row's lanes in one fixed order), beta = v^T p, w = p - beta v and the
// rank-2 update A -= 2 (v w^T + w v^T); v and w reach every lane through LDS
// (Vh and the scratch row ws).  The Householder vectors go to Vh (entries of
// rows R..63 are not written), the diagonal and off-diagonal of T to d and e.
// Run by one wave.
template <int R>
__device__ __forceinline__ void tridiag_in_registers(const double (*A)[kMaxBasis + 1], double (*Vh)[kMaxBasis],
                                                     double* d, double* e, double* ws, int n, int lane) {
  constexpr int LPR = 64 / R, C = R / LPR;
  static_assert(LPR == 2 || LPR == 4, "rows split over two or four lanes");
  const int row = lane / LPR, q = lane % LPR;
  double ar[C];
#pragma unroll
  for (int t = 0; t < C; ++t) {
    const int c = q * C + t;
    ar[t] = (row < n && c < n) ? A[row][c] : 0.0;
  }
#pragma unroll
  for (int k = 0; k + 2 < R; ++k) {
    if (k + 2 < n) {
      const int qk = k / C, tk = k % C;   // owner lane (within the row) and register of column k
      // x_row = A[row][k] on every lane of the row
      double xk = ar[tk];
      if (LPR == 4) {
        if (qk == 0) xk = mov_dpp_d<0x00>(xk);
        else if (qk == 1) xk = mov_dpp_d<0x55>(xk);
        else if (qk == 2) xk = mov_dpp_d<0xAA>(xk);
        else xk = mov_dpp_d<0xFF>(xk);
      } else {
        if (qk == 0) xk = mov_dpp_d<0xA0>(xk);   // quad_perm [0,0,2,2]
        else xk = mov_dpp_d<0xF5>(xk);           // quad_perm [1,1,3,3]
      }
      const bool mine = row > k && row < n;
      const double xr = mine ? xk : 0.0;
      const double nrm2 = wave_total(q == 0 ? xr * xr : 0.0);
      const double x0 = readlane_d(xk, (k + 1) * LPR);
      const double alpha = nrm2 > 0.0 ? -copysign(sqrt(nrm2), x0) : 0.0;
      const double vn2 = 2.0 * (nrm2 - alpha * x0);   // ||x - alpha e_{k+1}||^2
      const double vr = vn2 > 0.0 ? (xr - (row == k + 1 ? alpha : 0.0)) / sqrt(vn2) : 0.0;
      if (q == 0) Vh[k][row] = vr;
      const double dk = readlane_d(ar[tk], k * LPR + qk);
      if (lane == 0) {
        d[k] = dk;
        e[k] = alpha;
      }
      if (vn2 > 0.0) {
        wave_sync();   // Vh[k] complete before it is read back
        // v is zero in entries 0..k, so columns up to k add nothing
        double vc[C];
        double pp = 0.0;
#pragma unroll
        for (int t = 0; t < C; ++t) vc[t] = Vh[k][q * C + t];
#pragma unroll
        for (int t = 0; t < C; ++t) pp += ar[t] * vc[t];
        pp += mov_dpp_d<0xB1>(pp);                  // lane ^ 1
        if (LPR == 4) pp += mov_dpp_d<0x4E>(pp);    // lane ^ 2
        const double pr = mine ? pp : 0.0;
        const double beta = wave_total(q == 0 ? vr * pr : 0.0);
        const double wr = pr - beta * vr;
        if (q == 0) ws[row] = wr;
        wave_sync();
        double wc[C];
#pragma unroll
        for (int t = 0; t < C; ++t) wc[t] = ws[q * C + t];
#pragma unroll
        for (int t = 0; t < C; ++t) ar[t] -= 2.0 * (vr * wc[t] + wr * vc[t]);
        wave_sync();   // ws read by every lane before the next step writes it
      }
    }
  }
  // the last 2 x 2 block: element (r, c) is register c % C of lane r * LPR + c / C
  double dl = 0.0, dm = 0.0, el = 0.0;
  const int c0 = n - 2, c1 = n - 1;
#pragma unroll
  for (int t = 0; t < C; ++t) {
    if (c0 >= 0 && c0 % C == t) {
      dl = readlane_d(ar[t], c0 * LPR + c0 / C);
      el = readlane_d(ar[t], c1 * LPR + c0 / C);
    }
    if (c1 % C == t) dm = readlane_d(ar[t], c1 * LPR + c1 / C);
  }
  if (lane == 0) {
    if (n >= 2) {
      d[n - 2] = dl;
      e[n - 2] = el;
    }
    d[n - 1] = dm;
  }
}

// Gram row m_ij = m_ji = (v^A_j)^T v_i (j <= i) from the chunk partials (all
// GE_T threads: wave w sums columns w, w + 16, ... over the problem's chunks,
// each lane a chunk stride of 64 in chunk order, then the wave sum), then
// the lowest eigenpair of the (i+1) x (i+1) projected matrix M in the first
// wave (no step needs more than a wave-level reduction):
//  1. Householder tridiagonalisation T = Q^T M Q, Q = H_0 ... H_{n-3},
//     H_k = I - 2 v_k v_k^T;
//  2. the lowest eigenvalue of T by multisection on Sturm counts: the
//     bracket starts as the Gershgorin interval, one round of 64 shifts
//     spaced geometrically around the previous step's eigenvalue narrows it
//     (from the second step of a solve on), then each round the 64 lanes
//     test 64 equally spaced shifts inside it and it shrinks 65-fold, until
//     its width is 4 eps of the eigenvalue's magnitude;
//  3. its eigenvector by the twisted factorisation of T - lambda I;
//  4. back-transformation x = Q y.
constexpr int GE_T = 1024;
__global__ __launch_bounds__(GE_T) void gram_eig_kernel(const DavProb* __restrict__ probs, int nct,
                                                        const double* __restrict__ part, int i, int B,
                                                        double* __restrict__ M, double* __restrict__ svec,
                                                        double* __restrict__ lam, double* __restrict__ svec_prev) {
  __shared__ double A[kMaxBasis][kMaxBasis + 1];
  __shared__ double Vh[kMaxBasis][kMaxBasis];
  __shared__ double d[kMaxBasis], e[kMaxBasis], vb[kMaxBasis], wb[kMaxBasis], rowsum[kMaxBasis];
  const int p = blockIdx.x, lane = threadIdx.x & 63, wave = threadIdx.x >> 6, n = i + 1;
  double* Mp = M + (int64_t)p * B * B;
  // the first wave's loads go out first and complete during the sums: the
  // previous step's eigenvalue (written by this kernel's previous call in
  // the same solve; the first call of a solve has i = 0), the previous Ritz
  // vector (read before svec is overwritten below) and, up to order 16, the
  // stored rows (lane r reads row r)
  double lam_prev = 0.0, sp = 0.0, mrow[16];
  if (wave == 0) {
    lam_prev = i > 0 ? lam[p] : 0.0;
    sp = svec_prev && lane < i ? svec[(int64_t)p * B + lane] : 0.0;
#pragma unroll
    for (int c = 0; c < 16; ++c) mrow[c] = n <= 16 && lane < i && c < i ? Mp[(int64_t)lane * B + c] : 0.0;
  }
  {
    const DavProb pr = probs[p];
    for (int j = wave; j <= i; j += GE_T / 64) {
      const double* col = part + (int64_t)j * nct + pr.chunk0;
      double v = 0.0;
      int c = lane;
      for (; c + 15 * 64 < pr.nchunk; c += 16 * 64) {
        double t[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) t[u] = col[c + u * 64];
#pragma unroll
        for (int u = 0; u < 16; ++u) v += t[u];
      }
      for (; c < pr.nchunk; c += 64) v += col[c];
      v = wave_total(v);
      if (lane == 0) rowsum[j] = v;
    }
  }
  __syncthreads();
  if (wave != 0) return;
  // the new row and column from the sums, the rest from the stored matrix
  const double rv = lane <= i ? rowsum[lane] : 0.0;
  if (n <= 16) {
    if (lane < i) {
#pragma unroll
      for (int c = 0; c < 16; ++c)
        if (c < i) A[lane][c] = mrow[c];
    }
  } else {
    load_rows<8>(A, Mp, B, i, lane);
  }
  if (svec_prev && lane <= i) svec_prev[(int64_t)p * B + lane] = sp;
  if (lane < i) {
    A[i][lane] = rv;
    A[lane][i] = rv;
  }
  if (lane == i) A[i][i] = rv;
  if (lane <= i) {
    Mp[i * B + lane] = rv;
    Mp[lane * B + i] = rv;
  }
  wave_sync();
  // 1. tridiagonalisation (lane r owns row r of the trailing block).  Up to
  // 16 or 32 rows the row is held in registers (tridiag_in_registers);
  // larger matrices stay in LDS.
  if (n <= 16) {
    tridiag_in_registers<16>(A, Vh, d, e, vb, n, lane);
  } else if (n <= 32) {
    tridiag_in_registers<32>(A, Vh, d, e, vb, n, lane);
  } else {
    for (int k = 0; k + 2 < n; ++k) {
      const bool mine = lane > k && lane < n;
      const double xr = mine ? A[lane][k] : 0.0;
      const double nrm2 = wave_total(xr * xr);
      const double x0 = A[k + 1][k];
      const double alpha = nrm2 > 0.0 ? -copysign(sqrt(nrm2), x0) : 0.0;
      const double vn2 = 2.0 * (nrm2 - alpha * x0);   // ||x - alpha e_{k+1}||^2
      const double vr = vn2 > 0.0 ? (xr - (lane == k + 1 ? alpha : 0.0)) / sqrt(vn2) : 0.0;
      vb[lane] = vr;
      Vh[k][lane] = vr;
      if (lane == 0) {
        d[k] = A[k][k];
        e[k] = alpha;
      }
      wave_sync();
      if (vn2 > 0.0) {
        // four partial sums so that the LDS loads of a row are in flight together
        double p0 = 0.0, p1 = 0.0, p2 = 0.0, p3 = 0.0;
        if (mine) {
          int c = k + 1;
          for (; c + 3 < n; c += 4) {
            p0 += A[lane][c] * vb[c];
            p1 += A[lane][c + 1] * vb[c + 1];
            p2 += A[lane][c + 2] * vb[c + 2];
            p3 += A[lane][c + 3] * vb[c + 3];
          }
          for (; c < n; ++c) p0 += A[lane][c] * vb[c];
        }
        const double pr = (p0 + p1) + (p2 + p3);
        const double beta = wave_total(vr * pr);
        const double wr = pr - beta * vr;
        wb[lane] = wr;
        wave_sync();
        if (mine) {
#pragma unroll 4
          for (int c = k + 1; c < n; ++c) A[lane][c] -= 2.0 * (vr * wb[c] + wr * vb[c]);
        }
        wave_sync();
      }
    }
    if (lane == 0) {
      if (n >= 2) {
        d[n - 2] = A[n - 2][n - 2];
        e[n - 2] = A[n - 1][n - 2];
      }
      d[n - 1] = A[n - 1][n - 1];
    }
  }
  wave_sync();
  // 2. multisection for the lowest eigenvalue of T
  double glo = 1e308, ghi = -1e308, tn = 0.0, emax2 = 0.0;
  if (lane < n) {
    const double el = lane > 0 ? fabs(e[lane - 1]) : 0.0, er = lane < n - 1 ? fabs(e[lane]) : 0.0;
    glo = d[lane] - el - er;
    ghi = d[lane] + el + er;
    tn = fabs(d[lane]) + el + er;
    emax2 = er * er;
  }
  for (int o = 32; o > 0; o >>= 1) {
    glo = fmin(glo, __shfl_xor(glo, o, 64));
    ghi = fmax(ghi, __shfl_xor(ghi, o, 64));
    tn = fmax(tn, __shfl_xor(tn, o, 64));
    emax2 = fmax(emax2, __shfl_xor(emax2, o, 64));
  }
  const double eps = 2.220446049250313e-16;
  const double pivmin = 2.2250738585072014e-308 * fmax(1.0, emax2);
  double lo = glo - 2.0 * eps * tn - pivmin, hi = ghi + 2.0 * eps * tn + pivmin;
  // squared off-diagonal in LDS once (the Sturm recurrence reads it every round)
  if (lane + 1 < n) wb[lane] = e[lane] * e[lane];
  wave_sync();
  // number of eigenvalues of T below sigma (Sturm count of the LDL^T pivots).
  // One shift per lane: the recurrence is bound by the issue of its FP64
  // reciprocal and FMAs, so interleaving several shifts per lane costs about
  // proportionally more per round than it saves in rounds.
  auto count_below = [&](double sigma) {
    int cnt = 0;
    double q = d[0] - sigma;
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += q < 0.0;
#pragma unroll 4
    for (int j = 1; j < n; ++j) {
      // e_{j-1}^2 / q with the hardware reciprocal refined by one Newton step
      // (relative error ~1e-16, like a rounded division; only the sign of the
      // recurrence is used)
      double r = __builtin_amdgcn_rcp(q);
      r = fma(r, fma(-q, r, 1.0), r);
      q = (d[j] - sigma) - wb[j - 1] * r;
      if (fabs(q) < pivmin) q = -pivmin;
      cnt += q < 0.0;
    }
    return cnt;
  };
  // The 64 shifts of a round ascend with the lane.  The bracket becomes
  // [shift f - 1, shift f] for the first lane f whose count is >= 1 (lo kept
  // when f = 0), or [last shift, hi] when none is, so count(lo) = 0 and
  // count(hi) >= 1 hold throughout.
  auto narrow = [&](double sigma) {
    const unsigned long long below = __ballot(count_below(sigma) >= 1);
    if (below) {
      const int first = __ffsll((long long)below) - 1;
      hi = fmin(hi, readlane_d(sigma, first));
      if (first > 0) lo = fmax(lo, readlane_d(sigma, first - 1));
    } else {
      lo = fmax(lo, readlane_d(sigma, GT - 1));
    }
  };
  // a first round of shifts spaced geometrically on both sides of the
  // previous step's eigenvalue (32 a side, distances 2^-50 .. 2^12 of its
  // magnitude, ratio 4): the lowest eigenvalue moves little from step to
  // step, so the bracket usually shrinks to a few times the move at once.
  // Only a guess: the bracket rules above hold whatever it finds.
  if (i > 0 && isfinite(lam_prev)) {
    const double scale = fmax(fabs(lam_prev), 1e-3 * tn);
    const int side = lane < 32 ? 31 - lane : lane - 32;   // 0 nearest .. 31 farthest
    const double off = scale * exp2(-50.0 + 2.0 * (double)side);
    narrow(lane < 32 ? lam_prev - off : lam_prev + off);
  }
  // then rounds of 64 equally spaced shifts inside the bracket
  for (int round = 0; round < 24; ++round) {
    const double width = hi - lo;
    if (!(width > 4.0 * eps * fmax(fabs(lo), fabs(hi))) || width <= pivmin) break;
    narrow(lo + width * (double)(lane + 1) / (double)(GT + 1));
  }
  const double lambda = 0.5 * (lo + hi);
  // 3. the eigenvector of T for lambda by the twisted factorisation
  // (Dhillon and Parlett's "getvec"): the pivots of T - lambda I = L+ D+ L+^T
  // (forward) and = U- D- U-^T (backward), the twist index r where
  // |gamma_r| = |D+_r + D-_r - (d_r - lambda)| is smallest, z_r = 1 and the
  // other entries by the two recurrences outward from r.  The recurrences
  // are sequential: every lane runs them on the same (uniform) values read
  // from LDS (d, e, and e^2 in wb), and lane 0 stores the pivots and the
  // entries to scratch rows of A (free after the tridiagonalisation).  A
  // pivot of magnitude below pivmin is replaced by -pivmin (as in the Sturm
  // counts); the reciprocals use the hardware reciprocal refined by one
  // Newton step.
  auto recip = [](double q) {
    double r = __builtin_amdgcn_rcp(q);
    return fma(r, fma(-q, r, 1.0), r);
  };
  double* Dp = A[0];
  double* Dm = A[1];
  double* Y = A[2];
  double yv;
  if (!(tn > 0.0) || n == 1) {   // T = 0 or 1 x 1: a unit vector is an eigenvector
    yv = lane == 0 ? 1.0 : 0.0;
  } else {
    // the forward and the backward recurrence side by side (independent)
    double fw = d[0] - lambda, bw = d[n - 1] - lambda;
    if (fabs(fw) < pivmin) fw = -pivmin;
    if (fabs(bw) < pivmin) bw = -pivmin;
    if (lane == 0) {
      Dp[0] = fw;
      Dm[n - 1] = bw;
    }
#pragma unroll 2
    for (int k = 0; k + 1 < n; ++k) {
      const int kb = n - 2 - k;
      fw = (d[k + 1] - lambda) - wb[k] * recip(fw);
      bw = (d[kb] - lambda) - wb[kb] * recip(bw);
      if (fabs(fw) < pivmin) fw = -pivmin;
      if (fabs(bw) < pivmin) bw = -pivmin;
      if (lane == 0) {
        Dp[k + 1] = fw;
        Dm[kb] = bw;
      }
    }
    wave_sync();
    // twist index: the smallest |gamma_k| (the lowest k among equal ones)
    double g = lane < n ? fabs(Dp[lane] + Dm[lane] - (d[lane] - lambda)) : 1e308;
    int r = lane;
    for (int o = 32; o > 0; o >>= 1) {
      const double go = __shfl_xor(g, o, 64);
      const int ro = __shfl_xor(r, o, 64);
      if (go < g || (go == g && ro < r)) {
        g = go;
        r = ro;
      }
    }
    // z_r = 1; z_k = -(e_k / D+_k) z_{k+1} below r; z_{k+1} = -(e_k / D-_{k+1}) z_k above r
    if (lane == 0) Y[r] = 1.0;
    double z = 1.0;
    for (int k = r - 1; k >= 0; --k) {
      z = -e[k] * recip(Dp[k]) * z;
      if (lane == 0) Y[k] = z;
    }
    z = 1.0;
    for (int k = r; k + 1 < n; ++k) {
      z = -e[k] * recip(Dm[k + 1]) * z;
      if (lane == 0) Y[k + 1] = z;
    }
    wave_sync();
    yv = lane < n ? Y[lane] : 0.0;
    // unit length; the sign that makes the entries sum to a positive value
    // (the sign inverse iteration from the constant vector would give)
    const double nrm = sqrt(wave_total(yv * yv));
    const double sum = wave_total(yv);
    yv *= (sum < 0.0 ? -1.0 : 1.0) / nrm;
  }
  // 4. x = H_0 (H_1 (... (H_{n-3} y))) (entries of Vh past n are not read)
  double xr = lane < n ? yv : 0.0;
  for (int k = n - 3; k >= 0; --k) {
    const double v = lane < n ? Vh[k][lane] : 0.0;
    const double dv = wave_total(v * xr);
    xr -= 2.0 * dv * v;
  }
  if (lane < n) svec[(int64_t)p * B + lane] = xr;
  if (lane == 0) lam[p] = lambda;
}

// q = sum s_j v^A_j - lambda sum s_j v_j with partial ||q||^2; when x is
// non-null the Ritz vector x = sum s_j v_j is stored too, and when part_d is
// non-null the partial dots v_j^T q (the first Gram-Schmidt pass, columns
// j < J) and the partial ||q||^2 again (column J) as well.
//
// JR > 0 (J <= JR): the loop over the basis is unrolled JR times and the
// chunk's basis values stay in registers for the Gram-Schmidt dots (the
// same arithmetic in the same order as JR = 0).
template <int JR, typename TV>
__global__ __launch_bounds__(DT) void ritz_kernel(const Chunk* __restrict__ chunks, int nct, int J, int B,
                                                  const double* __restrict__ V, const TV* __restrict__ VA,
                                                  int64_t stride, const double* __restrict__ svec,
                                                  const double* __restrict__ lam, double* __restrict__ x,
                                                  double* __restrict__ q, double* __restrict__ part,
                                                  double* __restrict__ part_d, double* __restrict__ part_res,
                                                  const double* __restrict__ D) {
  __shared__ double ws[kMaxBasisD + 2][4];
  __shared__ double sv[kMaxBasis];
  const Chunk ch = chunks[blockIdx.x];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if ((int)threadIdx.x < J) sv[threadIdx.x] = svec[(int64_t)ch.prob * B + threadIdx.x];
  __syncthreads();
  const double l = lam[ch.prob];
  // positive preconditioner max(D - lambda, floor): amplification bounded by
  // 1 / floor (the plain D - lambda meets near-zero denominators while the
  // Ritz value is above some diagonal entries)
  const double floor_p = 1e-3 * fmax(fabs(l), 1.0);
  double qv[PER];
  double vr[JR > 0 ? JR : 1][PER];
  double nrm = 0.0, res = 0.0;
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = threadIdx.x + u * DT;
    qv[u] = 0.0;
#pragma unroll
    for (int j = 0; j < (JR > 0 ? JR : 1); ++j) vr[j][u] = 0.0;
    if (e >= ch.len) continue;
    double xv = 0.0, av = 0.0;
    if (JR > 0) {
#pragma unroll
      for (int j = 0; j < (JR > 0 ? JR : 1); ++j)
        if (j < J) {
          const double vv = ld_at(V + j * stride + ch.start, e);
          vr[j][u] = vv;
          xv += sv[j] * vv;
          av += sv[j] * (double)ld_at(VA + j * stride + ch.start, e);
        }
    } else {
#pragma unroll 4
      for (int j = 0; j < J; ++j) {
        xv += sv[j] * ld_at(V + j * stride + ch.start, e);
        av += sv[j] * (double)ld_at(VA + j * stride + ch.start, e);
      }
    }
    const double r = av - l * xv;
    res += r * r;
    double v = r;
    if (D) v = r / fmax(ld_at(D + ch.start, e) - l, floor_p);
    if (x) st_at(x + ch.start, e, xv);
    st_at(q + ch.start, e, v);
    qv[u] = v;
    nrm += v * v;
  }
  nrm = wave_sum(nrm);
  if (lane == 0) ws[kMaxBasisD][wave] = nrm;
  res = wave_sum(res);
  if (lane == 0) ws[kMaxBasisD + 1][wave] = res;
  if (part_d) {
    if (JR > 0) {
#pragma unroll
      for (int j = 0; j < (JR > 0 ? JR : 1); ++j)
        if (j < J) {
          double d = 0.0;
#pragma unroll
          for (int u = 0; u < PER; ++u) {
            const int e = threadIdx.x + u * DT;
            if (e < ch.len) d += vr[j][u] * qv[u];
          }
          d = wave_sum(d);
          if (lane == 0) ws[j][wave] = d;
        }
    } else {
#pragma unroll 4
      for (int j = 0; j < J; ++j) {
        double d = 0.0;
#pragma unroll
        for (int u = 0; u < PER; ++u) {
          const int e = threadIdx.x + u * DT;
          if (e < ch.len) d += ld_at(V + j * stride + ch.start, e) * qv[u];
        }
        d = wave_sum(d);
        if (lane == 0) ws[j][wave] = d;
      }
    }
  }
  __syncthreads();
  if (threadIdx.x == 0)
    part[blockIdx.x] = ((ws[kMaxBasisD][0] + ws[kMaxBasisD][1]) + ws[kMaxBasisD][2]) + ws[kMaxBasisD][3];
  if (threadIdx.x == 0)
    part_res[blockIdx.x] =
        ((ws[kMaxBasisD + 1][0] + ws[kMaxBasisD + 1][1]) + ws[kMaxBasisD + 1][2]) + ws[kMaxBasisD + 1][3];
  if (part_d && (int)threadIdx.x < J) {
    const int j = threadIdx.x;
    part_d[(int64_t)j * nct + blockIdx.x] = ((ws[j][0] + ws[j][1]) + ws[j][2]) + ws[j][3];
  }
  // column J of the first-pass partials: ||q||^2 before orthogonalisation
  if (part_d && threadIdx.x == 0)
    part_d[(int64_t)J * nct + blockIdx.x] =
        ((ws[kMaxBasisD][0] + ws[kMaxBasisD][1]) + ws[kMaxBasisD][2]) + ws[kMaxBasisD][3];
}

// First classical Gram-Schmidt pass q -= sum_j c_j v_j with c_j = red[p * ldr + j];
// red[p * ldr + J] holds ||q||^2 before the pass, kept in nq0[p].  Writes the
// partial dots v_j^T q of the result (columns j < J: the coefficients of a
// second pass) and its partial ||q||^2 (column J).
// JR > 0 (J <= JR): the basis loop unrolled JR times and the chunk's basis
// values kept in registers for the dots (same arithmetic and order).
template <int JR>
__global__ __launch_bounds__(DT) void update_kernel(const Chunk* __restrict__ chunks, int nct, int J,
                                                    const double* __restrict__ V, int64_t stride, int ldr,
                                                    const double* __restrict__ red,
                                                    double* __restrict__ q, double* __restrict__ part_out,
                                                    double* __restrict__ nq0) {
  __shared__ double cj[kMaxBasis];
  __shared__ double wsum[kMaxBasisD][4];
  const Chunk ch = chunks[blockIdx.x];
  if ((int)threadIdx.x < J) cj[threadIdx.x] = red[(int64_t)ch.prob * ldr + threadIdx.x];
  if (threadIdx.x == 0) nq0[ch.prob] = red[(int64_t)ch.prob * ldr + J];   // same value from every block
  __syncthreads();
  double qv[PER];
  double vr[JR > 0 ? JR : 1][PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = threadIdx.x + u * DT;
#pragma unroll
    for (int j = 0; j < (JR > 0 ? JR : 1); ++j) vr[j][u] = 0.0;
    if (e < ch.len) {
      double v = ld_at(q + ch.start, e);
      if (JR > 0) {
#pragma unroll
        for (int j = 0; j < (JR > 0 ? JR : 1); ++j)
          if (j < J) {
            const double vv = ld_at(V + j * stride + ch.start, e);
            vr[j][u] = vv;
            v -= cj[j] * vv;
          }
      } else {
#pragma unroll 4
        for (int j = 0; j < J; ++j) v -= cj[j] * ld_at(V + j * stride + ch.start, e);
      }
      st_at(q + ch.start, e, v);
      qv[u] = v;
    } else {
      qv[u] = 0.0;
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (JR > 0) {
#pragma unroll
    for (int j = 0; j < (JR > 0 ? JR : 1); ++j)
      if (j < J) {
        double s = 0.0;
#pragma unroll
        for (int u = 0; u < PER; ++u) {
          const int e = threadIdx.x + u * DT;
          if (e < ch.len) s += vr[j][u] * qv[u];
        }
        s = wave_sum(s);
        if (lane == 0) wsum[j][wave] = s;
      }
  } else {
#pragma unroll 4
    for (int j = 0; j < J; ++j) {
      double s = 0.0;
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int e = threadIdx.x + u * DT;
        if (e < ch.len) s += ld_at(V + j * stride + ch.start, e) * qv[u];
      }
      s = wave_sum(s);
      if (lane == 0) wsum[j][wave] = s;
    }
  }
  double s = 0.0;
#pragma unroll
  for (int u = 0; u < PER; ++u) s += qv[u] * qv[u];
  s = wave_sum(s);
  if (lane == 0) wsum[J][wave] = s;
  __syncthreads();
  if ((int)threadIdx.x <= J) {
    const int j = threadIdx.x;
    part_out[(int64_t)j * nct + blockIdx.x] = ((wsum[j][0] + wsum[j][1]) + wsum[j][2]) + wsum[j][3];
  }
}

// The new basis vector v_i (i = J - 1) and its product from t (after the
// first pass, in q) and the raw product H t (in VA_i): with the deferred
// second-pass coefficients c (when p2[p] is set)
//   v_i = s (t - sum_k c_k v_k),   H v_i = s (H t - sum_k c_k H v_k)
// (H is linear, so the product of the corrected vector is the corrected
// product), s = scale[p]; both are stored, then the Gram row partials
// part[c * nct + chunk] = sum over the chunk of (H v_c)[e] v_i[e], c <= i.
template <typename TV>
__global__ __launch_bounds__(DT) void fresh_dots_kernel(const Chunk* __restrict__ chunks, int nct, int J,
                                                        double* __restrict__ V, TV* __restrict__ VA,
                                                        int64_t stride, const double* __restrict__ q,
                                                        const double* __restrict__ scale,
                                                        const double* __restrict__ p2,
                                                        const double* __restrict__ cp, double* __restrict__ part) {
  __shared__ double ws[kMaxBasisD + 1][4];
  __shared__ double ck[kMaxBasis];
  const Chunk ch = chunks[blockIdx.x];
  const int i = J - 1;
  const double sc = scale[ch.prob];
  const bool two = p2[ch.prob] != 0.0;
  if (two && (int)threadIdx.x < i) ck[threadIdx.x] = cp[(int64_t)ch.prob * kMaxBasis + threadIdx.x];
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double* Vi = V + i * stride + ch.start;
  TV* VAi = VA + i * stride + ch.start;
  double yv[PER], av[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = threadIdx.x + u * DT;
    yv[u] = 0.0;
    av[u] = 0.0;
    if (e >= ch.len) continue;
    double v = ld_at(q + ch.start, e), a = (double)ld_at(VAi, e);
    if (two) {
      for (int k = 0; k < i; ++k) {
        v -= ck[k] * ld_at(V + k * stride + ch.start, e);
        a -= ck[k] * (double)ld_at(VA + k * stride + ch.start, e);
      }
    }
    v *= sc;
    const TV at = (TV)(a * sc);   // the product as stored (FP32 in the FP32 phase)
    st_at(Vi, e, v);
    st_at(VAi, e, at);
    yv[u] = v;
    av[u] = (double)at;
  }
#pragma unroll 4
  for (int c = 0; c < i; ++c) {
    const TV* Xc = VA + c * stride + ch.start;
    double s = 0.0;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = threadIdx.x + u * DT;
      if (e < ch.len) s += (double)ld_at(Xc, e) * yv[u];
    }
    s = wave_sum(s);
    if (lane == 0) ws[c][wave] = s;
  }
  double s = 0.0;
#pragma unroll
  for (int u = 0; u < PER; ++u) s += av[u] * yv[u];
  s = wave_sum(s);
  if (lane == 0) ws[i][wave] = s;
  __syncthreads();
  if ((int)threadIdx.x < J) {
    const int c = threadIdx.x;
    part[(int64_t)c * nct + blockIdx.x] = ((ws[c][0] + ws[c][1]) + ws[c][2]) + ws[c][3];
  }
}

// SplitMix64 (Steele, Lea, Flood 2014) and the Box-Muller cosine branch.
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__device__ __forceinline__ double gauss_at(uint64_t key, uint64_t idx) {
  const uint64_t g = 0x9E3779B97F4A7C15ull;
  const double u1 = (double)(mix64(key + (2 * idx + 1) * g) >> 11) * 0x1.0p-53;
  const double u2 = (double)(mix64(key + (2 * idx + 2) * g) >> 11) * 0x1.0p-53;
  return sqrt(-2.0 * log(1.0 - u1)) * cos(6.283185307179586476925286766559 * u2);
}

// Per problem (one workgroup): the second Gram-Schmidt pass is due when the
// first one lost more than half of ||t||^2 ("twice is enough": otherwise t
// is already orthogonal to working accuracy).  Its coefficients c = V^T t
// (the first pass's partial dots, summed here) go to cp for the next step's
// Gram row, which applies the pass; ||t||^2 after it is ||t||^2 - ||c||^2
// (V orthonormal).  A second pass that would leave less than 1e-4 of ||t||^2
// leaves rounding noise, whose norm that difference does not give
// accurately: treated as a breakdown.  Then accept t (scale = 1/||t||) or, on
// breakdown (||t|| below rtol of its value before orthogonalisation), restart
// from seeded Gaussian vectors orthogonalised twice against the basis (a
// rare path, done here in full: p2 = 0).
// out[c] = sum over the problem's chunks of part[c * nct + chunk], c < ncol:
// wave w of the block sums columns w, w + (waves), ..., each lane a chunk
// stride of 64 in chunk order, then the wave sum (one fixed order).
__device__ __forceinline__ void col_sums(const double* __restrict__ part, int nct, const DavProb& pr, int ncol,
                                         double* out) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int c = wave; c < ncol; c += nw) {
    const double* col = part + (int64_t)c * nct + pr.chunk0;
    double v = 0.0;
    int k = lane;
    for (; k + 7 * 64 < pr.nchunk; k += 8 * 64) {
      double t[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) t[u] = col[k + u * 64];
#pragma unroll
      for (int u = 0; u < 8; ++u) v += t[u];
    }
    for (; k < pr.nchunk; k += 64) v += col[k];
    v = wave_total(v);
    if (lane == 0) out[c] = v;
  }
  __syncthreads();
}

constexpr int FT = 1024;   // threads of the finalize workgroup
__global__ __launch_bounds__(FT) void finalize_kernel(const DavProb* __restrict__ probs, int nct, int J, int step,
                                                      int B, int64_t stride, const double* __restrict__ V,
                                                      double* __restrict__ q,
                                                      const double* __restrict__ part_n0,
                                                      const double* __restrict__ part_b,
                                                      const double* __restrict__ nq0,
                                                      const int64_t* __restrict__ blk_off,
                                                      const int32_t* __restrict__ blk_ptr, uint64_t seed,
                                                      double rtol, double* __restrict__ scale,
                                                      double* __restrict__ cp, double* __restrict__ p2,
                                                      int32_t* __restrict__ restarts,
                                                      int32_t* __restrict__ status) {
  __shared__ double sh[16];
  __shared__ double cj[kMaxBasis + 1];
  __shared__ double nn[1];
  const int p = blockIdx.x;
  const DavProb pr = probs[p];
  col_sums(part_n0, 0, pr, 1, nn);
  col_sums(part_b, nct, pr, J + 1, cj);
  const double nb = nn[0], n1 = cj[J];
  const bool two = !(n1 >= 0.5 * nq0[p]);
  double na = n1;
  if (two) {
    double c2 = 0.0;
    for (int j = 0; j < J; ++j) c2 += cj[j] * cj[j];
    na = n1 - c2;
    if (!(na >= 1e-4 * n1)) na = 0.0;
  }
  if (na >= rtol * rtol * nb && na > 0.0) {
    if (threadIdx.x == 0) {
      scale[p] = 1.0 / sqrt(na);
      p2[p] = two ? 1.0 : 0.0;
    }
    if (two && (int)threadIdx.x < J) cp[(int64_t)p * kMaxBasis + threadIdx.x] = cj[threadIdx.x];
    return;
  }
  if (threadIdx.x == 0) p2[p] = 0.0;
  for (int attempt = 0; attempt < 3; ++attempt) {
    const uint64_t key = seed + 0x632BE59BD9B4E019ull * (uint64_t)(1 + 65536ll * step + attempt);
    // fill the allowed elements (padding stays zero)
    for (int b = blk_ptr[p]; b < blk_ptr[p + 1]; ++b) {
      const int64_t o = blk_off[2 * b], sz = blk_off[2 * b + 1];
      for (int64_t e = threadIdx.x; e < sz; e += FT) q[pr.base + o + e] = gauss_at(key, (uint64_t)(o + e));
    }
    __syncthreads();
    double s = 0.0;
    for (int64_t e = threadIdx.x; e < pr.len; e += FT) s += q[pr.base + e] * q[pr.base + e];
    const double before = block_sum(s, sh);
    for (int pass = 0; pass < 2; ++pass) {
      for (int j = 0; j < J; ++j) {
        double d = 0.0;
        for (int64_t e = threadIdx.x; e < pr.len; e += FT) d += V[j * stride + pr.base + e] * q[pr.base + e];
        d = block_sum(d, sh);
        if (threadIdx.x == 0) cj[j] = d;
      }
      __syncthreads();
      for (int64_t e = threadIdx.x; e < pr.len; e += FT) {
        double v = q[pr.base + e];
        for (int j = 0; j < J; ++j) v -= cj[j] * V[j * stride + pr.base + e];
        q[pr.base + e] = v;
      }
      __syncthreads();
    }
    s = 0.0;
    for (int64_t e = threadIdx.x; e < pr.len; e += FT) s += q[pr.base + e] * q[pr.base + e];
    const double after = block_sum(s, sh);
    if (threadIdx.x == 0) restarts[p] += 1;
    if (after >= rtol * rtol * before && after > 0.0) {
      if (threadIdx.x == 0) scale[p] = 1.0 / sqrt(after);
      return;
    }
  }
  if (threadIdx.x == 0) {
    status[p] = 1;
    scale[p] = 0.0;
  }
}

__global__ void fill_zero_kernel(double* x, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] = 0.0;
}

// Thick restart of one problem's basis (one wave per problem).  s is the
// current Ritz vector (coordinates of the j-vector basis) and sp the previous
// step's Ritz vector padded with 0; the new basis is s and, when nkeep = 2,
// e = sp orthogonalised twice against s (or, if less than 1e-8 of it remains,
// the newest basis vector e_{j-1} orthogonalised the same way), normalised.
// Writes the coefficients S (column t of problem p at S[(p * 2 + t) * B]),
// the projected matrix S^T M S into rows and columns 0..nkeep-1 of M, and
// s = e_0 (the current Ritz vector is the first kept vector).
__global__ __launch_bounds__(GT) void restart_kernel(int j, int B, int nkeep, double* __restrict__ M,
                                                     double* __restrict__ svec,
                                                     const double* __restrict__ svec_prev,
                                                     double* __restrict__ S) {
  __shared__ double A[kMaxBasis][kMaxBasis + 1];
  const int p = blockIdx.x, lane = threadIdx.x;
  double* Mp = M + (int64_t)p * B * B;
  load_rows<8>(A, Mp, B, j, lane);
  const double sv = lane < j ? svec[(int64_t)p * B + lane] : 0.0;
  double ev = 0.0;
  if (nkeep == 2) {
    double pv = lane < j ? svec_prev[(int64_t)p * B + lane] : 0.0;
    for (int pass = 0; pass < 2; ++pass) pv -= sv * wave_total(sv * pv);
    double nn = sqrt(wave_total(pv * pv));
    if (!(nn > 1e-8)) {
      pv = lane == j - 1 ? 1.0 : 0.0;
      for (int pass = 0; pass < 2; ++pass) pv -= sv * wave_total(sv * pv);
      nn = sqrt(wave_total(pv * pv));
    }
    ev = pv / nn;
  }
  __syncthreads();
  // u = M s, w = M e (lane r: row r)
  double u = 0.0, w = 0.0;
  if (lane < j)
    for (int c = 0; c < j; ++c) {
      const double sc = readlane_d(sv, c), ec = readlane_d(ev, c);
      u += A[lane][c] * sc;
      w += A[lane][c] * ec;
    }
  else
    for (int c = 0; c < j; ++c) {   // keep every lane in the lane reads
      (void)readlane_d(sv, c);
      (void)readlane_d(ev, c);
    }
  const double m00 = wave_total(sv * u), m01 = wave_total(sv * w), m11 = wave_total(ev * w);
  if (lane < B) {
    S[((int64_t)p * 2 + 0) * B + lane] = sv;
    S[((int64_t)p * 2 + 1) * B + lane] = ev;
    svec[(int64_t)p * B + lane] = lane == 0 ? 1.0 : 0.0;
  }
  if (lane == 0) {
    Mp[0] = m00;
    if (nkeep == 2) {
      Mp[1] = m01;
      Mp[B] = m01;
      Mp[B + 1] = m11;
    }
  }
}

// In-place rotation of the basis (and, when VA is non-null, of its
// products): X_t <- sum_c S_ct X_c for t < nout, every input of an element
// read before its outputs are written (each element belongs to one thread).
template <typename TV>
__global__ __launch_bounds__(DT) void rotate_kernel(const Chunk* __restrict__ chunks, int J, int B, int nout,
                                                    const double* __restrict__ S, double* __restrict__ V,
                                                    TV* __restrict__ VA, int64_t stride) {
  __shared__ double sc[2][kMaxBasis];
  const Chunk ch = chunks[blockIdx.x];
  if ((int)threadIdx.x < J) {
    sc[0][threadIdx.x] = S[((int64_t)ch.prob * 2 + 0) * B + threadIdx.x];
    sc[1][threadIdx.x] = S[((int64_t)ch.prob * 2 + 1) * B + threadIdx.x];
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = threadIdx.x + u * DT;
    if (e >= ch.len) continue;
    double o0 = 0.0, o1 = 0.0, a0 = 0.0, a1 = 0.0;
    for (int c = 0; c < J; ++c) {
      const double v = ld_at(V + c * stride + ch.start, e);
      o0 += sc[0][c] * v;
      o1 += sc[1][c] * v;
      if (VA) {
        const double a = (double)ld_at(VA + c * stride + ch.start, e);
        a0 += sc[0][c] * a;
        a1 += sc[1][c] * a;
      }
    }
    st_at(V + ch.start, e, o0);
    if (nout == 2) st_at(V + stride + ch.start, e, o1);
    if (VA) {
      st_at(VA + ch.start, e, (TV)a0);
      if (nout == 2) st_at(VA + stride + ch.start, e, (TV)a1);
    }
  }
}

// Diagonal of H_eff (Davidson's preconditioner): for every psi block
// (a, s1, s2, c), D[i, j] = sum over flux-0 channels w of a, w'' of c of
// L(a, w, a)[i, i] C(w, w'') R(c, w'', c)[j, j] with
// C(w, w'') = sum_w' W1(w, s1, s1, w') W2(w', s2, s2, w'').  One workgroup
// per task (a row range of one block); C is formed in LDS first.
__global__ __launch_bounds__(DT) void diag_kernel(const DiagTask* __restrict__ tasks, const double* __restrict__ L,
                                                  const double* __restrict__ W1, const double* __restrict__ W2,
                                                  const double* __restrict__ R, double* __restrict__ D) {
  __shared__ double C[kMaxDiagChannels * kMaxDiagChannels];
  const DiagTask t = tasks[blockIdx.x];
  for (int idx = threadIdx.x; idx < t.nl * t.nr; idx += DT) {
    const int w = idx / t.nr, z = idx % t.nr;
    double c = 0.0;
    for (int v = 0; v < t.nm; ++v) c += W1[t.w1_off + (int64_t)w * t.nm + v] * W2[t.w2_off + (int64_t)v * t.nr + z];
    C[idx] = c;
  }
  __syncthreads();
  const int n = t.nrow * t.cols;
  for (int e = threadIdx.x; e < n; e += DT) {
    const int i = t.row0 + e / t.cols, jj = e % t.cols;
    double sum = 0.0;
    for (int w = 0; w < t.nl; ++w) {
      const double lw = L[t.l_off + ((int64_t)i * t.nl + w) * t.rows + i];
      double inner = 0.0;
      for (int z = 0; z < t.nr; ++z) inner += C[w * t.nr + z] * R[t.r_off + ((int64_t)jj * t.nr + z) * t.cols + jj];
      sum += lw * inner;
    }
    D[t.psi_off + (int64_t)i * t.cols + jj] = sum;
  }
}

// ---------------------------------------------------------------- launches --
static unsigned nchunks(const bsdmrg_plan_s* P) { return (unsigned)P->chunks.size(); }
static const DavProb* dav_probs(const bsdmrg_plan_s* P) { return P->d_dav_probs; }

hipError_t dav_fill_zero(double* x, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)blocks), dim3(256), 0, s, x, n);
  return hipGetLastError();
}

hipError_t dav_dots(const bsdmrg_plan_s* P, int J, const double* X, int64_t xstride, const double* y,
                    double* part, hipStream_t s, bool norm_col) {
  if (J < 0 || J > kMaxBasisD || (norm_col && J >= kMaxBasisD + 1)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(dots_kernel<double>, dim3(nchunks(P)), dim3(DT), 0, s, P->d_chunks, (int)nchunks(P), J, X,
                     xstride, y, part, norm_col ? 1 : 0);
  return hipGetLastError();
}

hipError_t dav_dots(const bsdmrg_plan_s* P, int J, const float* X, int64_t xstride, const double* y, double* part,
                    hipStream_t s) {
  if (J < 0 || J > kMaxBasisD) return hipErrorInvalidValue;
  hipLaunchKernelGGL(dots_kernel<float>, dim3(nchunks(P)), dim3(DT), 0, s, P->d_chunks, (int)nchunks(P), J, X,
                     xstride, y, part, 0);
  return hipGetLastError();
}

hipError_t dav_restart(const bsdmrg_plan_s* P, const DavBufs& b, int j, int nkeep, hipStream_t s) {
  if (j < 1 || j > b.B || nkeep < 1 || nkeep > 2 || (nkeep == 2 && j < 2)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(restart_kernel, dim3((unsigned)P->probs.size()), dim3(GT), 0, s, j, b.B, nkeep, b.M, b.svec,
                     b.svec_prev, b.Srot);
  return hipGetLastError();
}

hipError_t dav_rotate(const bsdmrg_plan_s* P, const DavBufs& b, int J, int nout, bool with_products,
                      hipStream_t s) {
  if (J < 1 || J > b.B || nout < 1 || nout > 2) return hipErrorInvalidValue;
  if (b.va32)
    hipLaunchKernelGGL(rotate_kernel<float>, dim3(nchunks(P)), dim3(DT), 0, s, P->d_chunks, J, b.B, nout, b.Srot,
                       b.V, with_products ? b.VAf : nullptr, b.n);
  else
    hipLaunchKernelGGL(rotate_kernel<double>, dim3(nchunks(P)), dim3(DT), 0, s, P->d_chunks, J, b.B, nout, b.Srot,
                       b.V, with_products ? b.VA : nullptr, b.n);
  return hipGetLastError();
}

hipError_t dav_diag(const bsdmrg_plan_s* P, const double* L, const double* W1, const double* W2, const double* R,
                    double* D, hipStream_t s) {
  hipError_t e = dav_fill_zero(D, P->psi_elems, s);
  if (e != hipSuccess || P->diag_tasks.empty()) return e;
  hipLaunchKernelGGL(diag_kernel, dim3((unsigned)P->diag_tasks.size()), dim3(DT), 0, s, P->d_diag_tasks, L, W1,
                     W2, R, D);
  return hipGetLastError();
}

hipError_t dav_psum(const bsdmrg_plan_s* P, int J, const double* part, double* red, int ldr, hipStream_t s) {
  hipLaunchKernelGGL(psum_kernel, dim3((unsigned)P->probs.size(), (unsigned)J), dim3(DT), 0, s, dav_probs(P),
                     (int)nchunks(P), J, part, ldr, red);
  return hipGetLastError();
}

hipError_t dav_normalize(const bsdmrg_plan_s* P, const double* part, double* red, const double* x, double* y,
                         hipStream_t s) {
  hipError_t e = dav_psum(P, 1, part, red, 1, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(normalize_kernel, dim3(nchunks(P)), dim3(DT), 0, s, P->d_chunks, 1, red, x, y);
  return hipGetLastError();
}

hipError_t dav_gram_eig(const bsdmrg_plan_s* P, const DavBufs& b, int i, hipStream_t s) {
  if (i < 0 || i >= kMaxBasis) return hipErrorInvalidValue;
  // the Gram row's sums and the eigensolve in one workgroup per problem
  hipLaunchKernelGGL(gram_eig_kernel, dim3((unsigned)P->probs.size()), dim3(GE_T), 0, s, dav_probs(P),
                     (int)nchunks(P), b.part_a, i, b.B, b.M, b.svec, b.lam, b.svec_prev);
  return hipGetLastError();
}

hipError_t dav_ritz(const bsdmrg_plan_s* P, const DavBufs& b, int i, bool want_x, double* part_d,
                    const double* D, hipStream_t s) {
  double* x = want_x ? b.x : nullptr;
  const int J = i + 1;
  const unsigned g = (unsigned)nchunks(P);
  const int nct = (int)nchunks(P);
  if (b.va32) {
    if (J <= 16)
      hipLaunchKernelGGL((ritz_kernel<16, float>), dim3(g), dim3(DT), 0, s, P->d_chunks, nct, J, b.B, b.V, b.VAf,
                         b.n, b.svec, b.lam, x, b.q, b.part_n0, part_d, b.part_res, D);
    else
      hipLaunchKernelGGL((ritz_kernel<0, float>), dim3(g), dim3(DT), 0, s, P->d_chunks, nct, J, b.B, b.V, b.VAf,
                         b.n, b.svec, b.lam, x, b.q, b.part_n0, part_d, b.part_res, D);
  } else {
    if (J <= 16)
      hipLaunchKernelGGL((ritz_kernel<16, double>), dim3(g), dim3(DT), 0, s, P->d_chunks, nct, J, b.B, b.V, b.VA,
                         b.n, b.svec, b.lam, x, b.q, b.part_n0, part_d, b.part_res, D);
    else
      hipLaunchKernelGGL((ritz_kernel<0, double>), dim3(g), dim3(DT), 0, s, P->d_chunks, nct, J, b.B, b.V, b.VA,
                         b.n, b.svec, b.lam, x, b.q, b.part_n0, part_d, b.part_res, D);
  }
  return hipGetLastError();
}

hipError_t dav_update(const bsdmrg_plan_s* P, const DavBufs& b, int J, const double* part_in, hipStream_t s) {
  if (J < 1 || J >= kMaxBasisD) return hipErrorInvalidValue;   // column J holds a norm
  hipError_t e = dav_psum(P, J + 1, part_in, b.red, kMaxBasis, s);
  if (e != hipSuccess) return e;
  if (J <= 16)
    hipLaunchKernelGGL(update_kernel<16>, dim3(nchunks(P)), dim3(DT), 0, s, P->d_chunks, (int)nchunks(P), J, b.V,
                       b.n, kMaxBasis, b.red, b.q, b.part_b, b.nq0);
  else
    hipLaunchKernelGGL(update_kernel<0>, dim3(nchunks(P)), dim3(DT), 0, s, P->d_chunks, (int)nchunks(P), J, b.V,
                       b.n, kMaxBasis, b.red, b.q, b.part_b, b.nq0);
  return hipGetLastError();
}

hipError_t dav_finalize(const bsdmrg_plan_s* P, const DavBufs& b, int J, int step, uint64_t seed, double rtol,
                        const int64_t* blk_off, const int32_t* blk_ptr, hipStream_t s) {
  if (J < 1 || J >= kMaxBasisD) return hipErrorInvalidValue;
  hipLaunchKernelGGL(finalize_kernel, dim3((unsigned)P->probs.size()), dim3(FT), 0, s, dav_probs(P),
                     (int)nchunks(P), J, step, b.B, b.n, b.V, b.q, b.part_n0, b.part_b, b.nq0, blk_off, blk_ptr,
                     seed, rtol, b.scale, b.cp, b.p2, b.restarts, b.status);
  return hipGetLastError();
}

hipError_t dav_fresh_dots(const bsdmrg_plan_s* P, const DavBufs& b, int J, hipStream_t s) {
  if (J < 1 || J > kMaxBasis || J > b.B) return hipErrorInvalidValue;
  if (b.va32)
    hipLaunchKernelGGL(fresh_dots_kernel<float>, dim3(nchunks(P)), dim3(DT), 0, s, P->d_chunks, (int)nchunks(P), J,
                       b.V, b.VAf, b.n, b.q, b.scale, b.p2, b.cp, b.part_a);
  else
    hipLaunchKernelGGL(fresh_dots_kernel<double>, dim3(nchunks(P)), dim3(DT), 0, s, P->d_chunks, (int)nchunks(P), J,
                       b.V, b.VA, b.n, b.q, b.scale, b.p2, b.cp, b.part_a);
  return hipGetLastError();
}

}  // namespace bsd
