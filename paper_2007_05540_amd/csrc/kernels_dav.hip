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

// Deterministic block sum (wave shuffles, then the four wave sums in order).
__device__ __forceinline__ double block_sum(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
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

// Per-block sums of J values per thread (vals[j] for the calling thread):
// wave butterflies, then the four wave sums added in order by thread j; one
// barrier for all J.  Writes part[j * nct + blockIdx.x].
__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// out[j] = sum over the problem's chunks of part[j * nct + chunk] for j < J
// (thread-strided sums, then the deterministic block tree); result in LDS.
__device__ __forceinline__ void sum_partials(const double* __restrict__ part, int nct, const DavProb& pr,
                                             int J, double* out, double* sh) {
  for (int j = 0; j < J; ++j) {
    double v = 0.0;
    for (int c = threadIdx.x; c < pr.nchunk; c += blockDim.x) v += part[(int64_t)j * nct + pr.chunk0 + c];
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
  double v = 0.0;
  for (int c = threadIdx.x; c < pr.nchunk; c += DT) v += part[(int64_t)j * nct + pr.chunk0 + c];
  v = block_sum(v, sh);
  if (threadIdx.x == 0) red[(int64_t)p * ldr + j] = v;
}

// part[j * nct + ch] = sum_{e in chunk ch} X_j[e] y[e], j < J (wave sums
// per j, one barrier, the four wave sums added in order).
__global__ __launch_bounds__(DT) void dots_kernel(const Chunk* __restrict__ chunks, int nct, int J,
                                                  const double* __restrict__ X, int64_t xstride,
                                                  const double* __restrict__ y, double* __restrict__ part) {
  __shared__ double ws[kMaxBasisD][4];
  const Chunk ch = chunks[blockIdx.x];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double yv[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = threadIdx.x + u * DT;
    yv[u] = e < ch.len ? y[ch.start + e] : 0.0;
  }
  for (int j = 0; j < J; ++j) {
    const double* Xj = X + j * xstride + ch.start;
    double s = 0.0;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = threadIdx.x + u * DT;
      if (e < ch.len) s += Xj[e] * yv[u];
    }
    s = wave_sum(s);
    if (lane == 0) ws[j][wave] = s;
  }
  __syncthreads();
  if ((int)threadIdx.x < J) {
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

// Gram row m_ij = m_ji = (v^A_j)^T v_i (j <= i) from the chunk partials, then
// the lowest eigenpair of the (i+1) x (i+1) projected matrix by parallel
// (round-robin ordered) Jacobi rotations: in every step the indices form
// ne/2 disjoint pairs, all rotations of a step are computed at once and
// applied in place as 2 x 2 block updates A <- J^T A J, V <- V J.  An odd
// size gets a zero dummy index that is never selected.  Warm start: the
// matrix grows by one row and column per step, so Jacobi starts from
// W^T M W with W = diag(previous eigenvectors, 1) (all but the new row and
// column are then already diagonal) and V = W; the eigenvectors are kept in
// evec for the next step.
constexpr int kMaxBasis = 64;
__global__ __launch_bounds__(DT) void gram_eig_kernel(int ldr, int i, int B, const double* __restrict__ red,
                                                      double* __restrict__ M, double* __restrict__ evec,
                                                      double* __restrict__ svec, double* __restrict__ lam) {
  __shared__ double A[kMaxBasis][kMaxBasis + 1];
  __shared__ double V[kMaxBasis][kMaxBasis + 1];
  __shared__ double T[kMaxBasis][kMaxBasis + 1];
  __shared__ double pc[kMaxBasis / 2], ps[kMaxBasis / 2];
  __shared__ int pp[kMaxBasis / 2], pq[kMaxBasis / 2];
  __shared__ double sh[16];
  const int p = blockIdx.x, tid = threadIdx.x, n = i + 1;
  const int ne = n + (n & 1);
  const int half = ne / 2;
  double* Mp = M + (int64_t)p * B * B;
  double* Ep = evec + (int64_t)p * B * B;
  if (tid <= i) {
    const double v = red[(int64_t)p * ldr + tid];
    Mp[i * B + tid] = v;
    Mp[tid * B + i] = v;
  }
  __threadfence_block();
  __syncthreads();
  for (int e = tid; e < ne * ne; e += DT) {
    const int r = e / ne, c = e % ne;
    A[r][c] = (r < n && c < n) ? Mp[r * B + c] : 0.0;
    // W = diag(previous eigenvectors (i x i), 1), identity on the dummy index
    V[r][c] = (r < i && c < i) ? Ep[r * B + c] : (r == c ? 1.0 : 0.0);
  }
  __syncthreads();
  if (i > 0) {
    for (int e = tid; e < n * n; e += DT) {   // T = A W
      const int r = e / n, c = e % n;
      double t = 0.0;
      for (int k = 0; k < n; ++k) t += A[r][k] * V[k][c];
      T[r][c] = t;
    }
    __syncthreads();
    for (int e = tid; e < n * n; e += DT) {   // A = W^T T
      const int r = e / n, c = e % n;
      double t = 0.0;
      for (int k = 0; k < n; ++k) t += V[k][r] * T[k][c];
      A[r][c] = t;
    }
    __syncthreads();
    for (int e = tid; e < n * n; e += DT) {   // exact symmetry of the start matrix
      const int r = e / n, c = e % n;
      if (r < c) {
        const double m = 0.5 * (A[r][c] + A[c][r]);
        T[r][c] = m;
      }
    }
    __syncthreads();
    for (int e = tid; e < n * n; e += DT) {
      const int r = e / n, c = e % n;
      if (r < c) A[r][c] = T[r][c];
      if (r > c) A[r][c] = T[c][r];
    }
    __syncthreads();
  }
  double f = 0.0;
  for (int e = tid; e < n * n; e += DT) f += A[e / n][e % n] * A[e / n][e % n];
  const double fro2 = block_sum(f, sh);
  const double tiny = 1e-17 * sqrt(fro2);
  for (int sweep = 0; sweep < 30; ++sweep) {
    double o = 0.0;
    for (int e = tid; e < n * n; e += DT) {
      const int r = e / n, c = e % n;
      if (r != c) o += A[r][c] * A[r][c];
    }
    const double off = block_sum(o, sh);
    if (off <= 1e-32 * fro2) break;
    for (int step = 0; step < ne - 1; ++step) {
      if (tid < half) {
        // circle method: position 0 fixed, the others rotate by one per step
        auto player = [&](int k) { return k == 0 ? 0 : 1 + ((k - 1 + step) % (ne - 1)); };
        const int a = player(tid), b = player(ne - 1 - tid);
        const int P = min(a, b), Q = max(a, b);
        const double apq = A[P][Q];
        double c = 1.0, sn = 0.0;
        if (fabs(apq) > tiny) {
          const double tau = (A[Q][Q] - A[P][P]) / (2.0 * apq);
          const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
          c = 1.0 / sqrt(1.0 + t * t);
          sn = t * c;
        }
        pp[tid] = P; pq[tid] = Q; pc[tid] = c; ps[tid] = sn;
      }
      __syncthreads();
      for (int e = tid; e < half * half; e += DT) {
        const int kr = e / half, kc = e % half;
        if (ps[kr] == 0.0 && ps[kc] == 0.0) continue;
        const int r0 = pp[kr], r1 = pq[kr], c0 = pp[kc], c1 = pq[kc];
        const double cr = pc[kr], sr = ps[kr], cc = pc[kc], sc = ps[kc];
        const double b00 = A[r0][c0], b01 = A[r0][c1], b10 = A[r1][c0], b11 = A[r1][c1];
        const double x00 = b00 * cc - b01 * sc, x01 = b00 * sc + b01 * cc;
        const double x10 = b10 * cc - b11 * sc, x11 = b10 * sc + b11 * cc;
        A[r0][c0] = cr * x00 - sr * x10;
        A[r1][c1] = sr * x01 + cr * x11;
        if (kr == kc) {
          A[r0][c1] = 0.0;
          A[r1][c0] = 0.0;
        } else {
          A[r0][c1] = cr * x01 - sr * x11;
          A[r1][c0] = sr * x00 + cr * x10;
        }
      }
      for (int e = tid; e < ne * half; e += DT) {
        const int r = e / half, kc = e % half;
        if (ps[kc] == 0.0) continue;
        const int c0 = pp[kc], c1 = pq[kc];
        const double cc = pc[kc], sc = ps[kc];
        const double v0 = V[r][c0], v1 = V[r][c1];
        V[r][c0] = v0 * cc - v1 * sc;
        V[r][c1] = v0 * sc + v1 * cc;
      }
      __syncthreads();
    }
  }
  int idx = 0;
  for (int r = 1; r < n; ++r)
    if (A[r][r] < A[idx][idx]) idx = r;
  if (tid < n) svec[(int64_t)p * B + tid] = V[tid][idx];
  if (tid == 0) lam[p] = A[idx][idx];
  for (int e = tid; e < n * n; e += DT) Ep[(e / n) * B + e % n] = V[e / n][e % n];
}

// q = sum s_j v^A_j - lambda sum s_j v_j with partial ||q||^2; when x is
// non-null the Ritz vector x = sum s_j v_j is stored too, and when part_d is
// non-null the partial dots v_j^T q (the first Gram-Schmidt pass) as well.
__global__ __launch_bounds__(DT) void ritz_kernel(const Chunk* __restrict__ chunks, int nct, int J, int B,
                                                  const double* __restrict__ V, const double* __restrict__ VA,
                                                  int64_t stride, const double* __restrict__ svec,
                                                  const double* __restrict__ lam, double* __restrict__ x,
                                                  double* __restrict__ q, double* __restrict__ part,
                                                  double* __restrict__ part_d) {
  __shared__ double ws[kMaxBasisD + 1][4];
  __shared__ double sv[kMaxBasis];
  const Chunk ch = chunks[blockIdx.x];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if ((int)threadIdx.x < J) sv[threadIdx.x] = svec[(int64_t)ch.prob * B + threadIdx.x];
  __syncthreads();
  const double l = lam[ch.prob];
  double qv[PER];
  double nrm = 0.0;
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = threadIdx.x + u * DT;
    qv[u] = 0.0;
    if (e >= ch.len) continue;
    const int64_t g = ch.start + e;
    double xv = 0.0, av = 0.0;
    for (int j = 0; j < J; ++j) {
      xv += sv[j] * V[j * stride + g];
      av += sv[j] * VA[j * stride + g];
    }
    const double v = av - l * xv;
    if (x) x[g] = xv;
    q[g] = v;
    qv[u] = v;
    nrm += v * v;
  }
  nrm = wave_sum(nrm);
  if (lane == 0) ws[kMaxBasisD][wave] = nrm;
  if (part_d) {
    for (int j = 0; j < J; ++j) {
      double d = 0.0;
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int e = threadIdx.x + u * DT;
        if (e < ch.len) d += V[j * stride + ch.start + e] * qv[u];
      }
      d = wave_sum(d);
      if (lane == 0) ws[j][wave] = d;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0)
    part[blockIdx.x] = ((ws[kMaxBasisD][0] + ws[kMaxBasisD][1]) + ws[kMaxBasisD][2]) + ws[kMaxBasisD][3];
  if (part_d && (int)threadIdx.x < J) {
    const int j = threadIdx.x;
    part_d[(int64_t)j * nct + blockIdx.x] = ((ws[j][0] + ws[j][1]) + ws[j][2]) + ws[j][3];
  }
}

// q -= sum_j c_j v_j with c_j = red[p * ldr + j]; mode 1 then writes the
// partial dots v_j^T q, mode 2 the partial ||q||^2.
__global__ __launch_bounds__(DT) void update_kernel(const Chunk* __restrict__ chunks, int nct, int J,
                                                    const double* __restrict__ V, int64_t stride, int ldr,
                                                    const double* __restrict__ red,
                                                    double* __restrict__ q, double* __restrict__ part_out,
                                                    int mode) {
  __shared__ double sh[16];
  __shared__ double cj[kMaxBasis];
  __shared__ double wsum[kMaxBasisD][4];
  const Chunk ch = chunks[blockIdx.x];
  if ((int)threadIdx.x < J) cj[threadIdx.x] = red[(int64_t)ch.prob * ldr + threadIdx.x];
  __syncthreads();
  double qv[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = threadIdx.x + u * DT;
    if (e < ch.len) {
      const int64_t g = ch.start + e;
      double v = q[g];
      for (int j = 0; j < J; ++j) v -= cj[j] * V[j * stride + g];
      q[g] = v;
      qv[u] = v;
    } else {
      qv[u] = 0.0;
    }
  }
  if (mode == 1) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int j = 0; j < J; ++j) {
      double s = 0.0;
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int e = threadIdx.x + u * DT;
        if (e < ch.len) s += V[j * stride + ch.start + e] * qv[u];
      }
      s = wave_sum(s);
      if (lane == 0) wsum[j][wave] = s;
    }
    __syncthreads();
    if ((int)threadIdx.x < J) {
      const int j = threadIdx.x;
      part_out[(int64_t)j * nct + blockIdx.x] = ((wsum[j][0] + wsum[j][1]) + wsum[j][2]) + wsum[j][3];
    }
  } else {
    double s = 0.0;
#pragma unroll
    for (int u = 0; u < PER; ++u) s += qv[u] * qv[u];
    s = block_sum(s, sh);
    if (threadIdx.x == 0) part_out[blockIdx.x] = s;
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

// Decide per problem: accept q (scale = 1/||q||) or, when orthogonalisation
// failed, restart from seeded Gaussian vectors orthogonalised twice against
// the basis (single workgroup per problem; a rare path).
__global__ __launch_bounds__(DT) void finalize_kernel(const DavProb* __restrict__ probs, int i, int B,
                                                      int64_t stride, const double* __restrict__ V,
                                                      double* __restrict__ q,
                                                      const double* __restrict__ part_n0,
                                                      const double* __restrict__ part_n1,
                                                      const int64_t* __restrict__ blk_off,
                                                      const int32_t* __restrict__ blk_ptr, uint64_t seed,
                                                      double rtol, double* __restrict__ scale,
                                                      int32_t* __restrict__ restarts,
                                                      int32_t* __restrict__ status) {
  __shared__ double sh[16];
  __shared__ double cj[kMaxBasis];
  __shared__ double nn[2];
  const int p = blockIdx.x;
  const DavProb pr = probs[p];
  sum_partials(part_n0, 0, pr, 1, nn, sh);
  sum_partials(part_n1, 0, pr, 1, nn + 1, sh);
  const double nb = nn[0], na = nn[1];
  if (na >= rtol * rtol * nb && na > 0.0) {
    if (threadIdx.x == 0) scale[p] = 1.0 / sqrt(na);
    return;
  }
  for (int attempt = 0; attempt < 3; ++attempt) {
    const uint64_t key = seed + 0x632BE59BD9B4E019ull * (uint64_t)(1 + 65536ll * i + attempt);
    // fill the allowed elements (padding stays zero)
    for (int b = blk_ptr[p]; b < blk_ptr[p + 1]; ++b) {
      const int64_t o = blk_off[2 * b], sz = blk_off[2 * b + 1];
      for (int64_t e = threadIdx.x; e < sz; e += DT) q[pr.base + o + e] = gauss_at(key, (uint64_t)(o + e));
    }
    __syncthreads();
    double s = 0.0;
    for (int64_t e = threadIdx.x; e < pr.len; e += DT) s += q[pr.base + e] * q[pr.base + e];
    const double before = block_sum(s, sh);
    for (int pass = 0; pass < 2; ++pass) {
      for (int j = 0; j <= i; ++j) {
        double d = 0.0;
        for (int64_t e = threadIdx.x; e < pr.len; e += DT) d += V[j * stride + pr.base + e] * q[pr.base + e];
        d = block_sum(d, sh);
        if (threadIdx.x == 0) cj[j] = d;
      }
      __syncthreads();
      for (int64_t e = threadIdx.x; e < pr.len; e += DT) {
        double v = q[pr.base + e];
        for (int j = 0; j <= i; ++j) v -= cj[j] * V[j * stride + pr.base + e];
        q[pr.base + e] = v;
      }
      __syncthreads();
    }
    s = 0.0;
    for (int64_t e = threadIdx.x; e < pr.len; e += DT) s += q[pr.base + e] * q[pr.base + e];
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

__global__ __launch_bounds__(DT) void scale_kernel(const Chunk* __restrict__ chunks,
                                                   const double* __restrict__ scale,
                                                   const double* __restrict__ x, double* __restrict__ y) {
  const Chunk ch = chunks[blockIdx.x];
  const double s = scale[ch.prob];
  for (int e = threadIdx.x; e < ch.len; e += DT) y[ch.start + e] = x[ch.start + e] * s;
}

__global__ void fill_zero_kernel(double* x, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] = 0.0;
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
                    double* part, hipStream_t s) {
  hipLaunchKernelGGL(dots_kernel, dim3(nchunks(P)), dim3(DT), 0, s, P->d_chunks, (int)nchunks(P), J, X,
                     xstride, y, part);
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
  hipError_t e = dav_psum(P, i + 1, b.part_a, b.red, kMaxBasis, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(gram_eig_kernel, dim3((unsigned)P->probs.size()), dim3(DT), 0, s, kMaxBasis, i, b.B,
                     b.red, b.M, b.evec, b.svec, b.lam);
  return hipGetLastError();
}

hipError_t dav_ritz(const bsdmrg_plan_s* P, const DavBufs& b, int i, bool want_x, double* part_d,
                    hipStream_t s) {
  hipLaunchKernelGGL(ritz_kernel, dim3(nchunks(P)), dim3(DT), 0, s, P->d_chunks, (int)nchunks(P), i + 1, b.B,
                     b.V, b.VA, b.n, b.svec, b.lam, want_x ? b.x : nullptr, b.q, b.part_n0, part_d);
  return hipGetLastError();
}

hipError_t dav_update(const bsdmrg_plan_s* P, const DavBufs& b, int J, const double* part_in,
                      double* part_out, int mode, hipStream_t s) {
  hipError_t e = dav_psum(P, J, part_in, b.red, kMaxBasis, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(update_kernel, dim3(nchunks(P)), dim3(DT), 0, s, P->d_chunks, (int)nchunks(P), J, b.V,
                     b.n, kMaxBasis, b.red, b.q, part_out, mode);
  return hipGetLastError();
}

hipError_t dav_finalize(const bsdmrg_plan_s* P, const DavBufs& b, int i, uint64_t seed, double rtol,
                        const int64_t* blk_off, const int32_t* blk_ptr, hipStream_t s) {
  hipLaunchKernelGGL(finalize_kernel, dim3((unsigned)P->probs.size()), dim3(DT), 0, s, dav_probs(P), i, b.B,
                     b.n, b.V, b.q, b.part_n0, b.part_n1, blk_off, blk_ptr, seed, rtol, b.scale, b.restarts,
                     b.status);
  return hipGetLastError();
}

hipError_t dav_scale_into(const bsdmrg_plan_s* P, const DavBufs& b, double* dst, hipStream_t s) {
  hipLaunchKernelGGL(scale_kernel, dim3(nchunks(P)), dim3(DT), 0, s, P->d_chunks, b.scale, b.q, dst);
  return hipGetLastError();
}

}  // namespace bsd
