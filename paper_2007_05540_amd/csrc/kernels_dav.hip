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

// part[j * nct + ch] = sum_{e in chunk ch} X_j[e] y[e], j < J
__global__ __launch_bounds__(DT) void dots_kernel(const Chunk* __restrict__ chunks, int nct, int J,
                                                  const double* __restrict__ X, int64_t xstride,
                                                  const double* __restrict__ y, double* __restrict__ part) {
  __shared__ double sh[16];
  const Chunk ch = chunks[blockIdx.x];
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
    s = block_sum(s, sh);
    if (threadIdx.x == 0) part[(int64_t)j * nct + blockIdx.x] = s;
  }
}

// y = x / ||x||_p with ||x||_p^2 = sum of the problem's chunk partials.
__global__ __launch_bounds__(DT) void normalize_kernel(const Chunk* __restrict__ chunks,
                                                       const DavProb* __restrict__ probs,
                                                       const double* __restrict__ part,
                                                       const double* __restrict__ x,
                                                       double* __restrict__ y) {
  __shared__ double inv;
  const Chunk ch = chunks[blockIdx.x];
  if (threadIdx.x == 0) {
    const DavProb pr = probs[ch.prob];
    double s = 0.0;
    for (int c = 0; c < pr.nchunk; ++c) s += part[pr.chunk0 + c];
    inv = 1.0 / sqrt(s);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < ch.len; e += DT) y[ch.start + e] = x[ch.start + e] * inv;
}

// Gram row m_ij = m_ji = (v^A_j)^T v_i (j <= i) from the chunk partials, then
// the lowest eigenpair of the (i+1) x (i+1) projected matrix by cyclic Jacobi
// rotations (one wave per problem, matrix in LDS).
constexpr int kMaxBasis = 64;
__global__ __launch_bounds__(64) void gram_eig_kernel(const DavProb* __restrict__ probs, int nct, int i,
                                                      int B, const double* __restrict__ part,
                                                      double* __restrict__ M, double* __restrict__ svec,
                                                      double* __restrict__ lam) {
  __shared__ double A[kMaxBasis][kMaxBasis + 1];
  __shared__ double V[kMaxBasis][kMaxBasis + 1];
  const int p = blockIdx.x, k = threadIdx.x, n = i + 1;
  const DavProb pr = probs[p];
  double* Mp = M + (int64_t)p * B * B;
  if (k <= i) {
    double s = 0.0;
    for (int c = 0; c < pr.nchunk; ++c) s += part[(int64_t)k * nct + pr.chunk0 + c];
    Mp[i * B + k] = s;
    Mp[k * B + i] = s;
  }
  __threadfence_block();
  __syncthreads();
  if (k < n)
    for (int c = 0; c < n; ++c) {
      A[k][c] = Mp[k * B + c];
      V[k][c] = (k == c) ? 1.0 : 0.0;
    }
  __syncthreads();
  // Frobenius norm (for the thresholds)
  double fro = 0.0;
  for (int r = 0; r < n; ++r)
    for (int c = 0; c < n; ++c) fro += A[r][c] * A[r][c];
  const double tiny = 1e-18 * sqrt(fro);
  for (int sweep = 0; sweep < 50; ++sweep) {
    double off = 0.0;
    for (int r = 0; r < n; ++r)
      for (int c = 0; c < n; ++c)
        if (r != c) off += A[r][c] * A[r][c];
    if (off <= 1e-34 * fro || off == 0.0) break;
    for (int pp = 0; pp < n - 1; ++pp)
      for (int qq = pp + 1; qq < n; ++qq) {
        const double apq = A[pp][qq];
        if (fabs(apq) <= tiny) continue;
        const double app = A[pp][pp], aqq = A[qq][qq];
        const double tau = (aqq - app) / (2.0 * apq);
        const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
        const double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
        __syncthreads();
        if (k < n) {
          const double akp = A[k][pp], akq = A[k][qq];
          A[k][pp] = c * akp - s * akq;
          A[k][qq] = s * akp + c * akq;
        }
        __syncthreads();
        if (k < n) {
          const double apk = A[pp][k], aqk = A[qq][k];
          A[pp][k] = c * apk - s * aqk;
          A[qq][k] = s * apk + c * aqk;
          const double vkp = V[k][pp], vkq = V[k][qq];
          V[k][pp] = c * vkp - s * vkq;
          V[k][qq] = s * vkp + c * vkq;
        }
        __syncthreads();
        if (k == 0) { A[pp][qq] = 0.0; A[qq][pp] = 0.0; }
        __syncthreads();
      }
  }
  int idx = 0;
  for (int r = 1; r < n; ++r)
    if (A[r][r] < A[idx][idx]) idx = r;
  if (k < n) svec[(int64_t)p * B + k] = V[k][idx];
  if (k == 0) lam[p] = A[idx][idx];
}

// x = sum s_j v_j, q = sum s_j v^A_j - lambda x, partial ||q||^2.
__global__ __launch_bounds__(DT) void ritz_kernel(const Chunk* __restrict__ chunks, int J, int B,
                                                  const double* __restrict__ V, const double* __restrict__ VA,
                                                  int64_t stride, const double* __restrict__ svec,
                                                  const double* __restrict__ lam, double* __restrict__ x,
                                                  double* __restrict__ q, double* __restrict__ part) {
  __shared__ double sh[16];
  __shared__ double sv[kMaxBasis];
  const Chunk ch = chunks[blockIdx.x];
  if ((int)threadIdx.x < J) sv[threadIdx.x] = svec[(int64_t)ch.prob * B + threadIdx.x];
  __syncthreads();
  const double l = lam[ch.prob];
  double nrm = 0.0;
  for (int u = 0; u < PER; ++u) {
    const int e = threadIdx.x + u * DT;
    if (e >= ch.len) break;
    const int64_t g = ch.start + e;
    double xv = 0.0, av = 0.0;
    for (int j = 0; j < J; ++j) {
      xv += sv[j] * V[j * stride + g];
      av += sv[j] * VA[j * stride + g];
    }
    const double qv = av - l * xv;
    x[g] = xv;
    q[g] = qv;
    nrm += qv * qv;
  }
  nrm = block_sum(nrm, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = nrm;
}

// q -= sum_j c_j v_j with c_j = sum of the problem's chunk partials of
// part_in; mode 1 then writes the partial dots v_j^T q, mode 2 ||q||^2.
__global__ __launch_bounds__(DT) void update_kernel(const Chunk* __restrict__ chunks,
                                                    const DavProb* __restrict__ probs, int nct, int J,
                                                    const double* __restrict__ V, int64_t stride,
                                                    const double* __restrict__ part_in,
                                                    double* __restrict__ q, double* __restrict__ part_out,
                                                    int mode) {
  __shared__ double sh[16];
  __shared__ double cj[kMaxBasis];
  const Chunk ch = chunks[blockIdx.x];
  const DavProb pr = probs[ch.prob];
  if ((int)threadIdx.x < J) {
    double s = 0.0;
    for (int c = 0; c < pr.nchunk; ++c) s += part_in[(int64_t)threadIdx.x * nct + pr.chunk0 + c];
    cj[threadIdx.x] = s;
  }
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
    for (int j = 0; j < J; ++j) {
      double s = 0.0;
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int e = threadIdx.x + u * DT;
        if (e < ch.len) s += V[j * stride + ch.start + e] * qv[u];
      }
      s = block_sum(s, sh);
      if (threadIdx.x == 0) part_out[(int64_t)j * nct + blockIdx.x] = s;
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
  const int p = blockIdx.x;
  const DavProb pr = probs[p];
  double nb = 0.0, na = 0.0;
  for (int c = 0; c < pr.nchunk; ++c) {
    nb += part_n0[pr.chunk0 + c];
    na += part_n1[pr.chunk0 + c];
  }
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

hipError_t dav_normalize(const bsdmrg_plan_s* P, const double* part, const double* x, double* y,
                         hipStream_t s) {
  hipLaunchKernelGGL(normalize_kernel, dim3(nchunks(P)), dim3(DT), 0, s, P->d_chunks, dav_probs(P), part,
                     x, y);
  return hipGetLastError();
}

hipError_t dav_gram_eig(const bsdmrg_plan_s* P, const DavBufs& b, int i, hipStream_t s) {
  hipLaunchKernelGGL(gram_eig_kernel, dim3((unsigned)P->probs.size()), dim3(64), 0, s, dav_probs(P),
                     (int)nchunks(P), i, b.B, b.part_a, b.M, b.svec, b.lam);
  return hipGetLastError();
}

hipError_t dav_ritz(const bsdmrg_plan_s* P, const DavBufs& b, int i, hipStream_t s) {
  hipLaunchKernelGGL(ritz_kernel, dim3(nchunks(P)), dim3(DT), 0, s, P->d_chunks, i + 1, b.B, b.V, b.VA, b.n,
                     b.svec, b.lam, b.x, b.q, b.part_n0);
  return hipGetLastError();
}

hipError_t dav_update(const bsdmrg_plan_s* P, const DavBufs& b, int J, const double* part_in,
                      double* part_out, int mode, hipStream_t s) {
  hipLaunchKernelGGL(update_kernel, dim3(nchunks(P)), dim3(DT), 0, s, P->d_chunks, dav_probs(P),
                     (int)nchunks(P), J, b.V, b.n, part_in, b.q, part_out, mode);
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
