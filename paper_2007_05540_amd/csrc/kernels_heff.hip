// Device kernels of the two-site effective-Hamiltonian product (gfx950).
//
// ggemm: grouped block GEMM.  One workgroup (4 waves, 2 x 2) computes one
// 64 x 64 tile of one task; the task's K-list segments are accumulated in the
// same MFMA accumulators (fixed order, no atomics).  Tiles are staged through
// LDS in BK = 16 slices stored k-major so that MFMA operand fetches are
// contiguous; the next slice is fetched from global memory into registers
// while the current slice is multiplied.
//   FP64: v_mfma_f64_16x16x4f64, FP32: v_mfma_f32_16x16x4f32.
// Operand layout of the 16x16x4 MFMA (both types): lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16].  Accumulator element r of lane l is
// D[l / 16 + 4 r][l % 16] for the FP64 instruction and D[4 (l / 16) + r][l % 16]
// for the FP32 one (checked on gfx950).
#include <hip/hip_runtime.h>

#include "bsdmrg_internal.h"
#include "kernels.h"

namespace bsd {

constexpr int BM = 64, BN = 64, BK = 16, NTHR = 256;

template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 op(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <>
struct Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 op(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

// TC: compute type; TA/TB: global operand types (converted on load);
// TO: output type; BT: B stored N x K (row-major) instead of K x N;
// AT: A stored K x M (row-major) instead of M x K.
template <typename TC, typename TA, typename TB, typename TO, bool BT, bool AT = false>
__global__ __launch_bounds__(NTHR) void ggemm_kernel(const GemmTile* __restrict__ tiles,
                                                     const GemmTask* __restrict__ tasks,
                                                     const GemmSeg* __restrict__ segs,
                                                     const TA* __restrict__ A,
                                                     const TB* __restrict__ B,
                                                     TO* __restrict__ C, TO* __restrict__ Cpart) {
  __shared__ TC As[BK][BM + 1];
  __shared__ TC Bs[BK][BN + 1];
  const GemmTile tile = tiles[blockIdx.x];
  const GemmTask task = tasks[tile.task];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  using V4 = typename Mfma<TC>::v4;
  V4 acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) acc[i][j] = V4{0, 0, 0, 0};

  // global -> register mapping
  const int a_row = tid >> 2, a_k = (tid & 3) * 4;          // A: 64 rows x 16 k
  const int at_k = tid >> 4, at_m = (tid & 15) * 4;         // A (TN): 16 k x 64 m
  const int bn_k = tid >> 4, bn_n = (tid & 15) * 4;         // B (NN): 16 k x 64 n
  const int bt_n = tid >> 2, bt_k = (tid & 3) * 4;          // B (NT): 64 n x 16 k
  TC ra[4], rb[4];

  int seg = task.seg0;
  const int seg_end = task.seg0 + task.nseg;
  int k0 = 0;
  GemmSeg s;
  if (seg < seg_end) s = segs[seg];

  auto load = [&](const GemmSeg& sg, int kk0) {
    const TA* Ap = A + sg.a_off;
    const TB* Bp = B + sg.b_off;
    if (!AT) {
      const int row = tile.m0 + a_row;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int k = kk0 + a_k + u;
        ra[u] = (row < task.M && k < sg.K) ? (TC)Ap[(int64_t)row * sg.lda + k] : (TC)0;
      }
    } else {
      const int k = kk0 + at_k;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int m = tile.m0 + at_m + u;
        ra[u] = (k < sg.K && m < task.M) ? (TC)Ap[(int64_t)k * sg.lda + m] : (TC)0;
      }
    }
    if (!BT) {
      const int k = kk0 + bn_k;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int n = tile.n0 + bn_n + u;
        rb[u] = (k < sg.K && n < task.N) ? (TC)Bp[(int64_t)k * sg.ldb + n] : (TC)0;
      }
    } else {
      const int n = tile.n0 + bt_n;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int k = kk0 + bt_k + u;
        rb[u] = (n < task.N && k < sg.K) ? (TC)Bp[(int64_t)n * sg.ldb + k] : (TC)0;
      }
    }
  };

  bool have = seg < seg_end;
  if (have) load(s, 0);
  while (have) {
    __syncthreads();
    if (!AT) {
#pragma unroll
      for (int u = 0; u < 4; ++u) As[a_k + u][a_row] = ra[u];
    } else {
#pragma unroll
      for (int u = 0; u < 4; ++u) As[at_k][at_m + u] = ra[u];
    }
    if (!BT) {
#pragma unroll
      for (int u = 0; u < 4; ++u) Bs[bn_k][bn_n + u] = rb[u];
    } else {
#pragma unroll
      for (int u = 0; u < 4; ++u) Bs[bt_k + u][bt_n] = rb[u];
    }
    __syncthreads();
    // advance to the next K slice (possibly the next segment) and prefetch it
    k0 += BK;
    if (k0 >= s.K) {
      ++seg;
      k0 = 0;
      have = seg < seg_end;
      if (have) s = segs[seg];
    }
    if (have) load(s, k0);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      TC a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = As[kk + (lane >> 4)][wm * 32 + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = Bs[kk + (lane >> 4)][wn * 32 + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = Mfma<TC>::op(a[i], b[j], acc[i][j]);
    }
  }

  TO* Cp = (task.cbuf ? Cpart : C) + task.c_off;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = tile.m0 + wm * 32 + i * 16 + Mfma<TC>::row(lane, r);
        const int col = tile.n0 + wn * 32 + j * 16 + (lane & 15);
        if (row < task.M && col < task.N) Cp[(int64_t)row * task.ldc + col] = (TO)acc[i][j][r];
      }
}

// MPO mixing (S2): each workgroup handles one row range of one task; every
// thread owns up to 16 elements and issues the 16 loads of a term together.
// coef == nullptr means unit coefficients (the split-K reduction).
template <typename T, typename TACC>
__global__ __launch_bounds__(NTHR) void mix_kernel(const MixItem* __restrict__ items,
                                                   const MixTask* __restrict__ tasks,
                                                   const MixTerm* __restrict__ terms,
                                                   const double* __restrict__ coef,
                                                   const T* __restrict__ src, T* __restrict__ dst) {
  constexpr int PER = 16;   // kMixItemElems = 4096 = 16 * 256
  __shared__ int64_t s_off[64];
  __shared__ int32_t s_ld[64];
  __shared__ TACC s_c[64];
  const MixItem it = items[blockIdx.x];
  const MixTask t = tasks[it.task];
  const int n = it.nrows * t.cols;
  int rr[PER], cc[PER];
  TACC acc[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int e = threadIdx.x + q * NTHR;
    rr[q] = it.row0 + e / t.cols;
    cc[q] = e % t.cols;
    acc[q] = 0;
  }
  for (int t0 = 0; t0 < t.nterm; t0 += 64) {
    const int nt = min(64, t.nterm - t0);
    __syncthreads();
    if ((int)threadIdx.x < nt) {
      const MixTerm m = terms[t.term0 + t0 + threadIdx.x];
      s_off[threadIdx.x] = m.src_off;
      s_ld[threadIdx.x] = m.ld_src;
      s_c[threadIdx.x] = coef ? (TACC)coef[m.coef] : (TACC)1;
    }
    __syncthreads();
    for (int j = 0; j < nt; ++j) {
      const T* sp = src + s_off[j];
      const int ld = s_ld[j];
      const TACC cj = s_c[j];
      T v[PER];
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int e = threadIdx.x + q * NTHR;
        v[q] = e < n ? sp[(int64_t)rr[q] * ld + cc[q]] : (T)0;
      }
#pragma unroll
      for (int q = 0; q < PER; ++q) acc[q] += cj * (TACC)v[q];
    }
  }
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int e = threadIdx.x + q * NTHR;
    if (e < n) dst[t.dst_off + (int64_t)rr[q] * t.ld_dst + cc[q]] = (T)acc[q];
  }
}

// WW coefficients: coef[i] = sum over pairs W1[e1] * W2[e2] (fixed order).
__global__ void coef_kernel(int n, const int32_t* __restrict__ ptr, const int64_t* __restrict__ e1,
                            const int64_t* __restrict__ e2, const double* __restrict__ W1,
                            const double* __restrict__ W2, double* __restrict__ coef) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int p = ptr[i]; p < ptr[i + 1]; ++p) s += W1[e1[p]] * W2[e2[p]];
  coef[i] = s;
}

__global__ void cast_f64_f32_kernel(int64_t n, const double* __restrict__ x, float* __restrict__ y) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (float)x[i];
}

// ---------------------------------------------------------------- launches --
template <typename TC, typename TA, typename TB, typename TO, bool BT, bool AT = false>
static hipError_t launch_gemm(const Stage& st, const TA* A, const TB* B, TO* C, TO* Cpart, hipStream_t s) {
  if (st.tiles.empty()) return hipSuccess;
  hipLaunchKernelGGL((ggemm_kernel<TC, TA, TB, TO, BT, AT>), dim3((unsigned)st.tiles.size()), dim3(NTHR), 0,
                     s, st.d_tiles, st.d_tasks, st.d_segs, A, B, C, Cpart);
  return hipGetLastError();
}

// FP64 grouped GEMM of any stage in one of the layouts NN, NT (B stored
// N x K) or TN (A stored K x M).
hipError_t launch_gemm_f64(const Stage& st, int layout, const double* A, const double* B, double* C,
                           double* Cpart, hipStream_t s) {
  if (layout == kNN) return launch_gemm<double, double, double, double, false, false>(st, A, B, C, Cpart, s);
  if (layout == kNT) return launch_gemm<double, double, double, double, true, false>(st, A, B, C, Cpart, s);
  return launch_gemm<double, double, double, double, false, true>(st, A, B, C, Cpart, s);
}

hipError_t launch_mix_tables(const MixItem* items, size_t n_items, const MixTask* tasks, const MixTerm* terms,
                             const double* coef, const double* src, double* dst, hipStream_t s) {
  if (n_items == 0) return hipSuccess;
  hipLaunchKernelGGL((mix_kernel<double, double>), dim3((unsigned)n_items), dim3(NTHR), 0, s, items, tasks,
                     terms, coef, src, dst);
  return hipGetLastError();
}

static hipError_t launch_reduce(const bsdmrg_plan_s* P, const double* part, double* out, hipStream_t s) {
  if (P->red_items.empty()) return hipSuccess;
  hipLaunchKernelGGL((mix_kernel<double, double>), dim3((unsigned)P->red_items.size()), dim3(NTHR), 0, s,
                     P->d_red_items, P->d_red_tasks, P->d_red_terms, (const double*)nullptr, part, out);
  return hipGetLastError();
}

hipError_t launch_s1_f64(const bsdmrg_plan_s* P, const double* L, const double* psi, double* T1,
                         hipStream_t s) {
  return launch_gemm<double, double, double, double, false>(P->s1, L, psi, T1, T1, s);
}
hipError_t launch_s3_f64(const bsdmrg_plan_s* P, const double* T2, const double* R, double* out,
                         double* part, hipStream_t s) {
  hipError_t e = launch_gemm<double, double, double, double, true>(P->s3, T2, R, out, part, s);
  if (e != hipSuccess) return e;
  return launch_reduce(P, part, out, s);
}
hipError_t launch_s1_f32(const bsdmrg_plan_s* P, const float* L, const double* psi, float* T1,
                         hipStream_t s) {
  return launch_gemm<float, float, double, float, false>(P->s1, L, psi, T1, T1, s);
}
hipError_t launch_s3_f32(const bsdmrg_plan_s* P, const float* T2, const float* R, double* out,
                         double* part, hipStream_t s) {
  hipError_t e = launch_gemm<float, float, float, double, true>(P->s3, T2, R, out, part, s);
  if (e != hipSuccess) return e;
  return launch_reduce(P, part, out, s);
}

hipError_t launch_mix_f64(const bsdmrg_plan_s* P, const double* coef, const double* T1, double* T2,
                          hipStream_t s) {
  if (P->mix_items.empty()) return hipSuccess;
  hipLaunchKernelGGL((mix_kernel<double, double>), dim3((unsigned)P->mix_items.size()), dim3(NTHR), 0, s,
                     P->d_mix_items, P->d_mix_tasks, P->d_mix_terms, coef, T1, T2);
  return hipGetLastError();
}
hipError_t launch_mix_f32(const bsdmrg_plan_s* P, const double* coef, const float* T1, float* T2,
                          hipStream_t s) {
  if (P->mix_items.empty()) return hipSuccess;
  hipLaunchKernelGGL((mix_kernel<float, float>), dim3((unsigned)P->mix_items.size()), dim3(NTHR), 0, s,
                     P->d_mix_items, P->d_mix_tasks, P->d_mix_terms, coef, T1, T2);
  return hipGetLastError();
}

hipError_t launch_coef(const bsdmrg_plan_s* P, const double* W1, const double* W2, double* coef,
                       hipStream_t s) {
  const int n = (int)P->n_coefs;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(coef_kernel, dim3((n + 255) / 256), dim3(256), 0, s, n, P->d_coef_ptr, P->d_coef_e1,
                     P->d_coef_e2, W1, W2, coef);
  return hipGetLastError();
}

hipError_t launch_cast(int64_t n, const double* x, float* y, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(cast_f64_f32_kernel, dim3((unsigned)blocks), dim3(256), 0, s, n, x, y);
  return hipGetLastError();
}

}  // namespace bsd
