// Device kernels of the two-site effective-Hamiltonian product (gfx950).
//
// ggemm: grouped block GEMM.  One workgroup (4 waves, 2 x 2) computes one
// 64 x 64 or 128 x 128 tile of one task; the task's K-list segments are accumulated in the
// same MFMA accumulators (fixed order, no atomics).  Operands are staged
// through double-buffered LDS slices (32 deep in k for FP32, 16 for FP64);
// the next slice is fetched from global memory into registers while the
// current slice is multiplied.
//   FP64: v_mfma_f64_16x16x4f64, FP32: v_mfma_f32_16x16x4f32.
// Operand layout of the 16x16x4 MFMA (both types): lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16].  Accumulator element r of lane l is
// D[l / 16 + 4 r][l % 16] for the FP64 instruction and D[4 (l / 16) + r][l % 16]
// for the FP32 one (checked on gfx950).
#include <hip/hip_runtime.h>

#include <type_traits>

#include "bsdmrg_internal.h"
#include "kernels.h"

namespace bsd {

constexpr int NTHR = 256;

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

// Raw buffer resource (gfx9 family: untyped, stride 0) over nbytes from p;
// loads at byte offsets at or past nbytes return zero.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p, int64_t nbytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)nbytes, 0x00020000);
}
template <typename T>
__device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t r, unsigned off);
template <>
__device__ __forceinline__ float buf_load<float>(__amdgpu_buffer_rsrc_t r, unsigned off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
}
template <>
__device__ __forceinline__ double buf_load<double>(__amdgpu_buffer_rsrc_t r, unsigned off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}

// LDS slice of one operand of a TM x TM tile (BKT deep in k): K-contiguous
// operands (A as M x K, B as N x K) are kept [row][k] with a row stride of
// BKT + 4 (FP32) or BKT + 1 (FP64), M/N-contiguous ones (A as K x M, B as
// K x N) [k][col] with a row stride of TM + 16 (FP32) or TM + 8 (FP64).  With these strides the
// MFMA operand reads (16 consecutive rows or columns at 4 k) spread evenly
// over the LDS banks, and so do the global->LDS writes of the M/N-contiguous
// operands (64 consecutive columns of one k).
template <typename TC, bool KC, int TM>
struct Slice {
  // k depth of a slice (one barrier per slice): 32 in FP32, 16 in FP64
  static constexpr int BKT = sizeof(TC) == 4 ? 32 : 16;
  static constexpr int LD = KC ? BKT + (sizeof(TC) == 4 ? 4 : 1) : TM + (sizeof(TC) == 4 ? 16 : 8);
  static constexpr int SIZE = KC ? TM * LD : BKT * LD;
  // element (row or column r of the tile, k of the slice)
  static __device__ __forceinline__ int at(int r, int k) { return KC ? r * LD + k : k * LD + r; }
};

// One wave's part of a grouped-GEMM tile: the whole K loop for a fixed
// number NI x NJ (0..2 each) of valid 16 x 16 sub-tiles of the wave's
// 32 x 32 quarter, so the MFMAs of a wave are straight-line code with the
// accumulators in fixed registers.  Every wave of the workgroup runs the
// same number of iterations and barriers whatever its NI x NJ.
//
// TC: compute type; TA/TB: global operand types (converted when written to
// LDS); TO: output type; BT: B stored N x K (row-major) instead of K x N;
// AT: A stored K x M (row-major) instead of M x K.
//
// Global -> LDS: a thread owns EPT = TM * BKT / 256 elements of each operand
// slice.  For a K-contiguous operand: k = tid % BKT and rows tid / BKT +
// (256 / BKT) u, so one load instruction reads consecutive k of a few rows.
// For an M/N-contiguous operand: column tid % TM and k = tid / TM +
// (256 / TM) u, so one load instruction reads 64 consecutive columns of one
// k.  Each load is a raw buffer load: a wave-uniform resource (the segment's
// block from the slice's first k to the block's end, rebuilt per slice in
// scalar registers) plus a per-thread 32-bit byte offset fixed for the
// segment, so a load costs no vector address arithmetic and a read past the
// block returns zero.  Loads keep their storage type until they are written
// to LDS, so they stay in flight across the MFMAs of the current slice.  LDS
// holds one slice, written after a barrier that follows the slice's MFMAs
// (two barriers per iteration): with the half-slice operand fragments this
// leaves room for five workgroups of 64 x 64 FP32 tiles per CU instead of
// four, and the next slice's loads still overlap the current MFMAs.
// One result element of a tile: the output (type TO) or, for a piece of a
// split K-list (cbuf != 0), the partial buffer, which holds the accumulation
// type TC (an FP32 accumulator in half the bytes of an FP64 output), read
// back by the fixed-order sum of the pieces.
template <typename TC, typename TO>
__device__ __forceinline__ void put_c(TO* __restrict__ C, TO* __restrict__ Cpart, int cbuf, int64_t idx, TC v) {
  if (cbuf) ((TC*)Cpart)[idx] = v;
  else C[idx] = (TO)v;
}

template <typename TC, typename TA, typename TB, typename TO, bool BT, bool AT, int TM, int NI, int NJ>
__device__ __forceinline__ void ggemm_wave(const GemmTile& tile, const GemmTask& task, const GemmSeg& first,
                                           const GemmSeg* __restrict__ segs, const TA* __restrict__ A,
                                           const TB* __restrict__ B, TO* __restrict__ C,
                                           TO* __restrict__ Cpart, TC* As, TC* Bs, int ni_rt, int nj_rt) {
  using SA = Slice<TC, !AT, TM>;
  using SB = Slice<TC, BT, TM>;
  constexpr int BKT = SA::BKT;        // k depth of a slice
  constexpr int EPT = TM * BKT / NTHR;   // elements of each operand per thread and slice
  constexpr int RSTEP = NTHR / BKT;   // row step of a thread's K-contiguous elements
  constexpr int KSTEP = NTHR / TM;    // k step of a thread's M/N-contiguous elements
  constexpr int WQ = TM / 2;          // rows / columns of a wave's quarter of the tile
  // sub-tiles per wave: NI x NJ fixed, or (NI < 0) up to TM / 32 each, chosen
  // at run time by wave-uniform branches
  constexpr int MI = NI >= 0 ? NI : TM / 32, MJ = NJ >= 0 ? NJ : TM / 32;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int l16 = lane & 15, g4 = lane >> 4;
  using V4 = typename Mfma<TC>::v4;
  V4 acc[MI > 0 ? MI : 1][MJ > 0 ? MJ : 1];
#pragma unroll
  for (int i = 0; i < (MI > 0 ? MI : 1); ++i)
#pragma unroll
    for (int j = 0; j < (MJ > 0 ? MJ : 1); ++j) acc[i][j] = V4{0, 0, 0, 0};

  // this thread's EPT elements of a slice: (row or column, k) per operand
  const int kc_k = tid % BKT, kc_r = tid / BKT;    // K-contiguous: k, first row (+RSTEP u)
  const int mc_c = tid % TM, mc_k = tid / TM;      // M/N-contiguous: column, first k (+KSTEP u)
  // validity of rows / columns (fixed for the tile)
  unsigned a_v = 0, b_v = 0;
#pragma unroll
  for (int u = 0; u < EPT; ++u) {
    a_v |= (unsigned)(tile.m0 + (AT ? mc_c : kc_r + RSTEP * u) < task.M) << u;
    b_v |= (unsigned)(tile.n0 + (BT ? kc_r + RSTEP * u : mc_c) < task.N) << u;
  }

  TA la[EPT];
  TB lb[EPT];
  unsigned va = 0, vb = 0;
  // Operands are read through buffer resources spanning exactly the
  // segment's block from the slice's first k on: a read past the block (rows
  // past the last one of a K-contiguous block, k past K of an M/N-contiguous
  // one) returns zero and touches no memory.  Reads that stay inside the
  // block but leave the tile (k past K within a K-contiguous row, columns
  // past the edge of an M/N-contiguous row) are zeroed by the masks.
  const TA* a_seg = nullptr;
  const TB* b_seg = nullptr;
  int64_t a_ext = 0, b_ext = 0;      // elements of the block from its start
  unsigned ao[EPT], bo[EPT];         // byte offsets of this thread's elements
  auto setup = [&](const GemmSeg& sg) {
    a_seg = A + sg.a_off;
    b_seg = B + sg.b_off;
    a_ext = AT ? (int64_t)(sg.K - 1) * sg.lda + task.M : (int64_t)(task.M - 1) * sg.lda + sg.K;
    b_ext = BT ? (int64_t)(task.N - 1) * sg.ldb + sg.K : (int64_t)(sg.K - 1) * sg.ldb + task.N;
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
      const unsigned ar = tile.m0 + (AT ? mc_c : kc_r + RSTEP * u);
      const unsigned br = tile.n0 + (BT ? kc_r + RSTEP * u : mc_c);
      ao[u] = (AT ? (unsigned)(mc_k + KSTEP * u) * sg.lda + ar : ar * sg.lda + kc_k) * sizeof(TA);
      bo[u] = (BT ? br * sg.ldb + kc_k : (unsigned)(mc_k + KSTEP * u) * sg.ldb + br) * sizeof(TB);
    }
  };
  auto load = [&](const GemmSeg& sg, int kk0) {
    const int64_t ash = (int64_t)kk0 * (AT ? sg.lda : 1);
    const int64_t bsh = (int64_t)kk0 * (BT ? 1 : sg.ldb);
    const __amdgpu_buffer_rsrc_t ra = make_rsrc(a_seg + ash, (a_ext - ash) * (int64_t)sizeof(TA));
    const __amdgpu_buffer_rsrc_t rb = make_rsrc(b_seg + bsh, (b_ext - bsh) * (int64_t)sizeof(TB));
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
      la[u] = buf_load<TA>(ra, ao[u]);
      lb[u] = buf_load<TB>(rb, bo[u]);
    }
    // K-contiguous operands: k past K of a row inside the block is the next
    // row's data; every element of a thread shares its k
    const bool kin = kk0 + kc_k < sg.K;
    va = (AT || kin) ? a_v : 0u;
    vb = (!BT || kin) ? b_v : 0u;
  };
  auto store = [&](int buf) {
    TC* as = As + buf * SA::SIZE;
    TC* bs = Bs + buf * SB::SIZE;
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
      const TC x = ((va >> u) & 1) ? (TC)la[u] : (TC)0;
      const TC y = ((vb >> u) & 1) ? (TC)lb[u] : (TC)0;
      as[AT ? SA::at(mc_c, mc_k + KSTEP * u) : SA::at(kc_r + RSTEP * u, kc_k)] = x;
      bs[BT ? SB::at(kc_r + RSTEP * u, kc_k) : SB::at(mc_c, mc_k + KSTEP * u)] = y;
    }
  };
  // MFMA k-step q of lane group g (lanes 16 g .. 16 g + 15) takes k = g QN + q
  // of the slice (any assignment of the slice's k to (g, q) is valid when A
  // and B use the same one): a lane's operands of a whole slice are QN
  // consecutive k, all read from LDS before the slice's MFMAs.
  auto compute = [&](int buf) {
    if (MI == 0 || MJ == 0) return;
    constexpr int QN = BKT / 4;
    const TC* as = As + buf * SA::SIZE;
    const TC* bs = Bs + buf * SB::SIZE;
    // the operands of a half slice at a time (fewer registers, so five
    // workgroups fit on a CU in FP32), the MFMAs in the same k order
    constexpr int QH = QN / 2;
#pragma unroll
    for (int q0 = 0; q0 < QN; q0 += QH) {
      TC a[MI > 0 ? MI : 1][QH], b[MJ > 0 ? MJ : 1][QH];
#pragma unroll
      for (int i = 0; i < MI; ++i)
        if (NI >= 0 || i < ni_rt)
#pragma unroll
          for (int q = 0; q < QH; ++q) a[i][q] = as[SA::at(wm * WQ + i * 16 + l16, g4 * QN + q0 + q)];
#pragma unroll
      for (int j = 0; j < MJ; ++j)
        if (NJ >= 0 || j < nj_rt)
#pragma unroll
          for (int q = 0; q < QH; ++q) b[j][q] = bs[SB::at(wn * WQ + j * 16 + l16, g4 * QN + q0 + q)];
#pragma unroll
      for (int q = 0; q < QH; ++q)
#pragma unroll
        for (int i = 0; i < MI; ++i)
#pragma unroll
          for (int j = 0; j < MJ; ++j)
            if ((NI >= 0 || i < ni_rt) && (NJ >= 0 || j < nj_rt))
              acc[i][j] = Mfma<TC>::op(a[i][q], b[j][q], acc[i][j]);
    }
  };

  int seg = task.seg0;
  const int seg_end = task.seg0 + task.nseg;
  int k0 = 0;
  GemmSeg s;
  bool have = seg < seg_end;
  if (have) {
    s = first;
    setup(s);
    load(s, 0);
    store(0);
  }
  __syncthreads();
  int buf = 0;
  while (have) {
    // advance to the next K slice (possibly the next segment) and fetch it
    k0 += BKT;
    if (k0 >= s.K) {
      ++seg;
      k0 = 0;
      have = seg < seg_end;
      if (have) {
        s = segs[seg];
        setup(s);
      }
    }
    if (have) load(s, k0);
    compute(buf);
    if (have) {
      // one LDS slice: every wave has read it before the next is stored
      __syncthreads();
      store(buf);
      __syncthreads();
    }
  }

#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < MJ; ++j)
      if ((NI >= 0 || i < ni_rt) && (NJ >= 0 || j < nj_rt))
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = tile.m0 + wm * WQ + i * 16 + Mfma<TC>::row(lane, r);
          const int col = tile.n0 + wn * WQ + j * 16 + l16;
          if (row < task.M && col < task.N)
            put_c<TC, TO>(C, Cpart, task.cbuf, task.c_off + (int64_t)row * task.ldc + col, acc[i][j][r]);
        }
}

// Grouped block GEMM: one workgroup per tile of one task, the task's K-list
// segments accumulated in the same MFMA accumulators (fixed order).  A tile
// is 64 x 64 (shape 0, each wave a 32 x 32 quarter) or, in launches built
// with BIG, 128 x 128 (shape 1, each wave a 64 x 64 quarter: half the LDS
// and global traffic per flop, for large blocks).
template <typename TC, typename TA, typename TB, typename TO, bool BT, bool AT, bool BIG>
__global__ __launch_bounds__(NTHR) __attribute__((amdgpu_waves_per_eu(BIG || sizeof(TC) == 4 ? 1 : 5))) void ggemm_kernel(const GemmTile* __restrict__ tiles,
                                                     const PTile* __restrict__ ftiles,
                                                     const GemmTask* __restrict__ tasks,
                                                     const GemmSeg* __restrict__ segs,
                                                     const TA* __restrict__ A,
                                                     const TB* __restrict__ B,
                                                     TO* __restrict__ C, TO* __restrict__ Cpart) {
  constexpr int TMX = BIG ? 128 : 64;
  __shared__ TC As[Slice<TC, !AT, TMX>::SIZE];
  __shared__ TC Bs[Slice<TC, BT, TMX>::SIZE];
  // the tile, its task's fields and its first K segment: from the flattened
  // table when the stage has one (one descriptor load), else from the tile,
  // task and segment tables (three dependent loads)
  GemmTile tile;
  GemmTask task;
  GemmSeg first{};
  if (ftiles) {
    const PTile r = ftiles[blockIdx.x];
    if (r.pad0 < 0) return;   // padding of the per-XCD schedule
    tile = GemmTile{r.pad0, r.m0, r.n0, r.pad1};
    task = GemmTask{r.c_off, r.ldc, r.M, r.N, r.seg0, r.nseg, 0, r.cbuf, 0};
    first = r.first;
  } else {
    tile = tiles[blockIdx.x];
    if (tile.task < 0) return;
    task = tasks[tile.task];
    if (task.nseg > 0) first = segs[task.seg0];
  }
  const int wave = threadIdx.x >> 6;
  if (BIG && tile.shape == 1) {
    // valid 16 x 16 sub-tiles of this wave's 64 x 64 quarter (wave-uniform)
    const int r0 = tile.m0 + (wave >> 1) * 64, c0 = tile.n0 + (wave & 1) * 64;
    const int ni = min(4, max(0, (task.M - r0 + 15) / 16));
    const int nj = min(4, max(0, (task.N - c0 + 15) / 16));
    if (ni == 4 && nj == 4)
      ggemm_wave<TC, TA, TB, TO, BT, AT, 128, 4, 4>(tile, task, first, segs, A, B, C, Cpart, As, Bs, 4, 4);
    else
      ggemm_wave<TC, TA, TB, TO, BT, AT, 128, -1, -1>(tile, task, first, segs, A, B, C, Cpart, As, Bs, ni, nj);
    return;
  }
  // valid 16 x 16 sub-tiles of this wave's 32 x 32 quarter (wave-uniform)
  const int r0 = tile.m0 + (wave >> 1) * 32, c0 = tile.n0 + (wave & 1) * 32;
  const int ni = r0 >= task.M ? 0 : (r0 + 16 < task.M ? 2 : 1);
  const int nj = c0 >= task.N ? 0 : (c0 + 16 < task.N ? 2 : 1);
  if (ni == 2 && nj == 2)
    ggemm_wave<TC, TA, TB, TO, BT, AT, 64, 2, 2>(tile, task, first, segs, A, B, C, Cpart, As, Bs, 2, 2);
  else if (ni == 2 && nj == 1)
    ggemm_wave<TC, TA, TB, TO, BT, AT, 64, 2, 1>(tile, task, first, segs, A, B, C, Cpart, As, Bs, 2, 1);
  else if (ni == 1 && nj == 2)
    ggemm_wave<TC, TA, TB, TO, BT, AT, 64, 1, 2>(tile, task, first, segs, A, B, C, Cpart, As, Bs, 1, 2);
  else if (ni == 1 && nj == 1)
    ggemm_wave<TC, TA, TB, TO, BT, AT, 64, 1, 1>(tile, task, first, segs, A, B, C, Cpart, As, Bs, 1, 1);
  else
    ggemm_wave<TC, TA, TB, TO, BT, AT, 64, 0, 0>(tile, task, first, segs, A, B, C, Cpart, As, Bs, 0, 0);
}

// MFMA work of one k-slice for a wave whose 32 x 32 quarter of the tile has
// NI x NJ valid 16 x 16 sub-tiles (the same lane / LDS layout as ggemm_wave).
template <typename TC, bool BT, bool AT, int NI, int NJ>
__device__ __forceinline__ void pslice_mfma(const TC* as, const TC* bs, typename Mfma<TC>::v4 (&acc)[2][2], int wm,
                                            int wn, int l16, int g4) {
  using SA = Slice<TC, !AT, 64>;
  using SB = Slice<TC, BT, 64>;
  constexpr int QN = SA::BKT / 4;
  TC a[NI][QN], b[NJ][QN];
#pragma unroll
  for (int i = 0; i < NI; ++i)
#pragma unroll
    for (int q = 0; q < QN; ++q) a[i][q] = as[SA::at(wm * 32 + i * 16 + l16, g4 * QN + q)];
#pragma unroll
  for (int j = 0; j < NJ; ++j)
#pragma unroll
    for (int q = 0; q < QN; ++q) b[j][q] = bs[SB::at(wn * 32 + j * 16 + l16, g4 * QN + q)];
#pragma unroll
  for (int q = 0; q < QN; ++q)
#pragma unroll
    for (int i = 0; i < NI; ++i)
#pragma unroll
      for (int j = 0; j < NJ; ++j) acc[i][j] = Mfma<TC>::op(a[i][q], b[j][q], acc[i][j]);
}

// Persistent grouped block GEMM: one workgroup per resident slot works
// through its own list of 64 x 64 tiles (assigned on the host: a task's
// tiles on one XCD, longest first over the slots of that XCD).  The k-slice
// after the current one is fetched into registers while the current one is
// multiplied, also across a tile change: the first slice of the next tile
// is in flight during the last MFMAs and the result stores of the current
// tile, and the record of the tile after that is prefetched one tile ahead,
// so a tile change exposes no load latency.  Per tile the K-list segments
// are accumulated in the same registers in segment order, as in
// ggemm_kernel (the outputs are bit-identical).  Tasks without segments
// have their output block written as zeros.
template <typename TC, typename TA, typename TB, typename TO, bool BT, bool AT>
__global__ __launch_bounds__(NTHR) void pgemm_kernel(const int32_t* __restrict__ wg_ptr,
                                                     const PTile* __restrict__ ptiles,
                                                     const GemmSeg* __restrict__ segs, const TA* __restrict__ A,
                                                     const TB* __restrict__ B, TO* __restrict__ C,
                                                     TO* __restrict__ Cpart) {
  constexpr int TM = 64;
  using SA = Slice<TC, !AT, TM>;
  using SB = Slice<TC, BT, TM>;
  constexpr int BKT = SA::BKT;
  constexpr int EPT = TM * BKT / NTHR;
  constexpr int RSTEP = NTHR / BKT;
  constexpr int KSTEP = NTHR / TM;
  __shared__ TC As[2 * SA::SIZE];
  __shared__ TC Bs[2 * SB::SIZE];
  const int t_begin = wg_ptr[blockIdx.x], t_end = wg_ptr[blockIdx.x + 1];
  if (t_begin >= t_end) return;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int l16 = lane & 15, g4 = lane >> 4;
  const int kc_k = tid % BKT, kc_r = tid / BKT;
  const int mc_c = tid % TM, mc_k = tid / TM;
  using V4 = typename Mfma<TC>::v4;

  // ---- load side: the tile, segment and k of the slice being fetched ----
  int lt = t_begin;          // index of the load tile
  PTile lrec;                // its record
  PTile nrec;                // record of tile lt + 1 (prefetched)
  int lseg = 0;              // segment index within the load tile (0 = inline first)
  GemmSeg ls;                // current segment of the load tile
  int lk0 = 0;
  unsigned a_v = 0, b_v = 0;
  TA la[EPT];
  TB lb[EPT];
  unsigned va = 0, vb = 0;
  const TA* a_seg = nullptr;
  const TB* b_seg = nullptr;
  int64_t a_ext = 0, b_ext = 0;
  unsigned ao[EPT], bo[EPT];

  auto tile_masks = [&](const PTile& r) {
    a_v = 0;
    b_v = 0;
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
      a_v |= (unsigned)(r.m0 + (AT ? mc_c : kc_r + RSTEP * u) < r.M) << u;
      b_v |= (unsigned)(r.n0 + (BT ? kc_r + RSTEP * u : mc_c) < r.N) << u;
    }
  };
  auto setup = [&](const GemmSeg& sg) {
    a_seg = A + sg.a_off;
    b_seg = B + sg.b_off;
    a_ext = AT ? (int64_t)(sg.K - 1) * sg.lda + lrec.M : (int64_t)(lrec.M - 1) * sg.lda + sg.K;
    b_ext = BT ? (int64_t)(lrec.N - 1) * sg.ldb + sg.K : (int64_t)(sg.K - 1) * sg.ldb + lrec.N;
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
      const unsigned ar = lrec.m0 + (AT ? mc_c : kc_r + RSTEP * u);
      const unsigned br = lrec.n0 + (BT ? kc_r + RSTEP * u : mc_c);
      ao[u] = (AT ? (unsigned)(mc_k + KSTEP * u) * sg.lda + ar : ar * sg.lda + kc_k) * sizeof(TA);
      bo[u] = (BT ? br * sg.ldb + kc_k : (unsigned)(mc_k + KSTEP * u) * sg.ldb + br) * sizeof(TB);
    }
  };
  auto load = [&](int kk0) {
    const int64_t ash = (int64_t)kk0 * (AT ? ls.lda : 1);
    const int64_t bsh = (int64_t)kk0 * (BT ? 1 : ls.ldb);
    const __amdgpu_buffer_rsrc_t ra = make_rsrc(a_seg + ash, (a_ext - ash) * (int64_t)sizeof(TA));
    const __amdgpu_buffer_rsrc_t rb = make_rsrc(b_seg + bsh, (b_ext - bsh) * (int64_t)sizeof(TB));
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
      la[u] = buf_load<TA>(ra, ao[u]);
      lb[u] = buf_load<TB>(rb, bo[u]);
    }
    const bool kin = kk0 + kc_k < ls.K;
    va = (AT || kin) ? a_v : 0u;
    vb = (!BT || kin) ? b_v : 0u;
  };
  auto store = [&](int buf) {
    TC* as = As + buf * SA::SIZE;
    TC* bs = Bs + buf * SB::SIZE;
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
      const TC x = ((va >> u) & 1) ? (TC)la[u] : (TC)0;
      const TC y = ((vb >> u) & 1) ? (TC)lb[u] : (TC)0;
      as[AT ? SA::at(mc_c, mc_k + KSTEP * u) : SA::at(kc_r + RSTEP * u, kc_k)] = x;
      bs[BT ? SB::at(kc_r + RSTEP * u, kc_k) : SB::at(mc_c, mc_k + KSTEP * u)] = y;
    }
  };
  // output block of a tile written as zeros (a task without K segments)
  auto zero_tile = [&](const PTile& r) {
    for (int e = tid; e < TM * TM; e += NTHR) {
      const int row = r.m0 + e / TM, col = r.n0 + e % TM;
      if (row < r.M && col < r.N) put_c<TC, TO>(C, Cpart, r.cbuf, r.c_off + (int64_t)row * r.ldc + col, (TC)0);
    }
  };
  // make tile index idx the load tile (record from nrec, which then
  // prefetches the following one); false when it has no segment
  auto enter_tile = [&](int idx) {
    lrec = nrec;
    if (idx + 1 < t_end) nrec = ptiles[idx + 1];
    lt = idx;
    lseg = 0;
    lk0 = 0;
    if (lrec.nseg == 0) return false;
    ls = lrec.first;
    tile_masks(lrec);
    setup(ls);
    return true;
  };
  // move the load position to the next slice (maybe in a later tile) and
  // fetch it; false when the workgroup's list is done
  auto advance = [&]() {
    lk0 += BKT;
    if (lk0 >= ls.K) {
      lk0 = 0;
      ++lseg;
      if (lseg < lrec.nseg) {
        ls = segs[lrec.seg0 + lseg];
        setup(ls);
      } else {
        bool found = false;
        for (int idx = lt + 1; idx < t_end && !found; ++idx) {
          found = enter_tile(idx);
          if (!found) zero_tile(lrec);
        }
        if (!found) return false;
      }
    }
    load(lk0);
    return true;
  };

  // ---- compute side: the tile whose slice is in LDS ----
  V4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = V4{0, 0, 0, 0};
  PTile crec;
  int ct = -1;
  int ni = 0, nj = 0;
  auto start_compute = [&]() {
    crec = lrec;
    ct = lt;
    const int r0 = crec.m0 + wm * 32, c0 = crec.n0 + wn * 32;
    ni = r0 >= crec.M ? 0 : (r0 + 16 < crec.M ? 2 : 1);
    nj = c0 >= crec.N ? 0 : (c0 + 16 < crec.N ? 2 : 1);
  };
  auto compute = [&](int buf) {
    const TC* as = As + buf * SA::SIZE;
    const TC* bs = Bs + buf * SB::SIZE;
    if (ni == 2 && nj == 2) pslice_mfma<TC, BT, AT, 2, 2>(as, bs, acc, wm, wn, l16, g4);
    else if (ni == 2 && nj == 1) pslice_mfma<TC, BT, AT, 2, 1>(as, bs, acc, wm, wn, l16, g4);
    else if (ni == 1 && nj == 2) pslice_mfma<TC, BT, AT, 1, 2>(as, bs, acc, wm, wn, l16, g4);
    else if (ni == 1 && nj == 1) pslice_mfma<TC, BT, AT, 1, 1>(as, bs, acc, wm, wn, l16, g4);
  };
  auto epilogue = [&]() {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        if (i < ni && j < nj) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = crec.m0 + wm * 32 + i * 16 + Mfma<TC>::row(lane, r);
            const int col = crec.n0 + wn * 32 + j * 16 + l16;
            if (row < crec.M && col < crec.N)
              put_c<TC, TO>(C, Cpart, crec.cbuf, crec.c_off + (int64_t)row * crec.ldc + col, acc[i][j][r]);
          }
        }
        acc[i][j] = V4{0, 0, 0, 0};
      }
  };

  // first tile with a segment (the ones before it are written as zeros)
  nrec = ptiles[t_begin];
  bool have = false;
  for (int idx = t_begin; idx < t_end && !have; ++idx) {
    have = enter_tile(idx);
    if (!have) zero_tile(lrec);
  }
  if (!have) return;
  load(0);
  store(0);
  start_compute();
  __syncthreads();
  int buf = 0;
  for (;;) {
    const bool more = advance();
    compute(buf);
    if (!more || lt != ct) {
      epilogue();
      if (!more) break;
      start_compute();
    }
    store(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
}

// MPO mixing (S2): each workgroup handles one row range of one task; every
// thread owns up to PER elements and issues the PER loads of a term together,
// from the term's block base (scalar registers) plus a 32-bit byte offset
// (source blocks below 2^29 elements: checked on the host).
// coef == nullptr means unit coefficients (the split-K reduction).
template <typename TS, typename T, typename TACC, int PER, int TR>
__device__ __forceinline__ void mix_body(int64_t dst_off, int ld_dst, int cols, int row0, int nrows, int term0,
                                         int nterm, const MixTerm* __restrict__ terms,
                                         const double* __restrict__ coef, const TS* __restrict__ src,
                                         T* __restrict__ dst) {
  const int n = nrows * cols;
  int rr[PER], cc[PER];
  TACC acc[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int e = threadIdx.x + q * NTHR;
    rr[q] = row0 + e / cols;
    cc[q] = e % cols;
    acc[q] = 0;
  }
  // terms read with a uniform index (scalar registers), TR (4 or 2) at a
  // time, then two, then one: the loads of a round are in flight together,
  // then they are added in term order; element offsets within a source block
  // are 32-bit
  auto load = [&](const MixTerm& m, TS* v) {
    const TS* sp = src + m.src_off;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = threadIdx.x + q * NTHR;
      v[q] = e < n ? *(const TS*)((const char*)sp + (unsigned)(rr[q] * m.ld_src + cc[q]) * (unsigned)sizeof(TS))
                   : (TS)0;
    }
  };
  int j = 0;
  if (TR == 4) {
    for (; j + 3 < nterm; j += 4) {
      const MixTerm m0 = terms[term0 + j], m1 = terms[term0 + j + 1];
      const MixTerm m2 = terms[term0 + j + 2], m3 = terms[term0 + j + 3];
      TS v0[PER], v1[PER], v2[PER], v3[PER];
      load(m0, v0);
      load(m1, v1);
      load(m2, v2);
      load(m3, v3);
      const TACC c0 = coef ? (TACC)coef[m0.coef] : (TACC)1;
      const TACC c1 = coef ? (TACC)coef[m1.coef] : (TACC)1;
      const TACC c2 = coef ? (TACC)coef[m2.coef] : (TACC)1;
      const TACC c3 = coef ? (TACC)coef[m3.coef] : (TACC)1;
#pragma unroll
      for (int q = 0; q < PER; ++q) acc[q] += c0 * (TACC)v0[q];
#pragma unroll
      for (int q = 0; q < PER; ++q) acc[q] += c1 * (TACC)v1[q];
#pragma unroll
      for (int q = 0; q < PER; ++q) acc[q] += c2 * (TACC)v2[q];
#pragma unroll
      for (int q = 0; q < PER; ++q) acc[q] += c3 * (TACC)v3[q];
    }
  }
  for (; j + 1 < nterm; j += 2) {
    const MixTerm m0 = terms[term0 + j], m1 = terms[term0 + j + 1];
    TS v0[PER], v1[PER];
    load(m0, v0);
    load(m1, v1);
    const TACC c0 = coef ? (TACC)coef[m0.coef] : (TACC)1;
    const TACC c1 = coef ? (TACC)coef[m1.coef] : (TACC)1;
#pragma unroll
    for (int q = 0; q < PER; ++q) acc[q] += c0 * (TACC)v0[q];
#pragma unroll
    for (int q = 0; q < PER; ++q) acc[q] += c1 * (TACC)v1[q];
  }
  if (j < nterm) {
    const MixTerm m0 = terms[term0 + j];
    TS v0[PER];
    load(m0, v0);
    const TACC c0 = coef ? (TACC)coef[m0.coef] : (TACC)1;
#pragma unroll
    for (int q = 0; q < PER; ++q) acc[q] += c0 * (TACC)v0[q];
  }
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int e = threadIdx.x + q * NTHR;
    if (e < n) dst[dst_off + (int64_t)rr[q] * ld_dst + cc[q]] = (T)acc[q];
  }
}

// The S2 (TR = 4: MPOs with many terms per output keep four terms' loads in
// flight) and split-K-sum (TR = 2: a few pieces) launches: one flattened
// descriptor per workgroup.
template <typename T, typename TACC, int PER, int TR>
__global__ __launch_bounds__(NTHR) void mix_kernel(const MixWork* __restrict__ work,
                                                   const MixTerm* __restrict__ terms,
                                                   const double* __restrict__ coef,
                                                   const T* __restrict__ src, T* __restrict__ dst) {
  const MixWork w = work[blockIdx.x];
  mix_body<T, T, TACC, PER, TR>(w.dst_off, w.ld_dst, w.cols, w.row0, w.nrows, w.term0, w.nterm, terms, coef, src,
                                dst);
}

// The fixed-order sum of FP32 split-K partials (the FP32 S3 launch) into the
// output (FP64, or FP32 for the products of the FP32 phase of a mixed
// Davidson solve): the pieces added in order in FP32, like the K-list within
// a piece (FP32 accumulation throughout the K-list).  Accumulating the loaded
// FP32 values directly keeps the loads of a round in flight together (a
// widening of each value would be placed beside its per-lane guarded load
// and wait for it).
template <int PER, typename TD>
__global__ __launch_bounds__(NTHR) void split_sum_f32_kernel(const MixWork* __restrict__ work,
                                                             const MixTerm* __restrict__ terms,
                                                             const float* __restrict__ src,
                                                             TD* __restrict__ dst) {
  const MixWork w = work[blockIdx.x];
  mix_body<float, TD, float, PER, 2>(w.dst_off, w.ld_dst, w.cols, w.row0, w.nrows, w.term0, w.nterm, terms,
                                          nullptr, src, dst);
}

// The adjoint and environment launches: item and task tables.
__global__ __launch_bounds__(NTHR) void mix_table_kernel(const MixItem* __restrict__ items,
                                                         const MixTask* __restrict__ tasks,
                                                         const MixTerm* __restrict__ terms,
                                                         const double* __restrict__ coef,
                                                         const double* __restrict__ src, double* __restrict__ dst) {
  const MixItem it = items[blockIdx.x];
  const MixTask t = tasks[it.task];
  mix_body<double, double, double, 16, 2>(t.dst_off, t.ld_dst, t.cols, it.row0, it.nrows, t.term0, t.nterm, terms,
                                          coef, src, dst);
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
  if (st.big)
    hipLaunchKernelGGL((ggemm_kernel<TC, TA, TB, TO, BT, AT, true>), dim3((unsigned)st.tiles.size()), dim3(NTHR),
                       0, s, st.d_tiles, st.d_ftiles, st.d_tasks, st.d_segs, A, B, C, Cpart);
  else
    hipLaunchKernelGGL((ggemm_kernel<TC, TA, TB, TO, BT, AT, false>), dim3((unsigned)st.tiles.size()),
                       dim3(NTHR), 0, s, st.d_tiles, st.d_ftiles, st.d_tasks, st.d_segs, A, B, C, Cpart);
  return hipGetLastError();
}

// Persistent variant (64 x 64 tiles, one workgroup per slot with tiles).
template <typename TC, typename TA, typename TB, typename TO, bool BT, bool AT = false>
static hipError_t launch_pgemm(const Stage& st, const TA* A, const TB* B, TO* C, TO* Cpart, hipStream_t s) {
  const int n_wg = (int)st.wg_ptr.size() - 1;
  if (n_wg <= 0) return hipSuccess;
  hipLaunchKernelGGL((pgemm_kernel<TC, TA, TB, TO, BT, AT>), dim3((unsigned)n_wg), dim3(NTHR), 0, s, st.d_wg_ptr,
                     st.d_ptiles, st.d_segs, A, B, C, Cpart);
  return hipGetLastError();
}

// The stage's launch: persistent or one workgroup per tile.
template <typename TC, typename TA, typename TB, typename TO, bool BT, bool AT = false>
static hipError_t launch_stage(const Stage& st, const TA* A, const TB* B, TO* C, TO* Cpart, hipStream_t s) {
  if (st.persistent) return launch_pgemm<TC, TA, TB, TO, BT, AT>(st, A, B, C, Cpart, s);
  return launch_gemm<TC, TA, TB, TO, BT, AT>(st, A, B, C, Cpart, s);
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
  hipLaunchKernelGGL(mix_table_kernel, dim3((unsigned)n_items), dim3(NTHR), 0, s, items, tasks, terms, coef, src,
                     dst);
  return hipGetLastError();
}

hipError_t launch_s3_reduce(const bsdmrg_plan_s* P, const double* part, double* out, bool f32_parts,
                            hipStream_t s) {
  if (P->red_items.empty()) return hipSuccess;
  if (f32_parts) {
    const float* pf = (const float*)part;
    if (P->mix_per == 8)
      hipLaunchKernelGGL((split_sum_f32_kernel<8, double>), dim3((unsigned)P->red_items.size()), dim3(NTHR), 0, s,
                         P->d_red_work, P->d_red_terms, pf, out);
    else
      hipLaunchKernelGGL((split_sum_f32_kernel<16, double>), dim3((unsigned)P->red_items.size()), dim3(NTHR), 0, s,
                         P->d_red_work, P->d_red_terms, pf, out);
    return hipGetLastError();
  }
  if (P->mix_per == 8)
    hipLaunchKernelGGL((mix_kernel<double, double, 8, 2>), dim3((unsigned)P->red_items.size()), dim3(NTHR), 0, s,
                       P->d_red_work, P->d_red_terms, (const double*)nullptr, part, out);
  else
    hipLaunchKernelGGL((mix_kernel<double, double, 16, 2>), dim3((unsigned)P->red_items.size()), dim3(NTHR), 0, s,
                       P->d_red_work, P->d_red_terms, (const double*)nullptr, part, out);
  return hipGetLastError();
}

hipError_t launch_s1_f64(const bsdmrg_plan_s* P, const double* L, const double* psi, double* T1,
                         hipStream_t s) {
  return launch_stage<double, double, double, double, false>(P->s1, L, psi, T1, T1, s);
}
hipError_t launch_s3_f64(const bsdmrg_plan_s* P, const double* T2, const double* R, double* out,
                         double* part, hipStream_t s) {
  hipError_t e = launch_s3_gemm_f64(P, T2, R, out, part, s);
  if (e != hipSuccess) return e;
  return launch_s3_reduce(P, part, out, false, s);
}
hipError_t launch_s3_gemm_f64(const bsdmrg_plan_s* P, const double* T2, const double* R, double* out,
                              double* part, hipStream_t s) {
  return launch_stage<double, double, double, double, true>(P->s3, T2, R, out, part, s);
}
hipError_t launch_s1_f32(const bsdmrg_plan_s* P, const float* L, const double* psi, float* T1,
                         hipStream_t s) {
  return launch_stage<float, float, double, float, false>(P->s1, L, psi, T1, T1, s);
}
hipError_t launch_s3_f32(const bsdmrg_plan_s* P, const float* T2, const float* R, double* out,
                         double* part, hipStream_t s) {
  hipError_t e = launch_s3_gemm_f32(P, T2, R, out, part, s);
  if (e != hipSuccess) return e;
  return launch_s3_reduce(P, part, out, true, s);
}
hipError_t launch_s3_gemm_f32(const bsdmrg_plan_s* P, const float* T2, const float* R, double* out,
                              double* part, hipStream_t s) {
  return launch_stage<float, float, float, double, true>(P->s3, T2, R, out, part, s);
}
hipError_t launch_s3_f32_out32(const bsdmrg_plan_s* P, const float* T2, const float* R, float* out, double* part,
                               hipStream_t s) {
  hipError_t e = launch_s3_gemm_f32_out32(P, T2, R, out, part, s);
  if (e != hipSuccess) return e;
  return launch_s3_reduce_out32(P, part, out, s);
}
hipError_t launch_s3_gemm_f32_out32(const bsdmrg_plan_s* P, const float* T2, const float* R, float* out,
                                    double* part, hipStream_t s) {
  return launch_stage<float, float, float, float, true>(P->s3, T2, R, out, (float*)part, s);
}
hipError_t launch_s3_reduce_out32(const bsdmrg_plan_s* P, const double* part, float* out, hipStream_t s) {
  if (P->red_items.empty()) return hipSuccess;
  const float* pf = (const float*)part;
  if (P->mix_per == 8)
    hipLaunchKernelGGL((split_sum_f32_kernel<8, float>), dim3((unsigned)P->red_items.size()), dim3(NTHR), 0, s,
                       P->d_red_work, P->d_red_terms, pf, out);
  else
    hipLaunchKernelGGL((split_sum_f32_kernel<16, float>), dim3((unsigned)P->red_items.size()), dim3(NTHR), 0, s,
                       P->d_red_work, P->d_red_terms, pf, out);
  return hipGetLastError();
}

hipError_t launch_mix_f64(const bsdmrg_plan_s* P, const double* coef, const double* T1, double* T2,
                          hipStream_t s) {
  if (P->mix_items.empty()) return hipSuccess;
  if (P->mix_per == 8)
    hipLaunchKernelGGL((mix_kernel<double, double, 8, 4>), dim3((unsigned)P->mix_items.size()), dim3(NTHR), 0, s,
                       P->d_mix_work, P->d_mix_terms, coef, T1, T2);
  else
    hipLaunchKernelGGL((mix_kernel<double, double, 16, 4>), dim3((unsigned)P->mix_items.size()), dim3(NTHR), 0, s,
                       P->d_mix_work, P->d_mix_terms, coef, T1, T2);
  return hipGetLastError();
}
hipError_t launch_mix_f32(const bsdmrg_plan_s* P, const double* coef, const float* T1, float* T2,
                          hipStream_t s) {
  if (P->mix_items.empty()) return hipSuccess;
  if (P->mix_per == 8)
    hipLaunchKernelGGL((mix_kernel<float, float, 8, 4>), dim3((unsigned)P->mix_items.size()), dim3(NTHR), 0, s,
                       P->d_mix_work, P->d_mix_terms, coef, T1, T2);
  else
    hipLaunchKernelGGL((mix_kernel<float, float, 16, 4>), dim3((unsigned)P->mix_items.size()), dim3(NTHR), 0, s,
                       P->d_mix_work, P->d_mix_terms, coef, T1, T2);
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

// Sparse-dense format (every operand one dense array, Sec. IV-A): the two
// MPO sites contracted over their shared channel, laid out as the A operand
// of the mixing GEMM, WW[(s1' s2' w''), (w s1 s2)] = sum_v W1(w, s1', s1, v)
// W2(v, s2', s2, w'') with W dense (k, d, d, k).
template <typename TO>
__global__ void dense_ww_kernel(int k, int d, const double* __restrict__ W1, const double* __restrict__ W2,
                                TO* __restrict__ WW) {
  const int n = d * d * k;
  const int64_t total = (int64_t)n * n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(e / n), c = (int)(e % n);
    const int s1p = r / (d * k), s2p = (r / k) % d, wpp = r % k;
    const int w = c / (d * d), s1 = (c / d) % d, s2 = c % d;
    double acc = 0.0;
    for (int v = 0; v < k; ++v)
      acc += W1[(((int64_t)w * d + s1p) * d + s1) * k + v] * W2[(((int64_t)v * d + s2p) * d + s2) * k + wpp];
    WW[e] = (TO)acc;
  }
}

hipError_t launch_dense_product(const bsdmrg_op_s* O, int precision, const double* L, const double* W1,
                                const double* W2, const double* R, const double* psi, double* out, void* T1,
                                void* T2, void* WW, float* Lf, float* Rf, hipStream_t s) {
  const int k = O->dn_k, d = O->dn_d;
  const int64_t n_ww = (int64_t)d * d * k * d * d * k;
  const unsigned ww_blocks = (unsigned)std::min<int64_t>((n_ww + 255) / 256, 1024);
  if (precision == 0) {
    hipLaunchKernelGGL(dense_ww_kernel<double>, dim3(ww_blocks), dim3(256), 0, s, k, d, W1, W2, (double*)WW);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = launch_stage<double, double, double, double, false>(O->g1, L, psi, (double*)T1,
                                                                                 (double*)T1, s);
    if (e == hipSuccess)
      e = launch_stage<double, double, double, double, false>(O->g3, (const double*)WW, (const double*)T1,
                                                              (double*)T2, (double*)T2, s);
    if (e == hipSuccess)
      e = launch_stage<double, double, double, double, true>(O->g2, (const double*)T2, R, out, out, s);
    return e;
  }
  const int64_t l_elems = O->dn_ma * k * O->dn_ma, r_elems = O->dn_mc * k * O->dn_mc;
  hipLaunchKernelGGL(dense_ww_kernel<float>, dim3(ww_blocks), dim3(256), 0, s, k, d, W1, W2, (float*)WW);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = launch_cast(l_elems, L, Lf, s);
  if (e == hipSuccess) e = launch_cast(r_elems, R, Rf, s);
  if (e == hipSuccess)
    e = launch_stage<float, float, double, float, false>(O->g1, Lf, psi, (float*)T1, (float*)T1, s);
  if (e == hipSuccess)
    e = launch_stage<float, float, float, float, false>(O->g3, (const float*)WW, (const float*)T1, (float*)T2,
                                                        (float*)T2, s);
  if (e == hipSuccess) e = launch_stage<float, float, float, double, true>(O->g2, (const float*)T2, Rf, out, out, s);
  return e;
}

hipError_t launch_cast(int64_t n, const double* x, float* y, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(cast_f64_f32_kernel, dim3((unsigned)blocks), dim3(256), 0, s, n, x, y);
  return hipGetLastError();
}

}  // namespace bsd
