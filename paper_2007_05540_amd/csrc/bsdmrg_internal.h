// Internal data structures of the bsdmrg library (host and device).
#pragma once

#include <array>
#include <cstdint>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/bsdmrg.h"

namespace bsd {

constexpr int kAlign = 32;          // block alignment in elements (256 B in FP64)
constexpr int kMaxOrder = 8;
constexpr int kChunk = 512;         // Davidson reduction chunk (elements)

using Charge = std::array<int32_t, 2>;
using Key = std::array<int32_t, kMaxOrder>;

struct Leg {
  int nc = 1;
  std::vector<Charge> q;
  std::vector<int64_t> d;
  int size() const { return (int)q.size(); }
  int find(const Charge& c) const;   // sector index with charge c, or -1
};

struct Layout {
  int order = 0;
  std::vector<Key> keys;
  std::vector<int64_t> offs;         // n_blocks + 1
  std::map<Key, int> index;
  int lookup(const Key& k) const {
    auto it = index.find(k);
    return it == index.end() ? -1 : it->second;
  }
  int64_t elems() const { return offs.empty() ? 0 : offs.back(); }
};

// Error state (thread-local message) ----------------------------------------
void set_error(const std::string& msg);
struct Error {
  bsdmrg_status code;
  std::string msg;
};

Leg leg_from(const bsdmrg_leg& l);                          // throws Error
Layout make_layout(const std::vector<const Leg*>& legs, const int32_t* signs);  // throws Error
inline int64_t round_up(int64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// GEMM tables: C[M x N] (row-major, ldc) = sum over segments A_s[M x K_s] B_s
// with A row-major (lda) and B row-major K x N (ldb) or, for the NT variant,
// stored N x K row-major (ldb).  Offsets are element offsets into the base
// pointers handed to the launch.
struct GemmSeg {
  int64_t a_off, b_off;
  int32_t lda, ldb, K, pad;
};
struct GemmTask {
  int64_t c_off;
  int32_t ldc, M, N, seg0, nseg, ksum;
  int32_t cbuf, pad;   // cbuf 0: output buffer, 1: split-K partial buffer
};
struct GemmTile {
  int32_t task, m0, n0, shape;   // shape 0: 64 x 64 tile, 1: 128 x 128 tile
};
constexpr int32_t kNoBigTiles = 1 << 30;   // big_min of a stage with 64 x 64 tiles only

// One 64 x 64 tile of the persistent grouped GEMM with everything its
// workgroup needs to start it: the task's output geometry and its first
// K segment inline (further segments come from the segment table).
struct PTile {
  int64_t c_off;
  int32_t m0, n0, M, N, ldc, cbuf;
  int32_t seg0, nseg, pad0, pad1;
  GemmSeg first;
};
static_assert(sizeof(PTile) == 80, "PTile layout");

// MPO mixing: dst rows x cols sub-matrix (row stride ld_dst) = sum over terms
// coef[c] * src sub-matrix (row stride ld_src).
struct MixTask {
  int64_t dst_off;
  int32_t ld_dst, rows, cols, term0, nterm, pad;
};
struct MixTerm {
  int64_t src_off;
  int32_t ld_src, coef;
};
struct MixItem {
  int32_t task, row0, nrows, pad;
};
// An item with its task's fields, as the S2 and split-K-sum launches read it
// (one descriptor load instead of two dependent ones).
struct MixWork {
  int64_t dst_off;
  int32_t ld_dst, cols, row0, nrows, term0, nterm;
};
static_assert(sizeof(MixWork) == 32, "MixWork layout");

// Davidson reduction chunks (never straddle two problems).
struct Chunk {
  int64_t start;
  int32_t len, prob;
};

// Diagonal of H_eff over one row range of one psi block (preconditioner):
// L block (a, w0, a) with nl flux-0 channels, R block (c, w0'', c) with nr,
// W1 block (w0, s1, s1, w0') nl x nm, W2 block (w0', s2, s2, w0'') nm x nr.
constexpr int kMaxDiagChannels = 64;
struct DiagTask {
  int64_t psi_off, l_off, r_off, w1_off, w2_off;
  int32_t rows, cols, nl, nm, nr, row0, nrow, pad;
};

// Per-problem descriptor of the Davidson kernels.
struct DavProb {
  int64_t base, len;      // element range of the problem inside a vector
  int32_t chunk0, nchunk; // its reduction chunks
};

// Strided block copy: dst[(r) * drs + (c) * dcs] = scale_c * src[r * sld + c]
// with an optional per-column (or per-row) factor.
struct CopyTask {
  int64_t src_off, dst_off;
  int32_t rows, cols;
  int32_t src_rs, src_cs;   // source strides (row, column)
  int32_t dst_rs, dst_cs;   // destination strides
  int32_t fac_off;          // index of the first factor (or -1)
  int32_t fac_on_rows;      // 1: factor indexed by row, 0: by column
};

// Sign gauge of column j of U (column-major, ld): the entry of largest
// magnitude (the first, in row order, within 1e-10 relative of the maximum)
// becomes positive.  One block per kept column; writes sign[col] = +-1 and
// the factors sign*S (for the side that absorbs S) and sign.
struct GaugeTask {
  int64_t u_off;
  int32_t rows, ld;
  int32_t s_idx;    // index of the singular value
};

// Partial inner product of a G sub-matrix and a T1 sub-matrix (adjoint).
struct BwdDot {
  int64_t g_off, t_off;
  int32_t ld_g, ld_t, cols, row0, nrows, pad;
};

// One-sided Jacobi SVD of one charge matrix: X (m x n, n <= m) is M or M^T.
// SVD of one charge matrix M (rows x cols); X = M or M^T is m x n, m >= n.
// Work (elements of the work array): X (m n), AV = [A; VJ] (2n x n, ld 2n:
// A = R^T in rows 0..n-1, the Jacobi rotations VJ in rows n..n+r-1), Z (m n),
// aux (4 n + 2: R diagonal, reflector factors, column norms, pivots, rank),
// sigma (n), order (n).  Block Jacobi: nb (even) blocks of b columns.
struct SvdTask {
  int64_t x_off, av_off, z_off, aux_off, sig_off, perm_off;
  int64_t u_off, s_off, vt_off;              // outputs
  int32_t m, n, rows, transposed;            // rows = rows of M
  int32_t b, nb, big_qr, pad1;               // big_qr: QR by the multi-workgroup kernels
};
struct SvdPair {      // one workgroup of a block-Jacobi step: sector, pair slot
  int32_t sec, slot;
};
struct SvdCols {      // one workgroup of the left-vector kernel: sector, first column
  int32_t sec, col0;
};

struct Stage {
  std::vector<GemmTask> tasks;
  std::vector<GemmSeg> segs;
  std::vector<GemmTile> tiles;
  GemmTask* d_tasks = nullptr;
  GemmSeg* d_segs = nullptr;
  GemmTile* d_tiles = nullptr;
  double flops = 0.0;
  int32_t big_min = kNoBigTiles;   // tasks with M and N >= big_min use 128 x 128 tiles
  bool big = false;                // the tile table holds 128 x 128 tiles
  void* d_tiles_own = nullptr;     // device tile tables allocated by a re-schedule (else inside the plan blob)
  // the tile table with each tile's task fields and first K segment inline
  // (same order; pad0 = task index or -1 for an empty tile, pad1 = shape);
  // launches of stages that upload it read one descriptor per workgroup
  std::vector<PTile> ftiles;
  PTile* d_ftiles = nullptr;
  // persistent launch: one workgroup per slot, its 64 x 64 tiles in
  // ptiles[wg_ptr[w] .. wg_ptr[w + 1])
  bool persistent = false;
  std::vector<PTile> ptiles;
  std::vector<int32_t> wg_ptr;
  PTile* d_ptiles = nullptr;       // device copies (inside the plan blob)
  int32_t* d_wg_ptr = nullptr;
};
// resident workgroup slots of a persistent launch per XCD: 4 workgroups of
// 64 x 64 tiles per CU (LDS and registers allow 4), 32 CUs per XCD
constexpr int kPersistentSlotsPerXcd = 128;

// Forward intermediate blocks kept for the adjoint.
struct T1Block {
  int32_t ap, f, s1, s2, c;   // a', left channel sector, s1, s2, c
  int64_t off;                // global offset in T1
};
struct T2Block {
  int32_t ap, s1p, s2p, g, c; // a', s1', s2', right channel sector, c
  int64_t off;                // global offset in T2
};

struct ProblemPlan {
  Leg a, s1, s2, c, wl, wm, wr;
  std::vector<T1Block> t1;
  std::vector<T2Block> t2;
  std::vector<double> w1_host, w2_host;
  std::vector<char> nz1, nz2;
  Layout psi, L, R, W1, W2;
  int64_t psi_base = 0, L_base = 0, R_base = 0, W1_base = 0, W2_base = 0;
  int64_t t1_base = 0, t2_base = 0, coef_base = 0;
  int64_t t1_elems = 0, t2_elems = 0, n_coefs = 0;
  int64_t dim = 0;   // allowed (non-padding) elements of psi: the dimension of the eigenproblem
  int32_t chunk0 = 0, nchunk = 0;
};

struct Backward;      // adjoint tables of the two-site energy (backward.cpp)
struct EnvBackward;   // adjoint tables of an environment extension (env_backward.cpp)

// Stage-1 block of an environment extension: X1(x', f, s, b), row-major
// (x' * channels of f) x b.
struct X1Block {
  int32_t xp, f, is, ib;
  int64_t off;
};

}  // namespace bsd

struct bsdmrg_plan_s {
  std::vector<bsd::ProblemPlan> probs;
  int64_t psi_elems = 0, L_elems = 0, R_elems = 0, W1_elems = 0, W2_elems = 0;
  int64_t t1_elems = 0, t2_elems = 0, n_coefs = 0;
  bsd::Stage s1, s3;
  // split-K of S3: partial tiles (in the accumulation type) summed in fixed
  // order by the mixing kernel (FP64) or the FP32 split sum
  int64_t s3_part_elems = 0;
  int32_t s3_split = 0;   // S3 split-K width (0: tasks not split)
  std::vector<bsd::MixTask> red_tasks;
  std::vector<bsd::MixTerm> red_terms;
  std::vector<bsd::MixItem> red_items;
  bsd::MixTerm* d_red_terms = nullptr;
  bsd::MixWork* d_red_work = nullptr;
  std::vector<bsd::MixTask> mix_tasks;
  std::vector<bsd::MixTerm> mix_terms;
  std::vector<bsd::MixItem> mix_items;
  std::vector<int32_t> mix_item_group;   // per item: the (problem, a', c) group whose T1 blocks it reads (host)
  int32_t mix_per = 16;                  // outputs per thread of the S2 and split-K-sum launches (8 or 16)
  int32_t n_mix_groups = 0;
  std::vector<int32_t> coef_ptr;     // CSR over coefficient pairs
  std::vector<int64_t> coef_e1, coef_e2;
  std::vector<bsd::Chunk> chunks;
  double flops_s2 = 0.0;
  bool on_device = false;
  void* d_blob = nullptr;            // one device allocation for all tables
  bsd::MixTerm* d_mix_terms = nullptr;
  bsd::MixWork* d_mix_work = nullptr;
  int32_t* d_coef_ptr = nullptr;
  int64_t* d_coef_e1 = nullptr;
  int64_t* d_coef_e2 = nullptr;
  bsd::Chunk* d_chunks = nullptr;
  std::vector<bsd::DavProb> dav_probs;
  std::vector<int64_t> blk_off;      // per psi block: (offset in problem, size)
  std::vector<int32_t> blk_ptr;      // per problem: first block (n_probs + 1)
  bsd::DavProb* d_dav_probs = nullptr;
  std::vector<bsd::DiagTask> diag_tasks;   // diagonal of H_eff (preconditioner)
  bsd::DiagTask* d_diag_tasks = nullptr;
  int64_t* d_blk_off = nullptr;
  int32_t* d_blk_ptr = nullptr;
  // backward-pass tables (built lazily)
  bsd::Backward* bwd = nullptr;
  // cached hipGraphs of fixed-iteration eigensolves (under mu)
  struct GraphCache* graph = nullptr;
  // guards the lazily built parts of a plan (graph cache, adjoint tables)
  std::mutex mu;
};

// Auxiliary operations (environment extension, two-site merge): one or two
// grouped-GEMM stages around an MPO-mixing stage whose coefficients are the
// entries of W itself.
struct bsdmrg_op_s {
  int kind = 0;                       // 1 env left, 2 env right, 3 merge, 4 dense two-site product
  bsd::Stage g1, g2;                  // first and last GEMM stage
  bsd::Stage g3;                      // dense product: the MPO mixing as a GEMM
  int64_t dn_ma = 0, dn_mc = 0;       // dense product: bond dimensions,
  int32_t dn_k = 0, dn_d = 0;         //   channels and physical dimension
  int layout1 = 0, layout2 = 0;       // kNN / kNT / kTN
  std::vector<bsd::MixTask> mix_tasks;
  std::vector<bsd::MixTerm> mix_terms;
  std::vector<bsd::MixItem> mix_items;
  int64_t x1_elems = 0, x2_elems = 0, out_elems = 0;
  double flops = 0.0;
  void* d_blob = nullptr;
  bsd::MixTask* d_mix_tasks = nullptr;
  bsd::MixTerm* d_mix_terms = nullptr;
  bsd::MixItem* d_mix_items = nullptr;
  // environment ops: legs x, s, y, wl, wr and the stage-1 blocks (adjoint)
  int side = 0;
  std::vector<bsd::Leg> legs;
  std::vector<bsd::X1Block> x1_blocks;
  bsd::EnvBackward* ebwd = nullptr;
  std::mutex mu;                      // guards the lazy build of ebwd
};
