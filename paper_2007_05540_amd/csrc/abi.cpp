// C ABI of the bsdmrg library: plans, the two-site product, the Davidson
// eigensolver.  No exception crosses this file's extern "C" functions.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <stdexcept>

#include "bsdmrg_internal.h"
#include "kernels.h"

bsdmrg_plan_s* build_plan(const bsdmrg_problem* probs, int n_probs);
namespace bsd {
const char* last_error_cstr();
void destroy_backward(bsdmrg_plan_s* P);
void destroy_graph(bsdmrg_plan_s* P);
int64_t heff_backward_bytes(bsdmrg_plan_s* P);
void heff_backward_run(bsdmrg_plan_s* P, const double* L, const double* W1, const double* W2, const double* R,
                       const double* psi, const double* g_host, double* d_psi, double* d_L, double* d_W1,
                       double* d_W2, double* d_R, void* ws, int64_t ws_bytes, hipStream_t s);
void heff_energy_run(bsdmrg_plan_s* P, const double* L, const double* W1, const double* W2, const double* R,
                     const double* psi, double* energy, void* ws, int64_t ws_bytes, hipStream_t s);
}  // namespace bsd

using namespace bsd;

#define HIPCHK(x)                                                                              \
  do {                                                                                         \
    hipError_t e_ = (x);                                                                       \
    if (e_ != hipSuccess) throw Error{BSDMRG_EHIP, std::string(#x) + ": " + hipGetErrorString(e_)}; \
  } while (0)

template <class F>
static bsdmrg_status guarded(F&& f) {
  try {
    f();
    return BSDMRG_OK;
  } catch (const Error& e) {
    set_error(e.msg);
    return e.code;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return BSDMRG_ENOMEM;
  } catch (const std::exception& e) {
    set_error(e.what());
    return BSDMRG_EINVAL;
  } catch (...) {
    set_error("unknown error");
    return BSDMRG_EINVAL;
  }
}

static inline size_t al256(size_t b) { return (b + 255) / 256 * 256; }

// Sub-allocator over a caller workspace.
struct Carve {
  char* base;
  size_t used = 0, cap;
  Carve(void* p, size_t c) : base((char*)p), cap(c) {}
  template <class T>
  T* take(size_t n) {
    T* p = (T*)(base ? base + used : nullptr);
    used += al256(n * sizeof(T));
    return p;
  }
};

struct ApplyWS {
  double* T1;
  double* T2;
  double* part;     // split-K partial tiles of S3 (FP32 values in the FP32 product)
  double* coef;
  float* L32;
  float* R32;
};

static ApplyWS carve_apply(const bsdmrg_plan_s* P, Carve& c) {
  ApplyWS w;
  w.T1 = c.take<double>(P->t1_elems);
  w.T2 = c.take<double>(P->t2_elems);
  w.part = c.take<double>(std::max<int64_t>(P->s3_part_elems, 1));
  w.coef = c.take<double>(std::max<int64_t>(P->n_coefs, 1));
  w.L32 = c.take<float>(P->L_elems);
  w.R32 = c.take<float>(P->R_elems);
  return w;
}

static size_t apply_bytes(const bsdmrg_plan_s* P) {
  Carve c(nullptr, 0);
  carve_apply(P, c);
  return c.used;
}

// Workspace of one product that holds only what the kernels of one
// precision touch: FP64 keeps T1 and T2 in FP64; FP32 keeps them in FP32
// plus the FP32 copies of L and R.  Same kernels as carve_apply's layout.
static ApplyWS carve_apply_prec(const bsdmrg_plan_s* P, int prec, Carve& c) {
  ApplyWS w{};
  const size_t el = prec == BSDMRG_F64 ? sizeof(double) : sizeof(float);
  w.T1 = (double*)c.take<char>((size_t)P->t1_elems * el);
  w.T2 = (double*)c.take<char>((size_t)P->t2_elems * el);
  w.part = c.take<double>(std::max<int64_t>(P->s3_part_elems, 1));
  w.coef = c.take<double>(std::max<int64_t>(P->n_coefs, 1));
  if (prec == BSDMRG_F32) {
    w.L32 = c.take<float>(P->L_elems);
    w.R32 = c.take<float>(P->R_elems);
  }
  return w;
}

namespace bsd {
int64_t heff_apply_bytes(const bsdmrg_plan_s* P) { return (int64_t)apply_bytes(P); }

// FP64 product that also hands back the intermediates (for the adjoint):
// the apply workspace sits at the start of ws.
void heff_forward_f64(const bsdmrg_plan_s* P, const double* L, const double* W1, const double* W2, const double* R,
                      const double* psi, double* out, void* ws, hipStream_t s, double** T1, double** T2,
                      double** coef) {
  Carve c(ws, (size_t)apply_bytes(P));
  ApplyWS w = carve_apply(P, c);
  HIPCHK(launch_coef(P, W1, W2, w.coef, s));
  HIPCHK(launch_s1_f64(P, L, psi, w.T1, s));
  HIPCHK(launch_mix_f64(P, w.coef, w.T1, w.T2, s));
  HIPCHK(launch_s3_f64(P, w.T2, R, out, w.part, s));
  *T1 = w.T1;
  *T2 = w.T2;
  *coef = w.coef;
}
}  // namespace bsd

static std::vector<MixWork> work_of(const std::vector<MixItem>& items, const std::vector<MixTask>& tasks) {
  std::vector<MixWork> w;
  w.reserve(items.size());
  for (const MixItem& it : items) {
    const MixTask& t = tasks[it.task];
    w.push_back(MixWork{t.dst_off, t.ld_dst, t.cols, it.row0, it.nrows, t.term0, t.nterm});
  }
  return w;
}

static void upload(bsdmrg_plan_s* P) {
  struct Part {
    const void* src;
    size_t bytes;
    void** dst;
  };
  const std::vector<MixWork> mix_work = work_of(P->mix_items, P->mix_tasks);
  const std::vector<MixWork> red_work = work_of(P->red_items, P->red_tasks);
  std::vector<Part> parts = {
      {mix_work.data(), mix_work.size() * sizeof(MixWork), (void**)&P->d_mix_work},
      {red_work.data(), red_work.size() * sizeof(MixWork), (void**)&P->d_red_work},
      {P->s1.tasks.data(), P->s1.tasks.size() * sizeof(GemmTask), (void**)&P->s1.d_tasks},
      {P->s1.segs.data(), P->s1.segs.size() * sizeof(GemmSeg), (void**)&P->s1.d_segs},
      {P->s1.tiles.data(), P->s1.tiles.size() * sizeof(GemmTile), (void**)&P->s1.d_tiles},
      {P->s1.ftiles.data(), P->s1.ftiles.size() * sizeof(PTile), (void**)&P->s1.d_ftiles},
      {P->s3.tasks.data(), P->s3.tasks.size() * sizeof(GemmTask), (void**)&P->s3.d_tasks},
      {P->s3.segs.data(), P->s3.segs.size() * sizeof(GemmSeg), (void**)&P->s3.d_segs},
      {P->s3.tiles.data(), P->s3.tiles.size() * sizeof(GemmTile), (void**)&P->s3.d_tiles},
      {P->s3.ftiles.data(), P->s3.ftiles.size() * sizeof(PTile), (void**)&P->s3.d_ftiles},
      {P->mix_terms.data(), P->mix_terms.size() * sizeof(MixTerm), (void**)&P->d_mix_terms},
      {P->red_terms.data(), P->red_terms.size() * sizeof(MixTerm), (void**)&P->d_red_terms},
      {P->coef_ptr.data(), P->coef_ptr.size() * sizeof(int32_t), (void**)&P->d_coef_ptr},
      {P->coef_e1.data(), P->coef_e1.size() * sizeof(int64_t), (void**)&P->d_coef_e1},
      {P->coef_e2.data(), P->coef_e2.size() * sizeof(int64_t), (void**)&P->d_coef_e2},
      {P->chunks.data(), P->chunks.size() * sizeof(Chunk), (void**)&P->d_chunks},
      {P->dav_probs.data(), P->dav_probs.size() * sizeof(DavProb), (void**)&P->d_dav_probs},
      {P->blk_off.data(), P->blk_off.size() * sizeof(int64_t), (void**)&P->d_blk_off},
      {P->blk_ptr.data(), P->blk_ptr.size() * sizeof(int32_t), (void**)&P->d_blk_ptr},
      {P->diag_tasks.data(), P->diag_tasks.size() * sizeof(DiagTask), (void**)&P->d_diag_tasks},
      {P->s1.ptiles.data(), P->s1.ptiles.size() * sizeof(PTile), (void**)&P->s1.d_ptiles},
      {P->s1.wg_ptr.data(), P->s1.wg_ptr.size() * sizeof(int32_t), (void**)&P->s1.d_wg_ptr},
      {P->s3.ptiles.data(), P->s3.ptiles.size() * sizeof(PTile), (void**)&P->s3.d_ptiles},
      {P->s3.wg_ptr.data(), P->s3.wg_ptr.size() * sizeof(int32_t), (void**)&P->s3.d_wg_ptr},
  };
  size_t total = 0;
  for (auto& p : parts) total += al256(std::max<size_t>(p.bytes, 1));
  HIPCHK(hipMalloc(&P->d_blob, total));
  std::vector<char> host(total, 0);
  size_t off = 0;
  for (auto& p : parts) {
    if (p.bytes) std::memcpy(host.data() + off, p.src, p.bytes);
    *p.dst = (char*)P->d_blob + off;
    off += al256(std::max<size_t>(p.bytes, 1));
  }
  HIPCHK(hipMemcpy(P->d_blob, host.data(), total, hipMemcpyHostToDevice));
  P->on_device = true;
}

// New tile schedule of one GEMM stage: the table is rebuilt, checked and
// uploaded to a buffer of its own; a captured graph holds the old table and
// is dropped.
static void reschedule_stage(bsdmrg_plan_s* P, Stage& st, int32_t big_min, const char* name) {
  if (big_min == 0) {
    // the persistent tables were built, checked and uploaded with the plan
    schedule_tiles(st, kNoBigTiles);
    st.big_min = 0;
    destroy_graph(P);
    st.persistent = true;
    return;
  }
  st.persistent = false;
  schedule_tiles(st, big_min);
  flatten_tiles(st);
  validate_tiles(st, name);
  destroy_graph(P);
  // both tile tables in one buffer: tiles, then (256-byte aligned) ftiles
  const size_t tb = al256(std::max<size_t>(st.tiles.size() * sizeof(GemmTile), 1));
  const size_t bytes = tb + std::max<size_t>(st.ftiles.size() * sizeof(PTile), 1);
  void* d = nullptr;
  HIPCHK(hipMalloc(&d, bytes));
  hipError_t e = hipMemcpy(d, st.tiles.data(), st.tiles.size() * sizeof(GemmTile), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy((char*)d + tb, st.ftiles.data(), st.ftiles.size() * sizeof(PTile), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(d);
    HIPCHK(e);
  }
  if (st.d_tiles_own) (void)hipFree(st.d_tiles_own);
  st.d_tiles_own = d;
  st.d_tiles = (GemmTile*)d;
  st.d_ftiles = (PTile*)((char*)d + tb);
}

static void check_ws(void* ws, int64_t have, size_t need) {
  if (need > 0 && !ws) throw Error{BSDMRG_EINVAL, "workspace pointer is NULL"};
  if ((size_t)have < need)
    throw Error{BSDMRG_EINVAL, "workspace too small: need " + std::to_string(need) + " bytes"};
}

static void need_device(const bsdmrg_plan_s* P) {
  if (!P) throw Error{BSDMRG_EINVAL, "plan is NULL"};
  if (!P->on_device) throw Error{BSDMRG_EINVAL, "plan was built host-only"};
}

// Operand preparation: WW coefficients (and FP32 copies of L, R).
static void prepare(const bsdmrg_plan_s* P, int prec, const double* L, const double* W1,
                    const double* W2, const double* R, const ApplyWS& w, hipStream_t s) {
  HIPCHK(launch_coef(P, W1, W2, w.coef, s));
  if (prec == BSDMRG_F32) {
    HIPCHK(launch_cast(P->L_elems, L, w.L32, s));
    HIPCHK(launch_cast(P->R_elems, R, w.R32, s));
  }
}

static void matvec(const bsdmrg_plan_s* P, int prec, const double* L, const double* R,
                   const ApplyWS& w, const double* psi, double* out, hipStream_t s) {
  if (prec == BSDMRG_F64) {
    HIPCHK(launch_s1_f64(P, L, psi, w.T1, s));
    HIPCHK(launch_mix_f64(P, w.coef, w.T1, w.T2, s));
    HIPCHK(launch_s3_f64(P, w.T2, R, out, w.part, s));
  } else {
    float* T1 = (float*)w.T1;
    float* T2 = (float*)w.T2;
    HIPCHK(launch_s1_f32(P, w.L32, psi, T1, s));
    HIPCHK(launch_mix_f32(P, w.coef, T1, T2, s));
    HIPCHK(launch_s3_f32(P, T2, w.R32, out, w.part, s));
  }
}

// The FP32 product with its result stored in FP32: the products of the FP32
// phase of a mixed Davidson solve, which are FP32-accurate.
static void matvec_out32(const bsdmrg_plan_s* P, const ApplyWS& w, const double* psi, float* out, hipStream_t s) {
  float* T1 = (float*)w.T1;
  float* T2 = (float*)w.T2;
  HIPCHK(launch_s1_f32(P, w.L32, psi, T1, s));
  HIPCHK(launch_mix_f32(P, w.coef, T1, T2, s));
  HIPCHK(launch_s3_f32_out32(P, T2, w.R32, out, w.part, s));
}

namespace bsd {
int64_t heff_apply_bytes_prec(const bsdmrg_plan_s* P, int prec) {
  Carve c(nullptr, 0);
  carve_apply_prec(P, prec, c);
  return (int64_t)c.used;
}

// One product with the per-precision workspace layout (carve_apply_prec);
// the caller has checked the plan, the operands and the workspace size.
void heff_apply_compact(const bsdmrg_plan_s* P, int prec, const double* L, const double* W1, const double* W2,
                        const double* R, const double* psi, double* out, void* ws, hipStream_t s) {
  Carve c(ws, (size_t)heff_apply_bytes_prec(P, prec));
  ApplyWS w = carve_apply_prec(P, prec, c);
  prepare(P, prec, L, W1, W2, R, w, s);
  matvec(P, prec, L, R, w, psi, out, s);
}
}  // namespace bsd

// ------------------------------------------------------------ Davidson ------
struct EigWS {
  ApplyWS a;
  DavBufs d;
};

// Basis size: the products of a phase without thick restart (<= 64), else
// the option's basis (0: 64).
static int basis_size(const bsdmrg_eig_opts* o) {
  if (o->restart_keep > 0) return o->basis > 0 ? o->basis : 64;
  int B = o->max_iter;
  if (o->precision == BSDMRG_F32_REFINE) B = std::max(B, o->refine_max_iter);
  return std::min(B, 64);
}

static EigWS carve_eig(const bsdmrg_plan_s* P, const bsdmrg_eig_opts* o, Carve& c) {
  EigWS w;
  w.a = carve_apply(P, c);
  const int B = basis_size(o);
  const int64_t n = P->psi_elems, nch = (int64_t)P->chunks.size(), np = (int64_t)P->probs.size();
  DavBufs& d = w.d;
  d.n = n;
  d.B = B;
  d.V = c.take<double>((size_t)B * n);
  d.VA = c.take<double>((size_t)B * n);
  d.VAf = (float*)d.VA;
  d.va32 = false;
  d.x = c.take<double>(n);
  d.q = c.take<double>(n);
  d.part_a = c.take<double>((size_t)(B + 1) * nch);
  d.part_b = c.take<double>((size_t)(B + 1) * nch);
  d.part_n0 = c.take<double>(nch);
  d.part_res = c.take<double>(nch);
  d.cp = c.take<double>((size_t)np * 64);
  d.p2 = c.take<double>(np);
  d.nq0 = c.take<double>(np);
  d.red = c.take<double>((size_t)np * 65);
  d.M = c.take<double>((size_t)np * B * B);
  d.svec = c.take<double>((size_t)np * B);
  d.svec_prev = c.take<double>((size_t)np * B);
  d.Srot = c.take<double>((size_t)np * 2 * B);
  d.lam = c.take<double>(np);
  d.scale = c.take<double>(np);
  // restarts and status share one region of np + 1 doubles (zero-filled)
  d.restarts = (int32_t*)c.take<double>(np + 1);
  d.status = d.restarts + np;
  d.D = o->precond ? c.take<double>(n) : nullptr;
  return w;
}

static void validate_opts(const bsdmrg_plan_s* P, const bsdmrg_eig_opts* o) {
  if (!o) throw Error{BSDMRG_EINVAL, "eig opts is NULL"};
  if (o->precision != BSDMRG_F64 && o->precision != BSDMRG_F32_REFINE)
    throw Error{BSDMRG_EINVAL, "eigensolve precision must be F64 or F32_REFINE"};
  if (o->restart_keep != 0 && o->restart_keep != 1) throw Error{BSDMRG_EINVAL, "restart_keep must be 0 or 1"};
  if (o->precond != 0 && o->precond != 1) throw Error{BSDMRG_EINVAL, "precond must be 0 or 1"};
  if (o->check_every < 0 || o->check_every > 4096) throw Error{BSDMRG_EINVAL, "check_every must be in 0..4096"};
  const bool mixed = o->precision == BSDMRG_F32_REFINE;
  if (o->restart_keep == 0) {
    if (o->max_iter < 1 || o->max_iter > 64) throw Error{BSDMRG_EINVAL, "max_iter must be in 1..64"};
    if (mixed && (o->refine_max_iter < 1 || o->refine_max_iter > 64))
      throw Error{BSDMRG_EINVAL, "refine_max_iter must be in 1..64"};
  } else {
    if (o->basis != 0 && (o->basis < 3 || o->basis > 64)) throw Error{BSDMRG_EINVAL, "basis must be 0 or 3..64"};
    if (o->max_iter < 1 || o->max_iter > 4096) throw Error{BSDMRG_EINVAL, "max_iter must be in 1..4096"};
    if (mixed && (o->refine_max_iter < 1 || o->refine_max_iter > 4096))
      throw Error{BSDMRG_EINVAL, "refine_max_iter must be in 1..4096"};
  }
  if (P->probs.size() > 1 && !o->fixed_iters)
    throw Error{BSDMRG_EINVAL, "a batch plan requires fixed_iters = 1"};
  if (!(o->restart_rtol >= 0.0) || std::isnan(o->tol) || std::isnan(o->tol_f32))
    throw Error{BSDMRG_EINVAL, "bad tolerances"};
}

// Captured solves of a plan, keyed by every pointer and option of the call
// (a fixed-iteration solve is fully determined by them).  Looked up, captured
// and launched under the plan's mutex, so calls from several threads with
// their own workspaces keep their own graphs.
struct GraphKey {
  const void* ptrs[6];
  bsdmrg_eig_opts o;
  bool operator==(const GraphKey& k) const {
    return std::memcmp(ptrs, k.ptrs, sizeof(ptrs)) == 0 && std::memcmp(&o, &k.o, sizeof(o)) == 0;
  }
};
struct SolveCounts {
  int it64 = 0, it32 = 0, thick = 0;
};
struct GraphEntry {
  GraphKey key;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  SolveCounts counts;
};
struct GraphCache {
  std::vector<GraphEntry> entries;   // oldest first
};
constexpr size_t kMaxGraphs = 8;

namespace bsd {
void destroy_graph(bsdmrg_plan_s* P) {
  if (!P->graph) return;
  for (GraphEntry& g : P->graph->entries) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
  }
  delete P->graph;
  P->graph = nullptr;
}
}  // namespace bsd

// A basis as large as the space it lives in makes the Ritz pair exact and
// leaves no new direction: a phase ends there (the smallest problem of a
// batch sets the cap for all).
static int64_t solve_dim(const bsdmrg_plan_s* P) {
  int64_t dim = INT64_MAX;
  for (const ProblemPlan& pp : P->probs) dim = std::min(dim, std::max<int64_t>(pp.dim, 1));
  return dim;
}

// Enqueue the whole solve (Alg. 1 with the bounded basis, the preconditioner
// and the FP32 -> FP64 switch documented in the header).  The sequence of
// launches depends only on the options and the plan, except in tol mode,
// where the host reads ||q|| after every Ritz step (one sync per step).
static void enqueue_solve(const bsdmrg_plan_s* P, const double* L, const double* W1, const double* W2,
                          const double* R, double* psi, const bsdmrg_eig_opts* o, EigWS& w,
                          hipStream_t s, SolveCounts& cnt, std::vector<double>& res, std::vector<int>& conv) {
  const DavBufs& d = w.d;
  const int64_t n = d.n;
  const int np = (int)P->probs.size();
  const int B = d.B;
  HIPCHK(launch_coef(P, W1, W2, w.a.coef, s));
  const bool mixed = o->precision == BSDMRG_F32_REFINE;
  if (mixed) {
    HIPCHK(launch_cast(P->L_elems, L, w.a.L32, s));
    HIPCHK(launch_cast(P->R_elems, R, w.a.R32, s));
  }
  if (d.D) HIPCHK(dav_diag(P, L, W1, W2, R, d.D, s));
  HIPCHK(dav_fill_zero(d.VA, (int64_t)B * n, s));
  HIPCHK(dav_fill_zero((double*)d.restarts, np + 1, s));
  HIPCHK(dav_dots(P, 1, psi, 0, psi, d.part_a, s));
  HIPCHK(dav_normalize(P, d.part_a, d.red, psi, d.V, s));
  struct Phase {
    int prec, budget;
    double tol;
  };
  std::vector<Phase> phases;
  if (mixed) {
    phases.push_back({BSDMRG_F32, o->max_iter, o->tol_f32});
    phases.push_back({BSDMRG_F64, o->refine_max_iter, o->tol});
  } else {
    phases.push_back({BSDMRG_F64, o->max_iter, o->tol});
  }
  // tol mode: the residual partials of a check are copied to pinned host
  // memory without waiting for them and examined at the next check, so the
  // device never idles for a host round trip between checks; when a lagged
  // check is converged, the current residual is read synchronously and the
  // solve stops if it is converged too.  The end of a phase reads the
  // current residual synchronously.
  const size_t nch = P->chunks.size();
  struct Lagged {
    double* h = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};
    ~Lagged() {
      for (hipEvent_t e : ev)
        if (e) (void)hipEventDestroy(e);
      if (h) (void)hipHostFree(h);
    }
  } lag;
  std::vector<double> hpart(nch);
  if (!o->fixed_iters) {
    HIPCHK(hipHostMalloc((void**)&lag.h, 2 * nch * sizeof(double), hipHostMallocDefault));
    for (hipEvent_t& e : lag.ev) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  }
  auto converged_from = [&](const double* hp, double tol) {
    bool all = true;
    for (int p = 0; p < np; ++p) {
      const DavProb& pr = P->dav_probs[p];
      double r = 0.0;
      for (int c = 0; c < pr.nchunk; ++c) r += hp[pr.chunk0 + c];
      res[p] = std::sqrt(r);
      conv[p] = res[p] <= tol;
      all = all && conv[p];
    }
    return all;
  };
  auto read_now = [&](double tol) {
    HIPCHK(hipMemcpyAsync(hpart.data(), d.part_res, nch * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return converged_from(hpart.data(), tol);
  };
  const int64_t dim = solve_dim(P);
  const bool thick = o->restart_keep > 0;
  int j = 1;          // basis size
  int step = 0;       // products so far (all phases): the random-restart key index
  cnt = SolveCounts{};
  for (size_t ph = 0; ph < phases.size(); ++ph) {
    const Phase& f = phases[ph];
    // the FP32 phase stores the products in FP32 (they are FP32-accurate);
    // every dot product, the Gram matrix and the Ritz vector stay FP64
    DavBufs dp = d;
    dp.va32 = f.prec == BSDMRG_F32;
    auto product = [&](const double* x, int slot) {
      if (dp.va32) matvec_out32(P, w.a, x, dp.VAf + (int64_t)slot * n, s);
      else matvec(P, f.prec, L, R, w.a, x, d.VA + (int64_t)slot * n, s);
    };
    auto gram_row = [&](int cols, const double* y) {
      if (dp.va32) HIPCHK(dav_dots(P, cols, dp.VAf, n, y, d.part_a, s));
      else HIPCHK(dav_dots(P, cols, d.VA, n, y, d.part_a, s));
    };
    int products = 0;
    int pend = -1, nextb = 0;   // buffer of the check in flight, next buffer
    int& counter = f.prec == BSDMRG_F64 ? cnt.it64 : cnt.it32;
    if (ph == 0) {
      product(d.V, 0);
      products = 1;
      ++step;
    } else {
      // switch: keep x and the previous Ritz vector (or x alone), then
      // recompute their products and the projected matrix in this precision
      const int nkeep = std::min({2, j, f.budget});
      HIPCHK(dav_restart(P, dp, j, nkeep, s));
      HIPCHK(dav_rotate(P, dp, j, nkeep, false, s));
      // the FP32 products shared this memory: clear it, since a product
      // does not write the padding of its vector (which must stay zero)
      if (phases[ph - 1].prec == BSDMRG_F32) HIPCHK(dav_fill_zero(d.VA, (int64_t)B * n, s));
      cnt.thick++;
      j = nkeep;
      for (int r = 0; r < j; ++r) {
        product(d.V + (int64_t)r * n, r);
        ++products;
        ++step;
        if (r + 1 < j) {
          gram_row(r + 1, d.V + (int64_t)r * n);
          HIPCHK(dav_gram_eig(P, dp, r, s));
        }
      }
    }
    bool fresh = false;   // the newest vector is the raw t of the last step (and VA_i its raw product)
    for (;;) {
      const int i = j - 1;
      if (fresh) HIPCHK(dav_fresh_dots(P, dp, j, s));
      else gram_row(j, d.V + (int64_t)i * n);
      fresh = false;
      HIPCHK(dav_gram_eig(P, dp, i, s));
      const bool last = products >= f.budget || j >= dim;
      // q, t and (unless this is the last step) the first Gram-Schmidt dots v_c^T t
      HIPCHK(dav_ritz(P, dp, i, false, last ? nullptr : d.part_a, d.D, s));
      const int every = std::max(1, o->check_every);
      if (!o->fixed_iters && !last && products % every == 0) {
        bool stop = false;
        if (pend >= 0) {
          HIPCHK(hipEventSynchronize(lag.ev[pend]));
          if (converged_from(lag.h + (size_t)pend * nch, f.tol)) stop = read_now(f.tol);
          pend = -1;
        }
        if (stop) {
          HIPCHK(dav_ritz(P, dp, i, true, nullptr, d.D, s));
          break;
        }
        HIPCHK(hipMemcpyAsync(lag.h + (size_t)nextb * nch, d.part_res, nch * sizeof(double), hipMemcpyDeviceToHost,
                              s));
        HIPCHK(hipEventRecord(lag.ev[nextb], s));
        pend = nextb;
        nextb ^= 1;
      }
      if (last) {
        if (!o->fixed_iters) (void)read_now(f.tol);   // also completes a check in flight
        HIPCHK(dav_ritz(P, dp, i, true, nullptr, d.D, s));
        break;
      }
      if (thick && j == B) {
        // thick restart to x and the previous Ritz vector; the dots of t
        // against the new basis (and ||t||^2) are taken again
        HIPCHK(dav_restart(P, dp, j, 2, s));
        HIPCHK(dav_rotate(P, dp, j, 2, true, s));
        cnt.thick++;
        j = 2;
        HIPCHK(dav_dots(P, j, d.V, n, d.q, d.part_a, s, true));
      }
      // the first Gram-Schmidt pass; the second one (when needed) and the
      // normalisation are deferred to the Gram row of the next step, which
      // applies them to t and, H being linear, to the product of t
      HIPCHK(dav_update(P, dp, j, d.part_a, s));
      HIPCHK(dav_finalize(P, dp, j, step - 1, o->seed, o->restart_rtol, P->d_blk_off, P->d_blk_ptr, s));
      product(d.q, j);
      fresh = true;
      ++j;
      ++products;
      ++step;
    }
    counter = products;
  }
  HIPCHK(dav_dots(P, 1, d.x, 0, d.x, d.part_a, s));
  HIPCHK(dav_normalize(P, d.part_a, d.red, d.x, psi, s));
}

extern "C" {

bsdmrg_status bsdmrg_layout(const bsdmrg_leg* legs, int32_t order, const int32_t* signs,
                            int64_t* n_blocks, int32_t* block_sectors, int64_t* offsets,
                            int64_t capacity) {
  return guarded([&] {
    if (!legs || !signs || !n_blocks || order < 1 || order > kMaxOrder)
      throw Error{BSDMRG_EINVAL, "layout: bad arguments"};
    std::vector<Leg> ls;
    for (int i = 0; i < order; ++i) ls.push_back(leg_from(legs[i]));
    std::vector<const Leg*> lp;
    for (auto& l : ls) lp.push_back(&l);
    Layout L = make_layout(lp, signs);
    *n_blocks = (int64_t)L.keys.size();
    if (capacity < (int64_t)L.keys.size()) throw Error{BSDMRG_ECAPACITY, "layout: capacity too small"};
    if (!block_sectors || !offsets) throw Error{BSDMRG_EINVAL, "layout: output arrays are NULL"};
    for (size_t b = 0; b < L.keys.size(); ++b)
      for (int i = 0; i < order; ++i) block_sectors[b * order + i] = L.keys[b][i];
    for (size_t b = 0; b <= L.keys.size(); ++b) offsets[b] = L.offs[b];
  });
}

bsdmrg_status bsdmrg_plan(const bsdmrg_problem* probs, int32_t n_probs, int32_t flags,
                          bsdmrg_plan_t* out) {
  return guarded([&] {
    if (!probs || n_probs < 1 || !out) throw Error{BSDMRG_EINVAL, "plan: bad arguments"};
    *out = nullptr;
    bsdmrg_plan_s* P = build_plan(probs, n_probs);
    if (!(flags & BSDMRG_PLAN_HOST_ONLY)) {
      try {
        upload(P);
      } catch (...) {
        if (P->d_blob) (void)hipFree(P->d_blob);
        delete P;
        throw;
      }
    }
    *out = P;
  });
}

bsdmrg_status bsdmrg_plan_query(bsdmrg_plan_t P, bsdmrg_plan_info* info) {
  return guarded([&] {
    if (!P || !info) throw Error{BSDMRG_EINVAL, "plan_query: NULL argument"};
    info->n_probs = (int64_t)P->probs.size();
    info->psi_elems = P->psi_elems;
    info->L_elems = P->L_elems;
    info->R_elems = P->R_elems;
    info->W1_elems = P->W1_elems;
    info->W2_elems = P->W2_elems;
    info->t1_elems = P->t1_elems;
    info->t2_elems = P->t2_elems;
    info->apply_workspace_bytes = (int64_t)apply_bytes(P);
    bool bwd_built = false;
    {
      std::lock_guard<std::mutex> lk(P->mu);
      bwd_built = P->bwd != nullptr;
    }
    info->backward_workspace_bytes = bwd_built ? heff_backward_bytes(P) : 0;
    info->flops_s1 = P->s1.flops;
    info->flops_s2 = P->flops_s2;
    info->flops_s3 = P->s3.flops;
    info->n_s1_tasks = (int64_t)P->s1.tasks.size();
    info->n_s3_tasks = (int64_t)P->s3.tasks.size();
    info->n_s1_tiles = (int64_t)P->s1.tiles.size();
    info->n_s3_tiles = (int64_t)P->s3.tiles.size();
    info->n_mix_terms = (int64_t)P->mix_terms.size();
    info->n_coefs = P->n_coefs;
    info->s1_big_min = P->s1.big_min;
    info->s3_big_min = P->s3.big_min;
    info->s3_split_k = P->s3_split;
  });
}

bsdmrg_status bsdmrg_plan_offsets(bsdmrg_plan_t P, int32_t p, int64_t* offs) {
  return guarded([&] {
    if (!P || !offs || p < 0 || p >= (int)P->probs.size()) throw Error{BSDMRG_EINVAL, "plan_offsets: bad arguments"};
    const ProblemPlan& q = P->probs[p];
    offs[0] = q.psi_base;
    offs[1] = q.L_base;
    offs[2] = q.R_base;
    offs[3] = q.W1_base;
    offs[4] = q.W2_base;
  });
}

bsdmrg_status bsdmrg_plan_tasks(bsdmrg_plan_t P, int32_t stage, int64_t* tasks4, int64_t capacity,
                                int64_t* n_tasks) {
  return guarded([&] {
    if (!P || !n_tasks || (stage != 1 && stage != 3)) throw Error{BSDMRG_EINVAL, "plan_tasks: bad arguments"};
    const Stage& st = stage == 1 ? P->s1 : P->s3;
    *n_tasks = (int64_t)st.tasks.size();
    if (capacity < *n_tasks) throw Error{BSDMRG_ECAPACITY, "plan_tasks: capacity too small"};
    if (!tasks4) throw Error{BSDMRG_EINVAL, "plan_tasks: NULL output"};
    for (size_t t = 0; t < st.tasks.size(); ++t) {
      tasks4[4 * t + 0] = st.tasks[t].M;
      tasks4[4 * t + 1] = st.tasks[t].N;
      tasks4[4 * t + 2] = st.tasks[t].ksum;
      tasks4[4 * t + 3] = st.tasks[t].nseg;
    }
  });
}

bsdmrg_status bsdmrg_plan_destroy(bsdmrg_plan_t P) {
  return guarded([&] {
    if (!P) return;
    destroy_graph(P);
    destroy_backward(P);
    for (Stage* st : {&P->s1, &P->s3})
      if (st->d_tiles_own) (void)hipFree(st->d_tiles_own);
    if (P->d_blob) (void)hipFree(P->d_blob);
    delete P;
  });
}

bsdmrg_status bsdmrg_heff_apply(bsdmrg_plan_t P, int32_t precision, const double* L, const double* W1,
                                const double* W2, const double* R, const double* psi, double* out,
                                void* workspace, int64_t workspace_bytes, hipStream_t stream) {
  return guarded([&] {
    need_device(P);
    if (precision != BSDMRG_F64 && precision != BSDMRG_F32)
      throw Error{BSDMRG_EINVAL, "heff_apply: precision must be F64 or F32"};
    if (!L || !W1 || !W2 || !R || !psi || !out) throw Error{BSDMRG_EINVAL, "heff_apply: NULL operand"};
    if (psi == out) throw Error{BSDMRG_EINVAL, "heff_apply: out must not alias psi"};
    const size_t need = apply_bytes(P);
    check_ws(workspace, workspace_bytes, need);
    Carve c(workspace, (size_t)workspace_bytes);
    ApplyWS w = carve_apply(P, c);
    prepare(P, precision, L, W1, W2, R, w, stream);
    matvec(P, precision, L, R, w, psi, out, stream);
  });
}

bsdmrg_status bsdmrg_heff_backward_workspace(bsdmrg_plan_t P, int64_t* bytes) {
  return guarded([&] {
    if (!P || !bytes) throw Error{BSDMRG_EINVAL, "heff_backward_workspace: NULL argument"};
    *bytes = heff_backward_bytes(P);
  });
}

bsdmrg_status bsdmrg_heff_backward(bsdmrg_plan_t P, const double* L, const double* W1, const double* W2,
                                   const double* R, const double* psi, const double* g_E, double* d_psi,
                                   double* d_L, double* d_W1, double* d_W2, double* d_R, void* workspace,
                                   int64_t workspace_bytes, hipStream_t stream) {
  return guarded([&] {
    need_device(P);
    if (!L || !W1 || !W2 || !R || !psi || !g_E) throw Error{BSDMRG_EINVAL, "heff_backward: NULL operand"};
    const double* ins[5] = {L, W1, W2, R, psi};
    double* outs[5] = {d_psi, d_L, d_W1, d_W2, d_R};
    for (double* o : outs)
      for (const double* i : ins)
        if (o && (const double*)o == i) throw Error{BSDMRG_EINVAL, "heff_backward: an output aliases an input"};
    for (size_t p = 0; p < P->probs.size(); ++p)
      if (!std::isfinite(g_E[p])) throw Error{BSDMRG_EINVAL, "heff_backward: g_E is not finite"};
    heff_backward_run(P, L, W1, W2, R, psi, g_E, d_psi, d_L, d_W1, d_W2, d_R, workspace, workspace_bytes, stream);
  });
}

bsdmrg_status bsdmrg_heff_energy(bsdmrg_plan_t P, const double* L, const double* W1, const double* W2,
                                 const double* R, const double* psi, double* energy, void* workspace,
                                 int64_t workspace_bytes, hipStream_t stream) {
  return guarded([&] {
    need_device(P);
    if (!L || !W1 || !W2 || !R || !psi || !energy) throw Error{BSDMRG_EINVAL, "heff_energy: NULL argument"};
    heff_energy_run(P, L, W1, W2, R, psi, energy, workspace, workspace_bytes, stream);
  });
}

bsdmrg_status bsdmrg_heff_diagonal(bsdmrg_plan_t P, const double* L, const double* W1, const double* W2,
                                   const double* R, double* D, hipStream_t stream) {
  return guarded([&] {
    need_device(P);
    if (!L || !W1 || !W2 || !R || !D) throw Error{BSDMRG_EINVAL, "heff_diagonal: NULL argument"};
    HIPCHK(dav_diag(P, L, W1, W2, R, D, stream));
  });
}

bsdmrg_status bsdmrg_eig_workspace(bsdmrg_plan_t P, const bsdmrg_eig_opts* o, int64_t* bytes) {
  return guarded([&] {
    if (!P || !bytes) throw Error{BSDMRG_EINVAL, "eig_workspace: NULL argument"};
    validate_opts(P, o);
    Carve c(nullptr, 0);
    carve_eig(P, o, c);
    *bytes = (int64_t)c.used;
  });
}

bsdmrg_status bsdmrg_eigensolve(bsdmrg_plan_t P, const double* L, const double* W1, const double* W2,
                                const double* R, double* psi, const bsdmrg_eig_opts* o, double* energy,
                                bsdmrg_eig_stats* stats, void* workspace, int64_t workspace_bytes,
                                hipStream_t s) {
  return guarded([&] {
    need_device(P);
    validate_opts(P, o);
    if (!L || !W1 || !W2 || !R || !psi || !energy || !stats)
      throw Error{BSDMRG_EINVAL, "eigensolve: NULL argument"};
    Carve c0(nullptr, 0);
    carve_eig(P, o, c0);
    check_ws(workspace, workspace_bytes, c0.used);
    Carve c(workspace, (size_t)workspace_bytes);
    EigWS w = carve_eig(P, o, c);
    const int np = (int)P->probs.size();
    std::vector<int> conv(np, 0);
    std::vector<double> res(np, 0.0);
    SolveCounts cnt;
    const bool graph = o->fixed_iters && o->use_graph && s != nullptr;
    if (graph) {
      std::lock_guard<std::mutex> lk(P->mu);
      if (!P->graph) P->graph = new GraphCache();
      GraphKey key{{L, W1, W2, R, psi, workspace}, *o};
      GraphEntry* hit = nullptr;
      for (GraphEntry& g : P->graph->entries)
        if (g.key == key) hit = &g;
      if (!hit) {
        GraphEntry G;
        G.key = key;
        HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        try {
          enqueue_solve(P, L, W1, W2, R, psi, o, w, s, G.counts, res, conv);
        } catch (...) {
          hipGraph_t g = nullptr;
          (void)hipStreamEndCapture(s, &g);
          if (g) (void)hipGraphDestroy(g);
          throw;
        }
        HIPCHK(hipStreamEndCapture(s, &G.graph));
        hipError_t e = hipGraphInstantiate(&G.exec, G.graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
          (void)hipGraphDestroy(G.graph);
          HIPCHK(e);
        }
        if (P->graph->entries.size() >= kMaxGraphs) {
          // an in-flight launch of the evicted graph completes normally
          GraphEntry& old = P->graph->entries.front();
          (void)hipGraphExecDestroy(old.exec);
          (void)hipGraphDestroy(old.graph);
          P->graph->entries.erase(P->graph->entries.begin());
        }
        P->graph->entries.push_back(G);
        hit = &P->graph->entries.back();
      }
      HIPCHK(hipGraphLaunch(hit->exec, s));
      cnt = hit->counts;
    } else {
      enqueue_solve(P, L, W1, W2, R, psi, o, w, s, cnt, res, conv);
    }
    std::vector<double> lam(np);
    std::vector<int32_t> rs(2 * np);
    std::vector<double> hpart(P->chunks.size());
    HIPCHK(hipMemcpyAsync(lam.data(), w.d.lam, np * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(rs.data(), w.d.restarts, 2 * np * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(hpart.data(), w.d.part_res, hpart.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    bool failed = false;
    for (int p = 0; p < np; ++p) {
      const DavProb& pr = P->dav_probs[p];
      double r = 0.0;
      for (int cc = 0; cc < pr.nchunk; ++cc) r += hpart[pr.chunk0 + cc];
      energy[p] = lam[p];
      stats[p].iters = cnt.it64;
      stats[p].iters_f32 = cnt.it32;
      stats[p].restarts = rs[p];
      stats[p].residual = std::sqrt(r);
      stats[p].converged = stats[p].residual <= o->tol;
      stats[p].thick_restarts = cnt.thick;
      stats[p].pad = 0;
      failed = failed || rs[np + p] != 0;
    }
    if (failed) throw Error{BSDMRG_ESOLVER, "eigensolve: reorthogonalisation failed after 3 restarts"};
  });
}

bsdmrg_status bsdmrg_stage_timing(bsdmrg_plan_t P, int32_t precision, const double* L, const double* W1,
                                  const double* W2, const double* R, const double* psi, double* out,
                                  void* workspace, int64_t workspace_bytes, int32_t reps, float* ms,
                                  hipStream_t s) {
  hipEvent_t ev[2] = {nullptr, nullptr};
  bsdmrg_status st = guarded([&] {
    need_device(P);
    if (precision != BSDMRG_F64 && precision != BSDMRG_F32 && precision != BSDMRG_F32_REFINE)
      throw Error{BSDMRG_EINVAL, "stage_timing: precision must be F64, F32 or F32_REFINE"};
    if (!L || !W1 || !W2 || !R || !psi || !out || !ms || reps < 1)
      throw Error{BSDMRG_EINVAL, "stage_timing: bad arguments"};
    // F32_REFINE: the stages as the FP32 phase of a mixed eigensolve runs
    // them (S3 and its split-K sum write FP32 products, here into out)
    const bool solve32 = precision == BSDMRG_F32_REFINE;
    if (solve32) precision = BSDMRG_F32;
    check_ws(workspace, workspace_bytes, apply_bytes(P));
    Carve c(workspace, (size_t)workspace_bytes);
    ApplyWS w = carve_apply(P, c);
    HIPCHK(hipEventCreate(&ev[0]));
    HIPCHK(hipEventCreate(&ev[1]));
    prepare(P, precision, L, W1, W2, R, w, s);
    float* T1f = (float*)w.T1;
    float* T2f = (float*)w.T2;
    for (int stage = 0; stage < 5; ++stage) {
      HIPCHK(hipEventRecord(ev[0], s));
      for (int r = 0; r < reps; ++r) {
        if (stage == 0) HIPCHK(launch_coef(P, W1, W2, w.coef, s));
        if (stage == 4) {
          if (solve32) HIPCHK(launch_s3_reduce_out32(P, w.part, (float*)out, s));
          else HIPCHK(launch_s3_reduce(P, w.part, out, precision == BSDMRG_F32, s));
        }
        if (precision == BSDMRG_F64) {
          if (stage == 1) HIPCHK(launch_s1_f64(P, L, psi, w.T1, s));
          if (stage == 2) HIPCHK(launch_mix_f64(P, w.coef, w.T1, w.T2, s));
          if (stage == 3) HIPCHK(launch_s3_gemm_f64(P, w.T2, R, out, w.part, s));
        } else {
          if (stage == 1) HIPCHK(launch_s1_f32(P, w.L32, psi, T1f, s));
          if (stage == 2) HIPCHK(launch_mix_f32(P, w.coef, T1f, T2f, s));
          if (stage == 3) {
            if (solve32) HIPCHK(launch_s3_gemm_f32_out32(P, T2f, w.R32, (float*)out, w.part, s));
            else HIPCHK(launch_s3_gemm_f32(P, T2f, w.R32, out, w.part, s));
          }
        }
      }
      HIPCHK(hipEventRecord(ev[1], s));
      HIPCHK(hipEventSynchronize(ev[1]));
      float t = 0.f;
      HIPCHK(hipEventElapsedTime(&t, ev[0], ev[1]));
      ms[stage] = t / reps;
    }
    if (solve32) {
      // out holds FP32 products, also where it has padding, which a product
      // leaves unwritten: cleared, then the FP32 product as with F32
      HIPCHK(dav_fill_zero(out, P->psi_elems, s));
      matvec(P, BSDMRG_F32, L, R, w, psi, out, s);
      HIPCHK(hipStreamSynchronize(s));
    }
  });
  for (auto e : ev)
    if (e) (void)hipEventDestroy(e);
  return st;
}

bsdmrg_status bsdmrg_plan_set_tiles(bsdmrg_plan_t P, int32_t s1_big_min, int32_t s3_big_min) {
  return guarded([&] {
    need_device(P);
    if (s1_big_min < 0 || s3_big_min < 0) throw Error{BSDMRG_EINVAL, "plan_set_tiles: big_min must be >= 0"};
    reschedule_stage(P, P->s1, std::min(s1_big_min, kNoBigTiles), "S1 tiles");
    reschedule_stage(P, P->s3, std::min(s3_big_min, kNoBigTiles), "S3 tiles");
  });
}

bsdmrg_status bsdmrg_plan_autotune(bsdmrg_plan_t P, int32_t precision, const double* L, const double* W1,
                                   const double* W2, const double* R, const double* psi, double* out,
                                   void* workspace, int64_t workspace_bytes, int32_t reps, int32_t* big_min,
                                   hipStream_t s) {
  hipEvent_t ev[2] = {nullptr, nullptr};
  bsdmrg_status st = guarded([&] {
    need_device(P);
    if (precision != BSDMRG_F64 && precision != BSDMRG_F32)
      throw Error{BSDMRG_EINVAL, "plan_autotune: precision must be F64 or F32"};
    if (!L || !W1 || !W2 || !R || !psi || !out || !big_min || reps < 1 || psi == out)
      throw Error{BSDMRG_EINVAL, "plan_autotune: bad arguments"};
    check_ws(workspace, workspace_bytes, apply_bytes(P));
    Carve c(workspace, (size_t)workspace_bytes);
    ApplyWS w = carve_apply(P, c);
    HIPCHK(hipEventCreate(&ev[0]));
    HIPCHK(hipEventCreate(&ev[1]));
    prepare(P, precision, L, W1, W2, R, w, s);
    matvec(P, precision, L, R, w, psi, out, s);   // T1 and T2 hold the values the stages see
    static const int32_t kCand[] = {kNoBigTiles, 0, 384, 256, 160, 96};
    for (int which = 0; which < 2; ++which) {
      Stage& sg = which == 0 ? P->s1 : P->s3;
      const char* name = which == 0 ? "S1 tiles" : "S3 tiles";
      auto launch = [&] {
        if (precision == BSDMRG_F64) {
          if (which == 0) HIPCHK(launch_s1_f64(P, L, psi, w.T1, s));
          else HIPCHK(launch_s3_gemm_f64(P, w.T2, R, out, w.part, s));
        } else {
          if (which == 0) HIPCHK(launch_s1_f32(P, w.L32, psi, (float*)w.T1, s));
          else HIPCHK(launch_s3_gemm_f32(P, (float*)w.T2, w.R32, out, w.part, s));
        }
      };
      int32_t best = kNoBigTiles;
      float best_t = 0.f;
      bool first = true;
      std::vector<std::vector<GemmTile>> seen;
      for (int32_t cand : kCand) {
        if (cand != 0) {   // tile classes that give the same one-workgroup-per-tile schedule are timed once
          Stage probe;
          probe.tasks = sg.tasks;
          schedule_tiles(probe, cand);
          bool dup = false;
          for (const auto& t : seen)
            dup = dup || (t.size() == probe.tiles.size() &&
                          std::memcmp(t.data(), probe.tiles.data(), t.size() * sizeof(GemmTile)) == 0);
          if (dup) continue;
          seen.push_back(probe.tiles);
        }
        reschedule_stage(P, sg, cand, name);
        launch();   // warm-up
        HIPCHK(hipEventRecord(ev[0], s));
        for (int r = 0; r < reps; ++r) launch();
        HIPCHK(hipEventRecord(ev[1], s));
        HIPCHK(hipEventSynchronize(ev[1]));
        float t = 0.f;
        HIPCHK(hipEventElapsedTime(&t, ev[0], ev[1]));
        if (first || t < 0.98f * best_t) {
          first = false;
          best = cand;
          best_t = t;
        }
      }
      reschedule_stage(P, sg, best, name);
      big_min[which] = best;
    }
    // out holds one product again (the S3 timing runs wrote split-K pieces only)
    matvec(P, precision, L, R, w, psi, out, s);
    HIPCHK(hipStreamSynchronize(s));
  });
  for (auto e : ev)
    if (e) (void)hipEventDestroy(e);
  return st;
}

const char* bsdmrg_last_error(void) { return last_error_cstr(); }

}  // extern "C"
