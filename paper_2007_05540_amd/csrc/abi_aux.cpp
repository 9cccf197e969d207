// C ABI of the sweep operations: truncated SVD split, environment extension,
// two-site merge.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <stdexcept>

#include "bsdmrg_internal.h"
#include "kernels.h"

namespace bsd {
bsdmrg_op_s* build_env(const bsdmrg_env_problem& in, int side);
bsdmrg_op_s* build_merge(const Leg& a, const Leg& s1, const Leg& b, const Leg& s2, const Leg& c);
void truncate_workspace(const bsdmrg_leg* legs, int64_t* bytes);
void truncate_run(const bsdmrg_leg* legs, const double* theta, const bsdmrg_trunc_opts* o, int32_t* new_n,
                  int32_t* new_q, int64_t* new_d, int32_t leg_cap, double* A, int64_t A_cap, int64_t* A_elems,
                  double* B, int64_t B_cap, int64_t* B_elems, double* svals, int64_t sv_cap, int64_t* n_kept,
                  double* discarded, void* ws, int64_t ws_bytes, hipStream_t st);
void destroy_env_backward(bsdmrg_op_s* O);
int64_t env_backward_bytes(bsdmrg_op_s* O);
void env_backward_run(bsdmrg_op_s* O, const double* env, const double* site, const double* d_out, double* d_W,
                      void* ws, int64_t ws_bytes, hipStream_t s);
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

static size_t al(size_t b) { return (b + 255) / 256 * 256; }

static void upload_op(bsdmrg_op_s* O) {
  struct Part { const void* src; size_t bytes; void** dst; };
  std::vector<Part> parts = {
      {O->g1.tasks.data(), O->g1.tasks.size() * sizeof(GemmTask), (void**)&O->g1.d_tasks},
      {O->g1.segs.data(), O->g1.segs.size() * sizeof(GemmSeg), (void**)&O->g1.d_segs},
      {O->g1.tiles.data(), O->g1.tiles.size() * sizeof(GemmTile), (void**)&O->g1.d_tiles},
      {O->g2.tasks.data(), O->g2.tasks.size() * sizeof(GemmTask), (void**)&O->g2.d_tasks},
      {O->g2.segs.data(), O->g2.segs.size() * sizeof(GemmSeg), (void**)&O->g2.d_segs},
      {O->g2.tiles.data(), O->g2.tiles.size() * sizeof(GemmTile), (void**)&O->g2.d_tiles},
      {O->mix_tasks.data(), O->mix_tasks.size() * sizeof(MixTask), (void**)&O->d_mix_tasks},
      {O->mix_terms.data(), O->mix_terms.size() * sizeof(MixTerm), (void**)&O->d_mix_terms},
      {O->mix_items.data(), O->mix_items.size() * sizeof(MixItem), (void**)&O->d_mix_items},
  };
  size_t total = 0;
  for (auto& p : parts) total += al(std::max<size_t>(p.bytes, 1));
  HIPCHK(hipMalloc(&O->d_blob, total));
  std::vector<char> host(total, 0);
  size_t off = 0;
  for (auto& p : parts) {
    if (p.bytes) std::memcpy(host.data() + off, p.src, p.bytes);
    *p.dst = (char*)O->d_blob + off;
    off += al(std::max<size_t>(p.bytes, 1));
  }
  HIPCHK(hipMemcpy(O->d_blob, host.data(), total, hipMemcpyHostToDevice));
}

static int64_t op_ws_bytes(const bsdmrg_op_s* O) { return (int64_t)(al(O->x1_elems * 8) + al(O->x2_elems * 8)); }

extern "C" {

bsdmrg_status bsdmrg_env_plan(const bsdmrg_env_problem* p, int32_t side, int32_t flags, bsdmrg_op_t* out) {
  return guarded([&] {
    if (!p || !out || (side != 0 && side != 1)) throw Error{BSDMRG_EINVAL, "env_plan: bad arguments"};
    *out = nullptr;
    bsdmrg_op_s* O = build_env(*p, side);
    try {
      if (!(flags & BSDMRG_PLAN_HOST_ONLY)) upload_op(O);
    } catch (...) {
      if (O->d_blob) (void)hipFree(O->d_blob);
      delete O;
      throw;
    }
    *out = O;
  });
}

bsdmrg_status bsdmrg_merge_plan(const bsdmrg_leg* legs, int32_t flags, bsdmrg_op_t* out) {
  return guarded([&] {
    if (!legs || !out) throw Error{BSDMRG_EINVAL, "merge_plan: bad arguments"};
    *out = nullptr;
    Leg a = leg_from(legs[0]), s1 = leg_from(legs[1]), b = leg_from(legs[2]), s2 = leg_from(legs[3]),
        c = leg_from(legs[4]);
    bsdmrg_op_s* O = build_merge(a, s1, b, s2, c);
    try {
      if (!(flags & BSDMRG_PLAN_HOST_ONLY)) upload_op(O);
    } catch (...) {
      if (O->d_blob) (void)hipFree(O->d_blob);
      delete O;
      throw;
    }
    *out = O;
  });
}

bsdmrg_status bsdmrg_op_query(bsdmrg_op_t O, int64_t* workspace_bytes, int64_t* out_elems, double* flops) {
  return guarded([&] {
    if (!O) throw Error{BSDMRG_EINVAL, "op_query: NULL op"};
    if (workspace_bytes) *workspace_bytes = op_ws_bytes(O);
    if (out_elems) *out_elems = O->out_elems;
    if (flops) *flops = O->flops;
  });
}

bsdmrg_status bsdmrg_op_destroy(bsdmrg_op_t O) {
  return guarded([&] {
    if (!O) return;
    destroy_env_backward(O);
    if (O->d_blob) (void)hipFree(O->d_blob);
    delete O;
  });
}

bsdmrg_status bsdmrg_env_update(bsdmrg_op_t O, const double* env, const double* mps, const double* W,
                                double* env_out, void* workspace, int64_t workspace_bytes, hipStream_t s) {
  return guarded([&] {
    if (!O || (O->kind != 1 && O->kind != 2)) throw Error{BSDMRG_EINVAL, "env_update: not an environment op"};
    if (!O->d_blob) throw Error{BSDMRG_EINVAL, "env_update: op was built host-only"};
    if (!env || !mps || !W || !env_out) throw Error{BSDMRG_EINVAL, "env_update: NULL operand"};
    if (workspace_bytes < op_ws_bytes(O) || (op_ws_bytes(O) > 0 && !workspace))
      throw Error{BSDMRG_EINVAL, "env_update: workspace too small"};
    double* X1 = (double*)workspace;
    double* X2 = (double*)((char*)workspace + al(O->x1_elems * 8));
    // left: A-op of stage 1 is the environment, B-op the MPS site;
    // right: A-op the environment, B-op the MPS site stored N x K
    HIPCHK(launch_gemm_f64(O->g1, O->layout1, env, mps, X1, X1, s));
    HIPCHK(launch_mix_tables(O->d_mix_items, O->mix_items.size(), O->d_mix_tasks, O->d_mix_terms, W, X1, X2, s));
    HIPCHK(launch_gemm_f64(O->g2, O->layout2, mps, X2, env_out, env_out, s));
  });
}

bsdmrg_status bsdmrg_env_backward_workspace(bsdmrg_op_t O, int64_t* bytes) {
  return guarded([&] {
    if (!O || !bytes) throw Error{BSDMRG_EINVAL, "env_backward_workspace: NULL argument"};
    if (O->kind != 1 && O->kind != 2) throw Error{BSDMRG_EINVAL, "env_backward_workspace: not an environment op"};
    *bytes = env_backward_bytes(O);
  });
}

bsdmrg_status bsdmrg_env_backward(bsdmrg_op_t O, const double* env, const double* mps, const double* d_out,
                                  double* d_W, void* workspace, int64_t workspace_bytes, hipStream_t s) {
  return guarded([&] {
    if (!O || (O->kind != 1 && O->kind != 2)) throw Error{BSDMRG_EINVAL, "env_backward: not an environment op"};
    if (!env || !mps || !d_out || !d_W) throw Error{BSDMRG_EINVAL, "env_backward: NULL operand"};
    if (d_W == env || d_W == mps || d_W == d_out) throw Error{BSDMRG_EINVAL, "env_backward: d_W aliases an input"};
    env_backward_run(O, env, mps, d_out, d_W, workspace, workspace_bytes, s);
  });
}

bsdmrg_status bsdmrg_merge(bsdmrg_op_t O, const double* A, const double* B, double* theta, hipStream_t s) {
  return guarded([&] {
    if (!O || O->kind != 3) throw Error{BSDMRG_EINVAL, "merge: not a merge op"};
    if (!O->d_blob) throw Error{BSDMRG_EINVAL, "merge: op was built host-only"};
    if (!A || !B || !theta) throw Error{BSDMRG_EINVAL, "merge: NULL operand"};
    HIPCHK(launch_gemm_f64(O->g1, O->layout1, A, B, theta, theta, s));
  });
}

bsdmrg_status bsdmrg_truncate_workspace(const bsdmrg_leg* theta_legs, int64_t* bytes) {
  return guarded([&] {
    if (!theta_legs || !bytes) throw Error{BSDMRG_EINVAL, "truncate_workspace: NULL argument"};
    truncate_workspace(theta_legs, bytes);
  });
}

bsdmrg_status bsdmrg_truncate(const bsdmrg_leg* theta_legs, const double* theta, const bsdmrg_trunc_opts* o,
                              int32_t* new_n_sectors, int32_t* new_charges, int64_t* new_dims,
                              int32_t leg_capacity, double* A, int64_t A_capacity, int64_t* A_elems, double* B,
                              int64_t B_capacity, int64_t* B_elems, double* svals, int64_t sv_capacity,
                              int64_t* n_kept, double* discarded, void* workspace, int64_t workspace_bytes,
                              hipStream_t stream) {
  return guarded([&] {
    if (!theta_legs) throw Error{BSDMRG_EINVAL, "truncate: NULL legs"};
    truncate_run(theta_legs, theta, o, new_n_sectors, new_charges, new_dims, leg_capacity, A, A_capacity, A_elems,
                 B, B_capacity, B_elems, svals, sv_capacity, n_kept, discarded, workspace, workspace_bytes, stream);
  });
}

}  // extern "C"
