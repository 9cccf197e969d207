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
bsdmrg_op_s* build_dense(int64_t ma, int64_t mc, int32_t k, int32_t d);
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
      {O->g3.tasks.data(), O->g3.tasks.size() * sizeof(GemmTask), (void**)&O->g3.d_tasks},
      {O->g3.segs.data(), O->g3.segs.size() * sizeof(GemmSeg), (void**)&O->g3.d_segs},
      {O->g3.tiles.data(), O->g3.tiles.size() * sizeof(GemmTile), (void**)&O->g3.d_tiles},
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

// dense product workspace: T1, T2, WW in FP64, or T1, T2, WW, L and R in FP32
static int64_t dense_ws_bytes(const bsdmrg_op_s* O, int precision) {
  const int64_t dk = (int64_t)O->dn_d * O->dn_d * O->dn_k;
  if (precision == BSDMRG_F64) return (int64_t)(al(O->x1_elems * 8) + al(O->x2_elems * 8) + al(dk * dk * 8));
  return (int64_t)(al(O->x1_elems * 4) + al(O->x2_elems * 4) + al(dk * dk * 4) +
                   al(O->dn_ma * O->dn_k * O->dn_ma * 4) + al(O->dn_mc * O->dn_k * O->dn_mc * 4));
}

static int64_t op_ws_bytes(const bsdmrg_op_s* O) {
  if (O->kind == 4) return std::max(dense_ws_bytes(O, BSDMRG_F64), dense_ws_bytes(O, BSDMRG_F32));
  return (int64_t)(al(O->x1_elems * 8) + al(O->x2_elems * 8));
}

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

bsdmrg_status bsdmrg_dense_plan(int64_t ma, int64_t mc, int32_t k, int32_t d, int32_t flags, bsdmrg_op_t* out) {
  return guarded([&] {
    if (!out) throw Error{BSDMRG_EINVAL, "dense_plan: NULL output"};
    *out = nullptr;
    bsdmrg_op_s* O = build_dense(ma, mc, k, d);
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

bsdmrg_status bsdmrg_dense_apply(bsdmrg_op_t O, int32_t precision, const double* L, const double* W1,
                                 const double* W2, const double* R, const double* psi, double* out,
                                 void* workspace, int64_t workspace_bytes, hipStream_t s) {
  return guarded([&] {
    if (!O || O->kind != 4) throw Error{BSDMRG_EINVAL, "dense_apply: not a dense product op"};
    if (!O->d_blob) throw Error{BSDMRG_EINVAL, "dense_apply: op was built host-only"};
    if (precision != BSDMRG_F64 && precision != BSDMRG_F32)
      throw Error{BSDMRG_EINVAL, "dense_apply: precision must be BSDMRG_F64 or BSDMRG_F32"};
    if (!L || !W1 || !W2 || !R || !psi || !out) throw Error{BSDMRG_EINVAL, "dense_apply: NULL operand"};
    if (out == psi) throw Error{BSDMRG_EINVAL, "dense_apply: out aliases psi"};
    const int64_t need = dense_ws_bytes(O, precision);
    if (!workspace || workspace_bytes < need)
      throw Error{BSDMRG_EINVAL, "dense_apply: workspace too small: need " + std::to_string(need) + " bytes"};
    const size_t es = precision == BSDMRG_F64 ? 8 : 4;
    const int64_t dk = (int64_t)O->dn_d * O->dn_d * O->dn_k;
    char* p = (char*)workspace;
    void* T1 = p;
    p += al(O->x1_elems * es);
    void* T2 = p;
    p += al(O->x2_elems * es);
    void* WW = p;
    p += al(dk * dk * es);
    float* Lf = precision == BSDMRG_F32 ? (float*)p : nullptr;
    if (Lf) p += al(O->dn_ma * O->dn_k * O->dn_ma * 4);
    float* Rf = precision == BSDMRG_F32 ? (float*)p : nullptr;
    HIPCHK(launch_dense_product(O, precision, L, W1, W2, R, psi, out, T1, T2, WW, Lf, Rf, s));
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

bsdmrg_status bsdmrg_param_derivative(int32_t n_sites, const double* const* dE_dW, const double* const* dW_dp,
                                      const int64_t* n_elems, double* terms, double* result, hipStream_t s) {
  return guarded([&] {
    if (n_sites < 1 || !dE_dW || !dW_dp || !n_elems || !terms || !result)
      throw Error{BSDMRG_EINVAL, "param_derivative: NULL argument or n_sites < 1"};
    for (int i = 0; i < n_sites; ++i) {
      if (n_elems[i] < 0) throw Error{BSDMRG_EINVAL, "param_derivative: negative element count"};
      if (n_elems[i] > 0 && (!dE_dW[i] || !dW_dp[i])) throw Error{BSDMRG_EINVAL, "param_derivative: NULL site"};
    }
    for (int base = 0; base < n_sites; base += kSiteDotGroup) {
      SiteDotGroup g{};
      const int count = std::min(kSiteDotGroup, n_sites - base);
      for (int b = 0; b < count; ++b) {
        g.x[b] = dE_dW[base + b];
        g.y[b] = dW_dp[base + b];
        g.n[b] = n_elems[base + b];
      }
      HIPCHK(launch_site_dots(g, count, base, terms, s));
    }
    HIPCHK(launch_ordered_sum(n_sites, terms, s));
    HIPCHK(hipMemcpyAsync(result, terms + n_sites, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
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
