// Launch wrappers of the device kernels (host-callable).
#pragma once

#include <hip/hip_runtime.h>

#include "bsdmrg_internal.h"

namespace bsd {

// two-site product stages
hipError_t launch_s1_f64(const bsdmrg_plan_s* P, const double* L, const double* psi, double* T1,
                         hipStream_t s);
hipError_t launch_s3_f64(const bsdmrg_plan_s* P, const double* T2, const double* R, double* out,
                         double* part, hipStream_t s);
hipError_t launch_s1_f32(const bsdmrg_plan_s* P, const float* L, const double* psi, float* T1,
                         hipStream_t s);
hipError_t launch_s3_f32(const bsdmrg_plan_s* P, const float* T2, const float* R, double* out,
                         double* part, hipStream_t s);
// S3 as its two launches: split-K GEMM pieces, then their fixed-order sum
hipError_t launch_s3_gemm_f64(const bsdmrg_plan_s* P, const double* T2, const double* R, double* out,
                              double* part, hipStream_t s);
hipError_t launch_s3_gemm_f32(const bsdmrg_plan_s* P, const float* T2, const float* R, double* out,
                              double* part, hipStream_t s);
// S3 in FP32 with FP32 output (the products of the FP32 phase of a mixed
// Davidson solve), split-K pieces summed
hipError_t launch_s3_f32_out32(const bsdmrg_plan_s* P, const float* T2, const float* R, float* out, double* part,
                               hipStream_t s);
hipError_t launch_s3_gemm_f32_out32(const bsdmrg_plan_s* P, const float* T2, const float* R, float* out,
                                    double* part, hipStream_t s);
hipError_t launch_s3_reduce_out32(const bsdmrg_plan_s* P, const double* part, float* out, hipStream_t s);
// f32_parts: the partials were written by the FP32 S3 launch (FP32 values in
// the partial buffer); else FP64 partials.
hipError_t launch_s3_reduce(const bsdmrg_plan_s* P, const double* part, double* out, bool f32_parts,
                            hipStream_t s);
hipError_t launch_mix_f64(const bsdmrg_plan_s* P, const double* coef, const double* T1, double* T2,
                          hipStream_t s);
hipError_t launch_mix_f32(const bsdmrg_plan_s* P, const double* coef, const float* T1, float* T2,
                          hipStream_t s);
hipError_t launch_coef(const bsdmrg_plan_s* P, const double* W1, const double* W2, double* coef,
                       hipStream_t s);
hipError_t launch_cast(int64_t n, const double* x, float* y, hipStream_t s);
// sparse-dense product of a dense op (precision 0: FP64, 1: FP32 MFMA with
// FP32 T1, T2, WW and L, R cast into Lf, Rf)
hipError_t launch_dense_product(const bsdmrg_op_s* O, int precision, const double* L, const double* W1,
                                const double* W2, const double* R, const double* psi, double* out, void* T1,
                                void* T2, void* WW, float* Lf, float* Rf, hipStream_t s);

enum { kNN = 0, kNT = 1, kTN = 2 };
hipError_t launch_copy(const void* d_tasks, int n, const double* src, double* dst, const double* fac,
                       hipStream_t s);
hipError_t launch_svd_qr(const void* d_tasks, int n, double* work, double* S, hipStream_t s);
hipError_t launch_svd_qr_big(const void* d_big, int n_big, const void* d_cols, int n_cols, int n_max,
                             const void* d_tasks, double* work, double* S, hipStream_t s);
hipError_t launch_svd_bjac(const void* d_pairs, int n_pairs, const void* d_tasks, double* work,
                           const double* active, double* rot, int step, hipStream_t s);
hipError_t launch_svd_finish(const void* d_tasks, int n, const void* d_cols, int n_cols, double* work, double* U,
                             double* S, double* Vt, hipStream_t s);
hipError_t launch_gauge(const void* d_tasks, int n, const double* U, const double* S, double* sign,
                        double* sgn_s, hipStream_t s);
hipError_t launch_gemm_f64(const Stage& st, int layout, const double* A, const double* B, double* C,
                           double* Cpart, hipStream_t s);
hipError_t launch_mix_tables(const MixItem* items, size_t n_items, const MixTask* tasks, const MixTerm* terms,
                             const double* coef, const double* src, double* dst, hipStream_t s);

// Davidson (Alg. 1) building blocks; every vector spans all problems of the
// plan, reductions are per problem through the chunk table.
struct DavBufs {
  double* V;        // basis, B vectors of n elements
  double* VA;       // products
  float* VAf;       // the products stored in FP32 (FP32 phase of a mixed solve; the memory of VA)
  bool va32;        // the launches read and write VAf instead of VA
  double* x;
  double* q;
  double* part_a;   // (B + 1) * nchunk partial sums
  double* part_b;
  double* part_n0;  // nchunk: ||t||^2 before orthogonalisation (t = q, or the preconditioned q)
  double* part_res; // nchunk: ||q||^2 (the residual)
  double* cp;       // n_probs * 64: coefficients of the deferred second Gram-Schmidt pass
  double* p2;       // n_probs: 1 when the deferred second pass applies, else 0
  double* nq0;      // n_probs: ||q||^2 before orthogonalisation (total)
  double* red;      // n_probs * 64 per-problem sums of partials
  double* M;        // n_probs * B * B projected matrices
  double* svec;     // n_probs * B Ritz vectors of M
  double* svec_prev;// n_probs * B the previous step's Ritz vector (thick restart)
  double* Srot;     // n_probs * 2 * B restart coefficients
  double* D;        // n (diagonal of H_eff) or null
  double* lam;      // n_probs
  double* scale;    // n_probs
  int32_t* restarts;  // n_probs
  int32_t* status;    // n_probs, non-zero when a restart failed
  int64_t n;        // vector length (all problems)
  int B;            // max basis size
};

hipError_t dav_fill_zero(double* x, int64_t n, hipStream_t s);
// part[j] (j < J) = chunk partials of X_j^T y; with norm_col also ||y||^2 as column J
hipError_t dav_dots(const bsdmrg_plan_s* P, int J, const double* X, int64_t xstride, const double* y,
                    double* part, hipStream_t s, bool norm_col = false);
hipError_t dav_dots(const bsdmrg_plan_s* P, int J, const float* X, int64_t xstride, const double* y, double* part,
                    hipStream_t s);
// thick restart coefficients (nkeep 1 or 2 vectors out of j) and the new projected matrix
hipError_t dav_restart(const bsdmrg_plan_s* P, const DavBufs& b, int j, int nkeep, hipStream_t s);
// V (and VA) <- V S in place, nout output vectors from J inputs
hipError_t dav_rotate(const bsdmrg_plan_s* P, const DavBufs& b, int J, int nout, bool with_products,
                      hipStream_t s);
// D = diagonal of H_eff (padding 0)
hipError_t dav_diag(const bsdmrg_plan_s* P, const double* L, const double* W1, const double* W2, const double* R,
                    double* D, hipStream_t s);
hipError_t dav_psum(const bsdmrg_plan_s* P, int J, const double* part, double* red, int ldr, hipStream_t s);
hipError_t dav_normalize(const bsdmrg_plan_s* P, const double* part, double* red, const double* x, double* y,
                         hipStream_t s);
hipError_t dav_gram_eig(const bsdmrg_plan_s* P, const DavBufs& b, int i, hipStream_t s);
// q and the new direction t (q, or q / (D - lambda) when D is non-null) into
// b.q, x when want_x; with part_d also the partial dots v_j^T t, j <= i, and
// ||t||^2 as column i + 1
hipError_t dav_ritz(const bsdmrg_plan_s* P, const DavBufs& b, int i, bool want_x, double* part_d,
                    const double* D, hipStream_t s);
// first Gram-Schmidt pass t -= V c (c from part_in), the partial dots of the
// result for the second pass into b.part_b
hipError_t dav_update(const bsdmrg_plan_s* P, const DavBufs& b, int J, const double* part_in, hipStream_t s);
// J: basis size; step: product index of the random-restart key.  Decides the
// second pass and the scale of the new vector (or restarts it at random)
hipError_t dav_finalize(const bsdmrg_plan_s* P, const DavBufs& b, int J, int step, uint64_t seed, double rtol,
                        const int64_t* blk_off, const int32_t* blk_ptr, hipStream_t s);
// basis vector i = J - 1 and its product from t (b.q) and its raw product
// (in VA_i): the deferred second pass and the scale applied to both, then
// the Gram row partials VA_c^T v_i (c <= i) into b.part_a
hipError_t dav_fresh_dots(const bsdmrg_plan_s* P, const DavBufs& b, int J, hipStream_t s);

// adjoint kernels (kernels_bwd.hip)
constexpr int kSiteDotGroup = 32;   // sites per launch of the chain-rule dots
struct SiteDotGroup {
  const double* x[kSiteDotGroup];
  const double* y[kSiteDotGroup];
  int64_t n[kSiteDotGroup];
};
hipError_t launch_site_dots(const SiteDotGroup& g, int count, int base, double* terms, hipStream_t s);
hipError_t launch_ordered_sum(int n, double* terms, hipStream_t s);
hipError_t launch_bwd_dots(const BwdDot* items, int n, const double* G, const double* T1, double* part,
                           hipStream_t s);
hipError_t launch_bwd_coef(int n, const int32_t* ptr, const double* part, const int64_t* idx, double* out,
                           hipStream_t s);
hipError_t launch_bwd_wgrad(int64_t n, const int32_t* ptr, const int32_t* coef, const int64_t* partner,
                            const double* dcoef, const double* Wother, double g, double* dW, hipStream_t s);
hipError_t launch_seg_scale(int64_t n, const int64_t* base, int np, const double* g, const double* x,
                            const double* y, double* out, hipStream_t s);

// XCD-aware tile schedule of a GEMM stage (schedule.cpp)
void schedule_tiles(Stage& st, int32_t big_min = kNoBigTiles);
void flatten_tiles(Stage& st);   // Stage::ftiles from the tiles, tasks and segments
void validate_tiles(const Stage& st, const char* name);
// persistent launch of a stage: 64 x 64 tiles dealt to slots_per_xcd
// workgroups per XCD (schedule.cpp), and its table check (validate.cpp)
void schedule_persistent(Stage& st, int slots_per_xcd);
void validate_ptiles(const Stage& st, const char* name);

// host-side table checks (validate.cpp)
void validate_gemm(const Stage& st, int layout, int64_t a_elems, int64_t b_elems, int64_t c_elems,
                   int64_t cpart_elems, const char* name);
void validate_mix(const std::vector<MixTask>& tasks, const std::vector<MixTerm>& terms,
                  const std::vector<MixItem>& items, int64_t src_elems, int64_t dst_elems, int64_t coef_elems,
                  const char* name, int64_t item_max = 4096);
void validate_copy(const std::vector<CopyTask>& tasks, int64_t src_elems, int64_t dst_elems, int64_t fac_elems,
                   const char* name);
void validate_heff_plan(const bsdmrg_plan_s* P);

}  // namespace bsd
