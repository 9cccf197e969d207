// Adjoint of the two-site energy functional
//   E = psi^T H_eff psi = sum psi(a',s1',s2',c') L(a',w,a) W1(w,s1',s1,w')
//                             W2(w',s2',s2,w'') R(c',w'',c) psi(a,s1,s2,c)
// (real tensors; the two-site form of the projected operator of Sec. II-C).
// E is linear in each of L, W1, W2 and R, so each gradient is the same
// contraction with that operand left out.  With the forward intermediates
// T1 = L psi and T2 = mix(T1) and the bra-side partial G = psi R:
//   B1  G(a',s1',s2',w'',c) = sum_c' psi(a',s1',s2',c') R(c',w'',c)   NN GEMM
//   B2  H(a',w,s1,s2,c) = sum WW(w,s1',s2',s1,s2,w'') G(...)            transposed mixing
//   dL(a',w,a)   = sum_{s1,s2,c} H(a',w,s1,s2,c) psi(a,s1,s2,c)         NT GEMM, K-list
//   dpsi         = H_eff psi + sum_{a',w} L(a',w,a) H(a',w,s1,s2,c)      forward + TN GEMM
//   dR(c',w'',c) = sum_{a',s1',s2'} psi(a',s1',s2',c') T2(...)           TN GEMM, K-list
//   dWW(t)       = <G sub-block, T1 sub-block> summed over the blocks sharing coefficient t
//   dW1(e1) = sum dWW(t) W2(e2), dW2(e2) = sum dWW(t) W1(e1) over the pairs of t.
// The W gradient covers every element of the W blocks present in the plan
// (blocks that are entirely zero are absent and get 0).  Every sum runs in a
// fixed order: results are bitwise reproducible.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <tuple>

#include "bsdmrg_internal.h"
#include "kernels.h"

namespace bsd {

constexpr int kItemB = 4096;

// FP64 product that hands back its intermediates (abi.cpp); the product's
// workspace sits at the start of ws.
void heff_forward_f64(const bsdmrg_plan_s* P, const double* L, const double* W1, const double* W2, const double* R,
                      const double* psi, double* out, void* ws, hipStream_t s, double** T1, double** T2,
                      double** coef);
int64_t heff_apply_bytes(const bsdmrg_plan_s* P);

struct Backward {
  Stage b1, dl, hpsi, dr;
  std::vector<MixTask> h_tasks;      // transposed mixing G -> H
  std::vector<MixTerm> h_terms;
  std::vector<MixItem> h_items;
  std::vector<BwdDot> dots;          // dWW partial dots, grouped by key
  std::vector<int32_t> dot_ptr;      // CSR: key -> dots
  int64_t n_keys = 0;
  std::vector<int32_t> w1_ptr, w2_ptr, w1_coef, w2_coef;   // CSR over W elements
  std::vector<int64_t> w1_part, w2_part;
  std::vector<int64_t> base;         // per operand (psi, L, R, W1, W2): problem bases + total
  void* d_blob = nullptr;
  int64_t* d_base = nullptr;
  BwdDot* d_dots = nullptr;
  int32_t* d_dot_ptr = nullptr;
  MixTask* d_h_tasks = nullptr;
  MixTerm* d_h_terms = nullptr;
  MixItem* d_h_items = nullptr;
  int32_t *d_w1_ptr = nullptr, *d_w2_ptr = nullptr, *d_w1_coef = nullptr, *d_w2_coef = nullptr;
  int64_t *d_w1_part = nullptr, *d_w2_part = nullptr;
};

void destroy_backward(bsdmrg_plan_s* P) {
  if (!P->bwd) return;
  if (P->bwd->d_blob) (void)hipFree(P->bwd->d_blob);
  delete P->bwd;
  P->bwd = nullptr;
}

static Key kk3(int a, int b, int c) { Key k{}; k[0] = a; k[1] = b; k[2] = c; return k; }
static Key kk4(int a, int b, int c, int d) { Key k{}; k[0] = a; k[1] = b; k[2] = c; k[3] = d; return k; }
static Charge add2(const Charge& a, const Charge& b) { return {a[0] + b[0], a[1] + b[1]}; }

#define HIPCHK(x)                                                                              \
  do {                                                                                         \
    hipError_t e_ = (x);                                                                       \
    if (e_ != hipSuccess) throw Error{BSDMRG_EHIP, std::string(#x) + ": " + hipGetErrorString(e_)}; \
  } while (0)

static size_t al(size_t b) { return (b + 255) / 256 * 256; }

static void build_backward(bsdmrg_plan_s* P) {
  auto* B = new Backward();
  try {
    // --- transposed mixing: invert the forward term lists ---------------------
    // H has the layout of T1; every T1 channel sub-matrix is one H task.
    std::map<int64_t, std::vector<std::pair<MixTerm, int>>> by_src;   // T1 sub offset -> (G term, rows)
    for (const MixTask& t : P->mix_tasks)
      for (int j = 0; j < t.nterm; ++j) {
        const MixTerm& m = P->mix_terms[t.term0 + j];
        by_src[m.src_off].push_back({MixTerm{t.dst_off, t.ld_dst, m.coef}, t.rows});
      }
    for (const ProblemPlan& p : P->probs)
      for (const T1Block& b : p.t1) {
        const int64_t nf = p.wl.d[b.f], bc = p.c.d[b.c], ba = p.a.d[b.ap];
        for (int iw = 0; iw < nf; ++iw) {
          const int64_t off = b.off + iw * bc;
          MixTask mt{off, (int32_t)(nf * bc), (int32_t)ba, (int32_t)bc, (int32_t)B->h_terms.size(), 0, 0};
          auto it = by_src.find(off);
          if (it != by_src.end())
            for (auto& tr : it->second) B->h_terms.push_back(tr.first);
          mt.nterm = (int32_t)B->h_terms.size() - mt.term0;
          const int task = (int)B->h_tasks.size();
          B->h_tasks.push_back(mt);
          const int rows_per = std::max<int64_t>(1, kItemB / bc);
          for (int r0 = 0; r0 < ba; r0 += rows_per)
            B->h_items.push_back(MixItem{task, r0, (int32_t)std::min<int64_t>(rows_per, ba - r0), 0});
        }
      }
    // --- GEMM stages ----------------------------------------------------------
    for (const ProblemPlan& p : P->probs) {
      std::map<Key, int64_t> t1, t2;   // (a', f, s1, s2, c) / (a', s1', s2', g) -> offset
      std::map<Key, int> t2c;
      for (const T1Block& b : p.t1) {
        Key k{};
        k[0] = b.ap; k[1] = b.f; k[2] = b.s1; k[3] = b.s2; k[4] = b.c;
        t1[k] = b.off;
      }
      for (const T2Block& b : p.t2) {
        t2[kk4(b.ap, b.s1p, b.s2p, b.g)] = b.off;
        t2c[kk4(b.ap, b.s1p, b.s2p, b.g)] = b.c;
      }
      // B1: G block = psi(a',s1',s2',c') R(c',g,c)
      for (const T2Block& b : p.t2) {
        const Charge qcp = add2(add2(p.a.q[b.ap], p.s1.q[b.s1p]), p.s2.q[b.s2p]);
        const int icp = p.c.find(qcp);
        const int pb = p.psi.lookup(kk4(b.ap, b.s1p, b.s2p, icp));
        const int rb = p.R.lookup(kk3(icp, b.g, b.c));
        if (icp < 0 || pb < 0 || rb < 0) throw Error{BSDMRG_EQN, "backward: G operands missing"};
        const int32_t M = (int32_t)p.a.d[b.ap], N = (int32_t)(p.wr.d[b.g] * p.c.d[b.c]), K = (int32_t)p.c.d[icp];
        B->b1.segs.push_back(GemmSeg{p.psi_base + p.psi.offs[pb], p.R_base + p.R.offs[rb], K, N, K, 0});
        B->b1.tasks.push_back(GemmTask{b.off, N, M, N, (int32_t)B->b1.segs.size() - 1, 1, K, 0, 0});
      }
      // dL block (a', f, a): sum over (s1, s2, c) of H block x psi block^T
      for (size_t lb = 0; lb < p.L.keys.size(); ++lb) {
        const int iap = p.L.keys[lb][0], f = p.L.keys[lb][1], ia = p.L.keys[lb][2];
        const int32_t M = (int32_t)(p.a.d[iap] * p.wl.d[f]), N = (int32_t)p.a.d[ia];
        GemmTask t{p.L_base + p.L.offs[lb], N, M, N, (int32_t)B->dl.segs.size(), 0, 0, 0, 0};
        for (size_t pb = 0; pb < p.psi.keys.size(); ++pb) {
          const Key& k = p.psi.keys[pb];
          if (k[0] != ia) continue;
          Key k1{};
          k1[0] = iap; k1[1] = f; k1[2] = k[1]; k1[3] = k[2]; k1[4] = k[3];
          auto it = t1.find(k1);
          if (it == t1.end()) continue;
          const int32_t K = (int32_t)p.c.d[k[3]];
          B->dl.segs.push_back(GemmSeg{it->second, p.psi_base + p.psi.offs[pb], K, K, K, 0});
          t.nseg++;
          t.ksum += K;
        }
        B->dl.tasks.push_back(t);
      }
      // H^T psi block (a, s1, s2, c): sum over f of L block^T x H block
      for (size_t pb = 0; pb < p.psi.keys.size(); ++pb) {
        const Key& k = p.psi.keys[pb];
        const int ia = k[0], ic = k[3];
        const int32_t M = (int32_t)p.a.d[ia], N = (int32_t)p.c.d[ic];
        GemmTask t{p.psi_base + p.psi.offs[pb], N, M, N, (int32_t)B->hpsi.segs.size(), 0, 0, 0, 0};
        for (int f = 0; f < p.wl.size(); ++f) {
          const int iap = p.a.find(add2(p.a.q[ia], p.wl.q[f]));
          if (iap < 0) continue;
          Key k1{};
          k1[0] = iap; k1[1] = f; k1[2] = k[1]; k1[3] = k[2]; k1[4] = ic;
          auto it = t1.find(k1);
          const int lb = p.L.lookup(kk3(iap, f, ia));
          if (it == t1.end() || lb < 0) continue;
          const int32_t K = (int32_t)(p.a.d[iap] * p.wl.d[f]);
          B->hpsi.segs.push_back(GemmSeg{p.L_base + p.L.offs[lb], it->second, M, N, K, 0});
          t.nseg++;
          t.ksum += K;
        }
        B->hpsi.tasks.push_back(t);
      }
      // dR block (c', g, c): sum over (a', s1', s2') of psi block^T x T2 block
      for (size_t rb = 0; rb < p.R.keys.size(); ++rb) {
        const int icp = p.R.keys[rb][0], g = p.R.keys[rb][1], ic = p.R.keys[rb][2];
        const int32_t M = (int32_t)p.c.d[icp], N = (int32_t)(p.wr.d[g] * p.c.d[ic]);
        GemmTask t{p.R_base + p.R.offs[rb], N, M, N, (int32_t)B->dr.segs.size(), 0, 0, 0, 0};
        for (size_t pb = 0; pb < p.psi.keys.size(); ++pb) {
          const Key& k = p.psi.keys[pb];
          if (k[3] != icp) continue;
          auto it = t2.find(kk4(k[0], k[1], k[2], g));
          if (it == t2.end() || t2c[kk4(k[0], k[1], k[2], g)] != ic) continue;
          const int32_t K = (int32_t)p.a.d[k[0]];
          B->dr.segs.push_back(GemmSeg{p.psi_base + p.psi.offs[pb], it->second, M, N, K, 0});
          t.nseg++;
          t.ksum += K;
        }
        B->dr.tasks.push_back(t);
      }
      // --- dWW keys over every element of the present W blocks ----------------
      struct WKey {
        int f, iw, s1p, s1, s2p, s2, g, iwpp;
        bool operator<(const WKey& o) const {
          return std::tie(f, iw, s1p, s1, s2p, s2, g, iwpp) < std::tie(o.f, o.iw, o.s1p, o.s1, o.s2p, o.s2, o.g, o.iwpp);
        }
      };
      std::map<WKey, std::vector<std::pair<int64_t, int64_t>>> keys;
      for (size_t b1 = 0; b1 < p.W1.keys.size(); ++b1) {
        if (!p.nz1[b1]) continue;
        const int f = p.W1.keys[b1][0], s1p = p.W1.keys[b1][1], s1 = p.W1.keys[b1][2], m = p.W1.keys[b1][3];
        for (size_t b2 = 0; b2 < p.W2.keys.size(); ++b2) {
          if (!p.nz2[b2] || p.W2.keys[b2][0] != m) continue;
          const int s2p = p.W2.keys[b2][1], s2 = p.W2.keys[b2][2], g = p.W2.keys[b2][3];
          const int64_t nf = p.wl.d[f], nm = p.wm.d[m], ng = p.wr.d[g];
          for (int iw = 0; iw < nf; ++iw)
            for (int iwpp = 0; iwpp < ng; ++iwpp) {
              auto& v = keys[WKey{f, iw, s1p, s1, s2p, s2, g, iwpp}];
              for (int im = 0; im < nm; ++im)
                v.push_back({p.W1.offs[b1] + iw * nm + im, p.W2.offs[b2] + im * ng + iwpp});
            }
        }
      }
      std::vector<std::vector<std::pair<int32_t, int64_t>>> w1rows(p.W1.elems()), w2rows(p.W2.elems());
      for (auto& kv : keys) {
        const WKey& k = kv.first;
        const int32_t kid = (int32_t)B->n_keys++;
        B->dot_ptr.push_back((int32_t)B->dots.size());
        for (int iap = 0; iap < p.a.size(); ++iap) {
          auto i2 = t2.find(kk4(iap, k.s1p, k.s2p, k.g));
          if (i2 == t2.end()) continue;
          const int ic = t2c[i2->first];
          Key k1{};
          k1[0] = iap; k1[1] = k.f; k1[2] = k.s1; k1[3] = k.s2; k1[4] = ic;
          auto i1 = t1.find(k1);
          if (i1 == t1.end()) continue;
          const int64_t ba = p.a.d[iap], bc = p.c.d[ic];
          const int rows_per = std::max<int64_t>(1, kItemB / bc);
          for (int r0 = 0; r0 < ba; r0 += rows_per)
            B->dots.push_back(BwdDot{i2->second + k.iwpp * bc, i1->second + k.iw * bc,
                                     (int32_t)(p.wr.d[k.g] * bc), (int32_t)(p.wl.d[k.f] * bc), (int32_t)bc,
                                     r0, (int32_t)std::min<int64_t>(rows_per, ba - r0), 0});
        }
        for (auto& pr : kv.second) {
          w1rows[pr.first].push_back({kid, p.W2_base + pr.second});
          w2rows[pr.second].push_back({kid, p.W1_base + pr.first});
        }
      }
      // CSR rows over the whole W buffers of this problem (batches concatenate)
      auto emit = [](std::vector<std::vector<std::pair<int32_t, int64_t>>>& rows, std::vector<int32_t>& ptr,
                     std::vector<int32_t>& coef, std::vector<int64_t>& part) {
        for (auto& r : rows) {
          if (ptr.empty()) ptr.push_back(0);
          for (auto& e : r) {
            coef.push_back(e.first);
            part.push_back(e.second);
          }
          ptr.push_back((int32_t)coef.size());
        }
      };
      emit(w1rows, B->w1_ptr, B->w1_coef, B->w1_part);
      emit(w2rows, B->w2_ptr, B->w2_coef, B->w2_part);
    }
    B->dot_ptr.push_back((int32_t)B->dots.size());
    for (int op = 0; op < 5; ++op) {
      for (const ProblemPlan& p : P->probs)
        B->base.push_back(op == 0 ? p.psi_base : op == 1 ? p.L_base : op == 2 ? p.R_base : op == 3 ? p.W1_base
                                                                                                    : p.W2_base);
      B->base.push_back(op == 0 ? P->psi_elems : op == 1 ? P->L_elems : op == 2 ? P->R_elems : op == 3 ? P->W1_elems
                                                                                                       : P->W2_elems);
    }
    if (B->w1_ptr.empty()) B->w1_ptr.push_back(0);
    if (B->w2_ptr.empty()) B->w2_ptr.push_back(0);
    schedule_tiles(B->b1);
    schedule_tiles(B->dl);
    schedule_tiles(B->hpsi);
    schedule_tiles(B->dr);
    // host checks of every table
    validate_gemm(B->b1, kNN, P->psi_elems, P->R_elems, P->t2_elems, 0, "backward G");
    validate_gemm(B->dl, kNT, P->t1_elems, P->psi_elems, P->L_elems, 0, "backward dL");
    validate_gemm(B->hpsi, kTN, P->L_elems, P->t1_elems, P->psi_elems, 0, "backward H^T psi");
    validate_gemm(B->dr, kTN, P->psi_elems, P->t2_elems, P->R_elems, 0, "backward dR");
    validate_mix(B->h_tasks, B->h_terms, B->h_items, P->t2_elems, P->t1_elems, P->n_coefs, "backward mixing");
    for (const BwdDot& d : B->dots)
      if (d.g_off < 0 || d.t_off < 0 || d.g_off + (int64_t)(d.row0 + d.nrows - 1) * d.ld_g + d.cols > P->t2_elems ||
          d.t_off + (int64_t)(d.row0 + d.nrows - 1) * d.ld_t + d.cols > P->t1_elems)
        throw Error{BSDMRG_EINVAL, "internal table check failed: backward dots"};
    if ((int64_t)B->w1_ptr.size() != P->W1_elems + 1 || (int64_t)B->w2_ptr.size() != P->W2_elems + 1)
      throw Error{BSDMRG_EINVAL, "internal table check failed: backward W rows"};
    auto check_csr = [&](const std::vector<int32_t>& ptr, const std::vector<int32_t>& coef,
                         const std::vector<int64_t>& part, int64_t other) {
      if (ptr.front() != 0 || ptr.back() != (int32_t)coef.size() || coef.size() != part.size())
        throw Error{BSDMRG_EINVAL, "internal table check failed: backward W CSR"};
      for (size_t i = 1; i < ptr.size(); ++i)
        if (ptr[i] < ptr[i - 1]) throw Error{BSDMRG_EINVAL, "internal table check failed: backward W CSR order"};
      for (size_t j = 0; j < coef.size(); ++j)
        if (coef[j] < 0 || coef[j] >= B->n_keys || part[j] < 0 || part[j] >= other)
          throw Error{BSDMRG_EINVAL, "internal table check failed: backward W entries"};
    };
    check_csr(B->w1_ptr, B->w1_coef, B->w1_part, P->W2_elems);
    check_csr(B->w2_ptr, B->w2_coef, B->w2_part, P->W1_elems);
    if ((int64_t)B->dot_ptr.size() != B->n_keys + 1 || B->dot_ptr.front() != 0 ||
        B->dot_ptr.back() != (int32_t)B->dots.size())
      throw Error{BSDMRG_EINVAL, "internal table check failed: backward dot keys"};
    for (size_t i = 1; i < B->dot_ptr.size(); ++i)
      if (B->dot_ptr[i] < B->dot_ptr[i - 1]) throw Error{BSDMRG_EINVAL, "internal table check failed: dot order"};
    for (const BwdDot& d : B->dots)
      if (d.nrows < 1 || d.cols < 1 || d.nrows * d.cols > kItemB * 2 || d.cols > d.ld_g || d.cols > d.ld_t)
        throw Error{BSDMRG_EINVAL, "internal table check failed: backward dot shape"};
    for (int op = 0; op < 5; ++op)
      for (size_t p = 0; p < P->probs.size(); ++p)
        if (B->base[op * (P->probs.size() + 1) + p] > B->base[op * (P->probs.size() + 1) + p + 1])
          throw Error{BSDMRG_EINVAL, "internal table check failed: backward problem bases"};
    for (const MixItem& it : B->h_items)
      if (it.nrows * B->h_tasks[it.task].cols > kItemB)
        throw Error{BSDMRG_EINVAL, "internal table check failed: backward mixing item size"};
  } catch (...) {
    delete B;
    throw;
  }
  P->bwd = B;
}

static void upload_backward(Backward* B) {
  try {
    struct Part { const void* src; size_t bytes; void** dst; };
    std::vector<Part> parts = {
        {B->b1.tasks.data(), B->b1.tasks.size() * sizeof(GemmTask), (void**)&B->b1.d_tasks},
        {B->b1.segs.data(), B->b1.segs.size() * sizeof(GemmSeg), (void**)&B->b1.d_segs},
        {B->b1.tiles.data(), B->b1.tiles.size() * sizeof(GemmTile), (void**)&B->b1.d_tiles},
        {B->dl.tasks.data(), B->dl.tasks.size() * sizeof(GemmTask), (void**)&B->dl.d_tasks},
        {B->dl.segs.data(), B->dl.segs.size() * sizeof(GemmSeg), (void**)&B->dl.d_segs},
        {B->dl.tiles.data(), B->dl.tiles.size() * sizeof(GemmTile), (void**)&B->dl.d_tiles},
        {B->hpsi.tasks.data(), B->hpsi.tasks.size() * sizeof(GemmTask), (void**)&B->hpsi.d_tasks},
        {B->hpsi.segs.data(), B->hpsi.segs.size() * sizeof(GemmSeg), (void**)&B->hpsi.d_segs},
        {B->hpsi.tiles.data(), B->hpsi.tiles.size() * sizeof(GemmTile), (void**)&B->hpsi.d_tiles},
        {B->dr.tasks.data(), B->dr.tasks.size() * sizeof(GemmTask), (void**)&B->dr.d_tasks},
        {B->dr.segs.data(), B->dr.segs.size() * sizeof(GemmSeg), (void**)&B->dr.d_segs},
        {B->dr.tiles.data(), B->dr.tiles.size() * sizeof(GemmTile), (void**)&B->dr.d_tiles},
        {B->h_tasks.data(), B->h_tasks.size() * sizeof(MixTask), (void**)&B->d_h_tasks},
        {B->h_terms.data(), B->h_terms.size() * sizeof(MixTerm), (void**)&B->d_h_terms},
        {B->h_items.data(), B->h_items.size() * sizeof(MixItem), (void**)&B->d_h_items},
        {B->dots.data(), B->dots.size() * sizeof(BwdDot), (void**)&B->d_dots},
        {B->dot_ptr.data(), B->dot_ptr.size() * sizeof(int32_t), (void**)&B->d_dot_ptr},
        {B->w1_ptr.data(), B->w1_ptr.size() * sizeof(int32_t), (void**)&B->d_w1_ptr},
        {B->w1_coef.data(), B->w1_coef.size() * sizeof(int32_t), (void**)&B->d_w1_coef},
        {B->w1_part.data(), B->w1_part.size() * sizeof(int64_t), (void**)&B->d_w1_part},
        {B->w2_ptr.data(), B->w2_ptr.size() * sizeof(int32_t), (void**)&B->d_w2_ptr},
        {B->w2_coef.data(), B->w2_coef.size() * sizeof(int32_t), (void**)&B->d_w2_coef},
        {B->w2_part.data(), B->w2_part.size() * sizeof(int64_t), (void**)&B->d_w2_part},
        {B->base.data(), B->base.size() * sizeof(int64_t), (void**)&B->d_base},
    };
    size_t total = 0;
    for (auto& q : parts) total += al(std::max<size_t>(q.bytes, 1));
    HIPCHK(hipMalloc(&B->d_blob, total));
    std::vector<char> host(total, 0);
    size_t off = 0;
    for (auto& q : parts) {
      if (q.bytes) std::memcpy(host.data() + off, q.src, q.bytes);
      *q.dst = (char*)B->d_blob + off;
      off += al(std::max<size_t>(q.bytes, 1));
    }
    HIPCHK(hipMemcpy(B->d_blob, host.data(), total, hipMemcpyHostToDevice));
  } catch (...) {
    if (B->d_blob) (void)hipFree(B->d_blob);
    B->d_blob = nullptr;
    throw;
  }
}

// Workspace of the adjoint (and of the energy evaluation), in carve order:
// the product's own workspace, G, H, H^T psi, H_eff psi, dot partials, dWW,
// per-problem scale factors, energy partials, per-problem energies.
struct BwdWS {
  double *G, *H, *hpsi, *fwd, *part, *dcoef, *g, *epart, *ered;
  int64_t bytes;
};

static BwdWS carve_bwd(const bsdmrg_plan_s* P, const Backward* B, void* ws) {
  BwdWS w{};
  const int64_t apply = heff_apply_bytes(P);
  char* base = (char*)ws;
  size_t off = (size_t)apply;
  auto take = [&](size_t n) {
    double* r = base ? (double*)(base + off) : nullptr;
    off += al(std::max<size_t>(n, 1) * 8);
    return r;
  };
  const size_t np = P->probs.size();
  w.G = take(P->t2_elems);
  w.H = take(P->t1_elems);
  w.hpsi = take(P->psi_elems);
  w.fwd = take(P->psi_elems);
  w.part = take(B->dots.size());
  w.dcoef = take(B->n_keys);
  w.g = take(np);
  w.epart = take(P->chunks.size());
  w.ered = take(np);
  w.bytes = (int64_t)off;
  return w;
}

// The adjoint tables are built on first use; the plan's mutex makes the
// build and upload happen once when several threads share the plan.
static void ensure_tables(bsdmrg_plan_s* P) {
  std::lock_guard<std::mutex> lk(P->mu);
  if (!P->bwd) build_backward(P);
  if (!P->bwd->d_blob) upload_backward(P->bwd);
}

void heff_backward_run(bsdmrg_plan_s* P, const double* L, const double* W1, const double* W2, const double* R,
                       const double* psi, const double* g_host, double* d_psi, double* d_L, double* d_W1,
                       double* d_W2, double* d_R, void* ws, int64_t ws_bytes, hipStream_t s) {
  ensure_tables(P);
  const Backward* B = P->bwd;
  const BwdWS need = carve_bwd(P, B, nullptr);
  if (!ws || ws_bytes < need.bytes)
    throw Error{BSDMRG_EINVAL, "heff_backward: workspace too small: need " + std::to_string(need.bytes) + " bytes"};
  const BwdWS w = carve_bwd(P, B, ws);
  const int np = (int)P->probs.size();
  HIPCHK(hipMemcpyAsync(w.g, g_host, np * sizeof(double), hipMemcpyHostToDevice, s));
  double *T1 = nullptr, *T2 = nullptr, *coef = nullptr;
  // forward: coefficients, T1, T2 and H_eff psi
  HIPCHK(dav_fill_zero(w.fwd, P->psi_elems, s));
  heff_forward_f64(P, L, W1, W2, R, psi, w.fwd, ws, s, &T1, &T2, &coef);
  // G = psi R and H = mix^T(G)
  HIPCHK(launch_gemm_f64(B->b1, kNN, psi, R, w.G, w.G, s));
  HIPCHK(launch_mix_tables(B->d_h_items, B->h_items.size(), B->d_h_tasks, B->d_h_terms, coef, w.G, w.H, s));
  if (d_psi) {
    HIPCHK(dav_fill_zero(w.hpsi, P->psi_elems, s));
    HIPCHK(launch_gemm_f64(B->hpsi, kTN, L, w.H, w.hpsi, w.hpsi, s));
    HIPCHK(launch_seg_scale(P->psi_elems, B->d_base + 0 * (np + 1), np, w.g, w.fwd, w.hpsi, d_psi, s));
  }
  if (d_L) {
    HIPCHK(dav_fill_zero(d_L, P->L_elems, s));
    HIPCHK(launch_gemm_f64(B->dl, kNT, w.H, psi, d_L, d_L, s));
    HIPCHK(launch_seg_scale(P->L_elems, B->d_base + 1 * (np + 1), np, w.g, d_L, nullptr, d_L, s));
  }
  if (d_R) {
    HIPCHK(dav_fill_zero(d_R, P->R_elems, s));
    HIPCHK(launch_gemm_f64(B->dr, kTN, psi, T2, d_R, d_R, s));
    HIPCHK(launch_seg_scale(P->R_elems, B->d_base + 2 * (np + 1), np, w.g, d_R, nullptr, d_R, s));
  }
  if (d_W1 || d_W2) {
    HIPCHK(launch_bwd_dots(B->d_dots, (int)B->dots.size(), w.G, T1, w.part, s));
    HIPCHK(launch_bwd_coef((int)B->n_keys, B->d_dot_ptr, w.part, nullptr, w.dcoef, s));
    if (d_W1) {
      HIPCHK(launch_bwd_wgrad(P->W1_elems, B->d_w1_ptr, B->d_w1_coef, B->d_w1_part, w.dcoef, W2, 1.0, d_W1, s));
      HIPCHK(launch_seg_scale(P->W1_elems, B->d_base + 3 * (np + 1), np, w.g, d_W1, nullptr, d_W1, s));
    }
    if (d_W2) {
      HIPCHK(launch_bwd_wgrad(P->W2_elems, B->d_w2_ptr, B->d_w2_coef, B->d_w2_part, w.dcoef, W1, 1.0, d_W2, s));
      HIPCHK(launch_seg_scale(P->W2_elems, B->d_base + 4 * (np + 1), np, w.g, d_W2, nullptr, d_W2, s));
    }
  }
  // g_host may be released once the call returns: finish the upload first
  HIPCHK(hipStreamSynchronize(s));
}

void heff_energy_run(bsdmrg_plan_s* P, const double* L, const double* W1, const double* W2, const double* R,
                     const double* psi, double* energy, void* ws, int64_t ws_bytes, hipStream_t s) {
  ensure_tables(P);
  const Backward* B = P->bwd;
  const BwdWS need = carve_bwd(P, B, nullptr);
  if (!ws || ws_bytes < need.bytes)
    throw Error{BSDMRG_EINVAL, "heff_energy: workspace too small: need " + std::to_string(need.bytes) + " bytes"};
  const BwdWS w = carve_bwd(P, B, ws);
  double *T1 = nullptr, *T2 = nullptr, *coef = nullptr;
  HIPCHK(dav_fill_zero(w.fwd, P->psi_elems, s));
  heff_forward_f64(P, L, W1, W2, R, psi, w.fwd, ws, s, &T1, &T2, &coef);
  HIPCHK(dav_dots(P, 1, psi, 0, w.fwd, w.epart, s));
  HIPCHK(dav_psum(P, 1, w.epart, w.ered, 1, s));
  HIPCHK(hipMemcpyAsync(energy, w.ered, P->probs.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
}

int64_t heff_backward_bytes(bsdmrg_plan_s* P) {
  std::lock_guard<std::mutex> lk(P->mu);
  if (!P->bwd) build_backward(P);
  return carve_bwd(P, P->bwd, nullptr).bytes;
}

}  // namespace bsd
