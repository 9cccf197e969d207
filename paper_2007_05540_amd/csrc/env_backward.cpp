// Adjoint of the environment extension with respect to the MPO tensor.
// The extension is linear in W, so for an output cotangent D:
//   left  (E = L, site A(x,s,y)):
//     dW(w,s',s,g) = sum A(x',s',y') L(x',w,x) A(x,s,y) D(y',g,y)
//                  = sum_{x',y} X1(x',w,s,y) Y(x',s',g,y),
//     X1 = L A (stage 1 of the extension), Y(x',s',g,y) = sum_y' A(x',s',y') D(y',g,y)  (NN GEMM)
//   right (E = R, site B(y,s,x)):
//     dW(g,s',s,w) = sum B(y',s',x') R(x',w,x) B(y,s,x) D(y',g,y)
//                  = sum_{x',y} Z1(x',w,s,y) Y(x',s',g,y),
//     Z1 = R B^T (stage 1 of the extension), Y(x',s',g,y) = sum_y' B(y',s',x') D(y',g,y)  (TN GEMM)
// Each W element is one sum of block dots over (x', y) blocks, in a fixed
// order.  The cotangent of the environment itself is the extension of the
// opposite side applied to D with the same site tensor (the same contraction
// read from the other end), so it needs no tables of its own.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>

#include "bsdmrg_internal.h"
#include "kernels.h"

namespace bsd {

namespace {
const int32_t kMpsS[3] = {1, 1, -1};
const int32_t kEnvS[3] = {-1, 1, 1};
const int32_t kWS[4] = {1, 1, -1, -1};
constexpr int kItemE = 4096;

Charge cadd(const Charge& a, const Charge& b) { return {a[0] + b[0], a[1] + b[1]}; }
Charge csub(const Charge& a, const Charge& b) { return {a[0] - b[0], a[1] - b[1]}; }
Key k3(int a, int b, int c) { Key k{}; k[0] = a; k[1] = b; k[2] = c; return k; }
Key k4(int a, int b, int c, int d) { Key k{}; k[0] = a; k[1] = b; k[2] = c; k[3] = d; return k; }
size_t al(size_t b) { return (b + 255) / 256 * 256; }
}  // namespace

#define HIPCHK(x)                                                                              \
  do {                                                                                         \
    hipError_t e_ = (x);                                                                       \
    if (e_ != hipSuccess) throw Error{BSDMRG_EHIP, std::string(#x) + ": " + hipGetErrorString(e_)}; \
  } while (0)

struct EnvBackward {
  Stage y;
  int layout_y = kNN;
  int64_t y_elems = 0, w_elems = 0;
  std::vector<BwdDot> dots;
  std::vector<int32_t> dot_ptr;     // key -> dots (keys = W elements of the allowed blocks)
  std::vector<int64_t> key_elem;    // key -> W element
  void* d_blob = nullptr;
  BwdDot* d_dots = nullptr;
  int32_t* d_dot_ptr = nullptr;
  int64_t* d_key_elem = nullptr;
};

void destroy_env_backward(bsdmrg_op_s* O) {
  if (!O->ebwd) return;
  if (O->ebwd->d_blob) (void)hipFree(O->ebwd->d_blob);
  delete O->ebwd;
  O->ebwd = nullptr;
}

static void build_env_backward(bsdmrg_op_s* O) {
  if (O->kind != 1 && O->kind != 2) throw Error{BSDMRG_EINVAL, "env_backward: not an environment op"};
  auto* B = new EnvBackward();
  try {
    const Leg &x = O->legs[0], &s = O->legs[1], &y = O->legs[2], &wl = O->legs[3], &wr = O->legs[4];
    const int side = O->side;
    const Leg& wi = side == 0 ? wl : wr;
    const Leg& wo = side == 0 ? wr : wl;
    Layout W = make_layout({&wl, &s, &s, &wr}, kWS);
    Layout M = side == 0 ? make_layout({&x, &s, &y}, kMpsS) : make_layout({&y, &s, &x}, kMpsS);
    Layout Eo = make_layout({&y, &wo, &y}, kEnvS);
    B->w_elems = W.elems();
    B->layout_y = side == 0 ? kNN : kTN;
    // Y blocks (x', s', g, y): one GEMM task each (the K-list has one segment)
    std::map<Key, int64_t> yb;
    int64_t cur = 0;
    for (int xp = 0; xp < x.size(); ++xp)
      for (int sp = 0; sp < s.size(); ++sp) {
        const Charge qyp = side == 0 ? cadd(x.q[xp], s.q[sp]) : csub(x.q[xp], s.q[sp]);
        const int iyp = y.find(qyp);
        if (iyp < 0) continue;
        const int mb = side == 0 ? M.lookup(k3(xp, sp, iyp)) : M.lookup(k3(iyp, sp, xp));
        if (mb < 0) continue;
        for (int g = 0; g < wo.size(); ++g) {
          const int ib = y.find(csub(qyp, wo.q[g]));
          if (ib < 0) continue;
          const int ob = Eo.lookup(k3(iyp, g, ib));
          if (ob < 0) continue;
          const int32_t Mr = (int32_t)x.d[xp], N = (int32_t)(wo.d[g] * y.d[ib]), K = (int32_t)y.d[iyp];
          B->y.segs.push_back(GemmSeg{M.offs[mb], Eo.offs[ob], side == 0 ? K : Mr, N, K, 0});
          B->y.tasks.push_back(GemmTask{cur, N, Mr, N, (int32_t)B->y.segs.size() - 1, 1, K, 0, 0});
          B->y.flops += 2.0 * Mr * N * (double)K;
          yb[k4(xp, sp, g, ib)] = cur;
          cur += round_up((int64_t)Mr * N);
        }
      }
    B->y_elems = cur;
    schedule_tiles(B->y);
    // stage-1 blocks grouped by (input channel sector, s)
    std::map<std::pair<int, int>, std::vector<X1Block>> by_fs;
    for (const X1Block& b : O->x1_blocks) by_fs[{b.f, b.is}].push_back(b);
    // one key per W element of every allowed block
    for (size_t wb = 0; wb < W.keys.size(); ++wb) {
      const int l = W.keys[wb][0], sp = W.keys[wb][1], is = W.keys[wb][2], r = W.keys[wb][3];
      const int f = side == 0 ? l : r, g = side == 0 ? r : l;
      const int64_t nl = wl.d[l], nr = wr.d[r], nf = wi.d[f], ng = wo.d[g];
      auto grp = by_fs.find({f, is});
      for (int64_t il = 0; il < nl; ++il)
        for (int64_t ir = 0; ir < nr; ++ir) {
          const int64_t iw = side == 0 ? il : ir, ig = side == 0 ? ir : il;
          B->dot_ptr.push_back((int32_t)B->dots.size());
          B->key_elem.push_back(W.offs[wb] + il * nr + ir);
          if (grp == by_fs.end()) continue;
          for (const X1Block& xb : grp->second) {
            auto it = yb.find(k4(xb.xp, sp, g, xb.ib));
            if (it == yb.end()) continue;
            const int64_t bx = x.d[xb.xp], bb = y.d[xb.ib];
            const int rows_per = (int)std::max<int64_t>(1, kItemE / bb);
            for (int r0 = 0; r0 < bx; r0 += rows_per)
              B->dots.push_back(BwdDot{it->second + ig * bb, xb.off + iw * bb, (int32_t)(ng * bb), (int32_t)(nf * bb),
                                       (int32_t)bb, r0, (int32_t)std::min<int64_t>(rows_per, bx - r0), 0});
          }
        }
    }
    B->dot_ptr.push_back((int32_t)B->dots.size());
    // host checks of every table
    validate_gemm(B->y, B->layout_y, M.elems(), Eo.elems(), B->y_elems, 0, "env adjoint Y");
    for (const BwdDot& d : B->dots)
      if (d.g_off < 0 || d.t_off < 0 || d.nrows < 1 || d.cols < 1 || d.cols > d.ld_g || d.cols > d.ld_t ||
          d.g_off + (int64_t)(d.row0 + d.nrows - 1) * d.ld_g + d.cols > B->y_elems ||
          d.t_off + (int64_t)(d.row0 + d.nrows - 1) * d.ld_t + d.cols > O->x1_elems)
        throw Error{BSDMRG_EINVAL, "internal table check failed: env adjoint dots"};
    for (size_t i = 1; i < B->dot_ptr.size(); ++i)
      if (B->dot_ptr[i] < B->dot_ptr[i - 1]) throw Error{BSDMRG_EINVAL, "internal table check failed: env keys"};
    for (int64_t e : B->key_elem)
      if (e < 0 || e >= B->w_elems) throw Error{BSDMRG_EINVAL, "internal table check failed: env key element"};
  } catch (...) {
    delete B;
    throw;
  }
  O->ebwd = B;
}

static void upload_env_backward(EnvBackward* B) {
  struct Part { const void* src; size_t bytes; void** dst; };
  std::vector<Part> parts = {
      {B->y.tasks.data(), B->y.tasks.size() * sizeof(GemmTask), (void**)&B->y.d_tasks},
      {B->y.segs.data(), B->y.segs.size() * sizeof(GemmSeg), (void**)&B->y.d_segs},
      {B->y.tiles.data(), B->y.tiles.size() * sizeof(GemmTile), (void**)&B->y.d_tiles},
      {B->dots.data(), B->dots.size() * sizeof(BwdDot), (void**)&B->d_dots},
      {B->dot_ptr.data(), B->dot_ptr.size() * sizeof(int32_t), (void**)&B->d_dot_ptr},
      {B->key_elem.data(), B->key_elem.size() * sizeof(int64_t), (void**)&B->d_key_elem},
  };
  size_t total = 0;
  for (auto& q : parts) total += al(std::max<size_t>(q.bytes, 1));
  HIPCHK(hipMalloc(&B->d_blob, total));
  try {
    std::vector<char> host(total, 0);
    size_t off = 0;
    for (auto& q : parts) {
      if (q.bytes) std::memcpy(host.data() + off, q.src, q.bytes);
      *q.dst = (char*)B->d_blob + off;
      off += al(std::max<size_t>(q.bytes, 1));
    }
    HIPCHK(hipMemcpy(B->d_blob, host.data(), total, hipMemcpyHostToDevice));
  } catch (...) {
    (void)hipFree(B->d_blob);
    B->d_blob = nullptr;
    throw;
  }
}

// The adjoint tables are built (and uploaded) on first use, under the op's
// mutex so that threads sharing the op build them once.
static EnvBackward* ensure_env_tables(bsdmrg_op_s* O, bool upload) {
  std::lock_guard<std::mutex> lk(O->mu);
  if (!O->ebwd) build_env_backward(O);
  if (upload && !O->ebwd->d_blob) upload_env_backward(O->ebwd);
  return O->ebwd;
}

int64_t env_backward_bytes(bsdmrg_op_s* O) {
  const EnvBackward* B = ensure_env_tables(O, false);
  return (int64_t)(al(std::max<int64_t>(O->x1_elems, 1) * 8) + al(std::max<int64_t>(B->y_elems, 1) * 8) +
                   al(std::max<size_t>(B->dots.size(), 1) * 8));
}

void env_backward_run(bsdmrg_op_s* O, const double* env, const double* site, const double* d_out, double* d_W,
                      void* ws, int64_t ws_bytes, hipStream_t s) {
  if (!O->d_blob) throw Error{BSDMRG_EINVAL, "env_backward: op was built host-only"};
  const int64_t need = env_backward_bytes(O);
  if (!ws || ws_bytes < need)
    throw Error{BSDMRG_EINVAL, "env_backward: workspace too small: need " + std::to_string(need) + " bytes"};
  EnvBackward* B = ensure_env_tables(O, true);
  double* X1 = (double*)ws;
  double* Y = (double*)((char*)ws + al(std::max<int64_t>(O->x1_elems, 1) * 8));
  double* part = (double*)((char*)Y + al(std::max<int64_t>(B->y_elems, 1) * 8));
  HIPCHK(launch_gemm_f64(O->g1, O->layout1, env, site, X1, X1, s));
  HIPCHK(launch_gemm_f64(B->y, B->layout_y, site, d_out, Y, Y, s));
  HIPCHK(dav_fill_zero(d_W, B->w_elems, s));
  HIPCHK(launch_bwd_dots(B->d_dots, (int)B->dots.size(), Y, X1, part, s));
  HIPCHK(launch_bwd_coef((int)B->key_elem.size(), B->d_dot_ptr, part, B->d_key_elem, d_W, s));
}

}  // namespace bsd
