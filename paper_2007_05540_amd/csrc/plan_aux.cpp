// Planners and executors of the environment extension and the two-site merge
// (Sec. II-C: the environments are extended from centre to centre while
// sweeping; the two-site tensor is the contraction of the two sites over the
// shared bond).  Every block pairing follows Alg. 2: blocks meet on equal
// sector labels of the contracted legs.
//
// Left:  X1(a',w,s,b) = sum_a L(a',w,a) A(a,s,b)                       NN GEMM
//        X2(a',s',w',b) = sum_{w,s} W(w,s',s,w') X1(a',w,s,b)          mixing
//        L'(b',w',b) = sum_{a',s'} A(a',s',b') X2(a',s',w',b)          TN GEMM
// Right: Z1(c',w',s,b) = sum_c R(c',w',c) B(b,s,c)                      NT GEMM
//        Z2(c',s',w,b) = sum_{w',s} W(w,s',s,w') Z1(c',w',s,b)          mixing
//        R'(b',w,b) = sum_{s',c'} B(b',s',c') Z2(c',s',w,b)            NN GEMM
// Merge: theta(a,s1,s2,c) = sum_b A(a,s1,b) B(b,s2,c)                   NN GEMM
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "bsdmrg_internal.h"
#include "kernels.h"

namespace bsd {

static const int32_t kEnvS[3] = {-1, 1, 1};
static const int32_t kMpsS[3] = {1, 1, -1};
static const int32_t kWS[4] = {1, 1, -1, -1};
static const int32_t kPsiS[4] = {1, 1, 1, -1};
constexpr int kTile = 64, kItem = 4096;

static Charge cadd(const Charge& a, const Charge& b) { return {a[0] + b[0], a[1] + b[1]}; }
static Charge csub(const Charge& a, const Charge& b) { return {a[0] - b[0], a[1] - b[1]}; }
static Key k3(int a, int b, int c) { Key k{}; k[0] = a; k[1] = b; k[2] = c; return k; }
static Key k4(int a, int b, int c, int d) { Key k{}; k[0] = a; k[1] = b; k[2] = c; k[3] = d; return k; }

static void add_items(bsdmrg_op_s* O, int task, int rows, int cols) {
  if (cols > kItem) throw Error{BSDMRG_EINVAL, "env: sector dimensions above 4096 are not supported"};
  int rows_per = std::max(1, kItem / std::max(1, cols));
  for (int r0 = 0; r0 < rows; r0 += rows_per)
    O->mix_items.push_back(MixItem{task, r0, std::min(rows_per, rows - r0), 0});
}

static bool w_nonzero(const Layout& L, const double* w, int b) {
  for (int64_t e = L.offs[b]; e < L.offs[b + 1]; ++e)
    if (w[e] != 0.0) return true;
  return false;
}

// side 0: left extension; side 1: right extension.
bsdmrg_op_s* build_env(const bsdmrg_env_problem& in, int side) {
  auto* O = new bsdmrg_op_s();
  try {
    Leg x = leg_from(in.x), s = leg_from(in.s), y = leg_from(in.y), wl = leg_from(in.wl), wr = leg_from(in.wr);
    for (auto d : s.d)
      if (d != 1) throw Error{BSDMRG_EINVAL, "env: physical sectors must have dimension 1"};
    if (!in.w_host) throw Error{BSDMRG_EINVAL, "env: W host array is required"};
    Layout W = make_layout({&wl, &s, &s, &wr}, kWS);
    std::vector<char> nz(W.keys.size());
    for (size_t b = 0; b < nz.size(); ++b) nz[b] = w_nonzero(W, in.w_host, (int)b);
    O->kind = side == 0 ? 1 : 2;
    O->side = side;
    O->legs = {x, s, y, wl, wr};
    const Leg& wi = side == 0 ? wl : wr;   // channel leg of the input environment
    const Leg& wo = side == 0 ? wr : wl;   // channel leg of the output environment
    Layout E = make_layout({&x, &wi, &x}, kEnvS);
    Layout M = side == 0 ? make_layout({&x, &s, &y}, kMpsS) : make_layout({&y, &s, &x}, kMpsS);
    Layout Eo = make_layout({&y, &wo, &y}, kEnvS);
    O->out_elems = Eo.elems();
    // stage 1 ---------------------------------------------------------------
    std::map<Key, int64_t> x1;   // (x', f, s, b) -> offset
    int64_t cur = 0;
    for (size_t eb = 0; eb < E.keys.size(); ++eb) {
      const int xp = E.keys[eb][0], f = E.keys[eb][1], xx = E.keys[eb][2];
      for (int is = 0; is < s.size(); ++is)
        for (int ib = 0; ib < y.size(); ++ib) {
          const int mb = side == 0 ? M.lookup(k3(xx, is, ib)) : M.lookup(k3(ib, is, xx));
          if (mb < 0) continue;
          const int32_t Mr = (int32_t)(x.d[xp] * wi.d[f]), K = (int32_t)x.d[xx], N = (int32_t)y.d[ib];
          GemmSeg g{E.offs[eb], M.offs[mb], K, side == 0 ? N : K, K, 0};
          O->g1.segs.push_back(g);
          O->g1.tasks.push_back(GemmTask{cur, N, Mr, N, (int32_t)O->g1.segs.size() - 1, 1, K, 0, 0});
          O->flops += 2.0 * Mr * N * (double)K;
          x1[k4(xp, f, is, ib)] = cur;
          O->x1_blocks.push_back(X1Block{xp, f, is, ib, cur});
          cur += round_up((int64_t)Mr * N);
        }
    }
    O->x1_elems = cur;
    O->layout1 = side == 0 ? kNN : kNT;
    // stage 2 (mixing with W entries) and stage 3 ----------------------------
    std::map<Key, int64_t> x2;   // (x', s', g, b) -> offset
    cur = 0;
    for (int xp = 0; xp < x.size(); ++xp)
      for (int sp = 0; sp < s.size(); ++sp) {
        // bra bond of the output: left q_b' = q_x' + q_s'; right q_b' = q_x' - q_s'
        const Charge qbp = side == 0 ? cadd(x.q[xp], s.q[sp]) : csub(x.q[xp], s.q[sp]);
        if (y.find(qbp) < 0) continue;
        for (int g = 0; g < wo.size(); ++g) {
          const int ib = y.find(csub(qbp, wo.q[g]));
          if (ib < 0) continue;
          const int64_t bx = x.d[xp], bb = y.d[ib], ng = wo.d[g];
          const int64_t off = cur;
          bool any = false;
          for (int ig = 0; ig < ng; ++ig) {
            MixTask mt{off + ig * bb, (int32_t)(ng * bb), (int32_t)bx, (int32_t)bb,
                       (int32_t)O->mix_terms.size(), 0, 0};
            for (int f = 0; f < wi.size(); ++f)
              for (int is = 0; is < s.size(); ++is) {
                auto it = x1.find(k4(xp, f, is, ib));
                if (it == x1.end()) continue;
                // W block: left (f, s', s, g) ; right (g, s', s, f)
                const int wb = side == 0 ? W.lookup(k4(f, sp, is, g)) : W.lookup(k4(g, sp, is, f));
                if (wb < 0 || !nz[wb]) continue;
                any = true;
                const int64_t nf = wi.d[f];
                for (int iw = 0; iw < nf; ++iw) {
                  const int64_t e = side == 0 ? W.offs[wb] + (int64_t)iw * ng + ig
                                              : W.offs[wb] + (int64_t)ig * nf + iw;
                  if (in.w_host[e] == 0.0) continue;
                  O->mix_terms.push_back(MixTerm{it->second + iw * bb, (int32_t)(nf * bb), (int32_t)e});
                }
              }
            mt.nterm = (int32_t)O->mix_terms.size() - mt.term0;
            O->mix_tasks.push_back(mt);
            add_items(O, (int)O->mix_tasks.size() - 1, (int)bx, (int)bb);
          }
          if (!any) {   // no structural contribution: drop the block again
            O->mix_items.erase(std::remove_if(O->mix_items.begin(), O->mix_items.end(),
                                              [&](const MixItem& m) {
                                                return m.task >= (int)O->mix_tasks.size() - ng;
                                              }),
                               O->mix_items.end());
            O->mix_tasks.resize(O->mix_tasks.size() - ng);
            continue;
          }
          x2[k4(xp, sp, g, ib)] = off;
          cur += round_up(bx * ng * bb);
        }
      }
    O->x2_elems = cur;
    // stage 3: one task per output block, K-list over s'
    for (size_t ob = 0; ob < Eo.keys.size(); ++ob) {
      const int ibp = Eo.keys[ob][0], g = Eo.keys[ob][1], ib = Eo.keys[ob][2];
      const int32_t Mr = (int32_t)y.d[ibp], N = (int32_t)(wo.d[g] * y.d[ib]);
      GemmTask t{Eo.offs[ob], N, Mr, N, (int32_t)O->g2.segs.size(), 0, 0, 0, 0};
      for (int sp = 0; sp < s.size(); ++sp) {
        const Charge qx = side == 0 ? csub(y.q[ibp], s.q[sp]) : cadd(y.q[ibp], s.q[sp]);
        const int xp = x.find(qx);
        if (xp < 0) continue;
        auto it = x2.find(k4(xp, sp, g, ib));
        if (it == x2.end()) continue;
        const int mb = side == 0 ? M.lookup(k3(xp, sp, ibp)) : M.lookup(k3(ibp, sp, xp));
        if (mb < 0) continue;
        const int32_t K = (int32_t)x.d[xp];
        // left: A-op = A(a',s',b') stored K x M (lda = b_b'); right: B(b',s',c') M x K (lda = b_c')
        GemmSeg sg{M.offs[mb], it->second, side == 0 ? Mr : K, N, K, 0};
        O->g2.segs.push_back(sg);
        t.nseg++;
        t.ksum += K;
        O->flops += 2.0 * Mr * N * (double)K;
      }
      O->g2.tasks.push_back(t);
    }
    O->layout2 = side == 0 ? kTN : kNN;
    schedule_tiles(O->g1);
    schedule_tiles(O->g2);
    validate_gemm(O->g1, O->layout1, E.elems(), M.elems(), O->x1_elems, 0, "env stage 1");
    validate_mix(O->mix_tasks, O->mix_terms, O->mix_items, O->x1_elems, O->x2_elems, W.elems(), "env mixing");
    validate_gemm(O->g2, O->layout2, M.elems(), O->x2_elems, O->out_elems, 0, "env stage 3");
  } catch (...) {
    delete O;
    throw;
  }
  return O;
}

bsdmrg_op_s* build_merge(const Leg& a, const Leg& s1, const Leg& b, const Leg& s2, const Leg& c) {
  auto* O = new bsdmrg_op_s();
  try {
    O->kind = 3;
    Layout A = make_layout({&a, &s1, &b}, kMpsS);
    Layout B = make_layout({&b, &s2, &c}, kMpsS);
    Layout T = make_layout({&a, &s1, &s2, &c}, kPsiS);
    O->out_elems = T.elems();
    for (size_t tb = 0; tb < T.keys.size(); ++tb) {
      const int ia = T.keys[tb][0], i1 = T.keys[tb][1], i2 = T.keys[tb][2], ic = T.keys[tb][3];
      // theta block (a, s1, s2, c) = A block (a, s1, b) as an (a s1) x b matrix
      // times B block (b, s2, c) as b x (s2 c) (physical sectors of any size)
      const int32_t M = (int32_t)(a.d[ia] * s1.d[i1]), N = (int32_t)(s2.d[i2] * c.d[ic]);
      GemmTask t{T.offs[tb], N, M, N, (int32_t)O->g1.segs.size(), 0, 0, 0, 0};
      const int ib = b.find(cadd(a.q[ia], s1.q[i1]));
      if (ib >= 0) {
        const int ab = A.lookup(k3(ia, i1, ib)), bb = B.lookup(k3(ib, i2, ic));
        if (ab >= 0 && bb >= 0) {
          const int32_t K = (int32_t)b.d[ib];
          O->g1.segs.push_back(GemmSeg{A.offs[ab], B.offs[bb], K, N, K, 0});
          t.nseg = 1;
          t.ksum = K;
          O->flops += 2.0 * M * N * (double)K;
        }
      }
      O->g1.tasks.push_back(t);
    }
    O->layout1 = kNN;
    schedule_tiles(O->g1);
    validate_gemm(O->g1, kNN, A.elems(), B.elems(), O->out_elems, 0, "merge");
  } catch (...) {
    delete O;
    throw;
  }
  return O;
}

// Sparse-dense two-site product (Sec. IV-A: every operand embedded in one
// dense array, the forbidden blocks stored as zeros) as three GEMM stages:
//   T1(a' w, s1 s2 c)       = L(a' w, a) psi(a, s1 s2 c)              NN, one task
//   T2[a'](s1' s2' w'', c)  = WW(s1' s2' w'', w s1 s2) T1[a'](w s1 s2, c)  NN, one task per a'
//   out(a' s1' s2', c')     = T2(a' s1' s2', w'' c) R(c', w'' c)^T      NT, one task
bsdmrg_op_s* build_dense(int64_t ma, int64_t mc, int32_t k, int32_t d) {
  if (ma < 1 || mc < 1 || k < 1 || d < 1 || d > 8)
    throw Error{BSDMRG_EINVAL, "dense_plan: need ma, mc, k >= 1 and 1 <= d <= 8"};
  const int64_t dd = (int64_t)d * d;
  const int64_t lim = (int64_t)1 << 30;
  if (ma * k >= lim || dd * mc >= lim || k * mc >= lim || ma * dd >= lim || dd * k >= lim)
    throw Error{BSDMRG_EINVAL, "dense_plan: a GEMM dimension reaches 2^30"};
  if ((ma * k) * ma >= ((int64_t)1 << 31) / 8 || ma * dd * k * mc >= ((int64_t)1 << 31) / 8 ||
      (mc * k) * mc >= ((int64_t)1 << 31) / 8)
    throw Error{BSDMRG_EINVAL, "dense_plan: an operand reaches 2 GiB (32-bit buffer offsets)"};
  auto* O = new bsdmrg_op_s();
  try {
    O->kind = 4;
    O->dn_ma = ma;
    O->dn_mc = mc;
    O->dn_k = k;
    O->dn_d = d;
    const int32_t kdd = (int32_t)(k * dd);
    O->g1.segs.push_back(GemmSeg{0, 0, (int32_t)ma, (int32_t)(dd * mc), (int32_t)ma, 0});
    O->g1.tasks.push_back(GemmTask{0, (int32_t)(dd * mc), (int32_t)(ma * k), (int32_t)(dd * mc), 0, 1, (int32_t)ma, 0, 0});
    for (int64_t ap = 0; ap < ma; ++ap) {
      O->g3.segs.push_back(GemmSeg{0, ap * kdd * mc, kdd, (int32_t)mc, kdd, 0});
      O->g3.tasks.push_back(GemmTask{ap * kdd * mc, (int32_t)mc, kdd, (int32_t)mc, (int32_t)ap, 1, kdd, 0, 0});
    }
    O->g2.segs.push_back(GemmSeg{0, 0, (int32_t)(k * mc), (int32_t)(k * mc), (int32_t)(k * mc), 0});
    O->g2.tasks.push_back(GemmTask{0, (int32_t)mc, (int32_t)(ma * dd), (int32_t)mc, 0, 1, (int32_t)(k * mc), 0, 0});
    O->x1_elems = ma * kdd * mc;   // T1
    O->x2_elems = ma * kdd * mc;   // T2
    O->out_elems = ma * dd * mc;
    O->flops = 2.0 * (double)(ma * k) * ma * (dd * mc) + 2.0 * (double)ma * mc * kdd * kdd +
               2.0 * (double)(ma * dd) * (k * mc) * mc;
    O->layout1 = kNN;
    O->layout2 = kNT;
    schedule_tiles(O->g1);
    schedule_tiles(O->g3);
    schedule_tiles(O->g2);
    validate_gemm(O->g1, kNN, ma * k * ma, ma * dd * mc, O->x1_elems, 0, "dense S1");
    validate_gemm(O->g3, kNN, (int64_t)kdd * kdd, O->x1_elems, O->x2_elems, 0, "dense mixing");
    validate_gemm(O->g2, kNT, O->x2_elems, mc * k * mc, O->out_elems, 0, "dense S3");
  } catch (...) {
    delete O;
    throw;
  }
  return O;
}

}  // namespace bsd
