// Contraction planner: Alg. 2 (pair the blocks whose labels agree on the
// contracted legs, key the products by the remaining labels) generalised to
// the four-operand two-site product of Sec. II-C,
//   out(a',s1',s2',c') = sum L(a',w,a) W1(w,s1',s1,w') W2(w',s2',s2,w'')
//                            R(c',w'',c) psi(a,s1,s2,c),
// evaluated in three stages:
//   S1  T1(a',w,s1,s2,c) = sum_a L(a',w,a) psi(a,s1,s2,c)        grouped GEMM
//   S2  T2(a',s1',s2',w'',c) = sum WW(w,s1',s2',s1,s2,w'') T1     MPO mixing
//       with WW = sum_w' W1 W2 combined element by element
//   S3  out(a',s1',s2',c') = sum_{w'',c} T2 R(c',w'',c)            grouped GEMM
// Every block of psi, T1, T2, out is a matrix (physical sectors have dim 1):
// a T1 block is (b_a' * n_w) x b_c, a T2 block b_a' x (n_w'' * b_c).  S1 has
// one K segment per task (a = a' - f_w is unique); S3 sums the w'' flux
// sectors of an output block as a K-list accumulated in registers, so no
// atomics and a fixed summation order.
#include <algorithm>
#include <array>
#include <cstring>
#include <numeric>
#include <unordered_map>

#include "bsdmrg_internal.h"
#include "kernels.h"

namespace bsd {

constexpr int kTileM = 64, kTileN = 64;
constexpr int kMixItemElems = 4096;
constexpr int kRedItemSmall = 1024;
constexpr int64_t kMinRedItems = 256;
// S3 split-K: a task whose K-list is longer than the width is cut into pieces
// of at most that width, summed afterwards in a fixed order.  The width is the
// widest of kSplitWidths (0: no split) that still leaves at least kMinS3Tiles
// tiles of 64 x 64 (three rounds of four workgroups on each of the 256 CUs),
// else kSplitK: splitting only to fill the chip, since every piece adds a
// partial block to write and sum.
constexpr int kSplitK = 512;
constexpr int kSplitWidths[] = {0, 4096, 2048, 1024};
constexpr int64_t kMinS3Tiles = 3072;

static const int32_t kPsiSigns[4] = {1, 1, 1, -1};
static const int32_t kEnvSigns[3] = {-1, 1, 1};
static const int32_t kWSigns[4] = {1, 1, -1, -1};

static Charge add(const Charge& a, const Charge& b) { return {a[0] + b[0], a[1] + b[1]}; }
static Charge sub(const Charge& a, const Charge& b) { return {a[0] - b[0], a[1] - b[1]}; }

static Key key3(int a, int b, int c) { Key k{}; k[0] = a; k[1] = b; k[2] = c; return k; }
static Key key4(int a, int b, int c, int d) { Key k{}; k[0] = a; k[1] = b; k[2] = c; k[3] = d; return k; }
// packed (a', f, s1, s2, c) of a T1 block for hashing: sector indices < 2^16,
// channel sectors and physical sectors < 2^8 (checked by the caller)
static uint64_t pack5(int a, int b, int c, int d, int e) {
  return ((uint64_t)a << 40) | ((uint64_t)b << 32) | ((uint64_t)c << 24) | ((uint64_t)d << 16) | (uint64_t)e;
}

static void plan_problem(bsdmrg_plan_s* P, int pi, const bsdmrg_problem& in) {
  ProblemPlan& p = P->probs[pi];
  p.a = leg_from(in.a); p.s1 = leg_from(in.s1); p.s2 = leg_from(in.s2); p.c = leg_from(in.c);
  p.wl = leg_from(in.wl); p.wm = leg_from(in.wm); p.wr = leg_from(in.wr);
  for (const Leg* l : {&p.s1, &p.s2})
    for (auto d : l->d)
      if (d != 1) throw Error{BSDMRG_EINVAL, "plan: physical sectors must have dimension 1"};
  if (!in.w1_host || !in.w2_host) throw Error{BSDMRG_EINVAL, "plan: W host arrays are required"};
  p.psi = make_layout({&p.a, &p.s1, &p.s2, &p.c}, kPsiSigns);
  p.L = make_layout({&p.a, &p.wl, &p.a}, kEnvSigns);
  p.R = make_layout({&p.c, &p.wr, &p.c}, kEnvSigns);
  p.W1 = make_layout({&p.wl, &p.s1, &p.s1, &p.wm}, kWSigns);
  p.W2 = make_layout({&p.wm, &p.s2, &p.s2, &p.wr}, kWSigns);

  p.psi_base = P->psi_elems; P->psi_elems += p.psi.elems();
  p.L_base = P->L_elems;     P->L_elems += p.L.elems();
  p.R_base = P->R_elems;     P->R_elems += p.R.elems();
  p.W1_base = P->W1_elems;   P->W1_elems += p.W1.elems();
  p.W2_base = P->W2_elems;   P->W2_elems += p.W2.elems();
  p.t1_base = P->t1_elems;
  p.t2_base = P->t2_elems;
  p.coef_base = P->n_coefs;

  // Non-zero W blocks (a W block that is entirely zero is structurally absent).
  auto nonzero = [](const Layout& L, const double* v, int b) {
    for (int64_t e = L.offs[b]; e < L.offs[b + 1]; ++e)
      if (v[e] != 0.0) return true;
    return false;
  };
  std::vector<char> nz1(p.W1.keys.size()), nz2(p.W2.keys.size());
  for (size_t b = 0; b < nz1.size(); ++b) nz1[b] = nonzero(p.W1, in.w1_host, (int)b);
  for (size_t b = 0; b < nz2.size(); ++b) nz2[b] = nonzero(p.W2, in.w2_host, (int)b);
  p.nz1 = nz1;
  p.nz2 = nz2;
  p.w1_host.assign(in.w1_host, in.w1_host + p.W1.elems());
  p.w2_host.assign(in.w2_host, in.w2_host + p.W2.elems());

  // ---- S1: one task per (psi block, left channel sector) ---------------
  if (p.a.size() >= (1 << 16) || p.c.size() >= (1 << 16) || p.wl.size() >= 256 || p.wm.size() >= 256 ||
      p.wr.size() >= 256 || p.s1.size() >= 256 || p.s2.size() >= 256)
    throw Error{BSDMRG_EINVAL, "plan: too many sectors on a leg"};
  std::unordered_map<uint64_t, std::pair<int64_t, int>> t1;   // (a', f, s1, s2, c) -> (offset, index)
  t1.reserve(p.psi.keys.size() * p.wl.size() * 2);
  std::vector<int64_t> t1_off;
  int64_t t1_cursor = 0;
  for (size_t pb = 0; pb < p.psi.keys.size(); ++pb) {
    const Key& k = p.psi.keys[pb];
    int ia = k[0], i1 = k[1], i2 = k[2], ic = k[3];
    for (int f = 0; f < p.wl.size(); ++f) {
      int iap = p.a.find(add(p.a.q[ia], p.wl.q[f]));
      if (iap < 0) continue;
      int lb = p.L.lookup(key3(iap, f, ia));
      if (lb < 0) throw Error{BSDMRG_EQN, "plan: missing L block"};
      const int32_t M = (int32_t)(p.a.d[iap] * p.wl.d[f]);
      const int32_t N = (int32_t)p.c.d[ic];
      const int32_t K = (int32_t)p.a.d[ia];
      GemmSeg s{p.L_base + p.L.offs[lb], p.psi_base + p.psi.offs[pb], K, N, K, 0};
      GemmTask t{p.t1_base + t1_cursor, N, M, N, (int32_t)P->s1.segs.size(), 1, K, 0, 0};
      P->s1.segs.push_back(s);
      P->s1.tasks.push_back(t);
      P->s1.flops += 2.0 * M * N * (double)K;
      t1[pack5(iap, f, i1, i2, ic)] = {t1_cursor, (int)t1_off.size()};
      p.t1.push_back(T1Block{iap, f, i1, i2, ic, p.t1_base + t1_cursor});
      t1_off.push_back(t1_cursor);
      t1_cursor += round_up((int64_t)M * N);
    }
  }
  p.t1_elems = t1_cursor;

  // ---- S2: T2 blocks (a', s1', s2', g, c) and their mixing terms ------------
  struct CoefKey {
    int f, iw, s1p, s1, s2p, s2, g, iwpp;
    uint64_t pack() const {   // f, g < 2^8; iw, iwpp < 2^12; physical sectors < 2^8
      return ((uint64_t)f << 56) | ((uint64_t)iw << 44) | ((uint64_t)s1p << 36) | ((uint64_t)s1 << 28) |
             ((uint64_t)s2p << 20) | ((uint64_t)s2 << 12) | ((uint64_t)g << 4) ^ ((uint64_t)iwpp * 0x9E3779B97F4A7C15ull);
    }
  };
  struct CoefEntry {
    CoefKey k;
    int id;
  };
  std::unordered_map<uint64_t, std::vector<CoefEntry>> coef_index;
  auto wstart = [](const Leg& l) {
    std::vector<int64_t> s(l.size() + 1, 0);
    for (int i = 0; i < l.size(); ++i) s[i + 1] = s[i] + l.d[i];
    return s;
  };
  (void)wstart;
  auto same = [](const CoefKey& a, const CoefKey& b) {
    return a.f == b.f && a.iw == b.iw && a.s1p == b.s1p && a.s1 == b.s1 && a.s2p == b.s2p && a.s2 == b.s2 &&
           a.g == b.g && a.iwpp == b.iwpp;
  };
  auto coef_of = [&](const CoefKey& ck) -> int {
    auto& bucket = coef_index[ck.pack()];
    for (const CoefEntry& ce : bucket)
      if (same(ce.k, ck)) return ce.id;
    // pairs over the middle channel: W1(f,iw; s1p, s1; m, im) W2(m, im; s2p, s2; g, iwpp)
    std::vector<std::pair<int64_t, int64_t>> pairs;
    for (int m = 0; m < p.wm.size(); ++m) {
      int b1 = p.W1.lookup(key4(ck.f, ck.s1p, ck.s1, m));
      int b2 = p.W2.lookup(key4(m, ck.s2p, ck.s2, ck.g));
      if (b1 < 0 || b2 < 0 || !nz1[b1] || !nz2[b2]) continue;
      const int64_t nm = p.wm.d[m], ng = p.wr.d[ck.g];
      for (int im = 0; im < nm; ++im) {
        int64_t e1 = p.W1.offs[b1] + (int64_t)ck.iw * nm + im;
        int64_t e2 = p.W2.offs[b2] + (int64_t)im * ng + ck.iwpp;
        if (in.w1_host[e1] != 0.0 && in.w2_host[e2] != 0.0)
          pairs.push_back({p.W1_base + e1, p.W2_base + e2});
      }
    }
    if (pairs.empty()) {
      bucket.push_back(CoefEntry{ck, -1});
      return -1;
    }
    int id = (int)(P->coef_ptr.size() - 1);
    for (auto& pr : pairs) { P->coef_e1.push_back(pr.first); P->coef_e2.push_back(pr.second); }
    P->coef_ptr.push_back((int32_t)P->coef_e1.size());
    p.n_coefs++;
    bucket.push_back(CoefEntry{ck, id});
    return id;
  };

  // (f, s1, s2) coupled to (s1', s2', g) through some middle channel sector
  // with non-zero W_i and W_{i+1} blocks; independent of the bond sectors,
  // so found once (lexicographic in (f, s1, s2))
  const int n1 = p.s1.size(), n2 = p.s2.size();
  std::vector<std::vector<std::array<int, 3>>> wlink((size_t)n1 * n2 * p.wr.size());
  for (int s1p = 0; s1p < n1; ++s1p)
    for (int s2p = 0; s2p < n2; ++s2p)
      for (int g = 0; g < p.wr.size(); ++g) {
        auto& lst = wlink[((size_t)s1p * n2 + s2p) * p.wr.size() + g];
        for (int f = 0; f < p.wl.size(); ++f)
          for (int i1 = 0; i1 < n1; ++i1)
            for (int i2 = 0; i2 < n2; ++i2)
              for (int m = 0; m < p.wm.size(); ++m) {
                int b1 = p.W1.lookup(key4(f, s1p, i1, m));
                int b2 = p.W2.lookup(key4(m, s2p, i2, g));
                if (b1 >= 0 && b2 >= 0 && nz1[b1] && nz2[b2]) {
                  lst.push_back({f, i1, i2});
                  break;
                }
              }
      }

  std::map<Key, std::pair<int64_t, int>> t2;   // (a', s1', s2', g) -> (offset, c)
  int64_t t2_cursor = 0;
  // mixing items that read the T1 blocks of one (a', c) sector pair form a
  // group (placed on one XCD so that the blocks are re-read from its L2)
  std::map<std::pair<int, int>, int32_t> group_of;
  for (int iap = 0; iap < p.a.size(); ++iap)
    for (int s1p = 0; s1p < p.s1.size(); ++s1p)
      for (int s2p = 0; s2p < p.s2.size(); ++s2p) {
        Charge qout = add(add(p.a.q[iap], p.s1.q[s1p]), p.s2.q[s2p]);   // = q_c'
        if (p.c.find(qout) < 0) continue;
        for (int g = 0; g < p.wr.size(); ++g) {
          int ic = p.c.find(sub(qout, p.wr.q[g]));
          if (ic < 0) continue;
          // block-level existence: a T1 block and non-zero W blocks connect
          const auto& lst = wlink[((size_t)s1p * n2 + s2p) * p.wr.size() + g];
          std::vector<std::pair<int, const std::pair<int64_t, int>*>> src;   // (link, T1 block)
          for (size_t li = 0; li < lst.size(); ++li) {
            auto it = t1.find(pack5(iap, lst[li][0], lst[li][1], lst[li][2], ic));
            if (it != t1.end()) src.push_back({(int)li, &it->second});
          }
          if (src.empty()) continue;
          const int64_t ba = p.a.d[iap], bc = p.c.d[ic], ng = p.wr.d[g];
          if (bc > kMixItemElems || ba > (1 << 30))
            throw Error{BSDMRG_EINVAL, "plan: sector dimensions above 4096 are not supported"};
          t2[key4(iap, s1p, s2p, g)] = {t2_cursor, ic};
          p.t2.push_back(T2Block{iap, s1p, s2p, g, ic, p.t2_base + t2_cursor});
          for (int iwpp = 0; iwpp < ng; ++iwpp) {
            MixTask mt{p.t2_base + t2_cursor + iwpp * bc, (int32_t)(ng * bc), (int32_t)ba,
                       (int32_t)bc, (int32_t)P->mix_terms.size(), 0, 0};
            for (const auto& sr : src) {
              const int f = lst[sr.first][0], i1 = lst[sr.first][1], i2 = lst[sr.first][2];
              const int64_t nf = p.wl.d[f];
              for (int iw = 0; iw < nf; ++iw) {
                int cidx = coef_of(CoefKey{f, iw, s1p, i1, s2p, i2, g, iwpp});
                if (cidx < 0) continue;
                P->mix_terms.push_back(MixTerm{p.t1_base + sr.second->first + iw * bc, (int32_t)(nf * bc), cidx});
              }
            }
            mt.nterm = (int32_t)P->mix_terms.size() - mt.term0;
            P->flops_s2 += 2.0 * mt.nterm * (double)ba * bc;
            const int task = (int)P->mix_tasks.size();
            P->mix_tasks.push_back(mt);
            // item size: up to kMixItemElems outputs, fewer for tasks with many
            // terms (their loads come in rounds of four, then two, then one
            // term), so that no workgroup runs much longer than the others
            const int64_t rounds = std::max<int64_t>(1, mt.nterm / 4 + (mt.nterm % 4 + 1) / 2);
            const int64_t item_elems = (int64_t)P->mix_per * 256;
            int rows_per = std::max<int64_t>(1, item_elems / std::max<int64_t>(1, bc * rounds));
            auto gi = group_of.emplace(std::make_pair(iap, ic), (int32_t)(P->n_mix_groups + group_of.size())).first;
            for (int r0 = 0; r0 < ba; r0 += rows_per) {
              P->mix_items.push_back(MixItem{task, r0, (int32_t)std::min<int64_t>(rows_per, ba - r0), 0});
              P->mix_item_group.push_back(gi->second);
            }
          }
          t2_cursor += round_up(ba * ng * bc);
        }
      }
  p.t2_elems = t2_cursor;
  P->n_mix_groups += (int32_t)group_of.size();

  // ---- S3: one task per output block, K-list over the w'' flux sectors ------
  for (size_t ob = 0; ob < p.psi.keys.size(); ++ob) {
    const Key& k = p.psi.keys[ob];
    int iap = k[0], s1p = k[1], s2p = k[2], icp = k[3];
    const int32_t M = (int32_t)p.a.d[iap], N = (int32_t)p.c.d[icp];
    GemmTask t{p.psi_base + p.psi.offs[ob], N, M, N, (int32_t)P->s3.segs.size(), 0, 0, 0, 0};
    for (int g = 0; g < p.wr.size(); ++g) {
      auto it = t2.find(key4(iap, s1p, s2p, g));
      if (it == t2.end()) continue;
      int ic = it->second.second;
      int rb = p.R.lookup(key3(icp, g, ic));
      if (rb < 0) throw Error{BSDMRG_EQN, "plan: missing R block"};
      const int32_t K = (int32_t)(p.wr.d[g] * p.c.d[ic]);
      P->s3.segs.push_back(GemmSeg{p.t2_base + it->second.first, p.R_base + p.R.offs[rb], K, K, K, 0});
      t.nseg++;
      t.ksum += K;
      P->s3.flops += 2.0 * M * N * (double)K;
    }
    P->s3.tasks.push_back(t);
  }
  // ---- diagonal of H_eff: flux-0 channels of L, W1, W2, R per psi block ----
  {
    const Charge zero{0, 0};
    const int f0 = p.wl.find(zero), m0 = p.wm.find(zero), g0 = p.wr.find(zero);
    if (f0 >= 0 && m0 >= 0 && g0 >= 0) {
      const int64_t nl = p.wl.d[f0], nm = p.wm.d[m0], nr = p.wr.d[g0];
      if (nl > kMaxDiagChannels || nr > kMaxDiagChannels)
        throw Error{BSDMRG_EINVAL, "plan: more than 64 channels in the flux-0 sector"};
      for (size_t pb = 0; pb < p.psi.keys.size(); ++pb) {
        const Key& k = p.psi.keys[pb];
        const int ia = k[0], i1 = k[1], i2 = k[2], ic = k[3];
        const int lb = p.L.lookup(key3(ia, f0, ia)), rb = p.R.lookup(key3(ic, g0, ic));
        const int b1 = p.W1.lookup(key4(f0, i1, i1, m0)), b2 = p.W2.lookup(key4(m0, i2, i2, g0));
        if (lb < 0 || rb < 0 || b1 < 0 || b2 < 0 || !nz1[b1] || !nz2[b2]) continue;   // diagonal 0
        const int32_t rows = (int32_t)p.a.d[ia], cols = (int32_t)p.c.d[ic];
        const int32_t per = std::max<int32_t>(1, kMixItemElems / cols);
        for (int32_t r0 = 0; r0 < rows; r0 += per)
          P->diag_tasks.push_back(DiagTask{p.psi_base + p.psi.offs[pb], p.L_base + p.L.offs[lb],
                                           p.R_base + p.R.offs[rb], p.W1_base + p.W1.offs[b1],
                                           p.W2_base + p.W2.offs[b2], rows, cols, (int32_t)nl, (int32_t)nm,
                                           (int32_t)nr, r0, std::min(per, rows - r0), 0});
      }
    }
  }
  P->t1_elems += p.t1_elems;
  P->t2_elems += p.t2_elems;
  P->n_coefs += p.n_coefs;
}

// 64 x 64 tiles of S3 if tasks with a K-list longer than w (> 0) are split.
static int64_t s3_tiles_at(const Stage& st, int w) {
  int64_t n = 0;
  for (const GemmTask& t : st.tasks) {
    const int64_t tiles = (int64_t)((t.M + kTileM - 1) / kTileM) * ((t.N + kTileN - 1) / kTileN);
    int64_t pieces = 1;
    if (w > 0 && t.ksum > w) {
      pieces = 0;
      for (int j = 0; j < t.nseg; ++j) pieces += (st.segs[t.seg0 + j].K + w - 1) / w;
    }
    n += tiles * pieces;
  }
  return n;
}

static int choose_split(const Stage& st) {
  for (int w : kSplitWidths)
    if (s3_tiles_at(st, w) >= kMinS3Tiles) return w;
  return kSplitK;
}

// Split every S3 task whose K-list is longer than the chosen width into
// pieces of at most that width (segments are cut along K: the A and B offsets
// move by k0 columns).  Each piece writes an M x N partial block; the pieces
// of a task are summed in piece order by the reduction tables.
static void split_k(bsdmrg_plan_s* P) {
  Stage& st = P->s3;
  const int w = choose_split(st);
  P->s3_split = w;
  if (w == 0) return;
  std::vector<GemmTask> tasks;
  std::vector<GemmSeg> segs;
  for (const GemmTask& t : st.tasks) {
    if (t.ksum <= w) {
      GemmTask u = t;
      u.seg0 = (int32_t)segs.size();
      for (int j = 0; j < t.nseg; ++j) segs.push_back(st.segs[t.seg0 + j]);
      tasks.push_back(u);
      continue;
    }
    MixTask red{t.c_off, t.ldc, t.M, t.N, (int32_t)P->red_terms.size(), 0, 0};
    for (int j = 0; j < t.nseg; ++j) {
      const GemmSeg& g = st.segs[t.seg0 + j];
      for (int k0 = 0; k0 < g.K; k0 += w) {
        const int32_t kk = std::min(w, g.K - k0);
        GemmSeg h{g.a_off + k0, g.b_off + k0, g.lda, g.ldb, kk, 0};
        GemmTask u{P->s3_part_elems, t.N, t.M, t.N, (int32_t)segs.size(), 1, kk, 1, 0};
        segs.push_back(h);
        tasks.push_back(u);
        P->red_terms.push_back(MixTerm{P->s3_part_elems, t.N, -1});
        P->s3_part_elems += round_up((int64_t)t.M * t.N);
      }
    }
    red.nterm = (int32_t)P->red_terms.size() - red.term0;
    P->red_tasks.push_back(red);
  }
  st.tasks.swap(tasks);
  st.segs.swap(segs);
  // reduction workgroups of whole rows, up to kMixItemElems outputs each, or
  // up to kRedItemSmall when the larger ones would number fewer than one per
  // CU (kMinRedItems)
  // (items of tasks with many pieces are smaller: the pieces are loaded in
  // rounds of two)
  auto rows_per = [](const MixTask& r, int item) {
    return std::max(1, item / std::max(1, r.cols * std::max(1, (r.nterm + 1) / 2)));
  };
  int64_t n_big = 0;
  const int big = P->mix_per * 256;
  for (const MixTask& r : P->red_tasks) n_big += (r.rows + rows_per(r, big) - 1) / rows_per(r, big);
  const int item = n_big < kMinRedItems ? std::min(kRedItemSmall, big) : big;
  for (int task = 0; task < (int)P->red_tasks.size(); ++task) {
    const MixTask& r = P->red_tasks[task];
    const int rp = rows_per(r, item);
    for (int r0 = 0; r0 < r.rows; r0 += rp) P->red_items.push_back(MixItem{task, r0, std::min(rp, r.rows - r0), 0});
  }
}

}  // namespace bsd

using namespace bsd;

// Order the mixing items so that the items of one group (they read the
// same T1 blocks) run on one XCD: workgroup i of a launch runs on XCD
// i mod 8, so the groups are dealt to 8 bins longest-first by work (rows x
// columns x terms) and slot i takes the next item of bin i mod 8 (of the
// fullest bin once its own is empty).  Every item computes the same values
// in any order.
static void order_mix_items(bsdmrg_plan_s* P) {
  constexpr int kXcd = 8;
  const size_t n = P->mix_items.size();
  if (n == 0) return;
  const int ng = P->n_mix_groups;
  std::vector<double> work(ng, 0.0);
  std::vector<std::vector<int>> items(ng);
  for (size_t i = 0; i < n; ++i) {
    const MixItem& it = P->mix_items[i];
    const MixTask& t = P->mix_tasks[it.task];
    const int g = P->mix_item_group[i];
    work[g] += (double)it.nrows * t.cols * std::max(1, t.nterm);
    items[g].push_back((int)i);
  }
  std::vector<int> gorder(ng);
  for (int g = 0; g < ng; ++g) gorder[g] = g;
  std::stable_sort(gorder.begin(), gorder.end(), [&](int a, int b) { return work[a] > work[b]; });
  std::vector<double> load(kXcd, 0.0);
  std::vector<std::vector<int>> bin(kXcd);
  for (int g : gorder) {
    if (items[g].empty()) continue;
    const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    load[x] += work[g];
    bin[x].insert(bin[x].end(), items[g].begin(), items[g].end());
  }
  std::vector<size_t> next(kXcd, 0);
  std::vector<MixItem> out;
  std::vector<int32_t> out_group;
  out.reserve(n);
  out_group.reserve(n);
  for (size_t i = 0; i < n; ++i) {
    int x = (int)(i % kXcd);
    if (next[x] == bin[x].size()) {
      size_t best = 0;
      for (int y = 0; y < kXcd; ++y)
        if (bin[y].size() - next[y] > best) {
          best = bin[y].size() - next[y];
          x = y;
        }
    }
    const int src = bin[x][next[x]++];
    out.push_back(P->mix_items[src]);
    out_group.push_back(P->mix_item_group[src]);
  }
  P->mix_items.swap(out);
  P->mix_item_group.swap(out_group);
}

bsdmrg_plan_s* build_plan(const bsdmrg_problem* probs, int n_probs) {
  auto* P = new bsdmrg_plan_s();
  try {
    P->probs.resize(n_probs);
    P->coef_ptr.push_back(0);
    // S2 and the split-K sums work on rows of c-sector width: eight outputs
    // per thread (items of up to 2048) when every row fits, else sixteen
    int64_t widest = 0;
    for (int i = 0; i < n_probs; ++i)
      for (auto d : leg_from(probs[i].c).d) widest = std::max<int64_t>(widest, d);
    P->mix_per = widest <= 2048 ? 8 : 16;
    for (int i = 0; i < n_probs; ++i) plan_problem(P, i, probs[i]);
    split_k(P);
    order_mix_items(P);
    schedule_tiles(P->s1);
    schedule_tiles(P->s3);
    flatten_tiles(P->s1);
    flatten_tiles(P->s3);
    schedule_persistent(P->s1, kPersistentSlotsPerXcd);
    schedule_persistent(P->s3, kPersistentSlotsPerXcd);
    validate_ptiles(P->s1, "S1 persistent tiles");
    validate_ptiles(P->s3, "S3 persistent tiles");
    // Davidson reduction chunks
    for (int i = 0; i < n_probs; ++i) {
      ProblemPlan& p = P->probs[i];
      p.chunk0 = (int32_t)P->chunks.size();
      for (int64_t s = 0; s < p.psi.elems(); s += kChunk)
        P->chunks.push_back(Chunk{p.psi_base + s, (int32_t)std::min<int64_t>(kChunk, p.psi.elems() - s), i});
      p.nchunk = (int32_t)P->chunks.size() - p.chunk0;
      P->dav_probs.push_back(DavProb{p.psi_base, p.psi.elems(), p.chunk0, p.nchunk});
      P->blk_ptr.push_back((int32_t)(P->blk_off.size() / 2));
      for (size_t b = 0; b < p.psi.keys.size(); ++b) {
        const Key& k = p.psi.keys[b];
        P->blk_off.push_back(p.psi.offs[b]);
        P->blk_off.push_back(p.a.d[k[0]] * p.c.d[k[3]]);
        p.dim += p.a.d[k[0]] * p.c.d[k[3]];
      }
    }
    P->blk_ptr.push_back((int32_t)(P->blk_off.size() / 2));
    validate_heff_plan(P);
  } catch (...) {
    delete P;
    throw;
  }
  return P;
}
