// Truncated SVD split of the two-site tensor (Sec. II-C, Fig. 1e; Sec. IV-A).
// theta(a,s1,s2,c) is wrapped into one matrix per charge q of the new bond
// (rows: the (a, s1) pairs with q_a + q_s1 = q; columns: the (s2, c) pairs
// with q_c - q_s2 = q; both in lexicographic order of their sector indices),
// each matrix is decomposed in FP64 on the device: QR with column pivoting
// (one workgroup per matrix up to 64 columns, else one launch per step over
// many workgroups) cut at the numerical rank, then block one-sided Jacobi on
// R^T (block pairs of a step in parallel workgroups, columns in LDS) until a
// sweep rotates nothing; the singular values of all charges are pooled and
// truncated on the host, and U, S, V^T are scattered into A(a,s1,b) and
// B(b,s2,c) with S absorbed in the direction of the sweep.  Physical sectors
// may have any dimension up to 64 (rows (a, s1) and columns (s2, c) of a
// charge matrix are then fused a-major and s2-major).  Readings of the silent points: see bsdmrg_truncate in the
// header (cutoff modes, degenerate groups, sign gauge).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "bsdmrg_internal.h"
#include "kernels.h"

namespace bsd {

static const int32_t kPsiS[4] = {1, 1, 1, -1};
static const int32_t kMpsS[3] = {1, 1, -1};

struct TSector {
  Charge q;
  std::vector<std::pair<int, int>> rk, ck;   // (a, s1) and (s2, c) sector pairs
  std::vector<int64_t> r0, c0;
  int64_t rows = 0, cols = 0, kmin = 0;
  int64_t mat, u, s, v;                       // X, U, S, Vt offsets (elements)
  int64_t jav, jz, jaux, jsig, jperm;         // SVD scratch offsets in the work array
  int32_t b = 1, nb = 2;                      // block-Jacobi blocks
};

struct TPlan {
  Leg a, s1, s2, c;
  Layout theta;
  std::vector<TSector> sec;
  int64_t n_mat = 0, n_u = 0, n_s = 0, n_v = 0, n_work = 0, n_pairs = 0, n_cols = 0, n_big = 0, n_bigcols = 0;
  int64_t n_gather = 0;
  size_t bytes = 0;
};

static size_t al(size_t b) { return (b + 255) / 256 * 256; }
constexpr int kSvdMaxSweeps = 60;   // block-Jacobi sweeps (a converged matrix stops earlier)
// Matrices with more columns than this are factorised by the multi-workgroup
// QR (one launch per step and phase, all such matrices of a truncation
// together); smaller ones by one workgroup each, whose QR runs at the L2
// bandwidth of one CU: above ~64 columns the per-column launches are faster
// (6x6 J1-J2 sweeps at m = 512: truncations 0.90 s per sweep with the cut at
// 256 columns, 0.77 s at 64; 4x16 Hubbard sweeps at m = 1024 -7%).
constexpr int64_t kQrBig = 64;

static TPlan make_tplan(const bsdmrg_leg* legs) {
  TPlan T;
  T.a = leg_from(legs[0]); T.s1 = leg_from(legs[1]); T.s2 = leg_from(legs[2]); T.c = leg_from(legs[3]);
  for (const Leg* l : {&T.s1, &T.s2})
    for (auto d : l->d)
      if (d > 64) throw Error{BSDMRG_EINVAL, "truncate: physical sectors above dimension 64"};
  T.theta = make_layout({&T.a, &T.s1, &T.s2, &T.c}, kPsiS);
  std::map<Charge, std::vector<std::pair<int, int>>> rows, cols;
  for (int ia = 0; ia < T.a.size(); ++ia)
    for (int i1 = 0; i1 < T.s1.size(); ++i1)
      rows[{T.a.q[ia][0] + T.s1.q[i1][0], T.a.q[ia][1] + T.s1.q[i1][1]}].push_back({ia, i1});
  for (int i2 = 0; i2 < T.s2.size(); ++i2)
    for (int ic = 0; ic < T.c.size(); ++ic)
      cols[{T.c.q[ic][0] - T.s2.q[i2][0], T.c.q[ic][1] - T.s2.q[i2][1]}].push_back({i2, ic});
  for (auto& kv : rows) {
    auto it = cols.find(kv.first);
    if (it == cols.end()) continue;
    TSector s;
    s.q = kv.first;
    s.rk = kv.second;
    s.ck = it->second;
    for (auto& r : s.rk) { s.r0.push_back(s.rows); s.rows += T.a.d[r.first] * T.s1.d[r.second]; }
    for (auto& c : s.ck) { s.c0.push_back(s.cols); s.cols += T.s2.d[c.first] * T.c.d[c.second]; }
    s.kmin = std::min(s.rows, s.cols);
    s.u = T.n_u; T.n_u += s.rows * s.kmin;
    s.v = T.n_v; T.n_v += s.kmin * s.cols;
    s.s = T.n_s; T.n_s += s.kmin;
    // SVD work: X (max x min), AV (2 min x min), Z (max x min), aux
    // (4 min + 2), sigma (min), order (min)
    s.mat = T.n_work; T.n_work += s.rows * s.cols;
    s.jav = T.n_work; T.n_work += 2 * s.kmin * s.kmin;
    s.jz = T.n_work; T.n_work += s.rows * s.cols;
    s.jaux = T.n_work; T.n_work += 4 * s.kmin + 2;
    s.jsig = T.n_work; T.n_work += s.kmin;
    s.jperm = T.n_work; T.n_work += s.kmin;
    // blocks of b columns: a pair of blocks (2b columns of 2 min rows at
    // most) fills the 16384 doubles of LDS of one workgroup; the widest such
    // b (at most 32): fewer, longer block-Jacobi steps per sweep
    if (s.kmin > 4096) throw Error{BSDMRG_EINVAL, "truncate: a charge sector has more than 4096 columns"};
    s.b = (int32_t)std::max<int64_t>(1, std::min<int64_t>(32, 16384 / (4 * s.kmin)));
    s.nb = (int32_t)((s.kmin + s.b - 1) / s.b);
    s.nb += s.nb & 1;
    if (s.nb < 2) s.nb = 2;
    T.n_pairs += s.nb / 2;
    T.n_cols += (s.kmin + 15) / 16;
    if (s.kmin > kQrBig) {
      T.n_big += 1;
      T.n_bigcols += (s.kmin + 15) / 16;
    }
    T.sec.push_back(s);
  }
  T.n_mat = T.n_work;
  // scatter copies: one per (row pair, i_1) into A and per (column pair, i_2) into B
  int64_t n_rk = 0, n_ck = 0;
  for (auto& s : T.sec) {
    for (auto& r : s.rk) n_rk += T.s1.d[r.second];
    for (auto& c : s.ck) n_ck += T.s2.d[c.first];
  }
  // gather copies: one per (theta block, i_1, i_2)
  T.n_gather = 0;
  for (const Key& k : T.theta.keys) T.n_gather += T.s1.d[k[1]] * T.s2.d[k[2]];
  T.bytes = al(T.n_work * 8) + al(T.n_u * 8) + al(T.n_s * 8) + al(T.n_v * 8) + al(T.n_s * 8) * 2 +
            al(T.n_gather * sizeof(CopyTask) + 1) + al(T.sec.size() * sizeof(SvdTask) + 1) +
            al(T.n_pairs * sizeof(SvdPair) + 1) + al(T.n_cols * sizeof(SvdCols) + 1) + al(T.sec.size() * 8) * 2 +
            al(T.n_big * sizeof(int32_t) + 1) + al(T.n_bigcols * sizeof(SvdCols) + 1) +
            al(T.n_s * sizeof(GaugeTask) + 1) + al((n_rk + n_ck) * sizeof(CopyTask) + 1);
  return T;
}

// Global selection of the kept singular values (ties by charge index, then
// index inside the charge).
static std::vector<int64_t> select_kept(const TPlan& T, const std::vector<double>& S, const bsdmrg_trunc_opts* o,
                                        double* discarded, std::vector<double>& kept_vals) {
  struct E { double v; int sec; int64_t j; };
  std::vector<E> pool;
  for (size_t q = 0; q < T.sec.size(); ++q)
    for (int64_t j = 0; j < T.sec[q].kmin; ++j) pool.push_back({S[T.sec[q].s + j], (int)q, j});
  std::stable_sort(pool.begin(), pool.end(), [](const E& x, const E& y) {
    if (x.v != y.v) return x.v > y.v;
    if (x.sec != y.sec) return x.sec < y.sec;
    return x.j < y.j;
  });
  double total2 = 0.0;
  for (auto& p : pool) total2 += p.v * p.v;
  const double norm = std::sqrt(total2);
  int64_t n_keep = 0;
  if (o->cutoff_mode == 0) {
    for (auto& p : pool) n_keep += p.v >= o->cutoff * norm;
  } else {
    n_keep = (int64_t)pool.size();
    double acc = 0.0;
    while (n_keep > 0 && acc + pool[n_keep - 1].v * pool[n_keep - 1].v <= o->cutoff * total2) {
      acc += pool[n_keep - 1].v * pool[n_keep - 1].v;
      --n_keep;
    }
  }
  n_keep = std::min<int64_t>(n_keep, o->max_m);
  if (n_keep > 0 && n_keep < (int64_t)pool.size()) {
    const double sd = pool[n_keep].v;
    int64_t n2 = n_keep;
    while (n2 > 0 && pool[n2 - 1].v - sd <= o->degen_rtol * pool[n2 - 1].v) --n2;
    if (n2 > 0) n_keep = n2;
  }
  std::vector<int64_t> counts(T.sec.size(), 0);
  double disc = 0.0;
  kept_vals.clear();
  for (int64_t i = 0; i < (int64_t)pool.size(); ++i) {
    if (i < n_keep) {
      counts[pool[i].sec]++;
      kept_vals.push_back(pool[i].v);
    } else {
      disc += pool[i].v * pool[i].v;
    }
  }
  *discarded = disc;
  return counts;
}

#define HIPCHK(x)                                                                              \
  do {                                                                                         \
    hipError_t e_ = (x);                                                                       \
    if (e_ != hipSuccess) throw Error{BSDMRG_EHIP, std::string(#x) + ": " + hipGetErrorString(e_)}; \
  } while (0)

void truncate_workspace(const bsdmrg_leg* legs, int64_t* bytes) { *bytes = (int64_t)make_tplan(legs).bytes; }

void truncate_run(const bsdmrg_leg* legs, const double* theta, const bsdmrg_trunc_opts* o, int32_t* new_n,
                  int32_t* new_q, int64_t* new_d, int32_t leg_cap, double* A, int64_t A_cap, int64_t* A_elems,
                  double* B, int64_t B_cap, int64_t* B_elems, double* svals, int64_t sv_cap, int64_t* n_kept,
                  double* discarded, void* ws, int64_t ws_bytes, hipStream_t st) {
  if (!o || !theta || !new_n || !new_q || !new_d || !A_elems || !B_elems || !n_kept || !discarded)
    throw Error{BSDMRG_EINVAL, "truncate: NULL argument"};
  if (o->direction != 0 && o->direction != 1) throw Error{BSDMRG_EINVAL, "truncate: direction must be 0 or 1"};
  if (o->cutoff_mode != 0 && o->cutoff_mode != 1) throw Error{BSDMRG_EINVAL, "truncate: bad cutoff_mode"};
  if (!(o->cutoff >= 0.0) || o->max_m < 1 || !(o->degen_rtol >= 0.0))
    throw Error{BSDMRG_EINVAL, "truncate: bad cutoff, max_m or degen_rtol"};
  TPlan T = make_tplan(legs);
  if (!ws || (size_t)ws_bytes < T.bytes) throw Error{BSDMRG_EINVAL, "truncate: workspace too small"};
  char* p = (char*)ws;
  auto take = [&](size_t bytes) { char* r = p; p += al(bytes); return r; };
  double* work = (double*)take(T.n_work * 8);
  double* U = (double*)take(T.n_u * 8);
  double* S = (double*)take(T.n_s * 8);
  double* V = (double*)take(T.n_v * 8);
  double* sign = (double*)take(T.n_s * 8);
  double* sgn_s = (double*)take(T.n_s * 8);
  char* gather_tab = take(T.n_gather * sizeof(CopyTask) + 1);
  char* svd_tab = take(T.sec.size() * sizeof(SvdTask) + 1);
  char* pair_tab = take(T.n_pairs * sizeof(SvdPair) + 1);
  char* cols_tab = take(T.n_cols * sizeof(SvdCols) + 1);
  double* d_active = (double*)take(T.sec.size() * 8);
  double* d_rot = (double*)take(T.sec.size() * 8);
  char* big_tab = take(T.n_big * sizeof(int32_t) + 1);
  char* bigcols_tab = take(T.n_bigcols * sizeof(SvdCols) + 1);
  char* gauge_tab = take(T.n_s * sizeof(GaugeTask) + 1);
  char* scatter_tab = p;

  // gather theta blocks into the column-major charge matrices
  std::vector<CopyTask> gt;
  for (size_t si = 0; si < T.sec.size(); ++si) {
    const TSector& s = T.sec[si];
    for (size_t r = 0; r < s.rk.size(); ++r)
      for (size_t c = 0; c < s.ck.size(); ++c) {
        Key k{};
        k[0] = s.rk[r].first; k[1] = s.rk[r].second; k[2] = s.ck[c].first; k[3] = s.ck[c].second;
        const int b = T.theta.lookup(k);
        if (b < 0) throw Error{BSDMRG_EQN, "truncate: theta block missing"};
        // block (a, s1, s2, c) row-major; matrix row r0 + i_a d1 + i_1, column
        // c0 + i_2 dc + i_c: one strided copy of an a x c sub-block per (i_1, i_2)
        const int32_t rows = (int32_t)T.a.d[k[0]], cols = (int32_t)T.c.d[k[3]];
        const int32_t d1 = (int32_t)T.s1.d[k[1]], d2 = (int32_t)T.s2.d[k[2]];
        for (int32_t i1 = 0; i1 < d1; ++i1)
          for (int32_t i2 = 0; i2 < d2; ++i2) {
            const int64_t src = T.theta.offs[b] + (int64_t)(i1 * d2 + i2) * cols;
            const int64_t mr = s.r0[r] + i1, mc = s.c0[c] + (int64_t)i2 * cols;
            if (s.rows >= s.cols)   // X = M, column-major (ld rows)
              gt.push_back(CopyTask{src, s.mat + mr + mc * s.rows, rows, cols, d1 * d2 * cols, 1, d1,
                                    (int32_t)s.rows, -1, 0});
            else                    // X = M^T, column-major (ld cols)
              gt.push_back(CopyTask{src, s.mat + mc + mr * s.cols, rows, cols, d1 * d2 * cols, 1,
                                    (int32_t)s.cols * d1, 1, -1, 0});
          }
      }
  }
  validate_copy(gt, T.theta.elems(), T.n_work, 0, "truncate gather");
  HIPCHK(hipMemcpyAsync(gather_tab, gt.data(), gt.size() * sizeof(CopyTask), hipMemcpyHostToDevice, st));
  HIPCHK(launch_copy(gather_tab, (int)gt.size(), theta, work, nullptr, st));
  std::vector<SvdTask> sv;
  std::vector<SvdPair> pairs;
  std::vector<SvdCols> colblk, bigcols;
  std::vector<int32_t> big;
  int nb_max = 0, n_big_max = 0;
  for (size_t si = 0; si < T.sec.size(); ++si) {
    const TSector& s = T.sec[si];
    const bool tr = s.rows < s.cols;
    sv.push_back(SvdTask{s.mat, s.jav, s.jz, s.jaux, s.jsig, s.jperm, s.u, s.s, s.v,
                         (int32_t)std::max(s.rows, s.cols), (int32_t)s.kmin, (int32_t)s.rows, tr ? 1 : 0,
                         s.b, s.nb, s.kmin > kQrBig ? 1 : 0, 0});
    const SvdTask& t = sv.back();
    const int64_t mn = (int64_t)t.m * t.n, nn = (int64_t)t.n * t.n;
    if (t.x_off + mn > T.n_work || t.av_off + 2 * nn > T.n_work || t.z_off + mn > T.n_work ||
        t.aux_off + 4 * t.n + 2 > T.n_work || t.sig_off + t.n > T.n_work || t.perm_off + t.n > T.n_work ||
        t.u_off + s.rows * s.kmin > T.n_u || t.vt_off + s.kmin * s.cols > T.n_v || t.s_off + t.n > T.n_s ||
        t.m < t.n || t.n < 1 || (t.transposed ? s.cols : s.rows) != t.m || t.b < 1 || t.nb < 2 || (t.nb & 1) ||
        (int64_t)t.nb * t.b < t.n || 4 * (int64_t)t.b * t.n > 16384)
      throw Error{BSDMRG_EINVAL, "internal table check failed: truncate SVD"};
    for (int q = 0; q < t.nb / 2; ++q) pairs.push_back(SvdPair{(int32_t)si, q});
    for (int c = 0; c < t.n; c += 16) colblk.push_back(SvdCols{(int32_t)si, c});
    nb_max = std::max(nb_max, (int)t.nb);
    if (t.big_qr) {
      big.push_back((int32_t)si);
      for (int c = 0; c < t.n; c += 16) bigcols.push_back(SvdCols{(int32_t)si, c});
      n_big_max = std::max(n_big_max, (int)t.n);
    }
  }
  if ((int64_t)big.size() != T.n_big || (int64_t)bigcols.size() != T.n_bigcols)
    throw Error{BSDMRG_EINVAL, "internal table check failed: truncate QR blocks"};
  if ((int64_t)pairs.size() != T.n_pairs || (int64_t)colblk.size() != T.n_cols)
    throw Error{BSDMRG_EINVAL, "internal table check failed: truncate SVD blocks"};
  HIPCHK(hipMemcpyAsync(svd_tab, sv.data(), sv.size() * sizeof(SvdTask), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(cols_tab, colblk.data(), colblk.size() * sizeof(SvdCols), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(big_tab, big.data(), big.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(bigcols_tab, bigcols.data(), bigcols.size() * sizeof(SvdCols), hipMemcpyHostToDevice, st));
  HIPCHK(launch_svd_qr(svd_tab, (int)sv.size(), work, S, st));
  HIPCHK(launch_svd_qr_big(big_tab, (int)big.size(), bigcols_tab, (int)bigcols.size(), n_big_max, svd_tab, work, S,
                           st));
  // block-Jacobi sweeps until a sweep rotates nothing (per matrix).  The
  // workgroup table of a sweep lists the pairs of the still active matrices,
  // those with the most blocks first, so that step t launches only the
  // prefix of matrices that have a step t (nb - 1 > t).
  std::vector<double> active(T.sec.size(), 1.0), rot(T.sec.size(), 0.0);
  std::vector<int> order(T.sec.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return sv[a].nb > sv[b].nb; });
  std::vector<SvdPair> live;
  std::vector<int> prefix(nb_max > 1 ? nb_max - 1 : 0, 0);
  bool converged = false;
  for (int sweep = 0; sweep < kSvdMaxSweeps; ++sweep) {
    live.clear();
    std::fill(prefix.begin(), prefix.end(), 0);
    for (int si : order) {
      if (active[si] == 0.0) continue;
      for (int q = 0; q < sv[si].nb / 2; ++q) live.push_back(SvdPair{si, q});
      for (int t = 0; t < sv[si].nb - 1; ++t) prefix[t] = (int)live.size();
    }
    if (live.empty()) {
      converged = true;
      break;
    }
    HIPCHK(hipMemcpyAsync(pair_tab, live.data(), live.size() * sizeof(SvdPair), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(d_active, active.data(), active.size() * 8, hipMemcpyHostToDevice, st));
    HIPCHK(dav_fill_zero(d_rot, (int64_t)T.sec.size(), st));
    for (int step = 0; step < nb_max - 1; ++step)
      if (prefix[step] > 0)
        HIPCHK(launch_svd_bjac(pair_tab, prefix[step], svd_tab, work, d_active, d_rot, step, st));
    HIPCHK(hipMemcpyAsync(rot.data(), d_rot, rot.size() * 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    bool any = false;
    for (size_t i = 0; i < active.size(); ++i) {
      active[i] = (active[i] != 0.0 && rot[i] != 0.0) ? 1.0 : 0.0;
      any = any || active[i] != 0.0;
    }
    if (!any) {
      converged = true;
      break;
    }
  }
  // a matrix still rotating after the last sweep has singular values that
  // are not yet accurate: refuse to truncate with them
  if (!converged)
    throw Error{BSDMRG_ESOLVER, "truncate: block-Jacobi SVD still rotating after " + std::to_string(kSvdMaxSweeps) +
                                    " sweeps"};
  HIPCHK(launch_svd_finish(svd_tab, (int)sv.size(), cols_tab, (int)colblk.size(), work, U, S, V, st));
  std::vector<double> hS(T.n_s);
  HIPCHK(hipMemcpyAsync(hS.data(), S, T.n_s * 8, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  bool any_nonzero = false;
  for (double v : hS) {
    if (!std::isfinite(v)) throw Error{BSDMRG_ESOLVER, "truncate: non-finite singular value (theta not finite?)"};
    any_nonzero = any_nonzero || v != 0.0;
  }
  if (!any_nonzero) throw Error{BSDMRG_ESOLVER, "truncate: theta is zero (no singular vector to keep)"};
  std::vector<double> kept;
  std::vector<int64_t> counts = select_kept(T, hS, o, discarded, kept);
  // new leg and output layouts
  std::vector<int> new_of(T.sec.size(), -1);
  Leg b;
  b.nc = T.a.nc;
  for (size_t si = 0; si < T.sec.size(); ++si)
    if (counts[si] > 0) {
      new_of[si] = b.size();
      b.q.push_back(T.sec[si].q);
      b.d.push_back(counts[si]);
    }
  *new_n = b.size();
  *n_kept = (int64_t)kept.size();
  if (b.size() == 0) throw Error{BSDMRG_ESOLVER, "truncate: nothing kept (theta is zero?)"};
  Layout LA = make_layout({&T.a, &T.s1, &b}, kMpsS);
  Layout LB = make_layout({&b, &T.s2, &T.c}, kMpsS);
  *A_elems = LA.elems();
  *B_elems = LB.elems();
  if (leg_cap < b.size() || A_cap < LA.elems() || B_cap < LB.elems() || sv_cap < (int64_t)kept.size())
    throw Error{BSDMRG_ECAPACITY, "truncate: output capacity too small (required sizes returned)"};
  if (!A || !B || !svals) throw Error{BSDMRG_EINVAL, "truncate: NULL output"};
  for (int i = 0; i < b.size(); ++i) {
    for (int cc = 0; cc < b.nc; ++cc) new_q[i * b.nc + cc] = b.q[i][cc];
    new_d[i] = b.d[i];
  }
  std::copy(kept.begin(), kept.end(), svals);
  // gauge of every kept column
  std::vector<GaugeTask> gg;
  std::vector<int64_t> gbase(T.sec.size(), 0);
  for (size_t si = 0; si < T.sec.size(); ++si) {
    gbase[si] = (int64_t)gg.size();
    for (int64_t j = 0; j < counts[si]; ++j)
      gg.push_back(GaugeTask{T.sec[si].u + j * T.sec[si].rows, (int32_t)T.sec[si].rows,
                             (int32_t)T.sec[si].rows, (int32_t)(T.sec[si].s + j)});
  }
  for (const GaugeTask& g : gg)
    if (g.u_off < 0 || g.u_off + g.rows > T.n_u || g.s_idx < 0 || g.s_idx >= T.n_s || g.rows < 1)
      throw Error{BSDMRG_EINVAL, "internal table check failed: truncate gauge"};
  HIPCHK(hipMemcpyAsync(gauge_tab, gg.data(), gg.size() * sizeof(GaugeTask), hipMemcpyHostToDevice, st));
  HIPCHK(launch_gauge(gauge_tab, (int)gg.size(), U, S, sign, sgn_s, st));
  // scatter: A(a,s1,b) from U, B(b,s2,c) from V^T
  std::vector<CopyTask> ta, tb;
  for (size_t si = 0; si < T.sec.size(); ++si) {
    if (counts[si] == 0) continue;
    const TSector& s = T.sec[si];
    const int ib = new_of[si];
    const int32_t nq = (int32_t)counts[si];
    // A block (a, s1, b) row-major [i_a][i_1][j] from U rows r0 + i_a d1 + i_1
    for (size_t r = 0; r < s.rk.size(); ++r) {
      Key k{};
      k[0] = s.rk[r].first; k[1] = s.rk[r].second; k[2] = ib;
      const int blk = LA.lookup(k);
      if (blk < 0) throw Error{BSDMRG_EQN, "truncate: A block missing"};
      const int32_t d1 = (int32_t)T.s1.d[k[1]];
      for (int32_t i1 = 0; i1 < d1; ++i1)
        ta.push_back(CopyTask{s.u + s.r0[r] + i1, LA.offs[blk] + (int64_t)i1 * nq, (int32_t)T.a.d[k[0]], nq, d1,
                              (int32_t)s.rows, d1 * nq, 1, (int32_t)gbase[si], 0});
    }
    // B block (b, s2, c) row-major [j][i_2][i_c] from V^T columns c0 + i_2 dc + i_c
    for (size_t c = 0; c < s.ck.size(); ++c) {
      Key k{};
      k[0] = ib; k[1] = s.ck[c].first; k[2] = s.ck[c].second;
      const int blk = LB.lookup(k);
      if (blk < 0) throw Error{BSDMRG_EQN, "truncate: B block missing"};
      const int32_t bc = (int32_t)T.c.d[k[2]], d2 = (int32_t)T.s2.d[k[1]];
      for (int32_t i2 = 0; i2 < d2; ++i2)
        tb.push_back(CopyTask{s.v + (s.c0[c] + (int64_t)i2 * bc) * s.kmin, LB.offs[blk] + (int64_t)i2 * bc, nq, bc, 1,
                              (int32_t)s.kmin, d2 * bc, 1, (int32_t)gbase[si], 1});
    }
  }
  validate_copy(ta, T.n_u, LA.elems(), (int64_t)gg.size(), "truncate scatter A");
  validate_copy(tb, T.n_v, LB.elems(), (int64_t)gg.size(), "truncate scatter B");
  std::vector<CopyTask> all(ta);
  all.insert(all.end(), tb.begin(), tb.end());
  HIPCHK(hipMemcpyAsync(scatter_tab, all.data(), all.size() * sizeof(CopyTask), hipMemcpyHostToDevice, st));
  HIPCHK(dav_fill_zero(A, LA.elems(), st));
  HIPCHK(dav_fill_zero(B, LB.elems(), st));
  const bool right = o->direction == 0;
  HIPCHK(launch_copy(scatter_tab, (int)ta.size(), U, A, right ? sign : sgn_s, st));
  HIPCHK(launch_copy(scatter_tab + ta.size() * sizeof(CopyTask), (int)tb.size(), V, B, right ? sgn_s : sign, st));
  HIPCHK(hipStreamSynchronize(st));
}

}  // namespace bsd
