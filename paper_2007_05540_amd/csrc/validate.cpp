// Host-side checks that every index table stays inside its buffers.  Run
// when a plan is built (and on the truncation tables before upload); a
// violation raises an error instead of launching a kernel that would read
// or write out of bounds.
#include <cstring>
#include <string>

#include "bsdmrg_internal.h"
#include "kernels.h"

namespace bsd {

static void fail(const std::string& what) { throw Error{BSDMRG_EINVAL, "internal table check failed: " + what}; }

void validate_gemm(const Stage& st, int layout, int64_t a_elems, int64_t b_elems, int64_t c_elems,
                   int64_t cpart_elems, const char* name) {
  for (size_t t = 0; t < st.tasks.size(); ++t) {
    const GemmTask& k = st.tasks[t];
    if (k.M < 1 || k.N < 1 || k.nseg < 0 || k.seg0 < 0 || k.seg0 + k.nseg > (int64_t)st.segs.size())
      fail(std::string(name) + ": task shape");
    if (k.N > k.ldc) fail(std::string(name) + ": ldc");
    const int64_t cl = k.cbuf ? cpart_elems : c_elems;
    if (k.c_off < 0 || k.c_off + (int64_t)(k.M - 1) * k.ldc + k.N > cl) fail(std::string(name) + ": C extent");
    int64_t ks = 0;
    for (int j = 0; j < k.nseg; ++j) {
      const GemmSeg& g = st.segs[k.seg0 + j];
      if (g.K < 1) fail(std::string(name) + ": K");
      ks += g.K;
      if (layout == kTN) {
        if (k.M > g.lda || g.a_off < 0 || g.a_off + (int64_t)(g.K - 1) * g.lda + k.M > a_elems)
          fail(std::string(name) + ": A extent (TN)");
      } else {
        if (g.K > g.lda || g.a_off < 0 || g.a_off + (int64_t)(k.M - 1) * g.lda + g.K > a_elems)
          fail(std::string(name) + ": A extent");
      }
      if (layout == kNT) {
        if (g.K > g.ldb || g.b_off < 0 || g.b_off + (int64_t)(k.N - 1) * g.ldb + g.K > b_elems)
          fail(std::string(name) + ": B extent (NT)");
      } else {
        if (k.N > g.ldb || g.b_off < 0 || g.b_off + (int64_t)(g.K - 1) * g.ldb + k.N > b_elems)
          fail(std::string(name) + ": B extent");
      }
    }
    if (ks != k.ksum) fail(std::string(name) + ": ksum");
    // the GEMM kernel reads a block through a buffer resource whose length in
    // bytes is a 31-bit number, with 32-bit byte offsets (8-byte elements)
    for (int j = 0; j < k.nseg; ++j) {
      const GemmSeg& g = st.segs[k.seg0 + j];
      const int64_t ea = layout == kTN ? (int64_t)(g.K - 1) * g.lda + k.M : (int64_t)(k.M - 1) * g.lda + g.K;
      const int64_t eb = layout == kNT ? (int64_t)(k.N - 1) * g.ldb + g.K : (int64_t)(g.K - 1) * g.ldb + k.N;
      if (ea > (int64_t)0x0FFFFFFF || eb > (int64_t)0x0FFFFFFF) fail(std::string(name) + ": block above 2^28 elements");
    }
  }
  validate_tiles(st, name);
}

void validate_tiles(const Stage& st, const char* name) {
  for (const GemmTile& tl : st.tiles) {
    if (tl.task == -1) continue;   // empty tile of the XCD schedule
    if (tl.task < 0 || tl.task >= (int64_t)st.tasks.size()) fail(std::string(name) + ": tile task");
    const GemmTask& k = st.tasks[tl.task];
    if (tl.m0 < 0 || tl.m0 >= k.M || tl.n0 < 0 || tl.n0 >= k.N) fail(std::string(name) + ": tile origin");
    if (tl.shape != 0 && !(tl.shape == 1 && st.big)) fail(std::string(name) + ": tile shape");
  }
  // the flattened table (when built) repeats each tile with its task's
  // fields and first segment
  if (st.ftiles.empty()) return;
  if (st.ftiles.size() != st.tiles.size()) fail(std::string(name) + ": flattened tile count");
  for (size_t i = 0; i < st.tiles.size(); ++i) {
    const GemmTile& tl = st.tiles[i];
    const PTile& r = st.ftiles[i];
    if (r.pad0 != tl.task) fail(std::string(name) + ": flattened tile task");
    if (tl.task < 0) continue;
    const GemmTask& k = st.tasks[tl.task];
    if (r.c_off != k.c_off || r.M != k.M || r.N != k.N || r.ldc != k.ldc || r.cbuf != k.cbuf || r.seg0 != k.seg0 ||
        r.nseg != k.nseg || r.m0 != tl.m0 || r.n0 != tl.n0 || r.pad1 != tl.shape)
      fail(std::string(name) + ": flattened tile record");
    if (k.nseg > 0 && std::memcmp(&r.first, &st.segs[k.seg0], sizeof(GemmSeg)) != 0)
      fail(std::string(name) + ": flattened tile first segment");
  }
}

// The persistent schedule covers every 64 x 64 tile of every task exactly
// once, and every record repeats its task's fields and first segment.
void validate_ptiles(const Stage& st, const char* name) {
  if (st.wg_ptr.empty() || st.wg_ptr.front() != 0 || st.wg_ptr.back() != (int32_t)st.ptiles.size())
    fail(std::string(name) + ": persistent workgroup table");
  for (size_t w = 0; w + 1 < st.wg_ptr.size(); ++w)
    if (st.wg_ptr[w] > st.wg_ptr[w + 1]) fail(std::string(name) + ": persistent workgroup order");
  int64_t expect = 0;
  for (const GemmTask& k : st.tasks) expect += (int64_t)((k.M + 63) / 64) * ((k.N + 63) / 64);
  if ((int64_t)st.ptiles.size() != expect) fail(std::string(name) + ": persistent tile count");
  std::vector<std::vector<char>> seen(st.tasks.size());
  for (size_t t = 0; t < st.tasks.size(); ++t)
    seen[t].assign((size_t)((st.tasks[t].M + 63) / 64) * ((st.tasks[t].N + 63) / 64), 0);
  for (const PTile& r : st.ptiles) {
    if (r.pad0 < 0 || r.pad0 >= (int32_t)st.tasks.size()) fail(std::string(name) + ": persistent tile task");
    const GemmTask& k = st.tasks[r.pad0];
    if (r.c_off != k.c_off || r.M != k.M || r.N != k.N || r.ldc != k.ldc || r.cbuf != k.cbuf || r.seg0 != k.seg0 ||
        r.nseg != k.nseg)
      fail(std::string(name) + ": persistent tile record");
    if (r.m0 < 0 || r.m0 >= k.M || r.n0 < 0 || r.n0 >= k.N || r.m0 % 64 || r.n0 % 64)
      fail(std::string(name) + ": persistent tile origin");
    if (k.nseg > 0 && std::memcmp(&r.first, &st.segs[k.seg0], sizeof(GemmSeg)) != 0)
      fail(std::string(name) + ": persistent tile first segment");
    char& f = seen[r.pad0][(size_t)(r.m0 / 64) * ((k.N + 63) / 64) + r.n0 / 64];
    if (f) fail(std::string(name) + ": persistent tile repeated");
    f = 1;
  }
}

void validate_mix(const std::vector<MixTask>& tasks, const std::vector<MixTerm>& terms,
                  const std::vector<MixItem>& items, int64_t src_elems, int64_t dst_elems, int64_t coef_elems,
                  const char* name, int64_t item_max) {
  for (const MixTask& t : tasks) {
    if (t.rows < 1 || t.cols < 1 || t.cols > t.ld_dst || t.dst_off < 0 ||
        t.dst_off + (int64_t)(t.rows - 1) * t.ld_dst + t.cols > dst_elems)
      fail(std::string(name) + ": dst extent");
    if (t.term0 < 0 || t.nterm < 0 || t.term0 + t.nterm > (int64_t)terms.size()) fail(std::string(name) + ": terms");
    for (int j = 0; j < t.nterm; ++j) {
      const MixTerm& m = terms[t.term0 + j];
      if (t.cols > m.ld_src || m.src_off < 0 || m.src_off + (int64_t)(t.rows - 1) * m.ld_src + t.cols > src_elems)
        fail(std::string(name) + ": src extent");
      // the mixing kernel addresses a source block with 32-bit byte offsets
      if ((int64_t)(t.rows - 1) * m.ld_src + t.cols > ((int64_t)1 << 29))
        fail(std::string(name) + ": source block above 2^29 elements");
      if (coef_elems >= 0 && (m.coef < 0 || m.coef >= coef_elems)) fail(std::string(name) + ": coef index");
    }
  }
  for (const MixItem& it : items) {
    if (it.task < 0 || it.task >= (int64_t)tasks.size()) fail(std::string(name) + ": item task");
    const MixTask& t = tasks[it.task];
    if (it.row0 < 0 || it.nrows < 1 || it.row0 + it.nrows > t.rows || (int64_t)it.nrows * t.cols > item_max)
      fail(std::string(name) + ": item rows");
  }
}

void validate_copy(const std::vector<CopyTask>& tasks, int64_t src_elems, int64_t dst_elems, int64_t fac_elems,
                   const char* name) {
  for (const CopyTask& t : tasks) {
    if (t.rows < 1 || t.cols < 1) fail(std::string(name) + ": shape");
    const int64_t s_last = t.src_off + (int64_t)(t.rows - 1) * t.src_rs + (int64_t)(t.cols - 1) * t.src_cs;
    const int64_t d_last = t.dst_off + (int64_t)(t.rows - 1) * t.dst_rs + (int64_t)(t.cols - 1) * t.dst_cs;
    if (t.src_off < 0 || s_last >= src_elems) fail(std::string(name) + ": src extent");
    if (t.dst_off < 0 || d_last >= dst_elems) fail(std::string(name) + ": dst extent");
    if (t.fac_off >= 0 && t.fac_off + (t.fac_on_rows ? t.rows : t.cols) > fac_elems)
      fail(std::string(name) + ": factor extent");
  }
}

void validate_heff_plan(const bsdmrg_plan_s* P) {
  validate_gemm(P->s1, kNN, P->L_elems, P->psi_elems, P->t1_elems, 0, "S1");
  validate_gemm(P->s3, kNT, P->t2_elems, P->R_elems, P->psi_elems, P->s3_part_elems, "S3");
  // the launches of S2 and of the split-K sums process 256 * mix_per outputs per workgroup
  validate_mix(P->mix_tasks, P->mix_terms, P->mix_items, P->t1_elems, P->t2_elems, P->n_coefs, "S2",
               256 * P->mix_per);
  validate_mix(P->red_tasks, P->red_terms, P->red_items, P->s3_part_elems, P->psi_elems, -1, "S3 reduce",
               256 * P->mix_per);
  for (size_t i = 0; i + 1 < P->coef_ptr.size(); ++i)
    for (int32_t k = P->coef_ptr[i]; k < P->coef_ptr[i + 1]; ++k)
      if (P->coef_e1[k] < 0 || P->coef_e1[k] >= P->W1_elems || P->coef_e2[k] < 0 || P->coef_e2[k] >= P->W2_elems)
        fail("WW coefficient pairs");
  for (const Chunk& c : P->chunks)
    if (c.start < 0 || c.len < 1 || c.len > kChunk || c.start + c.len > P->psi_elems) fail("chunks");
  for (size_t p = 0; p < P->dav_probs.size(); ++p) {
    const DavProb& d = P->dav_probs[p];
    if (d.base < 0 || d.base + d.len > P->psi_elems) fail("problem range");
    for (int32_t b = P->blk_ptr[p]; b < P->blk_ptr[p + 1]; ++b)
      if (P->blk_off[2 * b] < 0 || P->blk_off[2 * b] + P->blk_off[2 * b + 1] > d.len) fail("psi block table");
  }
  // diagonal tasks: every element read or written stays inside its buffer
  for (const DiagTask& t : P->diag_tasks) {
    if (t.rows < 1 || t.cols < 1 || t.nl < 1 || t.nm < 1 || t.nr < 1 || t.nl > kMaxDiagChannels ||
        t.nr > kMaxDiagChannels || t.row0 < 0 || t.nrow < 1 || t.row0 + t.nrow > t.rows ||
        (int64_t)t.nrow * t.cols > 4096)
      fail("diagonal task shape");
    if (t.psi_off < 0 || t.psi_off + (int64_t)t.rows * t.cols > P->psi_elems) fail("diagonal task psi range");
    if (t.l_off < 0 || t.l_off + (int64_t)t.rows * t.nl * t.rows > P->L_elems) fail("diagonal task L range");
    if (t.r_off < 0 || t.r_off + (int64_t)t.cols * t.nr * t.cols > P->R_elems) fail("diagonal task R range");
    if (t.w1_off < 0 || t.w1_off + (int64_t)t.nl * t.nm > P->W1_elems) fail("diagonal task W1 range");
    if (t.w2_off < 0 || t.w2_off + (int64_t)t.nm * t.nr > P->W2_elems) fail("diagonal task W2 range");
  }
}

}  // namespace bsd
