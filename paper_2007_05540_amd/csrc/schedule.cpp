// Tile schedule of a grouped-GEMM stage for the 8 XCDs of the MI355X.
//
// Workgroups of one launch are dispatched to the XCDs round-robin (workgroup
// i runs on XCD i mod 8) and every XCD has its own L2.  Tiles of one task
// share their A row panels and B column panels, so a task's tiles are kept on
// one XCD and run back to back there: the operand panels are fetched into
// that XCD's L2 once instead of once per XCD.  Tasks are distributed over
// the XCDs by longest-processing-time (LPT) bin packing on their cost
// (tiles x K); a task heavier than a quarter of an XCD's share is cut into
// row-panel chunks first.  Each XCD runs its chunks longest-K first, tiles of
// a chunk in row-panel order.  The per-XCD lists are interleaved into the
// launch order; shorter lists are padded with empty tiles (task = -1) that
// exit at once.  Tasks with M and N >= big_min are cut into 128 x 128 tiles,
// the others into 64 x 64 tiles.
#include <algorithm>
#include <numeric>

#include "bsdmrg_internal.h"
#include "kernels.h"

namespace bsd {

namespace {
constexpr int kXcd = 8;

struct Unit {
  int task, m_begin, m_end;   // row panels [m_begin, m_end) of the task (in tiles)
  double cost;
};
}  // namespace

void schedule_tiles(Stage& st, int32_t big_min) {
  st.tiles.clear();
  st.big_min = big_min;
  st.big = false;
  auto tsz = [&](const GemmTask& k) { return (k.M >= big_min && k.N >= big_min) ? 128 : 64; };
  std::vector<Unit> units;
  double total = 0.0;
  for (size_t t = 0; t < st.tasks.size(); ++t) {
    const GemmTask& k = st.tasks[t];
    const int ts = tsz(k);
    const int mt = std::max(1, (k.M + ts - 1) / ts), nt = std::max(1, (k.N + ts - 1) / ts);
    total += (double)mt * nt * (ts / 64) * (ts / 64) * (k.ksum + 16);
  }
  const double cap = std::max(1.0, total / (4.0 * kXcd));
  for (size_t t = 0; t < st.tasks.size(); ++t) {
    const GemmTask& k = st.tasks[t];
    const int ts = tsz(k);
    const int mt = std::max(1, (k.M + ts - 1) / ts), nt = std::max(1, (k.N + ts - 1) / ts);
    const double panel = (double)nt * (ts / 64) * (ts / 64) * (k.ksum + 16);
    const int per = std::max(1, (int)(cap / panel));
    for (int m = 0; m < mt; m += per) {
      const int e = std::min(mt, m + per);
      units.push_back(Unit{(int)t, m, e, panel * (e - m)});
    }
  }
  // LPT bin packing of the units over the XCDs
  std::vector<int> order(units.size());
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return units[a].cost > units[b].cost; });
  std::vector<double> load(kXcd, 0.0);
  std::vector<std::vector<int>> bins(kXcd);
  for (int u : order) {
    const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    bins[x].push_back(u);
    load[x] += units[u].cost;
  }
  // per XCD: chunks longest K first, tiles in row-panel order
  std::vector<std::vector<GemmTile>> lists(kXcd);
  size_t longest = 0;
  for (int x = 0; x < kXcd; ++x) {
    std::stable_sort(bins[x].begin(), bins[x].end(), [&](int a, int b) {
      return st.tasks[units[a].task].ksum > st.tasks[units[b].task].ksum;
    });
    for (int u : bins[x]) {
      const Unit& un = units[u];
      const GemmTask& k = st.tasks[un.task];
      const int ts = tsz(k);
      const int nt = std::max(1, (k.N + ts - 1) / ts);
      for (int m = un.m_begin; m < un.m_end; ++m)
        for (int n = 0; n < nt; ++n) lists[x].push_back(GemmTile{un.task, m * ts, n * ts, ts == 128 ? 1 : 0});
      if (ts == 128) st.big = true;
    }
    longest = std::max(longest, lists[x].size());
  }
  for (size_t q = 0; q < longest; ++q)
    for (int x = 0; x < kXcd; ++x)
      st.tiles.push_back(q < lists[x].size() ? lists[x][q] : GemmTile{-1, 0, 0, 0});
  // drop the empty tiles at the very end of the launch
  while (!st.tiles.empty() && st.tiles.back().task < 0) st.tiles.pop_back();
}

// The flattened tile table of a stage (its tasks, segments and tiles built).
void flatten_tiles(Stage& st) {
  st.ftiles.clear();
  st.ftiles.reserve(st.tiles.size());
  for (const GemmTile& t : st.tiles) {
    PTile r{};
    r.pad0 = t.task;
    if (t.task >= 0) {
      const GemmTask& k = st.tasks[t.task];
      r.c_off = k.c_off;
      r.m0 = t.m0;
      r.n0 = t.n0;
      r.M = k.M;
      r.N = k.N;
      r.ldc = k.ldc;
      r.cbuf = k.cbuf;
      r.seg0 = k.seg0;
      r.nseg = k.nseg;
      r.pad1 = t.shape;
      if (k.nseg > 0) r.first = st.segs[k.seg0];
    }
    st.ftiles.push_back(r);
  }
}

// Persistent schedule of a stage (64 x 64 tiles): slots_per_xcd workgroups
// per XCD, workgroup w on XCD w mod 8.  The tasks are spread over the XCDs
// as above (a task's tiles stay on one XCD: one L2 holds its panels); on each
// XCD the tiles are dealt longest first to the least loaded slot (LPT on
// k-slices plus a fixed per-tile cost), so the tiles of one task run at the
// same time on different slots and every slot ends at about the same time.
void schedule_persistent(Stage& st, int slots_per_xcd) {
  Stage flat;
  flat.tasks = st.tasks;
  schedule_tiles(flat, kNoBigTiles);   // the XCD binning, 64 x 64 tiles only
  std::vector<std::vector<GemmTile>> per_xcd(kXcd);
  for (size_t i = 0; i < flat.tiles.size(); ++i)
    if (flat.tiles[i].task >= 0) per_xcd[i % kXcd].push_back(flat.tiles[i]);
  const int S = std::max(1, slots_per_xcd);
  std::vector<std::vector<GemmTile>> slot_tiles((size_t)S * kXcd);
  for (int x = 0; x < kXcd; ++x) {
    auto& lst = per_xcd[x];
    auto cost = [&](const GemmTile& t) { return (double)st.tasks[t.task].ksum + 64.0; };
    std::stable_sort(lst.begin(), lst.end(), [&](const GemmTile& a, const GemmTile& b) { return cost(a) > cost(b); });
    std::vector<double> load(S, 0.0);
    for (const GemmTile& t : lst) {
      const int sl = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      load[sl] += cost(t);
      slot_tiles[(size_t)sl * kXcd + x].push_back(t);
    }
  }
  // drop trailing workgroups without tiles
  size_t n_wg = slot_tiles.size();
  while (n_wg > 0 && slot_tiles[n_wg - 1].empty()) --n_wg;
  st.ptiles.clear();
  st.wg_ptr.assign(1, 0);
  for (size_t w = 0; w < n_wg; ++w) {
    for (const GemmTile& t : slot_tiles[w]) {
      const GemmTask& k = st.tasks[t.task];
      PTile r{};
      r.c_off = k.c_off;
      r.m0 = t.m0;
      r.n0 = t.n0;
      r.M = k.M;
      r.N = k.N;
      r.ldc = k.ldc;
      r.cbuf = k.cbuf;
      r.seg0 = k.seg0;
      r.nseg = k.nseg;
      r.pad0 = t.task;   // for the table check
      if (k.nseg > 0) r.first = st.segs[k.seg0];
      st.ptiles.push_back(r);
    }
    st.wg_ptr.push_back((int32_t)st.ptiles.size());
  }
}

}  // namespace bsd
