// Legs and the canonical block layout (quantum-number block form, Sec. II-D;
// list format, Sec. IV-A).  Pure host code.
#include <algorithm>
#include <cstring>

#include "bsdmrg_internal.h"

namespace bsd {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }
const char* last_error_cstr() { return g_last_error.c_str(); }

int Leg::find(const Charge& c) const {
  auto it = std::lower_bound(q.begin(), q.end(), c);
  if (it == q.end() || *it != c) return -1;
  return (int)(it - q.begin());
}

Leg leg_from(const bsdmrg_leg& l) {
  if (l.n_sectors < 1 || l.n_charges < 1 || l.n_charges > 2 || !l.charges || !l.dims)
    throw Error{BSDMRG_EINVAL, "leg: need n_sectors >= 1, 1 <= n_charges <= 2, non-null arrays"};
  Leg out;
  out.nc = l.n_charges;
  for (int i = 0; i < l.n_sectors; ++i) {
    Charge c{0, 0};
    for (int j = 0; j < l.n_charges; ++j) c[j] = l.charges[i * l.n_charges + j];
    if (l.dims[i] < 1) throw Error{BSDMRG_EQN, "leg: sector dimension < 1"};
    if (i > 0 && !(out.q.back() < c)) throw Error{BSDMRG_EQN, "leg: charges not strictly ascending"};
    out.q.push_back(c);
    out.d.push_back(l.dims[i]);
  }
  return out;
}

// All allowed sector tuples in lexicographic order.  The first order-1 legs
// are enumerated; the charge rule fixes the last leg's charge, found by
// binary search, so the order stays lexicographic.
Layout make_layout(const std::vector<const Leg*>& legs, const int32_t* signs) {
  Layout L;
  const int n = (int)legs.size();
  if (n < 1 || n > kMaxOrder) throw Error{BSDMRG_EINVAL, "layout: order must be 1..8"};
  const int nc = legs[0]->nc;
  for (auto* l : legs)
    if (l->nc != nc) throw Error{BSDMRG_EINVAL, "layout: legs disagree on charge components"};
  for (int i = 0; i < n; ++i)
    if (signs[i] != 1 && signs[i] != -1) throw Error{BSDMRG_EINVAL, "layout: signs must be +-1"};
  L.order = n;
  L.offs.push_back(0);
  Key key{};
  std::vector<int> idx(n, 0);
  if (n == 1) {
    for (int s = 0; s < legs[0]->size(); ++s) {
      bool ok = true;
      for (int c = 0; c < nc; ++c) ok = ok && legs[0]->q[s][c] == 0;
      if (!ok) continue;
      key[0] = s;
      L.index[key] = (int)L.keys.size();
      L.keys.push_back(key);
      L.offs.push_back(L.offs.back() + round_up(legs[0]->d[s]));
    }
    return L;
  }
  while (true) {
    Charge need{0, 0};
    for (int i = 0; i < n - 1; ++i)
      for (int c = 0; c < nc; ++c) need[c] -= signs[i] * legs[i]->q[idx[i]][c];
    for (int c = 0; c < nc; ++c) need[c] *= signs[n - 1];   // sign_last * q_last = need
    int last = legs[n - 1]->find(need);
    if (last >= 0) {
      int64_t size = 1;
      for (int i = 0; i < n - 1; ++i) { key[i] = idx[i]; size *= legs[i]->d[idx[i]]; }
      key[n - 1] = last;
      size *= legs[n - 1]->d[last];
      L.index[key] = (int)L.keys.size();
      L.keys.push_back(key);
      L.offs.push_back(L.offs.back() + round_up(size));
    }
    int j = n - 2;
    while (j >= 0) {
      if (++idx[j] < legs[j]->size()) break;
      idx[j] = 0;
      --j;
    }
    if (j < 0) break;
  }
  return L;
}

}  // namespace bsd
