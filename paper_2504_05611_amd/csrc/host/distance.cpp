// Circuit-level distance of a detector error model: the fewest mechanisms whose
// detector flips cancel while some observable flips (Results, "Circuit-level
// distance of distributed primitives", Table I reports upper bounds found by
// a search of this kind).
//
// Breadth-first search over states (detection events still active, observable
// mask), level k holding the states reachable with k mechanisms.  Level 1 is
// every single mechanism; a state grows only by mechanisms that touch its
// smallest active detector.  Every logical error set can be ordered that way
// (start from any of its members; the rest always contains one that touches
// the current smallest active detector), so with no cap on the active set the
// first empty state with a non-zero mask is a minimum-weight logical error.
// Capping the active set (max_active) keeps the state space small and turns
// the result into an upper bound.
#include <algorithm>
#include <cstring>
#include <string>
#include <unordered_set>
#include <vector>

#include "internal.h"

namespace tmcs {

tmcs_status dem_distance(const Dem& D, int max_active, int max_weight, int64_t max_states, int32_t* weight) {
  *weight = 0;
  if (D.obs_words != 1) return fail(TMCS_EUNSUPPORTED, "the distance search takes at most 64 observables");
  struct State { std::vector<int32_t> dets; uint64_t obs; };
  auto key_of = [](const State& s) {
    std::string k((const char*)s.dets.data(), s.dets.size() * sizeof(int32_t));
    k.append((const char*)&s.obs, sizeof(uint64_t));
    return k;
  };
  auto col_dets = [&](int j) {
    return std::vector<int32_t>(D.row_idx.begin() + D.col_ptr[j], D.row_idx.begin() + D.col_ptr[j + 1]);
  };
  std::unordered_set<std::string> seen;
  std::vector<State> level;
  for (int j = 0; j < D.cols; ++j) {
    State s{col_dets(j), D.obs_mask[j]};
    if (s.dets.empty()) {
      if (s.obs) { *weight = 1; return TMCS_OK; }
      continue;
    }
    if ((int)s.dets.size() > max_active) continue;
    if (seen.insert(key_of(s)).second) level.push_back(std::move(s));
  }
  int64_t states = (int64_t)level.size();
  for (int w = 2; w <= max_weight && !level.empty(); ++w) {
    std::vector<State> next;
    for (const State& s : level) {
      const int d0 = s.dets[0];
      for (int32_t e = D.row_ptr[d0]; e < D.row_ptr[d0 + 1]; ++e) {
        const int j = D.col_idx[e];
        State t;
        const std::vector<int32_t> c = col_dets(j);
        std::set_symmetric_difference(s.dets.begin(), s.dets.end(), c.begin(), c.end(), std::back_inserter(t.dets));
        t.obs = s.obs ^ D.obs_mask[j];
        if (t.dets.empty()) {
          if (t.obs) { *weight = w; return TMCS_OK; }
          continue;
        }
        if ((int)t.dets.size() > max_active) continue;
        if (!seen.insert(key_of(t)).second) continue;
        if (++states > max_states) return TMCS_OK;    // search budget spent: nothing found within it
        next.push_back(std::move(t));
      }
    }
    level.swap(next);
  }
  return TMCS_OK;
}

}  // namespace tmcs
