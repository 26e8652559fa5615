// Compile a circuit into the layered instruction stream of the frame kernel.
//
// Measurement records are never stored: every record is XORed, as soon as it
// is measured, into the accumulator slots of the detectors and observables that
// contain it and into a private slot when a classically controlled Pauli reads
// it.  A detector's slot lives from its first record to its DETECTOR
// instruction, where it is written out and cleared; observables are written at
// the end.  Slots are assigned by a first-free allocator in program order, so
// the number of slots is the peak number of live accumulators.
#include <algorithm>
#include <cmath>
#include <set>

#include "program.h"

namespace tmcs {

namespace {

struct Emitter {
  Program* P;
  void layer(int32_t kind, const std::vector<int32_t>& items) {
    const int w = layer_item_width(kind);
    if (items.empty()) return;
    // split so that no frame qubit (or slot for FEED/CLEAR) repeats within a layer
    std::set<int32_t> used;
    std::vector<int32_t> cur;
    auto flush = [&]() {
      if (cur.empty()) return;
      P->layers.push_back(kind);
      P->layers.push_back((int32_t)cur.size() / w);
      P->layers.push_back((int32_t)P->data.size());
      P->data.insert(P->data.end(), cur.begin(), cur.end());
      P->num_layers++;
      cur.clear();
      used.clear();
    };
    for (size_t i = 0; i < items.size(); i += w) {
      std::vector<int32_t> keys;
      switch (kind) {
        case L_RESET: case L_H: keys = {items[i]}; break;
        case L_CX: keys = {items[i], items[i + 1]}; break;
        case L_MEAS: keys = {items[i]}; break;
        case L_FEED: keys = {items[i + 1]}; break;
        case L_NOISE: keys = {items[i + 2]}; if (items[i + 3] >= 0) keys.push_back(items[i + 3]); break;
        default: keys = {}; break;
      }
      bool clash = false;
      for (int32_t k : keys) clash |= used.count(k) > 0;
      if (clash) flush();
      for (int32_t k : keys) used.insert(k);
      cur.insert(cur.end(), items.begin() + i, items.begin() + i + w);
    }
    flush();
  }
};

}  // namespace

tmcs_status compile_program(const Circuit& c, Program* P) {
  const int nd = c.num_dets, no = c.num_obs;
  // targets: detector d -> d; observable o -> nd + o; feedback record r -> nd + no + j
  std::vector<std::vector<int32_t>> rec_targets(c.num_meas);
  std::vector<int32_t> fb_target(c.num_meas, -1);
  std::vector<int32_t> fb_last_op(c.num_meas, -1);
  int nfb = 0;
  {
    int ndet = 0;
    for (size_t i = 0; i < c.ops.size(); ++i) {
      const Op& op = c.ops[i];
      if (op.kind == OP_DET) {
        for (int32_t r : op.t) rec_targets[r].push_back(ndet);
        ++ndet;
      } else if (op.kind == OP_OBS) {
        for (int32_t r : op.t) rec_targets[r].push_back(nd + op.obs);
      } else if (op.kind == OP_CXREC || op.kind == OP_CZREC) {
        for (size_t k = 0; k + 1 < op.t.size(); k += 2) {
          const int32_t r = op.t[k];
          if (fb_target[r] < 0) {
            fb_target[r] = nd + no + nfb++;
            rec_targets[r].push_back(fb_target[r]);
          }
          fb_last_op[r] = (int32_t)i;
        }
      }
    }
  }
  // A record listed twice by one detector cancels; keep odd multiplicities only.
  for (auto& v : rec_targets) {
    std::sort(v.begin(), v.end());
    std::vector<int32_t> odd;
    for (size_t i = 0; i < v.size();) {
      size_t j = i;
      while (j < v.size() && v[j] == v[i]) ++j;
      if ((j - i) & 1) odd.push_back(v[i]);
      i = j;
    }
    v.swap(odd);
  }
  std::vector<int32_t> slot_of(nd + no + nfb, -1);
  std::vector<int32_t> free_slots;
  int next = 0;
  auto alloc = [&]() {
    if (!free_slots.empty()) { int s = free_slots.back(); free_slots.pop_back(); return s; }
    return next++;
  };
  Emitter E{P};
  int nm = 0, ndet = 0;
  int64_t site = 0;
  std::vector<double> tab;
  auto tab_index = [&](double p) {
    for (size_t i = 0; i < tab.size(); ++i)
      if (tab[i] == p) return (int)i;
    tab.push_back(p);
    return (int)tab.size() - 1;
  };
  size_t i = 0;
  while (i < c.ops.size()) {
    const Op& op = c.ops[i];
    std::vector<int32_t> items;
    switch (op.kind) {
      case OP_R:
      case OP_RX:
      case OP_BELL:
        E.layer(L_RESET, op.t);
        break;
      case OP_H:
        E.layer(L_H, op.t);
        break;
      case OP_CX:
        E.layer(L_CX, op.t);
        break;
      case OP_M:
      case OP_MX:
        for (int32_t q : op.t) {
          const int r = nm++;
          if (rec_targets[r].empty()) continue;   // a record nobody reads
          const int32_t s0 = (int32_t)P->mslots.size();
          for (int32_t t : rec_targets[r]) {
            if (slot_of[t] < 0) slot_of[t] = alloc();
            P->mslots.push_back(slot_of[t]);
          }
          items.insert(items.end(), {q, op.kind == OP_MX ? 1 : 0, s0, (int32_t)P->mslots.size()});
        }
        E.layer(L_MEAS, items);
        break;
      case OP_CXREC:
      case OP_CZREC: {
        std::vector<int32_t> clear;
        for (size_t k = 0; k + 1 < op.t.size(); k += 2) {
          const int32_t r = op.t[k];
          items.insert(items.end(), {slot_of[fb_target[r]], op.t[k + 1], op.kind == OP_CXREC ? 1 : 3});
        }
        E.layer(L_FEED, items);
        for (size_t k = 0; k + 1 < op.t.size(); k += 2) {
          const int32_t r = op.t[k];
          if (fb_last_op[r] == (int32_t)i && slot_of[fb_target[r]] >= 0) {
            clear.push_back(slot_of[fb_target[r]]);
            free_slots.push_back(slot_of[fb_target[r]]);
            slot_of[fb_target[r]] = -2;
          }
        }
        E.layer(L_CLEAR, clear);
        break;
      }
      case OP_XERR:
      case OP_ZERR:
      case OP_DEP1:
      case OP_DEP2: {
        // one noise layer (split only where a qubit repeats) for a run of
        // consecutive noise instructions: Pauli events commute, and the run's
        // sites stay consecutive
        auto is_noise = [](OpKind k) { return k == OP_XERR || k == OP_ZERR || k == OP_DEP1 || k == OP_DEP2; };
        while (i < c.ops.size() && is_noise(c.ops[i].kind)) {
          const Op& nop = c.ops[i];
          const int g = nop.kind == OP_DEP2 ? 2 : 1;
          const NoiseKind nk = nop.kind == OP_XERR ? NK_XERR : nop.kind == OP_ZERR ? NK_ZERR
                             : nop.kind == OP_DEP1 ? NK_DEP1 : NK_DEP2;
          const int ti = tab_index(nop.p);
          for (size_t k = 0; k < nop.t.size(); k += g) {
            items.insert(items.end(), {(int32_t)site, (int32_t)nk, nop.t[k], g == 2 ? nop.t[k + 1] : -1});
            P->site_kind.push_back((uint8_t)nk);
            P->site_tab.push_back((uint16_t)ti);
            P->events_per_shot += nop.p;
            ++site;
          }
          ++i;
        }
        E.layer(L_NOISE, items);
        continue;
      }
      case OP_DET: {
        // one EMIT layer for a run of consecutive DETECTOR instructions
        std::vector<int32_t> freed;
        while (i < c.ops.size() && c.ops[i].kind == OP_DET) {
          const int32_t s = slot_of[ndet];
          if (s < 0) return fail(TMCS_EINVAL, "detector without records");
          items.insert(items.end(), {s, ndet});
          freed.push_back(s);
          slot_of[ndet] = -2;
          ++ndet;
          ++i;
        }
        E.layer(L_EMIT, items);
        for (int32_t s : freed) free_slots.push_back(s);
        continue;
      }
      default:
        break;
    }
    ++i;
  }
  std::vector<int32_t> obs_items;
  for (int o = 0; o < no; ++o) {
    if (slot_of[nd + o] < 0) {
      // an observable without records is identically zero: give it a fresh slot
      slot_of[nd + o] = alloc();
    }
    obs_items.insert(obs_items.end(), {slot_of[nd + o], -(o + 1)});
  }
  E.layer(L_EMIT, obs_items);
  P->nslots = next;
  P->tab_p = tab;
  if (tab.size() > 65535) return fail(TMCS_EUNSUPPORTED, "too many distinct noise strengths");
  return TMCS_OK;
}

}  // namespace tmcs
