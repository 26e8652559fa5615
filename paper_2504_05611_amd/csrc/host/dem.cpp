// Detector error model by a backward sensitivity sweep.
//
// Walking the circuit from its end to its start, the library keeps for every
// qubit the set of outputs (detectors, then observables) that an X error, and
// a Z error, at the current point would flip, and for every measurement record
// the set of outputs its flip would flip.  The rules are the adjoint of the
// Pauli-frame rules:
//   DETECTOR / OBSERVABLE_INCLUDE : add the output to each of its records
//   CX rec -> q (conditional X)   : record r also flips sensX[q] (Z: sensZ[q])
//   M q  (record r)               : sensX[q] ^= rec[r]    (MX: sensZ[q] ^= rec[r])
//   R / RX / Bell preparation     : sensX[q] = sensZ[q] = {} (earlier errors erased)
//   H q                           : swap sensX[q], sensZ[q]
//   CX c t                        : sensX[c] ^= sensX[t]; sensZ[t] ^= sensZ[c]
// At a noise site, each Pauli component's symptom is the XOR of the
// sensitivities of its X and Z parts.  This yields every single-fault symptom
// in one pass over the circuit (the paper's DEM columns: one per distinct
// mechanism, Methods "Decoding" and Table III).
//
// Each channel is split into independent mechanisms with the same output
// distribution: X_ERROR/Z_ERROR one mechanism of probability p; DEPOLARIZE1 three
// of q1 = (1 - sqrt(1 - 4p/3))/2; DEPOLARIZE2 fifteen of
// q2 = (1 - (1 - 16p/15)^(1/8))/2, the eighth root taken as three square roots.
// Identical symptoms are merged in circuit order (site, then component) with
// p <- pa + pb - 2 pa pb; empty symptoms are dropped and observable-only
// symptoms (undetectable logical errors) are counted and excluded.  Columns are
// sorted by (detector list, observable mask) lexicographically.
//
// The same sweep checks that every detector and observable is deterministic in
// the noiseless circuit (Methods, "Simulation": detectors compare stabilizer
// measurements whose noiseless values agree).  Read backwards, an output is the
// outcome of a Pauli P times records; sensX[q] holds the outputs whose P
// anticommutes with X_q (a Z or Y on q) and sensZ[q] those whose P has an X or
// Y on q.  The output is random when P anticommutes with the operator that a
// reset prepares or a measurement measures at that point:
//   R q / M q (Z basis)  : outputs in sensZ[q];   RX q / MX q : outputs in sensX[q]
//   Bell pair (a, b)     : P restricted to (a, b) must lie in {II, XX, YY, ZZ},
//                          so sensX[a] = sensX[b] and sensZ[a] = sensZ[b]
//   start (all |0>)      : outputs in sensZ[q]
// Such a circuit is rejected with TMCS_ENONDETERMINISTIC.
#include <algorithm>
#include <cmath>
#include <string>
#include <unordered_map>

#include "internal.h"

namespace tmcs {

int channel_components(OpKind k) {
  switch (k) {
    case OP_XERR:
    case OP_ZERR: return 1;
    case OP_DEP1: return 3;
    case OP_DEP2: return 15;
    default: return 0;
  }
}

double mechanism_prob(OpKind k, double p) {
  switch (k) {
    case OP_XERR:
    case OP_ZERR: return p;
    case OP_DEP1: return (1.0 - std::sqrt(1.0 - 4.0 * p / 3.0)) / 2.0;
    case OP_DEP2: return (1.0 - std::sqrt(std::sqrt(std::sqrt(1.0 - 16.0 * p / 15.0)))) / 2.0;
    default: return 0.0;
  }
}

namespace {

using Set = std::vector<int32_t>;  // sorted, distinct

void sym_into(Set& a, const Set& b) {
  if (b.empty()) return;
  Set out;
  out.reserve(a.size() + b.size());
  size_t i = 0, j = 0;
  while (i < a.size() && j < b.size()) {
    if (a[i] < b[j]) out.push_back(a[i++]);
    else if (b[j] < a[i]) out.push_back(b[j++]);
    else { ++i; ++j; }
  }
  while (i < a.size()) out.push_back(a[i++]);
  while (j < b.size()) out.push_back(b[j++]);
  a.swap(out);
}

struct SetHash {
  size_t operator()(const Set& s) const {
    uint64_t h = 1469598103934665603ull;
    for (int32_t x : s) { h ^= (uint64_t)(uint32_t)x; h *= 1099511628211ull; }
    return (size_t)h;
  }
};

// Pauli on the first and second target of component c of channel k
// (0 = I, 1 = X, 2 = Y, 3 = Z): DEPOLARIZE1 c -> c+1; DEPOLARIZE2 c+1 = 4a + b.
void component_paulis(OpKind k, int c, int* a, int* b) {
  *b = 0;
  if (k == OP_XERR) *a = 1;
  else if (k == OP_ZERR) *a = 3;
  else if (k == OP_DEP1) *a = c + 1;
  else { *a = (c + 1) >> 2; *b = (c + 1) & 3; }
}

}  // namespace

tmcs_status build_dem(const Circuit& c, Dem* d) {
  const int Q = c.num_qubits;
  const int nd = c.num_dets;
  std::vector<Set> sx(Q), sz(Q), rec(c.num_meas);
  // record indices of measurement instructions, found by a forward count
  std::vector<int32_t> first_rec(c.ops.size(), 0), first_det(c.ops.size(), 0);
  std::vector<int64_t> first_site(c.ops.size(), 0);
  {
    int nm = 0, ndet = 0;
    int64_t ns = 0;
    for (size_t i = 0; i < c.ops.size(); ++i) {
      const Op& op = c.ops[i];
      first_rec[i] = nm;
      first_det[i] = ndet;
      first_site[i] = ns;
      if (op.kind == OP_M || op.kind == OP_MX) nm += (int)op.t.size();
      if (op.kind == OP_DET) ndet += 1;
      const int K = channel_components(op.kind);
      if (K) ns += (int64_t)op.t.size() / (op.kind == OP_DEP2 ? 2 : 1);
    }
  }
  // channel table: (kind, p) -> id, so contributions are stored compactly
  std::vector<std::pair<OpKind, double>> chans;
  auto chan_id = [&](OpKind k, double p) {
    for (size_t i = 0; i < chans.size(); ++i)
      if (chans[i].first == k && chans[i].second == p) return (int)i;
    chans.push_back({k, p});
    return (int)chans.size() - 1;
  };
  // outputs (detectors, then observables) found random in the noiseless circuit
  std::vector<char> nondet((size_t)nd + (size_t)std::max(c.num_obs, 0), 0);
  auto mark = [&](const Set& s) { for (int32_t x : s) nondet[x] = 1; };
  auto mark_diff = [&](const Set& a, const Set& b) { Set t = a; sym_into(t, b); mark(t); };
  std::unordered_map<Set, int32_t, SetHash> index;
  std::vector<Set> symptoms;
  std::vector<std::vector<uint16_t>> contrib;  // per symptom: channel ids, reverse circuit order

  for (size_t ii = c.ops.size(); ii-- > 0;) {
    const Op& op = c.ops[ii];
    switch (op.kind) {
      case OP_DET: {
        const int32_t det = first_det[ii];
        for (int32_t r : op.t) sym_into(rec[r], Set{det});
        break;
      }
      case OP_OBS:
        for (int32_t r : op.t) sym_into(rec[r], Set{nd + op.obs});
        break;
      case OP_CXREC:
        for (size_t i = 0; i + 1 < op.t.size(); i += 2) sym_into(rec[op.t[i]], sx[op.t[i + 1]]);
        break;
      case OP_CZREC:
        for (size_t i = 0; i + 1 < op.t.size(); i += 2) sym_into(rec[op.t[i]], sz[op.t[i + 1]]);
        break;
      case OP_M:
        for (size_t i = 0; i < op.t.size(); ++i) {
          mark(sz[op.t[i]]);
          sym_into(sx[op.t[i]], rec[first_rec[ii] + i]);
        }
        break;
      case OP_MX:
        for (size_t i = 0; i < op.t.size(); ++i) {
          mark(sx[op.t[i]]);
          sym_into(sz[op.t[i]], rec[first_rec[ii] + i]);
        }
        break;
      case OP_R:
      case OP_RX:
        for (int32_t q : op.t) {
          mark(op.kind == OP_R ? sz[q] : sx[q]);
          sx[q].clear();
          sz[q].clear();
        }
        break;
      case OP_BELL:
        for (size_t i = 0; i + 1 < op.t.size(); i += 2) {
          const int32_t a = op.t[i], b = op.t[i + 1];
          mark_diff(sx[a], sx[b]);
          mark_diff(sz[a], sz[b]);
          sx[a].clear(); sz[a].clear(); sx[b].clear(); sz[b].clear();
        }
        break;
      case OP_H:
        for (int32_t q : op.t) sx[q].swap(sz[q]);
        break;
      case OP_CX:
        for (size_t i = 0; i + 1 < op.t.size(); i += 2) {
          const int32_t a = op.t[i], b = op.t[i + 1];
          Set tx = sx[b];
          sym_into(sx[a], tx);
          Set tz = sz[a];
          sym_into(sz[b], tz);
        }
        break;
      case OP_XERR:
      case OP_ZERR:
      case OP_DEP1:
      case OP_DEP2: {
        const int K = channel_components(op.kind);
        const int g = op.kind == OP_DEP2 ? 2 : 1;
        const int cid = chan_id(op.kind, op.p);
        const int ns = (int)op.t.size() / g;
        for (int s = ns - 1; s >= 0; --s) {
          const int32_t q1 = op.t[g * s], q2 = g == 2 ? op.t[g * s + 1] : -1;
          for (int comp = K - 1; comp >= 0; --comp) {
            int a, b;
            component_paulis(op.kind, comp, &a, &b);
            Set sym;
            if (a == 1 || a == 2) sym_into(sym, sx[q1]);
            if (a == 2 || a == 3) sym_into(sym, sz[q1]);
            if (q2 >= 0) {
              if (b == 1 || b == 2) sym_into(sym, sx[q2]);
              if (b == 2 || b == 3) sym_into(sym, sz[q2]);
            }
            auto it = index.find(sym);
            int32_t id;
            if (it == index.end()) {
              id = (int32_t)symptoms.size();
              index.emplace(sym, id);
              symptoms.push_back(sym);
              contrib.emplace_back();
            } else {
              id = it->second;
            }
            contrib[id].push_back((uint16_t)cid);
          }
        }
        break;
      }
      default:
        break;
    }
  }
  for (int q = 0; q < Q; ++q) mark(sz[q]);      // every qubit starts in |0>
  for (size_t x = 0; x < nondet.size(); ++x)
    if (nondet[x]) {
      const bool det = (int)x < nd;
      return fail(TMCS_ENONDETERMINISTIC, std::string(det ? "detector " : "observable ") +
                                             std::to_string(det ? (int)x : (int)x - nd) +
                                             " is not deterministic in the noiseless circuit");
    }
  if (chans.size() > 65535) return fail(TMCS_EUNSUPPORTED, "too many distinct noise channels");

  struct Col { Set dets; std::vector<uint64_t> om; double p; };
  std::vector<Col> cols;
  int64_t undetectable = 0;
  if (c.num_obs > MAX_OBS) return fail(TMCS_EUNSUPPORTED, "more than 256 observables");
  const int OW = std::max(1, (c.num_obs + 63) / 64);
  for (size_t i = 0; i < symptoms.size(); ++i) {
    const Set& s = symptoms[i];
    // merge in circuit order: contributions were stored in reverse order
    double p = 0.0;
    bool first = true;
    for (auto it = contrib[i].rbegin(); it != contrib[i].rend(); ++it) {
      const double q = mechanism_prob(chans[*it].first, chans[*it].second);
      if (first) { p = q; first = false; }
      else p = p + q - 2.0 * p * q;
    }
    Col col;
    col.om.assign(OW, 0ull);
    bool any_obs = false;
    for (int32_t x : s) {
      if (x < nd) col.dets.push_back(x);
      else { col.om[(x - nd) >> 6] |= 1ull << ((x - nd) & 63); any_obs = true; }
    }
    col.p = p;
    if (col.dets.empty()) {
      if (any_obs) ++undetectable;
      continue;
    }
    cols.push_back(std::move(col));
  }
  // (detector list, observable mask as one integer): masks compare from their top word down
  std::sort(cols.begin(), cols.end(), [OW](const Col& a, const Col& b) {
    if (a.dets != b.dets) return a.dets < b.dets;
    for (int w = OW - 1; w >= 0; --w)
      if (a.om[w] != b.om[w]) return a.om[w] < b.om[w];
    return false;
  });
  d->rows = nd;
  d->cols = (int)cols.size();
  d->nobs = c.num_obs;
  d->undetectable = undetectable;
  d->col_ptr.assign(d->cols + 1, 0);
  d->priors.resize(d->cols);
  d->obs_words = OW;
  d->obs_mask.resize((size_t)d->cols * OW);
  std::vector<int32_t> row_cnt(nd, 0);
  for (int j = 0; j < d->cols; ++j) {
    d->col_ptr[j + 1] = d->col_ptr[j] + (int32_t)cols[j].dets.size();
    d->priors[j] = cols[j].p;
    for (int w = 0; w < OW; ++w) d->obs_mask[(size_t)j * OW + w] = cols[j].om[w];
    for (int32_t r : cols[j].dets) row_cnt[r]++;
    d->max_col_deg = std::max(d->max_col_deg, (int)cols[j].dets.size());
  }
  d->edges = d->col_ptr[d->cols];
  d->row_idx.resize(d->edges);
  for (int j = 0; j < d->cols; ++j)
    std::copy(cols[j].dets.begin(), cols[j].dets.end(), d->row_idx.begin() + d->col_ptr[j]);
  d->row_ptr.assign(nd + 1, 0);
  for (int r = 0; r < nd; ++r) {
    d->row_ptr[r + 1] = d->row_ptr[r] + row_cnt[r];
    d->max_row_deg = std::max(d->max_row_deg, row_cnt[r]);
  }
  d->col_idx.resize(d->edges);
  d->csc_edge.resize(d->edges);
  std::vector<int32_t> fillp(d->row_ptr.begin(), d->row_ptr.end() - 1);
  for (int j = 0; j < d->cols; ++j) {           // columns ascending => CSR rows sorted
    for (int32_t e = d->col_ptr[j]; e < d->col_ptr[j + 1]; ++e) {
      const int32_t r = d->row_idx[e];
      const int32_t pos = fillp[r]++;
      d->col_idx[pos] = j;
      d->csc_edge[e] = pos;
    }
  }
  // GF(2) rank of H (rows as bit vectors over the columns)
  const int64_t words = (d->cols + 63) / 64;
  if ((int64_t)nd * words > (int64_t)1 << 28)
    return fail(TMCS_EUNSUPPORTED, "DEM too large for the dense rank computation");
  std::vector<BitRow> rows(nd, BitRow(words, 0ull));
  for (int r = 0; r < nd; ++r)
    for (int32_t e = d->row_ptr[r]; e < d->row_ptr[r + 1]; ++e) {
      const int32_t j = d->col_idx[e];
      rows[r][j >> 6] |= 1ull << (j & 63);
    }
  d->rank = gf2_rank_rows(std::move(rows), d->cols);
  return TMCS_OK;
}

}  // namespace tmcs
