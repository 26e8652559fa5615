// Noisy Clifford circuits of the distributed operations.
//
// Operations (Methods: "Non-local CNOT circuit", "State teleportation circuit";
// Fig. 1b, 1c): Z-basis memory; non-local transversal CNOT CB1 -> CB2 through n
// ebit pairs (CX data->ebit_A, measure ebit_A, conditional X on ebit_B,
// CX ebit_B->data, H and measure ebit_B, conditional Z on the control data);
// teleportation CB1 -> CB3 (H on CB2, non-local CNOT CB2 -> CB3, transversal
// Bell measurement of CB1/CB2, conditional X/Z corrections on CB3).  Blocks are
// reset noisily, run rounds_before syndrome rounds, the operation, then
// rounds_after rounds (teleport: on CB3 only), then a Z readout of the data.
//
// Noise (Methods, "Simulation"): bit flip p after R (phase flip after RX); bit
// flip p before M (phase flip before MX); DEPOLARIZE1(p) after H; DEPOLARIZE2(p)
// after each CX including ebit-data CX; surface code: DEPOLARIZE1(p) on the
// data at the start of every round; BB code: DEPOLARIZE1(p) on every qubit of
// the block idle in a layer of the round (reset, each CX layer, measurement);
// ebit pairs: perfect Bell preparation then DEPOLARIZE2(p_ebit); classically
// controlled Paulis are noiseless.  X checks use RX/MX (no Hadamards in the
// rounds, as Table III's 1q counts 3n and 7n require).  Detectors: Z checks only
// (Methods, "Non-local CNOT circuit").  After a transversal CNOT c -> t, t's next
// Z detectors also include c's previous records (Z_t -> Z_c Z_t); after the
// teleportation CB3's next Z detectors compare with CB1's last round.
//
// Qubits: block b is [b*(n+nx+nz), ...) as data, X ancillas, Z ancillas; ebit
// pair k is (E0 + k, E0 + n + k) with E0 after the blocks.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <set>

#include "internal.h"

namespace tmcs {

namespace {

struct Block {
  int base;
  std::vector<int> data, xanc, zanc, all;
  std::vector<std::vector<int32_t>> prev;  // per Z check: records XORed next round
};

std::vector<int32_t> sym_diff(const std::vector<int32_t>& a, const std::vector<int32_t>& b) {
  std::set<int32_t> s(a.begin(), a.end());
  for (int32_t x : b) {
    auto it = s.find(x);
    if (it == s.end()) s.insert(x); else s.erase(it);
  }
  return std::vector<int32_t>(s.begin(), s.end());
}

struct Builder {
  Circuit* c;
  std::vector<int32_t> add(OpKind k, std::vector<int32_t> t, double p = 0.0, int obs = 0) {
    std::vector<int32_t> recs;
    if (k == OP_M || k == OP_MX) {
      for (size_t i = 0; i < t.size(); ++i) recs.push_back(c->num_meas + (int)i);
      c->num_meas += (int)t.size();
    }
    if (k == OP_XERR || k == OP_ZERR || k == OP_DEP1 || k == OP_DEP2) {
      if (t.empty()) return recs;
      c->num_sites += (int64_t)t.size() / (k == OP_DEP2 ? 2 : 1);
    }
    if (k == OP_DET) c->num_dets += 1;
    if (k == OP_OBS) c->num_obs = std::max(c->num_obs, obs + 1);
    if (t.empty() && k != OP_TICK) return recs;
    Op op;
    op.kind = k;
    op.p = p;
    op.obs = obs;
    op.t = std::move(t);
    c->ops.push_back(std::move(op));
    return recs;
  }
};

void syndrome_round(Builder& B, std::vector<Block*> blocks, const CodeBlock& code, double p) {
  std::vector<int32_t> xa, za, da;
  for (Block* b : blocks) {
    xa.insert(xa.end(), b->xanc.begin(), b->xanc.end());
    za.insert(za.end(), b->zanc.begin(), b->zanc.end());
    da.insert(da.end(), b->data.begin(), b->data.end());
  }
  B.add(OP_RX, xa);
  B.add(OP_R, za);
  B.add(OP_ZERR, xa, p);
  B.add(OP_XERR, za, p);
  B.add(OP_DEP1, da, p);
  B.add(OP_TICK, {});
  for (int t = 0; t < code.layers; ++t) {
    std::vector<int32_t> pairs;
    for (Block* b : blocks) {
      for (auto& rd : code.xs[t]) { pairs.push_back(b->xanc[rd.first]); pairs.push_back(b->data[rd.second]); }
      for (auto& rd : code.zs[t]) { pairs.push_back(b->data[rd.second]); pairs.push_back(b->zanc[rd.first]); }
    }
    B.add(OP_CX, pairs);
    B.add(OP_DEP2, pairs, p);
    if (code.kind == TMCS_BB) {
      std::set<int32_t> busy(pairs.begin(), pairs.end());
      std::vector<int32_t> idle;
      for (Block* b : blocks)
        for (int q : b->all)
          if (!busy.count(q)) idle.push_back(q);
      B.add(OP_DEP1, idle, p);
    }
    B.add(OP_TICK, {});
  }
  B.add(OP_XERR, za, p);
  B.add(OP_ZERR, xa, p);
  std::vector<int32_t> zrec = B.add(OP_M, za);
  B.add(OP_MX, xa);
  if (code.kind == TMCS_BB) B.add(OP_DEP1, da, p);
  size_t k = 0;
  for (Block* b : blocks) {
    for (int i = 0; i < code.nz; ++i, ++k) {
      B.add(OP_DET, sym_diff({zrec[k]}, b->prev[i]));
      b->prev[i] = {zrec[k]};
    }
  }
  B.add(OP_TICK, {});
}

void nonlocal_cnot(Builder& B, Block& ctl, Block& tgt, int e0, int n, const tmcs_circuit_spec& s) {
  std::vector<int32_t> ea, eb, pairs, cx1, cx2;
  for (int k = 0; k < n; ++k) { ea.push_back(e0 + k); eb.push_back(e0 + n + k); }
  for (int k = 0; k < n; ++k) { pairs.push_back(ea[k]); pairs.push_back(eb[k]); }
  B.add(OP_BELL, pairs);
  B.add(OP_DEP2, pairs, s.p_ebit);
  if (s.ebit_per_step > 0) {
    // decoherence of each ebit for its age in generation steps (T1 = T2)
    const int f = s.ebit_per_step, steps = (n + f - 1) / f;
    for (int k = 0; k < n; ++k) {
      const int age = steps - 1 - k / f;
      const double pk = 0.75 * (1.0 - std::exp(-(double)age * s.ebit_rate));
      if (pk > 0.0) B.add(OP_DEP1, {ea[k], eb[k]}, pk);
    }
  }
  B.add(OP_TICK, {});
  for (int k = 0; k < n; ++k) { cx1.push_back(ctl.data[k]); cx1.push_back(ea[k]); }
  B.add(OP_CX, cx1);
  B.add(OP_DEP2, cx1, s.p);
  B.add(OP_TICK, {});
  B.add(OP_XERR, ea, s.p);
  std::vector<int32_t> ra = B.add(OP_M, ea);
  B.add(OP_TICK, {});
  std::vector<int32_t> fx;
  for (int k = 0; k < n; ++k) { fx.push_back(ra[k]); fx.push_back(eb[k]); }
  B.add(OP_CXREC, fx);
  for (int k = 0; k < n; ++k) { cx2.push_back(eb[k]); cx2.push_back(tgt.data[k]); }
  B.add(OP_CX, cx2);
  B.add(OP_DEP2, cx2, s.p);
  B.add(OP_TICK, {});
  B.add(OP_H, eb);
  B.add(OP_DEP1, eb, s.p);
  B.add(OP_TICK, {});
  B.add(OP_XERR, eb, s.p);
  std::vector<int32_t> rb = B.add(OP_M, eb);
  B.add(OP_TICK, {});
  std::vector<int32_t> fz;
  for (int k = 0; k < n; ++k) { fz.push_back(rb[k]); fz.push_back(ctl.data[k]); }
  B.add(OP_CZREC, fz);
  B.add(OP_TICK, {});
  for (size_t i = 0; i < tgt.prev.size(); ++i) tgt.prev[i] = sym_diff(tgt.prev[i], ctl.prev[i]);
}

void final_readout(Builder& B, std::vector<Block*> blocks, const CodeBlock& code, double p) {
  std::vector<int32_t> da;
  for (Block* b : blocks) da.insert(da.end(), b->data.begin(), b->data.end());
  B.add(OP_XERR, da, p);
  std::vector<int32_t> rec = B.add(OP_M, da);
  size_t off = 0;
  std::vector<std::vector<int32_t>> per;
  for (Block* b : blocks) {
    std::vector<int32_t> r(rec.begin() + off, rec.begin() + off + code.n);
    off += code.n;
    per.push_back(r);
    for (int i = 0; i < code.nz; ++i) {
      std::vector<int32_t> sup;
      for (int j : code.hz[i]) sup.push_back(r[j]);
      B.add(OP_DET, sym_diff(sup, b->prev[i]));
    }
  }
  int o = 0;
  for (size_t bi = 0; bi < blocks.size(); ++bi) {
    for (auto& row : code.lz) {
      std::vector<int32_t> t;
      for (int j : row) t.push_back(per[bi][j]);
      B.add(OP_OBS, t, 0.0, o);
      ++o;
    }
  }
}

}  // namespace

tmcs_status build_circuit(const tmcs_circuit_spec& s, Circuit* c) {
  if (!(s.p >= 0.0 && s.p < 0.5) || !(s.p_ebit >= 0.0 && s.p_ebit < 0.5))
    return fail(TMCS_EINVAL, "p and p_ebit must lie in [0, 0.5)");
  if (s.ebit_per_step < 0 || !(s.ebit_rate >= 0.0 && s.ebit_rate < 1e300))
    return fail(TMCS_EINVAL, "ebit_per_step must be >= 0 and ebit_rate finite and >= 0");
  if (s.op != TMCS_MEMORY && s.op != TMCS_NONLOCAL_CNOT && s.op != TMCS_TELEPORT && s.op != TMCS_PAULI_STRING)
    return fail(TMCS_EINVAL, "unknown operation");
  if (s.op == TMCS_PAULI_STRING && (s.weight < 2 || s.weight > 63))
    return fail(TMCS_EINVAL, "a Pauli string needs weight in [2, 63]");
  if (s.rounds_before < 1 || s.rounds_before > 10000)
    return fail(TMCS_EINVAL, "rounds_before must be in [1, 10000]");
  if ((s.op == TMCS_NONLOCAL_CNOT || s.op == TMCS_TELEPORT) && (s.rounds_after < 1 || s.rounds_after > 10000))
    return fail(TMCS_EINVAL, "rounds_after must be in [1, 10000] for nlcnot/teleport");
  tmcs_status st = make_code(s, &c->code);
  if (st != TMCS_OK) return st;
  const CodeBlock& code = c->code;
  c->spec = s;
  const int nblocks = s.op == TMCS_MEMORY ? 1 : s.op == TMCS_NONLOCAL_CNOT ? 2 : s.op == TMCS_TELEPORT ? 3 : s.weight + 1;
  if ((int64_t)code.k * nblocks > MAX_OBS) return fail(TMCS_EUNSUPPORTED, "more than 256 logical observables");
  const int size = code.n + code.nx + code.nz;
  std::vector<Block> blocks(nblocks);
  for (int b = 0; b < nblocks; ++b) {
    Block& B = blocks[b];
    B.base = b * size;
    for (int i = 0; i < code.n; ++i) B.data.push_back(B.base + i);
    for (int i = 0; i < code.nx; ++i) B.xanc.push_back(B.base + code.n + i);
    for (int i = 0; i < code.nz; ++i) B.zanc.push_back(B.base + code.n + code.nx + i);
    for (int i = 0; i < size; ++i) B.all.push_back(B.base + i);
    B.prev.assign(code.nz, {});
  }
  const int e0 = nblocks * size;
  c->num_qubits = e0 + (s.op != TMCS_MEMORY ? 2 * code.n : 0);
  Builder Bd{c};
  std::vector<Block*> all;
  for (auto& b : blocks) all.push_back(&b);
  std::vector<int32_t> data;
  for (auto& b : blocks) data.insert(data.end(), b.data.begin(), b.data.end());
  Bd.add(OP_R, data);
  Bd.add(OP_XERR, data, s.p);
  Bd.add(OP_TICK, {});
  for (int r = 0; r < s.rounds_before; ++r) syndrome_round(Bd, all, code, s.p);
  if (s.op == TMCS_MEMORY) {
    final_readout(Bd, all, code, s.p);
    c->final_meas = code.n;
  } else if (s.op == TMCS_NONLOCAL_CNOT) {
    nonlocal_cnot(Bd, blocks[0], blocks[1], e0, code.n, s);
    for (int r = 0; r < s.rounds_after; ++r) syndrome_round(Bd, all, code, s.p);
    final_readout(Bd, all, code, s.p);
    c->final_meas = 2 * code.n;
  } else if (s.op == TMCS_PAULI_STRING) {
    const int w = s.weight;
    for (int m = 0; m < w; ++m) {
      Block &ctl = blocks[m], &tgt = blocks[m + 1];
      if (m < w - 1 && m % 2 == 0) {
        nonlocal_cnot(Bd, ctl, tgt, e0, code.n, s);
      } else {
        std::vector<int32_t> cx;
        for (int k = 0; k < code.n; ++k) { cx.push_back(ctl.data[k]); cx.push_back(tgt.data[k]); }
        Bd.add(OP_CX, cx);
        Bd.add(OP_DEP2, cx, s.p);
        Bd.add(OP_TICK, {});
        for (int i = 0; i < code.nz; ++i) tgt.prev[i] = sym_diff(tgt.prev[i], ctl.prev[i]);
      }
      std::vector<Block*> pair = {&ctl, &tgt};
      syndrome_round(Bd, pair, code, s.p);
    }
    final_readout(Bd, all, code, s.p);
    c->final_meas = nblocks * code.n;
  } else {
    Block &cb1 = blocks[0], &cb2 = blocks[1], &cb3 = blocks[2];
    std::vector<int32_t> d2(cb2.data.begin(), cb2.data.end());
    Bd.add(OP_H, d2);
    Bd.add(OP_DEP1, d2, s.p);
    Bd.add(OP_TICK, {});
    nonlocal_cnot(Bd, cb2, cb3, e0, code.n, s);
    std::vector<int32_t> bell;
    for (int k = 0; k < code.n; ++k) { bell.push_back(cb1.data[k]); bell.push_back(cb2.data[k]); }
    Bd.add(OP_CX, bell);
    Bd.add(OP_DEP2, bell, s.p);
    Bd.add(OP_TICK, {});
    std::vector<int32_t> d1(cb1.data.begin(), cb1.data.end());
    Bd.add(OP_H, d1);
    Bd.add(OP_DEP1, d1, s.p);
    Bd.add(OP_TICK, {});
    std::vector<int32_t> both = d1;
    both.insert(both.end(), d2.begin(), d2.end());
    Bd.add(OP_XERR, both, s.p);
    std::vector<int32_t> r = Bd.add(OP_M, both);
    Bd.add(OP_TICK, {});
    std::vector<int32_t> fx, fz;
    for (int k = 0; k < code.n; ++k) {
      fx.push_back(r[code.n + k]); fx.push_back(cb3.data[k]);
      fz.push_back(r[k]); fz.push_back(cb3.data[k]);
    }
    Bd.add(OP_CXREC, fx);
    Bd.add(OP_CZREC, fz);
    Bd.add(OP_TICK, {});
    for (int i = 0; i < code.nz; ++i) cb3.prev[i] = cb1.prev[i];
    std::vector<Block*> only3 = {&cb3};
    for (int q = 0; q < s.rounds_after; ++q) syndrome_round(Bd, only3, code, s.p);
    final_readout(Bd, only3, code, s.p);
    c->final_meas = code.n;
  }
  return TMCS_OK;
}

static const char* op_name(OpKind k) {
  switch (k) {
    case OP_R: return "R";
    case OP_RX: return "RX";
    case OP_M: return "M";
    case OP_MX: return "MX";
    case OP_H: return "H";
    case OP_CX: return "CX";
    case OP_BELL: return "BELL_PREP";
    case OP_XERR: return "X_ERROR";
    case OP_ZERR: return "Z_ERROR";
    case OP_DEP1: return "DEPOLARIZE1";
    case OP_DEP2: return "DEPOLARIZE2";
    case OP_TICK: return "TICK";
    default: return "?";
  }
}

std::string circuit_text(const Circuit& c) {
  std::string out;
  int nm = 0;
  char buf[64];
  for (const Op& op : c.ops) {
    switch (op.kind) {
      case OP_M:
      case OP_MX:
        out += op_name(op.kind);
        for (int q : op.t) { out += ' '; out += std::to_string(q); }
        nm += (int)op.t.size();
        break;
      case OP_XERR:
      case OP_ZERR:
      case OP_DEP1:
      case OP_DEP2:
        snprintf(buf, sizeof buf, "%s(%.17g)", op_name(op.kind), op.p);
        out += buf;
        for (int q : op.t) { out += ' '; out += std::to_string(q); }
        break;
      case OP_CXREC:
      case OP_CZREC:
        out += op.kind == OP_CXREC ? "CX" : "CZ";
        for (size_t i = 0; i + 1 < op.t.size(); i += 2) {
          out += " rec[-" + std::to_string(nm - op.t[i]) + "] " + std::to_string(op.t[i + 1]);
        }
        break;
      case OP_DET:
        out += "DETECTOR";
        for (int r : op.t) out += " rec[-" + std::to_string(nm - r) + "]";
        break;
      case OP_OBS:
        out += "OBSERVABLE_INCLUDE(" + std::to_string(op.obs) + ")";
        for (int r : op.t) out += " rec[-" + std::to_string(nm - r) + "]";
        break;
      case OP_TICK:
        out += "TICK";
        break;
      default:
        out += op_name(op.kind);
        for (int q : op.t) { out += ' '; out += std::to_string(q); }
    }
    out += '\n';
  }
  return out;
}

void circuit_counts(const Circuit& c, int64_t info[TMCS_INFO_LEN]) {
  for (int i = 0; i < TMCS_INFO_LEN; ++i) info[i] = 0;
  double events = 0.0;
  for (const Op& op : c.ops) {
    if (op.kind == OP_XERR || op.kind == OP_ZERR || op.kind == OP_DEP1 || op.kind == OP_DEP2)
      events += op.p * (double)(op.kind == OP_DEP2 ? op.t.size() / 2 : op.t.size());
    if (op.kind == OP_H || op.kind == OP_CXREC || op.kind == OP_CZREC)
      info[TMCS_INFO_GATES_1Q] += op.kind == OP_H ? (int64_t)op.t.size() : (int64_t)op.t.size() / 2;
    else if (op.kind == OP_CX)
      info[TMCS_INFO_GATES_2Q] += (int64_t)op.t.size() / 2;
  }
  info[TMCS_INFO_QUBITS] = c.num_qubits;
  info[TMCS_INFO_MEAS] = c.num_meas;
  info[TMCS_INFO_MEAS_FINAL] = c.final_meas;
  info[TMCS_INFO_DETECTORS] = c.num_dets;
  info[TMCS_INFO_OBSERVABLES] = c.num_obs;
  info[TMCS_INFO_NOISE_SITES] = c.num_sites;
  info[TMCS_INFO_INSTRUCTIONS] = (int64_t)c.ops.size();
  info[TMCS_INFO_CODE_N] = c.code.n;
  info[TMCS_INFO_CODE_K] = c.code.k;
  info[TMCS_INFO_EVENTS_PER_MSHOT] = (int64_t)std::llround(events * 1e6);
}

}  // namespace tmcs
