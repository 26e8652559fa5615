// Host-only check of the DEM builder's noiseless-determinism test: small
// hand-written circuits, built with g++ against the library's host sources.
// Prints one line per case: "<name> <status>".
#include <cstdio>
#include <string>
#include <vector>

#include "host/internal.h"

namespace tmcs {
static std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }
tmcs_status fail(tmcs_status st, const std::string& msg) { g_err = msg; return st; }
}  // namespace tmcs

using namespace tmcs;

struct B {
  Circuit c;
  explicit B(int q) { c.num_qubits = q; }
  B& op(OpKind k, std::vector<int32_t> t, double p = 0.0, int obs = 0) {
    Op o{k};
    o.t = std::move(t);
    o.p = p;
    o.obs = obs;
    if (k == OP_M || k == OP_MX) c.num_meas += (int)o.t.size();
    if (k == OP_DET) c.num_dets += 1;
    if (k == OP_OBS) c.num_obs = std::max(c.num_obs, obs + 1);
    if (k == OP_XERR || k == OP_ZERR || k == OP_DEP1) c.num_sites += (int64_t)o.t.size();
    c.ops.push_back(std::move(o));
    return *this;
  }
};

static void run(const char* name, const B& b) {
  Dem d;
  g_err.clear();
  const tmcs_status st = build_dem(b.c, &d);
  std::printf("%s %d %s\n", name, (int)st, g_err.c_str());
}

int main() {
  // Z-basis reset then Z measurement: deterministic
  run("reset_measure", B(1).op(OP_R, {0}).op(OP_XERR, {0}, 0.1).op(OP_M, {0}).op(OP_DET, {0}));
  // |+> measured in Z: random
  run("rx_measure_z", B(1).op(OP_RX, {0}).op(OP_M, {0}).op(OP_DET, {0}));
  // no reset: qubits start in |0>, H makes it random
  run("start_h_measure", B(1).op(OP_H, {0}).op(OP_M, {0}).op(OP_DET, {0}));
  // a repeated measurement of a random qubit: the parity of the two records is fixed
  run("repeat_measure", B(1).op(OP_RX, {0}).op(OP_M, {0}).op(OP_M, {0}).op(OP_DET, {0, 1}));
  // one half of a Bell pair: random; ZZ and XX parities: deterministic
  run("bell_half", B(2).op(OP_BELL, {0, 1}).op(OP_M, {0, 1}).op(OP_DET, {0}));
  run("bell_zz", B(2).op(OP_BELL, {0, 1}).op(OP_M, {0, 1}).op(OP_DET, {0, 1}));
  run("bell_xx", B(2).op(OP_BELL, {0, 1}).op(OP_MX, {0, 1}).op(OP_DET, {0, 1}));
  run("bell_zx", B(2).op(OP_BELL, {0, 1}).op(OP_M, {0}).op(OP_MX, {1}).op(OP_DET, {0, 1}));
  // teleportation of |0> from qubit 0 to qubit 2 through the pair (1, 2):
  // records 0 (X basis of q0) and 1 (Z basis of q1); the X correction from
  // record 1 makes q2's Z measurement deterministic, without it it is random
  run("teleport_corrected", B(3).op(OP_R, {0}).op(OP_BELL, {1, 2}).op(OP_CX, {0, 1}).op(OP_MX, {0}).op(OP_M, {1})
                                .op(OP_CXREC, {1, 2}).op(OP_CZREC, {0, 2}).op(OP_M, {2}).op(OP_DET, {2}));
  run("teleport_uncorrected", B(3).op(OP_R, {0}).op(OP_BELL, {1, 2}).op(OP_CX, {0, 1}).op(OP_MX, {0}).op(OP_M, {1})
                                  .op(OP_M, {2}).op(OP_DET, {2}));
  // a random observable
  run("random_observable", B(2).op(OP_R, {0, 1}).op(OP_M, {0}).op(OP_DET, {0}).op(OP_H, {1}).op(OP_M, {1})
                               .op(OP_OBS, {1}, 0.0, 0));
  return 0;
}
