// Host-only run of the circuit, code, DEM, program and distance builders, for a
// build with AddressSanitizer and UndefinedBehaviorSanitizer (g++ against the
// library's host sources).  Prints one line per case:
// "<name> <status> <detectors> <dem columns> <dem edges> <distance or -1>".
#include <cstdio>
#include <string>

#include "host/internal.h"
#include "host/program.h"

namespace tmcs {
static std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }
tmcs_status fail(tmcs_status st, const std::string& msg) { g_err = msg; return st; }
}  // namespace tmcs

using namespace tmcs;

static tmcs_circuit_spec sc(int d, int op, int rb, int ra) {
  tmcs_circuit_spec s{};
  s.code = TMCS_SC; s.d = d; s.op = op; s.rounds_before = rb; s.rounds_after = ra;
  s.p = 1e-3; s.p_ebit = 1e-2;
  return s;
}

static tmcs_circuit_spec bb(int l, int m, const int a[3][2], const int b[3][2], int op, int rb, int ra) {
  tmcs_circuit_spec s{};
  s.code = TMCS_BB; s.bb_l = l; s.bb_m = m;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 2; ++j) { s.bb_a[i][j] = a[i][j]; s.bb_b[i][j] = b[i][j]; }
  s.op = op; s.rounds_before = rb; s.rounds_after = ra; s.p = 4e-3; s.p_ebit = 4e-2;
  return s;
}

// build everything for one spec; the exact distance search (every detector may
// be active) when `dist` is set
static void run(const char* name, const tmcs_circuit_spec& s, bool dist) {
  Circuit c;
  tmcs_status st = build_circuit(s, &c);
  if (st != TMCS_OK) { printf("%s %d 0 0 0 -1\n", name, (int)st); return; }
  const std::string text = circuit_text(c);
  int64_t info[TMCS_INFO_LEN];
  circuit_counts(c, info);
  Dem D;
  if ((st = build_dem(c, &D)) != TMCS_OK) { printf("%s %d 0 0 0 -1\n", name, (int)st); return; }
  Program P;
  if ((st = compile_program(c, &P)) != TMCS_OK) { printf("%s %d 0 0 0 -1\n", name, (int)st); return; }
  int32_t w = -1;
  if (dist && (st = dem_distance(D, D.rows, 8, 4000000, &w)) != TMCS_OK) w = -2;
  printf("%s %d %lld %d %lld %d\n", name, (int)st, (long long)info[TMCS_INFO_DETECTORS], D.cols, (long long)D.edges,
         (int)w);
  (void)text;
}

int main() {
  const int a18[3][2] = {{0, 0}, {1, 0}, {0, 1}}, b18[3][2] = {{0, 0}, {2, 0}, {0, 2}};   // [[18,4,4]]
  const int a36[3][2] = {{1, 0}, {0, 2}, {0, 3}}, b36[3][2] = {{0, 0}, {2, 0}, {0, 1}};   // [[36,4,6]]
  run("sc3_memory", sc(3, TMCS_MEMORY, 3, 0), true);
  run("sc3_nlcnot", sc(3, TMCS_NONLOCAL_CNOT, 3, 3), true);
  run("sc3_teleport", sc(3, TMCS_TELEPORT, 3, 3), true);
  run("sc5_nlcnot", sc(5, TMCS_NONLOCAL_CNOT, 5, 5), false);
  run("sc5_teleport", sc(5, TMCS_TELEPORT, 4, 3), false);
  {
    tmcs_circuit_spec s = sc(5, TMCS_NONLOCAL_CNOT, 3, 3);
    s.ebit_per_step = 2;
    s.ebit_rate = 0.01;
    run("sc5_nlcnot_decoherence", s, false);
  }
  {
    tmcs_circuit_spec s = sc(3, TMCS_PAULI_STRING, 2, 0);
    s.weight = 3;
    run("sc3_pstring3", s, false);
  }
  run("bb18_memory", bb(3, 3, a18, b18, TMCS_MEMORY, 3, 0), true);
  run("bb18_nlcnot", bb(3, 3, a18, b18, TMCS_NONLOCAL_CNOT, 3, 3), false);
  run("bb18_teleport", bb(3, 3, a18, b18, TMCS_TELEPORT, 3, 3), false);
  run("bb36_nlcnot", bb(3, 6, a36, b36, TMCS_NONLOCAL_CNOT, 3, 3), false);
  {
    tmcs_circuit_spec s = bb(3, 6, a36, b36, TMCS_PAULI_STRING, 2, 0);
    s.weight = 2;
    run("bb36_pstring2", s, false);
  }
  // invalid specs fail cleanly
  run("bad_even_d", sc(4, TMCS_MEMORY, 3, 0), false);
  {
    tmcs_circuit_spec s = sc(3, TMCS_MEMORY, 3, 0);
    s.p = 0.7;
    run("bad_p", s, false);
  }
  {
    tmcs_circuit_spec s = sc(3, TMCS_MEMORY, 0, 0);
    run("bad_rounds", s, false);
  }
  return 0;
}
