"""Circuit specifications and seeds shared by the oracle and the GPU path.

This module holds parameters only (no arithmetic of the method): which code,
which distributed operation, how many syndrome rounds, which noise strengths,
how many shots and which seeds.  Both the CPU oracle and the product library
build their own codes, circuits and detector error models from these
parameters.

Codes
  * rotated surface code [[d^2, 1, d]] (Supplementary Note 2);
  * bivariate-bicycle codes from Supplementary Table IV, given as (l, m) and
    the three monomials x^i y^j of a(x, y) and of b(x, y).

Operations
  * ``memory``   : one block, Z-basis memory, ``rounds_before`` rounds;
  * ``nlcnot``   : non-local transversal CNOT between two blocks through an
    n-pair ebit layer (Methods, Non-local CNOT circuit; Fig. 1b);
  * ``teleport`` : logical teleportation CB1 -> CB3 through a logical Bell
    pair of CB2 and CB3 (Methods, State teleportation circuit; Fig. 1c).
  * ``pstring``  : Pauli-string parity of weight w (Methods, Pauli string
    compute): w data blocks and an ancilla, a chain of block CNOTs
    1 -> 2 -> ... -> w alternating non-local (first) and local, then a local
    CNOT w -> ancilla, one round on the two blocks after every CNOT.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import Tuple

Mono = Tuple[int, int]  # (power of x, power of y)

# Supplementary Table IV: (l, m, a(x,y), b(x,y)); a and b as monomial lists.
BB_CODES = {
    "bb18": (3, 3, ((0, 0), (1, 0), (0, 1)), ((0, 0), (2, 0), (0, 2))),      # [[18,4,4]]
    "bb36": (3, 6, ((1, 0), (0, 2), (0, 3)), ((0, 0), (2, 0), (0, 1))),      # [[36,4,6]]
    "bb54": (3, 9, ((1, 0), (0, 1), (0, 3)), ((0, 0), (2, 0), (0, 2))),      # [[54,4,8]]
    "bb90": (15, 3, ((9, 0), (0, 1), (0, 2)), ((0, 0), (2, 0), (7, 0))),     # [[90,8,10]]
    "bb144": (12, 6, ((3, 0), (0, 1), (0, 2)), ((1, 0), (2, 0), (0, 3))),    # [[144,12,12]]
}
BB_PARAMS = {"bb18": (18, 4, 4), "bb36": (36, 4, 6), "bb54": (54, 4, 8),
             "bb90": (90, 8, 10), "bb144": (144, 12, 12)}

MEMORY, NLCNOT, TELEPORT, PSTRING = "memory", "nlcnot", "teleport", "pstring"
SC, BB = "sc", "bb"


@dataclass(frozen=True)
class CircuitSpec:
    code: str = SC                  # "sc" | "bb"
    d: int = 3                      # surface-code distance (sc only)
    bb: str = ""                    # key of BB_CODES (bb only)
    op: str = MEMORY                # "memory" | "nlcnot" | "teleport"
    rounds_before: int = 3
    rounds_after: int = 0
    p: float = 1e-3
    p_ebit: float = 1e-3
    # ebit decoherence while the n ebits are generated (Methods, Decoherence):
    # ebit_per_step ebits are made together per generation step (0: no
    # decoherence), ebit_rate = t_gen / T with T1 = T2 = T
    ebit_per_step: int = 0
    ebit_rate: float = 0.0
    weight: int = 0                 # pstring: number of data blocks w (>= 2)

    def bb_params(self):
        return BB_CODES[self.bb]


def sc(d, op=MEMORY, rb=3, ra=0, p=1e-3, p_ebit=None):
    return CircuitSpec(code=SC, d=d, op=op, rounds_before=rb, rounds_after=ra,
                       p=p, p_ebit=p if p_ebit is None else p_ebit)


def bb(name, op=MEMORY, rb=3, ra=0, p=1e-3, p_ebit=None):
    return CircuitSpec(code=BB, bb=name, op=op, rounds_before=rb, rounds_after=ra,
                       p=p, p_ebit=p if p_ebit is None else p_ebit)


def pstring(code_spec: CircuitSpec, w: int, rounds=4) -> CircuitSpec:
    """Pauli-string compute of weight w on copies of code_spec's code (Methods:
    four rounds on every block first; ebit noise equal to the PER)."""
    return replace(code_spec, op=PSTRING, weight=w, rounds_before=rounds, rounds_after=1,
                   p_ebit=code_spec.p)


def line_width(spec: CircuitSpec) -> int:
    """Ebits generated together in the line schedule (Methods, Decoherence): d for
    surface codes; for BB codes the divisor of n closest to d (the smaller one on
    a tie)."""
    if spec.code == SC:
        return spec.d
    n, _, d = BB_PARAMS[spec.bb]
    divs = [f for f in range(1, n + 1) if n % f == 0]
    return min(divs, key=lambda f: (abs(f - d), f))


def with_decoherence(spec: CircuitSpec, rate: float, lines: bool) -> CircuitSpec:
    """spec with ebit decoherence at t_gen / T = rate, one ebit at a time or in lines."""
    return replace(spec, ebit_per_step=line_width(spec) if lines else 1, ebit_rate=rate)


@dataclass(frozen=True)
class Workload:
    name: str
    specs: Tuple[CircuitSpec, ...]   # one per instance (instance id = index)
    shots: int
    seed: int
    bp_iters: int
    description: str = ""
    extra: dict = field(default_factory=dict)


# The five workloads the benchmark and the parity tests are built around.
WORKLOADS = {
    "sc3_memory": Workload(
        "sc3_memory", (sc(3, MEMORY, 3, 0, 1e-3),), 10_000, 1, 30,
        "rotated SC d=3 Z-memory, 3 rounds, p=1e-3"),
    "sc5_nlcnot": Workload(
        "sc5_nlcnot", (sc(5, NLCNOT, 5, 5, 1e-3, 1e-2),), 1_000_000, 1, 30,
        "non-local transversal CNOT, two SC d=5 blocks, 25 ebit pairs, "
        "5/5 rounds, p=1e-3, p_ebit=1e-2"),
    "bb144_memory": Workload(
        "bb144_memory",
        (bb("bb144", MEMORY, 12, 0, 5e-4), bb("bb144", MEMORY, 12, 0, 1e-3),
         bb("bb144", MEMORY, 12, 0, 2e-3)),
        1_000_000, 1, 30,
        "BB [[144,12,12]] memory, 12 rounds, p in {5e-4, 1e-3, 2e-3}"),
    "bb144_teleport": Workload(
        "bb144_teleport", (bb("bb144", TELEPORT, 4, 3, 1e-3, 1e-2),), 1_000_000, 1, 20,
        "teleportation of a BB [[144,12,12]] block, 144 ebits, 4/4/4 + 3 rounds, "
        "p=1e-3, p_ebit=1e-2"),
    "sc5_pstring": Workload(
        "sc5_pstring", tuple(pstring(sc(5, p=1e-3), w) for w in (2, 3, 4, 5, 6)), 1_000_000, 1, 30,
        "Pauli-string compute of weight w = 2..6 on SC d=5 blocks (chain patterns 1, 10, 101, 1010, "
        "10101), 4 rounds first, one round after each CNOT, p = p_ebit = 1e-3"),
    "sc_nlcnot_mixed": Workload(
        "sc_nlcnot_mixed",
        tuple(sc(d, NLCNOT, d, d, p, 10 * p) for d in (11, 15, 21, 29)
              for p in (1e-4, 1e-3)),
        100_000, 1, 20,
        "mixed batch: non-local CNOT on SC d in {11,15,21,29}, d/d rounds, "
        "p in {1e-4, 1e-3}, p_ebit = 10p"),
}


def with_noise(spec: CircuitSpec, p: float, p_ebit: float | None = None) -> CircuitSpec:
    return replace(spec, p=p, p_ebit=p if p_ebit is None else p_ebit)
