"""Noisy Clifford circuits for memory, non-local CNOT and teleportation (oracle).

The circuit is a list of instructions ``(name, arg, targets)`` with absolute
measurement-record indices.  Instruction set and frame semantics:

  R / RX q..           reset to |0> / |+>
  M / MX q..           measure Z / X (one record each, in target order)
  H q..                Hadamard
  CX c t ..            CNOT pairs
  BELL_PREP a b ..     noiseless preparation of |Phi+> on each pair
  CXREC [(r, q)..]     X on q if record r is 1 (classically controlled)
  CZREC [(r, q)..]     Z on q if record r is 1
  X_ERROR(p) q..       X with probability p (one noise site per target)
  Z_ERROR(p) q..       Z with probability p
  DEPOLARIZE1(p) q..   X, Y, Z each with probability p/3
  DEPOLARIZE2(p) a b.. one of the 15 non-identity two-qubit Paulis, each p/15
  TICK                 layer separator
  DETECTOR [r..]       parity of records
  OBS(k) [r..]         parity of records, folded into logical observable k

Construction (Methods: Simulation, Non-local CNOT circuit, State teleportation
circuit; Fig. 1b/1c; Table III).  Readings where the paper is silent:

* Noise (Methods, Simulation): reset bit flip p after R (phase flip after
  RX); bit flip p before M (phase flip before MX); DEPOLARIZE1(p) after H;
  DEPOLARIZE2(p) after every CX, including ebit-data CX.  Surface code:
  DEPOLARIZE1(p) on every data qubit at the start of each round.  BB code:
  idle DEPOLARIZE1(p) on every qubit of the block left idle by a layer of the
  round (reset, each CX layer, measurement).  Ebits are prepared perfectly and
  then get DEPOLARIZE2(p_ebit); classically controlled Paulis are noiseless.
* Ebit decoherence (Methods, Decoherence), when spec.ebit_per_step > 0: the n
  ebits are made f = ebit_per_step at a time, the last group just before the
  non-local CNOT, so ebit k (generation order) has waited
  age_k = ceil(n / f) - 1 - floor(k / f) steps of t_gen.  Both halves then get
  the Pauli channel of [PhysRevA.90.062320] for t = age_k t_gen with T1 = T2 = T,
  p_X = p_Y = p_Z = (1 - exp(-t/T)) / 4, i.e. DEPOLARIZE1 with
  p = 3/4 (1 - exp(-age_k * ebit_rate)) (omitted where p = 0), applied right
  after the ebit's DEPOLARIZE2(p_ebit).
* X-type ancillas use RX/MX and there are no Hadamards in syndrome
  extraction (fixed by the 1q counts 3n / 7n of Table III).
* Detectors exist for Z checks only (Methods, Non-local CNOT circuit); after a
  transversal CNOT c -> t the target's next Z detectors also include the
  control's previous records; after teleportation CB3's next Z detectors
  compare with CB1's last round.
* The conditional Z of the non-local CNOT acts on the control block (gate
  teleportation); it touches only X-basis records.
* Schedules: surface code 4 interleaved CX layers (X checks NW, NE, SW, SE;
  Z checks NW, SW, NE, SE); BB code the interleaved depth-7 cycle of
  oracle.codes.BB_X_STEPS / BB_Z_STEPS (each step: one term of every X check
  and one term of every Z check on the other half of the data).
* Pauli-string compute (Methods, Pauli string compute): blocks 1..w and the
  ancilla start in |0> with rounds_before rounds on all of them; CNOT m -> m+1
  for m = 1..w-1 is non-local for odd m and local (transversal CX with
  DEPOLARIZE2(p)) for even m (patterns 1, 10, 101, ...), then a local CNOT
  w -> ancilla; after every CNOT one round on its two blocks only (the other
  blocks wait without noise); all blocks are then read out, every block's Z
  logicals being observables.  The non-local CNOTs reuse one ebit register.
* Qubits: block b occupies [b*(n+n_anc), (b+1)*(n+n_anc)) as data, X
  ancillas, Z ancillas; ebit pair k is (E0 + k, E0 + n + k) after the blocks.

Parity: gate/measurement/detector counts pinned against Table III's closed
forms; detector determinism pinned with the stabilizer tableau; circuit
distance of the d=3 surface-code operations pinned by brute force (Table I).
"""
from __future__ import annotations

import math

import numpy as np

from workloads import BB, CircuitSpec, MEMORY, NLCNOT, PSTRING, SC, TELEPORT

from .codes import make_code

NOISE_OPS = ("X_ERROR", "Z_ERROR", "DEPOLARIZE1", "DEPOLARIZE2")


class Circuit:
    def __init__(self):
        self.ops = []
        self.num_qubits = 0
        self.num_meas = 0
        self.num_dets = 0
        self.num_obs = 0
        self.num_sites = 0

    # ------------------------------------------------------------- emitters
    def add(self, name, arg, targets):
        if name in ("M", "MX"):
            first = self.num_meas
            self.num_meas += len(targets)
            self.ops.append((name, arg, list(targets)))
            return list(range(first, first + len(targets)))
        if name in NOISE_OPS:
            if len(targets) == 0:
                return None
            group = 2 if name == "DEPOLARIZE2" else 1
            self.num_sites += len(targets) // group
        if name == "DETECTOR":
            self.num_dets += 1
        if name == "OBS":
            self.num_obs = max(self.num_obs, arg + 1)
        if len(targets) == 0 and name not in ("TICK",):
            return None
        self.ops.append((name, arg, list(targets)))
        return None

    # ---------------------------------------------------------------- views
    def counts(self):
        """Table III style counts: 1q gates, 2q gates, measurements."""
        one = two = meas = 0
        for name, arg, t in self.ops:
            if name == "H":
                one += len(t)
            elif name in ("CXREC", "CZREC"):
                one += len(t)
            elif name == "CX":
                two += len(t) // 2
            elif name in ("M", "MX"):
                meas += len(t)
        return dict(q1=one, q2=two, meas=meas, dets=self.num_dets,
                    obs=self.num_obs, sites=self.num_sites, qubits=self.num_qubits)

    def text(self) -> str:
        """Canonical text form (stim-like, relative record indices)."""
        lines = []
        nm = 0
        for name, arg, t in self.ops:
            if name in ("M", "MX"):
                lines.append(name + " " + " ".join(str(q) for q in t))
                nm += len(t)
            elif name in NOISE_OPS:
                lines.append("%s(%.17g) %s" % (name, arg, " ".join(str(q) for q in t)))
            elif name in ("CXREC", "CZREC"):
                g = "CX" if name == "CXREC" else "CZ"
                lines.append(g + " " + " ".join("rec[-%d] %d" % (nm - r, q) for r, q in t))
            elif name == "DETECTOR":
                lines.append("DETECTOR " + " ".join("rec[-%d]" % (nm - r) for r in t))
            elif name == "OBS":
                lines.append("OBSERVABLE_INCLUDE(%d) " % arg +
                             " ".join("rec[-%d]" % (nm - r) for r in t))
            elif name == "TICK":
                lines.append("TICK")
            else:
                lines.append(name + " " + " ".join(str(q) for q in t))
        return "\n".join(lines) + "\n"


def _xor_lists(a, b):
    s = set(a) ^ set(b)
    return sorted(s)


class _Block:
    def __init__(self, code, base):
        self.code = code
        self.base = base
        n = code.n
        self.nx = code.hx.shape[0]
        self.nz = code.hz.shape[0]
        self.data = [base + i for i in range(n)]
        self.xanc = [base + n + i for i in range(self.nx)]
        self.zanc = [base + n + self.nx + i for i in range(self.nz)]
        self.all = list(range(base, base + n + self.nx + self.nz))
        self.prev = [[] for _ in range(self.nz)]  # records compared next round


def _syndrome_round(c: Circuit, blocks, spec):
    code = blocks[0].code
    p = spec.p
    xa = [q for b in blocks for q in b.xanc]
    za = [q for b in blocks for q in b.zanc]
    da = [q for b in blocks for q in b.data]
    c.add("RX", None, xa)
    c.add("R", None, za)
    c.add("Z_ERROR", p, xa)
    c.add("X_ERROR", p, za)
    c.add("DEPOLARIZE1", p, da)
    c.add("TICK", None, [])
    for t in range(code.sched_layers):
        pairs = []
        for b in blocks:
            for (r, dq) in code.x_sched[t]:
                pairs += [b.xanc[r], b.data[dq]]
            for (r, dq) in code.z_sched[t]:
                pairs += [b.data[dq], b.zanc[r]]
        c.add("CX", None, pairs)
        c.add("DEPOLARIZE2", p, pairs)
        if code.kind == BB:
            busy = set(pairs)
            idle = [q for b in blocks for q in b.all if q not in busy]
            c.add("DEPOLARIZE1", p, idle)
        c.add("TICK", None, [])
    c.add("X_ERROR", p, za)
    c.add("Z_ERROR", p, xa)
    zrec = c.add("M", None, za)
    c.add("MX", None, xa)
    if code.kind == BB:
        c.add("DEPOLARIZE1", p, da)
    k = 0
    for b in blocks:
        for i in range(b.nz):
            c.add("DETECTOR", None, _xor_lists([zrec[k]], b.prev[i]))
            b.prev[i] = [zrec[k]]
            k += 1
    c.add("TICK", None, [])


def ebit_decoherence(n: int, f: int, rate: float):
    """Per ebit (generation order): the DEPOLARIZE1 probability of its age."""
    if f <= 0:
        return [0.0] * n
    steps = -(-n // f)
    return [0.75 * (1.0 - math.exp(-(steps - 1 - k // f) * rate)) for k in range(n)]


def _nonlocal_cnot(c: Circuit, ctl: _Block, tgt: _Block, e0: int, spec):
    n = ctl.code.n
    p = spec.p
    ea = [e0 + k for k in range(n)]
    eb = [e0 + n + k for k in range(n)]
    pairs = [q for k in range(n) for q in (ea[k], eb[k])]
    c.add("BELL_PREP", None, pairs)
    c.add("DEPOLARIZE2", spec.p_ebit, pairs)
    for k, pk in enumerate(ebit_decoherence(n, spec.ebit_per_step, spec.ebit_rate)):
        if pk > 0.0:
            c.add("DEPOLARIZE1", pk, [ea[k], eb[k]])
    c.add("TICK", None, [])
    cx1 = [q for k in range(n) for q in (ctl.data[k], ea[k])]
    c.add("CX", None, cx1)
    c.add("DEPOLARIZE2", p, cx1)
    c.add("TICK", None, [])
    c.add("X_ERROR", p, ea)
    ra = c.add("M", None, ea)
    c.add("TICK", None, [])
    c.add("CXREC", None, [(ra[k], eb[k]) for k in range(n)])
    cx2 = [q for k in range(n) for q in (eb[k], tgt.data[k])]
    c.add("CX", None, cx2)
    c.add("DEPOLARIZE2", p, cx2)
    c.add("TICK", None, [])
    c.add("H", None, eb)
    c.add("DEPOLARIZE1", p, eb)
    c.add("TICK", None, [])
    c.add("X_ERROR", p, eb)
    rb = c.add("M", None, eb)
    c.add("TICK", None, [])
    c.add("CZREC", None, [(rb[k], ctl.data[k]) for k in range(n)])
    c.add("TICK", None, [])
    # Z_t -> Z_c Z_t: the target's next comparison includes the control's.
    for i in range(tgt.nz):
        tgt.prev[i] = _xor_lists(tgt.prev[i], ctl.prev[i])


def _final_readout(c: Circuit, blocks, spec, obs_base=0):
    da = [q for b in blocks for q in b.data]
    c.add("X_ERROR", spec.p, da)
    rec = c.add("M", None, da)
    off = 0
    per_block = []
    for b in blocks:
        r = rec[off: off + b.code.n]
        per_block.append(r)
        off += b.code.n
        for i in range(b.nz):
            support = np.nonzero(b.code.hz[i])[0]
            c.add("DETECTOR", None, _xor_lists([r[j] for j in support], b.prev[i]))
    o = obs_base
    for b, r in zip(blocks, per_block):
        for row in b.code.lz:
            c.add("OBS", o, [r[j] for j in np.nonzero(row)[0]])
            o += 1


def build_circuit(spec: CircuitSpec) -> Circuit:
    code = make_code(spec)
    if spec.rounds_before < 1:
        raise ValueError("rounds_before must be >= 1")
    if spec.op in (NLCNOT, TELEPORT) and spec.rounds_after < 1:
        raise ValueError("rounds_after must be >= 1 for nlcnot/teleport")
    if spec.op == PSTRING and spec.weight < 2:
        raise ValueError("a Pauli string needs weight >= 2")
    nblocks = {MEMORY: 1, NLCNOT: 2, TELEPORT: 3}.get(spec.op, spec.weight + 1)
    size = code.n + code.hx.shape[0] + code.hz.shape[0]
    blocks = [_Block(code, b * size) for b in range(nblocks)]
    e0 = nblocks * size
    c = Circuit()
    c.num_qubits = e0 + (2 * code.n if spec.op != MEMORY else 0)
    c.code = code
    c.spec = spec
    data = [q for b in blocks for q in b.data]
    c.add("R", None, data)
    c.add("X_ERROR", spec.p, data)
    c.add("TICK", None, [])
    for _ in range(spec.rounds_before):
        _syndrome_round(c, blocks, spec)
    if spec.op == MEMORY:
        _final_readout(c, blocks, spec)
    elif spec.op == NLCNOT:
        _nonlocal_cnot(c, blocks[0], blocks[1], e0, spec)
        for _ in range(spec.rounds_after):
            _syndrome_round(c, blocks, spec)
        _final_readout(c, blocks, spec)
    elif spec.op == PSTRING:
        w = spec.weight
        for m in range(w):
            ctl, tgt = blocks[m], blocks[m + 1]
            if m < w - 1 and m % 2 == 0:
                _nonlocal_cnot(c, ctl, tgt, e0, spec)
            else:
                cx = [q for k in range(code.n) for q in (ctl.data[k], tgt.data[k])]
                c.add("CX", None, cx)
                c.add("DEPOLARIZE2", spec.p, cx)
                c.add("TICK", None, [])
                for i in range(tgt.nz):
                    tgt.prev[i] = _xor_lists(tgt.prev[i], ctl.prev[i])
            _syndrome_round(c, [ctl, tgt], spec)
        _final_readout(c, blocks, spec)
    else:
        cb1, cb2, cb3 = blocks
        c.add("H", None, cb2.data)
        c.add("DEPOLARIZE1", spec.p, cb2.data)
        c.add("TICK", None, [])
        _nonlocal_cnot(c, cb2, cb3, e0, spec)
        bell = [q for k in range(code.n) for q in (cb1.data[k], cb2.data[k])]
        c.add("CX", None, bell)
        c.add("DEPOLARIZE2", spec.p, bell)
        c.add("TICK", None, [])
        c.add("H", None, cb1.data)
        c.add("DEPOLARIZE1", spec.p, cb1.data)
        c.add("TICK", None, [])
        both = cb1.data + cb2.data
        c.add("X_ERROR", spec.p, both)
        r = c.add("M", None, both)
        r1, r2 = r[:code.n], r[code.n:]
        c.add("TICK", None, [])
        c.add("CXREC", None, [(r2[k], cb3.data[k]) for k in range(code.n)])
        c.add("CZREC", None, [(r1[k], cb3.data[k]) for k in range(code.n)])
        c.add("TICK", None, [])
        for i in range(cb3.nz):
            cb3.prev[i] = list(cb1.prev[i])
        for _ in range(spec.rounds_after):
            _syndrome_round(c, [cb3], spec)
        _final_readout(c, [cb3], spec)
    return c
