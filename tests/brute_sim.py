"""Brute-force simulators used only to pin the oracle.

Two independent simulators of the circuit language subset:

* :class:`Tableau` -- the stabiliser-tableau method of Aaronson and Gottesman
  ("Improved simulation of stabilizer circuits", PRA 70, 052328, 2004):
  destabiliser and stabiliser rows, the phase-tracking row product, random
  and deterministic Z measurements.
* :class:`StateVector` -- dense amplitudes, gates as matrices, measurement by
  projection. Only for a handful of qubits; it pins the tableau code.

Both share only the circuit-text parser below (which is independent of the
oracle's and of the compiler's). A fault is injected by applying its Pauli at
its channel's place in a full simulation; its signature is the set of
detectors/observables whose value differs from the noiseless run. This is an
algorithm independent of frame propagation.
"""

from __future__ import annotations

import dataclasses
import random
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

NOISE1 = ("X_ERROR", "Y_ERROR", "Z_ERROR", "DEPOLARIZE1")
ALIASES = {"CNOT": "CX", "ZCX": "CX", "ZCZ": "CZ", "H_XZ": "H", "SQRT_Z": "S",
           "SQRT_Z_DAG": "S_DAG", "RZ": "R", "MZ": "M", "MRZ": "MR"}


@dataclasses.dataclass
class Instr:
    name: str
    args: Tuple[float, ...]
    targets: Tuple[int, ...]     # qubits, or k for rec[-k]


def parse(text: str) -> List[Instr]:
    out = []
    for line in text.splitlines():
        line = line.split("#", 1)[0].strip()
        if not line:
            continue
        head, _, rest = line.partition(" ")
        args: Tuple[float, ...] = ()
        if "(" in head:
            name, _, a = head.partition("(")
            args = tuple(float(x) for x in a.rstrip(")").split(",") if x.strip())
        else:
            name = head
        name = ALIASES.get(name.upper(), name.upper())
        tg = []
        for tok in rest.split():
            if tok.startswith("rec[-"):
                tg.append(int(tok[5:-1]))
            else:
                tg.append(int(tok))
        out.append(Instr(name, args, tuple(tg)))
    return out


def channels(instrs: Sequence[Instr]) -> List[Tuple[int, str, Tuple[int, ...], float]]:
    """(instruction index, kind, qubits, rate) per channel, in channel order."""
    out = []
    for k, ins in enumerate(instrs):
        if ins.name in NOISE1:
            out += [(k, ins.name, (q,), ins.args[0]) for q in ins.targets]
        elif ins.name == "DEPOLARIZE2":
            t = ins.targets
            out += [(k, ins.name, (t[i], t[i + 1]), ins.args[0]) for i in range(0, len(t), 2)]
    return out


# ---------------------------------------------------------------------------
# Tableau simulator
# ---------------------------------------------------------------------------

class Tableau:
    def __init__(self, n: int, rng: Optional[random.Random] = None, forced: int = 0):
        self.n = n
        self.x = np.zeros((2 * n + 1, n), dtype=np.uint8)
        self.z = np.zeros((2 * n + 1, n), dtype=np.uint8)
        self.r = np.zeros(2 * n + 1, dtype=np.uint8)
        for i in range(n):
            self.x[i, i] = 1
            self.z[n + i, i] = 1
        self.rng = rng
        self.forced = forced

    def copy(self) -> "Tableau":
        t = Tableau.__new__(Tableau)
        t.n, t.rng, t.forced = self.n, self.rng, self.forced
        t.x, t.z, t.r = self.x.copy(), self.z.copy(), self.r.copy()
        return t

    # Clifford generators
    def h(self, a):
        x, z = self.x, self.z
        self.r ^= x[:, a] & z[:, a]
        x[:, a], z[:, a] = z[:, a].copy(), x[:, a].copy()

    def s(self, a):
        self.r ^= self.x[:, a] & self.z[:, a]
        self.z[:, a] ^= self.x[:, a]

    def cx(self, a, b):
        x, z = self.x, self.z
        self.r ^= x[:, a] & z[:, b] & (x[:, b] ^ z[:, a] ^ 1)
        x[:, b] ^= x[:, a]
        z[:, a] ^= z[:, b]

    def pauli(self, q, px, pz):
        # conjugating by a Pauli flips the sign of every row that anticommutes
        self.r ^= (self.z[:, q] & px) ^ (self.x[:, q] & pz)

    def _rowsum(self, h, i):
        x1, z1 = self.x[i].astype(np.int64), self.z[i].astype(np.int64)
        x2, z2 = self.x[h].astype(np.int64), self.z[h].astype(np.int64)
        g = np.where((x1 == 1) & (z1 == 1), z2 - x2,
            np.where((x1 == 1) & (z1 == 0), z2 * (2 * x2 - 1),
            np.where((x1 == 0) & (z1 == 1), x2 * (1 - 2 * z2), 0)))
        tot = (2 * int(self.r[h]) + 2 * int(self.r[i]) + int(g.sum())) % 4
        self.r[h] = 1 if tot == 2 else 0
        self.x[h] ^= self.x[i]
        self.z[h] ^= self.z[i]

    def measure(self, a) -> Tuple[int, bool]:
        """Z measurement of qubit a -> (outcome, was_random)."""
        n = self.n
        ps = np.nonzero(self.x[n:2 * n, a])[0]
        if len(ps):
            p = n + int(ps[0])
            for i in range(2 * n):
                if i != p and self.x[i, a]:
                    self._rowsum(i, p)
            self.x[p - n], self.z[p - n], self.r[p - n] = self.x[p], self.z[p], self.r[p]
            self.x[p] = 0
            self.z[p] = 0
            self.z[p, a] = 1
            out = self.rng.randint(0, 1) if self.rng is not None else self.forced
            self.r[p] = out
            return out, True
        s = 2 * n
        self.x[s] = 0
        self.z[s] = 0
        self.r[s] = 0
        for i in range(n):
            if self.x[i, a]:
                self._rowsum(s, i + n)
        return int(self.r[s]), False


# ---------------------------------------------------------------------------
# State-vector simulator (a few qubits)
# ---------------------------------------------------------------------------

_I2 = np.eye(2, dtype=complex)
_H = np.array([[1, 1], [1, -1]], dtype=complex) / np.sqrt(2)
_S = np.array([[1, 0], [0, 1j]], dtype=complex)
_X = np.array([[0, 1], [1, 0]], dtype=complex)
_Y = np.array([[0, -1j], [1j, 0]], dtype=complex)
_Z = np.array([[1, 0], [0, -1]], dtype=complex)
_SX = np.array([[1 + 1j, 1 - 1j], [1 - 1j, 1 + 1j]], dtype=complex) / 2
ONE_Q = {"H": _H, "S": _S, "S_DAG": _S.conj().T, "SQRT_X": _SX, "SQRT_X_DAG": _SX.conj().T,
         "X": _X, "Y": _Y, "Z": _Z, "I": _I2}


class StateVector:
    def __init__(self, n: int, forced: int = 0):
        self.n = n
        self.psi = np.zeros([2] * n, dtype=complex)
        self.psi[(0,) * n] = 1.0
        self.forced = forced

    def copy(self) -> "StateVector":
        t = StateVector.__new__(StateVector)
        t.n, t.forced, t.psi = self.n, self.forced, self.psi.copy()
        return t

    def apply1(self, u, q):
        self.psi = np.moveaxis(np.tensordot(u, self.psi, axes=([1], [q])), 0, q)

    def apply2(self, u4, a, b):
        u = u4.reshape(2, 2, 2, 2)
        self.psi = np.moveaxis(np.tensordot(u, self.psi, axes=([2, 3], [a, b])), [0, 1], [a, b])

    def h(self, a):
        self.apply1(_H, a)

    def s(self, a):
        self.apply1(_S, a)

    def cx(self, a, b):
        u = np.eye(4, dtype=complex)[[0, 1, 3, 2]]
        self.apply2(u, a, b)

    def pauli(self, q, px, pz):
        if pz:
            self.apply1(_Z, q)
        if px:
            self.apply1(_X, q)

    def measure(self, a) -> Tuple[int, bool]:
        p1 = float(np.sum(np.abs(np.take(self.psi, 1, axis=a)) ** 2))
        p0 = 1.0 - p1
        rnd = p0 > 1e-9 and p1 > 1e-9
        out = self.forced if rnd else (1 if p1 > 0.5 else 0)
        proj = np.zeros(2)
        proj[out] = 1.0
        self.psi = self.psi * proj.reshape([2 if k == a else 1 for k in range(self.n)])
        self.psi /= np.linalg.norm(self.psi)
        return out, rnd


# ---------------------------------------------------------------------------
# Running a circuit
# ---------------------------------------------------------------------------

def _apply(sim, ins: Instr):
    """Apply one non-noise instruction; return list of measurement outcomes."""
    name, t = ins.name, ins.targets
    rec = []
    if name == "H":
        for q in t:
            sim.h(q)
    elif name in ("S", "S_DAG", "SQRT_X", "SQRT_X_DAG", "X", "Y", "Z", "I"):
        for q in t:
            if isinstance(sim, StateVector):
                sim.apply1(ONE_Q[name], q)
            elif name == "S":
                sim.s(q)
            elif name == "S_DAG":
                sim.s(q); sim.s(q); sim.s(q)
            elif name == "SQRT_X":
                sim.h(q); sim.s(q); sim.h(q)
            elif name == "SQRT_X_DAG":
                sim.h(q); sim.s(q); sim.s(q); sim.s(q); sim.h(q)
            elif name == "X":
                sim.pauli(q, 1, 0)
            elif name == "Y":
                sim.pauli(q, 1, 1)
            elif name == "Z":
                sim.pauli(q, 0, 1)
    elif name in ("CX", "CZ", "SWAP"):
        for i in range(0, len(t), 2):
            a, b = t[i], t[i + 1]
            if name == "CX":
                sim.cx(a, b)
            elif name == "CZ":
                sim.h(b); sim.cx(a, b); sim.h(b)
            else:
                sim.cx(a, b); sim.cx(b, a); sim.cx(a, b)
    elif name in ("R", "RX"):
        for q in t:
            if name == "RX":
                sim.h(q)
            m, _ = sim.measure(q)
            if m:
                sim.pauli(q, 1, 0)
            if name == "RX":
                sim.h(q)
    elif name in ("M", "MX", "MR", "MRX"):
        for q in t:
            xb = name in ("MX", "MRX")
            if xb:
                sim.h(q)
            m, _ = sim.measure(q)
            rec.append(m)
            if name in ("MR", "MRX") and m:
                sim.pauli(q, 1, 0)
            if xb:
                sim.h(q)
    elif name in ("TICK", "QUBIT_COORDS", "SHIFT_COORDS", "DETECTOR", "OBSERVABLE_INCLUDE"):
        pass
    else:
        raise ValueError(f"unsupported {name}")
    return rec


def n_qubits(instrs: Sequence[Instr]) -> int:
    m = -1
    for ins in instrs:
        if ins.name not in ("DETECTOR", "OBSERVABLE_INCLUDE", "TICK", "QUBIT_COORDS", "SHIFT_COORDS"):
            if ins.targets:
                m = max(m, max(ins.targets))
    return m + 1


def _annotations(instrs: Sequence[Instr]):
    """Detector and observable definitions as lists of absolute measurement ids."""
    nm = 0
    dets: List[List[int]] = []
    obs: Dict[int, List[int]] = {}
    for ins in instrs:
        if ins.name in ("M", "MX", "MR", "MRX"):
            nm += len(ins.targets)
        elif ins.name == "DETECTOR":
            dets.append([nm - k for k in ins.targets])
        elif ins.name == "OBSERVABLE_INCLUDE":
            obs.setdefault(int(ins.args[0]), []).extend(nm - k for k in ins.targets)
    nobs = (max(obs) + 1) if obs else 0
    return dets, [obs.get(k, []) for k in range(nobs)]


def _values(rec, dets, obs):
    dv = [sum(rec[m] for m in d) % 2 for d in dets]
    ov = [sum(rec[m] for m in o) % 2 for o in obs]
    return dv + ov


class Runner:
    """Simulates a circuit once, keeping a checkpoint before every noise
    instruction, then replays the suffix for each injected fault."""

    def __init__(self, text: str, engine: str = "tableau", forced: int = 0, seed: Optional[int] = None):
        self.instrs = parse(text)
        self.n = n_qubits(self.instrs)
        self.dets, self.obs = _annotations(self.instrs)
        self.chans = channels(self.instrs)
        rng = random.Random(seed) if seed is not None else None
        if engine == "tableau":
            sim = Tableau(self.n, rng=rng, forced=forced)
        else:
            sim = StateVector(self.n, forced=forced)
        self.checkpoints: Dict[int, Tuple[object, int]] = {}
        rec: List[int] = []
        for k, ins in enumerate(self.instrs):
            if ins.name in NOISE1 or ins.name == "DEPOLARIZE2":
                self.checkpoints[k] = (sim.copy(), len(rec))
                continue
            rec += _apply(sim, ins)
        self.record = rec
        self.values = _values(rec, self.dets, self.obs)

    def signature(self, channel: int, code: int) -> Tuple[int, ...]:
        """Flipped detector/observable indices when channel `channel` fires with
        Pauli `code` (bit0 x on first qubit, bit1 z on first, bit2 x on second,
        bit3 z on second)."""
        k, _, qs, _ = self.chans[channel]
        sim0, nrec = self.checkpoints[k]
        sim = sim0.copy()
        rec = list(self.record[:nrec])
        sim.pauli(qs[0], code & 1, (code >> 1) & 1)
        if len(qs) == 2:
            sim.pauli(qs[1], (code >> 2) & 1, (code >> 3) & 1)
        for ins in self.instrs[k + 1:]:
            if ins.name in NOISE1 or ins.name == "DEPOLARIZE2":
                continue
            rec += _apply(sim, ins)
        vals = _values(rec, self.dets, self.obs)
        return tuple(i for i, (a, b) in enumerate(zip(vals, self.values)) if a != b)


def channel_paulis(kind: str) -> List[int]:
    """Every non-identity Pauli a channel of this kind can apply, as codes."""
    if kind == "X_ERROR":
        return [1]
    if kind == "Y_ERROR":
        return [3]
    if kind == "Z_ERROR":
        return [2]
    if kind == "DEPOLARIZE1":
        return [1, 3, 2]
    out = []
    for a in range(4):
        for b in range(4):
            if a or b:
                out.append(a | (b << 2))
    return out


def pauli_probability(kind: str, rate: float) -> float:
    """Probability of one specific non-identity Pauli in the channel's own
    definition (not an independent split): r for flips, r/3 and r/15 for the
    depolarising channels."""
    if kind in ("X_ERROR", "Y_ERROR", "Z_ERROR"):
        return rate
    if kind == "DEPOLARIZE1":
        return rate / 3.0
    return rate / 15.0
