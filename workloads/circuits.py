"""Generators of realised, fully unrolled Clifford syndrome-measurement circuits.

Every generator returns a :class:`Circuit` holding Stim-format text (the circuit
language subset accepted by the compiler) plus the counts a caller needs to
build a per-channel rate array. Channels are enumerated in program order and,
within one noise instruction, in target-group order (one qubit, or one pair for
DEPOLARIZE2); this is the order in which a rate array overrides the rates
written in the text.

Workloads follow the paper's evaluation (Sec. 4): Z-basis memory experiments of
the rotated surface code and of the bivariate bicycle code [[144,12,12]], d
rounds, no REPEAT blocks, with circuit-level noise (Sec. 2.1.3): DEPOLARIZE1
after single-qubit gates and resets, DEPOLARIZE2 after each CX, X_ERROR before
each measurement. No idle noise is inserted.
"""

from __future__ import annotations

import dataclasses
import random
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np


# Operation codes of the compiler's binary circuit form (gp_circuit_ir in
# include/gp.h): the same circuit as the text, one entry per elementary
# operation in program order.
IR_CODES = {
    "I": 0, "X": 0, "Y": 0, "Z": 0,
    "H": 1, "H_XZ": 1, "S": 2, "S_DAG": 2, "SQRT_Z": 2, "SQRT_Z_DAG": 2, "SQRT_X": 3, "SQRT_X_DAG": 3,
    "CX": 4, "CNOT": 4, "ZCX": 4, "CZ": 5, "ZCZ": 5, "SWAP": 6,
    "R": 7, "RZ": 7, "RX": 8, "M": 9, "MZ": 9, "MX": 10, "MR": 11, "MRZ": 11, "MRX": 12,
    "X_ERROR": 16, "Y_ERROR": 17, "Z_ERROR": 18, "DEPOLARIZE1": 19, "DEPOLARIZE2": 20,
    "DETECTOR": 32, "OBSERVABLE_INCLUDE": 33,
}
_TWO_QUBIT = {"CX", "CNOT", "ZCX", "CZ", "ZCZ", "SWAP"}


@dataclasses.dataclass
class Circuit:
    text: str
    n_qubits: int
    n_channels: int
    n_measurements: int
    n_detectors: int
    n_observables: int
    rounds: int
    name: str
    #: the same circuit in binary form: arrays "code" (uint8), "q0", "q1"
    #: (uint32), "rate" (float64), one entry per operation, and "rec" (uint32,
    #: absolute measurement indices of the detectors' and observables' records)
    ir: Optional[Dict[str, np.ndarray]] = None

    def channel_kinds(self) -> List[str]:
        """Noise instruction name of each channel, in channel order."""
        kinds: List[str] = []
        for line in self.text.splitlines():
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            head = line.split()[0]
            name = head.split("(")[0].upper()
            tail = line[len(head):].split()
            if name in ("X_ERROR", "Y_ERROR", "Z_ERROR", "DEPOLARIZE1"):
                kinds += [name] * len(tail)
            elif name == "DEPOLARIZE2":
                kinds += [name] * (len(tail) // 2)
        return kinds


class _Builder:
    """Accumulates circuit text and keeps the running counts."""

    def __init__(self) -> None:
        self.lines: List[str] = []
        self.n_meas = 0
        self.n_det = 0
        self.n_obs = 0
        self.n_chan = 0
        self.max_q = -1
        # binary form: parallel lists, one entry per operation
        self._code: List[int] = []
        self._q0: List[int] = []
        self._q1: List[int] = []
        self._rate: List[float] = []
        self._rec: List[int] = []

    def _touch(self, qs: Sequence[int]) -> None:
        if qs:
            self.max_q = max(self.max_q, max(qs))

    def _op(self, name: str, q0: Sequence[int], q1, rate: float = 0.0) -> None:
        n = len(q0)
        self._code.extend([IR_CODES[name]] * n)
        self._q0.extend(q0)
        self._q1.extend([q1] * n if isinstance(q1, int) else q1)
        self._rate.extend([rate] * n)

    def gate(self, name: str, qs: Sequence[int]) -> None:
        if len(qs) == 0:
            return
        self._touch(qs)
        self.lines.append(name + " " + " ".join(str(q) for q in qs))
        if name in _TWO_QUBIT:
            self._op(name, qs[0::2], qs[1::2])
        else:
            self._op(name, qs, 0)

    def pairs(self, name: str, ps: Sequence[Tuple[int, int]]) -> None:
        flat = [q for p in ps for q in p]
        self.gate(name, flat)

    def noise1(self, name: str, p: float, qs: Sequence[int]) -> None:
        if len(qs) == 0 or p is None:
            return
        self._touch(qs)
        self.lines.append(f"{name}({p!r}) " + " ".join(str(q) for q in qs))
        self.n_chan += len(qs)
        self._op(name, qs, 0, p)

    def noise2(self, p: float, ps: Sequence[Tuple[int, int]]) -> None:
        if len(ps) == 0 or p is None:
            return
        flat = [q for pr in ps for q in pr]
        self._touch(flat)
        self.lines.append(f"DEPOLARIZE2({p!r}) " + " ".join(str(q) for q in flat))
        self.n_chan += len(ps)
        self._op("DEPOLARIZE2", flat[0::2], flat[1::2], p)

    def measure(self, name: str, qs: Sequence[int]) -> List[int]:
        """Emit a measurement instruction; return absolute measurement indices."""
        self.gate(name, qs)
        idx = list(range(self.n_meas, self.n_meas + len(qs)))
        self.n_meas += len(qs)
        return idx

    def _recs(self, meas: Sequence[int]) -> str:
        return " ".join(f"rec[{m - self.n_meas}]" for m in meas)

    def detector(self, meas: Sequence[int], coords: Optional[Sequence[float]] = None) -> int:
        c = "" if coords is None else "(" + ", ".join(repr(float(x)) for x in coords) + ")"
        self.lines.append(f"DETECTOR{c} " + self._recs(meas))
        self.n_det += 1
        self._op("DETECTOR", [0], [len(meas)])
        self._rec.extend(meas)
        return self.n_det - 1

    def observable(self, k: int, meas: Sequence[int]) -> None:
        self.lines.append(f"OBSERVABLE_INCLUDE({k}) " + self._recs(meas))
        self.n_obs = max(self.n_obs, k + 1)
        self._op("OBSERVABLE_INCLUDE", [k], [len(meas)])
        self._rec.extend(meas)

    def binary(self) -> Dict[str, np.ndarray]:
        """The circuit so far in the compiler's binary form."""
        return {"code": np.array(self._code, dtype=np.uint8), "q0": np.array(self._q0, dtype=np.uint32),
                "q1": np.array(self._q1, dtype=np.uint32), "rate": np.array(self._rate, dtype=np.float64),
                "rec": np.array(self._rec, dtype=np.uint32)}

    def tick(self) -> None:
        self.lines.append("TICK")

    def build(self, rounds: int, name: str, n_qubits: Optional[int] = None) -> Circuit:
        return Circuit(
            text="\n".join(self.lines) + "\n",
            n_qubits=(self.max_q + 1) if n_qubits is None else n_qubits,
            n_channels=self.n_chan,
            n_measurements=self.n_meas,
            n_detectors=self.n_det,
            n_observables=self.n_obs,
            rounds=rounds,
            name=name,
            ir=self.binary(),
        )


# ---------------------------------------------------------------------------
# Rotated surface code
# ---------------------------------------------------------------------------

def _rotated_layout(d: int):
    """Data qubit (r, c) -> r*d + c. Plaquette with corner index (i, j),
    0 <= i, j <= d, covers data (i-1, j-1), (i-1, j), (i, j-1), (i, j).
    Checkerboard: X type if (i + j) is even. Weight-2 plaquettes are kept on the
    top/bottom edges for X type and on the left/right edges for Z type.
    Returns lists of (type, corners) with corners = (TL, TR, BL, BR), None where
    the corner falls outside the lattice."""
    plaqs = []
    for i in range(d + 1):
        for j in range(d + 1):
            typ = "X" if (i + j) % 2 == 0 else "Z"
            interior = 1 <= i <= d - 1 and 1 <= j <= d - 1
            top_bottom = (i == 0 or i == d) and 1 <= j <= d - 1
            left_right = (j == 0 or j == d) and 1 <= i <= d - 1
            if not (interior or (top_bottom and typ == "X") or (left_right and typ == "Z")):
                continue

            def dq(r, c):
                return r * d + c if (0 <= r < d and 0 <= c < d) else None

            corners = (dq(i - 1, j - 1), dq(i - 1, j), dq(i, j - 1), dq(i, j))
            plaqs.append((typ, corners))
    return plaqs


def paper_noise(p: float) -> Dict[str, object]:
    """The paper's hardware-inspired preset (Sec. 4): p1 = pi = p/10 and
    p2 = pr = pm = p, with idle noise and resets that fail by a bit flip."""
    return {"p1": p / 10, "pi": p / 10, "p2": p, "pr": p, "pm": p, "reset_noise": "X_ERROR"}


def rotated_surface_code_memory(d: int, rounds: int, p: float = 1e-3,
                                p1: Optional[float] = None, p2: Optional[float] = None,
                                pm: Optional[float] = None, pr: Optional[float] = None,
                                pi: float = 0.0, reset_noise: str = "DEPOLARIZE1",
                                x_detectors: bool = True, ticks: bool = True) -> Circuit:
    """Z-basis memory of the distance-d rotated surface code, `rounds` rounds.

    CX order: X checks visit (TL, TR, BL, BR) ("Z" shape), Z checks visit
    (TL, BL, TR, BR) ("N" shape), so that hook errors of each type run
    perpendicular to the logical operator of the same type. Detectors: first
    round Z checks, consecutive-round parity of every check (X checks only if
    `x_detectors`), final data parity of every Z check. Observable 0: Z on data
    row 0. Noise: DEPOLARIZE1(p1) after one-qubit gates, DEPOLARIZE2(p2) after
    CX, X_ERROR(pm) before measurements, `reset_noise`(pr) after resets, and
    DEPOLARIZE1(pi) on the qubits idle in a gate layer when pi > 0.
    """
    p1 = p if p1 is None else p1
    p2 = p if p2 is None else p2
    pm = p if pm is None else pm
    pr = p if pr is None else pr
    plaqs = _rotated_layout(d)
    n_data = d * d
    anc = [n_data + k for k in range(len(plaqs))]
    xanc = [anc[k] for k, (t, _) in enumerate(plaqs) if t == "X"]
    zanc = [anc[k] for k, (t, _) in enumerate(plaqs) if t == "Z"]
    data = list(range(n_data))
    allq = data + anc
    order_x = (0, 1, 2, 3)
    order_z = (0, 2, 1, 3)
    b = _Builder()
    busy_h = set(xanc)
    idle_h = [q for q in allq if q not in busy_h]

    def idle(qs):
        if pi > 0 and qs:
            b.noise1("DEPOLARIZE1", pi, qs)

    b.gate("R", allq)
    b.noise1(reset_noise, pr, allq)
    if ticks:
        b.tick()
    last: Dict[int, int] = {}
    for rnd in range(rounds):
        b.gate("H", xanc)
        b.noise1("DEPOLARIZE1", p1, xanc)
        idle(idle_h)
        if ticks:
            b.tick()
        for layer in range(4):
            pairs = []
            for k, (typ, corners) in enumerate(plaqs):
                slot = order_x[layer] if typ == "X" else order_z[layer]
                q = corners[slot]
                if q is None:
                    continue
                pairs.append((anc[k], q) if typ == "X" else (q, anc[k]))
            b.pairs("CX", pairs)
            b.noise2(p2, pairs)
            busy = {q for pr_ in pairs for q in pr_}
            idle([q for q in allq if q not in busy])
            if ticks:
                b.tick()
        b.gate("H", xanc)
        b.noise1("DEPOLARIZE1", p1, xanc)
        idle(idle_h)
        if ticks:
            b.tick()
        b.noise1("X_ERROR", pm, anc)
        ms = b.measure("MR", anc)
        b.noise1(reset_noise, pr, anc)
        idle(data)
        cur = dict(zip(anc, ms))
        for k, (typ, _) in enumerate(plaqs):
            a = anc[k]
            if rnd == 0:
                if typ == "Z":
                    b.detector([cur[a]])
            elif typ == "Z" or x_detectors:
                b.detector([cur[a], last[a]])
        last = cur
        if ticks:
            b.tick()
    b.noise1("X_ERROR", pm, data)
    mdata = dict(zip(data, b.measure("M", data)))
    for k, (typ, corners) in enumerate(plaqs):
        if typ != "Z":
            continue
        ms = [mdata[q] for q in corners if q is not None]
        b.detector(ms + [last[anc[k]]])
    b.observable(0, [mdata[c] for c in range(d)])
    return b.build(rounds, f"rotated_surface_code_d{d}_r{rounds}")


def rotated_surface_code_checks(d: int):
    """(H_X, H_Z) parity-check matrices of the layout used above (tests only)."""
    plaqs = _rotated_layout(d)
    hx, hz = [], []
    for typ, corners in plaqs:
        row = np.zeros(d * d, dtype=np.uint8)
        for q in corners:
            if q is not None:
                row[q] = 1
        (hx if typ == "X" else hz).append(row)
    return np.array(hx), np.array(hz)


# ---------------------------------------------------------------------------
# Repetition code and the bit-flip example of the paper's Fig. 1
# ---------------------------------------------------------------------------

def repetition_code_memory(d: int, rounds: int, p_data: float = 0.0, p_meas: float = 0.0,
                           p2: float = 0.0, p1: float = 0.0,
                           data_noise: str = "X_ERROR") -> Circuit:
    """Bit-flip repetition code: data 0..d-1, ancilla d+i checks Z_i Z_{i+1}.

    p_data: `data_noise` on every data qubit before each round
    (phenomenological-style); p_meas: X_ERROR before each measurement;
    p2: DEPOLARIZE2 after every CX; p1: DEPOLARIZE1 after every reset.
    A rate of 0 omits the channel. Observable 0: final measurement of data 0.
    """
    data = list(range(d))
    anc = [d + i for i in range(d - 1)]
    b = _Builder()
    b.gate("R", data + anc)
    if p1:
        b.noise1("DEPOLARIZE1", p1, data + anc)
    b.tick()
    last: Dict[int, int] = {}
    for rnd in range(rounds):
        if p_data:
            b.noise1(data_noise, p_data, data)
        for off in (0, 1):
            pairs = [(i + off, anc[i]) for i in range(d - 1)]
            b.pairs("CX", pairs)
            if p2:
                b.noise2(p2, pairs)
            b.tick()
        if p_meas:
            b.noise1("X_ERROR", p_meas, anc)
        ms = b.measure("MR", anc)
        if p1:
            b.noise1("DEPOLARIZE1", p1, anc)
        cur = dict(zip(anc, ms))
        for a in anc:
            b.detector([cur[a]] if rnd == 0 else [cur[a], last[a]])
        last = cur
        b.tick()
    if p_meas:
        b.noise1("X_ERROR", p_meas, data)
    md = b.measure("M", data)
    for i, a in enumerate(anc):
        b.detector([md[i], md[i + 1], last[a]])
    b.observable(0, [md[0]])
    return b.build(rounds, f"repetition_d{d}_r{rounds}")


def bit_flip_code_fig1(error_after_second_cnot_layer: bool = True) -> Circuit:
    """The d = 3 bit-flip code of the paper's Fig. 1 over two rounds.

    Qubits 0, 2, 4 are data, 1 and 3 are ancillas. Round: CX 0->1, 2->3; then
    CX 2->1, 4->3; then MR 1 3. Detectors in declaration order: orange (first
    measurement of ancilla 1), green (first measurement of ancilla 3), blue
    (parity of the two ancilla-1 measurements), yellow (same for ancilla 3).
    The single noise channel is an X error on data qubit 2 placed after the
    second CNOT layer of the first round (the error called E12 in the figure).
    """
    b = _Builder()
    b.gate("R", [0, 1, 2, 3, 4])
    b.tick()
    ms_rounds = []
    for rnd in range(2):
        b.pairs("CX", [(0, 1), (2, 3)])
        b.tick()
        b.pairs("CX", [(2, 1), (4, 3)])
        if rnd == 0 and error_after_second_cnot_layer:
            b.noise1("X_ERROR", 0.01, [2])
        b.tick()
        ms_rounds.append(b.measure("MR", [1, 3]))
        b.tick()
    (a1, a3), (b1, b3) = ms_rounds
    b.detector([a1])       # orange
    b.detector([a3])       # green
    b.detector([a1, b1])   # blue
    b.detector([a3, b3])   # yellow
    return b.build(2, "bit_flip_fig1", n_qubits=5)


# ---------------------------------------------------------------------------
# Bivariate bicycle code [[144,12,12]]
# ---------------------------------------------------------------------------

def _shift(n: int, k: int) -> np.ndarray:
    m = np.zeros((n, n), dtype=np.uint8)
    for i in range(n):
        m[i, (i + k) % n] = 1
    return m


def bb_matrices(l: int = 12, m: int = 6):
    """A = x^3 + y + y^2, B = y^3 + x + x^2 with x = S_l (x) I_m, y = I_l (x) S_m.
    Returns the three permutation terms of A and of B."""
    x = np.kron(_shift(l, 1), np.eye(m, dtype=np.uint8))
    y = np.kron(np.eye(l, dtype=np.uint8), _shift(m, 1))

    def mpow(a, k):
        r = np.eye(a.shape[0], dtype=np.uint8)
        for _ in range(k):
            r = (r @ a) % 2
        return r.astype(np.uint8)

    a_terms = [mpow(x, 3), mpow(y, 1), mpow(y, 2)]
    b_terms = [mpow(y, 3), mpow(x, 1), mpow(x, 2)]
    return a_terms, b_terms


def _gf2_rank(mat: np.ndarray) -> int:
    a = (mat.copy() % 2).astype(np.uint8)
    rank = 0
    rows, cols = a.shape
    for c in range(cols):
        piv = None
        for r in range(rank, rows):
            if a[r, c]:
                piv = r
                break
        if piv is None:
            continue
        a[[rank, piv]] = a[[piv, rank]]
        for r in range(rows):
            if r != rank and a[r, c]:
                a[r] ^= a[rank]
        rank += 1
        if rank == rows:
            break
    return rank


def _gf2_nullspace(mat: np.ndarray) -> np.ndarray:
    a = (mat.copy() % 2).astype(np.uint8)
    rows, cols = a.shape
    pivots = []
    r = 0
    for c in range(cols):
        piv = None
        for k in range(r, rows):
            if a[k, c]:
                piv = k
                break
        if piv is None:
            continue
        a[[r, piv]] = a[[piv, r]]
        for k in range(rows):
            if k != r and a[k, c]:
                a[k] ^= a[r]
        pivots.append(c)
        r += 1
        if r == rows:
            break
    free = [c for c in range(cols) if c not in pivots]
    basis = []
    for f in free:
        v = np.zeros(cols, dtype=np.uint8)
        v[f] = 1
        for i, pc in enumerate(pivots):
            if a[i, f]:
                v[pc] = 1
        basis.append(v)
    return np.array(basis, dtype=np.uint8)


def bb_check_matrices(l: int = 12, m: int = 6):
    a_terms, b_terms = bb_matrices(l, m)
    a = sum(a_terms) % 2
    bm = sum(b_terms) % 2
    hx = np.concatenate([a, bm], axis=1).astype(np.uint8)
    hz = np.concatenate([bm.T, a.T], axis=1).astype(np.uint8)
    return hx, hz


def bb_logical_z(l: int = 12, m: int = 6) -> np.ndarray:
    """Basis of Z-type logical operators: ker(H_X) modulo rowspace(H_Z)."""
    hx, hz = bb_check_matrices(l, m)
    ker = _gf2_nullspace(hx)
    chosen: List[np.ndarray] = []
    base_rank = _gf2_rank(hz)
    cur = hz.copy()
    for v in ker:
        trial = np.concatenate([cur, v[None, :]], axis=0)
        if _gf2_rank(trial) > base_rank + len(chosen):
            chosen.append(v)
            cur = trial
    return np.array(chosen, dtype=np.uint8)


# Depth-8 syndrome cycle of a bivariate bicycle code: the CX slot (0..6) of
# each permutation term, X checks (A_k on L data, B_k on R data) and Z checks
# (B_k^T on L data, A_k^T on R data), then one slot of measure-and-reset.
# Chosen by exhaustive search over slot assignments in which every ancilla and
# every data qubit meets at most one CX per slot, subject to the condition that
# makes the interleaved X and Z checks measure the stabilisers: an X check and
# a Z check that share data qubits through the terms (A_k, B_m^T) on L and
# (B_m, A_k^T) on R see those two qubits in the same relative order
# (slot(A_k) > slot(B_m^T) exactly when slot(B_m) > slot(A_k^T)); with the nine
# sums a_k + b_m distinct, this is the condition term pair by term pair.
BB_DEPTH8_SLOTS = {"A": (0, 1, 5), "B": (2, 3, 4), "BT": (2, 3, 4), "AT": (5, 6, 1)}


def bivariate_bicycle_memory(rounds: int = 12, p: float = 1e-3, l: int = 12, m: int = 6,
                             schedule: str = "depth8", p1: Optional[float] = None, p2: Optional[float] = None,
                             pm: Optional[float] = None, pr: Optional[float] = None, pi: float = 0.0,
                             reset_noise: str = "DEPOLARIZE1") -> Circuit:
    """Z-basis memory of the bivariate bicycle code (default [[144,12,12]]).

    Qubits: L data 0..lm-1, R data lm..2lm-1, X ancillas, then Z ancillas.
    schedule "depth8" (default): X ancillas are prepared and read in the X
    basis (RX, then MRX each round), and the twelve permutation terms run in
    seven CX slots (BB_DEPTH8_SLOTS) followed by one slot of measure-and-reset:
    eight layers per round. schedule "sequential": X ancillas use H ... H and
    MR, the six terms of [A|B] run as six CX layers, then the six terms of
    [B^T|A^T] onto the Z ancillas. Noise: DEPOLARIZE1 after every one-qubit
    gate and reset, DEPOLARIZE2 after every CX, a flip before every
    measurement (Z_ERROR before an X-basis one, X_ERROR before a Z-basis one).
    The rates default to p; p1 (one-qubit gates), p2 (CX), pm (measurements),
    pr (resets) and pi (DEPOLARIZE1 on the qubits idle in a gate or
    measurement layer, when pi > 0) set them apart, as in the paper's preset
    (`paper_noise`). reset_noise "X_ERROR" makes a reset fail by a flip in its
    own basis (X_ERROR after a Z-basis reset, Z_ERROR after an X-basis one).
    """
    if schedule not in ("depth8", "sequential"):
        raise ValueError(f"unknown schedule {schedule!r}")
    if reset_noise not in ("DEPOLARIZE1", "X_ERROR"):
        raise ValueError(f"unknown reset noise {reset_noise!r}")
    p1 = p if p1 is None else p1
    p2 = p if p2 is None else p2
    pm = p if pm is None else pm
    pr = p if pr is None else pr
    nd = l * m
    a_terms, b_terms = bb_matrices(l, m)
    L = list(range(nd))
    R = list(range(nd, 2 * nd))
    xa = list(range(2 * nd, 3 * nd))
    za = list(range(3 * nd, 4 * nd))
    anc = xa + za
    data = L + R
    allq = data + anc
    b = _Builder()

    def reset_noise_on(z_basis, x_basis):
        # after resets: one DEPOLARIZE1 over both sets, or a flip in each set's basis
        if reset_noise == "DEPOLARIZE1":
            b.noise1("DEPOLARIZE1", pr, list(z_basis) + list(x_basis))
        else:
            if z_basis:
                b.noise1("X_ERROR", pr, z_basis)
            if x_basis:
                b.noise1("Z_ERROR", pr, x_basis)

    def idle(qs):
        if pi > 0 and qs:
            b.noise1("DEPOLARIZE1", pi, qs)

    def x_pairs(blk, t):   # X check i -> its data qubit of term t
        return [(xa[i], blk[int(np.nonzero(t[i])[0][0])]) for i in range(nd)]

    def z_pairs(blk, t):   # data qubit of term t^T of Z check i -> Z check i
        tt = t.T
        return [(blk[int(np.nonzero(tt[i])[0][0])], za[i]) for i in range(nd)]

    if schedule == "depth8":
        b.gate("R", data + za)
        b.gate("RX", xa)
        if reset_noise == "DEPOLARIZE1":
            b.noise1("DEPOLARIZE1", pr, allq)
        else:
            reset_noise_on(data + za, xa)
        b.tick()
        slots = [[] for _ in range(7)]
        for k in range(3):
            slots[BB_DEPTH8_SLOTS["A"][k]] += x_pairs(L, a_terms[k])
            slots[BB_DEPTH8_SLOTS["B"][k]] += x_pairs(R, b_terms[k])
            slots[BB_DEPTH8_SLOTS["BT"][k]] += z_pairs(L, b_terms[k])
            slots[BB_DEPTH8_SLOTS["AT"][k]] += z_pairs(R, a_terms[k])
    else:
        b.gate("R", allq)
        reset_noise_on(allq, [])
        b.tick()
    last: Dict[int, int] = {}
    for rnd in range(rounds):
        if schedule == "depth8":
            for pairs in slots:
                b.pairs("CX", pairs)
                b.noise2(p2, pairs)
                busy = {q for pr_ in pairs for q in pr_}
                idle([q for q in allq if q not in busy])
                b.tick()
            b.noise1("Z_ERROR", pm, xa)
            b.noise1("X_ERROR", pm, za)
            mx = b.measure("MRX", xa)
            mz = b.measure("MR", za)
            ms = mx + mz
            if reset_noise == "DEPOLARIZE1":
                b.noise1("DEPOLARIZE1", pr, anc)
            else:
                reset_noise_on(za, xa)
            idle(data)
        else:
            b.gate("H", xa)
            b.noise1("DEPOLARIZE1", p1, xa)
            idle([q for q in allq if q not in set(xa)])
            b.tick()
            # X checks: row i of A (on L) and of B (on R).
            for blk, terms in ((L, a_terms), (R, b_terms)):
                for t in terms:
                    pairs = x_pairs(blk, t)
                    b.pairs("CX", pairs)
                    b.noise2(p2, pairs)
                    busy = {q for pr_ in pairs for q in pr_}
                    idle([q for q in allq if q not in busy])
                    b.tick()
            b.gate("H", xa)
            b.noise1("DEPOLARIZE1", p1, xa)
            idle([q for q in allq if q not in set(xa)])
            b.tick()
            # Z checks: row i of B^T (on L) and of A^T (on R).
            for blk, terms in ((L, b_terms), (R, a_terms)):
                for t in terms:
                    pairs = z_pairs(blk, t)
                    b.pairs("CX", pairs)
                    b.noise2(p2, pairs)
                    busy = {q for pr_ in pairs for q in pr_}
                    idle([q for q in allq if q not in busy])
                    b.tick()
            b.noise1("X_ERROR", pm, anc)
            ms = b.measure("MR", anc)
            reset_noise_on(anc, [])
            idle(data)
        cur = dict(zip(anc, ms))
        if rnd == 0:
            for a in za:
                b.detector([cur[a]])
        else:
            for a in anc:
                b.detector([cur[a], last[a]])
        last = cur
        b.tick()
    b.noise1("X_ERROR", pm, data)
    md = b.measure("M", data)
    hx, hz = bb_check_matrices(l, m)
    for i, a in enumerate(za):
        supp = np.nonzero(hz[i])[0]
        b.detector([md[int(q)] for q in supp] + [last[a]])
    logicals = bb_logical_z(l, m)
    for k, v in enumerate(logicals):
        b.observable(k, [md[int(q)] for q in np.nonzero(v)[0]])
    tag = "" if schedule == "depth8" else "_seq"
    return b.build(rounds, f"bivariate_bicycle_{2 * nd}_r{rounds}{tag}")


# ---------------------------------------------------------------------------
# Mirror circuits: random Clifford layers followed by their inverse
# ---------------------------------------------------------------------------

_INVERSE = {"H": "H", "S": "S_DAG", "S_DAG": "S", "SQRT_X": "SQRT_X_DAG",
            "SQRT_X_DAG": "SQRT_X", "X": "X", "Y": "Y", "Z": "Z", "I": "I",
            "CX": "CX", "CZ": "CZ", "SWAP": "SWAP"}


def mirror_circuit(n: int, depth: int, seed: int, p: float = 0.05,
                   x_basis: Sequence[int] = ()) -> Circuit:
    """Random layers of {H, S, S_DAG, SQRT_X, SQRT_X_DAG, X, Y, Z, I, CX, CZ,
    SWAP} followed by the inverse layers, so every final measurement is
    deterministic. Qubits listed in `x_basis` are prepared with RX and read with
    MX. A DEPOLARIZE1 / DEPOLARIZE2 follows every gate; Y_ERROR and Z_ERROR
    channels are sprinkled in; one mid-circuit MR on an extra qubit checks
    measurement-reset handling. Every final measurement is a detector (one of
    them listed twice with another record, which must cancel), and observable 0
    is split over two OBSERVABLE_INCLUDE instructions."""
    rng = random.Random(seed)
    one_q = ["H", "S", "S_DAG", "SQRT_X", "SQRT_X_DAG", "X", "Y", "Z", "I"]
    two_q = ["CX", "CZ", "SWAP"]
    layers: List[List[Tuple[str, Tuple[int, ...]]]] = []
    for _ in range(depth):
        qs = list(range(n))
        rng.shuffle(qs)
        layer = []
        while qs:
            if len(qs) >= 2 and rng.random() < 0.5:
                a, c = qs.pop(), qs.pop()
                layer.append((rng.choice(two_q), (a, c)))
            else:
                layer.append((rng.choice(one_q), (qs.pop(),)))
        layers.append(layer)
    b = _Builder()
    zq = [q for q in range(n) if q not in x_basis]
    b.gate("R", zq + [n])
    b.gate("RX", list(x_basis))
    b.noise1("DEPOLARIZE1", p, list(range(n)))
    b.tick()

    def emit(layer, inverse):
        for g, qs in layer:
            name = _INVERSE[g] if inverse else g
            b.gate(name, list(qs))
            if len(qs) == 1:
                b.noise1("DEPOLARIZE1", p, list(qs))
            else:
                b.noise2(p, [qs])
        b.tick()

    for k, layer in enumerate(layers):
        emit(layer, False)
        if k == depth // 2:
            b.noise1("Y_ERROR", p, [0])
            b.noise1("Z_ERROR", p, [n - 1])
    # mid-circuit measure-and-reset of an extra qubit whose outcome is fixed
    b.noise1("X_ERROR", p, [n])
    m_extra = b.measure("MR", [n])
    b.detector(m_extra)
    for layer in reversed(layers):
        emit([(g, qs) for g, qs in reversed(layer)], True)
    b.noise1("X_ERROR", p, zq)
    b.noise1("Z_ERROR", p, list(x_basis))
    mz = dict(zip(zq, b.measure("M", zq)))
    mx = dict(zip(x_basis, b.measure("MX", list(x_basis))))
    allm = {**mz, **mx}
    for q in range(n):
        if q == 0 and n > 1:
            b.detector([allm[0], allm[1], allm[1]])
        else:
            b.detector([allm[q]])
    b.observable(0, [allm[0]])
    if n > 1:
        b.observable(0, [allm[n - 1]])
    return b.build(2 * depth, f"mirror_n{n}_d{depth}_s{seed}", n_qubits=n + 1)
