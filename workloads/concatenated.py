"""Adaptive syndrome measurement of the [[4,2,2]]-concatenated rotated surface
code (paper Sec. 5): seeded realised branches.

Layout. The outer code is the distance-d rotated surface code of
:func:`workloads.circuits.rotated_surface_code_memory`; each outer data qubit
is one logical qubit of an inner [[4,2,2]] (Iceberg) block with stabilisers
XXXX and ZZZZ on physical qubits (0, 1, 2, 3). The two logical qubits of a
block are X1 = X0 X1, Z1 = Z0 Z2 and X2 = X0 X2, Z2 = Z0 Z1 (each logical pair
anticommutes, the cross pairs commute, all commute with the stabilisers).

Pairing (Eq. 6). Outer data (r, c) is paired with (d-1-r, (c+2) mod d). The map
is an involution only when d divides 4; in general it is followed around each
of its cycles and consecutive elements are paired; a cycle of odd length
leaves one qubit, which gets a block of its own with only its first logical
qubit in use. :func:`iceberg_pairing_violations` counts the pairs that break
the two constraints of Sec. 5.1.1 (no outer check on both logical qubits of a
block; no block touched twice in one time step of the outer CX schedule).

Branch (one realised execution path, Sec. 5.2). Every cycle measures the
inner checks of every block, then the outer checks that run this cycle:
  * per cycle and block, a seeded mid-circuit outcome picks the block's inner
    variant: an extra syndrome round (the two inner checks are measured twice)
    or the flag-qubit variant (each inner check gets a flag qubit entangled
    after its first and before its last CX and read out on its own);
  * a second seeded outcome per cycle and block stands for the block's inner
    difference syndrome firing (probability `p_excite`): outer checks with a
    data qubit in a fired block run (Sec. 5.2.2), and every outer check runs
    in the first and last cycle and every `gamma` cycles (the refresh,
    Sec. 5.2.3; gamma = d/2 rounded down, at least 1);
  * detectors are instantiated dynamically (Sec. 5.2.4): a check execution
    gets a detector comparing it with the check's previous execution when
    there is one; a Z-type check's first execution is compared with the
    all-|0> start; a flag is a detector by itself.
Z-basis memory: all physical qubits start in |0>; the data blocks are read
out in the Z basis at the end, closing every Z-type check; observable 0 is
the outer logical Z along outer data row 0.

Noise is the uniform circuit-level model of the other workloads: DEPOLARIZE1
after resets, DEPOLARIZE2 after every CX, X_ERROR before Z-basis and Z_ERROR
before X-basis measurements.
"""

from __future__ import annotations

from typing import Dict, List, Optional, Sequence, Tuple

from .circuits import Circuit, _Builder, _rotated_layout
from .rates import splitmix64_uniform

# physical qubits (within a block) of the logical operators of logical 1 and 2
ICEBERG_X = ((0, 1), (0, 2))
ICEBERG_Z = ((0, 2), (0, 1))
# CX visiting order of outer checks, as in the plain surface-code workload
_ORDER_X = (0, 1, 2, 3)
_ORDER_Z = (0, 2, 1, 3)


def iceberg_pairing(d: int) -> List[Tuple[int, ...]]:
    """Blocks of outer data qubits (index r*d + c): pairs along the cycles of
    (r, c) -> (d-1-r, (c+2) mod d), and a single for each odd cycle's last element."""
    def step(q: int) -> int:
        r, c = divmod(q, d)
        return (d - 1 - r) * d + (c + 2) % d

    seen = [False] * (d * d)
    blocks: List[Tuple[int, ...]] = []
    for q0 in range(d * d):
        if seen[q0]:
            continue
        cyc = []
        q = q0
        while not seen[q]:
            seen[q] = True
            cyc.append(q)
            q = step(q)
        for i in range(0, len(cyc) - 1, 2):
            blocks.append((cyc[i], cyc[i + 1]))
        if len(cyc) % 2:
            blocks.append((cyc[-1],))
    return blocks


def iceberg_pairing_violations(d: int, blocks: Optional[Sequence[Tuple[int, ...]]] = None) -> Tuple[int, int]:
    """(checks holding both logical qubits of one block, repeated blocks within
    one CX time step of the outer schedule). The first must be 0 for the
    concatenation to keep the outer distance; the second only costs depth
    here (the lowering layers conflicting gates one after the other)."""
    blocks = iceberg_pairing(d) if blocks is None else blocks
    where = {q: k for k, b in enumerate(blocks) for q in b}
    plaqs = _rotated_layout(d)
    ft = 0
    for _, corners in plaqs:
        qs = [q for q in corners if q is not None]
        ft += len(qs) - len({where[q] for q in qs})
    sched = 0
    for s in range(4):
        used = []
        for typ, corners in plaqs:
            q = corners[(_ORDER_X if typ == "X" else _ORDER_Z)[s]]
            if q is not None:
                used.append(where[q])
        sched += len(used) - len(set(used))
    return ft, sched


def iceberg_branch_choices(d: int, seed: int, cycles: int, n_blocks: int, p_excite: float):
    """Seeded per (cycle, block) outcomes: variant (0 extra round, 1 flag) and fired."""
    u = splitmix64_uniform(seed, 2 * cycles * n_blocks)
    variant = [[int(u[2 * (t * n_blocks + k)] >= 0.5) for k in range(n_blocks)] for t in range(cycles)]
    fired = [[bool(u[2 * (t * n_blocks + k) + 1] < p_excite) for k in range(n_blocks)] for t in range(cycles)]
    return variant, fired


def iceberg_surface_branch(d: int, seed: int, cycles: Optional[int] = None, p: float = 1e-3,
                           p_excite: float = 0.25, gamma: Optional[int] = None) -> Circuit:
    """One realised branch of the adaptive [[4,2,2]] x rotated-surface-code
    memory experiment, outer distance d, `cycles` cycles (default d)."""
    cycles = d if cycles is None else cycles
    if cycles < 1:
        raise ValueError("at least one cycle")
    gamma = max(1, d // 2) if gamma is None else gamma
    blocks = iceberg_pairing(d)
    nb = len(blocks)
    where: Dict[int, Tuple[int, int]] = {q: (k, j) for k, b in enumerate(blocks) for j, q in enumerate(b)}
    plaqs = _rotated_layout(d)
    data = [4 * k + i for k in range(nb) for i in range(4)]
    az = [4 * nb + k for k in range(nb)]      # inner ZZZZ ancillas
    ax = [5 * nb + k for k in range(nb)]      # inner XXXX ancillas
    fz = [6 * nb + k for k in range(nb)]      # flags of the ZZZZ checks (read in X)
    fx = [7 * nb + k for k in range(nb)]      # flags of the XXXX checks (read in Z)
    oanc = [8 * nb + i for i in range(len(plaqs))]
    zbasis = az + fx + [oanc[i] for i, (t, _) in enumerate(plaqs) if t == "Z"]
    xbasis = ax + fz + [oanc[i] for i, (t, _) in enumerate(plaqs) if t == "X"]
    variant, fired = iceberg_branch_choices(d, seed, cycles, nb, p_excite)

    b = _Builder()
    b.gate("R", data + zbasis)
    b.gate("RX", xbasis)
    b.noise1("DEPOLARIZE1", p, data + zbasis + xbasis)
    b.tick()
    last: Dict[Tuple[str, int], int] = {}   # (check kind, index) -> its last measurement

    def cx_steps(steps: List[List[Tuple[int, int]]]) -> None:
        # a step whose pairs share a qubit (two checks on one block) is split,
        # in order, into instructions that touch each qubit once
        for pairs in steps:
            while pairs:
                used, now, rest = set(), [], []
                for pr in pairs:
                    if pr[0] in used or pr[1] in used:
                        rest.append(pr)
                    else:
                        now.append(pr)
                    used.update(pr)
                b.pairs("CX", now)
                b.noise2(p, now)
                b.tick()
                pairs = rest

    def measure(zq: List[int], xq: List[int]) -> Dict[int, int]:
        b.noise1("X_ERROR", p, zq)
        b.noise1("Z_ERROR", p, xq)
        out = dict(zip(zq, b.measure("MR", zq)))
        out.update(zip(xq, b.measure("MRX", xq)))
        b.noise1("DEPOLARIZE1", p, zq + xq)
        return out

    def close(kind: str, idx: int, m: int, z_type: bool) -> None:
        prev = last.get((kind, idx))
        if prev is not None:
            b.detector([m, prev])
        elif z_type:
            b.detector([m])
        last[(kind, idx)] = m

    for t in range(cycles):
        # inner layer: sub-round 0 for every block (flagged where chosen),
        # sub-round 1 for the blocks whose choice is an extra round
        for sub in (0, 1):
            members = [k for k in range(nb) if sub == 0 or variant[t][k] == 0]
            if not members:
                continue
            steps: List[List[Tuple[int, int]]] = [[] for _ in range(12)]
            flagged = []
            for k in members:
                q = [4 * k + i for i in range(4)]
                flag = sub == 0 and variant[t][k] == 1
                # ZZZZ: data -> az[k]; the flag fz[k] (|+>) is CX control onto az[k]
                zseq = [(q[0], az[k])] + ([(fz[k], az[k])] if flag else []) + [(q[1], az[k]), (q[2], az[k])] + \
                       ([(fz[k], az[k])] if flag else []) + [(q[3], az[k])]
                # XXXX: ax[k] -> data; ax[k] is CX control onto the flag fx[k] (|0>)
                xseq = [(ax[k], q[0])] + ([(ax[k], fx[k])] if flag else []) + [(ax[k], q[1]), (ax[k], q[2])] + \
                       ([(ax[k], fx[k])] if flag else []) + [(ax[k], q[3])]
                for i, pr in enumerate(zseq):
                    steps[i].append(pr)
                for i, pr in enumerate(xseq):
                    steps[6 + i].append(pr)
                if flag:
                    flagged.append(k)
            cx_steps(steps)
            ms = measure([az[k] for k in members] + [fx[k] for k in flagged],
                         [ax[k] for k in members] + [fz[k] for k in flagged])
            for k in members:
                close("iz", k, ms[az[k]], True)
                close("ix", k, ms[ax[k]], False)
            for k in flagged:
                b.detector([ms[fz[k]]])
                b.detector([ms[fx[k]]])
        # outer layer: the checks that run this cycle
        everything = t == 0 or t == cycles - 1 or t % gamma == 0
        run = []
        for i, (typ, corners) in enumerate(plaqs):
            qs = [q for q in corners if q is not None]
            if everything or any(fired[t][where[q][0]] for q in qs):
                run.append(i)
        if run:
            steps = []
            for s in range(4):
                for half in (0, 1):
                    pairs = []
                    for i in run:
                        typ, corners = plaqs[i]
                        q = corners[(_ORDER_X if typ == "X" else _ORDER_Z)[s]]
                        if q is None:
                            continue
                        k, j = where[q]
                        if typ == "X":
                            pairs.append((oanc[i], 4 * k + ICEBERG_X[j][half]))
                        else:
                            pairs.append((4 * k + ICEBERG_Z[j][half], oanc[i]))
                    steps.append(pairs)
            cx_steps(steps)
            ms = measure([oanc[i] for i in run if plaqs[i][0] == "Z"], [oanc[i] for i in run if plaqs[i][0] == "X"])
            for i in run:
                close("o", i, ms[oanc[i]], plaqs[i][0] == "Z")
        b.tick()

    # read out every data block in the Z basis; close the Z-type checks
    b.noise1("X_ERROR", p, data)
    md = dict(zip(data, b.measure("M", data)))
    for k in range(nb):
        b.detector([md[4 * k + i] for i in range(4)] + [last[("iz", k)]])

    def zbar(q: int) -> List[int]:
        k, j = where[q]
        return [md[4 * k + i] for i in ICEBERG_Z[j]]

    def odd(ms: List[int]) -> List[int]:
        cnt: Dict[int, int] = {}
        for m in ms:
            cnt[m] = cnt.get(m, 0) ^ 1
        return sorted(m for m, c in cnt.items() if c)

    for i, (typ, corners) in enumerate(plaqs):
        if typ != "Z":
            continue
        ms = [m for q in corners if q is not None for m in zbar(q)]
        b.detector(odd(ms) + [last[("o", i)]])
    b.observable(0, odd([m for c in range(d) for m in zbar(c)]))
    return b.build(cycles, f"iceberg_surface_d{d}_c{cycles}_s{seed}", n_qubits=8 * nb + len(plaqs))


def iceberg_surface_batch(d: int, n_branches: int = 256, seed: int = 0, cycles: Optional[int] = None,
                          p: float = 1e-3, p_excite: float = 0.25) -> List[Circuit]:
    """`n_branches` realised branches (seeds seed, seed + 1, ...)."""
    return [iceberg_surface_branch(d, seed + i, cycles=cycles, p=p, p_excite=p_excite) for i in range(n_branches)]
