"""Seeded synthetic circuit and state generators.

This module is shared by the CPU oracle and by the GPU engine as the common source of inputs. It holds
no state-vector arithmetic: it only draws random numbers and builds the FP64 gate matrices that both
sides receive verbatim (so no libm or device transcendental differences ever enter a comparison).

Conventions (mpiQulacs, Sec. II-A, Eqs. 2-4 and Sec. III-B):
  * qubit q is bit q of the amplitude index (qubit 0 is the least significant bit);
  * a k-qubit matrix acts on ``targets`` with ``targets[j]`` <-> bit j of its row/column index,
    row-major, psi' = U psi;
  * a diagonal gate is given by its 2^k diagonal entries in the same bit order;
  * a controlled gate applies U on its targets where every control bit is 1;
  * ``fswap`` is the fused-swap of Sec. III-D: swap(p+i, q+i) for i < s, ranges disjoint.

Gate definitions (the paper names RX/RZ/H but fixes no sign convention, Sec. IV-C/IV-F):
  RX(t) = exp(-i t X / 2), RZ(t) = diag(e^{-it/2}, e^{it/2}), H = [[1,1],[1,-1]]/sqrt(2),
  U3(t,p,l) = [[cos t/2, -e^{il} sin t/2], [e^{ip} sin t/2, e^{i(p+l)} cos t/2]].
Haar SU(4): QR of a complex Ginibre matrix with the phase of R's diagonal divided out
(Mezzadri 2007), then divided by det^{1/4}.

Workloads: the paper's Quantum Volume (Sec. IV-E) and QSB (Sec. IV-F) suites are not available, so the
random-circuit families below stand in for them with the same structure (random 1-qubit rotations,
CNOT/CZ layers, dense SU(4) on random qubit pairings).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

__all__ = [
    "Op", "Circuit", "u3", "rx", "rz", "h", "x_gate", "haar_su4", "dagger",
    "u3_cnot_layers", "mixed_layers", "su4_u3_random", "su4_u3_renorm", "su4_u3_error_run", "serving_batch",
    "hadamard_x11", "qsb", "quantum_volume", "ghz", "rx_sweep", "random_state", "random_circuit",
    "basis_state", "inverse_circuit",
]


@dataclass
class Op:
    """One circuit operation.

    kind: 'dense' | 'diag' | 'ctrl' | 'fswap'
    targets: target qubits (matrix bit j <-> targets[j]); for 'fswap' empty
    controls: control qubits for 'ctrl'
    mat: complex128 (2^k, 2^k) for 'dense'/'ctrl', (2^k,) for 'diag'
    p, q, s: fused-swap arguments
    label: gate name, for reporting only
    layer: 1-based layer the op belongs to (0 = none), for reporting and renormalisation cadence
    """
    kind: str
    targets: Tuple[int, ...] = ()
    controls: Tuple[int, ...] = ()
    mat: Optional[np.ndarray] = None
    p: int = 0
    q: int = 0
    s: int = 0
    label: str = ""
    layer: int = 0

    def qubits(self) -> Tuple[int, ...]:
        if self.kind == "fswap":
            return tuple(range(self.p, self.p + self.s)) + tuple(range(self.q, self.q + self.s))
        return tuple(self.controls) + tuple(self.targets)


@dataclass
class Circuit:
    n: int
    ops: List[Op] = field(default_factory=list)
    name: str = ""
    seed: Optional[int] = None
    # 1-based layer indices after which a complex64 state is renormalised (empty: never)
    renorm_after: Tuple[int, ...] = ()

    def __len__(self) -> int:
        return len(self.ops)

    def count(self, kinds: Sequence[str] = ("dense", "diag", "ctrl", "fswap")) -> int:
        return sum(1 for o in self.ops if o.kind in kinds)


# ----------------------------------------------------------------------------------------------------------
# gate matrices (inputs; complex128)
# ----------------------------------------------------------------------------------------------------------

def u3(theta: float, phi: float, lam: float) -> np.ndarray:
    c, s = math.cos(theta / 2.0), math.sin(theta / 2.0)
    return np.array([[c, -np.exp(1j * lam) * s],
                     [np.exp(1j * phi) * s, np.exp(1j * (phi + lam)) * c]], dtype=np.complex128)


def rx(theta: float) -> np.ndarray:
    c, s = math.cos(theta / 2.0), math.sin(theta / 2.0)
    return np.array([[c, -1j * s], [-1j * s, c]], dtype=np.complex128)


def rz(theta: float) -> np.ndarray:
    """Diagonal entries of RZ(theta)."""
    return np.array([np.exp(-0.5j * theta), np.exp(0.5j * theta)], dtype=np.complex128)


def h() -> np.ndarray:
    r = 1.0 / math.sqrt(2.0)
    return np.array([[r, r], [r, -r]], dtype=np.complex128)


def x_gate() -> np.ndarray:
    return np.array([[0, 1], [1, 0]], dtype=np.complex128)


def haar_su4(rng: np.random.Generator) -> np.ndarray:
    z = (rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4))) / math.sqrt(2.0)
    qm, r = np.linalg.qr(z)
    d = np.diag(r)
    qm = qm * (d / np.abs(d))
    det = np.linalg.det(qm)
    return (qm / det ** 0.25).astype(np.complex128)


def dagger(op: Op) -> Op:
    """The inverse of a unitary op (its conjugate transpose; fused-swaps are involutions)."""
    if op.kind == "fswap":
        return Op("fswap", p=op.p, q=op.q, s=op.s, label=op.label + "^-1", layer=op.layer)
    if op.kind == "diag":
        return Op("diag", op.targets, mat=np.conj(op.mat), label=op.label + "^-1", layer=op.layer)
    return Op(op.kind, op.targets, op.controls, mat=np.ascontiguousarray(np.conj(op.mat).T),
              label=op.label + "^-1", layer=op.layer)


def inverse_circuit(c: Circuit) -> Circuit:
    return Circuit(c.n, [dagger(o) for o in reversed(c.ops)], name=c.name + "^-1", seed=c.seed)


# ----------------------------------------------------------------------------------------------------------
# small builders
# ----------------------------------------------------------------------------------------------------------

def _dense(t, m, label, layer=0):
    return Op("dense", tuple(int(x) for x in t), mat=np.asarray(m, dtype=np.complex128), label=label, layer=layer)


def _diag(t, d, label, layer=0):
    return Op("diag", tuple(int(x) for x in t), mat=np.asarray(d, dtype=np.complex128), label=label, layer=layer)


def _ctrl(c, t, m, label, layer=0):
    return Op("ctrl", tuple(int(x) for x in t), tuple(int(x) for x in c), mat=np.asarray(m, dtype=np.complex128),
              label=label, layer=layer)


def _fswap(p, q, s, layer=0):
    return Op("fswap", p=int(p), q=int(q), s=int(s), label="FSWAP", layer=layer)


CZ_DIAG = np.array([1, 1, 1, -1], dtype=np.complex128)


def _u3_layer(rng, n, layer):
    ops = []
    for qb in range(n):  # angles drawn per qubit in ascending order
        th, ph, la = rng.uniform(0.0, 2.0 * math.pi, size=3)
        ops.append(_dense((qb,), u3(th, ph, la), "U3", layer))
    return ops


# ----------------------------------------------------------------------------------------------------------
# workload families
# ----------------------------------------------------------------------------------------------------------

def u3_cnot_layers(n: int = 16, seed: int = 16, layers: int = 10) -> Circuit:
    """Plain method, 16 qubits: per layer random U3 on every qubit, then CNOT on even neighbour pairs
    (0,1),(2,3).. on even layers and odd pairs (1,2),(3,4).. on odd layers (control = lower qubit);
    finally fused_swap(0, n-4, 4), i.e. qubits {12..15} <-> {0..3} at n=16."""
    rng = np.random.Generator(np.random.PCG64(seed))
    c = Circuit(n, name=f"u3_cnot_n{n}", seed=seed)
    for L in range(layers):
        c.ops += _u3_layer(rng, n, L + 1)
        start = 0 if L % 2 == 0 else 1
        for a in range(start, n - 1, 2):
            c.ops.append(_ctrl((a,), (a + 1,), x_gate(), "CNOT", L + 1))
    c.ops.append(_fswap(0, n - 4, 4, layers))
    return c


def mixed_layers(n: int = 28, seed: int = 28, layers: int = 20, toffolis: int = 32, swap_s: int = 6) -> Circuit:
    """Plain method, 28 qubits, unfused: per layer U3 on all, CZ on alternating neighbour pairs, RZ on all.
    Toffolis on ``toffolis`` random distinct triples (c1, c2, t), a quarter after layers 5/10/15/20;
    fused_swap(0, n-s, s) after layers 7/14/20."""
    rng = np.random.Generator(np.random.PCG64(seed))
    c = Circuit(n, name=f"mixed_n{n}", seed=seed)
    triples = []
    seen = set()
    while len(triples) < toffolis:
        tr = tuple(int(v) for v in rng.choice(n, size=3, replace=False))
        if tr not in seen:
            seen.add(tr)
            triples.append(tr)
    tof_after = {5: triples[0:8], 10: triples[8:16], 15: triples[16:24], 20: triples[24:32]}
    for L in range(1, layers + 1):
        c.ops += _u3_layer(rng, n, L)
        start = 0 if L % 2 == 1 else 1
        for a in range(start, n - 1, 2):
            c.ops.append(_diag((a, a + 1), CZ_DIAG, "CZ", L))
        for qb in range(n):
            c.ops.append(_diag((qb,), rz(rng.uniform(0.0, 2.0 * math.pi)), "RZ", L))
        for (c1, c2, t) in tof_after.get(L, []):
            c.ops.append(_ctrl((c1, c2), (t,), x_gate(), "TOFFOLI", L))
        if L in (7, 14, 20):
            c.ops.append(_fswap(0, n - swap_s, swap_s, L))
    return c


def _su4_u3_layers(n: int, seed: int, layers: int, name: str) -> Circuit:
    rng = np.random.Generator(np.random.PCG64(seed))
    c = Circuit(n, name=name, seed=seed)
    for L in range(1, layers + 1):
        perm = rng.permutation(n)
        for j in range(n // 2):
            c.ops.append(_dense((perm[2 * j], perm[2 * j + 1]), haar_su4(rng), "SU4", L))
        c.ops += _u3_layer(rng, n, L)
    return c


def su4_u3_random(n: int = 32, seed: int = 32, layers: int = 40) -> Circuit:
    """32-qubit random circuit: per layer a random qubit pairing (pi = permutation, pairs (pi[2j], pi[2j+1]))
    with a Haar SU(4) on each pair, then U3 on every qubit."""
    return _su4_u3_layers(n, seed, layers, f"su4_u3_n{n}")


def su4_u3_renorm(n: int = 33, seed: int = 33, layers: int = 40) -> Circuit:
    """Same family as su4_u3_random at 33 qubits (one qubit unpaired per layer); a complex64 state is
    renormalised after layers 10/20/30/40."""
    c = _su4_u3_layers(n, seed, layers, f"su4_u3_renorm_n{n}")
    c.renorm_after = tuple(L for L in range(10, layers + 1, 10))
    return c


def su4_u3_error_run(n: int = 24, seed: int = 24, layers: int = 40) -> Circuit:
    return su4_u3_renorm(n=n, seed=seed, layers=layers)


def _batch_circuit(rng: np.random.Generator, n: int, depth: int, idx: int) -> Circuit:
    c = Circuit(n, name=f"batch{idx}_n{n}_d{depth}")
    for L in range(1, depth + 1):
        c.ops += _u3_layer(rng, n, L)
        use_cnot = bool(rng.integers(0, 2))
        start = 0 if L % 2 == 1 else 1
        for a in range(start, n - 1, 2):
            if use_cnot:
                c.ops.append(_ctrl((a,), (a + 1,), x_gate(), "CNOT", L))
            else:
                c.ops.append(_diag((a, a + 1), CZ_DIAG, "CZ", L))
        for qb in range(n):
            c.ops.append(_diag((qb,), rz(rng.uniform(0.0, 2.0 * math.pi)), "RZ", L))
    return c


def serving_batch(count: int = 512, seed: int = 512, nmin: int = 10, nmax: int = 22, dmin: int = 10,
            dmax: int = 40) -> List[Circuit]:
    """Batched serving form: ``count`` independent circuits, n ~ U{nmin..nmax}, depth ~ U{dmin..dmax};
    per layer U3 on all, CNOT or CZ (coin flip per layer) on alternating pairs, RZ on all.
    Circuit j draws from SeedSequence(seed).spawn(count)[j]."""
    out = []
    for j, ss in enumerate(np.random.SeedSequence(seed).spawn(count)):
        rng = np.random.Generator(np.random.PCG64(ss))
        n = int(rng.integers(nmin, nmax + 1))
        d = int(rng.integers(dmin, dmax + 1))
        c = _batch_circuit(rng, n, d, j)
        c.seed = seed
        out.append(c)
    return out


def hadamard_x11(n: int, reps: int = 11) -> Circuit:
    """The Hadamard benchmark of Sec. IV-D: eleven H gates on each qubit."""
    c = Circuit(n, name=f"hadamard_x{reps}_n{n}")
    for r in range(reps):
        for qb in range(n):
            c.ops.append(_dense((qb,), h(), "H", r + 1))
    return c


def qsb(n: int, seed: int = 0, sets: int = 10) -> Circuit:
    """A QSB-structured circuit (Sec. IV-F): ``sets`` x (rotation layer RZ.RX.RZ on each qubit + CNOT layer
    with target i and control (i+1) mod n) + one more rotation layer. Angles are random."""
    rng = np.random.Generator(np.random.PCG64(seed))
    c = Circuit(n, name=f"qsb_n{n}", seed=seed)

    def rot(L):
        for qb in range(n):
            a, b, cc = rng.uniform(0.0, 2.0 * math.pi, size=3)
            c.ops.append(_diag((qb,), rz(a), "RZ", L))
            c.ops.append(_dense((qb,), rx(b), "RX", L))
            c.ops.append(_diag((qb,), rz(cc), "RZ", L))

    for L in range(1, sets + 1):
        rot(L)
        for i in range(n):
            c.ops.append(_ctrl(((i + 1) % n,), (i,), x_gate(), "CNOT", L))
    rot(sets + 1)
    return c


def ghz(n: int) -> Circuit:
    c = Circuit(n, name=f"ghz_n{n}")
    c.ops.append(_dense((0,), h(), "H"))
    for qb in range(n - 1):
        c.ops.append(_ctrl((qb,), (qb + 1,), x_gate(), "CNOT"))
    return c


def quantum_volume(n: int, seed: int = 0, depth: int = 10) -> Circuit:
    """Quantum Volume model circuit (Sec. IV-E): ``depth`` layers, each a random permutation of the qubit labels
    followed by a Haar SU(4) on every consecutive pair of the permuted labels (an odd n leaves one qubit idle).
    The reference generator the paper used is not available; this follows its prose."""
    rng = np.random.Generator(np.random.PCG64(seed))
    c = Circuit(n, name=f"qv_n{n}_d{depth}", seed=seed)
    for L in range(1, depth + 1):
        perm = rng.permutation(n)
        for j in range(n // 2):
            c.ops.append(_dense((perm[2 * j], perm[2 * j + 1]), haar_su4(rng), "SU4", L))
    return c


def rx_sweep(n: int, seed: int = 0) -> Circuit:
    """One random RX gate on each target qubit q = 0..n-1 in turn (the per-target gate-time sweep of
    Sec. IV-C)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    c = Circuit(n, name=f"rx_sweep_n{n}", seed=seed)
    for qb in range(n):
        c.ops.append(_dense((qb,), rx(rng.uniform(0.0, 2.0 * math.pi)), "RX", qb + 1))
    return c


def random_state(n: int, seed: int) -> np.ndarray:
    """A normalised complex128 state with i.i.d. Gaussian components."""
    rng = np.random.Generator(np.random.PCG64(seed))
    v = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    return (v / np.linalg.norm(v)).astype(np.complex128)


def basis_state(n: int, x: int) -> np.ndarray:
    v = np.zeros(1 << n, dtype=np.complex128)
    v[x] = 1.0
    return v


def _random_unitary(rng: np.random.Generator, dim: int) -> np.ndarray:
    z = (rng.standard_normal((dim, dim)) + 1j * rng.standard_normal((dim, dim))) / math.sqrt(2.0)
    qm, r = np.linalg.qr(z)
    d = np.diag(r)
    return (qm * (d / np.abs(d))).astype(np.complex128)


def random_circuit(n: int, seed: int, num_ops: int = 40, kmax: int = 3, kinds=("dense", "diag", "ctrl", "fswap"),
                   perm_frac: float = 0.2) -> Circuit:
    """A mixed random circuit over every op kind (for parity tests): dense k<=kmax with Haar-ish unitaries,
    diagonals with unit-modulus entries (some exactly +1/-1), controlled gates (some permutation
    targets), and fused-swaps with random non-overlapping ranges."""
    rng = np.random.Generator(np.random.PCG64(seed))
    c = Circuit(n, name=f"random_n{n}_s{seed}", seed=seed)
    for _ in range(num_ops):
        kind = kinds[int(rng.integers(0, len(kinds)))]
        if kind == "dense":
            k = int(rng.integers(1, min(kmax, n) + 1))
            t = tuple(int(v) for v in rng.choice(n, size=k, replace=False))
            if rng.random() < perm_frac:
                P = np.eye(1 << k, dtype=np.complex128)[rng.permutation(1 << k)]
                P = P * rng.choice([1, -1, 1j, -1j], size=(1 << k))[None, :]
                c.ops.append(_dense(t, P, "PERM"))
            else:
                c.ops.append(_dense(t, _random_unitary(rng, 1 << k), f"U{k}"))
        elif kind == "diag":
            k = int(rng.integers(1, min(kmax, n) + 1))
            t = tuple(int(v) for v in rng.choice(n, size=k, replace=False))
            d = np.exp(1j * rng.uniform(0, 2 * math.pi, size=1 << k))
            sel = rng.random(1 << k)
            d[sel < 0.2] = 1.0
            d[(sel >= 0.2) & (sel < 0.3)] = -1.0
            c.ops.append(_diag(t, d, f"D{k}"))
        elif kind == "ctrl":
            if n < 2:
                continue
            k = int(rng.integers(1, min(kmax, n - 1) + 1))
            cn = int(rng.integers(1, min(3, n - k) + 1))
            qs = [int(v) for v in rng.choice(n, size=k + cn, replace=False)]
            t, cc = tuple(qs[:k]), tuple(qs[k:])
            if rng.random() < 0.4:
                P = np.eye(1 << k, dtype=np.complex128)[rng.permutation(1 << k)]
                c.ops.append(_ctrl(cc, t, P, "CPERM"))
            else:
                c.ops.append(_ctrl(cc, t, _random_unitary(rng, 1 << k), f"CU{k}"))
        else:
            if n < 2:
                continue
            s = int(rng.integers(1, n // 2 + 1))
            p = int(rng.integers(0, n - 2 * s + 1))
            q = int(rng.integers(p + s, n - s + 1))
            if rng.random() < 0.5:
                p, q = q, p
            c.ops.append(_fswap(p, q, s))
    return c
