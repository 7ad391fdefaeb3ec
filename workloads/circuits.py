"""Seeded synthetic workloads for state-vector gate application.

This module only draws random numbers and lays out gate lists; it holds none of
the simulation arithmetic (no gate matrices except the Haar-random two-qubit
unitaries, which are themselves random *inputs*).  Both the FP64 reference
(``oracle/``) and the HIP library consume these gate lists, each through its own
gate table.

Conventions
-----------
* Qubit ``q`` is bit ``q`` of the amplitude index (little-endian).
* A gate is ``Gate(name, targets, controls, params, matrix)``.  ``name`` is one of
  ``h x y z s t rx ry rz p u3 matrix``.  Controls act on |1>.  ``matrix`` (only for
  ``name == "matrix"``) is a 2^k x 2^k complex array whose row/column index has
  ``targets[0]`` as its least significant bit.
* A ``BitSwap(lo, hi, width)`` entry is a physical relayout (the single-GPU
  stand-in for the global/local qubit exchange of distributed simulators, paper
  Sec. 2.1 "State-Vector Simulation" and Sec. 2.5); it leaves the logical state
  unchanged.

Workload shapes follow the paper's benchmark descriptions (Sec. 2.2) and the
layered random circuits the hot-path study is quoted on.  Where the paper is
silent (qubit pairing, angle law) the reading is: angles iid U[0, 2*pi), a
pairing is a uniformly random perfect matching of a shuffled qubit list whose
first element is the control.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple, Union

import numpy as np

TWO_PI = 2.0 * math.pi

GATE_NAMES = ("h", "x", "y", "z", "s", "t", "rx", "ry", "rz", "p", "u3", "matrix")
N_PARAMS = {"h": 0, "x": 0, "y": 0, "z": 0, "s": 0, "t": 0,
            "rx": 1, "ry": 1, "rz": 1, "p": 1, "u3": 3, "matrix": 0}


@dataclass(frozen=True)
class Gate:
    name: str
    targets: Tuple[int, ...]
    controls: Tuple[int, ...] = ()
    params: Tuple[float, ...] = ()
    matrix: Optional[np.ndarray] = field(default=None, compare=False)

    @property
    def qubits(self) -> Tuple[int, ...]:
        return tuple(self.targets) + tuple(self.controls)


@dataclass(frozen=True)
class BitSwap:
    lo: int
    hi: int
    width: int


Op = Union[Gate, BitSwap]


def cx(c: int, t: int) -> Gate:
    return Gate("x", (t,), (c,))


def cz(c: int, t: int) -> Gate:
    return Gate("z", (t,), (c,))


def cp(c: int, t: int, phi: float) -> Gate:
    return Gate("p", (t,), (c,), (float(phi),))


def circuit_seed(config: int, run: int) -> int:
    """Seed of run ``run`` (0 = warm-up) of workload ``config`` (1..5)."""
    return 1000 * config + run


def _angles(rng: np.random.Generator, k: int) -> Tuple[float, ...]:
    return tuple(float(x) for x in rng.uniform(0.0, TWO_PI, size=k))


def random_pairing(rng: np.random.Generator, n: int) -> List[Tuple[int, int]]:
    """Uniform random perfect matching of a shuffled qubit list (floor(n/2) pairs)."""
    perm = rng.permutation(n)
    return [(int(perm[2 * i]), int(perm[2 * i + 1])) for i in range(n // 2)]


def random_nonadjacent_pairing(rng: np.random.Generator, n: int,
                               max_tries: int = 10000) -> List[Tuple[int, int]]:
    """Random matching whose pairs all satisfy |a - b| >= 2 (rejection sampling)."""
    for _ in range(max_tries):
        pairs = random_pairing(rng, n)
        if all(abs(a - b) >= 2 for a, b in pairs):
            return pairs
    raise RuntimeError("no non-adjacent pairing found")


def layered_u3_pairing(n: int, layers: int, seed: int,
                       entangler: str = "cx") -> List[Gate]:
    """U3 on every qubit, then a two-qubit gate on each pair of a random matching.

    ``entangler`` is ``"cx"`` (every pair a CNOT) or ``"cx_or_cz"`` (a fair coin
    per pair).  n=12, 20 layers, ``"cx"`` is the 12-qubit complex128 workload;
    n=28, 20 layers, ``"cx_or_cz"`` the 28-qubit one.
    """
    rng = np.random.default_rng(seed)
    gates: List[Gate] = []
    for _ in range(layers):
        for q in range(n):
            gates.append(Gate("u3", (q,), (), _angles(rng, 3)))
        for a, b in random_pairing(rng, n):
            if entangler == "cx" or rng.integers(0, 2) == 0:
                gates.append(cx(a, b))
            else:
                gates.append(cz(a, b))
    return gates


def qft_ladder_block(n: int, width: int = 8) -> List[Gate]:
    """H + controlled-phase(pi/2^d) ladder on the ``width`` highest qubits.

    Textbook QFT order on qubits n-1 .. n-width: for j = 0..width-1, H on
    n-1-j, then CP(pi/2^d) with control n-1-j-d and target n-1-j for
    d = 1..width-1-j (8 H + 28 CP for width 8).
    """
    gates: List[Gate] = []
    for j in range(width):
        t = n - 1 - j
        gates.append(Gate("h", (t,)))
        for d in range(1, width - j):
            gates.append(cp(t - d, t, math.pi / (1 << d)))
    return gates


def share_layers(n: int, layers: int, seed: int, swap_every: int = 2,
                 swap_width: int = 6) -> List[Op]:
    """One GPU's share at full size (34q complex128 / 35q complex64 workload).

    Each layer: the QFT ladder on the 8 highest qubits, U3 on every qubit, CNOT
    on a random matching.  After every ``swap_every`` layers the top
    ``swap_width`` index bits are exchanged with the lowest ones.
    """
    rng = np.random.default_rng(seed)
    ops: List[Op] = []
    for layer in range(1, layers + 1):
        ops.extend(qft_ladder_block(n, 8))
        for q in range(n):
            ops.append(Gate("u3", (q,), (), _angles(rng, 3)))
        for a, b in random_pairing(rng, n):
            ops.append(cx(a, b))
        if swap_every and layer % swap_every == 0:
            ops.append(BitSwap(0, n - swap_width, swap_width))
    return ops


def haar_unitary(rng: np.random.Generator, d: int) -> np.ndarray:
    """Haar-random d x d unitary: QR of a complex Ginibre matrix with the phases of
    R's diagonal moved into Q (Mezzadri, Notices AMS 54, 2007)."""
    z = (rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))) / math.sqrt(2.0)
    q, r = np.linalg.qr(z)
    ph = np.diag(r) / np.abs(np.diag(r))
    return q * ph[np.newaxis, :]


def haar_su(rng: np.random.Generator, d: int) -> np.ndarray:
    u = haar_unitary(rng, d)
    det = np.linalg.det(u)
    return u / det ** (1.0 / d)


def u3_su4_layers(n: int, layers: int, seed: int) -> List[Gate]:
    """U3 on every qubit + Haar SU(4) on a random non-adjacent matching (30q, depth 40)."""
    rng = np.random.default_rng(seed)
    gates: List[Gate] = []
    for _ in range(layers):
        for q in range(n):
            gates.append(Gate("u3", (q,), (), _angles(rng, 3)))
        for a, b in random_nonadjacent_pairing(rng, n):
            gates.append(Gate("matrix", (a, b), (), (), haar_su(rng, 4)))
    return gates


def hea_circuit(q: int, depth: int, thetas: np.ndarray, phis: np.ndarray) -> List[Gate]:
    """Hardware-efficient ansatz: per layer RY(theta) RZ(phi) on every qubit, then
    the linear CNOT ladder i -> i+1.  ``thetas``/``phis`` have shape (depth, q)."""
    gates: List[Gate] = []
    for l in range(depth):
        for i in range(q):
            gates.append(Gate("ry", (i,), (), (float(thetas[l, i]),)))
            gates.append(Gate("rz", (i,), (), (float(phis[l, i]),)))
        for i in range(q - 1):
            gates.append(cx(i, i + 1))
    return gates


@dataclass
class HeaBatch:
    """A batch of HEA instances of uneven width (parameter-sweep workload)."""
    qubits: np.ndarray          # (B,) int
    depth: int
    thetas: List[np.ndarray]    # per instance (depth, q)
    phis: List[np.ndarray]

    def circuit(self, i: int) -> List[Gate]:
        return hea_circuit(int(self.qubits[i]), self.depth, self.thetas[i], self.phis[i])

    def num_gates(self) -> int:
        return sum(self.depth * (2 * int(q) + int(q) - 1) for q in self.qubits)


def hea_batch(batch: int, qmin: int, qmax: int, depth: int, seed: int) -> HeaBatch:
    rng = np.random.default_rng(seed)
    qs = rng.integers(qmin, qmax + 1, size=batch)
    thetas, phis = [], []
    for q in qs:
        thetas.append(rng.uniform(0.0, TWO_PI, size=(depth, int(q))))
        phis.append(rng.uniform(0.0, TWO_PI, size=(depth, int(q))))
    return HeaBatch(qs.astype(np.int64), depth, thetas, phis)


def rcs_circuit(n: int, seed: int) -> List[Gate]:
    """Random circuit sampling workload of paper Sec. 2.2 "Random Circuits":
    30n gates on random qubits; with probability 0.25 a CZ on two distinct
    qubits, otherwise one of H, RX, RY, RZ (equiprobable) with angle U[0, 2*pi)."""
    rng = np.random.default_rng(seed)
    gates: List[Gate] = []
    for _ in range(30 * n):
        if rng.random() < 0.25:
            a, b = (int(x) for x in rng.choice(n, size=2, replace=False))
            gates.append(cz(a, b))
        else:
            kind = ("h", "rx", "ry", "rz")[int(rng.integers(0, 4))]
            q = int(rng.integers(0, n))
            if kind == "h":
                gates.append(Gate("h", (q,)))
            else:
                gates.append(Gate(kind, (q,), (), (float(rng.uniform(0.0, TWO_PI)),)))
    return gates


def qpe_circuit(k: int, m: int) -> List[Gate]:
    """Textbook phase estimation of U = P(2*pi*phi), phi = m / 2^k, on eigenstate |1>.

    Counting qubits 0..k-1, eigen-qubit k.  Counting qubit j controls
    U^(2^(k-1-j)) = P(2*pi*phi*2^(k-1-j)); the adjoint of the H + controlled-phase
    ladder on the counting register then leaves m, counting qubit j holding bit j
    (paper Sec. 2.2 QPE: phases exactly representable with k bits).
    """
    phi = m / float(1 << k)
    gates: List[Gate] = [Gate("x", (k,))]
    for j in range(k):
        gates.append(Gate("h", (j,)))
    for j in range(k):
        gates.append(cp(j, k, TWO_PI * phi * (1 << (k - 1 - j))))
    # adjoint of qft_ladder_block on the k counting qubits (top qubit k-1)
    for j in range(k - 1, -1, -1):
        t = k - 1 - j
        for d in range(k - 1 - j, 0, -1):
            gates.append(cp(t - d, t, -math.pi / (1 << d)))
        gates.append(Gate("h", (t,)))
    return gates


def triangular_lattice_edges(rows: int, cols: int) -> List[Tuple[int, int]]:
    """Nearest-neighbour pairs of a triangular lattice of rows x cols sites with
    periodic boundaries in both directions (site (r, c) is qubit r * cols + c):
    each site bonds to its right, lower and lower-right neighbours, 3 rows*cols
    distinct bonds for rows, cols >= 3 (every site has six neighbours).  Stands
    in for the HamLib TFIM lattice of paper Sec. 2.2, whose data is not
    available here."""
    if rows < 3 or cols < 3:
        raise ValueError("need rows, cols >= 3 for distinct periodic bonds")
    edges = []
    for r in range(rows):
        for c in range(cols):
            q = r * cols + c
            for dr, dc in ((0, 1), (1, 0), (1, 1)):
                edges.append((q, ((r + dr) % rows) * cols + (c + dc) % cols))
    return edges


def tfim_trotter(rows: int, cols: int, steps: int, dt: float, J: float = 1.0, h: float = 1.0,
                 zz: str = "cx") -> List[Gate]:
    """First-order Suzuki-Trotter circuit for the transverse-field Ising model
    H = -J sum_<i,j> Z_i Z_j - h sum_i X_i (paper Eq. of the TFIM, Sec. 2.2) on
    the periodic triangular lattice: per step exp(i J dt Z_a Z_b) on every bond,
    then exp(i h dt X_q) = RX(-2 h dt) on every site.  The bond factor is
    exp(-i theta/2 Z_a Z_b) with theta = -2 J dt, given as CX(a, b) RZ_b(theta)
    CX(a, b) (zz="cx", the gate-level form of circuit benchmarks) or as its
    diagonal 4 x 4 matrix (zz="diag", an input matrix like the Haar unitaries)."""
    edges = triangular_lattice_edges(rows, cols)
    theta, phi = -2.0 * J * dt, -2.0 * h * dt
    gates: List[Gate] = []
    for _ in range(steps):
        for a, b in edges:
            if zz == "cx":
                gates += [cx(a, b), Gate("rz", (b,), (), (theta,)), cx(a, b)]
            elif zz == "diag":
                gates.append(Gate("matrix", (a, b), (), (),
                                  np.diag(np.exp(-0.5j * theta * np.array([1.0, -1.0, -1.0, 1.0])))))
            else:
                raise ValueError(zz)
        for q in range(rows * cols):
            gates.append(Gate("rx", (q,), (), (phi,)))
    return gates


def uniforms(seed: int, shots: int) -> np.ndarray:
    """Sampling uniforms in [0, 1) (the random numbers the sampler consumes)."""
    return np.random.default_rng(seed).random(shots)


def random_state(n: int, seed: int) -> np.ndarray:
    """Normalised complex Gaussian state (complex128) for readout tests."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    return v / np.linalg.norm(v)


def gate_count(ops: Sequence[Op]) -> int:
    return sum(1 for g in ops if isinstance(g, Gate))


def inverse(ops: Sequence[Op]) -> List[Op]:
    """Gate list of the adjoint circuit (mirror half).  Bit swaps are their own inverse."""
    out: List[Op] = []
    for g in reversed(list(ops)):
        if isinstance(g, BitSwap):
            out.append(g)
            continue
        nm, p = g.name, g.params
        if nm in ("h", "x", "y", "z"):
            out.append(g)
        elif nm == "s":
            out.append(Gate("p", g.targets, g.controls, (-math.pi / 2,)))
        elif nm == "t":
            out.append(Gate("p", g.targets, g.controls, (-math.pi / 4,)))
        elif nm in ("rx", "ry", "rz", "p"):
            out.append(Gate(nm, g.targets, g.controls, (-p[0],)))
        elif nm == "u3":
            # U3(t, f, l)^dagger = U3(-t, -l, -f)
            out.append(Gate("u3", g.targets, g.controls, (-p[0], -p[2], -p[1])))
        elif nm == "matrix":
            out.append(Gate("matrix", g.targets, g.controls, (), np.conj(g.matrix.T)))
        else:
            raise ValueError(nm)
    return out


def hea_z_terms(q: int) -> List[str]:
    """Pauli strings (qubit 0 first) for <Z_i> (i < q) and <Z_i Z_{i+1}> (i < q-1)."""
    terms = []
    for i in range(q):
        s = ["I"] * q
        s[i] = "Z"
        terms.append("".join(s))
    for i in range(q - 1):
        s = ["I"] * q
        s[i] = "Z"
        s[i + 1] = "Z"
        terms.append("".join(s))
    return terms
