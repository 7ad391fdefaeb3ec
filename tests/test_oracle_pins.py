"""Pins of the FP64 reference against facts fixed outside it.

Each check uses something other than the reference's own formula: numpy tensor
contraction / Kronecker products, scipy's matrix exponential, numpy's FFT,
closed forms, invariants and tiny brute force.  A plausible slip in the
reference (a dropped term, a wrong sign or index, a transposed operand) fails
at least one of them.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest
import scipy.linalg

import oracle
import workloads as W
from workloads import Gate

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
PX = np.array([[0, 1], [1, 0]], dtype=np.complex128)
PY = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
PZ = np.array([[1, 0], [0, -1]], dtype=np.complex128)
I2 = np.eye(2, dtype=np.complex128)


def tensor_apply(state, U, targets, controls=()):
    """Independent brute force: the controlled operator on (targets + controls) as
    a dense tensor, contracted with the state reshaped to a rank-n tensor."""
    n = state.size.bit_length() - 1
    qs = list(targets) + list(controls)
    k, m = len(targets), len(qs)
    d = 1 << m
    full = np.eye(d, dtype=np.complex128)
    full[d - (1 << k):, d - (1 << k):] = U  # all control bits (the high bits) = 1
    T = full.reshape([2] * (2 * m))
    psi = state.reshape([2] * n)  # axis a <-> qubit n-1-a
    in_axes = [m + (m - 1 - b) for b in range(m)]
    psi_axes = [n - 1 - qs[b] for b in range(m)]
    out = np.tensordot(T, psi, axes=(in_axes, psi_axes))
    dest = [n - 1 - qs[m - 1 - j] for j in range(m)]
    out = np.moveaxis(out, list(range(m)), dest)
    return np.ascontiguousarray(out.reshape(-1))


def kron_chain(ops_msb_first):
    out = np.array([[1.0 + 0j]])
    for o in ops_msb_first:
        out = np.kron(out, o)
    return out


ONE_Q = [("h", ()), ("x", ()), ("y", ()), ("z", ()), ("s", ()), ("t", ()),
         ("rx", (0.7,)), ("ry", (1.9,)), ("rz", (-2.3,)), ("p", (0.4,)), ("u3", (0.3, 1.1, -0.8))]


@pytest.mark.parametrize("name,params", ONE_Q)
def test_apply_all_placements_vs_tensor_contraction(name, params):
    n = 5
    U = oracle.gates.matrix(name, params)
    psi0 = W.random_state(n, 11)
    for t in range(n):
        others = [q for q in range(n) if q != t]
        ctrl_sets = [()] + [(c,) for c in others] + list(itertools.permutations(others, 2))[:6]
        for ctrls in ctrl_sets:
            got = oracle.apply_matrix(psi0.copy(), U, [t], ctrls)
            want = tensor_apply(psi0, U, [t], ctrls)
            assert np.max(np.abs(got - want)) < 1e-14, (name, t, ctrls)


@pytest.mark.parametrize("k", [2, 3, 4])
def test_apply_multi_target_vs_tensor_contraction(k):
    n = 7
    rng = np.random.default_rng(k)
    psi0 = W.random_state(n, 5 + k)
    for trial in range(12):
        qs = [int(x) for x in rng.permutation(n)]
        targets = qs[:k]
        c = int(rng.integers(0, min(2, n - k) + 1))
        controls = qs[k:k + c]
        U = W.haar_unitary(rng, 1 << k)
        got = oracle.apply_matrix(psi0.copy(), U, targets, controls)
        want = tensor_apply(psi0, U, targets, controls)
        assert np.max(np.abs(got - want)) < 1e-13, (targets, controls)


def test_one_qubit_gate_vs_kron_full_unitary():
    """Full 2^n x 2^n matrix product: qubit 0 is the rightmost Kronecker factor."""
    n = 6
    psi0 = W.random_state(n, 3)
    U = oracle.gates.matrix("u3", (0.9, -0.4, 2.2))
    for t in range(n):
        full = kron_chain([U if q == t else I2 for q in reversed(range(n))])
        got = oracle.apply_matrix(psi0.copy(), U, [t])
        assert np.max(np.abs(got - full @ psi0)) < 1e-14


def test_cnot_full_unitary():
    n = 3
    psi0 = W.random_state(n, 9)
    # CNOT control 2, target 0 as |0><0| (x) I (x) I + |1><1| (x) I (x) X
    P0 = np.diag([1, 0]).astype(np.complex128)
    P1 = np.diag([0, 1]).astype(np.complex128)
    full = kron_chain([P0, I2, I2]) + kron_chain([P1, I2, PX])
    got = oracle.apply_gate(psi0.copy(), W.cx(2, 0))
    assert np.max(np.abs(got - full @ psi0)) < 1e-15


def test_apply_rejects_bad_arguments():
    psi = oracle.zero_state(4)
    with pytest.raises(ValueError):
        oracle.apply_matrix(psi, oracle.gates.matrix("h"), [4])
    with pytest.raises(ValueError):
        oracle.apply_matrix(psi, oracle.gates.matrix("x"), [1], [1])
    with pytest.raises(ValueError):
        oracle.apply_matrix(psi, np.eye(4), [0, 0])


def test_gate_table_identities():
    g = oracle.gates.matrix
    pi = math.pi
    assert np.allclose(g("u3", (pi / 2, 0, pi)), g("h"), atol=1e-15)
    for th in (0.3, 1.7, -2.9):
        assert np.allclose(g("u3", (th, 0, 0)), g("ry", (th,)), atol=1e-15)
        assert np.allclose(g("u3", (th, -pi / 2, pi / 2)), g("rx", (th,)), atol=1e-15)
        assert np.allclose(g("rz", (th,)), np.exp(-0.5j * th) * g("u3", (0, 0, th)), atol=1e-15)
        assert np.allclose(g("p", (th,)), np.exp(0.5j * th) * g("rz", (th,)), atol=1e-15)
    assert np.allclose(g("s"), g("p", (pi / 2,)), atol=1e-15)
    assert np.allclose(g("t") @ g("t"), g("s"), atol=1e-15)
    assert np.allclose(g("x") @ g("y"), 1j * g("z"), atol=1e-15)
    assert np.allclose(g("h"), (g("x") + g("z")) / math.sqrt(2), atol=1e-15)
    assert np.allclose(g("x"), PX) and np.allclose(g("y"), PY) and np.allclose(g("z"), PZ)


@pytest.mark.parametrize("name,P", [("rx", PX), ("ry", PY), ("rz", PZ)])
def test_rotations_are_pauli_exponentials(name, P):
    for th in np.linspace(-7, 7, 15):
        want = scipy.linalg.expm(-0.5j * th * P)
        assert np.max(np.abs(oracle.gates.matrix(name, (th,)) - want)) < 1e-14


def test_gates_unitary():
    rng = np.random.default_rng(0)
    for name, params in ONE_Q:
        for _ in range(3):
            p = tuple(rng.uniform(0, 2 * math.pi, size=len(params)))
            U = oracle.gates.matrix(name, p)
            assert np.allclose(U @ U.conj().T, I2, atol=1e-15)


def test_uniform_superposition():
    n = 10
    a = oracle.run([Gate("h", (q,)) for q in range(n)], n)
    assert np.max(np.abs(a - 2.0 ** (-n / 2))) < 1e-15


def test_ghz():
    n = 9
    ops = [Gate("h", (0,))] + [W.cx(q, q + 1) for q in range(n - 1)]
    a = oracle.run(ops, n)
    want = np.zeros(1 << n, dtype=np.complex128)
    want[0] = want[-1] = 1 / math.sqrt(2)
    assert np.max(np.abs(a - want)) < 1e-15
    assert abs(oracle.expect_pauli(a, "X" * n) - 1) < 1e-14
    assert abs(oracle.expect_pauli(a, "Z" + "I" * (n - 2) + "Z") - 1) < 1e-14
    assert abs(oracle.expect_pauli(a, "Z" + "I" * (n - 1))) < 1e-14


@pytest.mark.parametrize("n,width,x", [(8, 8, 0b10110011), (10, 8, 0b1101000100), (6, 6, 5)])
def test_qft_ladder_of_basis_state_vs_fft(n, width, x):
    """H + CP(pi/2^d) ladder on the top `width` qubits maps |x> to the Fourier
    vector, output bits reversed (no final swaps)."""
    a = np.zeros(1 << n, dtype=np.complex128)
    a[x] = 1.0
    oracle.run(W.qft_ladder_block(n, width), n, a)
    M = 1 << width
    lo = n - width
    xh = x >> lo
    e = np.zeros(M, dtype=np.complex128)
    e[xh] = 1
    f = np.fft.ifft(e) * math.sqrt(M)  # f[y] = e^{2 pi i xh y / M} / sqrt(M)
    rev = [int(format(y, f"0{width}b")[::-1], 2) for y in range(M)]
    want = np.zeros(1 << n, dtype=np.complex128)
    low = x & ((1 << lo) - 1)
    for y in range(M):
        want[(rev[y] << lo) | low] = f[y]
    assert np.max(np.abs(a - want)) < 1e-14


def test_product_state_expectations():
    n = 8
    rng = np.random.default_rng(4)
    th = rng.uniform(0, 2 * math.pi, n)
    ph = rng.uniform(0, 2 * math.pi, n)
    ops = []
    for q in range(n):
        ops += [Gate("ry", (q,), (), (th[q],)), Gate("rz", (q,), (), (ph[q],))]
    a = oracle.run(ops, n)
    for i in range(n):
        s = ["I"] * n
        s[i] = "Z"
        assert abs(oracle.expect_pauli(a, "".join(s)) - math.cos(th[i])) < 1e-14
        s[i] = "X"
        assert abs(oracle.expect_pauli(a, "".join(s)) - math.sin(th[i]) * math.cos(ph[i])) < 1e-14
        s[i] = "Y"
        assert abs(oracle.expect_pauli(a, "".join(s)) - math.sin(th[i]) * math.sin(ph[i])) < 1e-14
    for i in range(n - 1):
        s = ["I"] * n
        s[i] = s[i + 1] = "Z"
        assert abs(oracle.expect_pauli(a, "".join(s)) - math.cos(th[i]) * math.cos(th[i + 1])) < 1e-14


def test_expectation_vs_kron_brute_force():
    n = 4
    psi = W.random_state(n, 21)
    P = {"I": I2, "X": PX, "Y": PY, "Z": PZ}
    for term in itertools.product("IXYZ", repeat=n):
        full = kron_chain([P[c] for c in reversed(term)])
        want = np.vdot(psi, full @ psi)
        got = oracle.expect_pauli(psi, "".join(term))
        assert abs(got - want) < 1e-14, term
        assert abs(got.imag) < 1e-14


def test_mirror_circuit_returns_to_zero():
    """A unitary followed by its adjoint is the identity (Sec. 2.1, A^-1 = A^dagger)."""
    n = 10
    ops = W.layered_u3_pairing(n, 10, 77, "cx_or_cz") + W.qft_ladder_block(n, 6)
    a = oracle.run(ops + W.inverse(ops), n)
    e0 = np.zeros(1 << n, dtype=np.complex128)
    e0[0] = 1
    assert np.max(np.abs(a - e0)) < 1e-12


def test_mirror_su4_and_rcs():
    n = 9
    for ops in (W.u3_su4_layers(n, 6, 5), W.rcs_circuit(n, 8)):
        a = oracle.run(ops + W.inverse(ops), n)
        assert abs(a[0] - 1) < 1e-12 and np.max(np.abs(a[1:])) < 1e-12


def test_norm_preserved_layered_12q():
    """|alpha|^2 + |beta|^2 = 1 generalised: unitaries keep the norm (Sec. 2.1)."""
    a = oracle.run(W.layered_u3_pairing(12, 20, W.circuit_seed(1, 1)), 12)
    assert abs(oracle.norm2(a) - 1) < 1e-13
    assert abs(np.sum(oracle.probabilities(a)) - 1) < 1e-13


def test_marginals_vs_tensor_sums():
    n = 8
    psi = W.random_state(n, 31)
    p = (np.abs(psi) ** 2).reshape([2] * n)  # axis a <-> qubit n-1-a
    rng = np.random.default_rng(2)
    for m in range(0, n + 1):
        for _ in range(3):
            Q = [int(x) for x in rng.permutation(n)[:m]]
            got = oracle.probabilities(psi, Q)
            keep = [n - 1 - q for q in Q]
            drop = tuple(a for a in range(n) if a not in keep)
            t = p.sum(axis=drop) if drop else p
            # remaining axes are in increasing axis order; reorder so that axis b <-> Q[m-1-b]
            kept_sorted = sorted(keep)
            order = [kept_sorted.index(n - 1 - Q[m - 1 - b]) for b in range(m)]
            want = np.transpose(t, order).reshape(-1) if m else np.array([t.sum()])
            assert np.max(np.abs(got - want)) < 1e-15, Q


def test_sampling_vs_searchsorted():
    n = 10
    psi = W.random_state(n, 41)
    u = W.uniforms(7, 5000)
    got = oracle.sample(psi, u)
    p = np.abs(psi) ** 2
    cdf = np.cumsum(p)
    want = np.searchsorted(cdf, u * cdf[-1], side="right")
    assert np.array_equal(got, want)


def test_sampling_edge_cases():
    psi = np.zeros(8, dtype=np.complex128)
    psi[5] = 1.0
    assert np.all(oracle.sample(psi, np.array([0.0, 0.5, 1 - 2 ** -53])) == 5)
    psi = np.zeros(4, dtype=np.complex128)
    psi[1] = psi[2] = 1 / math.sqrt(2)
    got = oracle.sample(psi, np.array([0.0, 0.49999, 0.5, 0.99]))
    assert list(got) == [1, 1, 2, 2]


def test_sampling_chi2():
    n = 5
    psi = W.random_state(n, 43)
    p = np.abs(psi) ** 2
    shots = 200000
    got = oracle.sample(psi, W.uniforms(9, shots))
    counts = np.bincount(got, minlength=1 << n)
    chi2 = np.sum((counts - shots * p) ** 2 / (shots * p))
    # 31 degrees of freedom: P(chi2 > 70) < 1e-4
    assert chi2 < 70


def test_qpe_exact_phase_every_shot():
    """Phases exactly representable with k bits are read out with certainty (Sec. 2.2 QPE)."""
    for k, m in ((5, 19), (7, 100), (6, 1)):
        a = oracle.run(W.qpe_circuit(k, m), k + 1)
        s = oracle.sample(a, W.uniforms(3, 1000))
        assert np.all(s == (m | (1 << k))), (k, m)


@pytest.mark.parametrize("n,lo,hi,w", [(10, 0, 5, 5), (12, 0, 6, 6), (11, 1, 6, 3), (9, 2, 5, 1)])
def test_bitswap_vs_tensor_transpose(n, lo, hi, w):
    psi = W.random_state(n, 51)
    perm = list(range(n))
    for b in range(w):
        a1, a2 = n - 1 - (lo + b), n - 1 - (hi + b)
        perm[a1], perm[a2] = perm[a2], perm[a1]
    want = np.transpose(psi.reshape([2] * n), perm).reshape(-1)
    got = oracle.bitswap(psi, lo, hi, w)
    assert np.array_equal(got, want)
    assert np.array_equal(oracle.bitswap(got, lo, hi, w), psi)


def test_bitswap_relayout_keeps_logical_state():
    """A gate on logical qubit q after the relayout acts on physical bit map[q]."""
    n, lo, hi, w = 10, 0, 7, 3
    psi = W.random_state(n, 61)
    ops = W.layered_u3_pairing(n, 2, 5, "cx_or_cz")
    want = oracle.run(ops, n, psi.copy())
    phys = oracle.bitswap(psi, lo, hi, w)
    qmap = oracle.apply_bitswap_map(list(range(n)), lo, hi, w)
    for g in ops:
        oracle.apply_matrix(phys, oracle.gate_matrix(g), [qmap[q] for q in g.targets],
                            [qmap[q] for q in g.controls])
    back = oracle.bitswap(phys, lo, hi, w)
    assert np.max(np.abs(back - want)) < 1e-14


def test_triangular_lattice_structure():
    for rows, cols in ((3, 3), (3, 11), (4, 5)):
        e = W.triangular_lattice_edges(rows, cols)
        n = rows * cols
        assert len(e) == 3 * n
        assert len({frozenset(x) for x in e}) == 3 * n and all(a != b for a, b in e)
        deg = np.bincount(np.array(e).reshape(-1), minlength=n)
        assert np.all(deg == 6)
    with pytest.raises(ValueError):
        W.triangular_lattice_edges(2, 5)


def full_op(ops_by_qubit, n):
    """Kronecker product of one-qubit matrices {qubit: M} (identity elsewhere)."""
    return kron_chain([ops_by_qubit.get(q, I2) for q in reversed(range(n))])


@pytest.mark.parametrize("zz", ["cx", "diag"])
def test_tfim_trotter_vs_matrix_exponentials(zz):
    """Each Trotter factor rebuilt independently as scipy's expm of the Pauli
    sums of the TFIM Hamiltonian (H = -J sum ZZ - h sum X) on 9 qubits."""
    rows, cols, steps, dt, J, h = 3, 3, 3, 0.13, 0.9, 1.7
    n = rows * cols
    a = oracle.run(W.tfim_trotter(rows, cols, steps, dt, J, h, zz), n)
    zz_sum = sum(full_op({p: PZ, q: PZ}, n) for p, q in W.triangular_lattice_edges(rows, cols))
    x_sum = sum(full_op({q: PX}, n) for q in range(n))
    step = scipy.linalg.expm(1j * h * dt * x_sum) @ scipy.linalg.expm(1j * J * dt * zz_sum)
    want = np.zeros(1 << n, dtype=np.complex128)
    want[0] = 1.0
    for _ in range(steps):
        want = step @ want
    assert np.max(np.abs(a - want)) < 1e-12


def test_tfim_closed_forms():
    rows, cols, steps, dt = 3, 4, 5, 0.21
    n = rows * cols
    E = len(W.triangular_lattice_edges(rows, cols))
    # no field: the Ising part is diagonal and |0...0> only picks up exp(i J dt E steps)
    a = oracle.run(W.tfim_trotter(rows, cols, steps, dt, J=1.3, h=0.0), n)
    assert abs(a[0] - np.exp(1j * 1.3 * dt * E * steps)) < 1e-13
    assert np.max(np.abs(a[1:])) < 1e-13
    # no coupling: a product of X rotations by 2 h dt steps on every qubit
    a = oracle.run(W.tfim_trotter(rows, cols, steps, dt, J=0.0, h=0.8, zz="diag"), n)
    for q in (0, 5, n - 1):
        s = ["I"] * n
        s[q] = "Z"
        assert abs(oracle.expect_pauli(a, "".join(s)) - math.cos(2 * 0.8 * dt * steps)) < 1e-13


def test_golden_paper_sizes():
    with open(os.path.join(GOLDEN, "paper_figures.json")) as f:
        gold = json.load(f)
    ex = gold["fp32_state_gib"]["example"]
    # complex64 = 8 bytes per amplitude
    assert (1 << ex["qubits"]) * 8 == ex["gib"] * 2 ** 30
    assert 2 ** (ex["qubits"] - gold["fp32_state_gib"]["formula_exponent_offset"]) == ex["gib"]
    n = 11
    ops = W.rcs_circuit(n, 1)
    assert len(ops) == gold["rcs_gate_count"]["per_qubit"] * n
    big = [g for s in range(10) for g in W.rcs_circuit(40, 100 + s)]
    frac_cz = sum(1 for g in big if g.controls) / len(big)
    # 12000 draws: standard deviation of the fraction is 0.004
    assert abs(frac_cz - gold["rcs_gate_count"]["cz_probability"]) < 0.02
