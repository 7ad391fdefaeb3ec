"""Parity of the HIP path with the FP64 reference, through the C ABI.

Tolerances: max |delta amplitude| <= 1e-12 for complex128 and <= 2e-5 for
complex64 (depth <= 200); bit-exact for the qubit-field exchange and index
work; read-outs compared on the very state the GPU holds (copied back), so
only the FP64 summation order differs.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from workloads import Gate

import paper_2511_14664_amd as svm
from paper_2511_14664_amd import _binding as B

from error_bounds import check_state, mirror_l2, state_bounds

pytestmark = pytest.mark.gpu

TOL = {B.SV_C128: 1e-12, B.SV_C64: 2e-5}
DTYPES = [B.SV_C128, B.SV_C64]
DNAME = {B.SV_C128: "c128", B.SV_C64: "c64"}


class State:
    """Library-owned device state (sv_create)."""

    def __init__(self, n, dtype):
        self.n, self.dtype = n, dtype
        self.h = B.sv_create(n, dtype)

    def close(self):
        if self.h:
            B.sv_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def load(self, psi):
        B.sv_copy_from_host(self.h, self.dtype, psi)
        return np.asarray(psi, dtype=B.amp_dtype(self.dtype)).astype(np.complex128)

    def host(self):
        return B.sv_copy_to_host(self.h, self.n, self.dtype).astype(np.complex128)

    def host_raw(self):
        return B.sv_copy_to_host(self.h, self.n, self.dtype)


def say(*a):
    print(*a, flush=True)


def maxerr(a, b):
    return float(np.max(np.abs(a - b)))


def run_checked(s, gates, opts, want, random_circuit=False):
    """Apply a circuit with its sweeps recorded, then compare the state with
    the oracle's: max |d amp| within TOL and ||d psi||_2 within the rounding
    bound of the recorded sweeps (``tests/error_bounds.py``)."""
    B.sv_profile_read(s.h)
    B.sv_profile_enable(s.h, True)
    st = B.sv_apply_circuit(s.h, gates, opts)
    recs = B.sv_profile_read(s.h, 1 << 14)
    B.sv_profile_enable(s.h, False)
    mx, l2, bound = check_state(s.host(), want, s.dtype == B.SV_C64, s.n, recs, gates, random_circuit)
    say(f"  max|d amp| {mx:.2e}, ||d psi||_2 {l2:.2e} (bound {bound:.2e})")
    return st, recs


# ---------------------------------------------------------------------------
# 12-qubit complex128 layered circuit: whole state and all probabilities
# ---------------------------------------------------------------------------
def test_layered_12q_c128_full_state_and_probabilities():
    n = 12
    gates = W.layered_u3_pairing(n, 20, W.circuit_seed(1, 1), "cx")
    assert len(gates) == 360
    want = oracle.run(gates, n)
    for mode in (B.SV_PLAN_PLAIN, B.SV_PLAN_GREEDY):
        say("12q c128 mode", mode)
        with State(n, B.SV_C128) as s:
            st = B.sv_apply_circuit(s.h, gates, B.make_opts(mode, 5))
            got = s.host()
            assert maxerr(got, want) <= 1e-12
            p = B.sv_probabilities(s.h, list(range(n)))
            assert maxerr(p, oracle.probabilities(want)) <= 1e-12
            assert st["gates"] == 360
            if mode == B.SV_PLAN_PLAIN:
                assert st["sweeps"] == 360
            else:
                assert st["sweeps"] < 60


# ---------------------------------------------------------------------------
# Every one-qubit kind at every target position, with controls
# ---------------------------------------------------------------------------
ONE_Q = [("h", ()), ("x", ()), ("y", ()), ("z", ()), ("s", ()), ("t", ()), ("rx", (0.7,)),
         ("ry", (1.9,)), ("rz", (-2.3,)), ("p", (0.4,)), ("u3", (0.3, 1.1, -0.8))]


@pytest.mark.parametrize("dtype", DTYPES, ids=DNAME.get)
def test_one_qubit_gates_every_position(dtype):
    n = 11
    psi = W.random_state(n, 3)
    with State(n, dtype) as s:
        for name, params in ONE_Q:
            for t in range(n):
                others = [q for q in range(n) if q != t]
                for ctrls in [(), (others[(t * 3) % (n - 1)],), (others[0], others[-1]),
                              tuple(others[1:4])]:
                    g = Gate(name, (t,), ctrls, params)
                    ref = s.load(psi)
                    B.sv_apply_circuit(s.h, [g])
                    got = s.host()
                    want = oracle.apply_gate(ref.copy(), g)
                    e = maxerr(got, want)
                    assert e <= TOL[dtype] / 10, (name, t, ctrls, e)


@pytest.mark.parametrize("dtype", DTYPES, ids=DNAME.get)
@pytest.mark.parametrize("n", [12, 16])
def test_one_target_low_targets_with_high_controls(dtype, n):
    """Targets inside one 128-byte line (index bits 1..3 of complex64, 0..2
    of complex128) with no control on the bits above them up to 8 swap
    partners between lanes (the other modes stay for controls on bits 4..8,
    3..8); every target and control placement against the reference."""
    psi = W.random_state(n, 5 + n)
    with State(n, dtype) as s:
        for t in ((1, 2, 3) if dtype == B.SV_C64 else (0, 1, 2)):
            for ctrls in [(), (9,), (n - 1,), (9, n - 2), (9, 10, n - 1), (0,), (5,), (8, n - 1), (3,)]:
                if t in ctrls:
                    continue
                for name, params in (("u3", (0.3, 1.1, -0.7)), ("h", ()), ("x", ())):
                    g = Gate(name, (t,), ctrls, params)
                    ref = s.load(psi)
                    B.sv_apply_circuit(s.h, [g])
                    got = s.host()
                    want = oracle.apply_gate(ref.copy(), g)
                    e = maxerr(got, want)
                    assert e <= TOL[dtype] / 10, (name, t, ctrls, e)


IN_LINE_CTRLS = [(0,), (1,), (2,), (3,), (1, 2), (0, 3), (0, 1, 2, 3), (2, 5), (3, -1), (0, 9), (1, 4, -1)]


@pytest.mark.parametrize("dtype", DTYPES, ids=DNAME.get)
@pytest.mark.parametrize("n", [13, 16])
def test_one_target_in_line_controls(dtype, n):
    """Controls on the index bits of one 128-byte line are tested per
    amplitude while whole lines are read and written: dense and diagonal
    one-target gates (d0 = 1 or not) at low and high targets against the
    reference, and every amplitude whose controls (or, for d0 = 1, target)
    are not all set comes back bit for bit as it went in."""
    psi = W.random_state(n, 17 + n)
    kinds = [("u3", (0.3, 1.1, -0.7)), ("x", ()), ("h", ()), ("z", ()), ("s", ()), ("rz", (0.9,)),
             ("p", (-1.3,))]
    idx = np.arange(1 << n)
    with State(n, dtype) as s:
        for t in (0, 1, 2, 3, 4, 7, n - 1):
            for cs in IN_LINE_CTRLS:
                ctrls = tuple(sorted({q % n for q in cs} - {t}))
                if not ctrls:
                    continue
                for name, params in kinds:
                    g = Gate(name, (t,), ctrls, params)
                    say(f"n={n} {DNAME[dtype]} {name} t={t} controls={ctrls}")
                    ref = s.load(psi)
                    B.sv_apply_circuit(s.h, [g])
                    raw = s.host_raw()
                    want = oracle.apply_gate(ref.copy(), g)
                    e = maxerr(raw.astype(np.complex128), want)
                    assert e <= TOL[dtype] / 10, (name, t, ctrls, e)
                    cm = sum(1 << q for q in ctrls)
                    keep = (idx & cm) != cm
                    if name in ("z", "s", "p"):
                        keep |= ((idx >> t) & 1) == 0
                    before = np.asarray(psi, dtype=B.amp_dtype(dtype))
                    assert np.array_equal(raw[keep].view(np.uint8), before[keep].view(np.uint8)), (name, t, ctrls)


@pytest.mark.parametrize("dtype", DTYPES, ids=DNAME.get)
@pytest.mark.parametrize("n", [8, 14, 17])
def test_multi_target_gates(dtype, n):
    """k = 2..6 targets at random and at the lowest/highest positions, 0-2
    controls; n = 8 takes the per-group path, n >= 14 the LDS tile."""
    rng = np.random.default_rng(n)
    psi = W.random_state(n, 5)
    with State(n, dtype) as s:
        for k in range(2, 7):
            placements = [list(range(k)), list(range(n - k, n))]
            for _ in range(3):
                placements.append([int(x) for x in rng.permutation(n)[:k]])
            for tg in placements:
                rest = [q for q in range(n) if q not in tg]
                for nc in (0, 1, 2):
                    if k + nc > n:
                        continue
                    ctl = [int(x) for x in rng.permutation(rest)[:nc]]
                    U = W.haar_unitary(rng, 1 << k)
                    say(f"n={n} {DNAME[dtype]} k={k} targets={tg} controls={ctl}")
                    ref = s.load(psi)
                    B.sv_apply_gate(s.h, U, tg, ctl)
                    want = oracle.apply_matrix(ref.copy(), U, tg, ctl)
                    e = maxerr(s.host(), want)
                    assert e <= TOL[dtype] / 10, (k, tg, ctl, e)


@pytest.mark.parametrize("dtype", DTYPES, ids=DNAME.get)
@pytest.mark.parametrize("kmax", [2, 3, 4, 5, 6])
def test_fused_circuits(dtype, kmax):
    n = 16
    gates = (W.layered_u3_pairing(n, 8, 9, "cx_or_cz") + W.qft_ladder_block(n, 8)
             + W.u3_su4_layers(n, 3, 4) + W.rcs_circuit(n, 11)[:200])
    want = oracle.run(gates, n)
    say(f"fused n={n} {DNAME[dtype]} kmax={kmax} gates={len(gates)}")
    with State(n, dtype) as s:
        st = B.sv_apply_circuit(s.h, gates, B.make_opts(B.SV_PLAN_GREEDY, kmax))
        e = maxerr(s.host(), want)
        assert e <= TOL[dtype], e
        assert st["sweeps"] < len(gates)


# ---------------------------------------------------------------------------
# Qubit bit-field exchange
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", DTYPES, ids=DNAME.get)
@pytest.mark.parametrize("n,lo,hi,w", [(14, 0, 8, 6), (16, 0, 10, 6), (13, 2, 7, 3), (12, 5, 9, 1), (12, 0, 6, 6)])
def test_bitswap_bit_exact(dtype, n, lo, hi, w):
    import torch

    psi = W.random_state(n, 13).astype(B.amp_dtype(dtype))
    with svm.StateVector(n, dtype) as sv:
        sv.from_host(psi)
        sv.swap_bits(lo, hi, w)
        sv.synchronize()
        raw = sv.buffer.cpu().numpy().view(B.amp_dtype(dtype)).copy()
        want = oracle.bitswap(psi.astype(np.complex128), lo, hi, w).astype(B.amp_dtype(dtype))
        assert np.array_equal(raw.view(np.uint8), want.view(np.uint8))
        assert sv.qubit_map() == oracle.apply_bitswap_map(list(range(n)), lo, hi, w)
        # logical read-out is unchanged, bit for bit
        assert np.array_equal(sv.to_host().view(np.uint8), psi.view(np.uint8))
        sv.swap_bits(lo, hi, w)
        sv.synchronize()
        raw2 = sv.buffer.cpu().numpy().view(B.amp_dtype(dtype))
        assert np.array_equal(raw2.view(np.uint8), psi.view(np.uint8))
        assert sv.qubit_map() == list(range(n))
    torch.cuda.synchronize()


@pytest.mark.parametrize("dtype", DTYPES, ids=DNAME.get)
@pytest.mark.parametrize("mode", [B.SV_PLAN_PLAIN, B.SV_PLAN_GREEDY])
def test_relaid_out_circuit_matches_swap_free_reference(dtype, mode):
    n = 16
    ops = W.share_layers(n, 4, 21, swap_every=2, swap_width=6)
    want = oracle.run(ops, n)
    with State(n, dtype) as s:
        seg = []
        for op in ops + [None]:
            if op is None or isinstance(op, W.BitSwap):
                if seg:
                    B.sv_apply_circuit(s.h, seg, B.make_opts(mode, 5))
                    seg = []
                if op is not None:
                    B.sv_swap_bits(s.h, op.lo, op.hi, op.width)
            else:
                seg.append(op)
        got = s.host()
        assert maxerr(got, want) <= TOL[dtype]
        # read-outs through the map
        p = B.sv_probabilities(s.h, [n - 1, 0, 3])
        assert maxerr(p, oracle.probabilities(want, [n - 1, 0, 3])) <= (1e-12 if dtype == B.SV_C128 else 1e-5)
        z = B.sv_expect_pauli(s.h, ["Z" + "I" * (n - 2) + "Z", "X" + "I" * (n - 1)])
        zw = [oracle.expect_pauli(want, "Z" + "I" * (n - 2) + "Z").real,
              oracle.expect_pauli(want, "X" + "I" * (n - 1)).real]
        assert maxerr(z, np.array(zw)) <= (1e-12 if dtype == B.SV_C128 else 1e-5)


# ---------------------------------------------------------------------------
# Read-outs on the GPU's own state
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", DTYPES, ids=DNAME.get)
@pytest.mark.parametrize("n", [5, 14, 20])
def test_marginals(dtype, n):
    rng = np.random.default_rng(n)
    psi = W.random_state(n, 17)
    with State(n, dtype) as s:
        ref = s.load(psi)
        qsets = [[], [0], [n - 1], list(range(n)), list(range(n))[::-1]]
        # low bins (segment fold), low + high bins, one low bin, many low bins
        qsets += [[q for q in Q if q < n] for Q in ([5, 4, 3, 2, 1, 0], [0, 13], [1], [3, 7, 11, 19],
                                                      list(range(10)), [11, 0, 16, 6, 12])]
        for m in (2, 3, min(7, n), min(12, n)):
            qsets.append([int(x) for x in rng.permutation(n)[:m]])
        for Q in qsets:
            say(f"marginal n={n} {DNAME[dtype]} Q={Q}")
            got = B.sv_probabilities(s.h, Q)
            want = oracle.probabilities(ref, Q)
            assert maxerr(got, want) <= 1e-12 * max(1.0, float(np.max(want))), Q


def test_marginal_folding_several_segments_per_workgroup():
    # 27 qubits with 10 bin bits below bit 12: the folded array would exceed
    # 2^24 doubles, so each workgroup folds two 4096-amplitude segments
    n = 27
    rng = np.random.default_rng(5)
    with State(n, B.SV_C64) as s:
        B.sv_apply_circuit(s.h, W.layered_u3_pairing(n, 2, W.circuit_seed(3, 1), "cx"))
        amp = s.host()
        for Q in (list(range(10)), [9, 3, 0, 22, 1, 2, 4, 5, 6, 7, 8], [int(x) for x in rng.permutation(12)[:10]] + [26]):
            say(f"marginal n={n} c64 Q={Q}")
            got = B.sv_probabilities(s.h, Q)
            want = oracle.probabilities(amp, Q)
            assert maxerr(got, want) <= 1e-12


@pytest.mark.parametrize("dtype", DTYPES, ids=DNAME.get)
def test_z_string_expectations_in_batches(dtype):
    n = 20
    rng = np.random.default_rng(11)
    psi = W.random_state(n, 23)
    terms = ["".join(rng.choice(list("IZ"), size=n)) for _ in range(45)] + ["I" * n]
    with State(n, dtype) as s:
        ref = s.load(psi)
        for sub in (terms, terms[:7], terms[:16], terms[:33]):
            got = B.sv_expect_pauli(s.h, sub)
            want = np.array([oracle.expect_pauli(ref, t).real for t in sub])
            assert maxerr(got, want) <= 1e-12


@pytest.mark.parametrize("dtype", DTYPES, ids=DNAME.get)
def test_pauli_expectations(dtype):
    n = 12
    rng = np.random.default_rng(7)
    psi = W.random_state(n, 19)
    terms = ["I" * n, "Z" * n, "X" * n, "Y" * n]
    for _ in range(40):
        terms.append("".join(rng.choice(list("IXYZ"), size=n)))
    for _ in range(20):
        terms.append("".join(rng.choice(list("IZ"), size=n)))
    with State(n, dtype) as s:
        ref = s.load(psi)
        got = B.sv_expect_pauli(s.h, terms)
        want = np.array([oracle.expect_pauli(ref, t).real for t in terms])
        assert maxerr(got, want) <= 1e-12


def sample_ok(state, u, got, tau):
    p = np.abs(state) ** 2
    cdf = np.cumsum(p)
    norm = cdf[-1]
    want = oracle.sample(state, u)
    bad = []
    for s in range(len(u)):
        if got[s] == want[s]:
            continue
        g = int(got[s])
        t = u[s] * norm
        lo = cdf[g - 1] if g > 0 else 0.0
        if not (lo - tau <= t < cdf[g] + tau and p[g] > 0):
            bad.append((s, g, int(want[s])))
    return bad


@pytest.mark.parametrize("dtype", DTYPES, ids=DNAME.get)
@pytest.mark.parametrize("n", [3, 12, 16, 19])
def test_sampling_index_agreement(dtype, n):
    psi = W.random_state(n, 23)
    u = W.uniforms(7, 3000)
    with State(n, dtype) as s:
        ref = s.load(psi)
        got = B.sv_sample(s.h, u)
        bad = sample_ok(ref, u, got, 1e-12)
        assert not bad, bad[:5]


def test_sampling_qpe_exact_phase():
    k, m = 9, 301
    n = k + 1
    with State(n, B.SV_C128) as s:
        B.sv_apply_circuit(s.h, W.qpe_circuit(k, m))
        out = B.sv_sample(s.h, W.uniforms(5, 1000))
        assert np.all(out == (m | (1 << k)))


def test_sampling_ghz_and_edges():
    n = 18
    ops = [Gate("h", (0,))] + [W.cx(q, q + 1) for q in range(n - 1)]
    with State(n, B.SV_C64) as s:
        B.sv_apply_circuit(s.h, ops)
        u = np.array([0.0, 0.25, 0.4999, 0.5001, 0.75, 1 - 2 ** -53])
        out = B.sv_sample(s.h, u)
        assert list(out[:3]) == [0, 0, 0] and list(out[3:]) == [(1 << n) - 1] * 3
        with pytest.raises(B.SvError):
            B.sv_sample(s.h, np.array([1.0]))
        assert B.sv_sample(s.h, np.array([])).size == 0


# ---------------------------------------------------------------------------
# Full-size 28-qubit workload in the benchmark's launch configuration
# ---------------------------------------------------------------------------
def split_layers(n, layers, seed):
    """Layered U3 + CNOT/CZ circuit that never couples qubits < n/2 with qubits
    >= n/2, so the state is a product of two half-size states the reference
    computes exactly."""
    h = n // 2
    lo = W.layered_u3_pairing(h, layers, seed, "cx_or_cz")
    hi = W.layered_u3_pairing(n - h, layers, seed + 1, "cx_or_cz")
    shift = [Gate(g.name, tuple(q + h for q in g.targets), tuple(q + h for q in g.controls), g.params, g.matrix)
             for g in hi]
    return lo, hi, lo + shift


@pytest.mark.parametrize("dtype", DTYPES, ids=DNAME.get)
def test_28q_product_circuit_full_state(dtype):
    """A 28-qubit layered circuit that never couples its two 14-qubit halves:
    the oracle's state is the product of the halves' states, compared with
    all 2^28 amplitudes the GPU holds under each plan."""
    n = 28
    lo, hi, gates = split_layers(n, 20, 77)
    a_lo = oracle.run(lo, 14)
    a_hi = oracle.run(hi, 14)
    want = np.outer(a_hi, a_lo).reshape(-1)
    for mode in (B.SV_PLAN_PASSES, B.SV_PLAN_GREEDY, B.SV_PLAN_PLAIN):
        say(f"28q product {DNAME[dtype]} mode={mode}")
        with State(n, dtype) as s:
            run_checked(s, gates, B.make_opts(mode, 5), want)
            norm = B.sv_probabilities(s.h, [])[0]
            assert abs(norm - 1) < (1e-12 if dtype == B.SV_C128 else 1e-5)
            if mode == B.SV_PLAN_PASSES:
                check_product_readouts(s, dtype, a_lo, a_hi)
                # the benchmark's 6-bit exchange (physical bits 0..5 <-> 22..27)
                # moves amplitudes without arithmetic and updates the qubit
                # map: the logical amplitudes read back are bit-identical
                before = s.host_raw()
                B.sv_swap_bits(s.h, 0, n - 6, 6)
                qmap = list(B.sv_qubit_map(s.h, n))
                assert qmap[:6] == list(range(22, 28)) and qmap[22:] == list(range(6))
                assert np.array_equal(before.view(np.uint8), s.host_raw().view(np.uint8))


def check_product_readouts(s, dtype, a_lo, a_hi):
    """The benchmark's read-outs on a product of two 14-qubit states: Z-string
    expectations factor into the halves' expectations; the 1000 shots agree
    index by index with the oracle's sampler run on the GPU's own state
    (copied back), up to the summation-order window at CDF steps."""
    zs = W.hea_z_terms(28)
    terms = zs[:32] + [zs[28 + 13]]  # the benchmark's 32 strings and Z13 Z14 across the halves
    got = B.sv_expect_pauli(s.h, terms)
    want = np.array([oracle.expect_pauli(a_lo, t[:14]).real * oracle.expect_pauli(a_hi, t[14:]).real
                     for t in terms])
    assert maxerr(got, want) <= TOL[dtype]
    u = W.uniforms(7, 1000)
    shots = B.sv_sample(s.h, u)
    bad = sample_ok(s.host(), u, shots, 1e-12)
    assert not bad, bad[:5]


def test_28q_marginal_low_bins_several_segments_per_workgroup():
    """Nine bin bits 0..8 at 28 qubits (complex64): each thread sums its
    loads over index bits 9..11 in registers, and the folded array would
    exceed 2^24 doubles, so each workgroup folds two segments.  The state is
    a product of two 14-qubit halves, so the marginals are the oracle's
    14-qubit marginals (times a one-qubit marginal of the upper half)."""
    n = 28
    lo, hi, gates = split_layers(n, 20, 91)
    a_lo = oracle.run(lo, 14)
    a_hi = oracle.run(hi, 14)
    with State(n, B.SV_C64) as s:
        B.sv_apply_circuit(s.h, gates, B.make_opts(B.SV_PLAN_PASSES))
        assert list(B.sv_qubit_map(s.h, n))[:9] == list(range(9))
        low = list(range(9))
        say("28q marginal over bits 0..8")
        got = B.sv_probabilities(s.h, low)
        assert maxerr(got, oracle.probabilities(a_lo, low)) <= TOL[B.SV_C64]
        say("28q marginal over bits 0..8 and 27")
        got = B.sv_probabilities(s.h, low + [27])
        want = np.outer(oracle.probabilities(a_hi, [13]), oracle.probabilities(a_lo, low)).reshape(-1)
        assert maxerr(got, want) <= TOL[B.SV_C64]


@pytest.mark.parametrize("dtype", DTYPES, ids=DNAME.get)
def test_28q_layered_mirror_returns_to_zero(dtype):
    n = 28
    gates = W.layered_u3_pairing(n, 20, W.circuit_seed(2, 1), "cx_or_cz")
    for mode in (B.SV_PLAN_PASSES, B.SV_PLAN_GREEDY):
        say(f"28q mirror {DNAME[dtype]} mode={mode}")
        with State(n, dtype) as s:
            B.sv_profile_enable(s.h, True)
            B.sv_apply_circuit(s.h, gates, B.make_opts(mode, 5))
            B.sv_apply_circuit(s.h, W.inverse(gates), B.make_opts(mode, 5))
            recs = B.sv_profile_read(s.h, 1 << 14)
            a0 = complex(B.sv_copy_to_host(s.h, n, dtype, 0, 1)[0])
            l2, res = mirror_l2(B.sv_probabilities(s.h, [])[0], a0, n)
            det, prob = state_bounds(recs, n, dtype == B.SV_C64)
            say(f"  ||psi - |0>||_2 {l2:.2e} (bounds: deterministic {det:.2e}, probabilistic {prob:.2e}; resolution {res:.1e})")
            assert l2 <= det + res
            p = B.sv_probabilities(s.h, [0, 27, 13])
            assert abs(p[0] - 1) <= 2 * det and np.all(np.abs(p[1:]) <= (det + res) ** 2)


# ---------------------------------------------------------------------------
# Torch-owned memory and stream
# ---------------------------------------------------------------------------
def test_statevector_on_torch_memory_and_stream():
    import torch

    n = 10
    gates = W.layered_u3_pairing(n, 5, 3, "cx_or_cz")
    want = oracle.run(gates, n)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        with svm.StateVector(n, B.SV_C128) as sv:
            sv.apply_circuit(gates, mode=B.SV_PLAN_GREEDY, max_fused=4)
            assert maxerr(sv.to_host(), want) <= 1e-12
    torch.cuda.synchronize()


# ---------------------------------------------------------------------------
# complex64 fused blocks with the three-term BF16 split on the matrix cores
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("kmax", [5, 6])
def test_bf16x3_fused_circuits(kmax):
    n = 16
    gates = (W.layered_u3_pairing(n, 8, 9, "cx_or_cz") + W.u3_su4_layers(n, 4, 4))
    want = oracle.run(gates, n)
    with State(n, B.SV_C64) as s:
        B.sv_profile_enable(s.h, True)
        st = B.sv_apply_circuit(s.h, gates, B.make_opts(B.SV_PLAN_GREEDY, kmax, B.SV_PREC_BF16X3))
        kinds = {r["kind_name"] for r in B.sv_profile_read(s.h)}
        assert "dense_bf16x3" in kinds
        e = maxerr(s.host(), want)
        say(f"bf16x3 kmax={kmax}: {st['sweeps']} sweeps, max|d amp| = {e:.2e}")
        assert e <= TOL[B.SV_C64]


def test_bf16x3_single_blocks_every_placement():
    n = 14
    rng = np.random.default_rng(21)
    psi = W.random_state(n, 22)
    with State(n, B.SV_C64) as s:
        for k in (5, 6):
            for tg in (list(range(k)), list(range(n - k, n)), [int(x) for x in rng.permutation(n)[:k]]):
                for ctl in ([], [q for q in range(n) if q not in tg][:1]):
                    if n - len(ctl) < 12:
                        continue
                    U = W.haar_unitary(rng, 1 << k)
                    ref = s.load(psi)
                    gate = Gate("matrix", tuple(tg), tuple(ctl), (), U)
                    B.sv_apply_circuit(s.h, [gate], B.make_opts(B.SV_PLAN_PLAIN, 1, B.SV_PREC_BF16X3))
                    want = oracle.apply_matrix(ref.copy(), U, tg, ctl)
                    e = maxerr(s.host(), want)
                    # one block: relative error ~2^-16 of amplitudes of size ~2^-7
                    assert e <= 1e-6, (k, tg, ctl, e)


# ---------------------------------------------------------------------------
# LDS passes (SV_PLAN_PASSES)
# ---------------------------------------------------------------------------
def pass_circuit(n, seed):
    """Layered circuit plus controlled one-qubit gates, 2..4-target matrix
    gates, a controlled matrix gate and (n >= 6) a 5-target matrix gate, which
    no pass kernel takes (its pass runs as ordinary sweeps)."""
    rng = np.random.default_rng(seed)
    gates = list(W.layered_u3_pairing(n, 6, W.circuit_seed(7, seed), "cx_or_cz"))
    for _ in range(6):
        q = [int(x) for x in rng.permutation(n)[:3]]
        gates.append(Gate("u3", (q[0],), tuple(q[1:1 + int(rng.integers(1, 3))]), tuple(rng.uniform(0, 6, 3))))
    for k in (2, 3, 4):
        q = [int(x) for x in rng.permutation(n)[:k]]
        gates.append(Gate("matrix", tuple(q), (), (), W.haar_unitary(rng, 1 << k)))
    q = [int(x) for x in rng.permutation(n)[:3]]
    gates.append(Gate("matrix", tuple(q[:2]), (q[2],), (), W.haar_unitary(rng, 4)))
    if n >= 6:
        q = [int(x) for x in rng.permutation(n)[:5]]
        gates.append(Gate("matrix", tuple(q), (), (), W.haar_unitary(rng, 32)))
    gates += list(W.layered_u3_pairing(n, 4, W.circuit_seed(8, seed), "cx"))
    return gates


@pytest.mark.parametrize("dtype", DTYPES, ids=DNAME.get)
@pytest.mark.parametrize("n", [9, 11, 12, 14, 20])
def test_pass_plan_matches_oracle(dtype, n):
    gates = pass_circuit(n, n)
    want = oracle.run(gates, n)
    for pq in (0, 4, 6, 8):
        say(f"passes n={n} {DNAME[dtype]} pass_qubits={pq}")
        with State(n, dtype) as s:
            st, _ = run_checked(s, gates, B.make_opts(B.SV_PLAN_PASSES, 5, B.SV_PREC_NATIVE, pq), want)
            assert st["gates"] == len(gates) and 1 <= st["sweeps"] < len(gates)


@pytest.mark.parametrize("dtype", DTYPES, ids=DNAME.get)
def test_pass_plan_after_relayout_and_profile_records(dtype):
    n = 16
    a = W.layered_u3_pairing(n, 5, W.circuit_seed(9, 1), "cx_or_cz")
    b = pass_circuit(n, 3)
    want = oracle.run(list(a) + list(b), n)
    with State(n, dtype) as s:
        B.sv_apply_circuit(s.h, a, B.make_opts(B.SV_PLAN_PASSES))
        B.sv_swap_bits(s.h, 0, n - 6, 6)
        B.sv_swap_bits(s.h, 2, 9, 3)
        B.sv_profile_read(s.h)
        B.sv_profile_enable(s.h, True)
        st = B.sv_apply_circuit(s.h, b, B.make_opts(B.SV_PLAN_PASSES))
        recs = B.sv_profile_read(s.h)
        assert maxerr(s.host(), want) <= TOL[dtype]
        kinds = {r["kind_name"] for r in recs}
        assert "pass" in kinds and len(recs) == st["sweeps"]
        assert sum(r["num_gates"] for r in recs) == len(b)
        # a pass holds at most 8 qubits above the tile's lowest bits, and at most the tile
        assert all(r["k"] <= r["tile_log"] and r["ms"] > 0 for r in recs if r["kind_name"] == "pass")


def phase_circuit(n, seed, layers=6):
    """Layers of U3 on every qubit and diagonal gates on random qubits across
    the register: CP (angles up to +-20 rad), CZ, RZ, doubly controlled P and
    2-qubit diagonal matrices.  Pass plans take most of them as per-tile
    phases on qubits outside the pass tile."""
    rng = np.random.default_rng(seed)
    gates = []
    for _ in range(layers):
        for q in range(n):
            gates.append(Gate("u3", (q,), (), tuple(float(x) for x in rng.uniform(0, 2 * math.pi, 3))))
        for _ in range(n):
            kind = int(rng.integers(0, 5))
            qs = [int(x) for x in rng.permutation(n)[:3]]
            if kind == 0:
                gates.append(W.cp(qs[0], qs[1], float(rng.uniform(-20, 20))))
            elif kind == 1:
                gates.append(W.cz(qs[0], qs[1]))
            elif kind == 2:
                gates.append(Gate("rz", (qs[0],), (), (float(rng.uniform(-9, 9)),)))
            elif kind == 3:
                gates.append(Gate("p", (qs[0],), (qs[1], qs[2]), (float(rng.uniform(0, 2 * math.pi)),)))
            else:
                d = np.diag(np.exp(1j * rng.uniform(0, 2 * math.pi, 4)))
                gates.append(Gate("matrix", (qs[0], qs[1]), (), (), d))
    return gates


@pytest.mark.parametrize("dtype", DTYPES, ids=DNAME.get)
@pytest.mark.parametrize("n", [13, 16, 20])
def test_pass_plan_phase_gates_match_oracle(dtype, n):
    gates = phase_circuit(n, 40 + n)
    want = oracle.run(gates, n)
    for pq in (6, 8):
        say(f"phase passes n={n} {DNAME[dtype]} pass_qubits={pq}")
        with State(n, dtype) as s:
            st, _ = run_checked(s, gates, B.make_opts(B.SV_PLAN_PASSES, 5, B.SV_PREC_NATIVE, pq), want)
            assert st["gates"] == len(gates)


def control_circuit(n, seed, layers=6):
    """Layers of H/U3 and controlled non-diagonal gates whose controls fall
    anywhere in the register: CX, doubly controlled U3 and controlled 2-qubit
    matrices, with some CZ.  Pass plans stage a block whose controls lie
    outside the tile as one matrix per value of those control bits."""
    rng = np.random.default_rng(seed)
    gates = []
    for layer in range(layers):
        for q in range(n):
            if layer % 2:
                gates.append(Gate("h", (q,)))
            else:
                gates.append(Gate("u3", (q,), (), tuple(float(x) for x in rng.uniform(0, 2 * math.pi, 3))))
        for _ in range(n):
            kind = int(rng.integers(0, 4))
            qs = [int(x) for x in rng.permutation(n)[:4]]
            if kind == 0:
                gates.append(W.cx(qs[0], qs[1]))
            elif kind == 1:
                gates.append(Gate("u3", (qs[0],), (qs[1], qs[2]), tuple(float(x) for x in rng.uniform(0, 2 * math.pi, 3))))
            elif kind == 2:
                gates.append(Gate("matrix", (qs[0], qs[1]), (qs[2],), (), W.haar_unitary(rng, 4)))
            else:
                gates.append(W.cz(qs[0], qs[1]))
    return gates


@pytest.mark.parametrize("dtype", DTYPES, ids=DNAME.get)
@pytest.mark.parametrize("n", [14, 20])
def test_pass_plan_outer_controls_match_oracle(dtype, n):
    gates = control_circuit(n, 60 + n)
    want = oracle.run(gates, n)
    for pq in (6, 8):
        say(f"outer-control passes n={n} {DNAME[dtype]} pass_qubits={pq}")
        with State(n, dtype) as s:
            st, _ = run_checked(s, gates, B.make_opts(B.SV_PLAN_PASSES, 5, B.SV_PREC_NATIVE, pq), want)
            assert st["gates"] == len(gates)


def term_heavy_circuit(n, reps, seed):
    """H on qubits 0..7, then controlled phases from each of them to six
    random qubits above, repeated: blocks whose phase gates reach many qubits
    outside the tile (per-tile phase terms), split where an H follows."""
    rng = np.random.default_rng(seed)
    gates = []
    for _ in range(reps):
        for q in range(8):
            gates.append(Gate("h", (q,)))
        for q in range(8):
            for o in rng.permutation(np.arange(8, n))[:6]:
                gates.append(W.cp(q, int(o), float(rng.uniform(-3, 3))))
    return gates


@pytest.mark.parametrize("dtype", DTYPES, ids=DNAME.get)
def test_pass_plan_term_heavy_matches_oracle(dtype):
    """The default plan, and passes of at most 6 qubits above the tile's
    lowest bits, which take most of the phase gates as per-tile phase terms
    (at least 20 blocks with terms)."""
    n = 20
    gates = term_heavy_circuit(n, 12, 5)
    want = oracle.run(gates, n)
    runs = [(0, B.SV_PREC_NATIVE), (6, B.SV_PREC_NATIVE)]
    if dtype == B.SV_C64:
        runs.append((6, B.SV_PREC_BF16X6))
    for pq, prec in runs:
        opts = B.make_opts(B.SV_PLAN_PASSES, 5, prec, pq)
        info = B.sv_pass_plan_info(n, dtype, gates, opts)
        assert info["gates"] == len(gates)
        if pq == 6:
            assert info["term_blocks"] >= 20
        say(f"term-heavy passes n={n} {DNAME[dtype]} pass qubits {pq or 8} precision {prec}: {info}")
        with State(n, dtype) as s:
            run_checked(s, gates, opts, want)


@pytest.mark.parametrize("dtype", DTYPES, ids=DNAME.get)
def test_pass_plan_non_unitary_diagonal_keeps_magnitudes(dtype):
    """Diagonal 2-qubit matrices whose entries are not all of modulus 1,
    mixed into the term-heavy circuit on a low and a high qubit: a pass may
    fold only unit-modulus diagonals in as per-tile phases, so these keep
    their magnitudes whatever the plan (the state's norm changes)."""
    n = 20
    rng = np.random.default_rng(17)
    gates = []
    for g in term_heavy_circuit(n, 6, 19):
        gates.append(g)
        if g.name == "p" and rng.random() < 0.3:
            q, o = g.controls[0], g.targets[0]
            d = np.diag(rng.uniform(0.7, 1.0, 4) * np.exp(1j * rng.uniform(0, 2 * math.pi, 4)))
            gates.append(Gate("matrix", (q, o), (), (), d))
    want = oracle.run(gates, n)
    assert abs(oracle.norm2(want) - 1.0) > 0.1
    for mode in (B.SV_PLAN_PASSES, B.SV_PLAN_GREEDY):
        say(f"non-unitary diagonals n={n} {DNAME[dtype]} mode={mode}")
        with State(n, dtype) as s:
            B.sv_apply_circuit(s.h, gates, B.make_opts(mode, 5))
            assert maxerr(s.host(), want) <= TOL[dtype]


@pytest.mark.parametrize("dtype", DTYPES, ids=DNAME.get)
@pytest.mark.parametrize("kmax", [2, 3, 5])
@pytest.mark.parametrize("n", [14, 20])
def test_pass_plan_small_blocks_match_oracle(dtype, kmax, n):
    """Pass blocks of at most kmax qubits (padded with identity to 16 x 16 on
    other tile slots).  The profile records count 126 algorithmic and 96
    matrix-core flops per amplitude per block."""
    gates = pass_circuit(n, 60 + n)
    want = oracle.run(gates, n)
    say(f"small-block passes n={n} {DNAME[dtype]} max_fused={kmax}")
    with State(n, dtype) as s:
        _, recs = run_checked(s, gates, B.make_opts(B.SV_PLAN_PASSES, kmax, B.SV_PREC_NATIVE, 8), want)
        recs = [r for r in recs if r["kind_name"] == "pass"]
    assert recs
    amps = 2.0 ** n
    for r in recs:
        blocks = r["flops"] / (126 * amps)
        assert blocks >= 1 and blocks == int(blocks) and r["mfma_flops"] == 96 * amps * blocks


@pytest.mark.parametrize("dtype", DTYPES, ids=DNAME.get)
@pytest.mark.parametrize("kind", ["layered", "controls", "phases"])
@pytest.mark.parametrize("n", [23, 24])
def test_pass_plan_large_states_match_oracle(dtype, kind, n):
    """States of 2^11 .. 2^13 pass tiles (more tiles than resident
    workgroups), with passes of three or more blocks, blocks with matrix
    variants and blocks with phase terms."""
    if kind == "layered":
        gates = W.layered_u3_pairing(n, 8, W.circuit_seed(2, n), "cx_or_cz")
    elif kind == "controls":
        gates = control_circuit(n, 70 + n)
    else:
        gates = phase_circuit(n, 80 + n, 3)
    want = oracle.run(gates, n)
    say(f"large-state passes n={n} {DNAME[dtype]} {kind}")
    with State(n, dtype) as s:
        _, recs = run_checked(s, gates, B.make_opts(B.SV_PLAN_PASSES), want, random_circuit=kind == "layered")
        recs = [r for r in recs if r["kind_name"] == "pass"]
    blocks = [round(r["flops"] / (126 * 2.0 ** n)) for r in recs]
    assert any(3 <= b <= 8 for b in blocks), blocks


@pytest.mark.parametrize("dtype", DTYPES, ids=DNAME.get)
@pytest.mark.parametrize("kind", ["mixed", "phases", "controls", "terms"])
@pytest.mark.parametrize("n", [14, 20])
def test_pass_plan_gate_order_search_matches_oracle(dtype, kind, n):
    """Passes split into blocks over random gate orders (pass_orders): a
    block's gates run in an order consistent with the circuit's
    dependencies, not in circuit order, with phase terms and matrix
    variants folded in the same way."""
    if kind == "mixed":
        gates = pass_circuit(n, 90 + n)
    elif kind == "phases":
        gates = phase_circuit(n, 91 + n, 4)
    elif kind == "controls":
        gates = control_circuit(n, 92 + n, 4)
    else:
        gates = term_heavy_circuit(n, 6, 93 + n)
    want = oracle.run(gates, n)
    for orders in (-1, 32):
        say(f"gate-order search n={n} {DNAME[dtype]} {kind} pass_orders={orders}")
        with State(n, dtype) as s:
            run_checked(s, gates, B.make_opts(B.SV_PLAN_PASSES, 5, B.SV_PREC_NATIVE, 8, orders), want)


@pytest.mark.parametrize("kind", ["mixed", "phases", "controls", "terms", "layered"])
@pytest.mark.parametrize("n", [13, 20, 23])
def test_pass_plan_bf16x6_matches_oracle(kind, n):
    """Complex64 passes with FP32-accurate split BF16 block products
    (SV_PREC_BF16X6): every kind of pass block (plain, matrix variants,
    per-tile phase terms), checked to the complex64 tolerance and the
    split form's rounding bound; the records show the split kernel ran."""
    if kind == "mixed":
        gates = pass_circuit(n, 110 + n)
    elif kind == "phases":
        gates = phase_circuit(n, 111 + n, 4)
    elif kind == "controls":
        gates = control_circuit(n, 112 + n, 4)
    elif kind == "terms":
        gates = term_heavy_circuit(n, 6, 113 + n)
    else:
        gates = W.layered_u3_pairing(n, 10, W.circuit_seed(2, n), "cx_or_cz")
    want = oracle.run(gates, n)
    say(f"bf16x6 passes n={n} {kind}")
    with State(n, B.SV_C64) as s:
        _, recs = run_checked(s, gates, B.make_opts(B.SV_PLAN_PASSES, 5, B.SV_PREC_BF16X6, 8), want,
                              random_circuit=kind == "layered")
    passes = [r for r in recs if r["kind_name"] == "pass"]
    assert passes and all(r["precision"] == B.SV_PREC_BF16X6 for r in passes)


def test_pass_plan_bf16x6_complex128_runs_native():
    n = 14
    gates = pass_circuit(n, 7)
    want = oracle.run(gates, n)
    with State(n, B.SV_C128) as s:
        _, recs = run_checked(s, gates, B.make_opts(B.SV_PLAN_PASSES, 5, B.SV_PREC_BF16X6, 8), want)
    assert all(r["precision"] == B.SV_PREC_NATIVE for r in recs)


@pytest.mark.parametrize("dtype", DTYPES, ids=DNAME.get)
def test_pass_plan_phase_gates_after_relayout(dtype):
    n = 18
    a = phase_circuit(n, 3, 2)
    b = phase_circuit(n, 4, 4) + W.qpe_circuit(8, 77)
    want = oracle.run(list(a) + list(b), n)
    with State(n, dtype) as s:
        B.sv_apply_circuit(s.h, a, B.make_opts(B.SV_PLAN_PASSES))
        B.sv_swap_bits(s.h, 0, n - 6, 6)
        B.sv_swap_bits(s.h, 3, 9, 2)
        say(f"phase passes after relayout {DNAME[dtype]} map={B.sv_qubit_map(s.h, n)}")
        B.sv_apply_circuit(s.h, b, B.make_opts(B.SV_PLAN_PASSES))
        assert maxerr(s.host(), want) <= TOL[dtype]


@pytest.mark.parametrize("dtype", DTYPES, ids=DNAME.get)
def test_pass_plan_qpe_exact_phase(dtype):
    k, m = 15, 0x5A5A & ((1 << 15) - 1)
    n = k + 1
    with State(n, dtype) as s:
        st = B.sv_apply_circuit(s.h, W.qpe_circuit(k, m), B.make_opts(B.SV_PLAN_PASSES))
        say(f"qpe passes n={n} {DNAME[dtype]}: {st['sweeps']} sweeps")
        out = B.sv_sample(s.h, W.uniforms(5, 1000))
        assert np.all(out == (m | (1 << k)))
        a = s.host()
        assert abs(abs(a[m | (1 << k)]) - 1.0) <= TOL[dtype] * 10


def with_new_angles(gates, seed):
    """The same gates on the same qubits with fresh rotation angles."""
    rng = np.random.default_rng(seed)
    out = []
    for g in gates:
        if g.name in ("u3", "rx", "ry", "rz", "p"):
            g = Gate(g.name, g.targets, g.controls, tuple(float(x) for x in rng.uniform(0, 2 * math.pi, len(g.params))))
        out.append(g)
    return out


@pytest.mark.parametrize("dtype", DTYPES, ids=DNAME.get)
def test_pass_plan_kept_per_structure(dtype):
    """A circuit of the same structure with new angles reuses the plan kept on
    the handle (new block matrices, same grouping); a relayout or other
    options make a new plan.  Every result against the oracle."""
    n = 18
    a = phase_circuit(n, 5, 3) + control_circuit(n, 6, 2)
    b = with_new_angles(a, 7)
    with State(n, dtype) as s:
        for gates, opts in ((a, B.make_opts(B.SV_PLAN_PASSES)), (b, B.make_opts(B.SV_PLAN_PASSES)),
                            (a, B.make_opts(B.SV_PLAN_PASSES, 5, B.SV_PREC_NATIVE, 6))):
            B.sv_reset(s.h)
            run_checked(s, gates, opts, oracle.run(gates, n))
        B.sv_reset(s.h)
        B.sv_swap_bits(s.h, 0, n - 6, 6)
        run_checked(s, b, B.make_opts(B.SV_PLAN_PASSES), oracle.run(b, n))


@pytest.mark.parametrize("dtype", DTYPES, ids=DNAME.get)
def test_pass_plan_forced_tile_width(dtype):
    """pass_tile: every kernel pass on the smallest tile or on twice it
    (the wide form: 512 threads); the records show the width used."""
    n = 20
    gates = pass_circuit(n, 21)
    want = oracle.run(gates, n)
    T0 = 12 if dtype == B.SV_C64 else 11
    for tile in (T0, T0 + 1):
        with State(n, dtype) as s:
            _, recs = run_checked(s, gates, B.make_opts(B.SV_PLAN_PASSES, 5, B.SV_PREC_NATIVE, 8, 0, tile), want)
        tiles = {r["tile_log"] for r in recs if r["kind_name"] == "pass"}
        say(f"  pass_tile {tile}: tiles used {tiles}")
        assert tiles and tiles <= {tile, T0} and tile in tiles
    with State(n, dtype) as s:
        for bad in (T0 - 1, T0 + 2):
            with pytest.raises(B.SvError):
                B.sv_apply_circuit(s.h, gates, B.make_opts(B.SV_PLAN_PASSES, 5, B.SV_PREC_NATIVE, 8, 0, bad))
        with pytest.raises(B.SvError):
            B.sv_apply_circuit(s.h, gates, B.make_opts(B.SV_PLAN_GREEDY, 5, B.SV_PREC_NATIVE, 0, 0, T0))
        if dtype == B.SV_C64:
            with pytest.raises(B.SvError):
                B.sv_apply_circuit(s.h, gates, B.make_opts(B.SV_PLAN_PASSES, 5, B.SV_PREC_BF16X6, 8, 0, T0 + 1))


def test_pass_plan_rejects_bad_options():
    with State(12, B.SV_C64) as s:
        for opts in (B.make_opts(B.SV_PLAN_PASSES, 5, B.SV_PREC_NATIVE, 3),
                     B.make_opts(B.SV_PLAN_PASSES, 5, B.SV_PREC_NATIVE, 9),
                     B.make_opts(B.SV_PLAN_GREEDY, 5, B.SV_PREC_NATIVE, 8)):
            with pytest.raises(B.SvError):
                B.sv_apply_circuit(s.h, [Gate("h", (0,))], opts)
    with pytest.raises(B.SvError):
        B.sv_plan_create(12, B.SV_C64, [Gate("h", (0,))], B.make_opts(B.SV_PLAN_PASSES))
