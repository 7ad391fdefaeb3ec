"""sv_readout: the marginal, Pauli expectation values and shots of one state in
one call (paper Sec. 2.1, "Measurement and Sampling"), through the C ABI.

Where every string is a Z string and the marginal's physical bits allow it, the
three share one read of the state (one fused sweep); otherwise they run one
after another.  Both routes are checked against the separate calls (FP64
sums in another grouping: 1e-13) and against the FP64 reference on the very
state the GPU holds (copied back): probabilities and expectation values to
1e-12, shots by index agreement within a CDF window of 1e-12 (the CDF runs
in physical index order, as in sv_sample).
"""
import numpy as np
import pytest

import oracle
import workloads as W

from paper_2511_14664_amd import _binding as B

pytestmark = pytest.mark.gpu

DTYPES = [B.SV_C128, B.SV_C64]
DNAME = {B.SV_C128: "c128", B.SV_C64: "c64"}


def say(*a):
    print(*a, flush=True)


def logical_of_physical(qmap, n):
    """Logical index held at each physical index (qmap[q]: physical bit of qubit q)."""
    idx = np.arange(1 << n, dtype=np.int64)
    out = np.zeros(1 << n, dtype=np.int64)
    for q in range(n):
        out |= ((idx >> int(qmap[q])) & 1) << q
    return out


def sample_bad(state, u, got, tau, log_of_phys):
    """Shots walk the CDF in physical index order (sv_sample): the reference
    samples the state in that order and maps the outcomes back."""
    phys_state = state[log_of_phys]
    phys_of_log = np.empty_like(log_of_phys)
    phys_of_log[log_of_phys] = np.arange(log_of_phys.size)
    p = np.abs(phys_state) ** 2
    cdf = np.cumsum(p)
    want = oracle.sample(phys_state, u)
    bad = []
    for s in range(len(u)):
        g = int(phys_of_log[int(got[s])])
        if g == want[s]:
            continue
        t = u[s] * cdf[-1]
        lo = cdf[g - 1] if g > 0 else 0.0
        if not (lo - tau <= t < cdf[g] + tau and p[g] > 0):
            bad.append((s, g, int(want[s])))
    return bad


def z_terms(n, count, seed):
    """count Z strings: single Z, neighbour pairs and random masks over all qubits."""
    rng = np.random.default_rng(seed)
    terms = W.hea_z_terms(n)[: min(count, 2 * n - 1)]
    while len(terms) < count:
        mask = rng.integers(0, 2, n)
        terms.append("".join("Z" if b else "I" for b in mask))
    return terms


def check(h, n, dtype, qubits, terms, u):
    host = B.sv_copy_to_host(h, n, dtype).astype(np.complex128)  # logical order
    probs, ex, shots = B.sv_readout(h, qubits, terms, u)
    # the separate calls on the same state
    if qubits is not None:
        want_p = B.sv_probabilities(h, qubits)
        assert probs.shape == want_p.shape
        assert np.max(np.abs(probs - want_p)) <= 1e-13
        ref_p = oracle.probabilities(host, qubits)
        assert np.max(np.abs(probs - ref_p)) <= 1e-12
    else:
        assert probs is None
    if terms:
        sep = B.sv_expect_pauli(h, terms)
        ref = np.array([oracle.expect_pauli(host, t).real for t in terms])
        err = np.max(np.abs(ex - ref))
        assert err <= 1e-12, err
        assert np.max(np.abs(ex - sep)) <= 1e-12
    else:
        assert ex.size == 0
    if u is not None and len(u):
        lop = logical_of_physical(B.sv_qubit_map(h, n), n)
        bad = sample_bad(host, np.asarray(u), shots, 1e-12, lop)
        sep_shots = B.sv_sample(h, np.asarray(u))
        assert np.mean(sep_shots == shots) >= 0.99
        assert not bad, bad[:5]
    else:
        assert shots.size == 0
    return probs, ex, shots


@pytest.mark.parametrize("dtype", DTYPES, ids=DNAME.get)
@pytest.mark.parametrize("n", [14, 17, 20])
def test_readout_fused_matches_separate_calls_and_oracle(dtype, n):
    psi = W.random_state(n, 31 + n)
    h = B.sv_create(n, dtype)
    try:
        B.sv_copy_from_host(h, dtype, psi)
        u = W.uniforms(5 + n, 1000)
        terms = z_terms(n, 32, n)
        # bins among bits 0..7 (both dtypes' register-summed fold) and bits >= 12
        qubits = [0, 3, 5, n - 1, n - 2]
        say(f"n={n} {DNAME[dtype]} fused marginal {qubits}, {len(terms)} Z strings, 1000 shots")
        check(h, n, dtype, qubits, terms, u)
        # parts on their own: no marginal; marginal only; shots only
        check(h, n, dtype, None, terms, u)
        check(h, n, dtype, [n - 1, 1], [], None)
        check(h, n, dtype, None, [], u)
    finally:
        B.sv_destroy(h)


@pytest.mark.parametrize("dtype", DTYPES, ids=DNAME.get)
def test_readout_after_exchange_headline_shape(dtype):
    """The benchmark's read-outs (marginal of the top qubits, 32 Z strings,
    1000 shots) after a 6-bit exchange, which puts six marginal qubits on
    physical bits 0..5 and leaves the others at bits >= 12."""
    n = 20
    psi = W.random_state(n, 77)
    h = B.sv_create(n, dtype)
    try:
        B.sv_copy_from_host(h, dtype, psi)
        B.sv_swap_bits(h, 0, n - 6, 6)
        u = W.uniforms(7, 1000)
        terms = W.hea_z_terms(n)[:32]
        qubits = list(range(n - 8, n))
        say(f"n={n} {DNAME[dtype]} after exchange: marginal {qubits}")
        check(h, n, dtype, qubits, terms, u)
    finally:
        B.sv_destroy(h)


@pytest.mark.parametrize("dtype", DTYPES, ids=DNAME.get)
@pytest.mark.parametrize("case", ["xy_term", "bin_bit_10", "small_state", "norm_only", "many_terms"])
def test_readout_fallback_routes(dtype, case):
    n = 12 if case == "small_state" else 16
    psi = W.random_state(n, 90 + n)
    h = B.sv_create(n, dtype)
    try:
        B.sv_copy_from_host(h, dtype, psi)
        u = W.uniforms(11, 500)
        qubits, terms = [1, n - 1], z_terms(n, 8, 3)
        if case == "xy_term":
            terms = terms + ["X" + "Z" * (n - 2) + "Y"]
        elif case == "bin_bit_10":
            qubits = [10, 2]
        elif case == "norm_only":
            qubits = []
        elif case == "many_terms":
            terms = z_terms(n, 40, 4)
        say(f"n={n} {DNAME[dtype]} fallback case {case}")
        check(h, n, dtype, qubits, terms, u)
    finally:
        B.sv_destroy(h)


def test_readout_rejects_bad_arguments():
    n = 14
    h = B.sv_create(n, B.SV_C64)
    try:
        for args in ((["Z" * (n - 1)], None), (["Q" * n], None)):
            with pytest.raises(B.SvError):
                B.sv_readout(h, [0], args[0], args[1])
        with pytest.raises(B.SvError):
            B.sv_readout(h, [0, 0], ["Z" * n], None)
        with pytest.raises(B.SvError):
            B.sv_readout(h, [0], ["Z" * n], [1.0])
        p, e, s = B.sv_readout(h, None, [], None)
        assert p is None and e.size == 0 and s.size == 0
    finally:
        B.sv_destroy(h)
