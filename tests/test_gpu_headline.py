"""The 28-qubit benchmark circuit itself, compared element by element with
the FP64 oracle at full size.

The circuit is the benchmark's: 20 layers of U3 on every qubit then CNOT or CZ
(fair coin) on a random perfect matching, 840 gates, seed 2001.  The oracle
runs it once (FP64, unfused, ~4 GiB of host memory) and its state serves every
case.  For complex128 and complex64 and the plain, greedy (<= 5-qubit blocks)
and LDS-pass plans (complex64 passes also with split BF16 block products),
all 2^28 amplitudes copied back from the GPU are compared:

* max |d amp| <= 1e-12 (complex128) / 2e-5 (complex64);
* ||d psi||_2 within the rounding bounds of ``tests/error_bounds.py``
  computed from the sweeps the library recorded and the oracle's own gates (deterministic, and the probabilistic
  bound with lambda = 6), and the largest relative error over amplitudes of
  modulus >= 2^-15 within the probabilistic per-amplitude bound;
* under the pass plan, the benchmark's read-outs on the GPU's own state: 1000
  shots index-exact against the oracle's sampler (outcomes may differ only
  where u * norm sits within 1e-12 of a CDF step: the GPU sums in another
  order), the same shots from the library's seeded stream, the 10-qubit
  marginal, Z-string expectations, and the 6-bit exchange, which must leave
  the logical amplitudes bit-identical.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W

from paper_2511_14664_amd import _binding as B

from error_bounds import amplitude_bound, oracle_bounds, state_bounds

pytestmark = pytest.mark.gpu

N = 28
TOL = {B.SV_C128: 1e-12, B.SV_C64: 2e-5}
DNAME = {B.SV_C128: "c128", B.SV_C64: "c64"}
MODES = {"passes": (B.SV_PLAN_PASSES, B.SV_PREC_NATIVE), "passes_bf16x6": (B.SV_PLAN_PASSES, B.SV_PREC_BF16X6),
         "greedy": (B.SV_PLAN_GREEDY, B.SV_PREC_NATIVE), "plain": (B.SV_PLAN_PLAIN, B.SV_PREC_NATIVE)}
CHUNK = 1 << 24


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def headline():
    gates = W.layered_u3_pairing(N, 20, W.circuit_seed(2, 1), "cx_or_cz")
    assert len(gates) == 840
    say(f"oracle: 28-qubit benchmark circuit, {len(gates)} gates, {oracle.num_threads()} threads ...")
    want = oracle.run(gates, N)
    say("oracle: done")
    return gates, want


def state_errors(got, want):
    """max |d a|, ||d psi||_2 and the largest |d a| / |a| over |a| >= 2^-15,
    accumulated in chunks (FP64)."""
    mx, l2, rel = 0.0, 0.0, 0.0
    big = 2.0 ** -15
    for i in range(0, want.size, CHUNK):
        g = got[i:i + CHUNK].astype(np.complex128)
        w = want[i:i + CHUNK]
        d = np.abs(g - w)
        mx = max(mx, float(d.max()))
        l2 += float(np.dot(d, d))
        aw = np.abs(w)
        sel = aw >= big
        if np.any(sel):
            rel = max(rel, float(np.max(d[sel] / aw[sel])))
    return mx, math.sqrt(l2), rel


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


def splitmix_uniforms(seed, count):
    """The library's documented shot stream, written out here from the
    SplitMix64 definition (Steele, Lea, Flood 2014)."""
    m = (1 << 64) - 1
    out = np.empty(count)
    for s in range(count):
        z = (seed + (s + 1) * 0x9E3779B97F4A7C15) & m
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & m
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & m
        z ^= z >> 31
        out[s] = (z >> 11) * 2.0 ** -53
    return out


CASES = [(B.SV_C128, "passes"), (B.SV_C128, "greedy"), (B.SV_C128, "plain"),
         (B.SV_C64, "passes"), (B.SV_C64, "passes_bf16x6"), (B.SV_C64, "greedy"), (B.SV_C64, "plain")]


@pytest.mark.parametrize("dtype,mode", CASES, ids=[f"{DNAME[d]}-{m}" for d, m in CASES])
def test_headline_circuit_full_state(headline, dtype, mode):
    gates, want = headline
    say(f"28q headline {DNAME[dtype]} mode={mode}: run")
    h = B.sv_create(N, dtype)
    try:
        B.sv_profile_enable(h, True)
        plan, prec = MODES[mode]
        st = B.sv_apply_circuit(h, gates, B.make_opts(plan, 5, prec))
        recs = B.sv_profile_read(h, 1 << 12)
        B.sv_profile_enable(h, False)
        assert st["gates"] == 840 and len(recs) == st["sweeps"]
        got = B.sv_copy_to_host(h, N, dtype)
        mx, l2, rel = state_errors(got, want)
        msg = f"28q headline {DNAME[dtype]} {mode}: {st['sweeps']} sweeps, max|d amp| {mx:.3e}, " \
              f"||d psi||_2 {l2:.3e}, max rel (|a| >= 2^-15) {rel:.3e}"
        det, prob = state_bounds(recs, N, dtype == B.SV_C64)
        odet, oprob = oracle_bounds(gates)
        det, prob = det + odet, math.hypot(prob, oprob)
        rel_bound = amplitude_bound(prob, N) / 2.0 ** -15
        msg += f"; bounds: ||d psi|| det {det:.3e} prob {prob:.3e}, rel {rel_bound:.3e}"
        say(msg)
        assert mx <= TOL[dtype]
        assert l2 <= prob <= det
        assert rel <= rel_bound
        if not mode.startswith("passes"):
            return
        check_readouts(h, dtype, got)
    finally:
        B.sv_destroy(h)


def check_readouts(h, dtype, got):
    """The benchmark step's read-outs and exchange on the state the GPU holds."""
    ref = np.asarray(got, dtype=np.complex128)
    u = W.uniforms(7, 1000)
    shots = B.sv_sample(h, u)
    bad = sample_ok(ref, u, shots, 1e-12)
    say(f"  shots: {len(u) - len(bad)} of {len(u)} index-exact")
    assert not bad, bad[:5]
    us = splitmix_uniforms(7, 1000)
    seeded = B.sv_sample_seeded(h, 1000, 7)
    assert np.array_equal(seeded, B.sv_sample(h, us))
    assert not sample_ok(ref, us, seeded, 1e-12)
    q = list(range(N - 10, N))
    p = B.sv_probabilities(h, q)
    assert np.max(np.abs(p - oracle.probabilities(ref, q))) <= 1e-12
    zs = W.hea_z_terms(N)
    terms = [zs[0], zs[13], zs[27], zs[N + 0], zs[N + 13], zs[N + 26]]
    e = B.sv_expect_pauli(h, terms)
    ew = np.array([oracle.expect_pauli(ref, t).real for t in terms])
    assert np.max(np.abs(e - ew)) <= 1e-12
    B.sv_swap_bits(h, 0, N - 6, 6)
    after = B.sv_copy_to_host(h, N, dtype)
    assert np.array_equal(after.view(np.uint8), got.view(np.uint8))
    say("  read-outs and exchange agree")


def test_headline_split_products_are_fp32_accurate(headline):
    """The split-BF16 pass path is at least as accurate as complex64 applied
    one gate at a time in FP32 on the vector units: its ||d psi||_2 and its
    largest relative error do not exceed the plain path's."""
    gates, want = headline
    err = {}
    for mode in ("plain", "passes_bf16x6"):
        plan, prec = MODES[mode]
        h = B.sv_create(N, B.SV_C64)
        try:
            B.sv_apply_circuit(h, gates, B.make_opts(plan, 5, prec))
            err[mode] = state_errors(B.sv_copy_to_host(h, N, B.SV_C64), want)
        finally:
            B.sv_destroy(h)
    say(f"c64 plain: ||d psi||_2 {err['plain'][1]:.3e}, rel {err['plain'][2]:.3e}; "
        f"split passes: ||d psi||_2 {err['passes_bf16x6'][1]:.3e}, rel {err['passes_bf16x6'][2]:.3e}")
    assert err["passes_bf16x6"][1] <= err["plain"][1]
    assert err["passes_bf16x6"][2] <= err["plain"][2]
