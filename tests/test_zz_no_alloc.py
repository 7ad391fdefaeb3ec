"""The allocation-free expectation entry point (sv_expect_pauli_noalloc),
through the C ABI, against sv_expect_pauli on the same state: two calls in a
row, the second on a smaller state with fewer strings, then the size limit.
Both entry points run the same kernels in the same order, so the results
must agree to the complex128 tolerance (in practice bit for bit)."""
import numpy as np
import pytest

import oracle
import workloads as W

from paper_2511_14664_amd import _binding as B

pytestmark = pytest.mark.gpu


def pauli_terms(n, count, seed):
    """Z-only strings (more than one launch batch of them) and general X/Y/Z
    strings, from a seeded generator."""
    rng = np.random.default_rng(seed)
    out = W.hea_z_terms(n)[:count // 2]
    while len(out) < count:
        out.append("".join(rng.choice(list("IXYZ"), n)))
    return out


@pytest.mark.parametrize("first,second", [((16, B.SV_C128, 200), (10, B.SV_C64, 5)),
                                          ((14, B.SV_C64, 256), (9, B.SV_C128, 40))])
def test_noalloc_expectations_match_the_allocating_entry_point(first, second):
    for n, dtype, count in (first, second):
        gates = W.layered_u3_pairing(n, 6, W.circuit_seed(1, n), "cx_or_cz")
        terms = pauli_terms(n, count, n)
        h = B.sv_create(n, dtype)
        try:
            B.sv_apply_circuit(h, gates, B.make_opts(B.SV_PLAN_GREEDY, 4))
            want = B.sv_expect_pauli(h, terms)
            got = B.sv_expect_pauli_noalloc(h, terms)
            print(f"n={n} dtype={dtype} terms={count}: max diff {float(np.max(np.abs(got - want))):.2e}, "
                  f"bit-identical {np.array_equal(got, want)}", flush=True)
            assert float(np.max(np.abs(got - want))) <= 1e-12
            # and both agree with the FP64 oracle on the state the GPU holds
            psi = B.sv_copy_to_host(h, n, dtype).astype(np.complex128)
            ref = np.array([oracle.expect_pauli(psi, t).real for t in terms[:12]])
            assert float(np.max(np.abs(got[:12] - ref))) <= 1e-12
        finally:
            B.sv_destroy(h)


def test_noalloc_rejects_more_terms_than_its_scratch_holds():
    n = 8
    h = B.sv_create(n, B.SV_C64)
    try:
        with pytest.raises(B.SvError) as e:
            B.sv_expect_pauli_noalloc(h, ["Z" * n] * (B.SV_NOALLOC_MAX_TERMS + 1))
        assert e.value.code == B.SV_EINVAL
        assert B.sv_expect_pauli_noalloc(h, []).size == 0
        assert abs(B.sv_expect_pauli_noalloc(h, ["Z" * n])[0] - 1.0) <= 1e-6
    finally:
        B.sv_destroy(h)
