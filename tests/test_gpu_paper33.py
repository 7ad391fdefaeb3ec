"""The paper's single-GPU workloads (Sec. 2.2), synthesised: random circuit
sampling (30n gates), textbook phase estimation and Trotterised
transverse-field Ising evolution at 33 qubits complex64 (64 GiB), the size the
paper runs on one GPU.

No host here holds a 33-qubit FP64 reference, so the full-size cases are
checked through results fixed by the mathematics: phase estimation of an
exactly representable phase returns the phase register value on every shot, a
random circuit or an Ising evolution followed by its adjoint returns to
|0...0>, and without a transverse field the Ising evolution only multiplies
|0...0> by exp(i J dt E steps).  Reduced twins of the generators are compared
with the FP64 reference amplitude by amplitude under every plan.
"""
import numpy as np
import pytest

import oracle
import workloads as W

from paper_2511_14664_amd import _binding as B

from error_bounds import check_state, mirror_l2, state_bounds

pytestmark = pytest.mark.gpu

TOL = {B.SV_C128: 1e-12, B.SV_C64: 2e-5}
PLANS = {"plain": B.make_opts(B.SV_PLAN_PLAIN), "greedy": B.make_opts(B.SV_PLAN_GREEDY, 5),
         "passes": B.make_opts(B.SV_PLAN_PASSES, 5, B.SV_PREC_NATIVE, 8)}


def say(*a):
    print(*a, flush=True)


def mirror(h, n, gates):
    """Run a circuit and its adjoint as LDS passes; the state returns to
    |0...0> up to rounding: ||psi - |0>||_2 within the deterministic rounding
    bound of the recorded sweeps.  Returns (||psi - |0>||_2, bound)."""
    B.sv_profile_enable(h, True)
    B.sv_apply_circuit(h, gates, PLANS["passes"])
    B.sv_apply_circuit(h, W.inverse(gates), PLANS["passes"])
    recs = B.sv_profile_read(h, 1 << 14)
    B.sv_profile_enable(h, False)
    a0 = complex(B.sv_copy_to_host(h, n, B.SV_C64, 0, 1)[0])
    l2, res = mirror_l2(B.sv_probabilities(h, [])[0], a0, n)
    det, prob = state_bounds(recs, n, True)
    say(f"  ||psi - |0>||_2 {l2:.2e} (bounds: deterministic {det:.2e}, probabilistic {prob:.2e}; resolution {res:.1e})")
    assert l2 <= det + res
    return l2, det


@pytest.mark.parametrize("plan", ["plain", "greedy", "passes"])
@pytest.mark.parametrize("dtype", [B.SV_C128, B.SV_C64], ids=["c128", "c64"])
def test_rcs_twin_20q_matches_reference(dtype, plan):
    n = 20
    gates = W.rcs_circuit(n, W.circuit_seed(6, 2))
    want = oracle.run(gates, n)
    say(f"rcs twin n={n} plan={plan}")
    h = B.sv_create(n, dtype)
    try:
        B.sv_profile_enable(h, True)
        st = B.sv_apply_circuit(h, gates, PLANS[plan])
        recs = B.sv_profile_read(h, 1 << 14)
        mx, l2, bound = check_state(B.sv_copy_to_host(h, n, dtype), want, dtype == B.SV_C64, n, recs, gates)
        say(f"  max|d amp| {mx:.2e}, ||d psi||_2 {l2:.2e} (bound {bound:.2e})")
        assert st["gates"] == len(gates) == 30 * n
    finally:
        B.sv_destroy(h)


@pytest.mark.parametrize("plan", ["greedy", "passes"])
def test_qpe_33q_every_shot_is_the_phase(plan):
    import torch

    n = 33
    k = n - 1
    m = 0x5A5A5A5A5A5A5A5A & ((1 << k) - 1)
    torch.cuda.empty_cache()
    say(f"qpe n={n} plan={plan}")
    h = B.sv_create(n, B.SV_C64)
    try:
        B.sv_apply_circuit(h, W.qpe_circuit(k, m), PLANS[plan])
        shots = B.sv_sample(h, W.uniforms(11, 1000))
        assert np.all(shots == (m | (1 << k)))
        p = B.sv_probabilities(h, [k - 3, k - 2, k - 1, k])
        want = np.zeros(16)
        want[((m >> (k - 3)) & 7) | 8] = 1.0
        assert float(np.max(np.abs(p - want))) <= 1e-5
    finally:
        B.sv_destroy(h)


def test_rcs_33q_mirror_returns_to_zero():
    import torch

    n = 33
    gates = W.rcs_circuit(n, W.circuit_seed(6, 1))
    torch.cuda.empty_cache()
    say(f"rcs mirror n={n}")
    h = B.sv_create(n, B.SV_C64)
    try:
        l2, det = mirror(h, n, gates)
        p = B.sv_probabilities(h, [n - 1])
        assert abs(p[0] - 1.0) <= 2 * det and abs(p.sum() - 1.0) <= 2 * det
    finally:
        B.sv_destroy(h)


@pytest.mark.parametrize("zz", ["cx", "diag"])
@pytest.mark.parametrize("plan", ["plain", "greedy", "passes"])
@pytest.mark.parametrize("dtype", [B.SV_C128, B.SV_C64], ids=["c128", "c64"])
def test_tfim_twin_18q_matches_reference(dtype, plan, zz):
    rows, cols = 3, 6
    n = rows * cols
    gates = W.tfim_trotter(rows, cols, 4, 0.1, 1.0, 1.0, zz)
    want = oracle.run(gates, n)
    say(f"tfim twin n={n} plan={plan} zz={zz}")
    h = B.sv_create(n, dtype)
    try:
        B.sv_profile_enable(h, True)
        B.sv_apply_circuit(h, gates, PLANS[plan])
        recs = B.sv_profile_read(h, 1 << 14)
        mx, l2, bound = check_state(B.sv_copy_to_host(h, n, dtype), want, dtype == B.SV_C64, n, recs, gates)
        say(f"  max|d amp| {mx:.2e}, ||d psi||_2 {l2:.2e} (bound {bound:.2e})")
    finally:
        B.sv_destroy(h)


@pytest.mark.parametrize("zz", ["cx", "diag"])
def test_tfim_33q_without_field_is_a_phase(zz):
    import torch

    rows, cols, steps, dt, J = 3, 11, 10, 0.1, 1.0
    n = rows * cols
    E = len(W.triangular_lattice_edges(rows, cols))
    torch.cuda.empty_cache()
    say(f"tfim h=0 n={n} zz={zz}")
    h = B.sv_create(n, B.SV_C64)
    try:
        B.sv_apply_circuit(h, W.tfim_trotter(rows, cols, steps, dt, J, 0.0, zz), PLANS["passes"])
        a = B.sv_copy_to_host(h, n, B.SV_C64, 0, 1 << 12)
        assert abs(a[0] - np.exp(1j * J * dt * E * steps)) <= 2e-5
        assert float(np.max(np.abs(a[1:]))) <= 2e-5
        p = B.sv_probabilities(h, [n - 2, n - 1])
        assert abs(p[0] - 1.0) <= 1e-5
    finally:
        B.sv_destroy(h)


def test_tfim_33q_mirror_returns_to_zero():
    import torch

    rows, cols = 3, 11
    n = rows * cols
    gates = W.tfim_trotter(rows, cols, 10, 0.1, 1.0, 1.0, "cx")
    torch.cuda.empty_cache()
    say(f"tfim mirror n={n}")
    h = B.sv_create(n, B.SV_C64)
    try:
        mirror(h, n, gates)
    finally:
        B.sv_destroy(h)
