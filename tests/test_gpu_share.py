"""One GPU's share of a distributed state at full size: 34 qubits complex128
and 35 qubits complex64 (256 GiB each), with the in-place exchange of the top 6
index bits with the lowest 6 every 2 layers.

No host holds a 256 GiB FP64 reference, so the full-size cases are checked
through properties that hold at any size (mirror circuit back to |0...0>,
norm, marginals of a basis state, the exchange applied twice is the identity
bit for bit), and a reduced twin of the same generator at 20 qubits is compared
with the FP64 reference amplitude by amplitude.
"""
import numpy as np
import pytest

import oracle
import workloads as W

from paper_2511_14664_amd import _binding as B

from error_bounds import check_state, mirror_l2, state_bounds

pytestmark = pytest.mark.gpu

TOL = {B.SV_C128: 1e-12, B.SV_C64: 2e-5}


def say(*a):
    print(*a, flush=True)


def run_ops(h, ops, mode=B.SV_PLAN_GREEDY, kmax=5):
    seg = []
    for op in list(ops) + [None]:
        if op is None or isinstance(op, W.BitSwap):
            if seg:
                B.sv_apply_circuit(h, seg, B.make_opts(mode, kmax))
                seg = []
            if op is not None:
                B.sv_swap_bits(h, op.lo, op.hi, op.width)
        else:
            seg.append(op)


@pytest.mark.parametrize("mode", [B.SV_PLAN_GREEDY, B.SV_PLAN_PASSES], ids=["greedy", "passes"])
@pytest.mark.parametrize("dtype", [B.SV_C128, B.SV_C64], ids=["c128", "c64"])
def test_share_twin_20q_matches_reference(dtype, mode):
    n = 20
    ops = W.share_layers(n, 10, W.circuit_seed(3, 1))
    want = oracle.run(ops, n)
    h = B.sv_create(n, dtype)
    try:
        B.sv_profile_enable(h, True)
        run_ops(h, ops, mode)
        recs = B.sv_profile_read(h, 1 << 14)
        got = B.sv_copy_to_host(h, n, dtype)
        mx, l2, bound = check_state(got, want, dtype == B.SV_C64, n, recs, ops)
        say(f"share twin {n}q: max|d amp| {mx:.2e}, ||d psi||_2 {l2:.2e} (bound {bound:.2e})")
        assert B.sv_qubit_map(h, n) != list(range(n))  # 5 exchanges: odd, so relaid out
    finally:
        B.sv_destroy(h)


@pytest.mark.parametrize("n,dtype", [(34, B.SV_C128), (35, B.SV_C64)], ids=["34q-c128", "35q-c64"])
def test_full_share_256gib(n, dtype):
    import torch

    torch.cuda.empty_cache()
    need = B.sv_state_bytes(n, dtype)
    free, total = torch.cuda.mem_get_info()
    say(f"{n}q share: need {need / 2**30:.0f} GiB, free {free / 2**30:.1f} of {total / 2**30:.1f} GiB")
    assert need == 256 * 2 ** 30
    if free < need + (2 << 30):
        pytest.skip(f"device has {free / 2**30:.1f} GiB free, the {n}-qubit share needs 258 GiB")
    h = B.sv_create(n, dtype)
    try:
        # exchange applied twice is the identity, bit for bit (windows at both ends)
        B.sv_apply_circuit(h, [W.Gate("h", (q,)) for q in (0, 3, 7, n - 1, n - 3)] +
                           [W.Gate("u3", (q,), (), (0.3 * q + 0.1, 0.2, -0.7)) for q in (1, 5, n - 2)],
                           B.make_opts(B.SV_PLAN_PLAIN))
        w = 1 << 20
        lo0 = B.sv_copy_to_host(h, n, dtype, 0, w)
        hi0 = B.sv_copy_to_host(h, n, dtype, (1 << n) - w, w)
        B.sv_swap_bits(h, 0, n - 6, 6)
        B.sv_swap_bits(h, 0, n - 6, 6)
        assert B.sv_qubit_map(h, n) == list(range(n))
        assert np.array_equal(B.sv_copy_to_host(h, n, dtype, 0, w).view(np.uint8), lo0.view(np.uint8))
        assert np.array_equal(B.sv_copy_to_host(h, n, dtype, (1 << n) - w, w).view(np.uint8), hi0.view(np.uint8))

        # two layers of the share workload (one exchange) and their mirror, as
        # greedy sweeps and as LDS passes (2^23 pass tiles: a 2-D grid)
        ops = W.share_layers(n, 2, W.circuit_seed(3, 1))
        for mode in (B.SV_PLAN_GREEDY, B.SV_PLAN_PASSES):
            B.sv_reset(h)
            say(f"{n}q: {W.gate_count(ops)} gates + exchanges, then the mirror (plan mode {mode})")
            B.sv_profile_read(h)
            B.sv_profile_enable(h, True)
            run_ops(h, ops, mode)
            norm = B.sv_probabilities(h, [])[0]
            assert abs(norm - 1) <= (1e-12 if dtype == B.SV_C128 else 1e-5)
            run_ops(h, W.inverse(ops), mode)
            recs = B.sv_profile_read(h, 1 << 14)
            B.sv_profile_enable(h, False)
            assert B.sv_qubit_map(h, n) == list(range(n))
            a0 = complex(B.sv_copy_to_host(h, n, dtype, 0, 1)[0])
            # the mirror returns to |0...0> up to rounding: ||psi - |0>||_2
            # within the rounding bound of the recorded sweeps
            l2, res = mirror_l2(B.sv_probabilities(h, [])[0], a0, n)
            det, prob = state_bounds(recs, n, dtype == B.SV_C64)
            say(f"  ||psi - |0>||_2 {l2:.2e} (bounds: deterministic {det:.2e}, probabilistic {prob:.2e}; resolution {res:.1e})")
            assert l2 <= det + res
            p = B.sv_probabilities(h, [0, n - 1, n // 2])
            assert abs(p[0] - 1) <= 2 * det and np.all(p[1:] <= (det + res) ** 2)
            s = B.sv_sample(h, W.uniforms(7, 1000))
            assert np.all(s == 0)
    finally:
        B.sv_destroy(h)
        torch.cuda.empty_cache()
