"""Host-only checks of the C ABI (no GPU needed): the library loads and exports
every entry point the header declares, arguments are validated on the host,
and the planner's fused blocks reproduce the unfused circuit (checked with the
FP64 reference)."""
import ctypes
import json
import os
import re

import numpy as np
import pytest

import oracle
import workloads as W
from workloads import Gate

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sv.h")

sv = pytest.importorskip("paper_2511_14664_amd", reason="libsv.so not built")
from paper_2511_14664_amd import _binding as B  # noqa: E402


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sv_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    lib = ctypes.CDLL(B.LIB_PATH)
    syms = declared_symbols()
    assert len(syms) >= 20
    for s in syms:
        assert hasattr(lib, s), s


def test_state_bytes_matches_paper_memory_formula():
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_figures.json")))
    ex = gold["fp32_state_gib"]["example"]
    assert B.sv_state_bytes(ex["qubits"], B.SV_C64) == ex["gib"] * 2 ** 30
    for n in (1, 12, 28, 35):
        assert B.sv_state_bytes(n, B.SV_C64) == 2 ** (n - 27) * 2 ** 30
        assert B.sv_state_bytes(n, B.SV_C128) == 2 * B.sv_state_bytes(n, B.SV_C64)
    for bad in (0, 41, -3):
        with pytest.raises(B.SvError) as e:
            B.sv_state_bytes(bad, B.SV_C64)
        assert e.value.code == B.SV_EINVAL
    with pytest.raises(B.SvError):
        B.sv_state_bytes(10, 7)


def test_create_rejects_before_touching_the_device(monkeypatch):
    with pytest.raises(B.SvError) as e:
        B.sv_create(0, B.SV_C64)
    assert e.value.code == B.SV_EINVAL
    monkeypatch.setenv("SV_MAX_DEVICE_BYTES", str(1 << 20))
    with pytest.raises(B.SvError) as e:
        B.sv_create(30, B.SV_C128)
    assert e.value.code == B.SV_ENOMEM
    assert "SV_MAX_DEVICE_BYTES" in B.sv_last_error()


@pytest.mark.parametrize("gate,msg", [
    (Gate("h", (5,)), "out of range"),
    (Gate("x", (1,), (1,)), "used twice"),
    (Gate("matrix", (0, 0), (), (), np.eye(4)), "used twice"),
    (Gate("rx", (0,), (), (float("nan"),)), "non-finite"),
    (Gate("u3", (0,), tuple(range(1, 5))), None),
])
def test_plan_validation(gate, msg):
    if msg is None:
        p = B.sv_plan_create(5, B.SV_C64, [gate])
        B.sv_plan_destroy(p)
        return
    with pytest.raises(B.SvError) as e:
        B.sv_plan_create(5, B.SV_C64, [gate])
    assert e.value.code == B.SV_EINVAL and msg in str(e.value)


def test_plan_option_validation():
    g = [Gate("h", (0,))]
    for opts in (B.make_opts(7, 5), B.make_opts(B.SV_PLAN_GREEDY, 0), B.make_opts(B.SV_PLAN_GREEDY, 7),
                 B.make_opts(B.SV_PLAN_GREEDY, 3, 9)):
        with pytest.raises(B.SvError):
            B.sv_plan_create(4, B.SV_C64, g, opts)


def _blocks(p):
    return [B.sv_plan_block(p, i) for i in range(B.sv_plan_num_blocks(p))]


def test_library_gate_table_matches_reference():
    rng = np.random.default_rng(1)
    for name in ("h", "x", "y", "z", "s", "t", "rx", "ry", "rz", "p", "u3"):
        params = tuple(rng.uniform(-7, 7, size=W.N_PARAMS[name]))
        p = B.sv_plan_create(3, B.SV_C128, [Gate(name, (1,), (), params)])
        (blk,) = _blocks(p)
        B.sv_plan_destroy(p)
        want = oracle.gates.matrix(name, params)
        assert np.max(np.abs(blk["matrix"] - want)) < 1e-15, name
        assert blk["targets"] == [1] and blk["num_gates"] == 1


def _apply_blocks_with_oracle(blocks, n):
    a = oracle.zero_state(n)
    for b in blocks:
        oracle.apply_matrix(a, b["matrix"], b["targets"], b["controls"])
    return a


@pytest.mark.parametrize("kmax", [1, 2, 3, 4, 5, 6])
def test_greedy_plan_reproduces_circuit(kmax):
    n = 10
    gates = W.layered_u3_pairing(n, 6, 5, "cx_or_cz") + W.qft_ladder_block(n, 5) + W.u3_su4_layers(n, 2, 3)
    p = B.sv_plan_create(n, B.SV_C128, gates, B.make_opts(B.SV_PLAN_GREEDY, kmax))
    blocks = _blocks(p)
    B.sv_plan_destroy(p)
    assert sum(b["num_gates"] for b in blocks) == len(gates)
    for b in blocks:
        assert len(b["targets"]) + len(b["controls"]) <= max(kmax, 2 if kmax == 1 else kmax) or b["num_gates"] == 1
        d = 1 << len(b["targets"])
        assert np.max(np.abs(b["matrix"] @ b["matrix"].conj().T - np.eye(d))) < 1e-12
    want = oracle.run(gates, n)
    got = _apply_blocks_with_oracle(blocks, n)
    assert np.max(np.abs(got - want)) < 1e-12
    if kmax >= 4:
        assert len(blocks) < len(gates) / 2


def test_plain_plan_is_one_block_per_gate():
    gates = W.layered_u3_pairing(8, 3, 2, "cx_or_cz")
    p = B.sv_plan_create(8, B.SV_C64, gates, B.make_opts(B.SV_PLAN_PLAIN))
    blocks = _blocks(p)
    B.sv_plan_destroy(p)
    assert len(blocks) == len(gates)
    for g, b in zip(gates, blocks):
        assert tuple(b["targets"]) == g.targets and tuple(b["controls"]) == g.controls


def test_greedy_fusion_ratio_on_28q_layers():
    gates = W.layered_u3_pairing(28, 20, W.circuit_seed(2, 1), "cx_or_cz")
    p = B.sv_plan_create(28, B.SV_C64, gates, B.make_opts(B.SV_PLAN_GREEDY, 5))
    nb = B.sv_plan_num_blocks(p)
    B.sv_plan_destroy(p)
    assert nb < len(gates) / 3, (nb, len(gates))


# ---------------------------------------------------------------------------
# LDS pass plans (host-only structure)
# ---------------------------------------------------------------------------
def wide_and_controlled(n, seed):
    """Layered circuit plus controlled gates, a 5-target matrix (no pass kernel
    takes it) and diagonal gates across the register."""
    rng = np.random.default_rng(seed)
    g = list(W.layered_u3_pairing(n, 4, W.circuit_seed(7, seed), "cx_or_cz"))
    q = [int(x) for x in rng.permutation(n)[:5]]
    g.append(Gate("matrix", tuple(q), (), (), W.haar_unitary(rng, 32)))
    for _ in range(3 * n):
        a, b, c = (int(x) for x in rng.permutation(n)[:3])
        g.append(W.cp(a, b, float(rng.uniform(0, 6))))
        g.append(Gate("u3", (a,), (b, c), tuple(float(x) for x in rng.uniform(0, 6, 3))))
    return g


@pytest.mark.parametrize("n,gates", [
    (28, W.layered_u3_pairing(28, 20, W.circuit_seed(2, 1), "cx_or_cz")),
    (33, W.rcs_circuit(33, W.circuit_seed(6, 1))),
    (33, W.qpe_circuit(32, 0x5A5A5A5A)),
    (33, W.tfim_trotter(3, 11, 10, 0.1, 1.0, 1.0, "cx")),
    (30, W.u3_su4_layers(30, 40, W.circuit_seed(5, 1))),
    (20, wide_and_controlled(20, 3)),
    (10, wide_and_controlled(10, 4)),
], ids=["layered28", "rcs33", "qpe33", "tfim33", "su4_30", "wide20", "small10"])
def test_pass_plan_covers_every_gate_once(n, gates):
    for dtype in (B.SV_C64, B.SV_C128):
        for pq in (4, 6, 8):
            info = B.sv_pass_plan_info(n, dtype, gates, B.make_opts(B.SV_PLAN_PASSES, 5, B.SV_PREC_NATIVE, pq))
            assert info["gates"] == len(gates), (dtype, pq, info)
            assert info["kernel_passes"] <= info["passes"]
            assert info["variant_blocks"] + info["term_blocks"] <= info["blocks"]


def test_pass_plan_structure_on_the_paper_workloads():
    c64 = B.SV_C64
    layered = B.sv_pass_plan_info(28, c64, W.layered_u3_pairing(28, 20, W.circuit_seed(2, 1), "cx_or_cz"))
    assert layered["passes"] <= 31 and layered["sweeps"] == 0
    # phase estimation: controlled-phase ladders across the tile boundary
    # (greedy 5-qubit fusion needs 121 sweeps, tile qubits alone 61 passes)
    qpe = B.sv_pass_plan_info(33, c64, W.qpe_circuit(32, 0x5A5A5A5A))
    assert qpe["passes"] <= 13 and qpe["term_blocks"] > 0
    # CX RZ CX bonds fuse into diagonal phase gates: the same plan as the
    # diagonal-matrix form of the bonds
    cx = B.sv_pass_plan_info(33, c64, W.tfim_trotter(3, 11, 10, 0.1, 1.0, 1.0, "cx"))
    dg = B.sv_pass_plan_info(33, c64, W.tfim_trotter(3, 11, 10, 0.1, 1.0, 1.0, "diag"))
    assert {k: v for k, v in cx.items() if k != "gates"} == {k: v for k, v in dg.items() if k != "gates"}
    assert cx["passes"] <= 60
    # dense SU(4) and U3 gates have no diagonal or controlled form
    su4 = B.sv_pass_plan_info(30, c64, W.u3_su4_layers(30, 40, W.circuit_seed(5, 1)))
    assert su4["variant_blocks"] == 0 and su4["term_blocks"] == 0
    # below the pass tile every pass falls back to fused sweeps
    small = B.sv_pass_plan_info(10, c64, wide_and_controlled(10, 4))
    assert small["kernel_passes"] == 0 and small["sweeps"] > 0


@pytest.mark.parametrize("n,gates", [
    (28, W.layered_u3_pairing(28, 20, W.circuit_seed(2, 1), "cx_or_cz")),
    (33, W.rcs_circuit(33, W.circuit_seed(6, 1))),
    (33, W.qpe_circuit(32, 0x5A5A5A5A)),
    (20, wide_and_controlled(20, 3)),
], ids=["layered28", "rcs33", "qpe33", "wide20"])
def test_pass_plan_gate_order_search(n, gates):
    """Planning over random gate orders (pass_orders: each pass split into
    blocks, and the whole circuit re-planned) still covers every gate once
    and never raises the plan's model time over circuit order and its
    reverse alone; the orders are seeded, so plans repeat."""
    def info(orders):
        return B.sv_pass_plan_info(n, B.SV_C64, gates, B.make_opts(B.SV_PLAN_PASSES, 5, B.SV_PREC_NATIVE, 8, orders))
    base = info(-1)
    assert base["cost_milli"] >= 1000 * base["passes"] // 2
    for orders in (0, 8, 32):
        i = info(orders)
        assert i["gates"] == len(gates)
        assert i["cost_milli"] <= base["cost_milli"], (orders, i, base)
        if orders == 0 and n < 32:
            assert i == base  # no search below 32 qubits by default
    assert info(16) == info(16)


def test_pass_orders_option_bounds():
    g = [Gate("h", (0,))]
    for orders in (-2, 65):
        with pytest.raises(B.SvError):
            B.sv_pass_plan_info(20, B.SV_C64, g, B.make_opts(B.SV_PLAN_PASSES, 5, B.SV_PREC_NATIVE, 8, orders))
    with pytest.raises(B.SvError):
        B.sv_plan_create(12, B.SV_C64, g, B.make_opts(B.SV_PLAN_GREEDY, 5, B.SV_PREC_NATIVE, 0, 4))
    B.sv_pass_plan_info(20, B.SV_C64, g, B.make_opts(B.SV_PLAN_PASSES, 5, B.SV_PREC_NATIVE, 8, 64))


def test_pass_plan_info_rejects_bad_input():
    g = [Gate("h", (0,))]
    for opts in (B.make_opts(B.SV_PLAN_GREEDY, 5), B.make_opts(B.SV_PLAN_PASSES, 5, B.SV_PREC_NATIVE, 3),
                 B.make_opts(B.SV_PLAN_PASSES, 5, B.SV_PREC_NATIVE, 9), B.make_opts(B.SV_PLAN_PASSES, 0)):
        with pytest.raises(B.SvError):
            B.sv_pass_plan_info(12, B.SV_C64, g, opts)
    with pytest.raises(B.SvError):
        B.sv_pass_plan_info(12, B.SV_C64, [Gate("h", (12,))])
    with pytest.raises(B.SvError):
        B.sv_pass_plan_info(0, B.SV_C64, g)


# ---------------------------------------------------------------------------
# The seeded shot stream (sv_uniforms / sv_sample_seeded), host only
# ---------------------------------------------------------------------------
_M64 = (1 << 64) - 1


def _splitmix64(seed, s):
    """s-th output of SplitMix64 (Steele, Lea, Flood, OOPSLA 2014) from state
    `seed`: the state advances by the golden-ratio increment and each output
    is the published 64-bit finaliser of the new state."""
    z = (seed + (s + 1) * 0x9E3779B97F4A7C15) & _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def test_splitmix64_reference_outputs():
    # the first outputs of the reference SplitMix64 generator from state 0
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "splitmix64_seed0.json")))
    assert [_splitmix64(0, s) for s in range(len(gold["outputs"]))] == [int(x, 16) for x in gold["outputs"]]


def test_uniform_stream_is_splitmix64():
    for seed in (0, 7, 2 ** 64 - 1, 0x0123456789ABCDEF):
        got = B.sv_uniforms(seed, 300)
        want = np.array([(_splitmix64(seed, s) >> 11) * 2.0 ** -53 for s in range(300)])
        assert np.array_equal(got, want)
        assert np.all((got >= 0) & (got < 1))
        # any window of the stream can be produced on its own
        assert np.array_equal(B.sv_uniforms(seed, 17, first=250), got[250:267])
    assert B.sv_uniforms(3, 0).size == 0
    with pytest.raises(B.SvError) as e:
        B.sv_uniforms(3, -1)
    assert e.value.code == B.SV_EINVAL


def test_sample_seeded_rejects_before_touching_the_device():
    with pytest.raises(B.SvError) as e:
        B.sv_sample_seeded(0, 10, 1)
    assert e.value.code == B.SV_EINVAL


def test_readout_rejects_before_touching_the_device():
    with pytest.raises(B.SvError) as e:
        B.sv_readout(0, [0], ["Z"], [0.5])
    assert e.value.code == B.SV_EINVAL
