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
