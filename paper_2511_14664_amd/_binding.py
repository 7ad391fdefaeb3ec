"""ctypes binding of libsv.so (include/sv.h), same names as the C entry points.

Argument marshalling only: every step of gate application and read-out runs
in the HIP library.  There is no fallback: if libsv.so is missing or fails to
load, importing this module raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Iterable, List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsv.so")

SV_OK, SV_EINVAL, SV_ENOMEM, SV_EDEVICE, SV_EUNSUPPORTED = 0, -1, -2, -3, -4
SV_C64, SV_C128 = 0, 1
SV_PLAN_PLAIN, SV_PLAN_GREEDY, SV_PLAN_LEARNED, SV_PLAN_PASSES = 0, 1, 2, 3
SV_PREC_NATIVE, SV_PREC_BF16X3, SV_PREC_BF16X6 = 0, 1, 2
SV_MAX_TARGETS, SV_MAX_CONTROLS = 6, 8
SV_NOALLOC_MAX_TERMS = 256

GATE_KIND = {"h": 0, "x": 1, "y": 2, "z": 3, "s": 4, "t": 5, "rx": 6, "ry": 7, "rz": 8,
             "p": 9, "u3": 10, "matrix": 11}

_ERRNAMES = {SV_EINVAL: "SV_EINVAL", SV_ENOMEM: "SV_ENOMEM", SV_EDEVICE: "SV_EDEVICE",
             SV_EUNSUPPORTED: "SV_EUNSUPPORTED"}


class SvError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__(f"{where}: {_ERRNAMES.get(code, code)}: {msg}")
        self.code = code


class sv_gate(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("num_targets", ctypes.c_int32),
                ("num_controls", ctypes.c_int32),
                ("targets", ctypes.c_int32 * SV_MAX_TARGETS),
                ("controls", ctypes.c_int32 * SV_MAX_CONTROLS),
                ("params", ctypes.c_double * 3),
                ("matrix", ctypes.POINTER(ctypes.c_double))]


class sv_plan_opts(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("max_fused", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("pass_qubits", ctypes.c_int32), ("pass_orders", ctypes.c_int32),
                ("pass_tile", ctypes.c_int32)]


class sv_run_stats(ctypes.Structure):
    _fields_ = [("gates", ctypes.c_int64), ("sweeps", ctypes.c_int64),
                ("fused_blocks", ctypes.c_int64), ("algorithmic_bytes", ctypes.c_double),
                ("flops", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
    # PyTorch ships its own HIP runtime under the same soname.  Loading torch
    # first makes libsv.so bind to that one, so the process holds a single HIP
    # runtime and torch-allocated memory and streams are valid in the library.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    P, I, U64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_uint64
    sig = {
        "sv_last_error": ([], ctypes.c_char_p),
        "sv_state_bytes": ([I, I, ctypes.POINTER(U64)], I),
        "sv_create": ([I, I, ctypes.POINTER(P)], I),
        "sv_create_on": ([P, U64, I, I, P, ctypes.POINTER(P)], I),
        "sv_destroy": ([P], I),
        "sv_set_stream": ([P, P], I),
        "sv_synchronize": ([P], I),
        "sv_reset": ([P], I),
        "sv_apply_gate": ([P, P, P, I, P, I], I),
        "sv_apply_circuit": ([P, ctypes.POINTER(sv_gate), I, ctypes.POINTER(sv_plan_opts),
                              ctypes.POINTER(sv_run_stats)], I),
        "sv_swap_bits": ([P, I, I, I], I),
        "sv_qubit_map": ([P, P], I),
        "sv_probabilities": ([P, P, I, P], I),
        "sv_expect_pauli": ([P, ctypes.POINTER(ctypes.c_char_p), I, P], I),
        "sv_expect_pauli_noalloc": ([P, ctypes.POINTER(ctypes.c_char_p), I, P], I),
        "sv_sample": ([P, P, I, P], I),
        "sv_sample_seeded": ([P, I, U64, P], I),
        "sv_readout": ([P, P, I, P, ctypes.POINTER(ctypes.c_char_p), I, P, P, I, P], I),
        "sv_uniforms": ([U64, U64, I, P], I),
        "sv_copy_to_host": ([P, P, U64, U64], I),
        "sv_copy_from_host": ([P, P, U64, U64], I),
        "sv_plan_create": ([I, I, ctypes.POINTER(sv_gate), I, ctypes.POINTER(sv_plan_opts),
                            ctypes.POINTER(P)], I),
        "sv_plan_num_blocks": ([P, ctypes.POINTER(I)], I),
        "sv_plan_block": ([P, I, P, P, P, P, P, P], I),
        "sv_apply_plan": ([P, P, ctypes.POINTER(sv_run_stats)], I),
        "sv_plan_destroy": ([P], I),
        "sv_pass_plan_info": ([I, I, ctypes.POINTER(sv_gate), I, ctypes.POINTER(sv_plan_opts), P], I),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


_lib = _load()


def _check(rc: int, where: str):
    if rc != SV_OK:
        raise SvError(rc, where, sv_last_error())


def sv_last_error() -> str:
    return _lib.sv_last_error().decode()


def amp_dtype(dtype: int):
    return np.complex64 if dtype == SV_C64 else np.complex128


# ---------------------------------------------------------------------------
# Gate lists
# ---------------------------------------------------------------------------
class Circuit:
    """A gate list marshalled once into an sv_gate array (kept alive here)."""

    def __init__(self, gates: Iterable):
        gates = [g for g in gates if hasattr(g, "name")]
        self.n_gates = len(gates)
        self.array = (sv_gate * max(1, len(gates)))()
        self._keep: List[np.ndarray] = []
        for i, g in enumerate(gates):
            s = self.array[i]
            s.kind = GATE_KIND[g.name]
            s.num_targets = len(g.targets)
            s.num_controls = len(g.controls)
            for j, q in enumerate(g.targets):
                s.targets[j] = int(q)
            for j, q in enumerate(g.controls):
                s.controls[j] = int(q)
            for j, p in enumerate(g.params):
                s.params[j] = float(p)
            if g.name == "matrix":
                m = np.ascontiguousarray(np.asarray(g.matrix, dtype=np.complex128))
                self._keep.append(m)
                s.matrix = m.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def make_opts(mode: int = SV_PLAN_PLAIN, max_fused: int = 5, precision: int = SV_PREC_NATIVE,
              pass_qubits: int = 0, pass_orders: int = 0, pass_tile: int = 0) -> sv_plan_opts:
    return sv_plan_opts(mode, max_fused, precision, pass_qubits, pass_orders, pass_tile)


def _as_circuit(gates) -> Circuit:
    return gates if isinstance(gates, Circuit) else Circuit(gates)


# ---------------------------------------------------------------------------
# Entry points
# ---------------------------------------------------------------------------
def sv_state_bytes(n: int, dtype: int) -> int:
    out = ctypes.c_uint64()
    _check(_lib.sv_state_bytes(n, dtype, ctypes.byref(out)), "sv_state_bytes")
    return out.value


def sv_create(n: int, dtype: int) -> int:
    h = ctypes.c_void_p()
    _check(_lib.sv_create(n, dtype, ctypes.byref(h)), "sv_create")
    return h.value


def sv_create_on(device_ptr: int, nbytes: int, n: int, dtype: int, stream: int = 0) -> int:
    h = ctypes.c_void_p()
    _check(_lib.sv_create_on(ctypes.c_void_p(device_ptr), nbytes, n, dtype,
                             ctypes.c_void_p(stream or None), ctypes.byref(h)), "sv_create_on")
    return h.value


def sv_destroy(h: int):
    _check(_lib.sv_destroy(ctypes.c_void_p(h)), "sv_destroy")


def sv_set_stream(h: int, stream: int):
    _check(_lib.sv_set_stream(ctypes.c_void_p(h), ctypes.c_void_p(stream or None)), "sv_set_stream")


def sv_synchronize(h: int):
    _check(_lib.sv_synchronize(ctypes.c_void_p(h)), "sv_synchronize")


def sv_reset(h: int):
    _check(_lib.sv_reset(ctypes.c_void_p(h)), "sv_reset")


def sv_apply_gate(h: int, U, targets: Sequence[int], controls: Sequence[int] = ()):
    U = np.ascontiguousarray(np.asarray(U, dtype=np.complex128))
    t = np.ascontiguousarray(np.asarray(list(targets), dtype=np.int32))
    c = np.ascontiguousarray(np.asarray(list(controls) or [0], dtype=np.int32))
    _check(_lib.sv_apply_gate(ctypes.c_void_p(h), U.ctypes.data, t.ctypes.data, len(targets),
                              c.ctypes.data if len(controls) else None, len(controls)), "sv_apply_gate")


def sv_apply_circuit(h: int, gates, opts: Optional[sv_plan_opts] = None) -> dict:
    circ = _as_circuit(gates)
    st = sv_run_stats()
    o = opts if opts is not None else make_opts()
    _check(_lib.sv_apply_circuit(ctypes.c_void_p(h), circ.array, circ.n_gates, ctypes.byref(o),
                                 ctypes.byref(st)), "sv_apply_circuit")
    return st.as_dict()


def sv_swap_bits(h: int, lo: int, hi: int, width: int):
    _check(_lib.sv_swap_bits(ctypes.c_void_p(h), lo, hi, width), "sv_swap_bits")


def sv_qubit_map(h: int, n: int) -> List[int]:
    m = np.zeros(n, dtype=np.int32)
    _check(_lib.sv_qubit_map(ctypes.c_void_p(h), m.ctypes.data), "sv_qubit_map")
    return [int(x) for x in m]


def sv_probabilities(h: int, qubits: Sequence[int]) -> np.ndarray:
    q = np.ascontiguousarray(np.asarray(list(qubits) or [0], dtype=np.int32))
    out = np.empty(1 << len(qubits), dtype=np.float64)
    _check(_lib.sv_probabilities(ctypes.c_void_p(h), q.ctypes.data if len(qubits) else None,
                                 len(qubits), out.ctypes.data), "sv_probabilities")
    return out


def sv_expect_pauli(h: int, terms: Sequence[str]) -> np.ndarray:
    arr = (ctypes.c_char_p * max(1, len(terms)))(*[t.encode() for t in terms])
    out = np.empty(max(1, len(terms)), dtype=np.float64)
    _check(_lib.sv_expect_pauli(ctypes.c_void_p(h), arr, len(terms), out.ctypes.data), "sv_expect_pauli")
    return out[:len(terms)]


def sv_expect_pauli_noalloc(h: int, terms: Sequence[str]) -> np.ndarray:
    arr = (ctypes.c_char_p * max(1, len(terms)))(*[t.encode() for t in terms])
    out = np.empty(max(1, len(terms)), dtype=np.float64)
    _check(_lib.sv_expect_pauli_noalloc(ctypes.c_void_p(h), arr, len(terms), out.ctypes.data),
           "sv_expect_pauli_noalloc")
    return out[:len(terms)]


def sv_sample(h: int, uniforms) -> np.ndarray:
    u = np.ascontiguousarray(np.asarray(uniforms, dtype=np.float64))
    out = np.empty(max(1, u.size), dtype=np.int64)
    _check(_lib.sv_sample(ctypes.c_void_p(h), u.ctypes.data, u.size, out.ctypes.data), "sv_sample")
    return out[:u.size]


def sv_sample_seeded(h: int, shots: int, seed: int) -> np.ndarray:
    out = np.empty(max(1, shots), dtype=np.int64)
    _check(_lib.sv_sample_seeded(ctypes.c_void_p(h), shots, seed, out.ctypes.data), "sv_sample_seeded")
    return out[:shots]


def sv_readout(h: int, qubits: Optional[Sequence[int]] = None, terms: Sequence[str] = (), uniforms=None):
    """sv_readout: (marginal or None, expectation values, samples) of one state."""
    want_p = qubits is not None
    q = np.ascontiguousarray(np.asarray(list(qubits or []) or [0], dtype=np.int32))
    m = len(qubits) if want_p else 0
    probs = np.empty(1 << m, dtype=np.float64) if want_p else None
    arr = (ctypes.c_char_p * max(1, len(terms)))(*[t.encode() for t in terms])
    expect = np.empty(max(1, len(terms)), dtype=np.float64)
    u = np.ascontiguousarray(np.asarray([] if uniforms is None else uniforms, dtype=np.float64))
    samples = np.empty(max(1, u.size), dtype=np.int64)
    _check(_lib.sv_readout(ctypes.c_void_p(h), q.ctypes.data if m else None, m,
                           probs.ctypes.data if want_p else None, arr, len(terms), expect.ctypes.data,
                           u.ctypes.data if u.size else None, u.size, samples.ctypes.data), "sv_readout")
    return probs, expect[:len(terms)], samples[:u.size]


def sv_uniforms(seed: int, count: int, first: int = 0) -> np.ndarray:
    out = np.empty(max(1, count), dtype=np.float64)
    _check(_lib.sv_uniforms(seed, first, count, out.ctypes.data), "sv_uniforms")
    return out[:count]


def sv_copy_to_host(h: int, n: int, dtype: int, first: int = 0, count: Optional[int] = None) -> np.ndarray:
    if count is None:
        count = (1 << n) - first
    out = np.empty(count, dtype=amp_dtype(dtype))
    _check(_lib.sv_copy_to_host(ctypes.c_void_p(h), out.ctypes.data, first, count), "sv_copy_to_host")
    return out


def sv_copy_from_host(h: int, dtype: int, src, first: int = 0):
    a = np.ascontiguousarray(np.asarray(src, dtype=amp_dtype(dtype)))
    _check(_lib.sv_copy_from_host(ctypes.c_void_p(h), a.ctypes.data, first, a.size), "sv_copy_from_host")


def sv_plan_create(n: int, dtype: int, gates, opts: Optional[sv_plan_opts] = None) -> int:
    circ = _as_circuit(gates)
    p = ctypes.c_void_p()
    o = opts if opts is not None else make_opts()
    _check(_lib.sv_plan_create(n, dtype, circ.array, circ.n_gates, ctypes.byref(o), ctypes.byref(p)),
           "sv_plan_create")
    return p.value


def sv_pass_plan_info(n: int, dtype: int, gates, opts: Optional[sv_plan_opts] = None) -> dict:
    circ = _as_circuit(gates)
    out = np.zeros(8, dtype=np.int64)
    o = opts if opts is not None else make_opts(SV_PLAN_PASSES)
    _check(_lib.sv_pass_plan_info(n, dtype, circ.array, circ.n_gates, ctypes.byref(o), out.ctypes.data),
           "sv_pass_plan_info")
    keys = ("passes", "kernel_passes", "blocks", "variant_blocks", "term_blocks", "sweeps", "gates", "cost_milli")
    return {k: int(v) for k, v in zip(keys, out)}


def sv_plan_num_blocks(p: int) -> int:
    out = ctypes.c_int()
    _check(_lib.sv_plan_num_blocks(ctypes.c_void_p(p), ctypes.byref(out)), "sv_plan_num_blocks")
    return out.value


def sv_plan_block(p: int, i: int) -> dict:
    k, c, ng = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    t = np.zeros(SV_MAX_TARGETS, dtype=np.int32)
    ctl = np.zeros(SV_MAX_CONTROLS, dtype=np.int32)
    _check(_lib.sv_plan_block(ctypes.c_void_p(p), i, ctypes.byref(k), t.ctypes.data, ctypes.byref(c),
                              ctl.ctypes.data, None, ctypes.byref(ng)), "sv_plan_block")
    d = 1 << k.value
    m = np.empty((d, d), dtype=np.complex128)
    _check(_lib.sv_plan_block(ctypes.c_void_p(p), i, None, None, None, None, m.ctypes.data, None),
           "sv_plan_block")
    return {"targets": [int(x) for x in t[:k.value]], "controls": [int(x) for x in ctl[:c.value]],
            "matrix": m, "num_gates": ng.value}


def sv_apply_plan(h: int, p: int) -> dict:
    st = sv_run_stats()
    _check(_lib.sv_apply_plan(ctypes.c_void_p(h), ctypes.c_void_p(p), ctypes.byref(st)), "sv_apply_plan")
    return st.as_dict()


def sv_plan_destroy(p: int):
    _check(_lib.sv_plan_destroy(ctypes.c_void_p(p)), "sv_plan_destroy")


# ---------------------------------------------------------------------------
# Sweep timing
# ---------------------------------------------------------------------------
class sv_sweep_record(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("k", ctypes.c_int32), ("c", ctypes.c_int32),
                ("lowest_target", ctypes.c_int32), ("highest_target", ctypes.c_int32),
                ("num_gates", ctypes.c_int32), ("bytes", ctypes.c_double), ("flops", ctypes.c_double),
                ("ms", ctypes.c_float), ("precision", ctypes.c_int32), ("mfma_flops", ctypes.c_double),
                ("blocks", ctypes.c_int32), ("term_blocks", ctypes.c_int32), ("variant_blocks", ctypes.c_int32),
                ("tile_log", ctypes.c_int32), ("tile_mask", ctypes.c_uint64)]


SWEEP_KIND = {0: "gate1", 1: "diag1", 2: "dense_tile", 3: "dense_mfma", 4: "dense_group", 5: "bitswap",
              6: "dense_bf16x3", 7: "pass"}

_lib.sv_profile_enable.argtypes = [ctypes.c_void_p, ctypes.c_int]
_lib.sv_profile_enable.restype = ctypes.c_int
_lib.sv_profile_read.argtypes = [ctypes.c_void_p, ctypes.POINTER(sv_sweep_record), ctypes.c_int,
                                 ctypes.POINTER(ctypes.c_int)]
_lib.sv_profile_read.restype = ctypes.c_int


def sv_profile_enable(h: int, enable: bool = True):
    _check(_lib.sv_profile_enable(ctypes.c_void_p(h), 1 if enable else 0), "sv_profile_enable")


def sv_profile_read(h: int, max_records: int = 1 << 16) -> List[dict]:
    buf = (sv_sweep_record * max_records)()
    cnt = ctypes.c_int()
    _check(_lib.sv_profile_read(ctypes.c_void_p(h), buf, max_records, ctypes.byref(cnt)), "sv_profile_read")
    out = []
    for i in range(min(cnt.value, max_records)):
        r = buf[i]
        d = {f: getattr(r, f) for f, _ in r._fields_}
        d["kind_name"] = SWEEP_KIND.get(r.kind, str(r.kind))
        out.append(d)
    return out


# ---------------------------------------------------------------------------
# Batches
# ---------------------------------------------------------------------------
class sv_batch_config(ctypes.Structure):
    _fields_ = [("tile_bits", ctypes.c_int32), ("low_bits", ctypes.c_int32),
                ("fuse_width", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return {"tile_bits": self.tile_bits, "low_bits": self.low_bits, "fuse_width": self.fuse_width}


_P = ctypes.c_void_p
_lib.sv_batch_create.argtypes = [ctypes.c_int, ctypes.c_int, _P, _P, _P, _P, _P, _P, ctypes.POINTER(_P)]
_lib.sv_batch_create.restype = ctypes.c_int
_lib.sv_batch_run.argtypes = [_P, _P, _P]
_lib.sv_batch_run.restype = ctypes.c_int
_lib.sv_batch_tune.argtypes = [_P, ctypes.c_int, ctypes.POINTER(sv_batch_config)]
_lib.sv_batch_tune.restype = ctypes.c_int
_lib.sv_batch_set_config.argtypes = [_P, ctypes.POINTER(sv_batch_config)]
_lib.sv_batch_set_config.restype = ctypes.c_int
_lib.sv_batch_get_config.argtypes = [_P, ctypes.POINTER(sv_batch_config)]
_lib.sv_batch_get_config.restype = ctypes.c_int
_lib.sv_batch_last_ms.argtypes = [_P, ctypes.POINTER(ctypes.c_double)]
_lib.sv_batch_last_ms.restype = ctypes.c_int
_lib.sv_batch_destroy.argtypes = [_P]
_lib.sv_batch_destroy.restype = ctypes.c_int


class Batch:
    """Marshalled batch inputs (gate arrays and Z masks kept alive here)."""

    def __init__(self, circuits: Sequence, qubits: Sequence[int], zmasks: Sequence[Sequence[int]]):
        self.circs = [_as_circuit(c) for c in circuits]
        self.ninst = len(self.circs)
        self.q = np.ascontiguousarray(np.asarray(qubits, dtype=np.int32))
        self.ng = np.ascontiguousarray(np.asarray([c.n_gates for c in self.circs], dtype=np.int32))
        self.gptr = (ctypes.c_void_p * self.ninst)(*[ctypes.addressof(c.array) for c in self.circs])
        self.z = [np.ascontiguousarray(np.asarray(list(z) or [0], dtype=np.uint64)) for z in zmasks]
        self.nt = np.ascontiguousarray(np.asarray([len(z) for z in zmasks], dtype=np.int32))
        self.zptr = (ctypes.c_void_p * self.ninst)(*[z.ctypes.data for z in self.z])
        self.total_terms = int(self.nt.sum())

    def gate_pointers(self, circuits=None):
        if circuits is None:
            return None
        circs = [_as_circuit(c) for c in circuits]
        self._keep_run = circs
        return (ctypes.c_void_p * len(circs))(*[ctypes.addressof(c.array) for c in circs])


def sv_batch_create(dtype: int, batch: Batch, stream: int = 0) -> int:
    h = ctypes.c_void_p()
    _check(_lib.sv_batch_create(dtype, batch.ninst, batch.q.ctypes.data, batch.gptr, batch.ng.ctypes.data,
                                batch.zptr, batch.nt.ctypes.data, ctypes.c_void_p(stream or None),
                                ctypes.byref(h)), "sv_batch_create")
    return h.value


def sv_batch_run(h: int, batch: Batch, circuits=None) -> np.ndarray:
    out = np.empty(max(1, batch.total_terms), dtype=np.float64)
    gp = batch.gate_pointers(circuits)
    _check(_lib.sv_batch_run(ctypes.c_void_p(h), gp, out.ctypes.data), "sv_batch_run")
    return out[:batch.total_terms]


def sv_batch_tune(h: int, repeats: int = 2) -> dict:
    c = sv_batch_config()
    _check(_lib.sv_batch_tune(ctypes.c_void_p(h), repeats, ctypes.byref(c)), "sv_batch_tune")
    return c.as_dict()


def sv_batch_set_config(h: int, tile_bits: int, low_bits: int, fuse_width: int):
    c = sv_batch_config(tile_bits, low_bits, fuse_width, 0)
    _check(_lib.sv_batch_set_config(ctypes.c_void_p(h), ctypes.byref(c)), "sv_batch_set_config")


def sv_batch_get_config(h: int) -> dict:
    c = sv_batch_config()
    _check(_lib.sv_batch_get_config(ctypes.c_void_p(h), ctypes.byref(c)), "sv_batch_get_config")
    return c.as_dict()


def sv_batch_last_ms(h: int) -> float:
    v = ctypes.c_double()
    _check(_lib.sv_batch_last_ms(ctypes.c_void_p(h), ctypes.byref(v)), "sv_batch_last_ms")
    return v.value


def sv_batch_destroy(h: int):
    _check(_lib.sv_batch_destroy(ctypes.c_void_p(h)), "sv_batch_destroy")


def sv_profile_read_raw(h: int, max_records: int = 1 << 16):
    """Recorded sweeps as an sv_sweep_record array (for sv_sweep_features)."""
    buf = (sv_sweep_record * max_records)()
    cnt = ctypes.c_int()
    _check(_lib.sv_profile_read(ctypes.c_void_p(h), buf, max_records, ctypes.byref(cnt)), "sv_profile_read")
    return buf, min(cnt.value, max_records)


# ---------------------------------------------------------------------------
# Learned cost model
# ---------------------------------------------------------------------------
SV_CM_FEATURES, SV_CM_HIDDEN = 16, 64
_F32P = ctypes.POINTER(ctypes.c_float)
for _name, _args in {
    "sv_costmodel_num_params": [ctypes.POINTER(ctypes.c_int)],
    "sv_costmodel_create": [ctypes.c_uint64, ctypes.POINTER(_P)],
    "sv_costmodel_get_params": [_P, _P],
    "sv_costmodel_set_params": [_P, _P],
    "sv_costmodel_grad": [_P, _P, _P, ctypes.c_int, _P, _F32P],
    "sv_costmodel_train": [_P, _P, _P, ctypes.c_int, ctypes.c_int, ctypes.c_float, _F32P],
    "sv_costmodel_predict": [_P, _P, ctypes.c_int, _P],
    "sv_costmodel_destroy": [_P],
    "sv_sweep_features": [ctypes.c_int, ctypes.c_int, _P, ctypes.c_int, _P],
    "sv_sweep_targets": [_P, ctypes.c_int, _P],
    "sv_set_costmodel": [_P, _P],
    "sv_costmodel_rank": [_P, ctypes.c_int, ctypes.c_int, ctypes.POINTER(sv_gate), ctypes.c_int, ctypes.c_int,
                          ctypes.POINTER(ctypes.c_int), _P],
}.items():
    _fn = getattr(_lib, _name)
    _fn.argtypes = _args
    _fn.restype = ctypes.c_int


def sv_costmodel_num_params() -> int:
    v = ctypes.c_int()
    _check(_lib.sv_costmodel_num_params(ctypes.byref(v)), "sv_costmodel_num_params")
    return v.value


def sv_costmodel_create(seed: int = 0) -> int:
    h = ctypes.c_void_p()
    _check(_lib.sv_costmodel_create(seed, ctypes.byref(h)), "sv_costmodel_create")
    return h.value


def sv_costmodel_get_params(m: int) -> np.ndarray:
    out = np.empty(sv_costmodel_num_params(), dtype=np.float32)
    _check(_lib.sv_costmodel_get_params(ctypes.c_void_p(m), out.ctypes.data), "sv_costmodel_get_params")
    return out


def sv_costmodel_set_params(m: int, p):
    p = np.ascontiguousarray(np.asarray(p, dtype=np.float32))
    if p.size != sv_costmodel_num_params():
        raise ValueError("wrong parameter count")
    _check(_lib.sv_costmodel_set_params(ctypes.c_void_p(m), p.ctypes.data), "sv_costmodel_set_params")


def _xy(x, y=None):
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float32).reshape(-1, SV_CM_FEATURES))
    if y is not None:
        y = np.ascontiguousarray(np.asarray(y, dtype=np.float32).ravel())
    return x, y


def sv_costmodel_grad(m: int, x, y):
    x, y = _xy(x, y)
    g = np.empty(sv_costmodel_num_params(), dtype=np.float32)
    L = ctypes.c_float()
    _check(_lib.sv_costmodel_grad(ctypes.c_void_p(m), x.ctypes.data, y.ctypes.data, x.shape[0], g.ctypes.data,
                                  ctypes.byref(L)), "sv_costmodel_grad")
    return float(L.value), g


def sv_costmodel_train(m: int, x, y, epochs: int, lr: float) -> float:
    x, y = _xy(x, y)
    L = ctypes.c_float()
    _check(_lib.sv_costmodel_train(ctypes.c_void_p(m), x.ctypes.data, y.ctypes.data, x.shape[0], epochs, lr,
                                   ctypes.byref(L)), "sv_costmodel_train")
    return float(L.value)


def sv_costmodel_predict(m: int, x) -> np.ndarray:
    x, _ = _xy(x)
    out = np.empty(x.shape[0], dtype=np.float32)
    _check(_lib.sv_costmodel_predict(ctypes.c_void_p(m), x.ctypes.data, x.shape[0], out.ctypes.data),
           "sv_costmodel_predict")
    return out


def sv_costmodel_destroy(m: int):
    _check(_lib.sv_costmodel_destroy(ctypes.c_void_p(m)), "sv_costmodel_destroy")


def sv_sweep_features(n: int, dtype: int, records, count: int) -> np.ndarray:
    out = np.empty((max(1, count), SV_CM_FEATURES), dtype=np.float32)
    _check(_lib.sv_sweep_features(n, dtype, records, count, out.ctypes.data), "sv_sweep_features")
    return out[:count]


def sv_sweep_targets(records, count: int) -> np.ndarray:
    out = np.empty(max(1, count), dtype=np.float32)
    _check(_lib.sv_sweep_targets(records, count, out.ctypes.data), "sv_sweep_targets")
    return out[:count]


def sv_set_costmodel(h: int, m: Optional[int]):
    _check(_lib.sv_set_costmodel(ctypes.c_void_p(h), ctypes.c_void_p(m or None)), "sv_set_costmodel")


def sv_costmodel_rank(m: int, n: int, dtype: int, gates, max_fused: int = 6):
    """(chosen, predicted ms): chosen is the greedy width 1..max_fused or 0 for
    the pass plan; predictions for widths 1..max_fused, then the pass plan."""
    circ = _as_circuit(gates)
    chosen = ctypes.c_int()
    pred = np.zeros(max_fused + 1, dtype=np.float32)
    _check(_lib.sv_costmodel_rank(ctypes.c_void_p(m), n, dtype, circ.array, circ.n_gates, max_fused,
                                  ctypes.byref(chosen), pred.ctypes.data), "sv_costmodel_rank")
    return chosen.value, pred
