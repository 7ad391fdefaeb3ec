"""FP64 reference state-vector simulator ("the oracle").

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by the
CPU-baseline leg of ``bench.py``; never by the product library, which shares no
code with it.  Arithmetic lives in ``sv_oracle.c`` (plain C, FP64, contraction
off) and ``gates.py``; this module only marshals numpy arrays.

Pins (``tests/test_oracle_pins.py``): tensor-contraction brute force for every
gate kind and placement, gate-table identities and matrix exponentials, closed
forms (uniform superposition, GHZ, QFT of a basis state against numpy's FFT,
product-state expectations, phase estimation with an exactly representable
phase), norm preservation, mirror circuits, library-routine checks of
marginals, sampling and the bit-field exchange.
"""
from __future__ import annotations

import ctypes
import os
from typing import Iterable, Sequence

import numpy as np

from . import gates as _gates

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from .build import build
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    I = ctypes.c_int
    lib.orc_zero_state.argtypes = [P, I]
    lib.orc_zero_state.restype = None
    lib.orc_apply.argtypes = [P, I, P, P, I, P, I]
    lib.orc_apply.restype = I
    lib.orc_probabilities.argtypes = [P, I, P, I, P]
    lib.orc_probabilities.restype = I
    lib.orc_inner.argtypes = [P, P, I, P]
    lib.orc_inner.restype = None
    lib.orc_sample.argtypes = [P, I, P, I, P]
    lib.orc_sample.restype = I
    lib.orc_bitswap.argtypes = [P, P, I, I, I, I]
    lib.orc_bitswap.restype = I
    _lib = lib
    return lib


def _nqubits(state: np.ndarray) -> int:
    n = int(state.size).bit_length() - 1
    if state.dtype != np.complex128 or (1 << n) != state.size or not state.flags.c_contiguous:
        raise ValueError("state must be a contiguous complex128 array of length 2^n")
    return n


def _i32(xs: Iterable[int]) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(list(xs), dtype=np.int32))


def zero_state(n: int) -> np.ndarray:
    a = np.empty(1 << n, dtype=np.complex128)
    _load().orc_zero_state(a.ctypes.data, n)
    return a


def gate_matrix(g) -> np.ndarray:
    return _gates.matrix(g.name, g.params, g.matrix)


def apply_matrix(state: np.ndarray, U: np.ndarray, targets: Sequence[int],
                 controls: Sequence[int] = ()) -> np.ndarray:
    """In place: apply U (2^k x 2^k, bit b of its index = targets[b]) with controls."""
    n = _nqubits(state)
    U = np.ascontiguousarray(np.asarray(U, dtype=np.complex128))
    k = len(targets)
    if U.shape != (1 << k, 1 << k):
        raise ValueError("matrix shape does not match target count")
    t = _i32(targets)
    c = _i32(controls) if len(controls) else np.zeros(1, dtype=np.int32)
    rc = _load().orc_apply(state.ctypes.data, n, U.ctypes.data, t.ctypes.data, k,
                           c.ctypes.data, len(controls))
    if rc != 0:
        raise ValueError(f"orc_apply rejected targets={targets} controls={controls} n={n}")
    return state


def apply_gate(state: np.ndarray, g) -> np.ndarray:
    return apply_matrix(state, gate_matrix(g), g.targets, g.controls)


def run(ops, n: int, state: np.ndarray | None = None) -> np.ndarray:
    """Apply a gate list to |0..0> (or to ``state`` in place).  ``BitSwap`` entries
    are physical relayouts that leave the logical state unchanged, so the
    reference skips them."""
    a = zero_state(n) if state is None else state
    for g in ops:
        if hasattr(g, "name"):
            apply_gate(a, g)
    return a


def probabilities(state: np.ndarray, qubits: Sequence[int] | None = None) -> np.ndarray:
    n = _nqubits(state)
    q = list(range(n)) if qubits is None else list(qubits)
    out = np.empty(1 << len(q), dtype=np.float64)
    qa = _i32(q) if q else np.zeros(1, dtype=np.int32)
    if _load().orc_probabilities(state.ctypes.data, n, qa.ctypes.data, len(q), out.ctypes.data) != 0:
        raise ValueError("bad qubit list")
    return out


def norm2(state: np.ndarray) -> float:
    return float(probabilities(state, [])[0])


def inner(a: np.ndarray, b: np.ndarray) -> complex:
    n = _nqubits(a)
    if _nqubits(b) != n:
        raise ValueError("size mismatch")
    out = np.empty(2, dtype=np.float64)
    _load().orc_inner(a.ctypes.data, b.ctypes.data, n, out.ctypes.data)
    return complex(out[0], out[1])


def expect_pauli(state: np.ndarray, term: str) -> complex:
    """<psi|P|psi> for a Pauli string (character q acts on qubit q): b = P|psi>
    built by applying each one-qubit Pauli, then <psi|b>."""
    n = _nqubits(state)
    if len(term) != n:
        raise ValueError("Pauli string length must equal the qubit count")
    b = state.copy()
    for q, ch in enumerate(term.upper()):
        if ch == "I":
            continue
        apply_matrix(b, _gates.PAULI[ch], [q])
    return inner(state, b)


def sample(state: np.ndarray, u: np.ndarray) -> np.ndarray:
    n = _nqubits(state)
    u = np.ascontiguousarray(np.asarray(u, dtype=np.float64))
    out = np.empty(u.size, dtype=np.int64)
    if _load().orc_sample(state.ctypes.data, n, u.ctypes.data, u.size, out.ctypes.data) != 0:
        raise MemoryError("orc_sample")
    return out


def bitswap(state: np.ndarray, lo: int, hi: int, width: int) -> np.ndarray:
    n = _nqubits(state)
    out = np.empty_like(state)
    if _load().orc_bitswap(state.ctypes.data, out.ctypes.data, n, lo, hi, width) != 0:
        raise ValueError("bad bit fields")
    return out


def apply_bitswap_map(qmap: list, lo: int, hi: int, width: int) -> list:
    """Logical->physical qubit map after exchanging physical fields [lo,lo+w) and [hi,hi+w)."""
    out = list(qmap)
    for q, p in enumerate(qmap):
        if lo <= p < lo + width:
            out[q] = p - lo + hi
        elif hi <= p < hi + width:
            out[q] = p - hi + lo
    return out


def num_threads() -> int:
    lib = _load()
    lib.orc_num_threads.restype = ctypes.c_int
    return int(lib.orc_num_threads())
