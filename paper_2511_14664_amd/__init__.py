"""MI355X-native state-vector gate application (gfx950 HIP behind a C ABI).

``_binding`` exposes the C entry points of ``include/sv.h`` under the same
names.  ``StateVector`` is a convenience wrapper that takes the device memory
from PyTorch (one tensor, caching allocator) and orders all work on the current
torch stream; PyTorch is used for memory and streams only.
"""
from __future__ import annotations

from typing import Optional, Sequence

import numpy as np

from ._binding import *  # noqa: F401,F403
from ._binding import (SV_C64, SV_C128, SV_PLAN_PLAIN, SV_PLAN_GREEDY, SV_PLAN_LEARNED,  # noqa: F401
                       SV_PREC_NATIVE, SV_PREC_BF16X3, Circuit, SvError, make_opts, LIB_PATH)
from . import _binding as _b


class StateVector:
    """n-qubit state in a torch-allocated HBM buffer."""

    def __init__(self, n: int, dtype: int = SV_C128, device: int = 0, stream=None):
        import torch

        self.n = n
        self.dtype = dtype
        nbytes = _b.sv_state_bytes(n, dtype)
        self._torch_device = torch.device("cuda", device)
        self.buffer = torch.empty(nbytes, dtype=torch.uint8, device=self._torch_device)
        s = stream if stream is not None else torch.cuda.current_stream(self._torch_device)
        self.stream = s
        with torch.cuda.device(self._torch_device):
            self.handle = _b.sv_create_on(self.buffer.data_ptr(), nbytes, n, dtype, s.cuda_stream)

    def close(self):
        if getattr(self, "handle", None):
            _b.sv_destroy(self.handle)
            self.handle = None
            self.buffer = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # --- gate application -------------------------------------------------
    def reset(self):
        _b.sv_reset(self.handle)

    def apply_gate(self, U, targets: Sequence[int], controls: Sequence[int] = ()):
        _b.sv_apply_gate(self.handle, U, targets, controls)

    def apply_circuit(self, gates, mode: int = SV_PLAN_PLAIN, max_fused: int = 5,
                      precision: int = SV_PREC_NATIVE) -> dict:
        return _b.sv_apply_circuit(self.handle, gates, make_opts(mode, max_fused, precision))

    def swap_bits(self, lo: int, hi: int, width: int):
        _b.sv_swap_bits(self.handle, lo, hi, width)

    def qubit_map(self):
        return _b.sv_qubit_map(self.handle, self.n)

    def synchronize(self):
        _b.sv_synchronize(self.handle)

    # --- read-out ---------------------------------------------------------
    def probabilities(self, qubits: Optional[Sequence[int]] = None) -> np.ndarray:
        return _b.sv_probabilities(self.handle, list(range(self.n)) if qubits is None else qubits)

    def expect_pauli(self, terms: Sequence[str]) -> np.ndarray:
        return _b.sv_expect_pauli(self.handle, terms)

    def sample(self, uniforms) -> np.ndarray:
        return _b.sv_sample(self.handle, uniforms)

    def sample_seeded(self, shots: int, seed: int) -> np.ndarray:
        return _b.sv_sample_seeded(self.handle, shots, seed)

    def readout(self, qubits: Optional[Sequence[int]] = None, terms: Sequence[str] = (), uniforms=None):
        """Marginal, expectation values and samples in one call (one read of the state where possible)."""
        return _b.sv_readout(self.handle, qubits, terms, uniforms)

    def to_host(self, first: int = 0, count: Optional[int] = None) -> np.ndarray:
        return _b.sv_copy_to_host(self.handle, self.n, self.dtype, first, count)

    def from_host(self, src, first: int = 0):
        _b.sv_copy_from_host(self.handle, self.dtype, src, first)
