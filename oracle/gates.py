"""Gate table of the FP64 reference (test infrastructure only).

Standard textbook one-qubit gates; rotations are R_P(theta) = exp(-i theta P / 2)
for the Pauli matrix P, the reading taken for the rotation gates the paper's
random-circuit workload names (Sec. 2.2 "Random Circuits").  U3 is the
three-angle form U3(theta, phi, lambda) =
[[cos(theta/2), -e^{i lambda} sin(theta/2)], [e^{i phi} sin(theta/2), e^{i(phi+lambda)} cos(theta/2)]].
This table is independent of the HIP library's own gate table.
"""
import math

import numpy as np

_SQ2 = 1.0 / math.sqrt(2.0)


def matrix(name, params=(), mat=None):
    """2^k x 2^k complex128 matrix of a gate (controls excluded)."""
    p = tuple(params)
    if name == "h":
        return np.array([[_SQ2, _SQ2], [_SQ2, -_SQ2]], dtype=np.complex128)
    if name == "x":
        return np.array([[0, 1], [1, 0]], dtype=np.complex128)
    if name == "y":
        return np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
    if name == "z":
        return np.array([[1, 0], [0, -1]], dtype=np.complex128)
    if name == "s":
        return np.array([[1, 0], [0, 1j]], dtype=np.complex128)
    if name == "t":
        return np.array([[1, 0], [0, np.exp(1j * math.pi / 4)]], dtype=np.complex128)
    if name == "rx":
        c, s = math.cos(p[0] / 2), math.sin(p[0] / 2)
        return np.array([[c, -1j * s], [-1j * s, c]], dtype=np.complex128)
    if name == "ry":
        c, s = math.cos(p[0] / 2), math.sin(p[0] / 2)
        return np.array([[c, -s], [s, c]], dtype=np.complex128)
    if name == "rz":
        return np.array([[np.exp(-0.5j * p[0]), 0], [0, np.exp(0.5j * p[0])]], dtype=np.complex128)
    if name == "p":
        return np.array([[1, 0], [0, np.exp(1j * p[0])]], dtype=np.complex128)
    if name == "u3":
        th, ph, la = p
        c, s = math.cos(th / 2), math.sin(th / 2)
        return np.array([[c, -np.exp(1j * la) * s],
                         [np.exp(1j * ph) * s, np.exp(1j * (ph + la)) * c]], dtype=np.complex128)
    if name == "matrix":
        return np.ascontiguousarray(np.asarray(mat, dtype=np.complex128))
    raise ValueError(f"unknown gate {name!r}")


PAULI = {
    "I": np.eye(2, dtype=np.complex128),
    "X": matrix("x"),
    "Y": matrix("y"),
    "Z": matrix("z"),
}
