"""Rounding-error bounds of the GPU path, from its arithmetic.

Used by the GPU parity tests to bound the state error against the FP64
oracle (complex64: u = 2^-24; the complex128 path performs the same
operations in FP64, u = 2^-53).  Every constant below follows from the operations the kernels
perform; none is fitted to an observed error.

Notation: u = 2^-24 (FP32 unit roundoff).  A sweep applies a d x d block
U = A + iB (FP64 product of the block's gates, unitary to ~1e-15, stored in
FP32) to each group v = x + iz of d amplitudes.  With T = (|A| + |B|)(|x| + |z|)
(entrywise moduli), ||T||_2 <= || |A| + |B| ||_F * sqrt(2) ||v||_2
<= sqrt(2 d) * sqrt(2) ||v||_2 = 2 sqrt(d) ||v||_2, since
sum (|A_ij| + |B_ij|)^2 <= 2 ||U||_F^2 = 2 d for a unitary U.

* Three-product form on the matrix cores (pass blocks, dense blocks of k >= 3,
  d = max(16, 2^k)): P1 = A x, P2 = B z, P3 = fl(A + B) fl(x + z), each a
  d-term dot product accumulated in the matrix core; Re = fl(P1 - P2),
  Im = fl(fl(P3 - P1) - P2) on the vector unit.  The matrix core's
  accumulation is charged 2 u per addition (covering truncating as well as
  round-to-nearest adders), the vector unit u.  With matrix entries carrying
  a relative error of at most m u (m = 1 for rounding to FP32; m = 8 once a
  pass rotates an entry by per-tile phases: FP32 sin/cos, two products and a
  sum), to first order |dRe| <= (2 d + m + 1) u T_i and
  |dIm| <= (4 d + 2 m + 5) u T_i, so
      eps_3M(d) = 2 sqrt(d) u sqrt((2 d + 9)^2 + (4 d + 21)^2)     (m = 8).
* Split BF16 form (SV_PREC_BF16X6 pass blocks, d = 16): both operands split
  exactly into three BF16 parts, each output row a sum of K = 2 d real
  products [Ur, -Ui] [x; z] or [Ui, Ur] [x; z] taken as six part products
  (the three dropped ones are below 2 u |a b| per product), accumulated in
  six matrix-core steps of K + 1 terms smallest first, so the last step (the
  products of the high parts) dominates: |dRe|, |dIm| <= (2 (2 d + 2) + 2 + m)
  u T_i, and
      eps_split(d) = 2 sqrt(d) u sqrt(2) (4 d + 14).
* Four-product form on the vector units (one-qubit sweeps, small-tile
  blocks, per-group blocks): each real output is a 2d-term dot product plus
  the matrix rounding, |dRe|, |dIm| <= (2 d + 2) u T_i, so
      eps_4M(d) = sqrt(2) (2 d + 2) u 2 sqrt(d).
* Diagonal one-qubit sweep: one complex product per amplitude,
  eps_diag = 5 u.  The index-bit exchange moves bytes: eps = 0.

Unitarity keeps earlier errors from growing, so after sweeps j = 1..N
||dpsi||_2 <= sum_j eps_j (to first order): the deterministic bound.

Under the probabilistic model of rounding (Higham and Mary, SIAM J. Sci.
Comput. 41(5), 2019: independent mean-zero rounding errors, so an n-term
error sum stays below lambda sqrt(n) u sum|a_k b_k| with probability at least
1 - 2 n exp(-lambda^2 (1 - u)^2 / 2)), each coefficient c above becomes
lambda sqrt(c), and the errors of different sweeps add in quadrature:
||dpsi||_2 <= sqrt(sum_j epsp_j^2), lambda = 6.  A random circuit spreads
each sweep's error over all 2^n amplitudes (its output amplitudes follow the
Porter-Thomas distribution), so each amplitude's error has standard deviation
||dpsi||_2 / 2^(n/2) and the largest of the 2^n stays below
sqrt(2 ln 2^(n+1)) times that with high probability: the per-amplitude bound
used for the relative error of the larger amplitudes.
"""
import math

U32 = 2.0 ** -24
U64 = 2.0 ** -53
LAMBDA = 6.0


def _d_of(rec):
    k = rec["k"]
    return 1 << k


def _eps(kind, d, probabilistic, u):
    """Bound on ||d y||_2 / ||v||_2 for one block of one sweep."""
    if kind == "3m":
        cr, ci = 2 * d + 9, 4 * d + 21
        scale = 2 * math.sqrt(d) * u
    elif kind == "split":
        cr = ci = 4 * d + 14
        scale = 2 * math.sqrt(d) * u
    elif kind == "4m":
        cr = ci = 2 * d + 2
        scale = 2 * math.sqrt(d) * u
    elif kind == "diag":
        return (LAMBDA * math.sqrt(5.0) if probabilistic else 5.0) * u
    else:
        return 0.0
    if probabilistic:
        return LAMBDA * math.sqrt(cr + ci) * scale
    return math.hypot(cr, ci) * scale


def sweep_terms(rec, n):
    """(kind, d, count) of the blocks one recorded sweep applies."""
    name = rec["kind_name"]
    if name == "pass":
        blocks = int(round(rec["flops"] / (126.0 * 2.0 ** n)))
        return ("split" if rec.get("precision") == 2 else "3m"), 16, blocks
    if name in ("dense_mfma",):
        return "3m", max(16, _d_of(rec)), 1
    if name in ("dense_tile", "dense_group"):
        return "4m", _d_of(rec), 1
    if name == "gate1":
        return "4m", 2, 1
    if name == "diag1":
        return "diag", 2, 1
    if name == "bitswap":
        return "exact", 0, 0
    raise ValueError(f"no rounding model for sweep kind {name}")


def state_bounds(records, n, complex64=True):
    """(deterministic, probabilistic) bounds on ||dpsi||_2 after the sweeps
    in `records` (sv_profile_read dicts) on an n-qubit state."""
    u = U32 if complex64 else U64
    det, prob2 = 0.0, 0.0
    for r in records:
        kind, d, cnt = sweep_terms(r, n)
        det += cnt * _eps(kind, d, False, u)
        prob2 += cnt * _eps(kind, d, True, u) ** 2
    return det, math.sqrt(prob2)


def oracle_bounds(gates):
    """(deterministic, probabilistic) bounds on the FP64 oracle's own
    ||dpsi||_2: each gate is one unfused application of its 2^k x 2^k matrix
    in the four-product form (u = 2^-53)."""
    det, prob2 = 0.0, 0.0
    for g in gates:
        if not hasattr(g, "name"):
            continue
        d = 1 << len(g.targets)
        det += _eps("4m", d, False, U64)
        prob2 += _eps("4m", d, True, U64) ** 2
    return det, math.sqrt(prob2)


def amplitude_bound(prob_l2, n):
    """Probabilistic bound on max_i |d a_i| for a random circuit's state."""
    return math.sqrt(2.0 * math.log(2.0) * (n + 1)) * prob_l2 / 2.0 ** (n / 2.0)


def state_l2(got, want, chunk=1 << 24):
    """max |d a| and ||d psi||_2 of a GPU state against the oracle's, in FP64."""
    import numpy as np

    mx, l2 = 0.0, 0.0
    for i in range(0, want.size, chunk):
        d = np.abs(np.asarray(got[i:i + chunk], dtype=np.complex128) - want[i:i + chunk])
        mx = max(mx, float(d.max()))
        l2 += float(np.dot(d, d))
    return mx, math.sqrt(l2)


def check_state(got, want, complex64, n, records, gates=(), random_circuit=False):
    """Assert max |d a| <= 1e-12 / 2e-5 and ||d psi||_2 within the rounding
    bound of the recorded sweeps plus the oracle's own gates (the
    probabilistic bound for a random circuit, else the deterministic one).
    Returns (max |d a|, ||d psi||_2, bound)."""
    mx, l2 = state_l2(got, want)
    det, prob = state_bounds(records, n, complex64)
    odet, oprob = oracle_bounds(gates)
    bound = math.hypot(prob, oprob) if random_circuit else det + odet
    assert mx <= (2e-5 if complex64 else 1e-12), (mx, l2, bound)
    assert l2 <= bound, (mx, l2, bound)
    return mx, l2, bound


def mirror_l2(norm2, a0, n):
    """||psi - |0...0>||_2 from the state's squared norm (an FP64 sum of 2^n
    terms) and its first amplitude, as sqrt(||psi||^2 - 2 Re a_0 + 1), with
    the resolution of that expression: the norm's FP64 sum carries an error
    up to (n + 1) 2^-53 (a tree of depth <= n) and the three-term sum adds
    3 * 2^-53 relative to its O(1) terms.  Returns (value, resolution)."""
    val = math.sqrt(max(0.0, norm2 - 2.0 * complex(a0).real + 1.0))
    res = math.sqrt(3.0 * (n + 4) * U64)
    return val, res
