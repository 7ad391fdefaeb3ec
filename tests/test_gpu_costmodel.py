"""Learned sweep cost model: GPU training kernels against the FP64 reference,
FP16 inference accuracy, learned planning correctness, and what the trained
network gains over the greedy plan on the 30-qubit SU(4) workload."""
import numpy as np
import pytest

import oracle
import workloads as W
from oracle import mlp

from paper_2511_14664_amd import _binding as B

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def data(n, seed):
    rng = np.random.default_rng(seed)
    X = rng.uniform(0, 1, (n, mlp.F)).astype(np.float32)
    y = (np.sin(3 * X[:, 0]) + X[:, 5] * X[:, 9] - 0.5 * X[:, 2]).astype(np.float32)
    return X, y


def test_param_count_matches_reference():
    assert B.sv_costmodel_num_params() == mlp.num_params() == 4929


def test_gpu_gradient_matches_reference():
    m = B.sv_costmodel_create(11)
    try:
        p = B.sv_costmodel_get_params(m)
        for n in (1, 7, 300, 5000):
            X, y = data(n, n)
            L, g = B.sv_costmodel_grad(m, X, y)
            Lr, gr = mlp.grad(p.astype(np.float64), X.astype(np.float64), y.astype(np.float64))
            assert abs(L - Lr) <= 1e-5 * max(1.0, abs(Lr)), (n, L, Lr)
            err = np.max(np.abs(g - gr)) / max(1e-12, np.max(np.abs(gr)))
            assert err <= 1e-4, (n, err)
    finally:
        B.sv_costmodel_destroy(m)


def test_fp16_inference_matches_reference_forward():
    m = B.sv_costmodel_create(12)
    try:
        X, y = data(2000, 3)
        B.sv_costmodel_train(m, X, y, 200, 3e-3)
        p = B.sv_costmodel_get_params(m).astype(np.float64)
        got = B.sv_costmodel_predict(m, X)
        want = mlp.forward(p, X.astype(np.float64))
        assert np.max(np.abs(got - want)) <= 2e-2 * max(1.0, np.max(np.abs(want)))
    finally:
        B.sv_costmodel_destroy(m)


def test_adam_steps_match_reference():
    m = B.sv_costmodel_create(13)
    try:
        X, y = data(500, 4)
        p = B.sv_costmodel_get_params(m).astype(np.float64)
        mo = np.zeros_like(p)
        vo = np.zeros_like(p)
        for t in range(1, 6):
            _, g = mlp.grad(p, X.astype(np.float64), y.astype(np.float64))
            p, mo, vo = mlp.adam_step(p, mo, vo, g, t, lr=1e-3)
        B.sv_costmodel_train(m, X, y, 5, 1e-3)
        got = B.sv_costmodel_get_params(m).astype(np.float64)
        # Adam moves every weight by ~lr per step whatever the gradient's size,
        # so a gradient that is zero up to rounding may step either way: almost
        # all weights must agree closely, none by more than the 5 steps allow
        d = np.abs(got - p)
        assert np.mean(d > 1e-4) < 0.01 and np.max(d) <= 5 * 2e-3
    finally:
        B.sv_costmodel_destroy(m)


def test_training_reduces_loss_and_rejects_bad_data():
    m = B.sv_costmodel_create(14)
    try:
        X, y = data(3000, 5)
        L0, _ = B.sv_costmodel_grad(m, X, y)
        B.sv_costmodel_train(m, X, y, 500, 3e-3)
        L1, _ = B.sv_costmodel_grad(m, X, y)
        assert L1 < 0.2 * L0
        Xb = X.copy()
        Xb[3, 2] = np.nan
        with pytest.raises(B.SvError):
            B.sv_costmodel_train(m, Xb, y, 1, 1e-3)
    finally:
        B.sv_costmodel_destroy(m)


def collect(n, dtype, gates, widths=(1, 2, 3, 4, 5, 6), plain=True, passes=True):
    """Sweep timings the library records itself (HIP events), as features and
    ln(ms per GB of algorithmic traffic): greedy plans of the given widths, the
    plain plan and the LDS pass plan."""
    h = B.sv_create(n, dtype)
    circ = B.Circuit(gates)
    try:
        B.sv_apply_circuit(h, circ, B.make_opts(B.SV_PLAN_GREEDY, 3))  # warm-up: code objects loaded
        B.sv_profile_read(h)
        B.sv_profile_enable(h, True)
        for k in widths:
            B.sv_reset(h)
            B.sv_apply_circuit(h, circ, B.make_opts(B.SV_PLAN_GREEDY, k))
        if plain:
            B.sv_reset(h)
            B.sv_apply_circuit(h, circ, B.make_opts(B.SV_PLAN_PLAIN))
        if passes:
            B.sv_reset(h)
            B.sv_apply_circuit(h, circ, B.make_opts(B.SV_PLAN_PASSES))
        recs, cnt = B.sv_profile_read_raw(h)
        X = B.sv_sweep_features(n, dtype, recs, cnt)
        y = B.sv_sweep_targets(recs, cnt)
        return X, y
    finally:
        B.sv_destroy(h)


def time_circuit(n, dtype, circ, opts, model=None, reps=2):
    import time

    h = B.sv_create(n, dtype)
    try:
        if model is not None:
            B.sv_set_costmodel(h, model)
        B.sv_apply_circuit(h, circ, opts)
        B.sv_synchronize(h)
        ts = []
        for _ in range(reps):
            B.sv_reset(h)
            B.sv_synchronize(h)
            t0 = time.perf_counter()
            st = B.sv_apply_circuit(h, circ, opts)
            B.sv_synchronize(h)
            ts.append(time.perf_counter() - t0)
        amp = B.sv_copy_to_host(h, n, dtype, 0, 4)
        return min(ts), st, amp
    finally:
        B.sv_destroy(h)


def test_learned_plan_is_correct_and_falls_back_without_model():
    n = 14
    gates = W.u3_su4_layers(n, 6, 3)
    want = oracle.run(gates, n)
    m = B.sv_costmodel_create(15)
    try:
        for dtype, tol in ((B.SV_C128, 1e-12), (B.SV_C64, 2e-5)):
            h = B.sv_create(n, dtype)
            try:
                B.sv_apply_circuit(h, gates, B.make_opts(B.SV_PLAN_LEARNED, 5))  # no model: greedy
                assert np.max(np.abs(B.sv_copy_to_host(h, n, dtype) - want)) <= tol
                B.sv_set_costmodel(h, m)
                B.sv_reset(h)
                B.sv_apply_circuit(h, gates, B.make_opts(B.SV_PLAN_LEARNED, 5))
                assert np.max(np.abs(B.sv_copy_to_host(h, n, dtype) - want)) <= tol
            finally:
                B.sv_destroy(h)
        k, pred = B.sv_costmodel_rank(m, n, B.SV_C64, gates, 5)
        assert 0 <= k <= 5 and len(pred) == 6 and np.all(np.isfinite(pred))
        assert pred[k - 1 if k else 5] == np.min(pred)
    finally:
        B.sv_costmodel_destroy(m)


def test_learned_planner_vs_greedy_on_30q_su4():
    """Train on timings of the 12-qubit and 28-qubit layered workloads (greedy
    widths 1..6, plain, passes), then plan the 30-qubit U3 + SU(4) circuit
    (depth 40, complex64).  Reports the wall time of the greedy and learned
    plans and the model's error on held-out sweeps."""
    Xs, ys = [], []
    for n, dtype, ent in ((12, B.SV_C128, "cx"), (28, B.SV_C64, "cx_or_cz"), (28, B.SV_C128, "cx_or_cz")):
        X, y = collect(n, dtype, W.layered_u3_pairing(n, 20, W.circuit_seed(1 if n == 12 else 2, 1), ent))
        Xs.append(X)
        ys.append(y)
    X = np.concatenate(Xs)
    y = np.concatenate(ys)
    say(f"training samples: {len(y)}")
    m = B.sv_costmodel_create(16)
    try:
        loss = B.sv_costmodel_train(m, X, y, 3000, 3e-3)
        say(f"training loss (ln ms)^2: {loss:.4f}")
        n = 30
        gates = W.u3_su4_layers(n, 40, W.circuit_seed(5, 1))
        circ = B.Circuit(gates)
        k, pred = B.sv_costmodel_rank(m, n, B.SV_C64, circ, 6)
        tg, sg, ag = time_circuit(n, B.SV_C64, circ, B.make_opts(B.SV_PLAN_GREEDY, 5))
        tl, sl, al = time_circuit(n, B.SV_C64, circ, B.make_opts(B.SV_PLAN_LEARNED, 6), model=m)
        say(f"30q SU(4): predicted ms by width 1..6, passes {np.round(pred, 1)}, chose {k or 'passes'}; greedy(5) {tg * 1e3:.1f} ms "
            f"({sg['sweeps']} sweeps), learned {tl * 1e3:.1f} ms ({sl['sweeps']} sweeps), gain {tg / tl:.3f}x")
        assert np.max(np.abs(ag - al)) <= 4e-5  # equal accuracy: same amplitudes within the complex64 bound
        assert tl <= 1.25 * tg
        # held-out: the model's fit on the evaluation workload's own sweeps, and
        # whether it ranks whole plans (widths 3..6) the way their measured
        # wall times do
        Xe, ye = collect(n, B.SV_C64, gates, widths=(3, 5), plain=False)
        pe = B.sv_costmodel_predict(m, Xe)
        mae = float(np.mean(np.abs(pe - ye)))
        # plans: greedy widths 3..6 and the pass plan (prediction index 6)
        cands = [(w, B.make_opts(B.SV_PLAN_GREEDY, w)) for w in (3, 4, 5, 6)] + [(0, B.make_opts(B.SV_PLAN_PASSES))]
        meas = [time_circuit(n, B.SV_C64, circ, o, reps=1)[0] for _, o in cands]
        pr = np.argsort(np.argsort([pred[w - 1] if w else pred[6] for w, _ in cands]))
        mr = np.argsort(np.argsort(meas))
        rho = float(np.corrcoef(pr, mr)[0, 1])
        say(f"held-out: mean |ln pred - ln meas| (ms/GB) = {mae:.3f}; plans [3, 4, 5, 6, passes]: measured ms "
            f"{np.round(np.array(meas) * 1e3, 1)}, Spearman(pred, meas) = {rho:.2f}")
        assert mae < 0.5
        assert rho >= 0.7
    finally:
        B.sv_costmodel_destroy(m)
