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
    assert B.sv_costmodel_num_params() == mlp.num_params() == 5313


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
    plain plan, and LDS pass plans of 5..8 pass qubits with and without the
    gate-order search, in every block arithmetic and tile width the pass
    kernels have."""
    h = B.sv_create(n, dtype)
    circ = B.Circuit(gates)
    try:
        B.sv_apply_circuit(h, circ, B.make_opts(B.SV_PLAN_GREEDY, 3))  # warm-up: code objects loaded
        B.sv_profile_read(h)
        B.sv_profile_enable(h, True)
        runs = [B.make_opts(B.SV_PLAN_GREEDY, k) for k in widths]
        if plain:
            runs.append(B.make_opts(B.SV_PLAN_PLAIN))
        if passes:
            T0 = 12 if dtype == B.SV_C64 else 11
            precs = (B.SV_PREC_NATIVE, B.SV_PREC_BF16X6) if dtype == B.SV_C64 else (B.SV_PREC_NATIVE,)
            for pq in (5, 6, 7, 8):
                for orders in (-1, 8):
                    for prec in precs:
                        tiles = (T0,) if prec == B.SV_PREC_BF16X6 or n < T0 + 7 else (T0, T0 + 1)
                        for tile in tiles:
                            runs.append(B.make_opts(B.SV_PLAN_PASSES, 5, prec, pq, orders, tile))
        X, y = [], []
        for o in runs:
            B.sv_reset(h)
            B.sv_apply_circuit(h, circ, o)
            recs, cnt = B.sv_profile_read_raw(h, 1 << 14)
            X.append(B.sv_sweep_features(n, dtype, recs, cnt))
            y.append(B.sv_sweep_targets(recs, cnt))
        return np.concatenate(X), np.concatenate(y)
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
                # the same structure again (the ranking is kept on the
                # handle), with fresh angles, and after a relayout
                gates2 = W.u3_su4_layers(n, 6, 3)
                for g in range(len(gates2)):
                    if gates2[g].name == "u3":
                        gates2[g] = W.Gate("u3", gates2[g].targets, (), (0.1 * g, 0.2, -0.3 * g))
                want2 = oracle.run(gates2, n)
                for relayout in (False, True):
                    B.sv_reset(h)
                    if relayout:
                        B.sv_swap_bits(h, 0, n - 6, 6)
                    B.sv_apply_circuit(h, gates2, B.make_opts(B.SV_PLAN_LEARNED, 5))
                    assert np.max(np.abs(B.sv_copy_to_host(h, n, dtype) - want2)) <= tol
            finally:
                B.sv_destroy(h)
        k, pred = B.sv_costmodel_rank(m, n, B.SV_C64, gates, 5)
        assert 0 <= k <= 5 and len(pred) == 6 and np.all(np.isfinite(pred))
        assert pred[k - 1 if k else 5] == np.min(pred)
    finally:
        B.sv_costmodel_destroy(m)


@pytest.fixture(scope="module")
def trained_model():
    """A model trained on the timings of the 12-qubit complex128 and the
    28-qubit complex64 / complex128 layered workloads (configurations 1-2)."""
    Xs, ys = [], []
    for n, dtype, ent in ((12, B.SV_C128, "cx"), (28, B.SV_C64, "cx_or_cz"), (28, B.SV_C128, "cx_or_cz")):
        X, y = collect(n, dtype, W.layered_u3_pairing(n, 20, W.circuit_seed(1 if n == 12 else 2, 1), ent))
        Xs.append(X)
        ys.append(y)
    say(f"training samples: {sum(len(y) for y in ys)}")
    m = B.sv_costmodel_create(16)
    loss = B.sv_costmodel_train(m, np.concatenate(Xs), np.concatenate(ys), 4000, 3e-3)
    say(f"training loss (ln ms/GB)^2: {loss:.4f}")
    yield m
    B.sv_costmodel_destroy(m)


def best_of(n, dtype, circ, opts, model=None, reps=5):
    """Median wall time of a circuit after one untimed application (the plan
    of this structure is then kept on the handle), and its first amplitudes."""
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
        return float(np.median(ts)), st, B.sv_copy_to_host(h, n, dtype, 0, 4096)
    finally:
        B.sv_destroy(h)


@pytest.mark.parametrize("workload", ["28q-layered", "30q-su4"])
def test_learned_plan_vs_the_best_fixed_heuristic(trained_model, workload):
    """The learned plan against the heuristic LDS pass plan (the best fixed
    plan: faster than greedy fusion on both workloads) at equal accuracy, in
    the benchmark's block arithmetic.  The 28-qubit layered circuit is the
    training configuration's own circuit; the 30-qubit U3 + SU(4) circuit
    (depth 40) is held out.  Both plans are kept per structure on the handle,
    so the timed runs pay no planning."""
    if workload == "28q-layered":
        n, gates = 28, W.layered_u3_pairing(28, 20, W.circuit_seed(2, 1), "cx_or_cz")
    else:
        n, gates = 30, W.u3_su4_layers(30, 40, W.circuit_seed(5, 1))
    circ = B.Circuit(gates)
    prec = B.SV_PREC_BF16X6
    tg, sg, _ = best_of(n, B.SV_C64, circ, B.make_opts(B.SV_PLAN_GREEDY, 5, prec), reps=3)
    tp, sp, ap = best_of(n, B.SV_C64, circ, B.make_opts(B.SV_PLAN_PASSES, 5, prec))
    tl, sl, al = best_of(n, B.SV_C64, circ, B.make_opts(B.SV_PLAN_LEARNED, 5, prec), model=trained_model)
    k, pred = B.sv_costmodel_rank(trained_model, n, B.SV_C64, circ, 5)
    say(f"{workload}: greedy(5) {tg * 1e3:.1f} ms ({sg['sweeps']} sweeps), passes {tp * 1e3:.1f} ms "
        f"({sp['sweeps']} sweeps), learned {tl * 1e3:.1f} ms ({sl['sweeps']} sweeps, choice {k or 'passes'}): "
        f"{tp / tl:.3f}x the pass heuristic, {tg / tl:.3f}x greedy; predicted ms by width 1..5, passes "
        f"{np.round(pred, 1)}")
    assert np.max(np.abs(ap - al)) <= 4e-5  # equal accuracy: the same amplitudes within the complex64 bound
    assert tp < tg
    # no slower than the best fixed plan beyond the run-to-run spread of a
    # median of five (about 1 %)
    assert tl <= 1.02 * tp


def test_learned_model_predicts_held_out_pass_times(trained_model):
    """Held out: the model's error on the 30-qubit SU(4) workload's own pass
    and sweep timings, and whether it ranks whole plans (greedy widths 3..6
    and the heuristic pass plan) the way their measured wall times do."""
    n = 30
    gates = W.u3_su4_layers(n, 40, W.circuit_seed(5, 1))
    circ = B.Circuit(gates)
    Xe, ye = collect(n, B.SV_C64, gates, widths=(3, 5), plain=False)
    pe = B.sv_costmodel_predict(trained_model, Xe)
    mae = float(np.mean(np.abs(pe - ye)))
    k, pred = B.sv_costmodel_rank(trained_model, n, B.SV_C64, circ, 6)
    cands = [(w, B.make_opts(B.SV_PLAN_GREEDY, w)) for w in (3, 4, 5, 6)]
    meas = [best_of(n, B.SV_C64, circ, o, reps=1)[0] for _, o in cands]
    pr = np.argsort(np.argsort([pred[w - 1] for w, _ in cands]))
    mr = np.argsort(np.argsort(meas))
    rho = float(np.corrcoef(pr, mr)[0, 1])
    say(f"held-out 30q SU(4): mean |ln pred - ln meas| (ms/GB) = {mae:.3f} over {len(ye)} sweeps; greedy "
        f"widths [3, 4, 5, 6]: measured ms {np.round(np.array(meas) * 1e3, 1)}, predicted "
        f"{np.round([pred[w - 1] for w, _ in cands], 1)}, Spearman {rho:.2f}")
    assert mae < 0.5
    assert rho >= 0.7
