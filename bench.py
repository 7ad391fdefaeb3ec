#!/usr/bin/env python3
"""Throughput of the state-vector gate-application path on one MI355X.

One step = one pass of the hot path over the 28-qubit complex64 layered random
circuit (U3 on every qubit + CNOT/CZ on a random matching, depth 20, 840
gates): reset to |0...0>, fusion planning, the fused sweeps, one in-place
exchange of the top 6 index bits with the lowest 6 (the single-device part of
the global/local qubit swap), then the read-outs: a 10-qubit marginal,
<Z_i> and <Z_i Z_i+1> expectation values, and 1000 shots.  The state lives in
HBM for the whole run; the timed region excludes circuit generation.

Prints one JSON line.  `value` is unfused gate applications per second.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "gate-apps/s & achieved HBM GB/s at 28–34 qubits, fused vs plain, 1 GPU"
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--qubits", type=int, default=28)
    ap.add_argument("--dtype", choices=["c64", "c128"], default="c64")
    ap.add_argument("--mode", choices=["plain", "greedy", "learned"], default="greedy")
    ap.add_argument("--max-fused", type=int, default=5)
    ap.add_argument("--no-plain", action="store_true", help="skip the plain (unfused) comparison run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain device copy of the state size (HBM counter calibration)")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1 "
                                   "(the multi-GPU exchange is described in DESIGN.md, not built)"}))
        sys.exit(2)

    import numpy as np
    import torch

    import workloads as W
    import paper_2511_14664_amd as svm
    from paper_2511_14664_amd import _binding as B

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)

    n = args.qubits
    dtype = B.SV_C64 if args.dtype == "c64" else B.SV_C128
    S = 8 if dtype == B.SV_C64 else 16
    gates = W.layered_u3_pairing(n, 20, W.circuit_seed(2, 1), "cx_or_cz")
    circ = B.Circuit(gates)
    mode = {"plain": B.SV_PLAN_PLAIN, "greedy": B.SV_PLAN_GREEDY, "learned": B.SV_PLAN_LEARNED}[args.mode]
    opts = B.make_opts(mode, args.max_fused)
    marg_q = list(range(n - 10, n))
    terms = W.hea_z_terms(n)[: 2 * 16]
    uni = W.uniforms(7, 1000)

    sv = svm.StateVector(n, dtype, device=0)
    stream = sv.stream

    def step(profile=False):
        B.sv_reset(sv.handle)
        st = B.sv_apply_circuit(sv.handle, circ, opts)
        B.sv_swap_bits(sv.handle, 0, n - 6, 6)
        B.sv_probabilities(sv.handle, marg_q)
        B.sv_expect_pauli(sv.handle, terms)
        B.sv_sample(sv.handle, uni)
        return st

    log(f"bench: {n} qubits {args.dtype} mode={args.mode} k<={args.max_fused}, {len(gates)} gates")
    for i in range(args.warmup):
        step()
        log(f"warmup {i} done")
    B.sv_profile_read(sv.handle)  # drop anything recorded so far
    torch.cuda.synchronize()

    B.sv_profile_enable(sv.handle, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = None
    for i in range(args.steps):
        stats = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    B.sv_profile_enable(sv.handle, False)
    recs = B.sv_profile_read(sv.handle, 1 << 18)
    ms_step = (t1 - t0) * 1e3 / args.steps
    gate_apps = len(gates) / (ms_step / 1e3)
    log(f"timed {args.steps} steps: {ms_step:.3f} ms/step, {gate_apps:.1f} gate-apps/s")

    # per-kernel-class totals from the live HIP-event records
    classes = {}
    for r in recs:
        key = (r["kind_name"], r["k"])
        c = classes.setdefault(key, {"ms": 0.0, "bytes": 0.0, "flops": 0.0, "launches": 0})
        c["ms"] += r["ms"]
        c["bytes"] += r["bytes"]
        c["flops"] += r["flops"]
        c["launches"] += 1
    sweep_ms = sum(c["ms"] for c in classes.values()) / args.steps
    sweep_bytes = sum(c["bytes"] for c in classes.values()) / args.steps
    dom_key = max(classes, key=lambda k: classes[k]["ms"])
    dom = classes[dom_key]
    avg_ms = dom["ms"] / dom["launches"]
    avg_bytes = dom["bytes"] / dom["launches"]
    achieved = avg_bytes / (avg_ms / 1e3) / 1e9
    breakdown = {f"{k[0]}_k{k[1]}": {"launches_per_step": v["launches"] / args.steps,
                                      "ms_per_step": round(v["ms"] / args.steps, 4),
                                      "GB/s": round(v["bytes"] / (v["ms"] / 1e3) / 1e9, 1) if v["ms"] > 0 else None}
                 for k, v in sorted(classes.items(), key=lambda kv: -kv[1]["ms"])}

    plain = None
    if not args.no_plain and args.mode != "plain":
        popts = B.make_opts(B.SV_PLAN_PLAIN)
        B.sv_reset(sv.handle)
        B.sv_apply_circuit(sv.handle, circ, popts)
        torch.cuda.synchronize()
        B.sv_profile_enable(sv.handle, True)
        t0 = time.perf_counter()
        B.sv_reset(sv.handle)
        pst = B.sv_apply_circuit(sv.handle, circ, popts)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        B.sv_profile_enable(sv.handle, False)
        precs = B.sv_profile_read(sv.handle, 1 << 18)
        p_ms = (t1 - t0) * 1e3
        p_kernel_ms = sum(r["ms"] for r in precs)
        p_bytes = sum(r["bytes"] for r in precs)
        g1 = [r for r in precs if r["kind_name"] == "gate1" and r["c"] == 0]
        g1_gbs = (sum(r["bytes"] for r in g1) / (sum(r["ms"] for r in g1) / 1e3) / 1e9) if g1 else None
        plain = {"ms_per_circuit": round(p_ms, 3), "gate_apps_per_s": round(len(gates) / (p_ms / 1e3), 1),
                 "sweeps": pst["sweeps"], "kernel_GB/s": round(p_bytes / (p_kernel_ms / 1e3) / 1e9, 1),
                 "dense_1q_GB/s": round(g1_gbs, 1) if g1_gbs else None}
        log(f"plain: {plain}")

    copy_cal = None
    if args.calibrate_copy:
        a = torch.empty(S << n, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        af, bf = a.view(torch.float32), b.view(torch.float32)
        torch.mul(af, 1.0, out=bf)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            torch.mul(af, 1.0, out=bf)
        e1.record()
        torch.cuda.synchronize()
        cms = e0.elapsed_time(e1) / 5
        copy_cal = {"bytes_per_launch": 2 * (S << n), "ms": round(cms, 4),
                    "GB/s": round(2 * (S << n) / (cms / 1e3) / 1e9, 1)}
        log(f"copy calibration: {copy_cal}")
        del a, b

    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        log("cpu baseline: FP64 reference on the same circuit (bounded sample) ...")
        a = oracle.zero_state(n)
        t0 = time.perf_counter()
        done = 0
        for g in gates:
            oracle.apply_gate(a, g)
            done += 1
            if done >= 3 and time.perf_counter() - t0 > args.cpu_seconds:
                break
        dt = time.perf_counter() - t0
        cpu = {"value": round(done / dt, 3), "unit": "gate-apps/s", "cores": oracle.num_threads(),
               "kind": "oracle",
               "sample": f"first {done} of the {len(gates)} gates of the same {n}-qubit circuit, "
                         f"unfused, FP64 complex128, {dt:.1f} s on host cores"}
        del a
        log(f"cpu baseline: {cpu}")

    out = {
        "metric": METRIC,
        "value": round(gate_apps, 2),
        "unit": "gate-apps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32" if dtype == B.SV_C64 else "fp64",
        "data": "synthetic",
        "config": {"workload": f"{n}-qubit random layered circuit (U3 on every qubit + CNOT/CZ on a random "
                               f"matching, depth 20, {len(gates)} gates), {args.dtype}, {args.mode} fusion "
                               f"<= {args.max_fused} qubits, + 6-bit index exchange, 10-qubit marginal, "
                               f"{len(terms)} Z-string expectations, 1000 shots",
                   "qubits": n, "state_bytes": S << n, "gates": len(gates),
                   "sweeps_per_step": stats["sweeps"] if stats else None, "parallelism": "single GPU"},
        "achieved_GB/s_all_sweeps": round(sweep_bytes / (sweep_ms / 1e3) / 1e9, 1),
        "sweep_ms_per_step": round(sweep_ms, 4),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": f"{dom_key[0]} k={dom_key[1]}", "avg_launch_ms": round(avg_ms, 5),
                     "bytes_per_launch": avg_bytes},
        "kernels": breakdown,
        "plain": plain,
        "copy_calibration": copy_cal,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    sv.close()


if __name__ == "__main__":
    main()
