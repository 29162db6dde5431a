#!/usr/bin/env python3
"""Benchmark of the batched phaseless-AFQMC walker step on one MI355X.

Workload (default): M=400 orbitals, 100+100 electrons, 1600 Cholesky vectors,
512 walkers at the trial, dt 0.005, QR every 5 steps, energy measured every
step, fields from the device Philox stream; synthetic seeded inputs
(paper_2003_01831_amd.synth, workload "m400").

Prints ONE JSON line: walker-steps/s of the headline precision (split-BF16x3
by default), the same rate for the plain FP64 path and complex FP32 on the same
GPU, the algorithmic TFLOP/s, the roofline entry of the dominant kernel (the
fused exchange contraction, timed with HIP events on the library stream), the
error against the CPU FP64 oracle on a 4-walker subset, and the oracle's own
rate on the host cores (cpu_baseline).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"fp64": 78.6, "cfp32": 157.3, "bf16x3": 2500.0}
DTYPE = {"fp64": "f64", "cfp32": "f32", "bf16x3": "bf16x3"}


def flops_per_walker_step(M, N, X, K=6, qr_every=5, real_trial=True):
    """Algorithmic flop count of one walker step (both spins, energy every step).
    The exchange and Coulomb terms use the real half-rotated Cholesky tensor of a
    real trial (4 flop per real-by-complex multiply-add); the complex-model count
    (8 flop per complex multiply-add everywhere) is returned alongside."""
    cm = 8.0
    ex_mac = 4.0 if real_trial else 8.0
    parts = {
        "overlap": cm * 2 * (N * N * M + N ** 3 + M * N * N),
        "coulomb": ex_mac * 2 * X * N * M,
        "exchange": ex_mac * 2 * X * N * N * M + cm * 2 * X * N * N,
        "abuild": 4.0 * M * M * X,
        "taylor": cm * K * M * M * 2 * N + 4.0 * 2 * M * M * 2 * N,
        "weight": cm * 2 * (N * N * M + N ** 3 / 3),
        "qr": cm * 2 * (2 * M * N * N - 2 * N ** 3 / 3) / max(qr_every, 1),
    }
    model = dict(parts)
    model["coulomb"] = 8.0 * 2 * X * N * M
    model["exchange"] = 8.0 * 2 * X * N * N * M + 8.0 * 2 * X * N * N
    return sum(parts.values()), parts, sum(model.values())


def profiled_traffic(kernel_src, profile_md, tag):
    """HBM bytes per launch of a kernel measured with rocprofv3 PMC counters
    (FETCH_SIZE/WRITE_SIZE, calibrated on a device copy) and recorded in the
    profile summary as `traffic_bytes_per_launch=B <tag>_sha256_16=H`, or None
    once the kernel source has changed since."""
    import hashlib
    import re
    try:
        sha = hashlib.sha256(open(kernel_src, "rb").read()).hexdigest()[:16]
        text = open(profile_md).read()
    except OSError:
        return None
    m = re.search(r"traffic_bytes_per_launch=(\d+) " + re.escape(tag) + r"_sha256_16=([0-9a-f]+)", text)
    if not m or m.group(2) != sha:
        return None
    return int(m.group(1))


def rel_max(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300)))


def trace_phases(lib, _lib):
    import ctypes as C
    phases = {}
    for i, name in enumerate(_lib.PHASES):
        ms, cnt = C.c_double(), C.c_int64()
        _lib.check(lib.afq_trace_query(i, C.byref(ms), C.byref(cnt)))
        phases[name] = (ms.value, cnt.value)
    return phases


def bench_uneven(a, torch, synth, api, _lib):
    """24 uneven systems (M in {32..256}, N = M/4 per spin, X = 4M, 16-128
    walkers) stepped together: every QR cycle of every system is one replay of
    a captured HIP graph whose branches are the systems."""
    shapes = synth.uneven_systems(24, seed=4000)
    dt, qr = 0.005, 5
    lib = _lib.load()
    t0 = time.perf_counter()
    pairs, e_shift = [], []
    flop_model = flop_real = 0.0
    ex_flops = 0.0
    for c in shapes:
        s = synth.make_system(c["M"], c["n_up"], c["n_dn"], c["n_chol"], seed=c["seed"])
        g = api.System.from_synth(s, precision=a.precision)
        probe = api.Walkers(g, 1)
        e_shift.append(float(probe.energy()[3][0]))
        probe.close()
        pairs.append((g, api.Walkers(g, c["n_walkers"])))
        fr, parts, fm = flops_per_walker_step(c["M"], c["n_up"], c["n_chol"], 6, qr)
        flop_model += fm * c["n_walkers"]
        flop_real += fr * c["n_walkers"]
        N = c["n_up"]
        ex_flops += 2 * (8.0 * c["n_chol"] * N * N * c["M"] + 8.0 * c["n_chol"] * N * N) * c["n_walkers"]
        del s
    nwt = sum(c["n_walkers"] for c in shapes)
    print(f"[bench] 24 systems, {nwt} walkers, built in {time.perf_counter() - t0:.1f}s", file=sys.stderr,
          flush=True)
    # per-kernel view: one eager traced step of every system (exchange launch times)
    lib.afq_trace_reset()
    lib.afq_trace_enable(1)
    for g, w in pairs:
        w.step(1, dt, seed=1, qr_every=0, e_shift=0.0, outputs=())
    torch.cuda.synchronize()
    lib.afq_trace_enable(0)
    ph = trace_phases(lib, _lib)
    lib.afq_trace_reset()
    for g, w in pairs:
        w.set(counter=0)
    b = api.Batch(pairs)
    # warm-up: eager steps up to the cycle boundary, then the graph capture
    b.step(2 * qr, dt, seed=11, qr_every=qr, e_shift=e_shift)
    torch.cuda.synchronize()
    steps = max(qr, (a.steps // qr) * qr)
    t = time.perf_counter()
    em = b.step(steps, dt, seed=11, qr_every=qr, e_shift=e_shift)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t
    value = nwt * steps / wall
    ex_ms, ex_cnt = ph["exchange"]
    achieved = ex_flops / (ex_ms / 1e3) / 1e12
    peak = PEAK_TFLOPS[a.precision]
    line = {
        "metric": "walker-steps/s + MFMA TFLOP/s, 24 uneven systems in one captured graph",
        "value": round(value, 3), "unit": "walker-steps/s", "n_gpus": 1, "steps": steps, "warmup": a.warmup,
        "ms_per_step": round(wall / steps * 1e3, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": DTYPE[a.precision], "data": "synthetic",
        "config": {"workload": f"uneven24: 24 systems, M in [32, 256], N_up=N_dn=M/4, Nchol=4M, {nwt} walkers, "
                               f"dt={dt}, QR every {qr}, graph of one QR cycle replayed",
                   "precision": a.precision, "walkers": nwt, "parallelism": "single GPU"},
        "alg_tflops": round(flop_model * steps / wall / 1e12, 3),
        "alg_tflops_real_lt": round(flop_real * steps / wall / 1e12, 3),
        "roofline": {"bound": "mfma", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
                     "frac": round(achieved / peak, 4), "traffic": None,
                     "kernel": "exchange kernels of all 24 systems (one eager traced step, sum of launch times)",
                     "launches": ex_cnt, "total_ms": round(ex_ms, 3)},
        "cpu_baseline": None,
        "eager_phase_ms_per_step": {k: round(v[0], 3) for k, v in ph.items()},
        "emix_last_mean": float(em[:, -1].mean().item()),
    }
    b.close()
    print(json.dumps(line))
    return 0


def bench_msd(a, torch, synth, api, _lib):
    """Orthogonal multi-determinant trial (256 determinants, rank <= 4 per
    spin) at M=128, 16+16 electrons, 512 Cholesky vectors, 256 walkers, FP64."""
    cfg = dict(synth.WORKLOADS["msd_m128"])
    M, nu, nd, X = cfg["M"], cfg["n_up"], cfg["n_dn"], cfg["n_chol"]
    nw = a.walkers or cfg["n_walkers"]
    dt, qr = cfg["dt"], cfg["qr_every"]
    lib = _lib.load()
    s = synth.make_system(M, nu, nd, X, seed=cfg["seed"])
    C, exc, coeffs = synth.make_msd(s, cfg["n_det"], cfg["occ_act"], cfg["vir_act"], cfg["k_max"],
                                    seed=cfg["msd_seed"])
    sysg = api.System.from_synth(s, precision="fp64")
    sysg.set_msd(C, exc, coeffs)
    probe = api.Walkers(sysg, 1)
    e_var = float(probe.energy()[3][0])
    probe.close()
    wk = api.Walkers(sysg, nw)
    wk.step(a.warmup, dt, seed=11, qr_every=qr, e_shift=e_var, outputs=())
    torch.cuda.synchronize()
    lib.afq_trace_reset()
    lib.afq_trace_enable(1)
    t = time.perf_counter()
    out = wk.step(a.steps, dt, seed=11, qr_every=qr, e_shift=e_var, outputs=("emix",))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t
    lib.afq_trace_enable(0)
    ph = trace_phases(lib, _lib)
    lib.afq_trace_reset()
    value = nw * a.steps / wall
    # the Omega GEMM: rows (X + 1) x (max(N_up, N_dn) + active virtuals of both spins), columns
    # every walker's N_up + N_dn orbitals, contraction over M; 8 flop per complex multiply-add
    nv = len({p for e in exc for sp in range(2) for p in e[sp][1]})
    nr = max(nu, nd) + nv
    om_ms, om_cnt = ph["msd_omega"]
    om_avg_s = om_ms / 1e3 / max(om_cnt, 1)
    chunks = max(om_cnt // max(a.steps, 1), 1)
    per_launch = 8.0 * (X + 1) * nr * M * (nu + nd) * nw / chunks
    achieved = per_launch / om_avg_s / 1e12
    peak = PEAK_TFLOPS["fp64"]
    cpu = None
    if not a.no_cpu:
        from oracle import msd as omsd
        dets = omsd.determinants(C, nu, nd, exc)
        W1 = synth.trial_walkers(s, 1)[0] + 0.05 * np.random.default_rng(5).standard_normal((M, nu + nd))
        nsub = 16
        tc = time.perf_counter()
        omsd.local_energy(s.h1, s.chol, dets[:nsub], coeffs[:nsub], W1, nu, nd)
        tc = time.perf_counter() - tc
        per_ws = tc * cfg["n_det"] / nsub          # one walker's energy over all determinants
        cpu = {"value": round(1.0 / per_ws, 6), "unit": "walker-steps/s", "cores": os.cpu_count(),
               "kind": "oracle",
               "sample": f"local energy of 1 walker over {nsub} of the {cfg['n_det']} determinants "
                         f"({tc:.1f}s), scaled by {cfg['n_det']}/{nsub}; excludes the propagation"}
    line = {
        "metric": "walker-steps/s, orthogonal multi-determinant trial (FP64)",
        "value": round(value, 3), "unit": "walker-steps/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": round(wall / a.steps * 1e3, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"msd_m128: M={M}, N_up=N_dn={nu}, Nchol={X}, {nw} walkers, {cfg['n_det']} "
                               f"determinants (rank <= {cfg['k_max']} per spin, active {cfg['occ_act']} occ + "
                               f"{cfg['vir_act']} virt), dt={dt}, QR every {qr}",
                   "precision": "fp64", "walkers": nw, "parallelism": "single GPU"},
        "roofline": {"bound": "mfma", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
                     "frac": round(achieved / peak, 4), "traffic": None,
                     "kernel": "[C_ref^H; C_V^H] L^g Theta GEMM (FP64 complex x complex), both spins, one walker chunk per launch",
                     "flop_per_launch": per_launch, "avg_launch_ms": round(om_avg_s * 1e3, 3),
                     "launches": om_cnt},
        "cpu_baseline": cpu,
        "phase_ms_per_step": {k: round(v[0] / a.steps, 3) for k, v in ph.items()},
        "emix_last": float(out["emix"][-1].item()),
    }
    print(json.dumps(line))
    return 0


def bench_kp(a, torch, synth, api, _lib):
    """k-point-blocked Cholesky (8 k-points, M=192, 6+6 electrons per k-point,
    96 vectors per momentum transfer), 256 walkers, FP64."""
    cfg = dict(synth.WORKLOADS["kp_m192"])
    nk, m, nu, nd, xq = cfg["nk"], cfg["m"], cfg["n_up"], cfg["n_dn"], cfg["xq"]
    nw = a.walkers or cfg["n_walkers"]
    dt, qr = cfg["dt"], cfg["qr_every"]
    M, Nu, Nd, XL = nk * m, nk * nu, nk * nd, nk * xq
    lib = _lib.load()
    ks = synth.make_kpoint_system(nk, m, nu, nd, xq, seed=cfg["seed"])
    sysg = api.System.from_kpoint(ks)
    probe = api.Walkers(sysg, 1)
    e_var = float(probe.energy()[3][0])
    probe.close()
    wk = api.Walkers(sysg, nw)
    wk.step(a.warmup, dt, seed=11, qr_every=qr, e_shift=e_var, outputs=())
    torch.cuda.synchronize()
    lib.afq_trace_reset()
    lib.afq_trace_enable(1)
    t = time.perf_counter()
    out = wk.step(a.steps, dt, seed=11, qr_every=qr, e_shift=e_var, outputs=("emix",))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t
    lib.afq_trace_enable(0)
    ph = trace_phases(lib, _lib)
    lib.afq_trace_reset()
    value = nw * a.steps / wall
    # trace kernel: per walker, spin, vector (Q, n), row block k1 and pair (a, k', b):
    # two length-m complex dot products (8 flop per multiply-add)
    tr_flop = sum(8.0 * 2 * m * (n * nk * n) * nk * XL for n in (nu, nd)) * nw
    ex_ms, ex_cnt = ph["exchange"]
    ex_avg_s = ex_ms / 1e3 / max(ex_cnt, 1)
    achieved = tr_flop / ex_avg_s / 1e12
    dense_flop = sum(2 * 8.0 * XL * (nk * n) ** 2 * M for n in (nu, nd)) * nw
    cpu = None
    if not a.no_cpu:
        from oracle import kpoint as okp
        h = okp.dense_one_body(ks.hk)
        L = okp.dense_factors(ks.Lk, ks.kq)
        T = okp.dense_trial(ks.phik, nu, nd)
        W1 = T + 0.05 * np.random.default_rng(5).standard_normal(T.shape)
        tc = time.perf_counter()
        okp.local_energy(h, L, T, W1, Nu, Nd)
        okp.force_bias(L, T, W1, Nu, Nd)
        tc = time.perf_counter() - tc
        cpu = {"value": round(1.0 / tc, 6), "unit": "walker-steps/s", "cores": os.cpu_count(), "kind": "oracle",
               "sample": f"local energy and force bias of 1 walker over the dense block vectors ({tc:.1f}s); "
                         f"excludes the propagation"}
    line = {
        "metric": "walker-steps/s, k-point-blocked Cholesky (FP64)",
        "value": round(value, 3), "unit": "walker-steps/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": round(wall / a.steps * 1e3, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"kp_m192: {nk} k-points, m={m}, {nu}+{nd} electrons per k-point (M={M}, "
                               f"N={Nu}+{Nd}), {xq} vectors per Q ({XL} complex vectors, {2 * XL} fields), "
                               f"{nw} walkers, dt={dt}, QR every {qr}",
                   "precision": "fp64", "walkers": nw, "parallelism": "single GPU"},
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_TFLOPS["fp64"], "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK_TFLOPS["fp64"], 4), "traffic": None,
                     "kernel": "k-point trace kernel (per row block and Q: Omega, Omega' blocks, FP64 VALU) "
                               "+ its row-block reduction",
                     "flop_per_launch": tr_flop, "avg_launch_ms": round(ex_avg_s * 1e3, 3), "launches": ex_cnt,
                     "dense_equivalent_flop": dense_flop},
        "cpu_baseline": cpu,
        "phase_ms_per_step": {k: round(v[0] / a.steps, 3) for k, v in ph.items()},
        "emix_last": float(out["emix"][-1].item()),
    }
    print(json.dumps(line))
    return 0


def measure_extras(a, extra, sysg, api, lib, _lib, torch, nw, dt, qr, e_var, M, nu, nd):
    """Population control and back-propagation at the headline size (outside the timed steps)."""
    # population control at this size: one comb of all walkers (host-synchronising)
    wk_pc = api.Walkers(sysg, nw)
    wk_pc.set(weights=np.random.default_rng(3).uniform(0.5, 1.5, nw))
    wk_pc.comb(0.5)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for r in range(5):
        wk_pc.comb((r + 0.5) / 5)
    torch.cuda.synchronize()
    extra["comb_ms"] = round((time.perf_counter() - t) / 5 * 1e3, 3)
    wk_pc.close()
    # back-propagated 1-RDM at this size: a window of 2 QR periods recorded by
    # ordinary steps, then the estimator (reversed walk of the trial + GEMMs)
    n_bp = 2 * qr
    wk_bp = api.Walkers(sysg, nw)
    wk_bp.step(1, dt, seed=12, qr_every=qr, e_shift=e_var)
    wk_bp.bp_begin(n_bp)
    torch.cuda.synchronize()
    t = time.perf_counter()
    wk_bp.step(n_bp, dt, seed=12, qr_every=qr, e_shift=e_var)
    torch.cuda.synchronize()
    rec_ms = (time.perf_counter() - t) / n_bp * 1e3
    lib.afq_trace_reset()
    lib.afq_trace_enable(1)
    t = time.perf_counter()
    P, _ = wk_bp.bp_rdm1(qr_every=qr)
    torch.cuda.synchronize()
    bp_ms = (time.perf_counter() - t) * 1e3
    lib.afq_trace_enable(0)
    bph = trace_phases(lib, _lib)
    lib.afq_trace_reset()
    Pn = P.cpu().numpy()
    prop_ms = sum(bph[k][0] for k in ("abuild", "taylor") if k in bph)
    est_flop = 2 * 8.0 * M * M * nw * nu      # P^s = Q Y^T over nw*n stacked columns, complex FP64
    extra["back_propagation"] = {
        "n_bp": n_bp, "recording_step_ms": round(rec_ms, 3), "rdm1_ms": round(bp_ms, 3),
        "rdm1_ms_per_window_step": round(bp_ms / n_bp, 3),
        "reverse_propagation_ms": round(prop_ms, 3), "qr_ms": round(bph.get("qr", (0.0, 0))[0], 3),
        "estimator_gemm_gflop": round(est_flop / 1e9, 3),
        "trace_err": float(max(abs(np.trace(Pn[0]).real - nu), abs(np.trace(Pn[1]).real - nd)))}
    del P
    wk_bp.close()


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="bf16x3", choices=list(PEAK_TFLOPS))
    ap.add_argument("--workload", default="m400")
    ap.add_argument("--walkers", type=int, default=None, help="override the walker count")
    ap.add_argument("--compare-steps", type=int, default=3, help="timed steps of the other precisions (0: skip)")
    ap.add_argument("--check-steps", type=int, default=2, help="steps of the 4-walker oracle check (0: skip)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the secondary measurements (comb, back-propagation window) after the timed steps")
    ap.add_argument("--exchange-form", default="auto", choices=["auto", "cholesky", "four_index"],
                    help="exchange form of the split-BF16x3 mode (auto: four-index where it pays)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run a device copy of this many MiB (calibrates HBM byte counters) and exit")
    a = ap.parse_args(argv)

    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the walker step shards by walkers (each GPU steps its own "
              "walkers, only the weighted energy sums are combined), so one GPU's share is the measured "
              "unit; use --gpus 1", file=sys.stderr)
        return 2

    import torch
    from paper_2003_01831_amd import synth, api, _lib

    if a.copy_probe_mib:
        n = a.copy_probe_mib * (1 << 20) // 8
        x = torch.ones(n, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": n * 8, "copy_probe_bytes_written": n * 8}))
        return 0

    if a.workload == "uneven24":
        return bench_uneven(a, torch, synth, api, _lib)
    if a.workload == "msd_m128":
        return bench_msd(a, torch, synth, api, _lib)
    if a.workload == "kp_m192":
        return bench_kp(a, torch, synth, api, _lib)

    cfg = dict(synth.WORKLOADS[a.workload])
    M, nu, nd, X = cfg["M"], cfg["n_up"], cfg["n_dn"], cfg["n_chol"]
    nw = a.walkers or cfg["n_walkers"]
    dt, qr = cfg["dt"], cfg["qr_every"]
    t0 = time.perf_counter()
    s = synth.make_system(M, nu, nd, X, seed=cfg["seed"])
    print(f"[bench] system generated in {time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)

    lib = _lib.load()
    t0 = time.perf_counter()
    sysg = api.System.from_synth(s, precision=a.precision, exchange_form=a.exchange_form)
    form, tensor_bytes = sysg.exchange_form()
    print(f"[bench] system set up in {time.perf_counter() - t0:.1f}s, exchange form {form} "
          f"({tensor_bytes / 1e9:.2f} GB tensor)", file=sys.stderr, flush=True)
    # E_shift = variational energy of the trial (walkers at the trial)
    probe = api.Walkers(sysg, 1)
    e_var = float(probe.energy()[3][0])
    probe.close()

    def timed(prec, steps, warmup):
        sysg.set_precision(prec)
        wk = api.Walkers(sysg, nw)
        if warmup:
            wk.step(warmup, dt, seed=11, qr_every=qr, e_shift=e_var, outputs=("emix",))
        torch.cuda.synchronize()
        lib.afq_trace_reset()
        lib.afq_trace_enable(1)
        torch.cuda.synchronize()
        t = time.perf_counter()
        out = wk.step(steps, dt, seed=11, qr_every=qr, e_shift=e_var, outputs=("emix",))
        torch.cuda.synchronize()
        wall = time.perf_counter() - t
        lib.afq_trace_enable(0)
        phases = trace_phases(lib, _lib)
        lib.afq_trace_reset()
        emix = out["emix"].cpu().numpy()
        wk.close()
        return wall, phases, emix

    print(f"[bench] timing {a.precision}: {a.warmup} warmup + {a.steps} steps, {nw} walkers", file=sys.stderr,
          flush=True)
    wall, phases, emix = timed(a.precision, a.steps, a.warmup)
    value = nw * a.steps / wall
    flop_ws, flop_parts, flop_model = flops_per_walker_step(M, nu, X, 6, qr)
    alg_tflops = flop_ws * nw * a.steps / wall / 1e12
    flop_exec = flop_ws
    if form == "four_index":
        flop_exec = flop_ws - flop_parts["exchange"] + 2 * 2.0 * (nu * M) ** 2

    ex_ms, ex_cnt = phases["exchange"]
    ex_avg_s = ex_ms / 1e3 / max(ex_cnt, 1)
    peak = PEAK_TFLOPS[a.precision]
    csrc = os.path.join(ROOT, "paper_2003_01831_amd", "csrc")
    if form == "four_index":
        # the quadratic form Theta^T W Theta over the upper block triangle of the
        # symmetric half-rotated tensor: (N M)^2 / 2 real-by-complex multiply-adds
        # (4 flop each) per walker and spin; spins that share the tensor are
        # contracted in one launch (one exchange phase per step), else one each
        NM = nu * M
        spins_per_launch = 2 if ex_cnt <= a.steps else 1
        per_launch_flops = 2.0 * NM * NM * nw * spins_per_launch
        traffic = None
        if a.workload == "m400" and nw == 512:
            traffic = profiled_traffic(os.path.join(csrc, "eri.hip"),
                                       os.path.join(ROOT, "profiles", "eri_bf16x3_m400.md"), "eri")
        roofline = {"bound": "mfma", "achieved": round(per_launch_flops / ex_avg_s / 1e12, 3), "peak": peak,
                    "unit": "TFLOP/s", "traffic": traffic,
                    "kernel": "four-index exchange kernel (W'' Theta-hat in split BF16x3, FP64 epilogue) "
                              "plus its per-walker reductions, %d spin%s per launch"
                              % (spins_per_launch, "s" if spins_per_launch > 1 else ""),
                    "flop_per_launch": per_launch_flops,
                    "avg_launch_ms": round(ex_avg_s * 1e3, 3), "launches": ex_cnt}
        roofline["frac"] = round(roofline["achieved"] / peak, 4)
        # every algorithmic product is three BF16 products (hi*hi + hi*lo + lo*hi)
        roofline["bf16_products_per_flop"] = 3
        roofline["mfma_pipe_frac"] = round(3 * roofline["achieved"] / peak, 4)
        # the same exchange term counted with the Cholesky-form model, for comparison
        roofline["cholesky_model_equivalent_tflops"] = round(
            (8.0 * X * nu * nu * M + 8.0 * X * nu * nu) * nw * spins_per_launch / ex_avg_s / 1e12, 3)
    else:
        # the exchange term of the general (complex L~) flop model, one spin per
        # launch; the real-L~ count the kernel actually needs is beside it
        per_launch_flops = (8.0 * X * nu * nu * M + 8.0 * X * nu * nu) * nw
        per_launch_real = flop_parts["exchange"] / 2 * nw
        achieved = per_launch_flops / ex_avg_s / 1e12
        traffic = None
        if a.precision == "bf16x3" and a.workload == "m400" and nw == 512:
            traffic = profiled_traffic(os.path.join(csrc, "exchange_big.hip"),
                                       os.path.join(ROOT, "profiles", "exchange_bf16x3_m400.md"), "exchange_big")
        roofline = {"bound": "mfma", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
                    "frac": round(achieved / peak, 4), "traffic": traffic,
                    "kernel": "exchange kernel (fused Omega = Lt Theta, tr Omega, tr Omega^2), one spin per launch",
                    "flop_per_launch": per_launch_flops,
                    "avg_launch_ms": round(ex_avg_s * 1e3, 3), "launches": ex_cnt,
                    "achieved_real_lt": round(per_launch_real / ex_avg_s / 1e12, 3)}
        if a.precision == "bf16x3":
            # split-BF16x3 issues three BF16 products per FP32-class product; against
            # that effective peak, count only the multiply-adds the real L~ needs
            roofline["real_lt_frac_of_bf16x3_effective_peak"] = round(roofline["achieved_real_lt"] / (peak / 3), 4)

    extra = {}
    if not a.no_extras:
        measure_extras(a, extra, sysg, api, lib, _lib, torch, nw, dt, qr, e_var, M, nu, nd)
    if a.compare_steps > 0:
        for prec in ("fp64", "cfp32", "bf16x3"):
            if prec == a.precision:
                continue
            print(f"[bench] timing {prec}: {a.compare_steps} steps", file=sys.stderr, flush=True)
            w2, ph2, _ = timed(prec, a.compare_steps, 1)
            extra[f"{prec}_walker_steps_per_s"] = round(nw * a.compare_steps / w2, 3)
            exm, exc = ph2["exchange"]
            # the other precisions run the Cholesky form: its complex-model count
            chol_launch = (8.0 * X * nu * nu * M + 8.0 * X * nu * nu) * nw
            extra[f"{prec}_exchange_tflops"] = round(chol_launch / (exm / 1e3 / max(exc, 1)) / 1e12, 3)
        sysg.set_precision(a.precision)
        if "fp64_walker_steps_per_s" in extra:
            extra["speedup_vs_fp64_path"] = round(value / extra["fp64_walker_steps_per_s"], 3)

    # error against the FP64 oracle and the oracle's own rate, on a 4-walker subset
    err, cpu = None, None
    if a.check_steps > 0:
        from oracle import afqmc
        nsub, ks = 4, a.check_steps
        fields = synth.make_fields(ks, nsub, X, seed=cfg["field_seed"])
        W0 = synth.trial_walkers(s, nsub)
        wk = api.Walkers(sysg, nsub)
        g = wk.step(ks, dt, fields=fields, qr_every=qr, e_shift=e_var)
        el, parts, _, _ = wk.energy()
        torch.cuda.synchronize()
        g = {k: v.cpu().numpy() for k, v in g.items()}
        if not a.no_cpu:
            try:
                import threadpoolctl
                threads = max([p.get("num_threads", 0) for p in threadpoolctl.threadpool_info()
                               if p.get("user_api") == "blas"] or [os.cpu_count()])
            except Exception:
                threads = os.cpu_count()
            print(f"[bench] oracle: {nsub} walkers x {ks} steps on the host", file=sys.stderr, flush=True)
            pre = afqmc.prepare(s.h1, s.chol, s.phi_t, nu, nd, dt)
            t = time.perf_counter()
            o = afqmc.run(s.h1, s.chol, s.phi_t, nu, nd, W0, np.ones(nsub), fields, dt, qr_every=qr,
                          e_shift=e_var, pre=pre)
            tc = time.perf_counter() - t
            oel, oparts, _ = afqmc.energy(s.h1, s.chol, s.phi_t, nu, nd, o["W"], o["w"])
            cpu = {"value": round(nsub * ks / tc, 4), "unit": "walker-steps/s", "cores": threads,
                   "kind": "oracle",
                   "sample": f"{nsub} walkers x {ks} steps of the same workload (numpy FP64, half-rotated "
                             f"energy), {tc:.1f}s; walkers are independent so the rate scales linearly",
                   "host_cpus": os.cpu_count()}
            pg = parts.cpu().numpy()
            err = {"precision": a.precision, "E_mix": rel_max(g["emix"], o["emix"]),
                   "E_L": rel_max(g["eloc"], o["eloc"]), "weights": rel_max(g["weights"], o["weights"]),
                   "ratio": rel_max(g["ratio"], o["ratio"]),
                   "E1": rel_max(pg[:, 0], oparts[:, 0]), "EJ": rel_max(pg[:, 1], oparts[:, 1]),
                   "EK": rel_max(pg[:, 2], oparts[:, 2])}
            err = {k: (v if isinstance(v, str) else float(f"{v:.3e}")) for k, v in err.items()}
        wk.close()

    line = {
        "metric": "walker-steps/s + MFMA TFLOP/s at M=400 vs plain FP64 path, err vs FP64 oracle",
        "value": round(value, 3), "unit": "walker-steps/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": round(wall / a.steps * 1e3, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": DTYPE[a.precision], "data": "synthetic",
        "config": {"workload": f"{a.workload}: M={M}, N_up=N_dn={nu}, Nchol={X}, {nw} walkers, dt={dt}, "
                               f"QR every {qr}, Taylor order 6, energy every step, Philox fields",
                   "precision": a.precision, "walkers": nw, "parallelism": "single GPU",
                   "exchange_form": form, "four_index_tensor_gb": round(tensor_bytes / 1e9, 3)},
        "alg_tflops": round(flop_model * nw * a.steps / wall / 1e12, 3),
        "alg_tflops_real_lt": round(alg_tflops, 3),
        "flop_per_walker_step": flop_model,
        "flop_per_walker_step_real_lt": flop_ws,
        # the algorithm actually run: with the four-index form the exchange term
        # is 2 (N M)^2 flop per spin instead of the Cholesky form's count
        "flop_per_walker_step_executed": flop_exec,
        "alg_tflops_executed": round(flop_exec * nw * a.steps / wall / 1e12, 3),
        "roofline": roofline,
        "cpu_baseline": cpu,
        "err_vs_fp64_oracle": err,
        "phase_ms_per_step": {k: round(v[0] / a.steps, 3) for k, v in phases.items()},
        "emix_last": float(emix[-1]),
    }
    line.update(extra)
    print(json.dumps(line))
    return 0


if __name__ == "__main__":
    sys.exit(main())
