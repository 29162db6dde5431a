#!/usr/bin/env python3
"""Benchmark of the batched phaseless-AFQMC walker step on one MI355X.

Workload (default): M=400 orbitals, 100+100 electrons, 1600 Cholesky vectors,
512 walkers at the trial, dt 0.005, QR every 5 steps, energy measured every
step, fields from the device Philox stream; synthetic seeded inputs
(paper_2003_01831_amd.synth, workload "m400").

Prints ONE JSON line: walker-steps/s of the headline precision (split-BF16x3
by default, with the exchange form the library chooses: the four-index form at
M=400), the same rate for the plain FP64 path with the same exchange form, and
both precisions (plus complex FP32) with the Cholesky form; the TFLOP/s of the
work each run executes (never a model count of an algorithm that did not run);
the roofline entry of the dominant kernel (timed with HIP events on the library
stream); the error against the CPU FP64 oracle on a 4-walker subset over 6
steps (a QR step included); the oracle's own rate on the host cores with all
BLAS threads and with one (cpu_baseline); and the adjoint (energy gradient) of
the differentiation workload: its time and its errors against the oracle.
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


def exchange_flops_executed(form, M, N, X, nw, spins=2):
    """Algorithmic flop of the exchange term that the chosen form computes
    (real half-rotated vectors of a real trial): the Cholesky form contracts
    Omega_n = Lt_n Theta (X N^2 M real-by-complex multiply-adds, 4 flop each,
    per walker and spin) and forms tr(Omega Omega) (8 X N^2); the four-index
    form contracts the quadratic form of the symmetric tensor, (N M)^2 / 2
    real-by-complex multiply-adds per walker and spin."""
    if form == "four_index":
        return 2.0 * (N * M) ** 2 * nw * spins
    return (4.0 * X * N * N * M + 8.0 * X * N * N) * nw * spins


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
    flop_exec = 0.0
    ex_flops = 0.0
    forms = {"cholesky": 0, "four_index": 0}
    for c in shapes:
        s = synth.make_system(c["M"], c["n_up"], c["n_dn"], c["n_chol"], seed=c["seed"])
        g = api.System.from_synth(s, precision=a.precision)
        probe = api.Walkers(g, 1)
        e_shift.append(float(probe.energy()[3][0]))
        probe.close()
        pairs.append((g, api.Walkers(g, c["n_walkers"])))
        used = g.exchange_form()[0]
        forms[used] += 1
        _, parts, _ = flops_per_walker_step(c["M"], c["n_up"], c["n_chol"], 6, qr)
        ex = exchange_flops_executed(used, c["M"], c["n_up"], c["n_chol"], c["n_walkers"])
        flop_exec += (sum(parts.values()) - parts["exchange"]) * c["n_walkers"] + ex
        ex_flops += ex
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
        # the work executed (each system's exchange counted for the form it ran)
        "tflops": round(flop_exec * steps / wall / 1e12, 3),
        "tflops_frac_of_peak": round(flop_exec * steps / wall / 1e12 / peak, 4),
        "exchange_forms": forms,
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
    if a.kp_trace == "valu":
        wk.set_exchange_variant(0, 1)
        wk.set_exchange_variant(1, 1)
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
    # two length-m complex dot products (8 flop per multiply-add; the MFMA
    # kernel's padded tiles are not counted)
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
        "roofline": {"bound": "mfma" if a.kp_trace == "mfma" else "alu", "achieved": round(achieved, 3),
                     "peak": PEAK_TFLOPS["fp64"], "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK_TFLOPS["fp64"], 4), "traffic": None,
                     "kernel": ("k-point trace kernel on FP64 MFMA (per group of row blocks and Q: Omega' tiles "
                                "to LDS, Omega tiles paired in their epilogue)" if a.kp_trace == "mfma" else
                                "k-point trace kernel on FP64 VALU (per row block and Q: Omega, Omega' blocks)")
                               + " + its row-block reduction",
                     "flop_per_launch": tr_flop, "avg_launch_ms": round(ex_avg_s * 1e3, 3), "launches": ex_cnt,
                     "dense_equivalent_flop": dense_flop},
        "cpu_baseline": cpu,
        "phase_ms_per_step": {k: round(v[0] / a.steps, 3) for k, v in ph.items()},
        "emix_last": float(out["emix"][-1].item()),
    }
    print(json.dumps(line))
    return 0


def measure_gradient(api, torch, synth):
    """Adjoint of the weighted mixed energy on the differentiation workload
    (M=64, 16+16 electrons, 256 vectors, 64 walkers perturbed by 0.1, weights
    in [0.5, 1.5]): milliseconds per afq_energy_backward call (all three
    gradients) and per afq_energy call, and the relative Frobenius error of each
    gradient against the oracle's adjoint, per precision."""
    from oracle import afqmc
    cfg = synth.WORKLOADS["grad_m64"]
    s = synth.make_system(cfg["M"], cfg["n_up"], cfg["n_dn"], cfg["n_chol"], seed=cfg["seed"])
    nw = cfg["n_walkers"]
    W = synth.perturbed_walkers(s, nw, cfg["perturb"], seed=cfg["field_seed"])
    w = synth.random_weights(nw, seed=7)
    print("[bench] gradient workload: oracle adjoint", file=sys.stderr, flush=True)
    rh, rl, rw = afqmc.energy_grad(s.h1, s.chol, s.phi_t, s.n_up, s.n_dn, W, w)

    def rel(x, r):
        return float(f"{np.linalg.norm((x - r).ravel()) / np.linalg.norm(r.ravel()):.3e}")

    out = {"workload": f"grad_m64: M={cfg['M']}, N_up=N_dn={cfg['n_up']}, Nchol={cfg['n_chol']}, {nw} walkers"}
    for prec in ("fp64", "cfp32", "bf16x3"):
        sysg = api.System.from_synth(s, precision=prec)
        wk = api.Walkers(sysg, nw, W, w)
        dh, dl, dw = api.energy_backward(sysg, wk, 1.0)
        wk.energy()
        torch.cuda.synchronize()
        reps = 5
        t = time.perf_counter()
        for _ in range(reps):
            api.energy_backward(sysg, wk, 1.0)
        torch.cuda.synchronize()
        tb = (time.perf_counter() - t) / reps
        t = time.perf_counter()
        for _ in range(reps):
            wk.energy()
        torch.cuda.synchronize()
        tf = (time.perf_counter() - t) / reps
        out[prec] = {"backward_ms": round(tb * 1e3, 3), "energy_ms": round(tf * 1e3, 3),
                     "err_d_h1": rel(dh.cpu().numpy(), rh), "err_d_chol": rel(dl.cpu().numpy(), rl),
                     "err_d_W": rel(dw.cpu().numpy(), rw)}
        wk.close()
        sysg.close()
    return out


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
    # the adjoint at this size: all three gradients (dL alone is X M^2 doubles)
    wk_g = api.Walkers(sysg, nw)
    wk_g.step(2, dt, seed=13, qr_every=qr, e_shift=e_var, outputs=())
    api.energy_backward(sysg, wk_g, 1.0)
    torch.cuda.synchronize()
    t = time.perf_counter()
    d = api.energy_backward(sysg, wk_g, 1.0)
    torch.cuda.synchronize()
    extra["backward_ms"] = round((time.perf_counter() - t) * 1e3, 3)
    del d
    wk_g.close()


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="bf16x3", choices=list(PEAK_TFLOPS))
    ap.add_argument("--workload", default="m400")
    ap.add_argument("--walkers", type=int, default=None, help="override the walker count")
    ap.add_argument("--compare-steps", type=int, default=5,
                    help="timed steps of the comparison runs (other precisions and forms; 0: skip)")
    ap.add_argument("--check-steps", type=int, default=6, help="steps of the 4-walker oracle check (0: skip)")
    ap.add_argument("--single-thread-steps", type=int, default=2,
                    help="steps of the 1-walker oracle run on one BLAS thread (0: skip)")
    ap.add_argument("--no-grad", dest="grad", action="store_false",
                    help="skip the adjoint measurement on the differentiation workload")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--kp-trace", default="mfma", choices=["mfma", "valu"],
                    help="k-point workload: exchange-trace kernel (FP64 MFMA or the FP64 VALU one)")
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

    def timed(prec, steps, warmup, form):
        """walls, traced phases and E_mix of `steps` steps of a fresh walker set
        after `warmup` untimed ones, in precision `prec` with exchange form `form`"""
        sysg.set_exchange_form(form)
        sysg.set_precision(prec)
        used, _ = sysg.exchange_form()
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
        return wall, phases, emix, used

    def summary(prec, steps, wall, phases, used):
        """walker-steps/s, executed TFLOP/s of the whole step and of the exchange
        launches, each with its fraction of the peak of the MFMA type used"""
        fe = flops_per_walker_step(M, nu, X, 6, qr)[1]
        step_flop = sum(fe.values()) - fe["exchange"] + exchange_flops_executed(used, M, nu, X, 1)
        ex_ms, ex_cnt = phases["exchange"]
        ex_flop = exchange_flops_executed(used, M, nu, X, nw) * steps
        pk = PEAK_TFLOPS[prec]
        out = {"walker_steps_per_s": round(nw * steps / wall, 3), "ms_per_step": round(wall / steps * 1e3, 3),
               "exchange_form": used, "steps_timed": steps,
               "step_tflops_executed": round(step_flop * nw * steps / wall / 1e12, 3),
               "exchange_tflops_executed": round(ex_flop / (ex_ms / 1e3) / 1e12, 3) if ex_ms > 0 else None,
               "peak_tflops": pk}
        out["step_frac_of_peak"] = round(out["step_tflops_executed"] / pk, 4)
        if out["exchange_tflops_executed"] is not None:
            out["exchange_frac_of_peak"] = round(out["exchange_tflops_executed"] / pk, 4)
        out["phase_ms_per_step"] = {k: round(v[0] / steps, 3) for k, v in phases.items() if v[0] > 0}
        return out

    print(f"[bench] timing {a.precision}: {a.warmup} warmup + {a.steps} steps, {nw} walkers", file=sys.stderr,
          flush=True)
    wall, phases, emix, form = timed(a.precision, a.steps, a.warmup, a.exchange_form)
    value = nw * a.steps / wall
    flop_model, flop_parts = flops_per_walker_step(M, nu, X, 6, qr)[2], flops_per_walker_step(M, nu, X, 6, qr)[1]
    flop_exec = sum(flop_parts.values()) - flop_parts["exchange"] + exchange_flops_executed(form, M, nu, X, 1)
    head = summary(a.precision, a.steps, wall, phases, form)

    ex_ms, ex_cnt = phases["exchange"]
    ex_avg_s = ex_ms / 1e3 / max(ex_cnt, 1)
    peak = PEAK_TFLOPS[a.precision]
    csrc = os.path.join(ROOT, "paper_2003_01831_amd", "csrc")
    if form == "four_index":
        # the quadratic form Theta^T W Theta over the upper block triangle of the
        # symmetric half-rotated tensor: (N M)^2 / 2 real-by-complex multiply-adds
        # (4 flop each) per walker and spin; spins that share the tensor are
        # contracted in one launch (one exchange phase per step), else one each
        spins_per_launch = 2 if ex_cnt <= a.steps else 1
        per_launch_flops = exchange_flops_executed(form, M, nu, X, nw, spins_per_launch)
        traffic = None
        if a.workload == "m400" and nw == 512 and a.precision == "bf16x3":
            traffic = profiled_traffic(os.path.join(csrc, "eri.hip"),
                                       os.path.join(ROOT, "profiles", "eri_bf16x3_m400.md"), "eri")
        kernel = ("four-index exchange kernel (W'' Theta-hat in split BF16x3, FP64 epilogue) plus its per-walker "
                  "reductions" if a.precision == "bf16x3" else
                  "four-index exchange (FP64 GEMMs over the upper block triangle of W', then per-walker dots)")
        roofline = {"bound": "mfma", "achieved": round(per_launch_flops / ex_avg_s / 1e12, 3), "peak": peak,
                    "unit": "TFLOP/s", "traffic": traffic,
                    "kernel": kernel + ", %d spin%s per launch" % (spins_per_launch, "s" if spins_per_launch > 1
                                                                    else ""),
                    "flop_per_launch": per_launch_flops,
                    "avg_launch_ms": round(ex_avg_s * 1e3, 3), "launches": ex_cnt}
    else:
        # the Cholesky form: Omega = Lt Theta with the real half-rotated vectors of
        # the real trial, one spin per launch
        per_launch_flops = exchange_flops_executed(form, M, nu, X, nw, 1)
        traffic = None
        if a.precision == "bf16x3" and a.workload == "m400" and nw == 512:
            traffic = profiled_traffic(os.path.join(csrc, "exchange_big.hip"),
                                       os.path.join(ROOT, "profiles", "exchange_bf16x3_m400.md"), "exchange_big")
        roofline = {"bound": "mfma", "achieved": round(per_launch_flops / ex_avg_s / 1e12, 3), "peak": peak,
                    "unit": "TFLOP/s", "traffic": traffic,
                    "kernel": "exchange kernel (fused Omega = Lt Theta, tr Omega, tr Omega^2), one spin per launch",
                    "flop_per_launch": per_launch_flops,
                    "avg_launch_ms": round(ex_avg_s * 1e3, 3), "launches": ex_cnt}
    roofline["frac"] = round(roofline["achieved"] / peak, 4)
    if a.precision == "bf16x3":
        # every algorithmic product is three BF16 products (hi*hi + hi*lo + lo*hi):
        # the MFMA pipes are busy about three times the fraction above
        roofline["bf16_products_per_flop"] = 3
        roofline["bf16_product_frac_of_peak"] = round(3 * roofline["achieved"] / peak, 4)

    extra = {}
    if not a.no_extras:
        measure_extras(a, extra, sysg, api, lib, _lib, torch, nw, dt, qr, e_var, M, nu, nd)

    # like-for-like comparisons on the same GPU: the FP64 path with the same
    # exchange form as the headline, then every precision with the Cholesky form
    cmp = {}
    if a.compare_steps > 0:
        runs = [("fp64", "auto")] if form == "four_index" else []
        runs += [(p, "cholesky") for p in ("bf16x3", "fp64", "cfp32")]
        for prec, frm in runs:
            print(f"[bench] timing {prec} ({frm} form): {a.compare_steps} steps", file=sys.stderr, flush=True)
            w2, ph2, _, used = timed(prec, a.compare_steps, 1, frm)
            cmp[f"{prec}_{used}"] = summary(prec, a.compare_steps, w2, ph2, used)
        sysg.set_exchange_form(a.exchange_form)
        sysg.set_precision(a.precision)
        same = cmp.get(f"fp64_{form}")
        if same is not None:
            # the headline against the plain FP64 path running the same algorithm
            extra["fp64_walker_steps_per_s"] = same["walker_steps_per_s"]
            extra["speedup_vs_fp64_path"] = round(value / same["walker_steps_per_s"], 3)
            extra["speedup_vs_fp64_path_form"] = form
        bc, fc = cmp.get("bf16x3_cholesky"), cmp.get("fp64_cholesky")
        if bc and fc:
            extra["speedup_bf16x3_vs_fp64_cholesky_form"] = round(bc["walker_steps_per_s"] / fc["walker_steps_per_s"],
                                                                  3)
        extra["compare"] = cmp

    # error against the FP64 oracle and the oracle's own rate, on a 4-walker
    # subset over check_steps steps (6 by default: QR after the fifth)
    err, cpu = None, None
    if a.check_steps > 0:
        from oracle import afqmc
        nsub, ks = 4, a.check_steps
        fields = synth.make_fields(ks, nsub, X, seed=cfg["field_seed"])
        W0 = synth.trial_walkers(s, nsub)
        wk = api.Walkers(sysg, nsub)
        g = wk.step(ks, dt, fields=fields, qr_every=qr, e_shift=e_var)
        el, parts, _, _ = wk.energy()
        Wg = wk.get()["W"].cpu().numpy()
        torch.cuda.synchronize()
        g = {k: v.cpu().numpy() for k, v in g.items()}
        if not a.no_cpu:
            import threadpoolctl

            def blas_threads():
                return max([p.get("num_threads", 0) for p in threadpoolctl.threadpool_info()
                            if p.get("user_api") == "blas"] or [0])

            threads = blas_threads() or os.cpu_count()
            print(f"[bench] oracle: {nsub} walkers x {ks} steps on the host ({threads} BLAS threads)",
                  file=sys.stderr, flush=True)
            pre = afqmc.prepare(s.h1, s.chol, s.phi_t, nu, nd, dt)
            t = time.perf_counter()
            o = afqmc.run(s.h1, s.chol, s.phi_t, nu, nd, W0, np.ones(nsub), fields, dt, qr_every=qr,
                          e_shift=e_var, pre=pre)
            tc = time.perf_counter() - t
            oel, oparts, _ = afqmc.energy(s.h1, s.chol, s.phi_t, nu, nd, o["W"], o["w"])
            cpu = {"value": round(nsub * ks / tc, 4), "unit": "walker-steps/s", "cores": threads,
                   "kind": "oracle",
                   "sample": f"{nsub} walkers x {ks} steps of the same workload (numpy FP64, half-rotated "
                             f"energy, QR after step 5), {tc:.1f}s; walkers are independent so the rate scales "
                             f"linearly",
                   "host_cpus": os.cpu_count()}
            if a.single_thread_steps > 0:
                n1 = a.single_thread_steps
                print(f"[bench] oracle: 1 walker x {n1} steps on 1 BLAS thread", file=sys.stderr, flush=True)
                with threadpoolctl.threadpool_limits(1, user_api="blas"):
                    t = time.perf_counter()
                    afqmc.run(s.h1, s.chol, s.phi_t, nu, nd, W0[:1], np.ones(1), fields[:n1, :1], dt,
                              qr_every=qr, e_shift=e_var, pre=pre)
                    t1 = time.perf_counter() - t
                cpu["single_thread"] = {"value": round(n1 / t1, 4), "unit": "walker-steps/s", "cores": 1,
                                        "sample": f"1 walker x {n1} steps, {t1:.1f}s"}
            pg = parts.cpu().numpy()
            err = {"precision": a.precision, "exchange_form": form, "steps": ks,
                   "E_mix": rel_max(g["emix"], o["emix"]),
                   "E_L": rel_max(g["eloc"], o["eloc"]), "weights": rel_max(g["weights"], o["weights"]),
                   "ratio": rel_max(g["ratio"], o["ratio"]),
                   "E1": rel_max(pg[:, 0], oparts[:, 0]), "EJ": rel_max(pg[:, 1], oparts[:, 1]),
                   "EK": rel_max(pg[:, 2], oparts[:, 2]),
                   "W": float(np.linalg.norm(Wg - o["W"]) / np.linalg.norm(o["W"]))}
            err = {k: (v if isinstance(v, (str, int)) else float(f"{v:.3e}")) for k, v in err.items()}
        wk.close()

    grad = None
    if a.grad and not a.no_cpu:
        grad = measure_gradient(api, torch, synth)

    line = {
        "metric": "walker-steps/s + MFMA TFLOP/s at M=400 vs plain FP64 path, err vs FP64 oracle",
        "value": round(value, 3), "unit": "walker-steps/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": round(wall / a.steps * 1e3, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": DTYPE[a.precision], "data": "synthetic",
        "config": {"workload": f"{a.workload}: M={M}, N_up=N_dn={nu}, Nchol={X}, {nw} walkers, dt={dt}, "
                               f"QR every {qr}, Taylor order 6, energy every step, Philox fields",
                   "precision": a.precision, "walkers": nw, "parallelism": "single GPU",
                   "exchange_form": form, "four_index_tensor_gb": round(tensor_bytes / 1e9, 3)},
        # TFLOP/s of the work this run executed (the exchange term counted for the
        # form that ran) and its fraction of the peak of the MFMA type used
        "tflops": head["step_tflops_executed"],
        "tflops_frac_of_peak": head["step_frac_of_peak"],
        "flop_per_walker_step_executed": flop_exec,
        # the general complex flop model (8 flop per complex multiply-add, Cholesky
        # form): a count for reference, not a rate of this run
        "flop_per_walker_step_model": flop_model,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "err_vs_fp64_oracle": err,
        "gradient": grad,
        "phase_ms_per_step": head["phase_ms_per_step"],
        "emix_last": float(emix[-1]),
    }
    line.update(extra)
    print(json.dumps(line))
    return 0


if __name__ == "__main__":
    sys.exit(main())
