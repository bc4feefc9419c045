"""Benchmark of the mu-mode hot path on one MI355X.

Workload: one Strang step of the 3-D cubic Gross-Pitaevskii equation
i psi_t = -1/2 Laplace psi + 1/2 |x|^2 psi + beta |psi|^2 psi, beta = 100,
n = 256 per direction on [-8, 8]^3 (homogeneous Dirichlet, second-order
finite differences), tau = 1e-3, complex64 state, the three mu-mode products
in split-precision MFMA with FP32 accumulation (--split: FP16x2, three
products, or BF16x3, six products), the nonlinear phase fused into the last
product.  Synthetic seeded Thomas-Fermi-like initial state.

Prints one JSON line.  The same step in plain FP64 (complex128 state, FP64
MFMA), in FP32 and in the other split scheme is timed beside it, the
per-launch durations of the mode-product kernels come from HIP events
recorded around each launch inside the timed region, and the FP64 CPU oracle
is timed on a bounded sample.
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

PEAK = {  # MI355X published dense peaks
    "bf16": 2516.6e12, "fp32": 157.3e12, "fp64": 78.6e12, "hbm": 8.0e12,
}
N, A, B, BETA, TAU, D = 256, -8.0, 8.0, 100.0, 1e-3, 3
FLOPS_PER_PRODUCT = 8.0 * N * N ** D            # complex MAC = 8 flops, n per output entry
FLOPS_PER_STEP = D * FLOPS_PER_PRODUCT
BYTES_PER_PRODUCT = 2 * 8 * N ** D                 # one read and one write of the complex64 state
SPLIT_PRODUCTS = {"bf16x3": 6, "fp16x2": 3}        # MFMA products per algorithmic product


# sources that determine the split product kernel; HBM traffic counters taken
# on another build of them are not reported
KERNEL_SOURCES = ["paper_2103_01691_amd/csrc/mode_tile.h", "paper_2103_01691_amd/csrc/mm_internal.h",
                  "paper_2103_01691_amd/csrc/kern_bf16x3.hip", "paper_2103_01691_amd/csrc/kern_fp16x2.hip",
                  "paper_2103_01691_amd/csrc/kern_bf16x3_ida.hip", "paper_2103_01691_amd/csrc/kern_fp16x2_ida.hip",
                  "paper_2103_01691_amd/csrc/kernels_common.hip", "paper_2103_01691_amd/build.py",
                  "paper_2103_01691_amd/csrc/mode_gauss.h", "paper_2103_01691_amd/csrc/kern_bf16x3_g.hip",
                  "paper_2103_01691_amd/csrc/kern_fp16x2_g.hip"]


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for s in KERNEL_SOURCES:
        p = os.path.join(ROOT, s)
        if os.path.exists(p):
            h.update(s.encode())
            with open(p, "rb") as f:
                h.update(f.read())
    return h.hexdigest()[:16]


def counter_traffic(summary, field="traffic_bytes_per_launch"):
    """A figure of a committed rocprofv3 summary (default: scaled FETCH_SIZE +
    WRITE_SIZE bytes per product launch), or None when it was taken on other
    kernel sources."""
    path = os.path.join(ROOT, "profiles", summary)
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith(("|", "#", "`")):
                k, _, v = line.partition(":")
                fields[k.strip()] = v.strip()
    if fields.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    try:
        return float(fields[field])
    except (KeyError, ValueError):
        return None


_T0 = time.perf_counter()


def log(msg):
    print(f"[{time.perf_counter() - _T0:6.1f} s] {msg}", file=sys.stderr, flush=True)


def build_operator(mm):
    # exp(-i tau H), H = -1/2 D2 + 1/2 x^2 (library FP64 builder)
    return mm.schrodinger_fd_exponential(N, A, B, 1.0, TAU)


def executed_share(tuned):
    """Fraction of the split MFMA work of the four-product form that one GPE
    step executes: the three-product (Gauss) kernels, tile classes 8 and 9,
    issue 3/4 of it.  A step runs mode 1 with the prologue phase (its own
    tune key, load path 0 + 8, else the plain one) and modes 2 and 3 on
    strided fibres (load path 1)."""
    cls = {t["load"]: t["class"] for t in tuned}
    m1 = cls.get(8, cls.get(0))
    m23 = cls.get(1)
    g = lambda c: 0.75 if c in (8, 9) else 1.0
    return (g(m1) + 2 * g(m23)) / 3


def time_path(ctx, mm, torch, E, psi0_np, prec, steps, warmup, profile, tune_ms=0, tune_file=None,
              identity_split=False):
    cdt = torch.complex128 if prec == "fp64" else torch.complex64
    npdt = np.complex128 if prec == "fp64" else np.complex64
    import synth
    psi = torch.from_numpy(synth.to_device_layout(psi0_np.astype(npdt))).cuda()
    op = ctx.mm_op_prepare(E, prec, identity_split=identity_split)
    ops = [op] * D
    tuned = []
    if tune_ms > 0 or tune_file:
        # tile shape of every mode product chosen by timing (the library's
        # autotuner), or read back from a tune file of an earlier run
        ctx.mm_tune_clear()
        if tune_file and os.path.exists(tune_file):
            ctx.mm_tune_load(tune_file)
        else:
            ctx.mm_autotune(psi, ops, max(tune_ms, 1))
            if tune_file:
                ctx.mm_tune_save(tune_file)
        tuned = [{"load": k[2], "rows": k[3], "fibres": k[5], "class": c, "us": round(us, 1)}
                 for k, c, us in ctx.mm_tune_entries()]
    if warmup > 0:
        ctx.gpe_strang_step(psi, ops, TAU, BETA, warmup)
    torch.cuda.synchronize()
    if profile:
        ctx.mm_profile_begin()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record()
    ctx.gpe_strang_step(psi, ops, TAU, BETA, steps)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev0.elapsed_time(ev1)
    recs = ctx.mm_profile_end() if profile else []
    op.destroy()
    del psi
    torch.cuda.empty_cache()
    return ms / steps, wall, recs, tuned


def timed(torch, fn, reps):
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    fn(reps)
    ev1.record()
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) * 1e-3


WORKLOADS = ("batch512", "ho128", "free256", "hkmp", "heat64", "vortex")


def other_workloads(ctx, mm, torch, only=WORKLOADS):
    """Throughput of the other scope workloads (their parity is tested in
    tests/); not the headline metric.  `only`: the subset to run (a profiler
    run of one workload)."""
    import synth
    out = {}
    gen = torch.Generator(device="cuda")
    gen.manual_seed(5)
    if "batch512" in only:
        out.update(_batch_workload(ctx, mm, torch, gen))
    if "ho128" in only:
        out.update(_ho_workload(ctx, mm, torch, gen))
    if "free256" in only:
        out.update(_free_workload(ctx, mm, torch))
    if "hkmp" in only:
        out.update(_hkmp_workload(ctx, mm, torch, gen))
    if "heat64" in only:
        out.update(_heat_workload(ctx, mm, torch, gen))
    if "vortex" in only:
        log("  vortex reconnection (Section 4.5)")
        out.update(_vortex_workload(ctx, mm, torch))
    return out


def _batch_workload(ctx, mm, torch, gen):
    import synth
    out = {}
    # batched: 512 instances of the mixed heat / Schroedinger workload, one
    # exponential step each, FP32, one captured graph per step; operators
    # shared per (kind, n) at tau = 1e-3 (the step's cost does not depend on tau)
    mix = synth.batch_mix(512, cfg_id=5)
    cache, tensors, ops = {}, [], []
    ideal = 0.0
    for inst in mix:
        cplx = inst["kind"] == "schrodinger"
        row = []
        for n in inst["dims"]:
            key = (inst["kind"], n)
            if key not in cache:
                if cplx:
                    E = mm.schrodinger_fd_exponential(n, -10.0, 10.0, 0.0, 1e-3)
                else:
                    E = mm.expm(mm.fd2_matrix(n, 0.0, 1.0), 1e-3).real.copy()
                cache[key] = ctx.mm_op_prepare(E, "fp32")
            row.append(cache[key])
        ops.append(row)
        shape = tuple(reversed(inst["dims"]))
        tensors.append(torch.randn(shape, dtype=torch.complex64 if cplx else torch.float32, device="cuda",
                                   generator=gen))
        N = float(np.prod(inst["dims"]))
        for n in inst["dims"]:
            flops = (8.0 if cplx else 2.0) * n * N
            nbytes = 2.0 * N * (8 if cplx else 4)
            ideal += max(flops / PEAK["fp32"], nbytes / PEAK["hbm"])
    ctx.mumode_expstep_batched(tensors, ops, 1)               # capture + first replay
    K = 20
    t_builtin = timed(torch, lambda k: ctx.mumode_expstep_batched(tensors, ops, k), K)
    # per-mode tiles chosen by the batch autotuner (timing the merged batch
    # step itself), then the step captured again with them
    tt0 = time.perf_counter()
    chosen = ctx.mm_autotune_batched(tensors, ops, 200)
    tune_s = time.perf_counter() - tt0
    ctx.mumode_expstep_batched(tensors, ops, 1)
    t = timed(torch, lambda k: ctx.mumode_expstep_batched(tensors, ops, k), K)
    out["batch512_fp32"] = {"instances_per_s": 512 * K / t, "ms_per_batch_step": 1e3 * t / K,
                            "roofline_frac": ideal / (t / K),
                            "ms_per_batch_step_builtin_tiles": 1e3 * t_builtin / K,
                            "autotune_s": tune_s,
                            "tuned_classes": {f"mode{m}_{'complex' if c else 'real'}": v for (m, c), v in chosen.items()},
                            "roofline": "sum over instances of max(flops / FP32 MFMA peak, bytes / HBM peak)"}
    ctx.mm_tune_clear()
    del tensors
    for o in cache.values():
        o.destroy()
    torch.cuda.empty_cache()
    return out


def _ho_workload(ctx, mm, torch, gen):
    out = {}
    # harmonic oscillator, Hermite n = 128, complex64, time-dependent potential
    m = 128
    Xl, _ = mm.hermite_nodes(m)
    Fl, Bl = mm.hermite_matrices(m)
    for prec in ("fp32", "bf16x3", "fp16x2"):
        Lh = ctx.mm_op_prepare(mm.hermite_ho_exponential(m, 0.02), prec)
        F, B = ctx.mm_op_prepare(Fl, prec), ctx.mm_op_prepare(Bl, prec)
        psi = torch.randn((m, m, m), dtype=torch.complex64, device="cuda", generator=gen)
        ctx.mm_autotune(psi, [Lh] * 3, 500)   # tiles for these shapes (kept in the context)
        ctx.ho_strang_step(psi, [F] * 3, [B] * 3, [Xl] * 3, 0.0, 0.02, 0.1, 2)
        K = 50
        t = timed(torch, lambda k: ctx.ho_strang_step(psi, [F] * 3, [B] * 3, [Xl] * 3, 0.0, 0.02, 0.1, k), K)
        out[f"ho128_{prec}"] = {"steps_per_s": K / t, "ms_per_step": 1e3 * t / K,
                                "tflops_effective": 3 * 8.0 * m * m ** 3 / (t / K) / 1e12}
        # the forward and backward Hermite transforms alone (Section 3): six
        # real-operator products on the complex state, each on the (re, im)
        # planes as real fibres (4 flops per complex entry and operator column)
        spec = torch.empty_like(psi)
        ctx.mumode_transform(spec, psi, [F] * 3)
        t6 = timed(torch, lambda k: [(ctx.mumode_transform(spec, psi, [F] * 3),
                                      ctx.mumode_transform(psi, spec, [B] * 3)) for _ in range(k)], K)
        out[f"ho128_{prec}"]["transforms_6pass_ms"] = 1e3 * t6 / K
        out[f"ho128_{prec}"]["transforms_6pass_tflops_effective"] = 6 * 4.0 * m * m ** 3 / (t6 / K) / 1e12
        for o in (Lh, F, B):
            o.destroy()
        del psi, spec
    return out


def _free_workload(ctx, mm, torch):
    import synth
    out = {}
    # free Schroedinger, d = 3, n = 256 on [-10, 10]^3, tau = 0.01: exact in
    # time, one expstep (three mode products) per step, 100 steps per call
    x0 = synth.wavepacket_initial(256, -10.0, 10.0, 3)
    Ef = mm.schrodinger_fd_exponential(256, -10.0, 10.0, 0.0, 0.01)
    fs = {}
    for prec in ("fp64", "fp32", "bf16x3", "fp16x2"):
        npdt = np.complex128 if prec == "fp64" else np.complex64
        psi = torch.from_numpy(synth.to_device_layout(x0.astype(npdt))).cuda()
        Eop = ctx.mm_op_prepare(Ef, prec)
        ctx.mm_autotune(psi, [Eop] * 3, 500)
        ctx.mumode_expstep(psi, [Eop] * 3, 2)
        t = timed(torch, lambda k: ctx.mumode_expstep(psi, [Eop] * 3, k), 100)
        fs[prec] = {"ms_per_step": 1e3 * t / 100, "steps_per_s": 100 / t,
                    "tflops_effective": FLOPS_PER_STEP / (t / 100) / 1e12}
        Eop.destroy()
        del psi
    out["free_schroedinger256_100steps"] = fs
    torch.cuda.empty_cache()
    return out


def _hkmp_workload(ctx, mm, torch, gen):
    out = {}
    # time-dependent Schroedinger problem of Section 4.4 in nodal Hermite
    # space, exponential midpoint rule: the mode-3 exponential is formed on
    # the device every step ("exp (int)"), then the three mode products
    for m in (128, 256):
        X, _ = mm.hermite_nodes(m)
        Bm = mm.hermite_ho_generator(m)
        K = 20
        g = np.zeros((K, 3), dtype=np.complex128)
        g[:, 2] = -1j * np.sin((np.arange(K) + 0.5) * 0.02) ** 2
        for prec, sdt in (("fp64", torch.complex128), ("fp32", torch.complex64)):
            psi = torch.randn((m, m, m), dtype=sdt, device="cuda", generator=gen)
            ctx.mumode_magnus_step(psi, [Bm] * 3, [None, None, X], g[:2], 0.02, 2, prec)
            t = timed(torch, lambda k: ctx.mumode_magnus_step(psi, [Bm] * 3, [None, None, X], g[:k], 0.02, k, prec), K)
            A = torch.from_numpy(np.ascontiguousarray((0.02 * (Bm - 1j * 0.5 * np.diag(X))).T)).cuda()
            Eo = torch.empty_like(A)
            t_exp = timed(torch, lambda k: [ctx.mm_expm_device(A, 1.0, Eo) for _ in range(k)], K)
            out[f"hkmp{m}_{prec}"] = {"ms_per_step": 1e3 * t / K, "ms_exp_int": 1e3 * t_exp / K,
                                      "note": "step = one device expm (mode 3) + three mode products; "
                                              "exp timed alone includes a host sync for its norm"}
            del psi, A, Eo
    out["hkmp_paper_v100_ms"] = {"n127_double": {"exp_int": 0.37, "mu_mode": 1.05},
                                 "n255_double": {"exp_int": 0.66, "mu_mode": 13.79},
                                 "n127_single": {"exp_int": 0.25, "mu_mode": 0.54},
                                 "n255_single": {"exp_int": 0.34, "mu_mode": 7.01},
                                 "source": "the paper's table for this problem (V100), context only"}
    return out


def _heat_workload(ctx, mm, torch, gen):
    out = {}
    # heat, d = 2, n = 64, FP64, 20 steps per call (launch-latency bound)
    E = mm.expm(mm.fd2_matrix(64, 0.0, 1.0), 1e-3).real.copy()
    Eop = ctx.mm_op_prepare(E, "fp64")
    u = torch.rand((64, 64), dtype=torch.float64, device="cuda", generator=gen)
    ctx.mumode_expstep(u, [Eop] * 2, 20)
    K = 20
    t = timed(torch, lambda k: [ctx.mumode_expstep(u, [Eop] * 2, 20) for _ in range(k)], K)
    ctx.mm_set_option(mm.MM_OPT_SMALL_RUN, 0)
    t_per = timed(torch, lambda k: [ctx.mumode_expstep(u, [Eop] * 2, 20) for _ in range(k)], K)
    ctx.mm_set_option(mm.MM_OPT_SMALL_RUN, 1)
    out["heat64x64_fp64_20steps"] = {"calls_per_s": K / t, "us_per_step": 1e6 * t / (20 * K),
                                     "us_per_step_one_launch_per_product": 1e6 * t_per / (20 * K),
                                     "note": "default: all 20 steps in one single-workgroup launch"}
    Eop.destroy()
    torch.cuda.empty_cache()
    return out


def _vortex_workload(ctx, mm, torch):
    import synth
    out = {}
    # vortex reconnection of Section 4.5: [-20, 20]^3 on graded non-uniform
    # nodes with homogeneous Neumann ends, symmetrised variable v = W^(1/2) u,
    # Strang steps of tau = 0.1 up to T = 25 (250 steps), the paper's n
    tau, T = 0.1, 25.0
    steps = int(round(T / tau))
    for n in (81, 141):
        xs = [synth.graded_nodes(n, -20.0, 20.0, 2.0)] * 3
        M, w = mm.nonuniform_neumann_d2(xs[0])
        E = mm.expm(M, 0.5j * tau)
        W = w[:, None, None] * w[None, :, None] * w[None, None, :]
        v0 = np.sqrt(W) * synth.vortex_pair_initial(xs)
        for prec in ("fp64", "fp32", "bf16x3", "fp16x2"):
            npdt = np.complex128 if prec == "fp64" else np.complex64
            v = torch.from_numpy(synth.to_device_layout(v0.astype(npdt))).cuda()
            Eop = ctx.mm_op_prepare(E, prec)
            ctx.mm_tune_clear()
            ctx.mm_autotune(v, [Eop] * 3, 300)
            ctx.vortex_strang_step(v, [Eop] * 3, [w] * 3, tau, 2)
            t = timed(torch, lambda k: ctx.vortex_strang_step(v, [Eop] * 3, [w] * 3, tau, k), steps)
            out[f"vortex{n}_{prec}"] = {"ms_per_step": 1e3 * t / steps, "s_to_T25": t,
                                        "tflops_effective": 3 * 8.0 * n * n ** 3 / (t / steps) / 1e12}
            Eop.destroy()
            del v
    ctx.mm_tune_clear()
    out["vortex_paper_cpu_s_to_T25"] = {"n81": 14.94, "n101": 29.51, "n121": 58.74, "n141": 102.40,
                                        "source": "the paper's figure for the mu-mode integrator (MATLAB, CPU), "
                                                  "context only"}
    torch.cuda.empty_cache()
    return out


def cpu_baseline(psi0, nsteps):
    from oracle import operators as op
    from oracle import schemes as sc
    E = op.ho_exponential(N, A, B, TAU)
    p = psi0.astype(np.complex64).astype(np.complex128)
    t0 = time.perf_counter()
    out = sc.gpe_strang(p, [E] * D, TAU, BETA, nsteps)
    dt = time.perf_counter() - t0
    return nsteps / dt, dt, out, p


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cpu-steps", type=int, default=16, help="oracle steps timed on the host (0: skip)")
    ap.add_argument("--no-side-paths", action="store_true", help="skip the FP64 / FP32 comparison paths")
    ap.add_argument("--split", default="fp16x2", choices=list(SPLIT_PRODUCTS),
                    help="split scheme of the timed path")
    ap.add_argument("--tune-ms", type=int, default=1500, help="autotuner budget per path (0: built-in tiles)")
    ap.add_argument("--tune-file", default=None,
                    help="timed path: load the tile choice from this file if it exists, else tune and save it")
    ap.add_argument("--no-workloads", action="store_true", help="skip the batched / HO / heat side measurements")
    ap.add_argument("--only-workload", choices=WORKLOADS, default=None,
                    help="profiling aid: run only this side workload, print its figures and exit")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="after timing, run one plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the library has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2103_01691_amd as mm
    import synth

    if args.only_workload:
        ctx = mm.Context(0)
        log(f"side workload {args.only_workload} alone")
        print(json.dumps(other_workloads(ctx, mm, torch, (args.only_workload,))), flush=True)
        ctx.close()
        return

    log("building operator (host FP64 expm)")
    E = build_operator(mm)
    log("building initial state")
    psi0 = synth.thomas_fermi_initial(N, A, B, D, BETA, cfg_id=4)
    ctx = mm.Context(0)

    split = args.split
    log(f"timing split {split}: {args.warmup} warmup + {args.steps} steps")
    ms, wall, recs, tuned = time_path(ctx, mm, torch, E, psi0, split, args.steps, args.warmup, True,
                                      args.tune_ms, args.tune_file)
    prod_ms = [t for _, t in recs]
    kinds = sorted(set(k for k, _ in recs))
    per_kind = {str(k): float(np.mean([t for kk, t in recs if kk == k])) for k in kinds}
    avg_launch_ms = float(np.mean(prod_ms)) if prod_ms else None
    achieved = FLOPS_PER_PRODUCT / (avg_launch_ms * 1e-3) if avg_launch_ms else None

    side = {}
    if not args.no_side_paths:
        for prec in ["fp64", "fp32"] + [p for p in SPLIT_PRODUCTS if p != split]:
            k = max(10, args.steps // 4)
            log(f"timing {prec}: {k} steps")
            pms, _, _, ptuned = time_path(ctx, mm, torch, E, psi0, prec, k, 5, False, args.tune_ms)
            eff = FLOPS_PER_STEP / (pms * 1e-3) / 1e12
            # MFMA work the path executes per step (split schemes: every
            # piece product) over the whole step time, against the dense
            # peak of the MFMA type it uses
            mult, peak = {"fp64": (1, PEAK["fp64"]), "fp32": (1, PEAK["fp32"])}.get(
                prec, (SPLIT_PRODUCTS.get(prec, 1), PEAK["bf16"]))
            if prec in SPLIT_PRODUCTS:
                mult *= executed_share(ptuned)
            side[prec] = {"ms_per_step": pms, "steps_per_s": 1e3 / pms, "tflops_effective": eff,
                          "executed_mfma_frac_per_step": mult * eff * 1e12 / peak}
            if prec in SPLIT_PRODUCTS:
                summ = f"mode_kernel_{prec}_gpe3d_n256.md"
                side[prec]["traffic_bytes_per_launch"] = counter_traffic(summ)
                side[prec]["mfma_busy_frac_counters"] = counter_traffic(summ, "mfma_busy_frac")
        # one step per call (a serving-style loop): every FP16x2 call starts
        # with a max-abs pass over the state, unless consecutive calls on the
        # tensor continue the running bound (MM_OPT_FP16X2_CHAIN)
        import synth
        psi = torch.from_numpy(synth.to_device_layout(psi0.astype(np.complex64))).cuda()
        op1 = ctx.mm_op_prepare(E, "fp16x2")
        percall = {}
        for chain in (0, 1):
            ctx.mm_set_option(mm.MM_OPT_FP16X2_CHAIN, chain)
            ctx.gpe_strang_step(psi, [op1] * D, TAU, BETA, 1)
            k = 50
            t = timed(torch, lambda r: [ctx.gpe_strang_step(psi, [op1] * D, TAU, BETA, 1) for _ in range(r)], k)
            percall["chained_bound" if chain else "max_abs_pass_each_call"] = 1e3 * t / k
        ctx.mm_set_option(mm.MM_OPT_FP16X2_CHAIN, 0)
        side["fp16x2_one_step_per_call_ms"] = percall
        op1.destroy()
        del psi
        # trajectory-accurate variants: operators prepared as L - I (identity
        # split), each product adding its input back in the epilogue
        for prec in SPLIT_PRODUCTS:
            k = max(10, args.steps // 4)
            log(f"timing {prec} with the identity split: {k} steps")
            pms, _, _, _ = time_path(ctx, mm, torch, E, psi0, prec, k, 5, False, args.tune_ms, identity_split=True)
            side[f"{prec}_identity_split"] = {"ms_per_step": pms, "steps_per_s": 1e3 / pms,
                                              "tflops_effective": FLOPS_PER_STEP / (pms * 1e-3) / 1e12}

    workloads = None
    if not args.no_workloads:
        log("timing the other workloads (batched, harmonic oscillator, small heat)")
        workloads = other_workloads(ctx, mm, torch)

    if args.calib_copy_mb > 0:
        # a plain copy kernel of known size: its FETCH_SIZE / WRITE_SIZE
        # counters calibrate the HBM traffic counters of the product kernels
        nbytes = args.calib_copy_mb << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # one GPU step vs the oracle on the identical cast input, plus the CPU baseline
    cpu = None
    parity = None
    if args.cpu_steps > 0:
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        log(f"oracle: {args.cpu_steps} FP64 steps on the host ({threads} threads)")
        sps, dt, ref, p0 = cpu_baseline(psi0, args.cpu_steps)
        cpu = {"value": sps, "unit": "steps/s", "cores": threads, "kind": "oracle",
               "sample": f"{args.cpu_steps} unmerged FP64 Strang steps of the full 256^3 GPE workload ({dt:.1f} s)"}
        psi = torch.from_numpy(synth.to_device_layout(psi0.astype(np.complex64))).cuda()
        op = ctx.mm_op_prepare(E, split)
        ctx.gpe_strang_step(psi, [op] * D, TAU, BETA, args.cpu_steps)
        torch.cuda.synchronize()
        got = synth.from_device_layout(psi.cpu().numpy()).astype(np.complex128)
        parity = float(np.linalg.norm((got - ref).ravel()) / np.linalg.norm(ref.ravel()))
        op.destroy()

    traffic = counter_traffic(f"mode_kernel_{split}_gpe3d_n256.md")
    out = {
        "metric": "3D n=256 steps/s & achieved TFLOP/s: split-precision MFMA vs plain FP64",
        "value": 1e3 / ms,
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": split,
        "data": "synthetic",
        "config": {"workload": f"gpe3d_strang_n256_split_{split}", "d": D, "n": N, "beta": BETA, "tau": TAU,
                   "domain": [A, B], "state": "complex64", "precision": f"split_{split}_fp32acc"},
        "tflops_effective": FLOPS_PER_STEP / (ms * 1e-3) / 1e12,
        "executed_mfma_frac_per_step": (SPLIT_PRODUCTS[split] * executed_share(tuned) * FLOPS_PER_STEP
                                        / (ms * 1e-3) / PEAK["bf16"]),
        "roofline": {
            "bound": "mfma", "achieved": achieved / 1e12 if achieved else None, "peak": PEAK["bf16"] / 1e12,
            "unit": "TFLOP/s", "frac": (achieved / PEAK["bf16"]) if achieved else None, "traffic": traffic,
            "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE x2 + WRITE_SIZE x1, copy-calibrated)",
            "algorithmic_bytes_per_launch": BYTES_PER_PRODUCT,
            "kernel": ("mode_kernel" + (" and gauss_kernel (three-product classes)"
                                        if any(t["class"] >= 8 for t in tuned) else "")
                       + f" (split {split}, complex 256x256 operator, one mu-mode product per launch)"),
            "avg_launch_ms": avg_launch_ms, "launches": len(prod_ms), "per_kind_ms": per_kind,
            "executed_mfma_frac": ((SPLIT_PRODUCTS[split] * executed_share(tuned) * achieved / PEAK["bf16"])
                                   if achieved else None),
            "mfma_busy_frac_counters": counter_traffic(f"mode_kernel_{split}_gpe3d_n256.md", "mfma_busy_frac"),
        },
        "tuned_tiles": tuned,
        "paths": side,
        "speedup_vs_fp64": (side["fp64"]["ms_per_step"] / ms) if "fp64" in side else None,
        "parity_rel_l2_vs_oracle": parity,
        "parity_steps": args.cpu_steps if parity is not None else None,
        "cpu_baseline": cpu,
        "other_workloads": workloads,
        "wall_s_timed": wall,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
