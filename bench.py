"""Benchmark: dense two-site DMRG updates at chi = 1024 on one MI355X.

Workload (dense two-site update, chi = 1024, d = 2): per update
    theta0 = A . B                       (contraction over the shared bond)
    20 Lanczos matvecs with the effective Hamiltonian L.W.W.R (Heisenberg MPO,
       bond dimension 5, Gaussian Hermitian environments (chi, 5, chi))
    trunc_svd of theta (2048 x 2048) with eps = 1e-8, chi <= 1024
    renormalised singular values, new site tensors A' = U s, B' = V^dagger
A step is one pass over a batch of `--updates` (default 64) independent
updates with seeded synthetic inputs already resident in HBM.  Two paths run
on the same inputs: plain FP64 (complex128 everywhere) and mixed (complex64
storage, split-BF16x3 contractions with FP32 accumulation, complex64-stored
Krylov vectors with FP64 recurrence and orthogonalisation arithmetic, FP64
Gram / orthogonalisation / eigensolve); the learned sketch
predicts the sketch rank of the randomized SVD and falls back to the plain
SVD when the discarded weight misses eps (always here: the cap binds).

Prints one JSON line (rank 0).  --gpus N with N > 1 exits: the benchmark
measures one GPU (the library has no multi-GPU path).
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

KERNEL_OF_CLASS = {  # kernel that carries each profiling class
    "c64_bf16x3_planes": ("gemm_planes_kernel<true>", "paper_2512_23917_amd/csrc/bf16x3.hip"),
    "c128_fp64": ("gemm_f64_kernel<cd,128,64>", "paper_2512_23917_amd/csrc/gemm.hip"),
    "hemv": ("tri_colC_kernel<cd,32>", "paper_2512_23917_amd/csrc/eig.hip"),
}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_gemm_planes_c64_chi1024.txt")

PEAKS = {  # MI355X published dense peaks
    "c128_fp64": (78.6e12, "TFLOP/s", "mfma"),
    "f64_fp64": (78.6e12, "TFLOP/s", "mfma"),
    "c64_fp32": (157.3e12, "TFLOP/s", "mfma"),
    "f32_fp32": (157.3e12, "TFLOP/s", "mfma"),
    "c64_bf16x3": (2.5e15, "TFLOP/s", "mfma"),
    "f32_bf16x3": (2.5e15, "TFLOP/s", "mfma"),
    "c64_bf16x3_planes": (2.5e15, "TFLOP/s", "mfma"),
    "f32_bf16x3_planes": (2.5e15, "TFLOP/s", "mfma"),
    "hemv": (8.0e12, "GB/s", "hbm"),
    "sweep_dot": (8.0e12, "GB/s", "hbm"),
    "sweep_axpy": (8.0e12, "GB/s", "hbm"),
    "reorth2_dot": (8.0e12, "GB/s", "hbm"),
    "reorth2_axpy": (8.0e12, "GB/s", "hbm"),
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_inputs(tci, ctx, n_upd, chi, complex_dtype_plain, with_plain, with_mixed):
    from paper_2512_23917_amd import synth
    import torch
    w = synth.heisenberg_mpo()
    plain, mixed = [], []
    wt = {}
    if with_plain:
        wt["plain"] = tci.Tensor.from_numpy(ctx, w, tci.C128)
    if with_mixed:
        wt["mixed"] = tci.Tensor.from_numpy(ctx, w.astype(np.complex64), tci.C64)
    t0 = time.time()
    for u in range(n_upd):
        g = synth.rng(2, u)
        a = synth.complex_gaussian(g, (chi, 2, chi))
        b = synth.complex_gaussian(g, (chi, 2, chi))
        left = synth.hermitian_environment(g, chi)
        right = synth.hermitian_environment(g, chi)
        if with_plain:
            plain.append([tci.Tensor.from_numpy(ctx, x, tci.C128) for x in (a, b, left, right)])
        if with_mixed:
            mixed.append([tci.Tensor.from_numpy(ctx, x.astype(np.complex64), tci.C64) for x in (a, b, left, right)])
        if u % 16 == 15:
            log(f"  inputs {u + 1}/{n_upd} ({time.time() - t0:.1f}s)")
    torch.cuda.synchronize()
    return plain, mixed, wt


def run_step(tci, ctx, ins, w, chi, n_matvec, params, thetas, prev=None):
    """One pass of the hot path over the batch; returns the split outputs and energies.
    prev: per update the bond's kept spectrum of the previous step (learned sketch)."""
    energies = []
    for u, (a, b, left, right) in enumerate(ins):
        tci.contract(ctx, a, "asm", b, "mtb", "astb", out=thetas[u])
        energies.append(tci.lanczos_ground(ctx, left, w, w, right, thetas[u], n_matvec))
    return tci.split_batched(ctx, thetas, params, prev_spectra=prev), energies


def time_path(tci, ctx, ins, w, chi, n_matvec, params, steps, warmup, dtype, profile=False, first_params=None):
    """first_params: parameters of the first pass (the learned sketch needs the
    spectra of a previous pass; the first one uses the plain SVD)."""
    import torch
    d = 2
    thetas = [tci.Tensor.empty(ctx, dtype, chi * d * d * chi) for _ in ins]
    for t in thetas:
        tci.reshape(ctx, t, (chi, d, d, chi))
    learned = first_params is not None
    out, prev = None, None
    for i in range(warmup):
        out = run_step(tci, ctx, ins, w, chi, n_matvec, first_params if (learned and prev is None) else params,
                       thetas, prev)
        prev = out[0][1] if learned else None
        log(f"  warmup {i + 1}/{warmup}")
    torch.cuda.synchronize()
    if profile:
        tci.profile_enable(ctx, True)
    t0 = time.perf_counter()
    for i in range(steps):
        out = run_step(tci, ctx, ins, w, chi, n_matvec, first_params if (learned and prev is None) else params,
                       thetas, prev)
        prev = out[0][1] if learned else None
        log(f"  step {i + 1}/{steps}")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = None
    if profile:
        prof = {}
        for tag in tci.profile_tags(ctx):
            prof[tag] = tci.profile_query(ctx, tag)
        tci.profile_enable(ctx, False)
    return dt, out, prof


def traffic_per_launch(kernel, src):
    """HBM bytes per launch of `kernel` from the committed counter summary, or
    None when there is none or the kernel's source changed since it was taken."""
    import hashlib
    if src is None or not os.path.exists(TRAFFIC_FILE):
        return None
    rec = {}
    with open(TRAFFIC_FILE) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                rec[k.strip()] = v.strip()
    if rec.get("kernel") != kernel:
        return None
    with open(os.path.join(ROOT, src), "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    if rec.get("source_sha256") != sha:
        return None
    try:
        return float(rec["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def bench_blocksparse(tci, ctx, n_upd=64, steps=3, eps=1e-8):
    """U(1) block-sparse batch: n_upd independent updates with chi drawn from
    {128, 256, 512, 1024} (21 outer / 22 middle sectors, binomial profile),
    Gaussian float32 blocks, charge-conserving gates, cap = the update's chi,
    all in one call.  The first call runs directly (and tunes the grouped GEMM
    tile), the second records the HIP graph; the timed calls replay it."""
    import torch
    from paper_2512_23917_amd import synth
    g = synth.rng(4, 9999)
    chis = [int(c) for c in g.choice([128, 256, 512, 1024], size=n_upd)]
    A, B, G = [], [], []
    for u, c in enumerate(chis):
        gu = synth.rng(4, 10000 + u)
        bl, bm, br = synth.u1_bond(c, 21), synth.u1_bond(c, 22), synth.u1_bond(c, 21)
        A.append(tci.BsTensor.from_blocks(ctx, bl, bm, {k: v.astype(np.float32)
                                                        for k, v in synth.u1_site_blocks(gu, bl, bm).items()}))
        B.append(tci.BsTensor.from_blocks(ctx, bm, br, {k: v.astype(np.float32)
                                                        for k, v in synth.u1_site_blocks(gu, bm, br).items()}))
        G.append(tci.Tensor.from_numpy(ctx, synth.u1_gate(gu), tci.F64))
    p = tci.update_params(chi_min=1, chi_max=1024, target_trunc_err=eps, direction=tci.DIR_LEFT,
                          precision=tci.PREC_FP32)
    times = []
    out = None
    for i in range(2 + steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = tci.bs_two_site_update_batched(ctx, A, B, G, p, chi_max_each=chis)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        log(f"  block-sparse call {i + 1}/{2 + steps}: {times[-1] * 1e3:.1f} ms")
    t = sum(times[2:]) / steps
    infos = out[3]
    return {"workload": f"U(1) block-sparse batch: {n_upd} updates, chi in {{128,256,512,1024}}, "
                        f"21/22 sectors, f32, eps={eps}, cap=chi, one call",
            "updates_per_s": round(n_upd / t, 3), "ms_per_call": round(1e3 * t, 2),
            "first_call_ms": round(1e3 * times[0], 2), "recording_call_ms": round(1e3 * times[1], 2),
            "chi_mix": {str(c): chis.count(c) for c in (128, 256, 512, 1024)},
            "kept_chi": [min(i.chi for i in infos), max(i.chi for i in infos)],
            "trunc_err_max": float(max(i.trunc_err for i in infos))}


def host_threads():
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    omp = os.environ.get("OMP_NUM_THREADS")
    return min(n, int(omp)) if omp and omp.isdigit() else n


def cpu_baseline(chi, n_matvec, budget_s=20.0):
    """Time the CPU oracle on slices of one update and scale to updates/s.

    Sample: (i) theta = A.B for 96 of the 1024 values of the left index of A
    (scale chi/96); (ii) one effective-Hamiltonian matvec restricted to 96 of
    the 1024 values of the left index a (the L-step and everything after it
    factor over a; scale chi/96), times n_matvec; (iii) the oracle's one-sided
    Jacobi SVD of a complex 800 x 800 Gaussian matrix, scaled by (2048/800)^3
    for the 2048 x 2048 truncated SVD.  Lanczos vector operations are linear in the
    vector length and are included in the matvec slice's scaling.
    """
    import oracle
    from oracle import dmrg as odmrg
    from paper_2512_23917_amd import synth
    g = synth.rng(2, 0)
    a = synth.complex_gaussian(g, (chi, 2, chi))
    b = synth.complex_gaussian(g, (chi, 2, chi))
    left = synth.hermitian_environment(g, chi)
    right = synth.hermitian_environment(g, chi)
    w = synth.heisenberg_mpo()
    x = synth.complex_gaussian(g, (chi, 2, 2, chi))
    oracle.build()
    rows = 96
    t0 = time.perf_counter()
    oracle.contract(a[:rows], "asm", b, "mtb", "astb")
    t_theta = (time.perf_counter() - t0) * (chi / rows)
    t0 = time.perf_counter()
    odmrg.heff_apply(np.ascontiguousarray(left[:rows]), w, w, right, x)
    t_mv = (time.perf_counter() - t0) * (chi / rows)
    n = 800
    m = synth.complex_gaussian(g, (n, n))
    t0 = time.perf_counter()
    oracle.svd_matrix(m)
    t_svd = (time.perf_counter() - t0) * (2 * chi / n) ** 3
    per_update = t_theta + n_matvec * t_mv + t_svd
    return dict(value=1.0 / per_update, unit="updates/s", cores=host_threads(), kind="oracle",
                sample=(f"oracle slices of one chi={chi} update: theta rows {rows}/{chi}, "
                        f"H_eff matvec on {rows}/{chi} left rows x{n_matvec}, Jacobi SVD {n}x{n} scaled "
                        f"(2048/{n})^3; per-update estimate {per_update:.1f}s "
                        f"(theta {t_theta:.1f}s, matvecs {n_matvec * t_mv:.1f}s, svd {t_svd:.1f}s)"))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--updates", type=int, default=64)
    ap.add_argument("--chi", type=int, default=1024)
    ap.add_argument("--nmatvec", type=int, default=20)
    ap.add_argument("--eps", type=float, default=1e-8)
    ap.add_argument("--mixed", choices=["bf16x3", "fp32"], default="bf16x3")
    ap.add_argument("--svd", choices=["learned", "plain"], default="learned",
                    help="truncated SVD of the mixed path: learned sketch rank (plain fallback) or plain")
    ap.add_argument("--model", default=None, help="sketch-model weights (default: the shipped file)")
    ap.add_argument("--plain-steps", type=int, default=1)
    ap.add_argument("--plain-warmup", type=int, default=1)
    ap.add_argument("--skip-plain", action="store_true")
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--skip-blocksparse", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a 1 GiB device-to-device copy three times (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark measures one GPU; --gpus must be 1"}))
        sys.exit(2)

    import torch
    if args.copy_probe:
        n = 1 << 30
        src = torch.ones(n // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": n, "copy_probe_bytes_written": n, "launches": 3}), flush=True)
        return
    from paper_2512_23917_amd import tci
    ctx = tci.Context(0)
    chi, U = args.chi, args.updates
    log(f"bench: {U} dense two-site DMRG updates, chi={chi}, {args.nmatvec} Lanczos matvecs, eps={args.eps}")
    plain_in, mixed_in, wt = make_inputs(tci, ctx, U, chi, tci.C128, not args.skip_plain, True)

    mixed_prec = tci.PREC_BF16X3 if args.mixed == "bf16x3" else tci.PREC_FP32
    ctx.set_precision(mixed_prec)
    pm = tci.update_params(chi_min=1, chi_max=chi, target_trunc_err=args.eps, direction=tci.DIR_RIGHT,
                           precision=mixed_prec)
    first = None
    model = None
    if args.svd == "learned":
        from paper_2512_23917_amd import sketch_train
        model = tci.SketchModel(ctx, path=args.model or sketch_train.DEFAULT_WEIGHTS)
        first = pm
        pm = tci.update_params(chi_min=1, chi_max=chi, target_trunc_err=args.eps, direction=tci.DIR_RIGHT,
                               precision=mixed_prec, svd_mode=tci.SVD_LEARNED, power_iters=2, seed=1)
        pm.sketch_model = model.h.value
    log("mixed path")
    t_mixed, (res_m, en_m), prof = time_path(tci, ctx, mixed_in, wt["mixed"], chi, args.nmatvec, pm,
                                              args.steps, args.warmup, tci.C64, profile=True, first_params=first)
    ups_mixed = U * args.steps / t_mixed
    infos_m = res_m[3]

    ups_plain = None
    en_p = None
    if not args.skip_plain:
        log("plain FP64 path")
        pp = tci.update_params(chi_min=1, chi_max=chi, target_trunc_err=args.eps, direction=tci.DIR_RIGHT,
                               precision=tci.PREC_FP64)
        t_plain, (res_p, en_p), _ = time_path(tci, ctx, plain_in, wt["plain"], chi, args.nmatvec, pp,
                                              args.plain_steps, args.plain_warmup, tci.C128)
        ups_plain = U * args.plain_steps / t_plain

    # dominant kernel class of the measured (mixed) path, summed over call sites
    roof = None
    classes = {}
    if prof:
        by_cls = {}
        for tag, (cnt, ms, work) in prof.items():
            cls = tag.split(":")[1]
            c = by_cls.setdefault(cls, [0, 0.0, 0.0, []])
            c[0] += cnt
            c[1] += ms
            c[2] += work
            c[3].append(tag.split(":")[0])
        cls = max(by_cls, key=lambda k: by_cls[k][1])
        cnt, ms, work, sites = by_cls[cls]
        peak, unit, bound = PEAKS.get(cls, (None, None, None))
        if peak:
            scale = 1e12 if unit == "TFLOP/s" else 1e9
            achieved = work / (ms * 1e-3)
            kname, ksrc = KERNEL_OF_CLASS.get(cls, (cls, None))
            roof = {"bound": bound, "achieved": round(achieved / scale, 2), "peak": peak / scale, "unit": unit,
                    "frac": round(achieved / peak, 4), "traffic": traffic_per_launch(kname, ksrc),
                    "kernel": kname, "call_sites": sorted(set(sites)), "class": cls,
                    "launches": cnt, "avg_launch_ms": round(ms / max(cnt, 1), 4),
                    "work_per_launch": work / max(cnt, 1)}
        share = {k: round(v[1] / (t_mixed * 1e3), 4) for k, v in sorted(prof.items(), key=lambda kv: -kv[1][1])[:8]}
        if roof:
            roof["time_share_top"] = share
        # every class of the mixed path: share of the timed region, achieved
        # rate and fraction of the matching peak (classes with a peak only)
        for k, (c_cnt, c_ms, c_work, _) in sorted(by_cls.items(), key=lambda kv: -kv[1][1]):
            c_peak, c_unit, c_bound = PEAKS.get(k, (None, None, None))
            entry = {"share": round(c_ms / (t_mixed * 1e3), 4), "launches": c_cnt}
            if c_peak:
                c_scale = 1e12 if c_unit == "TFLOP/s" else 1e9
                c_rate = c_work / (c_ms * 1e-3)
                entry.update({"rate": round(c_rate / c_scale, 2), "unit": c_unit, "bound": c_bound,
                              "frac": round(c_rate / c_peak, 4)})
            classes[k] = entry

    bs = None
    if not args.skip_blocksparse:
        log("U(1) block-sparse batch")
        bs = bench_blocksparse(tci, ctx)

    cpu = None
    if not args.skip_cpu:
        log("cpu baseline (oracle sample)")
        cpu = cpu_baseline(chi, args.nmatvec)

    chis = [i.chi for i in infos_m]
    line = {
        "metric": "two-site MPS updates/s at chi=1024, eps=1e-8: learned+mixed vs plain FP64",
        "value": round(ups_mixed, 4),
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * t_mixed / args.steps, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16x3+f64" if args.mixed == "bf16x3" else "f32+f64",
        "data": "synthetic (seeded Gaussian A, B; channel-paired Hermitian Gaussian L, R; Heisenberg MPO)",
        "config": {"workload": f"dense two-site DMRG update chi={chi} d=2 w=5, {args.nmatvec} Lanczos matvecs, "
                               f"trunc_svd eps={args.eps} cap {chi}, {U} updates per step",
                   "updates_per_step": U, "chi": chi, "precision": args.mixed},
        "plain_fp64_updates_per_s": None if ups_plain is None else round(ups_plain, 4),
        "speedup_vs_plain_fp64": None if ups_plain is None else round(ups_mixed / ups_plain, 3),
        "kept_chi": [min(chis), max(chis)],
        "trunc_err": [min(i.trunc_err for i in infos_m), max(i.trunc_err for i in infos_m)],
        "sketch": {"mode": args.svd,
                   "fallback_rate": float(np.mean([i.used_fallback for i in infos_m])),
                   "mean_sketch_rank": float(np.mean([i.sketch_rank for i in infos_m]))},
        "precision_detail": "c64 storage; split-BF16x3 MFMA contractions with FP32 accumulation; "
                            "Krylov basis stored in c64 with FP64 recurrence and orthogonalisation "
                            "arithmetic; FP64 Gram, orthogonalisation and eigensolve of the SVD",
        "energy_parity_mixed_vs_plain": None if en_p is None else
            float(max(abs(a - b) / abs(b) for a, b in zip(en_m, en_p))),
        "roofline": roof,
        "kernel_classes": classes,
        "cpu_baseline": cpu,
        "blocksparse": bs,
    }
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
