#!/usr/bin/env python
"""Fast CPD on one MI355X: EM iterations/s and time-to-converge at M=N=50k, D=3.

Workload (synthetic, seeded): the 50 000-point random spherical-harmonic
surface, scene = model pushed through a Gaussian-RBF field (beta = 1.5),
N(0, 0.02^2) noise, 20% of scene rows replaced by uniform outliers; Fast CPD
with the top K = 300 eigenpairs (randomized, p = 20, q = 2), lambda = 2,
w = 0.2, stop at |dsigma^2| < 1e-8.

A "step" is one full EM iteration (E-step passes A and B, the Fast M-step,
the sigma^2 update) on inputs already resident in HBM.  Warm-up steps run
first, then exactly --steps steps are timed between two synchronisations.
The eigen-prep (t_eig) and a full time-to-converge run are timed separately.

Prints one JSON line.  --gpus above 1 is refused: this path runs on one GPU.
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

METRIC = "time-to-converge (s) & EM iters/s at M=N=50k, 3D; vs plain CPD same GPU"

# Roofline of the E-step passes (ALU bound: O(M + N) bytes against O(M N)
# arithmetic).  The algorithmic work per model-scene pair is counted in FP32
# vector slots of the formulation each kernel implements, one slot being one
# lane-operation at the chip's FP32 vector rate (256 CU x 4 SIMD x 32 lanes x
# 2.4 GHz; x 2 FLOP per FMA = the published 157.3 TFLOP/s).  Non-packed FP32
# FMAs reach 23.4 lanes/cycle/SIMD on the chip (73% of that rate, a
# 32-chain microbenchmark), so the full vector rate, not half of it, is the
# ceiling even with packed FP32 disabled.  v_exp_f32 runs at a quarter of
# the rate (measured 6.8 lanes/cycle/SIMD) and does not overlap the FMAs of
# other waves, so an exponential counts 4 slots.
#   FP32  pass A: 3 sub + 3 (mul, 2 fma) for |y - x|^2, exp, add        = 11
#         pass B: the same 6, add L_n, exp, add (P1), 3 fma (PY), fma (t) = 16
#   BF16X pass A: |y - x|^2 from the matrix cores; exp, add            = 5
#         pass B: exp, sub L_n, add (P1), 3 fma (PY), fma (t)          = 10
# BF16X also spends one v_mfma_f32_16x16x32_bf16 per 256 pairs in the matrix
# pipe; it is not counted.
SLOTS = {("fp32", "passA"): 11, ("fp32", "passB"): 16,
         ("bf16x", "passA"): 5, ("bf16x", "passB"): 10}
PEAK_VALU_FP32_TFLOPS = 157.3  # 256 CU x 4 SIMD x 32 lanes x 2 (FMA) x 2.4 GHz
PEAK_EXP_PER_S = 19.66e12      # v_exp_f32 at a quarter of the vector rate
KERNEL_NAME = {("fp32", "passA"): "k_colsum", ("fp32", "passB"): "k_rowsum",
               ("bf16x", "passA"): "k_bfx_colsum", ("bf16x", "passB"): "k_bfx_rowsum"}
# HBM traffic of the dominant kernel per dispatch, from two rocprofv3 --pmc
# runs (FETCH_SIZE, WRITE_SIZE) scaled by the same counters on a device copy
# of known size; valid only while the kernel source is unchanged (sha256).
TRAFFIC = {
    "k_bfx_rowsum": {"sources": ["bf16x.hip", "bf16x_feat.hpp"],
                     "sha256": "52d80843f998d87370064ae0ad09c9558fb82ddcd7c7bb8209ed1f7aebf969b2",
                     "bytes_per_dispatch": 59.30e6 + 26.00e6,
                     "profile": "profiles/bf16x_rowsum_surface50k_traffic.md"},
    # one Fast M-step at 50k, K = 300: k_tpart4 + k_tmerge4 + k_apply4
    "fast_mstep_k300_50k": {"sources": ["mstep.hip"],
                            "sha256": "24d984a8e8d05c9e3f52dd2aacc18a5a025576108bbc1d099f837395345c1683",
                            "bytes_per_dispatch": (61.69e6 + 1.877e6) + (14.99e6 + 0.019e6)
                                                  + (62.80e6 + 2.425e6),
                            "profile": "profiles/bf16x_rowsum_surface50k_traffic.md"},
}


def traffic_of(key):
    """Measured HBM bytes per dispatch, or None once the source has changed."""
    tr = TRAFFIC.get(key)
    if tr and _source_hash(tr["sources"]) == tr["sha256"]:
        return tr["bytes_per_dispatch"]
    return None


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def _source_hash(names):
    """sha256 over the concatenated bytes of the named csrc files, in order."""
    import hashlib
    m = hashlib.sha256()
    for name in names:
        with open(os.path.join(ROOT, "paper_2006_06281_amd", "csrc", name), "rb") as f:
            m.update(f.read())
    return m.hexdigest()


def roofline_of(kern, pairs, precision):
    """Roofline entry for the dominant kernel (pass B), achieved from its
    average launch time measured with HIP events on the handle's stream."""
    out = {}
    for stage in ("passA", "passB"):
        t = kern[stage] * 1e-3
        slots = SLOTS[(precision, stage)]
        ach = pairs * slots * 2.0 / t / 1e12
        out[stage] = {"kernel": KERNEL_NAME[(precision, stage)], "avg_us": kern[stage] * 1e3,
                      "slots_per_pair": slots, "achieved": ach,
                      "frac": ach / PEAK_VALU_FP32_TFLOPS,
                      "exp_per_s": pairs / t, "exp_frac": pairs / t / PEAK_EXP_PER_S}
    b = out["passB"]
    traffic = traffic_of(b["kernel"])
    return {"bound": "alu", "kernel": b["kernel"] + " (E-step pass B)",
            "achieved": b["achieved"], "peak": PEAK_VALU_FP32_TFLOPS, "unit": "TFLOP/s",
            "frac": b["frac"], "traffic": traffic,
            "flop_model": "FMA-equivalent FP32 vector slots per pair (exp = 4) x pairs per launch",
            "stages": out}


def host_cpu():
    """The host's CPU model and logical CPU count."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "host_cpus": os.cpu_count()}


def cpu_baseline(pair, K, rows=20000):
    """The FP64 oracle as it stands, timed on this host on a bounded sample:
    the E-step and the sigma^2 pass on `rows` model rows against all scene
    points, scaled to M x N pairs, plus one full Fast M-step (K columns)."""
    from oracle import cpd64
    M, N = pair.M, pair.N
    Xs = pair.X[:rows]
    s2 = 0.01
    t0 = time.perf_counter()
    es = cpd64.estep(Xs, pair.Y, s2, pair.w)
    cpd64.sigma2_fast(Xs, pair.Y, s2, es, Xs)
    t_pairs = (time.perf_counter() - t0) * (M / rows)
    rng = np.random.default_rng(0)
    U, _ = np.linalg.qr(rng.standard_normal((M, K)))
    lam = np.sort(rng.random(K))[::-1]
    Yt = pair.X + 0.01
    t0 = time.perf_counter()
    cpd64.fast_mstep(pair.X, Yt, U, lam, pair.lam, s2)
    t_m = time.perf_counter() - t0
    per_iter = t_pairs + t_m
    return {"value": 1.0 / per_iter, "unit": "EM iters/s", "cores": cpd64.threads(),
            "kind": "oracle", **host_cpu(),
            "threads_note": "oracle thread pool = min(16, host CPUs): the host share of "
                            "one GPU is 16 cores",
            "sample": f"E-step + sigma^2 pass on {rows} of {M} model rows x {N} scene "
                      f"points scaled to M x N, plus one full Fast M-step (K={K}); "
                      f"{per_iter:.2f} s per iteration extrapolated"}


def converge_run(reg, pair, t_eig, warmup=3, reps=5):
    """cpd_register to |dsigma^2| < tol from the handle's start state (the
    state it holds when called: Xt and sigma^2), `warmup` untimed runs then
    the median of `reps` timed ones, each restarted from that state."""
    import torch
    X0, _, s20 = reg.state()
    runs = []
    for k in range(warmup + reps):
        reg.set_state(X0, s20)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = reg.register()
        torch.cuda.synchronize()
        if k >= warmup:
            runs.append((time.perf_counter() - t0, out))
    runs.sort(key=lambda r: r[0])
    t, out = runs[len(runs) // 2]
    rmse = float(np.sqrt(((out.Xt.double().cpu().numpy() - pair.Y_hat) ** 2).sum(1).mean()))
    return {"iters": out.iters, "converged": out.converged, "sigma2": out.sigma2,
            "time_to_converge_s": t_eig + t if out.converged else None,
            "time_to_converge_no_eig_s": t if out.converged else None,
            "run_s": t, "runs_s": [r[0] for r in runs], "protocol": f"median of {reps} after "
                                                                     f"{warmup} warm-up runs",
            "t_eig_s": t_eig, "t_c_s": out.t_c, "t_iter_s": out.t_iter,
            "t_o_s": out.t_o, "rmse_eq22": rmse}


PEAK_HBM_GBPS = 8000.0


def mstep_roofline(kern, M, K, elem=4):
    """The Fast M-step reads U (M x K) twice per iteration (U^T R, then
    U (h o T)); its algorithmic bytes are 2 M K elem, against HBM.  The
    measured bytes (counters) are attached for the 50k, K = 300 FP32 case."""
    t = kern["mstep"] * 1e-3
    ach = 2.0 * M * K * elem / t / 1e9
    traffic = traffic_of("fast_mstep_k300_50k") if (M, K, elem) == (50000, 300, 4) else None
    return {"bound": "hbm", "kernel": "Fast M-step (U^T R, U (h o T))", "achieved": ach,
            "peak": PEAK_HBM_GBPS, "unit": "GB/s", "frac": ach / PEAK_HBM_GBPS,
            "traffic": traffic, "bytes_model": "2 M K x 4 B (U read twice)", "avg_us": t * 1e6}


def fast_full_leg(fc, torch, X, Y, pair, precision):
    """Fast CPD with every eigenpair that is not round-off (FULL mode, eq. 17)
    at 50k: eigen-prep, per-iteration rate, and time-to-converge as configured
    (w = 0.2) and at the paper's w = 0.7 (the eigenpairs imported, not
    recomputed)."""
    kw = dict(precision=precision, beta=pair.beta, lam=pair.lam, w=pair.w, eig_mode="full",
              tol=1e-8, max_iter=1000)
    reg = fc.Registration(X, Y, **kw)
    _, _, s2_0 = reg.state()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reg.prepare()
    torch.cuda.synchronize()
    t_eig = time.perf_counter() - t0
    K = reg.K
    log(f"fast full 50k: eigen-prep {t_eig:.3f}s K={K} truncated={reg.eig_truncated}")
    reg.time_kernels(reps=5)
    reg.set_state(X, s2_0)
    kern = reg.time_kernels(reps=10)
    reg.set_state(X, s2_0)
    out = {"K": K, "truncated": reg.eig_truncated, "t_eig_s": t_eig, "kernels_ms": kern,
           "em_iters_per_s": 1000.0 / kern["iteration"],
           "mstep_roofline": mstep_roofline(kern, pair.M, K)}
    out["converge_w0.2"] = converge_run(reg, pair, t_eig, 1, 3)  # 1000 iterations: fewer runs
    U, lam = reg.export_eig()
    reg.close()
    reg7 = fc.Registration(X, Y, **dict(kw, w=0.7, eig_mode="import", K=K))
    reg7.prepare(U=U, lam=lam)
    out["converge_w0.7"] = converge_run(reg7, pair, t_eig)
    reg7.close()
    del U, lam
    torch.cuda.empty_cache()
    log(f"fast full 50k: {out['converge_w0.2']} / {out['converge_w0.7']}")
    return out


def train_net(fc, torch, M=2000, batch=32, triples=100_000, beta=2.0):
    """The warm-start network trained on the device's sphere recipe (cfg5:
    unit-sphere model + N(0, 0.01^2) jitter, RBF field with coefficients
    N(0, s^2), s = 0.3 sqrt(500 / M), 10% uniform outliers), bf16 kernels,
    Adam with a stepped learning rate."""
    coef = 0.3 * np.sqrt(500.0 / M)
    net = fc.WarmStartNet(seed=1)
    steps = -(-triples // batch)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for step in range(steps):
        lr = 1e-3 if step < 0.6 * steps else (3e-4 if step < 0.85 * steps else 1e-4)
        X, Y, V = fc.synth_pairs(batch, M, beta=beta, coef=coef, seed0=10_000_000 + batch * step)
        last = step == steps - 1 or step % 500 == 0
        loss = net.train_step(X, Y, V, beta=beta, lr=lr, want_loss=last)
        if last:
            log(f"warm: train step {step}/{steps} loss {loss:.4f}")
    torch.cuda.synchronize()
    return net, {"train_triples": steps * batch, "train_batch": batch,
                 "train_s": time.perf_counter() - t0, "train_loss_last": loss}


def plain_cpd_legs(fc, torch, X, Y, pair, kw, fast_ms_step):
    """The original CPD M-step (eq. 21) on the same GPU.

    50k: per-iteration time of original CPD on the same inputs (two timed
    iterations; a full run to convergence would take minutes per 100
    iterations).  10k: the 10 000-point surface workload (beta = 2,
    lambda = 3, w = 0.1, 5% outliers) run to |dsigma^2| < 1e-8 by original CPD
    and by Fast CPD with the full eigendecomposition, both in FP32 mode."""
    import synth
    out = {}
    # the original method's E-step runs in fp32 (BF16X is a Fast-CPD mode)
    reg = fc.Registration(X, Y, **dict(kw, method="original", eig_mode="full", K=0,
                                       precision="fp32"))
    reg.prepare()
    k = reg.time_kernels(reps=2)
    out["surface50k_ms_per_iter"] = k["iteration"]
    out["surface50k_mstep_ms"] = k["mstep"]
    out["surface50k_em_iters_per_s"] = 1000.0 / k["iteration"]
    out["fast_over_plain_iter_rate"] = k["iteration"] / fast_ms_step
    flop = pair.M ** 3 / 3.0
    ach = flop / (k["mstep"] * 1e-3) / 1e12
    out["mstep_roofline"] = {"bound": "mfma", "kernel": "original M-step (FP64 Cholesky, "
                                                         "solves, Phi W)",
                             "achieved": ach, "peak": 78.6, "unit": "TFLOP/s",
                             "frac": ach / 78.6, "traffic": None,
                             "flop_model": "M^3 / 3 per iteration (the factorisation)"}
    reg.close()
    del reg
    torch.cuda.empty_cache()
    log(f"plain CPD 50k: {k['iteration']:.1f} ms/iter (M-step {k['mstep']:.1f} ms)")
    p = synth.workload("surface10k")
    X10 = torch.as_tensor(p.X, dtype=torch.float32).cuda().contiguous()
    Y10 = torch.as_tensor(p.Y, dtype=torch.float32).cuda().contiguous()
    base = dict(precision="fp32", beta=p.beta, lam=p.lam, w=p.w, tol=1e-8, max_iter=1000)
    for name, extra in (("original", dict(method="original")),
                        ("fast_full", dict(method="fast", eig_mode="full"))):
        r = fc.Registration(X10, Y10, **base, **extra)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r.prepare()
        torch.cuda.synchronize()
        t_eig = time.perf_counter() - t0
        # original CPD takes seconds per run here: one run
        res = converge_run(r, p, t_eig, *((0, 1) if name == "original" else (3, 5)))
        if name == "fast_full":
            res["K"] = r.K
        out[f"surface10k_{name}"] = res
        log(f"surface10k {name}: {res}")
        r.close()
    o, f = out["surface10k_original"], out["surface10k_fast_full"]
    if o["time_to_converge_s"] and f["time_to_converge_s"]:
        out["surface10k_speedup_time_to_converge"] = o["time_to_converge_s"] / f["time_to_converge_s"]
    return out


def batch_leg(fc, torch, B=256, tune=True, single_n=8):
    """256 independent registrations (surface pairs, M_i, N_i ~ U{500..8000},
    beta_i ~ U[1, 3], lambda_i ~ U[1, 5], w = 0.1, 5% outliers), FULL
    eigen-prep per instance, advanced together by the batched path (FP32)."""
    import synth
    t0 = time.perf_counter()
    pairs = synth.batch_pairs(B=B)
    t_gen = time.perf_counter() - t0
    Xs = [torch.as_tensor(p.X, dtype=torch.float32).cuda() for p in pairs]
    Ys = [torch.as_tensor(p.Y, dtype=torch.float32).cuda() for p in pairs]
    br = fc.BatchRegistration(Xs, Ys, beta=[p.beta for p in pairs], lam=[p.lam for p in pairs],
                              w=0.1, eig_mode="full", tol=1e-8, max_iter=1000)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    br.prepare(tune=tune)
    torch.cuda.synchronize()
    t_prep = time.perf_counter() - t0
    info = br.info()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Xt, res = br.register()
    torch.cuda.synchronize()
    t_run = time.perf_counter() - t0
    iters = [r.iters for r in res]
    pairs_total = float(sum(p.M * p.N for p in pairs))
    rmse = [float(np.sqrt(((x.double().cpu().numpy() - p.Y_hat) ** 2).sum(1).mean()))
            for x, p in zip(Xt, pairs)]
    br.close()
    K = info["K"]
    # U (M_i x K_i FP32) is streamed twice per iteration (T = U^T R, then U T)
    u_bytes = float(sum(4 * p.M * k for p, k in zip(pairs, K)))
    single = single_instance_rate(fc, torch, Xs, Ys, pairs, n=single_n)
    single50 = single_50k_rate(fc, torch)
    pair_rate = float(sum(p.M * p.N * r.iters for p, r in zip(pairs, res))) / t_run
    return {"workload": "batch256: 256 surface pairs, M_i, N_i ~ U{500..8000}, beta_i ~ U[1,3], "
                        "lambda_i ~ U[1,5], w=0.1, 5% outliers; Fast CPD FULL eig, FP32, "
                        "tol 1e-8",
            "instances": B, "sum_MN": pairs_total, "gen_s": t_gen,
            "prepare_s": t_prep, "chunk": info["chunk"], "tile": info["tile"],
            "tune_ms_per_iter": {f"{c}/{t}": v for (c, t), v in info["tune_ms"].items()},
            "K_median": float(np.median(K)), "K_max": int(max(K)),
            "mstep_U_bytes_per_iter": 2 * u_bytes,
            "run_s": t_run, "converged": int(sum(r.converged for r in res)),
            "iters_max": max(iters), "iters_mean": float(np.mean(iters)),
            "instance_iters_per_s": float(sum(iters)) / t_run,
            "pair_updates_per_s": pair_rate,
            "single_instance": single,
            "batch_vs_single_pair_rate": pair_rate / single["pair_updates_per_s"],
            "single_50k": single50,
            "batch_vs_single_50k_pair_rate": pair_rate / single50["pair_updates_per_s"],
            "rmse_median": float(np.median(rmse)), "rmse_max": float(np.max(rmse))}


def single_instance_rate(fc, torch, Xs, Ys, pairs, n=8):
    """The same registrations one at a time through single handles (FP32,
    FULL eigen-prep, tol 1e-8) for the n largest instances: pair updates per
    second of register() alone, the reference rate for the batched path."""
    order = sorted(range(len(pairs)), key=lambda i: -pairs[i].M * pairs[i].N)[:n]
    work, t = 0.0, 0.0
    for i in order:
        p = pairs[i]
        r = fc.Registration(Xs[i], Ys[i], precision="fp32", beta=p.beta, lam=p.lam, w=0.1,
                            eig_mode="full", tol=1e-8, max_iter=1000)
        r.prepare()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = r.register()
        torch.cuda.synchronize()
        t += time.perf_counter() - t0
        work += float(p.M * p.N * out.iters)
        r.close()
    return {"instances": len(order), "which": "the largest M_i N_i", "register_s": t,
            "pair_updates_per_s": work / t}


def single_50k_rate(fc, torch, iters=30):
    """One large single-handle registration at full work for comparison: the
    surface50k pair in FP32, top-K = 300, `iters` EM iterations from the
    start state (culling inactive at that sigma^2), register() alone."""
    import synth
    p = synth.workload("surface50k")
    X = torch.as_tensor(p.X, dtype=torch.float32).cuda()
    Y = torch.as_tensor(p.Y, dtype=torch.float32).cuda()
    r = fc.Registration(X, Y, precision="fp32", beta=p.beta, lam=p.lam, w=p.w, eig_mode="topk",
                        K=300, tol=0.0, max_iter=iters)
    r.prepare()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = r.register()
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    r.close()
    return {"workload": "surface50k FP32 top-K=300", "iters": out.iters, "register_s": t,
            "pair_updates_per_s": float(p.M) * p.N * out.iters / t}


def warm_at_50k(fc, torch, net, M_train, beta, M=50000):
    """The trained network at 50k points (time-to-converge with and without
    the warm start, BF16X, top-K = 300).  The field is a density-weighted
    sum of coefficients, so W0 is scaled by M_train / M.  Two inputs: the
    sphere recipe the network was trained on (in distribution), and the
    50k surface workload with the paper's w = 0.7 (out of distribution)."""
    import synth
    out = {}
    cases = []
    X, Y, V = fc.synth_pairs(1, M, beta=beta, coef=0.3 * np.sqrt(500.0 / M), seed0=77)
    cases.append(("sphere50k", X[0].contiguous(), Y[0].contiguous(), (X + V)[0].double(),
                  dict(beta=beta, lam=3.0, w=0.1)))
    p = synth.workload("surface50k")
    cases.append(("surface50k_w0.7", torch.as_tensor(p.X, dtype=torch.float32).cuda().contiguous(),
                  torch.as_tensor(p.Y, dtype=torch.float32).cuda().contiguous(),
                  torch.as_tensor(p.Y_hat).cuda(), dict(beta=p.beta, lam=p.lam, w=0.7)))
    for name, Xc, Yc, gt, prm in cases:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        W0 = net.forward(Xc[None], Yc[None])[0] * (M_train / M)
        torch.cuda.synchronize()
        t_net = time.perf_counter() - t0
        reg = fc.Registration(Xc, Yc, precision="bf16x", eig_mode="topk", K=300, oversample=20,
                              power_iters=2, seed=0, tol=1e-8, max_iter=1000, **prm)
        t0 = time.perf_counter()
        reg.prepare()
        torch.cuda.synchronize()
        t_eig = time.perf_counter() - t0
        res = {}
        for tag, w0 in (("w0", None), ("net", W0.contiguous())):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            o = reg.register(W0=w0)
            torch.cuda.synchronize()
            run = time.perf_counter() - t0 + (t_net if tag == "net" else 0.0)
            rm = float((o.Xt.double() - gt).square().sum(1).mean().sqrt())
            res[tag] = {"iters": o.iters, "converged": o.converged, "run_s": run,
                        "time_to_converge_s": (t_eig + run) if o.converged else None,
                        "rmse_eq22": rm}
        res["t_eig_s"] = t_eig
        res["net_forward_s"] = t_net
        out[name] = res
        log(f"warm at 50k, {name}: {res}")
        reg.close()
    return out


def warm_leg(fc, torch, M=2000, batch=32, triples=100_000, held_out=1000, chunk=250,
             beta=2.0, lam=3.0, w=0.1):
    """Learned warm start at M = N = 2000: the network is trained on the GPU
    on `triples` pairs of the sphere recipe (unit-sphere model + N(0, 0.01^2)
    jitter, RBF field with coefficients N(0, s^2), s = 0.3 sqrt(500 / M) so
    the field has the size it has at M = 500, 10% uniform outliers in
    [-1.5, 1.5]^3), then `held_out` pairs from disjoint seeds are registered
    twice by the batched path (FULL eigen-prep, FP32, tol 1e-8): from W = 0
    and from the network's W0.  RMSE is against the true position x_m + v_m
    of every model point."""
    coef = 0.3 * np.sqrt(500.0 / M)
    net, tr = train_net(fc, torch, M=M, batch=batch, triples=triples, beta=beta)
    acc = {k: [] for k in ("it0", "itw", "cv0", "cvw", "r0", "rw", "i0", "iw")}
    t_run0 = t_runw = t_net = t_prep = 0.0
    for c0 in range(0, held_out, chunk):
        E = min(chunk, held_out - c0)
        X, Y, V = fc.synth_pairs(E, M, beta=beta, coef=coef, seed0=1 + c0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        W0 = net.forward(X, Y)
        torch.cuda.synchronize()
        t_net += time.perf_counter() - t0
        br = fc.BatchRegistration([X[i] for i in range(E)], [Y[i] for i in range(E)], beta=beta,
                                  lam=lam, w=w, eig_mode="full", tol=1e-8, max_iter=1000)
        t0 = time.perf_counter()
        br.prepare(tune=(c0 == 0))
        torch.cuda.synchronize()
        t_prep += time.perf_counter() - t0
        gt = (X + V).double()
        for tag, w0 in (("0", None), ("w", W0.reshape(-1, 3).contiguous())):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            Xt, res = br.register(W0=w0)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            if tag == "0":
                t_run0 += dt
            else:
                t_runw += dt
            acc["it" + tag] += [r.iters for r in res]
            acc["cv" + tag] += [r.converged for r in res]
            acc["r" + tag] += [float(((Xt[i].double() - gt[i]) ** 2).sum(1).mean().sqrt())
                               for i in range(E)]
        # RMSE of the starting positions: X (W = 0) and X + Phi W0
        for i in range(E):
            x = X[i].double()
            Phi = torch.exp(-torch.cdist(x, x).square() / (2.0 * beta * beta))
            acc["i0"].append(float((x - gt[i]).square().sum(1).mean().sqrt()))
            acc["iw"].append(float((x + Phi @ W0[i].double() - gt[i]).square().sum(1).mean().sqrt()))
        br.close()
        log(f"warm: held-out {c0 + E}/{held_out} registered")
    a = {k: np.asarray(v, dtype=np.float64) for k, v in acc.items()}
    at50k = warm_at_50k(fc, torch, net, M, beta)
    bumps = warm_bumps_leg(fc, torch, M=M)
    log(f"warm: bumps {bumps}")
    return {"at_50k": at50k, "bumps": bumps,
            "workload": f"warm{M}: M=N={M}, D=3, unit sphere + N(0,0.01^2), RBF field beta={beta:g} "
                        f"coef N(0,{coef:.4f}^2), 10% outliers; lambda={lam:g}, w={w:g}; "
                        f"Fast CPD FULL eig, FP32, tol 1e-8",
            **tr, "held_out": held_out,
            "net_forward_s": t_net, "prepare_s": t_prep,
            "iters_mean_w0": float(a["it0"].mean()), "iters_mean_net": float(a["itw"].mean()),
            "iters_median_w0": float(np.median(a["it0"])),
            "iters_median_net": float(np.median(a["itw"])),
            "converged_w0": int(a["cv0"].sum()), "converged_net": int(a["cvw"].sum()),
            "rmse_mean_w0": float(a["r0"].mean()), "rmse_mean_net": float(a["rw"].mean()),
            "rmse_median_w0": float(np.median(a["r0"])),
            "rmse_median_net": float(np.median(a["rw"])),
            "net_worse_rmse_1pct": int((a["rw"] > 1.01 * a["r0"]).sum()),
            "start_rmse_mean_w0": float(a["i0"].mean()),
            "start_rmse_mean_net": float(a["iw"].mean()),
            "run_s_w0": t_run0, "run_s_net": t_runw}


def warm_bumps_leg(fc, torch, M=2000, batch=32, steps=6000, held_out=500, chunk=250, beta=2.0,
                   lam=3.0, w=0.1):
    """The warm start where registration from W = 0 succeeds: the bumps
    recipe (unit sphere pushed out by six random Gaussian bumps, a moderate
    RBF field, 10% outliers), a network trained on it (Adam, lr 3e-5,
    output layer initialised at 1e-6 so training starts from W0 ~ 0), then
    `held_out` pairs from disjoint seeds registered by the batched path from
    W = 0 and from the network's W0; wall times include the forward pass."""
    coef = 0.004 * np.sqrt(1000.0 / M)
    net = fc.WarmStartNet(seed=1, out_scale=1e-6)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for step in range(steps):
        X, Y, V = fc.synth_pairs(batch, M, beta=beta, coef=coef, seed0=10_000_000 + batch * step,
                                 shape="bumps")
        net.train_step(X, Y, V, beta=beta, lr=3e-5, want_loss=False)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    X, Y, V = fc.synth_pairs(held_out, M, beta=beta, coef=coef, seed0=1, shape="bumps")
    gt = (X + V).double()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    W0 = net.forward(X, Y)
    torch.cuda.synchronize()
    t_net = time.perf_counter() - t0
    start0, startw = [], []
    for i in range(held_out):
        x = X[i].double()
        Phi = torch.exp(-torch.cdist(x, x).square() / (2.0 * beta * beta))
        start0.append(float((x - gt[i]).square().sum(1).mean().sqrt()))
        startw.append(float((x + Phi @ W0[i].double() - gt[i]).square().sum(1).mean().sqrt()))
    acc = {t: {"it": [], "cv": 0, "rm": [], "s": 0.0} for t in ("w0", "net")}
    for c0 in range(0, held_out, chunk):
        E = min(chunk, held_out - c0)
        br = fc.BatchRegistration([X[i] for i in range(c0, c0 + E)],
                                  [Y[i] for i in range(c0, c0 + E)], beta=beta, lam=lam, w=w,
                                  eig_mode="full", tol=1e-8, max_iter=1000)
        br.prepare(tune=(c0 == 0))
        for tag, w0 in (("w0", None), ("net", W0[c0:c0 + E].reshape(-1, 3).contiguous())):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            Xt, res = br.register(W0=w0)
            torch.cuda.synchronize()
            a = acc[tag]
            a["s"] += time.perf_counter() - t0
            a["it"] += [r.iters for r in res]
            a["cv"] += int(sum(r.converged for r in res))
            a["rm"] += [float((Xt[i].double() - gt[c0 + i]).square().sum(1).mean().sqrt())
                        for i in range(E)]
        br.close()
    out = {}
    for tag, a in acc.items():
        it, rm = np.array(a["it"], dtype=float), np.array(a["rm"])
        out[tag] = {"iters_mean": float(it.mean()), "iters_median": float(np.median(it)),
                    "converged": a["cv"], "rmse_mean": float(rm.mean()),
                    "rmse_median": float(np.median(rm)),
                    "run_s": a["s"] + (t_net if tag == "net" else 0.0)}
    return {"workload": f"bumps{M}: M=N={M}, unit sphere + six Gaussian bumps, RBF field "
                        f"beta={beta:g} coef N(0,{coef:.5f}^2), 10% outliers; lambda={lam:g}, "
                        f"w={w:g}; Fast CPD FULL eig, FP32, tol 1e-8",
            "train_steps": steps, "train_batch": batch, "train_s": t_train,
            "held_out": held_out, "net_forward_s": t_net,
            "start_rmse_mean_w0": float(np.mean(start0)),
            "start_rmse_mean_net": float(np.mean(startw)),
            "start_sq_error_vs_no_displacement": float(np.mean(np.square(startw)) /
                                                       np.mean(np.square(start0))),
            "from_w0": out["w0"], "from_net": out["net"]}


PEAK_BF16_MFMA_TFLOPS = 2500.0  # dense bf16 matrix rate of the MI355X


def net_gemm_flop(M, N, H=256):
    """Algorithmic matrix-core work of one warm-start training pair: every
    256 x 256 layer (three encoder layers on M + N points, the head's f Wa on
    M points) runs once forward and twice backward (input gradient and
    weight gradient), 2 FLOP per multiply-add."""
    rows = 3 * (M + N) + M
    return 3 * rows * 2 * H * H


def net_gemm_bytes(M, N, H=256):
    """Algorithmic HBM bytes of the same GEMMs for one pair, bf16 storage:
    each layer's forward reads its input and writes its output (R x H
    each), the input gradient reads dY and writes dX, the weight gradient
    reads X and dY: 3 x 2 x R x H x 2 bytes for R rows.  Their arithmetic
    intensity, H / 2 = 128 FLOP per byte at H = 256, is below the bf16
    ridge (2.5 PFLOP/s / 8 TB/s = 312), so HBM bounds them."""
    rows = 3 * (M + N) + M
    return 3 * 2 * rows * H * 2


def warm_train_leg(fc, torch, steps, warmup, M=2000, batch=32, beta=2.0):
    """Training throughput of the warm-start network alone: `warmup` then
    `steps` Adam steps of `batch` device-drawn pairs at M = N = 2000 (pair
    generation, forward, loss, backward, Adam), timed with HIP events on the
    current stream; the GEMM roofline is the algorithmic matrix-core FLOP of
    a step over the step time."""
    coef = 0.3 * np.sqrt(500.0 / M)
    net = fc.WarmStartNet(seed=1)
    st = torch.cuda.current_stream()

    def step(k):
        X, Y, V = fc.synth_pairs(batch, M, beta=beta, coef=coef, seed0=10_000_000 + batch * k)
        net.train_step(X, Y, V, beta=beta, lr=1e-3, want_loss=False)

    for k in range(warmup):
        step(k)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for k in range(steps):
        step(warmup + k)
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    flop = net_gemm_flop(M, M) * batch
    nbytes = net_gemm_bytes(M, M) * batch
    ach = flop / (ms * 1e-3) / 1e12
    bw = nbytes / (ms * 1e-3) / 1e9
    return {"ms_per_step": ms, "pairs_per_s": batch / (ms * 1e-3), "batch": batch, "M": M,
            "N": M, "gemm_flop_per_step": flop, "gemm_bytes_per_step": nbytes,
            "roofline": {"bound": "hbm", "kernel": "whole training step (all kernels)",
                         "achieved": bw, "peak": 8000.0, "unit": "GB/s", "frac": bw / 8000.0,
                         "traffic": None,
                         "bytes_model": "3 x 2 x (3 (M + N) + M) x 256 x 2 B per pair (bf16 "
                                        "GEMM operands; 128 FLOP/B, below the bf16 ridge)"},
            "mfma_view": {"achieved": ach, "peak": PEAK_BF16_MFMA_TFLOPS, "unit": "TFLOP/s",
                          "frac": ach / PEAK_BF16_MFMA_TFLOPS,
                          "flop_model": "3 x (3 (M + N) + M) x 2 x 256^2 per pair"}}


def table4_leg(fc, torch, sizes=(4000, 8000, 12000, 16000, 20000, 24000), iters=50):
    """The paper's scaling protocol (Section IV-B, Table IV) on synthetic
    stand-ins: scene = a random spherical-harmonic surface of M points, model
    = the same points under a random affine map; M = N; every method runs
    exactly `iters` iterations; the low-rank variants keep K = 0.1 M
    eigenpairs (randomized, p = 20, q = 2); beta = 2, lambda = 3, w = 0.1;
    FP32 E-step everywhere (the original and CPD-L solves are FP64).
    Times: t_eig (prepare, host wall), t_c / t_iter / t_o (device events
    inside cpd_register), t_total = t_eig + the register call's wall time."""
    import synth
    methods = (("CPD", dict(method="original")),
               ("CPD-L", dict(method="cpdl", eig_mode="topk")),
               ("Fast-CPD", dict(method="fast", eig_mode="full")),
               ("Fast-CPD-L", dict(method="fast", eig_mode="topk")))
    rows = []
    for M in sizes:
        p = synth.affine_pair(M, seed=M)
        X = torch.as_tensor(p.X, dtype=torch.float32).cuda().contiguous()
        Y = torch.as_tensor(p.Y, dtype=torch.float32).cuda().contiguous()
        for name, kw in methods:
            k = dict(kw)
            if k.get("eig_mode") == "topk":
                k.update(K=M // 10, oversample=20, power_iters=2, seed=0)
            r = fc.Registration(X, Y, precision="fp32", beta=p.beta, lam=p.lam, w=p.w, tol=0.0,
                                max_iter=iters, **k)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r.prepare()
            torch.cuda.synchronize()
            t_eig = time.perf_counter() - t0 if name != "CPD" else 0.0
            t0 = time.perf_counter()
            out = r.register()
            torch.cuda.synchronize()
            run = time.perf_counter() - t0
            rm = float(np.sqrt(((out.Xt.double().cpu().numpy() - p.Y_hat) ** 2).sum(1).mean()))
            row = {"M": M, "method": name, "K": r.K if name != "CPD" else M, "iters": out.iters,
                   "t_c": out.t_c, "t_eig": t_eig, "t_iter": out.t_iter, "t_o": out.t_o,
                   "t_f": t_eig + out.t_iter, "t_total": t_eig + run, "rmse_eq22": rm}
            rows.append(row)
            log(f"table4 {M} {name}: " + ", ".join(f"{a}={b:.4g}" if isinstance(b, float) else
                                                  f"{a}={b}" for a, b in row.items()))
            r.close()
        del X, Y
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--precision", default="bf16x", choices=["fp32", "bf16x"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-converge", action="store_true", help="skip time-to-converge")
    ap.add_argument("--no-plain", action="store_true", help="skip the original-CPD comparator")
    ap.add_argument("--no-full", action="store_true", help="skip Fast CPD with all eigenpairs")
    ap.add_argument("--no-warm", action="store_true", help="skip the learned warm start")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run two 256 MiB device-to-device copies first (a known-size "
                         "reference for hardware byte counters)")
    ap.add_argument("--workload", default="surface50k",
                    choices=["surface50k", "batch256", "warm2000", "warmtrain", "table4",
                             "converge07", "plain50k"],
                    help="batch256 / warm2000 / table4 / converge07 (surface50k at the "
                         "paper's w = 0.7, eigen-prep and one run to tolerance): that leg "
                         "alone, one JSON line of its own")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: this implementation has no multi-GPU path "
              "(each GPU would register its own instances).", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    import paper_2006_06281_amd as fc
    fc.require_device()

    if args.workload == "batch256":
        b = batch_leg(fc, torch)
        log(f"batch: {b}")
        slots = SLOTS[("fp32", "passA")] + SLOTS[("fp32", "passB")]
        ach = b["pair_updates_per_s"] * slots * 2.0 / 1e12
        print(json.dumps({"metric": "batched Fast CPD: instance EM iterations/s",
                          "value": b["instance_iters_per_s"], "unit": "instance EM iters/s",
                          "n_gpus": 1, "higher_is_better": True, "dtype": "f32",
                          "data": "synthetic", "config": {"workload": b["workload"]},
                          "roofline": {"bound": "alu", "kernel": "whole batched run (E-step "
                                                                 "passes dominate)",
                                       "achieved": ach, "peak": PEAK_VALU_FP32_TFLOPS,
                                       "unit": "TFLOP/s", "frac": ach / PEAK_VALU_FP32_TFLOPS,
                                       "traffic": None,
                                       "flop_model": f"{slots} FP32 vector slots per pair and "
                                                     "EM iteration (pass A + pass B, exp = 4)"},
                          "batch": b}), flush=True)
        return

    if args.workload == "table4":
        rows = table4_leg(fc, torch)
        last = [r for r in rows if r["M"] == max(x["M"] for x in rows)]
        fl = next(r for r in last if r["method"] == "Fast-CPD-L")
        print(json.dumps({"metric": "Table IV protocol: total time (s), 50 iterations, per method "
                                    "and size",
                          "value": fl["t_total"], "unit": "s (Fast-CPD-L, largest size)",
                          "n_gpus": 1, "higher_is_better": False, "dtype": "f32",
                          "data": "synthetic",
                          "config": {"workload": "table4: affine surface pairs M=N in "
                                                 "{4k..24k}, K=0.1M, 50 iterations"},
                          "table4": rows}), flush=True)
        return

    if args.workload == "warm2000":
        b = warm_leg(fc, torch)
        log(f"warm: {b}")
        ach = net_gemm_flop(2000, 2000) * b["train_triples"] / b["train_s"] / 1e12
        bw = net_gemm_bytes(2000, 2000) * b["train_triples"] / b["train_s"] / 1e9
        print(json.dumps({"metric": "learned warm start: mean EM iterations to tolerance, "
                                    "held-out pairs",
                          "value": b["iters_mean_net"], "unit": "EM iterations",
                          "n_gpus": 1, "higher_is_better": False, "dtype": "bf16 net, f32 EM",
                          "data": "synthetic", "config": {"workload": b["workload"]},
                          "roofline": {"bound": "hbm", "kernel": "network training (all "
                                                                 "kernels of a step)",
                                       "achieved": bw, "peak": 8000.0, "unit": "GB/s",
                                       "frac": bw / 8000.0, "traffic": None,
                                       "bytes_model": "3 x 2 x (3 (M + N) + M) x 256 x 2 B "
                                                      "per pair"},
                          "mfma_view": {"achieved": ach, "peak": PEAK_BF16_MFMA_TFLOPS,
                                        "unit": "TFLOP/s", "frac": ach / PEAK_BF16_MFMA_TFLOPS},
                          "warm_start": b}), flush=True)
        return

    if args.workload == "warmtrain":
        b = warm_train_leg(fc, torch, args.steps, args.warmup)
        log(f"warmtrain: {b}")
        print(json.dumps({"metric": "warm-start network training pairs/s",
                          "value": b["pairs_per_s"], "unit": "pairs/s", "n_gpus": 1,
                          "steps": args.steps, "warmup": args.warmup,
                          "ms_per_step": b["ms_per_step"], "higher_is_better": True,
                          "dtype": "bf16", "data": "synthetic",
                          "config": {"workload": "warm2000 training: batch 32 pairs, M=N=2000, "
                                                 "sphere recipe drawn on the device"},
                          "roofline": b["roofline"], "train": b}), flush=True)
        return

    if args.workload == "plain50k":
        pair = synth.workload("surface50k")
        X = torch.as_tensor(pair.X, dtype=torch.float32).cuda().contiguous()
        Y = torch.as_tensor(pair.Y, dtype=torch.float32).cuda().contiguous()
        reg = fc.Registration(X, Y, precision="fp32", method="original", beta=pair.beta,
                              lam=pair.lam, w=pair.w, tol=0.0, max_iter=1000)
        reg.prepare()
        k = reg.time_kernels(reps=args.steps)
        flop = pair.M ** 3 / 3.0
        log(f"plain50k: {k}")
        print(json.dumps({"metric": "original CPD (eq. 21) EM iterations/s at M=N=50k",
                          "value": 1000.0 / k["iteration"], "unit": "EM iters/s", "n_gpus": 1,
                          "steps": args.steps, "ms_per_step": k["iteration"],
                          "higher_is_better": True, "dtype": "f64 solve, f32 E-step",
                          "data": "synthetic",
                          "config": {"workload": "surface50k, original CPD, FP64 Cholesky"},
                          "roofline": {"bound": "mfma", "kernel": "M-step (Cholesky, solves, "
                                                                  "Phi W)",
                                       "achieved": flop / (k["mstep"] * 1e-3) / 1e12,
                                       "peak": 78.6, "unit": "TFLOP/s",
                                       "frac": flop / (k["mstep"] * 1e-3) / 1e12 / 78.6,
                                       "traffic": None, "flop_model": "M^3 / 3 per iteration"},
                          "kernels_ms": k}), flush=True)
        return

    if args.workload == "converge07":
        pair = synth.workload("surface50k")
        X = torch.as_tensor(pair.X, dtype=torch.float32).cuda().contiguous()
        Y = torch.as_tensor(pair.Y, dtype=torch.float32).cuda().contiguous()
        reg = fc.Registration(X, Y, precision=args.precision, beta=pair.beta, lam=pair.lam,
                              w=0.7, eig_mode="topk", K=300, oversample=20, power_iters=2,
                              seed=0, tol=1e-8, max_iter=1000)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reg.prepare()
        torch.cuda.synchronize()
        t_eig = time.perf_counter() - t0
        c = converge_run(reg, pair, t_eig)
        log(f"converge07: {c}")
        print(json.dumps({"metric": "time-to-converge (s), surface50k at w = 0.7",
                          "value": c["time_to_converge_s"], "unit": "s",
                          "n_gpus": 1, "higher_is_better": False,
                          "dtype": "bf16x-f32" if args.precision == "bf16x" else "f32",
                          "data": "synthetic",
                          "config": {"workload": "surface50k, w=0.7, Fast CPD top-K=300 "
                                                 "(p=20, q=2), tol 1e-8"},
                          "converge": c}), flush=True)
        return

    if args.copy_calibration:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(2):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 2 x 268435456 bytes device to device")
        del src, dst

    t0 = time.perf_counter()
    pair = synth.workload("surface50k")
    log(f"inputs generated in {time.perf_counter() - t0:.1f}s  M={pair.M} N={pair.N}")
    K, over, q = 300, 20, 2
    X = torch.as_tensor(pair.X, dtype=torch.float32).cuda().contiguous()
    Y = torch.as_tensor(pair.Y, dtype=torch.float32).cuda().contiguous()
    kw = dict(precision=args.precision, beta=pair.beta, lam=pair.lam, w=pair.w,
              eig_mode="topk", K=K, oversample=over, power_iters=q, seed=0, tol=1e-8,
              max_iter=1000)
    reg = fc.Registration(X, Y, **kw)
    _, _, s2_0 = reg.state()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reg.prepare()
    torch.cuda.synchronize()
    t_eig = time.perf_counter() - t0
    log(f"eigen-prep {t_eig:.3f}s  K={reg.K}")

    # per-stage device times (the roofline's live figures) at the initial
    # state, where no tile can be culled; then back to that state.  A kernel
    # trace shows pass B's dispatches 15% slower right after eigen-prep,
    # shortening steadily while the device is busy (across state resets, so
    # the clocks settling, not the state) and flat after about 30 ms of work;
    # 40 untimed repetitions (about 30 ms) come first.
    reg.time_kernels(reps=40)
    reg.set_state(X, s2_0)
    kern = reg.time_kernels(reps=20)
    log("stage ms: " + ", ".join(f"{k}={v:.4f}" for k, v in kern.items()))
    reg.set_state(X, s2_0)

    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        fc.cpd_step(reg.h, want_info=False)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        fc.cpd_step(reg.h, want_info=False)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_step = e0.elapsed_time(e1) / args.steps
    log(f"{args.steps} steps: {ms_step:.3f} ms/step")

    conv = None
    if not args.no_converge:
        conv = {}
        # As configured (w = 0.2), from the same start.
        reg.set_state(X, s2_0)
        conv["w=0.2"] = converge_run(reg, pair, t_eig, 1, 3)  # 1000 iterations: fewer runs
        log(f"w=0.2: {conv['w=0.2']}")
        # The same inputs with the paper's own outlier weight (Section IV,
        # w = 0.7): at w = 0.2 the uniform term does not absorb 20% outliers
        # at this size and the run stalls at sigma^2 ~ 0.05.
        reg7 = fc.Registration(X, Y, **dict(kw, w=0.7))
        t0 = time.perf_counter()
        reg7.prepare()
        torch.cuda.synchronize()
        t_eig7 = time.perf_counter() - t0
        conv["w=0.7"] = converge_run(reg7, pair, t_eig7)
        log(f"w=0.7: {conv['w=0.7']}")
        reg7.close()

    plain = None
    if not args.no_plain:
        plain = plain_cpd_legs(fc, torch, X, Y, pair, kw, ms_step)

    pairs = pair.M * pair.N
    roofline = roofline_of(kern, pairs, args.precision)

    full = None
    if not args.no_full:
        full = fast_full_leg(fc, torch, X, Y, pair, args.precision)

    warm = None
    if not args.no_warm:
        net, tr = train_net(fc, torch)
        warm = {"train": tr, "at_50k": warm_at_50k(fc, torch, net, 2000, 2.0)}
        del net
        torch.cuda.empty_cache()

    # The metric's four rows at M = N = 50k, one GPU.  Time-to-converge is
    # t_eig + the run to |dsigma^2| < 1e-8 (null when 1000 iterations do not
    # get there); "w=0.7" is the same inputs at the paper's outlier weight.
    def _ttc(c):
        return None if c is None else c["time_to_converge_s"]
    modes = {
        "fast_topk": {"K": K, "em_iters_per_s": 1000.0 / ms_step,
                      "time_to_converge_s": {w: _ttc(c) for w, c in (conv or {}).items()},
                      "iters": {w: c["iters"] for w, c in (conv or {}).items()},
                      "roofline": {k: roofline[k] for k in ("bound", "achieved", "peak", "unit",
                                                            "frac")},
                      "mstep_roofline": mstep_roofline(kern, pair.M, K)},
    }
    if full:
        modes["fast_full"] = {
            "K": full["K"], "truncated": full["truncated"],
            "em_iters_per_s": full["em_iters_per_s"],
            "time_to_converge_s": {"w=0.2": _ttc(full["converge_w0.2"]),
                                   "w=0.7": _ttc(full["converge_w0.7"])},
            "iters": {"w=0.2": full["converge_w0.2"]["iters"],
                      "w=0.7": full["converge_w0.7"]["iters"]},
            "roofline": roofline_of(full["kernels_ms"], pairs, args.precision)["stages"]["passB"],
            "mstep_roofline": full["mstep_roofline"]}
    if warm:
        s7 = warm["at_50k"]["surface50k_w0.7"]
        modes["warm_start"] = {
            "em_iters_per_s": 1000.0 / ms_step,
            "time_to_converge_s": {"w=0.7": s7["net"]["time_to_converge_s"],
                                   "w=0.7 from W=0": s7["w0"]["time_to_converge_s"]},
            "iters": {"w=0.7": s7["net"]["iters"], "w=0.7 from W=0": s7["w0"]["iters"]},
            "net_forward_s": s7["net_forward_s"],
            "note": "network trained on the sphere recipe at M=N=2000 (out of distribution "
                    "here); the in-distribution 50k case is in warm_start.at_50k.sphere50k",
            "roofline": {k: roofline[k] for k in ("bound", "achieved", "peak", "unit", "frac")}}
    if plain:
        it7 = (conv or {}).get("w=0.7", {}).get("iters")
        modes["plain_cpd"] = {
            "em_iters_per_s": plain["surface50k_em_iters_per_s"],
            "time_to_converge_s": {"w=0.7 (extrapolated)":
                                   None if it7 is None else it7 * plain["surface50k_ms_per_iter"] / 1e3},
            "extrapolation": "per-iteration time of original CPD at 50k x the iteration count "
                             "of Fast CPD top-K on the same inputs at w=0.7 (at 10k the oracle "
                             "takes 81 iterations for original CPD and 86 for Fast CPD)",
            "roofline": plain["mstep_roofline"]}

    cpu = None
    if not args.no_cpu:
        t0 = time.perf_counter()
        cpu = cpu_baseline(pair, K)
        log(f"cpu baseline {cpu['value']:.4f} it/s ({time.perf_counter() - t0:.1f}s)")

    rec = {
        "metric": METRIC, "value": 1000.0 / ms_step, "unit": "EM iters/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp32": "f32", "bf16x": "bf16x-f32"}[args.precision], "data": "synthetic",
        "config": {"workload": "surface50k: M=N=50000, D=3, spherical-harmonic surface, "
                               "GRBF field beta=1.5, 20% outliers, N(0,0.02^2) noise; Fast CPD "
                               "top-K=300 (p=20, q=2), lambda=2, w=0.2, tol 1e-8",
                   "M": pair.M, "N": pair.N, "D": 3, "K": K, "method": "fast-topk",
                   "precision": args.precision, "parallelism": "single-gpu"},
        "converge": conv, "kernels_ms": kern, "roofline": roofline, "cpu_baseline": cpu,
        "modes": modes, "plain_cpd": plain, "fast_full": full, "warm_start": warm,
        "host": host_cpu(),
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
