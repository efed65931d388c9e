#!/usr/bin/env python3
"""Benchmark of the descriptor hot path: voxel-iterations per second of one
loss/gradient evaluation (multigrid two-point correlations forward, float64
error, adjoint through every level) on one MI355X.

A step is one dmcr_loss_grad over one batch with the field, the target
descriptor and the workspace already resident in HBM.  The default workload
is a 3-D 256^3 two-phase U(0,1) field, P = 32, one level, spectra recomputed
in the adjoint.  The script prints one JSON line with the throughput, the
roofline figure of the dominant kernel (every launch carries a HIP event pair
stamped with the dispatch's own begin and end, in a second pass of the same
steps) and the FP64 oracle timed
on a bounded sample on the host cores.  Unless --no-serve is given it also runs
the continuous-batching serving workload (a Poisson stream of mixed 2-D/3-D,
2-3 phase reconstruction requests) and adds its latency percentiles and its
throughput against one-at-a-time reconstruction under "serving".
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "voxel·iterations/s (S2 fwd+adjoint) vs HBM roofline; p50/p99 solve latency"
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "3d256": dict(desc="3D 256^3 two-phase U(0,1) seed 0, P=32, 1 level, fwd+adjoint with recomputation",
                  shape=(256, 256, 256), C=1, L=1, P=32, recompute=True, batch=1),
    "2d512": dict(desc="2D 512^2 two-phase, P=64, 3-level multigrid (512/256/128), U(0,1) field",
                  shape=(512, 512), C=1, L=3, P=64, recompute=False, batch=1),
    "2d512b64": dict(desc="2D 512^2 two-phase, P=64, 3 levels, batch of 64 fields",
                     shape=(512, 512), C=1, L=3, P=64, recompute=False, batch=64),
    # the same step on batches whose passes (about 270 MB and 540 MB each) exceed the
    # 256 MB Infinity Cache, so that every pass streams from HBM
    "3d256b2": dict(desc="3D 256^3 two-phase U(0,1), P=32, 1 level, fwd+adjoint with recomputation, batch 2",
                    shape=(256, 256, 256), C=1, L=1, P=32, recompute=True, batch=2),
    "3d256b4": dict(desc="3D 256^3 two-phase U(0,1), P=32, 1 level, fwd+adjoint with recomputation, batch 4",
                    shape=(256, 256, 256), C=1, L=1, P=32, recompute=True, batch=4),
    "3d128": dict(desc="3D 128^3 three-phase (C=2), P=32, 3-level multigrid (128/64/32)",
                  shape=(128, 128, 128), C=2, L=3, P=32, recompute=False, batch=1),
    "2d256sbar": dict(desc="2D 256^2 two-phase, soft-threshold descriptor Sbar (alpha=10), P=31, "
                           "3 levels (256/128/64), direct path",
                      shape=(256, 256), C=1, L=3, P=31, recompute=False, batch=1, descriptor=1),
    # the short-displacement case that the shifted-product (direct) path is for
    "2d256direct": dict(desc="2D 256^2 two-phase, S2 product form, P=8, 1 level, batch 64, direct path",
                        shape=(256, 256), C=1, L=1, P=8, recompute=False, batch=64, path=2),
    "2d256s3": dict(desc="2D 256^2 two-phase, S2 (P=31, FFT) + three-point S3 (P3=4: 81 vectors, 3321 pairs), "
                         "3 levels (256/128/64), batch 8",
                    shape=(256, 256), C=1, L=3, P=31, recompute=False, batch=8, s3=4),
}

# Three-point blocks are dense FP32 contractions: the Gram product of the forward
# (N K3 multiply-adds, product form one more multiply) and the M x M cotangent
# product of the adjoint (N M^2 multiply-adds).  On the matrix cores (kernels
# named *_mf) the peak is MI355X's dense FP32 matrix rate, 157.3 TFLOP/s; the FMA
# kernels of small levels run against 256 CUs * 4 SIMDs * 16 lanes * 2 flops *
# 2.4 GHz = 78.6 TFLOP/s (no packed FP32).
MFMA_F32_PEAK_TFLOPS = 157.3
FMA_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12

# Soft-threshold pair terms are bound by FP32 vector issue, not HBM.  A wave64
# FP32 instruction takes 4 cycles of one 16-lane SIMD (packed FP32 is not used),
# the exp and reciprocal 4 times that.  Issue slots (lane-cycles) per term, counted
# from the formula with its constants folded (not from the compiled loop):
#   forward  f((a+b)/2)^2 accumulated: add, fma, exp, add, rcp, fma (f), fma (f f + acc)
#            = 5 plain + 2 quarter-rate = 13;
#   adjoint  K(r) f sigma (1 - sigma) accumulated, the voxel's own k1 phi + k0 and the
#            factor c1 alpha applied once per voxel: fma, exp, add, rcp, fma (f),
#            fma (sigma - sigma^2), mul, fma (acc) = 6 plain + 2 quarter-rate = 14.
# Peak terms/s = 256 CUs * 4 SIMDs * 16 lanes * 2.4 GHz / slots.
VALU_LANE_SLOTS_PER_S = 256 * 4 * 16 * 2.4e9
SOFT_SLOTS = {"direct_fwd_soft": 13, "direct_adj_soft": 14}

# Product-form pair terms on the direct path are one FP32 multiply-add each: the
# forward adds phi_i(x) phi_j(x + r) for every entry r of the block, the adjoint
# adds K(r) phi_j(x + r) over the full box for every channel pair.  They run
# against the same 78.6 TFLOP/s FMA rate (no packed FP32).
DIRECT_KERNELS = ("direct_fwd", "direct_adj")


# the sources the FFT-path kernels (the dominant kernels of every workload) compile from
KERNEL_SOURCES = ("dmcr_internal.h", "fft_path.hip", "fft_plane.hip", "fft_reg.h")


def level_P(spec, l):
    """P of level l as the library applies it: min(P_l, n_l / 2 - 1)."""
    return min(spec.max_disp[l], min(n >> l for n in spec.shape) // 2 - 1)


def K_level(spec, l):
    """Descriptor entries of level l (every pair): half box for autos, full box for crosses."""
    d = len(spec.shape)
    vol = (2 * level_P(spec, l) + 1) ** d
    return sum((vol + 1) // 2 if i == j else vol for (i, j) in spec.pairs)


def source_hash():
    """Hash of the FFT-path kernel sources: a stored counter profile is valid only for this code."""
    import hashlib
    d = os.path.join(ROOT, "paper_2103_09686_amd", "csrc")
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(f.encode())
        h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:16]


def stored_traffic(workload, kernel):
    """HBM bytes per dispatch of `kernel` from the committed rocprofv3 PMC summary of
    this workload (FETCH_SIZE and WRITE_SIZE scaled by the copy-kernel calibration),
    or None if there is none or the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "pmc_%s.txt" % workload)
    if not os.path.exists(path):
        return None
    src, table = None, {}
    for line in open(path):
        line = line.strip()
        if line.startswith("source_hash:"):
            src = line.split(":", 1)[1].strip()
        elif line and not line.startswith("#") and not line.startswith("kernel"):
            f = line.split()
            if len(f) >= 5:
                table[f[0]] = float(f[4]) * 1e6
    if src != source_hash():
        return None
    return table.get(kernel)


def calibrate_copy():
    """Plain device copies of known size (the calibration kernel for the HBM counters
    and the achievable-bandwidth reference)."""
    import torch
    torch.cuda.set_device(0)
    for mib in (64, 256, 1024):
        n = mib * 1024 * 1024 // 4
        a = torch.rand(n, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 10
        print(json.dumps(dict(copy_MiB=mib, us=round(ms * 1e3, 2), GBps_read_plus_write=round(2 * n * 4 / ms / 1e6, 1))),
              flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    # the GPU reaches its steady clock after about 0.1 s of sustained load: 500
    # steps of the 256^3 evaluation (0.11 s) cover it (after 5 the step is ~4% slower)
    ap.add_argument("--warmup", type=int, default=500)
    ap.add_argument("--settle", type=float, default=0.25,
                    help="seconds of sustained steps before the warm-up, so that the GPU clock is steady")
    ap.add_argument("--workload", default="3d256", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target oracle sample time")
    ap.add_argument("--calibrate-copy", action="store_true", help="time plain copies of 64/256/1024 MiB and exit")
    ap.add_argument("--fused-planes", action="store_true",
                    help="3-D levels with 256 x 256 planes take the fused one-pass plane transforms")
    ap.add_argument("--no-alternatives", action="store_true",
                    help="skip the second measurement of the step with the fused 256 x 256 plane transforms")
    ap.add_argument("--no-serve", action="store_true",
                    help="skip the continuous-batching serving workload (latency percentiles)")
    ap.add_argument("--requests", type=int, default=2000, help="serving: requests in the Poisson stream")
    ap.add_argument("--rate", type=float, default=20.0, help="serving: arrivals per second")
    ap.add_argument("--compare", type=int, default=100,
                    help="serving: requests in the batched vs one-at-a-time throughput comparison")
    ap.add_argument("--counters-only", action="store_true",
                    help="run the warm-up and timed steps only (for rocprofv3 --pmc runs): no per-launch "
                         "event pairs, no alternatives, no serving, no CPU baseline")
    ap.add_argument("--optimizer", action="store_true",
                    help="time L-BFGS iterations (m = 10, history full) of the workload's field instead")
    return ap.parse_args()


def optimizer_iterations(args, spec, phi, S_target):
    """L-BFGS iterations of one solver batch: the first 12 fill the history (m = 10),
    then args.steps iterations are timed (wall clock around blocking calls).  Prints
    one JSON line: ms per iteration, evaluations per iteration and the bytes that the
    vector passes of an iteration move, counted per pass."""
    import torch
    from paper_2103_09686_amd import dmcr
    B = phi.shape[0]
    opt = dmcr.Opt(m=10, max_iter=10 ** 6, tol_derr=0.0)
    sv = dmcr.Solver(spec, B, dmcr.Bounds(), opt)
    sv.phi.copy_(phi)
    sv.St.copy_(S_target)
    sv.start(list(range(B)))
    sv.iterate(12)
    torch.cuda.synchronize()
    ev0 = sum(sv.slots[b].evals for b in range(B))
    t0 = time.perf_counter()
    sv.iterate(args.steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    evals = (sum(sv.slots[b].evals for b in range(B)) - ev0) / (B * args.steps)
    out = dict(workload=args.workload, optimizer="lbfgs m=10", batch=B, iterations=args.steps,
               ms_per_iteration=round(dt * 1e3 / args.steps, 4), evaluations_per_iteration=round(evals, 3),
               E=[sv.slots[b].E for b in range(B)])
    print(json.dumps(out), flush=True)


def serving(n_requests, rate, n_compare):
    """Serving workload: Poisson stream (rate, n_requests), sizes uniform over 2-D
    128^2..1024^2 and 3-D 64^3..256^3, 2-3 phases, Boolean or GRF targets, stop at
    E <= 1e-4 or 2000 iterations.  Reports latency percentiles from arrival to result
    and the throughput of continuous batching against plain one-at-a-time GPU
    reconstruction on the same requests (all available at once)."""
    import copy

    import numpy as np
    import torch
    from paper_2103_09686_amd import dmcr, serve

    t0 = time.perf_counter()
    cache = serve.TargetCache(variants=2)
    stream = serve.request_stream(n_requests, rate, seed=0)
    reqs = serve.gpu_requests(stream, cache)
    prep = time.perf_counter() - t0
    print("serving: %d requests prepared in %.1f s" % (len(reqs), prep), file=sys.stderr, flush=True)
    opt = dmcr.Opt(max_iter=2000, tol_derr=1e-4)
    budget = int(0.6 * torch.cuda.mem_get_info()[0])
    srv = serve.Server(serve.GpuExecutor(opt=opt), budget_bytes=budget, iters_per_tick=4, threads=8,
                       asynchronous=True)
    done = srv.run(reqs)
    srv.close()
    live = serve.summary(done)
    print("serving (Poisson %.0f/s): %s" % (rate, live), file=sys.stderr, flush=True)
    # throughput comparison on the first n_compare requests, all available at t = 0;
    # both sides keep their result fields on the device for the rounded-field error
    base = serve.gpu_requests(stream[:n_compare], cache)
    for r in base:
        r.arrival = 0.0
    batched = copy.copy(base)
    ex = serve.GpuExecutor(opt=opt, keep_fields=True)
    srv = serve.Server(ex, budget_bytes=budget, iters_per_tick=4, threads=8, asynchronous=True)
    torch.cuda.synchronize()
    tb = time.perf_counter()
    bdone = srv.run([copy.copy(r) for r in batched])
    torch.cuda.synchronize()
    tb = time.perf_counter() - tb
    bfields = {}
    for g in srv.groups.values():
        bfields.update(g.fields_by_rid)
    brnd = serve.rounded_errors(bdone, bfields)
    srv.close()
    del bfields
    seq = [copy.copy(r) for r in base]
    bufs = serve.sequential_buffers(seq, opt)      # every class resident before the clock starts
    torch.cuda.synchronize()
    ts = time.perf_counter()
    _, sfields = serve.run_sequential(seq, opt=opt, bufs=bufs, keep_fields=True)
    torch.cuda.synchronize()
    ts = time.perf_counter() - ts
    srnd = serve.rounded_errors(seq, sfields)
    del sfields, bufs
    bsum, ssum = serve.summary(bdone), serve.summary(seq)

    def rnd_stats(rd):
        e = [v[0] for v in rd.values()]
        rel = [v[1] for v in rd.values()]
        return dict(rounded_E_p50=float(np.percentile(e, 50)), rounded_E_max=float(max(e)),
                    rounded_rel_err_p50=float(np.percentile(rel, 50)), rounded_rel_err_max=float(max(rel)))

    out = dict(requests=live["requests"], rate_per_s=rate, p50_s=round(live["p50_s"], 4),
               p99_s=round(live["p99_s"], 4), mean_s=round(live["mean_s"], 4),
               served_requests_per_s=round(live["requests_per_s"], 3),
               converged=live["converged"], max_final_E=live["max_final_E"],
               iters_per_request=dict(mean=round(live["iters_mean"], 2), p50=live["iters_p50"],
                                      p99=live["iters_p99"]),
               rel_err_p50=live.get("rel_err_p50"), rel_err_max=live.get("rel_err_max"),
               compare=dict(requests=n_compare, batched_requests_per_s=round(n_compare / tb, 2),
                            one_at_a_time_requests_per_s=round(n_compare / ts, 2), speedup=round(ts / tb, 2),
                            batched_max_E=max(r.final_E for r in bdone), one_at_a_time_max_E=max(r.final_E for r in seq),
                            batched_rel_err_max=bsum.get("rel_err_max"),
                            one_at_a_time_rel_err_max=ssum.get("rel_err_max"),
                            batched_iters_mean=round(bsum["iters_mean"], 2),
                            one_at_a_time_iters_mean=round(ssum["iters_mean"], 2),
                            batched_voxel_it_per_s=sum(r.voxels * r.iters for r in bdone) / tb,
                            one_at_a_time_voxel_it_per_s=sum(r.voxels * r.iters for r in seq) / ts,
                            batched_rounded=rnd_stats(brnd), one_at_a_time_rounded=rnd_stats(srnd)),
               prepare_s=round(prep, 1))
    print("serving compare: %s" % out["compare"], file=sys.stderr, flush=True)
    return out


def cpu_baseline(phi64, spec_kw, target_seconds):
    """Time the FP64 oracle on a bounded sample of one evaluation and scale it to the
    whole evaluation: forward over k_s sampled displacements (all voxels each) and
    adjoint at n_s sampled voxels (all displacements each)."""
    import numpy as np
    import oracle

    oracle.build()
    shape, P, L = spec_kw["shape"], spec_kw["P"], spec_kw["L"]
    d = len(shape)
    C = phi64.shape[0]
    kind = ["s2", "sbar", "stilde"][spec_kw.get("descriptor", 0)]
    ospec = oracle.Spec(shape=shape, n_channels=C, n_levels=L, descriptor=kind,
                        max_disp=tuple(min(P, min(s >> l for s in shape) // 2 - 1) for l in range(L)))
    if kind == "s2":
        fwd = oracle._native.corr
        adj_at = oracle._native.corr_adjoint_at
    else:
        c = oracle.soft_threshold_constants(ospec.alpha)
        fwd = lambda a, b, r: oracle._native.sbar(a, b, r, ospec.alpha, c)
        adj_at = lambda a, b, r, G, v: oracle._native.sbar_adjoint_at(a, b, r, ospec.alpha, c, G, v)
    lv = oracle.pyramid(phi64, L)
    rng = np.random.default_rng(0)
    # finest level, first pair: cost per displacement = N MACs, per voxel = K MACs (x2 in the adjoint)
    l0 = [e for e in ospec.layout() if e[0] == 0]
    (_, pair, off, k) = l0[0]
    rs = ospec.disp(0, pair)
    N = int(np.prod(shape))
    # calibrate with a tiny sample, then size the real ones: three independent
    # samples of each, a sixth of the budget apiece, and the median per-unit time
    t0 = time.perf_counter()
    fwd(lv[0][pair[0]], lv[0][pair[1]], rs[:4])
    t_per_r = max((time.perf_counter() - t0) / 4, 1e-6)
    k_s = int(max(8, min(len(rs), target_seconds / 6 / t_per_r)))
    G = rng.standard_normal(k)
    vox = rng.integers(0, min(shape), size=(64, d))
    t0 = time.perf_counter()
    adj_at(lv[0][pair[0]], lv[0][pair[1]], rs, G, vox)
    t_per_v = max((time.perf_counter() - t0) / 64, 1e-9)
    n_s = int(max(64, min(N, target_seconds / 6 / t_per_v)))
    reps_f, reps_a = [], []
    for _ in range(3):
        sel = rng.choice(len(rs), k_s, replace=False)
        t0 = time.perf_counter()
        fwd(lv[0][pair[0]], lv[0][pair[1]], rs[sel])
        reps_f.append(time.perf_counter() - t0)
        vox = rng.integers(0, min(shape), size=(n_s, d))
        t0 = time.perf_counter()
        adj_at(lv[0][pair[0]], lv[0][pair[1]], rs, G, vox)
        reps_a.append(time.perf_counter() - t0)
    t_fwd = sorted(reps_f)[1]
    t_adj = sorted(reps_a)[1]
    # whole evaluation: every (level, pair) block, forward over its displacements and
    # adjoint over its voxels, scaled by the measured per-unit times (cost ~ N_l * K_lp)
    t_full = 0.0
    for (l, p2, o2, k2) in ospec.layout():
        Nl = N >> (d * l)
        frac = (Nl / N)
        t_full += (t_fwd / k_s) * k2 * frac + (t_adj / n_s) * Nl * (k2 / k)
    sample = ("median of 3 samples, each %d of %d displacements (all %d voxels) forward + %d voxels "
              "(all %d displacements) adjoint of level 0, pair %s; scaled to all levels and pairs by N_l*K_lp"
              % (k_s, len(rs), N, n_s, len(rs), pair))
    P3 = spec_kw.get("s3", 0)
    if P3 > 0:
        # three-point blocks: forward and adjoint over all voxels for a sample of
        # the vector pairs, scaled by pairs and by N_l
        mode, alpha, cc = (0, 0.0, (0.0, 0.0, 0.0)) if kind == "s2" else \
            (1, ospec.alpha, oracle.soft_threshold_constants(ospec.alpha))
        vecs = oracle.box(d, min(P3, ospec.max_disp[0]))
        ia, ib = np.triu_indices(len(vecs))
        ks = min(len(ia), 64)
        sel = rng.choice(len(ia), ks, replace=False)
        t0 = time.perf_counter()
        oracle._native.s3(lv[0][0], vecs, ia[sel], ib[sel], mode, alpha, cc)
        t3f = time.perf_counter() - t0
        t0 = time.perf_counter()
        oracle._native.s3_adjoint(lv[0][0], vecs, ia[sel], ib[sel], mode, np.ones(ks), alpha, cc)
        t3a = time.perf_counter() - t0
        for l in range(L):
            Nl = N >> (d * l)
            M3 = (2 * min(P3, ospec.max_disp[l]) + 1) ** d
            t_full += C * (t3f + t3a) / ks * (M3 * (M3 + 1) // 2) * (Nl / N)
        sample += "; three-point: %d of %d pairs forward and adjoint over all voxels, scaled by pairs and N_l" % (
            ks, len(ia))
    return dict(value=N / t_full, unit="voxel·it/s", cores=oracle._native.num_threads(), kind="oracle",
                sample=sample, seconds=sum(reps_f) + sum(reps_a),
                spread=[round(min(reps_f) / max(reps_f), 3), round(min(reps_a) / max(reps_a), 3)])


def main():
    args = parse()
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2103_09686_amd import dmcr, synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    wl = WORKLOADS[args.workload]
    shape, C, L, P, B = wl["shape"], wl["C"], wl["L"], wl["P"], wl["batch"]
    flags = dmcr.FLAG_RECOMPUTE if wl["recompute"] else 0
    if args.fused_planes:
        flags |= dmcr.FLAG_FUSED_PLANES
    desc = wl.get("descriptor", dmcr.DESC_S2)
    spec = dmcr.make_spec(shape, C, L, P, flags=flags, descriptor=desc, s3_max_disp=wl.get("s3", 0),
                          path=wl.get("path", dmcr.PATH_AUTO))
    K = dmcr.dmcr_descriptor_size(spec)
    N = int(np.prod(shape))

    phi_h = np.stack([synth.uniform(shape, b, channels=C) for b in range(B)]).astype(np.float32)
    phi = torch.from_numpy(phi_h).cuda()
    # target descriptor: a seeded Boolean sphere medium (3-D) / disk medium (2-D), per channel
    tgt = np.concatenate([synth.boolean_spheres(shape, 6 if len(shape) == 3 else 4, 0.2 + 0.05 * c,
                                                seed=1000 + c)[0] for c in range(C)])
    S_t = dmcr.dmcr_descriptor_forward(spec, torch.from_numpy(tgt[None].astype(np.float32)).cuda())
    S_target = S_t.double().repeat(B, 1).contiguous()
    E = torch.empty(B, dtype=torch.float64, device="cuda")
    grad = torch.empty_like(phi)
    ws = dmcr.workspace(dmcr.dmcr_workspace_size(spec, B))
    stream = torch.cuda.current_stream()

    def step():
        dmcr.dmcr_loss_grad(spec, phi, S_target, E, grad, ws)

    if args.optimizer:
        optimizer_iterations(args, spec, phi, S_target)
        return

    import ctypes
    lib = dmcr.lib()
    lib.dmcr_profile_start.restype = ctypes.c_int
    lib.dmcr_profile_stop.restype = ctypes.c_int32

    class KStat(ctypes.Structure):
        _fields_ = [("name", ctypes.c_char * 48), ("launches", ctypes.c_int32),
                    ("total_ms", ctypes.c_double), ("bytes", ctypes.c_double)]

    lib.dmcr_profile_stop.argtypes = [ctypes.POINTER(KStat), ctypes.c_int32]

    def settle(fn):
        """Run the step for args.settle seconds of sustained load first: a fresh GPU runs
        its first ~0.1 s of load below its steady clock (the 256^3 step reads 4-6%
        slower there), which a handful of warm-up steps does not cover."""
        t_end = time.perf_counter() + args.settle
        while time.perf_counter() < t_end:
            for _ in range(8):
                fn()
            torch.cuda.synchronize()

    def timed(fn):
        """Settle, warm-up, then args.steps steps between two events on the launch stream:
        ms per step."""
        settle(fn)
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        wall0 = time.perf_counter()
        t0.record(stream)
        for _ in range(args.steps):
            fn()
        t1.record(stream)
        torch.cuda.synchronize()
        ms = t0.elapsed_time(t1) / args.steps
        print("timed %d steps: %.4f ms/step (wall %.3f s)" % (args.steps, ms, time.perf_counter() - wall0),
              file=sys.stderr, flush=True)
        return ms

    def kernel_table(fn):
        """Second pass of the same steps, every launch timed by the event pair it carries."""
        lib.dmcr_profile_start()
        for _ in range(args.steps):
            fn()
        stats = (KStat * 64)()
        nk = lib.dmcr_profile_stop(stats, 64)
        torch.cuda.synchronize()
        kern = []
        for i in range(min(nk, 64)):
            s = stats[i]
            kern.append(dict(name=s.name.decode(), launches=s.launches, avg_us=1e3 * s.total_ms / s.launches,
                             total_ms=s.total_ms, bytes_per_launch=s.bytes / s.launches,
                             GBps=(s.bytes / s.launches) / (s.total_ms / s.launches * 1e-3) / 1e9))
        kern.sort(key=lambda r: -r["total_ms"])
        for r in kern:
            print("  %-16s n=%-5d avg %9.2f us  %8.1f GB/s  (%.1f MB/launch)" %
                  (r["name"], r["launches"], r["avg_us"], r["GBps"], r["bytes_per_launch"] / 1e6),
                  file=sys.stderr, flush=True)
        return kern

    def step_percentiles(fn, n=1000):
        """Per-step GPU time: an event pair around each of n back-to-back steps on the
        launch stream (after the timed region, so the clock is steady)."""
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
        for a, b in evs:
            a.record(stream)
            fn()
            b.record(stream)
        torch.cuda.synchronize()
        t = sorted(a.elapsed_time(b) for a, b in evs)
        return dict(steps=n, p50_ms=round(t[n // 2], 5), p99_ms=round(t[int(0.99 * (n - 1))], 5),
                    max_ms=round(t[-1], 5))

    ms = timed(step)
    value = N * B / (ms * 1e-3)
    if args.counters_only:
        # for hardware-counter runs: the plain steps only (no event-stamped launches)
        print(json.dumps(dict(workload=args.workload, ms_per_step=ms, value=value)), flush=True)
        return
    step_time = step_percentiles(step)
    print("per-step GPU time: %s" % step_time, file=sys.stderr, flush=True)
    kern = kernel_table(step)
    dom = kern[0]
    prof_ms = sum(r["total_ms"] for r in kern) / args.steps
    if dom["name"] in SOFT_SLOTS:
        # pair terms per step: forward N_l * K_l (every pair), adjoint N_l * C^2 * box_l^d
        d = len(shape)
        terms = {"direct_fwd_soft": 0.0, "direct_adj_soft": 0.0}
        for l in range(L):
            Nl = N >> (d * l)
            box = 2 * level_P(spec, l) + 1
            terms["direct_fwd_soft"] += B * Nl * K_level(spec, l)
            terms["direct_adj_soft"] += B * Nl * C * C * box ** d
        per_launch = terms[dom["name"]] / L
        achieved = per_launch / (dom["avg_us"] * 1e-6) / 1e9
        peak = VALU_LANE_SLOTS_PER_S / SOFT_SLOTS[dom["name"]] / 1e9
        roofline = dict(bound="alu", kernel=dom["name"], achieved=round(achieved, 1), peak=round(peak, 1),
                        unit="Gterm/s", frac=round(achieved / peak, 4), traffic=None,
                        avg_us=round(dom["avg_us"], 2), terms_per_launch=per_launch)
    elif dom["name"] in DIRECT_KERNELS:
        # multiply-adds per step: forward N_l * K_l (every pair), adjoint N_l * C^2 * box_l^d
        d = len(shape)
        fl = {"direct_fwd": 0.0, "direct_adj": 0.0}
        for l in range(L):
            Nl = N >> (d * l)
            box = 2 * level_P(spec, l) + 1
            fl["direct_fwd"] += 2.0 * B * Nl * K_level(spec, l)
            fl["direct_adj"] += 2.0 * B * Nl * C * C * box ** d
        per_launch = fl[dom["name"]] / L
        achieved = per_launch / (dom["avg_us"] * 1e-6) / 1e12
        roofline = dict(bound="alu", kernel=dom["name"], achieved=round(achieved, 2), peak=round(FMA_PEAK_TFLOPS, 1),
                        unit="TFLOP/s", frac=round(achieved / FMA_PEAK_TFLOPS, 4), traffic=None,
                        avg_us=round(dom["avg_us"], 2), flops_per_launch=per_launch)
    elif dom["name"].startswith(("s3_fwd", "s3_adj_terms", "s3_adj_mf")):
        d = len(shape)
        flops = 0.0
        for l in range(L):
            Nl = N >> (d * l)
            P3 = min(spec.s3_max_disp, level_P(spec, l))
            M = (2 * P3 + 1) ** d
            if dom["name"].startswith("s3_fwd"):
                flops += B * C * Nl * (M * (M + 1) // 2) * (2 if desc else 3)
            else:
                flops += B * C * Nl * M * M * 2
        per_launch = flops / L
        achieved = per_launch / (dom["avg_us"] * 1e-6) / 1e12
        mf = "_mf" in dom["name"]
        peak = MFMA_F32_PEAK_TFLOPS if mf else FMA_PEAK_TFLOPS
        roofline = dict(bound="mfma" if mf else "alu", kernel=dom["name"], achieved=round(achieved, 2),
                        peak=round(peak, 1), unit="TFLOP/s", frac=round(achieved / peak, 4), traffic=None,
                        avg_us=round(dom["avg_us"], 2), flops_per_launch=per_launch)
    else:
        roofline = dict(bound="hbm", kernel=dom["name"], achieved=round(dom["GBps"], 1), peak=HBM_PEAK_GBS,
                        unit="GB/s", frac=round(dom["GBps"] / HBM_PEAK_GBS, 4),
                        traffic=stored_traffic(args.workload + ("fused" if args.fused_planes else ""), dom["name"]),
                        avg_us=round(dom["avg_us"], 2), bytes_per_launch=dom["bytes_per_launch"],
                        source_hash=source_hash())
    total_bytes = sum(r["bytes_per_launch"] * r["launches"] for r in kern) / args.steps
    step_roofline = dict(bytes_per_step=total_bytes, bytes_per_voxel=total_bytes / (N * B),
                         achieved_GBps=round(total_bytes / (ms * 1e-3) / 1e9, 1),
                         frac=round(total_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                         kernel_ms_sum=round(prof_ms, 4))
    if roofline["bound"] == "alu" and roofline["kernel"] in DIRECT_KERNELS:
        # the whole step against the FMA rate: every product term at two flops
        flops = sum(fl.values())
        step_roofline = dict(bound="alu", flops_per_step=flops,
                             frac=round(flops / (ms * 1e-3) / (FMA_PEAK_TFLOPS * 1e12), 4),
                             kernel_ms_sum=round(prof_ms, 4))
    if roofline["bound"] == "alu" and roofline["unit"] == "Gterm/s":
        # the whole step against FP32 issue: every soft term at its slot cost
        slots = sum(terms[k] * SOFT_SLOTS[k] for k in terms)
        step_roofline = dict(bound="alu", terms_per_step=sum(terms.values()), issue_slots_per_step=slots,
                             frac=round(slots / (ms * 1e-3) / VALU_LANE_SLOTS_PER_S, 4),
                             kernel_ms_sum=round(prof_ms, 4))

    out = dict(metric=METRIC, value=value, unit="voxel·it/s", n_gpus=1, steps=args.steps,
               warmup=args.warmup, settle_s=args.settle, ms_per_step=ms, step_time=step_time,
               higher_is_better=True, scaling="weak",
               vs_baseline=None, dtype="f32", data="synthetic",
               config=dict(workload=wl["desc"], shape=list(shape), channels=C, levels=L,
                           max_disp=[level_P(spec, l) for l in range(L)], K=K, batch=B,
                           path="direct" if desc or wl.get("path") == dmcr.PATH_DIRECT else "fft",
                           descriptor=["s2", "sbar", "stilde"][desc], s3_max_disp=spec.s3_max_disp,
                           recompute=wl["recompute"], fused_planes_256=bool(args.fused_planes),
                           parallelism="single GPU"),
               roofline=roofline, step_roofline=step_roofline)
    if len(shape) == 3 and shape[1] == shape[2] == 256 and not desc and not (args.fused_planes or
                                                                              args.no_alternatives):
        # the same step with the fused one-pass plane transforms of 256 x 256 planes (opt-in)
        spec_f = dmcr.make_spec(shape, C, L, P, flags=flags | dmcr.FLAG_FUSED_PLANES, descriptor=desc,
                                s3_max_disp=wl.get("s3", 0))
        ws_f = dmcr.workspace(dmcr.dmcr_workspace_size(spec_f, B))

        def step_f():
            dmcr.dmcr_loss_grad(spec_f, phi, S_target, E, grad, ws_f)

        print("alternative: fused 256 x 256 plane transforms", file=sys.stderr, flush=True)
        ms_f = timed(step_f)
        kern_f = kernel_table(step_f)
        bytes_f = sum(r["bytes_per_launch"] * r["launches"] for r in kern_f) / args.steps
        out["alternatives"] = [dict(
            flags="FUSED_PLANES", ms_per_step=ms_f, value=N * B / (ms_f * 1e-3),
            dominant_kernel=kern_f[0]["name"], dominant_avg_us=round(kern_f[0]["avg_us"], 2),
            dominant_frac=round(kern_f[0]["GBps"] / HBM_PEAK_GBS, 4), bytes_per_step=bytes_f,
            step_frac=round(bytes_f / (ms_f * 1e-3) / 1e9 / HBM_PEAK_GBS, 4))]
        del ws_f
    if not args.no_serve and args.workload == "3d256":
        out["serving"] = serving(args.requests, args.rate, args.compare)
    if not args.no_cpu_baseline:
        phi64 = phi_h[0].astype(np.float64)
        cb = cpu_baseline(phi64, dict(shape=shape, P=P, L=L, descriptor=desc, s3=wl.get("s3", 0)), args.cpu_seconds)
        out["cpu_baseline"] = dict(value=cb["value"], unit=cb["unit"], cores=cb["cores"], kind=cb["kind"],
                                   sample=cb["sample"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
