"""Benchmark of the visibility simulator hot path on one MI355X.

Headline workload: the diffuse sky with the learned beam -- 350 hex antennas
(14.6 m) with 2 feeds x 2 E-field axes, 3 145 728 equal-area pixels (nside-512
equivalent) with a log-normal brightness, the Fourier-feature network in place
of beam interpolation, BF16X3 product.  The full configuration has 64 LSTs x the
64 channels of 50-250 MHz that lie inside the network's 100-200 MHz band (4096
(t, nu) instances); one step here is a stated sample of them (by default 2
LSTs x 8 channels spread over the band, 16 instances), every step of Alg. 2 for
the whole sample in one matvis_simulate call, replayed from its captured
hipGraph.  All inputs are seeded synthetic arrays already resident in HBM when
timing starts.  The network is trained first, on the GPU, by the library's own
kernels (paper_2312_09763_amd.learned_beam, seeded), and the context
configuration is the autotuner's choice (matvis_autotune, cached in
paper_2312_09763_amd/tuning/).

metric: src * ant-pair * (t, nu) / s = n_src * n_ant (n_ant + 1) / 2 * n_t * n_nu / T.

Also on the same JSON line:
* roofline: the dominant kernel of the step -- the product over sources for
  the off-diagonal pairs of 128-antenna blocks, timed live with HIP events
  around each of its launches (a profiled pass over the same steps) -- against
  the bf16 dense MFMA peak.  Algorithmic flops per launch: for every visible
  source, 4 full block products V^00, V^11, V^10 and V^01 of n_I x n_J antennas
  for every block pair I > J (8 flops per complex multiply-add), x 3 products
  on BF16X3; the whole product (both launches) is reported beside it;
* error_vs_oracle: err_CS / err_F of the headline's visibilities against the
  FP64 direct sum with the interpolated beam, on sampled antenna pairs (plus
  the autocorrelations the Cauchy-Schwarz scale needs) of two instances;
* cpu_baseline: the FP64 direct-sum oracle on a bounded sample of the same
  workload (one instance, a seeded set of antenna pairs, every pixel), at the
  host's thread count and at one thread, with the CPU model;
* side_by_side: the same sample through the FP64 interpolated path, FP32 and
  BF16X3 with the interpolated beam;
* secondary: the 128-antenna, 50 000-source polarised workload (32 x 16
  instances) with its own product roofline and the bandwidth-bound steps;
* workloads, redundancy: the other synthetic workloads, and the sub-matrix
  product of App. A against the full product.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0}  # dense MFMA, MI355X
HBM_GBS = 8000.0
PRODUCTS = {"fp64": 1, "fp32": 1, "bf16x3": 3}
TUNING = os.path.join(ROOT, "paper_2312_09763_amd", "tuning", "gfx950.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def block_sizes(n_ant: int):
    return [min(128, n_ant - 128 * b) for b in range((n_ant + 127) // 128)]


def product_flops(path: str, n_ant: int, n_feed: int, n_ax: int, counts_t, n_freq: int):
    """Algorithmic (own-work) flops of one step's product, without the x3 of BF16X3:
    (whole product, first launch, block-pair launch).  Product over sources: per
    visible source, the V^00 and V^11 lower triangles and the full V^10 of every
    diagonal block, and four full n_I x n_J products for every block pair.  Z Z^H:
    4 N (N + 1) K over the lower triangle (N rows, K columns)."""
    M = float(np.sum(counts_t)) * n_freq  # visible sources summed over the step's instances
    if path == "sources":
        bs = block_sizes(n_ant)
        diag = sum(8.0 * (2 * n * n + n) for n in bs) * M
        pairs = sum(32.0 * bs[i] * bs[j] for i in range(len(bs)) for j in range(i)) * M
        return diag + pairs, diag, pairs
    N = n_ant * n_feed
    tot = 4.0 * N * (N + 1) * n_ax * M
    return tot, tot, 0.0


def hbm_steps(counts, n_time, n_src, n_comp, n_freq, steps_ms, cbytes=8):
    """Achieved HBM rate of the bandwidth-bound steps on their algorithmic bytes: the sky
    step reads X_eq per time (24 B per source) and writes index, s_hat and (za, az) per
    visible source (4 + 24 + 16 B); the beam step reads (za, az) (16 B) and writes one
    complex value per channel and component per visible source and time."""
    vis = float(np.sum(counts))
    by = {"sky": float(n_time * 24.0 * n_src + vis * 44.0), "beam": vis * (16.0 + cbytes * n_comp * n_freq)}
    return {k: {"bytes_per_step": b, "ms_per_step": steps_ms[k],
                "achieved_GBps": b / (steps_ms[k] / 1e3) / 1e9 if steps_ms[k] > 0 else None, "peak_GBps": HBM_GBS}
            for k, b in by.items()}


def profile_record(name: str):
    """A committed rocprofv3 summary (profiles/<name>.json): its HBM traffic and
    MFMA-busy figures, or None when it is missing or a source it depends on (the
    kernel, and the host code that sizes its launches) changed since it was taken."""
    import hashlib
    f = os.path.join(ROOT, "profiles", name + ".json")
    if not os.path.exists(f):
        return None
    rec = json.load(open(f))
    if "sources" not in rec or "sources_sha256_16" not in rec:
        return None
    h = hashlib.sha256()
    for src in rec["sources"]:
        h.update(open(os.path.join(ROOT, src), "rb").read())
    if h.hexdigest()[:16] != rec["sources_sha256_16"]:
        return None
    return rec


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def time_calls(ctx, d, vis, steps, stream):
    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(steps):
        ctx.simulate(**d, vis=vis)
    e1.record(stream)
    torch.cuda.synchronize()
    ctx.finish()
    return e0.elapsed_time(e1) / max(steps, 1)


def profiled(ctx, d, vis, steps):
    ctx.profile(True)
    for _ in range(steps):
        ctx.simulate(**d, vis=vis)
    prof = ctx.profile_read()
    ctx.profile(False)
    ctx.finish()
    return prof


def sample_pairs(n_ant: int, n: int, seed: int):
    """n seeded antenna pairs plus the autocorrelation of every antenna they use."""
    rng = np.random.Generator(np.random.PCG64(seed))
    a, b = rng.integers(0, n_ant, n), rng.integers(0, n_ant, n)
    pairs = sorted(set(zip(a.tolist(), b.tolist())))
    ants = sorted(set(a.tolist()) | set(b.tolist()))
    return pairs + [(x, x) for x in ants if (x, x) not in pairs]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n-time", type=int, default=2, help="LSTs in the headline's instance sample")
    ap.add_argument("--n-freq", type=int, default=8, help="channels in the headline's instance sample")
    ap.add_argument("--train-epochs", type=int, default=60,
                    help="epochs of the learned beam's training (0: untrained weights, for profiling runs only)")
    ap.add_argument("--profile-steps", type=int, default=2)
    ap.add_argument("--no-autotune", action="store_true", help="use the library's defaults")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--error-pairs", type=int, default=40)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of this many MiB (counter calibration)")
    ap.add_argument("--secondary-steps", type=int, default=10, help="steps of the 128-antenna workload (0 = skip)")
    ap.add_argument("--side-steps", type=int, default=1, help="steps of each side-by-side variant (0 = skip)")
    ap.add_argument("--side-precisions", default="bf16x3,fp32,fp64",
                    help="precisions of the side-by-side runs with the interpolated beam")
    ap.add_argument("--workload-steps", type=int, default=2, help="calls on each other workload (0 = skip)")
    ap.add_argument("--redundancy-steps", type=int, default=2, help="App. A comparison steps (0 = skip)")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        n = args.calibrate_copy << 20
        src = torch.ones(n // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the simulator shards (t, nu) instances "
              f"across GPUs with no communication; this benchmark measures one GPU.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2312_09763_amd import learned_beam
    from paper_2312_09763_amd import matvis as mv
    from paper_2312_09763_amd import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    stream = torch.cuda.current_stream()
    prec = "bf16x3"
    t0 = time.perf_counter()
    wl = synth.workload(5, n_time=args.n_time, n_freq=args.n_freq)
    log(f"workload5 sample: {wl.n_ant} antennas x {wl.n_feed} feeds, {wl.n_src} pixels, LSTs {wl.lsts}, "
        f"channels {np.round(wl.freqs / 1e6, 2)} MHz ({time.perf_counter() - t0:.1f} s to generate)")
    t0 = time.perf_counter()
    if args.train_epochs > 0:
        P, hist, _, _ = learned_beam.train(epochs=args.train_epochs)
    else:  # profiling runs only: the step's time does not depend on the weights
        P, hist = torch.from_numpy(synth.surrogate_init(0, sigma_v=1.0, az_max=4)).cuda(), [float("nan")]
    train_s = time.perf_counter() - t0
    log(f"learned beam: {args.train_epochs} epochs of 2^20 samples, loss {hist[0]:.3e} -> {hist[-1]:.3e} "
        f"({train_s:.1f} s)")
    d = mv.device_inputs(wl, prec)
    base = mv.config_for(wl, prec, beam_mode="surrogate")
    nu_range = (learned_beam.NU0, learned_beam.NU1)
    tune = {"source": "defaults"}
    cfg = base
    if not args.no_autotune:
        os.makedirs(os.path.dirname(TUNING), exist_ok=True)
        cached = os.path.exists(TUNING) and open(TUNING).read()
        t0 = time.perf_counter()
        cfg, tms = mv.autotune(base, **d, cache_path=TUNING, surrogate=P, nu_range=nu_range)
        tune = {"source": "cache" if cached and time.perf_counter() - t0 < 1.0 else "search",
                "search_s": round(time.perf_counter() - t0, 1), "tuned_ms_per_call": tms}
    tune.update({"tile": cfg.tile, "ksplit": cfg.ksplit, "src_chunk": cfg.src_chunk, "batch_time": cfg.batch_time,
                 "unfused": cfg.unfused})
    log(f"configuration: {tune}")

    ctx = mv.Context(cfg)
    ctx.set_surrogate(P, *nu_range)
    vis = torch.empty((wl.n_time, wl.n_freq, wl.n_ant, wl.n_ant, wl.n_feed, wl.n_feed), dtype=torch.complex64,
                      device="cuda")
    for _ in range(args.warmup):
        ctx.simulate(**d, vis=vis)
    ctx.finish()
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    ms_step = time_calls(ctx, d, vis, args.steps, stream)
    wall = (time.perf_counter() - wall0) / args.steps
    units = wl.work_units()
    value = units / (ms_step / 1e3)
    log(f"timed {args.steps} steps: {ms_step:.3f} ms/step (wall {wall * 1e3:.3f} ms/step), {value:.4e} units/s")

    # ---- live per-kernel timing for the roofline (same steps, launched directly)
    prof = profiled(ctx, d, vis, args.profile_steps)
    _, count, _, _ = ctx.step_sky(d["lsts"], d["src_radec"])
    counts = count.cpu().numpy().astype(np.int64)
    path = ctx.product_path
    tot_f, first_f, pair_f = product_flops(path, wl.n_ant, wl.n_feed, wl.n_ax, counts, wl.n_freq)
    k = PRODUCTS[prec]
    steps_ms = {s: round(v[0] / args.profile_steps, 4) for s, v in prof.items()}
    pair_ms, pair_n = prof["herk_pairs"]
    first_ms, first_n = prof["herk"]
    launch_ms = pair_ms / max(pair_n, 1)
    flops_launch = pair_f * k * args.profile_steps / max(pair_n, 1)
    achieved = flops_launch / (launch_ms / 1e3) / 1e12
    prod_ms = (pair_ms + first_ms) / args.profile_steps
    prod_tf = tot_f * k / (prod_ms / 1e3) / 1e12
    log(f"per-step device ms {steps_ms}; block-pair launch {launch_ms:.3f} ms x {pair_n / args.profile_steps:.0f} "
        f"per step at {achieved:.1f} TFLOP/s ({achieved / PEAK_TFLOPS[prec]:.3f} of peak); whole product "
        f"{prod_ms:.2f} ms/step at {prod_tf / PEAK_TFLOPS[prec]:.3f} of peak")
    kname = "k_herk_pairs"
    rec = profile_record("herk_pairs_bf16x3_workload5")
    roofline = {"bound": "mfma", "achieved": achieved, "peak": PEAK_TFLOPS[prec], "unit": "TFLOP/s",
                "frac": achieved / PEAK_TFLOPS[prec],
                "traffic": rec["traffic_bytes_per_launch"] if rec else None,
                "kernel": kname, "launch_ms": launch_ms, "launches_per_step": pair_n / args.profile_steps,
                "flops_per_launch": flops_launch, "useful_tflops": achieved / k,
                "mfma_busy_rocprof": rec.get("mfma_busy") if rec else None,
                "whole_product": {"ms_per_step": prod_ms, "tflops": prod_tf, "frac": prod_tf / PEAK_TFLOPS[prec],
                                  "first_launch_ms_per_step": first_ms / args.profile_steps,
                                  "pair_launch_ms_per_step": pair_ms / args.profile_steps}}

    # ---- error against the FP64 oracle (interpolated beam), two instances, sampled pairs
    import oracle
    from oracle import metrics
    err = None
    vis_h = vis.cpu().numpy()
    insts = [(0, 0), (wl.n_time - 1, wl.n_freq - 1)]
    pairs = sample_pairs(wl.n_ant, args.error_pairs, 7)
    grid = wl.beam.astype(np.complex64).astype(np.complex128)
    c0 = time.perf_counter()
    ref = oracle.simulate_pairs(wl.antpos, wl.freqs, wl.lsts, wl.ra, wl.dec, wl.flux, grid, wl.latitude, wl.dza,
                                wl.daz, wl.interp, instances=insts, pairs=pairs)
    pa, pb = np.array([p[0] for p in pairs]), np.array([p[1] for p in pairs])
    Vp = np.stack([vis_h[t, f][pa, pb] for (t, f) in insts]).astype(np.complex128)
    err = {"err_CS": float(metrics.err_cs_pairs(Vp, ref, pairs).max()),
           "err_F": float(metrics.err_f_pairs(Vp, ref).max()),
           "reference": "FP64 direct sum with the bicubic-interpolated beam (the learned beam's tolerance is 1e-3)",
           "instances": [[int(t), int(f)] for t, f in insts], "pairs": len(pairs),
           "oracle_s": round(time.perf_counter() - c0, 1)}
    log(f"error vs oracle: {err}")

    cpu = None if args.no_cpu_baseline else cpu_baseline(wl, grid)
    side = side_by_side(args, wl, vis, stream, cfg) if args.side_steps > 0 else None
    if side is not None:
        side["bf16x3+learned"] = {"ms_per_step": ms_step, "value": value, "product_path": path,
                                  "product_ms_per_step": prod_ms, "product_frac_of_peak": prod_tf / PEAK_TFLOPS[prec],
                                  "beam_ms_per_step": steps_ms["beam"]}
    ctx.close()
    del vis, d
    sec = secondary(args) if args.secondary_steps > 0 else None
    red = redundancy_section(args) if args.redundancy_steps > 0 else None
    wls = workloads_section(args) if args.workload_steps > 0 else None
    abeams = antenna_beams_section(args) if args.workload_steps > 0 else None

    out = {
        "metric": "src*ant-pair*(t,nu)/s",
        "value": value,
        "unit": "src*ant-pair*(t,nu)/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16x3 (f32 accumulate)",
        "data": "synthetic",
        "config": {"workload": "learned beam on the diffuse sky: 350-antenna hex array (14.6 m), 2 feeds x 2 axes, "
                               "3145728 equal-area pixels (nside 512) with log-normal brightness, learned beam "
                               "(Fourier-feature network of the direction, Chebyshev series in frequency) trained "
                               "on the 0.5 deg bicubic dipole beam, BF16X3 product; full "
                               "configuration 64 LSTs x 64 in-band channels (100-200 MHz of 128 over 50-250 MHz)",
                   "sample": f"{wl.n_time} LSTs x {wl.n_freq} channels = {wl.n_time * wl.n_freq} of the 4096 "
                             f"instances per step (LSTs {[round(x, 4) for x in wl.lsts.tolist()]} rad, channels "
                             f"{[round(x / 1e6, 2) for x in wl.freqs.tolist()]} MHz)",
                   "n_ant": wl.n_ant, "n_feed": wl.n_feed, "n_ax": wl.n_ax, "n_src": wl.n_src,
                   "n_time": wl.n_time, "n_freq": wl.n_freq, "precision": prec, "beam": "learned",
                   "product_path": path, "tuned": tune,
                   "learned_beam": {"epochs": args.train_epochs, "samples": 1 << 20, "final_loss": float(hist[-1]),
                                    "train_s": round(train_s, 1)}},
        "roofline": roofline,
        "step_ms": steps_ms,
        "hbm_steps": hbm_steps(counts, wl.n_time, wl.n_src, wl.n_feed * wl.n_ax, wl.n_freq, steps_ms),
        "error_vs_oracle": err,
        "cpu_baseline": cpu,
        "side_by_side": side,
        "secondary": sec,
        "redundancy": red,
        "workloads": wls,
        "antenna_beams": abeams,
    }
    print(json.dumps(out, default=float), flush=True)


def cpu_baseline(wl, grid):
    """The FP64 oracle on a bounded sample of the headline workload: one instance, a seeded
    set of antenna pairs over every pixel, at the host's thread count and at one thread."""
    import oracle
    threads = oracle.get_threads()
    res = {"unit": "src*ant-pair*(t,nu)/s", "kind": "oracle", "cpu_model": cpu_model(),
           "host_threads_available": os.cpu_count()}
    for n_thr, n_pairs in ((threads, 32 * threads), (1, 32)):
        oracle.set_threads(n_thr)
        pairs = sample_pairs(wl.n_ant, n_pairs, 11)[:n_pairs]
        c0 = time.perf_counter()
        oracle.simulate_pairs(wl.antpos, wl.freqs, wl.lsts, wl.ra, wl.dec, wl.flux, grid, wl.latitude, wl.dza,
                              wl.daz, wl.interp, instances=[(0, 0)], pairs=pairs)
        dt = time.perf_counter() - c0
        v = wl.n_src * len(pairs) / dt
        sample = (f"one instance (t=0, nu={wl.freqs[0] / 1e6:.2f} MHz) of the headline workload, {len(pairs)} seeded "
                  f"antenna pairs x all {wl.n_src} pixels, FP64 direct sum, {dt:.1f} s on {n_thr} thread(s)")
        if n_thr == threads:
            res.update({"value": v, "cores": n_thr, "sample": sample})
        else:
            res["single_thread"] = {"value": v, "cores": 1, "sample": sample}
        log(f"cpu baseline: {v:.3e} units/s on {n_thr} thread(s) ({dt:.1f} s)")
    oracle.set_threads(threads)
    return res


def side_by_side(args, wl, vis, stream, tuned):
    """The headline's sample through the FP64 interpolated path, FP32 and BF16X3 with the
    bicubic-interpolated beam (Z in device memory on FP64; formed in the product otherwise).
    BF16X3 takes the headline's tuned product configuration, FP32 and FP64 the defaults."""
    import torch
    from paper_2312_09763_amd import matvis as mv
    out = {}
    for vprec in [p for p in ("bf16x3", "fp32", "fp64") if p in args.side_precisions.split(",")]:
        vd = mv.device_inputs(wl, vprec)
        kw = dict(ksplit=tuned.ksplit, batch_time=tuned.batch_time, tile=tuned.tile) if vprec == "bf16x3" else {}
        with mv.Context(mv.config_for(wl, vprec, **kw)) as vctx:
            vvis = torch.empty(tuple(vis.shape), dtype=vctx.complex_dtype, device="cuda")
            vctx.simulate(**vd, vis=vvis)
            vctx.finish()
            vms = time_calls(vctx, vd, vvis, args.side_steps, stream)
            vprof = profiled(vctx, vd, vvis, 1)
            _, count, _, _ = vctx.step_sky(vd["lsts"], vd["src_radec"])
            counts = count.cpu().numpy().astype(np.int64)
            vpath = vctx.product_path
            tot, _, _ = product_flops(vpath, wl.n_ant, wl.n_feed, wl.n_ax, counts, wl.n_freq)
            pms = vprof["herk"][0] + vprof["herk_pairs"][0]
            vtf = tot * PRODUCTS[vprec] / (pms / 1e3) / 1e12 if pms > 0 else None
            vsteps = {k: round(v[0], 4) for k, v in vprof.items()}
            out[f"{vprec}+interpolated"] = {"ms_per_step": vms, "value": wl.work_units() / (vms / 1e3),
                                            "product_path": vpath, "product_ms_per_step": pms,
                                            "product_frac_of_peak": vtf / PEAK_TFLOPS[vprec] if vtf else None,
                                            "beam_ms_per_step": vprof["beam"][0],
                                            "hbm_steps": hbm_steps(counts, wl.n_time, wl.n_src, wl.n_feed * wl.n_ax,
                                                                   wl.n_freq, vsteps,
                                                                   16 if vprec == "fp64" else 8)}
            log(f"side by side {vprec} + interpolated beam: {vms:.2f} ms/step, product {pms:.2f} ms")
            del vvis
        del vd
        torch.cuda.empty_cache()
    return out


def secondary(args):
    """The 128-antenna polarised workload (50 000 sources, 32 LSTs x 16 channels, bicubic
    dipole beam; BF16X3): throughput, its product roofline (one 128-antenna block: the
    diagonal-block kernel) and the achieved HBM rate of the bandwidth-bound steps."""
    import torch
    from paper_2312_09763_amd import matvis as mv
    from paper_2312_09763_amd import synth
    prec = "bf16x3"
    wl = synth.workload(2)
    d = mv.device_inputs(wl, prec)
    stream = torch.cuda.current_stream()
    with mv.Context(mv.config_for(wl, prec)) as ctx:
        vis = ctx.simulate(**d)
        ctx.finish()
        ms = time_calls(ctx, d, vis, args.secondary_steps, stream)
        prof = profiled(ctx, d, vis, 2)
        _, count, _, _ = ctx.step_sky(d["lsts"], d["src_radec"])
        counts = count.cpu().numpy().astype(np.int64)
        path = ctx.product_path
    tot, _, _ = product_flops(path, wl.n_ant, wl.n_feed, wl.n_ax, counts, wl.n_freq)
    hm, hn = prof["herk"]
    launch_ms = hm / max(hn, 1)
    achieved = tot * PRODUCTS[prec] * 2 / max(hn, 1) / (launch_ms / 1e3) / 1e12
    steps_ms = {s: round(v[0] / 2, 4) for s, v in prof.items()}
    n_comp = wl.n_feed * wl.n_ax * wl.beam.shape[0]
    rec = profile_record("herk_coh_bf16x3_workload2")
    res = {"workload": "128-antenna polarised hex array, 50000 point sources, 32 LSTs x 16 channels 100-200 MHz, "
                       "dipole Jones beam 0.5 deg grid bicubic, BF16X3",
           "ms_per_step": ms, "value": wl.work_units() / (ms / 1e3), "product_path": path,
           "roofline": {"bound": "mfma", "kernel": "k_herk_coh<2, false, 96, false>", "achieved": achieved,
                        "peak": PEAK_TFLOPS[prec], "unit": "TFLOP/s", "frac": achieved / PEAK_TFLOPS[prec],
                        "launch_ms": launch_ms, "traffic": rec["traffic_bytes_per_launch"] if rec else None},
           "step_ms": steps_ms,
           "hbm_steps": hbm_steps(counts, wl.n_time, wl.n_src, n_comp, wl.n_freq, steps_ms)}
    log(f"secondary (128 antennas, 50k sources): {ms:.3f} ms/step, product launch {launch_ms:.3f} ms "
        f"({achieved / PEAK_TFLOPS[prec]:.3f} of peak), steps {steps_ms}")
    return res


def antenna_beams_section(args):
    """A beam per antenna (N_beam = N_ant, Sec. 3.5 / Sec. 6.1): 128 polarised antennas, each
    with its own dipole Jones beam on the 0.5 deg grid (bicubic), the 50 000-source sky, 4
    LSTs x 2 channels, BF16X3, against the same run with one shared beam.  The shared-beam
    run takes the product over sources; with a beam per antenna the axis sum cannot be
    taken per source first, so the product runs over the (source, axis) columns of Z."""
    import torch
    from paper_2312_09763_amd import matvis as mv
    from paper_2312_09763_amd import synth
    prec = "bf16x3"
    wl = synth.workload(2, n_time=4, n_freq=2)
    shared = wl.beam.astype(np.complex64)
    per_ant = synth.antenna_beams(wl.freqs, 0.5, wl.n_ant, seed=3)
    stream = torch.cuda.current_stream()
    res = {"workload": f"{wl.n_ant} polarised antennas, {wl.n_src} point sources, {wl.n_time} LSTs x {wl.n_freq} "
                       f"channels, 0.5 deg bicubic dipole beams, BF16X3"}
    for name, grid, bidx in (("shared_beam", shared, None),
                             ("beam_per_antenna", per_ant, np.arange(wl.n_ant, dtype=np.int32))):
        wl.beam = grid
        d = mv.device_inputs(wl, prec)
        bi = None if bidx is None else torch.from_numpy(bidx).cuda()
        with mv.Context(mv.config_for(wl, prec)) as ctx:
            vis = ctx.simulate(**d, beam_idx=bi)
            ctx.finish()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(args.workload_steps):
                ctx.simulate(**d, vis=vis, beam_idx=bi)
            e1.record(stream)
            torch.cuda.synchronize()
            ctx.finish()
            ms = e0.elapsed_time(e1) / args.workload_steps
            ctx.profile(True)
            ctx.simulate(**d, vis=vis, beam_idx=bi)
            prof = ctx.profile_read()
            ctx.profile(False)
            ctx.finish()
            res[name] = {"n_beam": int(grid.shape[0]), "ms_per_step": ms, "value": wl.work_units() / (ms / 1e3),
                         "product_path": ctx.product_path, "beam_ms": prof["beam"][0],
                         "product_ms": prof["herk"][0] + prof["herk_pairs"][0],
                         "step_ms": {k: round(v[0], 4) for k, v in prof.items()}}
            log(f"{name}: {ms:.2f} ms per step, beam {prof['beam'][0]:.3f} ms, product "
                f"{res[name]['product_ms']:.2f} ms, path {ctx.product_path}")
            del vis
        del d
    return res


def workloads_section(args):
    """Throughput of the other synthetic workloads on this GPU, in the metric's units:
    the 37-antenna scalar case (FP64, its stated precision), the batched uneven case at
    full size (FP32 and BF16X3) and the scalar diffuse sky at its full pixel count (one
    LST x 8 of its channels, a sample of its 64 x 128 instances, BF16X3)."""
    import torch
    from paper_2312_09763_amd import matvis as mv
    from paper_2312_09763_amd import synth
    cases = [(1, dict(), "fp64"), (4, dict(), "fp32"), (4, dict(), "bf16x3"), (3, dict(n_time=1, n_freq=8), "bf16x3")]
    out = {}
    made = {}
    stream = torch.cuda.current_stream()
    for cfg_id, kw, prec in cases:
        key = (cfg_id, tuple(sorted(kw.items())))
        if key not in made:
            made.clear()
            made[key] = synth.workload(cfg_id, **kw)
        wl = made[key]
        d = mv.device_inputs(wl, prec)
        with mv.Context(mv.config_for(wl, prec)) as ctx:
            vis = ctx.simulate(**d)
            ctx.finish()
            ms = time_calls(ctx, d, vis, args.workload_steps, stream)
            prof = profiled(ctx, d, vis, 1)
            _, count, _, _ = ctx.step_sky(d["lsts"], d["src_radec"])
            counts = count.cpu().numpy().astype(np.int64)
            path = ctx.product_path
        tot, _, _ = product_flops(path, wl.n_ant, wl.n_feed, wl.n_ax, counts, wl.n_freq)
        pms = prof["herk"][0] + prof["herk_pairs"][0]
        tf = tot * PRODUCTS[prec] / (pms / 1e3) / 1e12 if pms > 0 else None
        name = f"workload{cfg_id}_{prec}"
        out[name] = {"n_ant": wl.n_ant, "n_feed": wl.n_feed, "n_ax": wl.n_ax, "n_src": wl.n_src,
                     "instances": [wl.n_time, wl.n_freq], "ms_per_call": ms, "value": wl.work_units() / (ms / 1e3),
                     "product_path": path, "product_ms": pms, "product_tflops": tf,
                     "product_frac_of_peak": tf / PEAK_TFLOPS[prec] if tf else None,
                     "step_ms": {s: round(v[0], 4) for s, v in prof.items()}}
        log(f"{name}: {ms:.2f} ms per call, {wl.work_units() / (ms / 1e3):.3e} units/s, path {path}, "
            f"product {pms:.2f} ms" + (f" ({tf / PEAK_TFLOPS[prec]:.3f} of peak)" if tf else ""))
        del vis, d
    return out


def redundancy_section(args):
    """Full product V = Z Z^H against the sub-matrix product of App. A for the unique
    baselines of a redundant 350-antenna hexagon (the diffuse-sky array), BF16X3,
    FP32 and FP64 with Z in device memory, and BF16X3 and FP32 with Z formed in the
    product's stages; per-step device times from the profiled pass."""
    import torch
    from paper_2312_09763_amd import matvis as mv
    from paper_2312_09763_amd import synth
    wl = synth.workload(3, n_src=49152, n_time=4, n_freq=8)
    _, reps = mv.redundant_groups(wl.antpos, None, 1e-6)
    res = {"workload": f"{wl.n_ant}-antenna hexagon, {wl.n_src} equal-area pixels, {wl.n_time} LSTs x "
                       f"{wl.n_freq} channels, scalar Gaussian beam",
           "n_ant": wl.n_ant, "pairs": wl.n_ant * (wl.n_ant + 1) // 2, "unique_pairs": len(reps)}
    for key in ("bf16x3", "fp32", "fp64", "bf16x3_fused", "fp32_fused"):
        prec = key.replace("_fused", "")
        cfg = mv.config_for(wl, prec, unfused=(prec != "fp64" and not key.endswith("_fused")))
        d = mv.device_inputs(wl, prec)
        with mv.Context(cfg) as ctx:
            size = ctx.set_pairs(reps, 3)
            r = {"submatrix_size": size, "full_size": wl.n_ant ** 2, "compression": wl.n_ant ** 2 / size}
            for mode in ("full", "pairs"):
                run = ctx.simulate if mode == "full" else ctx.simulate_pairs
                run(**d)
                ctx.finish()
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(args.redundancy_steps):
                    run(**d)
                e1.record()
                torch.cuda.synchronize()
                ctx.finish()
                ctx.profile(True)
                run(**d)
                prof = ctx.profile_read()
                ctx.profile(False)
                ctx.finish()
                r[f"{mode}_ms_per_step"] = e0.elapsed_time(e1) / args.redundancy_steps
                r[f"{mode}_product_ms"] = prof["herk"][0] + prof["herk_pairs"][0]
                r[f"{mode}_reduce_ms"] = prof["reduce"][0]
            r["product_speedup"] = r["full_product_ms"] / r["pairs_product_ms"]
            r["step_speedup"] = r["full_ms_per_step"] / r["pairs_ms_per_step"]
            log(f"redundancy {key}: {len(reps)} unique pairs, compression {r['compression']:.1f}, product "
                f"{r['full_product_ms']:.2f} -> {r['pairs_product_ms']:.2f} ms, step {r['full_ms_per_step']:.2f} -> "
                f"{r['pairs_ms_per_step']:.2f} ms")
            res[key] = r
    return res


if __name__ == "__main__":
    main()
