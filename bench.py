"""Benchmark of the visibility simulator hot path on one MI355X.

Workload (the metric's configuration): 128-antenna hexagonal array with 2
feeds x 2 E-field axes, 50 000 point sources with power-law fluxes and
spectral indices, 32 LSTs over 24 h x 16 channels 100-200 MHz, a dipole-like
Jones beam on a 0.5 deg az/za grid with bicubic interpolation.  All inputs are
seeded synthetic arrays already resident in HBM when timing starts.

One step = one matvis_simulate call over every (t, nu) instance: rotation,
horizon compaction, beam interpolation, Z formation and V = Z Z^H, i.e. every
step of Alg. 2 for the whole batch, replayed from its captured hipGraph.

metric: src * ant-pair * (t, nu) / s = n_src * n_ant (n_ant + 1) / 2 * n_t * n_nu / T.

Also reported on the same JSON line:
* roofline: the product kernel, timed live with HIP events around each of its
  launches (a separate profiled pass over the same steps), against the MFMA
  peak of the arithmetic's dtype.  Algorithmic flops per instance, x 3
  products on BF16X3: 4 N (N + 1) K for Z Z^H over the lower triangle (N rows,
  K = n_ax x visible columns), and half that, 2 N (N + 1) K, on the path that
  sums the two axes per source first (three 128-antenna feed blocks over the
  visible sources);
* cpu_baseline: the FP64 direct-sum oracle on one full (t, nu) instance on the
  host cores, and the error of the GPU result on that instance;
* side_by_side: the same workload through the FP64 interpolated path, the FP32
  path, and BF16X3 with the learned beam in place of interpolation (its
  weights are a random initialisation: the time does not depend on them; the
  trained network's accuracy is measured by the tests);
* redundancy: the full product against the sub-matrix product of App. A;
* workloads: the same units on the other synthetic workloads (the 37-antenna
  scalar case, the batched uneven case, the diffuse-sky array at its full
  pixel count on a sample of its instances, scalar and polarised, with the
  interpolated and the learned beam).
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


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def measured_traffic(path: str):
    """HBM bytes per launch of the product kernel from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, scaled by a 1 GiB copy), or None when no
    summary exists for this path or a source it depends on (the kernel, and the host
    code that sizes its launches) changed since it was taken."""
    import hashlib
    f = os.path.join(ROOT, "profiles", {"sources": "herk_coh_bf16x3_workload2.json"}.get(path, "none.json"))
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
    return rec["traffic_bytes_per_launch"]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default="bf16x3", choices=["fp64", "fp32", "bf16x3"])
    ap.add_argument("--profile-steps", type=int, default=2)
    ap.add_argument("--unfused", action="store_true", help="write Z to HBM in its own step (FP32 / BF16X3)")
    ap.add_argument("--batch-time", type=int, default=0, help="times per device batch (0 = the library's choice)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--n-src", type=int, default=None, help="shrink the workload (smoke runs only)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of this many MiB (counter calibration)")
    ap.add_argument("--redundancy-steps", type=int, default=2,
                    help="time the full product against the sub-matrix product (App. A) on a 350-antenna "
                         "hexagon (0 = skip)")
    ap.add_argument("--workload-steps", type=int, default=2,
                    help="calls timed on each of the other workloads (0 = skip them)")
    ap.add_argument("--side-steps", type=int, default=2,
                    help="steps timed for each side-by-side variant (0 = skip them)")
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
    from paper_2312_09763_amd import matvis as mv
    from paper_2312_09763_amd import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    prec = args.precision
    wl = synth.workload(2, n_src=args.n_src)
    log(f"workload2: n_ant={wl.n_ant} n_src={wl.n_src} n_time={wl.n_time} n_freq={wl.n_freq} precision={prec}")
    cfg = mv.config_for(wl, prec, unfused=args.unfused, batch_time=args.batch_time)
    ctx = mv.Context(cfg)
    d = mv.device_inputs(wl, prec)
    vis = torch.empty((wl.n_time, wl.n_freq, wl.n_ant, wl.n_ant, wl.n_feed, wl.n_feed), dtype=ctx.complex_dtype,
                      device="cuda")
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        ctx.simulate(**d, vis=vis)
    ctx.finish()
    torch.cuda.synchronize()
    log("warmup done")

    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        ctx.simulate(**d, vis=vis)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ctx.finish()
    ms_step = e0.elapsed_time(e1) / args.steps
    units = wl.work_units()
    value = units / (ms_step / 1e3)
    log(f"timed {args.steps} steps: {ms_step:.3f} ms/step (wall {wall / args.steps * 1e3:.3f} ms/step)")

    # ---- live per-kernel timing for the roofline (same steps, launched directly)
    ctx.profile(True)
    for _ in range(args.profile_steps):
        ctx.simulate(**d, vis=vis)
    prof = ctx.profile_read()
    ctx.profile(False)
    ctx.finish()
    _, count, _, _ = ctx.step_sky(d["lsts"], d["src_radec"])
    counts = count.cpu().numpy().astype(np.int64)
    N = wl.n_ant * wl.n_feed
    K = wl.n_ax * counts  # per time
    path = ctx.product_path
    traffic = measured_traffic(path)
    per_col = 2.0 if path == "sources" else 4.0
    useful_flops_step = float(np.sum(per_col * N * (N + 1) * K) * wl.n_freq)
    herk_ms, herk_n = prof["herk"]
    herk_ms_launch = herk_ms / max(herk_n, 1)
    flops_launch = useful_flops_step * PRODUCTS[prec] * args.profile_steps / max(herk_n, 1)
    achieved = flops_launch / (herk_ms_launch / 1e3) / 1e12
    zform_ms, zform_n = prof["zform"]
    z_bytes_step = float(np.sum(N * (np.ceil(wl.n_ax * counts / 64.0) * 64) * 8.0) * wl.n_freq)
    steps_ms = {k: round(v[0] / args.profile_steps, 4) for k, v in prof.items()}
    log("per-step device ms:", steps_ms)
    # Algorithmic HBM bytes of the bandwidth-bound steps, per step.  Sky (rotation and
    # ordered compaction): per time, X_eq read once (24 B per source) and, per visible
    # source, index + s_hat + (za, az) written (4 + 24 + 16 B).  Beam: per visible
    # source and time, (za, az) read (16 B) and one complex64 per channel and beam
    # component written (the grid taps are L2 gathers, not counted).
    n_comp = wl.n_feed * wl.n_ax * wl.beam.shape[0]
    sky_bytes = float(wl.n_time * 24.0 * wl.n_src + np.sum(counts) * 44.0)
    beam_bytes = float(np.sum(counts) * (16.0 + 8.0 * n_comp * wl.n_freq))
    hbm_steps = {k: {"bytes_per_step": by, "ms_per_step": steps_ms[k],
                     "achieved_GBps": by / (steps_ms[k] / 1e3) / 1e9 if steps_ms[k] > 0 else None,
                     "peak_GBps": HBM_GBS}
                 for k, by in (("sky", sky_bytes), ("beam", beam_bytes))}

    # ---- side by side on the same workload: the FP64 interpolated path, FP32, and
    # BF16X3 with the learned beam (random-init weights: its time does not depend on them)
    side = {}
    if args.side_steps > 0:
        variants = [("fp64", "interpolated", {}), ("fp32", "interpolated", {}),
                    ("bf16x3", "learned", {"beam_mode": "surrogate"})]
        for vprec, beam, kw in variants:
            vcfg = mv.config_for(wl, vprec, **kw)
            vd = mv.device_inputs(wl, vprec)
            with mv.Context(vcfg) as vctx:
                if beam == "learned":
                    params = torch.from_numpy(synth.surrogate_init(0)).cuda()
                    vctx.set_surrogate(params, float(wl.freqs.min()), float(wl.freqs.max()))
                vvis = torch.empty_like(vis, dtype=vctx.complex_dtype)
                vctx.simulate(**vd, vis=vvis)
                vctx.finish()
                torch.cuda.synchronize()
                v0, v1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                v0.record(stream)
                for _ in range(args.side_steps):
                    vctx.simulate(**vd, vis=vvis)
                v1.record(stream)
                torch.cuda.synchronize()
                vctx.finish()
                vms = v0.elapsed_time(v1) / args.side_steps
                # the product kernel's own rate on this path, from one profiled step
                vctx.profile(True)
                vctx.simulate(**vd, vis=vvis)
                vprof = vctx.profile_read()
                vctx.profile(False)
                vctx.finish()
                vpath = vctx.product_path
                vflops = float(np.sum((2.0 if vpath == "sources" else 4.0) * N * (N + 1) * K) * wl.n_freq) * \
                    PRODUCTS[vprec]
                vtf = vflops / (vprof["herk"][0] / 1e3) / 1e12 if vprof["herk"][0] > 0 else None
                side[f"{vprec}+{beam}"] = {"ms_per_step": vms, "value": units / (vms / 1e3), "product_path": vpath,
                                           "product_ms_per_step": vprof["herk"][0],
                                           "product_tflops": vtf,
                                           "product_frac_of_peak": vtf / PEAK_TFLOPS[vprec] if vtf else None}
                log(f"side by side {vprec} + {beam} beam: {vms:.2f} ms/step")
                del vvis
        # the polarised sky (I, Q, U, V per source and channel) on the same path
        st = synth.polarised_stokes(wl.flux, wl.freqs, seed=1)
        pcfg = mv.config_for(wl, prec, polarised_sky=True)
        pd = mv.device_inputs(wl, prec, stokes=st)
        with mv.Context(pcfg) as pctx:
            pvis = torch.empty_like(vis)
            pctx.simulate(**pd, vis=pvis)
            pctx.finish()
            torch.cuda.synchronize()
            v0, v1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            v0.record(stream)
            for _ in range(args.side_steps):
                pctx.simulate(**pd, vis=pvis)
            v1.record(stream)
            torch.cuda.synchronize()
            pctx.finish()
            pms = v0.elapsed_time(v1) / args.side_steps
            side[f"{prec}+interpolated+polarised_sky"] = {"ms_per_step": pms, "value": units / (pms / 1e3),
                                                          "product_path": pctx.product_path}
            log(f"side by side {prec} + polarised sky: {pms:.2f} ms/step")
            del pvis
        side[f"{prec}+interpolated"] = {"ms_per_step": ms_step, "value": value, "product_path": ctx.product_path,
                                        "product_ms_per_step": herk_ms / args.profile_steps,
                                        "product_tflops": achieved, "product_frac_of_peak": achieved / PEAK_TFLOPS[prec]}

    red = redundancy_section(args) if args.redundancy_steps > 0 else None
    wls = workloads_section(args) if args.workload_steps > 0 else None

    # ---- CPU baseline: the FP64 oracle on one full instance, and the GPU error there
    cpu = None
    err = None
    if not args.no_cpu_baseline:
        import oracle
        from oracle import metrics
        t, f = 0, 0
        grid = wl.beam if prec == "fp64" else wl.beam.astype(np.complex64).astype(np.complex128)
        c0 = time.perf_counter()
        Vref = oracle.simulate(wl.antpos, wl.freqs, wl.lsts, wl.ra, wl.dec, wl.flux, grid, wl.latitude, wl.dza,
                               wl.daz, wl.interp, instances=[(t, f)])
        cdt = time.perf_counter() - c0
        sample_units = wl.n_src * wl.n_ant * (wl.n_ant + 1) / 2.0
        cpu = {"value": sample_units / cdt, "unit": "src*ant-pair*(t,nu)/s", "cores": oracle.get_threads(),
               "kind": "oracle",
               "sample": f"one full (t, nu) instance (t=0, nu={wl.freqs[f] / 1e6:.1f} MHz) of the same workload, "
                         f"all {wl.n_ant}x{wl.n_ant} antenna pairs, FP64 direct sum, {cdt:.1f} s"}
        Vg = vis[t, f].cpu().numpy().astype(np.complex128)[None]
        err = {"err_F": float(metrics.err_f(Vg, Vref).max()), "err_CS": float(metrics.err_cs(Vg, Vref).max()),
               "instance": [t, f]}
        log(f"oracle: {cdt:.1f} s on {oracle.get_threads()} threads; GPU error on that instance {err}")

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
        "dtype": {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16x3 (f32 accumulate)"}[prec],
        "data": "synthetic",
        "config": {"workload": "128-antenna polarised hex array, 50000 point sources, 32 LSTs x 16 channels "
                               "100-200 MHz, dipole Jones beam 0.5 deg grid bicubic",
                   "n_ant": wl.n_ant, "n_feed": wl.n_feed, "n_ax": wl.n_ax, "n_src": wl.n_src,
                   "n_time": wl.n_time, "n_freq": wl.n_freq, "precision": prec,
                   "product_path": path},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_TFLOPS[prec], "unit": "TFLOP/s",
                     "frac": achieved / PEAK_TFLOPS[prec], "traffic": traffic,
                     "kernel": {"z_in_hbm": "k_herk", "fused": "k_herk_fused", "fused_rows": "k_herk_b3_pair",
                                "fused_blocks": "k_herk_blk3",
                                "sources": "k_herk_coh<2, false>" if prec == "bf16x3" else "k_herk_coh<1, false>"}[path],
                     "launch_ms": herk_ms_launch, "flops_per_launch": flops_launch,
                     "useful_tflops": achieved / PRODUCTS[prec]},
        "zform": {"achieved_GBps": z_bytes_step * args.profile_steps / (zform_ms / 1e3) / 1e9 if zform_ms else None,
                  "peak_GBps": HBM_GBS},
        "step_ms": steps_ms,
        "hbm_steps": hbm_steps,
        "side_by_side": side,
        "redundancy": red,
        "workloads": wls,
        "cpu_baseline": cpu,
        "error_vs_oracle": err,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


def workloads_section(args):
    """Throughput of the other synthetic workloads on this GPU, in the metric's units:
    the 37-antenna scalar case (FP64, its stated precision), the batched uneven
    case at full size (FP32 and BF16X3), and the diffuse-sky array at its full
    pixel count (3 145 728 pixels, 350 antennas; one LST x 8 of its channels, a
    sample of the 64 x 128 instances), scalar with the BF16X3 product and
    polarised with the interpolated and the learned beam (random-init weights:
    the time does not depend on them)."""
    import torch
    from paper_2312_09763_amd import matvis as mv
    from paper_2312_09763_amd import synth
    cases = [(1, dict(), "fp64", "interpolated"), (4, dict(), "fp32", "interpolated"),
             (4, dict(), "bf16x3", "interpolated"), (3, dict(n_time=1, n_freq=8), "bf16x3", "interpolated"),
             (5, dict(n_time=1, n_freq=8), "bf16x3", "interpolated"), (5, dict(n_time=1, n_freq=8), "bf16x3", "learned")]
    out = {}
    made = {}
    stream = torch.cuda.current_stream()
    for cfg_id, kw, prec, beam in cases:
        key = (cfg_id, tuple(sorted(kw.items())))
        if key not in made:
            made.clear()  # keep one workload's arrays at a time
            made[key] = synth.workload(cfg_id, **kw)
        wl = made[key]
        extra = {"beam_mode": "surrogate"} if beam == "learned" else {}
        cfg = mv.config_for(wl, prec, **extra)
        d = mv.device_inputs(wl, prec)
        with mv.Context(cfg) as ctx:
            if beam == "learned":
                ctx.set_surrogate(torch.from_numpy(synth.surrogate_init(0)).cuda(), 100e6, 200e6)
            vis = ctx.simulate(**d)
            ctx.finish()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(args.workload_steps):
                ctx.simulate(**d, vis=vis)
            e1.record(stream)
            torch.cuda.synchronize()
            ctx.finish()
            ms = e0.elapsed_time(e1) / args.workload_steps
            ctx.profile(True)
            ctx.simulate(**d, vis=vis)
            prof = ctx.profile_read()
            ctx.profile(False)
            ctx.finish()
            _, count, _, _ = ctx.step_sky(d["lsts"], d["src_radec"])
            counts = count.cpu().numpy().astype(np.int64)
            path = ctx.product_path
        N = wl.n_ant * wl.n_feed
        K = wl.n_ax * counts
        flops = float(np.sum((2.0 if path == "sources" else 4.0) * N * (N + 1) * K) * wl.n_freq) * PRODUCTS[prec]
        herk_ms = prof["herk"][0]
        tf = flops / (herk_ms / 1e3) / 1e12 if herk_ms > 0 else None
        name = f"workload{cfg_id}_{prec}_{beam}"
        out[name] = {"n_ant": wl.n_ant, "n_feed": wl.n_feed, "n_ax": wl.n_ax, "n_src": wl.n_src,
                     "instances": [wl.n_time, wl.n_freq], "ms_per_call": ms,
                     "value": wl.work_units() / (ms / 1e3), "product_path": path, "product_ms": herk_ms,
                     "product_tflops": tf, "product_frac_of_peak": tf / PEAK_TFLOPS[prec] if tf else None,
                     "step_ms": {k: round(v[0], 4) for k, v in prof.items()}}
        log(f"{name}: {ms:.2f} ms per call, {wl.work_units() / (ms / 1e3):.3e} units/s, path {path}, "
            f"product {herk_ms:.2f} ms" + (f" ({tf / PEAK_TFLOPS[prec]:.3f} of peak)" if tf else ""))
        del vis, d
    return out


def redundancy_section(args):
    """Full product V = Z Z^H against the sub-matrix product of App. A for the unique
    baselines of a redundant 350-antenna hexagon (the diffuse-sky array), BF16X3,
    FP32 and FP64 with Z in device memory; per-step device times from the profiled pass."""
    import torch
    from paper_2312_09763_amd import matvis as mv
    from paper_2312_09763_amd import synth
    wl = synth.workload(3, n_src=49152, n_time=4, n_freq=8)
    _, reps = mv.redundant_groups(wl.antpos, None, 1e-6)
    res = {"workload": f"{wl.n_ant}-antenna hexagon, {wl.n_src} equal-area pixels, {wl.n_time} LSTs x "
                       f"{wl.n_freq} channels, scalar Gaussian beam",
           "n_ant": wl.n_ant, "pairs": wl.n_ant * (wl.n_ant + 1) // 2, "unique_pairs": len(reps)}
    for prec in ("bf16x3", "fp32", "fp64"):
        cfg = mv.config_for(wl, prec, unfused=(prec != "fp64"))
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
                r[f"{mode}_product_ms"] = prof["herk"][0]
                r[f"{mode}_reduce_ms"] = prof["reduce"][0]
            r["product_speedup"] = r["full_product_ms"] / r["pairs_product_ms"]
            r["step_speedup"] = r["full_ms_per_step"] / r["pairs_ms_per_step"]
            log(f"redundancy {prec}: {len(reps)} unique pairs, compression {r['compression']:.1f}, product "
                f"{r['full_product_ms']:.2f} -> {r['pairs_product_ms']:.2f} ms, step {r['full_ms_per_step']:.2f} -> "
                f"{r['pairs_ms_per_step']:.2f} ms")
            res[prec] = r
    return res


if __name__ == "__main__":
    main()
