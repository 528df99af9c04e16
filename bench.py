"""Benchmark of the EMDQ hot path on one MI355X.

One step = the whole path over one batch of synthetic input, inputs resident
in HBM: emdq_fit (per-match similarity fits as dual quaternions + EM inlier
reweighting over the N x N Gaussian weights) followed by emdq_warp (dense
per-pixel DQ blend on MFMA, Eq. (1), bilinear sample and colour merge into
the mosaic canvas).

Workloads (--workload):
  production  (default) 1280 x 1024 RGB uint8 frame, N = 2000 matches (30 %
              outliers, 8 Gaussian bumps), 4096 x 4096 RGBA FP32 canvas, FP32
  fhd-f32 / fhd-f16 / fhd-bf16
              1920 x 1080 frame, N = 4000 (30 % outliers), 1920 x 1080 canvas,
              with the blend's GEMM operands in the named precision
  batch64     64 independent pairs of mixed size (640x480 / 1280x1024 /
              1920x1080, N in [300, 3000], 10-40 % outliers), one canvas each,
              fitted and warped with the batched entry points
  batch64-learned
              the same, with the EM of every pair started from the learned
              prior (batched learned start + batched fit from it); both batch
              workloads also report plain single-pair calls on the same pairs

Prints one JSON line.  value = frame pixels x steps / wall time of the timed
steps (Mpix/s).  The roofline object covers the field + warp kernel, timed
with HIP events on the stream it runs on; cpu_baseline times the FP64 oracle
on the host cores on whole steps of the same workload (a bounded sample).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mpix/s dense EMDQ field+warp (N=2000); EM iters & px error learned vs plain"
PEAK_TFLOPS = {"f32": 157.3, "f16": 2500.0, "bf16": 2500.0}
# HBM traffic of the production field + warp kernel per launch, from rocprofv3
# FETCH_SIZE + WRITE_SIZE (KiB per dispatch) scaled by the copy-kernel
# calibration (factors 2.0 and 1.0): 15149.4 KiB x 2.0 + 18814.1 KiB x 1.0.
# Set to None whenever the kernel changes, until the counters are taken again.
TRAFFIC_BYTES = round((15149.4 * 2.0 + 18814.1 * 1.0) * 1024)
WORKLOADS = ("production", "fhd-f32", "fhd-f16", "fhd-bf16", "batch64", "batch64-learned")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--pair", type=int, default=1)
    ap.add_argument("--workload", choices=WORKLOADS, default="production")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="minimum host time of the oracle CPU baseline")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (3 times), for scaling "
                         "the FETCH_SIZE / WRITE_SIZE counters")
    return ap.parse_args()


def copy_calibration(mib):
    """A plain copy kernel of known size: reads and writes mib MiB."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": n * 4}), flush=True)


def cpu_baseline(pairs, min_seconds):
    """The FP64 oracle on the host: whole steps of the workload's pairs (EM fit
    + field, warp and merge of every frame pixel), cycling over the pairs
    until at least `min_seconds` have passed."""
    import oracle as O
    reps, px, t_fit, t_warp = 0, 0, 0.0, 0.0
    t_start = time.perf_counter()
    fits = []
    while True:
        P = pairs[reps % len(pairs)]
        W, H = P.cfg.width, P.cfg.height
        canvas = np.zeros((H, W, 4))
        t0 = time.perf_counter()
        f = O.fit(P.src, P.dst, W, H)
        t1 = time.perf_counter()
        O.warp(P.src, f.scale, f.q, f.mask, f.alpha, P.frame, canvas, 0, 0, 0, 0, W, H)
        t2 = time.perf_counter()
        if reps < len(pairs):
            fits.append(f)
        reps += 1
        px += W * H
        t_fit += t1 - t0
        t_warp += t2 - t1
        if t2 - t_start >= min_seconds:
            break
    total = t_fit + t_warp
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    first = pairs[0].cfg
    return fits, dict(value=round(px / total / 1e6, 4), unit="Mpix/s", cores=threads,
                      kind="oracle",
                      sample=f"{reps} whole pair steps ({min(reps, len(pairs))}"
                             f" distinct pairs, first {first.width}x{first.height} "
                             f"N={first.n_matches}): EM fit {t_fit / reps * 1e3:.0f} ms + "
                             f"field/warp/merge of every pixel {t_warp / reps * 1e3:.0f} ms "
                             f"per pair; FP64, OpenMP, {total:.1f} s in total")


def learned_vs_plain(E, torch, P, model, src, dst, stream, reps=5):
    """EM iterations, fit time and field error against the generator's
    ground truth, plain start (p = 1) against the learned start (kNN + MLP
    prior, emdq_learned_start + emdq_fit_from); outside the timed steps."""
    W, H = P.cfg.width, P.cfg.height
    weights = E.load_start_weights()
    p0 = torch.empty(P.cfg.n_matches, dtype=torch.float32, device="cuda")
    rng = np.random.default_rng(11)
    ix, iy = rng.integers(0, W, 4000), rng.integers(0, H, 4000)
    truth_px = P.truth_map(np.stack([ix, iy], 1).astype(np.float64))
    fld = torch.empty((H, W, 2), dtype=torch.float32, device="cuda")
    res = {}
    for name in ("learned", "plain"):   # the model ends with the plain fit
        ts = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if name == "plain":
                model.fit(src, dst, W, H, stream=stream)
            else:
                E.emdq_learned_start(src, dst, W, H, weights, p0, stream=stream)
                model.fit_from(src, dst, W, H, p0, stream=stream)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        r = model.results()
        model.field(0, 0, W, H, fld, stream=stream)
        f = fld.cpu().numpy()[iy, ix].astype(np.float64)
        e = np.sqrt(np.sum((f - truth_px) ** 2, 1))
        res[name] = dict(em_iters=r["iters"], fit_ms=round(float(np.median(ts)) * 1e3, 4),
                         n_inliers=r["n_in"], px_err_vs_truth_rms=round(float(np.sqrt(np.mean(e ** 2))), 4),
                         px_err_vs_truth_max=round(float(e.max()), 4),
                         mask_f1_vs_truth=round(float(2 * np.sum(r["mask"].astype(bool) & P.inlier)
                                                      / (r["mask"].sum() + P.inlier.sum())), 5))
    res["start"] = "16-NN features, 64-128-128-1 GELU MLP trained on synthetic pairs (start_mlp.npy)"
    return res


def truth_error(torch, pairs, models):
    """Mean over pairs of the rms field error against the generator's truth
    at 2000 sampled pixels per pair."""
    errs = []
    for P, m in zip(pairs, models):
        W, H = P.cfg.width, P.cfg.height
        rng = np.random.default_rng(P.seed)
        ix, iy = rng.integers(0, W, 2000), rng.integers(0, H, 2000)
        fld = torch.empty((H, W, 2), dtype=torch.float32, device="cuda")
        m.field(0, 0, W, H, fld)
        f = fld.cpu().numpy()[iy, ix].astype(np.float64)
        t = P.truth_map(np.stack([ix, iy], 1).astype(np.float64))
        errs.append(np.sqrt(np.mean(np.sum((f - t) ** 2, 1))))
    return round(float(np.mean(errs)), 4)


def plain_sequential(E, torch, pairs, srcs, dsts, frames, canvases, layouts, sizes, stream,
                     reps=3):
    """The same pairs through plain single-pair calls (emdq_fit with p = 1,
    then emdq_warp), one pair after the other: frames/s and field error."""
    models = [E.Model(P.cfg.n_matches) for P in pairs]

    def run():
        for m, s_, d_, f_, c_, (cw, ch, ox, oy), (w, h) in zip(models, srcs, dsts, frames,
                                                                canvases, layouts, sizes):
            m.fit(s_, d_, w, h, stream=stream)
            m.warp(f_, c_, ox, oy, 0, 0, w, h, stream=stream)
    run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        run()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return dict(frames_per_s=round(len(pairs) * reps / wall, 2),
                px_err_vs_truth_rms_mean=truth_error(torch, pairs, models))


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    import torch

    from paper_2103_07414_amd import emdq as E
    from paper_2103_07414_amd import synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    wl = args.workload
    prec = {"fhd-f16": "f16", "fhd-bf16": "bf16"}.get(wl, "f32")
    batched = wl.startswith("batch64")
    learned = wl == "batch64-learned"
    if batched:
        pairs = synth.gen_batch(64)
    else:
        pairs = [synth.gen_config(2 if wl == "production" else 4, args.pair)]
    models = [E.Model(P.cfg.n_matches) for P in pairs]
    for m in models:
        m.set_precision(prec)
    srcs = [torch.from_numpy(P.src).to(dev) for P in pairs]
    dsts = [torch.from_numpy(P.dst).to(dev) for P in pairs]
    frames = [torch.from_numpy(P.frame).to(dev) for P in pairs]
    layouts = [synth.canvas_layout(P.cfg) for P in pairs]
    canvases = [torch.zeros((ch, cw, 4), dtype=torch.float32, device=dev)
                for cw, ch, _, _ in layouts]
    sizes = [(P.cfg.width, P.cfg.height) for P in pairs]
    batch = E.Batch(len(pairs)) if batched else None
    if learned:
        start_w = E.load_start_weights()
        starts = [torch.empty(P.cfg.n_matches, dtype=torch.float32, device=dev) for P in pairs]

    def step(ev=None):
        if learned:
            batch.learned_start(srcs, dsts, sizes, start_w, starts, stream=stream)
            batch.fit(models, srcs, dsts, sizes, stream=stream, init_ps=starts)
        elif batch is not None:
            batch.fit(models, srcs, dsts, sizes, stream=stream)
        else:
            models[0].fit(srcs[0], dsts[0], *sizes[0], stream=stream)
        if ev is not None:
            ev[0].record(stream)
        if batch is not None:
            batch.warp(models, frames, canvases, [(ox, oy) for _, _, ox, oy in layouts],
                       [(0, 0, w, h) for w, h in sizes], stream=stream)
        else:
            cw, ch, ox, oy = layouts[0]
            models[0].warp(frames[0], canvases[0], ox, oy, 0, 0, *sizes[0], stream=stream)
        if ev is not None:
            ev[1].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    res = [m.results() for m in models]
    for r in res:
        if r["status"] < 0:
            raise SystemExit(f"fit failed: {E.status_string(r['status'])}")

    events = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(events[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    warp_ms = float(np.mean([a.elapsed_time(b) for a, b in events]))

    pix = sum(w * h for w, h in sizes)
    flops = sum(12.0 * w * h * r["n_in"] for (w, h), r in zip(sizes, res))
    achieved = flops / (warp_ms * 1e-3) / 1e12
    peak = PEAK_TFLOPS[prec]
    kernel = {"f32": "k_field<warp>", "f16": "k_field_half<warp,f16>",
              "bf16": "k_field_half<warp,bf16>"}[prec]
    if batch is not None:
        kernel = "k_field_b<warp>"
    roofline = dict(bound="mfma", achieved=round(achieved, 3), peak=peak, unit="TFLOP/s",
                    frac=round(achieved / peak, 4),
                    traffic=TRAFFIC_BYTES if wl == "production" else None, kernel=kernel,
                    algorithmic_flops_per_launch=flops, avg_launch_ms=round(warp_ms, 5))
    ms_per_step = wall / args.steps * 1e3
    if wl == "production":
        workload = ("single frame pair, plain EMDQ at production size: 1280x1024 RGB uint8 "
                    "frame, N=2000 matches (30% outliers, 8 bumps amp 15 px sigma 80 px), "
                    "field + bilinear warp + merge into a 4096x4096 RGBA FP32 canvas")
    elif batched:
        workload = ("64 independent pairs of mixed size (640x480 / 1280x1024 / 1920x1080, "
                    "N 300-3000, 10-40% outliers), batched fit + batched warp, one canvas each"
                    + (", EM started from the learned prior" if learned else ""))
    else:
        workload = (f"single 1920x1080 pair, N=4000 (30% outliers), field + warp into a "
                    f"1920x1080 RGBA FP32 canvas, blend operands {prec}")
    cfg = dict(workload=workload, pairs=len(pairs), pixels_per_step=pix,
               n_matches=sum(P.cfg.n_matches for P in pairs),
               n_inliers=sum(r["n_in"] for r in res),
               em_iters=[r["iters"] for r in res] if len(res) > 1 else res[0]["iters"],
               precision=prec)
    if len(pairs) == 1:
        cfg.update(frame=list(sizes[0]), canvas=list(layouts[0][:2]), seed=pairs[0].seed)
    out = dict(metric=METRIC, value=round(pix * args.steps / wall / 1e6, 3), unit="Mpix/s",
               n_gpus=1, steps=args.steps, warmup=args.warmup,
               ms_per_step=round(ms_per_step, 4), higher_is_better=True, scaling="weak",
               vs_baseline=None, dtype=prec if prec != "f32" else "f32", data="synthetic",
               config=cfg, warp_only_mpix_s=round(pix / (warp_ms * 1e-3) / 1e6, 2),
               fit_ms=round(ms_per_step - warp_ms, 4), roofline=roofline, learned_init=None)
    if wl == "production":
        out["learned_init"] = learned_vs_plain(E, torch, pairs[0], models[0], srcs[0], dsts[0],
                                               stream)
    if batched:
        out["this_form"] = dict(frames_per_s=round(len(pairs) * args.steps / wall, 2),
                                px_err_vs_truth_rms_mean=truth_error(torch, pairs, models))
        out["plain_single_pair_calls"] = plain_sequential(E, torch, pairs, srcs, dsts, frames,
                                                          canvases, layouts, sizes, stream)
    if not args.no_cpu_baseline:
        sample = pairs[:1] if len(pairs) == 1 else pairs[:4]
        fits, cpu = cpu_baseline(sample, args.cpu_seconds)
        out["cpu_baseline"] = cpu
        # px error of the GPU field against the oracle on sampled pixels of
        # the first pair, and mask agreement of the sampled pairs
        import oracle as O
        P, f = pairs[0], fits[0]
        W, H = sizes[0]
        fld = torch.empty((H, W, 2), dtype=torch.float32, device=dev)
        models[0].field(0, 0, W, H, fld)
        rng = np.random.default_rng(7)
        pts = rng.integers(0, [W, H], (2000, 2)).astype(np.float64)
        _, want = O.field_points(P.src, f.scale, f.q, f.mask, f.alpha, pts)
        got = fld.cpu().numpy()[pts[:, 1].astype(int), pts[:, 0].astype(int)]
        out["px_err_vs_oracle"] = float(np.abs(got - want).max())
        out["mask_equal_oracle"] = bool(all(np.array_equal(r["mask"], g.mask)
                                            for r, g in zip(res, fits)))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
