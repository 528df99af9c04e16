"""Benchmark of the EMDQ hot path on one MI355X.

One step = the whole path over one synthetic frame pair, inputs resident in
HBM: emdq_fit (per-match similarity fits as dual quaternions + EM inlier
reweighting over the N x N Gaussian weights) followed by emdq_warp (dense
per-pixel DQ blend on MFMA, Eq. (1), bilinear sample and colour merge into
the mosaic canvas).  Workload: 1280 x 1024 RGB uint8 frame, N = 2000 matches
(30 % outliers, 8 Gaussian bumps), 4096 x 4096 RGBA FP32 canvas.

Prints one JSON line.  value = frame pixels x steps / wall time of the timed
steps (Mpix/s).  The roofline object covers the field + warp kernel, timed
with HIP events on the stream it runs on; cpu_baseline times the FP64 oracle
on the host cores on whole steps of the same workload.
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
PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0
# HBM traffic of the field + warp kernel per launch, from rocprofv3
# FETCH_SIZE + WRITE_SIZE (KiB per dispatch) scaled by the copy-kernel
# calibration; None until measured for the current kernel.
TRAFFIC_BYTES = None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--pair", type=int, default=1)
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


def cpu_baseline(P, min_seconds):
    """The FP64 oracle on the host: whole steps (EM fit + field, warp and
    merge of every frame pixel) repeated for at least `min_seconds`."""
    import oracle as O
    W, H = P.cfg.width, P.cfg.height
    cw, ch, ox, oy = canvas_layout(P.cfg)
    canvas = np.zeros((H, W, 4))
    reps, t_fit, t_warp = 0, 0.0, 0.0
    t_start = time.perf_counter()
    while True:
        t0 = time.perf_counter()
        f = O.fit(P.src, P.dst, W, H)
        t1 = time.perf_counter()
        O.warp(P.src, f.scale, f.q, f.mask, f.alpha, P.frame, canvas, 0, 0, 0, 0, W, H)
        t2 = time.perf_counter()
        reps += 1
        t_fit += t1 - t0
        t_warp += t2 - t1
        if t2 - t_start >= min_seconds:
            break
    total = t_fit + t_warp
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    return f, dict(value=round(W * H * reps / total / 1e6, 4), unit="Mpix/s", cores=threads,
                   kind="oracle",
                   sample=f"{reps} whole steps on the same pair: EM fit ({f.iters} iterations, "
                          f"{t_fit / reps * 1e3:.0f} ms) + field/warp/merge of all {W}x{H} "
                          f"pixels ({t_warp / reps * 1e3:.0f} ms); FP64, OpenMP, "
                          f"{total:.1f} s in total")


def canvas_layout(cfg):
    from paper_2103_07414_amd import synth
    return synth.canvas_layout(cfg)


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
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
    P = synth.gen_config(2, args.pair)
    W, H = P.cfg.width, P.cfg.height
    cw, ch, ox, oy = synth.canvas_layout(P.cfg)
    src = torch.from_numpy(P.src).to(dev)
    dst = torch.from_numpy(P.dst).to(dev)
    frame = torch.from_numpy(P.frame).to(dev)
    canvas = torch.zeros((ch, cw, 4), dtype=torch.float32, device=dev)
    model = E.Model(P.cfg.n_matches)
    stream = torch.cuda.current_stream()

    def step(ev=None):
        model.fit(src, dst, W, H, stream=stream)
        if ev is not None:
            ev[0].record(stream)
        model.warp(frame, canvas, ox, oy, 0, 0, W, H, stream=stream)
        if ev is not None:
            ev[1].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    res = model.results()
    if res["status"] < 0:
        raise SystemExit(f"fit failed: {E.status_string(res['status'])}")

    events = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(events[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    warp_ms = float(np.mean([a.elapsed_time(b) for a, b in events]))

    n_in = res["n_in"]
    flops = 12.0 * W * H * n_in
    achieved = flops / (warp_ms * 1e-3) / 1e12
    roofline = dict(bound="mfma", achieved=round(achieved, 3), peak=PEAK_FP32_MFMA_TFLOPS,
                    unit="TFLOP/s", frac=round(achieved / PEAK_FP32_MFMA_TFLOPS, 4),
                    traffic=TRAFFIC_BYTES, kernel="k_field<warp>",
                    algorithmic_flops_per_launch=flops,
                    avg_launch_ms=round(warp_ms, 5))

    ms_per_step = wall / args.steps * 1e3
    out = dict(metric=METRIC, value=round(W * H * args.steps / wall / 1e6, 3), unit="Mpix/s",
               n_gpus=1, steps=args.steps, warmup=args.warmup,
               ms_per_step=round(ms_per_step, 4), higher_is_better=True, scaling="weak",
               vs_baseline=None, dtype="f32", data="synthetic",
               config=dict(workload="single frame pair, plain EMDQ at production size: "
                                    "1280x1024 RGB uint8 frame, N=2000 matches (30% outliers, "
                                    "8 bumps amp 15 px sigma 80 px), field + bilinear warp + "
                                    "merge into a 4096x4096 RGBA FP32 canvas",
                           frame=[W, H], n_matches=P.cfg.n_matches, canvas=[cw, ch],
                           seed=P.seed, em_iters=res["iters"], n_inliers=n_in),
               warp_only_mpix_s=round(W * H / (warp_ms * 1e-3) / 1e6, 2),
               fit_ms=round(ms_per_step - warp_ms, 4),
               roofline=roofline, learned_init=None)
    if not args.no_cpu_baseline:
        f, cpu = cpu_baseline(P, args.cpu_seconds)
        out["cpu_baseline"] = cpu
        # px error of the GPU field against the oracle on sampled pixels
        import oracle as O
        fld = torch.empty((H, W, 2), dtype=torch.float32, device=dev)
        model.field(0, 0, W, H, fld)
        rng = np.random.default_rng(7)
        pts = rng.integers(0, [W, H], (2000, 2)).astype(np.float64)
        _, want = O.field_points(P.src, f.scale, f.q, f.mask, f.alpha, pts)
        got = fld.cpu().numpy()[pts[:, 1].astype(int), pts[:, 0].astype(int)]
        out["px_err_vs_oracle"] = float(np.abs(got - want).max())
        out["mask_equal_oracle"] = bool(np.array_equal(res["mask"], f.mask))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
