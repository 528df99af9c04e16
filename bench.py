"""Benchmark of the EMDQ hot path on one MI355X.

One step = the whole path over one batch of synthetic input, inputs resident
in HBM: emdq_fit (per-match similarity fits as dual quaternions + EM inlier
reweighting over the N x N Gaussian weights) followed by emdq_warp (dense
per-pixel DQ blend on MFMA, Eq. (1), bilinear sample and colour merge into
the mosaic canvas).

Workloads (--workload):
  production  (default) 1280 x 1024 RGB uint8 frame, N = 2000 matches (30 %
              outliers, 8 Gaussian bumps), 4096 x 4096 RGBA FP32 canvas, FP32.
              Outside the timed steps it also reports the learned EM start
              against the plain one (EM iterations, inlier F1, px error) on
              this pair and on a 1920 x 1080, N = 5000 pair (40 % outliers,
              12 bumps of 25 px), and the 64-pair batch below three ways:
              batched with the learned start, batched with the plain start,
              and plain single-pair calls (frames/s and px error)
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
Unless --no-extras, steady_clocks repeats the timed steps after --settle more
untimed steps (the GPU's clocks take a few dozen steps to settle after idle);
it is reported beside the headline, not in it.
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
# HBM traffic of the production warp call (factor-table kernel + blend kernel)
# per call, from rocprofv3 FETCH_SIZE + WRITE_SIZE (KiB per dispatch) scaled by
# the copy-kernel calibration (a 256 MiB copy reads FETCH_SIZE 131,085.1 KiB
# and WRITE_SIZE 262,144.0 KiB): (57.75 + 43,018.16) x 262,144 / 131,085.1 +
# (12,609.0 + 18,814.06) x 1.0.  Set to None whenever the kernels change,
# until the counters are taken again.
TRAFFIC_BYTES = round(((57.75 + 43018.16) * 262144.0 / 131085.1 + (12609.0 + 18814.06)) * 1024)
# Average duration of the same call in the committed kernel trace of the
# production command (profiles/k_field_warp_f32_1280x1024_n2000.md): the two
# kernels' trace averages added, beside the live HIP-event duration the
# roofline fraction is computed from.
PROFILE = dict(file="profiles/k_field_warp_f32_1280x1024_n2000.md",
               kernels=["k_field_tables", "k_field<1, 4, 1, true>"],
               kernel_avg_us=[7.84, 195.67], avg_launch_ms=0.20351)
WORKLOADS = ("production", "fhd-f32", "fhd-f16", "fhd-bf16", "batch64", "batch64-learned")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--settle", type=int, default=50,
                    help="extra untimed steps before the steady-clock repeat (extras)")
    ap.add_argument("--pair", type=int, default=1)
    ap.add_argument("--workload", choices=WORKLOADS, default="production")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the reports after the timed steps (learned vs plain start, "
                         "batch forms), e.g. under a profiler")
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


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_threads(n):
    """Sets the OpenMP thread count of the oracle's parallel loops (the
    oracle is built with gcc -fopenmp, i.e. libgomp); returns the previous
    maximum."""
    import ctypes
    gomp = ctypes.CDLL("libgomp.so.1")
    prev = gomp.omp_get_max_threads()
    gomp.omp_set_num_threads(int(n))
    return prev


def oracle_step(O, P):
    """One whole oracle step of a pair: EM fit, then field, bilinear sample
    and merge of every frame pixel into a zero canvas.  Returns (fit, fit s,
    field+warp s)."""
    W, H = P.cfg.width, P.cfg.height
    canvas = np.zeros((H, W, 4))
    t0 = time.perf_counter()
    f = O.fit(P.src, P.dst, W, H)
    t1 = time.perf_counter()
    O.warp(P.src, f.scale, f.q, f.mask, f.alpha, P.frame, canvas, 0, 0, 0, 0, W, H)
    t2 = time.perf_counter()
    return f, t1 - t0, t2 - t1


def cpu_baseline(pairs, min_seconds, single_thread):
    """The FP64 oracle on the host: whole steps of the workload's pairs (EM fit
    + field, warp and merge of every frame pixel), cycling over the pairs
    until at least `min_seconds` have passed, on all host threads.  With
    `single_thread`, one step each of the small (320x240, N=200) and the
    production (1280x1024, N=2000) pair on one thread as well."""
    import oracle as O
    from paper_2103_07414_amd import synth
    reps, px, t_fit, t_warp = 0, 0, 0.0, 0.0
    t_start = time.perf_counter()
    fits = []
    while True:
        P = pairs[reps % len(pairs)]
        f, a, b = oracle_step(O, P)
        if reps < len(pairs):
            fits.append(f)
        reps += 1
        px += P.cfg.width * P.cfg.height
        t_fit += a
        t_warp += b
        if time.perf_counter() - t_start >= min_seconds:
            break
    total = t_fit + t_warp
    threads = oracle_threads(1)
    first = pairs[0].cfg
    out = dict(value=round(px / total / 1e6, 4), unit="Mpix/s", cores=threads,
               kind="oracle", cpu_model=cpu_model(), host_cpus=os.cpu_count(),
               sample=f"{reps} whole pair steps ({min(reps, len(pairs))}"
                      f" distinct pairs, first {first.width}x{first.height} "
                      f"N={first.n_matches}): EM fit {t_fit / reps * 1e3:.0f} ms + "
                      f"field/warp/merge of every pixel {t_warp / reps * 1e3:.0f} ms "
                      f"per pair; FP64, OpenMP on {threads} threads, {total:.1f} s in total")
    try:
        if single_thread:
            one = {}
            for name, cfg in (("small_320x240_n200", 1), ("production_1280x1024_n2000", 2)):
                P = synth.gen_config(cfg, 1)
                _, a, b = oracle_step(O, P)
                one[name] = dict(fit_ms=round(a * 1e3, 2), field_warp_ms=round(b * 1e3, 2),
                                 mpix_s=round(P.cfg.width * P.cfg.height / (a + b) / 1e6, 4))
            out["single_thread"] = one
    finally:
        oracle_threads(threads)
    return fits, out


def learned_vs_plain(E, torch, P, stream, reps=5):
    """EM iterations, inlier F1 and field error against the generator's ground
    truth, plain start (p = 1) against the learned start (kNN + MLP prior,
    emdq_learned_start + emdq_fit_from), on one pair; outside the timed
    steps."""
    dev = torch.device("cuda:0")
    W, H = P.cfg.width, P.cfg.height
    model = E.Model(P.cfg.n_matches)
    src, dst = torch.from_numpy(P.src).to(dev), torch.from_numpy(P.dst).to(dev)
    weights = E.load_start_weights()
    p0 = torch.empty(P.cfg.n_matches, dtype=torch.float32, device=dev)
    rng = np.random.default_rng(11)
    ix, iy = rng.integers(0, W, 4000), rng.integers(0, H, 4000)
    truth_px = P.truth_map(np.stack([ix, iy], 1).astype(np.float64))
    fld = torch.empty((H, W, 2), dtype=torch.float32, device=dev)
    res = {}
    for name in ("learned", "plain"):
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
        res[name] = dict(em_iters=r["iters"], status=r["status"],
                         fit_ms=round(float(np.median(ts)) * 1e3, 4),
                         n_inliers=r["n_in"], px_err_vs_truth_rms=round(float(np.sqrt(np.mean(e ** 2))), 4),
                         px_err_vs_truth_max=round(float(e.max()), 4),
                         mask_f1_vs_truth=round(float(2 * np.sum(r["mask"].astype(bool) & P.inlier)
                                                      / (r["mask"].sum() + P.inlier.sum())), 5))
    model.close()
    res["pair"] = dict(frame=[W, H], n_matches=P.cfg.n_matches, outliers=P.cfg.outlier_rate,
                       bumps=[P.cfg.n_bumps, P.cfg.bump_amp, P.cfg.bump_sigma], seed=P.seed)
    res["start"] = "16-NN features, 64-128-128-1 GELU MLP trained on synthetic pairs (start_mlp.npy)"
    return res


class Pairs:
    """Device copies of a list of pairs, a model and a canvas each, and the
    step functions that run them through the library."""

    def __init__(self, E, torch, pairs, prec="f32"):
        from paper_2103_07414_amd import synth
        dev = torch.device("cuda:0")
        self.E, self.torch, self.pairs = E, torch, pairs
        self.models = [E.Model(P.cfg.n_matches) for P in pairs]
        for m in self.models:
            m.set_precision(prec)
        self.srcs = [torch.from_numpy(P.src).to(dev) for P in pairs]
        self.dsts = [torch.from_numpy(P.dst).to(dev) for P in pairs]
        self.frames = [torch.from_numpy(P.frame).to(dev) for P in pairs]
        self.layouts = [synth.canvas_layout(P.cfg) for P in pairs]
        self.canvases = [torch.zeros((ch, cw, 4), dtype=torch.float32, device=dev)
                         for cw, ch, _, _ in self.layouts]
        self.sizes = [(P.cfg.width, P.cfg.height) for P in pairs]
        self.batch = None
        self.start_w = None
        self.starts = None
        self.warp_prepared = False

    def use_batch(self, learned):
        E, torch = self.E, self.torch
        self.batch = self.batch or E.Batch(len(self.pairs))
        if learned and self.start_w is None:
            self.start_w = E.load_start_weights()
            self.starts = [torch.empty(P.cfg.n_matches, dtype=torch.float32, device="cuda")
                           for P in self.pairs]
        self.learned = learned

    def fit(self, stream):
        if self.batch is None:
            for m, s_, d_, (w, h) in zip(self.models, self.srcs, self.dsts, self.sizes):
                m.fit(s_, d_, w, h, stream=stream)
        elif self.learned:
            self.batch.learned_start(self.srcs, self.dsts, self.sizes, self.start_w,
                                     self.starts, stream=stream)
            self.batch.fit(self.models, self.srcs, self.dsts, self.sizes, stream=stream,
                           init_ps=self.starts)
        else:
            self.batch.fit(self.models, self.srcs, self.dsts, self.sizes, stream=stream)

    def warp(self, stream):
        if self.batch is None:
            for m, f_, c_, (cw, ch, ox, oy), (w, h) in zip(self.models, self.frames,
                                                            self.canvases, self.layouts,
                                                            self.sizes):
                m.warp(f_, c_, ox, oy, 0, 0, w, h, stream=stream)
        else:
            # the batched warp's job table (pointers, regions, tile counts:
            # nothing that depends on a fit) is built once, as a pipeline
            # with fixed frame and canvas buffers does; each launch reads
            # the fits of that step
            if not self.warp_prepared:
                self.batch.prepare_warp(self.models, self.frames, self.canvases,
                                        [(ox, oy) for _, _, ox, oy in self.layouts],
                                        [(0, 0, w, h) for w, h in self.sizes])
                self.warp_prepared = True
            self.batch.launch(stream)

    def step(self, stream, ev=None):
        self.fit(stream)
        if ev is not None:
            ev[0].record(stream)
        self.warp(stream)
        if ev is not None:
            ev[1].record(stream)

    def frames_per_s(self, stream, steps):
        """Whole steps (fit + warp of every pair), timed on the wall clock."""
        torch = self.torch
        self.step(stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            self.step(stream)
        torch.cuda.synchronize()
        return len(self.pairs) * steps / (time.perf_counter() - t0)

    def truth_error(self):
        """Mean over pairs of the rms field error against the generator's
        truth at 2000 sampled pixels per pair."""
        torch = self.torch
        errs = []
        for P, m in zip(self.pairs, self.models):
            W, H = P.cfg.width, P.cfg.height
            rng = np.random.default_rng(P.seed)
            ix, iy = rng.integers(0, W, 2000), rng.integers(0, H, 2000)
            fld = torch.empty((H, W, 2), dtype=torch.float32, device="cuda")
            m.field(0, 0, W, H, fld)
            f = fld.cpu().numpy()[iy, ix].astype(np.float64)
            t = P.truth_map(np.stack([ix, iy], 1).astype(np.float64))
            errs.append(np.sqrt(np.mean(np.sum((f - t) ** 2, 1))))
        return round(float(np.mean(errs)), 4)

    def close(self):
        for m in self.models:
            m.close()
        if self.batch is not None:
            self.batch.close()


def batch_forms(E, torch, pairs, stream, steps=5):
    """The 64 mixed pairs three ways, on the same GPU: the batched entry
    points with the learned start, the batched entry points with the plain
    start, and plain single-pair calls (emdq_fit with p = 1, then emdq_warp,
    one pair after the other).  frames/s of whole steps and the mean field
    error against the generator's truth."""
    out = {}
    for name, batched, learned in (("learned_batched", True, True),
                                   ("plain_batched", True, False),
                                   ("plain_single_pair_calls", False, False)):
        R = Pairs(E, torch, pairs)
        if batched:
            R.use_batch(learned)
        fps = R.frames_per_s(stream, steps)
        res = [m.results() for m in R.models]
        out[name] = dict(frames_per_s=round(fps, 2), px_err_vs_truth_rms_mean=R.truth_error(),
                         em_iters_max=max(r["iters"] for r in res),
                         em_iters_mean=round(float(np.mean([r["iters"] for r in res])), 2))
        R.close()
    out["learned_batched_over_plain_single"] = round(
        out["learned_batched"]["frames_per_s"] / out["plain_single_pair_calls"]["frames_per_s"], 3)
    return out


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
    R = Pairs(E, torch, pairs, prec)
    if batched:
        R.use_batch(learned)
    models, sizes, layouts = R.models, R.sizes, R.layouts

    for _ in range(args.warmup):
        R.step(stream)
    torch.cuda.synchronize()
    res = [m.results() for m in models]
    for r in res:
        if r["status"] < 0:
            raise SystemExit(f"fit failed: {E.status_string(r['status'])}")

    def timed(steps):
        """Wall time of `steps` steps and the HIP-event time of each warp call."""
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(steps):
            R.step(stream, evs[k])
        torch.cuda.synchronize()
        return time.perf_counter() - t0, np.array([a.elapsed_time(b) for a, b in evs])

    wall, warp_times = timed(args.steps)
    warp_ms = float(np.mean(warp_times))

    pix = sum(w * h for w, h in sizes)
    flops = sum(12.0 * w * h * r["n_in"] for (w, h), r in zip(sizes, res))
    achieved = flops / (warp_ms * 1e-3) / 1e12
    peak = PEAK_TFLOPS[prec]
    # the warp call: the factor-table kernel, then the blend kernel
    kernel = {"f32": "k_field_tables + k_field<warp>",
              "f16": "k_half_tables<f16> + k_field_half<warp,f16>",
              "bf16": "k_half_tables<bf16> + k_field_half<warp,bf16>"}[prec]
    if batched:
        kernel = "k_field_tables_b + k_field_b<warp>"
    roofline = dict(bound="mfma", achieved=round(achieved, 3), peak=peak, unit="TFLOP/s",
                    frac=round(achieved / peak, 4),
                    traffic=TRAFFIC_BYTES if wl == "production" else None, kernel=kernel,
                    algorithmic_flops_per_launch=flops, avg_launch_ms=round(warp_ms, 5),
                    duration_source="HIP events recorded around every warp call (both "
                                    "kernels) on the stream it runs on, mean over the "
                                    "timed steps",
                    warp_ms_p10_median_p90=[round(float(q), 5) for q in
                                            np.quantile(warp_times, [0.1, 0.5, 0.9])])
    if wl == "production":
        roofline["profile"] = dict(PROFILE, frac_at_profile_duration=round(
            flops / (PROFILE["avg_launch_ms"] * 1e-3) / 1e12 / peak, 4))
    ms_per_step = wall / args.steps * 1e3
    if wl == "production":
        workload = ("single frame pair, plain EMDQ at production size: 1280x1024 RGB uint8 "
                    "frame, N=2000 matches (30% outliers, 8 bumps amp 15 px sigma 80 px), "
                    "field + bilinear warp + merge into a 4096x4096 RGBA FP32 canvas")
    elif batched:
        workload = ("64 independent pairs of mixed size (640x480 / 1280x1024 / 1920x1080, "
                    "N 300-3000, 10-40% outliers), batched fit + batched warp (its job table "
                    "prepared once), one canvas each"
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
               vs_baseline=None, dtype=prec, data="synthetic",
               config=cfg, warp_only_mpix_s=round(pix / (warp_ms * 1e-3) / 1e6, 2),
               fit_ms=round(ms_per_step - warp_ms, 4), roofline=roofline, learned_init=None)
    if not args.no_extras:
        # The same timed steps again once the GPU's clocks have settled: the
        # first few dozen steps after idle run at lower clocks.  Outside the
        # headline (which is the steps above).
        for _ in range(args.settle):
            R.step(stream)
        w2, t2 = timed(args.steps)
        m2 = float(np.mean(t2))
        out["steady_clocks"] = dict(
            untimed_steps_before=args.warmup + args.steps + args.settle, steps=args.steps,
            ms_per_step=round(w2 / args.steps * 1e3, 4),
            value=round(pix * args.steps / w2 / 1e6, 3), warp_ms=round(m2, 5),
            frac=round(flops / (m2 * 1e-3) / 1e12 / peak, 4))
    if wl == "production" and not args.no_extras:
        out["learned_init"] = learned_vs_plain(E, torch, pairs[0], stream)
        out["learned_init_fhd_n5000"] = learned_vs_plain(E, torch, synth.gen_config(5, 1),
                                                         stream)
        out["batch64"] = batch_forms(E, torch, synth.gen_batch(64), stream)
    if batched and not args.no_extras:
        out["this_form"] = dict(frames_per_s=round(len(pairs) * args.steps / wall, 2),
                                px_err_vs_truth_rms_mean=R.truth_error())
        S = Pairs(E, torch, pairs)
        out["plain_single_pair_calls"] = dict(frames_per_s=round(S.frames_per_s(stream, 3), 2),
                                              px_err_vs_truth_rms_mean=S.truth_error())
        S.close()
    if not args.no_cpu_baseline:
        sample = pairs[:1] if len(pairs) == 1 else pairs[:4]
        fits, cpu = cpu_baseline(sample, args.cpu_seconds, single_thread=wl == "production")
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
    R.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
