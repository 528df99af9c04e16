"""Trains the learned EM start (a per-match inlier prior) on the GPU with the
library's own kernels, on synthetic pairs labelled by the plain EMDQ fit.

For every pair: emdq_fit (plain start) gives the inlier mask used as the
label, emdq_start_features the 64 features of every match; then
emdq_start_train_step runs Adam minibatch steps (mean binary cross-entropy).
Writes the flat FP32 weight vector (W1[128][64], b1, W2[128][128], b2,
w3[128], b3) to start_mlp.npy, which emdq_learned_start reads.

Usage (needs the GPU):
  python -m paper_2103_07414_amd.train_start [--pairs 10000] [--epochs 2] [--out PATH]
"""
import argparse
import os
import time

import numpy as np

from paper_2103_07414_amd import emdq as E
from paper_2103_07414_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))
N_W = 24961


def random_pair(rng, seed):
    """A pair of random shape: 320x240 to 1920x1080, N 200-5000, 5-45 %
    outliers, 2-12 bumps of 5-25 px and width 40-100 px."""
    w, h = [(320, 240), (640, 480), (1280, 1024), (1920, 1080)][int(rng.integers(0, 4))]
    cfg = synth.PairConfig(w, h, int(rng.integers(200, 5001)), float(rng.uniform(0.05, 0.45)),
                           int(rng.integers(2, 13)), float(rng.uniform(5, 25)),
                           float(rng.uniform(40, 100)))
    return synth.gen_pair(cfg, seed, with_frame=False)


def init_weights(rng):
    """He-style initial weights for the 64-128-128-1 network."""
    parts = [rng.normal(0, np.sqrt(2 / 64), 128 * 64), np.zeros(128),
             rng.normal(0, np.sqrt(2 / 128), 128 * 128), np.zeros(128),
             rng.normal(0, np.sqrt(1 / 128), 128), np.zeros(1)]
    return np.concatenate(parts).astype(np.float32)


def main():
    import torch
    ap = argparse.ArgumentParser()
    ap.add_argument("--pairs", type=int, default=10000)
    ap.add_argument("--epochs", type=int, default=2)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--groups", type=int, default=64)
    ap.add_argument("--seed", type=int, default=77)
    ap.add_argument("--out", default=os.path.join(HERE, "start_mlp.npy"))
    args = ap.parse_args()
    rng = np.random.default_rng(args.seed)
    dev = torch.device("cuda:0")

    # ---- data: features and plain-EMDQ labels, all on the GPU
    t0 = time.perf_counter()
    model = E.Model(5000)
    feats, labels = [], []
    for i in range(args.pairs):
        P = random_pair(rng, 900000 + i)
        s = torch.from_numpy(P.src).to(dev)
        d = torch.from_numpy(P.dst).to(dev)
        model.fit(s, d, P.cfg.width, P.cfg.height)
        r = model.results()
        if r["status"] < 0:
            continue
        f = torch.empty((P.cfg.n_matches, 64), dtype=torch.float32, device=dev)
        E.emdq_start_features(s, d, P.cfg.width, P.cfg.height, f)
        feats.append(f)
        labels.append(torch.from_numpy(r["mask"].astype(np.float32)).to(dev))
        if (i + 1) % 1000 == 0:
            print(f"{i + 1} pairs labelled ({time.perf_counter() - t0:.0f} s)", flush=True)
    feat = torch.cat(feats)
    label = torch.cat(labels)
    del feats, labels
    M = int(label.shape[0])
    print(f"{M} samples from {args.pairs} pairs, inlier fraction {label.mean().item():.3f}",
          flush=True)

    # ---- Adam on the library's training kernels
    w = torch.from_numpy(init_weights(rng)).to(dev)
    m1, m2 = torch.zeros_like(w), torch.zeros_like(w)
    G = args.groups
    work = torch.zeros(E.emdq_start_train_work_floats(G), dtype=torch.float32, device=dev)
    steps_per_epoch = M // args.batch
    total = args.epochs * steps_per_epoch
    step = 0
    for ep in range(args.epochs):
        perm = rng.permutation(M).astype(np.int32)
        perm_dev = torch.from_numpy(perm).to(dev)
        run, cnt = 0.0, 0
        for b in range(steps_per_epoch):
            step += 1
            lr = args.lr * 0.5 * (1.0 + np.cos(np.pi * (step - 1) / total))   # cosine decay
            idx = perm_dev[b * args.batch:(b + 1) * args.batch]
            E.emdq_start_train_step(w, m1, m2, step, feat, label, idx, lr, G, work)
            if b % 50 == 0:
                run += float(work[G * (N_W + 1) + N_W].item())
                cnt += 1
        print(f"epoch {ep}: mean minibatch loss {run / max(cnt, 1):.4f} "
              f"({time.perf_counter() - t0:.0f} s)", flush=True)
    out = w.cpu().numpy().astype(np.float32)
    np.save(args.out, out)
    print(f"wrote {args.out} ({out.size} weights)", flush=True)


if __name__ == "__main__":
    main()
