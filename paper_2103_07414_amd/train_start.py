"""Trains the learned EM start (a per-match inlier prior) on synthetic pairs.

Offline, CPU only; writes `start_mlp.npy` (float32, the flat weight vector
W1[128][64], b1[128], W2[128][128], b2[128], w3[128], b3 in that order), which
the library's learned start reads from device memory.

Features of match i, from its 16 nearest other matches j (source distance,
ties by index), with g = sqrt(alpha) and displacement d = dst - src:
  g (x_j - x_i),  ss((d_j - d_i) / 8)  per neighbour, ss(t) = t / (1 + |t|);
network: two GELU layers of 128, sigmoid output.  Labels: the generator's
ground-truth inlier flags.

Usage: python -m paper_2103_07414_amd.train_start [--pairs 600] [--epochs 4]
"""
import argparse
import os

import numpy as np

from paper_2103_07414_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "start_mlp.npy")
K, NF, NH = 16, 64, 128


def alpha_of(w, h, alpha0=2e-4, ref_w=480, ref_h=270):
    s = (w / ref_w + h / ref_h) / 2.0
    return alpha0 / (s * s)


def features(src, dst, alpha):
    from scipy.spatial import cKDTree
    x = src.astype(np.float64)
    d = dst.astype(np.float64) - x
    n = len(x)
    k = min(K + 1, n)
    _, idx = cKDTree(x).query(x, k=k)
    idx = idx[:, 1:]                               # drop the match itself
    g = np.sqrt(alpha)
    f = np.zeros((n, NF))
    m = idx.shape[1]
    rel = g * (x[idx] - x[:, None, :])             # [n, m, 2]
    e = (d[idx] - d[:, None, :]) / 8.0
    e = e / (1.0 + np.abs(e))
    f4 = np.concatenate([rel, e], axis=2)           # [n, m, 4]
    f[:, :4 * m] = f4.reshape(n, 4 * m)
    return f


def random_pair(rng, seed):
    w, h = [(320, 240), (640, 480), (1280, 1024), (1920, 1080)][int(rng.integers(0, 4))]
    cfg = synth.PairConfig(w, h, int(rng.integers(200, 5001)), float(rng.uniform(0.05, 0.45)),
                           int(rng.integers(2, 13)), float(rng.uniform(5, 25)),
                           float(rng.uniform(40, 100)))
    return synth.gen_pair(cfg, seed, with_frame=False)


def main():
    import torch
    ap = argparse.ArgumentParser()
    ap.add_argument("--pairs", type=int, default=600)
    ap.add_argument("--epochs", type=int, default=4)
    ap.add_argument("--seed", type=int, default=77)
    args = ap.parse_args()
    torch.manual_seed(args.seed)
    rng = np.random.default_rng(args.seed)
    X, Y = [], []
    for i in range(args.pairs):
        P = random_pair(rng, 900000 + i)
        X.append(features(P.src, P.dst, alpha_of(P.cfg.width, P.cfg.height)))
        Y.append(P.inlier.astype(np.float64))
    X = torch.from_numpy(np.concatenate(X)).float()
    Y = torch.from_numpy(np.concatenate(Y)).float()
    print(f"{len(Y)} samples, inlier fraction {Y.mean():.3f}", flush=True)
    net = torch.nn.Sequential(torch.nn.Linear(NF, NH), torch.nn.GELU(),
                              torch.nn.Linear(NH, NH), torch.nn.GELU(), torch.nn.Linear(NH, 1))
    opt = torch.optim.Adam(net.parameters(), lr=2e-3)
    sched = torch.optim.lr_scheduler.CosineAnnealingLR(opt, args.epochs * (len(Y) // 4096 + 1))
    lossf = torch.nn.BCEWithLogitsLoss()
    for ep in range(args.epochs):
        perm = torch.randperm(len(Y))
        tot = 0.0
        for b in range(0, len(Y), 4096):
            sel = perm[b:b + 4096]
            opt.zero_grad()
            loss = lossf(net(X[sel]).squeeze(1), Y[sel])
            loss.backward()
            opt.step()
            sched.step()
            tot += loss.item() * len(sel)
        with torch.no_grad():
            acc = ((net(X).squeeze(1) > 0).float() == Y).float().mean().item()
        print(f"epoch {ep}: loss {tot / len(Y):.4f} accuracy {acc:.4f}", flush=True)
    l1, l2, l3 = net[0], net[2], net[4]
    w = torch.cat([l1.weight.reshape(-1), l1.bias, l2.weight.reshape(-1), l2.bias,
                   l3.weight.reshape(-1), l3.bias]).detach().numpy().astype(np.float32)
    assert w.size == NH * NF + NH + NH * NH + NH + NH + 1
    np.save(OUT, w)
    print(f"wrote {OUT} ({w.size} weights)")


if __name__ == "__main__":
    main()
