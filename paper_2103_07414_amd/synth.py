"""Seeded synthetic inputs for the EMDQ field + warp path.

This module only draws random numbers and shapes them into test inputs: feature
matches between a reference (mosaic-side) frame and a new frame, ground-truth
inlier labels, and an RGB uint8 texture for the new frame.  It contains none of
the EMDQ arithmetic (no weights, fits, dual quaternions, blending or warping),
so both the FP64 oracle and the GPU library can be fed from it.

The paper's data (in-vivo liver / lung videos, the Hamlyn and Mandala
sequences) is not available; these synthetic pairs stand in for it.  The
deformation model is a global similarity plus a few smooth Gaussian bumps,
i.e. a smooth non-rigid motion of the kind the paper handles (Sec. I and
Sec. II-A: smooth deformation, noisy matches with mismatches), with
uniformly-replaced outliers playing the role of SURF mismatches (Sec. II-B).

Draw order is fixed so the same seed always gives the same bytes.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np

__all__ = ["PairConfig", "CONFIGS", "gen_pair", "gen_config", "gen_texture",
           "config_seed", "canvas_layout", "gen_batch", "BATCH_FRAMES"]


@dataclass(frozen=True)
class PairConfig:
    """Shape of one synthetic frame pair."""
    width: int
    height: int
    n_matches: int
    outlier_rate: float
    n_bumps: int
    bump_amp: float
    bump_sigma: float
    canvas_w: int = 0          # 0: no canvas attached to this config
    canvas_h: int = 0
    rot_deg: float = 5.0       # global rotation drawn from U(-rot_deg, rot_deg)
    scale_lo: float = 0.95
    scale_hi: float = 1.05
    shift_px: float = 10.0     # global shift drawn from U(-shift_px, shift_px)^2
    noise_px: float = 1.0      # per-axis Gaussian match noise
    texture_sigma: float = 3.0  # periodic Gaussian blur of the white-noise texture


# Named workloads.  1: small correctness pair; 2: production-size pair
# (1280x1024, N=2000, 30% outliers, 4096^2 RGBA FP32 canvas); 4 and 5: the
# 1920x1080 mixed-precision and large-N shapes.
CONFIGS = {
    1: PairConfig(320, 240, 200, 0.20, 4, 5.0, 40.0, 640, 480),
    2: PairConfig(1280, 1024, 2000, 0.30, 8, 15.0, 80.0, 4096, 4096),
    4: PairConfig(1920, 1080, 4000, 0.30, 8, 15.0, 80.0, 1920, 1080),
    5: PairConfig(1920, 1080, 5000, 0.40, 12, 25.0, 80.0, 1920, 1080),
}


def config_seed(config: int, pair: int) -> int:
    """Seed of pair `pair` of workload `config`."""
    return 1000 * int(config) + int(pair)


def canvas_layout(cfg: PairConfig):
    """Canvas size and the offset that centres a W x H ROI in it."""
    cw = cfg.canvas_w or cfg.width
    ch = cfg.canvas_h or cfg.height
    return cw, ch, (cw - cfg.width) // 2, (ch - cfg.height) // 2


def gen_texture(width: int, height: int, rng: np.random.Generator,
                sigma: float = 3.0) -> np.ndarray:
    """Smooth RGB noise texture, uint8 [height, width, 3].

    Per channel: U(0,1) white noise, periodic Gaussian blur (in the Fourier
    domain), min-max stretch to [0, 255], round to nearest.
    """
    noise = rng.random((3, height, width))
    fy = np.fft.fftfreq(height)[:, None]
    fx = np.fft.fftfreq(width)[None, :]
    transfer = np.exp(-2.0 * (np.pi ** 2) * (sigma ** 2) * (fx ** 2 + fy ** 2))
    out = np.empty((height, width, 3), dtype=np.uint8)
    for c in range(3):
        blurred = np.real(np.fft.ifft2(np.fft.fft2(noise[c]) * transfer))
        lo, hi = blurred.min(), blurred.max()
        scaled = (blurred - lo) / (hi - lo) * 255.0
        out[..., c] = np.clip(np.rint(scaled), 0, 255).astype(np.uint8)
    return out


@dataclass
class Pair:
    """One synthetic pair.  Coordinates are pixel (column, row) with pixel
    centres at integers and the origin at the top-left pixel centre."""
    cfg: PairConfig
    seed: int
    src: np.ndarray            # float32 [N, 2], reference / mosaic-side positions
    dst: np.ndarray            # float32 [N, 2], positions in the new frame
    inlier: np.ndarray         # bool [N], ground-truth labels
    frame: np.ndarray          # uint8 [H, W, 3], texture of the new frame
    truth: dict = field(default_factory=dict)

    def truth_map(self, pts: np.ndarray) -> np.ndarray:
        """Ground-truth motion G(x) (float64) at points [M, 2]."""
        t = self.truth
        c = np.array(t["centre"])
        ct, st = np.cos(t["theta"]), np.sin(t["theta"])
        d = pts - c
        out = np.stack([ct * d[:, 0] - st * d[:, 1], st * d[:, 0] + ct * d[:, 1]], 1)
        out = c + t["scale"] * out + np.array(t["shift"])
        for (bx, by, ux, uy) in t["bumps"]:
            r2 = (pts[:, 0] - bx) ** 2 + (pts[:, 1] - by) ** 2
            g = t["bump_amp"] * np.exp(-r2 / (2.0 * t["bump_sigma"] ** 2))
            out[:, 0] += g * ux
            out[:, 1] += g * uy
        return out


def gen_pair(cfg: PairConfig, seed: int, with_frame: bool = True) -> Pair:
    """Draw one pair.  Fixed draw order:

    1. src ~ U([0, W-1] x [0, H-1])
    2. global similarity about the frame centre: angle, scale, shift
    3. bumps: centre ~ U(frame), direction ~ U(0, 2 pi)
    4. dst = G(src) + N(0, noise^2) per axis
    5. round(rate * N) outlier indices (no replacement) get dst ~ U(frame)
    6. texture of the new frame
    """
    rng = np.random.default_rng(seed)
    W, H, N = cfg.width, cfg.height, cfg.n_matches
    src = np.stack([rng.uniform(0.0, W - 1.0, N), rng.uniform(0.0, H - 1.0, N)], 1)
    theta = np.deg2rad(rng.uniform(-cfg.rot_deg, cfg.rot_deg))
    scale = rng.uniform(cfg.scale_lo, cfg.scale_hi)
    shift = rng.uniform(-cfg.shift_px, cfg.shift_px, 2)
    bumps = []
    for _ in range(cfg.n_bumps):
        bx = rng.uniform(0.0, W - 1.0)
        by = rng.uniform(0.0, H - 1.0)
        phi = rng.uniform(0.0, 2.0 * np.pi)
        bumps.append((float(bx), float(by), float(np.cos(phi)), float(np.sin(phi))))
    truth = dict(centre=((W - 1) / 2.0, (H - 1) / 2.0), theta=float(theta),
                 scale=float(scale), shift=(float(shift[0]), float(shift[1])),
                 bumps=bumps, bump_amp=cfg.bump_amp, bump_sigma=cfg.bump_sigma)
    pair = Pair(cfg, seed, src.astype(np.float32), None, None, None, truth)
    dst = pair.truth_map(src) + rng.normal(0.0, cfg.noise_px, (N, 2))
    n_out = int(round(cfg.outlier_rate * N))
    inlier = np.ones(N, dtype=bool)
    if n_out > 0:
        idx = rng.choice(N, size=n_out, replace=False)
        inlier[idx] = False
        dst[idx, 0] = rng.uniform(0.0, W - 1.0, n_out)
        dst[idx, 1] = rng.uniform(0.0, H - 1.0, n_out)
    pair.dst = dst.astype(np.float32)
    pair.inlier = inlier
    if with_frame:
        pair.frame = gen_texture(W, H, rng, cfg.texture_sigma)
    return pair


def gen_config(config: int, pair: int, with_frame: bool = True) -> Pair:
    """Pair `pair` of named workload `config` (seed = 1000 * config + pair)."""
    return gen_pair(CONFIGS[config], config_seed(config, pair), with_frame)


def similarity_matches(n: int, width: int, height: int, theta: float, scale: float,
                       shift, seed: int, centre=None):
    """Matches drawn from one exact similarity y = c + scale R (x - c) + shift
    (float32, no noise, no outliers); used for invariance checks."""
    rng = np.random.default_rng(seed)
    src = np.stack([rng.uniform(0.0, width - 1.0, n),
                    rng.uniform(0.0, height - 1.0, n)], 1).astype(np.float32)
    c = np.array(centre if centre is not None else ((width - 1) / 2.0, (height - 1) / 2.0))
    d = src.astype(np.float64) - c
    ct, st = np.cos(theta), np.sin(theta)
    dst = c + scale * np.stack([ct * d[:, 0] - st * d[:, 1], st * d[:, 0] + ct * d[:, 1]], 1)
    dst = dst + np.asarray(shift, dtype=np.float64)
    return src, dst.astype(np.float32)


# Mixed batch of independent pairs: frame size drawn from these, N ~ U[300, 3000],
# outlier rate ~ U(0.10, 0.40), 8 bumps of 15 px and sigma 80 px.
BATCH_FRAMES = ((640, 480), (1280, 1024), (1920, 1080))


def gen_batch(n_pairs: int = 64, seed: int = 3000, with_frame: bool = True):
    """A batch of `n_pairs` pairs of uneven size.  The shapes are drawn first
    from `seed` (frame index, N, outlier rate per pair, in that order); pair i
    is then drawn by gen_pair with seed 1000 * seed + i."""
    rng = np.random.default_rng(seed)
    pairs = []
    for i in range(n_pairs):
        w, h = BATCH_FRAMES[int(rng.integers(0, len(BATCH_FRAMES)))]
        n = int(rng.integers(300, 3001))
        rate = float(rng.uniform(0.10, 0.40))
        cfg = PairConfig(w, h, n, rate, 8, 15.0, 80.0, w, h)
        pairs.append(gen_pair(cfg, 1000 * seed + i, with_frame))
    return pairs
