"""The learned start's 16-nearest-neighbour search on point layouts that stress
a grid search: clusters with far outliers (most points in a few cells), exact
duplicates and integer lattices (many equal distances, decided by the match
index), collinear and identical points (a degenerate bounding box), sets with
fewer than 16 other matches, a large coordinate offset, and the largest pair
the grid takes next to the smallest one scanned pair by pair.  The features
are compared with the FP64 oracle's (neighbours chosen in FP64 on both sides,
ties by index), so a wrong or reordered neighbour shows as an error of the
size of a coordinate difference."""
import numpy as np
import pytest

import oracle as O

from gpu_util import check_start, emdq, oracle_start, to_dev, torch_or_skip

pytestmark = pytest.mark.gpu
W, H = 1280, 1024


def _layout(kind, n, rng):
    if kind == "uniform":
        return rng.uniform([0, 0], [W, H], (n, 2))
    if kind == "clusters":   # three tight clusters and a few far points
        c = rng.uniform([0, 0], [W, H], (3, 2))
        p = c[rng.integers(0, 3, n)] + rng.normal(0, 2.0, (n, 2))
        p[:5] = rng.uniform([-4000, -4000], [8000, 8000], (5, 2))
        return p
    if kind == "duplicates":   # every point four times
        p = rng.uniform([0, 0], [W, H], ((n + 3) // 4, 2))
        return np.repeat(p, 4, axis=0)[:n]
    if kind == "lattice":   # integer lattice, shuffled
        s = int(np.ceil(np.sqrt(n)))
        g = np.stack(np.meshgrid(np.arange(s), np.arange(s)), -1).reshape(-1, 2)[:n] * 8.0
        return g[rng.permutation(n)]
    if kind == "collinear":
        x = rng.uniform(0, W, n)
        return np.stack([x, np.full(n, 300.0)], 1)
    if kind == "identical":
        return np.tile([[640.0, 512.0]], (n, 1))
    if kind == "offset":   # far from the origin: rounding of the cell assignment
        return rng.uniform([0, 0], [W, H], (n, 2)) + 1.0e5
    raise ValueError(kind)


CASES = [("uniform", 2), ("uniform", 5), ("uniform", 17), ("uniform", 2000),
         ("clusters", 3000), ("duplicates", 1999), ("lattice", 1024), ("lattice", 7168),
         ("collinear", 700), ("identical", 40), ("offset", 1500),
         ("uniform", 5000), ("uniform", 7168), ("uniform", 7169)]


@pytest.mark.parametrize("kind,n", CASES)
def test_start_features_layouts(kind, n):
    torch = torch_or_skip()
    E = emdq()
    rng = np.random.default_rng([n, ord(kind[0]), len(kind)])
    src = _layout(kind, n, rng).astype(np.float32)
    dst = (src + rng.normal(0, 6.0, (n, 2))).astype(np.float32)
    print(f"start features {kind} n={n}", flush=True)
    out = torch.empty((n, 64), dtype=torch.float32, device="cuda")
    E.emdq_start_features(to_dev(src, torch), to_dev(dst, torch), W, H, out)
    want = O.init_features(src, dst, O.alpha(W, H))
    err = np.abs(out.cpu().numpy() - want).max()
    print(f"  max abs err {err:.2e}", flush=True)
    assert err <= 1e-5


@pytest.mark.parametrize("kind,n", [("clusters", 3000), ("lattice", 7168), ("uniform", 7169)])
def test_learned_start_layouts(kind, n):
    """The whole start (features and network) on the same layouts."""
    torch = torch_or_skip()
    E = emdq()
    rng = np.random.default_rng(7 + n)
    src = _layout(kind, n, rng).astype(np.float32)
    dst = (src + rng.normal(0, 6.0, (n, 2))).astype(np.float32)
    print(f"learned start {kind} n={n}", flush=True)
    out = torch.empty(n, dtype=torch.float32, device="cuda")
    E.emdq_learned_start(to_dev(src, torch), to_dev(dst, torch), W, H, E.load_start_weights(), out)
    wo = np.load(E.START_WEIGHTS, allow_pickle=False).astype(np.float64)
    check_start(out.cpu().numpy(), oracle_start(src, dst, W, H, wo), f"{kind} n={n}")
