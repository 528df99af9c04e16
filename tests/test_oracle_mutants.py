"""The oracle's pins catch plausible mistakes.

Each case plants one mistake in a copy of oracle/emdq_oracle.c (a dropped
term, a wrong sign or index, a transposed operand), builds it on the CPU and
runs the pin suite against it; the suite must fail."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "emdq_oracle.c")

MUTANTS = [
    ("transposed cross-covariance", "double num = C10 - C01,", "double num = C01 - C10,"),
    ("inverted scale ratio", "double s = sqrt(Vy / Vx);", "double s = sqrt(Vx / Vy);"),
    ("wrong sign in the translation", "double tx = my0 / s - (ct * mx0 - st * mx1);",
     "double tx = my0 / s - (ct * mx0 + st * mx1);"),
    ("scale not divided out of the translation", "double ty = my1 / s - (st * mx0 + ct * mx1);",
     "double ty = my1 - (st * mx0 + ct * mx1);"),
    ("wrong sign in the DQ dual part", "q[2] = 0.5 * (c * tx + s * ty);",
     "q[2] = 0.5 * (c * tx - s * ty);"),
    ("wrong sign in the DQ decode", "*ty = 2.0 * (s * dx + c * dy);",
     "*ty = 2.0 * (s * dx - c * dy);"),
    ("half angle dropped", "double c = cos(theta / 2.0), s = sin(theta / 2.0);",
     "double c = cos(theta), s = sin(theta);"),
    ("posterior weight dropped in the M-step",
     "w[j] = exp(-alpha * (dx * dx + dy * dy)) * p[j];",
     "w[j] = exp(-alpha * (dx * dx + dy * dy));"),
    ("Gaussian weight dropped in the M-step",
     "w[j] = exp(-alpha * (dx * dx + dy * dy)) * p[j];", "w[j] = p[j];"),
    ("blended scale not normalised", "sb /= W;                                    /* Eq. (2) */",
     ""),
    ("inlier mask ignored in the field", "for (int j = 0; j < n; ++j) wt[j] = mask[j] ? 1.0 : 0.0;\n#pragma omp parallel for schedule(dynamic, 1) reduction(| : bad)\n    for (int k = 0; k < h; ++k)\n        for (int i = 0; i < w; ++i) {\n            double *o",
     "for (int j = 0; j < n; ++j) wt[j] = 1.0;\n#pragma omp parallel for schedule(dynamic, 1) reduction(| : bad)\n    for (int k = 0; k < h; ++k)\n        for (int i = 0; i < w; ++i) {\n            double *o"),
    ("per-axis variance factor dropped", "double sigma2 = spe / (2.0 * sp);",
     "double sigma2 = spe / sp;"),
    ("Gaussian normaliser dropped", "double L = exp(-e2[i] / (2.0 * sigma2)) / (2.0 * pi * sigma2);",
     "double L = exp(-e2[i] / (2.0 * sigma2));"),
    ("inlier fraction not clamped", "if (gamma > prm->gamma_max) gamma = prm->gamma_max;", ""),
    ("stop rule without the second iteration", "if (k >= 2 && !changed) { converged = 1; break; }",
     "if (!changed) { converged = 1; break; }"),
    ("bilinear corner weights swapped", "rgb[c] = (1.0 - a) * (1.0 - b) * i00 + a * (1.0 - b) * i01",
     "rgb[c] = (1.0 - a) * (1.0 - b) * i00 + a * (1.0 - b) * i10"),
    ("merge count not capped", "px[3] = A + 1.0 < 30.0 ? A + 1.0 : 30.0;", "px[3] = A + 1.0;"),
    ("merge not a running average", "px[c] = (A * px[c] + v[c]) / (A + 1.0);",
     "px[c] = A * px[c] + v[c];"),
    ("resolution scale not averaged", "double s = ((double)w / ref_w + (double)h / ref_h) / 2.0;",
     "double s = ((double)w / ref_w + (double)h / ref_h);"),
    ("residual sign", "double ex = y[2 * i] - fx, ey = y[2 * i + 1] - fy;",
     "double ex = y[2 * i] + fx, ey = y[2 * i + 1] - fy;"),
    ("E-step blend weighted by p squared",
     "double w = exp(-alpha * (dx * dx + dy * dy)) * wt[j];",
     "double w = exp(-alpha * (dx * dx + dy * dy)) * wt[j] * wt[j];"),
    ("E-step blend with twice alpha",
     "if (oracle_blend_at(n, x, scale, q, p, alpha, x[2 * i], x[2 * i + 1], &fx, &fy) != 0) {",
     "if (oracle_blend_at(n, x, scale, q, p, 2.0 * alpha, x[2 * i], x[2 * i + 1], &fx, &fy) != 0) {"),
    ("E-step called with twice alpha in the EM loop",
     "oracle_estep(n, x, y, p, scale, q, alpha, e2);",
     "oracle_estep(n, x, y, p, scale, q, 2.0 * alpha, e2);"),
    ("final M-step with the final p dropped",
     "oracle_mstep(n, x, y, p, alpha, scale, q);   /* fit with the final p */", ""),
    ("displacement feature scale 4 instead of 8",
     "double ex = (y[2 * j] - x[2 * j] - dix) / 8.0,",
     "double ex = (y[2 * j] - x[2 * j] - dix) / 4.0,"),
    ("displacement feature sign flipped",
     "double ex = (y[2 * j] - x[2 * j] - dix) / 8.0,",
     "double ex = (dix - (y[2 * j] - x[2 * j])) / 8.0,"),
    ("displacement feature x and y swapped",
     "f[4 * r + 2] = ex / (1.0 + fabs(ex));\n            f[4 * r + 3] = ey / (1.0 + fabs(ey));",
     "f[4 * r + 2] = ey / (1.0 + fabs(ey));\n            f[4 * r + 3] = ex / (1.0 + fabs(ex));"),
    ("bfloat16 ties rounded away from zero", "return ldexp(rint(m * 256.0), e - 8);",
     "return ldexp(round(m * 256.0), e - 8);"),
    ("bfloat16 significand one bit short", "return ldexp(rint(m * 256.0), e - 8);",
     "return ldexp(rint(m * 128.0), e - 7);"),
    ("first hidden layer of the BF16 network not rounded", "h1[o] = oracle_bf16(gelu(a));",
     "h1[o] = gelu(a);"),
    ("second weight matrix of the BF16 network not rounded",
     "for (int k = 0; k < OR_NH; ++k) a += oracle_bf16(W2[o * OR_NH + k]) * h1[k];",
     "for (int k = 0; k < OR_NH; ++k) a += W2[o * OR_NH + k] * h1[k];"),
]


@pytest.mark.slow
@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_planted_mistake(name, old, new, tmp_path):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site not unique or missing: {name}"
    mutant = tmp_path / "emdq_oracle_mutant.c"
    mutant.write_text(src.replace(old, new))
    lib = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-std=gnu11", "-O1", "-fopenmp", "-fPIC", "-shared", "-o", str(lib),
                    str(mutant), "-lm"], check=True)
    env = dict(os.environ, ORACLE_LIB=str(lib), OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"no pin caught the planted mistake: {name}"
