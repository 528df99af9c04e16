/*
 * emdq_oracle.c -- plain, slow, FP64 CPU oracle of the EMDQ field + warp path.
 *
 * TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  The GPU library
 * shares no code, header, table or helper with it, and never calls it.
 *
 * Source: H. Zhou and J. Jayender, "Real-time Nonrigid Mosaicking of
 * Laparoscopy Images" (arXiv 2103.07414).
 *   Eq. (1)       node warp x_t = s (R x_0 + t), written as a scale and a
 *                 dual quaternion (DQ); footnote to Eq. (1): the image lies on
 *                 the z = 0 plane, so only 4 of the 8 DQ components are kept.
 *   Eqs. (2)-(3)  per-pixel scale and DQ = weighted means of the node ones.
 *   Eq. (4)       weight w = exp(-alpha |x_i,0 - x_p,0|^2).
 *   Eqs. (18)-(20) weighted similarity fit: SVD rotation, norm-ratio scale,
 *                 weighted-average translation (Sec. III-E).
 *   Sec. III-F    dense mosaicking of every pixel; Eqs. (23)-(24) TSDF-like
 *                 colour merge with a weight cap of 30.
 *   Sec. III-G    alpha = 2e-4 scaled by 1/s^2, s = (w/480 + h/270)/2.
 *   Sec. II-A     EMDQ: mismatch removal by expectation maximisation plus a
 *                 smooth DQ field interpolated among the inliers.
 *   Eq. (8)       uncertainty of the field: exp(beta d^2) to the nearest inlier.
 *   App. A        update of a node's warp function by a new (scale, DQ) that
 *                 is expressed in the current frame.
 *
 * The paper treats EMDQ as a black box and gives its inner rules elsewhere,
 * so the EM part follows this reading (it is the contract the GPU library is
 * held to):
 *   * every match i carries a similarity fitted to all matches j with weights
 *     w_ij = K_ij p_j, K_ij = exp(-alpha |x_i - x_j|^2) (Eq. (4) applied match
 *     to match, as Sec. III-E applies it node to node);
 *   * the fit centres on the weighted centroids, uses the det-corrected 2x2
 *     Procrustes rotation, the norm-ratio scale and the Eq. (20) translation;
 *   * E-step: blend the fits at each match (Eqs. (2)-(3)), normalise the DQ by
 *     the norm of its real part (dual-quaternion linear blending), predict
 *     y_i, and take the residual e_i; sigma^2 and the inlier fraction gamma are
 *     p-weighted estimates; p_i is the posterior of a Gaussian-inlier /
 *     uniform-outlier mixture over the new frame;
 *   * mask_i = (p_i > 0.5), the decision taken on p rounded to FP32; stop when
 *     the mask did not change (from the second iteration on) or at max_iter;
 *     then one more fit with the final p;
 *   * the dense field blends only the inliers (hard mask).
 *
 * Conventions: pixel coordinates (x = column, y = row), pixel centres at
 * integers, origin at the centre of the top-left pixel.  Planar DQ of a
 * rotation by theta about z and a translation t in the image plane:
 *   q = (cos(theta/2), sin(theta/2),
 *        (cos(theta/2) t_x + sin(theta/2) t_y) / 2,
 *        (cos(theta/2) t_y - sin(theta/2) t_x) / 2),
 * i.e. the w and z components of the real part and the x and y components of
 * the dual part of r + eps (1/2) t r.
 *
 * Status codes: 0 ok, 1 EM stopped at max_iter (results valid), -1 invalid
 * argument, -2 fewer than 2 matches, -3 no inliers, -4 non-finite input.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_WARN_NOT_CONVERGED 1
#define OR_EINVAL (-1)
#define OR_ETOOFEW (-2)
#define OR_ENOINLIERS (-3)
#define OR_ENONFINITE (-4)

typedef struct {
    double alpha0;      /* Eq. (4) coefficient at the reference resolution */
    int ref_w, ref_h;   /* reference resolution of Sec. III-G */
    int max_iter;       /* EM iteration cap */
    double p_thresh;    /* inlier threshold on the posterior */
    double gamma_min, gamma_max;  /* clamp of the inlier fraction */
    double sigma2_min;  /* floor of the inlier variance, px^2 */
} oracle_params;

void oracle_params_default(oracle_params *p)
{
    p->alpha0 = 2e-4;
    p->ref_w = 480;
    p->ref_h = 270;
    p->max_iter = 50;
    p->p_thresh = 0.5;
    p->gamma_min = 0.05;
    p->gamma_max = 0.95;
    p->sigma2_min = 1e-2;
}

/* Sec. III-G: alpha multiplied by 1/s^2, s = (w/480 + h/270)/2. */
double oracle_alpha(double alpha0, int ref_w, int ref_h, int w, int h)
{
    double s = ((double)w / ref_w + (double)h / ref_h) / 2.0;
    return alpha0 / (s * s);
}

/* ---------------------------------------------------------------- DQs --- */

/* Planar DQ of the rigid motion (rotation theta, translation t). */
void oracle_dq_from_rt(double theta, double tx, double ty, double q[4])
{
    double c = cos(theta / 2.0), s = sin(theta / 2.0);
    q[0] = c;
    q[1] = s;
    q[2] = 0.5 * (c * tx + s * ty);
    q[3] = 0.5 * (c * ty - s * tx);
}

/* Rotation (cos, sin) and translation of a planar DQ, after dividing it by
 * the norm of its real part.  Returns 0, or -1 if the real part is zero. */
int oracle_dq_decode(const double q[4], double *cos_t, double *sin_t,
                     double *tx, double *ty)
{
    double n = sqrt(q[0] * q[0] + q[1] * q[1]);
    if (!(n > 0.0)) return -1;
    double c = q[0] / n, s = q[1] / n, dx = q[2] / n, dy = q[3] / n;
    *cos_t = c * c - s * s;
    *sin_t = 2.0 * c * s;
    *tx = 2.0 * (c * dx - s * dy);
    *ty = 2.0 * (s * dx + c * dy);
    return 0;
}

/* Eq. (1): x_t = s (R x_0 + t) with R, t decoded from q. */
int oracle_warp_point(double scale, const double q[4], double x, double y,
                      double *ox, double *oy)
{
    double ct, st, tx, ty;
    if (oracle_dq_decode(q, &ct, &st, &tx, &ty) != 0) return -1;
    *ox = scale * (ct * x - st * y + tx);
    *oy = scale * (st * x + ct * y + ty);
    return 0;
}

/* -------------------------------------------------- weighted fit, M-step */

/* Weighted similarity fit of pairs (x_j -> y_j), Eqs. (18)-(20) with linear
 * weights and centroid centring.  Outputs the scale and the planar DQ.
 * Returns 0 for a regular fit, 1 when the degenerate rule was applied. */
int oracle_weighted_fit(int n, const double *x, const double *y, const double *w,
                        double *scale, double q[4])
{
    double S = 0.0, mx0 = 0.0, mx1 = 0.0, my0 = 0.0, my1 = 0.0;
    for (int j = 0; j < n; ++j) {
        S += w[j];
        mx0 += w[j] * x[2 * j];
        mx1 += w[j] * x[2 * j + 1];
        my0 += w[j] * y[2 * j];
        my1 += w[j] * y[2 * j + 1];
    }
    if (!(S > 0.0)) {               /* no weight at all: identity */
        *scale = 1.0;
        oracle_dq_from_rt(0.0, 0.0, 0.0, q);
        return 1;
    }
    mx0 /= S; mx1 /= S; my0 /= S; my1 /= S;
    /* second pass: centred cross-covariance C = sum w (y - ybar)(x - xbar)^T
     * and the centred spreads Vx, Vy */
    double C00 = 0.0, C01 = 0.0, C10 = 0.0, C11 = 0.0, Vx = 0.0, Vy = 0.0;
    for (int j = 0; j < n; ++j) {
        double ax = x[2 * j] - mx0, ay = x[2 * j + 1] - mx1;
        double bx = y[2 * j] - my0, by = y[2 * j + 1] - my1;
        C00 += w[j] * bx * ax;
        C01 += w[j] * bx * ay;
        C10 += w[j] * by * ax;
        C11 += w[j] * by * ay;
        Vx += w[j] * (ax * ax + ay * ay);
        Vy += w[j] * (bx * bx + by * by);
    }
    if (Vx <= 1e-12 * S || Vy <= 1e-12 * S) {
        /* all weighted sources (or targets) coincide: translation only */
        *scale = 1.0;
        oracle_dq_from_rt(0.0, my0 - mx0, my1 - mx1, q);
        return 1;
    }
    /* Eq. (18): R = U V^T of svd(C) with det(R) = +1.  For a 2x2 C the
     * maximiser of tr(R^T C) over rotations is theta = atan2(C10 - C01,
     * C00 + C11). */
    double num = C10 - C01, den = C00 + C11;
    double theta = (num == 0.0 && den == 0.0) ? 0.0 : atan2(num, den);
    /* Eq. (19): ratio of the weighted norms of the centred point sets. */
    double s = sqrt(Vy / Vx);
    /* Eq. (20): t = weighted average of (y / s - R x) = ybar / s - R xbar. */
    double ct = cos(theta), st = sin(theta);
    double tx = my0 / s - (ct * mx0 - st * mx1);
    double ty = my1 / s - (st * mx0 + ct * mx1);
    *scale = s;
    oracle_dq_from_rt(theta, tx, ty, q);
    return 0;
}

/* M-step: fit a similarity at every match i with weights K_ij p_j.
 * x, y: [n][2]; p: [n]; outputs scale[n], q[n][4]. */
void oracle_mstep(int n, const double *x, const double *y, const double *p,
                  double alpha, double *scale, double *q)
{
#pragma omp parallel
    {
        double *w = (double *)malloc(sizeof(double) * (size_t)n);
#pragma omp for schedule(static)
        for (int i = 0; i < n; ++i) {
            for (int j = 0; j < n; ++j) {
                double dx = x[2 * j] - x[2 * i], dy = x[2 * j + 1] - x[2 * i + 1];
                w[j] = exp(-alpha * (dx * dx + dy * dy)) * p[j];   /* Eq. (4) */
            }
            oracle_weighted_fit(n, x, y, w, &scale[i], &q[4 * i]);
        }
        free(w);
    }
}

/* ------------------------------------------------------------ blending --- */

/* Eqs. (2)-(4) at point z: weights w_j = exp(-alpha |z - x_j|^2) wt_j, blended
 * scale and DQ (weighted means), then Eq. (1).  Returns 0, or -1 when all
 * weights vanish. */
int oracle_blend_at(int n, const double *x, const double *scale, const double *q,
                    const double *wt, double alpha, double zx, double zy,
                    double *fx, double *fy)
{
    double W = 0.0, sb = 0.0, qb[4] = {0.0, 0.0, 0.0, 0.0};
    for (int j = 0; j < n; ++j) {
        if (wt[j] == 0.0) continue;
        double dx = zx - x[2 * j], dy = zy - x[2 * j + 1];
        double w = exp(-alpha * (dx * dx + dy * dy)) * wt[j];
        W += w;
        sb += w * scale[j];
        for (int c = 0; c < 4; ++c) qb[c] += w * q[4 * j + c];
    }
    if (!(W > 0.0)) return -1;
    sb /= W;                                    /* Eq. (2) */
    for (int c = 0; c < 4; ++c) qb[c] /= W;     /* Eq. (3) */
    return oracle_warp_point(sb, qb, zx, zy, fx, fy);   /* normalise + Eq. (1) */
}

/* E-step residuals: e2[i] = |y_i - F_i(x_i)|^2 where F_i blends all fits
 * with weights K_ij p_j.  A match with no weight gets +inf. */
void oracle_estep(int n, const double *x, const double *y, const double *p,
                  const double *scale, const double *q, double alpha, double *e2)
{
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) {
        double fx, fy;
        if (oracle_blend_at(n, x, scale, q, p, alpha, x[2 * i], x[2 * i + 1], &fx, &fy) != 0) {
            e2[i] = INFINITY;
            continue;
        }
        double ex = y[2 * i] - fx, ey = y[2 * i + 1] - fy;
        e2[i] = ex * ex + ey * ey;
    }
}

/* Posterior of the Gaussian-inlier / uniform-outlier mixture.
 * sigma2, gamma from the current p; returns the new p in p_out. */
void oracle_posterior(int n, const double *e2, const double *p, double u,
                      const oracle_params *prm, double *p_out,
                      double *sigma2_out, double *gamma_out)
{
    double sp = 0.0, spe = 0.0;
    for (int i = 0; i < n; ++i) {        /* fixed order */
        sp += p[i];
        if (p[i] > 0.0) spe += p[i] * e2[i];
    }
    double sigma2 = spe / (2.0 * sp);
    if (!(sigma2 >= prm->sigma2_min)) sigma2 = prm->sigma2_min;
    double gamma = sp / n;
    if (gamma < prm->gamma_min) gamma = prm->gamma_min;
    if (gamma > prm->gamma_max) gamma = prm->gamma_max;
    const double pi = 3.14159265358979323846;
    for (int i = 0; i < n; ++i) {
        double L = exp(-e2[i] / (2.0 * sigma2)) / (2.0 * pi * sigma2);
        double a = gamma * L, b = (1.0 - gamma) * u;
        p_out[i] = a / (a + b);
    }
    *sigma2_out = sigma2;
    *gamma_out = gamma;
}

static int all_finite(int n, const double *v)
{
    for (int i = 0; i < n; ++i)
        if (!isfinite(v[i])) return 0;
    return 1;
}

/* Full EM fit.  x = src (reference side), y = dst (new frame), [n][2].
 * Outputs scale[n], q[n][4], p[n], mask[n]; iters, sigma2, gamma (nullable).
 * frame_w, frame_h: size of the new frame (uniform outlier density 1/(w h)
 * and the Sec. III-G alpha scaling). */
int oracle_fit_init(int n, const double *x, const double *y, int frame_w, int frame_h,
                    const oracle_params *prm_in, const double *init_p, double *scale,
                    double *q, double *p, uint8_t *mask, int *iters, double *sigma2_out,
                    double *gamma_out);

int oracle_fit(int n, const double *x, const double *y, int frame_w, int frame_h,
               const oracle_params *prm_in, double *scale, double *q, double *p,
               uint8_t *mask, int *iters, double *sigma2_out, double *gamma_out)
{
    return oracle_fit_init(n, x, y, frame_w, frame_h, prm_in, NULL, scale, q, p, mask, iters,
                           sigma2_out, gamma_out);
}

/* EM fit starting from the posteriors init_p (null: p = 1, the plain start).
 * The starting mask is init_p > p_thresh, decided in FP32 as every later
 * mask. */
int oracle_fit_init(int n, const double *x, const double *y, int frame_w, int frame_h,
                    const oracle_params *prm_in, const double *init_p, double *scale,
                    double *q, double *p, uint8_t *mask, int *iters, double *sigma2_out,
                    double *gamma_out)
{
    oracle_params prm;
    if (prm_in) prm = *prm_in; else oracle_params_default(&prm);
    if (!x || !y || !scale || !q || !p || !mask) return OR_EINVAL;
    if (frame_w <= 0 || frame_h <= 0 || prm.max_iter < 1) return OR_EINVAL;
    if (n < 2) return OR_ETOOFEW;
    if (!all_finite(2 * n, x) || !all_finite(2 * n, y)) return OR_ENONFINITE;

    double alpha = oracle_alpha(prm.alpha0, prm.ref_w, prm.ref_h, frame_w, frame_h);
    double u = 1.0 / ((double)frame_w * (double)frame_h);
    double *e2 = (double *)malloc(sizeof(double) * (size_t)n);
    double *pn = (double *)malloc(sizeof(double) * (size_t)n);
    uint8_t *prev = (uint8_t *)malloc((size_t)n);
    for (int i = 0; i < n; ++i) {
        p[i] = init_p ? init_p[i] : 1.0;
        mask[i] = ((float)p[i] > (float)prm.p_thresh) ? 1 : 0;
    }
    if (init_p && !all_finite(n, init_p)) {   /* a non-finite input, like a coordinate */
        free(e2);
        free(pn);
        free(prev);
        return OR_ENONFINITE;
    }
    int k = 0, converged = 0, status = OR_OK;
    double sigma2 = 0.0, gamma = 0.0;
    while (1) {
        oracle_mstep(n, x, y, p, alpha, scale, q);
        oracle_estep(n, x, y, p, scale, q, alpha, e2);
        double sp = 0.0;
        for (int i = 0; i < n; ++i) sp += p[i];
        if (!(sp > 0.0)) { status = OR_ENOINLIERS; break; }
        oracle_posterior(n, e2, p, u, &prm, pn, &sigma2, &gamma);
        memcpy(prev, mask, (size_t)n);
        int changed = 0;
        for (int i = 0; i < n; ++i) {
            p[i] = pn[i];
            /* the threshold decision is taken on p rounded to FP32 */
            mask[i] = ((float)p[i] > (float)prm.p_thresh) ? 1 : 0;
            changed |= (mask[i] != prev[i]);
        }
        k += 1;
        if (k >= 2 && !changed) { converged = 1; break; }
        if (k >= prm.max_iter) break;
    }
    if (status == OR_OK) {
        oracle_mstep(n, x, y, p, alpha, scale, q);   /* fit with the final p */
        int n_in = 0;
        for (int i = 0; i < n; ++i) n_in += mask[i];
        if (n_in == 0) status = OR_ENOINLIERS;
        else if (!converged) status = OR_WARN_NOT_CONVERGED;
    }
    if (iters) *iters = k;
    if (sigma2_out) *sigma2_out = sigma2;
    if (gamma_out) *gamma_out = gamma;
    free(e2);
    free(pn);
    free(prev);
    return status;
}

/* ------------------------------------------------------- field and warp --- */

/* Dense field at the grid points (zx0 + i, zy0 + k), i < w, k < h, blending
 * the masked fits (Sec. II-A: interpolation among the inliers).
 * out: [h][w][2].  Returns 0 or -3 if some point has no weight. */
int oracle_field(int n, const double *x, const double *scale, const double *q,
                 const uint8_t *mask, double alpha, int zx0, int zy0, int w, int h,
                 double *out)
{
    double *wt = (double *)malloc(sizeof(double) * (size_t)n);
    int bad = 0;
    for (int j = 0; j < n; ++j) wt[j] = mask[j] ? 1.0 : 0.0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : bad)
    for (int k = 0; k < h; ++k)
        for (int i = 0; i < w; ++i) {
            double *o = out + 2 * ((size_t)k * w + i);
            if (oracle_blend_at(n, x, scale, q, wt, alpha, zx0 + i, zy0 + k, &o[0], &o[1]) != 0) {
                o[0] = o[1] = NAN;
                bad = 1;
            }
        }
    free(wt);
    return bad ? OR_ENOINLIERS : OR_OK;
}

/* Field at arbitrary points pts[m][2] -> out[m][2]. */
int oracle_field_points(int n, const double *x, const double *scale, const double *q,
                        const uint8_t *mask, double alpha, int m, const double *pts,
                        double *out)
{
    double *wt = (double *)malloc(sizeof(double) * (size_t)n);
    int bad = 0;
    for (int j = 0; j < n; ++j) wt[j] = mask[j] ? 1.0 : 0.0;
#pragma omp parallel for schedule(dynamic, 64) reduction(| : bad)
    for (int i = 0; i < m; ++i) {
        if (oracle_blend_at(n, x, scale, q, wt, alpha, pts[2 * i], pts[2 * i + 1],
                            &out[2 * i], &out[2 * i + 1]) != 0) {
            out[2 * i] = out[2 * i + 1] = NAN;
            bad = 1;
        }
    }
    free(wt);
    return bad ? OR_ENOINLIERS : OR_OK;
}

/* Bilinear sample of an RGB uint8 frame at (ux, uy).  Valid iff the point
 * lies in [0, fw-1] x [0, fh-1]; returns 0 and the three channels, or -1. */
int oracle_bilinear(const uint8_t *frame, int fw, int fh, int pitch,
                    double ux, double uy, double rgb[3])
{
    if (!(ux >= 0.0 && ux <= fw - 1.0 && uy >= 0.0 && uy <= fh - 1.0)) return -1;
    int x0 = (int)floor(ux), y0 = (int)floor(uy);
    int x1 = x0 + 1 < fw ? x0 + 1 : fw - 1;
    int y1 = y0 + 1 < fh ? y0 + 1 : fh - 1;
    double a = ux - x0, b = uy - y0;
    for (int c = 0; c < 3; ++c) {
        double i00 = frame[(size_t)y0 * pitch + 3 * x0 + c];
        double i01 = frame[(size_t)y0 * pitch + 3 * x1 + c];
        double i10 = frame[(size_t)y1 * pitch + 3 * x0 + c];
        double i11 = frame[(size_t)y1 * pitch + 3 * x1 + c];
        rgb[c] = (1.0 - a) * (1.0 - b) * i00 + a * (1.0 - b) * i01
               + (1.0 - a) * b * i10 + a * b * i11;
    }
    return 0;
}

/* Eqs. (23)-(24) as a running average with a capped count:
 * rgb <- (A rgb + v) / (A + 1), A <- min(A + 1, 30). */
void oracle_merge(double px[4], const double v[3])
{
    double A = px[3];
    for (int c = 0; c < 3; ++c) px[c] = (A * px[c] + v[c]) / (A + 1.0);
    px[3] = A + 1.0 < 30.0 ? A + 1.0 : 30.0;
}

/* Warp + merge: for every src grid point z = (zx0 + i, zy0 + k) (i < w,
 * k < h), u = F(z) is sampled in the new frame and merged into the canvas
 * pixel z + (ox, oy).  canvas: RGBA [ch][pitch_px][4] in double, updated in
 * place.  valid_out (nullable): [h][w] 1 where the sample was inside the
 * frame.  Returns 0, -1 on a bad rectangle, -3 if no inliers. */
int oracle_warp(int n, const double *x, const double *scale, const double *q,
                const uint8_t *mask, double alpha, const uint8_t *frame, int fw,
                int fh, int frame_pitch, double *canvas, int cw, int ch,
                int canvas_pitch_px, int ox, int oy, int zx0, int zy0, int w, int h,
                uint8_t *valid_out)
{
    if (zx0 + ox < 0 || zy0 + oy < 0 || zx0 + ox + w > cw || zy0 + oy + h > ch)
        return OR_EINVAL;
    double *wt = (double *)malloc(sizeof(double) * (size_t)n);
    int bad = 0;
    for (int j = 0; j < n; ++j) wt[j] = mask[j] ? 1.0 : 0.0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : bad)
    for (int k = 0; k < h; ++k)
        for (int i = 0; i < w; ++i) {
            double ux, uy, v[3];
            int valid = 0;
            if (oracle_blend_at(n, x, scale, q, wt, alpha, zx0 + i, zy0 + k, &ux, &uy) != 0)
                bad = 1;
            else if (oracle_bilinear(frame, fw, fh, frame_pitch, ux, uy, v) == 0) {
                size_t cy = (size_t)(zy0 + k + oy), cx = (size_t)(zx0 + i + ox);
                oracle_merge(canvas + 4 * (cy * canvas_pitch_px + cx), v);
                valid = 1;
            }
            if (valid_out) valid_out[(size_t)k * w + i] = (uint8_t)valid;
        }
    free(wt);
    return bad ? OR_ENOINLIERS : OR_OK;
}

/* ------------------------------------------- App. A, Eq. (8): node state --- */

/* Planar DQ of a pure translation t (trans2dq of App. A). */
void oracle_dq_translation(double tx, double ty, double q[4])
{
    oracle_dq_from_rt(0.0, tx, ty, q);
}

/* Rigid motion of a planar DQ as (cos, sin, tx, ty); q need not be unit. */
static void rigid_of(const double q[4], double m[4])
{
    oracle_dq_decode(q, &m[0], &m[1], &m[2], &m[3]);
}

/* a * b in the sense of App. A: the motion that applies a first, then b. */
void oracle_dq_then(const double a[4], const double b[4], double out[4])
{
    double ma[4], mb[4];
    rigid_of(a, ma);
    rigid_of(b, mb);
    /* b(a(x)) = Rb (Ra x + ta) + tb */
    double c = mb[0] * ma[0] - mb[1] * ma[1];
    double s = mb[1] * ma[0] + mb[0] * ma[1];
    double tx = mb[0] * ma[2] - mb[1] * ma[3] + mb[2];
    double ty = mb[1] * ma[2] + mb[0] * ma[3] + mb[3];
    oracle_dq_from_rt(atan2(s, c), tx, ty, out);
}

/* App. A warp-function update f(s_old, q_old, ds, dq):
 *   q1 = trans2dq((1 - s_old) / s_old * dt),  q2 = dq * q1,
 *   q_new = q_old * q2,  s_new = ds * s_old,
 * with dt the translation of dq and "*" applying its left operand first. */
void oracle_update(double s_old, const double q_old[4], double ds, const double dq[4],
                   double *s_new, double q_new[4])
{
    double md[4], q1[4], q2[4];
    rigid_of(dq, md);
    double k = (1.0 - s_old) / s_old;
    oracle_dq_translation(k * md[2], k * md[3], q1);
    oracle_dq_then(dq, q1, q2);
    oracle_dq_then(q_old, q2, q_new);
    *s_new = ds * s_old;
}

/* Eq. (8): uncertainty at the grid points z = (zx0 + i, zy0 + k):
 * min over the inliers j of exp(beta |z - x_j|^2).  out [h][w]; +inf when
 * there is no inlier. */
void oracle_uncertainty(int n, const double *x, const uint8_t *mask, double beta, int zx0,
                        int zy0, int w, int h, double *out)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int k = 0; k < h; ++k)
        for (int i = 0; i < w; ++i) {
            double best = INFINITY;
            for (int j = 0; j < n; ++j) {
                if (!mask[j]) continue;
                double dx = zx0 + i - x[2 * j], dy = zy0 + k - x[2 * j + 1];
                double u = exp(beta * (dx * dx + dy * dy));
                if (u < best) best = u;
            }
            out[(size_t)k * w + i] = best;
        }
}

/* Eqs. (2)-(3) at the point z over the inliers (mask), followed by the
 * normalisation of the blended DQ by the norm of its real part: the
 * node-level warp increment (Delta s, Delta q) that Sec. III-C reads off the
 * EMDQ field.  Returns 0, or -1 if no inlier carries weight at z. */
int oracle_blend_dq(int n, const double *x, const double *scale, const double *q,
                    const uint8_t *mask, double alpha, double zx, double zy, double *s_out,
                    double q_out[4])
{
    double W = 0.0, sb = 0.0, qb[4] = {0.0, 0.0, 0.0, 0.0};
    for (int j = 0; j < n; ++j) {
        if (!mask[j]) continue;
        double dx = zx - x[2 * j], dy = zy - x[2 * j + 1];
        double w = exp(-alpha * (dx * dx + dy * dy));
        W += w;
        sb += w * scale[j];
        for (int c = 0; c < 4; ++c) qb[c] += w * q[4 * j + c];
    }
    if (!(W > 0.0)) return -1;
    double nr = sqrt(qb[0] * qb[0] + qb[1] * qb[1]);
    if (!(nr > 0.0)) return -1;
    *s_out = sb / W;
    for (int c = 0; c < 4; ++c) q_out[c] = qb[c] / nr;   /* qb / W / (|r| / W) */
    return 0;
}

/* One tracking step of the deformation nodes (Sec. III-C, Sec. III-E):
 * for node i at position p_i in the frame the model's src points live in,
 *   (ds, dq) = the blend at p_i (Eqs. (2)-(3), normalised),
 *   dsig2    = min over the inliers j of exp(beta |p_i - x_j|^2)  (Eq. (8)),
 *   (s, q)  <- f(s, q, ds, dq)                                     (App. A),
 *   sig2    <- ds^2 sig2 + dsig2                                   (Eq. (9)),
 *   p_i     <- ds dq(p_i)                                          (Eq. (1)).
 * Arrays are updated in place.  Returns 0, or OR_ENOINLIERS if some node
 * has no weight (its entries are then NaN). */
int oracle_track_nodes(int n, const double *x, const double *scale, const double *q,
                       const uint8_t *mask, double alpha, double beta, int m, double *pos,
                       double *s_node, double *q_node, double *sig2)
{
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(| : bad)
    for (int i = 0; i < m; ++i) {
        double px = pos[2 * i], py = pos[2 * i + 1];
        double ds, dq[4];
        if (oracle_blend_dq(n, x, scale, q, mask, alpha, px, py, &ds, dq) != 0) {
            pos[2 * i] = pos[2 * i + 1] = s_node[i] = sig2[i] = NAN;
            for (int c = 0; c < 4; ++c) q_node[4 * i + c] = NAN;
            bad = 1;
            continue;
        }
        double u = INFINITY;                     /* Eq. (8) */
        for (int j = 0; j < n; ++j) {
            if (!mask[j]) continue;
            double dx = px - x[2 * j], dy = py - x[2 * j + 1];
            double e = exp(beta * (dx * dx + dy * dy));
            if (e < u) u = e;
        }
        double s_new, q_new[4];
        oracle_update(s_node[i], &q_node[4 * i], ds, dq, &s_new, q_new);
        sig2[i] = ds * ds * sig2[i] + u;
        double nx, ny;
        oracle_warp_point(ds, dq, px, py, &nx, &ny);
        pos[2 * i] = nx;
        pos[2 * i + 1] = ny;
        s_node[i] = s_new;
        for (int c = 0; c < 4; ++c) q_node[4 * i + c] = q_new[c];
    }
    return bad ? OR_ENOINLIERS : OR_OK;
}

/* ------------------------------------------------ learned EM start --- */
/*
 * Not in the paper: a learned starting point for the EM (a per-match
 * inlier prior), the next step the design takes beyond it.  Definition:
 *   neighbours  the K = 16 other matches nearest to match i by source
 *               distance, ordered by (squared distance in FP64, index);
 *               missing neighbours (n - 1 < K) give zero features;
 *   features    for neighbour rank r and neighbour j, with g = sqrt(alpha)
 *               and displacement d = dst - src:
 *                 f[4r]   = g (x_j - x_i)_x,  f[4r+1] = g (x_j - x_i)_y,
 *                 f[4r+2] = ss((d_j - d_i)_x / 8),  f[4r+3] = ss((d_j - d_i)_y / 8),
 *               ss(t) = t / (1 + |t|);
 *   network     h1 = gelu(W1 f + b1) (128), h2 = gelu(W2 h1 + b2) (128),
 *               p = sigmoid(w3 . h2 + b3), gelu(t) = t (1 + erf(t / sqrt 2)) / 2.
 */
#define OR_KNN 16
#define OR_NF (4 * OR_KNN)
#define OR_NH 128

void oracle_init_features(int n, const double *x, const double *y, double alpha,
                          double *feat)
{
    const double g = sqrt(alpha);
#pragma omp parallel for schedule(dynamic, 16)
    for (int i = 0; i < n; ++i) {
        double bd[OR_KNN];
        int bj[OR_KNN];
        int cnt = 0;
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            double dx = x[2 * j] - x[2 * i], dy = x[2 * j + 1] - x[2 * i + 1];
            double d2 = dx * dx + dy * dy;
            /* insertion into the sorted list of the best K by (d2, j) */
            int pos = cnt;
            while (pos > 0 && (bd[pos - 1] > d2 || (bd[pos - 1] == d2 && bj[pos - 1] > j)))
                --pos;
            if (pos >= OR_KNN) continue;
            int last = cnt < OR_KNN ? cnt : OR_KNN - 1;
            for (int k = last; k > pos; --k) { bd[k] = bd[k - 1]; bj[k] = bj[k - 1]; }
            bd[pos] = d2;
            bj[pos] = j;
            if (cnt < OR_KNN) ++cnt;
        }
        double *f = feat + (size_t)i * OR_NF;
        double dix = y[2 * i] - x[2 * i], diy = y[2 * i + 1] - x[2 * i + 1];
        for (int r = 0; r < OR_KNN; ++r) {
            if (r >= cnt) { f[4 * r] = f[4 * r + 1] = f[4 * r + 2] = f[4 * r + 3] = 0.0; continue; }
            int j = bj[r];
            double ex = (y[2 * j] - x[2 * j] - dix) / 8.0, ey = (y[2 * j + 1] - x[2 * j + 1] - diy) / 8.0;
            f[4 * r] = g * (x[2 * j] - x[2 * i]);
            f[4 * r + 1] = g * (x[2 * j + 1] - x[2 * i + 1]);
            f[4 * r + 2] = ex / (1.0 + fabs(ex));
            f[4 * r + 3] = ey / (1.0 + fabs(ey));
        }
    }
}

static double gelu(double t) { return 0.5 * t * (1.0 + erf(t / sqrt(2.0))); }

/* w: W1[128][64], b1[128], W2[128][128], b2[128], w3[128], b3 (row-major). */
void oracle_init_mlp(int n, const double *feat, const double *w, double *p_out)
{
    const double *W1 = w, *b1 = W1 + OR_NH * OR_NF, *W2 = b1 + OR_NH;
    const double *b2 = W2 + OR_NH * OR_NH, *w3 = b2 + OR_NH, *b3 = w3 + OR_NH;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) {
        const double *f = feat + (size_t)i * OR_NF;
        double h1[OR_NH], h2[OR_NH];
        for (int o = 0; o < OR_NH; ++o) {
            double a = b1[o];
            for (int k = 0; k < OR_NF; ++k) a += W1[o * OR_NF + k] * f[k];
            h1[o] = gelu(a);
        }
        for (int o = 0; o < OR_NH; ++o) {
            double a = b2[o];
            for (int k = 0; k < OR_NH; ++k) a += W2[o * OR_NH + k] * h1[k];
            h2[o] = gelu(a);
        }
        double z = b3[0];
        for (int k = 0; k < OR_NH; ++k) z += w3[k] * h2[k];
        p_out[i] = 1.0 / (1.0 + exp(-z));
    }
}

/* bfloat16 rounding: v to the nearest number with an 8-bit significand
 * (7 stored bits plus the implicit one) and FP32's exponent range, ties to
 * the even significand.  Written from that definition: v = m 2^e with
 * 0.5 <= |m| < 1, so m 2^8 is rounded to an integer, half to even (rint in
 * the default rounding mode), and scaled back.  Zero, infinities and NaN pass
 * through; magnitudes below FP32's normal range are not used here. */
double oracle_bf16(double v)
{
    if (v == 0.0 || !isfinite(v)) return v;
    int e;
    const double m = frexp(v, &e);
    return ldexp(rint(m * 256.0), e - 8);
}

/* The learned start's network with its two matrix products in BF16: the
 * features, W1, W2 and the first hidden layer rounded to BF16 before they
 * are multiplied; the products are exact and summed in FP64; the biases,
 * GELU, the second hidden layer and the output layer stay in full
 * precision.  Same weight layout as oracle_init_mlp. */
void oracle_init_mlp_bf16(int n, const double *feat, const double *w, double *p_out)
{
    const double *W1 = w, *b1 = W1 + OR_NH * OR_NF, *W2 = b1 + OR_NH;
    const double *b2 = W2 + OR_NH * OR_NH, *w3 = b2 + OR_NH, *b3 = w3 + OR_NH;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) {
        const double *f = feat + (size_t)i * OR_NF;
        double fb[OR_NF], h1[OR_NH], h2[OR_NH];
        for (int k = 0; k < OR_NF; ++k) fb[k] = oracle_bf16(f[k]);
        for (int o = 0; o < OR_NH; ++o) {
            double a = b1[o];
            for (int k = 0; k < OR_NF; ++k) a += oracle_bf16(W1[o * OR_NF + k]) * fb[k];
            h1[o] = oracle_bf16(gelu(a));
        }
        for (int o = 0; o < OR_NH; ++o) {
            double a = b2[o];
            for (int k = 0; k < OR_NH; ++k) a += oracle_bf16(W2[o * OR_NH + k]) * h1[k];
            h2[o] = gelu(a);
        }
        double z = b3[0];
        for (int k = 0; k < OR_NH; ++k) z += w3[k] * h2[k];
        p_out[i] = 1.0 / (1.0 + exp(-z));
    }
}

/* Mean binary cross-entropy of the learned start over n labelled samples
 * (label 1 = inlier) and its gradient with respect to the flat weight vector
 * (same layout as oracle_init_mlp), by the chain rule written out layer by
 * layer; gelu'(t) = Phi(t) + t phi(t).  grad: [N_WEIGHTS], overwritten. */
double oracle_start_grad(int n, const double *feat, const double *label, const double *w,
                         double *grad)
{
    const double *W1 = w, *b1 = W1 + OR_NH * OR_NF, *W2 = b1 + OR_NH;
    const double *b2 = W2 + OR_NH * OR_NH, *w3 = b2 + OR_NH, *b3 = w3 + OR_NH;
    double *gW1 = grad, *gb1 = gW1 + OR_NH * OR_NF, *gW2 = gb1 + OR_NH;
    double *gb2 = gW2 + OR_NH * OR_NH, *gw3 = gb2 + OR_NH, *gb3 = gw3 + OR_NH;
    const int nw = OR_NH * OR_NF + OR_NH + OR_NH * OR_NH + OR_NH + OR_NH + 1;
    for (int k = 0; k < nw; ++k) grad[k] = 0.0;
    double loss = 0.0;
    for (int i = 0; i < n; ++i) {
        const double *f = feat + (size_t)i * OR_NF;
        double a1[OR_NH], h1[OR_NH], a2[OR_NH], h2[OR_NH], d2[OR_NH], d1[OR_NH];
        for (int o = 0; o < OR_NH; ++o) {
            double a = b1[o];
            for (int k = 0; k < OR_NF; ++k) a += W1[o * OR_NF + k] * f[k];
            a1[o] = a;
            h1[o] = gelu(a);
        }
        for (int o = 0; o < OR_NH; ++o) {
            double a = b2[o];
            for (int k = 0; k < OR_NH; ++k) a += W2[o * OR_NH + k] * h1[k];
            a2[o] = a;
            h2[o] = gelu(a);
        }
        double z = b3[0];
        for (int k = 0; k < OR_NH; ++k) z += w3[k] * h2[k];
        double y = label[i];
        /* loss = softplus(z) - y z, stable form */
        loss += (z > 0 ? z + log1p(exp(-z)) : log1p(exp(z))) - y * z;
        double dz = 1.0 / (1.0 + exp(-z)) - y;
        gb3[0] += dz;
        for (int o = 0; o < OR_NH; ++o) {
            gw3[o] += dz * h2[o];
            double t = a2[o];
            double dg = 0.5 * (1.0 + erf(t / sqrt(2.0))) + t * exp(-0.5 * t * t) / sqrt(2.0 * M_PI);
            d2[o] = dz * w3[o] * dg;
        }
        for (int o = 0; o < OR_NH; ++o) {
            gb2[o] += d2[o];
            for (int k = 0; k < OR_NH; ++k) gW2[o * OR_NH + k] += d2[o] * h1[k];
        }
        for (int k = 0; k < OR_NH; ++k) {
            double s = 0.0;
            for (int o = 0; o < OR_NH; ++o) s += W2[o * OR_NH + k] * d2[o];
            double t = a1[k];
            double dg = 0.5 * (1.0 + erf(t / sqrt(2.0))) + t * exp(-0.5 * t * t) / sqrt(2.0 * M_PI);
            d1[k] = s * dg;
        }
        for (int o = 0; o < OR_NH; ++o) {
            gb1[o] += d1[o];
            for (int k = 0; k < OR_NF; ++k) gW1[o * OR_NF + k] += d1[o] * f[k];
        }
    }
    for (int k = 0; k < nw; ++k) grad[k] /= n;
    return loss / n;
}
