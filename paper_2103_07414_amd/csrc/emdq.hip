// emdq.hip -- EMDQ dense deformation field + warp for the MI355X (gfx950).
//
// Method: H. Zhou and J. Jayender, "Real-time Nonrigid Mosaicking of
// Laparoscopy Images" (arXiv 2103.07414), Sec. II-A (EMDQ), Eqs. (1)-(4),
// (18)-(20), Sec. III-F and Eqs. (23)-(24).  The public contract is
// include/emdq.h.
//
// Kernels
//   k_reset / k_load   model state reset; copy of the matches, finiteness check
//   k_mstep            per-match weighted similarity fit (Eqs. (18)-(20)) with
//                      weights exp(-alpha d^2) p_j (Eq. (4)); one wavefront per
//                      match, lanes stride the other matches, two-pass
//                      centred FP32 moments, FP64 re-fit of near-degenerate rows
//   k_estep            DQ blend at every match (Eqs. (2)-(3)), residuals; the
//                      last workgroup reduces (FP64, fixed order), updates the
//                      posteriors, the inlier mask and the stop flag
//   k_compact          packs the inliers for the field kernel (one workgroup,
//                      ordered scan)
//   k_field<MODE>      the W(P x N_in) . Q(N_in x 6) blend on FP32 MFMA, with
//                      the Gaussian factorised per axis, followed in registers
//                      by DQ normalisation, Eq. (1) and (MODE 1) the bilinear
//                      sample and colour merge
//
// Every reduction has a fixed order, and there are no floating-point atomics,
// so results are bit-reproducible.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "emdq.h"

namespace {

constexpr float kLog2e = 1.4426950408889634f;
constexpr int kWave = 64;
constexpr int kRowsPerBlock = 8;        // EM kernels: one wavefront per match
constexpr int kEmThreads = kWave * kRowsPerBlock;
constexpr int kMChunk = 2048;           // matches staged in LDS per M-step sweep
constexpr int kEChunk = 1024;           // matches (+ fits) staged per E-step sweep
constexpr int kCompactThreads = 1024;
constexpr int kFieldThreads = 256;      // 4 wavefronts per workgroup
constexpr int kTile = 32;               // 32 x 32 pixels per MFMA output tile
#ifndef EMDQ_RING
#define EMDQ_RING 4
#endif
#ifndef EMDQ_SCHED_MASK
#define EMDQ_SCHED_MASK 0x000F   // ALU, VALU, SALU, MFMA may cross
#endif
#ifndef EMDQ_SPLITK
#define EMDQ_SPLITK 4
#endif

constexpr int kRing = EMDQ_RING;       // field kernel: record ring depth (K steps)

typedef float f32x16 __attribute__((ext_vector_type(16)));

// Device-side record of the model.  Written by the EM kernels, read by the
// field kernel and, after a stream synchronisation, by the host.
struct DevState {
    int status;      // emdq_status of the fit (0 while running)
    int iter;        // EM iterations done
    int done;        // 1 once the stop rule fired
    int n_in;        // number of packed inliers
    unsigned ticket; // arrival counter of the E-step workgroups
    int changed;     // mask changed in the last iteration
    float sigma2;
    float gamma;
};

// ------------------------------------------------------------ helpers ----

__device__ __forceinline__ float wave_sum(float v) {
    // butterfly: every lane ends with the same bits (a + b == b + a)
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

__device__ __forceinline__ double wave_sum_d(double v) {
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

__device__ __forceinline__ float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }

__device__ __forceinline__ bool finite2(float2 v) {
    return __builtin_isfinite(v.x) && __builtin_isfinite(v.y);
}

// ------------------------------------------------------ state, loading ----

__global__ void k_reset(DevState *st) {
    if (threadIdx.x == 0) {
        st->status = 0;
        st->iter = 0;
        st->done = 0;
        st->n_in = 0;
        st->ticket = 0u;
        st->changed = 0;
        st->sigma2 = 0.f;
        st->gamma = 0.f;
    }
}

// xy[i] = (src_i, dst_i); p = 1, mask = 1; a non-finite coordinate sets the
// status to ENONFINITE (every writer stores the same value).
__global__ void k_load(const float2 *__restrict__ src, const float2 *__restrict__ dst, int n,
                       float4 *__restrict__ xy, float *__restrict__ p,
                       uint8_t *__restrict__ mask, DevState *st) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float2 a = src[i], b = dst[i];
    xy[i] = make_float4(a.x, a.y, b.x, b.y);
    p[i] = 1.f;
    mask[i] = 1;
    if (!finite2(a) || !finite2(b)) {
        atomicMin(&st->status, (int)EMDQ_ENONFINITE);
        atomicExch(&st->done, 1);
    }
}

// ------------------------------------------------- blend evaluation ----
//
// The blended sums are kept deviation-coded: with W = sum w, the sums of
// (q_c - 1) and (s - 1) instead of q_c and s (exact algebra, as the weights'
// own sum W restores sum w q_c = W + sum w (q_c - 1)).  The warp is then
// evaluated as a displacement D = F(z) - z:
//   s_hat = 1 + sg,  R_hat - I = [[-2 sn^2, -2 c sn], [2 c sn, -2 sn^2]] / n^2,
//   t_hat = 2 (c x - sn y, c y + sn x) / n^2,   n^2 = c^2 + sn^2,
//   D = sg z + (1 + sg) ((R_hat - I) z + t_hat),
// where c, sn, x, y, sg are the weighted means of q_c, q_s, q_x, q_y, s - 1.
// Nothing large cancels, so FP32 keeps ~1e-5 px on a ~1000 px coordinate.
__device__ __forceinline__ float2 blend_displacement(float W, float Cd, float Sn, float X, float Y,
                                                     float Gd, float zx, float zy) {
    const float iW = 1.f / W;
    const float c = 1.f + Cd * iW, sn = Sn * iW, x = X * iW, y = Y * iW, sg = Gd * iW;
    const float in2 = 1.f / (c * c + sn * sn);
    const float r00 = -2.f * sn * sn * in2, r10 = 2.f * c * sn * in2;
    const float tx = 2.f * (c * x - sn * y) * in2, ty = 2.f * (c * y + sn * x) * in2;
    const float s1 = 1.f + sg;
    return make_float2(sg * zx + s1 * (r00 * zx - r10 * zy + tx),
                       sg * zy + s1 * (r10 * zx + r00 * zy + ty));
}

// --------------------------------------------------------------- M-step ----

// Planar DQ from the half-angle direction (ch, sh) and the translation.
__device__ __forceinline__ float4 dq_make(float ch, float sh, float tx, float ty) {
    return make_float4(ch, sh, 0.5f * (ch * tx + sh * ty), 0.5f * (ch * ty - sh * tx));
}

// FP64 fit of one match, taken when the FP32 moments are too ill-conditioned
// to decide the degenerate case: two-pass centred sums over all matches,
// spread over the lanes of the wavefront.
__device__ void fit_row_f64(int i, const float4 *__restrict__ xy, const float *__restrict__ p,
                            int n, double alpha, int lane, float *scale_out, float4 *q_out) {
    const float4 me = xy[i];
    double S = 0, ax = 0, ay = 0, bx = 0, by = 0;
    for (int j = lane; j < n; j += kWave) {
        float4 v = xy[j];
        double dx = (double)v.x - me.x, dy = (double)v.y - me.y;
        double w = exp(-alpha * (dx * dx + dy * dy)) * (double)p[j];
        S += w;
        ax += w * v.x;
        ay += w * v.y;
        bx += w * v.z;
        by += w * v.w;
    }
    S = wave_sum_d(S);
    ax = wave_sum_d(ax);
    ay = wave_sum_d(ay);
    bx = wave_sum_d(bx);
    by = wave_sum_d(by);
    if (!(S > 0.0)) {
        *scale_out = 1.f;
        *q_out = make_float4(1.f, 0.f, 0.f, 0.f);
        return;
    }
    const double mx = ax / S, my = ay / S, nx = bx / S, ny = by / S;
    double c00 = 0, c01 = 0, c10 = 0, c11 = 0, vx = 0, vy = 0;
    for (int j = lane; j < n; j += kWave) {
        float4 v = xy[j];
        double dx = (double)v.x - me.x, dy = (double)v.y - me.y;
        double w = exp(-alpha * (dx * dx + dy * dy)) * (double)p[j];
        double a0 = v.x - mx, a1 = v.y - my, b0 = v.z - nx, b1 = v.w - ny;
        c00 += w * b0 * a0;
        c01 += w * b0 * a1;
        c10 += w * b1 * a0;
        c11 += w * b1 * a1;
        vx += w * (a0 * a0 + a1 * a1);
        vy += w * (b0 * b0 + b1 * b1);
    }
    c00 = wave_sum_d(c00);
    c01 = wave_sum_d(c01);
    c10 = wave_sum_d(c10);
    c11 = wave_sum_d(c11);
    vx = wave_sum_d(vx);
    vy = wave_sum_d(vy);
    if (vx <= 1e-12 * S || vy <= 1e-12 * S) {
        *scale_out = 1.f;
        *q_out = make_float4(1.f, 0.f, (float)(0.5 * (nx - mx)), (float)(0.5 * (ny - my)));
        return;
    }
    const double a = c00 + c11, b = c10 - c01;
    const double r = sqrt(a * a + b * b);
    double ct = 1.0, st = 0.0, ch = 1.0, sh = 0.0;
    if (r > 0.0) {
        ct = a / r;
        st = b / r;
        double hx, hy;
        if (a >= 0.0) { hx = r + a; hy = b; }
        else { double sg = b < 0.0 ? -1.0 : 1.0; hx = sg * b; hy = sg * (r - a); }
        const double hn = sqrt(hx * hx + hy * hy);
        ch = hx / hn;
        sh = hy / hn;
    }
    const double s = sqrt(vy / vx);
    const double tx = nx / s - (ct * mx - st * my);
    const double ty = ny / s - (st * mx + ct * my);
    *scale_out = (float)s;
    *q_out = make_float4((float)ch, (float)sh, (float)(0.5 * (ch * tx + sh * ty)),
                         (float)(0.5 * (ch * ty - sh * tx)));
}

// One wavefront per match i: weights w_j = exp(-alpha |x_j - x_i|^2) p_j.
// The workgroup stages the matches in LDS (coalesced, kMChunk at a time) and
// each wavefront sweeps them from there.  Pass 1: weight sum and weighted
// centroids, relative to (x_i, y_i).  Pass 2 (weights recomputed): centred
// cross-covariance terms and spreads, so no moment is formed by cancellation.
// Then the closed-form 2D Procrustes fit.
__global__ __launch_bounds__(kEmThreads) void k_mstep(
    const float4 *__restrict__ xy, const float *__restrict__ p, int n, float nal2,
    double alpha, float4 *__restrict__ q_out, float *__restrict__ s_out,
    const DevState *__restrict__ st, int final_pass) {
    __shared__ float4 s_xy[kMChunk];
    __shared__ float s_p[kMChunk];
    if (st->status < 0) return;
    if (!final_pass && st->done) return;
    const int lane = threadIdx.x & (kWave - 1);
    const int i = blockIdx.x * kRowsPerBlock + (threadIdx.x >> 6);
    const bool active = i < n;
    const float4 me = active ? xy[i] : make_float4(0.f, 0.f, 0.f, 0.f);
    const bool resident = n <= kMChunk;   // one staging serves both passes
    auto stage = [&](int c0, int cn) {
        __syncthreads();
        for (int t = threadIdx.x; t < cn; t += kEmThreads) {
            s_xy[t] = xy[c0 + t];
            s_p[t] = p[c0 + t];
        }
        __syncthreads();
    };

    float S = 0.f, Ax = 0.f, Ay = 0.f, Bx = 0.f, By = 0.f;
    for (int c0 = 0; c0 < n; c0 += kMChunk) {
        const int cn = min(kMChunk, n - c0);
        stage(c0, cn);
        if (active) {
#pragma unroll 4
            for (int t = lane; t < cn; t += kWave) {
                const float4 v = s_xy[t];
                const float dxx = v.x - me.x, dxy = v.y - me.y;   // x_j - x_i
                const float w = fast_exp2(nal2 * (dxx * dxx + dxy * dxy)) * s_p[t];
                S += w;
                Ax += w * dxx;
                Ay += w * dxy;
                Bx += w * (v.z - me.z);                          // y_j - y_i
                By += w * (v.w - me.w);
            }
        }
    }
    S = wave_sum(S);
    Ax = wave_sum(Ax);
    Ay = wave_sum(Ay);
    Bx = wave_sum(Bx);
    By = wave_sum(By);

    float mx = 0.f, my = 0.f, nx = 0.f, ny = 0.f;
    float vx = 0.f, vy = 0.f, a = 0.f, b = 0.f;
    const bool have_w = S > 0.f;
    if (have_w) {
        mx = Ax / S; my = Ay / S; nx = Bx / S; ny = By / S;
    }
    // weighted centroids in absolute coordinates
    const float cxx = me.x + mx, cxy = me.y + my, cyx = me.z + nx, cyy = me.w + ny;
    for (int c0 = 0; c0 < n; c0 += kMChunk) {
        const int cn = min(kMChunk, n - c0);
        if (!resident) stage(c0, cn);
        if (active && have_w) {
#pragma unroll 4
            for (int t = lane; t < cn; t += kWave) {
                const float4 v = s_xy[t];
                const float dxx = v.x - me.x, dxy = v.y - me.y;
                const float w = fast_exp2(nal2 * (dxx * dxx + dxy * dxy)) * s_p[t];
                const float ax = v.x - cxx, ay = v.y - cxy;    // x_j - xbar
                const float bx = v.z - cyx, by = v.w - cyy;    // y_j - ybar
                vx += w * (ax * ax + ay * ay);
                vy += w * (bx * bx + by * by);
                a += w * (bx * ax + by * ay);                  // C00 + C11
                b += w * (by * ax - bx * ay);                  // C10 - C01
            }
        }
    }
    if (!active) return;
    vx = wave_sum(vx);
    vy = wave_sum(vy);
    a = wave_sum(a);
    b = wave_sum(b);

    float scale;
    float4 q;
    // no weight, or a near-degenerate spread (below 1e-2 px^2): decide and
    // fit in FP64
    const bool need_f64 = !have_w || !(vx > 1e-2f * S) || !(vy > 1e-2f * S);
    if (need_f64) {
        fit_row_f64(i, xy, p, n, alpha, lane, &scale, &q);
    } else {
        const float r = sqrtf(a * a + b * b);
        float ct = 1.f, stt = 0.f, ch = 1.f, sh = 0.f;
        if (r > 0.f) {
            ct = a / r;
            stt = b / r;
            float hx, hy;
            if (a >= 0.f) { hx = r + a; hy = b; }
            else { const float sg = b < 0.f ? -1.f : 1.f; hx = sg * b; hy = sg * (r - a); }
            const float hn = sqrtf(hx * hx + hy * hy);
            ch = hx / hn;
            sh = hy / hn;
        }
        scale = sqrtf(vy / vx);
        const float cx = me.x + mx, cy = me.y + my;     // weighted centroid of x
        const float gx = me.z + nx, gy = me.w + ny;     // weighted centroid of y
        const float tx = gx / scale - (ct * cx - stt * cy);
        const float ty = gy / scale - (stt * cx + ct * cy);
        q = dq_make(ch, sh, tx, ty);
    }
    if (lane == 0) {
        q_out[i] = q;
        s_out[i] = scale;
    }
}

// --------------------------------------------------------------- E-step ----

// Blend of all fits at match i with weights exp(-alpha d^2) p_j (Eqs. (2)-(3)),
// normalisation, prediction y_hat = s (R x_i + t) (Eq. (1)), residual e_i^2.
// The last workgroup to finish turns the residuals into sigma^2, gamma, new
// posteriors, the mask and the stop decision.
__global__ __launch_bounds__(kEmThreads) void k_estep(
    const float4 *__restrict__ xy, float *__restrict__ p, const float4 *__restrict__ q,
    const float *__restrict__ s, int n, float nal2, double u, double sigma2_min,
    double gamma_min, double gamma_max, float p_thresh, int max_iter,
    float *__restrict__ e2, uint8_t *__restrict__ mask, DevState *st) {
    __shared__ float4 s_xy[kEChunk];
    __shared__ float4 s_q[kEChunk];
    __shared__ float2 s_ps[kEChunk];   // (p_j, s_j - 1)
    if (st->status < 0 || st->done) return;
    const int lane = threadIdx.x & (kWave - 1);
    const int i = blockIdx.x * kRowsPerBlock + (threadIdx.x >> 6);
    const bool active = i < n;
    const float4 me = active ? xy[i] : make_float4(0.f, 0.f, 0.f, 0.f);
    float W = 0.f, Gd = 0.f, Cd = 0.f, Sn = 0.f, X = 0.f, Y = 0.f;
    for (int c0 = 0; c0 < n; c0 += kEChunk) {
        const int cn = min(kEChunk, n - c0);
        __syncthreads();
        for (int t = threadIdx.x; t < cn; t += kEmThreads) {
            s_xy[t] = xy[c0 + t];
            s_q[t] = q[c0 + t];
            s_ps[t] = make_float2(p[c0 + t], s[c0 + t] - 1.f);
        }
        __syncthreads();
        if (active) {
#pragma unroll 4
            for (int t = lane; t < cn; t += kWave) {
                const float4 v = s_xy[t];
                const float2 ps = s_ps[t];
                const float dx = v.x - me.x, dy = v.y - me.y;
                const float w = fast_exp2(nal2 * (dx * dx + dy * dy)) * ps.x;
                const float4 qj = s_q[t];
                W += w;
                Gd += w * ps.y;
                Cd += w * (qj.x - 1.f);
                Sn += w * qj.y;
                X += w * qj.z;
                Y += w * qj.w;
            }
        }
    }
    if (active) {
        W = wave_sum(W);
        Gd = wave_sum(Gd);
        Cd = wave_sum(Cd);
        Sn = wave_sum(Sn);
        X = wave_sum(X);
        Y = wave_sum(Y);
        float err = __builtin_huge_valf();
        if (W > 0.f) {
            // e = y_i - F(x_i) = (y_i - x_i) - D(x_i)
            const float2 d = blend_displacement(W, Cd, Sn, X, Y, Gd, me.x, me.y);
            const float ex = (me.z - me.x) - d.x, ey = (me.w - me.y) - d.y;
            err = ex * ex + ey * ey;
        }
        if (lane == 0) e2[i] = err;
    }

    // ---- arrival: the last workgroup finishes the iteration
    __shared__ int last;
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const unsigned t = atomicAdd(&st->ticket, 1u);
        last = (t == gridDim.x - 1);
    }
    __syncthreads();
    if (!last) return;
    __threadfence();

    __shared__ double red_p[kEmThreads], red_pe[kEmThreads];
    __shared__ int any_changed;
    if (threadIdx.x == 0) any_changed = 0;
    double sp = 0.0, spe = 0.0;
    for (int r = threadIdx.x; r < n; r += kEmThreads) {
        const double pr = (double)p[r];
        const float er = __hip_atomic_load(&e2[r], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        sp += pr;
        if (pr > 0.0) spe += pr * (double)er;
    }
    red_p[threadIdx.x] = sp;
    red_pe[threadIdx.x] = spe;
    __syncthreads();
    for (int off = kEmThreads / 2; off >= 1; off >>= 1) {
        if (threadIdx.x < off) {
            red_p[threadIdx.x] += red_p[threadIdx.x + off];
            red_pe[threadIdx.x] += red_pe[threadIdx.x + off];
        }
        __syncthreads();
    }
    const double SP = red_p[0], SPE = red_pe[0];
    if (!(SP > 0.0)) {
        if (threadIdx.x == 0) {
            st->status = EMDQ_ENOINLIERS;
            st->done = 1;
            st->ticket = 0u;
        }
        return;
    }
    double sigma2 = SPE / (2.0 * SP);
    if (!(sigma2 >= sigma2_min)) sigma2 = sigma2_min;
    double gamma = SP / (double)n;
    gamma = gamma < gamma_min ? gamma_min : (gamma > gamma_max ? gamma_max : gamma);
    const double two_pi = 6.283185307179586;
    const double inv2s = 1.0 / (2.0 * sigma2);
    const double norm = 1.0 / (two_pi * sigma2);
    const double b = (1.0 - gamma) * u;
    int changed = 0;
    __syncthreads();
    for (int r = threadIdx.x; r < n; r += kEmThreads) {
        const float er = __hip_atomic_load(&e2[r], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const double a = gamma * exp(-(double)er * inv2s) * norm;
        const float pn = (float)(a / (a + b));
        p[r] = pn;
        const uint8_t m = pn > p_thresh ? 1 : 0;
        changed |= (m != mask[r]);
        mask[r] = m;
    }
    if (changed) atomicOr(&any_changed, 1);
    __syncthreads();
    if (threadIdx.x == 0) {
        const int it = st->iter + 1;
        st->iter = it;
        st->changed = any_changed;
        st->sigma2 = (float)sigma2;
        st->gamma = (float)gamma;
        if (it >= 2 && !any_changed) {
            st->done = 1;
        } else if (it >= max_iter) {
            st->done = 1;
            st->status = EMDQ_WARN_NOT_CONVERGED;
        }
        st->ticket = 0u;
        __threadfence();
    }
}

// ------------------------------------------------------------ compaction ----

// Packs the inliers in index order: packed[2k] = (x, y, q_c - 1, q_s),
// packed[2k+1] = (q_x, q_y, s - 1, 1) (deviation-coded, see
// blend_displacement).  One workgroup; each thread owns a
// contiguous run of matches, runs are ordered by an exclusive scan.
__global__ __launch_bounds__(kCompactThreads) void k_compact(
    const float4 *__restrict__ xy, const float4 *__restrict__ q, const float *__restrict__ s,
    const uint8_t *__restrict__ mask, int n, float4 *__restrict__ packed, DevState *st) {
    __shared__ int scan[kCompactThreads];
    if (st->status < 0) return;
    const int t = threadIdx.x;
    const int per = (n + kCompactThreads - 1) / kCompactThreads;
    const int b = t * per, e = min(b + per, n);
    int cnt = 0;
    for (int i = b; i < e; ++i) cnt += mask[i] ? 1 : 0;
    scan[t] = cnt;
    __syncthreads();
    for (int off = 1; off < kCompactThreads; off <<= 1) {   // inclusive scan
        const int v = t >= off ? scan[t - off] : 0;
        __syncthreads();
        scan[t] += v;
        __syncthreads();
    }
    int pos = scan[t] - cnt;
    for (int i = b; i < e; ++i) {
        if (!mask[i]) continue;
        const float4 v = xy[i], qi = q[i];
        packed[2 * pos] = make_float4(v.x, v.y, qi.x - 1.f, qi.y);
        packed[2 * pos + 1] = make_float4(qi.z, qi.w, s[i] - 1.f, 1.f);
        ++pos;
    }
    if (t == kCompactThreads - 1) {
        const int total = scan[t];
        st->n_in = total;
        if (total == 0) st->status = EMDQ_ENOINLIERS;
    }
}

// ------------------------------------------------------------ field / warp ----

// Output tile: 32 x 32 src grid points.  With the Gaussian factorised per
// axis, exp(-alpha |z - x_j|^2) = gy(z_y, j) gx(z_x, j), the six per-pixel sums
//   acc_c(z) = sum_j gy(z_y, j) [gx(z_x, j) Q_c(j)],  Q = (q_c, q_s, q_x, q_y, s, 1)
// are six 32 x 32 x N_in products A . B_c with A = gy (rows z_y, cols j) and
// B_c = gx Q_c (rows j, cols z_x), one v_mfma_f32_32x32x2f32 per pair of
// inliers and per c.  Operand layout of that instruction: lane l holds
// A[l % 32][l / 32] and B[l / 32][l % 32]; accumulator register r of lane l
// is C[8 (r / 4) + 4 (l / 32) + r % 4][l % 32].  Hence a lane owns pixels of
// one column z_x and all six sums of each of its 16 pixels, and lanes 0..31
// cover 32 consecutive z_x: canvas rows are read and written coalesced.
//
// SPLITK wavefronts share one tile and split the inliers; their partial sums
// are added through LDS in a fixed order, and each then finishes 16 / SPLITK
// of the tile's accumulator registers.
template <int SPLITK>
struct FieldLds {
    float part[SPLITK > 1 ? 4 : 1][SPLITK > 1 ? 6 * (16 - 16 / SPLITK) : 1][kWave];
};

enum { kModeField = 0, kModeWarp = 1 };

template <int MODE, int SPLITK>
__global__ __launch_bounds__(kFieldThreads) void k_field(
    const float4 *__restrict__ packed, const DevState *__restrict__ st, float nal2, int zx0,
    int zy0, int w, int h, int tiles_x, int n_tiles, float2 *__restrict__ out,
    const uint8_t *__restrict__ frame, int fw, int fh, int fpitch, float4 *__restrict__ canvas,
    int cpitch, int ox, int oy) {
    constexpr int kTilesPerWg = 4 / SPLITK;
    constexpr int kRegsOwned = 16 / SPLITK;
    __shared__ FieldLds<SPLITK> lds;

    const int wave = threadIdx.x >> 6, lane = threadIdx.x & (kWave - 1);
    const int tile = blockIdx.x * kTilesPerWg + wave / SPLITK;
    const int ks = wave % SPLITK;
    const int status = st->status;
    const int n_in = st->n_in;
    const bool bad = status < 0 || n_in <= 0;
    if (MODE == kModeWarp && bad) return;    // canvas left unchanged

    const int tx = tile % tiles_x, ty = tile / tiles_x;
    const int px0 = zx0 + tx * kTile, py0 = zy0 + ty * kTile;
    const int col = lane & 31, half = lane >> 5;
    const float zcol = (float)(px0 + col);   // z_x of the B operand column
    const float zrow = (float)(py0 + col);   // z_y of the A operand row

    f32x16 acc[6];
#pragma unroll
    for (int c = 0; c < 6; ++c)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[c][r] = 0.f;

    if (!bad && tile < n_tiles) {
        // wavefront-uniform K range (scalar loop control)
        const int kper = ((n_in + 2 * SPLITK - 1) / (2 * SPLITK)) * 2;   // even
        const int kb = __builtin_amdgcn_readfirstlane(ks * kper);
        const int ke = __builtin_amdgcn_readfirstlane(min(kb + kper, n_in));
        // Ring of kRing record buffers: step u of a group uses buffer u and
        // refills it for the same step of the next group, so every load has
        // kRing K steps (kRing x 6 MFMAs) to land.  The Gaussian factors of
        // step u + 1 are computed while the MFMAs of step u run.  The group
        // loop is fully unrolled, so the buffers stay in fixed registers.
        // Indices past the range are clamped to the last inlier and their
        // weight is zero.
        auto load = [&](int j0, float4 &r0, float4 &r1) {
            const int jl = min(j0 + half, n_in - 1);
            r0 = packed[2 * jl];
            r1 = packed[2 * jl + 1];
        };
        auto factors = [&](int j0, const float4 &r0, float &a, float &g) {
            const float dy = zrow - r0.y;
            a = fast_exp2(nal2 * dy * dy);
            const float dx = zcol - r0.x;
            const float gv = fast_exp2(nal2 * dx * dx);
            g = j0 + half < ke ? gv : 0.f;
        };
        float4 ra[kRing], rb[kRing];
#pragma unroll
        for (int u = 0; u < kRing; ++u) {
            load(kb + 2 * u, ra[u], rb[u]);
            __builtin_amdgcn_sched_barrier(0);   // issue in ring order
        }
        const int kend = kb + ((ke - kb + 2 * kRing - 1) / (2 * kRing)) * (2 * kRing);
        float a, g;
        factors(kb, ra[0], a, g);
        for (int j0 = kb; j0 < kend; j0 += 2 * kRing) {
#pragma unroll
            for (int u = 0; u < kRing; ++u) {
                const int j = j0 + 2 * u;
                const float4 r0 = ra[u], r1 = rb[u];
                acc[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, g * r0.z, acc[0], 0, 0, 0);
                float an, gn;   // next step (its record is already in the ring)
                factors(j + 2, ra[(u + 1) % kRing], an, gn);
                acc[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, g * r0.w, acc[1], 0, 0, 0);
                acc[2] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, g * r1.x, acc[2], 0, 0, 0);
                acc[3] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, g * r1.y, acc[3], 0, 0, 0);
                acc[4] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, g * r1.z, acc[4], 0, 0, 0);
                acc[5] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, g * r1.w, acc[5], 0, 0, 0);
                load(j + 2 * kRing, ra[u], rb[u]);
                a = an;
                g = gn;
                // memory operations keep their place (otherwise the loads
                // sink to their use); arithmetic may move across
                __builtin_amdgcn_sched_barrier(EMDQ_SCHED_MASK);
            }
        }
    }

    // ---- split-K reduction: wavefront ks keeps registers [ks*R, ks*R + R)
    const int rbase = ks * kRegsOwned;
    if constexpr (SPLITK > 1) {
        // publish the registers other wavefronts own
        int slot = 0;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            if (r >= rbase && r < rbase + kRegsOwned) continue;
#pragma unroll
            for (int c = 0; c < 6; ++c) lds.part[wave][slot * 6 + c][lane] = acc[c][r];
            ++slot;
        }
        __syncthreads();
        // add the partials in wavefront order 0, 1, ..., SPLITK-1
        const int wbase = (wave / SPLITK) * SPLITK;
#pragma unroll
        for (int rr = 0; rr < kRegsOwned; ++rr) {
            const int r = rbase + rr;
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                float sum = 0.f;
                for (int src = 0; src < SPLITK; ++src) {
                    float v;
                    if (src == ks) {
                        v = acc[c][r];
                    } else {
                        // slot of register r in wavefront src's list
                        const int src_base = src * kRegsOwned;
                        const int sl = r < src_base ? r : r - kRegsOwned;
                        v = lds.part[wbase + src][sl * 6 + c][lane];
                    }
                    sum = src == 0 ? v : sum + v;
                }
                acc[c][r] = sum;
            }
        }
    }
    if (tile >= n_tiles) return;

    // ---- epilogue: DQ normalisation, Eq. (1), then (warp) sample + merge
#pragma unroll
    for (int rr = 0; rr < kRegsOwned; ++rr) {
        const int r = rbase + rr;
        const int zx = px0 + col;
        const int zy = py0 + 8 * (r >> 2) + 4 * half + (r & 3);
        if (zx >= zx0 + w || zy >= zy0 + h) continue;
        const float fzx = (float)zx, fzy = (float)zy;
        const float2 d = blend_displacement(acc[5][r], acc[0][r], acc[1][r], acc[2][r],
                                            acc[3][r], acc[4][r], fzx, fzy);
        if constexpr (MODE == kModeField) {
            float2 o = bad ? make_float2(__builtin_nanf(""), __builtin_nanf(""))
                           : make_float2(fzx + d.x, fzy + d.y);
            out[(size_t)(zy - zy0) * w + (zx - zx0)] = o;
        } else {
            // u = z + d with integer z: the sample cell and the bilinear
            // weights come from d alone, so u is never rounded
            if (!(d.x >= -fzx && d.x <= (float)(fw - 1 - zx) && d.y >= -fzy &&
                  d.y <= (float)(fh - 1 - zy)))
                continue;
            const float flx = floorf(d.x), fly = floorf(d.y);
            const int x0 = zx + (int)flx, y0 = zy + (int)fly;
            const int x1 = min(x0 + 1, fw - 1), y1 = min(y0 + 1, fh - 1);
            const float a = d.x - flx, b = d.y - fly;
            const uint8_t *row0 = frame + (size_t)y0 * fpitch;
            const uint8_t *row1 = frame + (size_t)y1 * fpitch;
            const float w00 = (1.f - a) * (1.f - b), w01 = a * (1.f - b);
            const float w10 = (1.f - a) * b, w11 = a * b;
            float v[3];
#pragma unroll
            for (int ch = 0; ch < 3; ++ch)
                v[ch] = w00 * (float)row0[3 * x0 + ch] + w01 * (float)row0[3 * x1 + ch] +
                        w10 * (float)row1[3 * x0 + ch] + w11 * (float)row1[3 * x1 + ch];
            float4 *px = canvas + (size_t)(zy + oy) * cpitch + (zx + ox);
            float4 cur = *px;
            const float A = cur.w, A1 = A + 1.f;
            cur.x = (A * cur.x + v[0]) / A1;
            cur.y = (A * cur.y + v[1]) / A1;
            cur.z = (A * cur.z + v[2]) / A1;
            cur.w = fminf(A1, 30.f);
            *px = cur;
        }
    }
}

constexpr int kSplitK = EMDQ_SPLITK;

}  // namespace

// ================================================================ host ====

struct emdq_model_s {
    int n_max = 0;
    int device = 0;
    int n = 0;               // matches of the last fit / set_nodes
    float alpha = 0.f;       // Eq. (4) coefficient of the current model
    float4 *xy = nullptr;    // (src, dst) per match
    float *p = nullptr;
    uint8_t *mask = nullptr;
    float *e2 = nullptr;
    float4 *q = nullptr;
    float *s = nullptr;
    float4 *packed = nullptr;
    DevState *st = nullptr;
    DevState *host_st = nullptr;   // pinned
    hipStream_t last = nullptr;
};

namespace {

#define EMDQ_HIP(call)                                   \
    do {                                                 \
        if ((call) != hipSuccess) return EMDQ_EHIP;      \
    } while (0)

emdq_status check_launch() {
    return hipGetLastError() == hipSuccess ? EMDQ_OK : EMDQ_EHIP;
}

bool params_ok(const emdq_params &p) {
    return p.alpha0 > 0.f && p.ref_w > 0 && p.ref_h > 0 && p.max_iter >= 1 &&
           p.max_iter <= 100000 && p.p_thresh > 0.f && p.p_thresh < 1.f &&
           p.gamma_min > 0.f && p.gamma_max < 1.f && p.gamma_min <= p.gamma_max &&
           p.sigma2_min > 0.f && p.flags == 0u;
}

double alpha_d(const emdq_params &p, int w, int h) {
    const double s = ((double)w / p.ref_w + (double)h / p.ref_h) / 2.0;
    return (double)p.alpha0 / (s * s);
}

emdq_status launch_field(emdq_model m, int mode, int zx0, int zy0, int w, int h, float2 *out,
                         const uint8_t *frame, int fw, int fh, int fpitch, float4 *canvas,
                         int cpitch, int ox, int oy, hipStream_t stream) {
    const int tiles_x = (w + kTile - 1) / kTile, tiles_y = (h + kTile - 1) / kTile;
    const long long n_tiles = (long long)tiles_x * tiles_y;
    constexpr int tiles_per_wg = 4 / kSplitK;
    const long long blocks = (n_tiles + tiles_per_wg - 1) / tiles_per_wg;
    if (blocks > 0x7fffffffLL / kFieldThreads) return EMDQ_EINVAL;
    const float nal2 = -m->alpha * kLog2e;
    if (mode == kModeField)
        hipLaunchKernelGGL((k_field<kModeField, kSplitK>), dim3((unsigned)blocks),
                           dim3(kFieldThreads), 0, stream, m->packed, m->st, nal2, zx0, zy0, w,
                           h, tiles_x, (int)n_tiles, out, nullptr, 0, 0, 0, nullptr, 0, 0, 0);
    else
        hipLaunchKernelGGL((k_field<kModeWarp, kSplitK>), dim3((unsigned)blocks),
                           dim3(kFieldThreads), 0, stream, m->packed, m->st, nal2, zx0, zy0, w,
                           h, tiles_x, (int)n_tiles, nullptr, frame, fw, fh, fpitch, canvas,
                           cpitch, ox, oy);
    return check_launch();
}

}  // namespace

extern "C" {

void emdq_params_default(emdq_params *p) {
    if (!p) return;
    p->alpha0 = 2e-4f;
    p->ref_w = 480;
    p->ref_h = 270;
    p->max_iter = 50;
    p->p_thresh = 0.5f;
    p->gamma_min = 0.05f;
    p->gamma_max = 0.95f;
    p->sigma2_min = 1e-2f;
    p->flags = 0u;
}

float emdq_alpha(const emdq_params *p, int frame_w, int frame_h) {
    emdq_params d;
    if (!p) {
        emdq_params_default(&d);
        p = &d;
    }
    if (frame_w <= 0 || frame_h <= 0 || p->ref_w <= 0 || p->ref_h <= 0) return 0.f;
    return (float)alpha_d(*p, frame_w, frame_h);
}

const char *emdq_status_string(emdq_status s) {
    switch (s) {
    case EMDQ_OK: return "ok";
    case EMDQ_WARN_NOT_CONVERGED: return "EM stopped at max_iter";
    case EMDQ_EINVAL: return "invalid argument";
    case EMDQ_ETOOFEW: return "fewer than 2 matches";
    case EMDQ_ENOINLIERS: return "no inliers";
    case EMDQ_ENONFINITE: return "non-finite match coordinates";
    case EMDQ_EHIP: return "HIP runtime error";
    case EMDQ_ENOMEM: return "device allocation failed";
    }
    return "unknown status";
}

emdq_status emdq_model_create(int n_max, emdq_model *out) {
    if (!out || n_max < 2 || n_max > (1 << 26)) return EMDQ_EINVAL;
    *out = nullptr;
    emdq_model m = new (std::nothrow) emdq_model_s;
    if (!m) return EMDQ_ENOMEM;
    m->n_max = n_max;
    bool ok = hipGetDevice(&m->device) == hipSuccess;
    const size_t n = (size_t)n_max;
    ok = ok && hipMalloc((void **)&m->xy, n * sizeof(float4)) == hipSuccess;
    ok = ok && hipMalloc((void **)&m->p, n * sizeof(float)) == hipSuccess;
    ok = ok && hipMalloc((void **)&m->mask, n) == hipSuccess;
    ok = ok && hipMalloc((void **)&m->e2, n * sizeof(float)) == hipSuccess;
    ok = ok && hipMalloc((void **)&m->q, n * sizeof(float4)) == hipSuccess;
    ok = ok && hipMalloc((void **)&m->s, n * sizeof(float)) == hipSuccess;
    ok = ok && hipMalloc((void **)&m->packed, 2 * n * sizeof(float4)) == hipSuccess;
    ok = ok && hipMalloc((void **)&m->st, sizeof(DevState)) == hipSuccess;
    ok = ok && hipHostMalloc((void **)&m->host_st, sizeof(DevState), hipHostMallocDefault) ==
                   hipSuccess;
    if (ok) {
        // an empty model: status ENOINLIERS until a fit or set_nodes
        DevState init = {};
        init.status = EMDQ_ENOINLIERS;
        ok = hipMemcpy(m->st, &init, sizeof init, hipMemcpyHostToDevice) == hipSuccess;
    }
    if (!ok) {
        emdq_model_free(m);
        return EMDQ_ENOMEM;
    }
    *out = m;
    return EMDQ_OK;
}

void emdq_model_free(emdq_model m) {
    if (!m) return;
    if (m->last) (void)hipStreamSynchronize(m->last);
    (void)hipFree(m->xy);
    (void)hipFree(m->p);
    (void)hipFree(m->mask);
    (void)hipFree(m->e2);
    (void)hipFree(m->q);
    (void)hipFree(m->s);
    (void)hipFree(m->packed);
    (void)hipFree(m->st);
    if (m->host_st) (void)hipHostFree(m->host_st);
    delete m;
}

emdq_status emdq_fit(emdq_model m, const float *src_xy, const float *dst_xy, int n,
                     int frame_w, int frame_h, const emdq_params *params,
                     hipStream_t stream) {
    if (!m || !src_xy || !dst_xy) return EMDQ_EINVAL;
    emdq_params prm;
    if (params) prm = *params; else emdq_params_default(&prm);
    if (!params_ok(prm) || frame_w <= 0 || frame_h <= 0) return EMDQ_EINVAL;
    if (n < 2) return EMDQ_ETOOFEW;
    if (n > m->n_max) return EMDQ_EINVAL;
    m->last = stream;
    m->n = n;
    const double alpha = alpha_d(prm, frame_w, frame_h);
    m->alpha = (float)alpha;
    const float nal2 = -(float)alpha * kLog2e;
    const double u = 1.0 / ((double)frame_w * (double)frame_h);
    const unsigned em_blocks = (unsigned)((n + kRowsPerBlock - 1) / kRowsPerBlock);

    hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, stream, m->st);
    hipLaunchKernelGGL(k_load, dim3((n + 255) / 256), dim3(256), 0, stream,
                       (const float2 *)src_xy, (const float2 *)dst_xy, n, m->xy, m->p, m->mask,
                       m->st);
    if (check_launch() != EMDQ_OK) return EMDQ_EHIP;
    // EM: iterations are enqueued in chunks; every kernel returns at once
    // after the device-side stop flag is set, so a chunk may overshoot.
    int enqueued = 0;
    const int chunk = 4;
    while (true) {
        for (int c = 0; c < chunk && enqueued < prm.max_iter; ++c, ++enqueued) {
            hipLaunchKernelGGL(k_mstep, dim3(em_blocks), dim3(kEmThreads), 0, stream, m->xy,
                               m->p, n, nal2, alpha, m->q, m->s, m->st, 0);
            hipLaunchKernelGGL(k_estep, dim3(em_blocks), dim3(kEmThreads), 0, stream, m->xy,
                               m->p, m->q, m->s, n, nal2, u, (double)prm.sigma2_min,
                               (double)prm.gamma_min, (double)prm.gamma_max, prm.p_thresh,
                               prm.max_iter, m->e2, m->mask, m->st);
        }
        if (check_launch() != EMDQ_OK) return EMDQ_EHIP;
        EMDQ_HIP(hipMemcpyAsync(m->host_st, m->st, sizeof(DevState), hipMemcpyDeviceToHost,
                                stream));
        EMDQ_HIP(hipStreamSynchronize(stream));
        if (m->host_st->done || m->host_st->status < 0 || enqueued >= prm.max_iter) break;
    }
    // final fit with the final posteriors, then pack the inliers
    hipLaunchKernelGGL(k_mstep, dim3(em_blocks), dim3(kEmThreads), 0, stream, m->xy, m->p, n,
                       nal2, alpha, m->q, m->s, m->st, 1);
    hipLaunchKernelGGL(k_compact, dim3(1), dim3(kCompactThreads), 0, stream, m->xy, m->q,
                       m->s, m->mask, n, m->packed, m->st);
    return check_launch();
}

emdq_status emdq_model_set_nodes(emdq_model m, const float *x_xy, const float *scale,
                                 const float *q, const uint8_t *mask, int n, float alpha,
                                 hipStream_t stream) {
    if (!m || !x_xy || !scale || !q || n < 1 || n > m->n_max || !(alpha > 0.f))
        return EMDQ_EINVAL;
    m->last = stream;
    m->n = n;
    m->alpha = alpha;
    float4 *hxy = (float4 *)malloc((size_t)n * sizeof(float4));
    uint8_t *hm = (uint8_t *)malloc((size_t)n);
    if (!hxy || !hm) {
        free(hxy);
        free(hm);
        return EMDQ_ENOMEM;
    }
    for (int i = 0; i < n; ++i) {
        hxy[i] = make_float4(x_xy[2 * i], x_xy[2 * i + 1], 0.f, 0.f);
        hm[i] = mask ? (mask[i] ? 1 : 0) : 1;
    }
    emdq_status rc = EMDQ_OK;
    if (hipMemcpyAsync(m->xy, hxy, (size_t)n * sizeof(float4), hipMemcpyHostToDevice, stream) !=
            hipSuccess ||
        hipMemcpyAsync(m->q, q, (size_t)n * sizeof(float4), hipMemcpyHostToDevice, stream) !=
            hipSuccess ||
        hipMemcpyAsync(m->s, scale, (size_t)n * sizeof(float), hipMemcpyHostToDevice, stream) !=
            hipSuccess ||
        hipMemcpyAsync(m->mask, hm, (size_t)n, hipMemcpyHostToDevice, stream) != hipSuccess)
        rc = EMDQ_EHIP;
    if (rc == EMDQ_OK) {
        hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, stream, m->st);
        hipLaunchKernelGGL(k_compact, dim3(1), dim3(kCompactThreads), 0, stream, m->xy, m->q,
                           m->s, m->mask, n, m->packed, m->st);
        rc = check_launch();
    }
    // the staging buffers are released only after the copies completed
    if (hipStreamSynchronize(stream) != hipSuccess && rc == EMDQ_OK) rc = EMDQ_EHIP;
    free(hxy);
    free(hm);
    return rc;
}

emdq_status emdq_field(emdq_model m, int zx0, int zy0, int w, int h, float *out_xy,
                       hipStream_t stream) {
    if (!m || !out_xy || w < 0 || h < 0) return EMDQ_EINVAL;
    if (w == 0 || h == 0) return EMDQ_OK;
    m->last = stream;
    return launch_field(m, kModeField, zx0, zy0, w, h, (float2 *)out_xy, nullptr, 0, 0, 0,
                        nullptr, 0, 0, 0, stream);
}

emdq_status emdq_warp(emdq_model m, const uint8_t *frame_rgb, int fw, int fh,
                      int frame_pitch_bytes, float *canvas, int cw, int ch,
                      int canvas_pitch_px, int ox, int oy, int zx0, int zy0, int w, int h,
                      hipStream_t stream) {
    if (!m || !frame_rgb || !canvas) return EMDQ_EINVAL;
    if (fw <= 0 || fh <= 0 || cw <= 0 || ch <= 0 || w < 0 || h < 0) return EMDQ_EINVAL;
    if ((long long)frame_pitch_bytes < 3LL * fw || canvas_pitch_px < cw) return EMDQ_EINVAL;
    if (((uintptr_t)canvas & 15u) != 0) return EMDQ_EINVAL;
    if (w == 0 || h == 0) return EMDQ_OK;
    const long long cx0 = (long long)zx0 + ox, cy0 = (long long)zy0 + oy;
    if (cx0 < 0 || cy0 < 0 || cx0 + w > cw || cy0 + h > ch) return EMDQ_EINVAL;
    m->last = stream;
    return launch_field(m, kModeWarp, zx0, zy0, w, h, nullptr, frame_rgb, fw, fh,
                        frame_pitch_bytes, (float4 *)canvas, canvas_pitch_px, ox, oy, stream);
}

emdq_status emdq_model_status(emdq_model m, hipStream_t stream) {
    if (!m) return EMDQ_EINVAL;
    EMDQ_HIP(hipMemcpyAsync(m->host_st, m->st, sizeof(DevState), hipMemcpyDeviceToHost, stream));
    EMDQ_HIP(hipStreamSynchronize(stream));
    return (emdq_status)m->host_st->status;
}

emdq_status emdq_model_results(emdq_model m, float *scale, float *q, float *p, uint8_t *mask,
                               int *n_in, int *iters, float *sigma2, float *gamma,
                               hipStream_t stream) {
    if (!m) return EMDQ_EINVAL;
    const size_t n = (size_t)m->n;
    EMDQ_HIP(hipMemcpyAsync(m->host_st, m->st, sizeof(DevState), hipMemcpyDeviceToHost, stream));
    if (scale) EMDQ_HIP(hipMemcpyAsync(scale, m->s, n * 4, hipMemcpyDeviceToHost, stream));
    if (q) EMDQ_HIP(hipMemcpyAsync(q, m->q, n * 16, hipMemcpyDeviceToHost, stream));
    if (p) EMDQ_HIP(hipMemcpyAsync(p, m->p, n * 4, hipMemcpyDeviceToHost, stream));
    if (mask) EMDQ_HIP(hipMemcpyAsync(mask, m->mask, n, hipMemcpyDeviceToHost, stream));
    EMDQ_HIP(hipStreamSynchronize(stream));
    const DevState &s = *m->host_st;
    if (n_in) *n_in = s.n_in;
    if (iters) *iters = s.iter;
    if (sigma2) *sigma2 = s.sigma2;
    if (gamma) *gamma = s.gamma;
    return (emdq_status)s.status;
}

}  // extern "C"
