// emdq.hip -- EMDQ dense deformation field + warp for the MI355X (gfx950).
//
// Method: H. Zhou and J. Jayender, "Real-time Nonrigid Mosaicking of
// Laparoscopy Images" (arXiv 2103.07414), Sec. II-A (EMDQ), Eqs. (1)-(4),
// (18)-(20), Sec. III-F and Eqs. (23)-(24).  The public contract is
// include/emdq.h.
//
// Kernels
//   k_reset / k_load   model state reset; copy of the matches, finiteness check
//   k_mstep            posterior step of the previous iteration (FP64
//                      fixed-order sums, posteriors, inlier mask), then the
//                      per-match weighted similarity fit (Eqs. (18)-(20)) with
//                      weights exp(-alpha d^2) p_j (Eq. (4)); one wavefront per
//                      match, lanes stride the other matches, two-pass
//                      centred FP32 moments, FP64 re-fit of near-degenerate rows
//   k_estep            stop rule of the previous iteration; DQ blend at every
//                      match (Eqs. (2)-(3)), residuals, per-workgroup sums
//   k_mstep_s, k_estep_s, k_posterior
//                      the same EM in three launches per iteration (above
//                      kFusedMaxN matches): the posterior step and the stop
//                      rule in a one-workgroup kernel of their own
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
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>

#include "emdq.h"

namespace {

constexpr float kLog2e = 1.4426950408889634f;
constexpr int kWave = 64;
constexpr int kRowsPerBlock = 8;        // EM kernels: match rows per workgroup
template <int V> struct IntTag { static constexpr int value = V; };
constexpr int kEmThreads = kWave * kRowsPerBlock;
// E-step: match rows per wavefront (each staged match is read from LDS once
// for all of them), single pair and batch; the same bits either way
#ifndef EMDQ_E_ROWS
#define EMDQ_E_ROWS 1
#endif
#ifndef EMDQ_E_ROWS_BATCH
#define EMDQ_E_ROWS_BATCH 2
#endif
constexpr int e_threads(int rows) { return kWave * kRowsPerBlock / rows; }
constexpr int kEThreads = e_threads(EMDQ_E_ROWS);         // single-pair E-step workgroup
constexpr int kEThreadsB = e_threads(EMDQ_E_ROWS_BATCH);  // batched E-step workgroup
#ifndef EMDQ_MCHUNK
#define EMDQ_MCHUNK 2048
#endif
#ifndef EMDQ_ECHUNK
#define EMDQ_ECHUNK 1024
#endif
#ifndef EMDQ_ECHUNK_BATCH
#define EMDQ_ECHUNK_BATCH 512
#endif
#ifndef EMDQ_MCHUNK_BATCH
#define EMDQ_MCHUNK_BATCH 2048
#endif
#ifndef EMDQ_MSTEP_B_WAVES
#define EMDQ_MSTEP_B_WAVES 0   // batched M-step: wavefronts per SIMD the registers are held to (0: free)
#endif
constexpr int kMChunk = EMDQ_MCHUNK;    // matches staged in LDS per M-step sweep
constexpr int kEChunk = EMDQ_ECHUNK;    // matches (+ fits) staged per E-step sweep, single pair
constexpr int kEChunkB = EMDQ_ECHUNK_BATCH;   // the same, batched E-step (more workgroups per CU)
constexpr int kMChunkB = EMDQ_MCHUNK_BATCH;   // matches staged per batched M-step sweep
constexpr int kCompactThreads = 1024;
constexpr int kFieldThreads = 256;      // 4 wavefronts per workgroup
constexpr int kTile = 32;               // 32 x 32 pixels per MFMA output tile
constexpr int kHTxF = 128, kHTyF = 64;  // workgroup tile of the half-precision blend
constexpr int kBufferFlags = 0x00020000;   // raw buffer resource word 3 (gfx9 family)
#ifndef EMDQ_RING
#define EMDQ_RING 4
#endif
#ifndef EMDQ_SCHED_MASK
#define EMDQ_SCHED_MASK 0   // nothing crosses (measured faster than letting ALU cross)
#endif
#ifndef EMDQ_SPLITK
#define EMDQ_SPLITK 4
#endif

constexpr int kRing = EMDQ_RING;       // field kernel: record ring depth (K steps)
#ifndef EMDQ_FIELD_WAVES
#define EMDQ_FIELD_WAVES 3
#endif
// FP32 field kernel: wavefronts per SIMD the register allocation is held to
// (3 keeps at least two wavefronts on every SIMD through the last partial
// round of tiles; 4 spills)
constexpr int kFieldWaves = EMDQ_FIELD_WAVES;
// wavefronts per SIMD the FP32 field kernel's registers are held to, by row
// blocks per wavefront (two blocks hold 192 accumulators)
constexpr int field_waves(int rb) { return rb == 1 ? kFieldWaves : 2; }
#ifndef EMDQ_HALF_TABLES
#define EMDQ_HALF_TABLES 1  // half-precision blend: factor tables instead of in-loop exps
#endif
#ifndef EMDQ_WARP_BATCH
#define EMDQ_WARP_BATCH 1   // warp epilogue: a lane's pixels merged with batched loads
#endif
#ifndef EMDQ_MSTEP_ONEPASS
#define EMDQ_MSTEP_ONEPASS 1   // M-step: centred moments from one sweep's raw moments (0: a second sweep)
#endif
#ifndef EMDQ_MSTEP_WSHIFT
#define EMDQ_MSTEP_WSHIFT 1   // one-pass M-step: the weight's exponent from the moments' differences
#endif
#ifndef EMDQ_EM_CHUNK
#define EMDQ_EM_CHUNK 2
#endif
// single-pair EM: chunks end where the model's last fit stopped (1) or every
// EMDQ_EM_CHUNK iterations (0)
#ifndef EMDQ_EM_PREDICT
#define EMDQ_EM_PREDICT 1
#endif
constexpr int kEmChunk = EMDQ_EM_CHUNK; // EM iterations enqueued between stop-flag reads
#ifndef EMDQ_START_WGS
#define EMDQ_START_WGS 2048   // batched learned start: workgroups over all pairs
#endif
// learned start: one match per lane (1) or per wavefront (0) in the grid search
#ifndef EMDQ_START_LANE
#define EMDQ_START_LANE 1
#endif
// one match per lane: about this many workgroups for the features of one
// pair (WGS1; the single-pair start keeps one match per wavefront, which
// spreads one pair over more CUs) and for a batch (WGSB)
#ifndef EMDQ_START_LANE_WGS1
#define EMDQ_START_LANE_WGS1 32
#endif
#ifndef EMDQ_START_LANE_WGSB
#define EMDQ_START_LANE_WGSB 512
#endif
#ifndef EMDQ_FUSED_MAX_N
#define EMDQ_FUSED_MAX_N 2048
#endif
// FP32 blend with factor tables: XCD-aware order of the tiles (1) or the
// launch order (0)
#ifndef EMDQ_XCD_MAP
#define EMDQ_XCD_MAP 0
#endif
// single-pair EM: the host waits for a chunk's stop flag by polling its
// sequence number in pinned memory (1) or by an event (0)
#ifndef EMDQ_EM_POLL
#define EMDQ_EM_POLL 1
#endif
// single-pair EM: the state of a chunk's end is published by the next
// chunk's first M-step (1) or by the chunk's last E-step / posterior (0;
// measured as fast or faster at 2000 matches, slightly slower at 4000)
#ifndef EMDQ_PUBLISH_MSTEP
#define EMDQ_PUBLISH_MSTEP 0
#endif
// fused single-pair EM: a speculative compaction after every chunk (measured
// slower: its launches cost more than the host round trip they save)
#ifndef EMDQ_SPEC_COMPACT
#define EMDQ_SPEC_COMPACT 0
#endif
constexpr int kFusedMaxN = EMDQ_FUSED_MAX_N;   // single-pair fits: two launches per iteration up to this n

typedef float f32x16 __attribute__((ext_vector_type(16)));

// Device-side record of the model.  Written by the EM kernels, read by the
// field kernel and, after a stream synchronisation, by the host.
struct DevState {
    int status;      // emdq_status of the fit (0 while running)
    int iter;        // EM iterations done
    int done;        // 1 once the stop rule fired
    int n_in;        // number of packed inliers
    int changed;     // mask changed in the last iteration
    float sigma2;
    float gamma;
    int stop_at;     // single-pair fit: launch that ended the EM (em_stopped), 0 = running
    int packed;      // the inliers are packed (speculative compaction done)
    int fitted;      // batched fit: the final M-step of the stopped pair has run
    int seq;         // host copies only: sequence number of the publishing launch
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

// LDS written by some lanes of a wavefront and read by others of the same
// wavefront: keep the compiler from moving accesses across this point.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ bool finite2(float2 v) {
    return __builtin_isfinite(v.x) && __builtin_isfinite(v.y);
}

// ------------------------------------------------------ state, loading ----

// The state as a launch leaves it, copied into pinned host memory for the
// host's stop-flag reads, then its sequence number (system-scope release):
// the host polls the number, so no event has to be recorded.
__device__ __forceinline__ void publish_state(DevState *host_copy, const DevState *st, int seq) {
    *host_copy = *st;
    __hip_atomic_store(&host_copy->seq, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

__device__ __forceinline__ void reset_state(DevState *st) {
    st->status = 0;
    st->iter = 0;
    st->done = 0;
    st->n_in = 0;
    st->changed = 0;
    st->sigma2 = 0.f;
    st->gamma = 0.f;
    st->stop_at = 0;
    st->packed = 0;
    st->fitted = 0;
    st->seq = 0;
}

// The launches of a single-pair fit, numbered in enqueue order: the load is 1,
// iteration it (from 1) is the M-step 2 it and then the E-step 2 it + 1.  The
// launch that ends the EM stores its own number in stop_at with one 32-bit
// store, so a workgroup of that same launch reads either 0 or the launch's
// own number and carries on; every later launch returns at once.
constexpr int kOrdLoad = 1;
__device__ __forceinline__ bool em_stopped(int stop_at, int ordinal) {
    return stop_at != 0 && stop_at < ordinal;
}

__global__ void k_reset(DevState *st) {
    if (threadIdx.x == 0) reset_state(st);
}

// xy[i] = (src_i, dst_i); p = 1, mask = 1; cent[i] = 0 (the M-step's
// moment origin starts at the match itself); a non-finite coordinate sets
// the status to ENONFINITE (every writer stores the same value).
__device__ __forceinline__ void load_body(const float2 *__restrict__ src, const float2 *__restrict__ dst, int n,
                       float4 *__restrict__ xy, float *__restrict__ p,
                       uint8_t *__restrict__ mask, float4 *__restrict__ cent, DevState *st,
                       int block) {
    int i = block * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float2 a = src[i], b = dst[i];
    xy[i] = make_float4(a.x, a.y, b.x, b.y);
    p[i] = 1.f;
    mask[i] = 1;
    cent[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    if (!finite2(a) || !finite2(b)) {
        atomicMin(&st->status, (int)EMDQ_ENONFINITE);
        atomicExch(&st->done, 1);
        atomicExch(&st->stop_at, kOrdLoad);
    }
}

__global__ void k_load(const float2 *__restrict__ src, const float2 *__restrict__ dst, int n,
                       float4 *__restrict__ xy, float *__restrict__ p,
                       uint8_t *__restrict__ mask, float4 *__restrict__ cent, DevState *st) {
    load_body(src, dst, n, xy, p, mask, cent, st, blockIdx.x);
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
// Contraction is off in the EM arithmetic and in this function: every fused
// multiply-add is written out, so each kernel that inlines the code rounds
// exactly alike (batched and single-pair fits agree bit for bit).
__device__ __forceinline__ float2 blend_displacement(float W, float Cd, float Sn, float X, float Y,
                                                     float Gd, float zx, float zy) {
#pragma clang fp contract(off)
    const float iW = 1.f / W;
    const float c = __builtin_fmaf(Cd, iW, 1.f), sn = Sn * iW, x = X * iW, y = Y * iW,
                sg = Gd * iW;
    const float in2 = 1.f / __builtin_fmaf(c, c, sn * sn);
    const float r00 = -2.f * sn * sn * in2, r10 = 2.f * c * sn * in2;
    const float tx = 2.f * __builtin_fmaf(c, x, -(sn * y)) * in2,
                ty = 2.f * __builtin_fmaf(c, y, sn * x) * in2;
    const float s1 = 1.f + sg;
    return make_float2(
        __builtin_fmaf(sg, zx, s1 * (__builtin_fmaf(r00, zx, -(r10 * zy)) + tx)),
        __builtin_fmaf(sg, zy, s1 * (__builtin_fmaf(r10, zx, r00 * zy) + ty)));
}
// blend_displacement for the dense field's epilogue: the two divisions by
// hardware reciprocals (about 1 ulp; a relative error of ~1e-7 in the
// displacement, against the 1e-3 px bar), one instruction each instead of an
// IEEE division.  The EM keeps the divisions, so its residuals and the mask
// decisions are unchanged.
__device__ __forceinline__ float2 blend_displacement_field(float W, float Cd, float Sn, float X, float Y,
                                                     float Gd, float zx, float zy) {
#pragma clang fp contract(off)
    const float iW = __builtin_amdgcn_rcpf(W);
    const float c = __builtin_fmaf(Cd, iW, 1.f), sn = Sn * iW, x = X * iW, y = Y * iW,
                sg = Gd * iW;
    const float in2 = __builtin_amdgcn_rcpf(__builtin_fmaf(c, c, sn * sn));
    const float r00 = -2.f * sn * sn * in2, r10 = 2.f * c * sn * in2;
    const float tx = 2.f * __builtin_fmaf(c, x, -(sn * y)) * in2,
                ty = 2.f * __builtin_fmaf(c, y, sn * x) * in2;
    const float s1 = 1.f + sg;
    return make_float2(
        __builtin_fmaf(sg, zx, s1 * (__builtin_fmaf(r00, zx, -(r10 * zy)) + tx)),
        __builtin_fmaf(sg, zy, s1 * (__builtin_fmaf(r10, zx, r00 * zy) + ty)));
}

// ------------------------------------------------------------ posterior ----
//
// Gaussian-inlier / uniform-outlier mixture of Sec. II-A.  Each E-step
// workgroup leaves, for its rows, the FP64 sums (sum p_i, sum p_i e_i^2) in
// row order; partial_run and combine_partials add them over the workgroups
// in a fixed order, so every workgroup that finishes the iteration gets the
// same sigma^2 and gamma and hence the same posteriors.

struct PostParams {
    double u, sigma2_min, gamma_min, gamma_max;
    float p_thresh;
    int max_iter;
};

// p = a / (a + b), a = gamma exp(-e^2 / (2 sigma^2)) / (2 pi sigma^2),
// b = (1 - gamma) u (FP64)
// and, in FP32, p = 1 / (1 + 2^(e^2 s + l)) with s = log2(e) / (2 sigma^2),
// l = log2(b (2 pi sigma^2) / gamma); th = p_thresh
struct PostCoef {
    double gamma, inv2s, norm, b;
    float s, l, th;
};

// Half-width of the band around p_thresh in which the FP32 posterior is
// replaced by the FP64 one.  The FP32 form is off by less than 1e-5 (the
// exponent's rounding over |e^2 s| <= 150 and the 1-ulp exp2), so outside
// the band both forms fall on the same side of the threshold.
constexpr float kPostBand = 1e-3f;

// Every FP64 operation of the posterior step is rounded on its own
// (contraction off), so the kernels that inline it agree bit for bit.
__device__ __forceinline__ float post_p64(float e2, const PostCoef &c) {
#pragma clang fp contract(off)
    const double a = c.gamma * exp(-(double)e2 * c.inv2s) * c.norm;
    return (float)(a / (a + c.b));
}

// The posterior of a match: the FP32 form, or the FP64 one inside the band
// around p_thresh, so that the inlier mask is always decided as in FP64.
__device__ __forceinline__ float post_p(float e2, const PostCoef &c) {
#pragma clang fp contract(off)
    const float p = 1.f / (1.f + fast_exp2(__builtin_fmaf(e2, c.s, c.l)));
    return fabsf(p - c.th) > kPostBand ? p : post_p64(e2, c);
}

// Fixed-order sum of the E-step partials part[0, nb): thread t < kEmThreads
// adds part[t], part[t + kEmThreads], ... (partial_run); a butterfly per
// wavefront; then the first kRowsPerBlock wavefronts in order
// (combine_partials).  Every thread of a workgroup of at least kEmThreads
// threads calls both and gets the same bits, whichever workgroup and kernel
// it runs in.
// first: part[min(t, nb - 1)], loaded by the caller (so that the load can be
// issued early, unconditionally and in bounds)
__device__ __forceinline__ double2 partial_run(const double2 *__restrict__ part, int nb,
                                               double2 first) {
    const int t = threadIdx.x;
    double2 r = make_double2(0.0, 0.0);
    if (t < kEmThreads && t < nb) {
        r = first;   // 0 + part[t], exactly (the sums are not negative)
        for (int b = t + kEmThreads; b < nb; b += kEmThreads) {
            const double2 v = part[b];
            r.x += v.x;
            r.y += v.y;
        }
    }
    return r;
}

__device__ __forceinline__ double2 combine_partials(double2 run) {
    __shared__ double2 s_w[kRowsPerBlock];
    const int t = threadIdx.x;
    const double sp = wave_sum_d(run.x), spe = wave_sum_d(run.y);
    if (t < kEmThreads && (t & (kWave - 1)) == 0) s_w[t / kWave] = make_double2(sp, spe);
    __syncthreads();
    double2 r = s_w[0];
    for (int w = 1; w < kRowsPerBlock; ++w) {
        r.x += s_w[w].x;
        r.y += s_w[w].y;
    }
    return r;
}

// sigma^2 and gamma from the sums (clamped as the parameters say) and the
// posterior coefficients; false if no posterior weight is left.
__device__ __forceinline__ bool post_coef(double2 S, int n, const PostParams &pp,
                                          double *sigma2_out, PostCoef *c) {
#pragma clang fp contract(off)
    if (!(S.x > 0.0)) return false;
    double sigma2 = S.y / (2.0 * S.x);
    if (!(sigma2 >= pp.sigma2_min)) sigma2 = pp.sigma2_min;
    double gamma = S.x / (double)n;
    gamma = gamma < pp.gamma_min ? pp.gamma_min : (gamma > pp.gamma_max ? pp.gamma_max : gamma);
    c->gamma = gamma;
    c->inv2s = 1.0 / (2.0 * sigma2);
    c->norm = 1.0 / (6.283185307179586 * sigma2);
    c->b = (1.0 - gamma) * pp.u;
    c->s = (float)(c->inv2s * 1.4426950408889634);
    c->l = (float)log2(c->b / (c->gamma * c->norm));
    c->th = pp.p_thresh;
    *sigma2_out = sigma2;
    return true;
}

// The stop rule after the posteriors of iteration it: no mask change from
// the iteration before (from the second iteration on), or max_iter reached.
// Returns 0 (go on), 1 (converged) or 2 (not converged by max_iter).
__device__ __forceinline__ int stop_rule(int it, int any_changed, int max_iter) {
    if (it >= 2 && !any_changed) return 1;
    return it >= max_iter ? 2 : 0;
}

// --------------------------------------------------------------- M-step ----

// Planar DQ from the half-angle direction (ch, sh) and the translation.
__device__ __forceinline__ float4 dq_make(float ch, float sh, float tx, float ty) {
#pragma clang fp contract(off)
    return make_float4(ch, sh, 0.5f * __builtin_fmaf(ch, tx, sh * ty),
                       0.5f * __builtin_fmaf(ch, ty, -(sh * tx)));
}

// FP64 fit of one match, taken when the FP32 moments are too ill-conditioned
// to decide the degenerate case: two-pass centred sums over all matches,
// spread over the lanes of the wavefront.  p(j) gives the posterior of match j.
template <class PostOf>
__device__ void fit_row_f64(int i, const float4 *__restrict__ xy, const PostOf &p,
                            int n, double alpha, int lane, float *scale_out, float4 *q_out) {
#pragma clang fp contract(off)
    const float4 me = xy[i];
    double S = 0, ax = 0, ay = 0, bx = 0, by = 0;
    for (int j = lane; j < n; j += kWave) {
        float4 v = xy[j];
        double dx = (double)v.x - me.x, dy = (double)v.y - me.y;
        double w = exp(-alpha * (dx * dx + dy * dy)) * (double)p(j);
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
        double w = exp(-alpha * (dx * dx + dy * dy)) * (double)p(j);
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

// How an EM kernel runs.  kEmBatch: pairs of a batch; the stop flag is read
// first, so a pair that has stopped costs no loads.  kEmSingle: one pair,
// three launches per iteration (M-step, E-step, posterior kernel).
// kEmFused: one pair, two launches per iteration (below).  Both single-pair
// modes issue their first loads before they wait on the stop flag.
enum EmMode { kEmBatch = 0, kEmSingle = 1, kEmFused = 2 };

// A fused single-pair fit finishes the previous iteration at the start of its
// M-step (so an EM iteration is two launches): every workgroup sums the
// E-step partials, forms sigma^2, gamma and the posteriors of all matches
// (the same bits in every workgroup) and uses them as its weights; it stores
// the posteriors and the mask of its own rows and whether any of those mask
// bits changed.  The next E-step applies the stop rule from those flags.
struct EmFused {
    const float *e2;        // residuals of the previous E-step
    const double2 *part;    // its per-workgroup sums (sum p, sum p e^2)
    float *p_out;           // posteriors (own rows stored)
    uint8_t *mask;          // inlier mask (own rows stored)
    int *chg;               // per workgroup: a mask bit of its rows changed
    PostParams pp;
    int nb;                 // workgroups of the EM launches
    int it;                 // this iteration (from 1); posteriors of it - 1
    DevState *host_copy;    // pinned host memory or null: the state as the launch finds it
    int seq;                // sequence number published with host_copy
};

// One wavefront per match i: weights w_j = exp(-alpha |x_j - x_i|^2) p_j.
// The workgroup stages the matches in LDS (coalesced, kMChunk at a time) and
// each wavefront sweeps them from there once, accumulating the weight sum and
// the weighted first and second moments (spreads and the two cross terms of
// the 2D Procrustes fit) relative to an origin o; the centred moments follow
// as raw - S (mean - o)^2.  o is the match shifted by its weighted centroids
// of the previous M-step (cent, zeroed when a fit starts), so mean - o is the
// centroid's move in one iteration and the subtraction loses nothing that
// matters (measured: fits as close to the FP64 oracle as with a second sweep;
// with o = x_i, matches whose neighbours lie far to one side lost up to 50x).
// Rows whose centred spread is below 1e-2 px^2 of the weight are refitted in
// FP64.  (EMDQ_MSTEP_ONEPASS 0: a second sweep forms the centred moments.)
// Then the closed-form 2D Procrustes fit.  kEmFused: the posterior step first
// (EmFused); otherwise the posteriors are read from p.
template <int kMode, int kMChunk = ::kMChunk>
__device__ __forceinline__ void mstep_body(
    const float4 *__restrict__ xy, const float *p, int n, float nal2,
    double alpha, float4 *__restrict__ q_out, float *__restrict__ s_out,
    float4 *__restrict__ cent, DevState *st, int final_pass, const EmFused &F, int block) {
#pragma clang fp contract(off)
    __shared__ float4 s_xy[kMChunk];
    __shared__ float s_p[kMChunk];
    if (kMode == kEmBatch) {
        // a stopped pair's final fit is the first M-step after its stop (the
        // same inputs as a pass after the last iteration, so the same bits);
        // the posterior step that follows it marks the pair fitted
        if (st->status < 0 || st->fitted) return;
    }
    const int lane = threadIdx.x & (kWave - 1);
    const int i = block * kRowsPerBlock + (threadIdx.x >> 6);
    const bool active = i < n;
    const bool post = kMode == kEmFused && F.it >= 2;   // posteriors from F.e2 instead of p
    // staging: a chunk's loads into registers, then (posteriors formed) LDS
    constexpr int kPer = kMChunk / kEmThreads;
    float4 v[kPer];
    float r[kPer];   // e2 (post) or p of the staged matches
    auto load_chunk = [&](int c0, int cn) {
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const int t = threadIdx.x + k * kEmThreads;
            if (t < cn) {
                v[k] = xy[c0 + t];
                r[k] = post ? F.e2[c0 + t] : p[c0 + t];
            } else {
                v[k] = make_float4(0.f, 0.f, 0.f, 0.f);
                r[k] = 0.f;
            }
        }
    };
    PostCoef pc{};
    // fused mode: whether a mask bit of the workgroup's rows changed, OR-ed
    // over the workgroup by the first staging barrier
    int changed = 0;
    bool first_stage = true;
    auto store_chunk = [&](int cn) {
        float pv[kPer];
#pragma unroll
        for (int k = 0; k < kPer; ++k) pv[k] = post ? post_p(r[k], pc) : r[k];
        if (kMode == kEmFused && first_stage) {
            const int any = __syncthreads_or(changed);
            if (post && threadIdx.x == 0) F.chg[block] = any;
        } else {
            __syncthreads();
        }
        first_stage = false;
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const int t = threadIdx.x + k * kEmThreads;
            if (t < cn) { s_xy[t] = v[k]; s_p[t] = pv[k]; }
        }
        __syncthreads();
    };
    // single pair: every load of the first chunk (and of the posterior step)
    // is issued, unconditionally and in bounds, before the stop flag (loaded
    // last, so that one wait covers them all); the posterior loads are unused
    // when it = 1
    const float4 me = active ? xy[i] : make_float4(0.f, 0.f, 0.f, 0.f);
    // moment origin: the match shifted by its weighted centroids of the
    // previous M-step (zero at the first), so the centred moments lose
    // nothing to cancellation
    const float4 sh = EMDQ_MSTEP_ONEPASS && active ? cent[i] : make_float4(0.f, 0.f, 0.f, 0.f);
    const float4 o = make_float4(me.x + sh.x, me.y + sh.y, me.z + sh.z, me.w + sh.w);
    // One pass: the weight's exponent from the moments' differences
    // d = x_j - o, as nal2 |x_j - x_i|^2 = nal2 |d|^2 + 2 nal2 (o - x_i).d +
    // nal2 |o - x_i|^2 (o - x_i as the rounded o realises it; zero at the
    // first M-step, where this is nal2 |x_j - x_i|^2 itself).
    constexpr bool kShiftW = EMDQ_MSTEP_ONEPASS && EMDQ_MSTEP_WSHIFT;
    const float ox = o.x - me.x, oy = o.y - me.y;
    const float k1x = 2.f * nal2 * ox, k1y = 2.f * nal2 * oy;
    const float k0 = nal2 * __builtin_fmaf(ox, ox, oy * oy);
    double2 run = make_double2(0.0, 0.0);
    float e2_own = 0.f;
    uint8_t m_old = 0;
    if (kMode == kEmFused) {
        const double2 first = F.part[min((int)threadIdx.x, F.nb - 1)];
        const int ic = min(i, n - 1);
        e2_own = F.e2[ic];
        m_old = F.mask[ic];
        load_chunk(0, min(kMChunk, n));
        const int stop = __atomic_load_n(&st->stop_at, __ATOMIC_RELAXED);
        if (F.host_copy && block == 0 && threadIdx.x == 0) publish_state(F.host_copy, st, F.seq);
        if (em_stopped(stop, 2 * F.it)) return;
        if (post) run = partial_run(F.part, F.nb, first);
    } else if (kMode == kEmSingle) {
        load_chunk(0, min(kMChunk, n));
        const int status = st->status, done = st->done;
        if (F.host_copy && block == 0 && threadIdx.x == 0) publish_state(F.host_copy, st, F.seq);
        if (status < 0 || (!final_pass && done)) return;
    }
    if (post) {
        double sigma2;
        if (!post_coef(combine_partials(run), n, F.pp, &sigma2, &pc)) {
            if (block == 0 && threadIdx.x == 0) {
                st->status = EMDQ_ENOINLIERS;
                st->done = 1;
                st->stop_at = 2 * F.it;
            }
            return;
        }
        if (block == 0 && threadIdx.x == 0) {
            st->sigma2 = (float)sigma2;
            st->gamma = (float)pc.gamma;
        }
        if (active && lane == 0) {
            const float pn = post_p(e2_own, pc);
            const uint8_t m = pn > F.pp.p_thresh ? 1 : 0;
            changed = m != m_old;
            F.p_out[i] = pn;
            F.mask[i] = m;
        }
    }
    auto post_of = [&](int j) { return post ? post_p(F.e2[j], pc) : p[j]; };
    const bool resident = n <= kMChunk;   // one staging serves both passes
    bool preloaded = kMode != kEmBatch;   // the first chunk's registers are loaded already
    auto stage = [&](int c0, int cn) {
        if (!preloaded) load_chunk(c0, cn);
        store_chunk(cn);
        // the next chunk's loads go out now (its registers are free once
        // this chunk is in LDS) and land during this chunk's sweep
        if (c0 + kMChunk < n) load_chunk(c0 + kMChunk, min(kMChunk, n - c0 - kMChunk));
        preloaded = true;
    };

    // Fused mode (n <= kMChunk, so the matches are staged once): the first
    // pass keeps every weight in LDS and the second reads it back instead of
    // recomputing it (the same float either way).
    constexpr bool kKeepW = kMode == kEmFused && !EMDQ_MSTEP_ONEPASS;
    static_assert(!kKeepW || kFusedMaxN <= kMChunk, "fused M-step stages all matches once");
    __shared__ float s_w[kKeepW ? kRowsPerBlock * kMChunk : 1];
    float *const wrow = s_w + (kKeepW ? (threadIdx.x >> 6) * kMChunk : 0);
    auto weight = [&](const float4 &v, float pj) {
#pragma clang fp contract(off)
        const float dxx = v.x - me.x, dxy = v.y - me.y;   // x_j - x_i
        return fast_exp2(nal2 * __builtin_fmaf(dxx, dxx, dxy * dxy)) * pj;
    };
    float S = 0.f, Ax = 0.f, Ay = 0.f, Bx = 0.f, By = 0.f;
    float Pxx = 0.f, Pyy = 0.f, Pa = 0.f, Pb = 0.f;   // raw second moments (one pass)
    for (int c0 = 0; c0 < n; c0 += kMChunk) {
        const int cn = min(kMChunk, n - c0);
        stage(c0, cn);
        if (active) {
            auto acc1 = [&](const float4 &v, float pj, int t) {
#pragma clang fp contract(off)
                const float dxx = v.x - o.x, dxy = v.y - o.y;   // x_j - origin
                const float dyx = v.z - o.z, dyy = v.w - o.w;   // y_j - origin
                const float r2 = __builtin_fmaf(dxx, dxx, dxy * dxy);
                const float w =
                    kShiftW ? fast_exp2(__builtin_fmaf(
                                  nal2, r2, __builtin_fmaf(k1x, dxx, __builtin_fmaf(k1y, dxy, k0)))) *
                                  pj
                            : weight(v, pj);
                if (kKeepW) wrow[t] = w;
                S += w;
                Ax = __builtin_fmaf(w, dxx, Ax);
                Ay = __builtin_fmaf(w, dxy, Ay);
                Bx = __builtin_fmaf(w, dyx, Bx);
                By = __builtin_fmaf(w, dyy, By);
                if constexpr (EMDQ_MSTEP_ONEPASS) {
                    Pxx = __builtin_fmaf(w, r2, Pxx);
                    Pyy = __builtin_fmaf(w, __builtin_fmaf(dyx, dyx, dyy * dyy), Pyy);
                    Pa = __builtin_fmaf(w, __builtin_fmaf(dyx, dxx, dyy * dxy), Pa);
                    Pb = __builtin_fmaf(w, __builtin_fmaf(dyy, dxx, -(dyx * dxy)), Pb);
                }
            };
            int t = lane;
            for (; t + 3 * kWave < cn; t += 4 * kWave) {   // 4 LDS reads in flight
                const float4 v0 = s_xy[t], v1 = s_xy[t + kWave], v2 = s_xy[t + 2 * kWave],
                             v3 = s_xy[t + 3 * kWave];
                const float p0 = s_p[t], p1 = s_p[t + kWave], p2 = s_p[t + 2 * kWave],
                            p3 = s_p[t + 3 * kWave];
                acc1(v0, p0, t);
                acc1(v1, p1, t + kWave);
                acc1(v2, p2, t + 2 * kWave);
                acc1(v3, p3, t + 3 * kWave);
            }
            for (; t < cn; t += kWave) acc1(s_xy[t], s_p[t], t);
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
    const float cxx = o.x + mx, cxy = o.y + my, cyx = o.z + nx, cyy = o.w + ny;
    if constexpr (EMDQ_MSTEP_ONEPASS) {
        // centred moments from the raw ones: sum w (d - m)(e - n) = P - S m n
        Pxx = wave_sum(Pxx);
        Pyy = wave_sum(Pyy);
        Pa = wave_sum(Pa);
        Pb = wave_sum(Pb);
        if (have_w) {
            vx = Pxx - S * __builtin_fmaf(mx, mx, my * my);
            vy = Pyy - S * __builtin_fmaf(nx, nx, ny * ny);
            a = Pa - S * __builtin_fmaf(nx, mx, ny * my);
            b = Pb - S * __builtin_fmaf(ny, mx, -(nx * my));
        }
    }
    if (!resident) preloaded = false;   // the second sweep restages from the first chunk
    for (int c0 = 0; EMDQ_MSTEP_ONEPASS == 0 && c0 < n; c0 += kMChunk) {
        const int cn = min(kMChunk, n - c0);
        if (!resident) stage(c0, cn);
        if (active && have_w) {
            auto acc2 = [&](const float4 &v, float pj, int t) {
#pragma clang fp contract(off)
                const float w = kKeepW ? wrow[t] : weight(v, pj);
                const float ax = v.x - cxx, ay = v.y - cxy;    // x_j - xbar
                const float bx = v.z - cyx, by = v.w - cyy;    // y_j - ybar
                vx = __builtin_fmaf(w, __builtin_fmaf(ax, ax, ay * ay), vx);
                vy = __builtin_fmaf(w, __builtin_fmaf(bx, bx, by * by), vy);
                a = __builtin_fmaf(w, __builtin_fmaf(bx, ax, by * ay), a);      // C00 + C11
                b = __builtin_fmaf(w, __builtin_fmaf(by, ax, -(bx * ay)), b);   // C10 - C01
            };
            int t = lane;
            for (; t + 3 * kWave < cn; t += 4 * kWave) {
                const float4 v0 = s_xy[t], v1 = s_xy[t + kWave], v2 = s_xy[t + 2 * kWave],
                             v3 = s_xy[t + 3 * kWave];
                const float p0 = kKeepW ? 0.f : s_p[t], p1 = kKeepW ? 0.f : s_p[t + kWave],
                            p2 = kKeepW ? 0.f : s_p[t + 2 * kWave],
                            p3 = kKeepW ? 0.f : s_p[t + 3 * kWave];
                acc2(v0, p0, t);
                acc2(v1, p1, t + kWave);
                acc2(v2, p2, t + 2 * kWave);
                acc2(v3, p3, t + 3 * kWave);
            }
            for (; t < cn; t += kWave) acc2(s_xy[t], kKeepW ? 0.f : s_p[t], t);
        }
    }
    if (!active) return;
    if constexpr (!EMDQ_MSTEP_ONEPASS) {
        vx = wave_sum(vx);
        vy = wave_sum(vy);
        a = wave_sum(a);
        b = wave_sum(b);
    }

    float scale;
    float4 q;
    // no weight, or a near-degenerate spread (below 1e-2 px^2): decide and
    // fit in FP64
    const bool need_f64 = !have_w || !(vx > 1e-2f * S) || !(vy > 1e-2f * S);
    if (need_f64) {
        fit_row_f64(i, xy, post_of, n, alpha, lane, &scale, &q);
    } else {
        const float r = sqrtf(__builtin_fmaf(a, a, b * b));
        float ct = 1.f, stt = 0.f, ch = 1.f, sh = 0.f;
        if (r > 0.f) {
            ct = a / r;
            stt = b / r;
            float hx, hy;
            if (a >= 0.f) { hx = r + a; hy = b; }
            else { const float sg = b < 0.f ? -1.f : 1.f; hx = sg * b; hy = sg * (r - a); }
            const float hn = sqrtf(__builtin_fmaf(hx, hx, hy * hy));
            ch = hx / hn;
            sh = hy / hn;
        }
        scale = sqrtf(vy / vx);
        const float cx = o.x + mx, cy = o.y + my;       // weighted centroid of x
        const float gx = o.z + nx, gy = o.w + ny;       // weighted centroid of y
        const float tx = gx / scale - __builtin_fmaf(ct, cx, -(stt * cy));
        const float ty = gy / scale - __builtin_fmaf(stt, cx, ct * cy);
        q = dq_make(ch, sh, tx, ty);
    }
    if (lane == 0) {
        q_out[i] = q;
        s_out[i] = scale;
        if (EMDQ_MSTEP_ONEPASS)   // the next M-step's moment origin
            cent[i] = make_float4(sh.x + mx, sh.y + my, sh.z + nx, sh.w + ny);
    }
}

__global__ __launch_bounds__(kEmThreads) void k_mstep(
    const float4 *__restrict__ xy, const float *p, int n, float nal2, double alpha,
    float4 *__restrict__ q_out, float *__restrict__ s_out, float4 *__restrict__ cent,
    DevState *st, EmFused F) {
    mstep_body<kEmFused>(xy, p, n, nal2, alpha, q_out, s_out, cent, st, 0, F, blockIdx.x);
}

__global__ __launch_bounds__(kEmThreads) void k_mstep_s(
    const float4 *__restrict__ xy, const float *p, int n, float nal2, double alpha,
    float4 *__restrict__ q_out, float *__restrict__ s_out, float4 *__restrict__ cent,
    DevState *st, int final_pass, DevState *host_copy, int seq) {
    EmFused F{};
    F.host_copy = host_copy;
    F.seq = seq;
    mstep_body<kEmSingle>(xy, p, n, nal2, alpha, q_out, s_out, cent, st, final_pass, F,
                          blockIdx.x);
}

// --------------------------------------------------------------- E-step ----

// The stop decision of a single-pair fit, taken by the E-step of iteration
// it for iteration it - 1 from the M-step's per-workgroup flags.
struct EmStop {
    const int *chg;         // per M-step workgroup: a mask bit changed
    DevState *host_copy;    // pinned host memory or null: the state as the launch leaves it
    int max_iter;
    int it;                 // this iteration (from 1)
    int seq;                // sequence number published with host_copy
};

// Blend of all fits at match i with weights exp(-alpha d^2) p_j (Eqs. (2)-(3)),
// normalisation, prediction y_hat = s (R x_i + t) (Eq. (1)), residual e_i^2.
// The workgroup also leaves (sum p_i, sum p_i e_i^2) over its rows, in row
// order, in part[block].  kEmFused: first the stop rule (EmStop).  Each
// wavefront takes kERows consecutive rows (a workgroup of e_threads(kERows));
// kChunk matches (and fits) are staged in LDS per sweep.
template <int kMode, int kERows, int kChunk>
__device__ __forceinline__ void estep_body(
    const float4 *__restrict__ xy, const float *__restrict__ p, const float4 *__restrict__ q,
    const float *__restrict__ s, int n, float nal2, float *__restrict__ e2,
    double2 *__restrict__ part, int nb, DevState *st, const EmStop &stp, int block) {
#pragma clang fp contract(off)
    constexpr int kEThreads = e_threads(kERows);
    static_assert(kRowsPerBlock % kERows == 0 && kChunk % kEThreads == 0,
                  "whole rows per wavefront, whole staging rounds");
    __shared__ float4 s_xy[kChunk];
    __shared__ float4 s_q[kChunk];
    __shared__ float2 s_ps[kChunk];   // (p_j, s_j - 1)
    __shared__ double2 s_part[kRowsPerBlock];
    if (kMode == kEmBatch && (st->status < 0 || st->done)) return;
    const int lane = threadIdx.x & (kWave - 1);
    // the wavefront's rows i0, i0 + 1, ..., i0 + kERows - 1 (consecutive, so
    // the first is active if any is)
    const int i0 = block * kRowsPerBlock + (threadIdx.x >> 6) * kERows;
    const bool active = i0 < n;
    // staging: a chunk's loads into registers, then LDS
    constexpr int kPer = kChunk / kEThreads;
    float4 v[kPer], qv[kPer];
    float pv[kPer], sv[kPer];
    auto load_chunk = [&](int c0, int cn) {
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const int t = threadIdx.x + k * kEThreads;
            if (t < cn) {
                v[k] = xy[c0 + t];
                qv[k] = q[c0 + t];
                pv[k] = p[c0 + t];
                sv[k] = s[c0 + t];
            } else {
                v[k] = make_float4(0.f, 0.f, 0.f, 0.f);
                qv[k] = make_float4(0.f, 0.f, 0.f, 0.f);
                pv[k] = 0.f;
                sv[k] = 0.f;
            }
        }
    };
    auto store_chunk = [&](int cn) {
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const int t = threadIdx.x + k * kEThreads;
            if (t < cn) { s_xy[t] = v[k]; s_q[t] = qv[k]; s_ps[t] = make_float2(pv[k], sv[k] - 1.f); }
        }
        __syncthreads();
    };
    float4 me[kERows];
    float p_own[kERows];   // unconditional, in bounds; used if the row is active
#pragma unroll
    for (int r = 0; r < kERows; ++r) {
        me[r] = i0 + r < n ? xy[i0 + r] : make_float4(0.f, 0.f, 0.f, 0.f);
        p_own[r] = p[min(i0 + r, n - 1)];
    }
    if (kMode == kEmSingle) {
        // the first chunk's loads are issued before the stop flag's
        load_chunk(0, min(kChunk, n));
        const int status = st->status, done = st->done;
        if (status < 0 || done) return;
    } else if (kMode == kEmFused) {
        // every load of the first chunk and of the stop rule is issued before
        // the stop flag is waited on (all in bounds)
        // chg[min(t, nb - 1)] is one of the flags, so OR-ing it is harmless;
        // loaded unconditionally (unused when it = 1), the stop flag last
        const int chg0 = stp.chg[min((int)threadIdx.x, nb - 1)];
        load_chunk(0, min(kChunk, n));
        const int stop = __atomic_load_n(&st->stop_at, __ATOMIC_RELAXED);
        int any = stp.it >= 2 ? chg0 : 0;
        const bool lead = block == 0 && threadIdx.x == 0;
        auto publish = [&]() {
            if (lead && stp.host_copy) publish_state(stp.host_copy, st, stp.seq);
        };
        if (em_stopped(stop, 2 * stp.it + 1)) {
            publish();
            return;
        }
        if (stp.it >= 2) {   // the M-step before formed the posteriors of it - 1
            for (int b = threadIdx.x + kEThreads; b < nb; b += kEThreads) any |= stp.chg[b];
            any = __syncthreads_or(any);
            const int rule = stop_rule(stp.it - 1, any, stp.max_iter);
            if (lead) {
                st->iter = stp.it - 1;
                st->changed = any;
                if (rule) {
                    st->done = 1;
                    if (rule == 2) st->status = EMDQ_WARN_NOT_CONVERGED;
                    st->stop_at = 2 * stp.it + 1;
                }
            }
            if (rule) {
                publish();
                return;
            }
        }
        publish();   // nothing below changes the state
    }
    bool preloaded = kMode != kEmBatch;   // the first chunk's registers are loaded already
    float W[kERows], Gd[kERows], Cd[kERows], Sn[kERows], X[kERows], Y[kERows];
#pragma unroll
    for (int r = 0; r < kERows; ++r) W[r] = Gd[r] = Cd[r] = Sn[r] = X[r] = Y[r] = 0.f;
    for (int c0 = 0; c0 < n; c0 += kChunk) {
        const int cn = min(kChunk, n - c0);
        if (!preloaded) load_chunk(c0, cn);
        store_chunk(cn);
        // the next chunk's loads go out now (its registers are free once
        // this chunk is in LDS) and land during this chunk's sweep
        if (c0 + kChunk < n) load_chunk(c0 + kChunk, min(kChunk, n - c0 - kChunk));
        preloaded = true;
        if (active) {
            auto acc1 = [&](const float4 &v, const float2 &ps, const float4 &qj) {
#pragma clang fp contract(off)
                const float qc = qj.x - 1.f;
#pragma unroll
                for (int r = 0; r < kERows; ++r) {
                    const float dx = v.x - me[r].x, dy = v.y - me[r].y;
                    const float w = fast_exp2(nal2 * __builtin_fmaf(dx, dx, dy * dy)) * ps.x;
                    W[r] += w;
                    Gd[r] = __builtin_fmaf(w, ps.y, Gd[r]);
                    Cd[r] = __builtin_fmaf(w, qc, Cd[r]);
                    Sn[r] = __builtin_fmaf(w, qj.y, Sn[r]);
                    X[r] = __builtin_fmaf(w, qj.z, X[r]);
                    Y[r] = __builtin_fmaf(w, qj.w, Y[r]);
                }
            };
            int t = lane;
            for (; t + 3 * kWave < cn; t += 4 * kWave) {   // 4 LDS reads in flight
                const float4 v0 = s_xy[t], v1 = s_xy[t + kWave], v2 = s_xy[t + 2 * kWave],
                             v3 = s_xy[t + 3 * kWave];
                const float2 a0 = s_ps[t], a1 = s_ps[t + kWave], a2 = s_ps[t + 2 * kWave],
                             a3 = s_ps[t + 3 * kWave];
                const float4 q0 = s_q[t], q1 = s_q[t + kWave], q2 = s_q[t + 2 * kWave],
                             q3 = s_q[t + 3 * kWave];
                acc1(v0, a0, q0);
                acc1(v1, a1, q1);
                acc1(v2, a2, q2);
                acc1(v3, a3, q3);
            }
            for (; t < cn; t += kWave) acc1(s_xy[t], s_ps[t], s_q[t]);
        }
    }
#pragma unroll
    for (int r = 0; r < kERows; ++r) {
        const int i = i0 + r;
        double2 mine = make_double2(0.0, 0.0);
        if (i < n) {
            const float Wr = wave_sum(W[r]), Gr = wave_sum(Gd[r]), Cr = wave_sum(Cd[r]);
            const float Sr = wave_sum(Sn[r]), Xr = wave_sum(X[r]), Yr = wave_sum(Y[r]);
            float err = __builtin_huge_valf();
            if (Wr > 0.f) {
                // e = y_i - F(x_i) = (y_i - x_i) - D(x_i)
                const float2 d = blend_displacement(Wr, Cr, Sr, Xr, Yr, Gr, me[r].x, me[r].y);
                const float ex = (me[r].z - me[r].x) - d.x, ey = (me[r].w - me[r].y) - d.y;
                err = __builtin_fmaf(ex, ex, ey * ey);
            }
            if (lane == 0) {
                e2[i] = err;
                const double pr = (double)p_own[r];
                mine = make_double2(pr, pr > 0.0 ? pr * (double)err : 0.0);
            }
        }
        if (lane == 0) s_part[(threadIdx.x / kWave) * kERows + r] = mine;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double2 r = s_part[0];
        for (int w = 1; w < kRowsPerBlock; ++w) {
            r.x += s_part[w].x;
            r.y += s_part[w].y;
        }
        part[block] = r;
    }
}

__global__ __launch_bounds__(kEThreads) void k_estep(
    const float4 *__restrict__ xy, const float *__restrict__ p, const float4 *__restrict__ q,
    const float *__restrict__ s, int n, float nal2, float *__restrict__ e2,
    double2 *__restrict__ part, DevState *st, EmStop stp) {
    estep_body<kEmFused, EMDQ_E_ROWS, kEChunk>(xy, p, q, s, n, nal2, e2, part, gridDim.x, st, stp, blockIdx.x);
}

__global__ __launch_bounds__(kEThreads) void k_estep_s(
    const float4 *__restrict__ xy, const float *__restrict__ p, const float4 *__restrict__ q,
    const float *__restrict__ s, int n, float nal2, float *__restrict__ e2,
    double2 *__restrict__ part, DevState *st) {
    estep_body<kEmSingle, EMDQ_E_ROWS, kEChunk>(xy, p, q, s, n, nal2, e2, part, gridDim.x, st, EmStop{}, blockIdx.x);
}

// Finishes an EM iteration of one pair (one workgroup of kPostThreads >=
// kEmThreads threads; a batch pair, or a single pair in three launches per
// iteration): the E-step partials summed as partial_run / combine_partials
// do, sigma^2 and gamma, the posteriors (post_p) and mask of every match,
// and the stop rule.  The same arithmetic as the posterior step at the start of
// a fused M-step, so every mode gives the same bits.  host_copy (pinned host
// memory, may be null): the state as this kernel leaves it, so the host
// reads the stop flag without a copy.
constexpr int kPostThreads = 1024;

__device__ __forceinline__ void posterior_body(
    float *__restrict__ p, const float *__restrict__ e2, uint8_t *__restrict__ mask, int n,
    const double2 *__restrict__ part, int nb, const PostParams &pp, DevState *st,
    DevState *host_copy, int seq) {
#pragma clang fp contract(off)
    auto publish = [&]() {
        if (host_copy && threadIdx.x == 0) publish_state(host_copy, st, seq);
    };
    if (st->status < 0 || st->done) {
        publish();
        return;
    }
    double sigma2;
    PostCoef c;
    const double2 first = part[min((int)threadIdx.x, nb - 1)];
    if (!post_coef(combine_partials(partial_run(part, nb, first)), n, pp, &sigma2, &c)) {
        if (threadIdx.x == 0) {
            st->status = EMDQ_ENOINLIERS;
            st->done = 1;
        }
        publish();
        return;
    }
    int changed = 0;
    for (int r = threadIdx.x; r < n; r += kPostThreads) {
        const float pn = post_p(e2[r], c);
        p[r] = pn;
        const uint8_t m = pn > pp.p_thresh ? 1 : 0;
        changed |= (m != mask[r]);
        mask[r] = m;
    }
    changed = __syncthreads_or(changed);
    if (threadIdx.x == 0) {
        const int it = st->iter + 1;
        st->iter = it;
        st->changed = changed;
        st->sigma2 = (float)sigma2;
        st->gamma = (float)c.gamma;
        const int rule = stop_rule(it, changed, pp.max_iter);
        if (rule) st->done = 1;
        if (rule == 2) st->status = EMDQ_WARN_NOT_CONVERGED;
    }
    publish();
}

__global__ __launch_bounds__(kPostThreads) void k_posterior(
    float *__restrict__ p, const float *__restrict__ e2, uint8_t *__restrict__ mask, int n,
    const double2 *__restrict__ part, int nb, PostParams pp, DevState *st,
    DevState *host_copy, int seq) {
    posterior_body(p, e2, mask, n, part, nb, pp, st, host_copy, seq);
}

// ------------------------------------------------------------ compaction ----

// The stop rule after the last enqueued iteration of a single-pair fit, from
// the flags of its final M-step (chg null: no EM decision pending).
struct EmFinal {
    const int *chg;
    int nb, it, max_iter;
};

// Packs the inliers in index order: packed[2k] = (x, y, q_c - 1, q_s),
// packed[2k+1] = (q_x, q_y, s - 1, 1) (deviation-coded, see
// blend_displacement).  One workgroup; each thread owns a
// contiguous run of matches, runs are ordered by an exclusive scan.  First,
// if the EM is still running after its last iteration, the stop rule
// (EmFinal).
__device__ __forceinline__ void compact_body(
    const float4 *__restrict__ xy, const float4 *__restrict__ q, const float *__restrict__ s,
    const uint8_t *__restrict__ mask, int n, float4 *__restrict__ packed,
    float *__restrict__ xs, float *__restrict__ ys, DevState *st, const EmFinal &fin,
    int block) {
    __shared__ int scan[kCompactThreads];
    if (st->status < 0) return;
    const int t = threadIdx.x;
    if (fin.chg && st->stop_at == 0) {
        int any = 0;
        for (int k = t; k < fin.nb; k += kCompactThreads) any |= fin.chg[k];
        any = __syncthreads_or(any);   // also orders every read of st before the stores
        if (t == 0) {
            st->iter = fin.it;
            st->changed = any;
            const int rule = stop_rule(fin.it, any, fin.max_iter);
            if (rule) {
                st->done = 1;
                st->stop_at = 2 * fin.it + 3;   // after the final M-step, 2 (it + 1)
            }
            if (rule == 2) st->status = EMDQ_WARN_NOT_CONVERGED;
        }
    }
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
        xs[pos] = v.x;
        ys[pos] = v.y;
        ++pos;
    }
    if (t == kCompactThreads - 1) {
        const int total = scan[t];
        st->n_in = total;
        if (total == 0) st->status = EMDQ_ENOINLIERS;
    }
}

__global__ __launch_bounds__(kCompactThreads) void k_compact(
    const float4 *__restrict__ xy, const float4 *__restrict__ q, const float *__restrict__ s,
    const uint8_t *__restrict__ mask, int n, float4 *__restrict__ packed,
    float *__restrict__ xs, float *__restrict__ ys, DevState *st, EmFinal fin) {
    compact_body(xy, q, s, mask, n, packed, xs, ys, st, fin, blockIdx.x);
}

// Speculative compaction of a fused single-pair fit, enqueued after every
// chunk of EM iterations: once the EM has stopped (the M-step before the
// stopping E-step fitted with the final posteriors), the first one packs the
// inliers and the later ones return at once; before that they all return.
__global__ __launch_bounds__(kCompactThreads) void k_compact_spec(
    const float4 *__restrict__ xy, const float4 *__restrict__ q, const float *__restrict__ s,
    const uint8_t *__restrict__ mask, int n, float4 *__restrict__ packed,
    float *__restrict__ xs, float *__restrict__ ys, DevState *st) {
    if (st->stop_at == 0 || st->packed) return;
    compact_body(xy, q, s, mask, n, packed, xs, ys, st, EmFinal{}, blockIdx.x);
    __syncthreads();
    if (threadIdx.x == 0) st->packed = 1;
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
template <int SPLITK, int RB>
struct FieldLds {
    float part[SPLITK > 1 ? 4 : 1][SPLITK > 1 ? RB * 3 * (16 - 16 / SPLITK) : 1][kWave];
};

enum { kModeField = 0, kModeWarp = 1 };

// Sec. III-F, Eqs. (23)-(24): bilinear sample of the new frame at u = z + d
// and running-average merge into canvas pixel z + (ox, oy); pixels whose u
// leaves [0, fw-1] x [0, fh-1] are left unchanged.  With integer z the sample
// cell and the bilinear weights come from d alone, so u is never rounded.
[[maybe_unused]] __device__ __forceinline__ void warp_merge(int zx, int zy, float2 d,
                                           const uint8_t *__restrict__ frame, int fw, int fh,
                                           int fpitch, float4 *__restrict__ canvas, int cpitch,
                                           int ox, int oy) {
    const float fzx = (float)zx, fzy = (float)zy;
    if (!(d.x >= -fzx && d.x <= (float)(fw - 1 - zx) && d.y >= -fzy &&
          d.y <= (float)(fh - 1 - zy)))
        return;
    const float flx = floorf(d.x), fly = floorf(d.y);
    const int x0 = zx + (int)flx, y0 = zy + (int)fly;
    const int x1 = min(x0 + 1, fw - 1), y1 = min(y0 + 1, fh - 1);
    const float ax = d.x - flx, by = d.y - fly;
    const uint8_t *row0 = frame + (size_t)y0 * fpitch;
    const uint8_t *row1 = frame + (size_t)y1 * fpitch;
    const float w00 = (1.f - ax) * (1.f - by), w01 = ax * (1.f - by);
    const float w10 = (1.f - ax) * by, w11 = ax * by;
    float v[3];
#pragma unroll
    for (int ch = 0; ch < 3; ++ch)
        v[ch] = w00 * (float)row0[3 * x0 + ch] + w01 * (float)row0[3 * x1 + ch] +
                w10 * (float)row1[3 * x0 + ch] + w11 * (float)row1[3 * x1 + ch];
    float4 *px = canvas + (size_t)(zy + oy) * cpitch + (zx + ox);
    float4 cur = *px;
    const float A = cur.w, A1 = A + 1.f;
    const float rA1 = __builtin_amdgcn_rcpf(A1);   // A1 in [1, 31]: about 1 ulp
    cur.x = (A * cur.x + v[0]) * rA1;
    cur.y = (A * cur.y + v[1]) * rA1;
    cur.z = (A * cur.z + v[2]) * rA1;
    cur.w = fminf(A1, 30.f);
    *px = cur;
}

// warp_merge for NB pixels of one lane, with the same arithmetic for every
// pixel it merges.  All loads are issued before any is used: the sample cell
// of a pixel that is not merged is clamped into the frame, and the canvas
// read of a pixel outside the region goes to the region origin, so every
// load is in bounds and none waits behind another.  Only merged pixels are
// stored; the pixels are distinct, so no store feeds a later load.
template <int NB>
__device__ __forceinline__ void warp_merge_batch(const int (&zx)[NB], const int (&zy)[NB],
                                                 const float2 (&d)[NB], const bool (&live)[NB],
                                                 int zx0, int zy0,
                                                 const uint8_t *__restrict__ frame, int fw,
                                                 int fh, int fpitch, float4 *__restrict__ canvas,
                                                 int cpitch, int ox, int oy) {
    bool ok[NB];
    float ax[NB], by[NB];
    uint8_t p[NB][4][3];   // corners 00, 01, 10, 11; channels
    float4 cur[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        const float fzx = (float)zx[i], fzy = (float)zy[i];
        ok[i] = live[i] && d[i].x >= -fzx && d[i].x <= (float)(fw - 1 - zx[i]) &&
                d[i].y >= -fzy && d[i].y <= (float)(fh - 1 - zy[i]);
        const float dx = ok[i] ? d[i].x : 0.f, dy = ok[i] ? d[i].y : 0.f;
        const float flx = floorf(dx), fly = floorf(dy);
        const int x0 = min(max(zx[i] + (int)flx, 0), fw - 1);
        const int y0 = min(max(zy[i] + (int)fly, 0), fh - 1);
        const int x1 = min(x0 + 1, fw - 1), y1 = min(y0 + 1, fh - 1);
        ax[i] = dx - flx;
        by[i] = dy - fly;
        const uint8_t *row0 = frame + (size_t)y0 * fpitch;
        const uint8_t *row1 = frame + (size_t)y1 * fpitch;
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            p[i][0][ch] = row0[3 * x0 + ch];
            p[i][1][ch] = row0[3 * x1 + ch];
            p[i][2][ch] = row1[3 * x0 + ch];
            p[i][3][ch] = row1[3 * x1 + ch];
        }
        const int cx = live[i] ? zx[i] : zx0, cy = live[i] ? zy[i] : zy0;
        cur[i] = canvas[(size_t)(cy + oy) * cpitch + (cx + ox)];
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        if (!ok[i]) continue;
        const float w00 = (1.f - ax[i]) * (1.f - by[i]), w01 = ax[i] * (1.f - by[i]);
        const float w10 = (1.f - ax[i]) * by[i], w11 = ax[i] * by[i];
        float v[3];
#pragma unroll
        for (int ch = 0; ch < 3; ++ch)
            v[ch] = w00 * (float)p[i][0][ch] + w01 * (float)p[i][1][ch] +
                    w10 * (float)p[i][2][ch] + w11 * (float)p[i][3][ch];
        float4 c = cur[i];
        const float A = c.w, A1 = A + 1.f;
        const float rA1 = __builtin_amdgcn_rcpf(A1);   // A1 in [1, 31]: about 1 ulp
        c.x = (A * c.x + v[0]) * rA1;
        c.y = (A * c.y + v[1]) * rA1;
        c.z = (A * c.z + v[2]) * rA1;
        c.w = fminf(A1, 30.f);
        canvas[(size_t)(zy[i] + oy) * cpitch + (zx[i] + ox)] = c;
    }
}

// One per-axis Gaussian factor exp(-alpha d^2) = 2^(nal2 d^2), nal2 =
// -alpha log2(e), d = z - x_j along one axis.  The in-loop blend and the
// factor tables both call this, so both give the same bits.
__device__ __forceinline__ float axis_factor(float nal2, float d) {
    return fast_exp2(nal2 * d * d);
}

// Per-launch factor tables of the FP32 blend, inlier-major: gx[j * sx + c] =
// axis_factor(nal2, zx0 + c - x_j) for the region's columns c, gy[j * sy + r]
// likewise for its rows r (sx, sy: the region's width and height rounded up
// to whole tiles).  Null gx: the factors are computed in the blend's loop.
struct FieldTabs {
    const float *gx, *gy;
    int sx, sy;
};

// The tiles an FP16 blend of a region left to the FP32 blend (flags[b] != 0
// for its tile b, hx tiles per row; see k_field_fallback), and the field
// output pitch: out[(z_y - zy0) opitch + (z_x - zx0)] (opitch 0: the region
// width).
struct FieldFilter {
    const uint8_t *flags;
    int hx, opitch;
};

// RB row blocks of 32 share the B operands: a wavefront's tile is 32 RB rows x
// 32 columns and each pair of inliers costs RB + 1 exponentials and 6
// multiplies for 6 RB MFMAs; with factor tables (TAB), RB + 1 table loads
// and 5 multiplies (the weight column is the x factor itself).
template <int MODE, int SPLITK, int RB, bool TAB = false>
__device__ __forceinline__ void field_body(
    const float4 *__restrict__ packed, const DevState *__restrict__ st, float nal2, int zx0,
    int zy0, int w, int h, int tiles_x, int n_tiles, float2 *__restrict__ out,
    const uint8_t *__restrict__ frame, int fw, int fh, int fpitch, float4 *__restrict__ canvas,
    int cpitch, int ox, int oy, int block, FieldTabs tabs = FieldTabs{},
    FieldFilter filt = FieldFilter{}) {
    constexpr int kTilesPerWg = 4 / SPLITK;
    constexpr int kRegsOwned = 16 / SPLITK;
    __shared__ FieldLds<SPLITK, RB> lds;

    const int wave = threadIdx.x >> 6, lane = threadIdx.x & (kWave - 1);
    const int tile = block * kTilesPerWg + wave / SPLITK;
    const int ks = wave % SPLITK;
    const int status = st->status;
    const int n_in = st->n_in;
    const bool bad = status < 0 || n_in <= 0;
    if (MODE == kModeWarp && bad) return;    // canvas left unchanged

    int tx = tile % tiles_x, ty = tile / tiles_x;
    if (EMDQ_XCD_MAP && TAB && kTilesPerWg == 1 && tiles_x >= 16 && tile < n_tiles) {
        // Workgroups go to the 8 XCDs in turn (block b to XCD b % 8): give
        // XCD x the x-th run of tiles in an order of two column bands, each
        // row by row, so that its tiles are a compact block and share table
        // rows in its L2.
        const int q = n_tiles / 8, r = n_tiles % 8;
        const int xcd = block < 8 * q ? block % 8 : block - 8 * q;
        const int slot = block < 8 * q ? block / 8 : q;
        const int t = xcd * q + min(xcd, r) + slot;
        const int bw = (tiles_x + 1) / 2, c0 = bw * (n_tiles / tiles_x);
        if (t < c0) {
            tx = t % bw;
            ty = t / bw;
        } else {
            const int w1 = tiles_x - bw;
            tx = bw + (t - c0) % w1;
            ty = (t - c0) / w1;
        }
    }
    const int px0 = zx0 + tx * kTile, py0 = zy0 + ty * kTile * RB;
    const int opitch = filt.opitch > 0 ? filt.opitch : w;
    const int col = lane & 31, half = lane >> 5;
    const float zcol = (float)(px0 + col);   // z_x of the B operand column
    float zrow[RB];                          // z_y of the A operand rows
#pragma unroll
    for (int b = 0; b < RB; ++b) zrow[b] = (float)(py0 + kTile * b + col);

    f32x16 acc[RB][6];
#pragma unroll
    for (int b = 0; b < RB; ++b)
#pragma unroll
        for (int c = 0; c < 6; ++c)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[b][c][r] = 0.f;

    if (!bad && tile < n_tiles) {
        // Wavefront-uniform K range: a whole number of ring groups, so the
        // ranges of the SPLITK wavefronts never overlap; records past the
        // inliers read as zero (buffer range check) and add nothing.  The
        // buffer resource is rebuilt per step on the scalar unit, so record
        // addressing costs no vector instruction.
        constexpr int kGroup = 2 * kRing;
        const int kper = ((n_in + SPLITK * kGroup - 1) / (SPLITK * kGroup)) * kGroup;
        const int kb = __builtin_amdgcn_readfirstlane(ks * kper);
        const int kend = kb + kper;
        const int voff = half * 32;        // lanes 32..63 take the odd inlier
        auto factors = [&](const float4 &r0, float (&a)[RB], float &g) {
#pragma unroll
            for (int b = 0; b < RB; ++b) a[b] = axis_factor(nal2, zrow[b] - r0.y);
            g = axis_factor(nal2, zcol - r0.x);
        };
        auto load = [&](int j0, float4 &r0, float4 &r1) {
            const int jj = __builtin_amdgcn_readfirstlane(min(j0, n_in));
            const int bytes = __builtin_amdgcn_readfirstlane((n_in - jj) * 32);
            const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                (void *)(packed + 2 * jj), (short)0, bytes, kBufferFlags);
            r0 = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(rs, voff, 0, 0));
            r1 = __builtin_bit_cast(float4,
                                    __builtin_amdgcn_raw_buffer_load_b128(rs, voff + 16, 0, 0));
        };
        if constexpr (TAB) {
            // Factor tables: the A operands (rows) and the B factor (column)
            // of the lane's inlier j + half are table loads, 128 contiguous
            // bytes per half-wavefront; rows at or past n_in read as zero
            // (buffer range check), and so add nothing.  Same ring as below.
            const int lx = tx * kTile + col, ly = ty * kTile * RB + col;
            auto tload = [&](int j0, float4 &r0, float4 &r1, float (&ta)[RB], float &tg) {
                load(j0, r0, r1);
                const int jj = __builtin_amdgcn_readfirstlane(min(j0, n_in));
                const int rows = __builtin_amdgcn_readfirstlane(n_in - jj);
                const __amdgpu_buffer_rsrc_t rx = __builtin_amdgcn_make_buffer_rsrc(
                    (void *)(tabs.gx + (size_t)jj * tabs.sx), (short)0, rows * tabs.sx * 4,
                    kBufferFlags);
                const __amdgpu_buffer_rsrc_t ry = __builtin_amdgcn_make_buffer_rsrc(
                    (void *)(tabs.gy + (size_t)jj * tabs.sy), (short)0, rows * tabs.sy * 4,
                    kBufferFlags);
                tg = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(
                                                   rx, (half * tabs.sx + lx) * 4, 0, 0));
#pragma unroll
                for (int b = 0; b < RB; ++b)
                    ta[b] = __builtin_bit_cast(
                        float, __builtin_amdgcn_raw_buffer_load_b32(
                                   ry, (half * tabs.sy + ly + kTile * b) * 4, 0, 0));
            };
            float4 ra[kRing], rb[kRing];
            float ta[kRing][RB], tg[kRing];
#pragma unroll
            for (int u = 0; u < kRing; ++u) {
                tload(kb + 2 * u, ra[u], rb[u], ta[u], tg[u]);
                __builtin_amdgcn_sched_barrier(0);   // issue in ring order
            }
            for (int j0 = kb; j0 < kend; j0 += 2 * kRing) {
#pragma unroll
                for (int u = 0; u < kRing; ++u) {
                    const int j = j0 + 2 * u;
                    const float4 r0 = ra[u], r1 = rb[u];
                    const float q[5] = {r0.z, r0.w, r1.x, r1.y, r1.z};
                    float a[RB];
#pragma unroll
                    for (int bl = 0; bl < RB; ++bl) a[bl] = ta[u][bl];
                    const float g = tg[u];
#pragma unroll
                    for (int c = 0; c < 6; ++c) {
                        const float bop = c < 5 ? g * q[c] : g;
#pragma unroll
                        for (int bl = 0; bl < RB; ++bl)
                            acc[bl][c] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[bl], bop,
                                                                              acc[bl][c], 0, 0, 0);
                    }
                    tload(j + 2 * kRing, ra[u], rb[u], ta[u], tg[u]);
                    __builtin_amdgcn_sched_barrier(EMDQ_SCHED_MASK);
                }
            }
        } else {
        // Ring of kRing record buffers: step u of a group uses buffer u and
        // refills it for the same step of the next group, so every load has
        // kRing K steps to land.  The Gaussian factors of step u + 1 are
        // computed while the MFMAs of step u run.  The group loop is fully
        // unrolled, so the buffers stay in fixed registers.
        float4 ra[kRing], rb[kRing];
#pragma unroll
        for (int u = 0; u < kRing; ++u) {
            load(kb + 2 * u, ra[u], rb[u]);
            __builtin_amdgcn_sched_barrier(0);   // issue in ring order
        }
        float a[RB], g;
        factors(ra[0], a, g);
        for (int j0 = kb; j0 < kend; j0 += 2 * kRing) {
#pragma unroll
            for (int u = 0; u < kRing; ++u) {
                const int j = j0 + 2 * u;
                const float4 r0 = ra[u], r1 = rb[u];
                const float q[6] = {r0.z, r0.w, r1.x, r1.y, r1.z, r1.w};
                float an[RB], gn;   // next step (its record is already in the ring)
#pragma unroll
                for (int c = 0; c < 6; ++c) {
                    const float bop = g * q[c];
#pragma unroll
                    for (int bl = 0; bl < RB; ++bl)
                        acc[bl][c] =
                            __builtin_amdgcn_mfma_f32_32x32x2f32(a[bl], bop, acc[bl][c], 0, 0, 0);
                    if (c == 0) factors(ra[(u + 1) % kRing], an, gn);
                }
                load(j + 2 * kRing, ra[u], rb[u]);
#pragma unroll
                for (int bl = 0; bl < RB; ++bl) a[bl] = an[bl];
                g = gn;
                // memory operations keep their place (otherwise the loads
                // sink to their use)
                __builtin_amdgcn_sched_barrier(EMDQ_SCHED_MASK);
            }
        }
        }   // TAB
    }

    // ---- split-K reduction, then the epilogue, specialised per wavefront of
    // the tile: wavefront KS keeps registers [KS*R, KS*R + R) of every row
    // block.  ks is wavefront-uniform, so the switch below is a scalar
    // branch; with KS a compile-time constant those registers are fixed (a
    // runtime register index compiles to compare / select chains over all
    // 16 accumulator registers, thousands of VALU instructions that cannot
    // overlap the MFMA pipe).
    auto finish = [&](auto ks_tag) {
        constexpr int KS = decltype(ks_tag)::value;
        constexpr int rbase = KS * kRegsOwned;
        if constexpr (SPLITK > 1) {
            // two passes of three components each, so the partials need half
            // the LDS
#pragma unroll
            for (int c0 = 0; c0 < 6; c0 += 3) {
                if (c0 > 0) __syncthreads();   // the first pass's reads are done
                int slot = 0;
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    if (r >= rbase && r < rbase + kRegsOwned) continue;
#pragma unroll
                    for (int bl = 0; bl < RB; ++bl)
#pragma unroll
                        for (int c = 0; c < 3; ++c)
                            lds.part[wave][(slot * RB + bl) * 3 + c][lane] = acc[bl][c0 + c][r];
                    ++slot;
                }
                __syncthreads();
                // add the partials in wavefront order 0, 1, ..., SPLITK-1
                const int wbase = (wave / SPLITK) * SPLITK;
#pragma unroll
                for (int rr = 0; rr < kRegsOwned; ++rr) {
                    const int r = rbase + rr;
#pragma unroll
                    for (int bl = 0; bl < RB; ++bl)
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            float sum = 0.f;
                            for (int src = 0; src < SPLITK; ++src) {
                                float v;
                                if (src == KS) {
                                    v = acc[bl][c0 + c][r];
                                } else {
                                    // slot of register r in wavefront src's list
                                    const int src_base = src * kRegsOwned;
                                    const int sl = r < src_base ? r : r - kRegsOwned;
                                    v = lds.part[wbase + src][(sl * RB + bl) * 3 + c][lane];
                                }
                                sum = src == 0 ? v : sum + v;
                            }
                            acc[bl][c0 + c][r] = sum;
                        }
                }
            }
        }
        if (tile >= n_tiles) return;

        // ---- epilogue: DQ normalisation, Eq. (1), then (warp) sample + merge,
        // in groups of kGroupPix pixels per lane (fewer where more accumulator
        // registers are still live, so that nothing spills)
        constexpr int kGroupPix = SPLITK >= 4 ? 4 : 2;
        int pzx[kGroupPix], pzy[kGroupPix];
        float2 pd[kGroupPix];
        bool live[kGroupPix];
#pragma unroll
        for (int bl = 0; bl < RB; ++bl)
#pragma unroll
        for (int rr = 0; rr < kRegsOwned; ++rr) {
            const int r = rbase + rr, i = rr % kGroupPix;
            const int zx = px0 + col;
            const int zy = py0 + kTile * bl + 8 * (r >> 2) + 4 * half + (r & 3);
            const float fzx = (float)zx, fzy = (float)zy;
            pzx[i] = zx;
            pzy[i] = zy;
            live[i] = zx < zx0 + w && zy < zy0 + h;
            pd[i] = blend_displacement_field(acc[bl][5][r], acc[bl][0][r], acc[bl][1][r], acc[bl][2][r],
                                       acc[bl][3][r], acc[bl][4][r], fzx, fzy);
            if constexpr (MODE == kModeField) {
                if (live[i])
                    out[(size_t)(zy - zy0) * opitch + (zx - zx0)] =
                        bad ? make_float2(__builtin_nanf(""), __builtin_nanf(""))
                            : make_float2(fzx + pd[i].x, fzy + pd[i].y);
            } else if constexpr (!EMDQ_WARP_BATCH) {
                if (live[i]) warp_merge(zx, zy, pd[i], frame, fw, fh, fpitch, canvas, cpitch, ox, oy);
            } else if (i == kGroupPix - 1) {
                warp_merge_batch<kGroupPix>(pzx, pzy, pd, live, zx0, zy0, frame, fw, fh, fpitch,
                                            canvas, cpitch, ox, oy);
            }
        }
    };
    static_assert(SPLITK == 1 || SPLITK == 2 || SPLITK == 4, "split-K 1, 2 or 4");
    if constexpr (SPLITK == 1) {
        finish(IntTag<0>{});
    } else if constexpr (SPLITK == 2) {
        if (ks == 0) finish(IntTag<0>{});
        else finish(IntTag<1>{});
    } else {
        switch (ks) {
        case 0: finish(IntTag<0>{}); break;
        case 1: finish(IntTag<1>{}); break;
        case 2: finish(IntTag<2>{}); break;
        default: finish(IntTag<3>{}); break;
        }
    }
}

template <int MODE, int SPLITK, int RB, bool TAB>
__global__ __launch_bounds__(kFieldThreads) __attribute__((amdgpu_waves_per_eu(field_waves(RB), field_waves(RB)))) void k_field(
    const float4 *__restrict__ packed, const DevState *__restrict__ st, float nal2, int zx0,
    int zy0, int w, int h, int tiles_x, int n_tiles, float2 *__restrict__ out,
    const uint8_t *__restrict__ frame, int fw, int fh, int fpitch, float4 *__restrict__ canvas,
    int cpitch, int ox, int oy, FieldTabs tabs, FieldFilter filt) {
    field_body<MODE, SPLITK, RB, TAB>(packed, st, nal2, zx0, zy0, w, h, tiles_x, n_tiles, out,
                                      frame, fw, fh, fpitch, canvas, cpitch, ox, oy, blockIdx.x,
                                      tabs, filt);
}

// The FP32 blend of the tiles an FP16 blend of the same region left
// (FieldFilter): workgroup b looks at FP16 tile b (64 rows x 128 columns) and,
// if it is flagged, blends its four 64 x 32 tiles (two 32-row blocks per
// wavefront, split-K 4) one after the other; unflagged tiles return at once.
template <int MODE>
__global__ __launch_bounds__(kFieldThreads) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_field_fallback(
    const float4 *__restrict__ packed, const DevState *__restrict__ st, float nal2, int zx0,
    int zy0, int w, int h, float2 *__restrict__ out, const uint8_t *__restrict__ frame, int fw,
    int fh, int fpitch, float4 *__restrict__ canvas, int cpitch, int ox, int oy,
    FieldFilter filt) {
    if (!filt.flags[blockIdx.x]) return;
    const int rtx = (w + kTile - 1) / kTile, rty = (h + 2 * kTile - 1) / (2 * kTile);
    const int hxi = (int)blockIdx.x % filt.hx, hyi = (int)blockIdx.x / filt.hx;
    const FieldFilter all{nullptr, 0, filt.opitch};
    for (int k = 0; k < kHTxF / kTile; ++k) {
        const int tx = (kHTxF / kTile) * hxi + k;
        if (tx >= rtx) break;   // the same for every thread of the workgroup
        field_body<MODE, 4, 2, false>(packed, st, nal2, zx0, zy0, w, h, rtx, rtx * rty, out,
                                      frame, fw, fh, fpitch, canvas, cpitch, ox, oy,
                                      hyi * rtx + tx, FieldTabs{}, all);
        __syncthreads();   // the next tile reuses the split-K area of LDS
    }
}

// The factor tables of an FP32 blend over a region (FieldTabs): row j of
// each table belongs to inlier j; a thread owns four consecutive entries of
// the rows (x entries first, then y) and writes them for kTabRowsPerThread
// consecutive rows, whose coordinates it loads first, all at once.  Rows
// j >= n_in are not written (the blend reads them as zero).  Grid: x over the
// ceil((sx + sy) / 4) entry groups of a row, y over blocks of rows.
constexpr int kTabThreads = 256;
constexpr int kTabRowsPerThread = 8;

// Four consecutive entries z0 .. z0 + 3 of rows 0 .. min(nrows, 8) - 1 (row r
// at dst + r * stride, coordinate xj[r]).
__device__ __forceinline__ void table_rows(const float (&xj)[kTabRowsPerThread], int nrows,
                                           float nal2, float z0, float *dst, int stride) {
    const float z1 = z0 + 1.f, z2 = z0 + 2.f, z3 = z0 + 3.f;
#pragma unroll
    for (int r = 0; r < kTabRowsPerThread; ++r) {
        if (r >= nrows) break;
        float4 v;
        v.x = axis_factor(nal2, z0 - xj[r]);
        v.y = axis_factor(nal2, z1 - xj[r]);
        v.z = axis_factor(nal2, z2 - xj[r]);
        v.w = axis_factor(nal2, z3 - xj[r]);
        *(float4 *)(dst + (size_t)r * stride) = v;
    }
}
__global__ __launch_bounds__(kTabThreads) void k_field_tables(
    const float *__restrict__ xs, const float *__restrict__ ys,
    const DevState *__restrict__ st, float nal2, int zx0, int zy0, float *__restrict__ gx,
    float *__restrict__ gy, int sx, int sy) {
    const int n_in = st->status < 0 ? 0 : st->n_in;
    const int j0 = kTabRowsPerThread * (int)blockIdx.y;
    const int e = 4 * (int)(blockIdx.x * kTabThreads + threadIdx.x);
    if (j0 >= n_in || e >= sx + sy) return;
    const bool is_x = e < sx;   // sx is a multiple of 4: a group never straddles
    const float *src = is_x ? xs : ys;
    const int c0 = is_x ? e : e - sx;
    const int stride = is_x ? sx : sy;
    float *dst = (is_x ? gx : gy) + c0;
    float xj[kTabRowsPerThread];
#pragma unroll
    for (int r = 0; r < kTabRowsPerThread; ++r) xj[r] = src[min(j0 + r, n_in - 1)];
    table_rows(xj, n_in - j0, nal2, (float)((is_x ? zx0 : zy0) + c0), dst + (size_t)j0 * stride,
               stride);
}



// ------------------------------------------- half-precision field / warp ----
//
// The same blend with the two GEMM operands in FP16 or BF16 and FP32
// accumulation (v_mfma_f32_32x32x16_{f16,bf16}: lane l holds A[l % 32][8 (l / 32)
// + i] and B[8 (l / 32) + i][l % 32], i < 8; accumulator layout as above).
//
// Deviation coding per workgroup tile.  The blend is linear in the DQ
// components and the DQ product is bilinear, so for fixed unit DQs a, b
//   sum_j w_j (a q_j b) = a (sum_j w_j q_j) b,
// and normalising by the norm of the real part commutes with both products.
// Each workgroup takes a reference motion T0 = (R0, t0) and scale s0, the
// blend at its tile centre p, and blends q'_j = a q_j b with b the
// translation by p and a = R0^-1 composed with the translation by -c0,
// c0 = T0(p): q'_j is the motion u -> R0^T (T_j(u + p) - c0), close to the
// identity for the nodes that carry weight at the tile.  The stored values
// (q'_c - 1, q'_s, q'_x, q'_y, s_j - s0) are then small, which is what keeps
// the 11-bit (FP16) or 8-bit (BF16) operands accurate; the epilogue undoes
// the coding exactly: T(z) = R0 T'(z - p) + c0, s = s0 + mean(s_j - s0).
//
// Workgroup tile 64 rows x 128 columns; wavefront w owns columns
// [32 w, 32 w + 32) and both 32-row blocks, so each B operand (Gaussian x
// factor times one coded component, built in registers) feeds two MFMAs.
// The per-axis Gaussian factors of the next chunk of 64 inliers are computed
// into LDS while the MFMAs of the current chunk run (double buffer, one
// barrier per chunk).
enum { kDtF16 = 0, kDtBF16 = 1 };
constexpr int kHTx = kHTxF, kHTy = kHTyF, kHK = 64, kHStride = kHK + 8;   // LDS rows padded
constexpr int kTabRows = 4096;   // factor-table rows per axis (one slab of the region)
constexpr int kHalfFlagBytes = (kTabRows / kHTxF) * (kTabRows / kHTyF);   // tiles of a slab

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef _Float16 half4 __attribute__((ext_vector_type(4)));
typedef __bf16 bhalf8 __attribute__((ext_vector_type(8)));
typedef __bf16 bhalf4 __attribute__((ext_vector_type(4)));

template <int DT> struct HalfT;
template <> struct HalfT<kDtF16> {
    using T = _Float16;
    using V8 = half8;
    using V4 = half4;
    using Q = _Float16;   // coded node values in LDS
};
template <> struct HalfT<kDtBF16> {
    using T = __bf16;
    using V8 = bhalf8;
    using V4 = bhalf4;
    using Q = float;      // BF16 products are formed in FP32, then rounded
};

// Three chunk buffers: with factor tables, chunk c + 2 is stored while chunk
// c is multiplied, so chunk c + 1 is complete one barrier early and its
// first operands can be read before that barrier (the generating path uses
// two of them).
template <int DT>
struct alignas(16) HalfLds {
    typename HalfT<DT>::T gy[3][kHTy][kHStride];
    typename HalfT<DT>::T gx[3][kHTx][kHStride];
    typename HalfT<DT>::Q qd[3][5][kHK];
    float red[4][8];
};

// Operands of one K step of the half-precision blend, held in registers.
template <int DT> struct KOps;
template <> struct KOps<kDtF16> {
    half8 a0, a1, g;
    half8 q[5];
};
template <> struct KOps<kDtBF16> {
    bhalf8 a0, a1, g;
    float4 q[5][2];
};

// The MFMA operands of one K step: both row blocks' A and the six B.
// VALU instructions placed after each MFMA in the pipelined K step (F16:
// 20 packed multiplies for 12 MFMAs; BF16 forms its products in FP32)
template <int DT> constexpr int kHalfValu = DT == kDtF16 ? 3 : 9;
#ifndef EMDQ_HALF_LEAD
#define EMDQ_HALF_LEAD 6
#endif
// MFMAs of a K step issued before the first VALU that waits on its LDS reads
constexpr int kHalfLead = EMDQ_HALF_LEAD;
#ifndef EMDQ_HALF_SPREAD
#define EMDQ_HALF_SPREAD 1  // a K step's LDS reads interleaved with its MFMAs, not issued in a burst
#endif
#ifndef EMDQ_HALF_AHEAD
#define EMDQ_HALF_AHEAD 2   // K steps between a step's LDS operand reads and its MFMAs
#endif
template <int DT> struct KB {
    typename HalfT<DT>::V8 a0, a1, b[6];
};

// Planar DQ product (c1 + s1 k + eps (x1 i + y1 j)) (c2 + s2 k + eps (x2 i +
// y2 j)): the motion that applies the right operand first.
__device__ __forceinline__ float4 dq_mul(float4 a, float4 b) {
    return make_float4(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x,
                       a.x * b.z - a.y * b.w + a.z * b.x + a.w * b.y,
                       a.x * b.w + a.y * b.z + a.w * b.x - a.z * b.y);
}

template <int MODE, int DT>
__global__ __launch_bounds__(kFieldThreads) void k_field_half(
    const float4 *__restrict__ packed, const float *__restrict__ xs,
    const float *__restrict__ ys, const DevState *__restrict__ st, float ka, int zx0, int zy0,
    int w, int h, int tiles_x, float2 *__restrict__ out, const uint8_t *__restrict__ frame,
    int fw, int fh, int fpitch, float4 *__restrict__ canvas, int cpitch, int ox, int oy,
    const void *__restrict__ gx_tab, const void *__restrict__ gy_tab, int tab_stride,
    int opitch, uint8_t *__restrict__ tile_flags) {
    using T = typename HalfT<DT>::T;
    using V8 = typename HalfT<DT>::V8;
    using V4 = typename HalfT<DT>::V4;
    __shared__ HalfLds<DT> L;

    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & (kWave - 1);
    const int col = lane & 31, half = lane >> 5;
    const int status = st->status;
    const int n_in = st->n_in;
    const bool bad = status < 0 || n_in <= 0;
    if (MODE == kModeWarp && bad) return;

    const int px0 = zx0 + (int)(blockIdx.x % tiles_x) * kHTx;
    const int py0 = zy0 + (int)(blockIdx.x / tiles_x) * kHTy;
    const float pcx = (float)px0 + 0.5f * (kHTx - 1), pcy = (float)py0 + 0.5f * (kHTy - 1);

    // Table slices of a chunk (with factor tables; see below).  The first
    // chunk's are loaded before the reference blend, which they do not depend
    // on, so their latency overlaps it.
    V8 pgx[kHTx * 8 / kFieldThreads], pgy[kHTy * 8 / kFieldThreads];
    float4 pr0 = make_float4(0.f, 0.f, 0.f, 0.f), pr1 = pr0;
    const T *gxw =
        (const T *)gx_tab + (size_t)(px0 - zx0 + tid / 8) * tab_stride + 8 * (tid % 8);
    const T *gyw =
        (const T *)gy_tab + (size_t)(py0 - zy0 + tid / 8) * tab_stride + 8 * (tid % 8);
    constexpr size_t kRowStep = kFieldThreads / 8;   // rows per piece sweep
    auto fetch = [&](int jc) {
#pragma unroll
        for (int part = 0; part < kHTx * 8 / kFieldThreads; ++part)
            pgx[part] = *(const V8 *)(gxw + part * kRowStep * tab_stride + jc);
#pragma unroll
        for (int part = 0; part < kHTy * 8 / kFieldThreads; ++part)
            pgy[part] = *(const V8 *)(gyw + part * kRowStep * tab_stride + jc);
        if (wave == 3 && jc + lane < n_in) {
            pr0 = packed[2 * (jc + lane)];
            pr1 = packed[2 * (jc + lane) + 1];
        }
    };
    if (gx_tab && !bad) fetch(0);

    // ---- reference at the tile centre: FP32 blend over all inliers
    float sums[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (!bad) {
        // eight records per thread in flight at once (indices clamped, the
        // surplus ones weighted 0, which leaves the sums unchanged); the sums
        // keep the order j = tid, tid + 256, ...
        constexpr int kU = 8;
        const float nal2 = -ka * ka;
        for (int j0 = tid; j0 < n_in; j0 += kU * kFieldThreads) {
            float4 r0[kU], r1[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int j = min(j0 + u * kFieldThreads, n_in - 1);
                r0[u] = packed[2 * j];
                r1[u] = packed[2 * j + 1];
            }
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const float dx = pcx - r0[u].x, dy = pcy - r0[u].y;
                const float e = fast_exp2(nal2 * (dx * dx + dy * dy));
                const float wj = j0 + u * kFieldThreads < n_in ? e : 0.f;
                sums[0] += wj;
                sums[1] += wj * r0[u].z;
                sums[2] += wj * r0[u].w;
                sums[3] += wj * r1[u].x;
                sums[4] += wj * r1[u].y;
                sums[5] += wj * r1[u].z;
            }
        }
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) sums[c] = wave_sum(sums[c]);
    if (lane == 0)
#pragma unroll
        for (int c = 0; c < 6; ++c) L.red[wave][c] = sums[c];
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 6; ++c) sums[c] = ((L.red[0][c] + L.red[1][c]) + L.red[2][c]) + L.red[3][c];
    float ch0 = 1.f, sh0 = 0.f, d0x = 0.f, d0y = 0.f, sm1 = 0.f;
    {
        const float W0 = sums[0];
        const float C = 1.f + sums[1] / W0, S = sums[2] / W0;
        const float X = sums[3] / W0, Y = sums[4] / W0;
        const float in = 1.f / sqrtf(C * C + S * S);
        const float c = C * in, sn = S * in, dx = X * in, dy = Y * in;
        const float tx = 2.f * (c * dx - sn * dy), ty = 2.f * (sn * dx + c * dy);
        // (R0 - I) p + t0, rounded to 1/64 px so that c0 = p + d0 is exact
        const float ex = -2.f * sn * sn * pcx - 2.f * c * sn * pcy + tx;
        const float ey = 2.f * c * sn * pcx - 2.f * sn * sn * pcy + ty;
        const float gx = rintf(64.f * ex) * (1.f / 64.f), gy = rintf(64.f * ey) * (1.f / 64.f);
        const float g = sums[5] / W0;
        if (W0 > 0.f && __builtin_isfinite(c) && __builtin_isfinite(sn) &&
            __builtin_isfinite(gx) && __builtin_isfinite(gy) && __builtin_isfinite(g)) {
            ch0 = c;
            sh0 = sn;
            d0x = gx;
            d0y = gy;
            sm1 = g;
        }
    }
    const float cos0 = ch0 * ch0 - sh0 * sh0, sin0 = 2.f * ch0 * sh0;
    const float c0x = pcx + d0x, c0y = pcy + d0y;
    // a = R0^-1 (translation by -c0);  b = translation by p
    const float4 aq = make_float4(ch0, -sh0, -0.5f * (ch0 * c0x + sh0 * c0y),
                                  -0.5f * (ch0 * c0y - sh0 * c0x));
    const float4 bq = make_float4(1.f, 0.f, 0.5f * pcx, 0.5f * pcy);
    const float ch0m1 = -sh0 * sh0 / (1.f + ch0);   // ch0 - 1 without cancellation

    f32x16 acc[2][6];
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int c = 0; c < 6; ++c)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[b][c][r] = 0.f;

    if (!bad) {
        const int nchunks = (n_in + kHK - 1) / kHK;
        // generation roles: Gaussian x factor of column gcol for the 32
        // inliers [32 (wave / 2), +32) of a chunk, y factor of row `lane` for
        // the 16 inliers [16 wave, +16); wavefront 3 also codes the chunk's
        // node values (one inlier per lane)
        const int gcol = 64 * (wave & 1) + lane;
        const float zxa = ka * (float)(px0 + gcol), zya = ka * (float)(py0 + lane);
        const int jx = 32 * (wave >> 1), jy = 16 * wave;
        // Without factor tables each chunk's factors are generated here.
        auto gen = [&](int jc, int nb, int part) {
            const int bx = __builtin_amdgcn_readfirstlane(jc + jx + 8 * part);
            const int by = __builtin_amdgcn_readfirstlane(jc + jy + 4 * part);
            V8 gxv;
            V4 gyv;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const float d = ka * xs[bx + i] - zxa;
                const float e = fast_exp2(-(d * d));
                gxv[i] = (T)(bx + i < n_in ? e : 0.f);
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float d = ka * ys[by + i] - zya;
                const float e = fast_exp2(-(d * d));
                gyv[i] = (T)(by + i < n_in ? e : 0.f);
            }
            *(V8 *)&L.gx[nb][gcol][jx + 8 * part] = gxv;
            *(V4 *)&L.gy[nb][lane][jy + 4 * part] = gyv;
            if (part == 0 && wave == 3) {
                const int j = jc + lane;
                float v[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
                if (j < n_in) {
                    const float4 r0 = packed[2 * j], r1 = packed[2 * j + 1];
                    const float4 qj = make_float4(1.f + r0.z, r0.w, r1.x, r1.y);
                    const float4 qc = dq_mul(dq_mul(aq, qj), bq);
                    v[0] = ch0m1 + ch0 * r0.z + sh0 * r0.w;   // q'_c - 1
                    v[1] = qc.y;
                    v[2] = qc.z;
                    v[3] = qc.w;
                    v[4] = r1.z - sm1;                          // s_j - s0
                }
#pragma unroll
                for (int c = 0; c < 5; ++c) L.qd[nb][c][lane] = (typename HalfT<DT>::Q)v[c];
            }
        };
        // One K step of 16 inliers: the operands (both row blocks' y factors,
        // the x factors of the wavefront's columns, the coded node values)
        // are read from LDS by kload, then kmma forms the B operands and
        // issues the 12 MFMAs.  Splitting the two lets the reads of the
        // next step be issued before the MFMAs of this one.
        KOps<DT> cur;
        auto kload = [&](int buf, int s, KOps<DT> &o) {
            const int k8 = 16 * s + 8 * half;
            o.a0 = *(const V8 *)&L.gy[buf][col][k8];
            o.a1 = *(const V8 *)&L.gy[buf][32 + col][k8];
            o.g = *(const V8 *)&L.gx[buf][32 * wave + col][k8];
#pragma unroll
            for (int c = 0; c < 5; ++c) {
                if constexpr (DT == kDtF16) {
                    o.q[c] = *(const half8 *)&L.qd[buf][c][k8];
                } else {
                    o.q[c][0] = *(const float4 *)&L.qd[buf][c][k8];
                    o.q[c][1] = *(const float4 *)&L.qd[buf][c][k8 + 4];
                }
            }
        };
        // kbuild forms the B operands B_c = gx * (coded value c) and B_5 = gx
        auto kbuild = [&](const KOps<DT> &o, KB<DT> &k) {
            k.a0 = o.a0;
            k.a1 = o.a1;
            if constexpr (DT == kDtF16) {
#pragma unroll
                for (int c = 0; c < 5; ++c) k.b[c] = o.g * o.q[c];
            } else {
                float gf[8];
#pragma unroll
                for (int i = 0; i < 8; ++i) gf[i] = (float)o.g[i];
#pragma unroll
                for (int c = 0; c < 5; ++c) {
                    const float4 q0 = o.q[c][0], q1 = o.q[c][1];
                    const float qv[8] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w};
#pragma unroll
                    for (int i = 0; i < 8; ++i) k.b[c][i] = (T)(gf[i] * qv[i]);
                }
            }
            k.b[5] = o.g;
        };
        auto kmfma = [&](const KB<DT> &k) {
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                if constexpr (DT == kDtF16) {
                    acc[0][c] = __builtin_amdgcn_mfma_f32_32x32x16_f16(k.a0, k.b[c], acc[0][c], 0, 0, 0);
                    acc[1][c] = __builtin_amdgcn_mfma_f32_32x32x16_f16(k.a1, k.b[c], acc[1][c], 0, 0, 0);
                } else {
                    acc[0][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(k.a0, k.b[c], acc[0][c], 0, 0, 0);
                    acc[1][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(k.a1, k.b[c], acc[1][c], 0, 0, 0);
                }
            }
        };
        auto kmma = [&](const KOps<DT> &o) {
            KB<DT> k;
            kbuild(o, k);
            kmfma(k);
        };
        auto kstep = [&](int buf, int s) {
            kload(buf, s, cur);
            kmma(cur);
        };
        if (gx_tab) {
            // Tables (k_half_tables: rows of tab_stride values per grid column
            // / row of the region, valid up to n_in rounded up to kHK, zero
            // past n_in).  The next chunk's factors and node records are loaded
            // into registers one chunk ahead and stored to LDS after the
            // current chunk's MFMAs, so the loads' latency is hidden.
            // A chunk's slice of a table row is 64 values = 128 B, 8 pieces
            // of 16 B.  Workgroup thread e loads pieces e, e + 256, ... in
            // order, so 8 consecutive lanes read one row's aligned 128 B and
            // each load instruction touches 8 cache lines.
            auto store = [&](int jc, int nb) {
#pragma unroll
                for (int part = 0; part < kHTx * 8 / kFieldThreads; ++part)
                    *(V8 *)&L.gx[nb][part * kRowStep + tid / 8][8 * (tid % 8)] = pgx[part];
#pragma unroll
                for (int part = 0; part < kHTy * 8 / kFieldThreads; ++part)
                    *(V8 *)&L.gy[nb][part * kRowStep + tid / 8][8 * (tid % 8)] = pgy[part];
                if (wave == 3) {
                    float v[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
                    if (jc + lane < n_in) {
                        const float4 qj = make_float4(1.f + pr0.z, pr0.w, pr1.x, pr1.y);
                        const float4 qc = dq_mul(dq_mul(aq, qj), bq);
                        v[0] = ch0m1 + ch0 * pr0.z + sh0 * pr0.w;   // q'_c - 1
                        v[1] = qc.y;
                        v[2] = qc.z;
                        v[3] = qc.w;
                        v[4] = pr1.z - sm1;                           // s_j - s0
                    }
#pragma unroll
                    for (int c = 0; c < 5; ++c) L.qd[nb][c][lane] = (typename HalfT<DT>::Q)v[c];
                }
            };
            // Chunk c lives in buffer c % 3.  Iteration c multiplies chunk c,
            // stores chunk c + 2 (into the buffer chunk c - 1 used, free
            // since the previous barrier) and fetches chunk c + 3; chunk
            // c + 1 was stored before the previous barrier, so its first K
            // step is read while chunk c's last MFMAs run.
            store(0, 0);   // chunk 0 was fetched before the reference blend
            if (nchunks > 1) {
                fetch(kHK);
                store(kHK, 1);
            }
            if (nchunks > 2) fetch(2 * kHK);
            __syncthreads();
            // Software pipeline over K steps: step t issues the LDS reads of
            // step t + 1, then its own 12 MFMAs (operands formed during step
            // t - 1) interleaved with forming step t + 1's B operands, so
            // a single wavefront keeps the MFMA pipe fed.  The last step of a
            // chunk reads step 0 of the next chunk's buffer (after the last
            // chunk that is a stale buffer, read in bounds and never used).
            KB<DT> bcur, bnxt;
            kload(0, 0, cur);
            kbuild(cur, bcur);
            int buf = 0;
            if constexpr (EMDQ_HALF_AHEAD == 2) {
                // Two steps ahead: step t reads the operands of step t + 2,
                // issues its own MFMAs and forms step t + 1's B operands from
                // the reads of step t - 1, so no VALU waits on a read issued
                // in the same step.  Steps 0 and 1 of chunk c + 1 are read
                // during chunk c (that buffer was complete one barrier early).
                KOps<DT> nxt;
                kload(0, 1, cur);
                for (int c = 0; c < nchunks; ++c) {
                    const int nbuf = buf == 2 ? 0 : buf + 1;
#pragma unroll
                    for (int s = 0; s < 4; ++s) {
                        __builtin_amdgcn_sched_barrier(0);
                        kload(s < 2 ? buf : nbuf, (s + 2) & 3, nxt);
                        kmfma(bcur);
                        kbuild(cur, bnxt);
                        if constexpr (EMDQ_HALF_SPREAD) {
                            // one LDS read after each of the first 8 MFMAs,
                            // the products spread over all 12
#pragma unroll
                            for (int g = 0; g < 12; ++g) {
                                __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
                                if (g < 8) __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
                                __builtin_amdgcn_sched_group_barrier(0x002, DT == kDtF16 ? 2 : 8, 0);
                            }
                        } else {
                            // 8 LDS reads, then one MFMA per kHalfValu VALU
                            // instructions
                            __builtin_amdgcn_sched_group_barrier(0x100, 8, 0);
#pragma unroll
                            for (int g = 0; g < 12; ++g) {
                                __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
                                __builtin_amdgcn_sched_group_barrier(0x002, kHalfValu<DT>, 0);
                            }
                        }
                        __builtin_amdgcn_sched_barrier(0);
                        bcur = bnxt;
                        cur = nxt;
                    }
                    if (c + 2 < nchunks) {
                        store((c + 2) * kHK, nbuf == 2 ? 0 : nbuf + 1);
                        if (c + 3 < nchunks) fetch((c + 3) * kHK);
                    }
                    __syncthreads();
                    buf = nbuf;
                }
            } else
            for (int c = 0; c < nchunks; ++c) {
                const int nbuf = buf == 2 ? 0 : buf + 1;
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    __builtin_amdgcn_sched_barrier(0);
                    kload(s < 3 ? buf : nbuf, (s + 1) & 3, cur);
                    kmfma(bcur);
                    kbuild(cur, bnxt);
                    // 8 LDS reads, 4 MFMAs (the reads land), then one MFMA
                    // per kHalfValu VALU instructions
                    __builtin_amdgcn_sched_group_barrier(0x100, 8, 0);
                    __builtin_amdgcn_sched_group_barrier(0x008, kHalfLead, 0);
#pragma unroll
                    for (int g = 0; g < 12 - kHalfLead; ++g) {
                        __builtin_amdgcn_sched_group_barrier(0x002, kHalfValu<DT>, 0);
                        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
                    }
                    __builtin_amdgcn_sched_barrier(0);
                    bcur = bnxt;
                }
                if (c + 2 < nchunks) {
                    store((c + 2) * kHK, nbuf == 2 ? 0 : nbuf + 1);
                    if (c + 3 < nchunks) fetch((c + 3) * kHK);
                }
                __syncthreads();
                buf = nbuf;
            }
        } else {
#pragma unroll
            for (int part = 0; part < 4; ++part) gen(0, 0, part);
            __syncthreads();
            for (int c = 0; c < nchunks; ++c) {
                const int buf = c & 1;
                const bool more = c + 1 < nchunks;
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    kstep(buf, s);
                    if (more) gen((c + 1) * kHK, buf ^ 1, s);
                }
                __syncthreads();
            }
        }
    }

    // ---- FP16 range: a per-axis factor below FP16's normal range (2^-14)
    // is subnormal or zero, so inliers far from a pixel along an axis lose
    // their weight's precision or all of it.  Each such weight is below
    // 2^-24 in error, so where a pixel's weight sum is at least n_in 2^-13
    // the weight mass is off by at most 2^-11 of itself; a tile with a pixel
    // below that is left to the FP32 blend launched after this one
    // (tile_flags[tile] = 1, nothing written or merged here).
    if (tile_flags) {
        const float wmin = (float)n_in * 0x1p-13f;
        bool low = false;
#pragma unroll
        for (int bl = 0; bl < 2; ++bl)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int zx = px0 + 32 * wave + col;
                const int zy = py0 + 32 * bl + 8 * (r >> 2) + 4 * half + (r & 3);
                if (zx < zx0 + w && zy < zy0 + h && !(acc[bl][5][r] >= wmin)) low = true;
            }
        const bool tile_low = __syncthreads_or(low);
        if (tid == 0) tile_flags[blockIdx.x] = tile_low ? 1 : 0;
        if (tile_low) return;
    }

    // ---- epilogue: undo the coding, DQ normalisation, Eq. (1); the warp
    // merges the pixels in groups of kHGroup
    constexpr int kHGroup = 8;
    int pzx[kHGroup], pzy[kHGroup];
    float2 pd[kHGroup];
    bool live[kHGroup];
#pragma unroll
    for (int bl = 0; bl < 2; ++bl)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int zx = px0 + 32 * wave + col;
        const int zy = py0 + 32 * bl + 8 * (r >> 2) + 4 * half + (r & 3);
        const int gi = r % kHGroup;
        pzx[gi] = zx;
        pzy[gi] = zy;
        live[gi] = zx < zx0 + w && zy < zy0 + h;
        const float W = acc[bl][5][r];
        const float C = acc[bl][0][r] + W, S = acc[bl][1][r];
        const float X = acc[bl][2][r], Y = acc[bl][3][r];
        const float in2 = __builtin_amdgcn_rcpf(C * C + S * S), in = __builtin_amdgcn_sqrtf(in2);
        const float ch = C * in, sh = S * in;
        const float tx = 2.f * (C * X - S * Y) * in2, ty = 2.f * (S * X + C * Y) * in2;
        const float chc = ch0 * ch - sh0 * sh, shc = sh0 * ch + ch0 * sh;   // R0 R'
        const float ux = (float)zx - pcx, uy = (float)zy - pcy;
        const float ex = -2.f * shc * shc * ux - 2.f * chc * shc * uy + cos0 * tx - sin0 * ty + d0x;
        const float ey = 2.f * chc * shc * ux - 2.f * shc * shc * uy + sin0 * tx + cos0 * ty + d0y;
        const float sg = sm1 + acc[bl][4][r] * __builtin_amdgcn_rcpf(W);
        const float fzx = (float)zx, fzy = (float)zy;
        const float2 d = make_float2(ex + sg * (fzx + ex), ey + sg * (fzy + ey));
        pd[gi] = d;
        if constexpr (MODE == kModeField) {
            if (live[gi])
                out[(size_t)(zy - zy0) * opitch + (zx - zx0)] =
                    bad ? make_float2(__builtin_nanf(""), __builtin_nanf(""))
                        : make_float2(fzx + d.x, fzy + d.y);
        } else if constexpr (!EMDQ_WARP_BATCH) {
            if (live[gi]) warp_merge(zx, zy, d, frame, fw, fh, fpitch, canvas, cpitch, ox, oy);
        } else if (gi == kHGroup - 1) {
            warp_merge_batch<kHGroup>(pzx, pzy, pd, live, zx0, zy0, frame, fw, fh, fpitch, canvas,
                                      cpitch, ox, oy);
        }
    }
}

// Per-axis Gaussian factors of the half-precision blend, once per launch:
// row c of the x table holds gx(zx0 + c, j) = exp(-alpha (zx0 + c - x_j)^2),
// row r of the y table likewise for zy0 + r.  Each thread loads eight
// consecutive coordinates x_j once and writes them into kTabRowsPer rows
// (workgroup row blockIdx.y covers rows [kTabRowsPer blockIdx.y, +kTabRowsPer),
// x rows first; both row counts are multiples of kTabRowsPer).  Only j below
// n_in rounded up to the blend's K chunk is written (zero for j >= n_in): the
// blend reads no further.
constexpr int kTabRowsPer = 16;
static_assert(kHTx % kTabRowsPer == 0 && kHTy % kTabRowsPer == 0, "table row blocks");
template <int DT>
__global__ __launch_bounds__(256) void k_half_tables(
    const float *__restrict__ xs, const float *__restrict__ ys,
    const DevState *__restrict__ st, float ka, int zx0, int zy0, int rows_x, int tab_stride,
    void *__restrict__ gx_tab, void *__restrict__ gy_tab) {
    using T = typename HalfT<DT>::T;
    using V8 = typename HalfT<DT>::V8;
    const int n_in = st->status < 0 ? 0 : st->n_in;
    const int lim = min(tab_stride, (n_in + kHK - 1) / kHK * kHK);
    const int j0 = 8 * (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (j0 >= lim) return;
    const int row0 = kTabRowsPer * (int)blockIdx.y;
    const bool is_x = row0 < rows_x;
    const int r0 = is_x ? row0 : row0 - rows_x;
    const float *src = is_x ? xs : ys;
    // all eight loads in flight at once (n_in >= 1 here; indices clamped)
    float c[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) c[i] = ka * src[min(j0 + i, n_in - 1)];
    T *dst = (T *)(is_x ? gx_tab : gy_tab) + (size_t)r0 * tab_stride + j0;
    const int z0 = (is_x ? zx0 : zy0) + r0;
#pragma unroll 4
    for (int k = 0; k < kTabRowsPer; ++k) {
        const float za = ka * (float)(z0 + k);
        V8 v;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const float d = c[i] - za;
            v[i] = (T)(j0 + i < n_in ? fast_exp2(-(d * d)) : 0.f);
        }
        *(V8 *)(dst + (size_t)k * tab_stride) = v;
    }
}

// ---------------------------------------------- node tracking, uncertainty ----

__device__ __forceinline__ float wave_min(float v) {
    for (int off = 32; off >= 1; off >>= 1) v = fminf(v, __shfl_xor(v, off, kWave));
    return v;
}

// One tracking step of m deformation nodes against the model's inliers
// (Sec. III-C and III-E), one wavefront per node, lanes over the inliers:
//   (ds, dq) = blend at the node's position p (Eqs. (2)-(3)), normalised;
//   dsig2 = exp(beta d_min^2), d_min the distance to the nearest inlier
//           (Eq. (8): exp is increasing, so its minimum is at d_min);
//   App. A: q1 = translation by (1 - s)/s times the translation of dq,
//           q <- the motion "q, then dq, then q1", s <- ds s;
//   Eq. (9): sig2 <- ds^2 sig2 + dsig2;   p <- ds dq(p)  (Eq. (1)).
// A node with no weight (or a failed model) gets NaN everywhere.
__global__ __launch_bounds__(kEmThreads) void k_track(
    const float4 *__restrict__ packed, const DevState *__restrict__ st, float nal2, float beta,
    int m, float2 *__restrict__ pos, float *__restrict__ scale, float4 *__restrict__ q,
    float *__restrict__ sig2) {
    const int lane = threadIdx.x & (kWave - 1);
    const int i = blockIdx.x * kRowsPerBlock + (threadIdx.x >> 6);
    if (i >= m) return;
    const int n_in = st->n_in;
    const bool bad = st->status < 0 || n_in <= 0;
    const float2 p = pos[i];
    float W = 0.f, Gd = 0.f, Cd = 0.f, Sn = 0.f, X = 0.f, Y = 0.f;
    float d2min = __builtin_huge_valf();
    if (!bad)
        for (int j = lane; j < n_in; j += kWave) {
            const float4 r0 = packed[2 * j], r1 = packed[2 * j + 1];
            const float dx = r0.x - p.x, dy = r0.y - p.y;
            const float d2 = dx * dx + dy * dy;
            const float w = fast_exp2(nal2 * d2);
            W += w;
            Cd += w * r0.z;
            Sn += w * r0.w;
            X += w * r1.x;
            Y += w * r1.y;
            Gd += w * r1.z;
            d2min = fminf(d2min, d2);
        }
    W = wave_sum(W);
    Gd = wave_sum(Gd);
    Cd = wave_sum(Cd);
    Sn = wave_sum(Sn);
    X = wave_sum(X);
    Y = wave_sum(Y);
    d2min = wave_min(d2min);
    if (lane != 0) return;
    if (bad || !(W > 0.f)) {
        const float nan = __builtin_nanf("");
        pos[i] = make_float2(nan, nan);
        scale[i] = nan;
        q[i] = make_float4(nan, nan, nan, nan);
        sig2[i] = nan;
        return;
    }
    const float iW = 1.f / W;
    const float c = 1.f + Cd * iW, sn = Sn * iW, bx = X * iW, by = Y * iW, ds = 1.f + Gd * iW;
    const float in = 1.f / sqrtf(c * c + sn * sn);
    const float4 dq = make_float4(c * in, sn * in, bx * in, by * in);
    const float tx = 2.f * (dq.x * dq.z - dq.y * dq.w), ty = 2.f * (dq.y * dq.z + dq.x * dq.w);
    const float2 d = blend_displacement(W, Cd, Sn, X, Y, Gd, p.x, p.y);
    const float so = scale[i];
    const float k = (1.f - so) / so;
    const float4 q1 = make_float4(1.f, 0.f, 0.5f * k * tx, 0.5f * k * ty);
    float4 qn = dq_mul(dq_mul(q1, dq), q[i]);
    float nr = 1.f / sqrtf(qn.x * qn.x + qn.y * qn.y);
    if (qn.x < 0.f) nr = -nr;   // canonical sign, q_c >= 0
    q[i] = make_float4(qn.x * nr, qn.y * nr, qn.z * nr, qn.w * nr);
    scale[i] = ds * so;
    sig2[i] = ds * ds * sig2[i] + expf(beta * d2min);
    pos[i] = make_float2(p.x + d.x, p.y + d.y);
}

// Eq. (8) at every grid point z = (zx0 + i, zy0 + k): exp(beta d_min(z)^2),
// d_min the distance to the nearest inlier.  Workgroup tile 64 x 64 with
// centre c and half-diagonal r.  If D is the distance from c to its nearest
// inlier, every pixel of the tile has an inlier within D + r, and an inlier
// farther than D + 2r from c is farther than D + r from every pixel: only
// the inliers within D + 2r of c (plus 1 px against rounding) are scanned.
// The minimum does not depend on the scan order, so the candidate list is
// built with LDS atomics and the result is still deterministic.
constexpr int kUTile = 64, kUChunk = 2048, kUThreads = 256;

__global__ __launch_bounds__(kUThreads) void k_uncertainty(
    const float4 *__restrict__ packed, const DevState *__restrict__ st, float beta, int zx0,
    int zy0, int w, int h, int tiles_x, float *__restrict__ out) {
    __shared__ float2 cand[kUChunk];
    __shared__ float red[kUThreads / kWave];
    __shared__ int ncand;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid >> 6;
    const int n_in = st->n_in;
    const bool bad = st->status < 0 || n_in <= 0;
    const int px0 = zx0 + (int)(blockIdx.x % tiles_x) * kUTile;
    const int py0 = zy0 + (int)(blockIdx.x / tiles_x) * kUTile;
    const float cx = (float)px0 + 0.5f * (kUTile - 1), cy = (float)py0 + 0.5f * (kUTile - 1);
    constexpr float kHalfDiag = 0.5f * (kUTile - 1) * 1.41421357f;
    const int zx = px0 + lane;
    float m2[kUTile / 4];
#pragma unroll
    for (int k = 0; k < kUTile / 4; ++k) m2[k] = __builtin_huge_valf();
    if (!bad) {
        float dmin = __builtin_huge_valf();
        for (int j = tid; j < n_in; j += kUThreads) {
            const float4 r0 = packed[2 * j];
            const float dx = r0.x - cx, dy = r0.y - cy;
            dmin = fminf(dmin, sqrtf(dx * dx + dy * dy));
        }
        dmin = wave_min(dmin);
        if (lane == 0) red[wave] = dmin;
        __syncthreads();
        dmin = fminf(fminf(red[0], red[1]), fminf(red[2], red[3]));
        const float lim = dmin + 2.f * kHalfDiag + 1.f;
        for (int c0 = 0; c0 < n_in; c0 += kUChunk) {
            if (tid == 0) ncand = 0;
            __syncthreads();
            const int c1 = min(c0 + kUChunk, n_in);
            for (int j = c0 + tid; j < c1; j += kUThreads) {
                const float4 r0 = packed[2 * j];
                const float dx = r0.x - cx, dy = r0.y - cy;
                if (sqrtf(dx * dx + dy * dy) <= lim) cand[atomicAdd(&ncand, 1)] = make_float2(r0.x, r0.y);
            }
            __syncthreads();
            const int nc = ncand;
            for (int t = 0; t < nc; ++t) {
                const float2 v = cand[t];
                const float ex = (float)zx - v.x, ax = ex * ex;
#pragma unroll
                for (int k = 0; k < kUTile / 4; ++k) {
                    const float ey = (float)(py0 + wave + 4 * k) - v.y;
                    m2[k] = fminf(m2[k], fmaf(ey, ey, ax));
                }
            }
            __syncthreads();
        }
    }
    if (zx >= zx0 + w) return;
#pragma unroll
    for (int k = 0; k < kUTile / 4; ++k) {
        const int zy = py0 + wave + 4 * k;
        if (zy >= zy0 + h) break;
        out[(size_t)(zy - zy0) * w + (zx - zx0)] = bad ? __builtin_nanf("") : expf(beta * m2[k]);
    }
}

// ------------------------------------------------------ learned EM start ----
//
// A per-match inlier prior to start the EM from (not in the paper; the
// start p = 1 stays the default).  Match i looks at its 16 nearest other
// matches by source distance, ordered by (squared distance in FP64, index);
// per neighbour j the features are g (x_j - x_i) and ss((d_j - d_i) / 8),
// g = sqrt(alpha), d = dst - src, ss(t) = t / (1 + |t|); a 64 -> 128 -> 128
// -> 1 network with GELU layers and a sigmoid output maps them to p.
// Weights: W1[128][64], b1, W2[128][128], b2, w3[128], b3 (FP32, flat).
constexpr int kKnn = 16, kNFeat = 4 * kKnn, kNHid = 128;
constexpr int kStartWaves = 8, kStartThreads = kStartWaves * kWave;
static_assert(kNHid * kNFeat + kNHid + kNHid * kNHid + kNHid + kNHid + 1 == 24961,
              "weight vector size stated in the header");

// Neighbour search of pairs up to kGridMaxN matches: a uniform grid of at
// most kGridDim x kGridDim cells over the bounding box of the finite source
// points (about two per cell), counting-sorted into LDS by every workgroup.
constexpr int kGridMaxN = 7168, kGridDim = 50, kGridMaxCells = kGridDim * kGridDim;
static_assert(kGridMaxN % kStartThreads == 0, "grid points split evenly over the threads");

// The network runs on BF16 MFMA (v_mfma_f32_32x32x16_bf16, FP32
// accumulation) for a block of kMlpRows matches of a workgroup at a time, both
// layers transposed (outputs x matches):
//   layer 1  H1^T = W1 F^T:  A = W1 rows (16 features a step), B = the
//            block's features (from LDS, rounded to BF16);
//   layer 2  H2^T = W2 H1^T: B = H1 = bf16(gelu(layer 1 + b1)), written to
//            LDS by layer 1 (match-major, so it reads like the features);
//   output   z = w3 . gelu(H2^T + b2) + b3: each lane adds its rows, the two
//            halves are added, then the four output blocks in block order;
//            p = 1 / (1 + e^-z).
// Wavefront w < 4 computes output block w of each layer.  Rows are padded by
// 16 bytes against LDS bank conflicts.
constexpr int kMlpRows = 32;
constexpr int kMlpRounds = kMlpRows / 8;   // rounds of one match per wavefront
constexpr int kW1Stride = kNFeat + 8, kW2Stride = kNHid + 8, kFStride = kNFeat + 8;

struct alignas(16) StartLds {
    __bf16 w1[kNHid][kW1Stride];    // W1 rows (features contiguous)
    __bf16 w2[kNHid][kW2Stride];    // W2 rows
    float b1[kNHid], b2[kNHid], w3[kNHid];
    __bf16 f[kMlpRows][kFStride];   // features of the block's matches
    __bf16 h1[kMlpRows][kW2Stride]; // layer-1 output of the block's matches
    float zpart[4][kMlpRows];       // logit shares of the four output blocks
    float2 gp[kGridMaxN];        // points in cell order
    uint16_t gi[kGridMaxN];      // their match indices
    int gs[kGridMaxCells + 1];   // first point of every cell (counts while built)
    float gbox[kStartWaves][4];  // bounding-box partials, then (x0, y0, sx, sy)
    float gmargin;               // rounding allowance of the cell assignment
    int gbad[kStartWaves];       // a non-finite point seen by the wavefront
    int gdim[2];                 // nx, ny (nx = 0: no grid, every pair scanned)
    double kd[kStartWaves][kWave];   // candidates of the rank merge: distance
    int kj[kStartWaves][kWave];      // and index
};

__device__ __forceinline__ float gelu(float t) {
    return 0.5f * t * (1.f + erff(t * 0.70710678118654752f));
}

// GELU of the inference network with erf from the rational-exponential
// approximation of Abramowitz & Stegun (Handbook of Mathematical Functions,
// formula 7.1.26, after Hastings): erf(x) = 1 - t (a1 + t (a2 + t (a3 + t (a4 +
// t a5)))) e^(-x^2), t = 1 / (1 + p x), x >= 0, odd in x; absolute error below
// 1.5e-7.  Branch-free, a third of the instructions of the library erf; the
// network's inputs to it are then rounded to BF16 or summed into the logit,
// where this error is far below the BF16 rounding step.
__device__ __forceinline__ float gelu_fast(float t) {
    const float x = fabsf(t) * 0.70710678118654752f;
    const float u = __builtin_amdgcn_rcpf(1.f + 0.3275911f * x);
    const float poly =
        u * (0.254829592f + u * (-0.284496736f + u * (1.421413741f + u * (-1.453152027f + u * 1.061405429f))));
    const float e = 1.f - poly * fast_exp2(-kLog2e * x * x);   // erf(|t| / sqrt 2)
    return 0.5f * t * (1.f + copysignf(e, t));
}

// (a, ia) < (b, ib) lexicographically
__device__ __forceinline__ bool key_less(double a, int ia, double b, int ib) {
    return a < b || (a == b && ia < ib);
}

__device__ __forceinline__ double dist2_f64(float2 a, float2 b) {
#pragma clang fp contract(off)
    const double dx = (double)b.x - (double)a.x, dy = (double)b.y - (double)a.y;
    return dx * dx + dy * dy;   // rounded as written, no fused multiply-add
}

// grid cell of a coordinate (the same arithmetic when sorting and searching)
__device__ __forceinline__ int grid_cell(float v, float v0, float sv, int nv) {
    return min((int)((v - v0) / sv), nv - 1);
}


// The network on the block of kMlpRows matches whose features are in L.f
// (see StartLds): wavefront w < 4 computes output block w of each layer;
// row r's output goes to p_out[match_of(r)] when that is below n.  Three
// barriers; the block's features may be overwritten after the second.
template <class MatchOf>
__device__ __forceinline__ void start_mlp(StartLds &L, int wave, int lane, float b3,
                                          float *__restrict__ p_out, int n,
                                          const MatchOf &match_of) {
    const int col = lane & 31, half = lane >> 5;
    if (wave < 4) {
        const int ob = wave;
        f32x16 acc;
#pragma unroll
        for (int q = 0; q < 16; ++q) acc[q] = 0.f;
#pragma unroll
        for (int ks = 0; ks < kNFeat / 16; ++ks) {
            const bhalf8 wa = *(const bhalf8 *)&L.w1[32 * ob + col][16 * ks + 8 * half];
            const bhalf8 fb = *(const bhalf8 *)&L.f[col][16 * ks + 8 * half];
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wa, fb, acc, 0, 0, 0);
        }
        // H1[match][output] = bf16(gelu(layer 1 + b1))
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int o = 32 * ob + 8 * (q >> 2) + 4 * half + (q & 3);
            L.h1[col][o] = (__bf16)gelu_fast(acc[q] + L.b1[o]);
        }
    }
    __syncthreads();
    if (wave < 4) {
        const int ob2 = wave;
        f32x16 acc;
#pragma unroll
        for (int q = 0; q < 16; ++q) acc[q] = 0.f;
#pragma unroll
        for (int kk = 0; kk < kNHid / 16; ++kk) {
            const bhalf8 wa = *(const bhalf8 *)&L.w2[32 * ob2 + col][16 * kk + 8 * half];
            const bhalf8 hb = *(const bhalf8 *)&L.h1[col][16 * kk + 8 * half];
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wa, hb, acc, 0, 0, 0);
        }
        // this output block's share of the logit of match col: the lane's 16
        // rows, then the two halves (same order in both)
        float zp = 0.f;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int o = 32 * ob2 + 8 * (q >> 2) + 4 * half + (q & 3);
            zp += L.w3[o] * gelu_fast(acc[q] + L.b2[o]);
        }
        const float zo = __shfl_xor(zp, 32, kWave);
        if (half == 0) L.zpart[ob2][col] = zp + zo;
    }
    __syncthreads();
    if (wave == 0 && lane < kMlpRows) {
        // the four output blocks' shares added in block order
        const float z = ((L.zpart[0][lane] + L.zpart[1][lane]) + L.zpart[2][lane]) +
                        L.zpart[3][lane] + b3;
        const int im = match_of(lane);
        if (im < n) p_out[im] = 1.f / (1.f + expf(-z));
    }
}

// With feat_out set, the features are written out ([n][64]) and the network
// is not evaluated (wts and p_out unused).
__device__ __forceinline__ void start_body(const float2 *__restrict__ src,
                                           const float2 *__restrict__ dst, int n, float g,
                                           const float *__restrict__ wts,
                                           float *__restrict__ p_out,
                                           float *__restrict__ feat_out, int block,
                                           int nblocks, int lanes) {
    __shared__ StartLds L;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid >> 6;
    // lanes > 0: the grid search takes one match per lane, lanes matches per
    // wavefront, kStartWaves * lanes per workgroup and round; the workgroups
    // past the pair's matches have nothing to do (and every path below
    // strides over the others only)
    if (lanes > 0) {
        nblocks = min(nblocks, (n + kStartWaves * lanes - 1) / (kStartWaves * lanes));
        if (block >= nblocks) return;
    }
    float b3 = 0.f;
    if (!feat_out) {
        const float *W1 = wts, *B1 = W1 + kNHid * kNFeat, *W2 = B1 + kNHid;
        const float *B2 = W2 + kNHid * kNHid, *W3 = B2 + kNHid, *B3 = W3 + kNHid;
        // every load is issued before the first store (the pointer could
        // alias LDS as far as the compiler knows, which would otherwise keep
        // one load in flight at a time)
        constexpr int kR1 = kNHid * kNFeat / kStartThreads, kR2 = kNHid * kNHid / kStartThreads;
        static_assert(kR1 * kStartThreads == kNHid * kNFeat && kR2 * kStartThreads == kNHid * kNHid,
                      "weight matrices split evenly over the threads");
        float r1[kR1], r2[kR2];
#pragma unroll
        for (int k = 0; k < kR1; ++k) r1[k] = W1[tid + k * kStartThreads];
#pragma unroll
        for (int k = 0; k < kR2; ++k) r2[k] = W2[tid + k * kStartThreads];
        // rounded to BF16 (nearest, ties to even)
#pragma unroll
        for (int k = 0; k < kR1; ++k) {
            const int t = tid + k * kStartThreads;
            L.w1[t / kNFeat][t % kNFeat] = (__bf16)r1[k];
        }
#pragma unroll
        for (int k = 0; k < kR2; ++k) {
            const int t = tid + k * kStartThreads;
            L.w2[t / kNHid][t % kNHid] = (__bf16)r2[k];
        }
        for (int t = tid; t < kNHid; t += kStartThreads) {
            L.b1[t] = B1[t];
            L.b2[t] = B2[t];
            L.w3[t] = W3[t];
        }
        b3 = B3[0];
        // the weights are complete at the grid's first barrier, or at this one
        if (n > kGridMaxN) __syncthreads();
    }

    // ---- grid of the source points (pairs up to kGridMaxN matches); each
    // thread keeps its points in registers for the three passes
    constexpr int kPerThread = kGridMaxN / kStartThreads;
    bool grid = n <= kGridMaxN;
    float2 pv[kPerThread];
    if (grid) {
#pragma unroll
        for (int k = 0; k < kPerThread; ++k) {
            const int j = tid + k * kStartThreads;
            if (j < n) {
                pv[k] = src[j];
            } else {
                pv[k].x = __builtin_huge_valf();   // beyond n: never used
                pv[k].y = 0.f;
            }
        }
        float lo_x = __builtin_huge_valf(), lo_y = __builtin_huge_valf();
        float hi_x = -__builtin_huge_valf(), hi_y = -__builtin_huge_valf();
        bool bad = false;
#pragma unroll
        for (int k = 0; k < kPerThread; ++k) {
            if (tid + k * kStartThreads >= n) continue;
            const float2 v = pv[k];
            if (finite2(v)) {
                lo_x = fminf(lo_x, v.x);
                lo_y = fminf(lo_y, v.y);
                hi_x = fmaxf(hi_x, v.x);
                hi_y = fmaxf(hi_y, v.y);
            } else {
                bad = true;
            }
        }
        const bool wave_bad = __any(bad);
        for (int off = 32; off >= 1; off >>= 1) {
            lo_x = fminf(lo_x, __shfl_xor(lo_x, off, kWave));
            lo_y = fminf(lo_y, __shfl_xor(lo_y, off, kWave));
            hi_x = fmaxf(hi_x, __shfl_xor(hi_x, off, kWave));
            hi_y = fmaxf(hi_y, __shfl_xor(hi_y, off, kWave));
        }
        if (lane == 0) {
            L.gbox[wave][0] = lo_x;
            L.gbox[wave][1] = lo_y;
            L.gbox[wave][2] = hi_x;
            L.gbox[wave][3] = hi_y;
            L.gbad[wave] = wave_bad ? 1 : 0;
        }
        for (int c = tid; c <= kGridMaxCells; c += kStartThreads) L.gs[c] = 0;
        __syncthreads();
        if (tid == 0) {
            int any_bad = L.gbad[0];
            for (int w = 1; w < kStartWaves; ++w) {
                lo_x = fminf(lo_x, L.gbox[w][0]);
                lo_y = fminf(lo_y, L.gbox[w][1]);
                hi_x = fmaxf(hi_x, L.gbox[w][2]);
                hi_y = fmaxf(hi_y, L.gbox[w][3]);
                any_bad |= L.gbad[w];
            }
            int nx = 1, ny = 1;
            float sx = 1.f, sy = 1.f;
            if (lo_x <= hi_x) {   // some point is finite
                const float ex = hi_x - lo_x, ey = hi_y - lo_y;
                const float cells = fmaxf(1.f, 0.5f * (float)n);
                float side = sqrtf(ex * ey / cells);
                side = fmaxf(side, fmaxf(ex, ey) / (float)kGridDim);
                if (side > 0.f) {
                    nx = min(max((int)ceilf(ex / side), 1), kGridDim);
                    ny = min(max((int)ceilf(ey / side), 1), kGridDim);
                }
                if (ex > 0.f) sx = ex / (float)nx;
                if (ey > 0.f) sy = ey / (float)ny;
            } else {
                lo_x = lo_y = 0.f;
            }
            // a cell index below xa (above xb) puts a point left of x0 + xa sx
            // (right of x0 + (xb + 1) sx) up to the rounding of the
            // subtraction and the division: a few units in the last place of
            // the coordinates, far inside this allowance
            const float mag = fmaxf(fmaxf(fabsf(lo_x), fabsf(hi_x)), fmaxf(fabsf(lo_y), fabsf(hi_y)));
            L.gmargin = 1e-4f * fmaxf(sx, sy) + 4e-6f * mag;
            L.gbox[0][0] = lo_x;
            L.gbox[0][1] = lo_y;
            L.gbox[0][2] = sx;
            L.gbox[0][3] = sy;
            L.gdim[0] = any_bad ? 0 : nx;   // non-finite points: scan every pair
            L.gdim[1] = ny;
        }
        __syncthreads();
        grid = L.gdim[0] > 0;   // the same in every thread of the workgroup
    }
    if (grid) {
        const float gx0 = L.gbox[0][0], gy0 = L.gbox[0][1], gsx = L.gbox[0][2], gsy = L.gbox[0][3];
        const int gnx = L.gdim[0], gny = L.gdim[1];
#pragma unroll
        for (int k = 0; k < kPerThread; ++k) {   // counts
            if (tid + k * kStartThreads >= n) continue;
            const float2 v = pv[k];
            if (finite2(v))
                atomicAdd(&L.gs[grid_cell(v.y, gy0, gsy, gny) * gnx +
                                grid_cell(v.x, gx0, gsx, gnx) + 1], 1);
        }
        __syncthreads();
        if (wave == 0) {   // inclusive scan of the counts: gs[c] = first point of cell c
            int carry = 0;
            for (int c0 = 1; c0 <= gnx * gny; c0 += kWave) {
                int v = c0 + lane <= gnx * gny ? L.gs[c0 + lane] : 0;
                for (int off = 1; off < kWave; off <<= 1) {
                    const int u = __shfl_up(v, off, kWave);
                    if (lane >= off) v += u;
                }
                if (c0 + lane <= gnx * gny) L.gs[c0 + lane] = v + carry;
                carry += __shfl(v, kWave - 1, kWave);
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kPerThread; ++k) {   // scatter (order within a cell free)
            const int j = tid + k * kStartThreads;
            if (j >= n) continue;
            const float2 v = pv[k];
            if (finite2(v)) {
                const int c = grid_cell(v.y, gy0, gsy, gny) * gnx + grid_cell(v.x, gx0, gsx, gnx);
                const int pos = atomicAdd(&L.gs[c], 1);
                L.gp[pos] = v;
                L.gi[pos] = (uint16_t)j;
            }
        }
        __syncthreads();
        // gs[c] now holds the end of cell c, i.e. the start of cell c + 1
        if (lanes > 0) {
            // each cell's points by match index, so that a position in the
            // grid names the same match in every workgroup of the pair (the
            // one-match-per-lane rounds go by position)
            for (int c = tid; c < gnx * gny; c += kStartThreads) {
                const int a = c == 0 ? 0 : L.gs[c - 1], e = L.gs[c];
                for (int u = a + 1; u < e; ++u) {   // insertion sort, a few points
                    const uint16_t key = L.gi[u];
                    const float2 pt = L.gp[u];
                    int v = u - 1;
                    for (; v >= a && L.gi[v] > key; --v) {
                        L.gi[v + 1] = L.gi[v];
                        L.gp[v + 1] = L.gp[v];
                    }
                    L.gi[v + 1] = key;
                    L.gp[v + 1] = pt;
                }
            }
            __syncthreads();
        }
    }

    if (lanes > 0 && grid) {
        // ---- one match per lane: each lane searches the rings of cells
        // around its match on its own (the same rings and stopping rule as
        // below), keeping its sorted list of the 16 nearest by (squared
        // distance, index) -- the neighbours themselves, in order.  The
        // matches are taken in the grid's cell order (every point is finite
        // here), so the lanes of a wavefront search neighbouring cells.
        const float gx0 = L.gbox[0][0], gy0 = L.gbox[0][1];
        const float gsx = L.gbox[0][2], gsy = L.gbox[0][3];
        const int gnx = L.gdim[0], gny = L.gdim[1];
        const double margin = (double)L.gmargin;
        const int per_round = kStartWaves * lanes;
        const int li = wave * lanes + lane;   // the lane's place in a round
        for (int base = block * per_round; base < n; base += nblocks * per_round) {
            const int pos = base + li;
            const bool act = lane < lanes && pos < n;
            const int i = act ? (int)L.gi[pos] : 0;
            double bd[kKnn];
            int bj[kKnn];
#pragma unroll
            for (int k = 0; k < kKnn; ++k) { bd[k] = __builtin_huge_val(); bj[k] = 0x7fffffff; }
            auto insert = [&](double d2, int j) {
                if (!key_less(d2, j, bd[kKnn - 1], bj[kKnn - 1])) return;
#pragma unroll
                for (int k = kKnn - 1; k >= 1; --k) {
                    const bool shift = key_less(d2, j, bd[k - 1], bj[k - 1]);
                    const bool here = !shift && key_less(d2, j, bd[k], bj[k]);
                    bd[k] = shift ? bd[k - 1] : (here ? d2 : bd[k]);
                    bj[k] = shift ? bj[k - 1] : (here ? j : bj[k]);
                }
                if (key_less(d2, j, bd[0], bj[0])) { bd[0] = d2; bj[0] = j; }
            };
            const float2 xi = act ? L.gp[pos] : make_float2(0.f, 0.f);
            if (act) {
                const int cx = grid_cell(xi.x, gx0, gsx, gnx), cy = grid_cell(xi.y, gy0, gsy, gny);
                auto cell_start = [&](int c) { return c == 0 ? 0 : L.gs[c - 1]; };
                auto row = [&](int y, int xa, int xb) {   // cells xa..xb of row y
                    const int e = L.gs[y * gnx + xb];
                    for (int q = cell_start(y * gnx + xa); q < e; ++q) {
                        const int j = L.gi[q];
                        if (j != i) insert(dist2_f64(xi, L.gp[q]), j);
                    }
                };
                for (int R = 0;; ++R) {
                    const int xa = max(cx - R, 0), xb = min(cx + R, gnx - 1);
                    const int ya = max(cy - R, 0), yb = min(cy + R, gny - 1);
                    if (R == 0) {
                        row(cy, cx, cx);
                    } else {
                        if (cy - R >= 0) row(cy - R, xa, xb);
                        if (cy + R < gny) row(cy + R, xa, xb);
                        for (int y = max(cy - R + 1, 0); y <= min(cy + R - 1, gny - 1); ++y) {
                            if (cx - R >= 0) row(y, cx - R, cx - R);
                            if (cx + R < gnx) row(y, cx + R, cx + R);
                        }
                    }
                    if (xa == 0 && xb == gnx - 1 && ya == 0 && yb == gny - 1) break;
                    double bound = __builtin_huge_val();
                    if (xa > 0) bound = fmin(bound, (double)xi.x - ((double)gx0 + (double)xa * gsx));
                    if (xb < gnx - 1)
                        bound = fmin(bound, ((double)gx0 + (double)(xb + 1) * gsx) - (double)xi.x);
                    if (ya > 0) bound = fmin(bound, (double)xi.y - ((double)gy0 + (double)ya * gsy));
                    if (yb < gny - 1)
                        bound = fmin(bound, ((double)gy0 + (double)(yb + 1) * gsy) - (double)xi.y);
                    bound -= margin;
                    // 16 kept candidates closer than any unsearched point
                    if (bound > 0.0 && bd[kKnn - 1] < bound * bound) break;
                }
            }
            // ---- features of neighbour k (zero where fewer than 16 exist)
            float4 fv[kKnn];
            const float2 yi = act ? dst[i] : make_float2(0.f, 0.f);
#pragma unroll
            for (int k = 0; k < kKnn; ++k) {
                fv[k] = make_float4(0.f, 0.f, 0.f, 0.f);
                if (act && bj[k] != 0x7fffffff) {
                    const float2 xj = src[bj[k]], yj = dst[bj[k]];
                    float ex = ((yj.x - xj.x) - (yi.x - xi.x)) * 0.125f;
                    float ey = ((yj.y - xj.y) - (yi.y - xi.y)) * 0.125f;
                    fv[k] = make_float4(g * (xj.x - xi.x), g * (xj.y - xi.y),
                                        ex / (1.f + fabsf(ex)), ey / (1.f + fabsf(ey)));
                }
            }
            if (feat_out) {
                if (act)
#pragma unroll
                    for (int k = 0; k < kKnn; ++k)
                        *(float4 *)&feat_out[(size_t)i * kNFeat + 4 * k] = fv[k];
                continue;
            }
            // ---- the network on blocks of kMlpRows consecutive places
            for (int b0 = 0; b0 < per_round && base + b0 < n; b0 += kMlpRows) {   // uniform
                if (lane < lanes && li >= b0 && li < b0 + kMlpRows) {   // its own row
#pragma unroll
                    for (int k = 0; k < kKnn; ++k) {
                        bhalf4 fb;
                        fb[0] = (__bf16)fv[k].x;
                        fb[1] = (__bf16)fv[k].y;
                        fb[2] = (__bf16)fv[k].z;
                        fb[3] = (__bf16)fv[k].w;
                        *(bhalf4 *)&L.f[li - b0][4 * k] = fb;
                    }
                }
                __syncthreads();   // the block's features are complete
                const int lim = min(n, base + per_round);
                start_mlp(L, wave, lane, b3, p_out, n, [&](int r) {
                    const int q = base + b0 + r;
                    return q < lim ? (int)L.gi[q] : n;
                });
            }
        }
        return;
    }

    // The workgroup's matches in rounds t = 0, 1, ...: in round t wavefront w
    // takes match (block + t nblocks) kStartWaves + w.  Rounds are grouped by
    // kMlpRounds: the features of a group's matches (one per wavefront and
    // round) fill rows 8 (t % kMlpRounds) + w of the workgroup's block, then
    // the network runs once on the block.
    const int stride = nblocks * kStartWaves;
    for (int g0 = block * kStartWaves; g0 < n; g0 += kMlpRounds * stride) {   // workgroup-uniform
    for (int t = 0; t < kMlpRounds; ++t) {
        const int r = kStartWaves * t + wave;   // row of the block
        const int i = g0 + t * stride + wave;
        if (i >= n) {   // rows past the last match: zero features, no output
            if (!feat_out && lane < kKnn)
                *(uint2 *)&L.f[r][4 * lane] = make_uint2(0u, 0u);
            continue;
        }
        const float2 xi = src[i];
        // ---- per-lane sorted lists of the 16 nearest by (squared distance,
        // index)
        double bd[kKnn];
        int bj[kKnn];
#pragma unroll
        for (int k = 0; k < kKnn; ++k) { bd[k] = __builtin_huge_val(); bj[k] = 0x7fffffff; }
        double thresh = 0.0;   // grid search: the 16 nearest lie below it
        auto insert = [&](double d2, int j) {
            if (!key_less(d2, j, bd[kKnn - 1], bj[kKnn - 1])) return;
#pragma unroll
            for (int k = kKnn - 1; k >= 1; --k) {
                const bool shift = key_less(d2, j, bd[k - 1], bj[k - 1]);
                const bool here = !shift && key_less(d2, j, bd[k], bj[k]);
                bd[k] = shift ? bd[k - 1] : (here ? d2 : bd[k]);
                bj[k] = shift ? bj[k - 1] : (here ? j : bj[k]);
            }
            if (key_less(d2, j, bd[0], bj[0])) { bd[0] = d2; bj[0] = j; }
        };
        if (!grid) {
            for (int j = lane; j < n; j += kWave)
                if (j != i) insert(dist2_f64(xi, src[j]), j);
        } else {
            // Rings of cells around the match's cell, each ring searched
            // whole, until 16 of the kept candidates lie closer than the
            // nearest unsearched cell can: every point outside the searched
            // square is at least the distance to its edge (less a margin for
            // the rounding of the cell assignment).
            const float gx0 = L.gbox[0][0], gy0 = L.gbox[0][1];
            const float gsx = L.gbox[0][2], gsy = L.gbox[0][3];
            const int gnx = L.gdim[0], gny = L.gdim[1];
            const int cx = grid_cell(xi.x, gx0, gsx, gnx), cy = grid_cell(xi.y, gy0, gsy, gny);
            const double margin = (double)L.gmargin;
            thresh = __builtin_huge_val();
            auto range = [&](int a, int b) {   // points [a, b)
                for (int q = a + lane; q < b; q += kWave) {
                    const int j = L.gi[q];
                    if (j != i) insert(dist2_f64(xi, L.gp[q]), j);
                }
            };
            auto cell_start = [&](int c) { return c == 0 ? 0 : L.gs[c - 1]; };
            auto row = [&](int y, int xa, int xb) {   // cells xa..xb of row y
                range(cell_start(y * gnx + xa), L.gs[y * gnx + xb]);
            };
            for (int R = 0;; ++R) {
                const int xa = max(cx - R, 0), xb = min(cx + R, gnx - 1);
                const int ya = max(cy - R, 0), yb = min(cy + R, gny - 1);
                if (R == 0) {
                    row(cy, cx, cx);
                } else {
                    if (cy - R >= 0) row(cy - R, xa, xb);
                    if (cy + R < gny) row(cy + R, xa, xb);
                    for (int y = max(cy - R + 1, 0); y <= min(cy + R - 1, gny - 1); ++y) {
                        if (cx - R >= 0) row(y, cx - R, cx - R);
                        if (cx + R < gnx) row(y, cx + R, cx + R);
                    }
                }
                if (xa == 0 && xb == gnx - 1 && ya == 0 && yb == gny - 1) break;   // all searched
                double bound = __builtin_huge_val();
                if (xa > 0) bound = fmin(bound, (double)xi.x - ((double)gx0 + (double)xa * gsx));
                if (xb < gnx - 1)
                    bound = fmin(bound, ((double)gx0 + (double)(xb + 1) * gsx) - (double)xi.x);
                if (ya > 0) bound = fmin(bound, (double)xi.y - ((double)gy0 + (double)ya * gsy));
                if (yb < gny - 1)
                    bound = fmin(bound, ((double)gy0 + (double)(yb + 1) * gsy) - (double)xi.y);
                bound -= margin;
                if (bound > 0.0) {
                    const double b2 = bound * bound;
                    int cnt = 0;
#pragma unroll
                    for (int k = 0; k < kKnn; ++k) cnt += bd[k] < b2 ? 1 : 0;
                    for (int off = 32; off >= 1; off >>= 1) cnt += __shfl_xor(cnt, off, kWave);
                    if (cnt >= kKnn) { thresh = b2; break; }
                }
            }
        }
        int my_nbr = -1;
        bool merged = false;
        if (grid) {
            // ---- rank merge: the entries below the threshold (at least 16
            // of them, or every candidate once the whole grid was searched)
            // are gathered in LDS when they fit one per lane; each takes its
            // rank by (distance, index) among them, and the 16 lowest ranks
            // are the neighbours in order
            int cl = 0;
#pragma unroll
            for (int k = 0; k < kKnn; ++k) cl += bd[k] < thresh ? 1 : 0;   // a prefix of the list
            int pre = cl;
            for (int off = 1; off < kWave; off <<= 1) {
                const int u = __shfl_up(pre, off, kWave);
                if (lane >= off) pre += u;
            }
            const int total = __shfl(pre, kWave - 1, kWave);
            if (total <= kWave) {
                const int base = pre - cl;
#pragma unroll
                for (int k = 0; k < kKnn; ++k)
                    if (k < cl) {
                        L.kd[wave][base + k] = bd[k];
                        L.kj[wave][base + k] = bj[k];
                    }
                wave_sync();
                int rank = kWave;
                int mj = -1;
                if (lane < total) {
                    const double md = L.kd[wave][lane];
                    mj = L.kj[wave][lane];
                    rank = 0;
                    for (int u = 0; u < total; ++u)
                        rank += key_less(L.kd[wave][u], L.kj[wave][u], md, mj) ? 1 : 0;
                }
                wave_sync();
                if (rank < kKnn) L.kj[wave][rank] = mj;   // ranks are distinct
                wave_sync();
                if (lane < min(total, kKnn)) my_nbr = L.kj[wave][lane];
                wave_sync();
                merged = true;
            }
        }
        // ---- otherwise: 16 rounds of a wavefront arg-min over the list heads
#pragma unroll 1
        for (int r = 0; r < (merged ? 0 : kKnn); ++r) {
            double md = bd[0];
            int mj = bj[0];
            for (int off = 32; off >= 1; off >>= 1) {
                const double od = __shfl_xor(md, off, kWave);
                const int oj = __shfl_xor(mj, off, kWave);
                if (key_less(od, oj, md, mj)) { md = od; mj = oj; }
            }
            if (lane == r && mj != 0x7fffffff) my_nbr = mj;
            if (bj[0] == mj && mj != 0x7fffffff) {   // the owner pops its head
#pragma unroll
                for (int k = 0; k < kKnn - 1; ++k) { bd[k] = bd[k + 1]; bj[k] = bj[k + 1]; }
                bd[kKnn - 1] = __builtin_huge_val();
                bj[kKnn - 1] = 0x7fffffff;
            }
        }
        // ---- features (lane k < 16: neighbour k)
        if (lane < kKnn) {
            float4 fv = make_float4(0.f, 0.f, 0.f, 0.f);
            if (my_nbr >= 0) {
                const float2 xj = src[my_nbr], yj = dst[my_nbr], yi = dst[i];
                float ex = ((yj.x - xj.x) - (yi.x - xi.x)) * 0.125f;
                float ey = ((yj.y - xj.y) - (yi.y - xi.y)) * 0.125f;
                fv = make_float4(g * (xj.x - xi.x), g * (xj.y - xi.y), ex / (1.f + fabsf(ex)),
                                 ey / (1.f + fabsf(ey)));
            }
            if (feat_out) {
                *(float4 *)&feat_out[(size_t)i * kNFeat + 4 * lane] = fv;
            } else {
                bhalf4 fb;
                fb[0] = (__bf16)fv.x;
                fb[1] = (__bf16)fv.y;
                fb[2] = (__bf16)fv.z;
                fb[3] = (__bf16)fv.w;
                *(bhalf4 *)&L.f[r][4 * lane] = fb;
            }
        }
    }
    if (feat_out) continue;
    __syncthreads();   // the block's features are complete
    start_mlp(L, wave, lane, b3, p_out, n, [&](int r) {
        return g0 + (r / kStartWaves) * stride + r % kStartWaves;
    });
    // the next group's features overwrite the block only after the barrier
    // at its end, so these reads of zpart are done before zpart is written
    // again
    }
}

__global__ __launch_bounds__(kStartThreads) void k_start(
    const float2 *__restrict__ src, const float2 *__restrict__ dst, int n, float g,
    const float *__restrict__ wts, float *__restrict__ p_out, int lanes) {
    start_body(src, dst, n, g, wts, p_out, nullptr, blockIdx.x, gridDim.x, lanes);
}

__global__ __launch_bounds__(kStartThreads) void k_start_features(
    const float2 *__restrict__ src, const float2 *__restrict__ dst, int n, float g,
    float *__restrict__ feat_out, int lanes) {
    start_body(src, dst, n, g, nullptr, nullptr, feat_out, blockIdx.x, gridDim.x, lanes);
}

// Matches per wavefront of the one-match-per-lane search (0: one match per
// wavefront) for `matches` matches spread over about `wgs` workgroups.
int start_lanes(long long matches, int wgs) {
    if (!EMDQ_START_LANE) return 0;
    const long long l = (matches + (long long)kStartWaves * wgs - 1) / ((long long)kStartWaves * wgs);
    return (int)std::min<long long>(std::max<long long>(l, 8), kWave);
}

struct StartJob {
    const float2 *src, *dst;
    float *p_out;
    int n;
    float g;
};

// One launch for many pairs: blockIdx.y = pair, the pair's matches strided
// over the gridDim.x workgroups.
__global__ __launch_bounds__(kStartThreads) void k_start_b(const StartJob *__restrict__ jobs,
                                                           const float *__restrict__ wts,
                                                           int lanes) {
    const StartJob &J = jobs[blockIdx.y];
    start_body(J.src, J.dst, J.n, J.g, wts, J.p_out, nullptr, blockIdx.x, gridDim.x, lanes);
}

// EM start from given posteriors: xy as k_load, p = init_p, mask = p > thresh
// (FP32); a non-finite start or coordinate sets ENONFINITE.
__device__ __forceinline__ void load_from_body(
    const float2 *__restrict__ src, const float2 *__restrict__ dst,
    const float *__restrict__ init_p, int n, float p_thresh, float4 *__restrict__ xy,
    float *__restrict__ p, uint8_t *__restrict__ mask, float4 *__restrict__ cent, DevState *st,
    int block) {
    const int i = block * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float2 a = src[i], b = dst[i];
    const float pi = init_p[i];
    xy[i] = make_float4(a.x, a.y, b.x, b.y);
    p[i] = pi;
    mask[i] = pi > p_thresh ? 1 : 0;
    cent[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    if (!finite2(a) || !finite2(b) || !__builtin_isfinite(pi)) {
        atomicMin(&st->status, (int)EMDQ_ENONFINITE);
        atomicExch(&st->done, 1);
        atomicExch(&st->stop_at, kOrdLoad);
    }
}

__global__ void k_load_from(const float2 *__restrict__ src, const float2 *__restrict__ dst,
                            const float *__restrict__ init_p, int n, float p_thresh,
                            float4 *__restrict__ xy, float *__restrict__ p,
                            uint8_t *__restrict__ mask, float4 *__restrict__ cent, DevState *st) {
    load_from_body(src, dst, init_p, n, p_thresh, xy, p, mask, cent, st, blockIdx.x);
}


// ------------------------------------------------- learned start: training ----
//
// One Adam step of the learned start's network on a minibatch (mean binary
// cross-entropy; label 1 = inlier).  k_start_grad: workgroup gi takes the
// samples idx[gi], idx[gi + G], ... in that order, one at a time, all 256
// threads on one sample: thread t = (o, h) = (t / 2, t % 2) owns row o of W1
// (columns [32 h, 32 h + 32), kept in registers) and of W2 (columns
// [64 h, 64 h + 64)) and accumulates their gradients in registers; W2 sits
// in LDS with padded rows so that both its rows (forward) and its columns
// (backward) read without bank conflicts.  Each workgroup writes its partial
// gradient (and loss) to its own slot of the workspace; k_start_adam adds
// the slots in workgroup order, so a step is deterministic.
constexpr int kTrainThreads = 256;
constexpr int kNW = kNHid * kNFeat + kNHid + kNHid * kNHid + kNHid + kNHid + 1;
constexpr int kOffB1 = kNHid * kNFeat, kOffW2 = kOffB1 + kNHid, kOffB2 = kOffW2 + kNHid * kNHid;
constexpr int kOffW3 = kOffB2 + kNHid, kOffB3 = kOffW3 + kNHid;
constexpr int kSlot = kNW + 1;   // a workgroup's partial gradient, then its loss

__device__ __forceinline__ float gelu_grad(float t) {
    return 0.5f * (1.f + erff(t * 0.70710678118654752f)) +
           t * 0.39894228040143268f * expf(-0.5f * t * t);
}

__global__ __launch_bounds__(kTrainThreads) void k_start_grad(
    const float *__restrict__ wts, const float *__restrict__ feat,
    const float *__restrict__ label, const int *__restrict__ idx, int batch, int m_samples,
    float *__restrict__ work) {
    __shared__ float w2[kNHid][kNHid + 1];
    __shared__ float fL[kNFeat], a1L[kNHid], h1L[kNHid], d2L[kNHid], red[kTrainThreads / kWave];
    const int t = threadIdx.x, o = t >> 1, h = t & 1, lane = t & (kWave - 1), wave = t >> 6;
    const int G = gridDim.x, gi = blockIdx.x;
    for (int e = t; e < kNHid * kNHid; e += kTrainThreads) w2[e / kNHid][e % kNHid] = wts[kOffW2 + e];
    float w1r[32], gw1[32], gw2[64];
#pragma unroll
    for (int k = 0; k < 32; ++k) {
        w1r[k] = wts[o * kNFeat + 32 * h + k];
        gw1[k] = 0.f;
    }
#pragma unroll
    for (int k = 0; k < 64; ++k) gw2[k] = 0.f;
    const float b1 = wts[kOffB1 + o], b2 = wts[kOffB2 + o], w3 = wts[kOffW3 + o];
    const float b3 = wts[kOffB3];
    float gb1 = 0.f, gb2 = 0.f, gw3 = 0.f, gb3 = 0.f, loss = 0.f;
    __syncthreads();
    for (int sidx = gi; sidx < batch; sidx += G) {
        const int sm = idx[sidx];
        if (sm < 0 || sm >= m_samples) continue;   // uniform: the whole workgroup skips it
        if (t < kNFeat) fL[t] = feat[(size_t)sm * kNFeat + t];
        const float y = label[sm];
        __syncthreads();
        // layer 1: a1[o] from the two halves of row o
        float p = 0.f;
#pragma unroll
        for (int k = 0; k < 32; ++k) p = fmaf(w1r[k], fL[32 * h + k], p);
        p += __shfl_xor(p, 1, kWave);
        const float a1 = p + b1;
        if (h == 0) {
            a1L[o] = a1;
            h1L[o] = gelu(a1);
        }
        __syncthreads();
        // layer 2
        float q = 0.f;
#pragma unroll 16
        for (int k = 0; k < 64; ++k) q = fmaf(w2[o][64 * h + k], h1L[64 * h + k], q);
        q += __shfl_xor(q, 1, kWave);
        const float a2 = q + b2, h2 = gelu(a2);
        float zc = h == 0 ? w3 * h2 : 0.f;
        zc = wave_sum(zc);
        if (lane == 0) red[wave] = zc;
        __syncthreads();
        const float z = ((red[0] + red[1]) + red[2]) + red[3] + b3;
        const float dz = 1.f / (1.f + expf(-z)) - y;
        if (t == 0) {
            loss += (z > 0.f ? z + log1pf(expf(-z)) : log1pf(expf(z))) - y * z;
            gb3 += dz;
        }
        const float d2 = dz * w3 * gelu_grad(a2);
        if (h == 0) {
            gw3 += dz * h2;
            gb2 += d2;
            d2L[o] = d2;
        }
#pragma unroll
        for (int k = 0; k < 64; ++k) gw2[k] = fmaf(d2, h1L[64 * h + k], gw2[k]);
        __syncthreads();
        // back through W2: column o, rows of this thread's half
        float s = 0.f;
#pragma unroll 16
        for (int r = 0; r < 64; ++r) s = fmaf(w2[64 * h + r][o], d2L[64 * h + r], s);
        s += __shfl_xor(s, 1, kWave);
        const float d1 = s * gelu_grad(a1L[o]);
        if (h == 0) gb1 += d1;
#pragma unroll
        for (int k = 0; k < 32; ++k) gw1[k] = fmaf(d1, fL[32 * h + k], gw1[k]);
        __syncthreads();   // the next sample overwrites the LDS rows
    }
    float *slot = work + (size_t)gi * kSlot;
#pragma unroll
    for (int k = 0; k < 32; ++k) slot[o * kNFeat + 32 * h + k] = gw1[k];
#pragma unroll
    for (int k = 0; k < 64; ++k) slot[kOffW2 + o * kNHid + 64 * h + k] = gw2[k];
    if (h == 0) {
        slot[kOffB1 + o] = gb1;
        slot[kOffB2 + o] = gb2;
        slot[kOffW3 + o] = gw3;
    }
    if (t == 0) {
        slot[kOffB3] = gb3;
        slot[kNW] = loss;
    }
}

// Sums the G slots in order (mean over the batch), stores the gradient and
// the mean loss after the last slot, and applies Adam (step t >= 1).
__global__ void k_start_adam(float *__restrict__ wts, float *__restrict__ m1,
                             float *__restrict__ m2, float *__restrict__ work, int G, int batch,
                             float lr, float beta1, float beta2, float eps, int step) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k > kNW) return;
    float sum = 0.f;
    for (int gi = 0; gi < G; ++gi) sum += work[(size_t)gi * kSlot + k];
    const float gk = sum / (float)batch;
    work[(size_t)G * kSlot + k] = gk;   // k == kNW: the mean loss
    if (k == kNW) return;
    const float a = beta1 * m1[k] + (1.f - beta1) * gk;
    const float b = beta2 * m2[k] + (1.f - beta2) * gk * gk;
    m1[k] = a;
    m2[k] = b;
    const float ah = a / (1.f - powf(beta1, (float)step));
    const float bh = b / (1.f - powf(beta2, (float)step));
    wts[k] -= lr * ah / (sqrtf(bh) + eps);
}

constexpr int kSplitK = EMDQ_SPLITK;
// FP32 field launches take two 32-row blocks per wavefront (2 wavefronts per
// SIMD, 512 workgroups at once) from this many 32 x 64 tiles on, 1.5 such
// rounds; smaller launches keep one row block (3 wavefronts per SIMD, 768
// workgroups at once), whose rounds quantise them better.
#ifndef EMDQ_RB2_MIN_TILES
#define EMDQ_RB2_MIN_TILES 768
#endif
constexpr long long kRb2MinTiles = EMDQ_RB2_MIN_TILES;
// FP32 blend: factor tables (per model, kF32TabCols floats per match) for
// regions whose padded width + height fit; larger regions compute the
// factors in the loop.
#ifndef EMDQ_F32_TABLES
#define EMDQ_F32_TABLES 1
#endif
constexpr long long kF32TabCols = 4096;

inline long long tiles64(int w, int h) {
    return (long long)((w + kTile - 1) / kTile) * ((h + 2 * kTile - 1) / (2 * kTile));
}
inline int field_row_blocks(long long n64) { return n64 >= kRb2MinTiles ? 2 : 1; }

// ---------------------------------------------------------------- batches ----
//
// Many independent pairs in one launch per phase.  Every pair keeps its own
// model (buffers and DevState); a job table in device memory holds each
// pair's pointers and sizes.  EM phases use a 2D grid (blockIdx.y = pair,
// blockIdx.x = the pair's own workgroup, surplus workgroups of smaller pairs
// return at once); the field launch is flat over the pairs' tiles, each
// workgroup finding its pair by a binary search of the tile offsets.
struct EmJob {
    const float2 *src, *dst;
    const float *init_p;   // null: the plain start p = 1
    float4 *xy;
    float *p;
    uint8_t *mask;
    float *e2;
    double2 *part;       // E-step sums per workgroup
    float4 *q;
    float *s;
    float4 *cent;        // M-step moment origins (relative to each match)
    float4 *packed;
    float *xs, *ys;
    DevState *st;
    int n, blocks;       // matches; EM workgroups of this pair
    float nal2;
    double alpha, u;
};

struct FieldJob {
    const float4 *packed;
    const float *xs, *ys;   // the inlier coordinates (factor tables)
    FieldTabs tabs;         // factor tables of this pair (none: in-loop factors)
    const DevState *st;
    float2 *out;
    const uint8_t *frame;
    float4 *canvas;
    float nal2;
    int zx0, zy0, w, h, tiles_x, n_tiles, block_base;
    int fw, fh, fpitch, cpitch, ox, oy;
};

__global__ void k_reset_b(const EmJob *__restrict__ jobs) {
    if (threadIdx.x == 0) reset_state(jobs[blockIdx.x].st);
}

__global__ void k_load_b(const EmJob *__restrict__ jobs, float p_thresh) {
    const EmJob &J = jobs[blockIdx.y];
    if ((int)blockIdx.x * (int)blockDim.x >= J.n) return;
    if (J.init_p)
        load_from_body(J.src, J.dst, J.init_p, J.n, p_thresh, J.xy, J.p, J.mask, J.cent,
                       J.st, blockIdx.x);
    else
        load_body(J.src, J.dst, J.n, J.xy, J.p, J.mask, J.cent, J.st, blockIdx.x);
}

// The per-iteration batch kernels take blockIdx.y (x for the posterior step)
// as an index into act, the pairs still running, or as the pair when act is
// null.
__global__ __launch_bounds__(kEmThreads)
#if EMDQ_MSTEP_B_WAVES
__attribute__((amdgpu_waves_per_eu(EMDQ_MSTEP_B_WAVES, EMDQ_MSTEP_B_WAVES)))
#endif
void k_mstep_b(const EmJob *__restrict__ jobs,
                                                        const int *__restrict__ act) {
    const EmJob &J = jobs[act ? act[blockIdx.y] : (int)blockIdx.y];
    if ((int)blockIdx.x >= J.blocks) return;
    mstep_body<kEmBatch, kMChunkB>(J.xy, J.p, J.n, J.nal2, J.alpha, J.q, J.s, J.cent, J.st, 1, EmFused{},
                         blockIdx.x);
}

__global__ __launch_bounds__(kEThreadsB) void k_estep_b(const EmJob *__restrict__ jobs,
                                                        const int *__restrict__ act) {
    const EmJob &J = jobs[act ? act[blockIdx.y] : (int)blockIdx.y];
    if ((int)blockIdx.x >= J.blocks) return;
    estep_body<kEmBatch, EMDQ_E_ROWS_BATCH, kEChunkB>(J.xy, J.p, J.q, J.s, J.n, J.nal2, J.e2, J.part, J.blocks, J.st,
                         EmStop{}, blockIdx.x);
}

__global__ __launch_bounds__(kPostThreads) void k_posterior_b(
    const EmJob *__restrict__ jobs, const int *__restrict__ act, double sigma2_min,
    double gamma_min, double gamma_max, float p_thresh, int max_iter) {
    const EmJob &J = jobs[act ? act[blockIdx.x] : (int)blockIdx.x];
    // a pair found stopped has had its final fit in this iteration's M-step
    if (J.st->status >= 0 && J.st->done) {
        if (threadIdx.x == 0) J.st->fitted = 1;
        return;
    }
    const PostParams pp{J.u, sigma2_min, gamma_min, gamma_max, p_thresh, max_iter};
    posterior_body(J.p, J.e2, J.mask, J.n, J.part, J.blocks, pp, J.st, nullptr, 0);
}

__global__ __launch_bounds__(kCompactThreads) void k_compact_b(const EmJob *__restrict__ jobs) {
    const EmJob &J = jobs[blockIdx.x];
    compact_body(J.xy, J.q, J.s, J.mask, J.n, J.packed, J.xs, J.ys, J.st, EmFinal{}, 0);
}

__global__ void k_gather_states(const EmJob *__restrict__ jobs, int n_pairs,
                                DevState *__restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_pairs) out[i] = *jobs[i].st;
}

template <int MODE, int SPLITK, int RB, bool TAB>
__global__ __launch_bounds__(kFieldThreads) __attribute__((amdgpu_waves_per_eu(field_waves(RB), field_waves(RB)))) void k_field_b(const FieldJob *__restrict__ jobs,
                                                           int n_jobs) {
    int lo = 0, hi = n_jobs - 1;   // last job whose first workgroup is <= blockIdx.x
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].block_base <= (int)blockIdx.x) lo = mid; else hi = mid - 1;
    }
    const FieldJob &J = jobs[lo];
    field_body<MODE, SPLITK, RB, TAB>(J.packed, J.st, J.nal2, J.zx0, J.zy0, J.w, J.h,
                                      J.tiles_x, J.n_tiles, J.out, J.frame, J.fw, J.fh,
                                      J.fpitch, J.canvas, J.cpitch, J.ox, J.oy,
                                      (int)blockIdx.x - J.block_base, J.tabs);
}

// Batched factor tables: workgroup (blockIdx.x, blockIdx.y) writes rows
// [kTabRowsPerThread blockIdx.x, +kTabRowsPerThread) of pair blockIdx.y's
// tables (FieldJob::tabs; none: nothing to do), its threads striding over the
// entry groups of those rows.
__global__ __launch_bounds__(kTabThreads) void k_field_tables_b(const FieldJob *__restrict__ jobs) {
    const FieldJob &J = jobs[blockIdx.y];
    if (!J.tabs.gx) return;
    const int n_in = J.st->status < 0 ? 0 : J.st->n_in;
    const int j0 = kTabRowsPerThread * (int)blockIdx.x;
    if (j0 >= n_in) return;
    const int sx = J.tabs.sx, sy = J.tabs.sy;
    float xr[kTabRowsPerThread], yr[kTabRowsPerThread];
#pragma unroll
    for (int r = 0; r < kTabRowsPerThread; ++r) {
        xr[r] = J.xs[min(j0 + r, n_in - 1)];
        yr[r] = J.ys[min(j0 + r, n_in - 1)];
    }
    for (int e = 4 * (int)threadIdx.x; e < sx + sy; e += 4 * kTabThreads) {
        if (e < sx)
            table_rows(xr, n_in - j0, J.nal2, (float)(J.zx0 + e),
                       (float *)J.tabs.gx + (size_t)j0 * sx + e, sx);
        else
            table_rows(yr, n_in - j0, J.nal2, (float)(J.zy0 + e - sx),
                       (float *)J.tabs.gy + (size_t)j0 * sy + (e - sx), sy);
    }
}

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
    double2 *part = nullptr;   // EM: E-step sums per workgroup
    int *chg = nullptr;        // EM: per M-step workgroup, a mask bit changed
    float4 *q = nullptr;
    float *s = nullptr;
    float4 *cent = nullptr;  // EM: each match's M-step moment origin (previous centroids)
    float4 *packed = nullptr;
    float *xs = nullptr;     // inlier coordinates, SoA, padded by one chunk
    float *ys = nullptr;
    int precision = EMDQ_PREC_F32;
    void *half_tab = nullptr;   // x and y factor tables of the half-precision blend
    float *f32_tab = nullptr;   // factor tables of the FP32 blend: n_max x kF32TabCols
    uint8_t *half_flags = nullptr;   // FP16 blend: tiles left to the FP32 blend (one slab)
    int tab_stride = 0;         // values per table row: n_max rounded up to 64
    DevState *st = nullptr;
    DevState *host_st = nullptr;   // pinned
    DevState *em_st = nullptr;     // pinned [2]: stop flags read while the EM runs on
    DevState *em_st_dev = nullptr; // the same two slots, as the device addresses them
    hipEvent_t em_ev[2] = {};
    int em_seq = 0;                // sequence number of the last chunk enqueued
    int em_stop_it = 0;            // the iteration whose kernels saw the last fit's stop (0: none)
    int em_slot_seq[2] = {};       // the number each slot will be published with
};

namespace {

#define EMDQ_HIP(call)                                   \
    do {                                                 \
        if ((call) != hipSuccess) return EMDQ_EHIP;      \
    } while (0)

emdq_status check_launch() {
    return hipGetLastError() == hipSuccess ? EMDQ_OK : EMDQ_EHIP;
}

// The argument rules of emdq_warp (frame, canvas, target rectangle).
bool warp_args_ok(const uint8_t *frame_rgb, int fw, int fh, int frame_pitch_bytes,
                  const float *canvas, int cw, int ch, int canvas_pitch_px, int ox, int oy,
                  int zx0, int zy0, int w, int h) {
    if (!frame_rgb || !canvas) return false;
    if (fw <= 0 || fh <= 0 || cw <= 0 || ch <= 0 || w < 0 || h < 0) return false;
    if ((long long)frame_pitch_bytes < 3LL * fw || canvas_pitch_px < cw) return false;
    if (((uintptr_t)canvas & 15u) != 0) return false;
    if (w == 0 || h == 0) return true;
    const long long cx0 = (long long)zx0 + ox, cy0 = (long long)zy0 + oy;
    return !(cx0 < 0 || cy0 < 0 || cx0 + w > cw || cy0 + h > ch);
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

// host_sync = false: the EM's whole budget of max_iter iterations is
// enqueued without reading a stop flag (the kernels after the stop return at
// entry, so the bits are those of the host-synchronised fit).
emdq_status fit_impl(emdq_model m, const float *src_xy, const float *dst_xy, int n,
                     int frame_w, int frame_h, const emdq_params *params, const float *init_p,
                     hipStream_t stream, bool host_sync = true);

emdq_status launch_field(emdq_model m, int mode, int zx0, int zy0, int w, int h, float2 *out,
                         const uint8_t *frame, int fw, int fh, int fpitch, float4 *canvas,
                         int cpitch, int ox, int oy, hipStream_t stream) {
    const int rb = field_row_blocks(tiles64(w, h));   // FP32 path only
    const int tiles_x = (w + kTile - 1) / kTile;
    const int tiles_y = (h + kTile * rb - 1) / (kTile * rb);
    const long long n_tiles = (long long)tiles_x * tiles_y;
    constexpr int tiles_per_wg = 4 / kSplitK;
    const long long blocks = (n_tiles + tiles_per_wg - 1) / tiles_per_wg;
    if (blocks > 0x7fffffffLL / kFieldThreads) return EMDQ_EINVAL;
    if (m->precision != EMDQ_PREC_F32) {
        // Slabs of at most kTabRows columns and rows, each with its factor
        // tables computed first (the tables hold one slab).
        const float ka = sqrtf(m->alpha * kLog2e);
        const bool f16 = m->precision == EMDQ_PREC_F16;
        void *gxt = m->half_tab;
        void *gyt = m->half_tab ? (char *)m->half_tab + (size_t)kTabRows * m->tab_stride * 2 : nullptr;
        for (int sy = 0; sy < h; sy += kTabRows)
            for (int sx = 0; sx < w; sx += kTabRows) {
                const int sw = min(kTabRows, w - sx), sh = min(kTabRows, h - sy);
                const int hx = (sw + kHTx - 1) / kHTx, hy = (sh + kHTy - 1) / kHTy;
                const int zx = zx0 + sx, zy = zy0 + sy;
                if (gxt) {
                    const dim3 tg((unsigned)((m->tab_stride / 8 + 255) / 256),
                                  (unsigned)((hx * kHTx + hy * kHTy) / kTabRowsPer));
                    if (f16)
                        hipLaunchKernelGGL(k_half_tables<kDtF16>, tg, dim3(256), 0, stream,
                                           m->xs, m->ys, m->st, ka, zx, zy, hx * kHTx,
                                           m->tab_stride, gxt, gyt);
                    else
                        hipLaunchKernelGGL(k_half_tables<kDtBF16>, tg, dim3(256), 0, stream,
                                           m->xs, m->ys, m->st, ka, zx, zy, hx * kHTx,
                                           m->tab_stride, gxt, gyt);
                }
                // the slab's outputs are addressed through its own origin
                const unsigned nb = (unsigned)(hx * hy);
                uint8_t *flags = f16 ? m->half_flags : nullptr;
                if (mode == kModeField) {
                    auto k = f16 ? k_field_half<kModeField, kDtF16>
                                 : k_field_half<kModeField, kDtBF16>;
                    hipLaunchKernelGGL(k, dim3(nb), dim3(kFieldThreads), 0, stream, m->packed,
                                       m->xs, m->ys, m->st, ka, zx, zy, sw, sh, hx,
                                       out + (size_t)sy * w + sx, nullptr, 0, 0, 0, nullptr, 0, 0,
                                       0, gxt, gyt, m->tab_stride, w, flags);
                } else {
                    auto k = f16 ? k_field_half<kModeWarp, kDtF16>
                                 : k_field_half<kModeWarp, kDtBF16>;
                    hipLaunchKernelGGL(k, dim3(nb), dim3(kFieldThreads), 0, stream, m->packed,
                                       m->xs, m->ys, m->st, ka, zx, zy, sw, sh, hx, nullptr,
                                       frame, fw, fh, fpitch, canvas, cpitch, ox, oy, gxt, gyt,
                                       m->tab_stride, w, flags);
                }
                if (flags) {
                    // the tiles the FP16 blend left, in FP32 (one workgroup per FP16 tile)
                    const FieldFilter filt{flags, hx, w};
                    const float nal2 = -m->alpha * kLog2e;
                    if (mode == kModeField)
                        hipLaunchKernelGGL(k_field_fallback<kModeField>, dim3(nb),
                                           dim3(kFieldThreads), 0, stream, m->packed, m->st, nal2,
                                           zx, zy, sw, sh, out + (size_t)sy * w + sx, nullptr, 0,
                                           0, 0, nullptr, 0, 0, 0, filt);
                    else
                        hipLaunchKernelGGL(k_field_fallback<kModeWarp>, dim3(nb),
                                           dim3(kFieldThreads), 0, stream, m->packed, m->st, nal2,
                                           zx, zy, sw, sh, nullptr, frame, fw, fh, fpitch, canvas,
                                           cpitch, ox, oy, filt);
                }
            }
        return check_launch();
    }
    const float nal2 = -m->alpha * kLog2e;
    // factor tables when the region's padded rows fit the model's table
    // (same bits either way)
    FieldTabs tabs{};
    const long long sxp = (long long)tiles_x * kTile, syp = (long long)tiles_y * kTile * rb;
    if (m->f32_tab && m->n > 0 && sxp + syp <= kF32TabCols) {
        tabs.gx = m->f32_tab;
        tabs.gy = m->f32_tab + (size_t)m->n_max * sxp;
        tabs.sx = (int)sxp;
        tabs.sy = (int)syp;
        const unsigned gxb = (unsigned)((sxp + syp + 4 * kTabThreads - 1) / (4 * kTabThreads));
        const unsigned gyb = (unsigned)((m->n + kTabRowsPerThread - 1) / kTabRowsPerThread);
        hipLaunchKernelGGL(k_field_tables, dim3(gxb, gyb), dim3(kTabThreads), 0,
                           stream, m->xs, m->ys, m->st, nal2, zx0, zy0, (float *)tabs.gx,
                           (float *)tabs.gy, tabs.sx, tabs.sy);
    }
#define EMDQ_F(M, R, T, O, F, C)                                                                \
    hipLaunchKernelGGL((k_field<M, kSplitK, R, T>), dim3((unsigned)blocks),                  \
                       dim3(kFieldThreads), 0, stream, m->packed, m->st, nal2, zx0, zy0, w, h, \
                       tiles_x, (int)n_tiles, O, F, fw, fh, fpitch, C, cpitch, ox, oy, tabs, \
                       FieldFilter{})
#define EMDQ_FT(M, R, O, F, C)                 \
    do {                                       \
        if (tabs.gx) EMDQ_F(M, R, true, O, F, C); \
        else EMDQ_F(M, R, false, O, F, C);        \
    } while (0)
    if (mode == kModeField) {
        if (rb == 2) EMDQ_FT(kModeField, 2, out, nullptr, nullptr);
        else EMDQ_FT(kModeField, 1, out, nullptr, nullptr);
    } else {
        if (rb == 2) EMDQ_FT(kModeWarp, 2, nullptr, frame, canvas);
        else EMDQ_FT(kModeWarp, 1, nullptr, frame, canvas);
    }
#undef EMDQ_FT
#undef EMDQ_F
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
    const size_t nb = (n + kRowsPerBlock - 1) / kRowsPerBlock;
    ok = ok && hipMalloc((void **)&m->part, nb * sizeof(double2)) == hipSuccess;
    ok = ok && hipMalloc((void **)&m->chg, nb * sizeof(int)) == hipSuccess;
    ok = ok && hipMalloc((void **)&m->q, n * sizeof(float4)) == hipSuccess;
    ok = ok && hipMalloc((void **)&m->s, n * sizeof(float)) == hipSuccess;
    ok = ok && hipMalloc((void **)&m->cent, n * sizeof(float4)) == hipSuccess;
    ok = ok && hipMalloc((void **)&m->packed, 2 * n * sizeof(float4)) == hipSuccess;
    ok = ok && hipMalloc((void **)&m->xs, (n + kHK) * sizeof(float)) == hipSuccess;
    ok = ok && hipMalloc((void **)&m->ys, (n + kHK) * sizeof(float)) == hipSuccess;
    ok = ok && hipMalloc((void **)&m->st, sizeof(DevState)) == hipSuccess;
    if (ok && EMDQ_F32_TABLES && n_max <= 65535)
        ok = hipMalloc((void **)&m->f32_tab, n * kF32TabCols * sizeof(float)) == hipSuccess;
    ok = ok && hipHostMalloc((void **)&m->host_st, sizeof(DevState), hipHostMallocDefault) ==
                   hipSuccess;
    // coherent: the EM's E-step or posterior kernel stores the stop flags
    // straight into them
    ok = ok && hipHostMalloc((void **)&m->em_st, 2 * sizeof(DevState), hipHostMallocCoherent) ==
                   hipSuccess;
    // the slots start at sequence number 0 (the allocator may hand out memory
    // a freed model used, holding that model's numbers); this model's numbers
    // start at 1 and only grow, so a slot matches only once its chunk wrote it
    if (ok) memset(m->em_st, 0, 2 * sizeof(DevState));
    ok = ok && hipHostGetDevicePointer((void **)&m->em_st_dev, m->em_st, 0) == hipSuccess;
    for (int k = 0; ok && k < 2; ++k)
        ok = hipEventCreateWithFlags(&m->em_ev[k], hipEventDisableTiming) == hipSuccess;
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
    // Work still queued on the model's buffers is waited for by device, not
    // by the caller's stream: that stream may already be destroyed when the
    // model is released (garbage collection, process teardown), so the
    // model keeps no stream handle at all.
    int prev = 0;
    if (hipGetDevice(&prev) == hipSuccess && hipSetDevice(m->device) == hipSuccess) {
        (void)hipDeviceSynchronize();
        (void)hipSetDevice(prev);
    }
    (void)hipFree(m->xy);
    (void)hipFree(m->p);
    (void)hipFree(m->mask);
    (void)hipFree(m->e2);
    (void)hipFree(m->part);
    (void)hipFree(m->chg);
    (void)hipFree(m->q);
    (void)hipFree(m->cent);
    (void)hipFree(m->s);
    (void)hipFree(m->packed);
    (void)hipFree(m->xs);
    (void)hipFree(m->ys);
    (void)hipFree(m->half_tab);
    (void)hipFree(m->f32_tab);
    (void)hipFree(m->half_flags);
    (void)hipFree(m->st);
    if (m->host_st) (void)hipHostFree(m->host_st);
    if (m->em_st) (void)hipHostFree(m->em_st);
    for (int k = 0; k < 2; ++k)
        if (m->em_ev[k]) (void)hipEventDestroy(m->em_ev[k]);
    delete m;
}

emdq_status emdq_fit(emdq_model m, const float *src_xy, const float *dst_xy, int n,
                     int frame_w, int frame_h, const emdq_params *params,
                     hipStream_t stream) {
    return fit_impl(m, src_xy, dst_xy, n, frame_w, frame_h, params, nullptr, stream);
}

}  // extern "C"

namespace {

// Waits until pinned slot `slot` holds the state published with sequence
// number `seq` (by the last E-step or posterior kernel of a chunk); the
// stream is queried now and then so that a failed launch is reported rather
// than waited for.
emdq_status wait_published(emdq_model m, int slot, int seq, hipStream_t stream) {
    for (unsigned spins = 1;; ++spins) {
        if (__atomic_load_n(&m->em_st[slot].seq, __ATOMIC_ACQUIRE) == seq) return EMDQ_OK;
        if ((spins & 1023u) == 0u) {
            const hipError_t e = hipStreamQuery(stream);
            if (e == hipSuccess)   // everything enqueued has completed
                return __atomic_load_n(&m->em_st[slot].seq, __ATOMIC_ACQUIRE) == seq
                           ? EMDQ_OK : EMDQ_EHIP;
            if (e != hipErrorNotReady) return EMDQ_EHIP;
        }
    }
}

emdq_status fit_impl(emdq_model m, const float *src_xy, const float *dst_xy, int n,
                     int frame_w, int frame_h, const emdq_params *params, const float *init_p,
                     hipStream_t stream, bool host_sync) {
    if (!m || !src_xy || !dst_xy) return EMDQ_EINVAL;
    emdq_params prm;
    if (params) prm = *params; else emdq_params_default(&prm);
    if (!params_ok(prm) || frame_w <= 0 || frame_h <= 0) return EMDQ_EINVAL;
    if (n < 2) return EMDQ_ETOOFEW;
    if (n > m->n_max) return EMDQ_EINVAL;
    m->n = n;
    const double alpha = alpha_d(prm, frame_w, frame_h);
    m->alpha = (float)alpha;
    const float nal2 = -(float)alpha * kLog2e;
    const double u = 1.0 / ((double)frame_w * (double)frame_h);
    const unsigned em_blocks = (unsigned)((n + kRowsPerBlock - 1) / kRowsPerBlock);

    hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, stream, m->st);
    if (init_p)
        hipLaunchKernelGGL(k_load_from, dim3((n + 255) / 256), dim3(256), 0, stream,
                           (const float2 *)src_xy, (const float2 *)dst_xy, init_p, n,
                           prm.p_thresh, m->xy, m->p, m->mask, m->cent, m->st);
    else
        hipLaunchKernelGGL(k_load, dim3((n + 255) / 256), dim3(256), 0, stream,
                           (const float2 *)src_xy, (const float2 *)dst_xy, n, m->xy, m->p,
                           m->mask, m->cent, m->st);
    if (check_launch() != EMDQ_OK) return EMDQ_EHIP;
    const PostParams pp{u, (double)prm.sigma2_min, (double)prm.gamma_min, (double)prm.gamma_max,
                        prm.p_thresh, prm.max_iter};
    // Up to kFusedMaxN matches the posterior step runs inside the M-step (two
    // launches per iteration; every M-step workgroup forms all n
    // posteriors); above it in its own one-workgroup kernel (three launches).
    const bool fused = n <= kFusedMaxN;
    // M-step of iteration it (from 1); fused: the posteriors of iteration
    // it - 1 first, when it >= 2
    // pub: pinned slot the M-step publishes the state it finds into (the
    // previous chunk's end), or null
    auto mstep = [&](int it, int final_pass, DevState *pub = nullptr, int seq = 0) {
        if (fused) {
            const EmFused F{m->e2, m->part, m->p,          m->mask, m->chg, pp,
                            (int)em_blocks, it, pub, seq};
            hipLaunchKernelGGL(k_mstep, dim3(em_blocks), dim3(kEmThreads), 0, stream, m->xy,
                               m->p, n, nal2, alpha, m->q, m->s, m->cent, m->st, F);
        } else {
            hipLaunchKernelGGL(k_mstep_s, dim3(em_blocks), dim3(kEmThreads), 0, stream, m->xy,
                               m->p, n, nal2, alpha, m->q, m->s, m->cent, m->st, final_pass,
                               pub, seq);
        }
    };
    // EM: iterations are enqueued in chunks; every kernel returns at once
    // once the EM has stopped, so a chunk may overshoot.  The stop flag after
    // chunk k is read while chunk k + 1 already runs, so the GPU does not
    // wait for the host between chunks.
    // Fused fits also enqueue a speculative compaction after every chunk
    // (k_compact_spec), so the inliers are packed as soon as the EM stops,
    // without waiting for the host to read the stop flag.
    const bool spec = EMDQ_SPEC_COMPACT && fused && host_sync;
    int enqueued = 0;
    bool stopped = false;   // the host has read a stop flag
    for (int k = 0;; ++k) {
        // the chunk's last E-step (fused) or posterior kernel also stores the
        // state into host slot k & 1 with the chunk's sequence number (a
        // chunk holds at least one iteration: the loop leaves once max_iter
        // iterations are enqueued)
        const int seq = ++m->em_seq;
        m->em_slot_seq[k & 1] = seq;
        // chunks end where the model's last fit stopped, and run one
        // iteration at a time after it: if this fit stops there too, one
        // iteration instead of a whole chunk is enqueued past the stop
        // (the results do not depend on the chunking)
        int clen = kEmChunk;
        if (EMDQ_EM_PREDICT && host_sync && m->em_stop_it > 0)
            clen = enqueued < m->em_stop_it ? std::min(kEmChunk, m->em_stop_it - enqueued) : 1;
        for (int c = 0; c < clen && enqueued < prm.max_iter; ++c, ++enqueued) {
            // EMDQ_PUBLISH_MSTEP: the state at the end of chunk k - 1 is
            // published by the first M-step of chunk k as it starts (its
            // write completes while that kernel runs); otherwise by the last
            // E-step / posterior kernel of chunk k as it ends
            const bool last = c + 1 == clen || enqueued + 1 == prm.max_iter;
            DevState *slot =
                last && host_sync && !EMDQ_PUBLISH_MSTEP ? &m->em_st_dev[k & 1] : nullptr;
            const int it = enqueued + 1;
            if (EMDQ_PUBLISH_MSTEP && host_sync && c == 0 && k > 0)
                mstep(it, 0, &m->em_st_dev[(k - 1) & 1], m->em_slot_seq[(k - 1) & 1]);
            else
                mstep(it, 0);
            if (fused) {
                const EmStop X{m->chg, slot, prm.max_iter, it, seq};
                hipLaunchKernelGGL(k_estep, dim3(em_blocks), dim3(kEThreads), 0, stream, m->xy,
                                   m->p, m->q, m->s, n, nal2, m->e2, m->part, m->st, X);
            } else {
                hipLaunchKernelGGL(k_estep_s, dim3(em_blocks), dim3(kEThreads), 0, stream,
                                   m->xy, m->p, m->q, m->s, n, nal2, m->e2, m->part, m->st);
                hipLaunchKernelGGL(k_posterior, dim3(1), dim3(kPostThreads), 0, stream, m->p,
                                   m->e2, m->mask, n, m->part, (int)em_blocks, pp, m->st, slot,
                                   seq);
            }
        }
        if (spec)
            hipLaunchKernelGGL(k_compact_spec, dim3(1), dim3(kCompactThreads), 0, stream, m->xy,
                               m->q, m->s, m->mask, n, m->packed, m->xs, m->ys, m->st);
        if (check_launch() != EMDQ_OK) return EMDQ_EHIP;
        if (!host_sync) {
            if (enqueued >= prm.max_iter) break;
            continue;
        }
        if (!EMDQ_EM_POLL) EMDQ_HIP(hipEventRecord(m->em_ev[k & 1], stream));
        if (k > 0) {
            const int ps = (k - 1) & 1;
            if (EMDQ_EM_POLL) {
                const emdq_status wr = wait_published(m, ps, m->em_slot_seq[ps], stream);
                if (wr != EMDQ_OK) return wr;
            } else {
                EMDQ_HIP(hipEventSynchronize(m->em_ev[ps]));
            }
            const DevState &prev = m->em_st[ps];
            if (prev.done || prev.status < 0) {
                stopped = true;
                // fused: the E-step after the last iteration applies the
                // stop rule; otherwise the last iteration's posterior kernel
                m->em_stop_it = prev.status < 0 ? 0 : (fused ? prev.iter + 1 : prev.iter);
                break;
            }
        }
        if (enqueued >= prm.max_iter) {
            m->em_stop_it = 0;
            break;
        }
    }
    // once a stop flag was read, a fused fit is complete: the M-step before
    // the stopping E-step fitted with the final posteriors, and the
    // speculative compaction after that chunk packed the inliers
    if (spec && stopped) return check_launch();
    // the fit with the final posteriors (fused: the posteriors of the last
    // enqueued iteration first; not needed once a stop flag was read, as the
    // M-step before the stopping E-step fitted already), then (fused) the
    // last stop decision and the inliers packed
    if (!(fused && stopped)) mstep(enqueued + 1, 1);
    const EmFinal fin{fused ? m->chg : nullptr, (int)em_blocks, enqueued, prm.max_iter};
    hipLaunchKernelGGL(k_compact, dim3(1), dim3(kCompactThreads), 0, stream, m->xy, m->q,
                       m->s, m->mask, n, m->packed, m->xs, m->ys, m->st, fin);
    return check_launch();
}

}  // namespace

extern "C" {

emdq_status emdq_model_set_nodes(emdq_model m, const float *x_xy, const float *scale,
                                 const float *q, const uint8_t *mask, int n, float alpha,
                                 hipStream_t stream) {
    if (!m || !x_xy || !scale || !q || n < 1 || n > m->n_max || !(alpha > 0.f))
        return EMDQ_EINVAL;
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
                           m->s, m->mask, n, m->packed, m->xs, m->ys, m->st, EmFinal{});
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
    return launch_field(m, kModeField, zx0, zy0, w, h, (float2 *)out_xy, nullptr, 0, 0, 0,
                        nullptr, 0, 0, 0, stream);
}

emdq_status emdq_warp(emdq_model m, const uint8_t *frame_rgb, int fw, int fh,
                      int frame_pitch_bytes, float *canvas, int cw, int ch,
                      int canvas_pitch_px, int ox, int oy, int zx0, int zy0, int w, int h,
                      hipStream_t stream) {
    if (!m) return EMDQ_EINVAL;
    if (!warp_args_ok(frame_rgb, fw, fh, frame_pitch_bytes, canvas, cw, ch, canvas_pitch_px, ox,
                      oy, zx0, zy0, w, h))
        return EMDQ_EINVAL;
    if (w == 0 || h == 0) return EMDQ_OK;
    return launch_field(m, kModeWarp, zx0, zy0, w, h, nullptr, frame_rgb, fw, fh,
                        frame_pitch_bytes, (float4 *)canvas, canvas_pitch_px, ox, oy, stream);
}

emdq_status emdq_track_nodes(emdq_model m, float beta, int n_nodes, float *pos_xy,
                             float *scale, float *q, float *sigma2, hipStream_t stream) {
    if (!m || n_nodes < 0 || !(beta > 0.f) || !__builtin_isfinite(beta)) return EMDQ_EINVAL;
    if (n_nodes == 0) return EMDQ_OK;
    if (!pos_xy || !scale || !q || !sigma2) return EMDQ_EINVAL;
    if ((((uintptr_t)pos_xy) & 7u) || (((uintptr_t)q) & 15u)) return EMDQ_EINVAL;
    const float nal2 = -m->alpha * kLog2e;
    const unsigned blocks = (unsigned)((n_nodes + kRowsPerBlock - 1) / kRowsPerBlock);
    hipLaunchKernelGGL(k_track, dim3(blocks), dim3(kEmThreads), 0, stream, m->packed, m->st,
                       nal2, beta, n_nodes, (float2 *)pos_xy, scale, (float4 *)q, sigma2);
    return check_launch();
}

emdq_status emdq_uncertainty(emdq_model m, float beta, int zx0, int zy0, int w, int h,
                             float *out, hipStream_t stream) {
    if (!m || !out || w < 0 || h < 0 || !(beta > 0.f) || !__builtin_isfinite(beta))
        return EMDQ_EINVAL;
    if (w == 0 || h == 0) return EMDQ_OK;
    const long long tx = (w + kUTile - 1) / kUTile, ty = (h + kUTile - 1) / kUTile;
    if (tx * ty > 0x7fffffffLL) return EMDQ_EINVAL;
    hipLaunchKernelGGL(k_uncertainty, dim3((unsigned)(tx * ty)), dim3(kUThreads), 0, stream,
                       m->packed, m->st, beta, zx0, zy0, w, h, (int)tx, out);
    return check_launch();
}

emdq_status emdq_learned_start(const float *src_xy, const float *dst_xy, int n, int frame_w,
                               int frame_h, const emdq_params *params, const float *weights,
                               float *p_out, hipStream_t stream) {
    if (!src_xy || !dst_xy || !weights || !p_out || frame_w <= 0 || frame_h <= 0)
        return EMDQ_EINVAL;
    if (n < 2) return EMDQ_ETOOFEW;
    emdq_params prm;
    if (params) prm = *params; else emdq_params_default(&prm);
    if (!params_ok(prm)) return EMDQ_EINVAL;
    const float g = (float)sqrt(alpha_d(prm, frame_w, frame_h));
    int blocks = (n + kStartWaves - 1) / kStartWaves;
    if (blocks > 1024) blocks = 1024;   // each workgroup stages the weights once
    hipLaunchKernelGGL(k_start, dim3((unsigned)blocks), dim3(kStartThreads), 0, stream,
                       (const float2 *)src_xy, (const float2 *)dst_xy, n, g, weights, p_out, 0);
    return check_launch();
}

emdq_status emdq_start_features(const float *src_xy, const float *dst_xy, int n, int frame_w,
                                int frame_h, const emdq_params *params, float *feat_out,
                                hipStream_t stream) {
    if (!src_xy || !dst_xy || !feat_out || frame_w <= 0 || frame_h <= 0) return EMDQ_EINVAL;
    if (n < 2) return EMDQ_ETOOFEW;
    emdq_params prm;
    if (params) prm = *params; else emdq_params_default(&prm);
    if (!params_ok(prm)) return EMDQ_EINVAL;
    const float g = (float)sqrt(alpha_d(prm, frame_w, frame_h));
    int blocks = (n + kStartWaves - 1) / kStartWaves;
    if (blocks > 4096) blocks = 4096;
    const int lanes = start_lanes(n, EMDQ_START_LANE_WGS1);
    if (lanes > 0) blocks = (n + kStartWaves * lanes - 1) / (kStartWaves * lanes);
    hipLaunchKernelGGL(k_start_features, dim3((unsigned)blocks), dim3(kStartThreads), 0, stream,
                       (const float2 *)src_xy, (const float2 *)dst_xy, n, g, feat_out, lanes);
    return check_launch();
}

size_t emdq_start_train_work_floats(int groups) {
    if (groups < 1) return 0;
    return (size_t)(groups + 1) * (size_t)kSlot;
}

emdq_status emdq_start_train_step(float *weights, float *adam_m, float *adam_v, int step,
                                  const float *feat, const float *label, int m_samples,
                                  const int *idx, int batch, float lr, int groups, float *work,
                                  hipStream_t stream) {
    if (!weights || !adam_m || !adam_v || !feat || !label || !idx || !work) return EMDQ_EINVAL;
    if (m_samples < 1 || batch < 1 || step < 1 || groups < 1 || groups > 4096 || !(lr > 0.f))
        return EMDQ_EINVAL;
    if (groups > batch) groups = batch;
    hipLaunchKernelGGL(k_start_grad, dim3((unsigned)groups), dim3(kTrainThreads), 0, stream,
                       weights, feat, label, idx, batch, m_samples, work);
    hipLaunchKernelGGL(k_start_adam, dim3((kNW + 1 + 255) / 256), dim3(256), 0, stream, weights,
                       adam_m, adam_v, work, groups, batch, lr, 0.9f, 0.999f, 1e-8f, step);
    return check_launch();
}

emdq_status emdq_fit_from(emdq_model m, const float *src_xy, const float *dst_xy, int n,
                          int frame_w, int frame_h, const emdq_params *params,
                          const float *init_p, hipStream_t stream) {
    if (!init_p) return EMDQ_EINVAL;
    return fit_impl(m, src_xy, dst_xy, n, frame_w, frame_h, params, init_p, stream);
}

emdq_status emdq_model_set_precision(emdq_model m, emdq_precision precision) {
    if (!m) return EMDQ_EINVAL;
    if (precision != EMDQ_PREC_F32 && precision != EMDQ_PREC_F16 &&
        precision != EMDQ_PREC_BF16)
        return EMDQ_EINVAL;
    if (precision == EMDQ_PREC_F16 && !m->half_flags) {
        int prev = 0;
        if (hipGetDevice(&prev) != hipSuccess || hipSetDevice(m->device) != hipSuccess)
            return EMDQ_EHIP;
        const hipError_t e = hipMalloc((void **)&m->half_flags, kHalfFlagBytes);
        (void)hipSetDevice(prev);
        if (e != hipSuccess) {
            m->half_flags = nullptr;
            return EMDQ_ENOMEM;
        }
    }
    if (EMDQ_HALF_TABLES && precision != EMDQ_PREC_F32 && !m->half_tab) {
        const int stride = (m->n_max + 63) / 64 * 64;
        const size_t bytes = (size_t)2 * kTabRows * (size_t)stride * 2;
        int prev = 0;
        if (hipGetDevice(&prev) != hipSuccess || hipSetDevice(m->device) != hipSuccess)
            return EMDQ_EHIP;
        const hipError_t e = hipMalloc(&m->half_tab, bytes);
        (void)hipSetDevice(prev);
        if (e != hipSuccess) {
            m->half_tab = nullptr;
            return EMDQ_ENOMEM;
        }
        m->tab_stride = stride;
    }
    m->precision = precision;
    return EMDQ_OK;
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

// ---------------------------------------------------------------- batches ----

struct emdq_batch_s {
    int max_pairs = 0;
    EmJob *em_jobs = nullptr;        // device
    FieldJob *field_jobs = nullptr;  // device
    StartJob *start_jobs = nullptr;  // device
    FieldJob *prepared = nullptr;    // device: the table of emdq_batch_prepare
    int variant = -1;                // field-kernel shape (autotuner); -1: by size
    int prep_mode = -1, prep_pairs = 0, prep_variant = 0, prep_tab_rows = 0;
    long long prep_blocks = 0;
    DevState *states = nullptr;      // device, gathered per chunk
    DevState *host_states = nullptr; // pinned, two sets (read while the EM runs on)
    int *act = nullptr;              // device: the pairs still running
    int *host_act = nullptr;         // pinned, two sets: their uploads
    hipEvent_t em_ev[2] = {};
    static constexpr int kSlots = 4; // pinned staging ring for the job tables
    void *stage[kSlots] = {};
    hipEvent_t stage_done[kSlots] = {};
    int next_slot = 0;
    // the prepared whole step (emdq_batch_prepare_step): device job tables
    // and the launch shapes
    EmJob *step_em = nullptr;
    StartJob *step_start = nullptr;
    FieldJob *step_field = nullptr;
    bool step_ready = false;
    int step_pairs = 0, step_start_wgs = 0, step_start_lanes = 0, step_variant = 0,
        step_tab_rows = 0;
    int step_shape_blocks = 1, step_shape_n = 2;
    long long step_blocks = 0;
    const float *step_weights = nullptr;
    emdq_params step_prm = {};
};

namespace {

size_t batch_stage_bytes(int max_pairs) {
    size_t a = sizeof(EmJob);
    if (sizeof(FieldJob) > a) a = sizeof(FieldJob);
    if (sizeof(StartJob) > a) a = sizeof(StartJob);
    return a * (size_t)max_pairs;
}

// A staging slot whose previous upload has completed.
void *batch_slot(emdq_batch b, int *slot) {
    const int k = b->next_slot;
    b->next_slot = (k + 1) % emdq_batch_s::kSlots;
    if (hipEventSynchronize(b->stage_done[k]) != hipSuccess) return nullptr;
    *slot = k;
    return b->stage[k];
}

bool distinct_models(int n, const emdq_model *models) {
    for (int i = 0; i < n; ++i) {
        if (!models[i]) return false;
        for (int j = 0; j < i; ++j)
            if (models[i] == models[j]) return false;
    }
    return true;
}

emdq_status batch_region_ok(const emdq_region &r, int mode) {
    if (r.w < 0 || r.h < 0) return EMDQ_EINVAL;
    if (mode == kModeField) return (r.w && r.h && !r.out_xy) ? EMDQ_EINVAL : EMDQ_OK;
    if (!r.frame_rgb || !r.canvas) return EMDQ_EINVAL;
    if (r.fw <= 0 || r.fh <= 0 || r.cw <= 0 || r.ch <= 0) return EMDQ_EINVAL;
    if ((long long)r.frame_pitch_bytes < 3LL * r.fw || r.canvas_pitch_px < r.cw)
        return EMDQ_EINVAL;
    if (((uintptr_t)r.canvas & 15u) != 0) return EMDQ_EINVAL;
    const long long cx0 = (long long)r.zx0 + r.ox, cy0 = (long long)r.zy0 + r.oy;
    if (r.w && r.h && (cx0 < 0 || cy0 < 0 || cx0 + r.w > r.cw || cy0 + r.h > r.ch))
        return EMDQ_EINVAL;
    return EMDQ_OK;
}

// Field-kernel shapes the batched launch can use (split-K 4: one 32 x 32 tile
// per workgroup of four wavefronts; 2: two tiles; 1: four tiles).
constexpr int kBatchVariants = 4;
constexpr int kVariantSplitK[kBatchVariants] = {4, 2, 1, 4};
constexpr int kVariantRows[kBatchVariants] = {1, 1, 1, 2};   // 32-row blocks per wavefront

// Job table of a batched field / warp launch, the pairs ordered by match
// count (largest first), so the most expensive tiles are dispatched first.
emdq_status fill_field_jobs(FieldJob *jobs, int n_pairs, const emdq_model *models,
                            const emdq_region *regions, int splitk, int rows,
                            long long *blocks_out, int *tab_rows_out) {
    int tab_rows = 0;
    int *order = (int *)malloc(sizeof(int) * (size_t)n_pairs);
    if (!order) return EMDQ_ENOMEM;
    for (int i = 0; i < n_pairs; ++i) order[i] = i;
    for (int i = 1; i < n_pairs; ++i) {   // stable insertion sort by n, descending
        const int v = order[i];
        int k = i;
        while (k > 0 && models[order[k - 1]]->n < models[v]->n) {
            order[k] = order[k - 1];
            --k;
        }
        order[k] = v;
    }
    const int tiles_per_wg = 4 / splitk;
    long long base = 0;
    for (int q = 0; q < n_pairs; ++q) {
        const int i = order[q];
        const emdq_region &r = regions[i];
        emdq_model m = models[i];
        FieldJob &J = jobs[q];
        const int tiles_x = (r.w + kTile - 1) / kTile;
        const int tiles_y = (r.h + kTile * rows - 1) / (kTile * rows);
        const long long n_tiles = (r.w && r.h) ? (long long)tiles_x * tiles_y : 0;
        J.packed = m->packed;
        J.xs = m->xs;
        J.ys = m->ys;
        J.tabs = FieldTabs{};
        const long long sxp = (long long)tiles_x * kTile, syp = (long long)tiles_y * kTile * rows;
        if (m->f32_tab && n_tiles > 0 && sxp + syp <= kF32TabCols) {
            J.tabs.gx = m->f32_tab;
            J.tabs.gy = m->f32_tab + (size_t)m->n_max * sxp;
            J.tabs.sx = (int)sxp;
            J.tabs.sy = (int)syp;
            if (tab_rows >= 0) tab_rows = max(tab_rows, m->n_max);
        } else if (n_tiles > 0) {
            tab_rows = -1;   // a pair without tables: the whole launch computes in the loop
        }
        J.st = m->st;
        J.nal2 = -m->alpha * kLog2e;
        J.zx0 = r.zx0;
        J.zy0 = r.zy0;
        J.w = r.w;
        J.h = r.h;
        J.tiles_x = tiles_x;
        J.n_tiles = (int)n_tiles;
        J.block_base = (int)base;
        J.out = (float2 *)r.out_xy;
        J.frame = r.frame_rgb;
        J.fw = r.fw;
        J.fh = r.fh;
        J.fpitch = r.frame_pitch_bytes;
        J.canvas = (float4 *)r.canvas;
        J.cpitch = r.canvas_pitch_px;
        J.ox = r.ox;
        J.oy = r.oy;
        base += (n_tiles + tiles_per_wg - 1) / tiles_per_wg;
        if (base > 0x7fffffffLL / kFieldThreads) {
            free(order);
            return EMDQ_EINVAL;
        }
    }
    free(order);
    if (tab_rows < 0) {
        tab_rows = 0;
        for (int q = 0; q < n_pairs; ++q) jobs[q].tabs = FieldTabs{};
    }
    *blocks_out = base;
    *tab_rows_out = tab_rows;   // 0: no factor tables in this launch
    return EMDQ_OK;
}

void launch_field_b(int mode, int variant, unsigned blocks, const FieldJob *jobs, int n_jobs,
                    int tab_rows, hipStream_t stream) {
    if (tab_rows > 0)
        hipLaunchKernelGGL(k_field_tables_b,
                           dim3((unsigned)((tab_rows + kTabRowsPerThread - 1) / kTabRowsPerThread),
                                (unsigned)n_jobs),
                           dim3(kTabThreads), 0, stream, jobs);
#define EMDQ_FB(M, K, R)                                                                         \
    do {                                                                                         \
        if (tab_rows > 0)                                                                        \
            hipLaunchKernelGGL((k_field_b<M, K, R, true>), dim3(blocks), dim3(kFieldThreads), 0, \
                               stream, jobs, n_jobs);                                            \
        else                                                                                     \
            hipLaunchKernelGGL((k_field_b<M, K, R, false>), dim3(blocks), dim3(kFieldThreads),   \
                               0, stream, jobs, n_jobs);                                         \
    } while (0)
    if (mode == kModeField) {
        if (variant == 1) EMDQ_FB(kModeField, 2, 1);
        else if (variant == 2) EMDQ_FB(kModeField, 1, 1);
        else if (variant == 3) EMDQ_FB(kModeField, 4, 2);
        else EMDQ_FB(kModeField, 4, 1);
    } else {
        if (variant == 1) EMDQ_FB(kModeWarp, 2, 1);
        else if (variant == 2) EMDQ_FB(kModeWarp, 1, 1);
        else if (variant == 3) EMDQ_FB(kModeWarp, 4, 2);
        else EMDQ_FB(kModeWarp, 4, 1);
    }
#undef EMDQ_FB
}

// The batch's field-kernel shape: the one set by the autotuner or
// emdq_batch_set_variant, else split-K 4 with the row blocks the single-pair
// rule gives for the batch's total tile count.
int batch_variant(emdq_batch b, int n_pairs, const emdq_region *regions) {
    if (b->variant >= 0) return b->variant;
    long long n64 = 0;
    for (int i = 0; i < n_pairs; ++i) n64 += tiles64(regions[i].w, regions[i].h);
    return field_row_blocks(n64) == 2 ? 3 : 0;
}

emdq_status batch_regions_ok(emdq_batch b, int n_pairs, const emdq_model *models,
                             const emdq_region *regions, int mode) {
    if (!b || !models || !regions || n_pairs < 1 || n_pairs > b->max_pairs) return EMDQ_EINVAL;
    for (int i = 0; i < n_pairs; ++i) {
        if (!models[i]) return EMDQ_EINVAL;
        const emdq_status rc = batch_region_ok(regions[i], mode);
        if (rc != EMDQ_OK) return rc;
    }
    return EMDQ_OK;
}

emdq_status batch_field_launch(emdq_batch b, int n_pairs, const emdq_model *models,
                               const emdq_region *regions, int mode, hipStream_t stream) {
    emdq_status rc = batch_regions_ok(b, n_pairs, models, regions, mode);
    if (rc != EMDQ_OK) return rc;
    int slot = 0;
    FieldJob *jobs = (FieldJob *)batch_slot(b, &slot);
    if (!jobs) return EMDQ_EHIP;
    long long blocks = 0;
    const int v = batch_variant(b, n_pairs, regions);
    int tab_rows = 0;
    rc = fill_field_jobs(jobs, n_pairs, models, regions, kVariantSplitK[v], kVariantRows[v],
                         &blocks, &tab_rows);
    if (rc != EMDQ_OK) return rc;
    if (blocks == 0) return EMDQ_OK;
    EMDQ_HIP(hipMemcpyAsync(b->field_jobs, jobs, sizeof(FieldJob) * n_pairs,
                            hipMemcpyHostToDevice, stream));
    EMDQ_HIP(hipEventRecord(b->stage_done[slot], stream));
    launch_field_b(mode, v, (unsigned)blocks, b->field_jobs, n_pairs, tab_rows, stream);
    return check_launch();
}

// Cache of autotuner choices: one "emdq-autotune <tiles bucket> <matches
// bucket> <variant>" line per entry, buckets being rounded log2 of the total
// tile count and of the mean match count of the batch.
int cache_lookup(const char *path, int tb, int nb) {
    FILE *f = fopen(path, "r");
    if (!f) return -1;
    char tag[32];
    int a, c, v, found = -1;
    while (fscanf(f, "%31s %d %d %d", tag, &a, &c, &v) == 4)
        if (strcmp(tag, "emdq-autotune") == 0 && a == tb && c == nb && v >= 0 &&
            v < kBatchVariants)
            found = v;
    fclose(f);
    return found;
}

}  // namespace

// Launch shape of a batched EM: the 2D grid covers the largest pair.
struct BatchEmShape {
    int max_blocks = 1, max_n = 2;
};

// Validates the pairs of a batched fit and fills their job table (host
// memory); the models record the fit's size and alpha.
emdq_status fill_em_jobs(emdq_batch b, EmJob *jobs, int n_pairs, const emdq_model *models,
                         const float *const *src_xy, const float *const *dst_xy, const int *n,
                         const int *frame_w, const int *frame_h, const float *const *init_p,
                         const emdq_params *params, BatchEmShape *shape) {
    if (!b || !models || !src_xy || !dst_xy || !n || !frame_w || !frame_h) return EMDQ_EINVAL;
    if (n_pairs < 1 || n_pairs > b->max_pairs) return EMDQ_EINVAL;
    if (!distinct_models(n_pairs, models)) return EMDQ_EINVAL;
    emdq_params prm;
    if (params) prm = *params; else emdq_params_default(&prm);
    if (!params_ok(prm)) return EMDQ_EINVAL;
    for (int i = 0; i < n_pairs; ++i) {
        if (!src_xy[i] || !dst_xy[i] || frame_w[i] <= 0 || frame_h[i] <= 0) return EMDQ_EINVAL;
        if (init_p && !init_p[i]) return EMDQ_EINVAL;
        if (n[i] < 2) return EMDQ_ETOOFEW;
        if (n[i] > models[i]->n_max) return EMDQ_EINVAL;
    }
    BatchEmShape sh;
    for (int i = 0; i < n_pairs; ++i) {
        emdq_model m = models[i];
        const double alpha = alpha_d(prm, frame_w[i], frame_h[i]);
        m->n = n[i];
        m->alpha = (float)alpha;
        EmJob &J = jobs[i];
        J.src = (const float2 *)src_xy[i];
        J.dst = (const float2 *)dst_xy[i];
        J.init_p = init_p ? init_p[i] : nullptr;
        J.xy = m->xy;
        J.p = m->p;
        J.mask = m->mask;
        J.e2 = m->e2;
        J.part = m->part;
        J.q = m->q;
        J.s = m->s;
        J.cent = m->cent;
        J.packed = m->packed;
        J.xs = m->xs;
        J.ys = m->ys;
        J.st = m->st;
        J.n = n[i];
        J.blocks = (n[i] + kRowsPerBlock - 1) / kRowsPerBlock;
        J.nal2 = -(float)alpha * kLog2e;
        J.alpha = alpha;
        J.u = 1.0 / ((double)frame_w[i] * (double)frame_h[i]);
        if (J.blocks > sh.max_blocks) sh.max_blocks = J.blocks;
        if (n[i] > sh.max_n) sh.max_n = n[i];
    }
    *shape = sh;
    return EMDQ_OK;
}

// Enqueues the batched EM of the job table `jobs` (device).  host_stop: the
// host reads all pairs' stop flags between chunks of iterations and stops
// enqueuing once every pair has stopped; from the same flags it launches the
// next chunk's kernels over the pairs they show neither fitted nor failed
// (the kernels of the others would return at entry).  Otherwise the whole budget
// of max_iter iterations is enqueued over all pairs with no copy and no host
// synchronisation (the kernels of a stopped pair return at entry, so the
// results are the same bits), which a hipGraph can capture.
emdq_status enqueue_batch_em(emdq_batch b, const EmJob *jobs, int n_pairs,
                             const BatchEmShape &shape, const emdq_params &prm,
                             hipStream_t stream, bool host_stop) {
    const unsigned P = (unsigned)n_pairs;
    hipLaunchKernelGGL(k_reset_b, dim3(P), dim3(64), 0, stream, jobs);
    hipLaunchKernelGGL(k_load_b, dim3((unsigned)((shape.max_n + 255) / 256), P), dim3(256), 0,
                       stream, jobs, prm.p_thresh);
    if (check_launch() != EMDQ_OK) return EMDQ_EHIP;
    const int *act = nullptr;   // null: every pair
    unsigned n_act = P;
    auto mstep_b = [&]() {
        hipLaunchKernelGGL(k_mstep_b, dim3((unsigned)shape.max_blocks, n_act), dim3(kEmThreads),
                           0, stream, jobs, act);
    };
    int enqueued = 0;
    for (int k = 0;; ++k) {
        for (int c = 0; (c < kEmChunk || !host_stop) && enqueued < prm.max_iter;
             ++c, ++enqueued) {
            mstep_b();
            hipLaunchKernelGGL(k_estep_b, dim3((unsigned)shape.max_blocks, n_act),
                               dim3(kEThreadsB), 0, stream, jobs, act);
            hipLaunchKernelGGL(k_posterior_b, dim3(n_act), dim3(kPostThreads), 0, stream, jobs,
                               act, (double)prm.sigma2_min, (double)prm.gamma_min,
                               (double)prm.gamma_max, prm.p_thresh, prm.max_iter);
        }
        if (check_launch() != EMDQ_OK) return EMDQ_EHIP;
        if (!host_stop) break;
        hipLaunchKernelGGL(k_gather_states, dim3((P + 63) / 64), dim3(64), 0, stream, jobs,
                           n_pairs, b->states + (size_t)(k & 1) * b->max_pairs);
        if (check_launch() != EMDQ_OK) return EMDQ_EHIP;
        EMDQ_HIP(hipMemcpyAsync(b->host_states + (size_t)(k & 1) * b->max_pairs,
                                b->states + (size_t)(k & 1) * b->max_pairs,
                                sizeof(DevState) * n_pairs, hipMemcpyDeviceToHost, stream));
        EMDQ_HIP(hipEventRecord(b->em_ev[k & 1], stream));
        if (k > 0) {
            EMDQ_HIP(hipEventSynchronize(b->em_ev[(k - 1) & 1]));
            const DevState *prev = b->host_states + (size_t)((k - 1) & 1) * b->max_pairs;
            bool all = true;
            for (int i = 0; i < n_pairs; ++i) all = all && (prev[i].done || prev[i].status < 0);
            if (all) break;
            // the pairs not yet fitted; the upload from this set of the
            // pinned list went out before chunk k - 1, which has completed
            int *list = b->host_act + (size_t)(k & 1) * b->max_pairs;
            unsigned m = 0;
            for (int i = 0; i < n_pairs; ++i)
                if (prev[i].status >= 0 && !prev[i].fitted) list[m++] = i;
            if (m > 0 && m < n_act) {
                EMDQ_HIP(hipMemcpyAsync(b->act, list, sizeof(int) * m, hipMemcpyHostToDevice,
                                        stream));
                act = b->act;
                n_act = m;
            }
        }
        if (enqueued >= prm.max_iter) break;
    }
    // the final fit of the pairs that have not had it
    mstep_b();
    hipLaunchKernelGGL(k_compact_b, dim3(P), dim3(kCompactThreads), 0, stream, jobs);
    return check_launch();
}

// Validates the pairs of a batched learned start and fills their job table
// (host memory); *per receives the workgroups per pair.
emdq_status fill_start_jobs(emdq_batch b, StartJob *jobs, int n_pairs,
                            const float *const *src_xy, const float *const *dst_xy, const int *n,
                            const int *frame_w, const int *frame_h, const emdq_params *params,
                            float *const *p_out, int *per, int *lanes) {
    if (!b || !src_xy || !dst_xy || !n || !frame_w || !frame_h || !p_out) return EMDQ_EINVAL;
    if (n_pairs < 1 || n_pairs > b->max_pairs) return EMDQ_EINVAL;
    emdq_params prm;
    if (params) prm = *params; else emdq_params_default(&prm);
    if (!params_ok(prm)) return EMDQ_EINVAL;
    int max_n = 2;
    for (int i = 0; i < n_pairs; ++i) {
        if (!src_xy[i] || !dst_xy[i] || !p_out[i] || frame_w[i] <= 0 || frame_h[i] <= 0)
            return EMDQ_EINVAL;
        if (n[i] < 2) return EMDQ_ETOOFEW;
        jobs[i].src = (const float2 *)src_xy[i];
        jobs[i].dst = (const float2 *)dst_xy[i];
        jobs[i].p_out = p_out[i];
        jobs[i].n = n[i];
        jobs[i].g = (float)sqrt(alpha_d(prm, frame_w[i], frame_h[i]));
        if (n[i] > max_n) max_n = n[i];
    }
    // enough workgroups per pair to cover the largest one; about
    // EMDQ_START_WGS in all (one match per wavefront), or about 512 with
    // one match per lane
    int wgs = (EMDQ_START_WGS + n_pairs - 1) / n_pairs;
    const int need = (max_n + kStartWaves - 1) / kStartWaves;
    if (wgs > need) wgs = need;
    const int l = start_lanes((long long)max_n * n_pairs, EMDQ_START_LANE_WGSB);
    if (l > 0) wgs = (max_n + kStartWaves * l - 1) / (kStartWaves * l);
    *per = wgs;
    *lanes = l;
    return EMDQ_OK;
}

extern "C" {

emdq_status emdq_batch_create(int max_pairs, emdq_batch *out) {
    if (!out || max_pairs < 1 || max_pairs > 65535) return EMDQ_EINVAL;
    *out = nullptr;
    emdq_batch b = new (std::nothrow) emdq_batch_s;
    if (!b) return EMDQ_ENOMEM;
    b->max_pairs = max_pairs;
    const size_t n = (size_t)max_pairs;
    bool ok = hipMalloc((void **)&b->em_jobs, n * sizeof(EmJob)) == hipSuccess;
    ok = ok && hipMalloc((void **)&b->field_jobs, n * sizeof(FieldJob)) == hipSuccess;
    ok = ok && hipMalloc((void **)&b->start_jobs, n * sizeof(StartJob)) == hipSuccess;
    ok = ok && hipMalloc((void **)&b->prepared, n * sizeof(FieldJob)) == hipSuccess;
    ok = ok && hipMalloc((void **)&b->step_em, n * sizeof(EmJob)) == hipSuccess;
    ok = ok && hipMalloc((void **)&b->step_start, n * sizeof(StartJob)) == hipSuccess;
    ok = ok && hipMalloc((void **)&b->step_field, n * sizeof(FieldJob)) == hipSuccess;
    ok = ok && hipMalloc((void **)&b->states, 2 * n * sizeof(DevState)) == hipSuccess;
    ok = ok && hipHostMalloc((void **)&b->host_states, 2 * n * sizeof(DevState),
                             hipHostMallocDefault) == hipSuccess;
    ok = ok && hipMalloc((void **)&b->act, n * sizeof(int)) == hipSuccess;
    ok = ok && hipHostMalloc((void **)&b->host_act, 2 * n * sizeof(int),
                             hipHostMallocDefault) == hipSuccess;
    for (int k = 0; ok && k < 2; ++k)
        ok = hipEventCreateWithFlags(&b->em_ev[k], hipEventDisableTiming) == hipSuccess;
    for (int k = 0; ok && k < emdq_batch_s::kSlots; ++k) {
        ok = hipHostMalloc(&b->stage[k], batch_stage_bytes(max_pairs), hipHostMallocDefault) ==
             hipSuccess;
        ok = ok && hipEventCreateWithFlags(&b->stage_done[k], hipEventDisableTiming) ==
                       hipSuccess;
    }
    if (!ok) {
        emdq_batch_free(b);
        return EMDQ_ENOMEM;
    }
    *out = b;
    return EMDQ_OK;
}

void emdq_batch_free(emdq_batch b) {
    if (!b) return;
    for (int k = 0; k < emdq_batch_s::kSlots; ++k) {
        if (b->stage_done[k]) {
            (void)hipEventSynchronize(b->stage_done[k]);
            (void)hipEventDestroy(b->stage_done[k]);
        }
        if (b->stage[k]) (void)hipHostFree(b->stage[k]);
    }
    (void)hipFree(b->em_jobs);
    (void)hipFree(b->field_jobs);
    (void)hipFree(b->start_jobs);
    (void)hipFree(b->prepared);
    (void)hipFree(b->step_em);
    (void)hipFree(b->step_start);
    (void)hipFree(b->step_field);
    (void)hipFree(b->states);
    if (b->host_states) (void)hipHostFree(b->host_states);
    (void)hipFree(b->act);
    if (b->host_act) (void)hipHostFree(b->host_act);
    for (int k = 0; k < 2; ++k)
        if (b->em_ev[k]) (void)hipEventDestroy(b->em_ev[k]);
    delete b;
}

emdq_status emdq_batch_fit(emdq_batch b, int n_pairs, const emdq_model *models,
                           const float *const *src_xy, const float *const *dst_xy,
                           const int *n, const int *frame_w, const int *frame_h,
                           const float *const *init_p, const emdq_params *params,
                           hipStream_t stream) {
    if (!b) return EMDQ_EINVAL;
    emdq_params prm;
    if (params) prm = *params; else emdq_params_default(&prm);
    int slot = 0;
    EmJob *jobs = (EmJob *)batch_slot(b, &slot);
    if (!jobs) return EMDQ_EHIP;
    BatchEmShape shape;
    const emdq_status rc = fill_em_jobs(b, jobs, n_pairs, models, src_xy, dst_xy, n, frame_w,
                                        frame_h, init_p, params, &shape);
    if (rc != EMDQ_OK) return rc;
    EMDQ_HIP(hipMemcpyAsync(b->em_jobs, jobs, sizeof(EmJob) * n_pairs, hipMemcpyHostToDevice,
                            stream));
    EMDQ_HIP(hipEventRecord(b->stage_done[slot], stream));
    return enqueue_batch_em(b, b->em_jobs, n_pairs, shape, prm, stream, true);
}

emdq_status emdq_batch_learned_start(emdq_batch b, int n_pairs, const float *const *src_xy,
                                     const float *const *dst_xy, const int *n,
                                     const int *frame_w, const int *frame_h,
                                     const emdq_params *params, const float *weights,
                                     float *const *p_out, hipStream_t stream) {
    if (!b || !weights) return EMDQ_EINVAL;
    int slot = 0;
    StartJob *jobs = (StartJob *)batch_slot(b, &slot);
    if (!jobs) return EMDQ_EHIP;
    int per = 0, lanes = 0;
    const emdq_status rc = fill_start_jobs(b, jobs, n_pairs, src_xy, dst_xy, n, frame_w,
                                           frame_h, params, p_out, &per, &lanes);
    if (rc != EMDQ_OK) return rc;
    EMDQ_HIP(hipMemcpyAsync(b->start_jobs, jobs, sizeof(StartJob) * n_pairs,
                            hipMemcpyHostToDevice, stream));
    EMDQ_HIP(hipEventRecord(b->stage_done[slot], stream));
    hipLaunchKernelGGL(k_start_b, dim3((unsigned)per, (unsigned)n_pairs), dim3(kStartThreads), 0,
                       stream, b->start_jobs, weights, lanes);
    return check_launch();
}

emdq_status emdq_batch_autotune(emdq_batch b, int n_pairs, const emdq_model *models,
                                const emdq_region *regions, const char *cache_path,
                                int *variant_out, hipStream_t stream) {
    emdq_status rc = batch_regions_ok(b, n_pairs, models, regions, kModeField);
    if (rc != EMDQ_OK) return rc;
    long long tiles = 0;
    double nsum = 0.0;
    for (int i = 0; i < n_pairs; ++i) {
        tiles += (long long)((regions[i].w + kTile - 1) / kTile) * ((regions[i].h + kTile - 1) / kTile);
        nsum += models[i]->n;
    }
    const int tb = tiles > 0 ? (int)lround(log2((double)tiles)) : 0;
    const int nb = nsum > 0.0 ? (int)lround(log2(nsum / n_pairs)) : 0;
    int best = cache_path ? cache_lookup(cache_path, tb, nb) : -1;
    if (best < 0) {
        hipEvent_t e0, e1;
        EMDQ_HIP(hipEventCreate(&e0));
        EMDQ_HIP(hipEventCreate(&e1));
        float best_ms = 0.f;
        for (int v = 0; v < kBatchVariants && rc == EMDQ_OK; ++v) {
            b->variant = v;
            for (int rep = 0; rep < 2 && rc == EMDQ_OK; ++rep) {   // warm-up, then timed
                if (hipEventRecord(e0, stream) != hipSuccess) rc = EMDQ_EHIP;
                if (rc == EMDQ_OK)
                    rc = batch_field_launch(b, n_pairs, models, regions, kModeField, stream);
                if (rc == EMDQ_OK && hipEventRecord(e1, stream) != hipSuccess) rc = EMDQ_EHIP;
            }
            float ms = 0.f;
            if (rc == EMDQ_OK && (hipEventSynchronize(e1) != hipSuccess ||
                                  hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                rc = EMDQ_EHIP;
            if (rc == EMDQ_OK && (best < 0 || ms < best_ms)) {
                best = v;
                best_ms = ms;
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (rc != EMDQ_OK) {
            b->variant = -1;
            return rc;
        }
        if (cache_path) {
            FILE *f = fopen(cache_path, "a");
            if (f) {
                fprintf(f, "emdq-autotune %d %d %d\n", tb, nb, best);
                fclose(f);
            }
        }
    }
    b->variant = best;
    if (variant_out) *variant_out = best;
    return EMDQ_OK;
}

emdq_status emdq_batch_set_variant(emdq_batch b, int variant) {
    if (!b || variant < 0 || variant >= kBatchVariants) return EMDQ_EINVAL;
    b->variant = variant;
    return EMDQ_OK;
}

emdq_status emdq_batch_prepare(emdq_batch b, int warp, int n_pairs, const emdq_model *models,
                               const emdq_region *regions) {
    const int mode = warp ? kModeWarp : kModeField;
    emdq_status rc = batch_regions_ok(b, n_pairs, models, regions, mode);
    if (rc != EMDQ_OK) return rc;
    FieldJob *jobs = (FieldJob *)malloc(sizeof(FieldJob) * (size_t)n_pairs);
    if (!jobs) return EMDQ_ENOMEM;
    long long blocks = 0;
    const int v = batch_variant(b, n_pairs, regions);
    int tab_rows = 0;
    rc = fill_field_jobs(jobs, n_pairs, models, regions, kVariantSplitK[v], kVariantRows[v],
                         &blocks, &tab_rows);
    if (rc == EMDQ_OK &&
        hipMemcpy(b->prepared, jobs, sizeof(FieldJob) * n_pairs, hipMemcpyHostToDevice) !=
            hipSuccess)
        rc = EMDQ_EHIP;
    free(jobs);
    if (rc != EMDQ_OK) {
        b->prep_mode = -1;
        return rc;
    }
    b->prep_mode = mode;
    b->prep_pairs = n_pairs;
    b->prep_variant = v;
    b->prep_blocks = blocks;
    b->prep_tab_rows = tab_rows;
    return EMDQ_OK;
}

emdq_status emdq_batch_launch(emdq_batch b, hipStream_t stream) {
    if (!b || b->prep_mode < 0) return EMDQ_EINVAL;
    if (b->prep_blocks == 0) return EMDQ_OK;
    launch_field_b(b->prep_mode, b->prep_variant, (unsigned)b->prep_blocks, b->prepared,
                   b->prep_pairs, b->prep_tab_rows, stream);
    return check_launch();
}

emdq_status emdq_batch_prepare_step(emdq_batch b, int n_pairs, const emdq_model *models,
                                    const float *const *src_xy, const float *const *dst_xy,
                                    const int *n, const int *frame_w, const int *frame_h,
                                    const emdq_params *params, const float *start_weights,
                                    float *const *start_p, const emdq_region *regions) {
    if (!b) return EMDQ_EINVAL;
    b->step_ready = false;
    if (start_weights && !start_p) return EMDQ_EINVAL;
    emdq_status rc = batch_regions_ok(b, n_pairs, models, regions, kModeWarp);
    if (rc != EMDQ_OK) return rc;
    const size_t bytes = sizeof(EmJob) + sizeof(StartJob) + sizeof(FieldJob);
    char *host = (char *)malloc(bytes * (size_t)n_pairs);
    if (!host) return EMDQ_ENOMEM;
    EmJob *em = (EmJob *)host;
    StartJob *st = (StartJob *)(host + sizeof(EmJob) * (size_t)n_pairs);
    FieldJob *fj = (FieldJob *)(host + (sizeof(EmJob) + sizeof(StartJob)) * (size_t)n_pairs);
    BatchEmShape shape;
    int wgs = 0, lanes = 0, v = 0, tab_rows = 0;
    long long blocks = 0;
    rc = fill_em_jobs(b, em, n_pairs, models, src_xy, dst_xy, n, frame_w, frame_h,
                      start_weights ? (const float *const *)start_p : nullptr, params, &shape);
    if (rc == EMDQ_OK && start_weights)
        rc = fill_start_jobs(b, st, n_pairs, src_xy, dst_xy, n, frame_w, frame_h, params,
                             start_p, &wgs, &lanes);
    if (rc == EMDQ_OK) {
        v = batch_variant(b, n_pairs, regions);
        rc = fill_field_jobs(fj, n_pairs, models, regions, kVariantSplitK[v], kVariantRows[v],
                             &blocks, &tab_rows);
    }
    if (rc == EMDQ_OK &&
        (hipMemcpy(b->step_em, em, sizeof(EmJob) * n_pairs, hipMemcpyHostToDevice) !=
             hipSuccess ||
         hipMemcpy(b->step_start, st, sizeof(StartJob) * n_pairs, hipMemcpyHostToDevice) !=
             hipSuccess ||
         hipMemcpy(b->step_field, fj, sizeof(FieldJob) * n_pairs, hipMemcpyHostToDevice) !=
             hipSuccess))
        rc = EMDQ_EHIP;
    free(host);
    if (rc != EMDQ_OK) return rc;
    if (params) b->step_prm = *params; else emdq_params_default(&b->step_prm);
    b->step_pairs = n_pairs;
    b->step_start_wgs = wgs;
    b->step_start_lanes = lanes;
    b->step_weights = start_weights;
    b->step_variant = v;
    b->step_blocks = blocks;
    b->step_tab_rows = tab_rows;
    b->step_shape_blocks = shape.max_blocks;
    b->step_shape_n = shape.max_n;
    b->step_ready = true;
    return EMDQ_OK;
}

emdq_status emdq_batch_launch_step(emdq_batch b, hipStream_t stream) {
    if (!b || !b->step_ready) return EMDQ_EINVAL;
    const unsigned P = (unsigned)b->step_pairs;
    if (b->step_weights)
        hipLaunchKernelGGL(k_start_b, dim3((unsigned)b->step_start_wgs, P), dim3(kStartThreads),
                           0, stream, b->step_start, b->step_weights, b->step_start_lanes);
    BatchEmShape shape;
    shape.max_blocks = b->step_shape_blocks;
    shape.max_n = b->step_shape_n;
    const emdq_status rc =
        enqueue_batch_em(b, b->step_em, b->step_pairs, shape, b->step_prm, stream, false);
    if (rc != EMDQ_OK) return rc;
    if (b->step_blocks > 0)
        launch_field_b(kModeWarp, b->step_variant, (unsigned)b->step_blocks, b->step_field,
                       b->step_pairs, b->step_tab_rows, stream);
    return check_launch();
}

emdq_status emdq_batch_field(emdq_batch b, int n_pairs, const emdq_model *models,
                             const emdq_region *regions, hipStream_t stream) {
    return batch_field_launch(b, n_pairs, models, regions, kModeField, stream);
}

emdq_status emdq_batch_warp(emdq_batch b, int n_pairs, const emdq_model *models,
                            const emdq_region *regions, hipStream_t stream) {
    return batch_field_launch(b, n_pairs, models, regions, kModeWarp, stream);
}

}  // extern "C"


// ---------------------------------------------------- allocation-free entry ----
//
// emdq_fit_warp_static: emdq_fit followed by emdq_warp, with every device
// buffer of the model carved from one file-scope device array, so that the
// call allocates nothing.  Each device the library runs on holds its own copy
// of the array; its address is taken with hipGetSymbolAddress once per device
// (the array's name in host code is only a stand-in) and handed to the
// kernels like any model buffer.

namespace {

constexpr size_t round256(size_t b) { return (b + 255) / 256 * 256; }
constexpr size_t kStN = EMDQ_STATIC_MAX_N;
constexpr size_t kStNb = (kStN + kRowsPerBlock - 1) / kRowsPerBlock;
// byte offsets of the model's buffers in the array
constexpr size_t kStXy = 0;
constexpr size_t kStP = kStXy + round256(kStN * sizeof(float4));
constexpr size_t kStMask = kStP + round256(kStN * sizeof(float));
constexpr size_t kStE2 = kStMask + round256(kStN);
constexpr size_t kStPart = kStE2 + round256(kStN * sizeof(float));
constexpr size_t kStChg = kStPart + round256(kStNb * sizeof(double2));
constexpr size_t kStQ = kStChg + round256(kStNb * sizeof(int));
constexpr size_t kStS = kStQ + round256(kStN * sizeof(float4));
constexpr size_t kStCent = kStS + round256(kStN * sizeof(float));
constexpr size_t kStPacked = kStCent + round256(kStN * sizeof(float4));
constexpr size_t kStXs = kStPacked + round256(2 * kStN * sizeof(float4));
constexpr size_t kStYs = kStXs + round256((kStN + kHK) * sizeof(float));
constexpr size_t kStSt = kStYs + round256((kStN + kHK) * sizeof(float));
constexpr size_t kStBytes = kStSt + round256(sizeof(DevState));
static_assert(kStBytes < (1u << 20), "the static scratch stays under 1 MiB");

}  // namespace

static __device__ __align__(256) unsigned char scratch[kStBytes];

namespace {

constexpr int kStMaxDevices = 64;
std::mutex g_st_mu;
bool g_st_ready[kStMaxDevices];
emdq_model_s g_st_model[kStMaxDevices];   // host records; their pointers address `scratch`

// The model of the current device whose buffers live in `scratch`, set up on
// the first call on that device.
emdq_status static_model(emdq_model *out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return EMDQ_EHIP;
    if (dev < 0 || dev >= kStMaxDevices) return EMDQ_EINVAL;
    std::lock_guard<std::mutex> lock(g_st_mu);
    if (!g_st_ready[dev]) {
        unsigned char *ptr = nullptr;
        if (hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr)
            return EMDQ_EHIP;
        emdq_model_s &m = g_st_model[dev];
        m.n_max = (int)kStN;
        m.device = dev;
        m.xy = (float4 *)(ptr + kStXy);
        m.p = (float *)(ptr + kStP);
        m.mask = ptr + kStMask;
        m.e2 = (float *)(ptr + kStE2);
        m.part = (double2 *)(ptr + kStPart);
        m.chg = (int *)(ptr + kStChg);
        m.q = (float4 *)(ptr + kStQ);
        m.s = (float *)(ptr + kStS);
        m.cent = (float4 *)(ptr + kStCent);
        m.packed = (float4 *)(ptr + kStPacked);
        m.xs = (float *)(ptr + kStXs);
        m.ys = (float *)(ptr + kStYs);
        m.st = (DevState *)(ptr + kStSt);
        g_st_ready[dev] = true;
    }
    *out = &g_st_model[dev];
    return EMDQ_OK;
}

__global__ void k_export_state(const DevState *__restrict__ st, int *__restrict__ info) {
    if (threadIdx.x == 0) {
        info[0] = st->status;
        info[1] = st->iter;
        info[2] = st->n_in;
    }
}

}  // namespace

extern "C" {

emdq_status emdq_fit_warp_static(const float *src_xy, const float *dst_xy, int n,
                                 const emdq_params *params, const uint8_t *frame_rgb, int fw,
                                 int fh, int frame_pitch_bytes, float *canvas, int cw, int ch,
                                 int canvas_pitch_px, int ox, int oy, int zx0, int zy0, int w,
                                 int h, int *info, hipStream_t stream) {
    if (!src_xy || !dst_xy || !info) return EMDQ_EINVAL;
    if (!warp_args_ok(frame_rgb, fw, fh, frame_pitch_bytes, canvas, cw, ch, canvas_pitch_px, ox,
                      oy, zx0, zy0, w, h))
        return EMDQ_EINVAL;
    if (n < 2) return EMDQ_ETOOFEW;
    if (n > EMDQ_STATIC_MAX_N) return EMDQ_EINVAL;
    emdq_model m = nullptr;
    const emdq_status rc = static_model(&m);
    if (rc != EMDQ_OK) return rc;
    const emdq_status fr = fit_impl(m, src_xy, dst_xy, n, fw, fh, params, nullptr, stream,
                                    /*host_sync=*/false);
    if (fr != EMDQ_OK) return fr;
    if (w > 0 && h > 0) {
        const emdq_status wr = launch_field(m, kModeWarp, zx0, zy0, w, h, nullptr, frame_rgb, fw,
                                            fh, frame_pitch_bytes, (float4 *)canvas,
                                            canvas_pitch_px, ox, oy, stream);
        if (wr != EMDQ_OK) return wr;
    }
    hipLaunchKernelGGL(k_export_state, dim3(1), dim3(64), 0, stream, m->st, info);
    return check_launch();
}

}  // extern "C"
