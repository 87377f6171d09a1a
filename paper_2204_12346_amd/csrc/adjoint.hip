// Gradient of the deceased-count cost with respect to theta by the discrete
// adjoint of the RK4 scheme (reverse mode through every stage of every step).
//
// One particle per lane, one tile (64 particles of one problem) per
// wavefront, one wavefront per block:
//   1. forward pass: the loss kernel's integration (state s = b S, I, D; S
//      formed where beta changes), the cost, Dhat of every day, the
//      susceptible at every segment start and the state (s, I, S) every
//      `s` steps (checkpoints) -> workspace;
//   2. reverse sweep over the checkpoint intervals, last to first: replay
//      the interval from its checkpoint with exactly the forward pass's
//      operations, writing the state (s, I) before every step to the
//      wavefront's LDS slice, then walk the steps backwards, recomputing each
//      step's stages from its LDS state.  An interval longer than the LDS
//      slice holds is split into sub-intervals whose start states a first
//      replay stores in the workspace.
// For step n with stages Y1 = y, Y2 = y + h/2 k1, Y3 = y + h/2 k2,
// Y4 = y + h k3 and adjoint abar of y_{n+1}:
//   kbar4 = h/6 abar,             Ybar4 = J(Y4)^T kbar4
//   kbar3 = h/3 abar + h Ybar4,   Ybar3 = J(Y3)^T kbar3
//   kbar2 = h/3 abar + h/2 Ybar3, Ybar2 = J(Y2)^T kbar2
//   kbar1 = h/6 abar + h/2 Ybar2, Ybar1 = J(y)^T kbar1
//   a_n = abar + Ybar1 + Ybar2 + Ybar3 + Ybar4
//   thetabar += sum_s (df/dtheta)(Y_s)^T kbar_s
// and the cost's dl/dDhat_i is added to a_D at n = i * spd.
// State (S, I, D) (R never feeds back and no cost reads it): with
// p = b S I, b = beta/N, f = (-p, p - lam I, mu I) and u = kI - kS,
//   J^T k = (b I u,  b S u - lam kI + mu kD,  0),
//   df/dbeta . k = (S I / N) u,  df/dgamma . k = -I kI,  df/dmu . k = I (kD - kI).
// The stages are recomputed in the forward's scaled form, s_s = b S_s, which
// is the b S of J^T k; the beta sum is carried as sum s_s I_s u and divided
// by b at the segment's end (with beta = 0, s = 0 and S stays at its value
// S_k at the segment's start: there the sum is S_k sum I_s u).
// D never feeds back, so its adjoint is piecewise constant between samples:
// kbar_s.D = w_s h a_D with the RK4 weights w = (1/6, 1/3, 1/3, 1/6), and
// the D part of the mu sum is h/6 a_D (I1 + 2 I2 + 2 I3 + I4) per step,
// added a day at a time from the day's sum of J = I1 + 2 I2 + 2 I3 + I4,
// which the forward pass saves.
// The initial state depends on I0 through S0 = N - I0 - R0 - D0 and I = I0.
//
// Every replay repeats the forward pass's operations from a stored state,
// so the gradient is bitwise independent of the checkpoint interval and of
// the sub-interval length.
//
// The kernel runs in one of three modes: both passes (sird_loss_backward on
// its own), the forward pass alone (sird_loss given a workspace: the loss,
// and everything the reverse sweep reads, saved in the workspace), or the
// reverse sweep alone from such a workspace (sird_loss_backward with
// from_forward).  The saved forward is the same code as the forward pass of
// the first mode, so the gradient is bitwise the same either way.
#include <hip/hip_runtime.h>

#include <atomic>
#include <climits>
#include <cmath>
#include <mutex>
#include <string>
#include <type_traits>

#include "device.h"
#include "internal.h"

namespace sird {

struct BwdArgs {
    const sird_problem *probs;
    const sird_tile *tiles;
    const double *theta;
    const double *obs;
    const double *grad_loss;
    double *grad;
    double *loss_out;
    double *ws;
    int64_t P;       // slot stride of the workspace (total particles)
    int n_tiles;
    int obs_series;  // 1 or 3; the deceased counts are the last series
    int s;           // checkpoint interval in steps; 0: per problem, the whole
                     // days that fit an LDS sub-interval (lc steps; lc when
                     // a day is longer)
    int lc;          // steps of one LDS sub-interval
    int n_ck_max;    // checkpoints per particle (3 slots each)
    int n_sub_max;   // stored sub-interval starts per particle (3 slots each)
    int max_days;    // max W over problems (Dhat slots per particle - 1)
    int max_seg;     // max K over problems (segment-start slots)
    int lds_wave;    // doubles of LDS per wavefront
    int seg;         // 1: the segment-parallel sweep (checkpoints at every
                     // day start, then k_seg_transfer and k_seg_combine)
    int seg_rows;    // steps a wavefront of k_seg_transfer holds in LDS
    int max_pieces;  // bound on the segment-parallel sweep's pieces per problem
};

// Modes of k_backward.
enum BwdMode { kBoth = 0, kFwdOnly = 1, kRevOnly = 2 };

// LDS a wavefront of k_backward may take so that four fit on a compute unit
// (one per SIMD: 160 KiB of LDS per CU on gfx950).
constexpr int kBwdLdsBudget = 40 * 1024;
// The 64-bit operand of the raw buffer load and store builtins.
typedef unsigned int U32x2 __attribute__((ext_vector_type(2)));
// Word 3 of a raw buffer resource on gfx9-family chips (gfx950 included):
// untyped 32-bit data, no swizzle; the workspace loads use it.
constexpr int kBufferWord3 = 0x00020000;
// Bounds of the steps per LDS sub-interval.
constexpr int kLcMin = 8;
constexpr int kLcMax = 64;

// dl/dDhat_i of the cost; imax is the day MXSE takes its maximum on.
__device__ __forceinline__ double cost_grad(int kind, int i, int W, double D, double y,
                                            double w, int imax)
{
    const double n = (double)(W + 1);
    const double e = y - D;
    const double sg = e > 0.0 ? 1.0 : (e < 0.0 ? -1.0 : 0.0);
    switch (kind) {
    case SIRD_LOSS_SSRE: return i > 0 ? 2.0 * ((D - y) * w) * w : 0.0;
    case SIRD_LOSS_MSE: return -2.0 * e / n;
    case SIRD_LOSS_MXSE: return i == imax ? -2.0 * e : 0.0;
    case SIRD_LOSS_MAE: return -sg / n;
    case SIRD_LOSS_MAPE: return -100.0 * sg * w / n;
    default: return 0.0;
    }
}

// Sums of the reverse sweep.  The sums over stages 2 and 3 are kept apart
// from those over stages 1 and 4: the reverse step carries half the stage
// adjoints of stages 2 and 3 (see rev_step), whose terms count twice.
struct RevSums {
    double G14;   // over the segment's stages 1 and 4: s_s I_s u
    double G23;   // over the segment's stages 2 and 3: s_s I_s u / 2
    double Gv;    // over the segment's stages: I_s u
    double T14;   // over all stages 1 and 4: I_s kbar_s.I
    double T23;   // over all stages 2 and 3: I_s kbar_s.I / 2
};

// One stage of the reverse step: Ybar = J(Y_s)^T kbar; Ybar.S = b v with
// v = I_s u is returned as v (the next stage's kbar.S and the final sum
// take b in their constants); mkD = mu kbar_s.D.  G and T are the stage's
// pair of sums.
__device__ __forceinline__ void stage_adjoint(double ss, double Is, double kS, double kI,
                                              double mkD, double lam, double &v, double &YI,
                                              double &G, double &T)
{
    const double u = kI - kS;
    v = Is * u;
    YI = fma(ss, u, fma(-lam, kI, mkD));
    G = fma(ss, v, G);
    T = fma(Is, kI, T);
}

// The stages of one step from its start state (s, I), formed as the forward
// step forms them.
struct Stages {
    double s, I, s2, I2, s3, I3, s4, I4;
};

__device__ __forceinline__ void stages(Stages &z, const StepConst<double> &k)
{
    const double p1 = z.s * z.I;
    const double c1 = fma(-k.h2lam, z.I, z.I);
    z.s2 = fma(-k.h2b, p1, z.s);
    z.I2 = fma(k.h2, p1, c1);
    const double p2 = z.s2 * z.I2;
    const double c2 = fma(-k.h2lam, z.I2, z.I);
    z.s3 = fma(-k.h2b, p2, z.s);
    z.I3 = fma(k.h2, p2, c2);
    const double p3 = z.s3 * z.I3;
    const double c3 = fma(-k.hlam, z.I3, z.I);
    z.s4 = fma(-k.hb, p3, z.s);
    z.I4 = fma(k.h, p3, c3);
}

// One reverse step on the scaled adjoint (hS, hI) = h/6 a of (S, I): from
// h/6 a_{n+1} to h/6 a_n through the step's stages; a_D is constant here
// (m6 = h/6 mu a_D).  With the scaled adjoint, kbar4 = (hS, hI) and
// kbar1 = (hS, hI) + h/2 Ybar2 take no multiply, and stages 3 and 2 run on
// half their adjoints, kbar3/2 = (hS, hI) + h/2 Ybar4 and
// kbar2/2 = (hS, hI) + h/2 (Ybar3/2) (h/3 = 2 h/6; the stage adjoint is
// linear in kbar, and mu kbar.D / 2 = m6 for both): four multiplies fewer
// than forming h/6 a and h/3 a.  Ybar2/2 and Ybar3/2 count twice in the sums.
__device__ __forceinline__ void rev_step(const Stages &z, double &hS, double &hI,
                                         const StepConst<double> &k, double m6, RevSums &g)
{
    double v4, v3, v2, v1, Y4, Y3, Y2, Y1;
    // stage 4: kbar4 = h/6 a
    stage_adjoint(z.s4, z.I4, hS, hI, m6, k.lam, v4, Y4, g.G14, g.T14);
    // stage 3: kbar3 / 2 = h/6 a + h/2 Ybar4
    stage_adjoint(z.s3, z.I3, fma(k.h2b, v4, hS), fma(k.h2, Y4, hI), m6, k.lam, v3, Y3, g.G23,
                  g.T23);
    // stage 2: kbar2 / 2 = h/6 a + h/2 (Ybar3 / 2)
    stage_adjoint(z.s2, z.I2, fma(k.h2b, v3, hS), fma(k.h2, Y3, hI), m6, k.lam, v2, Y2, g.G23,
                  g.T23);
    // stage 1: kbar1 = h/6 a + h (Ybar2 / 2)
    stage_adjoint(z.s, z.I, fma(k.hb, v2, hS), fma(k.h, Y2, hI), m6, k.lam, v1, Y1, g.G14,
                  g.T14);

    // a_n = a + the four Ybar: h/6 a_n = h/6 a + h/6 (Y1 + 2 (Y2 + Y3) + Y4)
    // with the halved Y2, Y3; the S part is b V
    const double V = fma(2.0, v2 + v3, v1 + v4);
    g.Gv += V;
    hS = fma(k.h6b, V, hS);
    hI = fma(k.h6, fma(2.0, Y2 + Y3, Y1 + Y4), hI);
}

// dL/dbeta_k (before the upstream factor) from the segment's sums.
__device__ __forceinline__ double beta_grad(const RevSums &g, double b, double Sk, double invN)
{
    return b != 0.0 ? (fma(2.0, g.G23, g.G14) / b) * invN : (Sk * g.Gv) * invN;
}

__device__ __forceinline__ int seg_of(int n, int SS, int K)
{
    const int k = n / SS;
    return k > K - 1 ? K - 1 : k;
}

// First step of the segment after k, or INT_MAX when there is none inside
// the window.
__device__ __forceinline__ int next_seg_start(int k, int SS, int K, int T)
{
    const long n = (long)(k + 1) * SS;
    return (k + 1 < K && n < T) ? (int)n : INT_MAX;
}

// A segment change before step st, as the loss kernel makes it: S = s/b
// with the old beta (kept when beta = 0), the new beta, s = b S.
__device__ __forceinline__ void change_segment(SirdState<double> &y, StepConst<double> &sf,
                                               int &kf, int &next, const double *lb, int lane,
                                               double invN, int SS, int K, int T)
{
    unscale(y, sf);
    ++kf;
    set_beta(sf, lb[kf * kWave + lane], invN);
    rescale(y, sf);
    next = next_seg_start(kf, SS, K, T);
}

// The forward pass's integration from step st to step end (segment changes
// included), calling at() before the steps mark, mark + period, ... (it may
// store the state); the steps between calls run with no per-step test.
// jsum accumulates the steps' J.
template <typename At>
__device__ __forceinline__ void advance_marked(SirdState<double> &y, StepConst<double> &sf,
                                               int &kf, int &next, int &st, int end, int &mark,
                                               int period, const double *lb, int lane,
                                               double invN, int SS, int K, int T, double &jsum,
                                               At at)
{
    while (st < end) {
        if (st == next) change_segment(y, sf, kf, next, lb, lane, invN, SS, K, T);
        if (st == mark) {
            at();
            mark += period;
        }
        const int stop = min(min(end, next), mark);
#pragma unroll 2
        for (; st < stop; ++st) jsum += rk4_step<double, false, false>(y, sf);
    }
}

template <int KIND, int MODE>
__global__ void __launch_bounds__(4 * kWave) k_backward(BwdArgs a)
{
    extern __shared__ double lds[];
    const int lane = threadIdx.x & (kWave - 1);
    const int t = wave_tile_index();
    if (t >= a.n_tiles) return;
    // LDS of the wavefront: the observations and weights, the lane's betas,
    // and the states before the steps of one sub-interval
    double *const ly = lds + (size_t)(threadIdx.x / kWave) * a.lds_wave;
    double *const lw = ly + (a.max_days + 1);
    double *const lb = lw + (a.max_days + 1);              // [max_seg][64]
    // [3][64]: a prefetched checkpoint (s, I, S), parked until its replay
    double *const lck = lb + (size_t)a.max_seg * kWave + lane;
    // [2 + lc + 2][2][64]: (s, I) of the lane before each step of a
    // sub-interval, from row 2 on (two rows of slack at either end, which
    // the walk's read-ahead may touch and never uses)
    double *const lst = lb + (size_t)a.max_seg * kWave + 3 * kWave + 4 * kWave + lane;

    const sird_tile tl = a.tiles[t];
    const sird_problem P = a.probs[tl.prob];
    const int W = P.n_days, spd = P.steps_per_day, K = P.n_seg, n = P.n_part;
    const int T = W * spd;  // at most 2^30 (checked on the host)
    // steps per segment (a segment longer than the window is the window);
    // segments start at day starts
    const int SS = (int)min((long)P.seg_days * spd, (long)T + 1);
    const int pl = tl.p0 + lane;
    const bool active = pl < n;
    const int pc = active ? pl : n - 1;
    const size_t ld = (size_t)n;
    const double *th = a.theta + P.theta_off + pc;
    const size_t PS = (size_t)a.P;
    // Workspace: slot q of this lane's particle at wsb[q * PS] plus the
    // lane's byte offset (a uniform base and an offset register that never
    // changes, so a load in flight never holds an address register the
    // next instructions want); idle lanes address their stand-in column.
    //   checkpoint m: slots 3m..3m+2 (s, I, S); stored sub-interval start j:
    //   q_sub + 3j..; Dhat_i: q_day + i; S at segment k's start: q_seg + k;
    //   the sum of J over day i's steps: q_jd + i; MXSE's day and the loss:
    //   q_tail, q_tail + 1
    double *const wsb = a.ws + (size_t)(P.p_off + tl.p0);
    const uint32_t loff = (uint32_t)(pc - tl.p0) * (uint32_t)sizeof(double);
    auto slot = [&](size_t q) -> double & {
        return *(double *)((char *)(wsb + q * PS) + loff);
    };
    // loads through a buffer resource on the slot's (uniform) base: the
    // load's only address register is the lane offset
    auto load_at = [&](const double *base) -> double {
        const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
            (void *)base, (short)0, kWave * (int)sizeof(double), kBufferWord3);
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, loff, 0, 0));
    };
    auto load = [&](size_t q) -> double { return load_at(wsb + q * PS); };
    // a store through a buffer resource on a uniform slot address
    auto store_at = [&](double *base, double v) {
        const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
            (void *)base, (short)0, kWave * (int)sizeof(double), kBufferWord3);
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U32x2, v), r, loff, 0, 0);
    };
    const size_t q_sub = 3 * (size_t)a.n_ck_max;
    const size_t q_day = q_sub + 3 * (size_t)a.n_sub_max;
    const size_t q_seg = q_day + (size_t)(a.max_days + 1);
    const size_t q_jd = q_seg + (size_t)a.max_seg;
    const size_t q_tail = q_jd + (size_t)a.max_days;

    {
        // deceased counts: the last of the obs_series blocks of W+1 values
        const double *y = a.obs + P.obs_off + (size_t)(a.obs_series - 1) * (W + 1);
        for (int i = lane; i <= W; i += kWave) {
            const double yi = y[i];
            ly[i] = yi;
            lw[i] = 1.0 / fmax(yi, 1.0);
        }
#pragma unroll 4
        for (int k = 0; k < K; ++k) lb[k * kWave + lane] = th[(size_t)k * ld];
        wave_sync();
    }

    // this problem's checkpoint interval; a whole number of days when days
    // are the unit (the default, with a day no longer than lc steps, and the
    // segment-parallel sweep's forward pass, one day per interval); dpc: the
    // days per interval, 0 when steps are the unit
    const int dpc = a.seg ? 1 : ((a.s == 0 && spd <= a.lc) ? a.lc / spd : 0);
    const int sp = a.seg ? spd : (a.s > 0 ? a.s : (dpc > 0 ? dpc * spd : a.lc));

    const double gamma = th[(size_t)K * ld];
    const double mu = th[(size_t)(K + 1) * ld];
    const double I0 = th[(size_t)(K + 2) * ld];
    const double N = P.N;
    const double invN = 1.0 / N;
    StepConst<double> sc = step_const<double>(gamma, mu, spd);

    // ---------------------------------------------------- forward pass
    int imax = 0;
    if constexpr (MODE == kRevOnly) {
        imax = (int)load(q_tail);
        if (active && a.loss_out) a.loss_out[P.p_off + pl] = load(q_tail + 1);
    } else {
        SirdState<double> y;
        y.S = N - I0 - P.R0 - P.D0;
        y.I = I0;
        y.Rr = P.R0;
        y.D = P.D0;
        y.s = 0.0;
        y.eS = y.eI = y.eR = y.eD = 0.0;
        double acc = 0.0;
        cost_accum(KIND, acc, y.D, ly[0], lw[0], 0);
        if (active) slot(q_day) = y.D;
        int kf = 0;
        set_beta(sc, lb[lane], invN);
        rescale(y, sc);
        if (active) slot(q_seg) = y.S;
        int next = next_seg_start(0, SS, K, T);
        int st = 0, next_ck = 0;
        int kseen = 0;
        // the end of day `day` (the state after its steps, jd the sum of its
        // steps' J): S if a segment began with the day (it stays as the
        // segment change formed it: the integration carries s alone), the
        // cost, Dhat and the sum of J; the day slots are stepped a day at a
        // time, so their stores take no address arithmetic
        double *wday = wsb + (q_day + 1) * PS;
        double *wjd = wsb + q_jd * PS;
        auto end_of_day = [&](int day, double yo, double wo, double jd)
                              __attribute__((always_inline)) {
            if (kf != kseen) {
                if (active) slot(q_seg + kf) = y.S;
                kseen = kf;
            }
            const double prev = acc;
            cost_accum(KIND, acc, y.D, yo, wo, day + 1);
            if (KIND == SIRD_LOSS_MXSE && !(acc == prev)) imax = day + 1;
            if (active) {
                store_at(wday, y.D);
                store_at(wjd, jd);
            }
            wday += PS;
            wjd += PS;
        };
        if (dpc > 0) {
            // checkpoints at day starts: the loss kernel's day loop,
            // instantiated for days of a multiple of ten steps (blocks of ten
            // unrolled steps) and for others (unrolled by four), chosen
            // outside the loop so the state stays in its registers
            auto days = [&](auto tens) __attribute__((always_inline)) {
                constexpr bool TENS = decltype(tens)::value;
                double *wck = wsb;
                for (int day = 0; day < W; ++day) {
                    // the day's observation, read before its steps
                    const double yo = ly[day + 1], wo = lw[day + 1];
                    if (st == next) change_segment(y, sc, kf, next, lb, lane, invN, SS, K, T);
                    if (st == next_ck) {
                        if (active) {
                            store_at(wck, y.s);
                            store_at(wck + PS, y.I);
                            store_at(wck + 2 * PS, y.S);
                        }
                        wck += 3 * PS;
                        next_ck += sp;
                    }
                    double jd = 0.0;
                    if constexpr (TENS) {
                        for (int i = 0; i < spd; i += 10) {
#pragma unroll
                            for (int u = 0; u < 10; ++u) jd += rk4_step<double, false, false>(y, sc);
                        }
                    } else {
#pragma unroll 4
                        for (int i = 0; i < spd; ++i) jd += rk4_step<double, false, false>(y, sc);
                    }
                    st += spd;
                    end_of_day(day, yo, wo, jd);
                }
            };
            if (spd % 10 == 0)
                days(std::true_type{});
            else
                days(std::false_type{});
        } else {
            size_t cq = 0;
            for (int day = 0; day < W; ++day) {
                const double yo = ly[day + 1], wo = lw[day + 1];
                double jd = 0.0;
                advance_marked(y, sc, kf, next, st, st + spd, next_ck, sp, lb, lane, invN, SS,
                               K, T, jd, [&]() {
                                   if (active) {
                                       slot(cq) = y.s;
                                       slot(cq + 1) = y.I;
                                       slot(cq + 2) = y.S;
                                   }
                                   cq += 3;
                               });
                end_of_day(day, yo, wo, jd);
            }
        }
        const double L = cost_finish(KIND, acc, W);
        if (active && a.loss_out) a.loss_out[P.p_off + pl] = L;
        if constexpr (MODE == kFwdOnly) {
            if (active) {
                slot(q_tail) = (double)imax;
                slot(q_tail + 1) = L;
            }
            return;
        }
    }

    // ---------------------------------------------------- reverse sweep
    const double gl = a.grad_loss ? a.grad_loss[P.p_off + pc] : 1.0;
    double *gout = a.grad + P.theta_off + pc;
    const int k_last = seg_of(T - 1, SS, K);
    for (int k = k_last + 1; k < K; ++k)
        if (active) gout[(size_t)k * ld] = 0.0;  // segments past the window end

    double hS = 0.0, hI = 0.0;  // h/6 times the adjoint of (S, I)
    double aD = cost_grad(KIND, W, W, load(q_day + W), ly[W], lw[W], imax);
    double m6 = sc.h6 * (mu * aD);
    double muD = 0.0;  // sum over steps of h/6 a_D (I1 + 2 I2 + 2 I3 + I4)
    RevSums g{0.0, 0.0, 0.0, 0.0, 0.0};
    int kr = k_last;  // segment of the reverse position
    set_beta(sc, lb[kr * kWave + lane], invN);
    int seg_lo = kr * SS;  // first step of segment kr
    double Sk = load(q_seg + kr);
    // the next day start at or below the reverse position, and the slots of
    // its Dhat and sum of J (uniform addresses stepped down a day at a time,
    // so a day's loads take no address arithmetic)
    int dnext = (T - 1) / spd;
    const double *pday = wsb + (q_day + (size_t)dnext) * PS;
    const double *pjd = wsb + (q_jd + (size_t)dnext) * PS;

    // The step just reversed began day dnext (its Dhat is Dd, the day's sum
    // of J is Jd, its observation and weight yd, wd, all read before the
    // day's steps): add the mu sum's D part of the day with the day's a_D,
    // add the cost's gradient, and close segment kr if the step opened it.
    auto day_start = [&](int dstart, double Dd, double Jd, double yd, double wd)
                         __attribute__((always_inline)) {
        muD = fma(sc.h6 * aD, Jd, muD);
        aD += cost_grad(KIND, dnext, W, Dd, yd, wd, imax);
        m6 = sc.h6 * (mu * aD);
        if (dstart == seg_lo && kr > 0) {
            if (active) gout[(size_t)kr * ld] = beta_grad(g, sc.b, Sk, invN) * gl;
            g.G14 = 0.0;
            g.G23 = 0.0;
            g.Gv = 0.0;
            --kr;
            seg_lo -= SS;
            set_beta(sc, lb[kr * kWave + lane], invN);
            Sk = load(q_seg + kr);
        }
        --dnext;
        pday -= PS;
        pjd -= PS;
    };

    const int n_ck = (T + sp - 1) / sp;
    if (dpc > 0) {
        // Day-aligned intervals of L = sp steps (the last one may be shorter,
        // a whole number of days too): interval m is walked backwards while
        // interval m - 1 is replayed forwards, step for step, so the walk's
        // dependent chains and the replay's overlap.  One LDS slice holds
        // both: consecutive intervals are stored in opposite row orders
        // (interval m in ascending rows when n_ck - 1 - m is even), so the
        // replay writes each row right after the walk has read it; the
        // walk's read-ahead reaches two slack rows past either end.
        const int L = sp;
        const int R = 2 * kWave;  // doubles per row
        auto row_of = [&](bool asc, int i) { return lst + (asc ? i : L - 1 - i) * R; };
        // replay state of the interval before the walked one (kf: the
        // segment whose beta sf holds, -1 before the first replay)
        SirdState<double> yr;
        StepConst<double> sf = sc;
        int kf = -1, rnext = INT_MAX;
        // the segment of the latest replay start and its first step: replay
        // starts only move down, an interval at a time, from below T
        int k0 = k_last;
        int k0_lo = k_last * SS;
        auto replay_start = [&](int n0r, double s0, double I0r, double S0) {
            yr.s = s0;
            yr.I = I0r;
            yr.S = S0;
            yr.Rr = yr.D = 0.0;
            yr.eS = yr.eI = yr.eR = yr.eD = 0.0;
            while (n0r < k0_lo) {
                --k0;
                k0_lo -= SS;
            }
            // the previous replay may have ended in this segment: then sf
            // and rnext already belong to it
            if (k0 != kf) {
                kf = k0;
                set_beta(sf, lb[kf * kWave + lane], invN);
                rnext = next_seg_start(kf, SS, K, T);
            }
        };
        // one replayed day: spd steps from step rst into rows w, w + dw, ...
        auto replay_step = [&](double *&w, int dw) __attribute__((always_inline)) {
            w[0] = yr.s;
            w[kWave] = yr.I;
            w += dw;
            rk4_step<double, false, false>(yr, sf);
        };
        // Checkpoints reach the replay through LDS: loaded one interval
        // ahead and parked after the first day walked, so no load the replay
        // waits for is ever issued shortly before it (waits on loads cover
        // every load issued before).
        // mck: the checkpoint the next prefetch loads (one lower each time),
        // at slot address pck
        double ps_ = 0.0, pI_ = 0.0, pS_ = 0.0;
        int mck = n_ck - 2;
        const double *pck = wsb + 3 * (size_t)(mck > 0 ? mck : 0) * PS;
        auto prefetch = [&]() {
            if (mck >= 0) {
                ps_ = load_at(pck);
                pI_ = load_at(pck + PS);
                pS_ = load_at(pck + 2 * PS);
                if (mck > 0) pck -= 3 * PS;
            }
            --mck;
        };
        auto park = [&]() {
            lck[0] = ps_;
            lck[kWave] = pI_;
            lck[2 * kWave] = pS_;
        };
        {
            // the last interval alone, ascending
            const int n0 = (n_ck - 1) * L;
            const size_t q = 3 * (size_t)(n_ck - 1);
            replay_start(n0, load(q), load(q + 1), load(q + 2));
            prefetch();
            double *w = lst;
            for (int rst = n0; rst < T; rst += spd) {
                if (rst == rnext) change_segment(yr, sf, kf, rnext, lb, lane, invN, SS, K, T);
                for (int i = 0; i < spd; ++i) replay_step(w, R);
            }
            park();
        }
        for (int m = n_ck - 1; m >= 0; --m) {
            const int n0 = m * L;
            const int n1 = (n0 + L < T) ? n0 + L : T;
            const bool asc = ((n_ck - 1 - m) & 1) == 0;
            // walk: row of step n1 - 1, then one row per step towards n0
            double *r = asc ? lst + (n1 - 1 - n0) * R : lst + (L - 1 - (n1 - 1 - n0)) * R;
            const int dr = asc ? -R : R;
            // replay of interval m - 1 in the other order
            const bool rep = m > 0;
            double *w = row_of(!asc, 0);
            const int dw = asc ? -R : R;
            int rst = (m - 1) * L;
            if (rep) {
                replay_start(rst, lck[0], lck[kWave], lck[2 * kWave]);
                prefetch();
            }
            double ps = r[0], pI = r[kWave];
            double qs = r[dr], qI = r[dr + kWave];
            r -= dr;
            for (int hi = n1 - 1; hi >= n0; hi -= spd) {
                const int lo = hi - spd + 1;  // a day start
                const double Dd = load_at(pday);
                const double Jd = load_at(pjd);
                const double yd = ly[dnext], wd = lw[dnext];
                r += dr;
                Stages cur;
                cur.s = ps;
                cur.I = pI;
                ps = qs;
                pI = qI;
                qs = r[2 * dr];
                qI = r[2 * dr + kWave];
                stages(cur, sc);
                if (rep && rst == rnext)
                    change_segment(yr, sf, kf, rnext, lb, lane, invN, SS, K, T);
                if (rep) {
#pragma unroll 4
                    for (int st = hi; st > lo; --st) {
                        replay_step(w, dw);
                        Stages nxt;
                        nxt.s = ps;
                        nxt.I = pI;
                        ps = qs;
                        pI = qI;
                        r += dr;
                        qs = r[2 * dr];
                        qI = r[2 * dr + kWave];
                        stages(nxt, sc);
                        rev_step(cur, hS, hI, sc, m6, g);
                        cur = nxt;
                    }
                    replay_step(w, dw);
                    rst += spd;
                } else {
#pragma unroll 2
                    for (int st = hi; st > lo; --st) {
                        Stages nxt;
                        nxt.s = ps;
                        nxt.I = pI;
                        ps = qs;
                        pI = qI;
                        r += dr;
                        qs = r[2 * dr];
                        qI = r[2 * dr + kWave];
                        stages(nxt, sc);
                        rev_step(cur, hS, hI, sc, m6, g);
                        cur = nxt;
                    }
                }
                rev_step(cur, hS, hI, sc, m6, g);
                day_start(lo, Dd, Jd, yd, wd);
                if (hi == n1 - 1 && m >= 2) park();
            }
            // the replayed interval is longer than the walked one (only
            // after the last interval): its remaining days alone
            if (rep) {
                for (; rst < n0; rst += spd) {
                    if (rst == rnext) change_segment(yr, sf, kf, rnext, lb, lane, invN, SS, K, T);
                    for (int i = 0; i < spd; ++i) replay_step(w, dw);
                }
            }
        }
    } else {
    // the checkpoint of the interval to reverse next, loaded one interval
    // ahead
    double cs_, cI, cS;
    {
        const size_t q = 3 * (size_t)(n_ck - 1);
        cs_ = load(q);
        cI = load(q + 1);
        cS = load(q + 2);
    }
    for (int m = n_ck - 1; m >= 0; --m) {
        const int n0 = m * sp;
        const int n1 = (n0 + sp < T) ? n0 + sp : T;
        SirdState<double> ck;
        ck.s = cs_;
        ck.I = cI;
        ck.S = cS;
        ck.Rr = ck.D = 0.0;
        ck.eS = ck.eI = ck.eR = ck.eD = 0.0;
        // One sub-interval [b0, b1) from its start state y: replayed into
        // LDS, then walked backwards; prefetch: load the next interval's
        // checkpoint between the two.
        auto sub_interval = [&](int b0, int b1, SirdState<double> y, bool prefetch)
                                __attribute__((always_inline)) {
            // replay the sub-interval into LDS: (s, I) before every step
            {
                int kf = seg_of(b0, SS, K);
                StepConst<double> sf = sc;
                set_beta(sf, lb[kf * kWave + lane], invN);
                int next = next_seg_start(kf, SS, K, T);
                // the first row outside the loop: whatever load the start
                // state came from has landed before any loop below runs
                lst[0] = y.s;
                lst[kWave] = y.I;
                rk4_step<double, false, false>(y, sf);
                double *w = lst + 2 * kWave;
                for (int st = b0 + 1; st < b1;) {
                    if (st == next) change_segment(y, sf, kf, next, lb, lane, invN, SS, K, T);
                    const int stop = min(b1, next);
#pragma unroll 2
                    for (; st < stop; ++st, w += 2 * kWave) {
                        w[0] = y.s;
                        w[kWave] = y.I;
                        rk4_step<double, false, false>(y, sf);
                    }
                }
            }
            if (prefetch && m > 0) {
                // the next interval's checkpoint, loaded while this one is
                // walked (after the replay, whose first step waits for every
                // load in flight)
                const size_t q = 3 * (size_t)(m - 1);
                cs_ = load(q);
                cI = load(q + 1);
                cS = load(q + 2);
            }
            // walk it backwards; day starts take the cost's gradient, and the
            // first step of a segment closes that segment's beta sum.  Steps
            // hi down to lo of one day are reversed with no event between
            // them; the stages of the next step are formed before the
            // current step's adjoint (the two chains overlap) and the LDS
            // state of the step after that is read a step ahead.
            int st = b1 - 1;
            while (st >= b0) {
                const int dstart = dnext * spd;
                const int lo = dstart > b0 ? dstart : b0;
                // a run that ends at a day start loads that day's Dhat before
                // its steps and uses it after them (no load is left in flight
                // into the next replay, whose first step would wait for it)
                const double Dd = lo == dstart ? load_at(pday) : 0.0;
                const double Jd = lo == dstart ? load_at(pjd) : 0.0;
                const double yd = ly[dnext], wd = lw[dnext];
                // rows of steps st, st - 1, ...; two rows are read ahead,
                // which below lo reaches the two slack rows under row 0
                const double *r = lst + (st - b0) * (2 * kWave);
                Stages cur;
                cur.s = r[0];
                cur.I = r[kWave];
                double ps = r[-2 * kWave], pI = r[-kWave];
                double qs = r[-4 * kWave], qI = r[-3 * kWave];
                stages(cur, sc);
#pragma unroll 2
                for (; st > lo; --st) {
                    Stages nxt;
                    nxt.s = ps;
                    nxt.I = pI;
                    ps = qs;
                    pI = qI;
                    r -= 2 * kWave;
                    qs = r[-4 * kWave];
                    qI = r[-3 * kWave];
                    stages(nxt, sc);
                    rev_step(cur, hS, hI, sc, m6, g);
                    cur = nxt;
                }
                rev_step(cur, hS, hI, sc, m6, g);
                if (lo == dstart) day_start(dstart, Dd, Jd, yd, wd);
                st = lo - 1;
            }
        };
        const int nsub = (n1 - n0 + a.lc - 1) / a.lc;
        if (nsub == 1) {
            // the interval fits the LDS slice (the default interval): its
            // own code path, where no load is in flight at the replay
            sub_interval(n0, n1, ck, true);
            continue;
        }
        // with more than one sub-interval: replay up to the last one's start,
        // storing the starts of the ones between (the first starts at the
        // checkpoint, the last one's start stays in registers)
        SirdState<double> last = ck;
        {
            int kf = seg_of(n0, SS, K);
            StepConst<double> sf = sc;
            set_beta(sf, lb[kf * kWave + lane], invN);
            int next = next_seg_start(kf, SS, K, T);
            int st = n0, mark = n0 + a.lc;
            size_t sq = q_sub;
            double jdummy = 0.0;
            advance_marked(last, sf, kf, next, st, n0 + (nsub - 1) * a.lc, mark, a.lc, lb, lane,
                           invN, SS, K, T, jdummy, [&]() {
                               sq += 3;
                               if (active) {
                                   slot(sq) = last.s;
                                   slot(sq + 1) = last.I;
                                   slot(sq + 2) = last.S;
                               }
                           });
            // the last sub-interval may open a segment: its start state after
            // the change, as every stored start holds it
            if (st == next) change_segment(last, sf, kf, next, lb, lane, invN, SS, K, T);
        }
        for (int j = nsub - 1; j >= 0; --j) {
            const int b0 = n0 + j * a.lc;
            const int b1 = (b0 + a.lc < n1) ? b0 + a.lc : n1;
            SirdState<double> y = ck;
            if (j == nsub - 1) {
                y = last;
            } else if (j > 0) {
                const size_t q = q_sub + 3 * (size_t)j;
                y.s = load(q);
                y.I = load(q + 1);
                y.S = load(q + 2);
            }
            sub_interval(b0, b1, y, j == nsub - 1);
        }
    }
    }
    if (active) {
        const double tI = fma(2.0, g.T23, g.T14);  // sum over stages of I_s kbar_s.I
        gout[(size_t)kr * ld] = beta_grad(g, sc.b, Sk, invN) * gl;
        gout[(size_t)K * ld] = -tI * gl;
        gout[(size_t)(K + 1) * ld] = (muD - tI) * gl;
        gout[(size_t)(K + 2) * ld] = ((hI - hS) / sc.h6) * gl;
    }
}

// ------------------------------------------------ segment-parallel sweep
// The reverse sweep is affine in the (scaled) adjoint c = h/6 a of (S, I):
// a_D never depends on c (D does not feed back), and at any step it is the
// sum of the cost's dl/dDhat_i over the days after the step, known once the
// forward pass has saved Dhat.  So the sweep over one beta segment maps the
// adjoint c_end at the segment's end to c_start = A c_end + b, and the
// segment's sums (of s_s I_s u, I_s u and I_s kbar.I over its stages) are
// affine in c_end too, and so is the map of any run of days within a
// segment.  k_seg_transfer cuts every segment into pieces of at most
// kSegPieceDays days and runs every piece of every parameter vector at once
// (a wavefront per tile and piece, replaying each day from the checkpoint at
// its start), walking three adjoints backwards through the piece with the
// same reverse step as the sequential sweep: c = (1, 0) and c = (0, 1)
// without a_D (the columns of A, and the sums' slopes), and c = 0 with a_D
// (b, and the sums' offsets).  k_seg_combine then chains the pieces from the
// last, one lane per vector, adding up each segment's sums.  The gradient is the
// sequential sweep's up to rounding (its sums are added in another order).

// Workspace slots of one piece's affine map, after the two tail slots:
// A (c_S, c_I of both unit walks), b, and per walk the sums of s_s I_s u,
// I_s u and I_s kbar.I, then the piece's part of the mu sum's D part.
constexpr int kSegSlots = 16;
// A segment is walked in pieces of at most this many days, a wavefront each
// (a segment's map is the chain of its pieces' maps).
constexpr int kSegPieceDays = 7;

// The days [d0, d1) of segment k <= k_last (segments start at day starts;
// the last one runs to the window's end) and its number of pieces.
__device__ __forceinline__ int seg_pieces(int k, int k_last, int SS, int spd, int W, int &d0,
                                          int &d1)
{
    d0 = (k * SS) / spd;
    d1 = k == k_last ? W : ((k + 1) * SS) / spd;
    return (d1 - d0 + kSegPieceDays - 1) / kSegPieceDays;
}

// The workspace column of one lane: slot q of particle p at ws[q * stride + p],
// addressed as a uniform base (the tile's first particle) plus the lane's
// byte offset.
struct WsLane {
    double *base;
    size_t stride;
    uint32_t off;

    __device__ __forceinline__ double load(size_t q) const
    {
        const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(base + q * stride), (short)0, kWave * (int)sizeof(double), kBufferWord3);
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
    }
    __device__ __forceinline__ void store(size_t q, double v) const
    {
        const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(base + q * stride), (short)0, kWave * (int)sizeof(double), kBufferWord3);
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U32x2, v), r, off, 0, 0);
    }
};

// Slots of the segment-parallel sweep's workspace (no stored sub-interval
// starts): checkpoint d at 3d .. 3d + 2 (s, I, S), then Dhat, S at every
// segment start, the sums of J, the tail (MXSE's day, the loss) and the
// pieces' affine maps.
struct SegSlots {
    size_t day, seg, jd, tail, map;
    __device__ __forceinline__ SegSlots(const BwdArgs &a)
    {
        day = 3 * (size_t)a.n_ck_max;
        seg = day + (size_t)(a.max_days + 1);
        jd = seg + (size_t)a.max_seg;
        tail = jd + (size_t)a.max_days;
        map = tail + 2;
    }
};

// One wavefront per (tile, piece), one lane per parameter vector; pieces are
// numbered segment by segment from the first.
template <int KIND>
__global__ void __launch_bounds__(kWave) k_seg_transfer(BwdArgs a)
{
    extern __shared__ double lds[];
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = wave_uniform((int)blockIdx.x);
    const int t = wv / a.max_pieces;
    const int piece = wv - t * a.max_pieces;
    if (t >= a.n_tiles) return;
    const sird_tile tl = a.tiles[t];
    const sird_problem P = a.probs[tl.prob];
    const int W = P.n_days, spd = P.steps_per_day, K = P.n_seg, n = P.n_part;
    const int T = W * spd;
    const int SS = (int)min((long)P.seg_days * spd, (long)T + 1);
    const int k_last = seg_of(T - 1, SS, K);
    // the piece's segment k and days [d0, d1)
    int k = 0, j = piece, d0 = 0, d1 = 0;
    for (; k <= k_last; ++k) {
        const int np = seg_pieces(k, k_last, SS, spd, W, d0, d1);
        if (j < np) break;
        j -= np;
    }
    if (k > k_last) return;  // past the problem's last piece
    {
        const int s0 = d0 + j * kSegPieceDays;
        d1 = min(s0 + kSegPieceDays, d1);
        d0 = s0;
    }
    const int pl = tl.p0 + lane;
    const bool active = pl < n;
    const int pc = active ? pl : n - 1;
    const size_t ld = (size_t)n;
    const double *th = a.theta + P.theta_off + pc;
    const WsLane ws{a.ws + (size_t)(P.p_off + tl.p0), (size_t)a.P,
                    (uint32_t)(pc - tl.p0) * (uint32_t)sizeof(double)};
    const SegSlots q(a);
    // LDS of the wavefront: the deceased counts and their weights, then
    // [2 slack][seg_rows][2][64], (s, I) of the lane before each step of one
    // part of a day (the walk's read-ahead touches the slack rows below
    // row 0 and never uses them)
    double *const ly = lds;
    double *const lw = ly + (a.max_days + 1);
    double *const lst = lw + (a.max_days + 1) + 4 * kWave + lane;
    {
        const double *y = a.obs + P.obs_off + (size_t)(a.obs_series - 1) * (W + 1);
        for (int i = lane; i <= W; i += kWave) {
            const double yi = y[i];
            ly[i] = yi;
            lw[i] = 1.0 / fmax(yi, 1.0);
        }
        wave_sync();
    }
    const double gamma = th[(size_t)K * ld];
    const double mu = th[(size_t)(K + 1) * ld];
    StepConst<double> sc = step_const<double>(gamma, mu, spd);
    set_beta(sc, th[(size_t)k * ld], 1.0 / P.N);
    const int imax = (int)ws.load(q.tail);
    // a_D over the piece's last day: the cost's gradient at days W down to
    // d1, added in the sequential sweep's order; Dhat is loaded sixteen days
    // at a time (one memory round trip per sixteen days, not per day)
    double aD = cost_grad(KIND, W, W, ws.load(q.day + W), ly[W], lw[W], imax);
    for (int i0 = W - 1; i0 >= d1; i0 -= 16) {
        double Dv[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) Dv[i] = ws.load(q.day + (size_t)max(i0 - i, d1));
#pragma unroll
        for (int i = 0; i < 16; ++i)
            if (i0 - i >= d1)
                aD += cost_grad(KIND, i0 - i, W, Dv[i], ly[i0 - i], lw[i0 - i], imax);
    }
    // the three walks: unit c_S, unit c_I (no a_D), and c = 0 with a_D
    double c1S = 1.0, c1I = 0.0, c2S = 0.0, c2I = 1.0, c3S = 0.0, c3I = 0.0;
    RevSums g1{0.0, 0.0, 0.0, 0.0, 0.0}, g2 = g1, g3 = g1;
    double muD = 0.0;
    const int R = a.seg_rows;
    const int nparts = (spd + R - 1) / R;
    // the day's checkpoint, Dhat and sum of J are loaded a day ahead
    double nDd = ws.load(q.day + d1 - 1), nJd = ws.load(q.jd + d1 - 1);
    double nck_s = ws.load(3 * (size_t)(d1 - 1)), nck_I = ws.load(3 * (size_t)(d1 - 1) + 1);
    for (int d = d1 - 1; d >= d0; --d) {
        const double m6 = sc.h6 * (mu * aD);
        const double Dd = nDd, Jd = nJd, ck_s = nck_s, ck_I = nck_I;
        if (d > d0) {
            nDd = ws.load(q.day + d - 1);
            nJd = ws.load(q.jd + d - 1);
            nck_s = ws.load(3 * (size_t)(d - 1));
            nck_I = ws.load(3 * (size_t)(d - 1) + 1);
        }
        // the day's steps in parts of at most R, the last part first; a part
        // is replayed from the day's checkpoint
        for (int u = nparts - 1; u >= 0; --u) {
            const int b0 = u * R;
            const int b1 = min(spd, b0 + R);
            SirdState<double> y;
            y.s = ck_s;
            y.I = ck_I;
            y.S = y.Rr = y.D = 0.0;
            y.eS = y.eI = y.eR = y.eD = 0.0;
            for (int i = 0; i < b0; ++i) rk4_step<double, false, false>(y, sc);
            double *w = lst;
            for (int i = b0; i < b1; ++i, w += 2 * kWave) {
                w[0] = y.s;
                w[kWave] = y.I;
                rk4_step<double, false, false>(y, sc);
            }
            const double *r = lst + (size_t)(b1 - b0 - 1) * (2 * kWave);
            Stages cur;
            cur.s = r[0];
            cur.I = r[kWave];
            double ps = r[-2 * kWave], pI = r[-kWave];
            stages(cur, sc);
            for (int i = b1 - 1; i > b0; --i) {
                Stages nxt;
                nxt.s = ps;
                nxt.I = pI;
                r -= 2 * kWave;
                ps = r[-2 * kWave];
                pI = r[-kWave];
                stages(nxt, sc);
                rev_step(cur, c1S, c1I, sc, 0.0, g1);
                rev_step(cur, c2S, c2I, sc, 0.0, g2);
                rev_step(cur, c3S, c3I, sc, m6, g3);
                cur = nxt;
            }
            rev_step(cur, c1S, c1I, sc, 0.0, g1);
            rev_step(cur, c2S, c2I, sc, 0.0, g2);
            rev_step(cur, c3S, c3I, sc, m6, g3);
        }
        // the day start, as the sequential sweep takes it
        muD = fma(sc.h6 * aD, Jd, muD);
        aD += cost_grad(KIND, d, W, Dd, ly[d], lw[d], imax);
    }
    if (active) {
        const size_t m = q.map + (size_t)kSegSlots * piece;
        const double out[kSegSlots] = {c1S,
                                       c1I,
                                       c2S,
                                       c2I,
                                       c3S,
                                       c3I,
                                       fma(2.0, g1.G23, g1.G14),
                                       fma(2.0, g2.G23, g2.G14),
                                       fma(2.0, g3.G23, g3.G14),
                                       g1.Gv,
                                       g2.Gv,
                                       g3.Gv,
                                       fma(2.0, g1.T23, g1.T14),
                                       fma(2.0, g2.T23, g2.T14),
                                       fma(2.0, g3.T23, g3.T14),
                                       muD};
#pragma unroll
        for (int i = 0; i < kSegSlots; ++i) ws.store(m + i, out[i]);
    }
}

// One lane per parameter vector: the pieces' maps chained from the last
// (where c = 0) to the first, the gradient written.
__global__ void __launch_bounds__(256) k_seg_combine(BwdArgs a)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int t = wave_tile_index();
    if (t >= a.n_tiles) return;
    const sird_tile tl = a.tiles[t];
    const sird_problem P = a.probs[tl.prob];
    const int W = P.n_days, spd = P.steps_per_day, K = P.n_seg, n = P.n_part;
    const int T = W * spd;
    const int SS = (int)min((long)P.seg_days * spd, (long)T + 1);
    const int k_last = seg_of(T - 1, SS, K);
    const int pl = tl.p0 + lane;
    const bool active = pl < n;
    const int pc = active ? pl : n - 1;
    const size_t ld = (size_t)n;
    const double *th = a.theta + P.theta_off + pc;
    const WsLane ws{a.ws + (size_t)(P.p_off + tl.p0), (size_t)a.P,
                    (uint32_t)(pc - tl.p0) * (uint32_t)sizeof(double)};
    const SegSlots q(a);
    if (active && a.loss_out) a.loss_out[P.p_off + pl] = ws.load(q.tail + 1);
    const double gl = a.grad_loss ? a.grad_loss[P.p_off + pc] : 1.0;
    double *gout = a.grad + P.theta_off + pc;
    for (int k = k_last + 1; k < K; ++k)
        if (active) gout[(size_t)k * ld] = 0.0;  // segments past the window end
    const double invN = 1.0 / P.N;
    int total = 0, d0 = 0, d1 = 0;
    for (int k = 0; k <= k_last; ++k) total += seg_pieces(k, k_last, SS, spd, W, d0, d1);
    // the pieces from the last: a segment's sums over its pieces, its beta's
    // gradient after its first piece.  The chain is a few operations per
    // piece and its maps come from memory, so the maps are loaded four
    // pieces ahead (four register sets in turn).
    double cS = 0.0, cI = 0.0, tI = 0.0, muD = 0.0, G = 0.0, Gv = 0.0;
    int k = k_last;
    int left = seg_pieces(k, k_last, SS, spd, W, d0, d1);  // pieces of k to chain
    auto load_map = [&](double(&dst)[kSegSlots], int g) {
        if (g >= 0) {
#pragma unroll
            for (int i = 0; i < kSegSlots; ++i)
                dst[i] = ws.load(q.map + (size_t)kSegSlots * g + i);
        }
    };
    auto chain = [&](const double(&v)[kSegSlots]) {
        G += fma(v[6], cS, fma(v[7], cI, v[8]));
        Gv += fma(v[9], cS, fma(v[10], cI, v[11]));
        tI += fma(v[12], cS, fma(v[13], cI, v[14]));
        muD += v[15];
        const double nS = fma(v[0], cS, fma(v[2], cI, v[4]));
        const double nI = fma(v[1], cS, fma(v[3], cI, v[5]));
        cS = nS;
        cI = nI;
        if (--left == 0) {
            const double b = th[(size_t)k * ld] * invN;
            const double gk = b != 0.0 ? (G / b) * invN : (ws.load(q.seg + k) * Gv) * invN;
            if (active) gout[(size_t)k * ld] = gk * gl;
            G = Gv = 0.0;
            if (--k >= 0) left = seg_pieces(k, k_last, SS, spd, W, d0, d1);
        }
    };
    double m0[kSegSlots] = {}, m1[kSegSlots] = {}, m2[kSegSlots] = {}, m3[kSegSlots] = {};
    load_map(m0, total - 1);
    load_map(m1, total - 2);
    load_map(m2, total - 3);
    load_map(m3, total - 4);
    for (int g = total - 1; g >= 0; g -= 4) {
        chain(m0);
        load_map(m0, g - 4);
        if (g < 1) break;
        chain(m1);
        load_map(m1, g - 5);
        if (g < 2) break;
        chain(m2);
        load_map(m2, g - 6);
        if (g < 3) break;
        chain(m3);
        load_map(m3, g - 7);
    }
    if (active) {
        const double h6 = step_const<double>(0.0, 0.0, spd).h6;
        gout[(size_t)K * ld] = -tI * gl;
        gout[(size_t)(K + 1) * ld] = (muD - tI) * gl;
        gout[(size_t)(K + 2) * ld] = ((cI - cS) / h6) * gl;
    }
}

// Steps per LDS sub-interval: as many as fit the wavefront's share of LDS
// (four wavefronts per compute unit) next to the observations and betas,
// within [kLcMin, kLcMax].
static int lds_steps(const sird_batch *b)
{
    const long fixed = 8L * (2L * (b->max_days + 1) + (long)kWave * (b->max_d - 3 + 3 + 8));
    long lc = (kBwdLdsBudget - fixed) / (2L * kWave * 8);
    if (lc < kLcMin) lc = kLcMin;
    if (lc > kLcMax) lc = kLcMax;
    return (int)lc;
}

// Checkpoints per particle for ckpt_interval.  0: per problem the whole
// days that fit lc steps (an interval of at least (lc + 1)/2 steps, and at
// most one checkpoint a day), or lc steps when a day is longer.
static int64_t checkpoints(const sird_batch *b, int ckpt_interval)
{
    const int lc = lds_steps(b);
    if (ckpt_interval > 0) return (b->max_steps + ckpt_interval - 1) / ckpt_interval;
    const int64_t per_lc = (b->max_steps + lc - 1) / lc;
    int64_t aligned = (2 * b->max_steps + lc) / (lc + 1);
    if (aligned > b->max_days) aligned = b->max_days;
    return per_lc > aligned ? per_lc : aligned;
}

// A bound on the segment-parallel sweep's pieces of any problem: a segment
// of n days has ceil(n / kSegPieceDays) pieces, at most n / kSegPieceDays + 1.
static int seg_max_pieces(const sird_batch *b)
{
    return (b->max_days + kSegPieceDays - 1) / kSegPieceDays + (b->max_d - 3);
}

// Workspace slots per particle: 3 per checkpoint (s, I, S), 3 per LDS
// sub-interval of an interval longer than one (the first and last
// sub-intervals' slots go unused: the first starts at the checkpoint, the
// last one's start stays in registers), Dhat of every day, S at every
// segment start, every day's sum of J, the day MXSE peaks on and the loss.
static size_t ws_slots(const sird_batch *b, int ckpt_interval)
{
    if (ckpt_interval == SIRD_CKPT_SEGMENTS)
        return (size_t)(3 * (int64_t)b->max_days + b->max_days + 1 + (b->max_d - 3) +
                        b->max_days + 2 + (int64_t)kSegSlots * seg_max_pieces(b));
    const int lc = lds_steps(b);
    const int64_t n_ck = checkpoints(b, ckpt_interval);
    const int64_t n_sub =
        ckpt_interval > lc ? ((int64_t)ckpt_interval + lc - 1) / lc : 0;
    return (size_t)(3 * n_ck + 3 * n_sub + b->max_days + 1 + (b->max_d - 3) + b->max_days + 2);
}

template <int MODE>
static void launch_backward(int kind, int grid, int block, size_t lds, hipStream_t s,
                            const BwdArgs &a)
{
    switch (kind) {
    case SIRD_LOSS_SSRE:
        hipLaunchKernelGGL((k_backward<SIRD_LOSS_SSRE, MODE>), dim3(grid), dim3(block), lds, s, a);
        break;
    case SIRD_LOSS_MSE:
        hipLaunchKernelGGL((k_backward<SIRD_LOSS_MSE, MODE>), dim3(grid), dim3(block), lds, s, a);
        break;
    case SIRD_LOSS_MXSE:
        hipLaunchKernelGGL((k_backward<SIRD_LOSS_MXSE, MODE>), dim3(grid), dim3(block), lds, s, a);
        break;
    case SIRD_LOSS_MAE:
        hipLaunchKernelGGL((k_backward<SIRD_LOSS_MAE, MODE>), dim3(grid), dim3(block), lds, s, a);
        break;
    default:
        hipLaunchKernelGGL((k_backward<SIRD_LOSS_MAPE, MODE>), dim3(grid), dim3(block), lds, s,
                           a);
        break;
    }
}

size_t adjoint_workspace_bytes(const sird_batch *b, int ckpt_interval)
{
    return ws_slots(b, ckpt_interval) * (size_t)b->total_particles *
           sizeof(double);
}

// Host checks of a gradient call that do not concern the workspace; fills
// every field of *a but ws, and the launch shape.
static int adjoint_prepare(const sird_batch *batch, const double *theta, const double *obs,
                           int loss_kind, const double *grad_loss, double *grad_theta,
                           double *loss_out, int ckpt_interval, int mode, BwdArgs *a,
                           int *grid, size_t *lds, const char *who)
{
    const std::string w(who);
    int st = check_batch(batch, who);
    if (st) return st;
    if (!theta || !obs) return fail(SIRD_EINVAL, w + ": NULL array");
    if (mode != kFwdOnly && !grad_theta) return fail(SIRD_EINVAL, w + ": grad_theta is NULL");
    if (mode == kFwdOnly && !loss_out) return fail(SIRD_EINVAL, w + ": loss is NULL");
    if (batch->dtype != SIRD_F64)
        return fail(SIRD_EINVAL, w + ": the adjoint supports SIRD_F64 batches only");
    if (loss_kind < SIRD_LOSS_SSRE || loss_kind > SIRD_LOSS_MAPE)
        return fail(SIRD_EINVAL, w + ": the adjoint needs a deceased-count cost (loss_kind 0..4)");
    if (batch->models != 1 << SIRD_MODEL_RK4_SEGMENTS)
        return fail(SIRD_EINVAL, w + ": the adjoint supports the RK4 segment model only");
    const bool seg = ckpt_interval == SIRD_CKPT_SEGMENTS;
    if (ckpt_interval < 0 && !seg)
        return fail(SIRD_EINVAL, w + ": ckpt_interval < 0 (and not SIRD_CKPT_SEGMENTS)");
    if (batch->obs_len < 1) return fail(SIRD_EINVAL, w + ": batch planned without obs");
    *a = BwdArgs{};
    a->probs = batch->probs;
    a->tiles = batch->tiles;
    a->theta = theta;
    a->obs = obs;
    a->grad_loss = grad_loss;
    a->grad = grad_theta;
    a->loss_out = loss_out;
    a->P = batch->total_particles;
    a->n_tiles = batch->n_tiles;
    a->obs_series = batch->obs_series;
    a->s = seg ? 0 : ckpt_interval;
    a->lc = lds_steps(batch);
    a->n_ck_max = seg ? batch->max_days : (int)checkpoints(batch, ckpt_interval);
    a->n_sub_max = !seg && ckpt_interval > a->lc ? (ckpt_interval + a->lc - 1) / a->lc : 0;
    a->max_days = batch->max_days;
    a->max_seg = batch->max_d - 3;
    a->seg = seg ? 1 : 0;
    if (seg) {
        // rows of a k_seg_transfer wavefront: what fits kBwdLdsBudget next to
        // the observations, their weights and two slack rows
        const long rows = (kBwdLdsBudget / 8L - 2L * (batch->max_days + 1)) / (2L * kWave) - 2;
        if (rows < 1) return fail(SIRD_EINVAL, w + ": window too long for LDS");
        a->seg_rows = (int)(rows < kLcMax ? rows : kLcMax);
        a->max_pieces = seg_max_pieces(batch);
    }
    a->lds_wave = 2 * (batch->max_days + 1) + kWave * (a->max_seg + 3 + 2 * (4 + a->lc));
    *lds = sizeof(double) * (size_t)a->lds_wave;
    if (*lds > 65536) return fail(SIRD_EINVAL, w + ": window too long for LDS");
    *grid = batch->n_tiles;
    return SIRD_OK;
}

// Wavefronts per block of k_backward: four (one per SIMD of the compute unit
// a block lands on) when the device lets a block take four wavefronts' LDS,
// else one.
static int bwd_waves_per_block(size_t lds_per_wave)
{
    static std::atomic<int> per_block[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 1;
    int lim = per_block[dev].load(std::memory_order_relaxed);
    if (lim <= 0) {
        if (hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) !=
                hipSuccess ||
            lim <= 0)
            return 1;
        per_block[dev].store(lim, std::memory_order_relaxed);
    }
    return 4 * lds_per_wave <= (size_t)lim ? 4 : 1;
}

static void launch_seg_transfer(int kind, int grid, size_t lds, hipStream_t s,
                                const BwdArgs &a)
{
    switch (kind) {
    case SIRD_LOSS_SSRE:
        hipLaunchKernelGGL(k_seg_transfer<SIRD_LOSS_SSRE>, dim3(grid), dim3(kWave), lds, s, a);
        break;
    case SIRD_LOSS_MSE:
        hipLaunchKernelGGL(k_seg_transfer<SIRD_LOSS_MSE>, dim3(grid), dim3(kWave), lds, s, a);
        break;
    case SIRD_LOSS_MXSE:
        hipLaunchKernelGGL(k_seg_transfer<SIRD_LOSS_MXSE>, dim3(grid), dim3(kWave), lds, s, a);
        break;
    case SIRD_LOSS_MAE:
        hipLaunchKernelGGL(k_seg_transfer<SIRD_LOSS_MAE>, dim3(grid), dim3(kWave), lds, s, a);
        break;
    default:
        hipLaunchKernelGGL(k_seg_transfer<SIRD_LOSS_MAPE>, dim3(grid), dim3(kWave), lds, s, a);
        break;
    }
}

// The reverse sweep of the segment-parallel form: the pieces' maps, then
// their chain (grid: tiles).
static int seg_reverse(int loss_kind, int grid, hipStream_t stream, const BwdArgs &a,
                       const char *who)
{
    const size_t lds = sizeof(double) * (2 * (size_t)(a.max_days + 1) +
                                         (size_t)kWave * 2 * (size_t)(a.seg_rows + 2));
    launch_seg_transfer(loss_kind, grid * a.max_pieces, lds, stream, a);
    int st = hip_status(hipGetLastError(), who);
    if (st) return st;
    hipLaunchKernelGGL(k_seg_combine, dim3(tile_blocks(grid)), dim3(256), 0, stream, a);
    return hip_status(hipGetLastError(), who);
}

// grid: tiles (one wavefront each); lds: bytes per wavefront.
static int adjoint_launch(int mode, int loss_kind, int grid, size_t lds, hipStream_t stream,
                          const BwdArgs &a, const char *who)
{
    if (grid == 0) return SIRD_OK;
    if (a.seg && mode != kFwdOnly) {
        // the forward pass (checkpoints at every day start) unless it is
        // saved, then the pieces' maps and their chain
        if (mode == kBoth) {
            const int st = adjoint_launch(kFwdOnly, loss_kind, grid, lds, stream, a, who);
            if (st) return st;
        }
        return seg_reverse(loss_kind, grid, stream, a, who);
    }
    const int wpb = bwd_waves_per_block(lds);
    const int blocks = (grid + wpb - 1) / wpb;
    const int block = wpb * kWave;
    const size_t bytes = (size_t)wpb * lds;
    if (mode == kFwdOnly)
        launch_backward<kFwdOnly>(loss_kind, blocks, block, bytes, stream, a);
    else if (mode == kRevOnly)
        launch_backward<kRevOnly>(loss_kind, blocks, block, bytes, stream, a);
    else
        launch_backward<kBoth>(loss_kind, blocks, block, bytes, stream, a);
    return hip_status(hipGetLastError(), who);
}

int adjoint_enqueue(const sird_batch *batch, const double *theta, const double *obs,
                    int loss_kind, const double *grad_loss, double *grad_theta,
                    double *loss_out, int ckpt_interval, int mode, void *workspace,
                    size_t ws_bytes, hipStream_t stream, const char *who)
{
    const std::string w(who);
    BwdArgs a;
    int grid = 0;
    size_t lds = 0;
    int st = adjoint_prepare(batch, theta, obs, loss_kind, grad_loss, grad_theta, loss_out,
                             ckpt_interval, mode, &a, &grid, &lds, who);
    if (st) return st;
    if (!workspace) return fail(SIRD_EINVAL, w + ": NULL array");
    if (((uintptr_t)workspace & 255) != 0)
        return fail(SIRD_EINVAL, w + ": workspace not 256-byte aligned");
    if (ws_bytes < adjoint_workspace_bytes(batch, ckpt_interval))
        return fail(SIRD_ENOSPACE, w + ": workspace too small");
    a.ws = (double *)workspace;
    return adjoint_launch(mode, loss_kind, grid, lds, stream, a, who);
}

}  // namespace sird

using namespace sird;

extern "C" size_t sird_loss_backward_workspace(const sird_batch *batch, int ckpt_interval)
{
    if (check_batch(batch, "sird_loss_backward_workspace")) return 0;
    if (ckpt_interval < 0 && ckpt_interval != SIRD_CKPT_SEGMENTS) return 0;
    return adjoint_workspace_bytes(batch, ckpt_interval);
}

extern "C" int sird_loss_backward(const sird_batch *batch, const double *theta,
                                  const double *obs, int loss_kind, const double *grad_loss,
                                  double *grad_theta, double *loss_out, int ckpt_interval,
                                  int from_forward, void *workspace, size_t ws_bytes,
                                  void *stream)
{
    if (from_forward != 0 && from_forward != 1)
        return fail(SIRD_EINVAL, "sird_loss_backward: from_forward must be 0 or 1");
    return adjoint_enqueue(batch, theta, obs, loss_kind, grad_loss, grad_theta, loss_out,
                           ckpt_interval, from_forward ? kRevOnly : kBoth, workspace, ws_bytes,
                           (hipStream_t)stream, "sird_loss_backward");
}

// ------------------------------------------------ allocation-free gradient
// Workspace of sird_loss_backward_static: one array per GPU, placed by the
// loader with the code object and held until the process ends.  Host code
// never passes its name to a kernel (on the host the name is a stand-in,
// not a device address): the device address comes from
// hipGetSymbolAddress, taken once per device with that device current.
static __device__ __align__(256) unsigned char scratch[SIRD_STATIC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];

// Device address of this device's scratch (set up on the first call made
// with that device current), or a negative status.
int static_scratch(void **out, const char *who)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_status(e, who);
    if (dev < 0 || dev >= kMaxDevices)
        return fail(SIRD_EINVAL, std::string(who) + ": device ordinal out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(SIRD_EHIP, std::string(who) + ": hipGetSymbolAddress(scratch): " +
                                       hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return SIRD_OK;
}

}  // namespace

extern "C" int sird_loss_backward_static(const sird_batch *batch, const double *theta,
                                         const double *obs, int loss_kind,
                                         const double *grad_loss, double *grad_theta,
                                         double *loss_out, int ckpt_interval, void *stream)
{
    const char *who = "sird_loss_backward_static";
    BwdArgs a;
    int grid = 0;
    size_t lds = 0;
    int st = adjoint_prepare(batch, theta, obs, loss_kind, grad_loss, grad_theta, loss_out,
                             ckpt_interval, kBoth, &a, &grid, &lds, who);
    if (st) return st;
    const size_t need = adjoint_workspace_bytes(batch, ckpt_interval);
    if (need > (size_t)SIRD_STATIC_SCRATCH_BYTES)
        return fail(SIRD_ENOSPACE,
                    std::string(who) + ": the batch needs " + std::to_string(need) +
                        " bytes of workspace, above the static scratch of " +
                        std::to_string((size_t)SIRD_STATIC_SCRATCH_BYTES) +
                        "; use sird_loss_backward with a workspace");
    void *ws = nullptr;
    st = static_scratch(&ws, who);
    if (st) return st;
    a.ws = (double *)ws;
    return adjoint_launch(kBoth, loss_kind, grid, lds, (hipStream_t)stream, a, who);
}
