// Gradient of the deceased-count cost with respect to theta by the discrete
// adjoint of the RK4 scheme (reverse mode through every stage of every step).
//
// Per particle (one lane, one tile per wavefront):
//   1. forward pass: RK4 over the window, the cost, Dhat_i of every day and
//      the state (S, I, and the stages' scaled susceptible) every s steps
//      (checkpoints) -> workspace;
//   2. reverse sweep over the checkpoint intervals, last to first: replay
//      the interval from its checkpoint, keeping the state before every 8th
//      step in the workspace; then, chunk by chunk from the end, replay 8
//      steps into registers and walk them backwards.  For step n with stages
//      Y1 = y, Y2 = y + h/2 k1, Y3 = y + h/2 k2, Y4 = y + h k3 and adjoint
//      abar of y_{n+1}:
//        kbar4 = h/6 abar,           Ybar4 = J(Y4)^T kbar4
//        kbar3 = h/3 abar + h Ybar4,   Ybar3 = J(Y3)^T kbar3
//        kbar2 = h/3 abar + h/2 Ybar3, Ybar2 = J(Y2)^T kbar2
//        kbar1 = h/6 abar + h/2 Ybar2, Ybar1 = J(y)^T kbar1
//        a_n = abar + Ybar1 + Ybar2 + Ybar3 + Ybar4
//        thetabar += sum_s (df/dtheta)(Y_s)^T kbar_s
//      and the cost's dl/dDhat_i is added to a_D at n = i * spd.
// State (S, I, D) (R never feeds back and no cost reads it): with
// p = b S I, b = beta/N, f = (-p, p - lam I, mu I) and u = kI - kS,
//   J^T k = (b I u,  b S u - lam kI + mu kD,  0),
//   df/dbeta . k = (S I / N) u,  df/dgamma . k = -I kI,  df/dmu . k = I (kD - kI).
// D never feeds back, so its adjoint is piecewise constant between samples
// and kbar_s.D = w_s h a_D with the RK4 weights w = (1/6, 1/3, 1/3, 1/6).
// The initial state depends on I0 through S0 = N - I0 - R0 - D0 and I = I0.
//
// The forward pass here carries S next to s = b S (the form whose stages the
// reverse sweep recomputes); it agrees with the loss kernel, which carries
// s alone, to rounding.  Recomputation is deterministic (same operations
// from the same stored state), so the gradient is bitwise independent of
// the checkpoint interval.
//
// The kernel runs in one of three modes: both passes (sird_loss_backward on
// its own), the forward pass alone (sird_loss given a workspace: the loss,
// and everything the reverse sweep reads, saved in the workspace), or the
// reverse sweep alone from such a workspace (sird_loss_backward with
// from_forward).  The saved forward is the same code as the forward pass of
// the first mode, so the gradient is bitwise the same either way.
#include <hip/hip_runtime.h>

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
    int64_t P;  // slot stride of the workspace (total particles)
    int n_tiles;
    int obs_series;  // 1 or 3; the deceased counts are the last series
    int s;          // checkpoint interval in steps
    int n_ck_max;   // checkpoints per particle
    int max_days;   // max W over problems (Dhat slots per particle - 1)
    int lds_stride;
};

// Modes of k_backward.
enum BwdMode { kBoth = 0, kFwdOnly = 1, kRevOnly = 2 };

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

struct Grad {
    double beta;   // of the current segment, times N: sum of S_s I_s u over its stages
    double gamma;
    double mu;
};

// One stage of the reverse step: Ybar = J(Y_s)^T kbar and the parameter
// contributions; mkD = mu * kbar_s.D.  Ybar.S = b v with v = I_s u is
// returned as v: the next stage's kbar.S and the final sum take b in their
// constants.
__device__ __forceinline__ void stage_adjoint(double Ss, double Is, double bs, double kS,
                                              double kI, double mkD, double lam, double &v,
                                              double &YI, Grad &g, double &tI)
{
    const double u = kI - kS;
    v = Is * u;
    YI = fma(bs, u, fma(-lam, kI, mkD));
    g.beta = fma(Ss, v, g.beta);
    tI = fma(Is, kI, tI);
}

// One reverse step: (aS, aI) <- a_n from a_{n+1}; aD unchanged.
__device__ __forceinline__ void rk4_adjoint_step(double S, double I, double &aS, double &aI,
                                                 double aD, const StepConst<double> &k,
                                                 double mu, double h3, Grad &g)
{
    // recompute the stages
    const double bs1 = k.b * S;
    const double p1 = bs1 * I;
    const double q1 = fma(-k.lam, I, p1);
    const double S2 = fma(-k.h2, p1, S);
    const double I2 = fma(k.h2, q1, I);
    const double bs2 = k.b * S2;
    const double p2 = bs2 * I2;
    const double q2 = fma(-k.lam, I2, p2);
    const double S3 = fma(-k.h2, p2, S);
    const double I3 = fma(k.h2, q2, I);
    const double bs3 = k.b * S3;
    const double p3 = bs3 * I3;
    const double q3 = fma(-k.lam, I3, p3);
    const double S4 = fma(-k.h, p3, S);
    const double I4 = fma(k.h, q3, I);
    const double bs4 = k.b * S4;

    const double muaD = mu * aD;
    const double m6 = k.h6 * muaD;  // mu kbar_s.D for s = 1, 4
    const double m3 = h3 * muaD;    // mu kbar_s.D for s = 2, 3
    double tI = 0.0;                 // sum_s I_s kbar_s.I
    double v4, v3, v2, v1, Y4I, Y3I, Y2I, Y1I;
    // stage 4: kbar4 = h/6 abar
    const double k4S = k.h6 * aS, k4I = k.h6 * aI;
    stage_adjoint(S4, I4, bs4, k4S, k4I, m6, k.lam, v4, Y4I, g, tI);
    // stage 3: kbar3 = h/3 abar + h Ybar4
    const double h3S = h3 * aS, h3I = h3 * aI;
    stage_adjoint(S3, I3, bs3, fma(k.hb, v4, h3S), fma(k.h, Y4I, h3I), m3, k.lam, v3, Y3I, g,
                  tI);
    // stage 2: kbar2 = h/3 abar + h/2 Ybar3
    stage_adjoint(S2, I2, bs2, fma(k.h2b, v3, h3S), fma(k.h2, Y3I, h3I), m3, k.lam, v2, Y2I, g,
                  tI);
    // stage 1: kbar1 = h/6 abar + h/2 Ybar2
    stage_adjoint(S, I, bs1, fma(k.h2b, v2, k4S), fma(k.h2, Y2I, k4I), m6, k.lam, v1, Y1I, g,
                  tI);

    // gamma: -sum I_s kbar_s.I;  mu: sum I_s (kbar_s.D - kbar_s.I)
    const double J = fma(2.0, I2 + I3, I + I4);
    g.gamma -= tI;
    g.mu = fma(k.h6 * aD, J, g.mu - tI);
    aS = fma(k.b, (v1 + v2) + (v3 + v4), aS);
    aI = aI + ((Y1I + Y2I) + (Y3I + Y4I));
}

// Steps replayed into registers at a time in the reverse sweep.
constexpr int kChunk = 8;
// Chunk length of the aligned sweep: when it divides both the steps per day
// and the checkpoint interval, every day start, segment start and interval
// start falls on a chunk start, so a chunk's steps are replayed and
// reversed with no test between them.
constexpr int kAlign = 10;
// Threads per block of k_backward (four wavefronts).
constexpr int kBwdBlock = 256;

__device__ __forceinline__ int seg_of(int n, int SS, int K)
{
    const int k = n / SS;
    return k > K - 1 ? K - 1 : k;
}

template <int KIND, int MODE>
__global__ void __launch_bounds__(kBwdBlock) k_backward(BwdArgs a)
{
    extern __shared__ double lds[];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int t = wave_tile_index();
    if (t >= a.n_tiles) return;
    double *ly = lds + (size_t)wave * a.lds_stride;
    double *lw = ly + a.lds_stride / 2;

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
    // workspace of this particle: slot k at base[k * PS]
    double *const ck_ws = a.ws + (size_t)(P.p_off + pc);    // checkpoint m: 3m .. 3m+2 (S, I, s)
    double *const in_ws = ck_ws + (size_t)(3 * a.n_ck_max) * PS;  // chunk c: 3c .. 3c+2
    double *const day_ws = in_ws + (size_t)(3 * ((a.s + kChunk - 1) / kChunk)) * PS;  // Dhat_i
    // the forward pass's results the reverse sweep needs besides the
    // checkpoints and Dhat: the day MXSE peaks on, and the loss
    double *const tail_ws = day_ws + (size_t)(a.max_days + 1) * PS;

    {
        // deceased counts: the last of the obs_series blocks of W+1 values
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
    const double I0 = th[(size_t)(K + 2) * ld];
    const double N = P.N;
    const double invN = 1.0 / N;
    const double h3 = (1.0 / (double)spd) / 3.0;
    StepConst<double> sc = step_const<double>(gamma, mu, spd);

    // ---------------------------------------------------- forward pass
    // The S-carrying form of the forward kernel's step, day by day: a
    // segment change and the rescale s = b S at the start of a day, the
    // checkpoint (S, I, s) before every s-th step, the cost and Dhat at the
    // end of a day.
    int imax = 0;
    if constexpr (MODE == kRevOnly) {
        imax = active ? (int)tail_ws[0] : 0;
        if (active && a.loss_out) a.loss_out[P.p_off + pl] = tail_ws[PS];
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
    if (active) day_ws[0] = y.D;
    {
        int kseg = 0;
        set_beta(sc, th[0], invN);
        int st = 0, next_ck = 0;
        double *cp = ck_ws;
        double *dp = day_ws;
        for (int day = 0; day < W; ++day) {
            if (kseg < K - 1 && st == (kseg + 1) * SS) {
                ++kseg;
                set_beta(sc, th[(size_t)kseg * ld], invN);
            }
            rescale(y, sc);
            for (int sd = 0; sd < spd;) {
                if (st == next_ck) {
                    if (active) {
                        cp[0] = y.S;
                        cp[PS] = y.I;
                        cp[2 * PS] = y.s;
                    }
                    cp += 3 * PS;
                    next_ck += a.s;
                }
                const int run = min(spd - sd, next_ck - st);
#pragma unroll 2
                for (int i = 0; i < run; ++i) rk4_step<double, false>(y, sc);
                sd += run;
                st += run;
            }
            const double prev = acc;
            cost_accum(KIND, acc, y.D, ly[day + 1], lw[day + 1], day + 1);
            if (KIND == SIRD_LOSS_MXSE && !(acc == prev)) imax = day + 1;
            dp += PS;
            if (active) *dp = y.D;
        }
    }
    const double L = cost_finish(KIND, acc, W);
    if (active && a.loss_out) a.loss_out[P.p_off + pl] = L;
    if constexpr (MODE == kFwdOnly) {
        if (active) {
            tail_ws[0] = (double)imax;
            tail_ws[PS] = L;
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

    double aS = 0.0, aI = 0.0;
    const double DW = active ? day_ws[(size_t)W * PS] : 0.0;
    double aD = cost_grad(KIND, W, W, DW, ly[W], lw[W], imax);
    Grad g{0.0, 0.0, 0.0};
    int kr = k_last;  // segment of the reverse position
    set_beta(sc, th[(size_t)kr * ld], invN);
    int seg_lo = kr * SS;  // first step of segment kr

    const int n_ck = (T + a.s - 1) / a.s;
    const bool aligned = spd % kAlign == 0 && a.s % kAlign == 0;
    // the checkpoint of the interval to reverse next, loaded one interval
    // ahead
    double cS, cI, cs_;
    {
        const double *cp = ck_ws + (size_t)(3 * (n_ck - 1)) * PS;
        cS = active ? cp[0] : 0.0;
        cI = active ? cp[PS] : 0.0;
        cs_ = active ? cp[2 * PS] : 0.0;
    }
    for (int m = n_ck - 1; m >= 0; --m) {
        const int n0 = m * a.s;
        const int n1 = (n0 + a.s < T) ? n0 + a.s : T;
        const double ckS = cS, ckI = cI, cks = cs_;
        if (m > 0) {
            const double *cp = ck_ws + (size_t)(3 * (m - 1)) * PS;
            cS = active ? cp[0] : 0.0;
            cI = active ? cp[PS] : 0.0;
            cs_ = active ? cp[2 * PS] : 0.0;
        }
        if (aligned) {
            // Aligned sweep: chunks of kAlign steps; the interval and every
            // chunk are whole (T, s and the day are multiples of kAlign), a
            // chunk lies in one segment and only its first step can start a
            // day.  The operations are those of the general sweep below, in
            // the same order, so the gradient is bitwise the same.
            const int nc = (n1 - n0) / kAlign;
            // pass 1: chunk start states 1 .. nc-2 to the workspace; the last
            // chunk's stays in registers
            double lastS = ckS, lastI = ckI, lasts = cks;
            if (nc > 1) {
                SirdState<double> yr;
                yr.S = ckS;
                yr.I = ckI;
                yr.s = cks;
                yr.Rr = yr.D = 0.0;
                yr.eS = yr.eI = yr.eR = yr.eD = 0.0;
                int kf = seg_of(n0, SS, K);
                StepConst<double> sf = sc;
                set_beta(sf, th[(size_t)kf * ld], invN);
                double *ip = in_ws + 3 * PS;
                for (int c = 0; c < nc - 1; ++c) {
                    const int st = n0 + c * kAlign;
                    if (st % spd == 0) {
                        if (kf < K - 1 && st == (kf + 1) * SS) {
                            ++kf;
                            set_beta(sf, th[(size_t)kf * ld], invN);
                        }
                        rescale(yr, sf);
                    }
#pragma unroll
                    for (int i = 0; i < kAlign; ++i) rk4_step<double, false>(yr, sf);
                    if (c + 1 < nc - 1) {
                        if (active) {
                            ip[0] = yr.S;
                            ip[PS] = yr.I;
                            ip[2 * PS] = yr.s;
                        }
                        ip += 3 * PS;
                    }
                }
                lastS = yr.S;
                lastI = yr.I;
                lasts = yr.s;
            }
            // pass 2: chunks last to first, the next one's start state and
            // day-start Dhat loaded before the current one is walked
            double nS, nI, ns, nD;
            auto load_chunk = [&](int c) {
                if (c == 0) {
                    nS = ckS;
                    nI = ckI;
                    ns = cks;
                } else if (c == nc - 1) {
                    nS = lastS;
                    nI = lastI;
                    ns = lasts;
                } else {
                    const double *sp = in_ws + (size_t)(3 * c) * PS;
                    nS = active ? sp[0] : 0.0;
                    nI = active ? sp[PS] : 0.0;
                    ns = active ? sp[2 * PS] : 0.0;
                }
                const int cs = n0 + c * kAlign;
                nD = (active && cs % spd == 0) ? day_ws[(size_t)(cs / spd) * PS] : 0.0;
            };
            load_chunk(nc - 1);
            for (int c = nc - 1; c >= 0; --c) {
                const int cs = n0 + c * kAlign;
                SirdState<double> yr;
                yr.S = nS;
                yr.I = nI;
                yr.s = ns;
                yr.Rr = yr.D = 0.0;
                yr.eS = yr.eI = yr.eR = yr.eD = 0.0;
                const double Dd = nD;
                if (c > 0) load_chunk(c - 1);
                // the chunk is in the reverse's segment kr
                const bool day_start = cs % spd == 0;
                if (day_start) rescale(yr, sc);
                double Sa[kAlign], Ia[kAlign];
#pragma unroll
                for (int j = 0; j < kAlign; ++j) {
                    Sa[j] = yr.S;
                    Ia[j] = yr.I;
                    rk4_step<double, false>(yr, sc);
                }
#pragma unroll
                for (int j = kAlign - 1; j >= 0; --j)
                    rk4_adjoint_step(Sa[j], Ia[j], aS, aI, aD, sc, mu, h3, g);
                if (day_start) {
                    const int i = cs / spd;
                    aD += cost_grad(KIND, i, W, Dd, ly[i], lw[i], imax);
                    if (cs == seg_lo && kr > 0) {
                        // the chunk's first step opened segment kr
                        if (active) gout[(size_t)kr * ld] = (g.beta * invN) * gl;
                        g.beta = 0.0;
                        --kr;
                        seg_lo -= SS;
                        set_beta(sc, th[(size_t)kr * ld], invN);
                    }
                }
            }
            continue;
        }
        const int n_chunks = (n1 - n0 + kChunk - 1) / kChunk;
        // pass 1: replay the interval from its checkpoint with exactly the
        // forward pass's operations up to the start of its last chunk,
        // storing the state before the first step of every chunk but the
        // first (the checkpoint) and the last (kept in registers)
        double lastS = ckS, lastI = ckI, lasts = cks;
        if (n_chunks > 1) {
            SirdState<double> yr;
            yr.S = ckS;
            yr.I = ckI;
            yr.s = cks;
            yr.Rr = yr.D = 0.0;
            yr.eS = yr.eI = yr.eR = yr.eD = 0.0;
            int kf = seg_of(n0, SS, K);
            StepConst<double> sf = sc;
            set_beta(sf, th[(size_t)kf * ld], invN);
            const int stop = n0 + (n_chunks - 1) * kChunk;
            int st = n0, sd = n0 % spd, next_store = n0 + kChunk;
            double *ip = in_ws + 3 * PS;
            while (st < stop) {
                if (sd == 0) {
                    if (kf < K - 1 && st == (kf + 1) * SS) {
                        ++kf;
                        set_beta(sf, th[(size_t)kf * ld], invN);
                    }
                    rescale(yr, sf);
                }
                const int run = min(spd - sd, next_store - st);
#pragma unroll 2
                for (int i = 0; i < run; ++i) rk4_step<double, false>(yr, sf);
                st += run;
                sd += run;
                if (sd == spd) sd = 0;
                if (st == next_store && st < stop) {
                    if (active) {
                        ip[0] = yr.S;
                        ip[PS] = yr.I;
                        ip[2 * PS] = yr.s;
                    }
                    ip += 3 * PS;
                    next_store += kChunk;
                }
            }
            lastS = yr.S;
            lastI = yr.I;
            lasts = yr.s;
        }
        // pass 2: chunks last to first: replay kChunk steps into registers,
        // then walk them backwards.  The next chunk's start state, its day
        // starts (a mask) and their Dhat are loaded before the current
        // chunk is walked, so with one wavefront per SIMD their latency is
        // hidden.
        // With at least kChunk steps per day a chunk holds at most one day
        // start, kept in (nD1, nday1); else every day start j of the chunk
        // has its own (nD[j], nday[j]).
        const bool sparse = spd >= kChunk;
        double nS, nI, ns, nD[kChunk], nD1;
        int nday[kChunk], nday1;
        unsigned nmask;
        // chunk c starts at step cs = n0 + c kChunk = q spd + ph
        auto load_chunk = [&](int c, int cs, int q, int ph) {
            if (c == 0) {
                nS = ckS;
                nI = ckI;
                ns = cks;
            } else if (c == n_chunks - 1) {
                nS = lastS;
                nI = lastI;
                ns = lasts;
            } else {
                const double *sp = in_ws + (size_t)(3 * c) * PS;
                nS = active ? sp[0] : 0.0;
                nI = active ? sp[PS] : 0.0;
                ns = active ? sp[2 * PS] : 0.0;
            }
            const int len = (n1 - cs < kChunk) ? n1 - cs : kChunk;
            int jd = ph == 0 ? 0 : spd - ph;  // first day start in the chunk
            int d = ph == 0 ? q : q + 1;      // its day
            nmask = 0u;
            nD1 = 0.0;
            nday1 = d;
            if (sparse) {
                if (jd < len) {
                    nmask = 1u << jd;
                    if (active) nD1 = day_ws[(size_t)d * PS];
                }
                return;
            }
#pragma unroll
            for (int j = 0; j < kChunk; ++j) {
                nD[j] = 0.0;
                nday[j] = 0;
                if (j == jd && j < len) {
                    nmask |= 1u << j;
                    nday[j] = d;
                    if (active) nD[j] = day_ws[(size_t)d * PS];
                    ++d;
                    jd += spd;
                }
            }
        };
        int cs = n0 + (n_chunks - 1) * kChunk;
        int q = cs / spd, ph = cs - q * spd;
        load_chunk(n_chunks - 1, cs, q, ph);
        for (int c = n_chunks - 1; c >= 0; --c) {
            const int len = (n1 - cs < kChunk) ? n1 - cs : kChunk;
            SirdState<double> yr;
            yr.S = nS;
            yr.I = nI;
            yr.s = ns;
            yr.Rr = yr.D = 0.0;
            yr.eS = yr.eI = yr.eR = yr.eD = 0.0;
            double Dd[kChunk];
            int day[kChunk];
            if (!sparse) {
#pragma unroll
                for (int j = 0; j < kChunk; ++j) {
                    Dd[j] = nD[j];
                    day[j] = nday[j];
                }
            }
            const double Dd1 = nD1;
            const int day1 = nday1;
            const unsigned dmask = nmask;
            // the previous chunk's position
            const int pcs = cs - kChunk;
            int pq = q, pph = ph - kChunk;
            while (pph < 0) {
                pph += spd;
                --pq;
            }
            if (c > 0) load_chunk(c - 1, pcs, pq, pph);
            // segment of the chunk's first step: kr, or an earlier one when
            // a segment starts inside the chunk
            int kf = kr, lo = seg_lo;
            while (cs < lo) {
                --kf;
                lo -= SS;
            }
            StepConst<double> sf = sc;  // the reverse's segment: no reload
            if (kf != kr) set_beta(sf, th[(size_t)kf * ld], invN);
            int next_seg = (kf < K - 1) ? (kf + 1) * SS : T + 1;
            // replay, then walk back; a full chunk (every chunk but an
            // interval's last one, when the interval is not a multiple of
            // kChunk) has no per-step length test
            auto walk = [&](auto full) {
                constexpr bool FULL = decltype(full)::value;
                double Sa[kChunk], Ia[kChunk];
#pragma unroll
                for (int j = 0; j < kChunk; ++j) {
                    Sa[j] = Ia[j] = 0.0;
                    if (FULL || j < len) {
                        if (dmask & (1u << j)) {
                            if (cs + j == next_seg) {
                                ++kf;
                                next_seg = (kf < K - 1) ? next_seg + SS : T + 1;
                                set_beta(sf, th[(size_t)kf * ld], invN);
                            }
                            rescale(yr, sf);
                        }
                        Sa[j] = yr.S;
                        Ia[j] = yr.I;
                        rk4_step<double, false>(yr, sf);
                    }
                }
#pragma unroll
                for (int j = kChunk - 1; j >= 0; --j) {
                    if (FULL || j < len) {
                        rk4_adjoint_step(Sa[j], Ia[j], aS, aI, aD, sc, mu, h3, g);
                        if (dmask & (1u << j)) {
                            const int i = sparse ? day1 : day[j];
                            const double Dj = sparse ? Dd1 : Dd[j];
                            aD += cost_grad(KIND, i, W, Dj, ly[i], lw[i], imax);
                            if (cs + j == seg_lo && kr > 0) {
                                // the step just reversed opened segment kr
                                if (active) gout[(size_t)kr * ld] = (g.beta * invN) * gl;
                                g.beta = 0.0;
                                --kr;
                                seg_lo -= SS;
                                set_beta(sc, th[(size_t)kr * ld], invN);
                            }
                        }
                    }
                }
            };
            if (len == kChunk)
                walk(std::true_type{});
            else
                walk(std::false_type{});
            cs = pcs;
            q = pq;
            ph = pph;
        }
    }
    if (active) {
        gout[(size_t)kr * ld] = (g.beta * invN) * gl;
        gout[(size_t)K * ld] = g.gamma * gl;
        gout[(size_t)(K + 1) * ld] = g.mu * gl;
        gout[(size_t)(K + 2) * ld] = (aI - aS) * gl;
    }
}

// The checkpoint interval: as given, else ceil(sqrt(T)) rounded up to a
// multiple of kAlign (so that problems whose steps per day are a multiple
// of kAlign take the aligned sweep).
static int resolve_interval(const sird_batch *b, int ckpt_interval)
{
    if (ckpt_interval > 0) return ckpt_interval;
    const int s = (int)std::ceil(std::sqrt((double)b->max_steps));
    return (s + kAlign - 1) / kAlign * kAlign;
}

// Workspace slots per particle: 3 per checkpoint (S, I, s), 3 per chunk of
// one replayed interval (the first and last chunks' slots go unused: the
// first starts at the checkpoint, the last one's start stays in registers),
// Dhat of every day, the day MXSE peaks on and the loss.
static size_t ws_slots(const sird_batch *b, int s)
{
    const int64_t n_ck = (b->max_steps + s - 1) / s;
    const int64_t n_chunk = ((int64_t)s + kChunk - 1) / kChunk;
    return (size_t)(3 * n_ck + 3 * n_chunk + b->max_days + 1 + 2);
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
    return ws_slots(b, resolve_interval(b, ckpt_interval)) * (size_t)b->total_particles *
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
    if (ckpt_interval < 0) return fail(SIRD_EINVAL, w + ": ckpt_interval < 0");
    if (batch->obs_len < 1) return fail(SIRD_EINVAL, w + ": batch planned without obs");
    const int s = resolve_interval(batch, ckpt_interval);
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
    a->s = s;
    a->n_ck_max = (int)((batch->max_steps + s - 1) / s);
    a->max_days = batch->max_days;
    a->lds_stride = 2 * (batch->max_days + 1);
    *lds = (size_t)(kBwdBlock / kWave) * a->lds_stride * sizeof(double);
    if (*lds > 65536) return fail(SIRD_EINVAL, w + ": window too long for LDS");
    *grid = tile_blocks(batch->n_tiles);
    return SIRD_OK;
}

static int adjoint_launch(int mode, int loss_kind, int grid, size_t lds, hipStream_t stream,
                          const BwdArgs &a, const char *who)
{
    if (grid == 0) return SIRD_OK;
    if (mode == kFwdOnly)
        launch_backward<kFwdOnly>(loss_kind, grid, kBwdBlock, lds, stream, a);
    else if (mode == kRevOnly)
        launch_backward<kRevOnly>(loss_kind, grid, kBwdBlock, lds, stream, a);
    else
        launch_backward<kBoth>(loss_kind, grid, kBwdBlock, lds, stream, a);
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
    if (ckpt_interval < 0) return 0;
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
