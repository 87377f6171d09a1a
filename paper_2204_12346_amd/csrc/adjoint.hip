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
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>

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
    int kind;
    int obs_series;  // 1 or 3; the deceased counts are the last series
    int s;          // checkpoint interval in steps
    int n_ck_max;   // checkpoints per particle
    int lds_stride;
};

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
    double beta;   // of the current segment
    double gamma;
    double mu;
};

// One stage of the reverse step: Ybar = J(Y_s)^T kbar and the parameter
// contributions; mkD = mu * kbar_s.D.
__device__ __forceinline__ void stage_adjoint(double Ss, double Is, double bs, double kS,
                                              double kI, double mkD, double lam, double b,
                                              double invN, double &YS, double &YI, Grad &g,
                                              double &tI)
{
    const double u = kI - kS;
    YS = (b * Is) * u;
    YI = fma(bs, u, fma(-lam, kI, mkD));
    g.beta = fma((Ss * invN) * Is, u, g.beta);
    tI = fma(Is, kI, tI);
}

// One reverse step: (aS, aI) <- a_n from a_{n+1}; aD unchanged.
__device__ __forceinline__ void rk4_adjoint_step(double S, double I, double &aS, double &aI,
                                                 double aD, const StepConst<double> &k,
                                                 double mu, double invN, double h3, Grad &g)
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
    double Y4S, Y4I, Y3S, Y3I, Y2S, Y2I, Y1S, Y1I;
    // stage 4: kbar4 = h/6 abar
    const double k4S = k.h6 * aS, k4I = k.h6 * aI;
    stage_adjoint(S4, I4, bs4, k4S, k4I, m6, k.lam, k.b, invN, Y4S, Y4I, g, tI);
    // stage 3: kbar3 = h/3 abar + h Ybar4
    const double h3S = h3 * aS, h3I = h3 * aI;
    stage_adjoint(S3, I3, bs3, fma(k.h, Y4S, h3S), fma(k.h, Y4I, h3I), m3, k.lam, k.b, invN,
                  Y3S, Y3I, g, tI);
    // stage 2: kbar2 = h/3 abar + h/2 Ybar3
    stage_adjoint(S2, I2, bs2, fma(k.h2, Y3S, h3S), fma(k.h2, Y3I, h3I), m3, k.lam, k.b,
                  invN, Y2S, Y2I, g, tI);
    // stage 1: kbar1 = h/6 abar + h/2 Ybar2
    stage_adjoint(S, I, bs1, fma(k.h2, Y2S, k4S), fma(k.h2, Y2I, k4I), m6, k.lam, k.b, invN,
                  Y1S, Y1I, g, tI);

    // gamma: -sum I_s kbar_s.I;  mu: sum I_s (kbar_s.D - kbar_s.I)
    const double J = fma(2.0, I2 + I3, I + I4);
    g.gamma -= tI;
    g.mu = fma(k.h6 * aD, J, g.mu - tI);
    aS = aS + ((Y1S + Y2S) + (Y3S + Y4S));
    aI = aI + ((Y1I + Y2I) + (Y3I + Y4I));
    (void)q3;
}

// Steps replayed into registers at a time in the reverse sweep.
constexpr int kChunk = 8;

__device__ __forceinline__ int seg_of(int n, int SS, int K)
{
    const int k = n / SS;
    return k > K - 1 ? K - 1 : k;
}

__global__ void __launch_bounds__(256) k_backward(BwdArgs a)
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
    const long T = (long)W * spd;
    // steps per segment (a segment longer than the window is the window)
    const int SS = (int)min((long)P.seg_days * spd, T + 1);
    const int pl = tl.p0 + lane;
    const bool active = pl < n;
    const int pc = active ? pl : n - 1;
    const size_t ld = (size_t)n;
    const double *th = a.theta + P.theta_off + pc;
    const size_t PS = (size_t)a.P;
    double *wsp = a.ws + (size_t)(P.p_off + pc);
    const int ck_base = 0;  // checkpoint m: slots 3m (S), 3m+1 (I), 3m+2 (s)
    const int in_base = 3 * a.n_ck_max;  // chunk c of an interval: 3c .. 3c+2
    const int day_base = in_base + 3 * ((a.s + kChunk - 1) / kChunk);

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
    SirdState<double> y;
    y.S = N - I0 - P.R0 - P.D0;
    y.I = I0;
    y.Rr = P.R0;
    y.D = P.D0;
    y.s = 0.0;
    y.eS = y.eI = y.eR = y.eD = 0.0;
    double acc = 0.0;
    int imax = 0;
    cost_accum(a.kind, acc, y.D, ly[0], lw[0], 0);
    if (active) wsp[(size_t)day_base * PS] = y.D;
    {
        // the S-carrying form of the forward kernel's step: set_beta at
        // a segment start, rescale at a day start, then the step
        int k = 0;
        long next_seg = (K > 1) ? (long)SS : T + 1;
        set_beta(sc, th[0], invN);
        long next_ck = 0;
        int m = 0;
        int sd = 0, day = 0;
        for (long st = 0; st < T; ++st) {
            if (st == next_seg) {
                ++k;
                next_seg = (k < K - 1) ? next_seg + SS : T + 1;
                set_beta(sc, th[(size_t)k * ld], invN);
            }
            if (sd == 0) rescale(y, sc);
            if (st == next_ck) {
                if (active) {
                    wsp[(size_t)(ck_base + 3 * m) * PS] = y.S;
                    wsp[(size_t)(ck_base + 3 * m + 1) * PS] = y.I;
                    wsp[(size_t)(ck_base + 3 * m + 2) * PS] = y.s;
                }
                ++m;
                next_ck += a.s;
            }
            rk4_step<double, false>(y, sc);
            if (++sd == spd) {
                sd = 0;
                ++day;
                const double prev = acc;
                cost_accum(a.kind, acc, y.D, ly[day], lw[day], day);
                if (a.kind == SIRD_LOSS_MXSE && !(acc == prev)) imax = day;
                if (active) wsp[(size_t)(day_base + day) * PS] = y.D;
            }
        }
    }
    const double L = cost_finish(a.kind, acc, W);
    if (active && a.loss_out) a.loss_out[P.p_off + pl] = L;

    // ---------------------------------------------------- reverse sweep
    const double gl = a.grad_loss ? a.grad_loss[P.p_off + pc] : 1.0;
    double *gout = a.grad + P.theta_off + pc;
    const int k_last = seg_of(T - 1, SS, K);
    for (int k = k_last + 1; k < K; ++k)
        if (active) gout[(size_t)k * ld] = 0.0;  // segments past the window end

    double aS = 0.0, aI = 0.0;
    const double DW = active ? wsp[(size_t)(day_base + W) * PS] : 0.0;
    double aD = cost_grad(a.kind, W, W, DW, ly[W], lw[W], imax);
    Grad g{0.0, 0.0, 0.0};
    int kr = k_last;  // segment of the reverse position
    set_beta(sc, th[(size_t)kr * ld], invN);
    int seg_lo = kr * SS;  // first step of segment kr

    const int Ti = (int)T;  // at most 2^30 (checked on the host)
    const int n_ck = (Ti + a.s - 1) / a.s;
    for (int m = n_ck - 1; m >= 0; --m) {
        const int n0 = m * a.s;
        const int n1 = (n0 + a.s < Ti) ? n0 + a.s : Ti;
        // pass 1: replay the interval from its checkpoint with exactly the
        // forward pass's operations up to the start of its last chunk,
        // storing the state before the first step of every chunk but the
        // first (which is the checkpoint)
        const int n_chunks = (n1 - n0 + kChunk - 1) / kChunk;
        if (n_chunks > 1) {
            SirdState<double> yr;
            yr.S = active ? wsp[(size_t)(ck_base + 3 * m) * PS] : 0.0;
            yr.I = active ? wsp[(size_t)(ck_base + 3 * m + 1) * PS] : 0.0;
            yr.s = active ? wsp[(size_t)(ck_base + 3 * m + 2) * PS] : 0.0;
            yr.Rr = yr.D = 0.0;
            yr.eS = yr.eI = yr.eR = yr.eD = 0.0;
            int kf = seg_of(n0, SS, K);
            StepConst<double> sf = sc;
            set_beta(sf, th[(size_t)kf * ld], invN);
            int next_seg = (kf < K - 1) ? (kf + 1) * SS : Ti + 1;
            int sd = n0 % spd;
            for (int c = 1; c < n_chunks; ++c) {
                for (int j = 0; j < kChunk; ++j) {
                    const int st = n0 + (c - 1) * kChunk + j;
                    if (st == next_seg) {
                        ++kf;
                        next_seg = (kf < K - 1) ? next_seg + SS : Ti + 1;
                        set_beta(sf, th[(size_t)kf * ld], invN);
                    }
                    if (sd == 0) rescale(yr, sf);
                    rk4_step<double, false>(yr, sf);
                    if (++sd == spd) sd = 0;
                }
                if (active) {
                    wsp[(size_t)(in_base + 3 * c) * PS] = yr.S;
                    wsp[(size_t)(in_base + 3 * c + 1) * PS] = yr.I;
                    wsp[(size_t)(in_base + 3 * c + 2) * PS] = yr.s;
                }
            }
        }
        // pass 2: chunks last to first: replay kChunk steps into registers,
        // then walk them backwards.  The next chunk's start state, its day
        // boundaries and their Dhat are loaded before the current chunk is
        // walked, so with one wavefront per SIMD their latency is hidden.
        double nS, nI, ns, nD[kChunk];
        int nday[kChunk], nph;
        auto load_chunk = [&](int c) {
            // chunk 0 starts at the interval's checkpoint
            const int slot = c == 0 ? ck_base + 3 * m : in_base + 3 * c;
            nS = active ? wsp[(size_t)slot * PS] : 0.0;
            nI = active ? wsp[(size_t)(slot + 1) * PS] : 0.0;
            ns = active ? wsp[(size_t)(slot + 2) * PS] : 0.0;
            const int cs = n0 + c * kChunk;
            const int q = cs / spd;
            nph = cs - q * spd;  // step of the day at cs
            int ph = nph, d = nph == 0 ? q : q + 1;
#pragma unroll
            for (int j = 0; j < kChunk; ++j) {
                nday[j] = -1;
                nD[j] = 0.0;
                if (cs + j < n1 && ph == 0) {
                    nday[j] = d;
                    if (active) nD[j] = wsp[(size_t)(day_base + d) * PS];
                    ++d;
                }
                ph = (ph + 1 == spd) ? 0 : ph + 1;
            }
        };
        load_chunk(n_chunks - 1);
        for (int c = n_chunks - 1; c >= 0; --c) {
            const int cs = n0 + c * kChunk;
            const int len = (n1 - cs < kChunk) ? n1 - cs : kChunk;
            SirdState<double> yr;
            yr.S = nS;
            yr.I = nI;
            yr.s = ns;
            yr.Rr = yr.D = 0.0;
            yr.eS = yr.eI = yr.eR = yr.eD = 0.0;
            double Dd[kChunk];
            int day[kChunk];
#pragma unroll
            for (int j = 0; j < kChunk; ++j) {
                Dd[j] = nD[j];
                day[j] = nday[j];
            }
            int sd = nph;
            if (c > 0) load_chunk(c - 1);
            int kf = seg_of(cs, SS, K);
            StepConst<double> sf = sc;  // the reverse's segment: no reload
            if (kf != kr) set_beta(sf, th[(size_t)kf * ld], invN);
            int next_seg = (kf < K - 1) ? (kf + 1) * SS : Ti + 1;
            double Sa[kChunk], Ia[kChunk];
#pragma unroll
            for (int j = 0; j < kChunk; ++j) {
                Sa[j] = Ia[j] = 0.0;
                if (j < len) {
                    if (cs + j == next_seg) {
                        ++kf;
                        next_seg = (kf < K - 1) ? next_seg + SS : Ti + 1;
                        set_beta(sf, th[(size_t)kf * ld], invN);
                    }
                    if (sd == 0) rescale(yr, sf);
                    Sa[j] = yr.S;
                    Ia[j] = yr.I;
                    rk4_step<double, false>(yr, sf);
                    if (++sd == spd) sd = 0;
                }
            }
#pragma unroll
            for (int j = kChunk - 1; j >= 0; --j) {
                if (j < len) {
                    if (cs + j < seg_lo) {
                        if (active) gout[(size_t)kr * ld] = g.beta * gl;
                        g.beta = 0.0;
                        --kr;
                        seg_lo = kr * SS;
                        set_beta(sc, th[(size_t)kr * ld], invN);
                    }
                    rk4_adjoint_step(Sa[j], Ia[j], aS, aI, aD, sc, mu, invN, h3, g);
                    if (day[j] >= 0) {
                        const int i = day[j];
                        aD += cost_grad(a.kind, i, W, Dd[j], ly[i], lw[i], imax);
                    }
                }
            }
        }
    }
    if (active) {
        gout[(size_t)kr * ld] = g.beta * gl;
        gout[(size_t)K * ld] = g.gamma * gl;
        gout[(size_t)(K + 1) * ld] = g.mu * gl;
        gout[(size_t)(K + 2) * ld] = (aI - aS) * gl;
    }
}

static int resolve_interval(const sird_batch *b, int ckpt_interval)
{
    if (ckpt_interval > 0) return ckpt_interval;
    int s = (int)std::ceil(std::sqrt((double)b->max_steps));
    return s < 1 ? 1 : s;
}

// Workspace slots per particle: 3 per checkpoint (S, I, s), 3 per chunk of
// one replayed interval (the first chunk's slots go unused: it starts at
// the checkpoint), and Dhat of every day.
static size_t ws_slots(const sird_batch *b, int s)
{
    const int64_t n_ck = (b->max_steps + s - 1) / s;
    const int64_t n_chunk = ((int64_t)s + kChunk - 1) / kChunk;
    return (size_t)(3 * n_ck + 3 * n_chunk + b->max_days + 1);
}

}  // namespace sird

using namespace sird;

extern "C" size_t sird_loss_backward_workspace(const sird_batch *batch, int ckpt_interval)
{
    if (check_batch(batch, "sird_loss_backward_workspace")) return 0;
    if (ckpt_interval < 0) return 0;
    const int s = resolve_interval(batch, ckpt_interval);
    return ws_slots(batch, s) * (size_t)batch->total_particles * sizeof(double);
}

extern "C" int sird_loss_backward(const sird_batch *batch, const double *theta,
                                  const double *obs, int loss_kind, const double *grad_loss,
                                  double *grad_theta, double *loss_out, int ckpt_interval,
                                  void *workspace, size_t ws_bytes, void *stream)
{
    int st = check_batch(batch, "sird_loss_backward");
    if (st) return st;
    if (!theta || !obs || !grad_theta || !workspace)
        return fail(SIRD_EINVAL, "sird_loss_backward: NULL array");
    if (batch->dtype != SIRD_F64)
        return fail(SIRD_EINVAL, "sird_loss_backward: only SIRD_F64 batches are supported");
    if (loss_kind < SIRD_LOSS_SSRE || loss_kind > SIRD_LOSS_MAPE)
        return fail(SIRD_EINVAL, "sird_loss_backward: loss_kind must be a deceased-count cost");
    if (batch->models != 1 << SIRD_MODEL_RK4_SEGMENTS)
        return fail(SIRD_EINVAL, "sird_loss_backward: only the RK4 segment model is supported");
    if (ckpt_interval < 0) return fail(SIRD_EINVAL, "sird_loss_backward: ckpt_interval < 0");
    if (batch->obs_len < 1)
        return fail(SIRD_EINVAL, "sird_loss_backward: batch planned without obs");
    if (((uintptr_t)workspace & 255) != 0)
        return fail(SIRD_EINVAL, "sird_loss_backward: workspace not 256-byte aligned");
    const int s = resolve_interval(batch, ckpt_interval);
    const size_t need = ws_slots(batch, s) * (size_t)batch->total_particles * sizeof(double);
    if (ws_bytes < need) return fail(SIRD_ENOSPACE, "sird_loss_backward: workspace too small");
    BwdArgs a{};
    a.probs = batch->probs;
    a.tiles = batch->tiles;
    a.theta = theta;
    a.obs = obs;
    a.grad_loss = grad_loss;
    a.grad = grad_theta;
    a.loss_out = loss_out;
    a.ws = (double *)workspace;
    a.P = batch->total_particles;
    a.n_tiles = batch->n_tiles;
    a.kind = loss_kind;
    a.obs_series = batch->obs_series;
    a.s = s;
    a.n_ck_max = (int)((batch->max_steps + s - 1) / s);
    a.lds_stride = 2 * (batch->max_days + 1);
    const int block = 256;
    const size_t lds = (size_t)(block / kWave) * a.lds_stride * sizeof(double);
    if (lds > 65536) return fail(SIRD_EINVAL, "sird_loss_backward: window too long for LDS");
    const int grid = tile_blocks(batch->n_tiles);
    if (grid == 0) return SIRD_OK;
    hipLaunchKernelGGL(k_backward, dim3(grid), dim3(block), lds, (hipStream_t)stream, a);
    return hip_status(hipGetLastError(), "sird_loss_backward");
}
