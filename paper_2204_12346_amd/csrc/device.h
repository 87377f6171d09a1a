// Device-side building blocks of the gfx950 SIRD library: the RK4 step of
// eq. (SIRD), Philox4x64-10, wavefront helpers and the per-day cost
// accumulation of Sec. 3.1.
//
// Everything here is wave64 (CDNA4).  Control flow that depends on the
// problem (days, steps, segments) is uniform across a wavefront because a
// wavefront integrates 64 particles of one problem.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/sird.h"

namespace sird {

constexpr int kWave = 64;

// ---------------------------------------------------------------- RK4 step
// State (S, I, R, D) as in eq. (SIRD).  With b = beta/N the infection term
// is p = b S I and the right-hand side is (-p, p - lam I, gamma I, mu I),
// lam = gamma + mu.  Classical RK4 with stages Y1 = y, Y2 = y + h/2 k1,
// Y3 = y + h/2 k2, Y4 = y + h k3 and y+ = y + h/6 (k1 + 2k2 + 2k3 + k4).
// Only S and I feed back, so the update needs two sums,
//     P = p1 + 2p2 + 2p3 + p4,   J = I1 + 2I2 + 2I3 + I4,
// with S+ = S - h/6 P, I+ = I + h/6 (P - lam J), R+ = R + h/6 gamma J,
// D+ = D + h/6 mu J.
// The stages use the scaled susceptible s = b S, so p_s = s_s I_s costs one
// multiply, and s+ = s - b h/6 P.  With WITH_S the step also carries S
// (reset s = b S at the start of every day); without it s is the state and
// S = s/b is formed only where beta changes, which saves one FMA per step.
// In double without S and R: 22 VALU operations per step (3 mul, 3 add,
// 16 fma, 38 flops); S and R cost one FMA each.
template <typename R>
struct StepConst {
    R b;      // beta / N of the current segment
    R lam;    // gamma + mu
    R h;      // step
    R h2;     // h / 2
    R h6;     // h / 6
    R h6lam;  // h/6 * lam
    R h6mu;   // h/6 * mu
    R h6g;    // h/6 * gamma
    R hb;     // b h
    R h2b;    // b h / 2
    R h6b;    // b h / 6
    R h2lam;  // h/2 * lam
    R hlam;   // h * lam
};

// The state of one particle.  In float, S, I, R and D carry the running
// compensation of Kahan's summation (W. Kahan, "Further remarks on reducing
// truncation errors", CACM 1965): a step's increments are small next to the
// state (S is close to N early in an epidemic), and without compensation
// their rounding accumulates to ~1e-5 over 1800 steps.  In double the
// compensation fields stay zero and are never touched.
template <typename R>
struct SirdState {
    R S, I, Rr, D;
    R s;  // b S, the stages' scaled susceptible
    R eS, eI, eR, eD;
};

template <typename R>
__device__ __forceinline__ void kahan_add(R &s, R &e, R inc)
{
    const R y = inc - e;
    const R t = s + y;
    e = (t - s) - y;
    s = t;
}

// Compensated value of a state component, in double.
template <typename R>
__device__ __forceinline__ double state_value(R s, R e)
{
    return (double)s - (double)e;
}

// New segment: b = beta/N and the step constants that depend on it.  b is
// formed as beta times 1/N (1/N is taken once per particle), which saves a
// division per segment at one more rounding.
template <typename R>
__device__ __forceinline__ void set_beta(StepConst<R> &k, double beta, double invN)
{
    const double b = beta * invN;
    k.b = (R)b;
    k.hb = (R)((double)k.h * b);
    k.h2b = (R)((double)k.h2 * b);
    k.h6b = (R)((double)k.h6 * b);
}

// Start of a day (and of a segment): s = b S.
template <typename R>
__device__ __forceinline__ void rescale(SirdState<R> &y, const StepConst<R> &k)
{
    y.s = k.b * y.S;
}

// End of a segment integrated without S: S = s/b (S stays as it was when
// beta = 0, since then s = 0 and S does not change).
template <typename R>
__device__ __forceinline__ void unscale(SirdState<R> &y, const StepConst<R> &k)
{
    if (k.b != R(0)) y.S = y.s / k.b;
}

// Returns J = I1 + 2 I2 + 2 I3 + I4 (D+ - D = h/6 mu J), which callers that
// only integrate ignore.
template <typename R, bool WITH_R, bool WITH_S = true>
__device__ __forceinline__ R rk4_step(SirdState<R> &y, const StepConst<R> &k)
{
    // Stage I_{k+1} = I + c h (p_k - lam I_k) is formed as
    // fma(c h, p_k, I - c h lam I_k): the second term does not wait for
    // p_k, which takes three operations off the dependent chain of a step.
    const R s = y.s, I = y.I;
    const R p1 = s * I;
    const R c1 = fma(-k.h2lam, I, I);
    const R s2 = fma(-k.h2b, p1, s);
    const R I2 = fma(k.h2, p1, c1);

    const R p2 = s2 * I2;
    const R c2 = fma(-k.h2lam, I2, I);
    const R s3 = fma(-k.h2b, p2, s);
    const R I3 = fma(k.h2, p2, c2);

    const R p3 = s3 * I3;
    const R c3 = fma(-k.hlam, I3, I);
    const R s4 = fma(-k.hb, p3, s);
    const R I4 = fma(k.h, p3, c3);

    // p4 = s4 I4 is used only in P: formed inside it, p1 + p4 = fma(s4, I4, p1)
    const R P = fma(R(2), p2 + p3, fma(s4, I4, p1));
    const R J = fma(R(2), I2 + I3, I + I4);
    y.s = fma(-k.h6b, P, s);
    if constexpr (sizeof(R) == 8) {
        if (WITH_S) y.S = fma(-k.h6, P, y.S);
        y.I = fma(k.h6, P, fma(-k.h6lam, J, I));
        if (WITH_R) y.Rr = fma(k.h6g, J, y.Rr);
        y.D = fma(k.h6mu, J, y.D);
    } else {
        kahan_add(y.S, y.eS, -(k.h6 * P));
        kahan_add(y.I, y.eI, fma(k.h6, P, -(k.h6lam * J)));
        if (WITH_R) kahan_add(y.Rr, y.eR, k.h6g * J);
        kahan_add(y.D, y.eD, k.h6mu * J);
    }
    return J;
}

template <typename R>
__device__ __forceinline__ StepConst<R> step_const(double gamma, double mu, int spd)
{
    const double h = 1.0 / (double)spd;
    const double h6 = h / 6.0;
    StepConst<R> k;
    k.lam = (R)(gamma + mu);
    k.h = (R)h;
    k.h2 = (R)(0.5 * h);
    k.h6 = (R)h6;
    k.h6lam = (R)(h6 * (gamma + mu));
    k.h6mu = (R)(h6 * mu);
    k.h6g = (R)(h6 * gamma);
    k.h2lam = (R)(0.5 * h * (gamma + mu));
    k.hlam = (R)(h * (gamma + mu));
    k.b = k.hb = k.h2b = k.h6b = R(0);
    return k;
}

// ------------------------------------------------ Euler with the ramp of eq. (beta)
// The paper's own scheme (Sec. 3.1, 3.3): forward Euler, beta evaluated at
// the start of every step from the ramp beta1 -> beta2 over [t1, t2) (t in
// days from the window start), y+ = y + h f(t, y).  Per particle the
// constants beta1/N, beta2/N and the slope/N are formed once; a step costs
// the ramp (two compares, one fma, two selects) and 2 mul + 4 fma.  The ramp
// is evaluated in double for either state type: which side of t1 and t2 a
// step falls on must not depend on rounding t1, t2 to float.
template <typename R>
struct RampConst {
    double b1N, b2N, slopeN;  // beta1/N, beta2/N, (beta2 - beta1)/(t2 - t1)/N
    double t1, t2;
    R lam, h, hg, hmu;        // gamma + mu, step, h gamma, h mu
};

template <typename R>
__device__ __forceinline__ RampConst<R> ramp_const(double b1, double b2, double t1, double t2,
                                                   double gamma, double mu, double N, int spd)
{
    const double h = 1.0 / (double)spd;
    RampConst<R> c;
    c.b1N = b1 / N;
    c.b2N = b2 / N;
    c.slopeN = (b2 - b1) / (t2 - t1) / N;  // unused when t1 >= t2
    c.t1 = t1;
    c.t2 = t2;
    c.lam = (R)(gamma + mu);
    c.h = (R)h;
    c.hg = (R)(h * gamma);
    c.hmu = (R)(h * mu);
    return c;
}

// beta(t)/N of eq. (beta).
template <typename R>
__device__ __forceinline__ double ramp_bN(const RampConst<R> &c, double t)
{
    const double mid = fma(c.slopeN, t - c.t1, c.b1N);
    return (t < c.t1) ? c.b1N : ((t < c.t2) ? mid : c.b2N);
}

template <typename R, bool WITH_R>
__device__ __forceinline__ void euler_ramp_step(SirdState<R> &y, const RampConst<R> &c, double t)
{
    const R bN = (R)ramp_bN(c, t);
    const R I = y.I;
    const R p = bN * y.S * I;
    const R q = fma(-c.lam, I, p);
    if constexpr (sizeof(R) == 8) {
        y.S = fma(-c.h, p, y.S);
        if (WITH_R) y.Rr = fma(c.hg, I, y.Rr);
        y.D = fma(c.hmu, I, y.D);
        y.I = fma(c.h, q, I);
    } else {
        kahan_add(y.S, y.eS, -(c.h * p));
        if (WITH_R) kahan_add(y.Rr, y.eR, c.hg * I);
        kahan_add(y.D, y.eD, c.hmu * I);
        kahan_add(y.I, y.eI, c.h * q);
    }
}

// ------------------------------------------------------------ costs (3.1)
// Every cost of Sec. 3.1 is one of three accumulations of weighted daily
// errors e_i = (y_i - yhat_i) w_i over days 0..W, then a scale:
//   SSRE   sum e^2, w = 1/max(y,1) (0 on day 0)        scale 1
//   MSE    sum e^2, w = 1                              scale 1/n
//   MXSE   max e^2, w = 1                              scale 1
//   MAE    sum |e|, w = 1                              scale 1/n
//   MAPE   sum |e|, w = 1/max(y,1)                     scale 100/n
// (n = W + 1).  The F_IRD costs apply the same per series c in {I, R, D}
// with w = 1/(max y_c - min y_c) over the window (1 for a flat series), or
// 1/max(y,1) for MAPE, and take the largest of the three (NaN if any is
// NaN).  The forward kernels are specialised on the accumulation, so the
// daily update carries no branch on the cost kind.
enum CostAcc { kAccSq = 0, kAccAbs = 1, kAccMax = 2 };

// Per-kind constants of a cost, chosen on the host.
struct CostPlan {
    int series;     // 1 (D) or 3 (I, R, D)
    int acc;        // CostAcc
    int w_rel;      // weights 1/max(y, 1) instead of 1 (or 1/range)
    int skip0;      // weight 0 on day 0 (SSRE)
    double scale;   // 1 or 100
    int per_day;    // divide by n = W + 1
};

// Starting value of an accumulator: the max starts below any square so
// that day 0 always replaces it.
template <int ACC>
__device__ __forceinline__ double acc_init()
{
    return ACC == kAccMax ? -INFINITY : 0.0;
}

template <int ACC>
__device__ __forceinline__ void acc_day(double &acc, double e)
{
    if constexpr (ACC == kAccSq) {
        acc = fma(e, e, acc);
    } else if constexpr (ACC == kAccAbs) {
        acc += fabs(e);
    } else {
        const double sq = e * e;
        acc = (sq > acc || sq != sq) ? sq : acc;  // a NaN sticks
    }
}

__device__ __forceinline__ double cost_value(const CostPlan &c, double acc, int W)
{
    return (c.scale * acc) / (c.per_day ? (double)(W + 1) : 1.0);
}

// One day's contribution of a deceased-count cost in the form the adjoint
// differentiates; y the observation, w = 1/max(y, 1), i the day index.
__device__ __forceinline__ void cost_accum(int kind, double &acc, double D, double y,
                                           double w, int i)
{
    switch (kind) {
    case SIRD_LOSS_SSRE:
        if (i > 0) {
            const double r = (D - y) * w;
            acc = fma(r, r, acc);
        }
        break;
    case SIRD_LOSS_MSE: {
        const double e = y - D;
        acc = fma(e, e, acc);
        break;
    }
    case SIRD_LOSS_MXSE: {
        const double e = y - D;
        const double sq = e * e;
        if (i == 0 || sq > acc || sq != sq) acc = sq;  // a NaN sticks
        break;
    }
    case SIRD_LOSS_MAE: acc += fabs(y - D); break;
    case SIRD_LOSS_MAPE: acc += fabs((y - D) * w); break;
    default: break;
    }
}

__device__ __forceinline__ double cost_finish(int kind, double acc, int W)
{
    const double n = (double)(W + 1);
    if (kind == SIRD_LOSS_MSE || kind == SIRD_LOSS_MAE) return acc / n;
    if (kind == SIRD_LOSS_MAPE) return 100.0 * acc / n;
    return acc;
}

// --------------------------------------------------------- Philox4x64-10
// Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3"
// (SC'11): ten rounds of two 64x64->128 products with fixed multipliers,
// xor with the key, key bumped by Weyl constants between rounds.
struct Philox4x64 {
    uint64_t w[4];
};

__device__ __forceinline__ Philox4x64 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2,
                                                    uint64_t c3, uint64_t k0, uint64_t k1)
{
    constexpr uint64_t M0 = 0xD2E7470EE14C6C93ull;
    constexpr uint64_t M1 = 0xCA5A826395121157ull;
    constexpr uint64_t W0 = 0x9E3779B97F4A7C15ull;
    constexpr uint64_t W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
        const uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
        const uint64_t n0 = hi1 ^ c1 ^ k0;
        const uint64_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += W0;
        k1 += W1;
    }
    Philox4x64 out;
    out.w[0] = c0;
    out.w[1] = c1;
    out.w[2] = c2;
    out.w[3] = c3;
    return out;
}

// Top 53 bits scaled to [0, 1): exact in double.
__device__ __forceinline__ double u01(uint64_t x)
{
    return (double)(x >> 11) * 0x1.0p-53;
}

// ------------------------------------------------------- swarm, Sec. 3.3
// Everything the velocity/position update of one particle needs.
struct PsoMove {
    double w, c1, c2;
    uint64_t seed;
    const double *lo;       // box-shaped
    const double *hi;       // box-shaped
    double *x;              // theta-shaped
    double *v;              // theta-shaped
    const double *pbest_x;  // theta-shaped
    const double *gbest_x;  // box-shaped
};

// Velocity and position update of local particle pl of problem P at swarm
// iteration it.  The random numbers of dimension j sit in slot
// w = (j + 3) mod d: word w%4 of the Philox block with counter
// (it, pl, w/4, 1), r1 its high and r2 its low 32 bits times 2^-32.  The
// rotation puts the three trailing parameters (gamma, mu, I0) and the first
// leading one in block 0, so the integration can start after one block and
// move the later betas when it reaches them.  Every operation is a single
// rounded multiply or add (the library is built without contraction):
//   t = w v; t = t + (c1 r1)(pb - x); t = t + (c2 r2)(g - x);
//   v = t;   x = min(max(x + v, lo), hi).
// For the ramp model the positions of t1 and t2 (dimensions 2, 3) are then
// swapped when t1 > t2, so that every particle describes a ramp.
__device__ __forceinline__ void pso_move_particle(const PsoMove &m, const sird_problem &P,
                                                  int pl, uint64_t it);

// Dimension whose random numbers are in slot w of a d-dimensional particle.
__device__ __forceinline__ int move_slot_dim(int w, int d)
{
    return w >= 3 ? w - 3 : w + d - 3;
}

// Ramp model: keep t1 <= t2 (dimensions 2 and 3) of a theta-shaped array.
__device__ __forceinline__ void ramp_order(double *x, const sird_problem &P, int pl)
{
    const size_t n = (size_t)P.n_part;
    const size_t o2 = (size_t)P.theta_off + pl + 2 * n;
    const double a = x[o2], b = x[o2 + n];
    if (a > b) {
        x[o2] = b;
        x[o2 + n] = a;
    }
}

// Personal best of local particle pl given its loss f (NaN counts as +inf):
// strict improvement replaces pbest_f and copies x into pbest_x.
__device__ __forceinline__ void pso_pbest_particle(double f, const sird_problem &P, int pl,
                                                   double *pbest_f, double *pbest_x,
                                                   const double *x)
{
    if (f != f) f = INFINITY;
    if (f < pbest_f[P.p_off + pl]) {
        pbest_f[P.p_off + pl] = f;
        const int d = P.n_seg + 3;
        const size_t n = (size_t)P.n_part;
        const size_t base = (size_t)P.theta_off + pl;
        // eight loads in flight before their stores
        for (int j0 = 0; j0 < d; j0 += 8) {
            double t[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) t[u] = x[base + (size_t)min(j0 + u, d - 1) * n];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (j0 + u < d) pbest_x[base + (size_t)(j0 + u) * n] = t[u];
        }
    }
}

// ---------------------------------------------------------- wave helpers
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T>
__device__ __forceinline__ T wave_uniform(T v)
{
    return __builtin_amdgcn_readfirstlane(v);
}

// The dimensions of one Philox block of a particle's move, loaded ahead of
// the block's rounds so that the memory latency overlaps them.  Slots past
// d load the last dimension again and are never stored.
struct MoveBlock {
    double x[4], v[4], pb[4];
};

__device__ __forceinline__ void pso_move_load(const PsoMove &m, const sird_problem &P, int pl,
                                              int q, MoveBlock &b)
{
    const int d = P.n_seg + 3;
    const size_t n = (size_t)P.n_part;
    const size_t base = (size_t)P.theta_off + pl;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int w = min(4 * q + s, d - 1);
        const size_t o = base + (size_t)move_slot_dim(w, d) * n;
        b.x[s] = m.x[o];
        b.v[s] = m.v[o];
        b.pb[s] = m.pbest_x[o];
    }
}

// New velocity and position of the slots of block q from the values loaded
// by pso_move_load; x and v are stored and the new positions returned by
// slot in xn.
__device__ __forceinline__ void pso_move_commit(const PsoMove &m, const sird_problem &P, int pl,
                                                uint64_t it, int q, const MoveBlock &b,
                                                double (&xn)[4])
{
    const int d = P.n_seg + 3;
    const size_t n = (size_t)P.n_part;
    const size_t base = (size_t)P.theta_off + pl;
    const double *g = m.gbest_x + P.box_off;
    const double *lo = m.lo + P.box_off;
    const double *hi = m.hi + P.box_off;
    const Philox4x64 r = philox4x64_10(it, (uint64_t)pl, (uint64_t)q, 1, m.seed, P.stream);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int w = min(4 * q + s, d - 1);
        const int j = move_slot_dim(w, d);
        const double r1 = (double)(uint32_t)(r.w[s] >> 32) * 0x1.0p-32;
        const double r2 = (double)(uint32_t)r.w[s] * 0x1.0p-32;
        const double xo = b.x[s];
        double tv = m.w * b.v[s];
        const double a1 = m.c1 * r1;
        const double d1 = b.pb[s] - xo;
        const double a2 = m.c2 * r2;
        const double d2 = g[j] - xo;
        const double m1 = a1 * d1;
        tv = tv + m1;
        const double m2 = a2 * d2;
        tv = tv + m2;
        double x1 = xo + tv;
        if (x1 < lo[j]) x1 = lo[j];
        if (x1 > hi[j]) x1 = hi[j];
        xn[s] = x1;
        if (4 * q + s < d) {
            const size_t o = base + (size_t)j * n;
            m.v[o] = tv;
            m.x[o] = x1;
        }
    }
}

__device__ __forceinline__ void pso_move_block(const PsoMove &m, const sird_problem &P, int pl,
                                               uint64_t it, int q, double (&xn)[4])
{
    MoveBlock b;
    pso_move_load(m, P, pl, q, b);
    pso_move_commit(m, P, pl, it, q, b, xn);
}

// The same block with each slot loaded, updated and stored in turn: fewer
// registers, for use while an integration's state is live (its memory
// latency is then covered by the other wavefronts of the SIMD).
__device__ __forceinline__ void pso_move_block_seq(const PsoMove &m, const sird_problem &P,
                                                   int pl, uint64_t it, int q, double (&xn)[4])
{
    const int d = P.n_seg + 3;
    const size_t n = (size_t)P.n_part;
    const size_t base = (size_t)P.theta_off + pl;
    const double *g = m.gbest_x + P.box_off;
    const double *lo = m.lo + P.box_off;
    const double *hi = m.hi + P.box_off;
    const Philox4x64 r = philox4x64_10(it, (uint64_t)pl, (uint64_t)q, 1, m.seed, P.stream);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        if (4 * q + s >= d) break;
        const int j = move_slot_dim(4 * q + s, d);
        const size_t o = base + (size_t)j * n;
        const double r1 = (double)(uint32_t)(r.w[s] >> 32) * 0x1.0p-32;
        const double r2 = (double)(uint32_t)r.w[s] * 0x1.0p-32;
        const double xo = m.x[o];
        double tv = m.w * m.v[o];
        const double a1 = m.c1 * r1;
        const double d1 = m.pbest_x[o] - xo;
        const double a2 = m.c2 * r2;
        const double d2 = g[j] - xo;
        const double m1 = a1 * d1;
        tv = tv + m1;
        const double m2 = a2 * d2;
        tv = tv + m2;
        double x1 = xo + tv;
        if (x1 < lo[j]) x1 = lo[j];
        if (x1 > hi[j]) x1 = hi[j];
        m.v[o] = tv;
        m.x[o] = x1;
        xn[s] = x1;
    }
}

__device__ __forceinline__ void pso_move_particle(const PsoMove &m, const sird_problem &P,
                                                  int pl, uint64_t it)
{
    const int d = P.n_seg + 3;
    for (int q = 0; 4 * q < d; ++q) {
        double xn[4];
        pso_move_block(m, P, pl, it, q, xn);
    }
    if (P.model == SIRD_MODEL_EULER_RAMP) ramp_order(m.x, P, pl);
}

// The same move for the ramp model (d = 7: two blocks, slots (gamma, mu,
// I0, beta1) and (beta2, t1, t2)), with the new position also returned in
// xr by dimension (t1 <= t2 as stored): the caller integrates from
// registers instead of reading x back.
__device__ __forceinline__ void pso_move_ramp(const PsoMove &m, const sird_problem &P, int pl,
                                              uint64_t it, double (&xr)[7])
{
    double x0[4] = {0.0, 0.0, 0.0, 0.0}, x1[4] = {0.0, 0.0, 0.0, 0.0};
    pso_move_block_seq(m, P, pl, it, 0, x0);
    pso_move_block_seq(m, P, pl, it, 1, x1);
    xr[4] = x0[0];
    xr[5] = x0[1];
    xr[6] = x0[2];
    xr[0] = x0[3];
    xr[1] = x1[0];
    xr[2] = x1[1];
    xr[3] = x1[2];
    if (xr[2] > xr[3]) {
        const double t = xr[2];
        xr[2] = xr[3];
        xr[3] = t;
        const size_t n = (size_t)P.n_part;
        const size_t base = (size_t)P.theta_off + pl;
        m.x[base + 2 * n] = xr[2];
        m.x[base + 3 * n] = xr[3];
    }
}

// Index of this wavefront's tile in a launch of one wavefront per tile,
// made wavefront-uniform so that everything derived from it lives in SGPRs.
__device__ __forceinline__ int wave_tile_index()
{
    return wave_uniform((int)(blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave));
}

}  // namespace sird
