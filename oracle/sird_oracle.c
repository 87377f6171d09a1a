/*
 * Plain FP64 CPU oracle for the SIRD calibration hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * reference that the GPU library is checked against.  It shares no code,
 * header, constant or helper with the GPU library and is never linked into
 * it.  Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load it.
 *
 * What it computes, with the passage each part follows:
 *   - the SIRD right-hand side, eq. (SIRD) of Sec. 2.2, in the natural
 *     state (S, I, R, D);
 *   - a piecewise-constant transmission rate beta_k on segments of
 *     seg_days days (the library's replacement for the ramp of eq. (beta));
 *     the segment index is taken from the step index, so all four stages of
 *     a step use the same beta; the last segment extends to the end;
 *   - the ramp of eq. (beta) itself, for the Euler variant of Sec. 3.1/3.3;
 *   - classical RK4 with a fixed step h = 1/spd (the library's integrator),
 *     and forward Euler (the scheme named in Sec. 3.1 and Sec. 3.3);
 *   - the low-level costs MXSE, MSE, MAE, MAPE of Sec. 3.1 on the deceased
 *     compartment, plus the sum of squared relative errors (SSRE);
 *   - particle swarm optimisation as in Sec. 3.3 (inertia, cognitive and
 *     social coefficients; out-of-box positions set to the bound), driven
 *     by Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11);
 *   - the gradient of the discrete loss by forward-mode tangent propagation
 *     through every RK4 stage (an algorithm independent of the GPU's
 *     reverse-mode adjoint);
 *   - projected Adam (Kingma & Ba 2015) in box-normalised coordinates.
 *
 * Build: gcc -O2 -std=c99 -ffp-contract=off -fopenmp -shared -fPIC.
 * Evaluation order is the natural one; no contraction, no reordering.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ */
/* Philox4x64-10 (Salmon et al., SC'11).                               */
/* One round: two 64x64->128 products of the even counter words with  */
/* fixed multipliers, then a permutation/xor with the key; the key is  */
/* bumped by the Weyl constants between rounds.                        */
/* ------------------------------------------------------------------ */
#define ORC_PHILOX_M0 0xD2E7470EE14C6C93ULL
#define ORC_PHILOX_M1 0xCA5A826395121157ULL
#define ORC_PHILOX_W0 0x9E3779B97F4A7C15ULL /* golden ratio */
#define ORC_PHILOX_W1 0xBB67AE8584CAA73BULL /* sqrt(3) - 1 */

static void orc_mul128(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo)
{
    unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += ORC_PHILOX_W0;
            k1 += ORC_PHILOX_W1;
        }
        uint64_t hi0, lo0, hi1, lo1;
        orc_mul128(ORC_PHILOX_M0, x0, &hi0, &lo0);
        orc_mul128(ORC_PHILOX_M1, x2, &hi1, &lo1);
        uint64_t y0 = hi1 ^ x1 ^ k0;
        uint64_t y1 = lo1;
        uint64_t y2 = hi0 ^ x3 ^ k1;
        uint64_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Top 53 bits of a 64-bit word, scaled to [0, 1). */
double orc_u01(uint64_t w)
{
    return (double)(w >> 11) * (1.0 / 9007199254740992.0);
}

/* ------------------------------------------------------------------ */
/* Model: eq. (SIRD), Sec. 2.2.                                         */
/* ------------------------------------------------------------------ */
static void sird_rhs(double beta, double gamma, double mu, double N,
                     const double y[4], double k[4])
{
    double S = y[0], I = y[1];
    double infection = beta / N * S * I; /* (beta/N) S I */
    k[0] = -infection;
    k[1] = infection - (gamma + mu) * I;
    k[2] = gamma * I;
    k[3] = mu * I;
}

/* Segment of step n: all four stages of step n use beta_{k(n)}. */
static int seg_of_step(long n, int seg_days, int spd, int K)
{
    long k = n / ((long)seg_days * (long)spd);
    if (k > K - 1)
        k = K - 1;
    return (int)k;
}

/* eq. (beta): beta1 before t1, linear from beta1 to beta2 on [t1, t2),
 * beta2 from t2 on.  t is measured in days from the window start. */
double orc_beta_ramp(double t, double b1, double b2, double t1, double t2)
{
    if (t < t1)
        return b1;
    if (t < t2)
        return b1 + (b2 - b1) / (t2 - t1) * (t - t1);
    return b2;
}

static void rk4_step(double beta, double gamma, double mu, double N, double h,
                     double y[4])
{
    double k1[4], k2[4], k3[4], k4[4], yt[4];
    int c;
    sird_rhs(beta, gamma, mu, N, y, k1);
    for (c = 0; c < 4; ++c) yt[c] = y[c] + h / 2.0 * k1[c];
    sird_rhs(beta, gamma, mu, N, yt, k2);
    for (c = 0; c < 4; ++c) yt[c] = y[c] + h / 2.0 * k2[c];
    sird_rhs(beta, gamma, mu, N, yt, k3);
    for (c = 0; c < 4; ++c) yt[c] = y[c] + h * k3[c];
    sird_rhs(beta, gamma, mu, N, yt, k4);
    for (c = 0; c < 4; ++c)
        y[c] = y[c] + h / 6.0 * (k1[c] + 2.0 * k2[c] + 2.0 * k3[c] + k4[c]);
}

static void euler_step(double beta, double gamma, double mu, double N, double h,
                       double y[4])
{
    double k[4];
    int c;
    sird_rhs(beta, gamma, mu, N, y, k);
    for (c = 0; c < 4; ++c) y[c] = y[c] + h * k[c];
}

/* Parameter vector of the piecewise-constant model:
 *   theta = (beta_1 .. beta_K, gamma, mu, I0),  d = K + 3.
 * Initial state: S = N - I0 - R0 - D0, I = I0, R = R0, D = D0. */
static void initial_state(double N, double R0, double D0, double I0, double y[4])
{
    y[0] = N - I0 - R0 - D0;
    y[1] = I0;
    y[2] = R0;
    y[3] = D0;
}

/* Integrate one parameter vector with RK4 over W days at spd steps/day.
 * days (may be NULL): [4][W+1], compartment-major, state at every day.
 * steps (may be NULL): [4][T+1], state after every step (T = W*spd). */
void orc_integrate(int W, int spd, int seg_days, int K, double N, double R0,
                   double D0, const double *theta, double *days, double *steps)
{
    double y[4];
    double h = 1.0 / (double)spd;
    double gamma = theta[K], mu = theta[K + 1], I0 = theta[K + 2];
    long T = (long)W * spd;
    initial_state(N, R0, D0, I0, y);
    for (int c = 0; c < 4; ++c) {
        if (days) days[(long)c * (W + 1)] = y[c];
        if (steps) steps[(long)c * (T + 1)] = y[c];
    }
    for (long n = 0; n < T; ++n) {
        double beta = theta[seg_of_step(n, seg_days, spd, K)];
        rk4_step(beta, gamma, mu, N, h, y);
        for (int c = 0; c < 4; ++c) {
            if (steps) steps[(long)c * (T + 1) + n + 1] = y[c];
            if (days && (n + 1) % spd == 0)
                days[(long)c * (W + 1) + (n + 1) / spd] = y[c];
        }
    }
}

/* Paper-exact variant: forward Euler with the ramp of eq. (beta).
 * theta = (beta1, beta2, t1, t2, gamma, mu); the window starts from the
 * given state y0 = (S, I, R, D) (the paper takes it from the data on the
 * first day).  beta is evaluated at the start of each step. */
void orc_integrate_euler_ramp(int W, int spd, const double *theta,
                              const double *y0, double N, double *days)
{
    double y[4];
    double h = 1.0 / (double)spd;
    long T = (long)W * spd;
    for (int c = 0; c < 4; ++c) {
        y[c] = y0[c];
        days[(long)c * (W + 1)] = y[c];
    }
    for (long n = 0; n < T; ++n) {
        double t = (double)n * h;
        double beta = orc_beta_ramp(t, theta[0], theta[1], theta[2], theta[3]);
        euler_step(beta, theta[4], theta[5], N, h, y);
        if ((n + 1) % spd == 0)
            for (int c = 0; c < 4; ++c) days[(long)c * (W + 1) + (n + 1) / spd] = y[c];
    }
}

/* ------------------------------------------------------------------ */
/* Costs, Sec. 3.1.  Dhat and y hold days 0..W (n = W + 1 values).      */
/*   e_i = y_i - Dhat_i                                                 */
/*   SSRE = sum_{i=1..W} ((Dhat_i - y_i) / max(y_i, 1))^2               */
/*   MSE  = (1/n) sum e_i^2      MXSE = max e_i^2                        */
/*   MAE  = (1/n) sum |e_i|      MAPE = (100/n) sum |e_i / max(y_i,1)|   */
/* ------------------------------------------------------------------ */
enum { ORC_SSRE = 0, ORC_MSE = 1, ORC_MXSE = 2, ORC_MAE = 3, ORC_MAPE = 4 };

double orc_loss(int kind, int W, const double *Dhat, const double *y)
{
    int n = W + 1;
    double acc = 0.0;
    for (int i = 0; i <= W; ++i) {
        double e = y[i] - Dhat[i];
        double guard = y[i] > 1.0 ? y[i] : 1.0;
        switch (kind) {
        case ORC_SSRE:
            if (i >= 1) {
                double r = (Dhat[i] - y[i]) / guard;
                acc = acc + r * r;
            }
            break;
        case ORC_MSE: acc = acc + e * e; break;
        case ORC_MXSE: {
            /* a NaN anywhere makes the maximum NaN */
            double sq = e * e;
            if (i == 0 || sq > acc || isnan(sq)) acc = sq;
            break;
        }
        case ORC_MAE: acc = acc + fabs(e); break;
        case ORC_MAPE: acc = acc + fabs(e / guard); break;
        default: return NAN;
        }
    }
    if (kind == ORC_MSE || kind == ORC_MAE) acc = acc / (double)n;
    if (kind == ORC_MAPE) acc = 100.0 * acc / (double)n;
    return acc;
}

/* Losses of P parameter vectors (theta row-major [P][d]) on one problem. */
void orc_loss_batch(int W, int spd, int seg_days, int K, double N, double R0,
                    double D0, int P, const double *theta, const double *y,
                    int kind, double *loss, int nthreads)
{
    int d = K + 3;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(static)
#endif
    for (int p = 0; p < P; ++p) {
        double *days = (double *)malloc(sizeof(double) * 4 * (size_t)(W + 1));
        orc_integrate(W, spd, seg_days, K, N, R0, D0, theta + (long)p * d, days, NULL);
        double l = orc_loss(kind, W, days + 3L * (W + 1), y);
        loss[p] = l;
        free(days);
    }
}

/* ------------------------------------------------------------------ */
/* PSO, Sec. 3.3.                                                       */
/* Random numbers: Philox4x64-10, key = (seed, stream).                 */
/* A counter block (iteration, particle, m, purpose) yields four words.  */
/*   init (purpose 0): block m = j/2 serves dimensions 2m, 2m+1 with     */
/*     u_j = u01(word 2*(j&1)) (53 bits);                                */
/*   velocity (purpose 1): dimension j takes slot s = (j+3) mod d;       */
/*     block m = s/4 serves slots 4m..4m+3 and word s&3 gives            */
/*     r1_j = (high 32 bits) 2^-32 and r2_j = (low 32 bits) 2^-32.       */
/* Arrays are row-major [P][d].                                          */
/* ------------------------------------------------------------------ */
static void philox_block(uint64_t seed, uint64_t stream, uint64_t it, uint64_t p,
                         uint64_t m, uint64_t purpose, uint64_t out[4])
{
    uint64_t ctr[4] = {it, p, m, purpose};
    uint64_t key[2] = {seed, stream};
    orc_philox4x64_10(ctr, key, out);
}

void orc_pso_init(int P, int d, const double *lo, const double *hi,
                  uint64_t seed, uint64_t stream, double *x, double *v,
                  double *pbest_x, double *pbest_f, double *gbest_x,
                  double *gbest_f, int64_t *gbest_idx)
{
    for (int p = 0; p < P; ++p) {
        for (int j = 0; j < d; ++j) {
            uint64_t w[4];
            philox_block(seed, stream, 0, (uint64_t)p, (uint64_t)(j / 2), 0, w);
            double u = orc_u01(w[2 * (j % 2)]);
            double xv = lo[j] + u * (hi[j] - lo[j]);
            x[(long)p * d + j] = xv;
            v[(long)p * d + j] = 0.0;
            pbest_x[(long)p * d + j] = xv;
        }
        pbest_f[p] = INFINITY;
    }
    for (int j = 0; j < d; ++j) gbest_x[j] = lo[j];
    *gbest_f = INFINITY;
    *gbest_idx = -1;
}

/* Personal and global bests after evaluating f = loss(x).
 * NaN losses count as +inf.  Personal best: strict improvement.
 * Global best: argmin of the personal bests, lowest index on ties,
 * replacing the previous global best only on strict improvement.
 * margin (may be NULL): the smallest relative gap of any comparison
 * that decided an outcome in this update (near-tie detector). */
void orc_pso_bests(int P, int d, const double *f, const double *x,
                   double *pbest_x, double *pbest_f, double *gbest_x,
                   double *gbest_f, int64_t *gbest_idx, double *margin)
{
    double mrel = INFINITY;
    for (int p = 0; p < P; ++p) {
        double fp = isnan(f[p]) ? INFINITY : f[p];
        if (isfinite(fp) && isfinite(pbest_f[p])) {
            double scale = fabs(pbest_f[p]) > fabs(fp) ? fabs(pbest_f[p]) : fabs(fp);
            /* equal values come from equal positions and are decided
             * identically by any implementation: they are not near-ties */
            if (scale > 0.0 && fp != pbest_f[p]) {
                double g = fabs(fp - pbest_f[p]) / scale;
                if (g < mrel) mrel = g;
            }
        }
        if (fp < pbest_f[p]) {
            pbest_f[p] = fp;
            for (int j = 0; j < d; ++j) pbest_x[(long)p * d + j] = x[(long)p * d + j];
        }
    }
    int best = 0;
    for (int p = 1; p < P; ++p)
        if (pbest_f[p] < pbest_f[best]) best = p;
    /* gap between the winner and the runner-up */
    for (int p = 0; p < P; ++p) {
        if (p == best || !isfinite(pbest_f[p]) || !isfinite(pbest_f[best])) continue;
        if (pbest_f[p] == pbest_f[best]) continue;
        double scale = fabs(pbest_f[p]) > fabs(pbest_f[best]) ? fabs(pbest_f[p]) : fabs(pbest_f[best]);
        double g = scale > 0.0 ? fabs(pbest_f[p] - pbest_f[best]) / scale : 0.0;
        if (g < mrel) mrel = g;
    }
    if (P > 0 && isfinite(*gbest_f) && isfinite(pbest_f[best])) {
        double scale = fabs(*gbest_f) > fabs(pbest_f[best]) ? fabs(*gbest_f) : fabs(pbest_f[best]);
        double g = scale > 0.0 ? fabs(*gbest_f - pbest_f[best]) / scale : 0.0;
        if (g > 0.0 && g < mrel) mrel = g; /* an unchanged best (g == 0) decides nothing */
    }
    if (P > 0 && pbest_f[best] < *gbest_f) {
        *gbest_f = pbest_f[best];
        *gbest_idx = best;
        for (int j = 0; j < d; ++j) gbest_x[j] = pbest_x[(long)best * d + j];
    }
    if (margin) *margin = mrel;
}

/* Velocity and position update of iteration it, every operation a single
 * rounded IEEE multiply or add:
 *   t = w*v;  t = t + (c1*r1)*(pb - x);  t = t + (c2*r2)*(g - x);
 *   v = t;    x = min(max(x + v, lo), hi).
 * The paper does not say how the random numbers are drawn (Sec. 3.3).
 * Reading used here: dimension j of a d-dimensional particle takes slot
 * s = (j + 3) mod d; slot s is word s % 4 of the Philox block with counter
 * (it, p, s / 4, 1); r1 is that word's high and r2 its low 32 bits, each
 * times 2^-32.  (The slot order lists the last three parameters first.) */
void orc_pso_move(int P, int d, uint64_t it, double w, double c1, double c2,
                  const double *lo, const double *hi, uint64_t seed,
                  uint64_t stream, const double *pbest_x, const double *gbest_x,
                  double *x, double *v)
{
    for (int p = 0; p < P; ++p) {
        for (int j = 0; j < d; ++j) {
            uint64_t wd[4];
            int slot = (j + 3) % d;
            philox_block(seed, stream, it, (uint64_t)p, (uint64_t)(slot / 4), 1, wd);
            uint64_t word = wd[slot % 4];
            double r1 = (double)(word >> 32) * (1.0 / 4294967296.0);
            double r2 = (double)(word & 0xffffffffULL) * (1.0 / 4294967296.0);
            long o = (long)p * d + j;
            double xo = x[o];
            double t = w * v[o];
            double a1 = c1 * r1;
            double d1 = pbest_x[o] - xo;
            double a2 = c2 * r2;
            double d2 = gbest_x[j] - xo;
            double m1 = a1 * d1;
            t = t + m1;
            double m2 = a2 * d2;
            t = t + m2;
            v[o] = t;
            double xn = xo + t;
            if (xn < lo[j]) xn = lo[j];
            if (xn > hi[j]) xn = hi[j];
            x[o] = xn;
        }
    }
}

/* Whole PSO run on one problem: iters evaluations.  For it = 0..iters-1:
 * f = loss(x); bests; record (gbest_f, gbest_idx, margin); move unless last.
 * Final swarm state is returned through x, v, pbest_x, pbest_f, gbest_x. */
void orc_pso_run(int W, int spd, int seg_days, int K, double N, double R0,
                 double D0, const double *y, int kind, int P, const double *lo,
                 const double *hi, double w, double c1, double c2, uint64_t seed,
                 uint64_t stream, int iters, double *hist_f, int64_t *hist_idx,
                 double *hist_margin, double *x, double *v, double *pbest_x,
                 double *pbest_f, double *gbest_x, int nthreads)
{
    int d = K + 3;
    double gbest_f;
    int64_t gbest_idx;
    double *f = (double *)malloc(sizeof(double) * (size_t)(P > 0 ? P : 1));
    orc_pso_init(P, d, lo, hi, seed, stream, x, v, pbest_x, pbest_f, gbest_x,
                 &gbest_f, &gbest_idx);
    for (int it = 0; it < iters; ++it) {
        double margin;
        orc_loss_batch(W, spd, seg_days, K, N, R0, D0, P, x, y, kind, f, nthreads);
        orc_pso_bests(P, d, f, x, pbest_x, pbest_f, gbest_x, &gbest_f, &gbest_idx, &margin);
        if (hist_f) hist_f[it] = gbest_f;
        if (hist_idx) hist_idx[it] = gbest_idx;
        if (hist_margin) hist_margin[it] = margin;
        if (it < iters - 1)
            orc_pso_move(P, d, (uint64_t)it, w, c1, c2, lo, hi, seed, stream,
                         pbest_x, gbest_x, x, v);
    }
    free(f);
}

/* ------------------------------------------------------------------ */
/* Gradient of the discrete loss by forward-mode differentiation.       */
/* For each parameter j the tangent Ydot = dY/dtheta_j is carried       */
/* through every RK4 stage:                                             */
/*   kdot_s = J(Y_s) Ydot_s + (df/dtheta_j)(Y_s),                       */
/*   Ydot_2 = ydot + h/2 kdot_1, Ydot_3 = ydot + h/2 kdot_2,            */
/*   Ydot_4 = ydot + h kdot_3,                                          */
/*   ydot+ = ydot + h/6 (kdot_1 + 2 kdot_2 + 2 kdot_3 + kdot_4),        */
/* and dL/dtheta_j = sum_i (dl/dDhat_i) Ddot_i.                          */
/* ------------------------------------------------------------------ */

/* Jacobian-vector product of eq. (SIRD) plus the explicit parameter
 * derivative.  which: 0 = beta (of the active segment), 1 = gamma,
 * 2 = mu, -1 = none. */
static void sird_tangent(double beta, double gamma, double mu, double N,
                         const double y[4], const double yd[4], int which,
                         double kd[4])
{
    double S = y[0], I = y[1];
    double Sd = yd[0], Id = yd[1];
    /* d[(beta/N) S I] = (beta/N)(Sd I + S Id) */
    double infd = beta / N * (Sd * I + S * Id);
    double dI = -(gamma + mu) * Id;
    double dR = gamma * Id;
    double dD = mu * Id;
    double inf_beta = 0.0, dI_extra = 0.0, dR_extra = 0.0, dD_extra = 0.0;
    if (which == 0) inf_beta = S * I / N;
    if (which == 1) { dI_extra = -I; dR_extra = I; }
    if (which == 2) { dI_extra = -I; dD_extra = I; }
    kd[0] = -infd - inf_beta;
    kd[1] = infd + inf_beta + dI + dI_extra;
    kd[2] = dR + dR_extra;
    kd[3] = dD + dD_extra;
}

/* dl/dDhat_i for the cost of the given kind (index i of days 0..W). */
static double cost_dDhat(int kind, int W, int i, double Dhat, double y, int argmax)
{
    int n = W + 1;
    double e = y - Dhat;
    double guard = y > 1.0 ? y : 1.0;
    double s = (e > 0.0) ? 1.0 : ((e < 0.0) ? -1.0 : 0.0);
    switch (kind) {
    case ORC_SSRE: return i >= 1 ? 2.0 * ((Dhat - y) / guard) / guard : 0.0;
    case ORC_MSE: return -2.0 * e / (double)n;
    case ORC_MXSE: return i == argmax ? -2.0 * e : 0.0;
    case ORC_MAE: return -s / (double)n;
    case ORC_MAPE: return -100.0 * s / guard / (double)n;
    default: return NAN;
    }
}

/* scale (may be NULL): per component, the sum over days of the absolute
 * values of the terms dl/dDhat_i * dDhat_i/dtheta_j that the gradient adds
 * up -- the size the component's rounding error is relative to when the
 * terms cancel. */
void orc_loss_grad_fwd(int W, int spd, int seg_days, int K, double N, double R0,
                       double D0, const double *theta, const double *y, int kind,
                       double *loss, double *grad, double *scale)
{
    int d = K + 3;
    long T = (long)W * spd;
    double h = 1.0 / (double)spd;
    double gamma = theta[K], mu = theta[K + 1], I0 = theta[K + 2];
    double *days = (double *)malloc(sizeof(double) * 4 * (size_t)(W + 1));
    orc_integrate(W, spd, seg_days, K, N, R0, D0, theta, days, NULL);
    const double *Dhat = days + 3L * (W + 1);
    *loss = orc_loss(kind, W, Dhat, y);
    int argmax = 0;
    if (kind == ORC_MXSE) {
        double best = -1.0;
        for (int i = 0; i <= W; ++i) {
            double e = y[i] - Dhat[i];
            if (e * e > best) { best = e * e; argmax = i; }
        }
    }
    for (int j = 0; j < d; ++j) {
        double yv[4], yd[4];
        initial_state(N, R0, D0, I0, yv);
        yd[0] = yd[1] = yd[2] = yd[3] = 0.0;
        if (j == K + 2) { yd[0] = -1.0; yd[1] = 1.0; } /* dS0/dI0 = -1, dI0/dI0 = 1 */
        double g = cost_dDhat(kind, W, 0, Dhat[0], y[0], argmax) * yd[3];
        double gs = fabs(g);
        for (long n = 0; n < T; ++n) {
            int k = seg_of_step(n, seg_days, spd, K);
            double beta = theta[k];
            int which = -1;
            if (j == k) which = 0;
            if (j == K) which = 1;
            if (j == K + 1) which = 2;
            double k1[4], k2[4], k3[4], k4[4], kd1[4], kd2[4], kd3[4], kd4[4];
            double yt[4], ydt[4];
            int c;
            sird_rhs(beta, gamma, mu, N, yv, k1);
            sird_tangent(beta, gamma, mu, N, yv, yd, which, kd1);
            for (c = 0; c < 4; ++c) { yt[c] = yv[c] + h / 2.0 * k1[c]; ydt[c] = yd[c] + h / 2.0 * kd1[c]; }
            sird_rhs(beta, gamma, mu, N, yt, k2);
            sird_tangent(beta, gamma, mu, N, yt, ydt, which, kd2);
            for (c = 0; c < 4; ++c) { yt[c] = yv[c] + h / 2.0 * k2[c]; ydt[c] = yd[c] + h / 2.0 * kd2[c]; }
            sird_rhs(beta, gamma, mu, N, yt, k3);
            sird_tangent(beta, gamma, mu, N, yt, ydt, which, kd3);
            for (c = 0; c < 4; ++c) { yt[c] = yv[c] + h * k3[c]; ydt[c] = yd[c] + h * kd3[c]; }
            sird_rhs(beta, gamma, mu, N, yt, k4);
            sird_tangent(beta, gamma, mu, N, yt, ydt, which, kd4);
            for (c = 0; c < 4; ++c) {
                yv[c] = yv[c] + h / 6.0 * (k1[c] + 2.0 * k2[c] + 2.0 * k3[c] + k4[c]);
                yd[c] = yd[c] + h / 6.0 * (kd1[c] + 2.0 * kd2[c] + 2.0 * kd3[c] + kd4[c]);
            }
            if ((n + 1) % spd == 0) {
                int i = (int)((n + 1) / spd);
                double term = cost_dDhat(kind, W, i, Dhat[i], y[i], argmax) * yd[3];
                g = g + term;
                gs = gs + fabs(term);
            }
        }
        grad[j] = g;
        if (scale) scale[j] = gs;
    }
    free(days);
}

/* ------------------------------------------------------------------ */
/* Projected Adam (Kingma & Ba 2015) in box-normalised coordinates       */
/* u = (theta - lo)/(hi - lo).  One step t >= 1 for n vectors [n][d].   */
/* Dimensions with hi == lo are fixed and left untouched.               */
/* ------------------------------------------------------------------ */
void orc_adam_step(int n, int d, double *theta, const double *grad, double *m,
                   double *v, const double *lo, const double *hi, int t,
                   double lr, double b1, double b2, double eps)
{
    double bc1 = 1.0 - pow(b1, (double)t);
    double bc2 = 1.0 - pow(b2, (double)t);
    for (int q = 0; q < n; ++q) {
        for (int j = 0; j < d; ++j) {
            long o = (long)q * d + j;
            double width = hi[j] - lo[j];
            if (!(width > 0.0)) continue;
            double u = (theta[o] - lo[j]) / width;
            double gu = grad[o] * width;
            m[o] = b1 * m[o] + (1.0 - b1) * gu;
            v[o] = b2 * v[o] + (1.0 - b2) * gu * gu;
            double mhat = m[o] / bc1;
            double vhat = v[o] / bc2;
            u = u - lr * mhat / (sqrt(vhat) + eps);
            if (u < 0.0) u = 0.0;
            if (u > 1.0) u = 1.0;
            theta[o] = lo[j] + u * width;
        }
    }
}

/* ------------------------------------------------------------------ */
/* Projected L-BFGS (Liu & Nocedal 1989; two-loop recursion of Nocedal  */
/* 1980) in box-normalised coordinates u = (theta - lo)/(hi - lo) (with */
/* log theta for the last dimension when log_last is set), for          */
/* refining parameter vectors with gradients of the discrete loss.      */
/* Per vector (row q of [n][d] arrays; memory arrays [n][m][d]):         */
/* Every dot product over the d dimensions adds its rounded products in  */
/* pairs (orc_pair_dot), the order of a reduction across lanes.          */
/*  propose: r = H g_u by the two-loop recursion over the stored pairs   */
/*    (initial H = (s.y / y.y) I of the newest pair, I when none);       */
/*    p = -r; components at an active bound (u = 0 and p < 0, u = 1 and */
/*    p > 0) and fixed dimensions are zeroed; if g_u.p >= 0 the memory   */
/*    is dropped and p = -g_u (projected); with no stored pair the step  */
/*    is capped so that max |alpha p| <= 0.01;                           */
/*    n_trials trial points along p, trial t at the step a_t = alpha 2^t */
/*    (rows t n + q of [n_trials n][d] arrays):                          */
/*    u_t = clamp(u + a_t p, 0, 1), theta_t = lo + u_t (hi - lo).        */
/*  accept: among the trials with finite f_t passing Armijo              */
/*    f_t <= f + c1 a_t g_u.p, the one of lowest f_t (the first on ties) */
/*    is kept: the pair (u_t - u, g_u,t - g_u) is stored when s.y > 0,   */
/*    alpha = 1; with none, alpha is halved, and below 1e-20 the memory  */
/*    is dropped and alpha = 1.  One trial is classical backtracking by  */
/*    halving; more try longer steps in the same evaluation, which the   */
/*    ill-conditioned fits take (more progress per round).               */
/* ------------------------------------------------------------------ */
/* Box coordinate of dimension j: u = (phi(theta) - a)/w with phi the
 * identity, or the logarithm for the last dimension when log_last is set
 * (I0, which spans decades); w = 0 marks a fixed dimension. */
typedef struct { double a, w; int lg; } orc_coord;

static orc_coord orc_coord_of(const double *lo, const double *hi, int j, int d, int log_last)
{
    orc_coord c;
    c.lg = log_last && j == d - 1;
    if (c.lg) {
        c.a = log(lo[j]);
        c.w = log(hi[j]) - c.a;
    } else {
        c.a = lo[j];
        c.w = hi[j] - lo[j];
    }
    if (!(c.w > 0.0)) c.w = 0.0;
    return c;
}

static double orc_to_u(orc_coord c, double th)
{
    if (c.w == 0.0) return 0.0;
    return ((c.lg ? log(th) : th) - c.a) / c.w;
}

static double orc_from_u(orc_coord c, double u)
{
    double v = c.a + u * c.w;
    return c.lg ? exp(v) : v;
}

/* d loss / d u from d loss / d theta */
static double orc_grad_u(orc_coord c, double th, double g)
{
    return c.lg ? g * th * c.w : g * c.w;
}

/* sum over j < d (d <= 64) of a[j] b[j]: the products rounded, then added
 * in pairs over the dimensions padded with zeros to the next power of two
 * w -- first neighbours (0+1, 2+3, ...), then pairs of those, up to the
 * width w -- the order in which a reduction across lanes adds them. */
static double orc_pair_dot(const double *a, const double *b, int d)
{
    double v[64];
    int w = 1;
    while (w < d) w <<= 1;
    for (int j = 0; j < w; ++j) v[j] = j < d ? a[j] * b[j] : 0.0;
    for (int h = 1; h < w; h <<= 1)
        for (int j = 0; j < w; j += 2 * h) v[j] = v[j] + v[j + h];
    return v[0];
}

void orc_lbfgs_propose(int n, int d, int m, int log_last, int n_trials, const double *lo,
                       const double *hi, const double *theta, const double *grad,
                       const double *S, const double *Y, const double *rho, int *count,
                       const int *head, double *alpha, double *p_out, double *gp_out,
                       double *theta_t)
{
    for (int q = 0; q < n; ++q) {
        const double *th = theta + (long)q * d;
        const double *g = grad + (long)q * d;
        double gu[64], r[64], u[64], a[64];
        int cnt = count[q];
        for (int j = 0; j < d; ++j) {
            orc_coord c = orc_coord_of(lo, hi, j, d, log_last);
            gu[j] = orc_grad_u(c, th[j], g[j]);
            u[j] = orc_to_u(c, th[j]);
            r[j] = gu[j];
        }
        /* first loop: newest to oldest */
        for (int k = 0; k < cnt; ++k) {
            int slot = ((head[q] - 1 - k) % m + m) % m;
            const double *s = S + ((long)q * m + slot) * d;
            const double *y = Y + ((long)q * m + slot) * d;
            const double sr = orc_pair_dot(s, r, d);
            a[k] = rho[(long)q * m + slot] * sr;
            for (int j = 0; j < d; ++j) r[j] = r[j] - a[k] * y[j];
        }
        double h0 = 1.0;
        if (cnt > 0) {
            int slot = ((head[q] - 1) % m + m) % m;
            const double *s = S + ((long)q * m + slot) * d;
            const double *y = Y + ((long)q * m + slot) * d;
            const double sy = orc_pair_dot(s, y, d), yy = orc_pair_dot(y, y, d);
            if (yy > 0.0) h0 = sy / yy;
        }
        for (int j = 0; j < d; ++j) r[j] = h0 * r[j];
        /* second loop: oldest to newest */
        for (int k = cnt - 1; k >= 0; --k) {
            int slot = ((head[q] - 1 - k) % m + m) % m;
            const double *s = S + ((long)q * m + slot) * d;
            const double *y = Y + ((long)q * m + slot) * d;
            const double yr = orc_pair_dot(y, r, d);
            double b = rho[(long)q * m + slot] * yr;
            for (int j = 0; j < d; ++j) r[j] = r[j] + s[j] * (a[k] - b);
        }
        double *p = p_out + (long)q * d;
        for (int j = 0; j < d; ++j) {
            double w = orc_coord_of(lo, hi, j, d, log_last).w;
            double pj = -r[j];
            if (w == 0.0 || (u[j] <= 0.0 && pj < 0.0) || (u[j] >= 1.0 && pj > 0.0)) pj = 0.0;
            p[j] = pj;
        }
        double gp = orc_pair_dot(gu, p, d);
        if (!(gp < 0.0)) { /* not a descent direction: steepest descent */
            cnt = 0;
            for (int j = 0; j < d; ++j) {
                double w = orc_coord_of(lo, hi, j, d, log_last).w;
                double pj = -gu[j];
                if (w == 0.0 || (u[j] <= 0.0 && pj < 0.0) || (u[j] >= 1.0 && pj > 0.0)) pj = 0.0;
                p[j] = pj;
            }
            gp = orc_pair_dot(gu, p, d);
        }
        count[q] = cnt;
        if (cnt == 0) {
            double pmax = 0.0;
            for (int j = 0; j < d; ++j) if (fabs(p[j]) > pmax) pmax = fabs(p[j]);
            if (pmax > 0.0 && alpha[q] * pmax > 0.01) alpha[q] = 0.01 / pmax;
        }
        gp_out[q] = gp;
        /* trial t at the step alpha 2^t, in row t n + q */
        for (int t = 0; t < n_trials; ++t) {
            const double at = alpha[q] * (double)(1 << t);
            double *tt = theta_t + ((long)t * n + q) * d;
            for (int j = 0; j < d; ++j) {
                orc_coord c = orc_coord_of(lo, hi, j, d, log_last);
                if (c.w == 0.0) { tt[j] = th[j]; continue; }
                double ut = u[j] + at * p[j];
                if (ut < 0.0) ut = 0.0;
                if (ut > 1.0) ut = 1.0;
                tt[j] = orc_from_u(c, ut);
            }
        }
    }
}

void orc_lbfgs_accept(int n, int d, int m, int log_last, int n_trials, const double *lo,
                      const double *hi, double c1,
                      double *theta, double *grad, double *f, const double *theta_t,
                      const double *grad_t, const double *f_t, const double *gp,
                      double *S, double *Y, double *rho, int *count, int *head,
                      double *alpha)
{
    for (int q = 0; q < n; ++q) {
        /* the trial of lowest loss among those passing the Armijo test at
           their own step alpha 2^t (the first on ties) */
        int best = -1;
        double ft = 0.0;
        for (int t = 0; t < n_trials; ++t) {
            const double at = alpha[q] * (double)(1 << t);
            const double fx = f_t[(long)t * n + q];
            if (isfinite(fx) && fx <= f[q] + c1 * at * gp[q] && (best < 0 || fx < ft)) {
                best = t;
                ft = fx;
            }
        }
        if (best >= 0) {
            const double *tht = theta_t + ((long)best * n + q) * d;
            const double *grt = grad_t + ((long)best * n + q) * d;
            double sv[64], yv[64];
            for (int j = 0; j < d; ++j) {
                orc_coord c = orc_coord_of(lo, hi, j, d, log_last);
                double a = theta[(long)q * d + j], b = tht[j];
                sv[j] = orc_to_u(c, b) - orc_to_u(c, a);
                yv[j] = orc_grad_u(c, b, grt[j]) - orc_grad_u(c, a, grad[(long)q * d + j]);
            }
            const double sy = orc_pair_dot(sv, yv, d);
            if (sy > 0.0) {
                double *s = S + ((long)q * m + head[q]) * d;
                double *y = Y + ((long)q * m + head[q]) * d;
                for (int j = 0; j < d; ++j) { s[j] = sv[j]; y[j] = yv[j]; }
                rho[(long)q * m + head[q]] = 1.0 / sy;
                head[q] = (head[q] + 1) % m;
                if (count[q] < m) count[q] = count[q] + 1;
            }
            for (int j = 0; j < d; ++j) {
                theta[(long)q * d + j] = tht[j];
                grad[(long)q * d + j] = grt[j];
            }
            f[q] = ft;
            alpha[q] = 1.0;
        } else {
            alpha[q] = 0.5 * alpha[q];
            if (alpha[q] < 1e-20) {
                count[q] = 0;
                alpha[q] = 1.0;
            }
        }
    }
}

/* ------------------------------------------------------------------ */
/* The paper's own variant (Sec. 2.2, 3.1, 3.3): forward Euler with the  */
/* ramp of eq. (beta), parameter vector                                 */
/*   theta = (beta1, beta2, t1, t2, gamma, mu, I0)   (d = 7),           */
/* initial state S = N - I0 - R0 - D0, I0, R0, D0 (the paper takes it   */
/* from the data on the window's first day; I0 is then a fixed box      */
/* dimension).  beta is evaluated at the start of each step, t in days  */
/* from the window start.                                               */
/* ------------------------------------------------------------------ */
void orc_integrate_model(int model, int W, int spd, int seg_days, int K, double N, double R0,
                         double D0, const double *theta, double *days)
{
    if (model == 0) {
        orc_integrate(W, spd, seg_days, K, N, R0, D0, theta, days, NULL);
        return;
    }
    double th6[6] = {theta[0], theta[1], theta[2], theta[3], theta[4], theta[5]};
    double y0[4];
    initial_state(N, R0, D0, theta[6], y0);
    orc_integrate_euler_ramp(W, spd, th6, y0, N, days);
}

/* F_IRD of Sec. 3.1: the maximum over I, R, D of a low-level cost.  For
 * MXSE, MSE and MAE the errors are taken after the min-max normalisation
 * f_Y(y) = (y - min y)/(max y - min y) of the observed series (applied to
 * both the observation and the model value, so the error is
 * (y - yhat)/(max y - min y)); a flat observed series (max = min) is
 * normalised by 1.  MAPE is not normalised.  kind is the low-level cost
 * (ORC_MSE, ORC_MXSE, ORC_MAE, ORC_MAPE); n = W + 1 days. */
double orc_loss_ird(int kind, int W, const double *Ihat, const double *Rhat,
                    const double *Dhat, const double *yI, const double *yR, const double *yD)
{
    const double *yh[3] = {Ihat, Rhat, Dhat};
    const double *yo[3] = {yI, yR, yD};
    double F = -INFINITY;
    for (int c = 0; c < 3; ++c) {
        double lo = yo[c][0], hi = yo[c][0];
        for (int i = 1; i <= W; ++i) {
            if (yo[c][i] < lo) lo = yo[c][i];
            if (yo[c][i] > hi) hi = yo[c][i];
        }
        double range = hi - lo > 0.0 ? hi - lo : 1.0;
        double v;
        if (kind == ORC_MAPE) {
            v = orc_loss(ORC_MAPE, W, yh[c], yo[c]);
        } else {
            double *a = (double *)malloc(sizeof(double) * (size_t)(W + 1));
            double *b = (double *)malloc(sizeof(double) * (size_t)(W + 1));
            for (int i = 0; i <= W; ++i) {
                a[i] = (yh[c][i] - lo) / range;
                b[i] = (yo[c][i] - lo) / range;
            }
            v = orc_loss(kind, W, a, b);
            free(a);
            free(b);
        }
        if (isnan(v)) return NAN;
        if (v > F) F = v;
    }
    return F;
}

/* Losses of P parameter vectors of either model.  kind < 5: the D-only
 * costs of orc_loss on obs = y_D; kind 5..8: F_IRD with low-level cost
 * MXSE, MSE, MAE, MAPE on obs = [y_I; y_R; y_D] (3 (W+1) values). */
void orc_loss_batch_model(int model, int W, int spd, int seg_days, int K, double N, double R0,
                          double D0, int P, const double *theta, const double *obs, int kind,
                          double *loss, int nthreads)
{
    int d = K + 3;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(static)
#endif
    for (int p = 0; p < P; ++p) {
        double *days = (double *)malloc(sizeof(double) * 4 * (size_t)(W + 1));
        orc_integrate_model(model, W, spd, seg_days, K, N, R0, D0, theta + (long)p * d, days);
        long n1 = W + 1;
        double l;
        if (kind < 5) {
            l = orc_loss(kind, W, days + 3 * n1, obs);
        } else {
            static const int low[4] = {ORC_MXSE, ORC_MSE, ORC_MAE, ORC_MAPE};
            l = orc_loss_ird(low[kind - 5], W, days + n1, days + 2 * n1, days + 3 * n1, obs,
                             obs + n1, obs + 2 * n1);
        }
        loss[p] = l;
        free(days);
    }
}

/* After a move, keep a pair of dimensions (j, j+1) ordered (the ramp's
 * t1 <= t2): swap the positions when x_j > x_{j+1}. */
void orc_pso_sort_pair(int P, int d, int j, double *x)
{
    for (int p = 0; p < P; ++p) {
        double *r = x + (long)p * d;
        if (r[j] > r[j + 1]) {
            double t = r[j];
            r[j] = r[j + 1];
            r[j + 1] = t;
        }
    }
}

/* Whole PSO run of either model: as orc_pso_run, with the losses of
 * orc_loss_batch_model and, for the ramp model, (t1, t2) ordered after
 * every move. */
void orc_pso_run_model(int model, int W, int spd, int seg_days, int K, double N, double R0,
                       double D0, const double *obs, int kind, int P, const double *lo,
                       const double *hi, double w, double c1, double c2, uint64_t seed,
                       uint64_t stream, int iters, double *hist_f, int64_t *hist_idx,
                       double *hist_margin, double *x, double *v, double *pbest_x,
                       double *pbest_f, double *gbest_x, int nthreads)
{
    int d = K + 3;
    double gbest_f;
    int64_t gbest_idx;
    double *f = (double *)malloc(sizeof(double) * (size_t)(P > 0 ? P : 1));
    orc_pso_init(P, d, lo, hi, seed, stream, x, v, pbest_x, pbest_f, gbest_x, &gbest_f,
                 &gbest_idx);
    if (model == 1) orc_pso_sort_pair(P, d, 2, x);
    if (model == 1) orc_pso_sort_pair(P, d, 2, pbest_x);
    for (int it = 0; it < iters; ++it) {
        double margin;
        orc_loss_batch_model(model, W, spd, seg_days, K, N, R0, D0, P, x, obs, kind, f,
                             nthreads);
        orc_pso_bests(P, d, f, x, pbest_x, pbest_f, gbest_x, &gbest_f, &gbest_idx, &margin);
        if (hist_f) hist_f[it] = gbest_f;
        if (hist_idx) hist_idx[it] = gbest_idx;
        if (hist_margin) hist_margin[it] = margin;
        if (it < iters - 1) {
            orc_pso_move(P, d, (uint64_t)it, w, c1, c2, lo, hi, seed, stream, pbest_x,
                         gbest_x, x, v);
            if (model == 1) orc_pso_sort_pair(P, d, 2, x);
        }
    }
    free(f);
}
