// Refinement support: top-k selection of the swarm's personal bests, a
// gather of the selected parameter vectors into a refinement batch, and a
// projected Adam step (Kingma & Ba 2015) in box-normalised coordinates.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>

#include "device.h"
#include "internal.h"

namespace sird {

// ------------------------------------------------------------------ top-k
// Up to kTopkRounds the selection runs in k rounds, above it by ranks.
constexpr int kTopkRounds = 32;
constexpr int kTopkMax = 65536;

// One block per problem.  Round q selects the smallest (f, index) pair that
// is strictly greater than the pair selected in round q-1, so the k rounds
// emit the k smallest in (f, index) order.  NaN is ordered as +inf.
__device__ __forceinline__ bool key_less(double f, int i, double g, int j)
{
    return f < g || (f == g && i < j);
}

__global__ void __launch_bounds__(256) k_topk(const sird_problem *probs, const double *pbest_f,
                                              int k, int64_t *idx_out)
{
    __shared__ double sf[256 / kWave];
    __shared__ int si[256 / kWave];
    __shared__ double s_pf;
    __shared__ int s_pi;
    const int r = blockIdx.x;
    const sird_problem P = probs[r];
    const int n = P.n_part;
    const int tid = threadIdx.x;
    if (tid == 0) {
        s_pf = -INFINITY;
        s_pi = -1;
    }
    __syncthreads();
    for (int q = 0; q < k; ++q) {
        const double pf = s_pf;
        const int pi = s_pi;
        double bf = INFINITY;
        int bi = n;  // sentinel: nothing found
        for (int p = tid; p < n; p += blockDim.x) {
            double f = pbest_f[P.p_off + p];
            if (f != f) f = INFINITY;
            if (key_less(pf, pi, f, p) && key_less(f, p, bf, bi)) {
                bf = f;
                bi = p;
            }
        }
        for (int off = kWave / 2; off > 0; off >>= 1) {
            const double of = __shfl_xor(bf, off);
            const int oi = __shfl_xor(bi, off);
            if (key_less(of, oi, bf, bi)) {
                bf = of;
                bi = oi;
            }
        }
        if ((tid & (kWave - 1)) == 0) {
            sf[tid / kWave] = bf;
            si[tid / kWave] = bi;
        }
        __syncthreads();
        if (tid == 0) {
            for (int w = 1; w < (int)(blockDim.x / kWave); ++w)
                if (key_less(sf[w], si[w], bf, bi)) {
                    bf = sf[w];
                    bi = si[w];
                }
            idx_out[(size_t)r * k + q] = bi < n ? bi : -1;
            s_pf = bf;
            s_pi = bi;
        }
        __syncthreads();
    }
}

// Larger k: the rank of every particle, the number of particles whose
// (f, index) key is smaller, computed by one wavefront per 64-particle tile
// scanning its problem's n keys (broadcast 64 at a time by shuffles);
// a particle of rank < k is written to position rank.  Keys are distinct,
// so ranks are a permutation and the output equals the k-round selection.
// O(n^2) comparisons per problem, in parallel over its tiles.
__global__ void __launch_bounds__(256) k_topk_rank(const sird_problem *probs,
                                                   const sird_tile *tiles, int n_tiles,
                                                   const double *pbest_f, int k,
                                                   int64_t *idx_out)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int t = wave_tile_index();
    if (t >= n_tiles) return;
    const sird_tile tl = tiles[t];
    const sird_problem P = probs[tl.prob];
    const int n = P.n_part;
    const int p = tl.p0 + lane;
    double fp = INFINITY;
    if (p < n) {
        fp = pbest_f[P.p_off + p];
        if (fp != fp) fp = INFINITY;
    }
    int rank = 0;
    for (int q0 = 0; q0 < n; q0 += kWave) {
        double fq = INFINITY;
        if (q0 + lane < n) {
            fq = pbest_f[P.p_off + q0 + lane];
            if (fq != fq) fq = INFINITY;
        }
        const int m = min(kWave, n - q0);
        for (int j = 0; j < m; ++j) {
            const double g = __shfl(fq, j);
            rank += key_less(g, q0 + j, fp, p) ? 1 : 0;
        }
    }
    if (p < n && rank < k) idx_out[(size_t)tl.prob * k + rank] = p;
}

// Positions n..k-1 of every problem with fewer than k particles.
__global__ void __launch_bounds__(256) k_topk_pad(const sird_problem *probs, int k,
                                                  int64_t *idx_out)
{
    const int r = blockIdx.x;
    const int n = probs[r].n_part;
    for (int q = n + (int)threadIdx.x; q < k; q += blockDim.x) idx_out[(size_t)r * k + q] = -1;
}

// ----------------------------------------------------------------- gather
__global__ void __launch_bounds__(256) k_gather(const sird_problem *src, const double *src_theta,
                                                const double *src_lo, const sird_problem *dst,
                                                double *dst_theta, const int64_t *idx, int k,
                                                int n_prob)
{
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = gid / k;
    const int q = gid - r * k;
    if (r >= n_prob) return;
    const sird_problem S = src[r];
    const sird_problem D = dst[r];
    const int d = D.n_seg + 3;
    double *out = dst_theta + D.theta_off + q;
    if (S.n_seg != D.n_seg || D.n_part != k) {
        // shapes do not correspond: make the mistake visible
        if (q < D.n_part)
            for (int j = 0; j < d; ++j) out[(size_t)j * D.n_part] = NAN;
        return;
    }
    const int64_t p = idx[(size_t)r * k + q];
    for (int j = 0; j < d; ++j) {
        double v;
        if (p >= 0 && p < S.n_part)
            v = src_theta[S.theta_off + (size_t)j * S.n_part + p];
        else
            v = src_lo[S.box_off + j];
        out[(size_t)j * k] = v;
    }
}

// ------------------------------------------------------------------- Adam
struct AdamArgs {
    const sird_problem *probs;
    const sird_tile *tiles;
    int n_tiles;
    double *theta;
    const double *grad;
    double *m;
    double *v;
    const double *lo;
    const double *hi;
    double lr, b1, b2, eps, bc1, bc2;
};

__global__ void __launch_bounds__(256) k_adam(AdamArgs a)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int t = wave_tile_index();
    if (t >= a.n_tiles) return;
    const sird_tile tl = a.tiles[t];
    const sird_problem P = a.probs[tl.prob];
    const int n = P.n_part;
    const int pl = tl.p0 + lane;
    if (pl >= n) return;
    const int d = P.n_seg + 3;
    for (int j = 0; j < d; ++j) {
        const double lo = a.lo[P.box_off + j];
        const double width = a.hi[P.box_off + j] - lo;
        if (!(width > 0.0)) continue;
        const size_t o = (size_t)P.theta_off + (size_t)j * n + pl;
        double u = (a.theta[o] - lo) / width;
        const double gu = a.grad[o] * width;
        const double m = a.b1 * a.m[o] + (1.0 - a.b1) * gu;
        const double v = a.b2 * a.v[o] + (1.0 - a.b2) * gu * gu;
        a.m[o] = m;
        a.v[o] = v;
        const double mhat = m / a.bc1;
        const double vhat = v / a.bc2;
        u = u - a.lr * mhat / (sqrt(vhat) + a.eps);
        if (u < 0.0) u = 0.0;
        if (u > 1.0) u = 1.0;
        a.theta[o] = lo + u * width;
    }
}

// ---------------------------------------------------------------- L-BFGS
constexpr int kLbfgsMaxM = 32;
constexpr int kLbfgsMaxTrials = 8;

struct LbfgsArgs {
    const sird_problem *probs;
    const sird_tile *tiles;
    int n_tiles;
    int per_tile;  // wavefronts per tile: min(64, the batch's max_part)
    int n_trials;  // trial points per vector and round
    int64_t theta_len;
    int64_t total_particles;
    lbfgs_state st;
    const double *lo;
    const double *hi;
    double c1;
};

// Box coordinate of dimension j: u = (phi(theta) - a)/w, phi the identity,
// or the logarithm for the last dimension when log_last is set; w = 0 marks
// a fixed dimension.
struct Coord {
    double a, w;
    bool lg;
};

__device__ __forceinline__ Coord coord_of(const double *lo, const double *hi, int j, int d,
                                          int log_last)
{
    Coord c;
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

__device__ __forceinline__ double to_u(const Coord &c, double th)
{
    if (c.w == 0.0) return 0.0;
    return ((c.lg ? log(th) : th) - c.a) / c.w;
}

__device__ __forceinline__ double from_u(const Coord &c, double u)
{
    const double v = c.a + u * c.w;
    return c.lg ? exp(v) : v;
}

__device__ __forceinline__ double grad_u(const Coord &c, double th, double g)
{
    return c.lg ? g * th * c.w : g * c.w;
}

// The double held by lane j (a uniform j) in every lane's scalar registers.
__device__ __forceinline__ double lane_value(double x, int j)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(x), j);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(x), j);
    return __hiloint2double(hi, lo);
}

// The double of lane j's partner under a DPP row permutation CTRL.
template <int CTRL>
__device__ __forceinline__ double dpp_partner(double x)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), CTRL, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}

// x_0 + x_1 + ... + x_{d-1} over lanes 0..d-1 (d <= 64), returned to every
// lane.  In the first power-of-two block w >= d, lanes d..w-1 add zeros and
// neighbours are added in pairs, then pairs of those, up to w: at each level
// a lane adds the value of the lane whose index differs in that bit, so all
// lanes of a block hold the same bits, the pairwise sum the oracle's dot
// products compute.  Within a row of 16 the partners come by DPP (after the
// first two levels a block of four holds one value, so mirroring within
// eight or sixteen lanes finds the same partner value as flipping bit 2 or
// 3).
__device__ __forceinline__ double pair_sum(double x, int d)
{
    const int lane = threadIdx.x & (kWave - 1);
    double s = lane < d ? x : 0.0;
    if (d > 1) s = s + dpp_partner<0xB1>(s);   // quad_perm [1,0,3,2]: bit 0
    if (d > 2) s = s + dpp_partner<0x4E>(s);   // quad_perm [2,3,0,1]: bit 1
    if (d > 4) s = s + dpp_partner<0x141>(s);  // row_half_mirror: bit 2
    if (d > 8) s = s + dpp_partner<0x140>(s);  // row_mirror: bit 3
    if (d > 16) s = s + __shfl_xor(s, 16);
    if (d > 32) s = s + __shfl_xor(s, 32);
    return lane_value(s, 0);  // lane 0's, uniform across the wavefront
}

// One wavefront per parameter vector, lane j for dimension j (d <= 64).  All
// stored pairs are loaded at once, and every dot product is summed across the
// lanes in pairs (pair_sum), the order the oracle's dot products take, without
// a memory round trip per pair.
__global__ void __launch_bounds__(256) k_lbfgs_propose(LbfgsArgs a)
{
    const int j = threadIdx.x & (kWave - 1);
    const int v = wave_tile_index();  // the vector: lane v % per_tile of tile v / per_tile
    const int t = v / a.per_tile;
    if (t >= a.n_tiles) return;
    const sird_tile tl = a.tiles[t];
    const sird_problem P = a.probs[tl.prob];
    const int pl = tl.p0 + v % a.per_tile;
    if (pl >= P.n_part) return;
    const int d = P.n_seg + 3;
    const bool on = j < d;
    const int m = a.st.m;
    const size_t n = (size_t)P.n_part;
    const size_t cj = (size_t)P.theta_off + (size_t)(on ? j : 0) * n + pl;
    const size_t pidx = (size_t)P.p_off + pl;
    const int lgl = a.st.log_last;
    const Coord c = coord_of(a.lo + P.box_off, a.hi + P.box_off, on ? j : 0, d, lgl);
    const double th = a.st.theta[cj];
    const double gu = grad_u(c, th, a.st.grad[cj]);
    int cnt = a.st.count[pidx];
    const int head = a.st.head[pidx];
    // the stored pairs, newest first: pair k in slot head - 1 - k (mod m).
    // All m slots of the memory are allocated, so every load reads a valid
    // slot and all are issued together, without branches; pairs past cnt
    // are zeroed afterwards.
    double Sk[kLbfgsMaxM], Yk[kLbfgsMaxM], rho[kLbfgsMaxM];
    {
        int slot = min(max(head, 0), m - 1);  // a valid state has 0 <= head < m
#pragma unroll
        for (int k = 0; k < kLbfgsMaxM; ++k) {
            slot = (slot == 0 ? m : slot) - 1;
            Sk[k] = a.st.S[(size_t)slot * a.theta_len + cj];
            Yk[k] = a.st.Y[(size_t)slot * a.theta_len + cj];
            rho[k] = a.st.rho[(size_t)slot * a.total_particles + pidx];
        }
#pragma unroll
        for (int k = 0; k < kLbfgsMaxM; ++k) {
            if (k >= cnt) Sk[k] = Yk[k] = rho[k] = 0.0;
        }
    }
    double r = gu;
    double coef[kLbfgsMaxM];
#pragma unroll
    for (int k = 0; k < kLbfgsMaxM; ++k) {  // newest to oldest
        coef[k] = 0.0;
        if (k < cnt) {
            coef[k] = rho[k] * pair_sum(Sk[k] * r, d);
            r = r - coef[k] * Yk[k];
        }
    }
    double h0 = 1.0;
    if (cnt > 0) {
        const double sy = pair_sum(Sk[0] * Yk[0], d);
        const double yy = pair_sum(Yk[0] * Yk[0], d);
        if (yy > 0.0) h0 = sy / yy;
    }
    r = h0 * r;
#pragma unroll
    for (int k = kLbfgsMaxM - 1; k >= 0; --k) {  // oldest to newest
        if (k < cnt) {
            const double b = rho[k] * pair_sum(Yk[k] * r, d);
            r = r + Sk[k] * (coef[k] - b);
        }
    }
    // direction p = -r, projected
    const double u = to_u(c, th);
    double p = -r;
    if (c.w == 0.0 || (u <= 0.0 && p < 0.0) || (u >= 1.0 && p > 0.0)) p = 0.0;
    double gp = pair_sum(gu * p, d);
    if (!(gp < 0.0)) {  // not a descent direction: steepest descent
        cnt = 0;
        p = -gu;
        if (c.w == 0.0 || (u <= 0.0 && p < 0.0) || (u >= 1.0 && p > 0.0)) p = 0.0;
        gp = pair_sum(gu * p, d);
    }
    double alpha = a.st.alpha[pidx];
    if (cnt == 0) {
        double pmax = 0.0;
        for (int i = 0; i < d; ++i) pmax = fmax(pmax, fabs(lane_value(p, i)));
        if (pmax > 0.0 && alpha * pmax > 0.01) alpha = 0.01 / pmax;
    }
    if (j == 0) {
        a.st.count[pidx] = cnt;
        a.st.alpha[pidx] = alpha;
        a.st.gp[pidx] = gp;
    }
    if (on) {
        // trial t at the step alpha 2^t, in the t-th theta-shaped block
        for (int tr = 0; tr < a.n_trials; ++tr) {
            const double at = alpha * (double)(1 << tr);
            double tt = th;
            if (c.w != 0.0) {
                double ut = u + at * p;
                if (ut < 0.0) ut = 0.0;
                if (ut > 1.0) ut = 1.0;
                tt = from_u(c, ut);
            }
            a.st.theta_t[(size_t)tr * a.theta_len + cj] = tt;
        }
    }
}

// A wavefront per parameter vector, lane j for dimension j, as the proposal:
// the Armijo test on every trial point, the one of lowest loss among those
// that pass (the first on ties), and on acceptance the new pair (kept when
// s.y > 0, s.y summed in pairs) and the step.
__global__ void __launch_bounds__(256) k_lbfgs_accept(LbfgsArgs a)
{
    const int j = threadIdx.x & (kWave - 1);
    const int v = wave_tile_index();
    const int t = v / a.per_tile;
    if (t >= a.n_tiles) return;
    const sird_tile tl = a.tiles[t];
    const sird_problem P = a.probs[tl.prob];
    const int pl = tl.p0 + v % a.per_tile;
    if (pl >= P.n_part) return;
    const int d = P.n_seg + 3;
    const bool on = j < d;
    const int m = a.st.m;
    const size_t n = (size_t)P.n_part;
    const size_t cj = (size_t)P.theta_off + (size_t)(on ? j : 0) * n + pl;
    const size_t pidx = (size_t)P.p_off + pl;
    const double alpha = a.st.alpha[pidx];
    const double f0 = a.st.f[pidx], gp = a.st.gp[pidx];
    int best = -1;
    double ft = 0.0;
    for (int tr = 0; tr < a.n_trials; ++tr) {
        const double at = alpha * (double)(1 << tr);
        const double fx = a.st.f_t[(size_t)tr * a.total_particles + pidx];
        if (isfinite(fx) && fx <= f0 + a.c1 * at * gp && (best < 0 || fx < ft)) {
            best = tr;
            ft = fx;
        }
    }
    if (best >= 0) {
        const Coord c =
            coord_of(a.lo + P.box_off, a.hi + P.box_off, on ? j : 0, d, a.st.log_last);
        const size_t ct = (size_t)best * a.theta_len + cj;
        const double tt = a.st.theta_t[ct], th = a.st.theta[cj];
        const double gt = a.st.grad_t[ct], g = a.st.grad[cj];
        const double sj = to_u(c, tt) - to_u(c, th);
        const double yj = grad_u(c, tt, gt) - grad_u(c, th, g);
        const double sy = pair_sum(sj * yj, d);
        const int head = a.st.head[pidx];
        if (sy > 0.0 && on) {
            a.st.S[(size_t)head * a.theta_len + cj] = sj;
            a.st.Y[(size_t)head * a.theta_len + cj] = yj;
        }
        if (on) {
            a.st.theta[cj] = tt;
            a.st.grad[cj] = gt;
        }
        if (j == 0) {
            if (sy > 0.0) {
                a.st.rho[(size_t)head * a.total_particles + pidx] = 1.0 / sy;
                a.st.head[pidx] = (head + 1) % m;
                if (a.st.count[pidx] < m) a.st.count[pidx] = a.st.count[pidx] + 1;
            }
            a.st.f[pidx] = ft;
            a.st.alpha[pidx] = 1.0;
        }
    } else if (j == 0) {
        const double half = 0.5 * alpha;
        if (half < 1e-20) {
            a.st.count[pidx] = 0;
            a.st.alpha[pidx] = 1.0;
        } else {
            a.st.alpha[pidx] = half;
        }
    }
}

static int check_lbfgs(const sird_batch *b, const lbfgs_state *st, const double *lo,
                       const double *hi, const char *who)
{
    int s = check_batch(b, who);
    if (s) return s;
    const std::string w(who);
    if (!st || !lo || !hi) return fail(SIRD_EINVAL, w + ": NULL argument");
    if (!st->theta || !st->grad || !st->f || !st->theta_t || !st->grad_t || !st->f_t ||
        !st->S || !st->Y || !st->rho || !st->alpha || !st->gp || !st->count || !st->head)
        return fail(SIRD_EINVAL, w + ": NULL state array");
    if (st->m < 1 || st->m > kLbfgsMaxM) return fail(SIRD_EINVAL, w + ": m must be in 1..32");
    if (st->log_last != 0 && st->log_last != 1)
        return fail(SIRD_EINVAL, w + ": log_last must be 0 or 1");
    if (st->n_trials < 0 || st->n_trials > kLbfgsMaxTrials)
        return fail(SIRD_EINVAL, w + ": n_trials must be in 0..8");
    if (b->max_d > 64) return fail(SIRD_EINVAL, w + ": d > 64");
    return SIRD_OK;
}

static LbfgsArgs lbfgs_args(const sird_batch *b, const lbfgs_state *st, const double *lo,
                            const double *hi, double c1)
{
    LbfgsArgs a{};
    a.probs = b->probs;
    a.tiles = b->tiles;
    a.n_tiles = b->n_tiles;
    // a tile holds particles p0 .. p0 + 63 of one problem, so no tile has
    // more vectors than the largest problem
    a.per_tile = (b->max_part > 0 && b->max_part < kWave) ? b->max_part : kWave;
    a.theta_len = b->theta_len;
    a.total_particles = b->total_particles;
    a.st = *st;
    a.n_trials = st->n_trials > 0 ? st->n_trials : 1;
    a.lo = lo;
    a.hi = hi;
    a.c1 = c1;
    return a;
}

}  // namespace sird

using namespace sird;

extern "C" int sird_lbfgs_propose(const sird_batch *batch, const lbfgs_state *state,
                                  const double *lo, const double *hi, void *stream)
{
    int st = check_lbfgs(batch, state, lo, hi, "sird_lbfgs_propose");
    if (st) return st;
    // a wavefront per parameter vector (per_tile per tile), four per block
    if (batch->n_tiles == 0) return SIRD_OK;
    const LbfgsArgs a = lbfgs_args(batch, state, lo, hi, 0.0);
    const int64_t waves = (int64_t)batch->n_tiles * a.per_tile;
    hipLaunchKernelGGL(k_lbfgs_propose, dim3((unsigned)((waves + 3) / 4)), dim3(4 * kWave), 0,
                       (hipStream_t)stream, a);
    return hip_status(hipGetLastError(), "sird_lbfgs_propose");
}

extern "C" int sird_lbfgs_accept(const sird_batch *batch, const lbfgs_state *state,
                                 const double *lo, const double *hi, double c1, void *stream)
{
    int st = check_lbfgs(batch, state, lo, hi, "sird_lbfgs_accept");
    if (st) return st;
    if (!(c1 > 0.0 && c1 < 1.0)) return fail(SIRD_EINVAL, "sird_lbfgs_accept: c1 outside (0,1)");
    // a wavefront per parameter vector (per_tile per tile), four per block
    if (batch->n_tiles == 0) return SIRD_OK;
    const LbfgsArgs a = lbfgs_args(batch, state, lo, hi, c1);
    const int64_t waves = (int64_t)batch->n_tiles * a.per_tile;
    hipLaunchKernelGGL(k_lbfgs_accept, dim3((unsigned)((waves + 3) / 4)), dim3(4 * kWave), 0,
                       (hipStream_t)stream, a);
    return hip_status(hipGetLastError(), "sird_lbfgs_accept");
}

extern "C" int pso_topk(const sird_batch *batch, const double *pbest_f, int k,
                        int64_t *idx_out, void *stream)
{
    int st = check_batch(batch, "pso_topk");
    if (st) return st;
    if (!pbest_f || !idx_out) return fail(SIRD_EINVAL, "pso_topk: NULL array");
    if (k < 1 || k > kTopkMax)
        return fail(SIRD_EINVAL, "pso_topk: k must be in [1, 65536]");
    hipStream_t s = (hipStream_t)stream;
    if (k <= kTopkRounds) {
        hipLaunchKernelGGL(k_topk, dim3(batch->n_prob), dim3(256), 0, s, batch->probs, pbest_f,
                           k, idx_out);
        return hip_status(hipGetLastError(), "pso_topk");
    }
    hipLaunchKernelGGL(k_topk_pad, dim3(batch->n_prob), dim3(256), 0, s, batch->probs, k,
                       idx_out);
    st = hip_status(hipGetLastError(), "pso_topk");
    if (st) return st;
    const int grid = tile_blocks(batch->n_tiles);
    if (grid == 0) return SIRD_OK;
    hipLaunchKernelGGL(k_topk_rank, dim3(grid), dim3(256), 0, s, batch->probs, batch->tiles,
                       batch->n_tiles, pbest_f, k, idx_out);
    return hip_status(hipGetLastError(), "pso_topk");
}

extern "C" int sird_gather(const sird_batch *src, const double *src_theta,
                           const double *src_lo, const sird_batch *dst, double *dst_theta,
                           const int64_t *idx, int k, void *stream)
{
    int st = check_batch(src, "sird_gather(src)");
    if (st) return st;
    st = check_batch(dst, "sird_gather(dst)");
    if (st) return st;
    if (!src_theta || !src_lo || !dst_theta || !idx)
        return fail(SIRD_EINVAL, "sird_gather: NULL array");
    if (src->n_prob != dst->n_prob)
        return fail(SIRD_EINVAL, "sird_gather: batches have different problem counts");
    if (k < 1 || (int64_t)k * dst->n_prob != dst->total_particles)
        return fail(SIRD_EINVAL, "sird_gather: dst must hold k particles per problem");
    const int64_t total = (int64_t)k * src->n_prob;
    const int grid = (int)((total + 255) / 256);
    hipLaunchKernelGGL(k_gather, dim3(grid), dim3(256), 0, (hipStream_t)stream, src->probs,
                       src_theta, src_lo, dst->probs, dst_theta, idx, k, src->n_prob);
    return hip_status(hipGetLastError(), "sird_gather");
}

extern "C" int sird_adam_step(const sird_batch *batch, double *theta, const double *grad,
                              double *m, double *v, const double *lo, const double *hi,
                              int64_t t, const adam_params *params, void *stream)
{
    int st = check_batch(batch, "sird_adam_step");
    if (st) return st;
    if (!theta || !grad || !m || !v || !lo || !hi || !params)
        return fail(SIRD_EINVAL, "sird_adam_step: NULL argument");
    if (t < 1) return fail(SIRD_EINVAL, "sird_adam_step: t must be >= 1");
    if (!(params->beta1 >= 0.0 && params->beta1 < 1.0 && params->beta2 >= 0.0 &&
          params->beta2 < 1.0 && params->eps >= 0.0 && std::isfinite(params->lr)))
        return fail(SIRD_EINVAL, "sird_adam_step: bad coefficients");
    AdamArgs a{};
    a.probs = batch->probs;
    a.tiles = batch->tiles;
    a.n_tiles = batch->n_tiles;
    a.theta = theta;
    a.grad = grad;
    a.m = m;
    a.v = v;
    a.lo = lo;
    a.hi = hi;
    a.lr = params->lr;
    a.b1 = params->beta1;
    a.b2 = params->beta2;
    a.eps = params->eps;
    a.bc1 = 1.0 - std::pow(params->beta1, (double)t);
    a.bc2 = 1.0 - std::pow(params->beta2, (double)t);
    const int grid = tile_blocks(batch->n_tiles);
    if (grid == 0) return SIRD_OK;
    hipLaunchKernelGGL(k_adam, dim3(grid), dim3(256), 0, (hipStream_t)stream, a);
    return hip_status(hipGetLastError(), "sird_adam_step");
}
