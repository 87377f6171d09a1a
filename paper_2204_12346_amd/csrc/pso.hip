// Particle swarm kernels (Sec. 3.3): initialisation, personal bests, the
// per-problem global argmin, and the velocity/position update with Philox
// random numbers.  The update is written as separately rounded multiplies
// and adds (the library is compiled without contraction), so it is bitwise
// reproducible given equal inputs.
//
// Launch shapes: the per-particle kernels run one wavefront per 64-particle
// tile (the same tiles as the integration); the argmin runs one 256-thread
// block per problem and reduces with cross-lane shuffles, then through LDS.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>

#include "device.h"
#include "internal.h"

namespace sird {

struct PsoArgs {
    const sird_problem *probs;
    const sird_tile *tiles;
    int n_tiles;
    int n_prob;
    double w, c1, c2;
    uint64_t seed;
    const double *lo;
    const double *hi;
    pso_state st;
};

static PsoArgs make_args(const sird_batch *b, const pso_params *p, const pso_state *st)
{
    PsoArgs a{};
    a.probs = b->probs;
    a.tiles = b->tiles;
    a.n_tiles = b->n_tiles;
    a.n_prob = b->n_prob;
    a.w = p->w;
    a.c1 = p->c1;
    a.c2 = p->c2;
    a.seed = p->seed;
    a.lo = p->lo;
    a.hi = p->hi;
    a.st = *st;
    return a;
}

__global__ void __launch_bounds__(256) k_pso_init(PsoArgs a)
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
    const double *lo = a.lo + P.box_off;
    const double *hi = a.hi + P.box_off;
    const size_t base = (size_t)P.theta_off + pl;
    for (int m = 0; 2 * m < d; ++m) {
        const Philox4x64 r = philox4x64_10(0, (uint64_t)pl, (uint64_t)m, 0, a.seed, P.stream);
        for (int jj = 0; jj < 2; ++jj) {
            const int j = 2 * m + jj;
            if (j >= d) break;
            const double u = u01(r.w[2 * jj]);
            const double x = lo[j] + u * (hi[j] - lo[j]);
            const size_t o = base + (size_t)j * n;
            a.st.x[o] = x;
            a.st.v[o] = 0.0;
            a.st.pbest_x[o] = x;
        }
    }
    a.st.pbest_f[P.p_off + pl] = INFINITY;
}

__global__ void __launch_bounds__(256) k_pso_init_problems(PsoArgs a)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r == 0) {
        a.st.iter[0] = 0;
        a.st.iter[1] = 0;
    }
    if (r >= a.n_prob) return;
    const sird_problem P = a.probs[r];
    const int d = P.n_seg + 3;
    for (int j = 0; j < d; ++j) a.st.gbest_x[P.box_off + j] = a.lo[P.box_off + j];
    a.st.gbest_f[r] = INFINITY;
    a.st.gbest_idx[r] = -1;
}

// Personal bests: strict improvement, NaN counts as +inf.
__global__ void __launch_bounds__(256) k_pso_pbest(PsoArgs a)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int t = wave_tile_index();
    if (t >= a.n_tiles) return;
    const sird_tile tl = a.tiles[t];
    const sird_problem P = a.probs[tl.prob];
    const int n = P.n_part;
    const int pl = tl.p0 + lane;
    if (pl >= n) return;
    double f = a.st.f[P.p_off + pl];
    if (f != f) f = INFINITY;
    if (f < a.st.pbest_f[P.p_off + pl]) {
        a.st.pbest_f[P.p_off + pl] = f;
        const int d = P.n_seg + 3;
        const size_t base = (size_t)P.theta_off + pl;
        for (int j = 0; j < d; ++j) a.st.pbest_x[base + (size_t)j * n] = a.st.x[base + (size_t)j * n];
    }
}

// (f, index) lexicographic order: lowest index wins ties.
__device__ __forceinline__ bool better(double f, int i, double bf, int bi)
{
    return f < bf || (f == bf && i < bi);
}

// Global best of one problem per block: argmin of pbest_f, then replace the
// previous global best only on strict improvement, and record the history.
__global__ void __launch_bounds__(256) k_pso_gbest(PsoArgs a)
{
    __shared__ double sf[256 / kWave];
    __shared__ int si[256 / kWave];
    __shared__ int s_take;
    const int r = blockIdx.x;
    const sird_problem P = a.probs[r];
    const int n = P.n_part;
    const int tid = threadIdx.x;
    double bf = INFINITY;
    int bi = n;  // sentinel above every index
    for (int p = tid; p < n; p += blockDim.x) {
        const double f = a.st.pbest_f[P.p_off + p];
        if (better(f, p, bf, bi)) {
            bf = f;
            bi = p;
        }
    }
    for (int off = kWave / 2; off > 0; off >>= 1) {
        const double of = __shfl_xor(bf, off);
        const int oi = __shfl_xor(bi, off);
        if (better(of, oi, bf, bi)) {
            bf = of;
            bi = oi;
        }
    }
    if ((tid & (kWave - 1)) == 0) {
        sf[tid / kWave] = bf;
        si[tid / kWave] = bi;
    }
    __syncthreads();
    const uint64_t it = a.st.iter[0];
    if (tid == 0) {
        for (int k = 1; k < (int)(blockDim.x / kWave); ++k)
            if (better(sf[k], si[k], bf, bi)) {
                bf = sf[k];
                bi = si[k];
            }
        int take = 0;
        if (n > 0 && bi < n && bf < a.st.gbest_f[r]) {
            a.st.gbest_f[r] = bf;
            a.st.gbest_idx[r] = bi;
            take = 1;
        }
        s_take = take;
        si[0] = bi;
        if (a.st.hist_f && (int64_t)it < a.st.hist_len) {
            a.st.hist_f[(size_t)it * a.n_prob + r] = a.st.gbest_f[r];
            if (a.st.hist_idx) a.st.hist_idx[(size_t)it * a.n_prob + r] = a.st.gbest_idx[r];
        }
    }
    __syncthreads();
    if (s_take) {
        const int d = P.n_seg + 3;
        const int b = si[0];
        for (int j = tid; j < d; j += blockDim.x)
            a.st.gbest_x[P.box_off + j] = a.st.pbest_x[(size_t)P.theta_off + (size_t)j * n + b];
    }
}

// Velocity and position update, then the last block advances the iteration.
__global__ void __launch_bounds__(256) k_pso_move(PsoArgs a)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int t = wave_tile_index();
    const uint64_t it = a.st.iter[0];
    if (t < a.n_tiles) {
        const sird_tile tl = a.tiles[t];
        const sird_problem P = a.probs[tl.prob];
        const int n = P.n_part;
        const int pl = tl.p0 + lane;
        if (pl < n) {
            const int d = P.n_seg + 3;
            const double *lo = a.lo + P.box_off;
            const double *hi = a.hi + P.box_off;
            const double *g = a.st.gbest_x + P.box_off;
            const size_t base = (size_t)P.theta_off + pl;
            for (int m = 0; 2 * m < d; ++m) {
                const Philox4x64 r =
                    philox4x64_10(it, (uint64_t)pl, (uint64_t)m, 1, a.seed, P.stream);
                for (int jj = 0; jj < 2; ++jj) {
                    const int j = 2 * m + jj;
                    if (j >= d) break;
                    const double r1 = u01(r.w[2 * jj]);
                    const double r2 = u01(r.w[2 * jj + 1]);
                    const size_t o = base + (size_t)j * n;
                    const double xo = a.st.x[o];
                    double tv = a.w * a.st.v[o];
                    const double a1 = a.c1 * r1;
                    const double d1 = a.st.pbest_x[o] - xo;
                    const double a2 = a.c2 * r2;
                    const double d2 = g[j] - xo;
                    const double m1 = a1 * d1;
                    tv = tv + m1;
                    const double m2 = a2 * d2;
                    tv = tv + m2;
                    a.st.v[o] = tv;
                    double xn = xo + tv;
                    if (xn < lo[j]) xn = lo[j];
                    if (xn > hi[j]) xn = hi[j];
                    a.st.x[o] = xn;
                }
            }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const unsigned long long done =
            atomicAdd((unsigned long long *)&a.st.iter[1], 1ull);
        if (done == (unsigned long long)gridDim.x - 1) {
            atomicExch((unsigned long long *)&a.st.iter[1], 0ull);
            atomicExch((unsigned long long *)&a.st.iter[0], (unsigned long long)(it + 1));
        }
    }
}

static int check_pso(const sird_batch *b, const pso_params *p, const pso_state *st,
                     const char *who)
{
    int s = check_batch(b, who);
    if (s) return s;
    const std::string w(who);
    if (!p || !st) return fail(SIRD_EINVAL, w + ": params or state is NULL");
    if (!p->lo || !p->hi) return fail(SIRD_EINVAL, w + ": lo/hi is NULL");
    if (!st->x || !st->v || !st->pbest_x || !st->pbest_f || !st->gbest_x || !st->gbest_f ||
        !st->gbest_idx || !st->iter)
        return fail(SIRD_EINVAL, w + ": NULL swarm array");
    if (!std::isfinite(p->w) || !std::isfinite(p->c1) || !std::isfinite(p->c2))
        return fail(SIRD_EINVAL, w + ": non-finite coefficient");
    if (st->hist_len < 0) return fail(SIRD_EINVAL, w + ": hist_len < 0");
    if (st->hist_len > 0 && !st->hist_f) return fail(SIRD_EINVAL, w + ": hist_f is NULL");
    return SIRD_OK;
}

int pso_step_enqueue(const sird_batch *b, const pso_params *p, const pso_state *st,
                     hipStream_t s)
{
    PsoArgs a = make_args(b, p, st);
    const int tb = tile_blocks(b->n_tiles);
    if (tb > 0) hipLaunchKernelGGL(k_pso_pbest, dim3(tb), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_pso_gbest, dim3(b->n_prob), dim3(256), 0, s, a);
    // The move kernel always runs (at least one block) so the iteration
    // counter advances even for a batch without particles.
    hipLaunchKernelGGL(k_pso_move, dim3(tb > 0 ? tb : 1), dim3(256), 0, s, a);
    return hip_status(hipGetLastError(), "pso_step");
}

int forward_loss(const sird_batch *b, const double *theta, const double *obs, int kind,
                 double *loss, hipStream_t s);

int pso_iterate_enqueue(const sird_batch *b, const pso_params *p, const pso_state *st,
                        const double *obs, int kind, int n_iters, hipStream_t s)
{
    for (int i = 0; i < n_iters; ++i) {
        int r = forward_loss(b, st->x, obs, kind, st->f, s);
        if (r) return r;
        r = pso_step_enqueue(b, p, st, s);
        if (r) return r;
    }
    return SIRD_OK;
}

int check_iterate(const sird_batch *b, const pso_params *p, const pso_state *st,
                  const double *obs, int kind, int n_iters, const char *who)
{
    int r = check_pso(b, p, st, who);
    if (r) return r;
    const std::string w(who);
    if (!st->f) return fail(SIRD_EINVAL, w + ": state->f is NULL");
    if (!obs) return fail(SIRD_EINVAL, w + ": obs is NULL");
    if (b->obs_len < 1) return fail(SIRD_EINVAL, w + ": batch planned without obs");
    if (kind < SIRD_LOSS_SSRE || kind > SIRD_LOSS_MAPE)
        return fail(SIRD_EINVAL, w + ": unknown loss_kind");
    if (n_iters < 0) return fail(SIRD_EINVAL, w + ": n_iters < 0");
    return SIRD_OK;
}

}  // namespace sird

using namespace sird;

extern "C" int pso_init(const sird_batch *batch, const pso_params *params,
                        const pso_state *state, void *stream)
{
    int r = check_pso(batch, params, state, "pso_init");
    if (r) return r;
    hipStream_t s = (hipStream_t)stream;
    PsoArgs a = make_args(batch, params, state);
    const int tb = tile_blocks(batch->n_tiles);
    if (tb > 0) hipLaunchKernelGGL(k_pso_init, dim3(tb), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_pso_init_problems, dim3((batch->n_prob + 255) / 256), dim3(256), 0, s,
                       a);
    return hip_status(hipGetLastError(), "pso_init");
}

extern "C" int pso_step(const sird_batch *batch, const pso_params *params,
                        const pso_state *state, void *stream)
{
    int r = check_pso(batch, params, state, "pso_step");
    if (r) return r;
    if (!state->f) return fail(SIRD_EINVAL, "pso_step: state->f is NULL");
    return pso_step_enqueue(batch, params, state, (hipStream_t)stream);
}

extern "C" int sird_pso_iterate(const sird_batch *batch, const pso_params *params,
                                const pso_state *state, const double *obs, int loss_kind,
                                int n_iters, void *stream)
{
    int r = check_iterate(batch, params, state, obs, loss_kind, n_iters, "sird_pso_iterate");
    if (r) return r;
    return pso_iterate_enqueue(batch, params, state, obs, loss_kind, n_iters,
                               (hipStream_t)stream);
}
