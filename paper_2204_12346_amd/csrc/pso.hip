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
    int it_back;       // the move uses counter iter[0] - it_back
    int move_advance;  // the move kernel advances iter[0] (else it does not)
    int gbest_advance; // the global-best kernel advances iter[0]
};

__host__ __device__ static PsoMove move_of(const PsoArgs &a)
{
    PsoMove m;
    m.w = a.w;
    m.c1 = a.c1;
    m.c2 = a.c2;
    m.seed = a.seed;
    m.lo = a.lo;
    m.hi = a.hi;
    m.x = a.st.x;
    m.v = a.st.v;
    m.pbest_x = a.st.pbest_x;
    m.gbest_x = a.st.gbest_x;
    return m;
}

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
    a.it_back = 0;
    a.move_advance = 1;
    a.gbest_advance = 0;
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
    if (P.model == SIRD_MODEL_EULER_RAMP) {
        ramp_order(a.st.x, P, pl);
        ramp_order(a.st.pbest_x, P, pl);
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
    const int pl = tl.p0 + lane;
    if (pl >= P.n_part) return;
    pso_pbest_particle(a.st.f[P.p_off + pl], P, pl, a.st.pbest_f, a.st.pbest_x, a.st.x);
}

// (f, index) lexicographic order: lowest index wins ties.
__device__ __forceinline__ bool better(double f, int i, double bf, int bi)
{
    return f < bf || (f == bf && i < bi);
}

// Global best of a problem: argmin of pbest_f (lowest index among equal
// values), then replace the previous global best only on strict
// improvement, and record the history.

// Strided argmin over pbest_f of one problem, with up to 8 loads in flight.
__device__ __forceinline__ void gbest_scan(const double *f, int n, int first, int stride,
                                           double &bf, int &bi)
{
    bf = INFINITY;
    bi = n;  // sentinel above every index
#pragma unroll 16
    for (int p = first; p < n; p += stride) {
        const double v = f[p];
        if (better(v, p, bf, bi)) {
            bf = v;
            bi = p;
        }
    }
}

// Butterfly over the wavefront: every lane ends with the wavefront's argmin.
__device__ __forceinline__ void wave_argmin(double &bf, int &bi)
{
    for (int off = kWave / 2; off > 0; off >>= 1) {
        const double of = __shfl_xor(bf, off);
        const int oi = __shfl_xor(bi, off);
        if (better(of, oi, bf, bi)) {
            bf = of;
            bi = oi;
        }
    }
}

// Compare the problem's argmin (bf, bi) with its global best and record the
// history row of iteration it; one thread.  Returns whether bi was taken.
__device__ __forceinline__ bool gbest_commit(const PsoArgs &a, int r, int n, double bf, int bi,
                                             uint64_t it)
{
    bool take = false;
    if (n > 0 && bi < n && bf < a.st.gbest_f[r]) {
        a.st.gbest_f[r] = bf;
        a.st.gbest_idx[r] = bi;
        take = true;
    }
    if (a.st.hist_f && (int64_t)it < a.st.hist_len) {
        a.st.hist_f[(size_t)it * a.n_prob + r] = a.st.gbest_f[r];
        if (a.st.hist_idx) a.st.hist_idx[(size_t)it * a.n_prob + r] = a.st.gbest_idx[r];
    }
    return take;
}

// After every block has read iter[0] (= it): advance it once.  One thread
// per block; the block must have passed a barrier after its read.
__device__ __forceinline__ void gbest_advance_iteration(const PsoArgs &a, uint64_t it)
{
    if (gridDim.x == 1) {
        // this block is the only reader
        a.st.iter[0] = it + 1;
        return;
    }
    // the last block out advances the iteration
    __threadfence();
    const unsigned long long done = atomicAdd((unsigned long long *)&a.st.iter[1], 1ull);
    if (done == (unsigned long long)gridDim.x - 1) {
        atomicExch((unsigned long long *)&a.st.iter[1], 0ull);
        atomicExch((unsigned long long *)&a.st.iter[0], (unsigned long long)(it + 1));
    }
}

// Problems of more than kGbestWaveMax particles: one block per problem,
// 1024 threads, so that ten thousand particles cost about two memory
// latencies.
constexpr int kGbestBlock = 1024;
// Smaller problems: one wavefront per problem and sixteen problems per block,
// so that a batch of many problems needs few blocks (every block takes one
// same-address atomic to advance the iteration, and those serialise).
constexpr int kGbestWaveMax = 4096;
constexpr int kGbestWaveBlock = 1024;

__global__ void __launch_bounds__(kGbestBlock) k_pso_gbest(PsoArgs a)
{
    __shared__ double sf[kGbestBlock / kWave];
    __shared__ int si[kGbestBlock / kWave];
    __shared__ int s_take;
    const int r = blockIdx.x;
    const sird_problem P = a.probs[r];
    const int n = P.n_part;
    const int tid = threadIdx.x;
    double bf;
    int bi;
    gbest_scan(a.st.pbest_f + P.p_off, n, tid, blockDim.x, bf, bi);
    wave_argmin(bf, bi);
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
        s_take = gbest_commit(a, r, n, bf, bi, it) ? 1 : 0;
        si[0] = bi;
    }
    __syncthreads();
    if (s_take) {
        const int d = P.n_seg + 3;
        const int b = si[0];
        for (int j = tid; j < d; j += blockDim.x)
            a.st.gbest_x[P.box_off + j] = a.st.pbest_x[(size_t)P.theta_off + (size_t)j * n + b];
    }
    if (a.gbest_advance && tid == 0) gbest_advance_iteration(a, it);
}

__global__ void __launch_bounds__(kGbestWaveBlock) k_pso_gbest_waves(PsoArgs a)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int r = (int)(blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave);
    const uint64_t it = a.st.iter[0];
    if (r < a.n_prob) {
        const sird_problem P = a.probs[r];
        const int n = P.n_part;
        double bf;
        int bi;
        gbest_scan(a.st.pbest_f + P.p_off, n, lane, kWave, bf, bi);
        wave_argmin(bf, bi);
        int take = 0;
        if (lane == 0) take = gbest_commit(a, r, n, bf, bi, it) ? 1 : 0;
        if (wave_uniform(take)) {
            const int d = P.n_seg + 3;
            for (int j = lane; j < d; j += kWave)
                a.st.gbest_x[P.box_off + j] =
                    a.st.pbest_x[(size_t)P.theta_off + (size_t)j * n + bi];
        }
    }
    if (!a.gbest_advance) return;
    __syncthreads();
    if (threadIdx.x == 0) gbest_advance_iteration(a, it);
}

static int launch_gbest(const sird_batch *b, const PsoArgs &a, hipStream_t s)
{
    if (b->max_part <= kGbestWaveMax) {
        const int ppb = kGbestWaveBlock / kWave;
        hipLaunchKernelGGL(k_pso_gbest_waves, dim3((b->n_prob + ppb - 1) / ppb),
                           dim3(kGbestWaveBlock), 0, s, a);
    } else {
        hipLaunchKernelGGL(k_pso_gbest, dim3(b->n_prob), dim3(kGbestBlock), 0, s, a);
    }
    return SIRD_OK;
}

// Velocity and position update with counter iter[0] - it_back; then, if
// move_advance, the last block advances the iteration.
__global__ void __launch_bounds__(256) k_pso_move(PsoArgs a)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int t = wave_tile_index();
    const uint64_t it0 = a.st.iter[0];
    const uint64_t it = it0 - (uint64_t)a.it_back;
    if (t < a.n_tiles) {
        const sird_tile tl = a.tiles[t];
        const sird_problem P = a.probs[tl.prob];
        const int pl = tl.p0 + lane;
        if (pl < P.n_part) pso_move_particle(move_of(a), P, pl, it);
    }
    if (!a.move_advance) return;
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const unsigned long long done =
            atomicAdd((unsigned long long *)&a.st.iter[1], 1ull);
        if (done == (unsigned long long)gridDim.x - 1) {
            atomicExch((unsigned long long *)&a.st.iter[1], 0ull);
            atomicExch((unsigned long long *)&a.st.iter[0], (unsigned long long)(it0 + 1));
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
    launch_gbest(b, a, s);
    // The move kernel always runs (at least one block) so the iteration
    // counter advances even for a batch without particles.
    hipLaunchKernelGGL(k_pso_move, dim3(tb > 0 ? tb : 1), dim3(256), 0, s, a);
    return hip_status(hipGetLastError(), "pso_step");
}

int forward_iterate(const sird_batch *b, const PsoMove &mv, const pso_state *st,
                    const double *obs, int kind, bool move, hipStream_t s);

// n_iters iterations with the swarm fused into the integration kernel:
// iteration i integrates x (first moving it with the previous iteration's
// counter when i > 0) and updates the personal bests in the same kernel,
// then the global-best kernel advances the iteration; a final move kernel
// completes the last iteration without advancing the counter.  The result
// is bitwise that of n_iters x [sird_loss; pso_step].
static int evaluate_enqueue(const sird_batch *b, const pso_params *p, const pso_state *st,
                            const double *obs, int kind, bool move_first, hipStream_t s)
{
    PsoArgs a = make_args(b, p, st);
    return forward_iterate(b, move_of(a), st, obs, kind, move_first, s);
}

static int gbest_enqueue(const sird_batch *b, const pso_params *p, const pso_state *st,
                         hipStream_t s)
{
    PsoArgs a = make_args(b, p, st);
    a.gbest_advance = 1;
    launch_gbest(b, a, s);
    return hip_status(hipGetLastError(), "pso_gbest");
}

static int complete_move_enqueue(const sird_batch *b, const pso_params *p,
                                 const pso_state *st, hipStream_t s)
{
    PsoArgs a = make_args(b, p, st);
    a.it_back = 1;
    a.move_advance = 0;
    const int tb = tile_blocks(b->n_tiles);
    if (tb > 0) hipLaunchKernelGGL(k_pso_move, dim3(tb), dim3(256), 0, s, a);
    return hip_status(hipGetLastError(), "pso_complete_move");
}

int pso_iterate_enqueue(const sird_batch *b, const pso_params *p, const pso_state *st,
                        const double *obs, int kind, int n_iters, hipStream_t s)
{
    if (n_iters <= 0) return SIRD_OK;
    for (int i = 0; i < n_iters; ++i) {
        int r = evaluate_enqueue(b, p, st, obs, kind, i > 0, s);
        if (r) return r;
        r = gbest_enqueue(b, p, st, s);
        if (r) return r;
    }
    return complete_move_enqueue(b, p, st, s);
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
    r = check_kind(b, kind, who);
    if (r) return r;
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

extern "C" int pso_evaluate(const sird_batch *batch, const pso_params *params,
                            const pso_state *state, const double *obs, int loss_kind,
                            int move_first, void *stream)
{
    int r = check_iterate(batch, params, state, obs, loss_kind, 1, "pso_evaluate");
    if (r) return r;
    return evaluate_enqueue(batch, params, state, obs, loss_kind, move_first != 0,
                            (hipStream_t)stream);
}

extern "C" int pso_gbest(const sird_batch *batch, const pso_params *params,
                         const pso_state *state, void *stream)
{
    int r = check_pso(batch, params, state, "pso_gbest");
    if (r) return r;
    return gbest_enqueue(batch, params, state, (hipStream_t)stream);
}

extern "C" int pso_complete_move(const sird_batch *batch, const pso_params *params,
                                 const pso_state *state, void *stream)
{
    int r = check_pso(batch, params, state, "pso_complete_move");
    if (r) return r;
    return complete_move_enqueue(batch, params, state, (hipStream_t)stream);
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
