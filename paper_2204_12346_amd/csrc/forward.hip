// Forward integration kernels: RK4 over the calibration window of every
// particle, fused with the per-day cost (sird_loss) or writing the daily
// trajectory (sird_integrate).
//
// Mapping: one particle per lane, one tile (64 particles of one problem) per
// wavefront, so every loop bound is wavefront-uniform and lives in scalar
// registers.  The whole state stays in VGPRs; per day the wavefront reads one
// (y_i, 1/max(y_i,1)) pair that it staged in its own LDS slice at the start of
// the tile.  Tiles are ordered longest-first; with persistent > 0 a fixed set
// of resident wavefronts pulls tiles from a device counter instead of relying
// on the dispatcher's order.
#include <hip/hip_runtime.h>

#include <string>

#include "device.h"
#include "internal.h"

namespace sird {

struct FwdArgs {
    const sird_problem *probs;
    const sird_tile *tiles;
    int32_t *sched;
    const double *theta;
    const double *obs;
    double *loss;
    double *traj;
    int n_tiles;
    int n_waves;   // resident wavefronts of a persistent launch, else 0
    int loss_kind;
    int lds_stride;  // doubles per wavefront slice: 2 * (max_days + 1)
    // swarm fused into the integration (sird_pso_iterate): theta is the
    // swarm's x, loss its f; before integrating, a particle is moved with
    // counter iter[0] - 1 when do_move; after, its personal best is updated
    PsoMove mv;
    double *pbest_f;
    double *pbest_x;
    const uint64_t *iter;
    int do_move;
};

// S, I, R, D of one day into a [4][W+1][n] trajectory block.
template <typename R>
__device__ __forceinline__ void store_day(double *o, size_t comp_stride, const SirdState<R> &y)
{
    o[0] = state_value(y.S, y.eS);
    o[comp_stride] = state_value(y.I, y.eI);
    o[2 * comp_stride] = state_value(y.Rr, y.eR);
    o[3 * comp_stride] = state_value(y.D, y.eD);
}

template <typename R, bool TRAJ, bool FUSED>
__device__ __forceinline__ void fwd_tile(const FwdArgs &a, int t, int lane, double *ly,
                                         double *lw)
{
    const sird_tile tl = a.tiles[t];
    const sird_problem P = a.probs[tl.prob];
    const int W = P.n_days, spd = P.steps_per_day, seg = P.seg_days, K = P.n_seg;
    const int n = P.n_part;
    const int pl = tl.p0 + lane;
    const bool active = pl < n;
    const int pc = active ? pl : n - 1;  // idle lanes integrate a valid column
    const size_t ld = (size_t)n;
    const double *th = a.theta + P.theta_off + pc;

    if (!TRAJ) {
        const double *y = a.obs + P.obs_off;
        for (int i = lane; i <= W; i += kWave) {
            const double yi = y[i];
            ly[i] = yi;
            lw[i] = 1.0 / fmax(yi, 1.0);
        }
        wave_sync();
    }
    if (FUSED && a.do_move && active) pso_move_particle(a.mv, P, pl, a.iter[0] - 1);

    const double gamma = th[(size_t)K * ld];
    const double mu = th[(size_t)(K + 1) * ld];
    const double I0 = th[(size_t)(K + 2) * ld];
    const double N = P.N;
    StepConst<R> sc = step_const<R>(gamma, mu, spd);

    SirdState<R> y;
    y.S = (R)(N - I0 - P.R0 - P.D0);
    y.I = (R)I0;
    y.Rr = (R)P.R0;
    y.D = (R)P.D0;
    y.s = R(0);
    y.eS = y.eI = y.eR = y.eD = R(0);

    double acc = 0.0;
    double *tr = nullptr;
    const size_t comp_stride = (size_t)(W + 1) * ld;
    if (TRAJ) {
        tr = a.traj + P.traj_off + pc;
        if (active) store_day(tr, comp_stride, y);
    } else {
        cost_accum(a.loss_kind, acc, state_value(y.D, y.eD), ly[0], lw[0], 0);
    }

    int day = 0;
    double beta_next = th[0];
    for (int k = 0; k < K; ++k) {
        const double beta_k = beta_next;
        if (k + 1 < K) beta_next = th[(size_t)(k + 1) * ld];  // prefetch
        const int dend = (k == K - 1) ? W : min(W, (k + 1) * seg);
        if (day >= dend) continue;
        set_beta(sc, beta_k, N);
        for (; day < dend; ++day) {
            rescale(y, sc);
#pragma unroll 2
            for (int s = 0; s < spd; ++s) rk4_step<R, TRAJ>(y, sc);
            const int i = day + 1;
            if (TRAJ) {
                if (active) store_day(tr + (size_t)i * ld, comp_stride, y);
            } else {
                cost_accum(a.loss_kind, acc, state_value(y.D, y.eD), ly[i], lw[i], i);
            }
        }
    }
    if (!TRAJ && active) {
        const double L = cost_finish(a.loss_kind, acc, W);
        a.loss[P.p_off + pl] = L;
        if (FUSED) pso_pbest_particle(L, P, pl, a.pbest_f, a.pbest_x, a.mv.x);
    }
    if (!TRAJ) wave_sync();  // LDS slice reads done before it is restaged
}

template <typename R, bool TRAJ, bool FUSED>
__global__ void __launch_bounds__(1024) k_forward(FwdArgs a)
{
    extern __shared__ double lds[];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    double *ly = lds + (size_t)wave * a.lds_stride;
    double *lw = ly + a.lds_stride / 2;
    if (a.n_waves > 0) {
        for (;;) {
            int t = 0;
            if (lane == 0) t = atomicAdd(&a.sched[0], 1);
            t = wave_uniform(t);
            if (t >= a.n_tiles) break;
            fwd_tile<R, TRAJ, FUSED>(a, t, lane, ly, lw);
        }
        // The last wavefront out resets the counters for the next launch.
        if (lane == 0) {
            __threadfence();
            const int done = atomicAdd(&a.sched[1], 1);
            if (done == a.n_waves - 1) {
                atomicExch(&a.sched[0], 0);
                atomicExch(&a.sched[1], 0);
            }
        }
    } else {
        const int t = wave_tile_index();
        if (t < a.n_tiles) fwd_tile<R, TRAJ, FUSED>(a, t, lane, ly, lw);
    }
}

template <typename R, bool TRAJ, bool FUSED = false>
static int launch_forward(const sird_batch *b, FwdArgs a, hipStream_t s, const char *who)
{
    const int block = integ_block(b);
    const int wpb = block / kWave;
    a.lds_stride = 2 * (b->max_days + 1);
    const size_t lds = TRAJ ? 0 : (size_t)wpb * a.lds_stride * sizeof(double);
    if (lds > 65536)
        return fail(SIRD_EINVAL, std::string(who) +
                                     ": block too large for the window length (LDS > 64 KiB)");
    int grid;
    if (b->persistent > 0) {
        grid = (b->persistent + wpb - 1) / wpb;
        a.n_waves = grid * wpb;
    } else {
        grid = (a.n_tiles + wpb - 1) / wpb;
        a.n_waves = 0;
    }
    if (grid == 0) return SIRD_OK;
    hipLaunchKernelGGL((k_forward<R, TRAJ, FUSED>), dim3(grid), dim3(block), lds, s, a);
    return hip_status(hipGetLastError(), who);
}

int forward_loss(const sird_batch *b, const double *theta, const double *obs, int kind,
                 double *loss, hipStream_t s)
{
    FwdArgs a{};
    a.probs = b->probs;
    a.tiles = b->tiles;
    a.sched = b->sched;
    a.theta = theta;
    a.obs = obs;
    a.loss = loss;
    a.n_tiles = b->n_tiles;
    a.loss_kind = kind;
    if (b->dtype == SIRD_F32) return launch_forward<float, false>(b, a, s, "sird_loss");
    return launch_forward<double, false>(b, a, s, "sird_loss");
}

int forward_iterate(const sird_batch *b, const PsoMove &mv, const pso_state *st,
                    const double *obs, int kind, bool move, hipStream_t s)
{
    FwdArgs a{};
    a.probs = b->probs;
    a.tiles = b->tiles;
    a.sched = b->sched;
    a.theta = st->x;
    a.obs = obs;
    a.loss = st->f;
    a.n_tiles = b->n_tiles;
    a.loss_kind = kind;
    a.mv = mv;
    a.pbest_f = st->pbest_f;
    a.pbest_x = st->pbest_x;
    a.iter = st->iter;
    a.do_move = move ? 1 : 0;
    if (b->dtype == SIRD_F32) return launch_forward<float, false, true>(b, a, s, "sird_pso_iterate");
    return launch_forward<double, false, true>(b, a, s, "sird_pso_iterate");
}

}  // namespace sird

using namespace sird;

extern "C" int sird_loss(const sird_batch *batch, const double *theta, const double *obs,
                         int loss_kind, double *loss, void *stream)
{
    int st = check_batch(batch, "sird_loss");
    if (st) return st;
    if (!theta || !obs || !loss) return fail(SIRD_EINVAL, "sird_loss: NULL array");
    if (loss_kind < SIRD_LOSS_SSRE || loss_kind > SIRD_LOSS_MAPE)
        return fail(SIRD_EINVAL, "sird_loss: unknown loss_kind");
    if (batch->obs_len < 1) return fail(SIRD_EINVAL, "sird_loss: batch planned without obs");
    return forward_loss(batch, theta, obs, loss_kind, loss, (hipStream_t)stream);
}

extern "C" int sird_integrate(const sird_batch *batch, const double *theta, double *traj,
                              void *stream)
{
    int st = check_batch(batch, "sird_integrate");
    if (st) return st;
    if (!theta || !traj) return fail(SIRD_EINVAL, "sird_integrate: NULL array");
    if (batch->traj_len < 1)
        return fail(SIRD_EINVAL, "sird_integrate: batch planned without traj");
    FwdArgs a{};
    a.probs = batch->probs;
    a.tiles = batch->tiles;
    a.sched = batch->sched;
    a.theta = theta;
    a.traj = traj;
    a.n_tiles = batch->n_tiles;
    hipStream_t s = (hipStream_t)stream;
    if (batch->dtype == SIRD_F32) return launch_forward<float, true>(batch, a, s, "sird_integrate");
    return launch_forward<double, true>(batch, a, s, "sird_integrate");
}
