// Forward integration kernels: the model of every particle over its
// calibration window (RK4 with piecewise-constant beta, or the paper's
// forward Euler with the ramp of eq. (beta)), fused with the per-day cost
// (sird_loss, the swarm iteration) or writing the daily trajectory
// (sird_integrate).
//
// Mapping: one particle per lane, one tile (64 particles of one problem) per
// wavefront, so every loop bound is wavefront-uniform and lives in scalar
// registers.  The whole state stays in VGPRs; per day the wavefront reads the
// observations and weights that it staged in its own LDS slice at the start
// of the tile: (y_i, 1/max(y_i,1)) for a deceased-count cost, or the six
// values (y_I, y_R, y_D, w_I, w_R, w_D) of an F_IRD cost, whose min-max
// ranges the wavefront reduces with cross-lane shuffles while staging.
// Tiles are ordered longest-first; with persistent > 0 a fixed set of
// resident wavefronts pulls tiles from a device counter instead of relying
// on the dispatcher's order.  The kernel is specialised per model; a batch
// that mixes models gets one launch per model, each skipping the other's
// tiles.
#include <hip/hip_runtime.h>

#include <atomic>
#include <string>
#include <type_traits>

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
    const int32_t *pairs;  // first tile of each wavefront's tile pair (two particles per lane)
    int n_pairs;
    int n_tiles;
    int n_waves;     // resident wavefronts of a persistent launch, else 0
    int obs_series;  // 1 (D) or 3 (I, R, D)
    int lds_stride;  // doubles per wavefront slice: 2 or 6 times (max_days + 1)
    CostPlan cost;
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

// Deceased-count costs: (y_i, w_i) pairs of the D series (the last of the
// obs_series blocks), one 16-byte LDS read per day.
__device__ __forceinline__ void stage_d(const FwdArgs &a, const sird_problem &P, int lane,
                                        double *ly)
{
    const int W = P.n_days;
    const double *y = a.obs + P.obs_off + (size_t)(a.obs_series - 1) * (W + 1);
    // four loads in flight before their LDS stores
    for (int i0 = lane; i0 <= W; i0 += 4 * kWave) {
        double yv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) yv[u] = y[min(i0 + u * kWave, W)];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = i0 + u * kWave;
            if (i <= W) {
                ly[2 * i] = yv[u];
                ly[2 * i + 1] = a.cost.w_rel ? 1.0 / fmax(yv[u], 1.0) : 1.0;
            }
        }
    }
}

// F_IRD: per day (y_I, y_R, y_D, w_I, w_R, w_D); w = 1/range of the series
// (1 for a flat one), or 1/max(y, 1) for MAPE.  The ranges are reduced
// across the wavefront with shuffles.
__device__ __forceinline__ void stage_ird(const FwdArgs &a, const sird_problem &P, int lane,
                                          double *ly)
{
    const int W = P.n_days;
    const double *y = a.obs + P.obs_off;
    double lo[3], hi[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        lo[c] = INFINITY;
        hi[c] = -INFINITY;
    }
    for (int i = lane; i <= W; i += kWave) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double v = y[(size_t)c * (W + 1) + i];
            ly[6 * i + c] = v;
            lo[c] = fmin(lo[c], v);
            hi[c] = fmax(hi[c], v);
        }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        for (int off = kWave / 2; off > 0; off >>= 1) {
            lo[c] = fmin(lo[c], __shfl_xor(lo[c], off));
            hi[c] = fmax(hi[c], __shfl_xor(hi[c], off));
        }
    }
    double inv_range[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double r = hi[c] - lo[c];
        inv_range[c] = 1.0 / (r > 0.0 ? r : 1.0);
    }
    for (int i = lane; i <= W; i += kWave) {
#pragma unroll
        for (int c = 0; c < 3; ++c)
            ly[6 * i + 3 + c] = a.cost.w_rel ? 1.0 / fmax(ly[6 * i + c], 1.0) : inv_range[c];
    }
}

// NS: observed series of the cost (1 or 3), 0 when writing trajectories;
// ACC: the cost's accumulation (CostAcc).
template <typename R, bool TRAJ, bool FUSED, int MODEL, int NS, int ACC>
__device__ __forceinline__ void fwd_tile(const FwdArgs &a, int t, int lane, double *ly)
{
    constexpr bool WITH_R = TRAJ || NS == 3;
    const sird_tile tl = a.tiles[t];
    const sird_problem P = a.probs[tl.prob];
    if (P.model != MODEL) return;  // wavefront-uniform; the other launch has it
    const int W = P.n_days, spd = P.steps_per_day, K = P.n_seg;
    const int n = P.n_part;
    const int pl = tl.p0 + lane;
    const bool active = pl < n;
    const int pc = active ? pl : n - 1;  // idle lanes integrate a valid column
    const size_t ld = (size_t)n;
    const double *th = a.theta + P.theta_off + pc;

    if (!TRAJ) {
        if (NS == 3)
            stage_ird(a, P, lane, ly);
        else
            stage_d(a, P, lane, ly);
        wave_sync();
    }
    // Moving the swarm first: the ramp model's parameters (d = 7) come from
    // the move's registers (idle lanes take the box's lower corner); the
    // RK4 model moves Philox block 0 (gamma, mu, I0, beta_0) here and each
    // later block of four betas in the segment loop, four segments ahead of
    // its last one, so the swarm's memory traffic is spread over the
    // integration instead of stalling every wavefront at its start.
    const bool lazy = MODEL == SIRD_MODEL_RK4_SEGMENTS && FUSED && a.do_move;
    const uint64_t it = FUSED && a.do_move ? a.iter[0] - 1 : 0;
    double xr[7];
    double mv0[4] = {0.0, 0.0, 0.0, 0.0};
    if constexpr (MODEL == SIRD_MODEL_EULER_RAMP) {
        if (FUSED && a.do_move) {
            if (active) {
                pso_move_ramp(a.mv, P, pl, it, xr);
            } else {
#pragma unroll
                for (int j = 0; j < 7; ++j) xr[j] = a.mv.lo[P.box_off + j];
            }
        } else {
#pragma unroll
            for (int j = 0; j < 7; ++j) xr[j] = th[(size_t)j * ld];
        }
    } else if (lazy && active) {
        pso_move_block_seq(a.mv, P, pl, it, 0, mv0);
    }
    const bool from_move = lazy && active;

    const bool ramp = MODEL == SIRD_MODEL_EULER_RAMP;
    const double gamma = ramp ? xr[4] : (from_move ? mv0[0] : th[(size_t)K * ld]);
    const double mu = ramp ? xr[5] : (from_move ? mv0[1] : th[(size_t)(K + 1) * ld]);
    const double I0 = ramp ? xr[6] : (from_move ? mv0[2] : th[(size_t)(K + 2) * ld]);
    const double N = P.N;

    SirdState<R> y;
    y.S = (R)(N - I0 - P.R0 - P.D0);
    y.I = (R)I0;
    y.Rr = (R)P.R0;
    y.D = (R)P.D0;
    y.s = R(0);
    y.eS = y.eI = y.eR = y.eD = R(0);

    double acc[3] = {acc_init<ACC>(), acc_init<ACC>(), acc_init<ACC>()};
    double *tr = nullptr;
    const size_t comp_stride = (size_t)(W + 1) * ld;
    if (TRAJ) tr = a.traj + P.traj_off + pc;
    // the state after day i: stored, or added to the cost; o holds the
    // day's observations and weights ((y, w) of a deceased-count cost, or
    // (y_I, y_R, y_D, w_I, w_R, w_D)), read from LDS before the day's steps
    // so that the read's latency overlaps them
    struct DayObs {
        double v[NS == 3 ? 6 : 2];
    };
    auto emit = [&](int i, const DayObs &o) {
        if constexpr (TRAJ) {
            if (active) store_day(tr + (size_t)i * ld, comp_stride, y);
        } else if constexpr (NS == 3) {
            acc_day<ACC>(acc[0], (o.v[0] - state_value(y.I, y.eI)) * o.v[3]);
            acc_day<ACC>(acc[1], (o.v[1] - state_value(y.Rr, y.eR)) * o.v[4]);
            acc_day<ACC>(acc[2], (o.v[2] - state_value(y.D, y.eD)) * o.v[5]);
        } else {
            acc_day<ACC>(acc[0], (o.v[0] - state_value(y.D, y.eD)) * o.v[1]);
        }
    };
    auto day_obs = [&](int i) {
        DayObs o{};
        if constexpr (!TRAJ && NS == 1) {
            o.v[0] = ly[2 * i];
            o.v[1] = ly[2 * i + 1];
        } else if constexpr (!TRAJ && NS == 3) {
#pragma unroll
            for (int c = 0; c < 6; ++c) o.v[c] = ly[6 * i + c];
        }
        return o;
    };
    if constexpr (!TRAJ && NS == 1) {
        // SSRE leaves out day 0
        const double e0 = (ly[0] - state_value(y.D, y.eD)) * ly[1];
        acc_day<ACC>(acc[0], a.cost.skip0 ? 0.0 : e0);
    } else {
        emit(0, day_obs(0));
    }

    if constexpr (MODEL == SIRD_MODEL_RK4_SEGMENTS) {
        // the cost needs only I and D: in double, s = b S is the state
        // within a segment (S is formed at segment ends); trajectories and
        // the compensated float state carry S
        constexpr bool WITH_S = TRAJ || sizeof(R) != 8;
        StepConst<R> sc = step_const<R>(gamma, mu, spd);
        const double invN = 1.0 / N;
        const int seg = P.seg_days;
        // the segments and their days, instantiated twice: days of a
        // multiple of ten steps run in blocks of ten unrolled steps, other
        // days unrolled by four; choosing outside the day loop keeps the
        // loop-carried state in the same registers from day to day
        auto segments = [&](auto tens) {
            constexpr bool TENS = decltype(tens)::value;
            int day = 0;
            double beta_next = from_move ? mv0[3] : th[0];
            for (int k = 0; k < K; ++k) {
                const double beta_k = beta_next;
                if (k + 1 < K) {
                    if (lazy && (k & 3) == 0) {
                        // block k/4 + 1: slots k+4 .. k+7, beta_{k+1} .. beta_{k+4}
                        double xn[4] = {0.0, 0.0, 0.0, 0.0};
                        if (active) pso_move_block_seq(a.mv, P, pl, it, k / 4 + 1, xn);
                        beta_next = active ? xn[0] : th[(size_t)(k + 1) * ld];
                    } else {
                        beta_next = th[(size_t)(k + 1) * ld];  // prefetch
                    }
                }
                const int dend = (k == K - 1) ? W : (int)min((long)W, (long)(k + 1) * seg);
                if (day >= dend) continue;
                if (!WITH_S && day > 0) unscale(y, sc);
                set_beta(sc, beta_k, invN);
                if (!WITH_S) rescale(y, sc);
                for (; day < dend; ++day) {
                    if (WITH_S) rescale(y, sc);
                    const DayObs o = day_obs(day + 1);
                    if constexpr (TENS) {
                        for (int s = 0; s < spd; s += 10) {
#pragma unroll
                            for (int u = 0; u < 10; ++u) rk4_step<R, WITH_R, WITH_S>(y, sc);
                        }
                    } else {
#pragma unroll 4
                        for (int s = 0; s < spd; ++s) rk4_step<R, WITH_R, WITH_S>(y, sc);
                    }
                    emit(day + 1, o);
                }
            }
        };
        if (spd % 10 == 0)
            segments(std::true_type{});
        else
            segments(std::false_type{});
    } else {
        const RampConst<R> rc = ramp_const<R>(xr[0], xr[1], xr[2], xr[3], gamma, mu, N, spd);
        const double h = 1.0 / (double)spd;
        int64_t step = 0;
        for (int day = 0; day < W; ++day) {
            const DayObs o = day_obs(day + 1);
            // the ramp is evaluated at the start of each step, t = step h
            for (int s = 0; s < spd; ++s, ++step)
                euler_ramp_step<R, WITH_R>(y, rc, (double)step * h);
            emit(day + 1, o);
        }
    }
    if (!TRAJ && active) {
        double L = cost_value(a.cost, acc[0], W);
        if constexpr (NS == 3) {
            // the largest of the three series, NaN if any is NaN
            const double v1 = cost_value(a.cost, acc[1], W);
            const double v2 = cost_value(a.cost, acc[2], W);
            const bool nan = L != L || v1 != v1 || v2 != v2;
            L = fmax(L, fmax(v1, v2));
            if (nan) L = NAN;
        }
        a.loss[P.p_off + pl] = L;
        if (FUSED) pso_pbest_particle(L, P, pl, a.pbest_f, a.pbest_x, a.mv.x);
    }
    if (!TRAJ) wave_sync();  // LDS slice reads done before it is restaged
}

template <typename R, bool TRAJ, bool FUSED, int MODEL, int NS, int ACC>
__global__ void __launch_bounds__(1024) k_forward(FwdArgs a)
{
    extern __shared__ double lds[];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    double *ly = lds + (size_t)wave * a.lds_stride;
    if (a.n_waves > 0) {
        for (;;) {
            int t = 0;
            if (lane == 0) t = atomicAdd(&a.sched[0], 1);
            t = wave_uniform(t);
            if (t >= a.n_tiles) break;
            fwd_tile<R, TRAJ, FUSED, MODEL, NS, ACC>(a, t, lane, ly);
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
        if (t < a.n_tiles) fwd_tile<R, TRAJ, FUSED, MODEL, NS, ACC>(a, t, lane, ly);
    }
}

// Two particles per lane: the wavefront integrates the tile pair starting
// at tile pairs[w] (two consecutive 64-particle tiles of one problem, or a
// problem's last tile alone), lane l taking local particles p0 + l and
// p0 + 64 + l.  Only for the RK4 model with a deceased-count cost.  Each
// particle goes through exactly the operations fwd_tile applies to it (the
// two particles' steps are interleaved, which gives the scheduler two
// independent dependency chains), so the results are bitwise those of one
// particle per lane; the observations are staged and read once per pair.
template <typename R, bool FUSED, int ACC>
__device__ __forceinline__ void fwd_pair(const FwdArgs &a, int w, int lane, double *ly)
{
    constexpr int PPL = 2;
    const int t = a.pairs[w];
    const sird_tile tl = a.tiles[t];
    const sird_problem P = a.probs[tl.prob];
    if (P.model != SIRD_MODEL_RK4_SEGMENTS) return;
    const bool two = t + 1 < a.n_tiles && a.tiles[t + 1].prob == tl.prob &&
                     a.tiles[t + 1].p0 == tl.p0 + kWave;
    const int W = P.n_days, spd = P.steps_per_day, K = P.n_seg;
    const int n = P.n_part;
    const size_t ld = (size_t)n;
    int pl[PPL];
    bool active[PPL];
    const double *th[PPL];
#pragma unroll
    for (int j = 0; j < PPL; ++j) {
        pl[j] = tl.p0 + j * kWave + lane;
        active[j] = pl[j] < n && (j == 0 || two);
        th[j] = a.theta + P.theta_off + (active[j] ? pl[j] : n - 1);
    }

    stage_d(a, P, lane, ly);
    wave_sync();

    const bool lazy = FUSED && a.do_move;
    const uint64_t it = FUSED && a.do_move ? a.iter[0] - 1 : 0;
    double mv0[PPL][4];
    bool from_move[PPL];
#pragma unroll
    for (int j = 0; j < PPL; ++j) {
#pragma unroll
        for (int u = 0; u < 4; ++u) mv0[j][u] = 0.0;
        from_move[j] = lazy && active[j];
        if (from_move[j]) pso_move_block_seq(a.mv, P, pl[j], it, 0, mv0[j]);
    }
    constexpr bool WITH_S = sizeof(R) != 8;
    const double N = P.N;
    const double invN = 1.0 / N;
    SirdState<R> y[PPL];
    StepConst<R> sc[PPL];
    double acc[PPL];
    double beta_next[PPL];
#pragma unroll
    for (int j = 0; j < PPL; ++j) {
        const double gamma = from_move[j] ? mv0[j][0] : th[j][(size_t)K * ld];
        const double mu = from_move[j] ? mv0[j][1] : th[j][(size_t)(K + 1) * ld];
        const double I0 = from_move[j] ? mv0[j][2] : th[j][(size_t)(K + 2) * ld];
        y[j].S = (R)(N - I0 - P.R0 - P.D0);
        y[j].I = (R)I0;
        y[j].Rr = (R)P.R0;
        y[j].D = (R)P.D0;
        y[j].s = R(0);
        y[j].eS = y[j].eI = y[j].eR = y[j].eD = R(0);
        sc[j] = step_const<R>(gamma, mu, spd);
        acc[j] = acc_init<ACC>();
        // SSRE leaves out day 0
        const double e0 = (ly[0] - state_value(y[j].D, y[j].eD)) * ly[1];
        acc_day<ACC>(acc[j], a.cost.skip0 ? 0.0 : e0);
        beta_next[j] = from_move[j] ? mv0[j][3] : th[j][0];
    }
    const int seg = P.seg_days;
    int day = 0;
    for (int k = 0; k < K; ++k) {
        double beta_k[PPL];
#pragma unroll
        for (int j = 0; j < PPL; ++j) {
            beta_k[j] = beta_next[j];
            if (k + 1 < K) {
                if (lazy && (k & 3) == 0) {
                    double xn[4] = {0.0, 0.0, 0.0, 0.0};
                    if (active[j]) pso_move_block_seq(a.mv, P, pl[j], it, k / 4 + 1, xn);
                    beta_next[j] = active[j] ? xn[0] : th[j][(size_t)(k + 1) * ld];
                } else {
                    beta_next[j] = th[j][(size_t)(k + 1) * ld];  // prefetch
                }
            }
        }
        const int dend = (k == K - 1) ? W : (int)min((long)W, (long)(k + 1) * seg);
        if (day >= dend) continue;
#pragma unroll
        for (int j = 0; j < PPL; ++j) {
            if (!WITH_S && day > 0) unscale(y[j], sc[j]);
            set_beta(sc[j], beta_k[j], invN);
            if (!WITH_S) rescale(y[j], sc[j]);
        }
        for (; day < dend; ++day) {
            if (WITH_S) {
#pragma unroll
                for (int j = 0; j < PPL; ++j) rescale(y[j], sc[j]);
            }
            const double yo = ly[2 * (day + 1)], wo = ly[2 * (day + 1) + 1];
#pragma unroll 4
            for (int st = 0; st < spd; ++st) {
#pragma unroll
                for (int j = 0; j < PPL; ++j) rk4_step<R, false, WITH_S>(y[j], sc[j]);
            }
#pragma unroll
            for (int j = 0; j < PPL; ++j)
                acc_day<ACC>(acc[j], (yo - state_value(y[j].D, y[j].eD)) * wo);
        }
    }
#pragma unroll
    for (int j = 0; j < PPL; ++j) {
        if (active[j]) {
            const double L = cost_value(a.cost, acc[j], W);
            a.loss[P.p_off + pl[j]] = L;
            if (FUSED) pso_pbest_particle(L, P, pl[j], a.pbest_f, a.pbest_x, a.mv.x);
        }
    }
    wave_sync();  // LDS slice reads done before it is restaged
}

template <typename R, bool FUSED, int ACC>
__global__ void __launch_bounds__(1024) k_forward_pairs(FwdArgs a)
{
    extern __shared__ double lds[];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    double *ly = lds + (size_t)wave * a.lds_stride;
    const int w = wave_tile_index();
    if (w < a.n_pairs) fwd_pair<R, FUSED, ACC>(a, w, lane, ly);
}

// The constants of each cost kind (Sec. 3.1).
static CostPlan cost_plan(int kind)
{
    switch (kind) {
    case SIRD_LOSS_SSRE: return {1, kAccSq, 1, 1, 1.0, 0};
    case SIRD_LOSS_MSE: return {1, kAccSq, 0, 0, 1.0, 1};
    case SIRD_LOSS_MXSE: return {1, kAccMax, 0, 0, 1.0, 0};
    case SIRD_LOSS_MAE: return {1, kAccAbs, 0, 0, 1.0, 1};
    case SIRD_LOSS_MAPE: return {1, kAccAbs, 1, 0, 100.0, 1};
    case SIRD_LOSS_IRD_MXSE: return {3, kAccMax, 0, 0, 1.0, 0};
    case SIRD_LOSS_IRD_MSE: return {3, kAccSq, 0, 0, 1.0, 1};
    case SIRD_LOSS_IRD_MAE: return {3, kAccAbs, 0, 0, 1.0, 1};
    default: return {3, kAccAbs, 1, 0, 100.0, 1};  // SIRD_LOSS_IRD_MAPE
    }
}

// LDS to reserve per block so that a compute unit (4 SIMDs, its LDS shared
// by the blocks resident on it) holds at most waves_per_simd wavefronts per
// SIMD: with wpb wavefronts per block that is nb = 4 waves_per_simd / wpb
// blocks, so each block claims more than 1/(nb + 1) of the LDS (rounded up
// to the 512-byte allocation unit) and at most 1/nb of it.  0 if no
// reservation does it.
static size_t occupancy_lds(int waves_per_simd, int wpb)
{
    // LDS per compute unit of each device, queried once
    static std::atomic<int> lds_per_cu[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return 0;
    int per_cu = dev < 64 ? lds_per_cu[dev].load(std::memory_order_relaxed) : 0;
    if (per_cu <= 0) {
        if (hipDeviceGetAttribute(&per_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor,
                                  dev) != hipSuccess || per_cu <= 0)
            return 0;
        if (dev < 64) lds_per_cu[dev].store(per_cu, std::memory_order_relaxed);
    }
    const int nb = 4 * waves_per_simd / wpb;
    if (nb < 1) return 0;
    const size_t bytes = ((size_t)per_cu / (nb + 1) / 512 + 1) * 512;
    return bytes <= (size_t)per_cu / nb ? bytes : 0;
}

template <typename R, bool TRAJ, bool FUSED, int NS, int ACC>
static int launch_forward(const sird_batch *b, FwdArgs a, hipStream_t s, const char *who)
{
    const int block = integ_block(b);
    const int wpb = block / kWave;
    a.obs_series = b->obs_series;
    a.lds_stride = (NS == 3 ? 6 : 2) * (b->max_days + 1);
    size_t lds = TRAJ ? 0 : (size_t)wpb * a.lds_stride * sizeof(double);
    if (lds > 65536)
        return fail(SIRD_EINVAL, std::string(who) +
                                     ": block too large for the window length (LDS > 64 KiB)");
    if (b->waves_per_simd > 0) {
        const size_t cap = occupancy_lds(b->waves_per_simd, wpb);
        if (cap == 0 || cap > 65536)
            return fail(SIRD_EINVAL, std::string(who) +
                                         ": waves_per_simd too small for the block size");
        if (lds < cap) lds = cap;
    }
    if constexpr (!TRAJ && NS == 1) {
        // two particles per lane: the tile pairs of the batch, one per
        // wavefront (RK4-only batches without the persistent queue)
        if (b->ppl == 2 && b->persistent == 0 && b->models == 1 << SIRD_MODEL_RK4_SEGMENTS) {
            a.pairs = b->pair_tiles;
            a.n_pairs = b->n_pairs;
            a.n_waves = 0;
            const int pgrid = (b->n_pairs + wpb - 1) / wpb;
            if (pgrid == 0) return SIRD_OK;
            hipLaunchKernelGGL((k_forward_pairs<R, FUSED, ACC>), dim3(pgrid), dim3(block), lds,
                               s, a);
            return hip_status(hipGetLastError(), who);
        }
    }
    int grid;
    if (b->persistent > 0) {
        grid = (b->persistent + wpb - 1) / wpb;
        a.n_waves = grid * wpb;
    } else {
        grid = (a.n_tiles + wpb - 1) / wpb;
        a.n_waves = 0;
    }
    if (grid == 0) return SIRD_OK;
    if (b->models & (1 << SIRD_MODEL_RK4_SEGMENTS)) {
        hipLaunchKernelGGL((k_forward<R, TRAJ, FUSED, SIRD_MODEL_RK4_SEGMENTS, NS, ACC>),
                           dim3(grid), dim3(block), lds, s, a);
        const int st = hip_status(hipGetLastError(), who);
        if (st) return st;
    }
    if (b->models & (1 << SIRD_MODEL_EULER_RAMP)) {
        hipLaunchKernelGGL((k_forward<R, TRAJ, FUSED, SIRD_MODEL_EULER_RAMP, NS, ACC>),
                           dim3(grid), dim3(block), lds, s, a);
        const int st = hip_status(hipGetLastError(), who);
        if (st) return st;
    }
    return SIRD_OK;
}

// Instantiation for the cost of kind: series and accumulation.
template <typename R, bool FUSED>
static int launch_cost(const sird_batch *b, FwdArgs a, int kind, hipStream_t s,
                       const char *who)
{
    a.cost = cost_plan(kind);
    const bool three = a.cost.series == 3;
    switch (a.cost.acc) {
    case kAccSq:
        return three ? launch_forward<R, false, FUSED, 3, kAccSq>(b, a, s, who)
                     : launch_forward<R, false, FUSED, 1, kAccSq>(b, a, s, who);
    case kAccAbs:
        return three ? launch_forward<R, false, FUSED, 3, kAccAbs>(b, a, s, who)
                     : launch_forward<R, false, FUSED, 1, kAccAbs>(b, a, s, who);
    default:
        return three ? launch_forward<R, false, FUSED, 3, kAccMax>(b, a, s, who)
                     : launch_forward<R, false, FUSED, 1, kAccMax>(b, a, s, who);
    }
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
    if (b->dtype == SIRD_F32) return launch_cost<float, false>(b, a, kind, s, "sird_loss");
    return launch_cost<double, false>(b, a, kind, s, "sird_loss");
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
    a.mv = mv;
    a.pbest_f = st->pbest_f;
    a.pbest_x = st->pbest_x;
    a.iter = st->iter;
    a.do_move = move ? 1 : 0;
    if (b->dtype == SIRD_F32) return launch_cost<float, true>(b, a, kind, s, "sird_pso_iterate");
    return launch_cost<double, true>(b, a, kind, s, "sird_pso_iterate");
}

}  // namespace sird

using namespace sird;

extern "C" int sird_loss(const sird_batch *batch, const double *theta, const double *obs,
                         int loss_kind, double *loss, int ckpt_interval, void *workspace,
                         size_t ws_bytes, void *stream)
{
    int st = check_batch(batch, "sird_loss");
    if (st) return st;
    if (!theta || !obs || !loss) return fail(SIRD_EINVAL, "sird_loss: NULL array");
    st = check_kind(batch, loss_kind, "sird_loss");
    if (st) return st;
    if (batch->obs_len < 1) return fail(SIRD_EINVAL, "sird_loss: batch planned without obs");
    if (workspace)  // the adjoint's forward pass, saving its checkpoints
        return adjoint_enqueue(batch, theta, obs, loss_kind, nullptr, nullptr, loss,
                               ckpt_interval, 1, workspace, ws_bytes, (hipStream_t)stream,
                               "sird_loss");
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
    if (batch->dtype == SIRD_F32)
        return launch_forward<float, true, false, 0, 0>(batch, a, s, "sird_integrate");
    return launch_forward<double, true, false, 0, 0>(batch, a, s, "sird_integrate");
}
