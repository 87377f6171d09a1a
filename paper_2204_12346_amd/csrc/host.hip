// Host-side part of the C ABI: status strings, problem-table validation,
// the longest-first tile plan and the per-call batch checks.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/sird.h"
#include "internal.h"

namespace sird {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

int fail(int status, const std::string &msg)
{
    set_error(msg);
    return status;
}

int hip_status(hipError_t e, const char *who)
{
    if (e == hipSuccess) return SIRD_OK;
    return fail(SIRD_EHIP, std::string(who) + ": " + hipGetErrorString(e));
}

int check_batch(const sird_batch *b, const char *who)
{
    const std::string w(who);
    if (!b) return fail(SIRD_EINVAL, w + ": batch is NULL");
    if (b->n_prob < 1) return fail(SIRD_EINVAL, w + ": n_prob < 1");
    if (b->n_tiles < 0) return fail(SIRD_EINVAL, w + ": n_tiles < 0");
    if (b->max_days < 1 || b->max_d < 4 || b->max_steps < 1)
        return fail(SIRD_EINVAL, w + ": batch not planned (max_days/max_d/max_steps)");
    if (!b->probs) return fail(SIRD_EINVAL, w + ": probs is NULL");
    if (b->n_tiles > 0 && !b->tiles) return fail(SIRD_EINVAL, w + ": tiles is NULL");
    if (b->dtype != SIRD_F64 && b->dtype != SIRD_F32)
        return fail(SIRD_EINVAL, w + ": dtype must be SIRD_F64 or SIRD_F32");
    if (b->block != 0 && (b->block < 64 || b->block > 1024 || b->block % 64 != 0))
        return fail(SIRD_EINVAL, w + ": block must be 0 or a multiple of 64 in [64, 1024]");
    if (b->persistent < 0) return fail(SIRD_EINVAL, w + ": persistent < 0");
    if (b->waves_per_simd < 0 || b->waves_per_simd > 8)
        return fail(SIRD_EINVAL, w + ": waves_per_simd must be in [0, 8]");
    if (b->persistent > 0 && !b->sched)
        return fail(SIRD_EINVAL, w + ": persistent launch needs sched counters");
    if (b->obs_series != 1 && b->obs_series != 3)
        return fail(SIRD_EINVAL, w + ": obs_series must be 1 or 3");
    if (b->models < 1 || b->models > 3)
        return fail(SIRD_EINVAL, w + ": models must be a non-empty mask of SIRD_MODEL_*");
    if (b->ppl < 0 || b->ppl > 2) return fail(SIRD_EINVAL, w + ": ppl must be 0, 1 or 2");
    if (b->ppl == 2 && b->n_tiles > 0 && (!b->pair_tiles || b->n_pairs < 1 ||
                                          b->n_pairs > b->n_tiles))
        return fail(SIRD_EINVAL, w + ": ppl = 2 needs the pair table (sird_plan_pairs)");
    return SIRD_OK;
}

int check_kind(const sird_batch *b, int kind, const char *who)
{
    const std::string w(who);
    if (kind < SIRD_LOSS_SSRE || kind > SIRD_LOSS_IRD_MAPE)
        return fail(SIRD_EINVAL, w + ": unknown loss_kind");
    if (is_ird(kind) && b->obs_series != 3)
        return fail(SIRD_EINVAL, w + ": the F_IRD costs need a batch with obs_series = 3");
    return SIRD_OK;
}

int integ_block(const sird_batch *b) { return b->block ? b->block : 256; }

}  // namespace sird

using namespace sird;

extern "C" const char *sird_status_string(int status)
{
    switch (status) {
    case SIRD_OK: return "SIRD_OK: success";
    case SIRD_EINVAL: return "SIRD_EINVAL: invalid argument";
    case SIRD_ENOSPACE: return "SIRD_ENOSPACE: workspace or output too small";
    case SIRD_EHIP: return "SIRD_EHIP: HIP runtime error";
    default: return "unknown status";
    }
}

extern "C" const char *sird_last_error(void) { return g_last_error.c_str(); }

static bool range_ok(int64_t off, int64_t count, int64_t len)
{
    return off >= 0 && count >= 0 && off <= len && count <= len - off;
}

extern "C" int sird_problem_validate(const sird_problem *probs, int n_prob,
                                     int64_t total_particles, int64_t theta_len,
                                     int64_t obs_len, int64_t traj_len, int64_t box_len,
                                     int obs_series)
{
    if (!probs) return fail(SIRD_EINVAL, "sird_problem_validate: probs is NULL");
    if (n_prob < 1) return fail(SIRD_EINVAL, "sird_problem_validate: n_prob < 1");
    if (obs_series != 1 && obs_series != 3)
        return fail(SIRD_EINVAL, "sird_problem_validate: obs_series must be 1 or 3");
    for (int r = 0; r < n_prob; ++r) {
        const sird_problem &p = probs[r];
        char buf[160];
        auto bad = [&](const char *what) {
            std::snprintf(buf, sizeof buf, "sird_problem_validate: problem %d: %s", r, what);
            return fail(SIRD_EINVAL, buf);
        };
        if (p.n_days < 1) return bad("n_days < 1");
        if (p.steps_per_day < 1) return bad("steps_per_day < 1");
        if (p.seg_days < 1) return bad("seg_days < 1");
        if (p.n_seg < 1) return bad("n_seg < 1");
        if (p.n_part < 0) return bad("n_part < 0");
        if (p.model != SIRD_MODEL_RK4_SEGMENTS && p.model != SIRD_MODEL_EULER_RAMP)
            return bad("unknown model");
        if (p.model == SIRD_MODEL_EULER_RAMP && p.n_seg != 4)
            return bad("the ramp model needs n_seg = 4");
        if ((int64_t)p.n_days * p.steps_per_day > (int64_t)1 << 30)
            return bad("n_days * steps_per_day too large");
        if (p.n_days > (1 << 20) || p.n_seg > (1 << 20)) return bad("n_days or n_seg too large");
        if (!(p.N > 0.0) || !std::isfinite(p.N)) return bad("N must be finite and > 0");
        if (!(p.R0 >= 0.0) || !(p.D0 >= 0.0) || !std::isfinite(p.R0) || !std::isfinite(p.D0))
            return bad("R0 and D0 must be finite and >= 0");
        const int64_t d = (int64_t)p.n_seg + 3;
        if (!range_ok(p.p_off, p.n_part, total_particles)) return bad("particle range");
        if (!range_ok(p.theta_off, d * p.n_part, theta_len)) return bad("theta block");
        if (obs_len > 0 && !range_ok(p.obs_off, obs_series * ((int64_t)p.n_days + 1), obs_len))
            return bad("obs block");
        if (traj_len > 0 && !range_ok(p.traj_off, 4 * ((int64_t)p.n_days + 1) * p.n_part, traj_len))
            return bad("traj block");
        if (!range_ok(p.box_off, d, box_len)) return bad("box block");
    }
    return SIRD_OK;
}

extern "C" int sird_plan_tiles(const sird_problem *probs, int n_prob, sird_tile *tiles_out,
                               int max_tiles)
{
    if (!probs || n_prob < 1) return fail(SIRD_EINVAL, "sird_plan_tiles: bad problem table");
    std::vector<sird_tile> t;
    for (int r = 0; r < n_prob; ++r) {
        if (probs[r].n_part < 0) return fail(SIRD_EINVAL, "sird_plan_tiles: n_part < 0");
        for (int p0 = 0; p0 < probs[r].n_part; p0 += kTileParticles) t.push_back({r, p0});
    }
    if ((int64_t)t.size() > (int64_t)max_tiles || (max_tiles > 0 && !tiles_out && !t.empty()))
        return fail(SIRD_ENOSPACE, "sird_plan_tiles: tile table too small");
    std::stable_sort(t.begin(), t.end(), [&](const sird_tile &a, const sird_tile &b) {
        const int64_t ta = (int64_t)probs[a.prob].n_days * probs[a.prob].steps_per_day;
        const int64_t tb = (int64_t)probs[b.prob].n_days * probs[b.prob].steps_per_day;
        return ta > tb;
    });
    for (size_t i = 0; i < t.size(); ++i) tiles_out[i] = t[i];
    return (int)t.size();
}

extern "C" int sird_plan_pairs(const sird_tile *tiles, int n_tiles, int32_t *pairs_out,
                               int max_pairs)
{
    if (n_tiles < 0 || (n_tiles > 0 && (!tiles || !pairs_out)))
        return fail(SIRD_EINVAL, "sird_plan_pairs: bad tile table");
    int np = 0;
    for (int t = 0; t < n_tiles;) {
        if (np >= max_pairs) return fail(SIRD_ENOSPACE, "sird_plan_pairs: pairs_out too small");
        pairs_out[np++] = t;
        const bool two = t + 1 < n_tiles && tiles[t + 1].prob == tiles[t].prob &&
                         tiles[t + 1].p0 == tiles[t].p0 + kTileParticles;
        t += two ? 2 : 1;
    }
    return np;
}

extern "C" int sird_batch_plan(sird_batch *batch, const sird_problem *probs_host, int n_prob,
                               int64_t total_particles, int64_t theta_len, int64_t obs_len,
                               int64_t traj_len, int64_t box_len, int obs_series, int n_tiles,
                               const sird_problem *probs_dev, const sird_tile *tiles_dev,
                               int32_t *sched_dev)
{
    if (!batch) return fail(SIRD_EINVAL, "sird_batch_plan: batch is NULL");
    int st = sird_problem_validate(probs_host, n_prob, total_particles, theta_len, obs_len,
                                   traj_len, box_len, obs_series);
    if (st != SIRD_OK) return st;
    int64_t tiles = 0;
    int max_days = 0, max_d = 0, models = 0, max_part = 0;
    int64_t max_steps = 0;
    for (int r = 0; r < n_prob; ++r) {
        const sird_problem &p = probs_host[r];
        models |= 1 << p.model;
        tiles += (p.n_part + kTileParticles - 1) / kTileParticles;
        max_days = std::max(max_days, p.n_days);
        max_part = std::max(max_part, p.n_part);
        max_d = std::max(max_d, p.n_seg + 3);
        max_steps = std::max(max_steps, (int64_t)p.n_days * p.steps_per_day);
    }
    if (tiles != n_tiles)
        return fail(SIRD_EINVAL, "sird_batch_plan: n_tiles does not match the problem table");
    if (!probs_dev) return fail(SIRD_EINVAL, "sird_batch_plan: probs_dev is NULL");
    if (n_tiles > 0 && !tiles_dev) return fail(SIRD_EINVAL, "sird_batch_plan: tiles_dev is NULL");
    batch->n_prob = n_prob;
    batch->n_tiles = n_tiles;
    batch->max_days = max_days;
    batch->max_d = max_d;
    batch->max_steps = max_steps;
    batch->total_particles = total_particles;
    batch->theta_len = theta_len;
    batch->obs_len = obs_len;
    batch->traj_len = traj_len;
    batch->box_len = box_len;
    batch->probs = probs_dev;
    batch->tiles = tiles_dev;
    batch->sched = sched_dev;
    batch->obs_series = obs_series;
    batch->models = models;
    batch->max_part = max_part;
    return SIRD_OK;
}
