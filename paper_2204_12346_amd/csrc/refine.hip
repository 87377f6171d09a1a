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

}  // namespace sird

using namespace sird;

extern "C" int pso_topk(const sird_batch *batch, const double *pbest_f, int k,
                        int64_t *idx_out, void *stream)
{
    int st = check_batch(batch, "pso_topk");
    if (st) return st;
    if (!pbest_f || !idx_out) return fail(SIRD_EINVAL, "pso_topk: NULL array");
    if (k < 1 || k > 1024) return fail(SIRD_EINVAL, "pso_topk: k must be in [1, 1024]");
    hipLaunchKernelGGL(k_topk, dim3(batch->n_prob), dim3(256), 0, (hipStream_t)stream,
                       batch->probs, pbest_f, k, idx_out);
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
