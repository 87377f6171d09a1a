// HIP-graph capture of the calibration iteration: iters_per_launch
// repetitions of [sird_loss -> pso_step] recorded once and replayed, so a
// long run costs one graph launch per iters_per_launch iterations.  The
// swarm's iteration counter lives in device memory and the kernels reset
// their own counters, so the graph holds kernel nodes only (no memsets).
#include <hip/hip_runtime.h>

#include <new>
#include <string>

#include "device.h"
#include "internal.h"

namespace sird {

int pso_iterate_enqueue(const sird_batch *b, const pso_params *p, const pso_state *st,
                        const double *obs, int kind, int n_iters, hipStream_t s);
int check_iterate(const sird_batch *b, const pso_params *p, const pso_state *st,
                  const double *obs, int kind, int n_iters, const char *who);

struct GraphHandle {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

}  // namespace sird

using namespace sird;

extern "C" int sird_graph_create(const sird_batch *batch, const pso_params *params,
                                 const pso_state *state, const double *obs, int loss_kind,
                                 int iters_per_launch, void **graph_out)
{
    int r = check_iterate(batch, params, state, obs, loss_kind, iters_per_launch,
                          "sird_graph_create");
    if (r) return r;
    if (!graph_out) return fail(SIRD_EINVAL, "sird_graph_create: graph_out is NULL");
    if (iters_per_launch < 1)
        return fail(SIRD_EINVAL, "sird_graph_create: iters_per_launch < 1");
    *graph_out = nullptr;
    hipStream_t cs = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_status(e, "sird_graph_create(stream)");
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(cs);
        return hip_status(e, "sird_graph_create(begin capture)");
    }
    r = pso_iterate_enqueue(batch, params, state, obs, loss_kind, iters_per_launch, cs);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(cs, &g);
    if (r != SIRD_OK || e2 != hipSuccess) {
        (void)hipStreamDestroy(cs);
        if (g) (void)hipGraphDestroy(g);
        return r != SIRD_OK ? r : hip_status(e2, "sird_graph_create(end capture)");
    }
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(cs);
        (void)hipGraphDestroy(g);
        return hip_status(e, "sird_graph_create(instantiate)");
    }
    // upload the executable graph now, so that the first launch does not
    // pay for it
    e = hipGraphUpload(x, cs);
    if (e == hipSuccess) e = hipStreamSynchronize(cs);
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess) {
        (void)hipGraphExecDestroy(x);
        (void)hipGraphDestroy(g);
        return hip_status(e, "sird_graph_create(upload)");
    }
    GraphHandle *h = new (std::nothrow) GraphHandle;
    if (!h) {
        (void)hipGraphExecDestroy(x);
        (void)hipGraphDestroy(g);
        return fail(SIRD_EINVAL, "sird_graph_create: out of host memory");
    }
    h->graph = g;
    h->exec = x;
    *graph_out = h;
    return SIRD_OK;
}

extern "C" int sird_graph_launch(void *graph, int n_launches, void *stream)
{
    if (!graph) return fail(SIRD_EINVAL, "sird_graph_launch: graph is NULL");
    if (n_launches < 0) return fail(SIRD_EINVAL, "sird_graph_launch: n_launches < 0");
    GraphHandle *h = (GraphHandle *)graph;
    for (int i = 0; i < n_launches; ++i) {
        hipError_t e = hipGraphLaunch(h->exec, (hipStream_t)stream);
        if (e != hipSuccess) return hip_status(e, "sird_graph_launch");
    }
    return SIRD_OK;
}

extern "C" int sird_graph_destroy(void *graph)
{
    if (!graph) return SIRD_OK;
    GraphHandle *h = (GraphHandle *)graph;
    hipError_t e1 = h->exec ? hipGraphExecDestroy(h->exec) : hipSuccess;
    hipError_t e2 = h->graph ? hipGraphDestroy(h->graph) : hipSuccess;
    delete h;
    if (e1 != hipSuccess) return hip_status(e1, "sird_graph_destroy");
    return hip_status(e2, "sird_graph_destroy");
}
