// Host-side internals shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "../../include/sird.h"

namespace sird {

// Particles per tile: one wavefront of 64 lanes, one particle per lane.
constexpr int kTileParticles = 64;

// Thread-local error message behind sird_last_error().
void set_error(const std::string &msg);
int fail(int status, const std::string &msg);

// Scalar checks of a batch that every device call repeats (cheap; the table
// itself is checked by sird_batch_plan).
int check_batch(const sird_batch *b, const char *who);

// A cost kind this batch can evaluate: SIRD_LOSS_* in [0, 8]; the F_IRD
// kinds need three observed series.
int check_kind(const sird_batch *b, int kind, const char *who);

inline bool is_ird(int kind) { return kind >= SIRD_LOSS_IRD_MXSE; }

// Map a HIP status after enqueueing to SIRD_OK / SIRD_EHIP.
int hip_status(hipError_t e, const char *who);

// Threads per block of the integration kernels for this batch.
int integ_block(const sird_batch *b);

// Launch geometry of the per-tile kernels: blocks of 256 threads, one
// wavefront per tile.
inline int tile_blocks(int n_tiles) { return (n_tiles + 3) / 4; }

// The discrete adjoint (adjoint.hip).  mode 0: forward pass and reverse
// sweep; 1: the forward pass alone, saving the loss and what the reverse
// sweep reads in the workspace (loss_out required); 2: the reverse sweep
// alone from a workspace that mode 1 filled with the same theta, obs, kind
// and interval.  All host checks run before anything is enqueued.
int adjoint_enqueue(const sird_batch *batch, const double *theta, const double *obs,
                    int loss_kind, const double *grad_loss, double *grad_theta,
                    double *loss_out, int ckpt_interval, int mode, void *workspace,
                    size_t ws_bytes, hipStream_t stream, const char *who);
size_t adjoint_workspace_bytes(const sird_batch *b, int ckpt_interval);

}  // namespace sird
