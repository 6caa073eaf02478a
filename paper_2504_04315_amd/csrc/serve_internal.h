// Internal interface between the serving scheduler (serve.cpp) and the
// persistent multi-session kernels (k_serve.hip).
#pragma once

#include <vector>

#include "npm_internal.h"

namespace npm {

constexpr int kMaxRoundRequests = 256;

// One request of a round as the scheduler hands it to the launcher.
struct ServeRequest {
    int kind;                    // 0 query, 1 train
    int64_t n;
    const float *pos, *dir, *rad, *spdf;
    float *lobes, *pdf, *sdir, *spdf_out;
    double *stats;
    uint64_t seed;
    uint32_t stream_id;
    npm_ctx *ctx;
    int32_t session;
};

// Pinned host staging and device copy of a round's descriptors.
struct RoundBuffers {
    void *host = nullptr;
    void *dev = nullptr;
    size_t bytes = 0;
};

hipError_t round_buffers_init(RoundBuffers *b);
void round_buffers_free(RoundBuffers *b);
// Whether the persistent kernels are instantiated for this network shape.
bool serve_supports(const npm_config *cfg);
// Enqueues one round on `s`: the persistent query kernel over every query of
// the round, the persistent backward kernel over every training batch, and
// the Adam step of each session that trained.
hipError_t serve_launch_round(RoundBuffers *b, const std::vector<ServeRequest> &reqs,
                              hipStream_t s);

}  // namespace npm
