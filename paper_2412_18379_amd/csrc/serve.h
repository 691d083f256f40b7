// Serving loop: continuous batching of CNN-SNS jobs on resident meshes.
#pragma once

#include <memory>

#include "common.h"

namespace cnnsns {

cnnsns_server server_create(int64_t hbm_budget_bytes, int32_t max_inflight, int32_t queue_depth, int32_t precision,
                            const cnnsns_cnn* w);
uint64_t server_submit(cnnsns_server s, cnnsns_mesh m, const float* vel, int64_t n, const double* xp,
                       const double* origin, const int32_t* start, int32_t* host, int32_t* iters,
                       hipStream_t stream);
bool server_poll(cnnsns_server s, uint64_t job_id, double* latency_ms);
void server_wait(cnnsns_server s, uint64_t job_id, double* latency_ms);
void server_destroy(cnnsns_server s);

}  // namespace cnnsns
