// The log-add-exp reduce_by_index on the bucket-partitioned histogram path
// (defined with that path; used by the log-add-exp entry points).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/pvjp.h"

namespace pvjp {

// Whether the partitioned form serves (dtype, m): FP32 with bins beyond one
// block's LDS and at most 2^22 of them.
bool hist_lae_partition_ok(pvjp_dtype dtype, int64_t m);
// hs[b] = log sum of e^x over bin b (-inf for an empty bin or -inf elements
// only); ws: at least pvjp_hist_ws_bytes(PVJP_ADD, PVJP_F32, n, m) bytes,
// 256-byte aligned.
void hist_lae_partitioned(const int32_t* inds, const float* x, int64_t n, int32_t m, float* hs, char* ws,
                          hipStream_t st);

}  // namespace pvjp
