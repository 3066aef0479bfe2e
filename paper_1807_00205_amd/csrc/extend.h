// Launch interfaces of the region operations: extension and q-gram
// similarity (internal).
#pragma once
#include "sdf_impl.h"

namespace sdf {

// Extension of regions (extend.hip): in/out are device arrays of n regions
// with validated bounds (they may alias).  Throws on a scratch overflow.
struct ExtStats {
    unsigned long long events = 0, restarts = 0, ranks = 0;  // insertions, continued attempts
    unsigned long long rank_us = 0, loop_us = 0;  // workgroup time in gathering/ranking, phases
    unsigned long long slowest_us = 0;            // the slowest region's time
};
void launch_extend(const IndexView &ix, const sdf_region *in, uint64_t n, double tau,
                   uint64_t max_len, sdf_region *out, ExtStats *stats, hipStream_t st);

// q-gram similarity (qgram.hip): out[i] = Q of region i (device arrays).
uint32_t qgram_max_q();
void launch_qgram(const IndexView &ix, const sdf_region *reg, uint64_t n, uint32_t q,
                  unsigned long long *out, hipStream_t st);

}  // namespace sdf
