// serve_policy.cpp -- scheduling policy of the serving loop (host only).
#include "serve_policy.h"

#include <algorithm>

namespace qsched {

size_t admit_count(const std::vector<size_t> &queued_bytes, size_t mem_used, size_t budget,
                   size_t free_slots)
{
    size_t k = 0;
    for (; k < queued_bytes.size() && k < free_slots; k++) {
        if (queued_bytes[k] > budget || mem_used > budget - queued_bytes[k]) break;
        mem_used += queued_bytes[k];
    }
    return k;
}

uint64_t tick_scale(uint64_t backlog_items, uint64_t tick_items)
{
    uint64_t scale = 1;
    while (scale < kMaxTickScale && backlog_items > 4 * scale * tick_items) scale *= 2;
    return scale;
}

std::vector<uint64_t> tick_shares(const std::vector<uint64_t> &left, uint64_t tick_items)
{
    uint64_t backlog = 0;
    for (uint64_t l : left) backlog += l;
    uint64_t budget = tick_scale(backlog, tick_items) * tick_items;
    std::vector<uint64_t> share(left.size(), 0);
    for (size_t k = 0; k < left.size(); k++) {
        const uint64_t fair = std::max<uint64_t>(1, budget / (left.size() - k));
        share[k] = std::min(left[k], fair);
        budget = budget > share[k] ? budget - share[k] : 0;
    }
    return share;
}

}  // namespace qsched
