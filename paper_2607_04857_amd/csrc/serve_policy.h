// serve_policy.h -- scheduling policy of the serving loop (host only, no HIP).
//
// Two decisions, taken on every scheduler tick of the server:
//   * admission: requests enter device slots in arrival order while a slot
//     is free and the device-memory budget allows; the first request that
//     does not fit stops admission (no later request overtakes it);
//   * work per tick: every admitted request with unissued walk items gets a
//     share of the tick's item budget, water-filled so that requests with
//     few items left finish in this tick and the rest share what remains;
//     under a backlog the budget grows (see tick_scale).
// The server (server.cpp) applies them to its device state; a CPU test
// drives the same functions with a mock device.
#pragma once

#include <cstddef>
#include <cstdint>
#include <vector>

namespace qsched {

// How many requests at the head of the queue to admit now.  queued_bytes:
// device bytes of the queued requests, head first; mem_used: bytes held by
// admitted requests; budget: the server's device-memory budget; free_slots:
// free device slots.
size_t admit_count(const std::vector<size_t> &queued_bytes, size_t mem_used, size_t budget,
                   size_t free_slots);

// Largest tick budget multiplier: at 64 a tick gives each resident wave
// about 128 items, so the drain at the tick's end (at most one item per
// wave) costs under 1% of the tick.
constexpr uint64_t kMaxTickScale = 64;

// Budget multiplier for a tick: 1, doubled while the unissued work exceeds
// four ticks' worth at the current multiplier, up to kMaxTickScale (fewer
// tick boundaries under a backlog, where requests wait anyway).
uint64_t tick_scale(uint64_t backlog_items, uint64_t tick_items);

// Items each walking request issues in one tick.  left: unissued items per
// request, ascending (fewest first); tick_items: items per tick at scale 1.
// Returns one share per request (same order): share[k] <= left[k], every
// request with items left gets at least one, and the shares sum to at most
// tick_scale(sum(left), tick_items) * tick_items, or to the number of
// requests when that is larger.
std::vector<uint64_t> tick_shares(const std::vector<uint64_t> &left, uint64_t tick_items);

}  // namespace qsched
