#pragma once
#include <cstdint>
#include <vector>

#include "common.h"

namespace mplpxx {
// eu[e] < ev[e] for every edge; fills step_ptr (S+1 entries) and order (m).
// kind: MPLPXX_SCHED_AUTO / _GREEDY (round-robin for complete graphs, greedy
// matchings otherwise) or MPLPXX_SCHED_COLOR (edge colouring otherwise).
void build_schedule(int n, const std::vector<int>& eu, const std::vector<int>& ev, std::vector<int>& step_ptr,
                    std::vector<int>& order, int kind = 0);

// A validated graph with its schedule and per-slot metadata.
struct GraphPrep {
  int S = 0;
  std::vector<int> step_ptr, order;  // schedule (edge ids of the input list)
  std::vector<int> slot_of_edge;     // inverse of order
  std::vector<SlotInfo> slots;       // per slot: edge, nodes (u < v), positions
  std::vector<int> flip;             // per input edge: 1 if given as (v, u)
  std::vector<int> deg;              // per node
};

// Validates edges (range, self loops, duplicates) and builds the schedule;
// returns MPLPXX_OK or MPLPXX_EINVAL (with the message in mplpxx_last_error).
int prepare_graph(int n, int m, const int32_t* edges, GraphPrep& g, int kind = 0);
}  // namespace mplpxx
