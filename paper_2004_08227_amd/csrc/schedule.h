#pragma once
#include <vector>

namespace mplpxx {
// eu[e] < ev[e] for every edge; fills step_ptr (S+1 entries) and order (m).
void build_schedule(int n, const std::vector<int>& eu, const std::vector<int>& ev, std::vector<int>& step_ptr,
                    std::vector<int>& order);
}  // namespace mplpxx
