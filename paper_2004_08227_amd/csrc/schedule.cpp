// Edge schedule of Alg. 1 ("Compute Edge Schedule", Sec. 6 of the MPLP++
// paper): the queue is a sequence of matchings that together cover every
// edge once.  A complete graph gets the round-robin 1-factorization (n-1
// rounds for even n, n rounds for odd n, the minimum possible); any other
// graph gets greedy maximal matchings, each round scanning the remaining
// edges in ascending (u, v) order and keeping an edge when both of its nodes
// are still free.  Edges inside one round are listed in ascending (u, v).
#include <algorithm>
#include <cstdint>
#include <vector>

#include "host_util.h"
#include "schedule.h"

namespace mplpxx {

static inline int64_t key_of(int u, int v, int64_t n) { return (int64_t)u * n + v; }

void build_schedule(int n, const std::vector<int>& eu, const std::vector<int>& ev, std::vector<int>& step_ptr,
                    std::vector<int>& order) {
  const int64_t m = (int64_t)eu.size();
  step_ptr.clear();
  order.clear();
  step_ptr.push_back(0);
  if (m == 0) return;
  // edge ids sorted by (u, v)
  std::vector<int> by_key(m);
  for (int64_t e = 0; e < m; ++e) by_key[e] = (int)e;
  std::sort(by_key.begin(), by_key.end(), [&](int a, int b) { return key_of(eu[a], ev[a], n) < key_of(eu[b], ev[b], n); });
  std::vector<int64_t> keys(m);
  for (int64_t i = 0; i < m; ++i) keys[i] = key_of(eu[by_key[i]], ev[by_key[i]], n);
  auto edge_id = [&](int a, int b) -> int {
    const int u = std::min(a, b), v = std::max(a, b);
    const int64_t k = key_of(u, v, n);
    auto it = std::lower_bound(keys.begin(), keys.end(), k);
    return (it != keys.end() && *it == k) ? by_key[it - keys.begin()] : -1;
  };
  auto by_uv = [&](int a, int b) { return key_of(eu[a], ev[a], n) < key_of(eu[b], ev[b], n); };

  if (m == (int64_t)n * (n - 1) / 2) {
    // round-robin: a ring of N-1 positions plus a fixed node N-1; with odd n
    // the fixed node is a dummy and its partner sits the round out
    const int N = n + (n & 1);
    const int R = N - 1;
    std::vector<int> round;
    for (int r = 0; r < R; ++r) {
      round.clear();
      if (N - 1 < n) round.push_back(edge_id(N - 1, r));
      for (int k = 1; k <= N / 2 - 1; ++k) {
        const int a = (r + k) % R;
        const int b = (r - k + R) % R;
        round.push_back(edge_id(a, b));
      }
      std::sort(round.begin(), round.end(), by_uv);
      order.insert(order.end(), round.begin(), round.end());
      step_ptr.push_back((int)order.size());
    }
    return;
  }
  // greedy maximal matchings in (u, v) order
  std::vector<int> rest(by_key.begin(), by_key.end()), next;
  std::vector<int> used(n, -1);
  int round_id = 0;
  while (!rest.empty()) {
    next.clear();
    for (int e : rest) {
      if (used[eu[e]] != round_id && used[ev[e]] != round_id) {
        used[eu[e]] = used[ev[e]] = round_id;
        order.push_back(e);
      } else {
        next.push_back(e);
      }
    }
    step_ptr.push_back((int)order.size());
    rest.swap(next);
    ++round_id;
  }
}

int prepare_graph(int n, int m, const int32_t* edges, GraphPrep& g) {
  std::vector<int> eu(m), ev(m);
  g.flip.assign(m, 0);
  for (int e = 0; e < m; ++e) {
    const int a = edges[2 * e], b = edges[2 * e + 1];
    if (a < 0 || a >= n || b < 0 || b >= n) return fail(MPLPXX_EINVAL, "edge %d: node index out of range", e);
    if (a == b) return fail(MPLPXX_EINVAL, "edge %d: self loop", e);
    eu[e] = std::min(a, b);
    ev[e] = std::max(a, b);
    g.flip[e] = a > b;
  }
  {
    std::vector<int64_t> keys(m);
    for (int e = 0; e < m; ++e) keys[e] = (int64_t)eu[e] * n + ev[e];
    std::sort(keys.begin(), keys.end());
    for (int e = 1; e < m; ++e)
      if (keys[e] == keys[e - 1])
        return fail(MPLPXX_EINVAL, "duplicate edge (%lld, %lld)", (long long)(keys[e] / n), (long long)(keys[e] % n));
  }
  build_schedule(n, eu, ev, g.step_ptr, g.order);
  g.S = (int)g.step_ptr.size() - 1;
  if ((int)g.order.size() != m) return fail(MPLPXX_EINVAL, "internal: schedule does not cover the edges");
  g.slot_of_edge.assign(m, -1);
  g.slots.resize(m);
  g.deg.assign(n, 0);
  for (int i = 0; i < m; ++i) {
    const int e = g.order[i];
    g.slot_of_edge[e] = i;
    SlotInfo si{};
    si.e = e;
    si.u = eu[e];
    si.v = ev[e];
    si.pos_u = g.deg[si.u]++;
    si.pos_v = g.deg[si.v]++;
    g.slots[i] = si;
  }
  for (int i = 0; i < m; ++i) {
    g.slots[i].deg_u = g.deg[g.slots[i].u];
    g.slots[i].deg_v = g.deg[g.slots[i].v];
  }
  for (int k = 0; k < g.S; ++k)
    for (int i = g.step_ptr[k]; i < g.step_ptr[k + 1]; ++i) g.slots[i].step = k;
  return MPLPXX_OK;
}

}  // namespace mplpxx
