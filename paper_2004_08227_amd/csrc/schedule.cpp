// Edge schedule of Alg. 1 ("Compute Edge Schedule", Sec. 6 of the MPLP++
// paper): the queue is a sequence of matchings that together cover every
// edge once.  A complete graph gets the round-robin 1-factorization (n-1
// rounds for even n, n rounds for odd n, the minimum possible); any other
// graph gets greedy maximal matchings, each round scanning the remaining
// edges in ascending (u, v) order and keeping an edge when both of its nodes
// are still free.  Edges inside one round are listed in ascending (u, v).
//
// On request (kind MPLPXX_SCHED_COLOR) a graph that is not complete gets
// instead the matchings of a proper edge colouring with at most Delta + 1
// colours (Misra and Gries' constructive proof of Vizing's theorem), one
// round per colour in colour order: fewer rounds than the greedy matchings
// when the graph is irregular or dense, i.e. a shorter chain of dependent
// steps per iteration.  Every choice is fixed so that the schedule is a
// function of the edge set alone (the oracle implements the same rule):
//  * edges are coloured in ascending (u, v), u < v, with u the fan's centre;
//  * "a colour free on x" is the smallest colour no edge at x has;
//  * the fan F = [v, ...] is extended, while possible, by the neighbour y
//    not yet in F whose edge (u, y) has the smallest colour that is free on
//    the fan's last node;
//  * c = the colour free on u, d = the colour free on the fan's last node;
//    the path from u whose edges alternate d, c, d, ... is swapped c <-> d;
//  * w = the first node of F (in fan order) on which d is free and up to
//    which F is still a fan; the prefix up to w is rotated (each edge takes
//    the colour of the next fan edge) and (u, w) gets d.
#include <algorithm>
#include <cstdint>
#include <string>
#include <vector>

#include "host_util.h"
#include "schedule.h"

namespace mplpxx {

static inline int64_t key_of(int u, int v, int64_t n) { return (int64_t)u * n + v; }

// Misra-Gries edge colouring; colour[e] in [0, Delta].  at[x * C + c] = the
// edge of colour c at node x, or -1.
static void color_edges(int n, const std::vector<int>& eu, const std::vector<int>& ev, const std::vector<int>& by_key,
                        std::vector<int>& colour, int& ncolours) {
  const int64_t m = (int64_t)eu.size();
  std::vector<int> deg(n, 0);
  for (int64_t e = 0; e < m; ++e) {
    ++deg[eu[e]];
    ++deg[ev[e]];
  }
  const int C = *std::max_element(deg.begin(), deg.end()) + 1;
  ncolours = C;
  colour.assign(m, -1);
  std::vector<int> at((size_t)n * C, -1);
  auto other = [&](int e, int x) { return eu[e] == x ? ev[e] : eu[e]; };
  auto free_on = [&](int x, int c) { return at[(size_t)x * C + c] < 0; };
  auto first_free = [&](int x) {
    int c = 0;
    while (!free_on(x, c)) ++c;
    return c;
  };
  auto set_colour = [&](int e, int c) {
    if (colour[e] >= 0) {
      at[(size_t)eu[e] * C + colour[e]] = -1;
      at[(size_t)ev[e] * C + colour[e]] = -1;
    }
    colour[e] = c;
    if (c >= 0) {
      at[(size_t)eu[e] * C + c] = e;
      at[(size_t)ev[e] * C + c] = e;
    }
  };
  std::vector<int> fan, fan_edge, path;
  std::vector<char> in_fan(n, 0);
  for (int e0 : by_key) {
    const int u = eu[e0], v = ev[e0];
    // maximal fan of u starting at v
    fan.assign(1, v);
    fan_edge.assign(1, e0);
    in_fan[v] = 1;
    for (;;) {
      const int x = fan.back();
      int next = -1, next_e = -1;
      for (int c = 0; c < C; ++c) {
        if (!free_on(x, c)) continue;
        const int e = at[(size_t)u * C + c];
        if (e < 0) continue;
        const int y = other(e, u);
        if (in_fan[y]) continue;
        next = y;
        next_e = e;
        break;
      }
      if (next < 0) break;
      fan.push_back(next);
      fan_edge.push_back(next_e);
      in_fan[next] = 1;
    }
    for (int y : fan) in_fan[y] = 0;
    const int c = first_free(u);
    const int d = first_free(fan.back());
    if (c != d) {
      // the path from u alternating d, c, d, ...: swap its colours
      path.clear();
      int x = u, want = d;
      for (;;) {
        const int e = at[(size_t)x * C + want];
        if (e < 0) break;
        path.push_back(e);
        x = other(e, x);
        want = want == d ? c : d;
      }
      for (int e : path) set_colour(e, colour[e] == c ? -2 : -3);   // clear first
      for (int e : path) {
        const int was = colour[e];
        colour[e] = -1;
        set_colour(e, was == -2 ? d : c);
      }
    }
    // w: the first fan node with d free, up to which F is still a fan
    size_t wi = 0;
    bool found = false;
    for (size_t i = 0; i < fan.size(); ++i) {
      if (i > 0) {
        const int ci = colour[fan_edge[i]];
        if (ci < 0 || !free_on(fan[i - 1], ci)) break;
      }
      if (free_on(fan[i], d)) {
        wi = i;
        found = true;
        break;
      }
    }
    if (!found) wi = 0;  // (cannot happen for a proper colouring; keeps the loop total)
    // rotate the prefix: edge i takes the colour of edge i + 1, (u, w) gets d
    for (size_t i = 0; i < wi; ++i) {
      const int cn = colour[fan_edge[i + 1]];
      set_colour(fan_edge[i + 1], -1);
      set_colour(fan_edge[i], cn);
    }
    set_colour(fan_edge[wi], d);
  }
}

void build_schedule(int n, const std::vector<int>& eu, const std::vector<int>& ev, std::vector<int>& step_ptr,
                    std::vector<int>& order, int kind) {
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

  if (kind == MPLPXX_SCHED_COLOR && m != (int64_t)n * (n - 1) / 2) {
    std::vector<int> colour;
    int C = 0;
    color_edges(n, eu, ev, by_key, colour, C);
    std::vector<std::vector<int>> rounds(C);
    for (int e : by_key) rounds[colour[e]].push_back(e);   // ascending (u, v) within a colour
    for (const auto& r : rounds) {
      if (r.empty()) continue;
      order.insert(order.end(), r.begin(), r.end());
      step_ptr.push_back((int)order.size());
    }
    return;
  }
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

// A schedule is valid when its rounds list every edge exactly once and no
// node twice within a round (Alg. 1: the rounds are matchings).  The
// engines rely on both: the updates of a round run concurrently, and a
// node's updates are counted in schedule order.
static bool schedule_is_valid(int n, const std::vector<int>& eu, const std::vector<int>& ev,
                              const std::vector<int>& step_ptr, const std::vector<int>& order, std::string* why) {
  const int m = (int)eu.size();
  if ((int)order.size() != m || step_ptr.empty() || step_ptr.front() != 0 || step_ptr.back() != m) {
    *why = "the rounds do not cover the edges";
    return false;
  }
  std::vector<char> seen(m, 0);
  std::vector<int> round_of(n, -1);
  for (int k = 0; k + 1 < (int)step_ptr.size(); ++k) {
    if (step_ptr[k + 1] < step_ptr[k]) {
      *why = "round boundaries out of order";
      return false;
    }
    for (int i = step_ptr[k]; i < step_ptr[k + 1]; ++i) {
      const int e = order[i];
      if (e < 0 || e >= m || seen[e]) {
        *why = "an edge is missing or listed twice";
        return false;
      }
      seen[e] = 1;
      for (int x : {eu[e], ev[e]}) {
        if (round_of[x] == k) {
          *why = "round " + std::to_string(k) + " is not a matching (node " + std::to_string(x) + ")";
          return false;
        }
        round_of[x] = k;
      }
    }
  }
  return true;
}

int prepare_graph(int n, int m, const int32_t* edges, GraphPrep& g, int kind) {
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
  build_schedule(n, eu, ev, g.step_ptr, g.order, kind);
  g.S = (int)g.step_ptr.size() - 1;
  {
    std::string why;
    if (!schedule_is_valid(n, eu, ev, g.step_ptr, g.order, &why))
      return fail(MPLPXX_EINVAL, "internal: invalid schedule (%s)", why.c_str());
  }
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
