/* Pairwise tables of the 6D-pose-shaped synthetic workload (input
 * generation only; no solver arithmetic).  For edge e = (u, v):
 *   table[e][s][t] = (float) min((dp - dq)^2, tau),
 *   dp = |P[u][s] - P[v][t]|, dq = |Q[u] - Q[v]|,
 * every operation in FP64 in this exact order:
 *   d = sqrt((dx*dx + dy*dy) + dz*dz), c = (dp - dq) * (dp - dq).
 * The numpy fallback in workloads.py performs the same operations, so both
 * produce the same bits (IEEE add, multiply and sqrt are correctly rounded).
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fno-fast-math. */
#include <math.h>
#include <stdint.h>

void pose_tables(int64_t m, int L, const int32_t* edges, const double* P /* [n][L][3] */,
                 const double* Q /* [n][3] */, double tau, float* out /* [m][L][L] */) {
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < m; ++e) {
    const int u = edges[2 * e], v = edges[2 * e + 1];
    const double qx = Q[3 * u] - Q[3 * v], qy = Q[3 * u + 1] - Q[3 * v + 1], qz = Q[3 * u + 2] - Q[3 * v + 2];
    const double dq = sqrt((qx * qx + qy * qy) + qz * qz);
    float* o = out + e * (int64_t)L * L;
    const double* pu = P + (int64_t)u * L * 3;
    const double* pv = P + (int64_t)v * L * 3;
    for (int s = 0; s < L; ++s) {
      for (int t = 0; t < L; ++t) {
        const double dx = pu[3 * s] - pv[3 * t], dy = pu[3 * s + 1] - pv[3 * t + 1], dz = pu[3 * s + 2] - pv[3 * t + 2];
        const double dp = sqrt((dx * dx + dy * dy) + dz * dz);
        const double d = dp - dq;
        const double c = d * d;
        o[s * L + t] = (float)(c < tau ? c : tau);
      }
    }
  }
}
