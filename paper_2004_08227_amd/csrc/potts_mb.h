// Mailbox engine (persistent, FP32) for models with structured pairwise
// costs (Potts th(s,t) = w [s != t], truncated linear w min(|s - t|, tau))
// and L <= 64: the single-model counterpart of the wave engine's structured
// instances.  A workgroup is one compute wave (label l on lane l, the three
// passes of potts_passes.h) plus the two sync waves of the dense engine,
// which poll the mailboxes of the next step's two nodes and deliver them to
// LDS.  The tables hold the cost's parameters per slot.  For Potts costs
// every value is formed by the same IEEE operations as in the dense
// engines, so the results are bitwise those of the dense engine on the
// expanded table.
//
// Per step both kinds of waves meet at one barrier (the step's nodes are in
// LDS); there is no mid-step barrier as in mb_run, since the compute wave
// exchanges nothing with other waves.  The sync waves then go on to the next
// step's nodes, which go to the other half of the double buffer (slot
// parity); they come back to this half only after the compute wave has
// reached the next step's barrier, i.e. after it has read this step's
// values, so the next gathers overlap its passes.
#pragma once
#include "potts_passes.h"

namespace mplpxx {

constexpr int kPottsNT = 64;  // compute threads of the Potts instance

template <bool PHI_LDS, int KIND = MPLPXX_COST_POTTS>
__device__ __forceinline__ bool mb_run_potts(const MbView& v_in, int first_in, int stride_in, int iters_in,
                                             SmemMB<64, kPottsNT>& sm, float* phi_lds, long long spin_limit,
                                             int* err) {
  MbView v = v_in;
  v.L = uni(v.L);
  v.m = uni(v.m);
  v.n = uni(v.n);
  const int first = uni(first_in), stride = uni(stride_in), iters = uni(iters_in);
  const int tid = threadIdx.x;
  const int L = v.L;
  const int wave = tid >> 6, lane = tid & 63;
  if (first >= v.m) return true;
  const int owned = (v.m - first + stride - 1) / stride;
  const int total = owned * iters;
  if (tid >= kPottsNT) {
    // ---- sync waves: wait for (or read) the step's two nodes ----
    const bool is_sync_u = wave == kPottsNT / 64;
    SlotInfo si = ld_const(v.slots + first);
    int parity = 0, it = 0, j = 0;
    for (int q = 0; q < total; ++q) {
      const int slot = first + j * stride;
      const unsigned want_u = (unsigned)it * (unsigned)si.deg_u + (unsigned)si.pos_u;
      const unsigned want_v = (unsigned)it * (unsigned)si.deg_v + (unsigned)si.pos_v;
      int nxt = slot + stride;
      if (nxt >= v.m) nxt = first;
      nxt = uni(nxt);
      const bool last_iter = it == iters - 1;
      const SlotInfo si_next = ld_const(v.slots + nxt);
      if (v.stamps && last_iter && lane == 0 && is_sync_u) v.stamps[(size_t)slot * kStampStride + 0] = wall_clock64();
      const int node = is_sync_u ? si.u : si.v;
      const unsigned want = is_sync_u ? want_u : want_v;
      float* dst = is_sync_u ? sm.uu[parity] : sm.uv[parity];
      float* dst_hi = is_sync_u ? sm.uh[parity] : sm.vh[parity];
      float* dst_lo = is_sync_u ? sm.ul[parity] : sm.vl[parity];
      unsigned seen = 0;
      if (!sync_gather<64>(v.mb + (size_t)node * L, L, want, dst, dst_hi, dst_lo, &sm.cc[parity][is_sync_u ? 0 : 1],
                           spin_limit, err, &seen)) {
        if (lane == 0) {
          if (ld_dev(err) == 0 || seen != (want & 0xFFFFu)) report_timeout(err, slot, node, want & 0xFFFFu, seen);
          sm.abort_flag = 1;
        }
      }
      if (v.stamps && last_iter && lane == 0) v.stamps[(size_t)slot * kStampStride + (is_sync_u ? 1 : 2)] = wall_clock64();
      __syncthreads();
      if (sm.abort_flag) return false;
      si = si_next;
      parity ^= 1;
      if (++j == owned) { j = 0; ++it; }
    }
    return true;
  }

  // ---- the compute wave: lane = label ----
  const bool lout = lane < L;                  // this lane's label is real
  const int li = lout ? lane : L - 1;          // in range for every lane
  // lanes without a label store to one scratch word (per kind of store)
  float* sink_f = reinterpret_cast<float*>(v.sink + kPottsNT);
  SlotInfo si = ld_const(v.slots + first);
  int parity = 0, it = 0, j = 0;
  for (int q = 0; q < total; ++q) {
    const int slot = first + j * stride;
    const unsigned want_u = (unsigned)it * (unsigned)si.deg_u + (unsigned)si.pos_u;
    const unsigned want_v = (unsigned)it * (unsigned)si.deg_v + (unsigned)si.pos_v;
    int nxt = slot + stride;
    if (nxt >= v.m) nxt = first;
    nxt = uni(nxt);
    const bool last_iter = it == iters - 1;
    const SlotInfo si_next = ld_const(v.slots + nxt);
    // the slot's cost parameters and old messages (each label's message is
    // written and read only by this lane, so program order suffices)
    const float* prm = v.tables + (size_t)slot * cost_params(KIND);
    float* ph = PHI_LDS ? phi_lds + (size_t)j * 2 * L : v.phi + (size_t)slot * 2 * L;
    const float fu = ph[li], fv = ph[L + li];
    __syncthreads();  // the step's nodes are in LDS
    if (sm.abort_flag) return false;
    const float au = sm.uu[parity][li] - fu;  // centred (hi - c) + lo, minus the message
    const float av = sm.uv[parity][li] - fv;
    const float hu = sm.uh[parity][li], lu = sm.ul[parity][li];
    const float hv = sm.vh[parity][li], lv = sm.vl[parity][li];
    const float delta = 0.5f * (sm.cc[parity][0] - sm.cc[parity][1]);
    float phu, phv;
    structured_passes<KIND>(au, av, prm, lout, L, delta, phu, phv);
    float nhu, nlu, nhv, nlv;
    comp_update(hu, lu, fu, phu, nhu, nlu);
    comp_update(hv, lv, fv, phv, nhv, nlv);
    // push back (every lane issues the same stores)
    mb_store(lout ? v.mb + (size_t)si.u * L + lane : v.sink, mb_pack(nhu, nlu, want_u + 1));
    mb_store(lout ? v.mb + (size_t)si.v * L + lane : v.sink + 1, mb_pack(nhv, nlv, want_v + 1));
    if (PHI_LDS) {
      if (lout) {
        ph[lane] = phu;
        ph[L + lane] = phv;
      }
    } else {
      *(lout ? ph + lane : sink_f) = phu;
      *(lout ? ph + L + lane : sink_f + 1) = phv;
    }
    {
      const bool st = v.stamps && last_iter && tid == 0;
      long long* dst = st ? v.stamps + (size_t)slot * kStampStride + 3 : reinterpret_cast<long long*>(v.sink + kPottsNT + 1);
      *dst = st ? (long long)wall_clock64() : 0;
    }
    si = si_next;
    parity ^= 1;
    if (++j == owned) { j = 0; ++it; }
  }
  return true;
}

}  // namespace mplpxx
