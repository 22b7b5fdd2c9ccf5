// SMICE as the search's second key (Algorithm 1's selection, MICE of Section
// II.C): among the feasible masks of the chosen level, the one whose clusters'
// largest member errors, summed over clusters and snapshots, are smallest.
//
// Only clusters that a mask can touch are summed (the others add the same
// constant to every mask): every kept slot's cluster (the slot and the
// reduced slots below it down to the next kept one), every zone target's
// cluster, and every chain head's cluster (the head's own members, whose
// error is fixed when the head lies outside Omega_g, plus the reduced slots
// at the top of each chain below it).  A cluster's error on a phase is
// max(|V_super| - lo, hi - |V_super|) over its member groups (lo, hi: the
// groups' extreme |V^|), so each group enters once per phase, as in the
// per-mask scoring.
//
//   k_smice_prep   (1 block)  distinct heads, zone targets grouped by their
//                             anchor chain in Omega_g order, head maxima zeroed
//   k_smice_hconst (grid)     fixed error of each outside head's cluster
//   k_smice_score  (grid)     SMICE of every candidate mask (and of mask 0)
//   k_smice_argmin (1 block)  the smallest SMICE, tie rule, margin, flags
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "okr_device.h"
#include "okr_internal.h"

namespace okr {

// Node of Omega_g with flattened index q (ranges: start, end, cumulative).
__device__ __forceinline__ int sm_omega_node(const Topo& T, const int* rg, int nr, int q) {
  int r = 0;
  while (r + 1 < nr && rg[3 * (r + 1) + 2] <= q) ++r;
  return T.pre[rg[3 * r] + (q - rg[3 * r + 2])];
}

// Zone entry of the lowest present phase of node i, or -1 if i is not a
// zone target of this segment.
__device__ __forceinline__ int sm_first_entry(const Topo& T, const State& St, int i, int nz) {
  const unsigned ph = T.phase[i];
  for (int p = 0; p < 3; ++p)
    if (ph >> p & 1u) {
      const int e = St.zent_of[i * 3 + p];
      return (e >= 0 && e < nz) ? e : -1;
    }
  return -1;
}

__global__ __launch_bounds__(256) void k_smice_prep(const SegHdr* __restrict__ hdrs, const int* __restrict__ segs,
                                                    size_t lstride, const int* __restrict__ tab, Topo T, State St,
                                                    int* __restrict__ stab, double* __restrict__ hK, int S) {
  __shared__ int s_cnt[256][kMaxK];  // per thread: zone targets of its Omega range per anchor chain
  __shared__ int s_tot[kMaxK + 1];
  __shared__ int s_hnode[kMaxK], s_hin[kMaxK], s_chx[kMaxK], s_nh;
  const int g = segs[blockIdx.z];
  const SegHdr H = load_hdr_g(hdrs, g);
  tab = lane_ptr(tab, lstride);
  stab = lane_ptr(stab, lstride);
  hK = lane_ptr(hK, lstride);
  const int tid = threadIdx.x;
  if (!H.valid) {
    if (tid == 0) {
      stab[SM_NH] = 0;
      stab[SM_NZN] = 0;
    }
    return;
  }
  const int nch = H.nchains;
  const int* chains = tab + H.o_chain;
  if (tid == 0) {  // distinct heads in chain order
    int nh = 0;
    for (int c = 0; c < nch; ++c) {
      const int hd = chains[c * kChainInts + C_HEAD];
      int x = 0;
      while (x < nh && s_hnode[x] != hd) ++x;
      if (x == nh) {
        s_hnode[nh] = hd;
        s_hin[nh] = chains[c * kChainInts + C_OUTER] >= 0 ? 1 : 0;
        ++nh;
      }
      s_chx[c] = x;
    }
    s_nh = nh;
  }
  for (int c = 0; c < nch; ++c) s_cnt[tid][c] = 0;
  __syncthreads();
  const int nh = s_nh;
  for (int t = tid; t < nh * S; t += blockDim.x) hK[t] = 0.0;
  // zone targets in Omega_g order: thread tid owns a contiguous range of it
  const int* rg = tab + H.o_range;
  const int nom = H.nomega, per = (nom + 255) / 256;
  const int q0 = min(nom, tid * per), q1 = min(nom, q0 + per);
  for (int q = q0; q < q1; ++q) {
    const int i = sm_omega_node(T, rg, H.nrange, q);
    const int e = sm_first_entry(T, St, i, H.nz);
    if (e >= 0) s_cnt[tid][tab[H.o_zent + 3 * e + 2]]++;
  }
  __syncthreads();
  if (tid < nch) {  // exclusive scan over threads, per chain
    int acc = 0;
    for (int t = 0; t < 256; ++t) {
      const int v = s_cnt[t][tid];
      s_cnt[t][tid] = acc;
      acc += v;
    }
    s_tot[tid] = acc;
  }
  __syncthreads();
  if (tid == 0) {
    int acc = 0;
    for (int c = 0; c < nch; ++c) {
      const int v = s_tot[c];
      s_tot[c] = acc;
      stab[SM_ZOFF + c] = acc;
      acc += v;
    }
    s_tot[nch] = acc;
    stab[SM_ZOFF + nch] = acc;
    stab[SM_NZN] = acc;
    stab[SM_NH] = nh;
  }
  if (tid < nch) stab[SM_CHX + tid] = s_chx[tid];
  if (tid < nh) {
    stab[SM_HNODE + tid] = s_hnode[tid];
    stab[SM_HIN + tid] = s_hin[tid];
  }
  __syncthreads();
  for (int q = q0; q < q1; ++q) {
    const int i = sm_omega_node(T, rg, H.nrange, q);
    const int e = sm_first_entry(T, St, i, H.nz);
    if (e < 0) continue;
    const int c = tab[H.o_zent + 3 * e + 2];
    const int at = s_tot[c] + s_cnt[tid][c]++;
    int* zr = stab + SM_ZREC + at * kZrecInts;
    zr[0] = i;
    const unsigned ph = T.phase[i];
    for (int p = 0; p < 3; ++p) {
      const int ep = St.zent_of[i * 3 + p];
      zr[1 + p] = ((ph >> p & 1u) && ep >= 0 && ep < H.nz) ? ep : -1;
    }
    int hx = -1;
    for (int x = 0; x < nh; ++x)
      if (s_hnode[x] == i) hx = x;
    zr[4] = hx;
  }
}

// Fixed error of the cluster of every head outside Omega_g, per snapshot:
// the largest error over its members (every node whose super-node it is,
// itself included) and their phases, against its unchanging voltage.
__global__ __launch_bounds__(256) void k_smice_hconst(const SegHdr* __restrict__ hdrs, const int* __restrict__ segs,
                                                      size_t lstride, Topo T, State St,
                                                      const double2* __restrict__ Vcur,
                                                      const double* __restrict__ absV,
                                                      const int* __restrict__ stab, double* __restrict__ hK, int S) {
  __shared__ int s_hnode[kMaxK], s_hin[kMaxK];
  const int g = segs[blockIdx.z];
  const SegHdr H = load_hdr_g(hdrs, g);
  if (!H.valid) return;
  stab = lane_ptr(stab, lstride);
  hK = lane_ptr(hK, lstride);
  const int nh = stab[SM_NH];
  if (threadIdx.x < nh) {
    s_hnode[threadIdx.x] = stab[SM_HNODE + threadIdx.x];
    s_hin[threadIdx.x] = stab[SM_HIN + threadIdx.x];
  }
  __syncthreads();
  const int n = T.n;
  const long total = (long)n * S;
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
    const int l = (int)(t / n), i = (int)(t % n);
    const int sp = St.sup[i];
    int x = -1;
    for (int y = 0; y < nh; ++y)
      if (s_hnode[y] == sp && !s_hin[y]) x = y;
    if (x < 0) continue;
    const unsigned ph = T.phase[i];
    double e = 0.0;
    for (int p = 0; p < 3; ++p)
      if (ph >> p & 1u) {
        const double2 v = Vcur[((size_t)l * n + sp) * 3 + p];
        e = fmax(e, fabs(vmag(v) - absV[((size_t)l * n + i) * 3 + p]));
      }
    atomicMax((unsigned long long*)&hK[x * S + l], (unsigned long long)__double_as_longlong(e));
  }
}

// Voltage shift at the bottom of one chain for mask m (the currents its
// reduced slots move to their super-nodes), added to B.
__device__ __forceinline__ void sm_shift_chain(const cint* cr, const double2* Pl, uint32_t m, double2 (&B)[3]) {
  const int ns = cr[C_NSLOT], pair0 = cr[C_PAIR0], bit0 = cr[C_BIT0];
  const int phw0 = cr[C_PHW0], phw1 = cr[C_PHW1], phw2 = cr[C_PHW2];
  int sidx = 0;
  for (int r = 0; r < ns; ++r) {
    if ((m >> (bit0 + r)) & 1u) {
      const int w = r < 8 ? phw0 : (r < 16 ? phw1 : phw2);
      const int ph = (w >> (3 * (r & 7))) & 7;
      const double2* pr = Pl + (pair0 + ((r * (r + 1)) >> 1) + sidx) * 3;
#pragma unroll
      for (int p = 0; p < 3; ++p)
        if (ph >> p & 1) B[p] = cadd(B[p], pr[p]);  // the slot's present phases only
    } else {
      sidx = r + 1;
    }
  }
}

// Error of one member group (extreme |V^| lo, hi) against a super-node
// magnitude.
__device__ __forceinline__ double sm_group(double mag, double lo, double hi) { return fmax(mag - lo, hi - mag); }

// SMICE over the clusters a mask can touch, summed over the snapshots, for
// every feasible mask of the chosen level (others: +inf) and for mask 0.
// One mask per thread; per-thread head maxima in LDS.
constexpr int kSmiceThreads = 128;
__global__ __launch_bounds__(kSmiceThreads) void k_smice_score(
    const SegHdr* __restrict__ hdrs, const int* __restrict__ segs, size_t lstride, const int* __restrict__ tab,
    const double2* __restrict__ P, const TargetRec* __restrict__ srec, const double2* __restrict__ headV,
    const TargetRec* __restrict__ zrec, const int* __restrict__ stab, const double* __restrict__ hK,
    const MaskScore* __restrict__ fin, const TileRec* __restrict__ tiles, const DevDecision* __restrict__ decs,
    SelParams sp, double* __restrict__ smv, double* __restrict__ smv0) {
  __shared__ double s_acc[kMaxK][kSmiceThreads];
  const int g = segs[blockIdx.z];
  const SegHdr H = load_hdr_g(hdrs, g);
  if (!H.valid) return;
  const DevDecision d = decs[g];
  if (!d.found) return;
  const uint32_t nmask = 1u << H.k;
  // thread i: lane i % 64 of scoring tile i / 64 (tile_mask), so that the
  // tile record of its mask is at hand
  const uint32_t L = (uint32_t)H.lanebits;
  const uint32_t ti = blockIdx.x * kSmiceThreads + threadIdx.x;
  const uint32_t tile = ti / kScoreBlock, q = ti % kScoreBlock;
  if ((tile << __popc(L)) >= nmask || (q >> __popc(L)) != 0) return;
  const uint32_t m = tile_mask(L, tile, q, H.k);
  tab = lane_ptr(tab, lstride);
  P = lane_ptr(P, lstride);
  srec = lane_ptr(srec, lstride);
  headV = lane_ptr(headV, lstride);
  zrec = lane_ptr(zrec, lstride);
  stab = lane_ptr(stab, lstride);
  hK = lane_ptr(hK, lstride);
  fin = lane_ptr(fin, lstride);
  tiles = lane_ptr(tiles, lstride);
  smv = lane_ptr(smv, lstride);
  smv0 = lane_ptr(smv0, lstride);
  // (a tile stores the scores of its best feasible level only: a tile whose
  // best is below the chosen level has no feasible mask at it)
  const bool cand = __popc(m) == d.popcount && tiles[tile].best == d.popcount &&
                    feasible(fin[m], sp.e_bar);
  if (!cand && m != 0) {
    smv[m] = INFINITY;
    return;
  }
  const int tid = threadIdx.x;
  const int S = H.S, nh = stab[SM_NH];
  const cint* chains = as_cint(tab + H.o_chain);
  const cint* nest = as_cint(tab + H.o_nest);
  const int* zr0 = stab + SM_ZREC;
  double total = 0.0;
  for (int l = 0; l < S; ++l) {
    const double2* Pl = P + (size_t)l * H.npairs * 3;
    const TargetRec* Tl = srec + (size_t)l * H.nslots * 3;
    const double2* Hl = headV + (size_t)l * H.nchains * 3;
    const TargetRec* Zl = zrec + (size_t)l * H.nz;
    for (int x = 0; x < nh; ++x) s_acc[x][tid] = stab[SM_HIN + x] ? 0.0 : hK[x * S + l];
    double tot = 0.0;
    for (int c = 0; c < H.nchains; ++c) {
      const cint* cr = chains + c * kChainInts;
      double2 B[3];
#pragma unroll
      for (int p = 0; p < 3; ++p) B[p] = make_double2(0.0, 0.0);
      const int nl = cr[C_NEST_LEN], no = cr[C_NEST_OFF];
      for (int q = 0; q + 1 < nl; ++q) sm_shift_chain(chains + nest[no + q] * kChainInts, Pl, m, B);
      // the head's magnitude (moved by the outer chains when it lies below one)
      const int hph = cr[C_PHASE];
      const bool inner = cr[C_OUTER] >= 0;
      double smag[3];
#pragma unroll
      for (int p = 0; p < 3; ++p) {
        const double2 v = inner ? cadd(Hl[c * 3 + p], B[p]) : Hl[c * 3 + p];
        smag[p] = (hph >> p & 1) ? vmag(v) : 0.0;
      }
      const int hx = stab[SM_CHX + c];
      const int ns = cr[C_NSLOT], s0 = cr[C_SLOT0], pair0 = cr[C_PAIR0], bit0 = cr[C_BIT0];
      const int phw0 = cr[C_PHW0], phw1 = cr[C_PHW1], phw2 = cr[C_PHW2];
      int sidx = 0;
      bool open = false;
      double cl = 0.0;
      for (int r = 0; r < ns; ++r) {
        const int w = r < 8 ? phw0 : (r < 16 ? phw1 : phw2);
        const int ph = (w >> (3 * (r & 7))) & 7;
        const TargetRec* tr = Tl + (s0 + r) * 3;
        if ((m >> (bit0 + r)) & 1u) {  // reduced: its group joins the current super-node's cluster
          const double2* pr = Pl + (pair0 + ((r * (r + 1)) >> 1) + sidx) * 3;
          double er = 0.0;
#pragma unroll
          for (int p = 0; p < 3; ++p) {
            if (!(ph >> p & 1)) continue;
            B[p] = cadd(B[p], pr[p]);
            er = fmax(er, sm_group(smag[p], tr[p].lo, tr[p].hi));
          }
          if (sidx == 0) s_acc[hx][tid] = fmax(s_acc[hx][tid], er);
          else cl = fmax(cl, er);
        } else {  // kept: closes the cluster above, opens its own
          if (open) tot += cl;
          double er = 0.0;
#pragma unroll
          for (int p = 0; p < 3; ++p) {
            if (!(ph >> p & 1)) continue;
            const double mg = vmag(cadd(tr[p].W, B[p]));
            smag[p] = mg;
            er = fmax(er, sm_group(mg, tr[p].lo, tr[p].hi));
          }
          cl = er;
          open = true;
          sidx = r + 1;
        }
      }
      if (open) tot += cl;
      // zone targets anchored at this chain: their voltage moves with the
      // chain's bottom shift; a target that heads chains below keeps the
      // maximum for the head's cluster
      for (int z = stab[SM_ZOFF + c], ze = stab[SM_ZOFF + c + 1]; z < ze; ++z) {
        const int* zr = zr0 + z * kZrecInts;
        double ez = 0.0;
#pragma unroll
        for (int p = 0; p < 3; ++p) {
          const int e = zr[1 + p];
          if (e < 0) continue;
          const TargetRec t = Zl[e];
          ez = fmax(ez, sm_group(vmag(cadd(t.W, B[p])), t.lo, t.hi));
        }
        if (zr[4] >= 0) s_acc[zr[4]][tid] = fmax(s_acc[zr[4]][tid], ez);
        else tot += ez;
      }
    }
    for (int x = 0; x < nh; ++x) tot += s_acc[x][tid];
    total += tot;
  }
  if (m == 0) *smv0 = total;
  smv[m] = cand ? total : INFINITY;
}

// The decision under SMICE: the smallest SMICE among the candidates, the
// lowest mask within tol of it, the margin to the next one outside, and the
// ambiguity flags (a candidate within tol/100 of the tie-window edge, or a
// mask at the chosen level or above near the e_bar / band boundary).
__global__ __launch_bounds__(1024) void k_smice_argmin(const SegHdr* __restrict__ hdrs, const int* __restrict__ segs,
                                                       size_t lstride, const MaskScore* __restrict__ fin,
                                                       const TileRec* __restrict__ tiles,
                                                       const double* __restrict__ smv,
                                                       const double* __restrict__ smv0, double tol,
                                                       DevDecision* __restrict__ decs) {
  __shared__ double shd[16];
  __shared__ int shi[16];
  __shared__ unsigned shu[16];
  const int g = segs[blockIdx.z];
  const SegHdr H = load_hdr_g(hdrs, g);
  if (!H.valid) return;
  DevDecision d = decs[g];
  if (!d.found) return;
  fin = lane_ptr(fin, lstride);
  tiles = lane_ptr(tiles, lstride);
  smv = lane_ptr(smv, lstride);
  smv0 = lane_ptr(smv0, lstride);
  const uint32_t nm = 1u << H.k;
  const int ntiles = (int)(nm >> __popc((uint32_t)H.lanebits));
  double smin = INFINITY;
  for (uint32_t m = threadIdx.x; m < nm; m += blockDim.x) smin = fmin(smin, smv[m]);
  smin = block_reduce(smin, [](double a, double b) { return fmin(a, b); }, shd);
  const double thr = smin + tol, atol = tol / 100.0;
  unsigned pick = 0xffffffffu;
  double runner = INFINITY;
  int amb = 0;
  for (uint32_t m = threadIdx.x; m < nm; m += blockDim.x) {
    const double v = smv[m];
    if (!(v < INFINITY)) continue;
    if (fabs(v - thr) <= atol) amb = 1;
    if (v <= thr) pick = min(pick, m);
    else runner = fmin(runner, v);
  }
  for (int t = threadIdx.x; t < ntiles; t += blockDim.x)
    if (tiles[t].near >= d.popcount) amb = 1;
  pick = block_reduce(pick, [](unsigned a, unsigned b) { return min(a, b); }, shu);
  amb = block_reduce(amb, [](int a, int b) { return a | b; }, shi);
  runner = block_reduce(runner, [](double a, double b) { return fmin(a, b); }, shd);
  if (threadIdx.x == 0 && pick != 0xffffffffu) {
    d.mask = pick;
    d.e_loc = fin[pick].e;
    d.ambiguous = amb;
    d.key_gap = runner - smin;
    d.smice_rise = smv[pick] - *smv0;
    decs[g] = d;
  }
}

}  // namespace okr
