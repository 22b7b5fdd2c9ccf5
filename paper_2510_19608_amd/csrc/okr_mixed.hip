// Mixed-precision search of one segment: FP32 screening of every mask in
// difference form, then FP64 rescoring of a shortlist that provably contains
// every mask the FP64 decision depends on, so that the decision equals the
// FP64 path's whenever |e32 - e64| <= delta and |slack32 - slack64| <= delta.
//
//   k_build_mixed    FP32 tables from the FP64 ones (P, cluster offsets)
//   k_score_fp32     every mask, FP32; tile records of sure / possible /
//                    uncertain feasibility (band delta + amb around e_bar and
//                    the voltage band)                      [okr_score.hip]
//   k_mixed_select_a list A: uncertain masks at or above the best sure level
//   k_score_fp64     (list mode) FP64 scores of a mask list, the per-mask
//                    FP64 scoring kernel itself             [okr_score.hip]
//   k_mixed_select_b best level P*; list B: possibly feasible masks at P*
//                    whose FP32 error is within tie + 2 delta + amb of the
//                    smallest FP64-confirmed one
//   k_mixed_final    FP64 arg-min over list B, ambiguity from A and B
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "okr_device.h"
#include "okr_internal.h"

namespace okr {

__global__ __launch_bounds__(256) void k_build_mixed(const SegHdr* __restrict__ hdrs, const int* __restrict__ segs,
                                                     size_t lstride, const int* __restrict__ tab, int n,
                                                     const double2* __restrict__ Vcur,
                                                     const double2* __restrict__ P,
                                                     const TargetRec* __restrict__ srec,
                                                     const double2* __restrict__ headV,
                                                     const TargetRec* __restrict__ zrec, double vmin, double vmax,
                                                     Pair32* __restrict__ P32, Rec32* __restrict__ S32,
                                                     Head32* __restrict__ H32, Rec32* __restrict__ Z32) {
  const SegHdr H = load_hdr(hdrs, segs);
  if (!H.valid) return;
  tab = lane_ptr(tab, lstride);
  P = lane_ptr(P, lstride);
  srec = lane_ptr(srec, lstride);
  headV = lane_ptr(headV, lstride);
  zrec = lane_ptr(zrec, lstride);
  P32 = lane_ptr(P32, lstride);
  S32 = lane_ptr(S32, lstride);
  H32 = lane_ptr(H32, lstride);
  Z32 = lane_ptr(Z32, lstride);
  const int part = blockIdx.y, S = H.S;
  const int stride = gridDim.x * blockDim.x;
  const float NEG = -INFINITY, POS = INFINITY;
  if (part == 0) {
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < S * H.npairs * 3; t += stride) {
      const int l = t / (H.npairs * 3), rem = t % (H.npairs * 3), q = rem / 3, p = rem % 3;
      const int* pr = tab + H.o_pair + q * kPairInts;
      const double2 pv = P[((size_t)l * H.npairs + q) * 3 + p];
      const TargetRec r = srec[((size_t)l * H.nslots + pr[PR_RSLOT]) * 3 + p];
      Pair32 o;
      o.P = make_float2((float)pv.x, (float)pv.y);
      const int rphase = tab[H.o_slot + pr[PR_RSLOT] * kSlotInts + SL_PHASE];
      if (rphase >> p & 1) {
        const double ws = sqrt(cabs2(Vcur[((size_t)l * n + pr[PR_SUPER]) * 3 + p]));
        o.a = (float)(ws - r.lo);
        o.b = (float)(r.hi - ws);
      } else {
        o.a = NEG;
        o.b = NEG;
      }
      P32[t] = o;
    }
  } else if (part == 1) {
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < S * H.nslots * 3; t += stride) {
      const int s = (t / 3) % H.nslots, p = t % 3;
      const TargetRec r = srec[t];
      const int ph = tab[H.o_slot + s * kSlotInts + SL_PHASE];
      const double w = sqrt(cabs2(r.W));
      Rec32 o;
      o.W = make_float2((float)r.W.x, (float)r.W.y);
      o.w = (float)w;
      o.pad = 0.f;
      if (ph >> p & 1) {
        o.a = (float)(w - r.lo);
        o.b = (float)(r.hi - w);
        o.bmin = (float)(w - vmin);
        o.bmax = (float)(vmax - w);
      } else {
        o.a = NEG; o.b = NEG; o.bmin = POS; o.bmax = POS;
      }
      S32[t] = o;
    }
  } else if (part == 2) {
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < S * H.nchains * 3; t += stride) {
      const double2 v = headV[t];
      Head32 o;
      o.W = make_float2((float)v.x, (float)v.y);
      o.w = (float)sqrt(cabs2(v));
      o.pad = 0.f;
      H32[t] = o;
    }
  } else {
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < S * H.nz; t += stride) {
      const TargetRec r = zrec[t];
      const double w = sqrt(cabs2(r.W));
      Rec32 o;
      o.W = make_float2((float)r.W.x, (float)r.W.y);
      o.w = (float)w;
      o.a = (float)(w - r.lo);
      o.b = (float)(r.hi - w);
      o.bmin = (float)(w - vmin);
      o.bmax = (float)(vmax - w);
      o.pad = 0.f;
      Z32[t] = o;
    }
  }
}

__device__ __forceinline__ bool skip_segment(const SegHdr& H, const int* status) {
  return !H.valid || (*status & (16 | 32));
}

// List A: masks whose FP32 verdict is uncertain, at or above the best level
// holding a surely feasible mask.
__global__ __launch_bounds__(1024) void k_mixed_select_a(const SegHdr* __restrict__ hdrs, const int* __restrict__ segs,
                                                         size_t lstride, const MaskScore32* __restrict__ fin,
                                                         const TileRec32* __restrict__ tiles, SelParams sp,
                                                         const int* __restrict__ status, MixedState* __restrict__ ms,
                                                         uint32_t* __restrict__ listA, int* __restrict__ countA) {
  __shared__ int shi[16];
  __shared__ int cnt;
  __shared__ uint32_t s_lp[64];  // lane part of the mask of each of a tile's lanes
  const int g = segs[blockIdx.z];
  const SegHdr H = load_hdr_g(hdrs, g);
  if (threadIdx.x < 64) s_lp[threadIdx.x] = lane_part((uint32_t)H.lanebits, threadIdx.x);
  fin = lane_ptr(fin, lstride);
  tiles = lane_ptr(tiles, lstride);
  listA = lane_ptr(listA, lstride);
  countA = lane_ptr(countA, lstride);
  if (threadIdx.x == 0) cnt = 0;
  if (skip_segment(H, status)) {
    if (threadIdx.x == 0) { *countA = 0; ms[g].lo_level = -1; ms[g].hi_level = -1; }
    return;
  }
  const uint32_t nm = 1u << H.k;
  const uint32_t L = (uint32_t)H.lanebits;  // tile t, lane j holds tile_mask(L, t, j, k)
  const int lb = __popc(L);
  const int ntiles = (int)(nm >> lb);
  int lo = -1, hi = -1;
  for (int t = threadIdx.x; t < ntiles; t += blockDim.x) {
    lo = max(lo, tiles[t].sure);
    hi = max(hi, tiles[t].poss);
  }
  lo = block_reduce(lo, [](int a, int b) { return max(a, b); }, shi);
  hi = block_reduce(hi, [](int a, int b) { return max(a, b); }, shi);
  const double dd = sp.delta + sp.amb;
  for (int t = threadIdx.x; t < ntiles; t += blockDim.x) {
    if (tiles[t].unc < lo || tiles[t].unc < 0) continue;
    const uint32_t tb = tile_part(L, (uint32_t)t, H.k);
    for (int j = 0; j < 64; ++j) {
      if (j >> lb) break;
      const uint32_t mm = tb | s_lp[j];
      const MaskScore32 r = fin[mm];
      const bool sure = (double)r.e <= sp.e_bar - dd && (double)r.slack >= dd;
      const bool poss = (double)r.e <= sp.e_bar + dd && (double)r.slack >= -dd;
      if (poss && !sure && __popc(mm) >= lo) listA[atomicAdd(&cnt, 1)] = mm;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    *countA = cnt;
    ms[g].lo_level = lo;
    ms[g].hi_level = hi;
    ms[g].nA = cnt;
  }
}

// Best level P* and list B.
__global__ __launch_bounds__(1024) void k_mixed_select_b(const SegHdr* __restrict__ hdrs, const int* __restrict__ segs,
                                                         size_t lstride, const MaskScore32* __restrict__ fin,
                                                         const TileRec32* __restrict__ tiles, SelParams sp,
                                                         const int* __restrict__ status, MixedState* __restrict__ ms,
                                                         const uint32_t* __restrict__ listA,
                                                         const int* __restrict__ countA,
                                                         const MaskScore* __restrict__ scoreA,
                                                         uint32_t* __restrict__ listB, int* __restrict__ countB) {
  __shared__ int shi[16];
  __shared__ double shd[16];
  __shared__ int cnt;
  __shared__ uint32_t s_lp[64];  // lane part of the mask of each of a tile's lanes
  const int g = segs[blockIdx.z];
  const SegHdr H = load_hdr_g(hdrs, g);
  if (threadIdx.x < 64) s_lp[threadIdx.x] = lane_part((uint32_t)H.lanebits, threadIdx.x);
  fin = lane_ptr(fin, lstride);
  tiles = lane_ptr(tiles, lstride);
  listA = lane_ptr(listA, lstride);
  countA = lane_ptr(countA, lstride);
  scoreA = lane_ptr(scoreA, lstride);
  listB = lane_ptr(listB, lstride);
  countB = lane_ptr(countB, lstride);
  if (threadIdx.x == 0) cnt = 0;
  if (skip_segment(H, status)) {
    if (threadIdx.x == 0) { *countB = 0; ms[g].best = -1; }
    return;
  }
  const uint32_t nm = 1u << H.k;
  const uint32_t L = (uint32_t)H.lanebits;  // tile t, lane j holds tile_mask(L, t, j, k)
  const int lb = __popc(L);
  const int ntiles = (int)(nm >> lb);
  const double dd = sp.delta + sp.amb;
  const int nA = *countA;
  int best = ms[g].lo_level;
  for (int q = threadIdx.x; q < nA; q += blockDim.x)
    if (feasible(scoreA[q], sp.e_bar)) best = max(best, __popc(listA[q]));
  best = block_reduce(best, [](int a, int b) { return max(a, b); }, shi);
  // upper bound on the smallest FP64 error at level best
  double eup = INFINITY;
  if (best >= 0) {
    for (int t = threadIdx.x; t < ntiles; t += blockDim.x) {
      if (tiles[t].sure < best) continue;
      const uint32_t tb = tile_part(L, (uint32_t)t, H.k);
      for (int j = 0; j < 64; ++j) {
        if (j >> lb) break;
        const uint32_t mm = tb | s_lp[j];
        const MaskScore32 r = fin[mm];
        if (__popc(mm) == best && (double)r.e <= sp.e_bar - dd && (double)r.slack >= dd)
          eup = fmin(eup, (double)r.e + sp.delta);
      }
    }
    for (int q = threadIdx.x; q < nA; q += blockDim.x)
      if (__popc(listA[q]) == best && feasible(scoreA[q], sp.e_bar)) eup = fmin(eup, scoreA[q].e);
  }
  eup = block_reduce(eup, [](double a, double b) { return fmin(a, b); }, shd);
  const double bound = eup + sp.tie + sp.delta + sp.amb;
  if (best >= 0) {
    for (int t = threadIdx.x; t < ntiles; t += blockDim.x) {
      if (tiles[t].poss < best) continue;
      const uint32_t tb = tile_part(L, (uint32_t)t, H.k);
      for (int j = 0; j < 64; ++j) {
        if (j >> lb) break;
        const uint32_t mm = tb | s_lp[j];
        const MaskScore32 r = fin[mm];
        const bool poss = (double)r.e <= sp.e_bar + dd && (double)r.slack >= -dd;
        if (poss && __popc(mm) == best && (double)r.e <= bound) listB[atomicAdd(&cnt, 1)] = mm;
      }
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    *countB = cnt;
    ms[g].best = best;
    ms[g].nB = cnt;
    ms[g].e_up = eup;
  }
}

// FP64 arg-min over list B; ambiguity from the FP64 scores of A and B; the
// largest FP32 deviation seen on refined masks is kept for reporting.
__global__ __launch_bounds__(1024) void k_mixed_final(const SegHdr* __restrict__ hdrs, const int* __restrict__ segs,
                                                      size_t lstride, SelParams sp, const int* __restrict__ status,
                                                      MixedState* __restrict__ ms, const MaskScore32* __restrict__ fin,
                                                      const uint32_t* __restrict__ listA, const int* __restrict__ countA,
                                                      const MaskScore* __restrict__ scoreA,
                                                      const uint32_t* __restrict__ listB, const int* __restrict__ countB,
                                                      const MaskScore* __restrict__ scoreB,
                                                      DevDecision* __restrict__ decs, int* __restrict__ redo) {
  __shared__ double shd[16];
  __shared__ int shi[16];
  __shared__ unsigned shu[16];
  const int g = segs[blockIdx.z];
  const SegHdr H = load_hdr_g(hdrs, g);
  fin = lane_ptr(fin, lstride);
  listA = lane_ptr(listA, lstride);
  countA = lane_ptr(countA, lstride);
  scoreA = lane_ptr(scoreA, lstride);
  listB = lane_ptr(listB, lstride);
  countB = lane_ptr(countB, lstride);
  scoreB = lane_ptr(scoreB, lstride);
  DevDecision* dec = decs + g;
  const int best = ms[g].best;
  if (threadIdx.x == 0) redo[g] = 0;
  if (skip_segment(H, status) || best < 0) {
    if (threadIdx.x == 0) {
      DevDecision d;
      d.mask = 0; d.popcount = 0; d.e_loc = 0.0; d.e_min = 0.0; d.ambiguous = skip_segment(H, status) ? 0 : 1;
      d.found = 0;
      d.key_gap = INFINITY;
      d.smice_rise = 0.0;
      *dec = d;
    }
    return;
  }
  const int nA = *countA, nB = *countB;
  double emin = INFINITY, dev = 0.0;
  for (int q = threadIdx.x; q < nB; q += blockDim.x) {
    const MaskScore r = scoreB[q];
    if (feasible(r, sp.e_bar)) emin = fmin(emin, r.e);
    if (r.e <= 2.0 * sp.e_bar) dev = fmax(dev, fabs((double)fin[listB[q]].e - r.e));
  }
  emin = block_reduce(emin, [](double a, double b) { return fmin(a, b); }, shd);
  const double thr = emin + sp.tie;
  unsigned pick = 0xffffffffu;
  int amb = 0;
  double runner = INFINITY;  // among the FP64-rescored masks of list B
  for (int q = threadIdx.x; q < nB; q += blockDim.x) {
    const MaskScore r = scoreB[q];
    if (!feasible(r, sp.e_bar)) continue;
    if (fabs(r.e - thr) <= sp.amb) amb = 1;
    if (r.e <= thr) pick = min(pick, listB[q]);
    else runner = fmin(runner, r.e);
  }
  for (int q = threadIdx.x; q < nA; q += blockDim.x) {
    const MaskScore r = scoreA[q];
    if (__popc(listA[q]) >= best && near_boundary(r, sp.e_bar, sp.amb)) amb = 1;
    if (r.e <= 2.0 * sp.e_bar) dev = fmax(dev, fabs((double)fin[listA[q]].e - r.e));
  }
  pick = block_reduce(pick, [](unsigned a, unsigned b) { return min(a, b); }, shu);
  amb = block_reduce(amb, [](int a, int b) { return a | b; }, shi);
  dev = block_reduce(dev, [](double a, double b) { return fmax(a, b); }, shd);
  runner = block_reduce(runner, [](double a, double b) { return fmin(a, b); }, shd);
  if (threadIdx.x == 0) {
    DevDecision d;
    double epick = 0.0;
    for (int q = 0; q < nB; ++q)
      if (listB[q] == pick) epick = scoreB[q].e;
    d.mask = pick == 0xffffffffu ? 0u : pick;
    d.popcount = best;
    d.e_loc = epick;
    d.e_min = emin;
    d.ambiguous = amb;
    d.found = pick != 0xffffffffu;
    d.key_gap = runner - emin;
    d.smice_rise = 0.0;
    *dec = d;
    ms[g].max_dev = dev;
    // the shortlists are complete only while |e32 - e64| <= delta: past the
    // bound the segment is scored again in FP64 over every mask (and that
    // decision replaces this one)
    redo[g] = dev > sp.delta ? 1 : 0;
  }
}

}  // namespace okr
