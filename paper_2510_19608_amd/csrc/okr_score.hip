// Candidate scoring kernels: every mask of a segment (FP64, and the FP32
// difference-form screen of the mixed-precision search) and FP64 rescoring of
// a mask list.  Built with NaNs excluded (no input or intermediate here is
// NaN), which lets max/min compile to single instructions.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "okr_device.h"
#include "okr_internal.h"

namespace okr {

// ---------------------------------------------------------------- scoring --
constexpr int kStageBatch = 2;  // LDS-stage chunks each thread loads before it stores any

// Tile record of one wave's 64 masks (lane q holds mask
// tile_mask(lanebits, tile, q, k), final score r): highest feasible level,
// smallest error at that level, highest level of a mask near the e_bar /
// band boundary.
__device__ __forceinline__ int tile_record(const MaskScore& r, uint32_t m, uint32_t tile, bool valid,
                                           const SelParams& sp, TileRec* __restrict__ tiles) {
  const int pc = __popc(m);
  const bool feas = valid && feasible(r, sp.e_bar);
  int best = feas ? pc : -1;
  int nearl = (valid && near_boundary(r, sp.e_bar, sp.amb)) ? pc : -1;
  for (int o = 32; o > 0; o >>= 1) {
    best = max(best, __shfl_xor(best, o, 64));
    nearl = max(nearl, __shfl_xor(nearl, o, 64));
  }
  double em = (feas && pc == best) ? r.e : INFINITY;
  for (int o = 32; o > 0; o >>= 1) em = fmin(em, __shfl_xor(em, o, 64));
  if ((threadIdx.x & 63) == 0) {
    TileRec t;
    t.best = best;
    t.near = nearl;
    t.emin = em;
    tiles[tile] = t;
  }
  return best;
}

// Whether a mask's final score is stored: every mask when all are wanted
// (dumps, surrogate targets), else only the masks the arg-min can read -- a
// tile's masks at its best feasible level (no mask of a lower level of the
// tile can be at the chosen level) and mask 0 (the decision's error when no
// mask is feasible).
__device__ __forceinline__ bool keep_score(bool full, uint32_t m, int tile_best) {
  return full || __popc(m) == tile_best || m == 0;
}

// LDS stage of one pass of the per-mask kernel, in 16-byte chunks: chunk i
// of one index space over the pair rows, slot records (2 chunks each), chain
// heads and the first zone records (2 chunks each) of the pass's M snapshots
// (element r * M + j of each table, snapshot j fastest, M a power of two, so
// the LDS writes are contiguous).  stage_issue loads kStageBatch chunks per
// thread, from chunk b on (past the end the last chunk is loaded again and
// not stored); stage_store writes them to the buffer at chunk bb of the LDS,
// a chain head's magnitude too.
struct StageMap {
  int nP, nT, nH, nst;  // chunks of the pair, slot, head tables; all chunks
  int oT, oH, oZ, oHm;  // their offsets in a buffer (pairs at 0), head magnitudes
};
template <int M>
__device__ __forceinline__ void stage_issue(const StageMap& S, int b, int l, int l1, const SegHdr& H,
                                            const double2* __restrict__ P, const TargetRec* __restrict__ srec,
                                            const double2* __restrict__ headV, const TargetRec* __restrict__ zrec,
                                            uint4 (&v)[kStageBatch], int (&dst)[kStageBatch]) {
  constexpr int LM = M == 4 ? 2 : (M == 2 ? 1 : 0);
#pragma unroll
  for (int u = 0; u < kStageBatch; ++u) {
    const int i0 = b + u * kScoreThreads + (int)threadIdx.x;
    const int i = min(i0, S.nst - 1);
    // its table by selects, no branches, so the loads issue back to back
    const int iT = i - S.nP, iH = iT - S.nT, iZ = iH - S.nH;
    const bool isP = i < S.nP, isT = !isP && iT < S.nT, isH = !isP && !isT && iH < S.nH;
    const bool rec = !isP && !isH;  // slot and zone records: 2 chunks each
    const int ii = isP ? i : (isT ? iT : (isH ? iH : iZ));
    const int j = rec ? (ii >> 1) & (M - 1) : ii & (M - 1);
    const int chunk = rec ? ((ii >> (LM + 1)) << 1) + (ii & 1) : ii >> LM;
    const uint4* base =
        isP ? (const uint4*)P : (isT ? (const uint4*)srec : (isH ? (const uint4*)headV : (const uint4*)zrec));
    const int per = isP ? H.npairs * 3 : (isT ? H.nslots * 6 : (isH ? H.nchains * 3 : H.nz * 2));  // per snapshot
    dst[u] = i0 < S.nst ? (isP ? 0 : (isT ? S.oT : (isH ? S.oH : S.oZ))) + ii : -1;
    v[u] = base[(size_t)min(l + j, l1 - 1) * per + chunk];
  }
}
__device__ __forceinline__ void stage_store(const StageMap& S, unsigned char* lds, int bb,
                                            const uint4 (&v)[kStageBatch], const int (&dst)[kStageBatch]) {
  uint4* buf = (uint4*)lds + bb;
  double* Hm = (double*)(buf + S.oHm);
#pragma unroll
  for (int u = 0; u < kStageBatch; ++u) {
    if (dst[u] < 0) continue;
    buf[dst[u]] = v[u];
    if (dst[u] >= S.oH && dst[u] < S.oZ) {  // a chain head: its magnitude too
      const double2 hv =
          make_double2(__hiloint2double((int)v[u].y, (int)v[u].x), __hiloint2double((int)v[u].w, (int)v[u].z));
      Hm[dst[u] - S.oH] = (hv.x != 0.0 || hv.y != 0.0) ? hmag(hv) : 0.0;
    }
  }
}

// Per-mask FP64 scoring, snapshot-vectorised: one mask per lane; a block's 4
// waves form groups of ws waves (1, 2 or 4) over 64 consecutive masks each,
// the waves of a group splitting the segment's chains (each chain's terms,
// nesting path and zone entries included, are independent of the others')
// and folding their maxima and minima in LDS at the end.  The block's
// snapshot group is walked in passes of M snapshots staged together in LDS
// (snapshot fastest), every chain's terms for the M snapshots at once
// (score_chain_sv).  A pass past the group's last snapshot repeats it.  With
// one snapshot group the block writes the final per-mask scores and tile
// records itself; with several, the last block of a tile to finish (ticket
// counter) folds the groups.  Final per-mask scores are stored for every
// mask only with full_fin (keep_score).  Dynamic LDS per snapshot: pcap pairs, kcap
// slots and chains, zcap zone records (later zone records are read from
// global memory).
template <int M>
__global__ __launch_bounds__(kScoreThreads) void k_score_fp64(
    const SegHdr* __restrict__ hdrs, const int* __restrict__ segs, size_t lstride, const int* __restrict__ tab,
    const double2* __restrict__ P, const TargetRec* __restrict__ srec, const double2* __restrict__ headV,
    const TargetRec* __restrict__ zrec, const double* __restrict__ econst, int snaps_per_group, int SG, int pcap,
    int kcap, int zcap, int ws, SelParams sp, MaskScore* __restrict__ part, MaskScore* __restrict__ fin,
    TileRec* __restrict__ tiles, int* __restrict__ tickets, const int* __restrict__ gates, int full_fin) {
  constexpr int NW = kScoreThreads / 64;
  extern __shared__ __align__(16) unsigned char sv_lds[];
  __shared__ double f_e[NW][64], f_qn[NW][64], f_qx[NW][64];
  const int g = *as_cint(segs + blockIdx.z);
  const SegHdr H = load_hdr(hdrs, segs);
  if (!H.valid || (gates && gates[g] == 0)) return;
  // blocks past this segment's masks (a chunk's launch covers its largest segment)
  const uint32_t nmask = 1u << H.k;
  const uint32_t bmasks = kScoreBlock * (NW / ws);
  if ((uint64_t)blockIdx.x * bmasks >= nmask) return;
  tab = lane_ptr(tab, lstride);
  P = lane_ptr(P, lstride);
  srec = lane_ptr(srec, lstride);
  headV = lane_ptr(headV, lstride);
  zrec = lane_ptr(zrec, lstride);
  econst = lane_ptr(econst, lstride);
  part = lane_ptr(part, lstride);
  fin = lane_ptr(fin, lstride);
  tiles = lane_ptr(tiles, lstride);
  tickets = lane_ptr(tickets, lstride);
  const int tid = threadIdx.x;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lane = tid & 63;
  const int c0 = w % ws;  // this wave's first chain within its group
  // this wave's tile and this lane's mask (the lane bits vary across the wave)
  const uint32_t L = (uint32_t)H.lanebits;
  const uint32_t tile = blockIdx.x * (NW / ws) + (uint32_t)(w / ws);
  const uint32_t m = tile_mask(L, tile, (uint32_t)lane, H.k);
  const bool tile_ok = (tile << __popc(L)) < nmask;  // (a block's last waves can lie past the masks)
  const bool valid = tile_ok && ((uint32_t)lane >> __popc(L)) == 0;
  const int sg = blockIdx.y;
  const int l0 = sg * snaps_per_group;
  const int l1 = min(H.S, l0 + snaps_per_group);
  const cint* chains = as_cint(tab + H.o_chain);
  const cint* nest = as_cint(tab + H.o_nest);
  const int zst = min(H.nz, zcap);
  const int cP = H.npairs * 3, cT = H.nslots * 6, cH = H.nchains * 3, cZ = zst * 2;  // 16-byte chunks per snapshot
  double e = 0.0, qmn[M], qmx[M];
#pragma unroll
  for (int j = 0; j < M; ++j) {
    qmn[j] = INFINITY;
    qmx[j] = -INFINITY;
  }
  // LDS: the pass's tables packed to this segment's own sizes.  The launch
  // allocates the layout of the capacities (pcap pairs, kcap slots and
  // chains, zcap zone records per snapshot, for the chunk's largest
  // segment); when two packed buffers fit in it, the next pass is staged
  // while this one is computed (its first loads in flight during the
  // compute, one barrier per pass), else passes stage and compute in turn.
  constexpr int LM = M == 4 ? 2 : (M == 2 ? 1 : 0);
  StageMap SM;
  SM.nP = cP << LM;
  SM.nT = cT << LM;
  SM.nH = cH << LM;
  SM.nst = SM.nP + SM.nT + SM.nH + (cZ << LM);
  SM.oT = SM.nP;
  SM.oH = SM.oT + SM.nT;
  SM.oZ = SM.oH + SM.nH;
  SM.oHm = SM.nst;  // then doubles: the head magnitudes (nchains * 3 * M), the constant errors (M)
  const int nEc = H.nchains * 3 * M;             // (index of the first constant error among them)
  const int ubuf = SM.oHm + (nEc + M + 1) / 2;  // chunks per buffer
  // (the allocation: the capacities' layout and 16 bytes, which covers the
  // rounding of the packed one)
  const size_t cap_bytes = (size_t)M * ((size_t)pcap * 3 * sizeof(double2) +
                                        (size_t)kcap * 3 * (sizeof(TargetRec) + sizeof(double2) + sizeof(double)) +
                                        (size_t)zcap * sizeof(TargetRec) + sizeof(double)) +
                           16;
  const bool dbl = (size_t)2 * ubuf * 16 <= cap_bytes;
  const int npass = (l1 - l0 + M - 1) / M;
  uint4 sv[kStageBatch];
  int sd[kStageBatch];
  auto stage_all = [&](int l, int bb, int from) {  // chunks from `from` on, issued and stored in turn
    for (int b = from; b < SM.nst; b += kStageBatch * kScoreThreads) {
      stage_issue<M>(SM, b, l, l1, H, P, srec, headV, zrec, sv, sd);
      stage_store(SM, sv_lds, bb, sv, sd);
    }
    if (tid < M) ((double*)((uint4*)sv_lds + bb + SM.oHm))[nEc + tid] = econst[min(l + tid, l1 - 1)];
  };
  if (npass > 0) stage_all(l0, 0, 0);
  __syncthreads();
  for (int pi = 0; pi < npass; ++pi) {
    const int l = l0 + pi * M;
    const int cb = dbl ? (pi & 1) * ubuf : 0;  // this pass's buffer
    const int nb = dbl ? ubuf - cb : 0;        // the next pass's
    const bool ahead = dbl && pi + 1 < npass;
    if (ahead) stage_issue<M>(SM, 0, l + M, l1, H, P, srec, headV, zrec, sv, sd);
    uint4* buf = (uint4*)sv_lds + cb;
    const double2* Ps = (const double2*)buf;
    const TargetRec* Ts = (const TargetRec*)(buf + SM.oT);
    const double2* Hv = (const double2*)(buf + SM.oH);
    const TargetRec* Zs = (const TargetRec*)(buf + SM.oZ);
    const double* Hm = (const double*)(buf + SM.oHm);
    const double* Ec = Hm + nEc;
    double el[M];
    const TargetRec* zg[M];
#pragma unroll
    for (int j = 0; j < M; ++j) {
      el[j] = Ec[j];
      zg[j] = zrec + (size_t)min(l + j, l1 - 1) * H.nz;
    }
    for (int c = c0; c < H.nchains; c += ws)
      if (chains[c * kChainInts + C_PMASK] & L)  // (the others below)
        score_chain_sv<M>(chains, nest, c, Ps, Ts, Hv, Hm, Zs, zst, zg, m, el, qmn, qmx);
#pragma unroll
    for (int j = 0; j < M; ++j) e = fmax(e, el[j]);
    if (ahead) {
      stage_store(SM, sv_lds, nb, sv, sd);
      stage_all(l + M, nb, kStageBatch * kScoreThreads);
      __syncthreads();
    } else if (pi + 1 < npass) {
      __syncthreads();  // every wave is done with the buffer
      stage_all(l + M, 0, 0);
      __syncthreads();
    }
  }
  double qmin = qmn[0], qmax = qmx[0];
#pragma unroll
  for (int j = 1; j < M; ++j) {
    qmin = fmin(qmin, qmn[j]);
    qmax = fmax(qmax, qmx[j]);
  }
  // Chains whose terms depend on no lane bit (none of their own and their
  // nesting path's mask bits among the 6 that vary across the wave) are the same
  // for the wave's 64 masks: the wave evaluates each once, one snapshot per
  // lane, from the tables in global memory, and every lane takes the maxima
  // and minima over the snapshots.
  {
    const uint32_t mu = (uint32_t)__builtin_amdgcn_readfirstlane((int)m);
    double ue = 0.0, uqn = INFINITY, uqx = -INFINITY;
    bool any = false;
    for (int c = c0; c < H.nchains; c += ws) {
      if (chains[c * kChainInts + C_PMASK] & L) continue;
      any = true;
      for (int l = l0 + lane; l < l1; l += 64) {
        double e1[1] = {0.0}, qn1[1] = {INFINITY}, qx1[1] = {-INFINITY};
        const TargetRec* zl = zrec + (size_t)l * H.nz;
        const TargetRec* const zg1[1] = {zl};
        score_chain_sv<1, true>(chains, nest, c, P + (size_t)l * H.npairs * 3, srec + (size_t)l * H.nslots * 3,
                                headV + (size_t)l * H.nchains * 3, nullptr, zl, H.nz, zg1, mu, e1, qn1, qx1);
        ue = fmax(ue, e1[0]);
        uqn = fmin(uqn, qn1[0]);
        uqx = fmax(uqx, qx1[0]);
      }
    }
    if (any) {
      for (int o = 32; o > 0; o >>= 1) {
        ue = fmax(ue, __shfl_xor(ue, o, 64));
        uqn = fmin(uqn, __shfl_xor(uqn, o, 64));
        uqx = fmax(uqx, __shfl_xor(uqx, o, 64));
      }
      e = fmax(e, ue);
      qmin = fmin(qmin, uqn);
      qmax = fmax(qmax, uqx);
    }
  }
  // fold the chains of a group's waves into its first wave (max and min are
  // exact in any order)
  if (ws > 1) {
    f_e[w][lane] = e;
    f_qn[w][lane] = qmin;
    f_qx[w][lane] = qmax;
    __syncthreads();
    if (c0 != 0) return;
    for (int q = 1; q < ws; ++q) {
      e = fmax(e, f_e[w + q][lane]);
      qmin = fmin(qmin, f_qn[w + q][lane]);
      qmax = fmax(qmax, f_qx[w + q][lane]);
    }
  }
  if (!tile_ok) return;
  MaskScore r;
  r.e = e;
  r.slack = band_slack(qmin, qmax, sp.vmin, sp.vmax);
  if (SG == 1) {  // the block holds every snapshot: final scores and tile record directly
    const int tb = tile_record(r, m, tile, valid, sp, tiles);
    if (valid && keep_score(full_fin, m, tb)) fin[m] = r;
    return;
  }
  if (valid) part[(size_t)sg * nmask + m] = r;
  __threadfence();
  int t = 0;
  if (lane == 0) t = atomicAdd(&tickets[tile], 1);
  t = __shfl(t, 0, 64);
  if (t != SG - 1) return;
  __threadfence();
  // last block of this tile: combine the snapshot groups
  r.e = 0.0;
  r.slack = INFINITY;
  if (valid) {
    for (int q = 0; q < SG; ++q) {
      const volatile MaskScore* x = part + (size_t)q * nmask + m;
      r.e = fmax(r.e, x->e);
      r.slack = fmin(r.slack, x->slack);
    }
  }
  const int tb = tile_record(r, m, tile, valid, sp, tiles);
  if (valid && keep_score(full_fin, m, tb)) fin[m] = r;
  if (lane == 0) tickets[tile] = 0;  // ready for the next launch
}

#define OKR_SCORE64_INST(M_)                                                                                               \
  template __global__ void k_score_fp64<M_>(const SegHdr*, const int*, size_t, const int*, const double2*,              \
                                          const TargetRec*, const double2*, const TargetRec*, const double*, int, int, \
                                          int, int, int, int, SelParams, MaskScore*, MaskScore*, TileRec*, int*,       \
                                          const int*, int);
OKR_SCORE64_INST(1)
OKR_SCORE64_INST(2)
OKR_SCORE64_INST(4)
#undef OKR_SCORE64_INST

// ------------------------------------------------- chain-term kernels --
// Exact FP64 terms of chains for given mask bits, one lane per (item,
// snapshot), folded into per-item accumulators by 64-bit atomics on the IEEE
// bit patterns.  Items are either (listed mask, chain) pairs -- the scores of
// a short mask list -- or chain patterns -- the factored form's table: for
// chain c and assignment u of its C_PMASK bits (bit j of u at the j-th lowest
// set bit), the chain's terms.  Every folded value is a non-negative double
// (errors max(|V| - lo, hi - |V|) with lo <= hi, squared magnitudes), and for
// those the bit patterns order like the values; max and min are exact, so the
// results equal the per-mask kernel's.  qmax starts at +0 instead of -inf:
// band_slack treats both alike (no kept node-phase).
//
// A block serves one snapshot (blockIdx.y) of one segment (blockIdx.z of a
// chunk): it first stages the chain records and nesting paths and the
// snapshot's pair, slot, head and first zcap zone records in LDS (one
// coalesced round trip), then walks every item's chain from there.
enum { kTermsList = 0, kTermsPatterns = 1 };
constexpr int kTermsBlock = 256;  // threads of a chain-term block

__device__ __forceinline__ int terms_count(int mode, const SegHdr& H, const int* count, int cap) {
  return mode == kTermsList ? min(*count, cap) * H.nchains : H.npat;
}

__global__ void k_terms_init(const SegHdr* __restrict__ hdrs, const int* __restrict__ segs, size_t lstride, int mode,
                             const int* __restrict__ count, int cap, const double* __restrict__ econst,
                             unsigned long long* __restrict__ acc, unsigned long long* __restrict__ ecmax) {
  const SegHdr H = load_hdr(hdrs, segs);
  if (!H.valid) return;
  count = lane_ptr(count, lstride);
  econst = lane_ptr(econst, lstride);
  acc = lane_ptr(acc, lstride);
  ecmax = lane_ptr(ecmax, lstride);
  const int n = mode == kTermsList ? min(*count, cap) : H.npat;
  const int t0 = blockIdx.x * blockDim.x + threadIdx.x, stride = gridDim.x * blockDim.x;
  for (int q = t0; q < n; q += stride) {
    acc[3 * q] = 0ull;
    acc[3 * q + 1] = (unsigned long long)__double_as_longlong(INFINITY);
    acc[3 * q + 2] = 0ull;
  }
  if (mode == kTermsPatterns && ecmax) {
    if (t0 == 0) *ecmax = 0ull;
  }
}

__global__ __launch_bounds__(kTermsBlock) void k_chain_terms(
    const SegHdr* __restrict__ hdrs, const int* __restrict__ segs, size_t lstride, int mode,
    const int* __restrict__ tab, const double2* __restrict__ P, const TargetRec* __restrict__ srec,
    const double2* __restrict__ headV, const TargetRec* __restrict__ zrec, const double* __restrict__ econst,
    const uint32_t* __restrict__ list, const int* __restrict__ count, int cap, int icap, int zcap,
    unsigned long long* __restrict__ acc, unsigned long long* __restrict__ ecmax) {
  extern __shared__ __align__(16) unsigned char ct_lds[];
  const SegHdr H = load_hdr(hdrs, segs);
  if (!H.valid) return;
  tab = lane_ptr(tab, lstride);
  P = lane_ptr(P, lstride);
  srec = lane_ptr(srec, lstride);
  headV = lane_ptr(headV, lstride);
  zrec = lane_ptr(zrec, lstride);
  econst = lane_ptr(econst, lstride);
  list = lane_ptr(list, lstride);
  count = lane_ptr(count, lstride);
  acc = lane_ptr(acc, lstride);
  ecmax = lane_ptr(ecmax, lstride);
  const int items = terms_count(mode, H, count, cap);
  const int l = blockIdx.y;
  if (mode == kTermsPatterns && ecmax && blockIdx.x == 0 && threadIdx.x == 0)
    atomicMax(ecmax, (unsigned long long)__double_as_longlong(econst[l]));
  if ((int)(blockIdx.x * blockDim.x) >= items) return;  // whole block idle
  // stage: chain records and nesting paths (ints [0, o_slot)), then this
  // snapshot's pairs, slot records, heads and first zone records
  const int nint = H.o_slot;
  const int zst = min(H.nz, zcap);
  int* si = (int*)ct_lds;
  double2* sP = (double2*)(ct_lds + (size_t)((icap * 4 + 15) / 16) * 16);
  TargetRec* sS = (TargetRec*)(sP + (size_t)H.npairs * 3);
  double2* sH = (double2*)(sS + (size_t)H.nslots * 3);
  TargetRec* sZ = (TargetRec*)(sH + (size_t)H.nchains * 3);
  const uint4* gP = (const uint4*)(P + (size_t)l * H.npairs * 3);
  const uint4* gS = (const uint4*)(srec + (size_t)l * H.nslots * 3);
  const uint4* gH = (const uint4*)(headV + (size_t)l * H.nchains * 3);
  const uint4* gZ = (const uint4*)(zrec + (size_t)l * H.nz);
  const int cP = H.npairs * 3, cS = H.nslots * 6, cH = H.nchains * 3, cZ = zst * 2;
  for (int i = threadIdx.x; i < nint; i += blockDim.x) si[i] = tab[i];
  for (int i = threadIdx.x; i < cP + cS + cH + cZ; i += blockDim.x) {
    if (i < cP) ((uint4*)sP)[i] = gP[i];
    else if (i < cP + cS) ((uint4*)sS)[i - cP] = gS[i - cP];
    else if (i < cP + cS + cH) ((uint4*)sH)[i - cP - cS] = gH[i - cP - cS];
    else ((uint4*)sZ)[i - cP - cS - cH] = gZ[i - cP - cS - cH];
  }
  __syncthreads();
  const int* chains = si + H.o_chain;
  const int* nest = si + H.o_nest;
  const int nch = H.nchains;
  const double ec = econst[l];
  if (mode == kTermsList) {
    // a block's items cover consecutive listed masks (each with all its
    // chains): fold them in LDS first, then one global atomic per mask
    __shared__ unsigned long long s_acc[3 * (kTermsBlock + 2)];
    for (int base = blockIdx.x * blockDim.x; base < items; base += gridDim.x * blockDim.x) {
      const int q0 = base / nch, q1 = min(items - 1, base + (int)blockDim.x - 1) / nch;
      for (int i = threadIdx.x; i <= q1 - q0; i += blockDim.x) {
        s_acc[3 * i] = 0ull;
        s_acc[3 * i + 1] = (unsigned long long)__double_as_longlong(INFINITY);
        s_acc[3 * i + 2] = 0ull;
      }
      __syncthreads();
      const int it = base + threadIdx.x;
      if (it < items) {
        const int q = it / nch, c = it - q * nch;
        const uint32_t mm[1] = {list[q]};
        double el[1] = {ec}, qn[1] = {INFINITY}, qx[1] = {0.0};
        score_chain<true, 1>(chains, nest, c, sP, sS, sH, (const double*)nullptr, sZ, zst, zrec + (size_t)l * H.nz,
                             mm, el, qn, qx);
        unsigned long long* a = s_acc + 3 * (q - q0);
        atomicMax(&a[0], (unsigned long long)__double_as_longlong(el[0]));
        if (qn[0] < INFINITY) atomicMin(&a[1], (unsigned long long)__double_as_longlong(qn[0]));
        if (qx[0] > 0.0) atomicMax(&a[2], (unsigned long long)__double_as_longlong(qx[0]));
      }
      __syncthreads();
      for (int i = threadIdx.x; i <= q1 - q0; i += blockDim.x) {
        const int q = q0 + i;
        atomicMax(&acc[3 * q], s_acc[3 * i]);
        if (s_acc[3 * i + 1] != (unsigned long long)__double_as_longlong(INFINITY))
          atomicMin(&acc[3 * q + 1], s_acc[3 * i + 1]);
        if (s_acc[3 * i + 2] != 0ull) atomicMax(&acc[3 * q + 2], s_acc[3 * i + 2]);
      }
      __syncthreads();
    }
    return;
  }
  int c = 0;  // (a thread's items increase, so its chain index only moves forward)
  for (int it = blockIdx.x * blockDim.x + threadIdx.x; it < items; it += gridDim.x * blockDim.x) {
    while (c + 1 < nch && chains[(c + 1) * kChainInts + C_PBASE] <= it) ++c;
    const uint32_t u = (uint32_t)(it - chains[c * kChainInts + C_PBASE]);
    uint32_t pm = (uint32_t)chains[c * kChainInts + C_PMASK], mask = 0;
    for (int j = 0; pm; ++j) {  // deposit bit j of u at the j-th lowest bit of C_PMASK
      const uint32_t low = pm & (0u - pm);
      if (u >> j & 1u) mask |= low;
      pm ^= low;
    }
    const uint32_t mm[1] = {mask};
    double el[1] = {0.0}, qn[1] = {INFINITY}, qx[1] = {0.0};
    score_chain<true, 1>(chains, nest, c, sP, sS, sH, (const double*)nullptr, sZ, zst, zrec + (size_t)l * H.nz, mm,
                         el, qn, qx);
    atomicMax(&acc[3 * it], (unsigned long long)__double_as_longlong(el[0]));
    if (qn[0] < INFINITY) atomicMin(&acc[3 * it + 1], (unsigned long long)__double_as_longlong(qn[0]));
    if (qx[0] > 0.0) atomicMax(&acc[3 * it + 2], (unsigned long long)__double_as_longlong(qx[0]));
  }
}

// Scores of a short mask list from its accumulators.
__global__ void k_list_finish(const int* __restrict__ count, const unsigned long long* __restrict__ acc, int cap,
                              SelParams sp, MaskScore* __restrict__ out, size_t lstride) {
  count = lane_ptr(count, lstride);
  acc = lane_ptr(acc, lstride);
  out = lane_ptr(out, lstride);
  const int n = min(*count, cap);
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n; q += gridDim.x * blockDim.x) {
    MaskScore r;
    r.e = __longlong_as_double((long long)acc[3 * q]);
    r.slack = band_slack(__longlong_as_double((long long)acc[3 * q + 1]),
                         __longlong_as_double((long long)acc[3 * q + 2]), sp.vmin, sp.vmax);
    out[q] = r;
  }
}

// Every mask's score from the pattern table (one thread per mask): the
// largest constant error and each chain's entry for the mask's bits, then
// the band slack; per-mask scores and 64-mask tile records as the per-mask
// scoring kernel writes them.
constexpr int kPatLds = 1024;  // pattern-table entries staged in LDS

__global__ __launch_bounds__(256) void k_fac_combine(const SegHdr* __restrict__ hdrs, const int* __restrict__ segs,
                                                     size_t lstride, const int* __restrict__ tab,
                                                     const unsigned long long* __restrict__ pat,
                                                     const unsigned long long* __restrict__ ecmax, SelParams sp,
                                                     MaskScore* __restrict__ fin, TileRec* __restrict__ tiles) {
  __shared__ int s_pm[kMaxK], s_pb[kMaxK];
  __shared__ double s_pat[3 * kPatLds];
  const SegHdr H = load_hdr(hdrs, segs);
  if (!H.valid) return;
  if ((uint64_t)blockIdx.x * blockDim.x >= ((uint64_t)1 << H.k)) return;  // past this segment's masks
  tab = lane_ptr(tab, lstride);
  pat = lane_ptr(pat, lstride);
  ecmax = lane_ptr(ecmax, lstride);
  fin = lane_ptr(fin, lstride);
  tiles = lane_ptr(tiles, lstride);
  const int tid = threadIdx.x;
  const int nch = H.nchains;
  if (tid < nch) {
    s_pm[tid] = tab[H.o_chain + tid * kChainInts + C_PMASK];
    s_pb[tid] = tab[H.o_chain + tid * kChainInts + C_PBASE];
  }
  const int np = min(H.npat, kPatLds);
  for (int i = tid; i < 3 * np; i += blockDim.x) s_pat[i] = __longlong_as_double((long long)pat[i]);
  __syncthreads();
  const uint32_t nmask = 1u << H.k;
  const uint32_t L = (uint32_t)H.lanebits;
  const uint32_t tile = (blockIdx.x * blockDim.x + tid) / kScoreBlock;
  const uint32_t m = tile_mask(L, tile, (uint32_t)(tid & (kScoreBlock - 1)), H.k);
  const bool tile_ok = (tile << __popc(L)) < nmask;
  const bool valid = tile_ok && ((uint32_t)(tid & (kScoreBlock - 1)) >> __popc(L)) == 0;
  double e = __longlong_as_double((long long)*ecmax), qn = INFINITY, qx = 0.0;
  for (int c = 0; c < nch; ++c) {
    uint32_t pm = (uint32_t)__builtin_amdgcn_readfirstlane(s_pm[c]);
    const int pb = __builtin_amdgcn_readfirstlane(s_pb[c]);
    uint32_t u = 0;
    int j = 0;
    while (pm) {  // gather the mask's bits at C_PMASK's positions, run by run
      const int b = __builtin_ctz(pm);
      const int run = __builtin_ctz(~(pm >> b));
      const uint32_t ones = (1u << run) - 1u;
      u |= ((m >> b) & ones) << j;
      j += run;
      pm &= ~(ones << b);
    }
    const int idx = pb + (int)u;
    double pe, pn, px;
    if (idx < kPatLds) {
      pe = s_pat[3 * idx];
      pn = s_pat[3 * idx + 1];
      px = s_pat[3 * idx + 2];
    } else {
      pe = __longlong_as_double((long long)pat[3 * idx]);
      pn = __longlong_as_double((long long)pat[3 * idx + 1]);
      px = __longlong_as_double((long long)pat[3 * idx + 2]);
    }
    e = fmax(e, pe);
    qn = fmin(qn, pn);
    qx = fmax(qx, px);
  }
  MaskScore r;
  r.e = e;
  r.slack = band_slack(qn, qx, sp.vmin, sp.vmax);
  if (valid) fin[m] = r;
  if (tile_ok) tile_record(r, m, tile, valid, sp, tiles);
}

// d = |W + S| - |W| in difference form (w = |W| given):
// d = (2 Re(conj(W) S) + |S|^2) / (|W + S| + |W|).  The hardware square root
// and reciprocal (each within 1 ulp) suffice: |W| ~ 1 and |d| <~ 0.05, so
// they add well under 1e-8 absolute to d.
__device__ __forceinline__ float diff32(float2 W, float w, float2 S) {
  const float vx = W.x + S.x, vy = W.y + S.y;
  const float m = __builtin_amdgcn_sqrtf(vx * vx + vy * vy);
  const float num = 2.f * (W.x * S.x + W.y * S.y) + (S.x * S.x + S.y * S.y);
  return num * __builtin_amdgcn_rcpf(m + w);
}

// FP32 chain walk for M masks per lane (as walk_chain): d is the difference
// |W + S| - |W| of a slot's voltage; a non-nested head is unaffected (d = 0).
template <bool ERR, int M>
__device__ __forceinline__ void walk32(const int* __restrict__ cr, const Pair32* Ps, const Rec32* Ss,
                                       const Head32* Hs, int c, const uint32_t (&m)[M], float2 (&B)[M][3],
                                       float (&el)[M], float (&slack)[M]) {
  float2 S[M][3];
  float dd[M][3];  // d of the current super on each phase
#pragma unroll
  for (int i = 0; i < M; ++i)
#pragma unroll
    for (int p = 0; p < 3; ++p) {
      S[i][p] = B[i][p];
      dd[i][p] = 0.f;
    }
  if (ERR && cr[C_OUTER] >= 0) {
    const int hph = cr[C_PHASE];
    const Head32* hv = Hs + c * 3;
#pragma unroll
    for (int p = 0; p < 3; ++p)
      if (hph >> p & 1) {
        const Head32 h = hv[p];
#pragma unroll
        for (int i = 0; i < M; ++i) dd[i][p] = diff32(h.W, h.w, B[i][p]);
      }
  }
  const int ns = cr[C_NSLOT], s0 = cr[C_SLOT0], pair0 = cr[C_PAIR0], bit0 = cr[C_BIT0];
  const int phw0 = cr[C_PHW0], phw1 = cr[C_PHW1], phw2 = cr[C_PHW2];
  int sidx[M];
#pragma unroll
  for (int i = 0; i < M; ++i) sidx[i] = 0;
  for (int r = 0; r < ns; ++r) {
    const int w = r < 8 ? phw0 : (r < 16 ? phw1 : phw2);
    const int ph = (w >> (3 * (r & 7))) & 7;
    const int prow = pair0 + ((r * (r + 1)) >> 1);
    const Rec32* tr = Ss + (s0 + r) * 3;
    bool red[M];
    float rf[M];
    const Pair32* pp[M];
#pragma unroll
    for (int i = 0; i < M; ++i) {
      red[i] = (m[i] >> (bit0 + r)) & 1u;
      rf[i] = red[i] ? 1.f : 0.f;
      pp[i] = Ps + (prow + sidx[i]) * 3;
    }
#pragma unroll
    for (int p = 0; p < 3; ++p) {
      if (!(ph >> p & 1)) continue;
      Rec32 t;
      if (ERR) t = tr[p];
#pragma unroll
      for (int i = 0; i < M; ++i) {
        const Pair32 q = pp[i][p];
        S[i][p].x = fmaf(rf[i], q.P.x, S[i][p].x);
        S[i][p].y = fmaf(rf[i], q.P.y, S[i][p].y);
        if (ERR) {
          const float d = diff32(t.W, t.w, S[i][p]);
          const float ek = fmaxf(t.a + d, t.b - d);
          const float er = fmaxf(q.a + dd[i][p], q.b - dd[i][p]);
          el[i] = fmaxf(el[i], red[i] ? er : ek);
          slack[i] = red[i] ? slack[i] : fminf(slack[i], fminf(t.bmin + d, t.bmax - d));
          dd[i][p] = red[i] ? dd[i][p] : d;
        }
      }
    }
#pragma unroll
    for (int i = 0; i < M; ++i) sidx[i] = red[i] ? sidx[i] : r + 1;
  }
#pragma unroll
  for (int i = 0; i < M; ++i)
#pragma unroll
    for (int p = 0; p < 3; ++p) B[i][p] = S[i][p];
}

// FP32 screen of every mask (M masks per lane, layout as in k_score_fp64):
// tile records of sure / possible / uncertain feasibility.
template <int M>
__global__ __launch_bounds__(kScoreThreads) void k_score_fp32(
    const SegHdr* __restrict__ hdrs, const int* __restrict__ segs, size_t lstride, const int* __restrict__ tab,
    const Pair32* __restrict__ P32, const Rec32* __restrict__ S32, const Head32* __restrict__ H32,
    const Rec32* __restrict__ Z32, const double* __restrict__ econst, int snaps_per_group, int SG, SelParams sp,
    MaskScore32* __restrict__ part, MaskScore32* __restrict__ fin, TileRec32* __restrict__ tiles,
    int* __restrict__ tickets) {
  __shared__ Pair32 Ps[kMaxPairs * 3];
  __shared__ Rec32 Ts[kMaxK * 3];
  __shared__ Head32 Hv[kMaxK * 3];
  __shared__ Rec32 Zs[kZoneLds];
  __shared__ double s_ec;
  __shared__ int ticket;
  const SegHdr H = load_hdr(hdrs, segs);
  if (!H.valid) return;
  // blocks past this segment's masks (a chunk's launch covers its largest segment)
  if ((uint64_t)blockIdx.x * (kScoreThreads * M) >= ((uint64_t)1 << H.k)) return;
  tab = lane_ptr(tab, lstride);
  P32 = lane_ptr(P32, lstride);
  S32 = lane_ptr(S32, lstride);
  H32 = lane_ptr(H32, lstride);
  Z32 = lane_ptr(Z32, lstride);
  econst = lane_ptr(econst, lstride);
  part = lane_ptr(part, lstride);
  fin = lane_ptr(fin, lstride);
  tiles = lane_ptr(tiles, lstride);
  tickets = lane_ptr(tickets, lstride);
  const int tid = threadIdx.x;
  // lane set i of the block: tile x[i] / 64 (tile_mask over the segment's lane bits)
  const uint32_t L = (uint32_t)H.lanebits;
  uint32_t x[M], m[M];
#pragma unroll
  for (int i = 0; i < M; ++i) {
    x[i] = blockIdx.x * (kScoreThreads * M) + i * kScoreThreads + tid;
    m[i] = tile_mask(L, x[i] / kScoreBlock, x[i] % kScoreBlock, H.k);
  }
  const int sg = blockIdx.y;
  const int l0 = sg * snaps_per_group;
  const int l1 = min(H.S, l0 + snaps_per_group);
  const int* chains = tab + H.o_chain;
  const int* nest = tab + H.o_nest;
  const Stage z = stage_sizes(H);
  float e[M], slack[M];
#pragma unroll
  for (int i = 0; i < M; ++i) {
    e[i] = 0.f;
    slack[i] = INFINITY;
  }
  for (int l = l0; l < l1; ++l) {
    {
      const uint4* P_l = (const uint4*)(P32 + (size_t)l * H.npairs * 3);
      const uint4* S_l = (const uint4*)(S32 + (size_t)l * H.nslots * 3);
      const uint4* H_l = (const uint4*)(H32 + (size_t)l * H.nchains * 3);
      const uint4* Z_l = (const uint4*)(Z32 + (size_t)l * H.nz);
      for (int i = tid; i < z.total; i += kScoreThreads)
        stage_put(z, i, stage_src(z, i, P_l, S_l, H_l, Z_l), (uint4*)Ps, (uint4*)Ts, (uint4*)Hv, (double*)nullptr,
                  (uint4*)Zs);
      if (tid == 0) s_ec = econst[l];
      __syncthreads();
    }
    const Rec32* Zl = Z32 + (size_t)l * H.nz;
    float el[M];
    const float ec = (float)s_ec;
#pragma unroll
    for (int i = 0; i < M; ++i) el[i] = ec;
    for (int c = 0; c < H.nchains; ++c) {
      const int* cr = chains + c * kChainInts;
      if (!(cr[C_PMASK] & L)) continue;  // the same for the wave's lanes: below
      float2 B[M][3];
#pragma unroll
      for (int i = 0; i < M; ++i)
#pragma unroll
        for (int p = 0; p < 3; ++p) B[i][p] = make_float2(0.f, 0.f);
      const int nl = cr[C_NEST_LEN], no = cr[C_NEST_OFF];
      for (int q = 0; q + 1 < nl; ++q) {
        const int oc = nest[no + q];
        walk32<false, M>(chains + oc * kChainInts, Ps, Ts, Hv, oc, m, B, el, slack);
      }
      walk32<true, M>(cr, Ps, Ts, Hv, c, m, B, el, slack);
#pragma unroll
      for (int p = 0; p < 3; ++p)
        for (int q = cr[C_ZOFF0 + p], qe = q + cr[C_ZCNT0 + p]; q < qe; ++q) {
          Rec32 t;
          if (q < kZoneLds) t = Zs[q];
          else t = Zl[q];
#pragma unroll
          for (int i = 0; i < M; ++i) {
            const float d = diff32(t.W, t.w, B[i][p]);
            el[i] = fmaxf(el[i], fmaxf(t.a + d, t.b - d));
            slack[i] = fminf(slack[i], fminf(t.bmin + d, t.bmax - d));
          }
        }
    }
#pragma unroll
    for (int i = 0; i < M; ++i) e[i] = fmaxf(e[i], el[i]);
    __syncthreads();
  }
  // Chains none of whose bits is among the lane bits (the 6 that vary across
  // a wave's lanes) have the same terms for the wave's 64 masks of each of
  // its M mask sets:
  // evaluated once per wave and mask set, one snapshot per lane, from the
  // tables in global memory, folded across the lanes.
  {
    const int lane = tid & 63;
    for (int c = 0; c < H.nchains; ++c) {
      const int* cr = chains + c * kChainInts;
      if (cr[C_PMASK] & L) continue;
      const int nl = cr[C_NEST_LEN], no = cr[C_NEST_OFF];
#pragma unroll
      for (int i = 0; i < M; ++i) {
        const uint32_t mi[1] = {(uint32_t)__builtin_amdgcn_readfirstlane((int)m[i])};
        float ue = 0.f, us = INFINITY;
        for (int l = l0 + lane; l < l1; l += 64) {
          const Pair32* P_l = P32 + (size_t)l * H.npairs * 3;
          const Rec32* S_l = S32 + (size_t)l * H.nslots * 3;
          const Head32* H_l = H32 + (size_t)l * H.nchains * 3;
          const Rec32* Z_l = Z32 + (size_t)l * H.nz;
          float2 B[1][3];
#pragma unroll
          for (int p = 0; p < 3; ++p) B[0][p] = make_float2(0.f, 0.f);
          float el1[1] = {0.f}, sl1[1] = {INFINITY};
          for (int q = 0; q + 1 < nl; ++q) {
            const int oc = nest[no + q];
            walk32<false, 1>(chains + oc * kChainInts, P_l, S_l, H_l, oc, mi, B, el1, sl1);
          }
          walk32<true, 1>(cr, P_l, S_l, H_l, c, mi, B, el1, sl1);
#pragma unroll
          for (int p = 0; p < 3; ++p)
            for (int q = cr[C_ZOFF0 + p], qe = q + cr[C_ZCNT0 + p]; q < qe; ++q) {
              const Rec32 t = Z_l[q];
              const float d = diff32(t.W, t.w, B[0][p]);
              el1[0] = fmaxf(el1[0], fmaxf(t.a + d, t.b - d));
              sl1[0] = fminf(sl1[0], fminf(t.bmin + d, t.bmax - d));
            }
          ue = fmaxf(ue, el1[0]);
          us = fminf(us, sl1[0]);
        }
        for (int o = 32; o > 0; o >>= 1) {
          ue = fmaxf(ue, __shfl_xor(ue, o, 64));
          us = fminf(us, __shfl_xor(us, o, 64));
        }
        e[i] = fmaxf(e[i], ue);
        slack[i] = fminf(slack[i], us);
      }
    }
  }
  const uint32_t nmask = 1u << H.k;
#pragma unroll
  for (int i = 0; i < M; ++i)
    if (x[i] < nmask) {
      MaskScore32 r;
      r.e = e[i];
      r.slack = slack[i];
      part[(size_t)sg * nmask + m[i]] = r;
    }
  // every wave's partial scores are written and visible before the block
  // takes its ticket (the last block to take one reads them all)
  __threadfence();
  __syncthreads();
  if (tid == 0) ticket = atomicAdd(&tickets[blockIdx.x], 1);
  __syncthreads();
  if (ticket != SG - 1) return;
  __threadfence();
  const double dlt = sp.delta + sp.amb;
#pragma unroll
  for (int i = 0; i < M; ++i) {
    const bool valid = x[i] < nmask;
    MaskScore32 r;
    r.e = 0.f;
    r.slack = INFINITY;
    if (valid) {
      for (int q = 0; q < SG; ++q) {
        const volatile MaskScore32* x = part + (size_t)q * nmask + m[i];
        r.e = fmaxf(r.e, x->e);
        r.slack = fminf(r.slack, x->slack);
      }
      fin[m[i]] = r;
    }
    const bool sure = valid && (double)r.e <= sp.e_bar - dlt && (double)r.slack >= dlt;
    const bool poss = valid && (double)r.e <= sp.e_bar + dlt && (double)r.slack >= -dlt;
    const int pc = __popc(m[i]);
    int a = sure ? pc : -1, b = poss ? pc : -1, c = (poss && !sure) ? pc : -1;
    for (int o = 32; o > 0; o >>= 1) {
      a = max(a, __shfl_xor(a, o, 64));
      b = max(b, __shfl_xor(b, o, 64));
      c = max(c, __shfl_xor(c, o, 64));
    }
    const uint32_t tile = x[i] / kScoreBlock;
    if ((tid & 63) == 0 && tile * kScoreBlock < nmask) {
      TileRec32 t;
      t.sure = a;
      t.poss = b;
      t.unc = c;
      t.pad = 0;
      tiles[tile] = t;
    }
  }
  if (tid == 0) tickets[blockIdx.x] = 0;
}

#define OKR_SCORE32_INST(M_)                                                                                   \
  template __global__ void k_score_fp32<M_>(const SegHdr*, const int*, size_t, const int*, const Pair32*, const Rec32*,       \
                                            const Head32*, const Rec32*, const double*, int, int, SelParams,  \
                                            MaskScore32*, MaskScore32*, TileRec32*, int*);
OKR_SCORE32_INST(1)
OKR_SCORE32_INST(2)
OKR_SCORE32_INST(4)
#undef OKR_SCORE32_INST

}  // namespace okr
