// Device-side construction of one segment's tables from the cumulative kept
// state (no host round trip between segments).
//
//   k_build_struct  (1 block)  chains, slots, pairs, nesting, Omega ranges,
//                              zone entries grouped by (chain, phase)
//   k_build_values  (grid)     P = Z(super -> reduced) A, record voltages,
//                              min/max initialisation
//   k_build_members (grid)     cluster min/max |V^| and the constant error of
//                              clusters whose super-node is outside Omega_g
//
// The tables have the layout the scoring kernel reads (okr_internal.h).
#include <hip/hip_runtime.h>
#include <limits.h>
#include <math.h>
#include <stdint.h>

#include "okr_internal.h"

namespace okr {

__device__ __forceinline__ double2 b_cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 b_cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// status bit set when a structural invariant fails (the segment is then
// skipped by the scoring path and the call reports an error)
constexpr int kStatusBuild = 64;
constexpr int kOmegaLds = 4096;  // Omega_g nodes whose zone classification is kept in shared memory
// structural part of a segment's tables (chains, nesting, slots, pairs, ranges)
constexpr int kTabLds = kMaxK * kChainInts + kMaxK * kMaxK + kMaxK * kSlotInts + kMaxPairs * kPairInts + 3 * kMaxK;

// Child of kept node h on the tree path down to its descendant v.
__device__ __forceinline__ int child_toward(const Topo& T, int h, int v) {
  const int pv = T.pos[v];
  for (int q = T.ch_off[h]; q < T.ch_off[h + 1]; ++q) {
    const int x = T.ch[q];
    if (T.pos[x] <= pv && pv < T.pos[x] + T.size[x]) return x;
  }
  return -1;
}

__global__ __launch_bounds__(256) void k_build_struct(Topo T, State St, const int* __restrict__ segs, size_t lstride,
                                                      int S, SegHdr* __restrict__ hdrs, int* __restrict__ tab,
                                                      int tab_cap, int* __restrict__ status) {
  __shared__ int s_top[kMaxK], s_slotnode[kMaxK], s_slotbit[kMaxK], s_slotchain[kMaxK];
  __shared__ int s_cslot0[kMaxK + 1], s_head[kMaxK], s_outer[kMaxK], s_jslot[kMaxK];
  __shared__ int s_spos[kMaxK], s_ssize[kMaxK], s_sph[kMaxK];           // segment node j
  __shared__ int s_tpos[kMaxK], s_tsize[kMaxK], s_thead[kMaxK], s_thph[kMaxK];  // its chain top
  __shared__ int s_cpos[kMaxK], s_csize[kMaxK], s_chph[kMaxK];          // chain c: top pos/size, head phase
  __shared__ int s_rs[kMaxK], s_rcum[kMaxK + 1];                       // Omega_g ranges: start, cumulative size
  __shared__ int s_seg[kMaxK], s_thpos[kMaxK], s_first[kMaxK];          // segment node j, its top's head position,
                                                                        // first segment node with its top
  __shared__ int s_chpos[kMaxK], s_rkeep[kMaxK], s_depth[kMaxK];        // chain c: head position, new range, nesting
  __shared__ int s_pmask[kMaxK];                                        // chain c: mask bits of its nesting path
  __shared__ int s_okey[kMaxK];  // chain c: (preorder position << 5) | j of the deepest segment node above its head
  // exclusive prefix sums over the chains (entry nch: the totals) of: nesting
  // depth, pairs, new Omega_g range, its nodes, chain patterns
  __shared__ int s_xs[5][kMaxK + 1];
  __shared__ int s_keycnt[kMaxK * 3], s_keyoff[kMaxK * 3], s_keycur[kMaxK * 3];
  __shared__ SegHdr s_h;
  __shared__ int s_err, s_nch;
  __shared__ int s_cw[kMaxK];                 // chain c: its per-lane scoring work
  __shared__ uint32_t s_clos[kMaxK];          // chain c: chains whose terms depend on c's bits
  __shared__ int s_zi[kOmegaLds], s_zk[kOmegaLds];  // zone pass: node and key of Omega index q
  __shared__ int s_tab[kTabLds];                     // structural tables before they are written out
  const int g = segs[blockIdx.z];
  tab = lane_ptr(tab, lstride);
  const int* parent = T.parent;
  const int* segment = T.segment;
  const int tid = threadIdx.x;
  const int o0 = T.seg_off[g];
  const int k = T.seg_off[g + 1] - o0;
  if (tid == 0) {
    // an earlier segment failed: leave every later one invalid (its scratch
    // maps may be stale)
    s_err = ((*status & kStatusBuild) || k < 1 || k > kMaxK) ? 1 : 0;
    s_nch = 0;
  }
  if (tid < kMaxK) {
    s_okey[tid] = -1;
    s_rkeep[tid] = 1;
  }
  __syncthreads();
  // chain top of every segment node: the highest node above it reachable
  // through segment or reduced nodes (runs of reduced nodes are crossed in
  // one step: their nearest kept ancestor is known)
  if (!s_err && tid < k) {
    const int e = T.seg_nodes[o0 + tid];
    int c = T.seg_top[e], guard = 0;  // (runs of this segment's nodes climbed at plan time)
    for (;;) {
      const int p = parent[c];
      if (p < 0 || ++guard > T.n) break;
      if (segment[p] == g) { c = T.seg_top[p]; continue; }
      if (St.kept[p]) break;
      const int h = St.sup[p];
      const int x = (h >= 0 && h != p) ? child_toward(T, h, p) : -1;
      if (x < 0) { atomicOr(&s_err, 1); break; }
      c = x;
    }
    s_top[tid] = c;
    s_spos[tid] = T.pos[e];
    s_ssize[tid] = T.size[e];
    s_sph[tid] = T.phase[e];
    const int hd = parent[c];
    s_tpos[tid] = T.pos[c];
    s_tsize[tid] = T.size[c];
    s_thead[tid] = hd;
    s_thph[tid] = hd >= 0 ? T.phase[hd] : 0;
    s_thpos[tid] = hd >= 0 ? T.pos[hd] : -1;
    s_seg[tid] = e;
  }
  __syncthreads();
  // chains: one per distinct chain top, ordered by the tops' preorder
  // positions (distinct nodes, so the order is strict); slots chain by chain,
  // top to bottom (segment nodes are in preorder).  One thread per segment
  // node, shared-memory data only from here on.
  if (!s_err && tid < k) {
    const int top = s_top[tid];
    int j0 = tid;  // first segment node with this chain top
    for (int q = tid - 1; q >= 0; --q)
      if (s_top[q] == top) j0 = q;
    s_first[tid] = j0;
  }
  __syncthreads();
  if (!s_err && tid < k) {
    const int j = tid, j0 = s_first[j], tp = s_tpos[j];
    int c = 0, before = 0, within = 0, nch = 0;
    for (int q = 0; q < k; ++q) {
      const bool lower = s_tpos[q] < tp;  // q's chain comes before j's
      const bool opens = s_first[q] == q;
      nch += opens;
      c += opens && lower;
      before += lower;
      within += (s_first[q] == j0) && q < j;
    }
    const int s = before + within;
    s_jslot[j] = s;
    s_slotnode[s] = s_seg[j];
    s_slotbit[s] = j;
    s_slotchain[s] = c;
    if (j0 == j) {
      s_cpos[c] = tp;
      s_csize[c] = s_tsize[j];
      s_chph[c] = s_thph[j];
      s_head[c] = s_thead[j];
      s_chpos[c] = s_thpos[j];
      s_cslot0[c] = before;
    }
    if (j == 0) {
      s_nch = nch;
      s_cslot0[nch] = k;
    }
  }
  __syncthreads();
  // per chain: the outer chain (whose bottom slot is the deepest segment node
  // above the head), the path and consecutive-bit invariants, and whether its
  // top's subtree starts a new Omega_g range (laminar intervals in preorder:
  // a top inside an earlier top's subtree adds nothing)
  const int nch = s_nch;
  // over (chain, segment node) pairs: the deepest segment node whose subtree
  // holds the chain's head (positions are distinct, so the largest key is
  // that node); over (chain, earlier chain) pairs: whether the chain's top
  // lies in an earlier chain top's subtree (then it starts no new range)
  if (!s_err) {
    for (int x = tid; x < nch * k; x += blockDim.x) {
      const int c = x / k, j = x - c * k, ph = s_chpos[c];
      if (ph >= 0 && s_spos[j] <= ph && ph < s_spos[j] + s_ssize[j]) atomicMax(&s_okey[c], (s_spos[j] << 5) | j);
    }
    for (int x = tid; x < nch * nch; x += blockDim.x) {
      const int c = x / nch, q = x - c * nch;
      if (q < c && s_cpos[q] <= s_cpos[c] && s_cpos[c] < s_cpos[q] + s_csize[q]) s_rkeep[c] = 0;
    }
  }
  __syncthreads();
  if (!s_err && tid < nch) {
    const int c = tid;
    const int best = s_okey[c] >= 0 ? (s_okey[c] & 31) : -1;
    int oc = -1;
    if (best >= 0) {
      const int s = s_jslot[best];
      oc = s_slotchain[s];
      if (s != s_cslot0[oc + 1] - 1 || oc >= c) atomicOr(&s_err, 1);
    }
    s_outer[c] = oc;
    // every chain is a path: each slot lies below the previous one (the first
    // below the chain top); its nodes have at most one child, so its slots
    // are consecutive segment nodes in preorder: consecutive mask bits
    int pu = s_cpos[c], su = s_csize[c];
    const int s0 = s_cslot0[c], s1 = s_cslot0[c + 1];
    for (int s = s0; s < s1; ++s) {
      const int j = s_slotbit[s], pv = s_spos[j];
      if (!(pu <= pv && pv < pu + su) || (s > s0 && pv == pu) || j != s_slotbit[s0] + (s - s0))
        atomicOr(&s_err, 1);
      pu = pv;
      su = s_ssize[j];
    }
  }
  __syncthreads();
  if (tid < nch) {
    // nesting depth (outer chains have smaller indices) and the mask bits of
    // the chains on the nesting path, the chain itself included
    int d = 0, pm = 0;
    if (!s_err)
      for (int x = tid; x >= 0; x = s_outer[x]) {
        ++d;
        pm |= ((1 << (s_cslot0[x + 1] - s_cslot0[x])) - 1) << s_slotbit[s_cslot0[x]];
      }
    s_depth[tid] = d;
    s_pmask[tid] = pm;
  }
  __syncthreads();
  // the chains' table offsets: prefix sums in one wave (lane = chain)
  if (tid < 64) {
    int v[5] = {0, 0, 0, 0, 0};
    if (tid < nch) {
      const int n = s_cslot0[tid + 1] - s_cslot0[tid];
      v[0] = s_depth[tid];
      v[1] = n * (n + 1) / 2;
      v[2] = s_rkeep[tid];
      v[3] = s_rkeep[tid] ? s_csize[tid] : 0;
      v[4] = 1 << __popc(s_pmask[tid]);
    }
#pragma unroll
    for (int i = 0; i < 5; ++i) {
      int x = v[i];
      for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o, 64);
        if (tid >= o) x += y;
      }
      if (tid <= nch) s_xs[i][tid] = x - v[i];
    }
  }
  __syncthreads();
  // table layout
  const int nest_tot = s_xs[0][nch], npairs = s_xs[1][nch], nr = s_xs[2][nch], nom = s_xs[3][nch],
            npat = s_xs[4][nch];
  const int o_nest = nch * kChainInts, o_slot = o_nest + nest_tot, o_pair = o_slot + k * kSlotInts;
  const int o_range = o_pair + npairs * kPairInts, o_zent = o_range + 3 * nr;
  if (tid == 0) {
    SegHdr H;
    for (int q = 0; q < (int)(sizeof(SegHdr) / sizeof(int)); ++q) ((int*)&H)[q] = 0;
    H.g = g;
    H.k = k;
    H.S = S;
    H.o_chain = 0;
    H.o_nest = o_nest;
    H.o_slot = o_slot;
    H.o_pair = o_pair;
    H.o_range = o_range;
    H.o_zent = o_zent;
    H.nrange = nr;
    H.nomega = nom;
    H.nchains = nch;
    H.nslots = k;
    H.npairs = npairs;
    H.npat = npat;
    // the structural part must fit the segment's table (and the shared image,
    // which holds the largest possible one)
    if (o_zent > tab_cap || o_zent > kTabLds) s_err = 1;
    // the chain patterns number at most 2^(k+1) (a nesting forest whose
    // chains hold k bits in all): the pattern table's capacity
    if (npat > (2 << k)) s_err = 1;
    H.valid = s_err ? 0 : 1;
    s_h = H;
  }
  if (tid < kMaxK * 3) {
    s_keycnt[tid] = 0;
    s_keycur[tid] = 0;
  }
  __syncthreads();
  if (s_err) {
    if (tid == 0) {
      SegHdr H = s_h;
      H.valid = 0;
      hdrs[g] = H;
      atomicOr(status, kStatusBuild);
    }
    return;
  }
  // records: one thread per chain, one per slot
  if (tid < nch) {
    const int c = tid, s0 = s_cslot0[c], n = s_cslot0[c + 1] - s0;
    const int nest_off = s_xs[0][c], pair0 = s_xs[1][c], ridx = s_xs[2][c], rcum = s_xs[3][c], pbase = s_xs[4][c];
    const int d = s_depth[c];
    int q = d - 1;
    for (int x = c; x >= 0; x = s_outer[x]) s_tab[o_nest + nest_off + q--] = x;
    if (s_rkeep[c]) {
      s_tab[o_range + 3 * ridx] = s_cpos[c];
      s_tab[o_range + 3 * ridx + 1] = s_cpos[c] + s_csize[c];
      s_tab[o_range + 3 * ridx + 2] = rcum;
    }
    int phw[3] = {0, 0, 0};
    for (int r = 0; r < n; ++r) phw[r >> 3] |= s_sph[s_slotbit[s0 + r]] << (3 * (r & 7));
    int* cr = s_tab + c * kChainInts;
    cr[C_HEAD] = s_head[c];
    cr[C_NSLOT] = n;
    cr[C_SLOT0] = s0;
    cr[C_NEST_OFF] = nest_off;
    cr[C_NEST_LEN] = d;
    cr[C_OUTER] = s_outer[c];
    cr[C_PHASE] = s_chph[c];
    cr[C_BIT0] = s_slotbit[s0];
    cr[C_PAIR0] = pair0;
    cr[C_PHW0] = phw[0];
    cr[C_PHW1] = phw[1];
    cr[C_PHW2] = phw[2];
    cr[C_PMASK] = s_pmask[c];
    cr[C_PBASE] = pbase;
    for (int p = 0; p < 3; ++p) {
      cr[C_ZOFF0 + p] = 0;  // zone ranges filled after the zone pass
      cr[C_ZCNT0 + p] = 0;
    }
  }
  if (tid < k) {
    // slot s = r-th slot of chain c: pairs (super, reduced) with the super
    // node the head or one of the r slots above it
    const int s = tid, c = s_slotchain[s], s0 = s_cslot0[c], r = s - s0;
    const int pb = s_xs[1][c] + r * (r + 1) / 2;
    int* sr = s_tab + o_slot + s * kSlotInts;
    sr[SL_NODE] = s_slotnode[s];
    sr[SL_BIT] = s_slotbit[s];
    sr[SL_PHASE] = s_sph[s_slotbit[s]];
    sr[SL_PAIRBASE] = pb;
    sr[SL_CHAIN] = c;
    for (int sx = 0; sx <= r; ++sx) {
      int* pr = s_tab + o_pair + (pb + sx) * kPairInts;
      pr[PR_RNODE] = s_slotnode[s];
      pr[PR_SUPER] = (sx == 0) ? s_head[c] : s_slotnode[s0 + sx - 1];
      pr[PR_RSLOT] = s;
    }
    St.slot_of[s_slotnode[s]] = s;
  }
  __syncthreads();
  // the structural tables, built in shared memory, written out by all threads
  for (int q = tid; q < o_zent; q += blockDim.x) tab[q] = s_tab[q];
  // Omega_g ranges for the zone pass (shared copy)
  if (tid < nch && s_rkeep[tid]) {
    s_rs[s_xs[2][tid]] = s_cpos[tid];
    s_rcum[s_xs[2][tid]] = s_xs[3][tid];
  }
  if (tid == 0) s_rcum[nr] = nom;
  __syncthreads();
  SegHdr H = s_h;
  // zone targets: kept nodes of Omega_g outside the segment; anchor = chain
  // whose bottom slot is the first segment node above the target.  The
  // counting pass keeps what it found for the first kOmegaLds nodes in
  // shared memory, so the placing pass re-reads nothing for them; ranges,
  // slot chains and chain bottoms come from shared memory throughout.
  auto classify = [&](int q, int& node, int& key) {  // key = chain * 8 | phase bits, -1: not a target
    int r = 0;
    while (r + 1 < nr && s_rcum[r + 1] <= q) ++r;
    const int i = T.pre[s_rs[r] + (q - s_rcum[r])];
    node = i;
    key = -1;
    if (segment[i] == g || !St.kept[i]) return;
    const int pi = T.pos[i];
    int best = -1;
    for (int j = 0; j < k; ++j)
      if (s_spos[j] < pi && pi < s_spos[j] + s_ssize[j] && (best < 0 || s_spos[j] > s_spos[best])) best = j;
    const int s = (best >= 0) ? s_jslot[best] : -1;
    if (s < 0) { atomicOr(&s_err, 1); return; }
    const int c = s_slotchain[s];
    if (s != s_cslot0[c + 1] - 1) { atomicOr(&s_err, 1); return; }  // must be the chain's bottom
    key = c * 8 + (int)T.phase[i];
  };
  for (int q = threadIdx.x; q < nom; q += blockDim.x) {
    int i, key;
    classify(q, i, key);
    if (q < kOmegaLds) {
      s_zi[q] = i;
      s_zk[q] = key;
    }
    if (key < 0) continue;
    for (int p = 0; p < 3; ++p)
      if (key >> p & 1) atomicAdd(&s_keycnt[(key >> 3) * 3 + p], 1);
  }
  __syncthreads();
  // zone entries grouped by key (chain, phase): offsets by an exclusive sum
  if (!s_err && tid < nch * 3) {
    int acc = 0;
    for (int q = 0; q < tid; ++q) acc += s_keycnt[q];
    const int cnt = s_keycnt[tid];
    s_keyoff[tid] = acc;
    int* cr = tab + H.o_chain + (tid / 3) * kChainInts;
    cr[C_ZOFF0 + tid % 3] = acc;
    cr[C_ZCNT0 + tid % 3] = cnt;
    if (tid == nch * 3 - 1) {
      s_h.nz = acc + cnt;
      s_h.total_ints = H.o_zent + 3 * (acc + cnt);
      if (s_h.total_ints > tab_cap) s_err = 1;
    }
  }
  // Lane bits of the scoring kernel: a wave's 64 lanes vary 6 mask bits, and
  // a chain none of whose bits (its own and its nesting path's) is among them
  // is evaluated once per wave instead of per lane.  Chosen greedily: take
  // the bits of the chain that adds the least per-lane work per bit gained
  // (work of a chain: 2 per slot-phase, 1 per zone record, 1 per slot walked
  // on its nesting path), until 6 bits are taken.
  if (!s_err && tid < nch) {
    const int c = tid;
    int wk = 0;
    for (int q = s_cslot0[c]; q < s_cslot0[c + 1]; ++q) wk += 2 * __popc(s_sph[s_slotbit[q]]);
    for (int p = 0; p < 3; ++p) wk += s_keycnt[c * 3 + p];
    for (int x = s_outer[c]; x >= 0; x = s_outer[x]) wk += s_cslot0[x + 1] - s_cslot0[x];
    s_cw[c] = wk;
    const int n = s_cslot0[c + 1] - s_cslot0[c];
    const uint32_t own = ((1u << n) - 1u) << s_slotbit[s_cslot0[c]];
    uint32_t cl = 0;
    for (int d = 0; d < nch; ++d)
      if ((uint32_t)s_pmask[d] & own) cl |= 1u << d;
    s_clos[c] = cl;
  }
  __syncthreads();
  // the greedy choice itself in one wave (candidates in lanes, wave-wide
  // minimum; the chosen bits and the chains they touch kept in registers)
  if (tid < 64) {
    uint32_t lane_bits = 0, touched = 0;
    for (int need = s_err ? 0 : min(6, k); need > 0;) {
      long long key = LLONG_MAX;
      if (tid < nch) {
        const int c = tid;
        const int n = s_cslot0[c + 1] - s_cslot0[c];
        const uint32_t own = ((1u << n) - 1u) << s_slotbit[s_cslot0[c]];
        const int nb = min(__popc(own & ~lane_bits), need);
        if (nb > 0) {
          int add = 0;
          for (uint32_t x = s_clos[c] & ~touched; x; x &= x - 1) add += s_cw[__builtin_ctz(x)];
          // added work per bit, in 1/720 units (exact for 1..6 bits), then the chain
          key = ((long long)(add * (720 / nb)) << 8) | c;
        }
      }
      for (int o = 32; o > 0; o >>= 1) {
        const long long other = __shfl_xor(key, o, 64);
        key = other < key ? other : key;
      }
      const int best = (int)(key & 255);
      const int n = s_cslot0[best + 1] - s_cslot0[best];
      uint32_t free_bits = (((1u << n) - 1u) << s_slotbit[s_cslot0[best]]) & ~lane_bits;
      for (int b = 0; b < need && free_bits; ++b, free_bits &= free_bits - 1) lane_bits |= free_bits & (0u - free_bits);
      touched |= s_clos[best];
      need = min(6, k) - __popc(lane_bits);
    }
    if (tid == 0) s_h.lanebits = (int)lane_bits;
  }
  __syncthreads();
  if (!s_err)
    for (int q = threadIdx.x; q < nom; q += blockDim.x) {
      int i, key;
      if (q < kOmegaLds) {
        i = s_zi[q];
        key = s_zk[q];
      } else {
        classify(q, i, key);
      }
      if (key < 0) continue;
      const int c = key >> 3;
      for (int p = 0; p < 3; ++p) {
        if (!(key >> p & 1)) continue;
        const int idx = s_keyoff[c * 3 + p] + atomicAdd(&s_keycur[c * 3 + p], 1);
        int* ze = tab + H.o_zent + 3 * idx;
        ze[0] = i;
        ze[1] = p;
        ze[2] = c;
        St.zent_of[i * 3 + p] = idx;
      }
    }
  __syncthreads();
  if (threadIdx.x == 0) {
    H = s_h;
    if (s_err) {
      H.valid = 0;
      atomicOr(status, kStatusBuild);
    }
    hdrs[g] = H;
  }
}

// Node of Omega_g with flattened index q (ranges: start, end, cumulative).
__device__ __forceinline__ int omega_node(const Topo& T, const int* rg, int nr, int q) {
  int r = 0;
  while (r + 1 < nr && rg[3 * (r + 1) + 2] <= q) ++r;
  return T.pre[rg[3 * r] + (q - rg[3 * r + 2])];
}

__global__ __launch_bounds__(256) void k_build_values(const SegHdr* __restrict__ hdrs, const int* __restrict__ segs,
                                                      size_t lstride, const int* __restrict__ tab, int n,
                                                      const double2* __restrict__ Zroot,
                                                      const double2* __restrict__ Vcur,
                                                      const double2* __restrict__ A, double2* __restrict__ P,
                                                      TargetRec* __restrict__ srec, double2* __restrict__ headV,
                                                      TargetRec* __restrict__ zrec, double* __restrict__ econst) {
  const SegHdr H = load_hdr(hdrs, segs);
  if (!H.valid) return;
  tab = lane_ptr(tab, lstride);
  P = lane_ptr(P, lstride);
  srec = lane_ptr(srec, lstride);
  headV = lane_ptr(headV, lstride);
  zrec = lane_ptr(zrec, lstride);
  econst = lane_ptr(econst, lstride);
  const int part = blockIdx.y;
  const int S = H.S;
  const int stride = gridDim.x * blockDim.x;
  if (part == 0) {
    // P = Z(super -> reduced) A_reduced with Z(s -> r) = Zroot(r) - Zroot(s),
    // the series impedance of the path between them
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < S * H.npairs; t += stride) {
      const int l = t / H.npairs, q = t % H.npairs;
      const int* pr = tab + H.o_pair + q * kPairInts;
      const double2* zr = Zroot + (size_t)pr[PR_RNODE] * 9;
      const double2* zs = Zroot + (size_t)pr[PR_SUPER] * 9;
      double2 Z[9];
      for (int e = 0; e < 9; ++e) Z[e] = make_double2(zr[e].x - zs[e].x, zr[e].y - zs[e].y);
      const double2* a = A + ((size_t)l * n + pr[PR_RNODE]) * 3;
      double2* o = P + ((size_t)l * H.npairs + q) * 3;
      for (int r = 0; r < 3; ++r)
        o[r] = b_cadd(b_cadd(b_cmul(Z[r * 3], a[0]), b_cmul(Z[r * 3 + 1], a[1])), b_cmul(Z[r * 3 + 2], a[2]));
    }
  } else if (part == 1) {
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < S * H.nslots * 3; t += stride) {
      const int l = t / (H.nslots * 3), rem = t % (H.nslots * 3), s = rem / 3, p = rem % 3;
      const int node = tab[H.o_slot + s * kSlotInts + SL_NODE];
      TargetRec rec;
      rec.W = Vcur[((size_t)l * n + node) * 3 + p];
      rec.lo = INFINITY;
      rec.hi = 0.0;
      srec[((size_t)l * H.nslots + s) * 3 + p] = rec;
    }
  } else if (part == 2) {
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < S * H.nchains; t += stride) {
      const int l = t / H.nchains, c = t % H.nchains;
      const int head = tab[H.o_chain + c * kChainInts + C_HEAD];
      for (int p = 0; p < 3; ++p) headV[((size_t)l * H.nchains + c) * 3 + p] = Vcur[((size_t)l * n + head) * 3 + p];
    }
  } else if (part == 3) {
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < S * H.nz; t += stride) {
      const int l = t / H.nz, q = t % H.nz;
      const int* ze = tab + H.o_zent + q * 3;
      TargetRec rec;
      rec.W = Vcur[((size_t)l * n + ze[0]) * 3 + ze[1]];
      rec.lo = INFINITY;
      rec.hi = 0.0;
      zrec[(size_t)l * H.nz + q] = rec;
    }
  } else {
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < S; t += stride) econst[t] = 0.0;
  }
}

__device__ __forceinline__ void atomic_min_nonneg(double* a, double v) {
  atomicMin((unsigned long long*)a, (unsigned long long)__double_as_longlong(v));
}
__device__ __forceinline__ void atomic_max_nonneg(double* a, double v) {
  atomicMax((unsigned long long*)a, (unsigned long long)__double_as_longlong(v));
}

// Cluster statistics: every node of Omega_g contributes |V^| to the cluster of
// its current super-node (a slot, a zone target, or a head outside Omega_g,
// whose error is mask-independent and folds into econst).
__global__ __launch_bounds__(256) void k_build_members(const SegHdr* __restrict__ hdrs, const int* __restrict__ segs,
                                                       size_t lstride, const int* __restrict__ tab, Topo T, State St,
                                                       const double2* __restrict__ Vcur,
                                                       const double* __restrict__ absV, TargetRec* __restrict__ srec,
                                                       TargetRec* __restrict__ zrec, double* __restrict__ econst) {
  const int g = segs[blockIdx.z];
  const SegHdr H = load_hdr_g(hdrs, g);
  if (!H.valid) return;
  tab = lane_ptr(tab, lstride);
  srec = lane_ptr(srec, lstride);
  zrec = lane_ptr(zrec, lstride);
  econst = lane_ptr(econst, lstride);
  const int n = T.n;
  const int* rg = tab + H.o_range;
  const long total = (long)H.nomega * H.S;
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
    const int l = (int)(t / H.nomega), q = (int)(t % H.nomega);
    const int i = omega_node(T, rg, H.nrange, q);
    const int sp = St.sup[i];
    const unsigned ph = T.phase[i];
    const double* av = absV + ((size_t)l * n + i) * 3;
    if (T.segment[sp] == g) {
      const int s = St.slot_of[sp];
      if (s < 0 || s >= H.nslots) continue;
      TargetRec* r = srec + ((size_t)l * H.nslots + s) * 3;
      for (int p = 0; p < 3; ++p)
        if (ph >> p & 1u) { atomic_min_nonneg(&r[p].lo, av[p]); atomic_max_nonneg(&r[p].hi, av[p]); }
    } else {
      for (int p = 0; p < 3; ++p) {
        if (!(ph >> p & 1u)) continue;
        const int zi = St.zent_of[sp * 3 + p];
        if (zi >= H.nz) continue;
        if (zi >= 0) {
          TargetRec* r = zrec + (size_t)l * H.nz + zi;
          atomic_min_nonneg(&r->lo, av[p]);
          atomic_max_nonneg(&r->hi, av[p]);
        } else {
          const double2 v = Vcur[((size_t)l * n + sp) * 3 + p];
          atomic_max_nonneg(&econst[l], fabs(sqrt(v.x * v.x + v.y * v.y) - av[p]));
        }
      }
    }
  }
}

}  // namespace okr
