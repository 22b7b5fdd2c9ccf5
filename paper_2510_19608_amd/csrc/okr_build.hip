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

// Child of kept node h on the tree path down to its descendant v.
__device__ __forceinline__ int child_toward(const Topo& T, int h, int v) {
  const int pv = T.pos[v];
  for (int q = T.ch_off[h]; q < T.ch_off[h + 1]; ++q) {
    const int x = T.ch[q];
    if (T.pos[x] <= pv && pv < T.pos[x] + T.size[x]) return x;
  }
  return -1;
}

__global__ __launch_bounds__(256) void k_build_struct(Topo T, State St, int g, int S, SegHdr* __restrict__ hdrs,
                                                      int* __restrict__ tab, int tab_cap, int* __restrict__ status) {
  __shared__ int s_top[kMaxK], s_tops[kMaxK], s_slotnode[kMaxK], s_slotbit[kMaxK], s_slotchain[kMaxK];
  __shared__ int s_cslot0[kMaxK + 1], s_head[kMaxK], s_outer[kMaxK], s_jslot[kMaxK];
  __shared__ int s_spos[kMaxK], s_ssize[kMaxK], s_sph[kMaxK];           // segment node j
  __shared__ int s_tpos[kMaxK], s_tsize[kMaxK], s_thead[kMaxK], s_thph[kMaxK];  // its chain top
  __shared__ int s_cpos[kMaxK], s_csize[kMaxK], s_chph[kMaxK];          // chain c: top pos/size, head phase
  __shared__ int s_rs[kMaxK], s_re[kMaxK], s_rcum[kMaxK + 1];
  __shared__ int s_keycnt[kMaxK * 3], s_keyoff[kMaxK * 3], s_keycur[kMaxK * 3];
  __shared__ SegHdr s_h;
  __shared__ int s_err, s_nch;
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
  __syncthreads();
  // chain top of every segment node: the highest node above it reachable
  // through segment or reduced nodes (runs of reduced nodes are crossed in
  // one step: their nearest kept ancestor is known)
  if (!s_err && tid < k) {
    const int e = T.seg_nodes[o0 + tid];
    int c = e, guard = 0;
    for (;;) {
      const int p = parent[c];
      if (p < 0 || ++guard > T.n) break;
      if (segment[p] == g) { c = p; continue; }
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
  }
  __syncthreads();
  if (tid == 0 && !s_err) {
    // distinct chain tops (shared-memory data only from here on)
    int nch = 0, tj[kMaxK];
    for (int j = 0; j < k; ++j) {
      const int c = s_top[j];
      bool seen = false;
      for (int q = 0; q < nch; ++q) seen |= (s_tops[q] == c);
      if (!seen) {
        tj[nch] = j;
        s_tops[nch++] = c;
      }
    }
    // chains in preorder of their tops
    for (int a = 1; a < nch; ++a) {
      const int v = s_tops[a], vj = tj[a];
      int b = a - 1;
      while (b >= 0 && s_tpos[tj[b]] > s_tpos[vj]) {
        s_tops[b + 1] = s_tops[b];
        tj[b + 1] = tj[b];
        --b;
      }
      s_tops[b + 1] = v;
      tj[b + 1] = vj;
    }
    for (int c = 0; c < nch; ++c) {
      s_cpos[c] = s_tpos[tj[c]];
      s_csize[c] = s_tsize[tj[c]];
      s_chph[c] = s_thph[tj[c]];
    }
    // slots chain by chain, top to bottom (segment nodes are in preorder)
    int ns = 0;
    for (int c = 0; c < nch; ++c) {
      s_cslot0[c] = ns;
      for (int j = 0; j < k; ++j)
        if (s_top[j] == s_tops[c]) {
          s_slotnode[ns] = T.seg_nodes[o0 + j];
          s_slotbit[ns] = j;
          s_slotchain[ns] = c;
          s_jslot[j] = ns;
          ++ns;
        }
      s_head[c] = s_thead[tj[c]];
    }
    s_cslot0[nch] = ns;
    if (ns != k) s_err = 1;
    s_nch = nch;
  }
  __syncthreads();
  // outer chain: the chain whose bottom slot is the deepest segment node
  // above the head (a subtree test against every segment node)
  if (!s_err && tid < s_nch) {
    const int c = tid, hd = s_head[c];
    const int ph = hd >= 0 ? T.pos[hd] : -1;
    int best = -1;
    for (int j = 0; j < k; ++j)
      if (hd >= 0 && s_spos[j] <= ph && ph < s_spos[j] + s_ssize[j] && (best < 0 || s_spos[j] > s_spos[best]))
        best = j;
    s_outer[c] = -1;
    if (best >= 0) {
      const int u = T.seg_nodes[o0 + best];
      int s = -1;
      for (int q = 0; q < k; ++q)
        if (s_slotnode[q] == u) s = q;
      const int oc = s >= 0 ? s_slotchain[s] : -1;
      if (s < 0 || s != s_cslot0[oc + 1] - 1 || oc >= c) atomicOr(&s_err, 1);
      else s_outer[c] = oc;
    }
  }
  __syncthreads();
  if (tid == 0) {
    int err = s_err;
    const int nch = s_nch, ns = k;
    SegHdr H;
    for (int q = 0; q < (int)(sizeof(SegHdr) / sizeof(int)); ++q) ((int*)&H)[q] = 0;
    H.g = g;
    H.k = k;
    H.S = S;
    // table layout
    int o = 0;
    H.o_chain = o; o += nch * kChainInts;
    H.o_nest = o;
    if (o + nch * nch > tab_cap) err = 1;
    int nest_off[kMaxK], nest_len[kMaxK];
    for (int c = 0; c < nch && !err; ++c) {
      int d = 0;
      for (int x = c; x >= 0; x = s_outer[x]) ++d;
      nest_off[c] = o - H.o_nest;
      nest_len[c] = d;
      int q = d - 1;
      for (int x = c; x >= 0; x = s_outer[x]) tab[o + q--] = x;
      o += d;
    }
    // every chain is a path: each slot lies below the previous one (the
    // first below the chain top)
    for (int c = 0; c < nch && !err; ++c) {
      int pu = s_cpos[c], su = s_csize[c];
      for (int s = s_cslot0[c]; s < s_cslot0[c + 1]; ++s) {
        const int j = s_slotbit[s], pv = s_spos[j];
        if (!(pu <= pv && pv < pu + su) || (s > s_cslot0[c] && pv == pu)) { err = 1; break; }
        pu = pv;
        su = s_ssize[j];
      }
    }
    H.o_slot = o; o += ns * kSlotInts;
    H.o_pair = o;
    int npairs = 0, pairbase[kMaxK];
    for (int c = 0; c < nch && !err; ++c)
      for (int s = s_cslot0[c]; s < s_cslot0[c + 1]; ++s) {
        const int r = s - s_cslot0[c];
        pairbase[s] = npairs;
        for (int sx = 0; sx <= r; ++sx) {
          if (npairs >= kMaxPairs || o + kPairInts > tab_cap) { err = 1; break; }
          tab[o + PR_RNODE] = s_slotnode[s];
          tab[o + PR_SUPER] = (sx == 0) ? s_head[c] : s_slotnode[s_cslot0[c] + sx - 1];
          tab[o + PR_RSLOT] = s;
          o += kPairInts;
          ++npairs;
        }
      }
    // Omega_g ranges in preorder: union of the chain tops' subtrees
    int nr = 0;
    for (int c = 0; c < nch && !err; ++c) {
      const int a = s_cpos[c], b = a + s_csize[c];
      int q = nr - 1;
      while (q >= 0 && s_rs[q] > a) { s_rs[q + 1] = s_rs[q]; s_re[q + 1] = s_re[q]; --q; }
      s_rs[q + 1] = a;
      s_re[q + 1] = b;
      ++nr;
    }
    int m = 0;
    for (int q = 0; q < nr; ++q) {
      if (m > 0 && s_rs[q] < s_re[m - 1]) {
        s_re[m - 1] = max(s_re[m - 1], s_re[q]);
      } else {
        s_rs[m] = s_rs[q];
        s_re[m] = s_re[q];
        ++m;
      }
    }
    nr = m;
    s_rcum[0] = 0;
    for (int q = 0; q < nr; ++q) s_rcum[q + 1] = s_rcum[q] + (s_re[q] - s_rs[q]);
    H.o_range = o;
    if (o + 3 * nr > tab_cap) err = 1;
    for (int q = 0; q < nr && !err; ++q) {
      tab[o + 3 * q] = s_rs[q];
      tab[o + 3 * q + 1] = s_re[q];
      tab[o + 3 * q + 2] = s_rcum[q];
    }
    o += 3 * nr;
    H.nrange = nr;
    H.nomega = s_rcum[nr];
    H.o_zent = o;
    H.nchains = nch;
    H.nslots = ns;
    H.npairs = npairs;
    // chain and slot records (zone ranges filled after the zone pass)
    for (int c = 0; c < nch && !err; ++c) {
      int* cr = tab + H.o_chain + c * kChainInts;
      cr[C_HEAD] = s_head[c];
      cr[C_NSLOT] = s_cslot0[c + 1] - s_cslot0[c];
      cr[C_SLOT0] = s_cslot0[c];
      cr[C_NEST_OFF] = nest_off[c];
      cr[C_NEST_LEN] = nest_len[c];
      cr[C_OUTER] = s_outer[c];
      cr[C_PHASE] = s_chph[c];
      cr[C_BIT0] = s_slotbit[s_cslot0[c]];
      cr[C_PAIR0] = pairbase[s_cslot0[c]];
      int phw[3] = {0, 0, 0};
      for (int s = s_cslot0[c]; s < s_cslot0[c + 1]; ++s) {
        const int r = s - s_cslot0[c];
        phw[r >> 3] |= s_sph[s_slotbit[s]] << (3 * (r & 7));
        // a chain's nodes have at most one child, so its slots are consecutive
        // segment nodes in preorder: consecutive mask bits
        if (s_slotbit[s] != s_slotbit[s_cslot0[c]] + r) err = 1;
      }
      cr[C_PHW0] = phw[0];
      cr[C_PHW1] = phw[1];
      cr[C_PHW2] = phw[2];
      for (int p = 0; p < 3; ++p) { cr[C_ZOFF0 + p] = 0; cr[C_ZCNT0 + p] = 0; }
    }
    for (int s = 0; s < ns && !err; ++s) {
      int* sr = tab + H.o_slot + s * kSlotInts;
      sr[SL_NODE] = s_slotnode[s];
      sr[SL_BIT] = s_slotbit[s];
      sr[SL_PHASE] = s_sph[s_slotbit[s]];
      sr[SL_PAIRBASE] = pairbase[s];
      sr[SL_CHAIN] = s_slotchain[s];
      St.slot_of[s_slotnode[s]] = s;
    }
    for (int q = 0; q < kMaxK * 3; ++q) { s_keycnt[q] = 0; s_keycur[q] = 0; }
    H.valid = err ? 0 : 1;
    s_h = H;
    s_err = err;
  }
  __syncthreads();
  SegHdr H = s_h;
  if (s_err) {
    if (threadIdx.x == 0) {
      H.valid = 0;
      hdrs[g] = H;
      atomicOr(status, kStatusBuild);
    }
    return;
  }
  const int nr = H.nrange, nom = H.nomega;
  const int* rg = tab + H.o_range;
  // zone targets: kept nodes of Omega_g outside the segment; anchor = chain
  // whose bottom slot is the first segment node above the target
  for (int pass = 0; pass < 2; ++pass) {
    for (int q = threadIdx.x; q < nom; q += blockDim.x) {
      int r = 0;
      while (r + 1 < nr && rg[3 * (r + 1) + 2] <= q) ++r;
      const int i = T.pre[rg[3 * r] + (q - rg[3 * r + 2])];
      if (segment[i] == g || !St.kept[i]) continue;
      // anchor: the deepest segment node whose subtree holds i
      const int pi = T.pos[i];
      int best = -1;
      for (int j = 0; j < k; ++j)
        if (s_spos[j] < pi && pi < s_spos[j] + s_ssize[j] && (best < 0 || s_spos[j] > s_spos[best])) best = j;
      const int s = (best >= 0) ? s_jslot[best] : -1;
      if (s < 0) { atomicOr(&s_err, 1); continue; }
      const int c = tab[H.o_slot + s * kSlotInts + SL_CHAIN];
      const int* cr = tab + H.o_chain + c * kChainInts;
      if (s != cr[C_SLOT0] + cr[C_NSLOT] - 1) { atomicOr(&s_err, 1); continue; }  // must be the chain's bottom
      const unsigned ph = T.phase[i];
      for (int p = 0; p < 3; ++p) {
        if (!(ph >> p & 1u)) continue;
        const int key = c * 3 + p;
        if (pass == 0) {
          atomicAdd(&s_keycnt[key], 1);
        } else {
          const int idx = s_keyoff[key] + atomicAdd(&s_keycur[key], 1);
          int* ze = tab + H.o_zent + 3 * idx;
          ze[0] = i;
          ze[1] = p;
          ze[2] = c;
          St.zent_of[i * 3 + p] = idx;
        }
      }
    }
    __syncthreads();
    if (pass == 0 && threadIdx.x == 0) {
      int acc = 0;
      for (int key = 0; key < H.nchains * 3; ++key) {
        s_keyoff[key] = acc;
        int* cr = tab + H.o_chain + (key / 3) * kChainInts;
        cr[C_ZOFF0 + key % 3] = acc;
        cr[C_ZCNT0 + key % 3] = s_keycnt[key];
        acc += s_keycnt[key];
      }
      s_h.nz = acc;
      s_h.total_ints = H.o_zent + 3 * acc;
      if (s_h.total_ints > tab_cap) s_err = 1;
    }
    __syncthreads();
    if (s_err) break;
  }
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

__global__ __launch_bounds__(256) void k_build_values(const SegHdr* __restrict__ hdrs, int g,
                                                      const int* __restrict__ tab, int n,
                                                      const double2* __restrict__ Zroot,
                                                      const double2* __restrict__ Vcur,
                                                      const double2* __restrict__ A, double2* __restrict__ P,
                                                      TargetRec* __restrict__ srec, double2* __restrict__ headV,
                                                      TargetRec* __restrict__ zrec, double* __restrict__ econst) {
  const SegHdr H = hdrs[g];
  if (!H.valid) return;
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
__global__ __launch_bounds__(256) void k_build_members(const SegHdr* __restrict__ hdrs, int g,
                                                       const int* __restrict__ tab, Topo T, State St,
                                                       const double2* __restrict__ Vcur,
                                                       const double* __restrict__ absV, TargetRec* __restrict__ srec,
                                                       TargetRec* __restrict__ zrec, double* __restrict__ econst) {
  const SegHdr H = hdrs[g];
  if (!H.valid) return;
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
