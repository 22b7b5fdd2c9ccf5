// Greedy single-move reduction search (Algorithm 1, Section IV) and the
// evaluation of a fixed reduction over many scenarios (Section VI), on
// gfx950: kernels and the C ABI of include/okr_greedy.h.
//
// Design.  The full network is radial with the slack as source, so with the
// currents fixed its solution is V = V0 - sum_j Zcp(., j) I_j, where Zcp(y, j)
// is the series impedance of the common part of the root paths of y and j,
// i.e. Zroot(lca(y, j)).  Moving the aggregated load current J of super-node
// r to super-node s therefore changes node y's voltage by
//     dV_y = (Zroot(lca(y, r)) - Zroot(lca(y, s))) J,
// which is nonzero exactly on the subtrees of w = lca(r, s)'s children
// towards r and towards s.  Lowest common ancestors are O(1) lookups in a
// sparse table over the Euler tour (built once per topology).  Every
// iteration keeps each cluster's MICE, their total, block maxima over DFS
// positions and the member lists; one block scores one candidate by
// re-scoring only the clusters whose super-node lies in those two subtrees
// and the merged cluster, and one block picks the move, applies it to the
// voltages with the scoring's expression and rebuilds the cluster state.
// A search starts from the exact fixed-current solve (a level-synchronous
// sweep), which also serves the evaluation of a given assignment.

#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/okr_greedy.h"
#include "okr_device.h"
#include "okr_internal.h"

namespace okr {

__global__ void k_branch_z(int, const int*, const uint8_t*, const int*, const int*, const double2*, const double2*,
                           double2*, int*);
__global__ void k_powerflow(int, const int*, const uint8_t*, const int*, const int*, int, const int*, const int*,
                            const double2*, const double2*, double2, double2, double2, double, int, double, double,
                            double2*, double2*, double2*, double*, int*, int*);
__global__ void k_from_vhat(int, int, const uint8_t*, const double2*, const double2*, double, double, double2*,
                            double*, int*);
__global__ void k_zroot(int, const int*, const int*, const int*, int, const double2*, double2*);

struct GState {
  int iter;  // moves applied
  int done;  // no feasible candidate left
  int s, r;  // the move chosen by the last pick
};

struct GStep {  // layout of okr_greedy_step
  int cand, s, r, ambiguous, n_cand, n_feasible;
  double smice, emax;
};

constexpr int kGreedyThreads = 256;
constexpr int kGreedyPickThreads = 1024;
constexpr int kGreedyMaxS = 64;      // scenarios of a search (moved currents staged in LDS)
constexpr int kGreedyMaxN = 12288;   // nodes of a search (member counts in LDS)
constexpr int kSmallCluster = 8;    // clusters up to this size are scored by one lane
constexpr int kGreedyFullSN = 6144;  // S x n up to which every candidate scores every node

// O(1) lowest common ancestors: the Euler tour of the DFS (E = 2n - 1
// entries), every node's first index in it, and a sparse table of the
// shallowest node over power-of-two ranges of the tour (level k at st[k * E]).
struct LcaTab {
  const int* first;
  const int* st;
  const int* depth;
  int E;
  __device__ __forceinline__ int lca(int u, int v) const {
    int a = first[u], b = first[v];
    if (a > b) {
      const int t = a;
      a = b;
      b = t;
    }
    const int k = 31 - __clz(b - a + 1);
    const int x = st[(size_t)k * E + a], y = st[(size_t)k * E + b - (1 << k) + 1];
    return depth[x] <= depth[y] ? x : y;
  }
};

// The child of w whose subtree holds t (t strictly below w): children are
// stored in increasing DFS position.
__device__ __forceinline__ int child_toward(const int* ch_off, const int* ch, const int* pos, int w, int t) {
  int lo = ch_off[w], hi = ch_off[w + 1] - 1;
  const int q = pos[t];
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (pos[ch[mid]] <= q) lo = mid;
    else hi = mid - 1;
  }
  return ch[lo];
}

// Voltage change at node y of moving load current J (one scenario, 3 phases)
// from r to s: (Zroot(lca(y, r)) - Zroot(lca(y, s))) J; `moved` is false when
// both lca are the same node (no change).
struct MoveDelta {
  double2 dZ[9];
  bool moved;
  __device__ __forceinline__ void at(const LcaTab& T, const double2* Zr, int y, int r, int s) {
    between(Zr, T.lca(y, r), T.lca(y, s));
  }
  // a = lca(y, r), b = lca(y, s), when already known
  __device__ __forceinline__ void between(const double2* Zr, int a, int b) {
    moved = a != b;
    if (moved) {
      const double2* Za = Zr + (size_t)a * 9;
      const double2* Zb = Zr + (size_t)b * 9;
#pragma unroll
      for (int q = 0; q < 9; ++q) dZ[q] = csub(Za[q], Zb[q]);
    }
  }
  __device__ __forceinline__ double2 dv(int p, const double2* J) const {
    return cadd(cadd(cmul(dZ[p * 3], J[0]), cmul(dZ[p * 3 + 1], J[1])), cmul(dZ[p * 3 + 2], J[2]));
  }
};

// Per-iteration cluster state (device): MICE of every cluster per scenario
// (0 for nodes that are not super-nodes), their sum, the largest MICE over
// scenarios by DFS position and its maxima over blocks of 64 positions, and
// every cluster's members (CSR, any order: only maxima are taken over them).
// The member counts are built in LDS: a search takes at most kGreedyMaxN
// nodes.
struct Clusters {
  double* mice;   // [S][n]
  double* arr;    // [n], by DFS position
  double* bmax;   // [ceil(n / 64)]
  int* moff;      // [n + 1]
  int* mem;       // [n]
  double* tot;    // [1]
};

// Largest error over scenarios' phases of member x against magnitudes mag
// (3 per scenario): e_l = max_p ||V^_x| - mag_p|.
__device__ __forceinline__ double member_err(const double* absV, int n, int x, int l, unsigned ph,
                                             const double* mag) {
  const size_t xb = ((size_t)l * n + x) * 3;
  double e = 0.0;
#pragma unroll
  for (int p = 0; p < 3; ++p)
    if (ph >> p & 1u) e = fmax(e, fabs(absV[xb + p] - mag[p]));
  return e;
}

// Builds the cluster state of the current assignment and voltages (one
// block; called with every thread).  Member counts and fill pointers live in
// LDS (lcnt, n ints); every cluster's MICE is a wave-wide maximum over its
// members (one wave per super-node, 64 members at a time), so large clusters
// cost neither serial walks nor same-address atomics.
__device__ void cluster_prep(int n, int S, const uint8_t* phase, const int* pre, const int* sup, const double2* V,
                             const double* absV, const Clusters& C, int* lcnt, int* shi, double* shd) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int y = threadIdx.x; y < n; y += blockDim.x) lcnt[y] = 0;
  __syncthreads();
  for (int x = threadIdx.x; x < n; x += blockDim.x) atomicAdd(&lcnt[sup[x]], 1);
  __syncthreads();
  // member offsets: each thread scans a contiguous chunk, the chunk sums are
  // scanned across the block
  const int chunk = (n + blockDim.x - 1) / blockDim.x, c0 = threadIdx.x * chunk, c1 = min(n, c0 + chunk);
  int loc = 0;
  for (int y = c0; y < c1; ++y) loc += lcnt[y];
  const int base = block_exclusive_scan(loc, shi);
  for (int y = c0, acc = base; y < c1; ++y) {
    const int c = lcnt[y];
    C.moff[y] = acc;
    lcnt[y] = acc;  // fill pointer
    acc += c;
  }
  if (threadIdx.x == blockDim.x - 1) C.moff[n] = base + loc;
  __syncthreads();
  for (int x = threadIdx.x; x < n; x += blockDim.x) C.mem[atomicAdd(&lcnt[sup[x]], 1)] = x;
  __syncthreads();
  // MICE of every cluster (0 for nodes that are not super-nodes): a lane
  // takes a cluster of at most kSmallCluster members, a wave the larger ones
  for (int y0 = wv * 64; y0 < n; y0 += nw * 64) {
    const int y = y0 + lane;
    const bool is = y < n && sup[y] == y;
    const int m0 = is ? C.moff[y] : 0, m1 = is ? C.moff[y + 1] : 0;
    const bool big = is && m1 - m0 > kSmallCluster;
    if (y < n && !big)
      for (int l = 0; l < S; l += 2) {  // two scenarios per pass over the members
        const int l1 = l + 1 < S ? l + 1 : l;
        double mx0 = 0.0, mx1 = 0.0;
        if (is) {
          double mag0[3], mag1[3];
#pragma unroll
          for (int p = 0; p < 3; ++p) {
            mag0[p] = sqrt(cabs2(V[((size_t)l * n + y) * 3 + p]));
            mag1[p] = sqrt(cabs2(V[((size_t)l1 * n + y) * 3 + p]));
          }
          for (int k = m0; k < m1; ++k) {
            const int m = C.mem[k];
            const unsigned ph = phase[m];
            mx0 = fmax(mx0, member_err(absV, n, m, l, ph, mag0));
            mx1 = fmax(mx1, member_err(absV, n, m, l1, ph, mag1));
          }
        }
        C.mice[(size_t)l * n + y] = mx0;
        if (l1 != l) C.mice[(size_t)l1 * n + y] = mx1;
      }
    unsigned long long mask = __ballot(big);
    while (mask) {
      const int bit = __ffsll((long long)mask) - 1;
      mask &= mask - 1;
      const int u = y0 + bit, k0 = __shfl(m0, bit, 64), k1 = __shfl(m1, bit, 64);
      for (int l = 0; l < S; l += 2) {  // two scenarios per pass over the members
        const int l1 = l + 1 < S ? l + 1 : l;
        double mag0[3], mag1[3];
#pragma unroll
        for (int p = 0; p < 3; ++p) {
          mag0[p] = sqrt(cabs2(V[((size_t)l * n + u) * 3 + p]));
          mag1[p] = sqrt(cabs2(V[((size_t)l1 * n + u) * 3 + p]));
        }
        double mx0 = 0.0, mx1 = 0.0;
        for (int k = k0 + lane; k < k1; k += 64) {
          const int m = C.mem[k];
          const unsigned ph = phase[m];
          mx0 = fmax(mx0, member_err(absV, n, m, l, ph, mag0));
          mx1 = fmax(mx1, member_err(absV, n, m, l1, ph, mag1));
        }
        for (int o = 32; o > 0; o >>= 1) {
          mx0 = fmax(mx0, __shfl_xor(mx0, o, 64));
          mx1 = fmax(mx1, __shfl_xor(mx1, o, 64));
        }
        if (lane == 0) {
          C.mice[(size_t)l * n + u] = mx0;
          if (l1 != l) C.mice[(size_t)l1 * n + u] = mx1;
        }
      }
    }
  }
  __syncthreads();
  for (int q = threadIdx.x; q < n; q += blockDim.x) {
    double m = 0.0;
    for (int l = 0; l < S; ++l) m = fmax(m, C.mice[(size_t)l * n + pre[q]]);
    C.arr[q] = m;
  }
  double t = 0.0;
  for (int q = threadIdx.x; q < S * n; q += blockDim.x) t += C.mice[q];
  t = block_reduce(t, [](double a, double b) { return a + b; }, shd);
  __syncthreads();
  // block maxima: a wave per block of 64 positions, a position per lane
  for (int k = wv; k < (n + 63) / 64; k += nw) {
    const int q = k * 64 + lane;
    double m = q < n ? C.arr[q] : 0.0;
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
    if (lane == 0) C.bmax[k] = m;
  }
  if (threadIdx.x == 0) *C.tot = t;
  __syncthreads();
}

// Fixed-current solve of one scenario on the radial network: branch currents
// by subtree sums of the load currents I (deepest level first), then
// V(x) = V(parent) - z_x Ib(x) level by level from the slack (V0).  One block.
__device__ void sweep_block(int n, const int* parent, const uint8_t* phase, const int* lvl_off,
                            const int* lvl_nodes, int nlev, const int* ch_off, const int* ch, const double2* z,
                            const double2 (&v0)[3], const double2* I, double2* Ib, double2* V) {
  for (int q = threadIdx.x; q < n * 3; q += blockDim.x) Ib[q] = I[q];
  __syncthreads();
  for (int lev = nlev - 2; lev >= 0; --lev) {
    for (int q = lvl_off[lev] + threadIdx.x; q < lvl_off[lev + 1]; q += blockDim.x) {
      const int i = lvl_nodes[q];
      double2 s0 = Ib[i * 3], s1 = Ib[i * 3 + 1], s2 = Ib[i * 3 + 2];
      for (int e = ch_off[i]; e < ch_off[i + 1]; ++e) {
        const int c = ch[e];
        s0 = cadd(s0, Ib[c * 3]);
        s1 = cadd(s1, Ib[c * 3 + 1]);
        s2 = cadd(s2, Ib[c * 3 + 2]);
      }
      Ib[i * 3] = s0;
      Ib[i * 3 + 1] = s1;
      Ib[i * 3 + 2] = s2;
    }
    __syncthreads();
  }
  if (threadIdx.x < 3) V[threadIdx.x] = (phase[0] >> threadIdx.x & 1u) ? v0[threadIdx.x] : make_double2(0.0, 0.0);
  __syncthreads();
  for (int lev = 1; lev < nlev; ++lev) {
    for (int q = lvl_off[lev] + threadIdx.x; q < lvl_off[lev + 1]; q += blockDim.x) {
      const int i = lvl_nodes[q], pv = parent[i];
      const double2* zi = z + (size_t)i * 9;
      const double2 j0 = Ib[i * 3], j1 = Ib[i * 3 + 1], j2 = Ib[i * 3 + 2];
      for (int p = 0; p < 3; ++p) {
        double2 v = make_double2(0.0, 0.0);
        if (phase[i] >> p & 1u) {
          const double2 d = cadd(cadd(cmul(zi[p * 3], j0), cmul(zi[p * 3 + 1], j1)), cmul(zi[p * 3 + 2], j2));
          v = csub(V[pv * 3 + p], d);
        }
        V[i * 3 + p] = v;
      }
    }
    __syncthreads();
  }
}

// Start of the search: every node its own super-node, I = the load currents.
__global__ void k_greedy_init(int n, int S, const double2* __restrict__ A, double2* __restrict__ Iagg,
                              int* __restrict__ sup, GState* __restrict__ gs) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < (size_t)S * n * 3) Iagg[t] = A[t];
  if (t < (size_t)n) sup[t] = (int)t;
  if (t == 0) {
    gs->iter = 0;
    gs->done = 0;
    gs->s = gs->r = -1;
  }
}

// Fixed-current solve of every scenario (one block each) from Iagg.
__global__ __launch_bounds__(kGreedyThreads) void k_greedy_sweep(
    int n, const int* __restrict__ parent, const uint8_t* __restrict__ phase, const int* __restrict__ lvl_off,
    const int* __restrict__ lvl_nodes, int nlev, const int* __restrict__ ch_off, const int* __restrict__ ch,
    const double2* __restrict__ z, double2 v0a, double2 v0b, double2 v0c, const double2* __restrict__ Iagg,
    double2* __restrict__ Ib, double2* __restrict__ V) {
  const size_t base = (size_t)blockIdx.x * n * 3;
  const double2 v0[3] = {v0a, v0b, v0c};
  sweep_block(n, parent, phase, lvl_off, lvl_nodes, nlev, ch_off, ch, z, v0, Iagg + base, Ib + base, V + base);
}

// Cluster state of the search's starting point (one block).
__global__ __launch_bounds__(kGreedyPickThreads) void k_greedy_prep(int n, int S, const uint8_t* __restrict__ phase,
                                                                    const int* __restrict__ pre,
                                                                    const int* __restrict__ sup,
                                                                    const double2* __restrict__ V,
                                                                    const double* __restrict__ absV, Clusters C) {
  extern __shared__ __align__(16) unsigned char g_lds[];
  __shared__ int shi[kGreedyPickThreads];
  __shared__ double shd[kGreedyPickThreads / 64];
  cluster_prep(n, S, phase, pre, sup, V, absV, C, (int*)g_lds, shi, shd);
}

// Score of one candidate per block (grid: 2n blocks, id = blockIdx.x):
// SMICE (+inf when infeasible) and the largest error (-1 when the id is not a
// candidate in this state).  Only the clusters the move can change are
// scored again: with w = lca(r, s), voltages change exactly on the subtrees
// of w's children towards r and towards s (DFS intervals I_r, I_s), so the
// clusters whose super-node lies there (which, other than r's and s's, lie
// wholly inside them) and the merged cluster s + r; every other cluster keeps
// its MICE.  SMICE = (total - old MICE of the changed clusters) + their new
// MICE; the largest error is the maximum of the new MICE and of the other
// clusters' (block maxima over DFS positions outside the intervals and w).
__global__ __launch_bounds__(kGreedyThreads) void k_greedy_score(
    int n, int S, const int* __restrict__ parent, const uint8_t* __restrict__ phase, const int* __restrict__ pos,
    const int* __restrict__ size, const int* __restrict__ pre, const int* __restrict__ ch_off,
    const int* __restrict__ ch, const int* __restrict__ sup, LcaTab T, const double2* __restrict__ Zr,
    const double2* __restrict__ Iagg, const double2* __restrict__ Vcur, const double* __restrict__ absV,
    double e_bar, const GState* __restrict__ gs, Clusters C, double* __restrict__ sm, double* __restrict__ em) {
  __shared__ double2 J[kGreedyMaxS * 3];
  __shared__ double magS[kGreedyMaxS * 3];
  __shared__ unsigned long long newS[kGreedyMaxS];
  __shared__ double red[kGreedyThreads / 64];
  if (gs->done) return;
  const int cand = blockIdx.x, x = cand >> 1, dir = cand & 1, tid = threadIdx.x;
  int r = -1, s = -1;
  if (x > 0) {
    const int a = sup[x], b = sup[parent[x]];
    if (a != b) {
      r = dir ? b : a;
      s = dir ? a : b;
      if (r == 0 || (phase[r] & ~phase[s])) r = -1;
    }
  }
  if (r < 0) {  // not a candidate (uniform over the block)
    if (tid == 0) {
      sm[cand] = INFINITY;
      em[cand] = -1.0;
    }
    return;
  }
  const int w = T.lca(r, s);
  int a1 = 0, b1 = 0, a2 = 0, b2 = 0;  // I_r = [a1, b1), I_s = [a2, b2)
  if (r != w) {
    const int c = child_toward(ch_off, ch, pos, w, r);
    a1 = pos[c];
    b1 = a1 + size[c];
  }
  if (s != w) {
    const int c = child_toward(ch_off, ch, pos, w, s);
    a2 = pos[c];
    b2 = a2 + size[c];
  }
  const int qw = pos[w];
  MoveDelta msd;
  msd.between(Zr, w, s);  // lca(s, r) = w, lca(s, s) = s
  for (int q = tid; q < S * 3; q += kGreedyThreads) {
    J[q] = Iagg[((size_t)(q / 3) * n + r) * 3 + q % 3];
  }
  for (int l = tid; l < S; l += kGreedyThreads) newS[l] = 0ull;
  __syncthreads();
  for (int l = tid; l < S; l += kGreedyThreads) {
#pragma unroll
    for (int p = 0; p < 3; ++p) {  // unrolled: msd.dZ stays in registers
      double2 v = Vcur[((size_t)l * n + s) * 3 + p];
      if (msd.moved) v = cadd(v, msd.dv(p, J + l * 3));
      magS[l * 3 + p] = sqrt(cabs2(v));
    }
  }
  __syncthreads();
  double olds = 0.0, news = 0.0, emx = 0.0;
  // clusters whose super-node lies in I_r or I_s (other than r and s), the
  // two intervals walked as one range: each wave takes 64 positions at a
  // time; a lane scores the cluster of its position when it has at most
  // kSmallCluster members, and the wave scores the larger ones together (64
  // members at a time)
  {
    const int lane = tid & 63, wv = tid >> 6, L1 = b1 - a1, L = L1 + (b2 - a2);
    for (int c0 = wv * 64; c0 < L; c0 += kGreedyThreads) {
      const int qi = c0 + lane;  // index into I_r then I_s
      int u = -1, m0 = 0, m1 = 0;
      bool is = false;
      if (qi < L) {
        u = pre[qi < L1 ? a1 + qi : a2 + (qi - L1)];
        is = sup[u] == u && u != r && u != s;
        if (is) {
          m0 = C.moff[u];
          m1 = C.moff[u + 1];
        }
      }
      const bool big = is && m1 - m0 > kSmallCluster;
      // in I_r, lca(u, s) = w; in I_s, lca(u, r) = w: one lca to look up
      const bool inR = qi < L1;
      if (is && !big) {
        MoveDelta md;
        const int a = T.lca(u, inR ? r : s);
        md.between(Zr, inR ? a : w, inR ? w : a);
        for (int l = 0; l < S; l += 2) {  // two scenarios per pass over the members
          const int l1 = l + 1 < S ? l + 1 : l;
          double mag0[3], mag1[3];
#pragma unroll
          for (int p = 0; p < 3; ++p) {
            double2 v0 = Vcur[((size_t)l * n + u) * 3 + p], v1 = Vcur[((size_t)l1 * n + u) * 3 + p];
            if (md.moved) {
              v0 = cadd(v0, md.dv(p, J + l * 3));
              v1 = cadd(v1, md.dv(p, J + l1 * 3));
            }
            mag0[p] = sqrt(cabs2(v0));
            mag1[p] = sqrt(cabs2(v1));
          }
          double mx0 = 0.0, mx1 = 0.0;
          for (int k = m0; k < m1; ++k) {
            const int m = C.mem[k];
            const unsigned ph = phase[m];
            mx0 = fmax(mx0, member_err(absV, n, m, l, ph, mag0));
            mx1 = fmax(mx1, member_err(absV, n, m, l1, ph, mag1));
          }
          olds += C.mice[(size_t)l * n + u];
          news += mx0;
          emx = fmax(emx, mx0);
          if (l1 != l) {
            olds += C.mice[(size_t)l1 * n + u];
            news += mx1;
            emx = fmax(emx, mx1);
          }
        }
      }
      unsigned long long mask = __ballot(big);
      while (mask) {
        const int bit = __ffsll((long long)mask) - 1;
        mask &= mask - 1;
        const int uu = __shfl(u, bit, 64), k0 = __shfl(m0, bit, 64), k1 = __shfl(m1, bit, 64);
        const bool uinR = __shfl(qi, bit, 64) < L1;
        MoveDelta md;
        const int a = T.lca(uu, uinR ? r : s);
        md.between(Zr, uinR ? a : w, uinR ? w : a);
        for (int l = 0; l < S; l += 2) {  // two scenarios per pass over the members
          const int l1 = l + 1 < S ? l + 1 : l;
          double mag0[3], mag1[3];
#pragma unroll
          for (int p = 0; p < 3; ++p) {
            double2 v0 = Vcur[((size_t)l * n + uu) * 3 + p], v1 = Vcur[((size_t)l1 * n + uu) * 3 + p];
            if (md.moved) {
              v0 = cadd(v0, md.dv(p, J + l * 3));
              v1 = cadd(v1, md.dv(p, J + l1 * 3));
            }
            mag0[p] = sqrt(cabs2(v0));
            mag1[p] = sqrt(cabs2(v1));
          }
          double mx0 = 0.0, mx1 = 0.0;
          for (int k = k0 + lane; k < k1; k += 64) {
            const int m = C.mem[k];
            const unsigned ph = phase[m];
            mx0 = fmax(mx0, member_err(absV, n, m, l, ph, mag0));
            mx1 = fmax(mx1, member_err(absV, n, m, l1, ph, mag1));
          }
          for (int o = 32; o > 0; o >>= 1) {
            mx0 = fmax(mx0, __shfl_xor(mx0, o, 64));
            mx1 = fmax(mx1, __shfl_xor(mx1, o, 64));
          }
          if (lane == 0) {
            olds += C.mice[(size_t)l * n + uu];
            news += mx0;
            emx = fmax(emx, mx0);
            if (l1 != l) {
              olds += C.mice[(size_t)l1 * n + uu];
              news += mx1;
              emx = fmax(emx, mx1);
            }
          }
        }
      }
    }
  }
  // the merged cluster: r's members, and s's own when s's voltage moves
  for (int pass = 0; pass < 2; ++pass) {
    const int y = pass ? s : r;
    if (pass && !msd.moved) break;
    for (int k = C.moff[y] + tid; k < C.moff[y + 1]; k += kGreedyThreads) {
      const int m = C.mem[k];
      const unsigned ph = phase[m];
      for (int l = 0; l < S; ++l)
        atomicMax(&newS[l], (unsigned long long)__double_as_longlong(member_err(absV, n, m, l, ph, magS + l * 3)));
    }
  }
  // every other cluster keeps its MICE: largest over positions outside
  // I_r, I_s and w's
  double umax = 0.0;
  const int nb = (n + 63) / 64;
  for (int k = tid; k < nb; k += kGreedyThreads) {
    const int lo = k * 64, hi = min(n, lo + 64);
    const bool touch = (lo <= qw && qw < hi) || (lo < b1 && a1 < hi) || (lo < b2 && a2 < hi);
    if (!touch) umax = fmax(umax, C.bmax[k]);
  }
  // a touched block holds an end of I_r or I_s or w's position, or lies
  // wholly inside I_r or I_s (nothing to add): the five blocks that hold
  // those positions are read by one wave each, a position per lane (a block
  // named twice gives the same maximum)
  for (int j = tid >> 6; j < 5; j += kGreedyThreads / 64) {
    const int k = j == 0   ? qw >> 6
                  : j == 1 ? (a1 < b1 ? a1 >> 6 : -1)
                  : j == 2 ? (a1 < b1 ? (b1 - 1) >> 6 : -1)
                  : j == 3 ? (a2 < b2 ? a2 >> 6 : -1)
                           : (a2 < b2 ? (b2 - 1) >> 6 : -1);
    const int q = k * 64 + (tid & 63);
    if (k >= 0 && q < n && q != qw && !(a1 <= q && q < b1) && !(a2 <= q && q < b2)) umax = fmax(umax, C.arr[q]);
  }
  __syncthreads();
  olds = block_reduce(olds, [](double a, double b) { return a + b; }, red);
  news = block_reduce(news, [](double a, double b) { return a + b; }, red);
  emx = block_reduce(fmax(emx, umax), [](double a, double b) { return fmax(a, b); }, red);
  if (tid == 0) {
    for (int l = 0; l < S; ++l) {
      double v = __longlong_as_double((long long)newS[l]);
      if (!msd.moved) v = fmax(v, C.mice[(size_t)l * n + s]);
      olds += C.mice[(size_t)l * n + s] + C.mice[(size_t)l * n + r];
      news += v;
      emx = fmax(emx, v);
    }
    em[cand] = emx;
    sm[cand] = emx <= e_bar ? (*C.tot - olds) + news : INFINITY;
  }
}

// The iteration's move (one block of 1024): the smallest SMICE among
// feasible candidates, ties within tie_tol to the lowest id; the step is
// recorded, r's current joins s's, r's cluster is reassigned, every node's
// voltage takes the move's change (the expression the scoring evaluated),
// and the cluster state is rebuilt.  With no feasible candidate the search
// is marked done.
__global__ __launch_bounds__(kGreedyPickThreads) void k_greedy_pick_apply(
    int n, int S, const int* __restrict__ parent, const uint8_t* __restrict__ phase, const int* __restrict__ pre,
    const int* __restrict__ pos, const int* __restrict__ size, const int* __restrict__ ch_off,
    const int* __restrict__ ch, LcaTab T, const double2* __restrict__ Zr, const double* __restrict__ absV, const double* __restrict__ sm,
    const double* __restrict__ em, double e_bar, double tie, double amb, GState* __restrict__ gs,
    GStep* __restrict__ steps, int* __restrict__ sup, double2* __restrict__ Iagg, double2* __restrict__ V,
    Clusters C) {
  extern __shared__ __align__(16) unsigned char g_lds[];
  __shared__ double shd[kGreedyPickThreads / 64];
  __shared__ int shi[kGreedyPickThreads];
  __shared__ double2 J[kGreedyMaxS * 3];
  if (gs->done) return;
  const int tid = threadIdx.x, ncand = 2 * n;
  double mn = INFINITY;
  int nact = 0, nfeas = 0;
  for (int c = tid; c < ncand; c += kGreedyPickThreads) {
    mn = fmin(mn, sm[c]);
    nact += em[c] >= 0.0;
    nfeas += sm[c] < INFINITY;
  }
  mn = block_reduce(mn, [](double a, double b) { return fmin(a, b); }, shd);
  nact = block_reduce(nact, [](int a, int b) { return a + b; }, shi);
  nfeas = block_reduce(nfeas, [](int a, int b) { return a + b; }, shi);
  if (!(mn < INFINITY)) {
    if (tid == 0) gs->done = 1;
    return;
  }
  const double thr = mn + tie;
  int win = 0x7fffffff, fl = 0;
  for (int c = tid; c < ncand; c += kGreedyPickThreads) {
    const double v = sm[c];
    if (v <= thr) win = min(win, c);
    if (v < INFINITY && fabs(v - thr) <= amb) fl = 1;
    if (em[c] >= 0.0 && fabs(em[c] - e_bar) <= amb) fl = 1;
  }
  win = block_reduce(win, [](int a, int b) { return min(a, b); }, shi);
  fl = block_reduce(fl, [](int a, int b) { return max(a, b); }, shi);
  const int wx = win >> 1, wa = sup[wx], wb = sup[parent[wx]];
  const int r = (win & 1) ? wb : wa, s = (win & 1) ? wa : wb;
  for (int q = tid; q < S * 3; q += kGreedyPickThreads) J[q] = Iagg[((size_t)(q / 3) * n + r) * 3 + q % 3];
  __syncthreads();  // sup and Iagg read by every thread before they change
  if (tid == 0) {
    GStep st;
    st.cand = win;
    st.s = s;
    st.r = r;
    st.ambiguous = fl;
    st.n_cand = nact;
    st.n_feasible = nfeas;
    st.smice = sm[win];
    st.emax = em[win];
    steps[gs->iter] = st;
    gs->s = s;
    gs->r = r;
    gs->iter += 1;
  }
  for (int q = tid; q < S * 3; q += kGreedyPickThreads) {
    const size_t lr = ((size_t)(q / 3) * n + r) * 3 + q % 3, ls = ((size_t)(q / 3) * n + s) * 3 + q % 3;
    Iagg[ls] = cadd(Iagg[ls], J[q]);
    Iagg[lr] = make_double2(0.0, 0.0);
  }
  for (int u = tid; u < n; u += kGreedyPickThreads)
    if (sup[u] == r) sup[u] = s;
  // only the subtrees of w = lca(r, s)'s children towards r and s (DFS
  // intervals I_r, I_s) change; in I_r, lca(x, s) = w, in I_s lca(x, r) = w
  const int w = T.lca(r, s);
  int a1 = 0, b1 = 0, a2 = 0, b2 = 0;
  if (r != w) {
    const int c = child_toward(ch_off, ch, pos, w, r);
    a1 = pos[c];
    b1 = a1 + size[c];
  }
  if (s != w) {
    const int c = child_toward(ch_off, ch, pos, w, s);
    a2 = pos[c];
    b2 = a2 + size[c];
  }
  for (int xn = tid; xn < n; xn += kGreedyPickThreads) {
    const int q = pos[xn];
    const bool inR = a1 <= q && q < b1;
    if (!inR && !(a2 <= q && q < b2)) continue;
    MoveDelta md;
    const int a = T.lca(xn, inR ? r : s);
    md.between(Zr, inR ? a : w, inR ? w : a);
    for (int l = 0; l < S; ++l) {
      const size_t vb = ((size_t)l * n + xn) * 3;
#pragma unroll
      for (int p = 0; p < 3; ++p) V[vb + p] = cadd(V[vb + p], md.dv(p, J + l * 3));
    }
  }
  __syncthreads();
  cluster_prep(n, S, phase, pre, sup, V, absV, C, (int*)g_lds, shi, shd);
}

// ---- full-scoring form --------------------------------------------------

// Every node's largest error per scenario against its super-node's voltage
// in the current state (e0[l][x]); the full-form scoring reads it for nodes
// whose super-node's voltage a move leaves unchanged.
__device__ __forceinline__ void node_errors(int n, int S, const uint8_t* phase, const int* sup, const double2* V,
                                            const double* absV, double* e0, int t0, int dt) {
  for (int t = t0; t < n * S; t += dt) {
    const int x = t % n, l = t / n;
    const unsigned ph = phase[x];
    const size_t vb = ((size_t)l * n + sup[x]) * 3, xb = ((size_t)l * n + x) * 3;
    double ex = 0.0;
#pragma unroll
    for (int p = 0; p < 3; ++p)
      if (ph >> p & 1u) ex = fmax(ex, fabs(absV[xb + p] - sqrt(cabs2(V[vb + p]))));
    e0[t] = ex;
  }
}

__global__ __launch_bounds__(kGreedyThreads) void k_greedy_e0(int n, int S, const uint8_t* __restrict__ phase,
                                                               const int* __restrict__ sup,
                                                               const double2* __restrict__ V,
                                                               const double* __restrict__ absV,
                                                               double* __restrict__ e0) {
  node_errors(n, S, phase, sup, V, absV, e0, blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x);
}

struct PathRec {
  int node, lo, hi;  // an ancestor and the DFS position range of its subtree
};

// Depth of lca(y, t) where path[d] is t's ancestor at depth d (d <= dmax) and
// q is y's DFS position: the deepest d whose subtree range holds q.
__device__ __forceinline__ int lca_depth(const PathRec* path, int dmax, int q) {
  int lo = 0, hi = dmax;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (path[mid].lo <= q && q < path[mid].hi) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Root paths of r and s in LDS: pr[d] / ps[d] = the ancestor at depth d and
// its DFS position range (every depth up to the node's own has one).
__device__ __forceinline__ void load_paths(int n, const int* pos, const int* size, const int* depth, int r, int s,
                                           PathRec* pr, PathRec* ps) {
  const int qr = pos[r], qs = pos[s];
  for (int u = threadIdx.x; u < n; u += blockDim.x) {
    const int lo = pos[u], hi = lo + size[u];
    if (lo <= qr && qr < hi) pr[depth[u]] = PathRec{u, lo, hi};
    if (lo <= qs && qs < hi) ps[depth[u]] = PathRec{u, lo, hi};
  }
}

// DFS intervals of the subtrees of w = lca(r, s)'s children towards r and
// towards s (empty when r or s is w itself), from the staged root paths:
// only nodes in them can change voltage when r's current moves to s.
struct MoveIntervals {
  int a1, b1, a2, b2;
  __device__ __forceinline__ void from(const PathRec* pr, int dr, const PathRec* ps, int ds, int qs) {
    const int dw = lca_depth(pr, min(dr, ds), qs);
    a1 = b1 = a2 = b2 = 0;
    if (dr > dw) {
      a1 = pr[dw + 1].lo;
      b1 = pr[dw + 1].hi;
    }
    if (ds > dw) {
      a2 = ps[dw + 1].lo;
      b2 = ps[dw + 1].hi;
    }
  }
  __device__ __forceinline__ bool holds(int q) const { return (a1 <= q && q < b1) || (a2 <= q && q < b2); }
};

// MoveDelta with the lowest common ancestors found in the root paths of r
// and s staged in LDS (binary search by DFS position; the full-scoring form).
struct PathDelta {
  double2 dZ[9];
  bool moved;
  __device__ __forceinline__ void at(const PathRec* pr, int dr, const PathRec* ps, int ds, const double2* Zr, int qy,
                                     int dy) {
    const int da = lca_depth(pr, min(dy, dr), qy), db = lca_depth(ps, min(dy, ds), qy);
    moved = da != db;
    if (moved) {
      const double2* Za = Zr + (size_t)pr[da].node * 9;
      const double2* Zb = Zr + (size_t)ps[db].node * 9;
#pragma unroll
      for (int q = 0; q < 9; ++q) dZ[q] = csub(Za[q], Zb[q]);
    }
  }
  __device__ __forceinline__ double2 dv(int p, const double2* J) const {
    return cadd(cadd(cmul(dZ[p * 3], J[0]), cmul(dZ[p * 3 + 1], J[1])), cmul(dZ[p * 3 + 2], J[2]));
  }
};

// Full-scoring form (every node of every candidate; for S * n up to
// kGreedyFullSN): one candidate per block (grid: 2n blocks, id =
// blockIdx.x), SMICE (+inf when infeasible) and the largest error (-1 when
// the id is not a candidate).  Dynamic LDS: S * n cluster maxima (uint64 bit
// patterns), then the root paths of r and s.
__global__ __launch_bounds__(kGreedyThreads) void k_greedy_score_full(
    int n, int S, const int* __restrict__ parent, const uint8_t* __restrict__ phase, const int* __restrict__ pos,
    const int* __restrict__ size, const int* __restrict__ depth, const int* __restrict__ sup,
    const double2* __restrict__ Zr, const double2* __restrict__ Iagg, const double2* __restrict__ Vcur,
    const double* __restrict__ absV, const double* __restrict__ e0, double e_bar, const GState* __restrict__ gs,
    double* __restrict__ sm, double* __restrict__ em) {
  extern __shared__ __align__(16) unsigned char g_lds[];
  __shared__ double2 J[kGreedyMaxS * 3];
  __shared__ double red[kGreedyThreads / 64];
  if (gs->done) return;
  const int cand = blockIdx.x, x = cand >> 1, dir = cand & 1, tid = threadIdx.x;
  int r = -1, s = -1;
  if (x > 0) {
    const int a = sup[x], b = sup[parent[x]];
    if (a != b) {
      r = dir ? b : a;
      s = dir ? a : b;
      if (r == 0 || (phase[r] & ~phase[s])) r = -1;
    }
  }
  if (r < 0) {  // not a candidate (uniform over the block)
    if (tid == 0) {
      sm[cand] = INFINITY;
      em[cand] = -1.0;
    }
    return;
  }
  unsigned long long* mice = (unsigned long long*)g_lds;
  PathRec* pr = (PathRec*)(mice + (size_t)S * n);
  const int dr = depth[r], ds = depth[s];
  PathRec* ps = pr + dr + 1;
  for (int q = tid; q < S * n; q += kGreedyThreads) mice[q] = 0ull;
  load_paths(n, pos, size, depth, r, s, pr, ps);
  for (int q = tid; q < S * 3; q += kGreedyThreads) J[q] = Iagg[((size_t)(q / 3) * n + r) * 3 + q % 3];
  __syncthreads();
  MoveIntervals mi;
  mi.from(pr, dr, ps, ds, pos[s]);
  double emax = 0.0;
  for (int xn = tid; xn < n; xn += kGreedyThreads) {
    const int y0 = sup[xn], y = y0 == r ? s : y0;
    const int qy = pos[y];
    if (y0 != r && !mi.holds(qy)) {  // same super-node, same voltage: the stored errors
      for (int l = 0; l < S; ++l) {
        const double ex = e0[(size_t)l * n + xn];
        atomicMax(&mice[(size_t)l * n + y], (unsigned long long)__double_as_longlong(ex));
        emax = fmax(emax, ex);
      }
      continue;
    }
    PathDelta md;
    if (mi.holds(qy)) md.at(pr, dr, ps, ds, Zr, qy, depth[y]);
    else md.moved = false;
    const unsigned ph = phase[xn];
    for (int l = 0; l < S; ++l) {
      const size_t vb = ((size_t)l * n + y) * 3, xb = ((size_t)l * n + xn) * 3;
      double ex = 0.0;
#pragma unroll
      for (int p = 0; p < 3; ++p) {
        if (!(ph >> p & 1u)) continue;
        double2 v = Vcur[vb + p];
        if (md.moved) v = cadd(v, md.dv(p, J + l * 3));
        ex = fmax(ex, fabs(absV[xb + p] - sqrt(cabs2(v))));
      }
      atomicMax(&mice[(size_t)l * n + y], (unsigned long long)__double_as_longlong(ex));
      emax = fmax(emax, ex);
    }
  }
  __syncthreads();
  // SMICE: every thread sums its strided share in order, then a fixed tree
  double acc = 0.0;
  for (int q = tid; q < S * n; q += kGreedyThreads) acc += __longlong_as_double((long long)mice[q]);
  for (int o = 32; o > 0; o >>= 1) {
    acc += __shfl_xor(acc, o, 64);
    emax = fmax(emax, __shfl_xor(emax, o, 64));
  }
  if ((tid & 63) == 0) red[tid >> 6] = acc;
  __syncthreads();
  const double tot = (red[0] + red[1]) + (red[2] + red[3]);
  __syncthreads();
  if ((tid & 63) == 0) red[tid >> 6] = emax;
  __syncthreads();
  if (tid == 0) {
    const double e = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    em[cand] = e;
    sm[cand] = e <= e_bar ? tot : INFINITY;
  }
}

// The move of the full-scoring form (one block of 1024): as
// k_greedy_pick_apply without the cluster state.  Dynamic LDS: the two root
// paths.
__global__ __launch_bounds__(kGreedyPickThreads) void k_greedy_pick_apply_full(
    int n, int S, const int* __restrict__ parent, const int* __restrict__ pos, const int* __restrict__ size,
    const int* __restrict__ depth, const double2* __restrict__ Zr, const double* __restrict__ sm,
    const double* __restrict__ em, double e_bar, double tie, double amb, GState* __restrict__ gs,
    GStep* __restrict__ steps, int* __restrict__ sup, double2* __restrict__ Iagg, double2* __restrict__ V,
    const uint8_t* __restrict__ phase, const double* __restrict__ absV, double* __restrict__ e0) {
  extern __shared__ __align__(16) unsigned char g_lds[];
  __shared__ double shd[kGreedyPickThreads / 64];
  __shared__ int shi[kGreedyPickThreads / 64];
  __shared__ double2 J[kGreedyMaxS * 3];
  if (gs->done) return;
  const int tid = threadIdx.x, ncand = 2 * n;
  double mn = INFINITY;
  int nact = 0, nfeas = 0;
  for (int c = tid; c < ncand; c += kGreedyPickThreads) {
    mn = fmin(mn, sm[c]);
    nact += em[c] >= 0.0;
    nfeas += sm[c] < INFINITY;
  }
  mn = block_reduce(mn, [](double a, double b) { return fmin(a, b); }, shd);
  nact = block_reduce(nact, [](int a, int b) { return a + b; }, shi);
  nfeas = block_reduce(nfeas, [](int a, int b) { return a + b; }, shi);
  if (!(mn < INFINITY)) {
    if (tid == 0) gs->done = 1;
    return;
  }
  const double thr = mn + tie;
  int win = 0x7fffffff, fl = 0;
  for (int c = tid; c < ncand; c += kGreedyPickThreads) {
    const double v = sm[c];
    if (v <= thr) win = min(win, c);
    if (v < INFINITY && fabs(v - thr) <= amb) fl = 1;
    if (em[c] >= 0.0 && fabs(em[c] - e_bar) <= amb) fl = 1;
  }
  win = block_reduce(win, [](int a, int b) { return min(a, b); }, shi);
  fl = block_reduce(fl, [](int a, int b) { return max(a, b); }, shi);
  const int wx = win >> 1, wa = sup[wx], wb = sup[parent[wx]];
  const int r = (win & 1) ? wb : wa, s = (win & 1) ? wa : wb;
  PathRec* pr = (PathRec*)g_lds;
  const int dr = depth[r], ds = depth[s];
  PathRec* ps = pr + dr + 1;
  load_paths(n, pos, size, depth, r, s, pr, ps);
  for (int q = tid; q < S * 3; q += kGreedyPickThreads) J[q] = Iagg[((size_t)(q / 3) * n + r) * 3 + q % 3];
  __syncthreads();  // sup and Iagg read by every thread before they change
  if (tid == 0) {
    GStep st;
    st.cand = win;
    st.s = s;
    st.r = r;
    st.ambiguous = fl;
    st.n_cand = nact;
    st.n_feasible = nfeas;
    st.smice = sm[win];
    st.emax = em[win];
    steps[gs->iter] = st;
    gs->s = s;
    gs->r = r;
    gs->iter += 1;
  }
  for (int q = tid; q < S * 3; q += kGreedyPickThreads) {
    const size_t lr = ((size_t)(q / 3) * n + r) * 3 + q % 3, ls = ((size_t)(q / 3) * n + s) * 3 + q % 3;
    Iagg[ls] = cadd(Iagg[ls], J[q]);
    Iagg[lr] = make_double2(0.0, 0.0);
  }
  for (int u = tid; u < n; u += kGreedyPickThreads)
    if (sup[u] == r) sup[u] = s;
  MoveIntervals mi;
  mi.from(pr, dr, ps, ds, pos[s]);
  for (int t = tid; t < n * S; t += kGreedyPickThreads) {
    const int xn = t % n, l = t / n;
    const int qx = pos[xn];
    if (!mi.holds(qx)) continue;
    PathDelta md;
    md.at(pr, dr, ps, ds, Zr, qx, depth[xn]);
    if (!md.moved) continue;
    const size_t vb = ((size_t)l * n + xn) * 3;
#pragma unroll
    for (int p = 0; p < 3; ++p) V[vb + p] = cadd(V[vb + p], md.dv(p, J + l * 3));
  }
  __syncthreads();
  node_errors(n, S, phase, sup, V, absV, e0, tid, kGreedyPickThreads);
}

// ---- radialization (Section V) --------------------------------------------

// Critical nodes of a kept set (one block, level by level): a node that is
// not kept is critical when three or more of its tree directions reach a
// kept node through nodes that are not kept (its degree in the sub-tree that
// spans the kept nodes of its Kron clique).  Writes the radialized kept set
// and, for both kept sets, every node's nearest kept proper ancestor (-1 at
// the slack).  Scratch: down, up, cnt (n ints each).
__global__ __launch_bounds__(kGreedyPickThreads) void k_radialize(
    int n, const int* __restrict__ parent, const int* __restrict__ ch_off, const int* __restrict__ ch,
    const int* __restrict__ lvl_off, const int* __restrict__ lvl_nodes, int nlev, const int* __restrict__ sup,
    int* __restrict__ down, int* __restrict__ up, int* __restrict__ cnt, uint8_t* __restrict__ kept_rad,
    int* __restrict__ kp_rad, int* __restrict__ kp_mesh, int* __restrict__ ncrit) {
  __shared__ int shi[kGreedyPickThreads / 64];
  // down[x]: x is kept, or a kept node lies below x through non-kept nodes;
  // cnt[x]: children c with down[c]
  for (int lev = nlev - 1; lev >= 0; --lev) {
    for (int q = lvl_off[lev] + threadIdx.x; q < lvl_off[lev + 1]; q += blockDim.x) {
      const int x = lvl_nodes[q];
      int c = 0;
      for (int e = ch_off[x]; e < ch_off[x + 1]; ++e) c += down[ch[e]];
      cnt[x] = c;
      down[x] = (sup[x] == x || c > 0) ? 1 : 0;
    }
    __syncthreads();
  }
  // up[x]: the direction towards the parent reaches a kept node
  for (int lev = 0; lev < nlev; ++lev) {
    for (int q = lvl_off[lev] + threadIdx.x; q < lvl_off[lev + 1]; q += blockDim.x) {
      const int x = lvl_nodes[q];
      if (x == 0) {
        up[x] = 0;
        continue;
      }
      const int p = parent[x];
      up[x] = (sup[p] == p || up[p] || cnt[p] - down[x] > 0) ? 1 : 0;
    }
    __syncthreads();
  }
  int nc = 0;
  for (int x = threadIdx.x; x < n; x += blockDim.x) {
    const bool kept = sup[x] == x;
    const bool crit = !kept && up[x] + cnt[x] >= 3;
    nc += crit;
    kept_rad[x] = (kept || crit) ? 1 : 0;
  }
  nc = block_reduce(nc, [](int a, int b) { return a + b; }, shi);
  if (threadIdx.x == 0) *ncrit = nc;
  __syncthreads();
  for (int lev = 0; lev < nlev; ++lev) {
    for (int q = lvl_off[lev] + threadIdx.x; q < lvl_off[lev + 1]; q += blockDim.x) {
      const int x = lvl_nodes[q];
      if (x == 0) {
        kp_rad[x] = kp_mesh[x] = -1;
        continue;
      }
      const int p = parent[x];
      kp_rad[x] = kept_rad[p] ? p : kp_rad[p];
      kp_mesh[x] = sup[p] == p ? p : kp_mesh[p];
    }
    __syncthreads();
  }
}

// Voltage check of a radial reduced network (one thread per node and
// scenario): for every kept node x, the voltage of the radial network whose
// edges join each kept node to its nearest kept proper ancestor kp, with the
// aggregated load currents, is V0 - sum_j Zroot(a(lca(x, j))) I_j, a(v) = v
// when v is kept, else kp[v]; its largest distance from the full network's
// voltage V goes to *dv (bit pattern of a non-negative double).  Zero when
// every kept pair's lowest common ancestor is kept, i.e. when the network is
// radial with the same voltages.
__global__ __launch_bounds__(kGreedyThreads) void k_radial_check(
    int n, int S, const uint8_t* __restrict__ phase, LcaTab T, const double2* __restrict__ Zr,
    const int* __restrict__ sup, const uint8_t* __restrict__ kept_rad, const int* __restrict__ kp, int use_rad,
    const double2* __restrict__ Iagg, const double2* __restrict__ V, double2 v0a, double2 v0b, double2 v0c,
    unsigned long long* __restrict__ dv) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  double e = 0.0;
  if (t < n * S) {
    const int x = t % n, l = t / n;
    const bool kx = use_rad ? kept_rad[x] != 0 : sup[x] == x;
    if (kx) {
      const double2 v0[3] = {v0a, v0b, v0c};
      double2 acc[3] = {v0[0], v0[1], v0[2]};
      for (int j = 1; j < n; ++j) {
        if (sup[j] != j) continue;  // only super-nodes carry current
        int a = T.lca(x, j);
        const bool ka = use_rad ? kept_rad[a] != 0 : sup[a] == a;
        if (!ka) a = kp[a];
        const double2* Za = Zr + (size_t)a * 9;
        const double2* Ij = Iagg + ((size_t)l * n + j) * 3;
#pragma unroll
        for (int p = 0; p < 3; ++p)
          acc[p] = csub(acc[p], cadd(cadd(cmul(Za[p * 3], Ij[0]), cmul(Za[p * 3 + 1], Ij[1])), cmul(Za[p * 3 + 2], Ij[2])));
      }
      const double2* Vx = V + ((size_t)l * n + x) * 3;
#pragma unroll
      for (int p = 0; p < 3; ++p)
        if (phase[x] >> p & 1u) e = fmax(e, sqrt(cabs2(csub(acc[p], Vx[p]))));
    }
  }
  for (int o = 32; o > 0; o >>= 1) e = fmax(e, __shfl_xor(e, o, 64));
  if ((threadIdx.x & 63) == 0 && e > 0.0) atomicMax(dv, (unsigned long long)__double_as_longlong(e));
}

// I = A I^ for a given assignment: one thread per (scenario, node, phase)
// adds its cluster's members' currents in node order (members of super-node
// y: mem[moff[y] .. moff[y + 1]); zero for nodes that are not super-nodes).
__global__ void k_greedy_aggregate(int n, int S, const int* __restrict__ moff, const int* __restrict__ mem,
                                   const double2* __restrict__ A, double2* __restrict__ Iagg) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (size_t)S * n * 3) return;
  const int p = (int)(t % 3), y = (int)((t / 3) % n);
  const size_t base = (t / 3 / n) * n * 3;
  double2 acc = make_double2(0.0, 0.0);
  for (int q = moff[y]; q < moff[y + 1]; ++q) acc = cadd(acc, A[base + (size_t)mem[q] * 3 + p]);
  Iagg[t] = acc;
}

// Largest error of the current state per scenario (one block each): every
// node against its super-node's voltage.
__global__ __launch_bounds__(kGreedyThreads) void k_greedy_err(int n, const uint8_t* __restrict__ phase,
                                                               const int* __restrict__ sup,
                                                               const double2* __restrict__ V,
                                                               const double* __restrict__ absV,
                                                               double* __restrict__ err) {
  __shared__ double shd[16];
  const size_t base = (size_t)blockIdx.x * n * 3;
  double e = 0.0;
  for (int x = threadIdx.x; x < n; x += blockDim.x)
    for (int p = 0; p < 3; ++p)
      if (phase[x] >> p & 1u) e = fmax(e, fabs(absV[base + x * 3 + p] - sqrt(cabs2(V[base + sup[x] * 3 + p]))));
  e = block_reduce(e, [](double a, double b) { return fmax(a, b); }, shd);
  if (threadIdx.x == 0) err[blockIdx.x] = e;
}

}  // namespace okr

using namespace okr;

struct okr_greedy {
  hipStream_t stream = nullptr;
  std::string err;
  bool planned = false;
  int n = 0, S = 0, nlev = 0;
  std::vector<int> parent, pos, size, depth, lvl_off, lvl_nodes, ch_off, ch;
  std::vector<uint8_t> phase;
  // workspace layout (byte offsets)
  size_t o_topo = 0, o_phase = 0, o_z = 0, o_Zr = 0, o_Vhat = 0, o_A = 0, o_absV = 0, o_I = 0, o_V = 0, o_Ib = 0,
         o_sup = 0, o_sm = 0, o_em = 0, o_steps = 0, o_gs = 0, o_status = 0, o_iters = 0, o_err = 0, total = 0;
  // packed int arrays: parent, pos, size, depth, lvl_off, lvl_nodes, ch_off, ch
  size_t t_parent = 0, t_pos = 0, t_size = 0, t_depth = 0, t_lvl_off = 0, t_lvl_nodes = 0, t_ch_off = 0, t_ch = 0,
         t_pre = 0, t_first = 0, t_st = 0;
  int euler_len = 0;
  // cluster state of the search
  size_t o_mice = 0, o_arr = 0, o_bmax = 0, o_moff = 0, o_mem = 0, o_tot = 0;
  // radialization: 5 int arrays of n, kept flags, counter, two maxima
  size_t o_rad = 0, o_radk = 0, o_radx = 0;
  size_t o_e0 = 0;  // every node's error per scenario in the current state
  std::vector<int> topo_host;
};

#define OKRG_FAIL(g, code, ...)            \
  do {                                     \
    char _b[512];                          \
    snprintf(_b, sizeof _b, __VA_ARGS__);  \
    (g)->err = _b;                         \
    return code;                           \
  } while (0)

#define OKRG_HIP(g, call)                                                                   \
  do {                                                                                      \
    hipError_t _e = (call);                                                                 \
    if (_e != hipSuccess) OKRG_FAIL(g, OKR_E_HIP, "%s: %s", #call, hipGetErrorString(_e)); \
  } while (0)

extern "C" int okr_greedy_create(okr_greedy** g, void* hip_stream) {
  if (!g) return OKR_E_ARG;
  okr_greedy* G = new (std::nothrow) okr_greedy();
  if (!G) return OKR_E_ARG;
  G->stream = static_cast<hipStream_t>(hip_stream);
  *g = G;
  return OKR_OK;
}

extern "C" int okr_greedy_destroy(okr_greedy* g) {
  if (!g) return OKR_E_ARG;
  delete g;
  return OKR_OK;
}

extern "C" const char* okr_greedy_last_error(const okr_greedy* g) { return g ? g->err.c_str() : "null handle"; }

extern "C" int okr_greedy_plan(okr_greedy* g, int32_t n, const int32_t* parent, const uint8_t* phase, int32_t S,
                               size_t* workspace_bytes) {
  if (!g) return OKR_E_ARG;
  g->planned = false;
  if (!parent || !phase || !workspace_bytes || n < 1 || S < 1) OKRG_FAIL(g, OKR_E_ARG, "null argument, n < 1 or S < 1");
  g->n = n;
  g->S = S;
  g->parent.assign(parent, parent + n);
  g->phase.assign(phase, phase + n);
  if (g->parent[0] != -1) OKRG_FAIL(g, OKR_E_NOT_TREE, "parent[0] must be -1");
  for (int i = 1; i < n; ++i)
    if (g->parent[i] < 0 || g->parent[i] >= n || g->parent[i] == i)
      OKRG_FAIL(g, OKR_E_NOT_TREE, "parent[%d] = %d out of range", i, g->parent[i]);
  g->ch_off.assign(n + 1, 0);
  for (int i = 1; i < n; ++i) g->ch_off[g->parent[i] + 1]++;
  for (int i = 0; i < n; ++i) g->ch_off[i + 1] += g->ch_off[i];
  g->ch.assign(std::max(n - 1, 1), 0);
  {
    std::vector<int> fill(n, 0);
    for (int i = 1; i < n; ++i) g->ch[g->ch_off[g->parent[i]] + fill[g->parent[i]]++] = i;
  }
  std::vector<int> pre;
  pre.reserve(n);
  {
    std::vector<int> st{0};
    while (!st.empty() && (int)pre.size() <= n) {
      const int v = st.back();
      st.pop_back();
      pre.push_back(v);
      for (int e = g->ch_off[v + 1] - 1; e >= g->ch_off[v]; --e) st.push_back(g->ch[e]);
    }
  }
  if ((int)pre.size() != n) OKRG_FAIL(g, OKR_E_NOT_TREE, "parent[] is not a tree rooted at node 0");
  g->pos.assign(n, 0);
  for (int q = 0; q < n; ++q) g->pos[pre[q]] = q;
  g->size.assign(n, 1);
  for (int q = n - 1; q >= 1; --q) g->size[g->parent[pre[q]]] += g->size[pre[q]];
  g->depth.assign(n, 0);
  int dmax = 0;
  for (int q = 1; q < n; ++q) {
    const int v = pre[q];
    g->depth[v] = g->depth[g->parent[v]] + 1;
    dmax = std::max(dmax, g->depth[v]);
  }
  g->nlev = dmax + 1;
  g->lvl_off.assign(g->nlev + 1, 0);
  for (int i = 0; i < n; ++i) g->lvl_off[g->depth[i] + 1]++;
  for (int d = 0; d < g->nlev; ++d) g->lvl_off[d + 1] += g->lvl_off[d];
  g->lvl_nodes.assign(n, 0);
  {
    std::vector<int> fill(g->nlev, 0);
    for (int i = 0; i < n; ++i) g->lvl_nodes[g->lvl_off[g->depth[i]] + fill[g->depth[i]]++] = i;
  }
  for (int i = 0; i < n; ++i) {
    if (g->phase[i] == 0 || g->phase[i] > 7) OKRG_FAIL(g, OKR_E_PHASE, "node %d has phase mask %d", i, g->phase[i]);
    if (i > 0 && (g->phase[i] & ~g->phase[g->parent[i]]))
      OKRG_FAIL(g, OKR_E_PHASE, "phases of node %d are not a subset of its parent's", i);
  }
  // packed topology
  g->topo_host.clear();
  auto put = [&](const std::vector<int>& v) {
    const size_t at = g->topo_host.size();
    g->topo_host.insert(g->topo_host.end(), v.begin(), v.end());
    return at;
  };
  g->t_parent = put(g->parent);
  g->t_pos = put(g->pos);
  g->t_size = put(g->size);
  g->t_depth = put(g->depth);
  g->t_lvl_off = put(g->lvl_off);
  g->t_lvl_nodes = put(g->lvl_nodes);
  g->t_ch_off = put(g->ch_off);
  g->t_ch = put(g->ch);
  g->t_pre = put(pre);
  // Euler tour of the DFS (children in increasing id, i.e. increasing DFS
  // position), first occurrences, and the sparse table of shallowest nodes
  {
    std::vector<int> euler, first(n, -1);
    euler.reserve(2 * (size_t)n);
    std::vector<std::pair<int, int>> stk{{0, g->ch_off[0]}};
    euler.push_back(0);
    first[0] = 0;
    while (!stk.empty()) {
      const int v = stk.back().first, e = stk.back().second;
      if (e < g->ch_off[v + 1]) {
        stk.back().second = e + 1;
        const int c = g->ch[e];
        first[c] = (int)euler.size();
        euler.push_back(c);
        stk.push_back({c, g->ch_off[c]});
      } else {
        stk.pop_back();
        if (!stk.empty()) euler.push_back(stk.back().first);
      }
    }
    const int E = (int)euler.size();
    int L = 1;
    while ((1 << L) <= E) ++L;
    std::vector<int> sp((size_t)L * E);
    for (int i = 0; i < E; ++i) sp[i] = euler[i];
    for (int k = 1; k < L; ++k)
      for (int i = 0; i < E; ++i) {
        const int a = sp[(size_t)(k - 1) * E + i];
        const int j = i + (1 << (k - 1));
        const int b = j < E ? sp[(size_t)(k - 1) * E + j] : a;
        sp[(size_t)k * E + i] = g->depth[a] <= g->depth[b] ? a : b;
      }
    g->euler_len = E;
    g->t_first = put(first);
    g->t_st = put(sp);
  }
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off += (bytes + 255) & ~size_t(255);
    return at;
  };
  const size_t c3 = (size_t)S * n * 3;
  g->o_topo = take(sizeof(int) * g->topo_host.size());
  g->o_phase = take(n);
  g->o_z = take(sizeof(double2) * 9 * n);
  g->o_Zr = take(sizeof(double2) * 9 * n);
  g->o_Vhat = take(sizeof(double2) * c3);
  g->o_A = take(sizeof(double2) * c3);
  g->o_absV = take(sizeof(double) * c3);
  g->o_I = take(sizeof(double2) * c3);
  g->o_V = take(sizeof(double2) * c3);
  g->o_Ib = take(sizeof(double2) * c3);
  g->o_sup = take(sizeof(int) * n);
  g->o_sm = take(sizeof(double) * 2 * n);
  g->o_em = take(sizeof(double) * 2 * n);
  g->o_steps = take(sizeof(GStep) * n);
  g->o_gs = take(sizeof(GState));
  g->o_status = take(sizeof(int) * 4);
  g->o_iters = take(sizeof(int) * S);
  g->o_err = take(sizeof(double) * S);
  g->o_mice = take(sizeof(double) * (size_t)S * n);
  g->o_arr = take(sizeof(double) * n);
  g->o_bmax = take(sizeof(double) * ((n + 63) / 64));
  g->o_moff = take(sizeof(int) * (n + 1));
  g->o_mem = take(sizeof(int) * n);
  g->o_tot = take(sizeof(double));
  g->o_rad = take(sizeof(int) * 5 * (size_t)n);
  g->o_radk = take(n);
  g->o_radx = take(sizeof(unsigned long long) * 4);
  g->o_e0 = take(sizeof(double) * (size_t)S * n);
  g->total = off;
  *workspace_bytes = off;
  g->planned = true;
  return OKR_OK;
}

namespace {
struct GPtrs {
  int *topo, *parent, *pos, *size, *depth, *lvl_off, *lvl_nodes, *ch_off, *ch, *pre, *first, *sp, *sup, *status,
      *iters;
  Clusters C;
  uint8_t* phase;
  double2 *z, *Zr, *Vhat, *A, *I, *V, *Ib;
  double *absV, *sm, *em, *err, *e0;
  GStep* steps;
  GState* gs;
};

GPtrs gptrs(const okr_greedy* g, void* ws) {
  char* b = (char*)ws;
  GPtrs p;
  p.topo = (int*)(b + g->o_topo);
  p.parent = p.topo + g->t_parent;
  p.pos = p.topo + g->t_pos;
  p.size = p.topo + g->t_size;
  p.depth = p.topo + g->t_depth;
  p.lvl_off = p.topo + g->t_lvl_off;
  p.lvl_nodes = p.topo + g->t_lvl_nodes;
  p.ch_off = p.topo + g->t_ch_off;
  p.ch = p.topo + g->t_ch;
  p.pre = p.topo + g->t_pre;
  p.first = p.topo + g->t_first;
  p.sp = p.topo + g->t_st;
  p.C.mice = (double*)(b + g->o_mice);
  p.C.arr = (double*)(b + g->o_arr);
  p.C.bmax = (double*)(b + g->o_bmax);
  p.C.moff = (int*)(b + g->o_moff);
  p.C.mem = (int*)(b + g->o_mem);
  p.C.tot = (double*)(b + g->o_tot);
  p.phase = (uint8_t*)(b + g->o_phase);
  p.z = (double2*)(b + g->o_z);
  p.Zr = (double2*)(b + g->o_Zr);
  p.Vhat = (double2*)(b + g->o_Vhat);
  p.A = (double2*)(b + g->o_A);
  p.absV = (double*)(b + g->o_absV);
  p.I = (double2*)(b + g->o_I);
  p.V = (double2*)(b + g->o_V);
  p.Ib = (double2*)(b + g->o_Ib);
  p.sup = (int*)(b + g->o_sup);
  p.sm = (double*)(b + g->o_sm);
  p.em = (double*)(b + g->o_em);
  p.steps = (GStep*)(b + g->o_steps);
  p.gs = (GState*)(b + g->o_gs);
  p.status = (int*)(b + g->o_status);
  p.iters = (int*)(b + g->o_iters);
  p.err = (double*)(b + g->o_err);
  p.e0 = (double*)(b + g->o_e0);
  return p;
}

// Common set-up of a run or an evaluation: topology upload, branch
// impedances, impedances from the root, scenario library (load flow unless
// V^ is given); returns the status word and the largest load-flow count.
int setup(okr_greedy* g, const GPtrs& p, const okr_yblocks* Y, const okr_loads* L, const okr_greedy_params* prm) {
  const hipStream_t st = g->stream;
  const int n = g->n, S = g->S;
  OKRG_HIP(g, hipMemcpyAsync(p.topo, g->topo_host.data(), sizeof(int) * g->topo_host.size(), hipMemcpyHostToDevice, st));
  OKRG_HIP(g, hipMemcpyAsync(p.phase, g->phase.data(), n, hipMemcpyHostToDevice, st));
  OKRG_HIP(g, hipMemsetAsync(p.status, 0, sizeof(int) * 4, st));
  hipLaunchKernelGGL(k_branch_z, dim3((n + 127) / 128), dim3(128), 0, st, n, (const int*)p.parent,
                     (const uint8_t*)p.phase, (const int*)p.ch_off, (const int*)p.ch, (const double2*)Y->Y_diag,
                     (const double2*)Y->Y_off, p.z, p.status);
  hipLaunchKernelGGL(k_zroot, dim3(1), dim3(1024), 0, st, n, (const int*)p.parent, (const int*)p.lvl_off,
                     (const int*)p.lvl_nodes, g->nlev, (const double2*)p.z, p.Zr);
  const size_t c3 = (size_t)S * n * 3;
  const double2* V0 = (const double2*)L->V0;
  if (prm->flags & OKR_FLAG_VHAT_GIVEN) {
    OKRG_HIP(g, hipMemcpyAsync(p.Vhat, L->Vhat, sizeof(double2) * c3, hipMemcpyDeviceToDevice, st));
    hipLaunchKernelGGL(k_from_vhat, dim3((unsigned)((c3 + 255) / 256)), dim3(256), 0, st, n, S,
                       (const uint8_t*)p.phase, (const double2*)L->S_load, (const double2*)p.Vhat, 0.0, 1e300, p.A,
                       p.absV, p.status);
  } else {
    hipLaunchKernelGGL(k_powerflow, dim3(S), dim3(256), 0, st, n, (const int*)p.parent, (const uint8_t*)p.phase,
                       (const int*)p.lvl_off, (const int*)p.lvl_nodes, g->nlev, (const int*)p.ch_off,
                       (const int*)p.ch, (const double2*)p.z, (const double2*)L->S_load, V0[0], V0[1], V0[2],
                       prm->pf_tol > 0 ? prm->pf_tol : 1e-13, prm->pf_maxit > 0 ? prm->pf_maxit : 100, 0.0, 1e300,
                       p.Vhat, p.Ib, p.A, p.absV, p.iters, p.status);
  }
  OKRG_HIP(g, hipGetLastError());
  return OKR_OK;
}

int check_status(okr_greedy* g, int hs) {
  if (hs & 1) OKRG_FAIL(g, OKR_E_SINGULAR, "a present-phase branch block is singular");
  if (hs & 2) OKRG_FAIL(g, OKR_E_PHASE, "nonzero admittance entries on absent phases");
  if (hs & (4 | 8)) OKRG_FAIL(g, OKR_E_UNSUPPORTED, "admittance blocks asymmetric or with shunts");
  if (hs & 16) OKRG_FAIL(g, OKR_E_PF_DIVERGED, "load flow did not converge");
  return OKR_OK;
}

int check_call(okr_greedy* g, const okr_yblocks* Y, const okr_loads* L, const okr_greedy_params* prm, void* ws) {
  if (!g->planned) OKRG_FAIL(g, OKR_E_ARG, "okr_greedy_plan has not succeeded");
  if (!Y || !L || !prm || !Y->Y_diag || !Y->Y_off || !L->S_load || !L->V0) OKRG_FAIL(g, OKR_E_ARG, "null argument");
  if (L->S != g->S) OKRG_FAIL(g, OKR_E_ARG, "loads->S = %d, planned for %d", L->S, g->S);
  if ((prm->flags & OKR_FLAG_VHAT_GIVEN) && !L->Vhat) OKRG_FAIL(g, OKR_E_ARG, "OKR_FLAG_VHAT_GIVEN without Vhat");
  if (!ws) OKRG_FAIL(g, OKR_E_WORKSPACE, "no workspace");
  return OKR_OK;
}
// An assignment: super-nodes are their own super-node, every cluster is
// connected (one member whose parent lies outside it), the slack is a
// super-node, and a member's phases lie within its super-node's.
int check_assignment(okr_greedy* g, const int32_t* super) {
  const int n = g->n;
  std::vector<int> top(n, -1);
  for (int x = 0; x < n; ++x) {
    const int s = super[x];
    if (s < 0 || s >= n || super[s] != s) OKRG_FAIL(g, OKR_E_ARG, "super[%d] = %d is not a super-node", x, s);
    if (g->phase[x] & ~g->phase[s]) OKRG_FAIL(g, OKR_E_ARG, "node %d has phases outside its super-node's", x);
  }
  if (super[0] != 0) OKRG_FAIL(g, OKR_E_ARG, "the slack must stay its own super-node");
  for (int x = 0; x < n; ++x) {  // each cluster has one node whose parent lies outside it
    const int s = super[x];
    if (x == 0 || super[g->parent[x]] != s) {
      if (top[s] >= 0) OKRG_FAIL(g, OKR_E_ARG, "the cluster of super-node %d is not connected", s);
      top[s] = x;
    }
  }
  return OKR_OK;
}
}  // namespace

extern "C" int okr_greedy_run(okr_greedy* g, const okr_yblocks* Y, const okr_loads* L, const okr_greedy_params* prm,
                              void* ws, okr_greedy_result* out) {
  if (!g) return OKR_E_ARG;
  int rc = check_call(g, Y, L, prm, ws);
  if (rc) return rc;
  if (!out || !out->super || !out->steps || !out->err_per_snapshot) OKRG_FAIL(g, OKR_E_ARG, "null result buffer");
  const int n = g->n, S = g->S;
  if (S > kGreedyMaxS) OKRG_FAIL(g, OKR_E_UNSUPPORTED, "the search takes at most %d scenarios", kGreedyMaxS);
  // every candidate scores every node while the cluster table fits in LDS;
  // beyond that (or when asked) only the clusters a move can change
  const size_t lds_full = sizeof(unsigned long long) * (size_t)S * n + sizeof(PathRec) * 2 * (size_t)g->nlev;
  const size_t lds_paths = sizeof(PathRec) * 2 * (size_t)g->nlev;
  // (the full-scoring kernel also holds about 3 KB of static LDS)
  const bool incremental =
      (prm->flags & OKR_GREEDY_INCREMENTAL) || (size_t)S * n > kGreedyFullSN || lds_full > 60 * 1024;
  if (incremental && n > kGreedyMaxN)
    OKRG_FAIL(g, OKR_E_UNSUPPORTED, "the search takes at most %d nodes", kGreedyMaxN);
  const size_t lds_cnt = sizeof(int) * (size_t)n;
  const hipStream_t st = g->stream;
  const GPtrs p = gptrs(g, ws);
  hipEvent_t ev[3];
  for (auto& e : ev) OKRG_HIP(g, hipEventCreate(&e));
  struct EvGuard {
    hipEvent_t* e;
    ~EvGuard() {
      for (int i = 0; i < 3; ++i) (void)hipEventDestroy(e[i]);
    }
  } guard{ev};
  OKRG_HIP(g, hipEventRecord(ev[0], st));
  rc = setup(g, p, Y, L, prm);
  if (rc) return rc;
  const double2* V0 = (const double2*)L->V0;
  const size_t c3 = (size_t)S * n * 3;
  hipLaunchKernelGGL(k_greedy_init, dim3((unsigned)((std::max(c3, (size_t)n) + 255) / 256)), dim3(256), 0, st, n, S,
                     (const double2*)p.A, p.I, p.sup, p.gs);
  hipLaunchKernelGGL(k_greedy_sweep, dim3(S), dim3(kGreedyThreads), 0, st, n, (const int*)p.parent,
                     (const uint8_t*)p.phase, (const int*)p.lvl_off, (const int*)p.lvl_nodes, g->nlev,
                     (const int*)p.ch_off, (const int*)p.ch, (const double2*)p.z, V0[0], V0[1], V0[2],
                     (const double2*)p.I, p.Ib, p.V);
  LcaTab T;
  T.first = p.first;
  T.st = p.sp;
  T.depth = p.depth;
  T.E = g->euler_len;
  if (incremental)
    hipLaunchKernelGGL(k_greedy_prep, dim3(1), dim3(kGreedyPickThreads), lds_cnt, st, n, S, (const uint8_t*)p.phase,
                       (const int*)p.pre, (const int*)p.sup, (const double2*)p.V, (const double*)p.absV, p.C);
  else
    hipLaunchKernelGGL(k_greedy_e0, dim3((unsigned)(((size_t)n * S + kGreedyThreads - 1) / kGreedyThreads)),
                       dim3(kGreedyThreads), 0, st, n, S, (const uint8_t*)p.phase, (const int*)p.sup,
                       (const double2*)p.V, (const double*)p.absV, p.e0);
  OKRG_HIP(g, hipGetLastError());
  OKRG_HIP(g, hipEventRecord(ev[1], st));
  const double e_bar = prm->e_bar, tie = prm->tie_tol > 0 ? prm->tie_tol : 1e-11;
  const double amb = prm->amb_tol > 0 ? prm->amb_tol : 1e-13;
  // at most one move per enqueued iteration: the cap is the number enqueued
  const int cap = prm->max_iter > 0 ? std::min(prm->max_iter, n - 1) : n - 1;
  GState hs{};
  int enq = 0;
  constexpr int kBatch = 32;  // moves enqueued between checks of the done flag
  const bool timing = (prm->flags & OKR_FLAG_TIMING) != 0;
  std::vector<hipEvent_t> tev(timing ? 2 * kBatch : 0);
  for (auto& e : tev) OKRG_HIP(g, hipEventCreate(&e));
  struct TevGuard {
    std::vector<hipEvent_t>* v;
    ~TevGuard() {
      for (hipEvent_t e : *v) (void)hipEventDestroy(e);
    }
  } tguard{&tev};
  double score_ms = 0.0;
  int launches = 0;
  // one iteration's two launches (and the timing events around the scoring)
  auto enqueue_iteration = [&](int t) -> hipError_t {
    if (timing) {
      const hipError_t e = hipEventRecord(tev[2 * t], st);
      if (e != hipSuccess) return e;
    }
    if (incremental) {
      hipLaunchKernelGGL(k_greedy_score, dim3(2 * n), dim3(kGreedyThreads), 0, st, n, S, (const int*)p.parent,
                         (const uint8_t*)p.phase, (const int*)p.pos, (const int*)p.size, (const int*)p.pre,
                         (const int*)p.ch_off, (const int*)p.ch, (const int*)p.sup, T, (const double2*)p.Zr,
                         (const double2*)p.I, (const double2*)p.V, (const double*)p.absV, e_bar,
                         (const GState*)p.gs, p.C, p.sm, p.em);
      if (timing) {
        const hipError_t e = hipEventRecord(tev[2 * t + 1], st);
        if (e != hipSuccess) return e;
      }
      hipLaunchKernelGGL(k_greedy_pick_apply, dim3(1), dim3(kGreedyPickThreads), lds_cnt, st, n, S,
                         (const int*)p.parent, (const uint8_t*)p.phase, (const int*)p.pre, (const int*)p.pos,
                         (const int*)p.size, (const int*)p.ch_off, (const int*)p.ch, T, (const double2*)p.Zr,
                         (const double*)p.absV, (const double*)p.sm, (const double*)p.em, e_bar, tie, amb, p.gs,
                         p.steps, p.sup, p.I, p.V, p.C);
    } else {
      hipLaunchKernelGGL(k_greedy_score_full, dim3(2 * n), dim3(kGreedyThreads), lds_full, st, n, S,
                         (const int*)p.parent, (const uint8_t*)p.phase, (const int*)p.pos, (const int*)p.size,
                         (const int*)p.depth, (const int*)p.sup, (const double2*)p.Zr, (const double2*)p.I,
                         (const double2*)p.V, (const double*)p.absV, (const double*)p.e0, e_bar,
                         (const GState*)p.gs, p.sm, p.em);
      if (timing) {
        const hipError_t e = hipEventRecord(tev[2 * t + 1], st);
        if (e != hipSuccess) return e;
      }
      hipLaunchKernelGGL(k_greedy_pick_apply_full, dim3(1), dim3(kGreedyPickThreads), lds_paths, st, n, S,
                         (const int*)p.parent, (const int*)p.pos, (const int*)p.size, (const int*)p.depth,
                         (const double2*)p.Zr, (const double*)p.sm, (const double*)p.em, e_bar, tie, amb, p.gs,
                         p.steps, p.sup, p.I, p.V, (const uint8_t*)p.phase, (const double*)p.absV, p.e0);
    }
    return hipGetLastError();
  };
  // Without timing, a full batch of iterations is captured once into a graph
  // and replayed (the launches' arguments do not change between
  // iterations; the state lives in the workspace).  No memset is captured.
  hipGraphExec_t bexec = nullptr;
  struct GraphGuard {
    hipGraphExec_t* e;
    ~GraphGuard() {
      if (*e) (void)hipGraphExecDestroy(*e);
    }
  } gguard{&bexec};
  if (!timing && st != nullptr && cap >= kBatch) {
    hipGraph_t graph = nullptr;
    OKRG_HIP(g, hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    hipError_t ce = hipSuccess;
    for (int t = 0; t < kBatch && ce == hipSuccess; ++t) ce = enqueue_iteration(t);
    const hipError_t ee = hipStreamEndCapture(st, &graph);
    if (ce != hipSuccess || ee != hipSuccess)
      OKRG_FAIL(g, OKR_E_HIP, "graph capture failed: %s", hipGetErrorString(ce != hipSuccess ? ce : ee));
    const hipError_t ie = hipGraphInstantiate(&bexec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess) OKRG_FAIL(g, OKR_E_HIP, "graph instantiate failed: %s", hipGetErrorString(ie));
  }
  while (enq < cap) {
    const int b = std::min(kBatch, cap - enq);
    if (bexec && b == kBatch) {
      OKRG_HIP(g, hipGraphLaunch(bexec, st));
    } else {
      for (int t = 0; t < b; ++t) OKRG_HIP(g, enqueue_iteration(t));
    }
    OKRG_HIP(g, hipGetLastError());
    const int before = hs.iter;
    OKRG_HIP(g, hipMemcpyAsync(&hs, p.gs, sizeof(GState), hipMemcpyDeviceToHost, st));
    OKRG_HIP(g, hipStreamSynchronize(st));
    // score launches that did work: one per move, plus the one that found none
    const int ran = std::min(b, hs.iter - before + (hs.done ? 1 : 0));
    launches += ran;
    if (timing)
      for (int t = 0; t < ran; ++t) {
        float ms = 0.f;
        OKRG_HIP(g, hipEventElapsedTime(&ms, tev[2 * t], tev[2 * t + 1]));
        score_ms += ms;
      }
    enq += b;
    if (hs.done) break;
  }
  OKRG_HIP(g, hipEventRecord(ev[2], st));
  hipLaunchKernelGGL(k_greedy_err, dim3(S), dim3(kGreedyThreads), 0, st, n, (const uint8_t*)p.phase,
                     (const int*)p.sup, (const double2*)p.V, (const double*)p.absV, p.err);
  OKRG_HIP(g, hipGetLastError());
  int status[4] = {0, 0, 0, 0};
  std::vector<int> iters(S, 0);
  OKRG_HIP(g, hipMemcpyAsync(status, p.status, sizeof(status), hipMemcpyDeviceToHost, st));
  if (!(prm->flags & OKR_FLAG_VHAT_GIVEN))
    OKRG_HIP(g, hipMemcpyAsync(iters.data(), p.iters, sizeof(int) * S, hipMemcpyDeviceToHost, st));
  OKRG_HIP(g, hipMemcpyAsync(&hs, p.gs, sizeof(GState), hipMemcpyDeviceToHost, st));
  OKRG_HIP(g, hipMemcpyAsync(out->super, p.sup, sizeof(int) * n, hipMemcpyDeviceToHost, st));
  OKRG_HIP(g, hipMemcpyAsync(out->err_per_snapshot, p.err, sizeof(double) * S, hipMemcpyDeviceToHost, st));
  OKRG_HIP(g, hipStreamSynchronize(st));
  rc = check_status(g, status[0]);
  if (rc) return rc;
  if (hs.iter > 0)
  {
    OKRG_HIP(g, hipMemcpyAsync(out->steps, p.steps, sizeof(GStep) * hs.iter, hipMemcpyDeviceToHost, st));
    OKRG_HIP(g, hipStreamSynchronize(st));
  }
  out->n_steps = hs.iter;
  out->n_kept = n - hs.iter;
  out->n_score_launches = launches;
  out->incremental = incremental ? 1 : 0;
  out->t_score_ms = score_ms;
  {
    int64_t sc = 0;
    for (int i = 0; i < hs.iter; ++i) sc += out->steps[i].n_cand;
    out->n_scored = sc;
  }
  double mx = 0.0;
  for (int l = 0; l < S; ++l) mx = std::max(mx, out->err_per_snapshot[l]);
  out->max_err = mx;
  float a = 0.f, b = 0.f;
  OKRG_HIP(g, hipEventElapsedTime(&a, ev[0], ev[1]));
  OKRG_HIP(g, hipEventElapsedTime(&b, ev[1], ev[2]));
  out->t_pf_ms = a;
  out->t_search_ms = b;
  int im = 0;
  for (int v : iters) im = std::max(im, v);
  out->pf_iterations = im;
  return OKR_OK;
}

extern "C" int okr_greedy_evaluate(okr_greedy* g, const okr_yblocks* Y, const okr_loads* L, const int32_t* super,
                                   const okr_greedy_params* prm, void* ws, double* err, double* max_err) {
  if (!g) return OKR_E_ARG;
  int rc = check_call(g, Y, L, prm, ws);
  if (rc) return rc;
  if (!super || !err) OKRG_FAIL(g, OKR_E_ARG, "null assignment or output");
  const int n = g->n, S = g->S;
  rc = check_assignment(g, super);
  if (rc) return rc;
  const GPtrs p = gptrs(g, ws);
  const hipStream_t st = g->stream;
  rc = setup(g, p, Y, L, prm);
  if (rc) return rc;
  const double2* V0 = (const double2*)L->V0;
  // members of every cluster in node order (CSR), staged in the candidate
  // score buffers (unused by an evaluation)
  std::vector<int> csr(2 * (size_t)n + 1, 0);
  for (int x = 0; x < n; ++x) csr[super[x] + 1]++;
  for (int y = 0; y < n; ++y) csr[y + 1] += csr[y];
  {
    std::vector<int> fill(csr.begin(), csr.begin() + n);
    for (int x = 0; x < n; ++x) csr[n + 1 + fill[super[x]]++] = x;
  }
  int* moff = (int*)p.sm;
  OKRG_HIP(g, hipMemcpyAsync(p.sup, super, sizeof(int) * n, hipMemcpyHostToDevice, st));
  OKRG_HIP(g, hipMemcpyAsync(moff, csr.data(), sizeof(int) * csr.size(), hipMemcpyHostToDevice, st));
  const size_t c3 = (size_t)S * n * 3;
  hipLaunchKernelGGL(k_greedy_aggregate, dim3((unsigned)((c3 + 255) / 256)), dim3(256), 0, st, n, S,
                     (const int*)moff, (const int*)(moff + n + 1), (const double2*)p.A, p.I);
  hipLaunchKernelGGL(k_greedy_sweep, dim3(S), dim3(kGreedyThreads), 0, st, n, (const int*)p.parent,
                     (const uint8_t*)p.phase, (const int*)p.lvl_off, (const int*)p.lvl_nodes, g->nlev,
                     (const int*)p.ch_off, (const int*)p.ch, (const double2*)p.z, V0[0], V0[1], V0[2],
                     (const double2*)p.I, p.Ib, p.V);
  hipLaunchKernelGGL(k_greedy_err, dim3(S), dim3(kGreedyThreads), 0, st, n, (const uint8_t*)p.phase,
                     (const int*)p.sup, (const double2*)p.V, (const double*)p.absV, p.err);
  OKRG_HIP(g, hipGetLastError());
  int status[4] = {0, 0, 0, 0};
  OKRG_HIP(g, hipMemcpyAsync(status, p.status, sizeof(status), hipMemcpyDeviceToHost, st));
  OKRG_HIP(g, hipMemcpyAsync(err, p.err, sizeof(double) * S, hipMemcpyDeviceToHost, st));
  OKRG_HIP(g, hipStreamSynchronize(st));
  rc = check_status(g, status[0]);
  if (rc) return rc;
  if (max_err) {
    double mx = 0.0;
    for (int l = 0; l < S; ++l) mx = std::max(mx, err[l]);
    *max_err = mx;
  }
  return OKR_OK;
}

extern "C" int okr_greedy_radialize(okr_greedy* g, const okr_yblocks* Y, const okr_loads* L, const int32_t* super,
                                    const okr_greedy_params* prm, void* ws, uint8_t* kept_radial,
                                    int32_t* kept_parent, int32_t* n_critical, double* dv_radial,
                                    double* dv_meshed) {
  if (!g) return OKR_E_ARG;
  int rc = check_call(g, Y, L, prm, ws);
  if (rc) return rc;
  if (!super || !kept_radial || !kept_parent || !n_critical) OKRG_FAIL(g, OKR_E_ARG, "null assignment or output");
  rc = check_assignment(g, super);
  if (rc) return rc;
  const int n = g->n, S = g->S;
  const GPtrs p = gptrs(g, ws);
  const hipStream_t st = g->stream;
  rc = setup(g, p, Y, L, prm);
  if (rc) return rc;
  const double2* V0 = (const double2*)L->V0;
  std::vector<int> csr(2 * (size_t)n + 1, 0);
  for (int x = 0; x < n; ++x) csr[super[x] + 1]++;
  for (int y = 0; y < n; ++y) csr[y + 1] += csr[y];
  {
    std::vector<int> fill(csr.begin(), csr.begin() + n);
    for (int x = 0; x < n; ++x) csr[n + 1 + fill[super[x]]++] = x;
  }
  int* moff = (int*)p.sm;
  OKRG_HIP(g, hipMemcpyAsync(p.sup, super, sizeof(int) * n, hipMemcpyHostToDevice, st));
  OKRG_HIP(g, hipMemcpyAsync(moff, csr.data(), sizeof(int) * csr.size(), hipMemcpyHostToDevice, st));
  const size_t c3 = (size_t)S * n * 3;
  hipLaunchKernelGGL(k_greedy_aggregate, dim3((unsigned)((c3 + 255) / 256)), dim3(256), 0, st, n, S,
                     (const int*)moff, (const int*)(moff + n + 1), (const double2*)p.A, p.I);
  hipLaunchKernelGGL(k_greedy_sweep, dim3(S), dim3(kGreedyThreads), 0, st, n, (const int*)p.parent,
                     (const uint8_t*)p.phase, (const int*)p.lvl_off, (const int*)p.lvl_nodes, g->nlev,
                     (const int*)p.ch_off, (const int*)p.ch, (const double2*)p.z, V0[0], V0[1], V0[2],
                     (const double2*)p.I, p.Ib, p.V);
  char* b = (char*)ws;
  int* rad = (int*)(b + g->o_rad);
  int *down = rad, *up = rad + n, *cnt = rad + 2 * n, *kp_rad = rad + 3 * n, *kp_mesh = rad + 4 * n;
  uint8_t* krad = (uint8_t*)(b + g->o_radk);
  unsigned long long* x = (unsigned long long*)(b + g->o_radx);  // [0] critical count, [1] dv radial, [2] dv meshed
  OKRG_HIP(g, hipMemsetAsync(x, 0, sizeof(unsigned long long) * 4, st));
  hipLaunchKernelGGL(k_radialize, dim3(1), dim3(kGreedyPickThreads), 0, st, n, (const int*)p.parent,
                     (const int*)p.ch_off, (const int*)p.ch, (const int*)p.lvl_off, (const int*)p.lvl_nodes, g->nlev,
                     (const int*)p.sup, down, up, cnt, krad, kp_rad, kp_mesh, (int*)x);
  LcaTab T;
  T.first = p.first;
  T.st = p.sp;
  T.depth = p.depth;
  T.E = g->euler_len;
  // the check costs n x n per scenario: the first four scenarios suffice
  // (a missed critical node shows in any scenario that loads its branches)
  const int Sc = std::min(S, 4);
  const unsigned nb = (unsigned)(((size_t)n * Sc + kGreedyThreads - 1) / kGreedyThreads);
  hipLaunchKernelGGL(k_radial_check, dim3(nb), dim3(kGreedyThreads), 0, st, n, Sc, (const uint8_t*)p.phase, T,
                     (const double2*)p.Zr, (const int*)p.sup, (const uint8_t*)krad, (const int*)kp_rad, 1,
                     (const double2*)p.I, (const double2*)p.V, V0[0], V0[1], V0[2], x + 1);
  hipLaunchKernelGGL(k_radial_check, dim3(nb), dim3(kGreedyThreads), 0, st, n, Sc, (const uint8_t*)p.phase, T,
                     (const double2*)p.Zr, (const int*)p.sup, (const uint8_t*)krad, (const int*)kp_mesh, 0,
                     (const double2*)p.I, (const double2*)p.V, V0[0], V0[1], V0[2], x + 2);
  OKRG_HIP(g, hipGetLastError());
  int status[4] = {0, 0, 0, 0};
  unsigned long long hx[4] = {0, 0, 0, 0};
  OKRG_HIP(g, hipMemcpyAsync(status, p.status, sizeof(status), hipMemcpyDeviceToHost, st));
  OKRG_HIP(g, hipMemcpyAsync(hx, x, sizeof(hx), hipMemcpyDeviceToHost, st));
  OKRG_HIP(g, hipMemcpyAsync(kept_radial, krad, n, hipMemcpyDeviceToHost, st));
  OKRG_HIP(g, hipMemcpyAsync(kept_parent, kp_rad, sizeof(int) * n, hipMemcpyDeviceToHost, st));
  OKRG_HIP(g, hipStreamSynchronize(st));
  rc = check_status(g, status[0]);
  if (rc) return rc;
  int nc;
  std::memcpy(&nc, &hx[0], sizeof(int));
  *n_critical = nc;
  double d1, d2;
  std::memcpy(&d1, &hx[1], sizeof(double));
  std::memcpy(&d2, &hx[2], sizeof(double));
  if (dv_radial) *dv_radial = d1;
  if (dv_meshed) *dv_meshed = d2;
  return OKR_OK;
}
