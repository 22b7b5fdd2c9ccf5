// Host side of the C ABI: validation, DFS renumbering, per-segment index
// tables from the cumulative kept state, launch sequencing and outputs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/okr.h"
#include "okr_internal.h"

namespace okr {
// kernels (okr_kernels.hip)
__global__ void k_branch_z(int, const int*, const uint8_t*, const int*, const int*, const double2*, const double2*,
                           double2*, int*);
__global__ void k_powerflow(int, const int*, const uint8_t*, const int*, const int*, int, const int*, const int*,
                            const double2*, const double2*, double2, double2, double2, double, int, double, double,
                            double2*, double2*, double2*, double*, int*, int*);
__global__ void k_from_vhat(int, int, const uint8_t*, const double2*, const double2*, double, double, double2*,
                            double*, int*);
__global__ void k_seg_fill(const int*, SegHdr, int, const double2*, const double2*, const double2*, const double*,
                           double2*, TargetRec*, double2*, TargetRec*, double*);
__global__ void k_score_fp64(const int*, SegHdr, const double2*, const TargetRec*, const double2*, const TargetRec*,
                             const double*, int, int, SelParams, MaskScore*, MaskScore*, TileRec*, int*);
__global__ void k_argmin(const MaskScore*, const TileRec*, int, SelParams, DevDecision*);
__global__ void k_sqrt_selftest(const double*, double*, int);
__global__ void k_apply(const int*, SegHdr, int, const DevDecision*, const double2*, const TargetRec*,
                        const TargetRec*, double2*, double2*);
__global__ void k_final_err(int, const uint8_t*, const int*, const double2*, const double*, double*);
__global__ void k_kron_yeq(int, const int*, const uint8_t*, const int*, const double2*, double2*, double2*, int*);
__global__ void k_kron_diag(int, const uint8_t*, const int*, const int*, const int*, const double2*, double2*);
}  // namespace okr

using namespace okr;

namespace {

constexpr int kMaxSnapGroups = 32;

struct Layout {
  size_t z, Vhat, Vcur, A, J, absV, status, iters, topo, tab, P, srec, headV, zrec, econst, res, fin, tiles,
      tickets, dec, fin_int, yeq, Ykd, Yko, err, total;
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Snapshot groups of a scoring launch: enough blocks to fill the chip (about
// 8192 waves), each group a contiguous run of snapshots.
int snap_groups(int k, int S, int* spg) {
  const int mblocks = (int)((((uint64_t)1 << k) + kScoreBlock - 1) / kScoreBlock);
  int SG = std::min(S, std::max(1, 8192 / mblocks));
  SG = std::min(SG, kMaxSnapGroups);
  *spg = (S + SG - 1) / SG;
  return (S + *spg - 1) / *spg;
}

}  // namespace

struct okr_handle {
  hipStream_t stream = nullptr;
  std::string err;
  // plan
  bool planned = false;
  int n = 0, S = 0, nseg = 0, kmax = 0, nlev = 0;
  int64_t ncand = 0;
  std::vector<int> parent, segment, pre, pos, size, ch_off, ch, lvl_off, lvl_nodes;
  std::vector<uint8_t> phase, eligible;
  std::vector<std::vector<int>> seg_nodes;
  Layout L{};
  int topo_ints = 0, tab_ints_max = 0, zent_max = 0;
  // search state
  std::vector<uint8_t> kept, in_omega;
  std::vector<int> sup, zidx;
  // pinned staging
  int* h_tab = nullptr;
  size_t h_tab_bytes = 0;
  DevDecision* h_dec = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  // per-mask score dumps
  std::vector<std::vector<double>> dump_e, dump_s;
  std::vector<int> dump_k;
};

#define OKR_FAIL(h, code, ...)                                  \
  do {                                                          \
    char _b[512];                                               \
    snprintf(_b, sizeof _b, __VA_ARGS__);                       \
    (h)->err = _b;                                              \
    return code;                                                \
  } while (0)

#define OKR_HIP(h, call)                                                               \
  do {                                                                                 \
    hipError_t _e = (call);                                                            \
    if (_e != hipSuccess) OKR_FAIL(h, OKR_E_HIP, "%s: %s", #call, hipGetErrorString(_e)); \
  } while (0)

extern "C" int okr_create(okr_handle** h, void* hip_stream) {
  if (!h) return OKR_E_ARG;
  okr_handle* H = new (std::nothrow) okr_handle();
  if (!H) return OKR_E_ARG;
  H->stream = static_cast<hipStream_t>(hip_stream);
  *h = H;
  return OKR_OK;
}

extern "C" int okr_destroy(okr_handle* h) {
  if (!h) return OKR_E_ARG;
  if (h->h_tab) (void)hipHostFree(h->h_tab);
  if (h->h_dec) (void)hipHostFree(h->h_dec);
  if (h->ev0) (void)hipEventDestroy(h->ev0);
  if (h->ev1) (void)hipEventDestroy(h->ev1);
  delete h;
  return OKR_OK;
}

extern "C" const char* okr_last_error(const okr_handle* h) { return h ? h->err.c_str() : "null handle"; }

// ------------------------------------------------------------------- plan --
extern "C" int okr_plan(okr_handle* h, const okr_topology* topo, const okr_margins* mg, int32_t S,
                        size_t* workspace_bytes, okr_sizes* sizes) {
  if (!h) return OKR_E_ARG;
  h->planned = false;
  if (!topo || !mg || !workspace_bytes || S < 1) OKR_FAIL(h, OKR_E_ARG, "null argument or S < 1");
  const int n = topo->n;
  if (n < 1 || !topo->parent || !topo->phase || !topo->eligible || !topo->segment)
    OKR_FAIL(h, OKR_E_ARG, "topology arrays missing or n < 1");
  h->n = n;
  h->S = S;
  h->parent.assign(topo->parent, topo->parent + n);
  h->phase.assign(topo->phase, topo->phase + n);
  h->eligible.assign(topo->eligible, topo->eligible + n);
  h->segment.assign(topo->segment, topo->segment + n);
  if (h->parent[0] != -1) OKR_FAIL(h, OKR_E_NOT_TREE, "parent[0] must be -1");
  for (int i = 1; i < n; ++i)
    if (h->parent[i] < 0 || h->parent[i] >= n || h->parent[i] == i)
      OKR_FAIL(h, OKR_E_NOT_TREE, "parent[%d] = %d out of range", i, h->parent[i]);
  // children CSR (increasing id) and reachability from the slack
  h->ch_off.assign(n + 1, 0);
  for (int i = 1; i < n; ++i) h->ch_off[h->parent[i] + 1]++;
  for (int i = 0; i < n; ++i) h->ch_off[i + 1] += h->ch_off[i];
  h->ch.assign(std::max(n - 1, 1), 0);
  {
    std::vector<int> fill(n, 0);
    for (int i = 1; i < n; ++i) h->ch[h->ch_off[h->parent[i]] + fill[h->parent[i]]++] = i;
  }
  // DFS preorder, subtree sizes, BFS levels
  h->pre.clear();
  h->pre.reserve(n);
  {
    std::vector<int> st{0};
    while (!st.empty()) {
      int v = st.back();
      st.pop_back();
      h->pre.push_back(v);
      for (int e = h->ch_off[v + 1] - 1; e >= h->ch_off[v]; --e) st.push_back(h->ch[e]);
      if ((int)h->pre.size() > n) break;
    }
  }
  if ((int)h->pre.size() != n) OKR_FAIL(h, OKR_E_NOT_TREE, "parent[] is not a tree rooted at node 0");
  h->pos.assign(n, 0);
  for (int q = 0; q < n; ++q) h->pos[h->pre[q]] = q;
  h->size.assign(n, 1);
  for (int q = n - 1; q >= 1; --q) h->size[h->parent[h->pre[q]]] += h->size[h->pre[q]];
  {
    std::vector<int> depth(n, 0);
    int dmax = 0;
    for (int q = 1; q < n; ++q) {
      int v = h->pre[q];
      depth[v] = depth[h->parent[v]] + 1;
      dmax = std::max(dmax, depth[v]);
    }
    h->nlev = dmax + 1;
    h->lvl_off.assign(h->nlev + 1, 0);
    for (int i = 0; i < n; ++i) h->lvl_off[depth[i] + 1]++;
    for (int d = 0; d < h->nlev; ++d) h->lvl_off[d + 1] += h->lvl_off[d];
    h->lvl_nodes.assign(n, 0);
    std::vector<int> fill(h->nlev, 0);
    for (int i = 0; i < n; ++i) h->lvl_nodes[h->lvl_off[depth[i]] + fill[depth[i]]++] = i;
  }
  // phases, eligibility, segments
  for (int i = 0; i < n; ++i) {
    if (h->phase[i] == 0 || h->phase[i] > 7) OKR_FAIL(h, OKR_E_PHASE, "node %d has phase mask %d", i, h->phase[i]);
    if (i > 0 && (h->phase[i] & ~h->phase[h->parent[i]]))
      OKR_FAIL(h, OKR_E_PHASE, "phases of node %d are not a subset of its parent's", i);
  }
  int nseg = 0;
  for (int i = 0; i < n; ++i) {
    const bool el = h->eligible[i] != 0;
    if (el && i == 0) OKR_FAIL(h, OKR_E_UNSUPPORTED, "the slack cannot be eligible");
    if (el && h->ch_off[i + 1] - h->ch_off[i] > 1)
      OKR_FAIL(h, OKR_E_UNSUPPORTED, "eligible node %d has more than one child", i);
    if (el != (h->segment[i] >= 0)) OKR_FAIL(h, OKR_E_ARG, "segment[%d] must be >= 0 exactly when eligible", i);
    nseg = std::max(nseg, h->segment[i] + 1);
  }
  h->seg_nodes.assign(nseg, {});
  for (int q = 0; q < n; ++q) {
    int v = h->pre[q];
    if (h->segment[v] >= 0) h->seg_nodes[h->segment[v]].push_back(v);
  }
  h->kmax = 0;
  h->ncand = 0;
  for (int g = 0; g < nseg; ++g) {
    const int k = (int)h->seg_nodes[g].size();
    if (k == 0) OKR_FAIL(h, OKR_E_ARG, "segment id %d is empty", g);
    if (k > kMaxK) OKR_FAIL(h, OKR_E_UNSUPPORTED, "segment %d has %d eligible nodes (max %d)", g, k, kMaxK);
    h->kmax = std::max(h->kmax, k);
    h->ncand += int64_t(1) << k;
  }
  h->nseg = nseg;
  // workspace layout
  const size_t c3 = (size_t)S * n * 3;
  h->zent_max = 3 * n;
  h->topo_ints = n /*parent*/ + (n + 1) /*ch_off*/ + std::max(n - 1, 1) /*ch*/ + (h->nlev + 1) + n /*levels*/ +
                 (n + 3) / 4 /*phase bytes*/;
  h->tab_ints_max = kMaxK * kChainInts + kMaxK * kMaxK + kMaxK * kSlotInts + n + kMaxPairs * kPairInts +
                    h->zent_max * 3 + (h->zent_max + 1) + (kMaxK + 1) + (n + 3 * n) + 3 * n + 64;
  Layout& L = h->L;
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = align256(off + bytes); return o; };
  L.z = take(sizeof(double2) * 9 * n);
  L.Vhat = take(sizeof(double2) * c3);
  L.Vcur = take(sizeof(double2) * c3);
  L.A = take(sizeof(double2) * c3);
  L.J = take(sizeof(double2) * c3);
  L.absV = take(sizeof(double) * c3);
  L.status = take(64);
  L.iters = take(sizeof(int) * S);
  L.topo = take(sizeof(int) * h->topo_ints);
  L.tab = take(sizeof(int) * h->tab_ints_max);
  L.P = take(sizeof(double2) * 3 * (size_t)S * kMaxPairs);
  L.srec = take(sizeof(TargetRec) * 3 * (size_t)S * kMaxK);
  L.headV = take(sizeof(double2) * 3 * (size_t)S * kMaxK);
  L.zrec = take(sizeof(TargetRec) * (size_t)S * h->zent_max);
  L.econst = take(sizeof(double) * S);
  {
    size_t most = 1;
    for (int k = 1; k <= h->kmax; ++k) {
      int spg;
      most = std::max(most, (size_t)snap_groups(k, S, &spg) << k);
    }
    L.res = take(sizeof(MaskScore) * most);
  }
  {
    const size_t nm = (size_t)1 << h->kmax, nt = (nm + 63) / 64;
    L.fin = take(sizeof(MaskScore) * nm);
    L.tiles = take(sizeof(TileRec) * nt);
    L.tickets = take(sizeof(int) * nt);
  }
  L.dec = take(sizeof(DevDecision) + 64);
  L.fin_int = take(sizeof(int) * (size_t)(4 * n + 1) + n);
  L.yeq = take(sizeof(double2) * 9 * n);
  L.Ykd = take(sizeof(double2) * 9 * n);
  L.Yko = take(sizeof(double2) * 9 * n);
  L.err = take(sizeof(double) * S);
  L.total = off;
  *workspace_bytes = L.total;
  if (sizes) {
    sizes->n_segments = nseg;
    sizes->k_max = h->kmax;
    sizes->n_candidates = h->ncand;
  }
  h->planned = true;
  return OKR_OK;
}

// ---------------------------------------------------- segment index tables --
namespace {

struct SegBuild {
  SegHdr hdr{};
  std::vector<int> tab;
  double flops = 0.0;  // algorithmic FP64 flops of scoring every mask over all snapshots
};

// Builds the index tables of segment g from the kept state (see the design doc,
// "scoring formulation").  Omega_g, chains, slot clusters, zone targets.
void build_segment(okr_handle* h, int g, SegBuild& B) {
  const int n = h->n;
  const std::vector<int>& par = h->parent;
  const std::vector<int>& seg = h->segment;
  const std::vector<int>& nodes = h->seg_nodes[g];
  const int k = (int)nodes.size();
  // chain tops
  std::vector<int> top(k);
  for (int j = 0; j < k; ++j) {
    int c = nodes[j];
    while (par[c] >= 0 && (seg[par[c]] == g || !h->kept[par[c]])) c = par[c];
    top[j] = c;
  }
  std::vector<int> tops(top);
  std::sort(tops.begin(), tops.end(), [&](int a, int b) { return h->pos[a] < h->pos[b]; });
  tops.erase(std::unique(tops.begin(), tops.end()), tops.end());
  const int nch = (int)tops.size();
  std::vector<std::vector<int>> cslots(nch);
  for (int j = 0; j < k; ++j) {
    const int c = int(std::lower_bound(tops.begin(), tops.end(), top[j],
                                       [&](int a, int b) { return h->pos[a] < h->pos[b]; }) - tops.begin());
    cslots[c].push_back(j);  // nodes are in preorder, so slots come top to bottom
  }
  // slot numbering: chain order, top to bottom
  std::vector<int> slot_node, slot_bit, slot_chain;
  std::vector<int> node_slot_local;  // position in chain (0-based)
  for (int c = 0; c < nch; ++c)
    for (int r = 0; r < (int)cslots[c].size(); ++r) {
      slot_node.push_back(nodes[cslots[c][r]]);
      slot_bit.push_back(cslots[c][r]);
      slot_chain.push_back(c);
    }
  auto slot_of_node = [&](int v) {
    for (int s = 0; s < k; ++s)
      if (slot_node[s] == v) return s;
    return -1;
  };
  // chain paths (top .. bottom slot), heads, outer chains
  std::vector<std::vector<int>> paths(nch);
  std::vector<int> head(nch), outer(nch), bottom_slot(nch), slot0(nch);
  {
    int s = 0;
    for (int c = 0; c < nch; ++c) {
      slot0[c] = s;
      s += (int)cslots[c].size();
      bottom_slot[c] = s - 1;
      int v = slot_node[s - 1];
      std::vector<int> p;
      while (true) {
        p.push_back(v);
        if (v == tops[c]) break;
        v = par[v];
      }
      std::reverse(p.begin(), p.end());
      paths[c] = p;
      head[c] = par[tops[c]];
    }
  }
  auto chain_of_bottom = [&](int v) {
    for (int c = 0; c < nch; ++c)
      if (slot_node[bottom_slot[c]] == v) return c;
    return -1;
  };
  auto first_g_above = [&](int v) {
    int u = par[v];
    while (u >= 0 && seg[u] != g) u = par[u];
    return u;
  };
  for (int c = 0; c < nch; ++c) {
    int u = head[c];
    while (u >= 0 && seg[u] != g) u = par[u];
    outer[c] = (u >= 0) ? chain_of_bottom(u) : -1;
  }
  // Omega_g = union of the subtrees of the chain tops (preorder ranges)
  std::vector<std::pair<int, int>> ranges;
  for (int c = 0; c < nch; ++c) ranges.push_back({h->pos[tops[c]], h->pos[tops[c]] + h->size[tops[c]]});
  std::sort(ranges.begin(), ranges.end());
  std::vector<std::pair<int, int>> merged;
  for (auto& r : ranges) {
    if (!merged.empty() && r.first < merged.back().second)
      merged.back().second = std::max(merged.back().second, r.second);
    else
      merged.push_back(r);
  }
  for (auto& r : merged)
    for (int q = r.first; q < r.second; ++q) h->in_omega[h->pre[q]] = 1;
  // clusters
  std::vector<std::vector<int>> smem(k);
  std::vector<int> zt_node, zt_anchor;
  std::vector<std::vector<int>> zmem;
  std::vector<int> hm;  // member, head, phase
  for (auto& r : merged)
    for (int q = r.first; q < r.second; ++q) {
      const int i = h->pre[q];
      const int t = h->sup[i];
      if (seg[t] == g) {
        smem[slot_of_node(t)].push_back(i);
      } else if (h->in_omega[t]) {
        if (t == i) {  // groups are created at t, which preorder visits before its members
          h->zidx[t] = (int)zt_node.size();
          zt_node.push_back(t);
          zmem.push_back({});
          zt_anchor.push_back(chain_of_bottom(first_g_above(t)));
        }
        zmem[h->zidx[t]].push_back(i);
      } else {
        hm.push_back(i);
        hm.push_back(t);
        hm.push_back(h->phase[i]);
      }
    }
  for (int t : zt_node) h->zidx[t] = -1;
  for (auto& r : merged)
    for (int q = r.first; q < r.second; ++q) h->in_omega[h->pre[q]] = 0;
  // zone entries sorted by (anchor chain, phase)
  struct ZE { int node, phase, chain, group; };
  std::vector<ZE> ze;
  for (int zi = 0; zi < (int)zt_node.size(); ++zi)
    for (int p = 0; p < 3; ++p)
      if (h->phase[zt_node[zi]] >> p & 1) ze.push_back({zt_node[zi], p, zt_anchor[zi], zi});
  std::stable_sort(ze.begin(), ze.end(), [](const ZE& a, const ZE& b) {
    return a.chain != b.chain ? a.chain < b.chain : a.phase < b.phase;
  });
  // nesting paths
  std::vector<std::vector<int>> nestp(nch);
  for (int c = 0; c < nch; ++c) {
    std::vector<int> p;
    for (int x = c; x >= 0; x = outer[x]) p.push_back(x);
    std::reverse(p.begin(), p.end());
    nestp[c] = p;
  }
  // ---- emit tables
  SegHdr& H = B.hdr;
  std::vector<int>& T = B.tab;
  T.clear();
  H = SegHdr{};
  H.k = k;
  H.nchains = nch;
  H.nslots = k;
  H.S = h->S;
  H.o_chain = (int)T.size();
  T.resize(T.size() + nch * kChainInts, 0);
  H.o_nest = (int)T.size();
  std::vector<int> nest_off(nch);
  for (int c = 0; c < nch; ++c) {
    nest_off[c] = (int)T.size() - H.o_nest;
    for (int x : nestp[c]) T.push_back(x);
  }
  H.o_path = (int)T.size();
  std::vector<int> path_off(nch);
  for (int c = 0; c < nch; ++c) {
    path_off[c] = (int)T.size() - H.o_path;
    for (int v : paths[c]) T.push_back(v);
  }
  H.o_slot = (int)T.size();
  T.resize(T.size() + k * kSlotInts, 0);
  H.o_pair = (int)T.size();
  int npairs = 0;
  std::vector<int> pairbase(k);
  for (int c = 0; c < nch; ++c) {
    const int j = (int)cslots[c].size();
    for (int r = 0; r < j; ++r) {
      const int s = slot0[c] + r;
      pairbase[s] = npairs;
      // position of slot r in the path
      const int rpos = (int)(std::find(paths[c].begin(), paths[c].end(), slot_node[s]) - paths[c].begin());
      for (int sup_i = 0; sup_i <= r; ++sup_i) {
        int from = 0;
        if (sup_i > 0) {
          const int sv = slot_node[slot0[c] + sup_i - 1];
          from = (int)(std::find(paths[c].begin(), paths[c].end(), sv) - paths[c].begin()) + 1;
        }
        T.push_back(slot_node[s]);
        T.push_back(from);
        T.push_back(rpos);
        T.push_back(path_off[c]);
        ++npairs;
      }
    }
  }
  H.npairs = npairs;
  H.o_zent = (int)T.size();
  for (auto& e : ze) {
    T.push_back(e.node);
    T.push_back(e.phase);
    T.push_back(e.chain);
  }
  H.nz = (int)ze.size();
  H.o_smemoff = (int)T.size();
  T.resize(T.size() + k + 1, 0);
  H.o_zmemoff = (int)T.size();
  T.resize(T.size() + H.nz + 1, 0);
  H.o_mem = (int)T.size();
  {
    int cnt = 0;
    for (int s = 0; s < k; ++s) {
      T[H.o_smemoff + s] = cnt;
      for (int v : smem[s]) { T.push_back(v); ++cnt; }
    }
    T[H.o_smemoff + k] = cnt;
    for (int q = 0; q < H.nz; ++q) {
      T[H.o_zmemoff + q] = cnt;
      for (int v : zmem[ze[q].group])
        if (h->phase[v] >> ze[q].phase & 1) { T.push_back(v); ++cnt; }
    }
    T[H.o_zmemoff + H.nz] = cnt;
    H.nmem = cnt;
  }
  H.o_h = (int)T.size();
  for (int v : hm) T.push_back(v);
  H.nh = (int)hm.size() / 3;
  H.total_ints = (int)T.size();
  // fill chain and slot records
  for (int c = 0; c < nch; ++c) {
    int* cr = &T[H.o_chain + c * kChainInts];
    cr[C_HEAD] = head[c];
    cr[C_NSLOT] = (int)cslots[c].size();
    cr[C_SLOT0] = slot0[c];
    cr[C_NEST_OFF] = nest_off[c];
    cr[C_NEST_LEN] = (int)nestp[c].size();
    cr[C_PATH_OFF] = path_off[c];
    cr[C_PATH_LEN] = (int)paths[c].size();
    cr[C_OUTER] = outer[c];
    for (int p = 0; p < 3; ++p) { cr[C_ZOFF0 + p] = 0; cr[C_ZCNT0 + p] = 0; }
  }
  for (int q = 0; q < H.nz; ++q) {
    int* cr = &T[H.o_chain + ze[q].chain * kChainInts];
    if (cr[C_ZCNT0 + ze[q].phase] == 0) cr[C_ZOFF0 + ze[q].phase] = q;
    cr[C_ZCNT0 + ze[q].phase]++;
  }
  double fl = 0.0;
  for (int s = 0; s < k; ++s) {
    int* sr = &T[H.o_slot + s * kSlotInts];
    sr[SL_NODE] = slot_node[s];
    sr[SL_BIT] = slot_bit[s];
    sr[SL_PHASE] = h->phase[slot_node[s]];
    sr[SL_PAIRBASE] = pairbase[s];
    sr[SL_PATHPOS] = (int)(std::find(paths[slot_chain[s]].begin(), paths[slot_chain[s]].end(), slot_node[s]) -
                           paths[slot_chain[s]].begin());
    sr[SL_CHAIN] = slot_chain[s];
    const int np = __builtin_popcount(h->phase[slot_node[s]]);
    // per mask: reduced -> 6 (voltage rise) + 4|phi| (cluster error); kept -> 14|phi|
    fl += 0.5 * (6.0 + 4.0 * np) + 0.5 * (14.0 * np);
  }
  fl += 14.0 * H.nz;
  B.flops = fl * double(int64_t(1) << k) * h->S;
}

// Every index the kernels follow, checked against its buffer before upload.
// Returns an empty string when consistent.
std::string validate_tables(const okr_handle* h, const SegBuild& B) {
  const SegHdr& H = B.hdr;
  const std::vector<int>& T = B.tab;
  const int n = h->n;
  char buf[160];
  auto bad = [&](const char* what, int a, int b) {
    snprintf(buf, sizeof buf, "internal table check failed: %s (%d, %d)", what, a, b);
    return std::string(buf);
  };
  if (H.k < 1 || H.k > kMaxK || H.nslots != H.k) return bad("k", H.k, H.nslots);
  if (H.nchains < 1 || H.nchains > H.k) return bad("nchains", H.nchains, H.k);
  if (H.npairs < 1 || H.npairs > kMaxPairs) return bad("npairs", H.npairs, kMaxPairs);
  if (H.nz < 0 || H.nz > h->zent_max) return bad("nz", H.nz, h->zent_max);
  if (H.total_ints != (int)T.size() || H.total_ints > h->tab_ints_max) return bad("size", H.total_ints, (int)T.size());
  auto in = [&](int o, int cnt) { return o >= 0 && cnt >= 0 && o + cnt <= H.total_ints; };
  if (!in(H.o_chain, H.nchains * kChainInts) || !in(H.o_slot, H.k * kSlotInts) ||
      !in(H.o_pair, H.npairs * kPairInts) || !in(H.o_zent, H.nz * 3) || !in(H.o_zmemoff, H.nz + 1) ||
      !in(H.o_smemoff, H.k + 1) || !in(H.o_mem, H.nmem) || !in(H.o_h, H.nh * 3))
    return bad("offsets", H.total_ints, 0);
  int slots_seen = 0;
  for (int c = 0; c < H.nchains; ++c) {
    const int* cr = &T[H.o_chain + c * kChainInts];
    if (cr[C_HEAD] < 0 || cr[C_HEAD] >= n) return bad("head", c, cr[C_HEAD]);
    if (cr[C_NSLOT] < 1 || cr[C_SLOT0] != slots_seen) return bad("chain slots", c, cr[C_NSLOT]);
    slots_seen += cr[C_NSLOT];
    if (cr[C_OUTER] >= c) return bad("outer", c, cr[C_OUTER]);
    if (cr[C_NEST_LEN] < 1 || !in(H.o_nest + cr[C_NEST_OFF], cr[C_NEST_LEN])) return bad("nest", c, cr[C_NEST_LEN]);
    for (int q = 0; q < cr[C_NEST_LEN]; ++q) {
      const int x = T[H.o_nest + cr[C_NEST_OFF] + q];
      if (x < 0 || x > c || (q + 1 == cr[C_NEST_LEN] && x != c)) return bad("nest entry", c, x);
    }
    if (!in(H.o_path + cr[C_PATH_OFF], cr[C_PATH_LEN])) return bad("path", c, cr[C_PATH_LEN]);
    for (int p = 0; p < 3; ++p)
      if (cr[C_ZOFF0 + p] < 0 || cr[C_ZCNT0 + p] < 0 || cr[C_ZOFF0 + p] + cr[C_ZCNT0 + p] > H.nz)
        return bad("zone range", c, p);
    int pb = -1;
    for (int r = 0; r < cr[C_NSLOT]; ++r) {
      const int* sr = &T[H.o_slot + (cr[C_SLOT0] + r) * kSlotInts];
      if (sr[SL_NODE] < 0 || sr[SL_NODE] >= n) return bad("slot node", c, r);
      if (sr[SL_BIT] < 0 || sr[SL_BIT] >= H.k) return bad("slot bit", c, r);
      if (sr[SL_PHASE] < 1 || sr[SL_PHASE] > 7) return bad("slot phase", c, r);
      // pairs (super 0..r) of slot r: pairbase + r must stay inside the table
      if (sr[SL_PAIRBASE] < 0 || sr[SL_PAIRBASE] + r >= H.npairs || sr[SL_PAIRBASE] <= pb) return bad("pairbase", c, r);
      pb = sr[SL_PAIRBASE];
    }
  }
  if (slots_seen != H.k) return bad("slot count", slots_seen, H.k);
  for (int q = 0; q < H.npairs; ++q) {
    const int* pr = &T[H.o_pair + q * kPairInts];
    if (pr[PR_RNODE] < 0 || pr[PR_RNODE] >= n) return bad("pair node", q, pr[PR_RNODE]);
    if (pr[PR_FROM] < 0 || pr[PR_FROM] > pr[PR_TO]) return bad("pair range", q, pr[PR_FROM]);
    if (!in(H.o_path + pr[PR_PATHOFF], pr[PR_TO] + 1)) return bad("pair path", q, pr[PR_TO]);
    for (int x = pr[PR_FROM]; x <= pr[PR_TO]; ++x) {
      const int v = T[H.o_path + pr[PR_PATHOFF] + x];
      if (v < 0 || v >= n) return bad("path node", q, v);
    }
  }
  for (int q = 0; q < H.nz; ++q) {
    const int* ze = &T[H.o_zent + q * 3];
    if (ze[0] < 0 || ze[0] >= n || ze[1] < 0 || ze[1] > 2 || ze[2] < 0 || ze[2] >= H.nchains)
      return bad("zone entry", q, ze[0]);
  }
  auto csr_ok = [&](int o, int cnt) {
    if (T[o] != (o == H.o_smemoff ? 0 : T[H.o_smemoff + H.k])) return false;
    for (int q = 0; q < cnt; ++q)
      if (T[o + q + 1] < T[o + q] || T[o + q + 1] > H.nmem) return false;
    return true;
  };
  if (!csr_ok(H.o_smemoff, H.k) || !csr_ok(H.o_zmemoff, H.nz)) return bad("member offsets", H.nmem, 0);
  for (int q = 0; q < H.nmem; ++q)
    if (T[H.o_mem + q] < 0 || T[H.o_mem + q] >= n) return bad("member", q, T[H.o_mem + q]);
  for (int q = 0; q < H.nh; ++q) {
    const int* hq = &T[H.o_h + q * 3];
    if (hq[0] < 0 || hq[0] >= n || hq[1] < 0 || hq[1] >= n) return bad("head member", q, hq[0]);
  }
  return std::string();
}

}  // namespace

// ------------------------------------------------------------ the search --
extern "C" int okr_reduce_feeder(okr_handle* h, const okr_yblocks* Y, const okr_topology* topo,
                                 const okr_loads* loads, const okr_margins* mg, void* d_workspace,
                                 size_t workspace_bytes, okr_result* out) {
  using clk = std::chrono::steady_clock;
  if (!h) return OKR_E_ARG;
  if (!h->planned) OKR_FAIL(h, OKR_E_ARG, "okr_plan() must succeed first");
  if (!Y || !topo || !loads || !mg || !out || !Y->Y_diag || !Y->Y_off || !loads->V0)
    OKR_FAIL(h, OKR_E_ARG, "null argument");
  if (!out->super || !out->kept_parent || (!out->seg && h->nseg > 0))
    OKR_FAIL(h, OKR_E_ARG, "result buffers super, kept_parent and seg are required");
  if (topo->n != h->n || loads->S != h->S) OKR_FAIL(h, OKR_E_ARG, "topology or S differs from the plan");
  if (!d_workspace || workspace_bytes < h->L.total)
    OKR_FAIL(h, OKR_E_WORKSPACE, "workspace %zu bytes < planned %zu", workspace_bytes, h->L.total);
  const bool vhat_given = (mg->flags & OKR_FLAG_VHAT_GIVEN) != 0;
  if (!vhat_given && !loads->S_load) OKR_FAIL(h, OKR_E_ARG, "S_load is required");
  if (!loads->S_load) OKR_FAIL(h, OKR_E_ARG, "S_load is required (load currents)");
  if (vhat_given && !loads->Vhat) OKR_FAIL(h, OKR_E_ARG, "OKR_FLAG_VHAT_GIVEN without Vhat");
  if (mg->precision != OKR_PRECISION_FP64 && mg->precision != OKR_PRECISION_MIXED)
    OKR_FAIL(h, OKR_E_ARG, "unknown precision %d", mg->precision);
  if (!(mg->v_min < mg->v_max) || !(mg->e_bar >= 0) || !(mg->tie_tol >= 0) || !(mg->amb_tol >= 0))
    OKR_FAIL(h, OKR_E_ARG, "bad margins");
  const bool timing = (mg->flags & OKR_FLAG_TIMING) != 0;
  const bool dump = (mg->flags & OKR_FLAG_DUMP_SCORES) != 0;
  const int n = h->n, S = h->S;
  const Layout& L = h->L;
  char* ws = static_cast<char*>(d_workspace);
  auto dptr = [&](size_t o) { return static_cast<void*>(ws + o); };
  double2* z = (double2*)dptr(L.z);
  double2* Vhat = (double2*)dptr(L.Vhat);
  double2* Vcur = (double2*)dptr(L.Vcur);
  double2* A = (double2*)dptr(L.A);
  double2* J = (double2*)dptr(L.J);
  double* absV = (double*)dptr(L.absV);
  int* status = (int*)dptr(L.status);
  int* iters = (int*)dptr(L.iters);
  int* dtopo = (int*)dptr(L.topo);
  int* dtab = (int*)dptr(L.tab);
  double2* P = (double2*)dptr(L.P);
  TargetRec* srec = (TargetRec*)dptr(L.srec);
  double2* headV = (double2*)dptr(L.headV);
  TargetRec* zrec = (TargetRec*)dptr(L.zrec);
  double* econst = (double*)dptr(L.econst);
  MaskScore* res = (MaskScore*)dptr(L.res);
  MaskScore* mfin = (MaskScore*)dptr(L.fin);
  TileRec* tiles = (TileRec*)dptr(L.tiles);
  int* tickets = (int*)dptr(L.tickets);
  DevDecision* ddec = (DevDecision*)dptr(L.dec);
  int* fin = (int*)dptr(L.fin_int);
  double2* yeq = (double2*)dptr(L.yeq);
  double2* Ykd = (double2*)dptr(L.Ykd);
  double2* Yko = (double2*)dptr(L.Yko);
  double* derr = (double*)dptr(L.err);
  hipStream_t st = h->stream;
  const auto t0 = clk::now();
  // pinned staging for tables and the decision record (host memory only)
  const size_t need = sizeof(int) * (size_t)std::max(h->tab_ints_max, std::max(h->topo_ints, 4 * n + 1 + n)) + 1024;
  if (h->h_tab_bytes < need) {
    if (h->h_tab) (void)hipHostFree(h->h_tab);
    h->h_tab = nullptr;
    h->h_tab_bytes = 0;
    OKR_HIP(h, hipHostMalloc((void**)&h->h_tab, need, hipHostMallocDefault));
    h->h_tab_bytes = need;
  }
  if (!h->h_dec) OKR_HIP(h, hipHostMalloc((void**)&h->h_dec, sizeof(DevDecision), hipHostMallocDefault));
  if (!h->ev0) OKR_HIP(h, hipEventCreate(&h->ev0));
  if (!h->ev1) OKR_HIP(h, hipEventCreate(&h->ev1));

  // ---- topology upload: parent, ch_off, ch, lvl_off, lvl_nodes, phase bytes
  int* ht = h->h_tab;
  int o = 0;
  const int o_par = o; std::memcpy(ht + o, h->parent.data(), sizeof(int) * n); o += n;
  const int o_choff = o; std::memcpy(ht + o, h->ch_off.data(), sizeof(int) * (n + 1)); o += n + 1;
  const int o_ch = o; std::memcpy(ht + o, h->ch.data(), sizeof(int) * h->ch.size()); o += (int)h->ch.size();
  const int o_loff = o; std::memcpy(ht + o, h->lvl_off.data(), sizeof(int) * (h->nlev + 1)); o += h->nlev + 1;
  const int o_lnod = o; std::memcpy(ht + o, h->lvl_nodes.data(), sizeof(int) * n); o += n;
  const int o_ph = o; std::memcpy(ht + o, h->phase.data(), n); o += (n + 3) / 4;
  OKR_HIP(h, hipMemcpyAsync(dtopo, ht, sizeof(int) * o, hipMemcpyHostToDevice, st));
  OKR_HIP(h, hipMemsetAsync(status, 0, 64, st));
  OKR_HIP(h, hipMemsetAsync(tickets, 0, sizeof(int) * ((((size_t)1 << h->kmax) + 63) / 64), st));
  const int* d_par = dtopo + o_par;
  const int* d_choff = dtopo + o_choff;
  const int* d_ch = dtopo + o_ch;
  const uint8_t* d_ph = (const uint8_t*)(dtopo + o_ph);

  hipLaunchKernelGGL(k_branch_z, dim3((n + 127) / 128), dim3(128), 0, st, n, d_par, d_ph, d_choff, d_ch,
                     (const double2*)Y->Y_diag, (const double2*)Y->Y_off, z, status);
  OKR_HIP(h, hipGetLastError());
  // ---- a2: scenario library
  const double2* V0 = (const double2*)loads->V0;
  if (vhat_given) {
    OKR_HIP(h, hipMemcpyAsync(Vhat, loads->Vhat, sizeof(double2) * (size_t)S * n * 3, hipMemcpyDeviceToDevice, st));
    const size_t tot = (size_t)S * n * 3;
    hipLaunchKernelGGL(k_from_vhat, dim3((tot + 255) / 256), dim3(256), 0, st, n, S, d_ph,
                       (const double2*)loads->S_load, Vhat, mg->v_min, mg->v_max, A, absV, status);
  } else {
    hipLaunchKernelGGL(k_powerflow, dim3(S), dim3(256), 0, st, n, d_par, d_ph, dtopo + o_loff, dtopo + o_lnod,
                       h->nlev, d_choff, d_ch, z, (const double2*)loads->S_load, V0[0], V0[1], V0[2],
                       mg->pf_tol > 0 ? mg->pf_tol : 1e-13, mg->pf_maxit > 0 ? mg->pf_maxit : 100, mg->v_min,
                       mg->v_max, Vhat, J, A, absV, iters, status);
  }
  OKR_HIP(h, hipGetLastError());
  OKR_HIP(h, hipMemcpyAsync(Vcur, Vhat, sizeof(double2) * (size_t)S * n * 3, hipMemcpyDeviceToDevice, st));
  int hstatus = 0;
  OKR_HIP(h, hipMemcpyAsync(h->h_dec, status, sizeof(int), hipMemcpyDeviceToHost, st));
  OKR_HIP(h, hipStreamSynchronize(st));
  std::memcpy(&hstatus, h->h_dec, sizeof(int));
  if (hstatus & 1) OKR_FAIL(h, OKR_E_SINGULAR, "a present-phase branch block is singular");
  if (hstatus & 2) OKR_FAIL(h, OKR_E_PHASE, "nonzero admittance entries on absent phases");
  if (hstatus & (4 | 8)) OKR_FAIL(h, OKR_E_UNSUPPORTED, "admittance blocks asymmetric or with shunts");
  if (hstatus & 16) OKR_FAIL(h, OKR_E_PF_DIVERGED, "load flow did not converge");
  const bool base_out = (hstatus & 32) != 0;
  const auto t1 = clk::now();

  // ---- a3-a9: segments in order against the cumulative state
  h->kept.assign(n, 1);
  h->in_omega.assign(n, 0);
  h->zidx.assign(n, -1);
  h->sup.resize(n);
  for (int i = 0; i < n; ++i) h->sup[i] = i;
  if (dump) {
    h->dump_e.assign(h->nseg, {});
    h->dump_s.assign(h->nseg, {});
    h->dump_k.assign(h->nseg, 0);
  }
  out->score_kernel_ms = 0.0;
  out->algorithmic_flops = 0.0;
  out->n_score_launches = 0;
  out->warnings = base_out ? OKR_W_BASE_OUT_OF_BAND : 0;
  SegBuild B;
  SelParams sp;
  sp.e_bar = mg->e_bar;
  sp.vmin = mg->v_min;
  sp.vmax = mg->v_max;
  sp.tie = mg->tie_tol;
  sp.amb = mg->amb_tol;
  for (int g = 0; g < h->nseg; ++g) {
    okr_segment_result& R = out->seg[g];
    std::memset(&R, 0, sizeof R);
    R.segment = g;
    R.k = (int)h->seg_nodes[g].size();
    if (base_out) continue;
    build_segment(h, g, B);
    const SegHdr& H = B.hdr;
    {
      const std::string why = validate_tables(h, B);
      if (!why.empty()) OKR_FAIL(h, OKR_E_ARG, "segment %d: %s", g, why.c_str());
    }
    std::memcpy(h->h_tab, B.tab.data(), sizeof(int) * H.total_ints);
    OKR_HIP(h, hipMemcpyAsync(dtab, h->h_tab, sizeof(int) * H.total_ints, hipMemcpyHostToDevice, st));
    {
      const int items = std::max(std::max(S * H.npairs, S * H.nslots * 3), std::max(S * H.nchains, std::max(S * H.nz, S)));
      hipLaunchKernelGGL(k_seg_fill, dim3((items + 127) / 128, 5), dim3(128), 0, st, dtab, H, n, z, Vcur, A, absV,
                         P, srec, headV, zrec, econst);
      OKR_HIP(h, hipGetLastError());
    }
    const uint32_t nmask = 1u << H.k;
    const int mblocks = (int)((nmask + kScoreBlock - 1) / kScoreBlock);
    int spg;
    const int SG = snap_groups(H.k, S, &spg);
    if (timing) OKR_HIP(h, hipEventRecord(h->ev0, st));
    hipLaunchKernelGGL(k_score_fp64, dim3(mblocks, SG), dim3(kScoreBlock), 0, st, dtab, H, P, srec, headV, zrec,
                       econst, spg, SG, sp, res, mfin, tiles, tickets);
    OKR_HIP(h, hipGetLastError());
    if (timing) OKR_HIP(h, hipEventRecord(h->ev1, st));
    hipLaunchKernelGGL(k_argmin, dim3(1), dim3(1024), 0, st, mfin, tiles, H.k, sp, ddec);
    OKR_HIP(h, hipGetLastError());
    hipLaunchKernelGGL(k_apply, dim3(S), dim3(64), 0, st, dtab, H, n, ddec, P, srec, zrec, Vcur, A);
    OKR_HIP(h, hipGetLastError());
    OKR_HIP(h, hipMemcpyAsync(h->h_dec, ddec, sizeof(DevDecision), hipMemcpyDeviceToHost, st));
    if (dump) {
      h->dump_e[g].resize(nmask);
      h->dump_s[g].resize(nmask);
      h->dump_k[g] = H.k;
      std::vector<MaskScore> tmp(nmask);
      OKR_HIP(h, hipMemcpyAsync(tmp.data(), mfin, sizeof(MaskScore) * nmask, hipMemcpyDeviceToHost, st));
      OKR_HIP(h, hipStreamSynchronize(st));
      for (uint32_t m = 0; m < nmask; ++m) { h->dump_e[g][m] = tmp[m].e; h->dump_s[g][m] = tmp[m].slack; }
    }
    OKR_HIP(h, hipStreamSynchronize(st));
    const DevDecision d = *h->h_dec;
    R.mask = d.mask;
    R.popcount = d.popcount;
    R.e_loc = d.e_loc;
    R.e_min = d.e_min;
    R.ambiguous = d.ambiguous;
    R.n_scored = (int)nmask;
    R.flops = B.flops;
    if (timing) {
      float ms = 0.f;
      OKR_HIP(h, hipEventElapsedTime(&ms, h->ev0, h->ev1));
      R.score_ms = ms;
      out->score_kernel_ms += ms;
    }
    out->algorithmic_flops += B.flops;
    out->n_score_launches++;
    // cumulative kept state and super-nodes over Omega_g
    const std::vector<int>& nodes = h->seg_nodes[g];
    for (int j = 0; j < H.k; ++j)
      if (d.mask >> j & 1u) h->kept[nodes[j]] = 0;
    if (d.mask) {
      for (int j = 0; j < H.k; ++j) {
        int c = nodes[j];
        while (h->parent[c] >= 0 && (h->segment[h->parent[c]] == g || !h->kept[h->parent[c]])) c = h->parent[c];
        for (int q = h->pos[c]; q < h->pos[c] + h->size[c]; ++q) {
          const int v = h->pre[q];
          h->sup[v] = h->kept[v] ? v : h->sup[h->parent[v]];
        }
      }
    }
  }
  const auto t2 = clk::now();

  // ---- final outputs: aggregation map, Y_Kron blocks, errors
  std::vector<int> kp(n, -1), kc_off(n + 1, 0), kc;
  int nk = 0;
  for (int i = 0; i < n; ++i) {
    out->super[i] = h->sup[i];
    if (h->kept[i]) {
      ++nk;
      if (i > 0) kp[i] = h->sup[h->parent[i]];
    }
    out->kept_parent[i] = kp[i];
  }
  for (int i = 1; i < n; ++i)
    if (kp[i] >= 0) kc_off[kp[i] + 1]++;
  for (int i = 0; i < n; ++i) kc_off[i + 1] += kc_off[i];
  kc.assign(std::max(kc_off[n], 1), 0);
  {
    std::vector<int> fill(n, 0);
    for (int i = 1; i < n; ++i)
      if (kp[i] >= 0) kc[kc_off[kp[i]] + fill[kp[i]]++] = i;
  }
  out->n_kept = nk;
  int* hf = h->h_tab;
  std::memcpy(hf, h->sup.data(), sizeof(int) * n);
  std::memcpy(hf + n, kp.data(), sizeof(int) * n);
  std::memcpy(hf + 2 * n, kc_off.data(), sizeof(int) * (n + 1));
  std::memcpy(hf + 3 * n + 1, kc.data(), sizeof(int) * std::max(n - 1, 1));
  uint8_t* hk = (uint8_t*)(hf + 4 * n + 1);
  std::memcpy(hk, h->kept.data(), n);
  OKR_HIP(h, hipMemcpyAsync(fin, hf, sizeof(int) * (4 * n + 1) + n, hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(k_kron_yeq, dim3((n + 127) / 128), dim3(128), 0, st, n, d_par, d_ph, fin + n, z, yeq, Yko,
                     status);
  hipLaunchKernelGGL(k_kron_diag, dim3((n + 127) / 128), dim3(128), 0, st, n, (const uint8_t*)(fin + 4 * n + 1),
                     fin + n, fin + 2 * n, fin + 3 * n + 1, yeq, Ykd);
  hipLaunchKernelGGL(k_final_err, dim3(S), dim3(256), 0, st, n, d_ph, fin, Vcur, absV, derr);
  OKR_HIP(h, hipGetLastError());
  if (out->Yk_diag) OKR_HIP(h, hipMemcpyAsync(out->Yk_diag, Ykd, sizeof(double2) * 9 * n, hipMemcpyDeviceToHost, st));
  if (out->Yk_off) OKR_HIP(h, hipMemcpyAsync(out->Yk_off, Yko, sizeof(double2) * 9 * n, hipMemcpyDeviceToHost, st));
  if (out->err_per_snapshot)
    OKR_HIP(h, hipMemcpyAsync(out->err_per_snapshot, derr, sizeof(double) * S, hipMemcpyDeviceToHost, st));
  if (out->Vhat) OKR_HIP(h, hipMemcpyAsync(out->Vhat, Vhat, sizeof(double2) * (size_t)S * n * 3, hipMemcpyDeviceToHost, st));
  std::vector<int> hiters(S, 0);
  if (!vhat_given) OKR_HIP(h, hipMemcpyAsync(hiters.data(), iters, sizeof(int) * S, hipMemcpyDeviceToHost, st));
  OKR_HIP(h, hipMemcpyAsync(h->h_dec, status, sizeof(int), hipMemcpyDeviceToHost, st));
  OKR_HIP(h, hipStreamSynchronize(st));
  std::memcpy(&hstatus, h->h_dec, sizeof(int));
  if (hstatus & 1) OKR_FAIL(h, OKR_E_SINGULAR, "a Kron-reduced branch block is singular");
  out->pf_iterations = hiters.empty() ? 0 : *std::max_element(hiters.begin(), hiters.end());
  out->max_err = 0.0;
  if (out->err_per_snapshot)
    for (int l = 0; l < S; ++l) out->max_err = std::max(out->max_err, out->err_per_snapshot[l]);
  const auto t3 = clk::now();
  auto ms = [](clk::duration d) { return std::chrono::duration<double, std::milli>(d).count(); };
  out->t_setup_ms = 0.0;
  out->t_pf_ms = ms(t1 - t0);
  out->t_search_ms = ms(t2 - t1);
  out->t_final_ms = ms(t3 - t2);
  return base_out ? OKR_W_BASE_OUT_OF_BAND : OKR_OK;
}

extern "C" int okr_dump_scores(okr_handle* h, int32_t segment, double* e, double* slack, int32_t* k) {
  if (!h) return OKR_E_ARG;
  if (segment < 0 || segment >= (int)h->dump_e.size() || h->dump_e[segment].empty())
    OKR_FAIL(h, OKR_E_ARG, "no scores kept for segment %d (set OKR_FLAG_DUMP_SCORES)", segment);
  const size_t nm = h->dump_e[segment].size();
  if (e) std::memcpy(e, h->dump_e[segment].data(), sizeof(double) * nm);
  if (slack) std::memcpy(slack, h->dump_s[segment].data(), sizeof(double) * nm);
  if (k) *k = h->dump_k[segment];
  return OKR_OK;
}

// Self-test of the scoring kernel's square root (device pointers, n values).
extern "C" int okr_selftest_sqrt(const double* d_x, double* d_y, int n, void* stream) {
  if (!d_x || !d_y || n < 0) return OKR_E_ARG;
  hipLaunchKernelGGL(k_sqrt_selftest, dim3((n + 255) / 256), dim3(256), 0, static_cast<hipStream_t>(stream), d_x,
                     d_y, n);
  return hipGetLastError() == hipSuccess ? OKR_OK : OKR_E_HIP;
}
