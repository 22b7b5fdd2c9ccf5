// Host side of the C ABI: validation, DFS renumbering and the static tables
// of the plan, workspace layout, and the launch sequence of a search (one
// stream of kernels, optionally replayed as a captured hipGraph; one host
// synchronisation at the end).
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/okr.h"
#include "okr_internal.h"

namespace okr {
// kernels (okr_kernels.hip, okr_build.hip)
__global__ void k_branch_z(int, const int*, const uint8_t*, const int*, const int*, const double2*, const double2*,
                           double2*, int*);
__global__ void k_powerflow(int, const int*, const uint8_t*, const int*, const int*, int, const int*, const int*,
                            const double2*, const double2*, double2, double2, double2, double, int, double, double,
                            double2*, double2*, double2*, double*, int*, int*);
__global__ void k_powerflow_lds(int, const int*, const uint8_t*, const int*, const int*, int, const int*, const int*,
                                const double2*, const double2*, double2, double2, double2, double, int, double, double,
                                double2*, double2*, double2*, double*, int*, int*);
__global__ void k_powerflow_bfs(int, const uint8_t*, const int*, const int*, int, const int*, const int*,
                                const double2*, const double2*, double2, double2, double2, double, int, double, double,
                                double2*, double2*, double2*, double*, int*, int*);
__global__ void k_from_vhat(int, int, const uint8_t*, const double2*, const double2*, double, double, double2*,
                            double*, int*);
__global__ void k_build_struct(Topo, State, const int*, size_t, int, SegHdr*, int*, int, int*);
__global__ void k_zroot(int, const int*, const int*, const int*, int, const double2*, double2*);
__global__ void k_build_values(const SegHdr*, const int*, size_t, const int*, int, const double2*, const double2*,
                               const double2*, double2*, TargetRec*, double2*, TargetRec*, double*);
__global__ void k_build_members(const SegHdr*, const int*, size_t, const int*, Topo, State, const double2*,
                                const double*, TargetRec*, TargetRec*, double*);
template <int M>
__global__ void k_score_fp64(const SegHdr*, const int*, size_t, const int*, const double2*, const TargetRec*,
                           const double2*, const TargetRec*, const double*, int, int, int, int, int, int, SelParams,
                           MaskScore*, MaskScore*, TileRec*, int*, const int*, int);
__global__ void k_terms_init(const SegHdr*, const int*, size_t, int, const int*, int, const double*,
                             unsigned long long*, unsigned long long*);
__global__ void k_chain_terms(const SegHdr*, const int*, size_t, int, const int*, const double2*, const TargetRec*,
                              const double2*, const TargetRec*, const double*, const uint32_t*, const int*, int, int,
                              int, unsigned long long*, unsigned long long*);
__global__ void k_list_finish(const int*, const unsigned long long*, int, SelParams, MaskScore*, size_t);
__global__ void k_surr_rank(const SegHdr*, int, const int*, const float*, const float*, const SurrSlot*, const double*,
                            const uint32_t*, int, const __bf16*, const __bf16*, const float*, float, uint32_t*,
                            const int*, int);
__global__ void k_fac_combine(const SegHdr*, const int*, size_t, const int*, const unsigned long long*,
                              const unsigned long long*, SelParams, MaskScore*, TileRec*);
__global__ void k_argmin(const SegHdr*, const int*, size_t, const MaskScore*, const TileRec*, SelParams, const int*,
                         DevDecision*, const int*);
__global__ void k_apply(const SegHdr*, const int*, size_t, const int*, Topo, State, const DevDecision*,
                        const double2*, const TargetRec*, const TargetRec*, double2*, double2*);
__global__ void k_init_state(int, State, int*, int, int*, int, int, size_t);
__global__ void k_copy2(const double2*, double2*, size_t);
__global__ void k_final_err(int, const uint8_t*, const int*, const double2*, const double*, double*);
__global__ void k_kron_yeq(Topo, State, const double2*, double2*, double2*, int*, int*);
__global__ void k_kron_diag(Topo, State, const double2*, double2*);
__global__ void k_sqrt_selftest(const double*, double*, int);
__global__ void k_build_mixed(const SegHdr*, const int*, size_t, const int*, int, const double2*, const double2*,
                              const TargetRec*, const double2*, const TargetRec*, double, double, Pair32*, Rec32*,
                              Head32*, Rec32*);
template <int M>
__global__ void k_score_fp32(const SegHdr*, const int*, size_t, const int*, const Pair32*, const Rec32*, const Head32*,
                             const Rec32*, const double*, int, int, SelParams, MaskScore32*, MaskScore32*, TileRec32*,
                             int*);
__global__ void k_mixed_select_a(const SegHdr*, const int*, size_t, const MaskScore32*, const TileRec32*, SelParams,
                                 const int*, MixedState*, uint32_t*, int*);
__global__ void k_mixed_select_b(const SegHdr*, const int*, size_t, const MaskScore32*, const TileRec32*, SelParams,
                                 const int*, MixedState*, const uint32_t*, const int*, const MaskScore*, uint32_t*,
                                 int*);
__global__ void k_mixed_final(const SegHdr*, const int*, size_t, SelParams, const int*, MixedState*,
                              const MaskScore32*, const uint32_t*, const int*, const MaskScore*, const uint32_t*,
                              const int*, const MaskScore*, DevDecision*, int*);
__global__ void k_surr_tables(const SegHdr*, int, const int*, int, const double2*, const double2*, const double2*,
                              const TargetRec*, float*, float*, SurrSlot*);
__global__ void k_surr_features(const SegHdr*, int, const int*, const float*, const float*, const SurrSlot*,
                                const double*, const uint32_t*, int, int, float*, __bf16*, const int*, int);
__global__ void k_level_masks(int, int, int, int, uint32_t*);
__global__ void k_surr_stage(const SegHdr*, int, const uint32_t*, int, int, int*);
__global__ void k_surr_target(const SegHdr*, int, const MaskScore*, float*);
template <int EPI>
__global__ void k_gemm_nt(const __bf16*, int, const __bf16*, int, int, float*, int, const float*, float*, __bf16*,
                          __bf16*, int, const float*, float*, const int*, int);
__global__ void k_rowdot_finish(const float*, int, int, const float*, float*, const int*, int);
__global__ void k_batch_cast(const float*, int, __bf16*, __bf16*);
__global__ void k_loss_dy(const float*, const float*, int, float*, float*);
__global__ void k_dz2(const float*, const float*, const float*, int, __bf16*, __bf16*);
__global__ void k_dz1(const float*, const float*, int, __bf16*);
__global__ void k_colsums_part(const float*, const float*, const float*, const float*, const float*, int, float*);
__global__ void k_colsums_final(const float*, int, float*, float*, float*, float*);
__global__ void k_copy_cols(const float*, int, float*, int, int);
__global__ void k_sum_splits(const float*, int, int, float*);
__global__ void k_adam(float*, const float*, float*, float*, int, float, float, float);
__global__ void k_refresh_weights(const float*, __bf16*, __bf16*, __bf16*);
__global__ void k_topk(const SegHdr*, int, const uint32_t*, const uint32_t*, int, int, const int*, uint32_t*, int*,
                       const int*, int);
__global__ void k_surr_decide(const SegHdr*, int, SelParams, const int*, const uint32_t*, const int*,
                              const MaskScore*, DevDecision*, int*);
__global__ void k_zero_f32(float*, int);
__global__ void k_smice_prep(const SegHdr*, const int*, size_t, const int*, Topo, State, int*, double*, int);
__global__ void k_smice_hconst(const SegHdr*, const int*, size_t, Topo, State, const double2*, const double*,
                               const int*, double*, int);
__global__ void k_smice_score(const SegHdr*, const int*, size_t, const int*, const double2*, const TargetRec*,
                              const double2*, const TargetRec*, const int*, const double*, const MaskScore*,
                              const TileRec*, const DevDecision*, SelParams, double*, double*);
__global__ void k_smice_argmin(const SegHdr*, const int*, size_t, const MaskScore*, const TileRec*, const double*,
                               const double*, double, DevDecision*);
}  // namespace okr

using namespace okr;

namespace {

constexpr int kMaxSnapGroups = 32;
constexpr int kMaxLanes = 8;      // segments per chunk (each needs a scratch block)
constexpr int kDefaultLanes = 8;
constexpr int kStatusInts = 16;
constexpr double kMixedDelta = 1e-8;  // bound on |e32 - e64| used by the shortlist
constexpr double kSmiceTol = 1e-9;    // default SMICE tie window
// Dynamic LDS of the load flow with its iterates in shared memory (0: too
// large, the global-memory form runs).
constexpr size_t kPfLdsMax = 150 * 1024;
size_t pf_lds_bytes(int n, int nlev) {
  const size_t b = (size_t)n * 3 * 2 * sizeof(double2) + sizeof(int) * ((size_t)4 * n + nlev + 2) + (size_t)n;
  return b <= kPfLdsMax ? b : 0;
}
// Dynamic LDS of the breadth-first form (iterates in global memory, the
// queue tables in LDS as 16-bit positions; 0: not usable, the node-order
// global form runs).
size_t pf_bfs_lds_bytes(int n, int nlev) {
  const size_t b = sizeof(int) * ((size_t)nlev + 1) + sizeof(uint16_t) * ((size_t)3 * n + 1) + (size_t)n;
  return (n < 65536 && b <= kPfLdsMax) ? b : 0;
}
constexpr int kSmiceThreadsHost = 128;  // masks per block of the SMICE scoring

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Snapshot groups of the scoring launches (per-mask FP64, FP32 screen) for
// segments of k nodes, each group a contiguous run of snapshots: a
// group of about 8 snapshots for segments of up to 9 nodes, 16 up to 12, 32
// up to 16 and 64 above, scaled by (S / 96)^0.37 for S above 96 (a fit to
// the autotuner's picks on MI355X on the 1000-, 6000- and 8400-node
// workloads: 24, 96 and 288 snapshots, segments of 8 to 20 nodes).
int score64_groups_default(int k, int S, int* spg) {
  const double base = k <= 9 ? 8.0 : (k <= 12 ? 16.0 : (k <= 16 ? 32.0 : 64.0));
  const double want = base * (S > 96 ? std::pow(S / 96.0, 0.37) : 1.0);
  int SG = (int)std::ceil(S / want - 1e-9);
  SG = std::max(1, std::min(std::min(SG, S), kMaxSnapGroups));
  *spg = (S + SG - 1) / SG;
  return (S + *spg - 1) / *spg;
}

// Launch shape of the FP32 screen: masks per lane by segment size, snapshot
// groups by the per-mask FP64 kernel's rule (on MI355X 10% faster than a
// block-count target on the 8400-node workload, within 2% on the 6000-node
// one).  The workspace planner sizes the screen's partial scores from this
// same function.
int screen32_shape(int k, int S, int* spg, int* mpl) {
  *mpl = k >= 12 ? 4 : (k >= 10 ? 2 : 1);
  return score64_groups_default(k, S, spg);
}

struct Layout {
  size_t topo, z, Zroot, Vhat, Vcur, A, J, absV, kept, sup, slot_of, zent_of, status, iters, hdrs, decs, tab, P, srec,
      headV, zrec, econst, part, fin, tiles, tickets, kp, yeq, Ykd, Yko, err;
  // factored FP64 scoring: chain-pattern table, largest constant error;
  // accumulators of the short-list scoring
  size_t pat, ecmax, lacc;
  // mixed precision
  size_t P32, S32, H32, Z32, part32, fin32, tiles32, listA, listB, scoreA, scoreB, counts, mstate;
  // results the host reads after a search, contiguous (one transfer):
  // status .. err, from res0, res_bytes long
  size_t res0, res_bytes;
  // surrogate: feature tables (always), ranking buffers (when planned with top_k)
  size_t spz, szs, sss, skeys, slist, sscore, scount, sgates, sW1b, sW2b, sW2tb, slevel,
      sstage;
  // SMICE key (when planned with it): prep table, fixed head maxima, per-mask SMICE, mask 0's
  size_t stab, hK, smv, smv0;
  size_t lane0, lane_stride;  // per-lane scratch block (tab .. scount)
  size_t total;
};

// offsets (in int32) of the static topology arrays inside the topology buffer
struct TopoOffsets {
  int parent, phase, segment, pos, size, pre, ch_off, ch, lvl_off, lvl_nodes, bfs_cf, bfs_pp, seg_off, seg_nodes,
      chunks, seg_top, total;
};

}  // namespace

struct okr_handle {
  hipStream_t stream = nullptr;
  std::string err;
  // plan
  bool planned = false;
  int n = 0, S = 0, nseg = 0, kmax = 0, nlev = 0, tab_cap = 0, topk = 0;
  bool smice = false;  // planned with SMICE as the key (its buffers exist)
  int64_t ncand = 0;
  std::vector<int> parent, segment, pre, pos, size, ch_off, ch, lvl_off, lvl_nodes, bfs_cf, bfs_pp, seg_off, seg_nodes;
  std::vector<uint8_t> phase, eligible;
  Layout L{};
  TopoOffsets TO{};
  std::vector<int> topo_host;  // packed static arrays uploaded at each call
  // page-locked host copy of the result block (allocated by the first call
  // that may allocate; the no-allocation entry point copies region by region)
  void* rstage = nullptr;
  size_t rstage_bytes = 0;
  // page-locked copy of topo_host (the upload at each call is then a plain
  // asynchronous transfer); filled again after every plan
  void* tstage = nullptr;
  size_t tstage_bytes = 0;
  bool tstage_fresh = false;
  // timing
  std::vector<hipEvent_t> ev;
  // captured graph of one whole search, and the arguments it was captured with
  hipGraphExec_t gexec = nullptr;
  std::vector<uint64_t> gkey;
  // per-mask score dumps (FP64 scores, or FP32 screening scores in MIXED)
  std::vector<std::vector<MaskScore>> dump;
  std::vector<std::vector<MaskScore32>> dump32;
  // shape of the FP64 scoring launches, autotuned per segment size (0 = the
  // default rule): snapshot groups and masks per lane; values forced while
  // tuning; the partial-score capacity (masks x groups) of the workspace
  std::vector<int> sg_tuned, mpl_tuned, ws_tuned;
  int sg_force = 0, mpl_force = 0, ws_force = 0;
  size_t part_cap = 0;
  // segment chunks: every search step is one launch over a chunk of
  // mutually independent segments (chunk c = chunk_segs[chunk_off[c] ..
  // chunk_off[c + 1]), at most nlanes of them, each with its own scratch
  // block); chunk_k = the chunk's largest segment size
  int nlanes = 1;
  std::vector<int> chunk_off, chunk_segs, chunk_k;
};

namespace {
// Launch shape of the per-mask FP64 scoring for a chunk of nz segments whose
// largest has k nodes: snapshots per pass, waves sharing each 64 masks'
// chains, snapshot groups.  Each is forced (while autotuning), tuned for
// (k, nz), or the default rule.
int shape_key(int k, int nz) { return k * (kMaxLanes + 1) + nz; }
int tuned(const std::vector<int>& t, int k, int nz) {
  const int i = shape_key(k, nz);
  return i < (int)t.size() ? t[i] : 0;
}
// Defaults follow the autotuner's picks on MI355X for the 1000-, 6000- and
// 8400-node workloads (segments of 8 to 20 nodes, chunks of 1-8 segments):
// 4 snapshots per pass up to 14 nodes (and for a lone segment up to 16), 2 up
// to 19, then 1; 4 waves per 64 masks up to 14 nodes in chunks of up to 5
// (else 2), from 15 nodes one in chunks of three or more or from 18 nodes,
// else 4 for a lone segment of 15 and 2 otherwise.
int score_mpl(const okr_handle* h, int k, int nz) {
  if (h->mpl_force) return h->mpl_force;
  const int t = tuned(h->mpl_tuned, k, nz);
  if (t) return t;
  if (k <= 14 || (nz == 1 && k <= 16)) return 4;
  return k <= 19 ? 2 : 1;
}
int score_ws(const okr_handle* h, int k, int nz) {
  if (h->ws_force) return h->ws_force;
  const int t = tuned(h->ws_tuned, k, nz);
  if (t) return t;
  if (k <= 14) return nz <= 5 ? 4 : 2;
  if (nz >= 3 || k >= 18) return 1;
  return (nz == 1 && k <= 15) ? 4 : 2;
}

// Snapshot groups of the FP64 scoring launch for a segment of k nodes: the
// forced or tuned count, else the default rule, within the planned
// partial-score capacity; spg = snapshots per group.
// LDS of the snapshot-vectorised FP64 scoring kernel: spp snapshots of
// pairs, slot records, chain heads and their magnitudes, the first kSvZone
// zone records, and the constant errors.
constexpr int kSvZone = 128;
constexpr size_t kSvLdsMax = 60 * 1024;
size_t sv_lds_bytes(int spp, int k) {
  const size_t pcap = (size_t)k * (k + 1) / 2;
  return (size_t)spp * (pcap * 3 * sizeof(double2) + (size_t)k * 3 * (sizeof(TargetRec) + sizeof(double2) + sizeof(double)) +
                        kSvZone * sizeof(TargetRec) + sizeof(double)) +
         16;  // (the kernel packs the tables to the segment's own sizes: rounding room)
}
// LDS of the chain-term kernel for segments of up to k nodes: chain records
// and nesting paths, one snapshot's pairs, slot and head records, and the
// first kTermsZone zone records.
constexpr int kTermsZone = 256;
int terms_icap(int k) { return k * kChainInts + k * k; }
size_t terms_lds_bytes(int k) {
  const size_t pcap = (size_t)k * (k + 1) / 2;
  return ((size_t)terms_icap(k) * 4 + 15) / 16 * 16 + pcap * 3 * sizeof(double2) +
         (size_t)k * 3 * (sizeof(TargetRec) + sizeof(double2)) + kTermsZone * sizeof(TargetRec);
}

// Snapshots per pass: the wanted count (1, 2 or 4), at most the group's
// snapshots, within the LDS budget.
int sv_spp(int want, int k, int spg) {
  int spp = want >= 4 ? 4 : (want >= 2 ? 2 : 1);
  while (spp > 1 && (spp > spg || sv_lds_bytes(spp, k) > kSvLdsMax)) spp /= 2;
  return spp;
}

// (within the partial-score capacity of the workspace)
int snap_groups(const okr_handle* h, int k, int nz, int* spg) {
  const int S = h->S;
  int SG = h->sg_force ? h->sg_force : tuned(h->sg_tuned, k, nz);
  if (SG <= 0) SG = score64_groups_default(k, S, spg);
  SG = std::min(std::min(SG, S), kMaxSnapGroups);
  while (SG > 1 && ((size_t)SG << k) > h->part_cap) --SG;
  *spg = (S + SG - 1) / SG;
  return (S + *spg - 1) / *spg;
}
}  // namespace

#define OKR_FAIL(h, code, ...)            \
  do {                                    \
    char _b[512];                         \
    snprintf(_b, sizeof _b, __VA_ARGS__); \
    (h)->err = _b;                        \
    return code;                          \
  } while (0)

#define OKR_HIP(h, call)                                                                   \
  do {                                                                                     \
    hipError_t _e = (call);                                                                \
    if (_e != hipSuccess) OKR_FAIL(h, OKR_E_HIP, "%s: %s", #call, hipGetErrorString(_e)); \
  } while (0)

static void drop_graph(okr_handle* h) {
  if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
  h->gexec = nullptr;
  h->gkey.clear();
}

static void drop_events(okr_handle* h) {
  for (hipEvent_t e : h->ev) (void)hipEventDestroy(e);
  h->ev.clear();
}

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
  drop_graph(h);
  drop_events(h);
  if (h->rstage) (void)hipHostFree(h->rstage);
  if (h->tstage) (void)hipHostFree(h->tstage);
  delete h;
  return OKR_OK;
}

namespace {
// The method's own work of scoring segment g's 2^k candidates over S
// snapshots, from the kept state before the segment (keep): per candidate
// and snapshot, 2|phi_r| per reduced node r and hop to its super-node (the
// moved current), 8|phi_e|^2 + 2|phi_e| per edge carrying it (the voltage
// change), 2|phi| per segment node (the shift below the segment), 10 per
// node-phase of the affected region (magnitude, error, margins); plus 18 per
// reduced node per candidate (series sums of the Kron step).  The first two
// terms are averaged exactly over the masks, chain by chain: a reduced node's
// current climbs through reduced nodes to the first kept one, so only the
// segment nodes of its own chain matter.
double method_flops(const okr_handle* h, int g, const std::vector<uint8_t>& keep, int S) {
  const int k = h->seg_off[g + 1] - h->seg_off[g];
  const int* nodes = h->seg_nodes.data() + h->seg_off[g];
  auto ph = [&](int v) { return (double)__builtin_popcount(h->phase[v]); };
  // chain tops: climb through segment nodes and reduced nodes
  std::vector<int> top(k);
  for (int j = 0; j < k; ++j) {
    int c = nodes[j];
    while (h->parent[c] >= 0 && (h->segment[h->parent[c]] == g || !keep[h->parent[c]])) c = h->parent[c];
    top[j] = c;
  }
  // node-phases of the affected region: union of the tops' subtrees
  std::vector<std::pair<int, int>> iv;
  for (int j = 0; j < k; ++j) iv.push_back({h->pos[top[j]], h->pos[top[j]] + h->size[top[j]]});
  std::sort(iv.begin(), iv.end());
  double np_omega = 0.0;
  int reach = -1;
  for (auto& r : iv) {
    for (int q = std::max(r.first, reach); q < r.second; ++q) np_omega += ph(h->pre[q]);
    reach = std::max(reach, r.second);
  }
  double per = 10.0 * np_omega;
  for (int j = 0; j < k; ++j) per += 2.0 * ph(nodes[j]);
  // moved currents and voltage changes, chain by chain
  std::vector<char> done(k, 0);
  for (int j0 = 0; j0 < k; ++j0) {
    if (done[j0]) continue;
    // the chain: the path from its top down to its deepest segment node
    int bottom = nodes[j0];
    std::vector<int> bits;  // segment positions in this chain
    for (int j = 0; j < k; ++j)
      if (top[j] == top[j0]) {
        bits.push_back(j);
        done[j] = 1;
        if (h->pos[nodes[j]] > h->pos[bottom]) bottom = nodes[j];
      }
    std::vector<int> path;  // bottom .. top
    for (int c = bottom;; c = h->parent[c]) {
      path.push_back(c);
      if (c == top[j0]) break;
    }
    std::reverse(path.begin(), path.end());  // top .. bottom
    const int L = (int)path.size(), b = (int)bits.size();
    std::vector<int> bit_of(L, -1);
    for (int i = 0; i < L; ++i)
      for (int t = 0; t < b; ++t)
        if (nodes[bits[t]] == path[i]) bit_of[i] = t;
    double acc = 0.0;
    std::vector<char> carry(L);
    for (uint32_t m = 0; m < (1u << b); ++m) {
      int stop = -1;  // index of the nearest kept node above (-1: the head)
      std::fill(carry.begin(), carry.end(), 0);
      for (int i = 0; i < L; ++i) {
        if (bit_of[i] < 0) continue;  // reduced earlier: the current passes through
        if (!(m >> bit_of[i] & 1u)) {
          stop = i;
          continue;
        }
        acc += 2.0 * ph(path[i]) * (i - stop);
        for (int t = i; t > stop; --t) carry[t] = 1;
      }
      for (int i = 0; i < L; ++i)
        if (carry[i]) acc += 8.0 * ph(path[i]) * ph(path[i]) + 2.0 * ph(path[i]);
    }
    per += acc / double(1u << b);
  }
  const double masks = double(int64_t(1) << k);
  return per * masks * S + 18.0 * 0.5 * k * masks;
}
}  // namespace

extern "C" const char* okr_last_error(const okr_handle* h) { return h ? h->err.c_str() : "null handle"; }

// ------------------------------------------------------------------- plan --
extern "C" int okr_plan(okr_handle* h, const okr_topology* topo, const okr_margins* mg, int32_t S,
                        size_t* workspace_bytes, okr_sizes* sizes) {
  if (!h) return OKR_E_ARG;
  h->planned = false;
  h->tstage_fresh = false;
  drop_graph(h);
  if (!topo || !mg || !workspace_bytes || S < 1) OKR_FAIL(h, OKR_E_ARG, "null argument or S < 1");
  if (mg->secondary != OKR_SECONDARY_MAXERR && mg->secondary != OKR_SECONDARY_SMICE)
    OKR_FAIL(h, OKR_E_ARG, "unknown secondary key %d", mg->secondary);
  h->smice = mg->secondary == OKR_SECONDARY_SMICE;
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
    // breadth-first queue order: the root, then each listed node's children
    // in child-list order.  Every level is then a contiguous run, and the
    // children of the node at position q are the contiguous positions
    // bfs_cf[q] .. bfs_cf[q+1]-1, in child-list order; bfs_pp[q] is the
    // position of the parent.
    h->lvl_nodes.assign(1, 0);
    h->lvl_nodes.reserve(n);
    h->bfs_cf.assign(n + 1, 0);
    h->bfs_pp.assign(n, 0);
    for (int q = 0; q < n; ++q) {
      const int v = h->lvl_nodes[q];
      h->bfs_cf[q] = (int)h->lvl_nodes.size();
      for (int e = h->ch_off[v]; e < h->ch_off[v + 1]; ++e) {
        h->bfs_pp[h->lvl_nodes.size()] = q;
        h->lvl_nodes.push_back(h->ch[e]);
      }
    }
    h->bfs_cf[n] = n;
    for (int q = 1; q < n; ++q)
      if (depth[h->lvl_nodes[q]] < depth[h->lvl_nodes[q - 1]]) OKR_FAIL(h, OKR_E_NOT_TREE, "level order broken");
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
  std::vector<std::vector<int>> seg_nodes(nseg);
  for (int q = 0; q < n; ++q) {
    int v = h->pre[q];
    if (h->segment[v] >= 0) seg_nodes[h->segment[v]].push_back(v);
  }
  h->kmax = 0;
  h->ncand = 0;
  h->seg_off.assign(nseg + 1, 0);
  h->seg_nodes.clear();
  for (int g = 0; g < nseg; ++g) {
    const int k = (int)seg_nodes[g].size();
    if (k == 0) OKR_FAIL(h, OKR_E_ARG, "segment id %d is empty", g);
    if (k > kMaxK) OKR_FAIL(h, OKR_E_UNSUPPORTED, "segment %d has %d eligible nodes (max %d)", g, k, kMaxK);
    h->kmax = std::max(h->kmax, k);
    h->ncand += int64_t(1) << k;
    h->seg_off[g + 1] = h->seg_off[g] + k;
    h->seg_nodes.insert(h->seg_nodes.end(), seg_nodes[g].begin(), seg_nodes[g].end());
  }
  h->nseg = nseg;
  // Segment chunks.  A segment's search reads and writes state only inside
  // the subtrees of its possible chain tops (climb from each node through
  // segment nodes of any segment: every node that a chain of the segment can
  // ever pass lies there) and at the heads above them (moved currents land
  // there).  Segments that share none of that are independent, so their
  // order does not matter.  Every segment gets a level one above the highest
  // level of the earlier segments it conflicts with; each level's segments
  // (largest first) are cut into chunks of at most nlanes, and the chunks
  // run level by level: conflicting segments keep their order.
  {
    const int want = mg->lanes > 0 ? std::min(mg->lanes, kMaxLanes) : kDefaultLanes;
    h->nlanes = std::max(1, std::min(want, nseg));
    std::vector<std::vector<std::pair<int, int>>> iv(nseg);
    std::vector<std::vector<int>> heads(nseg);
    for (int g = 0; g < nseg; ++g) {
      for (int q = h->seg_off[g]; q < h->seg_off[g + 1]; ++q) {
        int c = h->seg_nodes[q];
        while (h->parent[c] >= 0 && h->segment[h->parent[c]] >= 0) c = h->parent[c];
        iv[g].push_back({h->pos[c], h->pos[c] + h->size[c]});
        heads[g].push_back(h->parent[c]);
      }
      std::sort(iv[g].begin(), iv[g].end());
      std::vector<std::pair<int, int>> mgd;
      for (auto& r : iv[g]) {
        if (!mgd.empty() && r.first < mgd.back().second) mgd.back().second = std::max(mgd.back().second, r.second);
        else mgd.push_back(r);
      }
      iv[g] = mgd;
      std::sort(heads[g].begin(), heads[g].end());
      heads[g].erase(std::unique(heads[g].begin(), heads[g].end()), heads[g].end());
    }
    auto inside = [&](int v, const std::vector<std::pair<int, int>>& R) {
      if (v < 0) return false;
      const int pv = h->pos[v];
      for (auto& r : R)
        if (r.first <= pv && pv < r.second) return true;
      return false;
    };
    auto conflict = [&](int a, int b) {
      size_t i = 0, j = 0;
      while (i < iv[a].size() && j < iv[b].size()) {
        if (iv[a][i].first < iv[b][j].second && iv[b][j].first < iv[a][i].second) return true;
        if (iv[a][i].second <= iv[b][j].second) ++i;
        else ++j;
      }
      for (int x : heads[a])
        if (inside(x, iv[b]) || std::binary_search(heads[b].begin(), heads[b].end(), x)) return true;
      for (int x : heads[b])
        if (inside(x, iv[a])) return true;
      return false;
    };
    std::vector<int> level(nseg, 0);
    int nlev_seg = 0;
    for (int g = 0; g < nseg; ++g) {
      for (int b = g - 1; b >= 0; --b)
        if (level[b] + 1 > level[g] && conflict(g, b)) level[g] = level[b] + 1;
      nlev_seg = std::max(nlev_seg, level[g] + 1);
    }
    std::vector<int> order(nseg);
    for (int g = 0; g < nseg; ++g) order[g] = g;
    auto ksz = [&](int g) { return h->seg_off[g + 1] - h->seg_off[g]; };
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
      if (level[a] != level[b]) return level[a] < level[b];
      if (ksz(a) != ksz(b)) return ksz(a) > ksz(b);
      return a < b;
    });
    h->chunk_off.assign(1, 0);
    h->chunk_segs.clear();
    h->chunk_k.clear();
    for (int i = 0; i < nseg; ++i) {
      const int g = order[i];
      const int c0 = h->chunk_off.back();
      const int m = (int)h->chunk_segs.size() - c0;
      if (m > 0 && (m == h->nlanes || level[h->chunk_segs[c0]] != level[g])) {
        h->chunk_off.push_back((int)h->chunk_segs.size());
        h->chunk_k.push_back(0);
      }
      if (h->chunk_k.empty()) h->chunk_k.push_back(0);
      h->chunk_segs.push_back(g);
      h->chunk_k.back() = std::max(h->chunk_k.back(), ksz(g));
    }
    if (!h->chunk_segs.empty()) h->chunk_off.push_back((int)h->chunk_segs.size());
  }
  // packed static topology
  TopoOffsets& TO = h->TO;
  std::vector<int>& tp = h->topo_host;
  tp.clear();
  auto put = [&](const std::vector<int>& v) {
    const int o = (int)tp.size();
    tp.insert(tp.end(), v.begin(), v.end());
    return o;
  };
  TO.parent = put(h->parent);
  TO.segment = put(h->segment);
  TO.pos = put(h->pos);
  TO.size = put(h->size);
  TO.pre = put(h->pre);
  TO.ch_off = put(h->ch_off);
  TO.ch = put(h->ch);
  TO.lvl_off = put(h->lvl_off);
  TO.lvl_nodes = put(h->lvl_nodes);
  TO.bfs_cf = put(h->bfs_cf);
  TO.bfs_pp = put(h->bfs_pp);
  TO.seg_off = put(h->seg_off);
  TO.seg_nodes = put(h->seg_nodes.empty() ? std::vector<int>{0} : h->seg_nodes);
  TO.chunks = put(h->chunk_segs.empty() ? std::vector<int>{0} : h->chunk_segs);
  {
    // static part of the chain-top climb: through nodes of the same segment
    // (preorder: a parent's entry is final before its children's)
    std::vector<int> top(n, -1);
    for (int q = 0; q < n; ++q) {
      const int v = h->pre[q];
      if (h->segment[v] < 0) continue;
      const int pv = h->parent[v];
      top[v] = (pv >= 0 && h->segment[pv] == h->segment[v]) ? top[pv] : v;
    }
    TO.seg_top = put(top);
  }
  TO.phase = (int)tp.size();
  tp.resize(tp.size() + (n + 3) / 4, 0);
  std::memcpy(tp.data() + TO.phase, h->phase.data(), n);
  TO.total = (int)tp.size();
  // table capacity of one segment (layout written by k_build_struct)
  h->tab_cap = kMaxK * kChainInts + kMaxK * kMaxK + n + kMaxK * kSlotInts + kMaxPairs * kPairInts + 3 * kMaxK +
               9 * n + 64;
  // workspace layout
  const size_t c3 = (size_t)S * n * 3;
  Layout& L = h->L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  L.topo = take(sizeof(int) * TO.total);
  L.z = take(sizeof(double2) * 9 * n);
  L.Zroot = take(sizeof(double2) * 9 * n);
  L.Vhat = take(sizeof(double2) * c3);
  L.Vcur = take(sizeof(double2) * c3);
  L.A = take(sizeof(double2) * c3);
  L.J = take(sizeof(double2) * c3);
  L.absV = take(sizeof(double) * c3);
  L.kept = take(n);
  L.slot_of = take(sizeof(int) * n);
  L.zent_of = take(sizeof(int) * 3 * n);
  // per-segment scratch (one block per chunk position z, at + z * lane_stride)
  L.lane0 = off;
  L.tab = take(sizeof(int) * h->tab_cap);
  L.P = take(sizeof(double2) * 3 * (size_t)S * kMaxPairs);
  L.srec = take(sizeof(TargetRec) * 3 * (size_t)S * kMaxK);
  L.headV = take(sizeof(double2) * 3 * (size_t)S * kMaxK);
  L.zrec = take(sizeof(TargetRec) * (size_t)S * 3 * n);
  L.econst = take(sizeof(double) * S);
  {
    // partial scores: every default shape, and room to tune up to 32 groups
    // for segments of up to 16 nodes
    size_t most = (size_t)std::min(S, kMaxSnapGroups) << std::min(h->kmax, 16);
    for (int k = 1; k <= h->kmax; ++k) {
      int spg;
      most = std::max(most, (size_t)score64_groups_default(k, S, &spg) << k);
    }
    L.part = take(sizeof(MaskScore) * most);
    h->part_cap = most;
    const size_t nkey = (size_t)shape_key(h->kmax + 1, 0);
    if (h->sg_tuned.size() != nkey) {  // tuning survives a re-plan of the same sizes
      h->sg_tuned.assign(nkey, 0);
      h->mpl_tuned.assign(nkey, 0);
      h->ws_tuned.assign(nkey, 0);
    }
    const size_t nm = (size_t)1 << h->kmax, nt = (nm + 63) / 64;
    L.fin = take(sizeof(MaskScore) * nm);
    L.tiles = take(sizeof(TileRec) * nt);
    L.tickets = take(sizeof(int) * nt);
    L.pat = take(sizeof(PatScore) * 2 * nm);
    L.ecmax = take(sizeof(double));
    L.lacc = take(sizeof(unsigned long long) * 3 * nm);
  }
  {
    size_t most = 1;
    for (int k = 1; k <= h->kmax; ++k) {
      int spg, mpl;
      most = std::max(most, (size_t)screen32_shape(k, S, &spg, &mpl) << k);
    }
    const size_t nm = (size_t)1 << h->kmax, nt = (nm + 63) / 64;
    L.P32 = take(sizeof(Pair32) * 3 * (size_t)S * kMaxPairs);
    L.S32 = take(sizeof(Rec32) * 3 * (size_t)S * kMaxK);
    L.H32 = take(sizeof(Head32) * 3 * (size_t)S * kMaxK);
    L.Z32 = take(sizeof(Rec32) * (size_t)S * 3 * n);
    L.part32 = take(sizeof(MaskScore32) * most);
    L.fin32 = take(sizeof(MaskScore32) * nm);
    L.tiles32 = take(sizeof(TileRec32) * nt);
    L.listA = take(sizeof(uint32_t) * nm);
    L.listB = take(sizeof(uint32_t) * nm);
    L.scoreA = take(sizeof(MaskScore) * nm);
    L.scoreB = take(sizeof(MaskScore) * nm);
    L.counts = take(sizeof(int) * 4);
  }
  h->topk = (mg->top_k > 0) ? mg->top_k : 0;
  {
    L.spz = take(sizeof(float) * kMaxPairs);
    L.szs = take(sizeof(float) * kMaxPairs);
    L.sss = take(sizeof(SurrSlot) * kMaxK);
    const size_t mp = h->topk ? std::max((size_t)64, (size_t)1 << h->kmax) : 0;
    L.skeys = take(sizeof(uint32_t) * mp);
    L.slevel = take(sizeof(uint32_t) * mp);
    L.slist = take(sizeof(uint32_t) * std::max(h->topk, 1));
    L.sscore = take(sizeof(MaskScore) * std::max(h->topk, 1));
    L.scount = take(sizeof(int) * 4);
  }
  {
    const size_t on = h->smice ? 1 : 0;
    L.stab = take(sizeof(int) * on * ((size_t)SM_ZREC + (size_t)kZrecInts * n));
    L.hK = take(sizeof(double) * on * (size_t)kMaxK * S);
    L.smv = take(sizeof(double) * on * ((size_t)1 << h->kmax));
    L.smv0 = take(sizeof(double) * on);
  }
  L.lane_stride = off - L.lane0;
  off = L.lane0 + L.lane_stride * (size_t)h->nlanes;
  // per-segment records and shared weights
  L.sstage = take(sizeof(int) * std::max(nseg, 1));
  L.sW1b = take(sizeof(uint16_t) * kSurrH * kSurrF * (h->topk ? 1 : 0));
  L.sW2b = take(sizeof(uint16_t) * kSurrH * kSurrH * (h->topk ? 1 : 0));
  L.sW2tb = take(8);
  L.yeq = take(sizeof(double2) * 9 * n);
  // the results the host reads, contiguous
  L.res0 = off;
  L.status = take(sizeof(int) * kStatusInts);
  L.iters = take(sizeof(int) * S);
  L.hdrs = take(sizeof(SegHdr) * std::max(nseg, 1));
  L.decs = take(sizeof(DevDecision) * std::max(nseg, 1));
  L.mstate = take(sizeof(MixedState) * std::max(nseg, 1));
  L.sgates = take(sizeof(int) * std::max(nseg, 1));
  L.sup = take(sizeof(int) * n);
  L.kp = take(sizeof(int) * n);
  L.Ykd = take(sizeof(double2) * 9 * n);
  L.Yko = take(sizeof(double2) * 9 * n);
  L.err = take(sizeof(double) * S);
  L.res_bytes = off - L.res0;
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

// ------------------------------------------------------------ the search --
namespace {

struct Ptrs {
  Topo T;
  State St;
  const int *lvl_off, *lvl_nodes, *bfs_cf, *bfs_pp, *chunks;
  double2 *z, *Zroot, *Vhat, *Vcur, *A, *J, *P, *headV, *yeq, *Ykd, *Yko;
  double *absV, *econst, *err;
  int *status, *iters, *tab, *tickets, *kp;
  SegHdr* hdrs;
  DevDecision* decs;
  TargetRec *srec, *zrec;
  MaskScore *part, *fin;
  TileRec* tiles;
  unsigned long long *pat, *ecmax, *lacc;
  Pair32* P32;
  Rec32 *S32, *Z32;
  Head32* H32;
  MaskScore32 *part32, *fin32;
  TileRec32* tiles32;
  uint32_t *listA, *listB;
  MaskScore *scoreA, *scoreB;
  int* counts;
  MixedState* mstate;
  float *spz, *szs;
  SurrSlot* sss;
  __bf16 *sW1b, *sW2b, *sW2tb;
  uint32_t *skeys, *slist, *slevel;
  MaskScore* sscore;
  int *scount, *sgates, *sstage;
  int* stab;
  double *hK, *smv, *smv0;
};

// Device pointers, with the scratch block of chunk position `lane`.
Ptrs pointers(okr_handle* h, void* d_workspace, int lane = 0) {
  const Layout& L = h->L;
  char* ws = static_cast<char*>(d_workspace);
  const size_t lo = L.lane_stride * (size_t)lane;
  auto at = [&](size_t o) {
    const bool lane_scoped = o >= L.lane0 && o < L.lane0 + L.lane_stride;
    return static_cast<void*>(ws + o + (lane_scoped ? lo : 0));
  };
  Ptrs p{};
  int* tp = (int*)at(L.topo);
  const TopoOffsets& TO = h->TO;
  p.T.n = h->n;
  p.T.parent = tp + TO.parent;
  p.T.phase = (const uint8_t*)(tp + TO.phase);
  p.T.segment = tp + TO.segment;
  p.T.pos = tp + TO.pos;
  p.T.size = tp + TO.size;
  p.T.pre = tp + TO.pre;
  p.T.ch_off = tp + TO.ch_off;
  p.T.ch = tp + TO.ch;
  p.T.seg_off = tp + TO.seg_off;
  p.T.seg_nodes = tp + TO.seg_nodes;
  p.T.seg_top = tp + TO.seg_top;
  p.lvl_off = tp + TO.lvl_off;
  p.lvl_nodes = tp + TO.lvl_nodes;
  p.bfs_cf = tp + TO.bfs_cf;
  p.bfs_pp = tp + TO.bfs_pp;
  p.chunks = tp + TO.chunks;
  p.St.kept = (uint8_t*)at(L.kept);
  p.St.sup = (int*)at(L.sup);
  p.St.slot_of = (int*)at(L.slot_of);
  p.St.zent_of = (int*)at(L.zent_of);
  p.z = (double2*)at(L.z);
  p.Zroot = (double2*)at(L.Zroot);
  p.Vhat = (double2*)at(L.Vhat);
  p.Vcur = (double2*)at(L.Vcur);
  p.A = (double2*)at(L.A);
  p.J = (double2*)at(L.J);
  p.absV = (double*)at(L.absV);
  p.status = (int*)at(L.status);
  p.iters = (int*)at(L.iters);
  p.hdrs = (SegHdr*)at(L.hdrs);
  p.decs = (DevDecision*)at(L.decs);
  p.tab = (int*)at(L.tab);
  p.P = (double2*)at(L.P);
  p.srec = (TargetRec*)at(L.srec);
  p.headV = (double2*)at(L.headV);
  p.zrec = (TargetRec*)at(L.zrec);
  p.econst = (double*)at(L.econst);
  p.part = (MaskScore*)at(L.part);
  p.fin = (MaskScore*)at(L.fin);
  p.tiles = (TileRec*)at(L.tiles);
  p.pat = (unsigned long long*)at(L.pat);
  p.ecmax = (unsigned long long*)at(L.ecmax);
  p.lacc = (unsigned long long*)at(L.lacc);
  p.tickets = (int*)at(L.tickets);
  p.kp = (int*)at(L.kp);
  p.yeq = (double2*)at(L.yeq);
  p.Ykd = (double2*)at(L.Ykd);
  p.Yko = (double2*)at(L.Yko);
  p.err = (double*)at(L.err);
  p.P32 = (Pair32*)at(L.P32);
  p.S32 = (Rec32*)at(L.S32);
  p.H32 = (Head32*)at(L.H32);
  p.Z32 = (Rec32*)at(L.Z32);
  p.part32 = (MaskScore32*)at(L.part32);
  p.fin32 = (MaskScore32*)at(L.fin32);
  p.tiles32 = (TileRec32*)at(L.tiles32);
  p.listA = (uint32_t*)at(L.listA);
  p.listB = (uint32_t*)at(L.listB);
  p.scoreA = (MaskScore*)at(L.scoreA);
  p.scoreB = (MaskScore*)at(L.scoreB);
  p.counts = (int*)at(L.counts);
  p.mstate = (MixedState*)at(L.mstate);
  p.spz = (float*)at(L.spz);
  p.szs = (float*)at(L.szs);
  p.sss = (SurrSlot*)at(L.sss);
  p.skeys = (uint32_t*)at(L.skeys);
  p.slist = (uint32_t*)at(L.slist);
  p.sscore = (MaskScore*)at(L.sscore);
  p.scount = (int*)at(L.scount);
  p.sgates = (int*)at(L.sgates);
  p.slevel = (uint32_t*)at(L.slevel);
  p.sstage = (int*)at(L.sstage);
  p.sW1b = (__bf16*)at(L.sW1b);
  p.sW2b = (__bf16*)at(L.sW2b);
  p.sW2tb = (__bf16*)at(L.sW2tb);
  p.stab = (int*)at(L.stab);
  p.hK = (double*)at(L.hK);
  p.smv = (double*)at(L.smv);
  p.smv0 = (double*)at(L.smv0);
  return p;
}

// FP64 scores of list[0 .. *count) (at most cap masks) of one segment into
// out: one lane per (listed mask, chain, snapshot), folded by atomics.  w
// holds the segment's scratch pointers and segp its id in device memory.
// FP64 scores of a mask list per chunk position (list, count and out in each
// position's scratch block; cap bounds every list): accumulators, chain
// terms of every (listed mask, chain), final scores.
void list_score(const okr_handle* h, const Ptrs& w, const int* segp, int nz, int k, const uint32_t* list,
                const int* count, int cap, MaskScore* out, const SelParams& sp, hipStream_t st) {
  const size_t ls = h->L.lane_stride;
  const int fb = std::max(1, std::min(64, (cap + 255) / 256));
  hipLaunchKernelGGL(k_terms_init, dim3(fb, 1, nz), dim3(256), 0, st, (const SegHdr*)w.hdrs, segp, ls, (int)0, count,
                     cap, (const double*)w.econst, w.lacc, (unsigned long long*)nullptr);
  // blocks per (segment, snapshot): each stages the snapshot's records, so
  // as few as fill the chip (about 1024 blocks in all), at most one per 256
  // items and 16
  const size_t pairs = (size_t)h->S * nz;
  const int cb = std::max(1, std::min({16, (int)(((size_t)cap * k + 255) / 256), (int)((1024 + pairs - 1) / pairs)}));
  hipLaunchKernelGGL(k_chain_terms, dim3(cb, h->S, nz), dim3(256), terms_lds_bytes(k), st, (const SegHdr*)w.hdrs,
                     segp, ls, (int)0, (const int*)w.tab, (const double2*)w.P, (const TargetRec*)w.srec,
                     (const double2*)w.headV, (const TargetRec*)w.zrec, (const double*)w.econst, list, count, cap,
                     terms_icap(k), kTermsZone, w.lacc, (unsigned long long*)nullptr);
  hipLaunchKernelGGL(k_list_finish, dim3(fb, 1, nz), dim3(256), 0, st, count, (const unsigned long long*)w.lacc, cap,
                     sp, out, ls);
}

void enqueue_search(okr_handle* h, void* ws, const okr_yblocks* Y, const okr_loads* loads,
                    const okr_margins* mg, hipStream_t st, const std::vector<hipEvent_t>* ev,
                    std::vector<std::vector<MaskScore>>* dump, std::vector<std::vector<MaskScore32>>* dump32,
                    float* feat_out, float* targ_out) {
  const int n = h->n, S = h->S;
  const Ptrs p = pointers(h, ws);
  std::vector<Ptrs> lp(h->nlanes);
  for (int l = 0; l < h->nlanes; ++l) lp[l] = pointers(h, ws, l);
  const bool vhat_given = (mg->flags & OKR_FLAG_VHAT_GIVEN) != 0;
  const int ntick = (int)((((size_t)1 << h->kmax) + 63) / 64);
  const int ninit = std::max(n, std::max(kStatusInts, ntick));
  hipLaunchKernelGGL(k_init_state, dim3((ninit + 255) / 256), dim3(256), 0, st, n, p.St, p.status, kStatusInts,
                     p.tickets, ntick, h->nlanes, h->L.lane_stride);
  hipLaunchKernelGGL(k_branch_z, dim3((n + 127) / 128), dim3(128), 0, st, n, p.T.parent, p.T.phase, p.T.ch_off,
                     p.T.ch, (const double2*)Y->Y_diag, (const double2*)Y->Y_off, p.z, p.status);
  hipLaunchKernelGGL(k_zroot, dim3(1), dim3(1024), 0, st, n, p.T.parent, p.lvl_off, p.lvl_nodes, h->nlev,
                     (const double2*)p.z, p.Zroot);
  const size_t c3 = (size_t)S * n * 3;
  if (vhat_given) {
    hipLaunchKernelGGL(k_copy2, dim3(1024), dim3(256), 0, st, (const double2*)loads->Vhat, p.Vhat, c3);
    hipLaunchKernelGGL(k_from_vhat, dim3((unsigned)((c3 + 255) / 256)), dim3(256), 0, st, n, S, p.T.phase,
                       (const double2*)loads->S_load, (const double2*)p.Vhat, mg->v_min, mg->v_max, p.A, p.absV,
                       p.status);
  } else {
    const double2* V0 = (const double2*)loads->V0;
    // iterates and tree in LDS where both fit, else the breadth-first form
    // with the queue tables in LDS, else everything in global memory (one
    // block per snapshot in each form; the breadth-first form's block of 512
    // takes most levels of the large feeders in one round: 1.23 -> 1.08 ms
    // on the 6000-node and 4.12 -> 3.85 ms on the 8400-node feeder against
    // 256)
    const size_t pf_lds = pf_lds_bytes(n, h->nlev), pf_bfs = pf_bfs_lds_bytes(n, h->nlev);
    const double tol = mg->pf_tol > 0 ? mg->pf_tol : 1e-13;
    const int maxit = mg->pf_maxit > 0 ? mg->pf_maxit : 100;
    if (pf_lds || !pf_bfs)
      hipLaunchKernelGGL(pf_lds ? k_powerflow_lds : k_powerflow, dim3(S), dim3(256), pf_lds, st, n, p.T.parent,
                         p.T.phase, p.lvl_off, p.lvl_nodes, h->nlev, p.T.ch_off, p.T.ch, (const double2*)p.z,
                         (const double2*)loads->S_load, V0[0], V0[1], V0[2], tol, maxit, mg->v_min, mg->v_max,
                         p.Vhat, p.J, p.A, p.absV, p.iters, p.status);
    else
      hipLaunchKernelGGL(k_powerflow_bfs, dim3(S), dim3(512), pf_bfs, st, n, p.T.phase, p.lvl_off, p.lvl_nodes,
                         h->nlev, p.bfs_cf, p.bfs_pp, (const double2*)p.z, (const double2*)loads->S_load, V0[0],
                         V0[1], V0[2], tol, maxit, mg->v_min, mg->v_max, p.Vhat, p.J, p.A, p.absV, p.iters,
                         p.status);
  }
  hipLaunchKernelGGL(k_copy2, dim3(1024), dim3(256), 0, st, (const double2*)p.Vhat, p.Vcur, c3);
  SelParams sp;
  sp.e_bar = mg->e_bar;
  sp.vmin = mg->v_min;
  sp.vmax = mg->v_max;
  sp.tie = mg->tie_tol;
  sp.amb = mg->amb_tol;
  sp.delta = mg->mixed_delta > 0.0 ? mg->mixed_delta : kMixedDelta;
  const bool mixed = mg->precision == OKR_PRECISION_MIXED;
  const bool factored = mg->precision == OKR_PRECISION_FP64_FACTORED;
  const bool surr = mg->top_k > 0 && mg->top_k <= h->topk && mg->surrogate != nullptr &&
                    mg->precision == OKR_PRECISION_FP64;
  if (surr)
    hipLaunchKernelGGL(k_refresh_weights, dim3((kSurrH * kSurrH + 255) / 256), dim3(256), 0, st, mg->surrogate,
                       p.sW1b, p.sW2b, (__bf16*)nullptr);
  const int members_blocks = std::min(2048, std::max(1, (int)(((size_t)n * S + 255) / 256)));
  // per-mask feature rows of segment g start at foff[g] (segments in id order)
  std::vector<size_t> foff(h->nseg + 1, 0);
  for (int g = 0; g < h->nseg; ++g) foff[g + 1] = foff[g] + ((size_t)1 << (h->seg_off[g + 1] - h->seg_off[g]));
  const size_t lstride = h->L.lane_stride;
  const int nchunk = (int)h->chunk_k.size();
  // every mask's final FP64 score is stored only when it is read back
  const int full_fin = (dump || feat_out) ? 1 : 0;
  for (int c = 0; c < nchunk; ++c) {
    const int c0 = h->chunk_off[c], nz = h->chunk_off[c + 1] - c0;
    const int* segs = p.chunks + c0;  // device copy of this chunk's segment ids
    const int kc = h->chunk_k[c];
    const Ptrs& q = lp[0];  // scratch of chunk position 0; position z is z * lstride further
    hipLaunchKernelGGL(k_build_struct, dim3(1, 1, nz), dim3(256), 0, st, q.T, q.St, segs, lstride, S, q.hdrs, q.tab,
                       h->tab_cap, q.status);
    hipLaunchKernelGGL(k_build_values, dim3(256, 5, nz), dim3(256), 0, st, (const SegHdr*)q.hdrs, segs, lstride,
                       (const int*)q.tab, n, (const double2*)q.Zroot, (const double2*)q.Vcur, (const double2*)q.A, q.P,
                       q.srec, q.headV, q.zrec, q.econst);
    hipLaunchKernelGGL(k_build_members, dim3(members_blocks, 1, nz), dim3(256), 0, st, (const SegHdr*)q.hdrs, segs,
                       lstride, (const int*)q.tab, q.T, q.St, (const double2*)q.Vcur, (const double*)q.absV, q.srec,
                       q.zrec, q.econst);
    const uint32_t nmask = 1u << kc;
    int spg;
    const int SG = snap_groups(h, kc, nz, &spg);
    // per-mask FP64 launch: one mask per lane, groups of ws waves sharing the
    // chains of 64 masks, spp snapshots per pass, LDS for spp snapshots
    const int sws = score_ws(h, kc, nz);
    const uint32_t bmask = kScoreBlock * (kScoreThreads / 64 / sws);
    const int mblocks = (int)((nmask + bmask - 1) / bmask);
    const int pcap = kc * (kc + 1) / 2;
    const int spp = sv_spp(score_mpl(h, kc, nz), kc, spg);
    const size_t lds = sv_lds_bytes(spp, kc);
    const int* gates = surr ? q.sgates : nullptr;
    for (int z = 0; z < nz; ++z) {
      const int g = h->chunk_segs[c0 + z];
      const int k = h->seg_off[g + 1] - h->seg_off[g];
      const uint32_t nm = 1u << k;
      const Ptrs& w = lp[z];
      if (surr || feat_out) {
        hipLaunchKernelGGL(k_surr_tables, dim3(kMaxPairs + kMaxK), dim3(64), 0, st, (const SegHdr*)w.hdrs, g,
                           (const int*)w.tab, n, (const double2*)w.Zroot, (const double2*)w.P, (const double2*)w.A,
                           (const TargetRec*)w.srec, w.spz, w.szs, w.sss);
      }
      if (!surr) continue;
      // Rank the masks with the surrogate and rescore the top-k exactly.
      // Stage 1 ranks only the top levels (popcount >= L1, at least 4 top_k
      // masks); when they hold top_k masks predicted feasible, those are the
      // top_k of the full ranking (predicted-feasible masks rank by level
      // first) and stage 2, the ranking of every mask, is skipped on device.
      const int K = mg->top_k;
      // predicted feasible: predicted ln error within the calibrated margin of ln(e_bar)
      const float ln_ebar = (float)(std::log(mg->e_bar) + (double)mg->surrogate_margin);
      int L1 = k;
      uint64_t N1 = 1;
      while (L1 > 0 && N1 < (uint64_t)4 * K) {
        --L1;
        uint64_t cb = 1;
        for (int r = 1; r <= L1; ++r) cb = cb * (uint64_t)(k - L1 + r) / (uint64_t)r;
        N1 += cb;
      }
      const bool staged = N1 < nm;
      int* stage = w.sstage + g;
      auto rank = [&](const uint32_t* masks, int nrow, const int* flag, int skip_if) {
        hipLaunchKernelGGL(k_surr_rank, dim3((nrow + 31) / 32), dim3(512), 0, st, (const SegHdr*)w.hdrs, g,
                           (const int*)w.tab, (const float*)w.spz, (const float*)w.szs, (const SurrSlot*)w.sss,
                           (const double*)w.econst, masks, nrow, (const __bf16*)w.sW1b, (const __bf16*)w.sW2b,
                           mg->surrogate, ln_ebar, w.skeys, flag, skip_if);
      };
      if (staged) {
        hipLaunchKernelGGL(k_level_masks, dim3(((int)N1 + 63) / 64 * 64 / 64), dim3(64), 0, st, k, L1, (int)N1,
                           ((int)N1 + 63) / 64 * 64, w.slevel);
        rank(w.slevel, (int)N1, (const int*)nullptr, 0);
        hipLaunchKernelGGL(k_surr_stage, dim3(1), dim3(256), 0, st, (const SegHdr*)w.hdrs, g,
                           (const uint32_t*)w.skeys, (int)N1, K, stage);
        hipLaunchKernelGGL(k_topk, dim3(1), dim3(1024), 0, st, (const SegHdr*)w.hdrs, g, (const uint32_t*)w.skeys,
                           (const uint32_t*)w.slevel, (int)N1, K, (const int*)w.status, w.slist, w.scount,
                           (const int*)stage, 0);
        rank((const uint32_t*)nullptr, (int)nm, (const int*)stage, 1);
        hipLaunchKernelGGL(k_topk, dim3(1), dim3(1024), 0, st, (const SegHdr*)w.hdrs, g, (const uint32_t*)w.skeys,
                           (const uint32_t*)nullptr, (int)nm, K, (const int*)w.status, w.slist, w.scount,
                           (const int*)stage, 1);
      } else {
        rank((const uint32_t*)nullptr, (int)nm, (const int*)nullptr, 0);
        hipLaunchKernelGGL(k_topk, dim3(1), dim3(1024), 0, st, (const SegHdr*)w.hdrs, g, (const uint32_t*)w.skeys,
                           (const uint32_t*)nullptr, (int)nm, K, (const int*)w.status, w.slist, w.scount,
                           (const int*)nullptr, 0);
      }
      // one segment: its own position's buffers are the launch's position 0
      list_score(h, w, p.chunks + c0 + z, 1, k, w.slist, w.scount, K, w.sscore, sp, st);
      hipLaunchKernelGGL(k_surr_decide, dim3(1), dim3(1024), 0, st, (const SegHdr*)w.hdrs, g, sp,
                         (const int*)w.status, (const uint32_t*)w.slist, (const int*)w.scount,
                         (const MaskScore*)w.sscore, w.decs, w.sgates + g);
    }
    if (!mixed) {
      // timing: the factored form's three launches between two recorded
      // events; the per-mask kernel's own start and end through its launch
      // (no marker packets around it)
      if (ev && factored) (void)hipEventRecord((*ev)[2 * c], st);
      hipEvent_t e0 = (ev && !factored) ? (*ev)[2 * c] : nullptr;
      hipEvent_t e1 = (ev && !factored) ? (*ev)[2 * c + 1] : nullptr;
      if (factored) {
        // pattern table (up to 2^(k+1) patterns), then every mask.  The
        // chain terms take one block per (segment, snapshot), looping over
        // all patterns: each block stages the snapshot's records once (with
        // 16 blocks per snapshot, each staging them, the launch took 2.7x
        // as long on the 8400-node feeder and 2.0x on the 6000-node one)
        const int pb = (int)std::min<uint64_t>(16, std::max<uint64_t>(1, ((uint64_t)2 << kc) / 256));
        hipLaunchKernelGGL(k_terms_init, dim3(pb, 1, nz), dim3(256), 0, st, (const SegHdr*)q.hdrs, segs, lstride, (int)1,
                           (const int*)nullptr, 0, (const double*)q.econst, q.pat, q.ecmax);
        hipLaunchKernelGGL(k_chain_terms, dim3(1, S, nz), dim3(256), terms_lds_bytes(kc), st, (const SegHdr*)q.hdrs,
                           segs, lstride, (int)1, (const int*)q.tab, (const double2*)q.P, (const TargetRec*)q.srec,
                           (const double2*)q.headV, (const TargetRec*)q.zrec, (const double*)q.econst,
                           (const uint32_t*)nullptr, (const int*)nullptr, 0, terms_icap(kc), kTermsZone, q.pat,
                           q.ecmax);
        hipLaunchKernelGGL(k_fac_combine, dim3((nmask + 255) / 256, 1, nz), dim3(256), 0, st, (const SegHdr*)q.hdrs,
                           segs, lstride, (const int*)q.tab, (const unsigned long long*)q.pat,
                           (const unsigned long long*)q.ecmax, sp, q.fin, q.tiles);
      } else {
#define OKR_SCORE64(M_)                                                                                             \
  hipExtLaunchKernelGGL(k_score_fp64<M_>, dim3(mblocks, SG, nz), dim3(kScoreThreads), lds, st, e0, e1, 0,            \
                        (const SegHdr*)q.hdrs, segs, lstride, (const int*)q.tab, (const double2*)q.P,              \
                        (const TargetRec*)q.srec, (const double2*)q.headV, (const TargetRec*)q.zrec,               \
                        (const double*)q.econst, spg, SG, pcap, kc, kSvZone, sws, sp, q.part, q.fin, q.tiles,      \
                        q.tickets, gates, full_fin)
        if (spp == 4) OKR_SCORE64(4);
        else if (spp == 2) OKR_SCORE64(2);
        else OKR_SCORE64(1);
#undef OKR_SCORE64
      }
      if (ev && factored) (void)hipEventRecord((*ev)[2 * c + 1], st);
      hipLaunchKernelGGL(k_argmin, dim3(1, 1, nz), dim3(1024), 0, st, (const SegHdr*)q.hdrs, segs, lstride,
                         (const MaskScore*)q.fin, (const TileRec*)q.tiles, sp, (const int*)q.status, q.decs, gates);
      if (mg->secondary == OKR_SECONDARY_SMICE && !surr) {
        // SMICE of the feasible masks of the chosen level, and the decision under it
        hipLaunchKernelGGL(k_smice_prep, dim3(1, 1, nz), dim3(256), 0, st, (const SegHdr*)q.hdrs, segs, lstride,
                           (const int*)q.tab, q.T, q.St, q.stab, q.hK, S);
        hipLaunchKernelGGL(k_smice_hconst, dim3(members_blocks, 1, nz), dim3(256), 0, st, (const SegHdr*)q.hdrs, segs,
                           lstride, q.T, q.St, (const double2*)q.Vcur, (const double*)q.absV, (const int*)q.stab,
                           q.hK, S);
        hipLaunchKernelGGL(k_smice_score, dim3((nmask + kSmiceThreadsHost - 1) / kSmiceThreadsHost, 1, nz),
                           dim3(kSmiceThreadsHost), 0, st, (const SegHdr*)q.hdrs, segs, lstride, (const int*)q.tab,
                           (const double2*)q.P, (const TargetRec*)q.srec, (const double2*)q.headV,
                           (const TargetRec*)q.zrec, (const int*)q.stab, (const double*)q.hK,
                           (const MaskScore*)q.fin, (const TileRec*)q.tiles, (const DevDecision*)q.decs, sp, q.smv,
                           q.smv0);
        hipLaunchKernelGGL(k_smice_argmin, dim3(1, 1, nz), dim3(1024), 0, st, (const SegHdr*)q.hdrs, segs, lstride,
                           (const MaskScore*)q.fin, (const TileRec*)q.tiles, (const double*)q.smv,
                           (const double*)q.smv0, mg->smice_tol > 0.0 ? mg->smice_tol : kSmiceTol, q.decs);
      }
      for (int z = 0; z < nz; ++z) {
        const int g = h->chunk_segs[c0 + z];
        const uint32_t nm = 1u << (h->seg_off[g + 1] - h->seg_off[g]);
        const Ptrs& w = lp[z];
        if (feat_out && !surr) {
          hipLaunchKernelGGL(k_surr_features, dim3((nm + 255) / 256), dim3(256), 0, st, (const SegHdr*)w.hdrs, g,
                             (const int*)w.tab, (const float*)w.spz, (const float*)w.szs, (const SurrSlot*)w.sss,
                             (const double*)w.econst, (const uint32_t*)nullptr, (int)nm, (int)nm,
                             feat_out + foff[g] * kSurrF, (__bf16*)nullptr, (const int*)nullptr, 0);
          if (targ_out)
            hipLaunchKernelGGL(k_surr_target, dim3((nm + 255) / 256), dim3(256), 0, st, (const SegHdr*)w.hdrs, g,
                               (const MaskScore*)w.fin, targ_out + foff[g]);
        }
        if (dump) {
          (*dump)[g].resize(nm);
          (void)hipMemcpyAsync((*dump)[g].data(), w.fin, sizeof(MaskScore) * nm, hipMemcpyDeviceToHost, st);
        }
      }
    } else {
      // mixed precision, one launch per step over the chunk: FP32 tables and
      // screen, shortlist A and its FP64 scores, shortlist B and its FP64
      // scores, the decision; then the FP64 scoring and arg-min of the
      // segments whose FP32 deviation exceeded the bound (gated on device)
      int spg32, mpl32;
      const int SG32 = screen32_shape(kc, S, &spg32, &mpl32);
      hipLaunchKernelGGL(k_build_mixed, dim3(256, 4, nz), dim3(256), 0, st, (const SegHdr*)q.hdrs, segs, lstride,
                         (const int*)q.tab, n, (const double2*)q.Vcur, (const double2*)q.P, (const TargetRec*)q.srec,
                         (const double2*)q.headV, (const TargetRec*)q.zrec, mg->v_min, mg->v_max, q.P32, q.S32, q.H32,
                         q.Z32);
      if (ev) (void)hipEventRecord((*ev)[2 * c], st);
      const int mblocks32 = (int)((nmask + kScoreThreads * mpl32 - 1) / (kScoreThreads * mpl32));
#define OKR_SCORE32(M_)                                                                                          \
  hipLaunchKernelGGL(k_score_fp32<M_>, dim3(mblocks32, SG32, nz), dim3(kScoreThreads), 0, st, (const SegHdr*)q.hdrs, \
                     segs, lstride, (const int*)q.tab, (const Pair32*)q.P32, (const Rec32*)q.S32,                  \
                     (const Head32*)q.H32, (const Rec32*)q.Z32, (const double*)q.econst, spg32, SG32, sp, q.part32,  \
                     q.fin32, q.tiles32, q.tickets)
      if (mpl32 == 4) OKR_SCORE32(4);
      else if (mpl32 == 2) OKR_SCORE32(2);
      else OKR_SCORE32(1);
#undef OKR_SCORE32
      if (ev) (void)hipEventRecord((*ev)[2 * c + 1], st);
      int* cA = q.counts;
      int* cB = q.counts + 1;
      hipLaunchKernelGGL(k_mixed_select_a, dim3(1, 1, nz), dim3(1024), 0, st, (const SegHdr*)q.hdrs, segs, lstride,
                         (const MaskScore32*)q.fin32, (const TileRec32*)q.tiles32, sp, (const int*)q.status, q.mstate,
                         q.listA, cA);
      list_score(h, q, segs, nz, kc, q.listA, cA, (int)nmask, q.scoreA, sp, st);
      hipLaunchKernelGGL(k_mixed_select_b, dim3(1, 1, nz), dim3(1024), 0, st, (const SegHdr*)q.hdrs, segs, lstride,
                         (const MaskScore32*)q.fin32, (const TileRec32*)q.tiles32, sp, (const int*)q.status, q.mstate,
                         (const uint32_t*)q.listA, (const int*)cA, (const MaskScore*)q.scoreA, q.listB, cB);
      list_score(h, q, segs, nz, kc, q.listB, cB, (int)nmask, q.scoreB, sp, st);
      hipLaunchKernelGGL(k_mixed_final, dim3(1, 1, nz), dim3(1024), 0, st, (const SegHdr*)q.hdrs, segs, lstride, sp,
                         (const int*)q.status, q.mstate, (const MaskScore32*)q.fin32, (const uint32_t*)q.listA,
                         (const int*)cA, (const MaskScore*)q.scoreA, (const uint32_t*)q.listB, (const int*)cB,
                         (const MaskScore*)q.scoreB, q.decs, q.sgates);
      {
        const int* redo = q.sgates;
#define OKR_SCORE64(M_)                                                                                             \
  hipLaunchKernelGGL(k_score_fp64<M_>, dim3(mblocks, SG, nz), dim3(kScoreThreads), lds, st, (const SegHdr*)q.hdrs, segs, \
                     lstride, (const int*)q.tab, (const double2*)q.P, (const TargetRec*)q.srec,                      \
                     (const double2*)q.headV, (const TargetRec*)q.zrec, (const double*)q.econst, spg, SG, pcap, kc,   \
                     kSvZone, sws, sp, q.part, q.fin, q.tiles, q.tickets, redo, full_fin)
        if (spp == 4) OKR_SCORE64(4);
        else if (spp == 2) OKR_SCORE64(2);
        else OKR_SCORE64(1);
#undef OKR_SCORE64
        hipLaunchKernelGGL(k_argmin, dim3(1, 1, nz), dim3(1024), 0, st, (const SegHdr*)q.hdrs, segs, lstride,
                           (const MaskScore*)q.fin, (const TileRec*)q.tiles, sp, (const int*)q.status, q.decs, redo);
      }
      if (dump)
        for (int z = 0; z < nz; ++z) {
          const int g = h->chunk_segs[c0 + z];
          const uint32_t nm = 1u << (h->seg_off[g + 1] - h->seg_off[g]);
          (*dump32)[g].resize(nm);
          (void)hipMemcpyAsync((*dump32)[g].data(), lp[z].fin32, sizeof(MaskScore32) * nm, hipMemcpyDeviceToHost, st);
        }
    }
    hipLaunchKernelGGL(k_apply, dim3(S, 1, nz), dim3(64), 0, st, (const SegHdr*)q.hdrs, segs, lstride,
                       (const int*)q.tab, q.T, q.St, (const DevDecision*)q.decs, (const double2*)q.P,
                       (const TargetRec*)q.srec, (const TargetRec*)q.zrec, q.Vcur, q.A);
  }
  hipLaunchKernelGGL(k_kron_yeq, dim3((n + 127) / 128), dim3(128), 0, st, p.T, p.St, (const double2*)p.z, p.yeq,
                     p.Yko, p.kp, p.status);
  hipLaunchKernelGGL(k_kron_diag, dim3((n + 127) / 128), dim3(128), 0, st, p.T, p.St, (const double2*)p.yeq, p.Ykd);
  hipLaunchKernelGGL(k_final_err, dim3(S), dim3(256), 0, st, n, p.T.phase, (const int*)p.St.sup,
                     (const double2*)p.Vcur, (const double*)p.absV, p.err);
}

uint64_t bits(double x) {
  uint64_t u;
  std::memcpy(&u, &x, sizeof u);
  return u;
}

}  // namespace

static int reduce_feeder_impl(okr_handle* h, const okr_yblocks* Y, const okr_topology* topo,
                              const okr_loads* loads, const okr_margins* mg, void* d_workspace,
                              size_t workspace_bytes, okr_result* out, bool may_alloc);

extern "C" int okr_reduce_feeder(okr_handle* h, const okr_yblocks* Y, const okr_topology* topo,
                                 const okr_loads* loads, const okr_margins* mg, void* d_workspace,
                                 size_t workspace_bytes, okr_result* out) {
  return reduce_feeder_impl(h, Y, topo, loads, mg, d_workspace, workspace_bytes, out, true);
}

// The no-allocation entry point's workspace: one array per GPU, resolved to
// its device address once per device (host code must never use the array's
// name as a device pointer).
static __device__ __align__(256) unsigned char scratch[OKR_NOALLOC_SCRATCH_BYTES];
namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

extern "C" int okr_reduce_feeder_noalloc(okr_handle* h, const okr_yblocks* Y, const okr_topology* topo,
                                         const okr_loads* loads, const okr_margins* mg, okr_result* out) {
  if (!h) return OKR_E_ARG;
  if (!mg) OKR_FAIL(h, OKR_E_ARG, "null margins");
  if (mg->flags & (OKR_FLAG_TIMING | OKR_FLAG_GRAPH | OKR_FLAG_AUTOTUNE | OKR_FLAG_DUMP_SCORES))
    OKR_FAIL(h, OKR_E_ARG, "okr_reduce_feeder_noalloc takes none of the timing, graph, autotune or dump flags");
  if (!h->planned) OKR_FAIL(h, OKR_E_ARG, "okr_plan() must succeed first");
  if (h->L.total > OKR_NOALLOC_SCRATCH_BYTES)
    OKR_FAIL(h, OKR_E_WORKSPACE, "planned workspace %zu bytes exceeds the static scratch of %zu bytes", h->L.total,
             (size_t)OKR_NOALLOC_SCRATCH_BYTES);
  int dev = -1;
  OKR_HIP(h, hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) OKR_FAIL(h, OKR_E_ARG, "device %d out of range", dev);
  void* ws = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
      void* ptr = nullptr;
      const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !ptr)
        OKR_FAIL(h, OKR_E_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
      g_scratch_ptr[dev] = ptr;
    }
    ws = g_scratch_ptr[dev];
  }
  return reduce_feeder_impl(h, Y, topo, loads, mg, ws, OKR_NOALLOC_SCRATCH_BYTES, out, false);
}

static int reduce_feeder_impl(okr_handle* h, const okr_yblocks* Y, const okr_topology* topo,
                              const okr_loads* loads, const okr_margins* mg, void* d_workspace,
                              size_t workspace_bytes, okr_result* out, bool may_alloc) {
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
  if (!loads->S_load) OKR_FAIL(h, OKR_E_ARG, "S_load is required (load currents)");
  if (vhat_given && !loads->Vhat) OKR_FAIL(h, OKR_E_ARG, "OKR_FLAG_VHAT_GIVEN without Vhat");
  if (mg->precision != OKR_PRECISION_FP64 && mg->precision != OKR_PRECISION_MIXED &&
      mg->precision != OKR_PRECISION_FP64_FACTORED)
    OKR_FAIL(h, OKR_E_ARG, "unknown precision %d", mg->precision);
  if (!(mg->v_min < mg->v_max) || !(mg->e_bar >= 0) || !(mg->tie_tol >= 0) || !(mg->amb_tol >= 0))
    OKR_FAIL(h, OKR_E_ARG, "bad margins");
  const bool timing = (mg->flags & OKR_FLAG_TIMING) != 0;
  const bool dump = (mg->flags & OKR_FLAG_DUMP_SCORES) != 0;
  const bool graph = (mg->flags & OKR_FLAG_GRAPH) != 0 && !timing && !dump && !out->features;
  if (mg->top_k > 0 && mg->surrogate && mg->top_k > h->topk)
    OKR_FAIL(h, OKR_E_ARG, "top_k %d exceeds the planned %d", mg->top_k, h->topk);
  if (out->targets && mg->precision == OKR_PRECISION_MIXED) OKR_FAIL(h, OKR_E_ARG, "targets need FP64 scores");
  if (mg->secondary != OKR_SECONDARY_MAXERR && mg->secondary != OKR_SECONDARY_SMICE)
    OKR_FAIL(h, OKR_E_ARG, "unknown secondary key %d", mg->secondary);
  if (mg->secondary == OKR_SECONDARY_SMICE) {
    if (!h->smice) OKR_FAIL(h, OKR_E_ARG, "SMICE as the key needs a plan made with it (okr_margins.secondary)");
    if (mg->precision == OKR_PRECISION_MIXED || (mg->top_k > 0 && mg->surrogate))
      OKR_FAIL(h, OKR_E_UNSUPPORTED, "SMICE as the key needs every feasible mask of the chosen level scored in FP64 "
                                     "(OKR_PRECISION_FP64 or FP64_FACTORED, no surrogate)");
    if (!(mg->smice_tol >= 0)) OKR_FAIL(h, OKR_E_ARG, "bad smice_tol");
  }
  const int n = h->n, S = h->S, nseg = h->nseg;
  hipStream_t st = h->stream;
  const Ptrs p = pointers(h, d_workspace);
  if (!(mg->flags & OKR_FLAG_VHAT_GIVEN)) {  // (set before any capture)
    if (pf_lds_bytes(n, h->nlev) > 64 * 1024)
      OKR_HIP(h, hipFuncSetAttribute(reinterpret_cast<const void*>(&k_powerflow_lds),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)kPfLdsMax));
    else if (!pf_lds_bytes(n, h->nlev) && pf_bfs_lds_bytes(n, h->nlev) > 64 * 1024)
      OKR_HIP(h, hipFuncSetAttribute(reinterpret_cast<const void*>(&k_powerflow_bfs),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)kPfLdsMax));
  }
  const auto t0 = clk::now();
  {
    const size_t tb = sizeof(int) * h->TO.total;
    if (may_alloc && h->tstage_bytes < tb) {
      if (h->tstage) (void)hipHostFree(h->tstage);
      h->tstage = nullptr;
      h->tstage_bytes = 0;
      OKR_HIP(h, hipHostMalloc(&h->tstage, tb, hipHostMallocDefault));
      h->tstage_bytes = tb;
      h->tstage_fresh = false;
    }
    if (may_alloc && h->tstage) {
      if (!h->tstage_fresh) std::memcpy(h->tstage, h->topo_host.data(), tb);
      h->tstage_fresh = true;
      OKR_HIP(h, hipMemcpyAsync((void*)p.T.parent, h->tstage, tb, hipMemcpyHostToDevice, st));
    } else {
      OKR_HIP(h, hipMemcpyAsync((void*)p.T.parent, h->topo_host.data(), tb, hipMemcpyHostToDevice, st));
    }
  }
  if (dump) {
    h->dump.assign(nseg, {});
    h->dump32.assign(nseg, {});
  }
  if (timing && (int)h->ev.size() < 2 * nseg) {
    drop_events(h);
    h->ev.resize(2 * std::max(nseg, 1), nullptr);
    for (auto& e : h->ev) OKR_HIP(h, hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
  }
  if (mg->flags & OKR_FLAG_AUTOTUNE) {
    // time the scoring launches of a whole search once per candidate group
    // count; keep the fastest per segment size
    if ((int)h->ev.size() < 2 * nseg) {
      drop_events(h);
      h->ev.resize(2 * std::max(nseg, 1), nullptr);
      for (auto& e : h->ev) OKR_HIP(h, hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
    }
    // (the FP64 scoring kernel is tuned whatever the call's precision)
    okr_margins mt = *mg;
    mt.precision = OKR_PRECISION_FP64;
    mt.top_k = 0;
    mt.surrogate = nullptr;
    // tsum[k][mpl index][waves index][groups]
    const int NG = kMaxSnapGroups + 1;
    const int nkey = shape_key(h->kmax + 1, 0);
    std::vector<double> tsum((size_t)nkey * 3 * 3 * NG, 0.0);
    auto T_ = [&](int key, int mi, int wi, int c) -> double& {
      return tsum[(((size_t)key * 3 + mi) * 3 + wi) * NG + c];
    };
    for (int mi = 0; mi < 3; ++mi)
      for (int wi = 0; wi < 3; ++wi)
        for (int c = 1; c <= std::min(S, kMaxSnapGroups); c *= 2) {
          h->sg_force = c;
          h->mpl_force = 1 << mi;
          h->ws_force = 1 << wi;
          enqueue_search(h, d_workspace, Y, loads, &mt, st, &h->ev, nullptr, nullptr, nullptr, nullptr);
          const hipError_t e1 = hipGetLastError(), e2 = hipStreamSynchronize(st);
          if (e1 != hipSuccess || e2 != hipSuccess) {
            h->sg_force = h->mpl_force = h->ws_force = 0;
            OKR_FAIL(h, OKR_E_HIP, "autotune run failed: %s", hipGetErrorString(e1 != hipSuccess ? e1 : e2));
          }
          for (int cc = 0; cc < (int)h->chunk_k.size(); ++cc) {
            const int k = h->chunk_k[cc], nzc = h->chunk_off[cc + 1] - h->chunk_off[cc];
            int spg;
            const int used = snap_groups(h, k, nzc, &spg);
            float ms = 0.f;
            const hipError_t ee = hipEventElapsedTime(&ms, h->ev[2 * cc], h->ev[2 * cc + 1]);
            if (ee != hipSuccess) {
              h->sg_force = h->mpl_force = h->ws_force = 0;
              OKR_FAIL(h, OKR_E_HIP, "autotune timing failed: %s", hipGetErrorString(ee));
            }
            if (used == c) T_(shape_key(k, nzc), mi, wi, c) += ms;
          }
          h->sg_force = h->mpl_force = h->ws_force = 0;
        }
    for (int key = 0; key < nkey; ++key) {
      int bc = 0, bm = 0, bw = 0;
      for (int mi = 0; mi < 3; ++mi)
        for (int wi = 0; wi < 3; ++wi)
          for (int c = 1; c <= kMaxSnapGroups; c *= 2)
            if (T_(key, mi, wi, c) > 0.0 && (bc == 0 || T_(key, mi, wi, c) < T_(key, bm, bw, bc))) {
              bc = c;
              bm = mi;
              bw = wi;
            }
      h->sg_tuned[key] = bc;
      h->mpl_tuned[key] = bc ? 1 << bm : 0;
      h->ws_tuned[key] = bc ? 1 << bw : 0;
    }
    drop_graph(h);  // a captured search used the earlier group counts
  }
  if (graph && st == nullptr) OKR_FAIL(h, OKR_E_ARG, "OKR_FLAG_GRAPH needs a non-null stream (the null stream cannot be captured)");
  if (graph) {
    const double2* V0 = (const double2*)loads->V0;
    const std::vector<uint64_t> key = {
        (uint64_t)d_workspace, (uint64_t)Y->Y_diag, (uint64_t)Y->Y_off, (uint64_t)loads->S_load,
        (uint64_t)loads->Vhat, (uint64_t)st, (uint64_t)mg->flags, bits(mg->e_bar), bits(mg->v_min),
        bits(mg->v_max), bits(mg->tie_tol), bits(mg->amb_tol), bits(mg->pf_tol), (uint64_t)mg->pf_maxit,
        bits(V0[0].x), bits(V0[0].y), bits(V0[1].x), bits(V0[1].y), bits(V0[2].x), bits(V0[2].y),
        (uint64_t)mg->precision, (uint64_t)(int64_t)mg->top_k, (uint64_t)mg->surrogate,
        bits((double)mg->surrogate_margin), bits(mg->mixed_delta), (uint64_t)mg->secondary, bits(mg->smice_tol)};
    if (!h->gexec || key != h->gkey) {
      drop_graph(h);
      OKR_HIP(h, hipStreamSynchronize(st));
      OKR_HIP(h, hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
      // one stream inside the capture (segments in order)
      enqueue_search(h, d_workspace, Y, loads, mg, st, nullptr, nullptr, nullptr, nullptr, nullptr);
      hipGraph_t gobj = nullptr;
      const hipError_t ec = hipStreamEndCapture(st, &gobj);
      if (ec != hipSuccess) OKR_FAIL(h, OKR_E_HIP, "graph capture failed: %s", hipGetErrorString(ec));
      const hipError_t ei = hipGraphInstantiate(&h->gexec, gobj, nullptr, nullptr, 0);
      (void)hipGraphDestroy(gobj);
      if (ei != hipSuccess) {
        h->gexec = nullptr;
        OKR_FAIL(h, OKR_E_HIP, "graph instantiate failed: %s", hipGetErrorString(ei));
      }
      h->gkey = key;
    }
    OKR_HIP(h, hipGraphLaunch(h->gexec, st));
  } else {
    enqueue_search(h, d_workspace, Y, loads, mg, st, timing ? &h->ev : nullptr, dump ? &h->dump : nullptr,
                   dump ? &h->dump32 : nullptr, out->features, out->targets);
    OKR_HIP(h, hipGetLastError());
  }
  // results (one synchronisation)
  std::vector<DevDecision> decs(std::max(nseg, 1));
  std::vector<SegHdr> hdrs(std::max(nseg, 1));
  std::vector<MixedState> mstate(std::max(nseg, 1));
  std::vector<int> gates(std::max(nseg, 1), 1);
  const bool surr_used = mg->top_k > 0 && mg->top_k <= h->topk && mg->surrogate && mg->precision == OKR_PRECISION_FP64;
  const bool mixed = mg->precision == OKR_PRECISION_MIXED;
  std::vector<int> sup(n), kp(n), iters(S, 0), status(kStatusInts, 0);
  // (destination, result-block offset, bytes) of every result read back
  struct Piece {
    void* dst;
    size_t off, bytes;
  };
  std::vector<Piece> pieces;
  auto want = [&](void* dst, size_t off, size_t bytes) {
    if (dst && bytes) pieces.push_back({dst, off, bytes});
  };
  const Layout& L = h->L;
  if (nseg > 0) {
    want(decs.data(), L.decs, sizeof(DevDecision) * nseg);
    want(hdrs.data(), L.hdrs, sizeof(SegHdr) * nseg);
    if (mixed) want(mstate.data(), L.mstate, sizeof(MixedState) * nseg);
    if (surr_used || mixed) want(gates.data(), L.sgates, sizeof(int) * nseg);
  }
  want(sup.data(), L.sup, sizeof(int) * n);
  want(kp.data(), L.kp, sizeof(int) * n);
  want(status.data(), L.status, sizeof(int) * kStatusInts);
  if (!vhat_given) want(iters.data(), L.iters, sizeof(int) * S);
  want(out->Yk_diag, L.Ykd, sizeof(double2) * 9 * n);
  want(out->Yk_off, L.Yko, sizeof(double2) * 9 * n);
  want(out->err_per_snapshot, L.err, sizeof(double) * S);
  if (may_alloc && h->rstage_bytes < L.res_bytes) {
    if (h->rstage) (void)hipHostFree(h->rstage);
    h->rstage = nullptr;
    h->rstage_bytes = 0;
    OKR_HIP(h, hipHostMalloc(&h->rstage, L.res_bytes, hipHostMallocDefault));
    h->rstage_bytes = L.res_bytes;
  }
  const bool staged = may_alloc && h->rstage;
  if (staged) {  // the whole result block in one transfer, then placed on the host
    OKR_HIP(h, hipMemcpyAsync(h->rstage, (const char*)d_workspace + L.res0, L.res_bytes, hipMemcpyDeviceToHost, st));
  } else {
    for (const Piece& q : pieces)
      OKR_HIP(h, hipMemcpyAsync(q.dst, (const char*)d_workspace + q.off, q.bytes, hipMemcpyDeviceToHost, st));
  }
  if (out->Vhat)
    OKR_HIP(h, hipMemcpyAsync(out->Vhat, p.Vhat, sizeof(double2) * (size_t)S * n * 3, hipMemcpyDeviceToHost, st));
  OKR_HIP(h, hipStreamSynchronize(st));
  if (staged)
    for (const Piece& q : pieces) std::memcpy(q.dst, (const char*)h->rstage + (q.off - L.res0), q.bytes);
  const auto t1 = clk::now();
  const int hs = status[0];
  if (hs & 1) OKR_FAIL(h, OKR_E_SINGULAR, "a present-phase branch block is singular");
  if (hs & 2) OKR_FAIL(h, OKR_E_PHASE, "nonzero admittance entries on absent phases");
  if (hs & (4 | 8)) OKR_FAIL(h, OKR_E_UNSUPPORTED, "admittance blocks asymmetric or with shunts");
  if (hs & 16) OKR_FAIL(h, OKR_E_PF_DIVERGED, "load flow did not converge");
  if (hs & 64) OKR_FAIL(h, OKR_E_ARG, "internal: a segment's tables failed a structural check");
  const bool base_out = (hs & 32) != 0;
  out->warnings = base_out ? OKR_W_BASE_OUT_OF_BAND : 0;
  out->score_kernel_ms = 0.0;
  out->algorithmic_flops = 0.0;
  out->kernel_form_flops = 0.0;
  std::vector<uint8_t> keep_before(n, 1);  // kept state before each segment, in segment order
  const int nchunk = (int)h->chunk_k.size();
  out->n_score_launches = nchunk;
  std::vector<int> chunk_of(std::max(nseg, 1), 0);
  for (int c = 0; c < nchunk; ++c)
    for (int i = h->chunk_off[c]; i < h->chunk_off[c + 1]; ++i) chunk_of[h->chunk_segs[i]] = c;
  std::vector<float> chunk_ms(std::max(nchunk, 1), 0.f);
  if (timing)
    for (int c = 0; c < nchunk; ++c) {
      OKR_HIP(h, hipEventElapsedTime(&chunk_ms[c], h->ev[2 * c], h->ev[2 * c + 1]));
      out->score_kernel_ms += chunk_ms[c];
    }
  for (int g = 0; g < nseg; ++g) {
    okr_segment_result& R = out->seg[g];
    std::memset(&R, 0, sizeof R);
    const int k = h->seg_off[g + 1] - h->seg_off[g];
    R.segment = g;
    R.k = k;
    R.mask = decs[g].mask;
    R.popcount = decs[g].popcount;
    R.e_loc = decs[g].e_loc;
    R.e_min = decs[g].e_min;
    R.ambiguous = decs[g].ambiguous;
    R.key_gap = decs[g].key_gap;
    R.smice_rise = mg->secondary == OKR_SECONDARY_SMICE ? decs[g].smice_rise : NAN;
    R.n_scored = 1 << k;
    {
      // launch shape of the segment's chunk (set by its largest segment)
      const int kc = h->chunk_k[chunk_of[g]];
      int spg;
      const int nzc = h->chunk_off[chunk_of[g] + 1] - h->chunk_off[chunk_of[g]];
      R.score_groups = snap_groups(h, kc, nzc, &spg);
      R.score_mpl = sv_spp(score_mpl(h, kc, nzc), kc, spg);
      R.score_waves = score_ws(h, kc, nzc);
      R.chunk = chunk_of[g];
    }
    // the scoring kernel's own FP64 work: per slot and mask, reduced ->
    // 6 + 4|phi|, kept -> 14|phi| (half the masks each); per zone entry 14
    double fl = 0.0;
    for (int q = h->seg_off[g]; q < h->seg_off[g + 1]; ++q) {
      const int np = __builtin_popcount(h->phase[h->seg_nodes[q]]);
      fl += 0.5 * (6.0 + 4.0 * np) + 0.5 * (14.0 * np);
    }
    fl += 14.0 * hdrs[g].nz;
    const bool per_mask = mg->precision != OKR_PRECISION_FP64_FACTORED;
    R.kernel_flops = per_mask ? fl * double(int64_t(1) << k) * S : 0.0;
    out->kernel_form_flops += R.kernel_flops;
    R.flops = per_mask ? method_flops(h, g, keep_before, S) : 0.0;
    out->algorithmic_flops += R.flops;
    for (int j = 0; j < k; ++j)  // the state the next segments see
      if (decs[g].mask >> j & 1u) keep_before[h->seg_nodes[h->seg_off[g] + j]] = 0;
    if (mixed) {  // (every mask again in FP64 when the deviation exceeded the bound)
      R.n_refined = mstate[g].nA + mstate[g].nB + (gates[g] ? (1 << k) : 0);
      R.fp32_dev = mstate[g].max_dev;
    }
    if (surr_used) {
      R.n_refined = std::min(mg->top_k, 1 << k);
      R.n_scored = R.n_refined + (gates[g] ? (1 << k) : 0);
    }
    if (timing) {  // the chunk's scoring time, split evenly over its segments
      const int c = chunk_of[g];
      R.score_ms = chunk_ms[c] / (float)(h->chunk_off[c + 1] - h->chunk_off[c]);
    }
  }
  int nk = 0;
  for (int i = 0; i < n; ++i) {
    out->super[i] = sup[i];
    out->kept_parent[i] = kp[i];
    nk += (sup[i] == i);
  }
  out->n_kept = nk;
  out->pf_iterations = iters.empty() ? 0 : *std::max_element(iters.begin(), iters.end());
  out->max_err = 0.0;
  if (out->err_per_snapshot)
    for (int l = 0; l < S; ++l) out->max_err = std::max(out->max_err, out->err_per_snapshot[l]);
  out->t_setup_ms = 0.0;
  out->t_pf_ms = 0.0;
  out->t_search_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
  out->t_final_ms = 0.0;
  return base_out ? OKR_W_BASE_OUT_OF_BAND : OKR_OK;
}

extern "C" int okr_dump_scores(okr_handle* h, int32_t segment, double* e, double* slack, int32_t* k) {
  if (!h) return OKR_E_ARG;
  const bool have = segment >= 0 && segment < (int)h->dump.size() &&
                    (!h->dump[segment].empty() || (segment < (int)h->dump32.size() && !h->dump32[segment].empty()));
  if (!have) OKR_FAIL(h, OKR_E_ARG, "no scores kept for segment %d (set OKR_FLAG_DUMP_SCORES)", segment);
  const std::vector<MaskScore>& d = h->dump[segment];
  for (size_t m = 0; m < d.size(); ++m) {
    if (e) e[m] = d[m].e;
    if (slack) slack[m] = d[m].slack;
  }
  if (d.empty() && segment < (int)h->dump32.size()) {
    const std::vector<MaskScore32>& d32 = h->dump32[segment];
    for (size_t m = 0; m < d32.size(); ++m) {
      if (e) e[m] = d32[m].e;
      if (slack) slack[m] = d32[m].slack;
    }
  }
  if (k) *k = h->seg_off[segment + 1] - h->seg_off[segment];
  return OKR_OK;
}

// Self-test of the scoring kernel's square root (device pointers, n values).
extern "C" int okr_selftest_sqrt(const double* d_x, double* d_y, int n, void* stream) {
  if (!d_x || !d_y || n < 0) return OKR_E_ARG;
  hipLaunchKernelGGL(k_sqrt_selftest, dim3((n + 255) / 256), dim3(256), 0, static_cast<hipStream_t>(stream), d_x,
                     d_y, n);
  return hipGetLastError() == hipSuccess ? OKR_OK : OKR_E_HIP;
}

// ------------------------------------------------------------ surrogate --
namespace {

struct SurrWork {
  __bf16 *Xb, *Xt, *H1b, *H1t, *dZ2b, *dZ2t, *dZ1t, *W1b, *W2b, *W2tb;
  float *Z1, *Z2, *part, *y, *dy, *dH1, *gW1full, *grads, *m, *v, *loss, *colpart, *gpart;
  size_t bytes;
};

constexpr int kMaxEpochs = 4096;
constexpr int kColChunkHost = 256;  // rows per partial column sum (k_colsums_part)
constexpr int kSplitK = 256;        // batch rows per K slice of the weight-gradient GEMMs

// K slices of the weight-gradient GEMMs for a batch of B rows (B % 64 == 0).
int surr_splits(int B) { return (B % kSplitK == 0) ? B / kSplitK : 1; }

SurrWork surr_layout(int B, void* base) {
  SurrWork w{};
  size_t off = 0;
  char* b = static_cast<char*>(base);
  auto take = [&](size_t bytes) {
    void* p = b ? (void*)(b + off) : nullptr;
    off = align256(off + bytes);
    return p;
  };
  const size_t bf = sizeof(uint16_t), f4 = sizeof(float);
  w.Xb = (__bf16*)take(bf * B * kSurrF);
  w.Xt = (__bf16*)take(bf * 64 * B);
  w.H1b = (__bf16*)take(bf * B * kSurrH);
  w.H1t = (__bf16*)take(bf * kSurrH * B);
  w.dZ2b = (__bf16*)take(bf * B * kSurrH);
  w.dZ2t = (__bf16*)take(bf * kSurrH * B);
  w.dZ1t = (__bf16*)take(bf * kSurrH * B);
  w.W1b = (__bf16*)take(bf * kSurrH * kSurrF);
  w.W2b = (__bf16*)take(bf * kSurrH * kSurrH);
  w.W2tb = (__bf16*)take(bf * kSurrH * kSurrH);
  w.Z1 = (float*)take(f4 * B * kSurrH);
  w.Z2 = (float*)take(f4 * B * kSurrH);
  w.part = (float*)take(f4 * (kSurrH / 32) * B);
  w.y = (float*)take(f4 * B);
  w.dy = (float*)take(f4 * B);
  w.dH1 = (float*)take(f4 * B * kSurrH);
  w.gW1full = (float*)take(f4 * kSurrH * 64);
  w.grads = (float*)take(f4 * kSurrParams);
  w.m = (float*)take(f4 * kSurrParams);
  w.v = (float*)take(f4 * kSurrParams);
  w.loss = (float*)take(f4 * kMaxEpochs);
  w.colpart = (float*)take(f4 * (3 * kSurrH + 1) * ((B + kColChunkHost - 1) / kColChunkHost));
  w.gpart = (float*)take(f4 * kSurrH * kSurrH * surr_splits(B));
  w.bytes = off;
  return w;
}

// Forward of one batch (B rows of FP32 features at X) into w.y; with `train`
// the pre-activations and the transposed activations are kept for backward.
void surr_forward(const SurrWork& w, const float* prm, const float* X, int B, bool train, hipStream_t st) {
  hipLaunchKernelGGL(k_batch_cast, dim3((B * 64 + 255) / 256), dim3(256), 0, st, X, B, w.Xb, w.Xt);
  hipLaunchKernelGGL(k_gemm_nt<1>, dim3(kSurrH / 64, B / 64), dim3(256), 0, st, (const __bf16*)w.Xb, kSurrF,
                     (const __bf16*)w.W1b, kSurrF, kSurrF, (float*)nullptr, kSurrH, prm + kOffB1,
                     train ? w.Z1 : (float*)nullptr, w.H1b, train ? w.H1t : (__bf16*)nullptr, B, (const float*)nullptr,
                     (float*)nullptr, (const int*)nullptr, 0);
  hipLaunchKernelGGL(k_gemm_nt<2>, dim3(kSurrH / 64, B / 64), dim3(256), 0, st, (const __bf16*)w.H1b, kSurrH,
                     (const __bf16*)w.W2b, kSurrH, kSurrH, (float*)nullptr, kSurrH, prm + kOffB2,
                     train ? w.Z2 : (float*)nullptr, (__bf16*)nullptr, (__bf16*)nullptr, B, prm + kOffW3, w.part,
                     (const int*)nullptr, 0);
  hipLaunchKernelGGL(k_rowdot_finish, dim3((B + 255) / 256), dim3(256), 0, st, (const float*)w.part, kSurrH / 32, B,
                     prm + kOffB3, w.y, (const int*)nullptr, 0);
}

// Loss gradient of one batch into w.grads; the batch loss is added to *loss.
void surr_backward(const SurrWork& w, const float* prm, const float* t, int B, float* loss, hipStream_t st) {
  hipLaunchKernelGGL(k_loss_dy, dim3((B + 255) / 256), dim3(256), 0, st, (const float*)w.y, t, B, w.dy, loss);
  hipLaunchKernelGGL(k_dz2, dim3((B * kSurrH + 255) / 256), dim3(256), 0, st, (const float*)w.Z2, (const float*)w.dy,
                     prm + kOffW3, B, w.dZ2b, w.dZ2t);
  // dW2 = dZ2^T H1, K = B split into slices of kSplitK rows
  const int splits = surr_splits(B);
  hipLaunchKernelGGL(k_gemm_nt<0>, dim3(kSurrH / 64, kSurrH / 64, splits), dim3(256), 0, st, (const __bf16*)w.dZ2t,
                     B, (const __bf16*)w.H1t, B, B, w.gpart, kSurrH, (const float*)nullptr, (float*)nullptr,
                     (__bf16*)nullptr, (__bf16*)nullptr, kSurrH, (const float*)nullptr, (float*)nullptr,
                     (const int*)nullptr, 0);
  hipLaunchKernelGGL(k_sum_splits, dim3(kSurrH * kSurrH / 256), dim3(256), 0, st, (const float*)w.gpart, splits,
                     kSurrH * kSurrH, w.grads + kOffW2);
  // dH1 = dZ2 W2
  hipLaunchKernelGGL(k_gemm_nt<0>, dim3(kSurrH / 64, B / 64), dim3(256), 0, st, (const __bf16*)w.dZ2b, kSurrH,
                     (const __bf16*)w.W2tb, kSurrH, kSurrH, w.dH1, kSurrH, (const float*)nullptr, (float*)nullptr,
                     (__bf16*)nullptr, (__bf16*)nullptr, B, (const float*)nullptr, (float*)nullptr,
                     (const int*)nullptr, 0);
  hipLaunchKernelGGL(k_dz1, dim3((B * kSurrH + 255) / 256), dim3(256), 0, st, (const float*)w.dH1, (const float*)w.Z1,
                     B, w.dZ1t);
  // dW1 = dZ1^T X (X^T padded to 64 rows), split like dW2
  hipLaunchKernelGGL(k_gemm_nt<0>, dim3(1, kSurrH / 64, splits), dim3(256), 0, st, (const __bf16*)w.dZ1t, B,
                     (const __bf16*)w.Xt, B, B, w.gpart, 64, (const float*)nullptr, (float*)nullptr,
                     (__bf16*)nullptr, (__bf16*)nullptr, kSurrH, (const float*)nullptr, (float*)nullptr,
                     (const int*)nullptr, 0);
  hipLaunchKernelGGL(k_sum_splits, dim3(kSurrH * 64 / 256), dim3(256), 0, st, (const float*)w.gpart, splits,
                     kSurrH * 64, w.gW1full);
  hipLaunchKernelGGL(k_copy_cols, dim3((kSurrH * kSurrF + 255) / 256), dim3(256), 0, st, (const float*)w.gW1full, 64,
                     w.grads + kOffW1, kSurrH, kSurrF);
  const int nchunk = (B + kColChunkHost - 1) / kColChunkHost;
  hipLaunchKernelGGL(k_colsums_part, dim3(nchunk), dim3(kSurrH + 1), 0, st, (const float*)w.Z1, (const float*)w.dH1,
                     (const float*)w.Z2, (const float*)w.dy, prm + kOffW3, B, w.colpart);
  hipLaunchKernelGGL(k_colsums_final, dim3((3 * kSurrH + 1 + 255) / 256), dim3(256), 0, st, (const float*)w.colpart,
                     nchunk, w.grads + kOffB1, w.grads + kOffB2, w.grads + kOffW3, w.grads + kOffB3);
}

void surr_refresh(const SurrWork& w, const float* prm, hipStream_t st) {
  hipLaunchKernelGGL(k_refresh_weights, dim3((kSurrH * kSurrH + 255) / 256), dim3(256), 0, st, prm, w.W1b, w.W2b,
                     w.W2tb);
}

}  // namespace

extern "C" int okr_surrogate_workspace(int32_t batch, size_t* bytes) {
  if (!bytes || batch < 64 || batch % 64) return OKR_E_ARG;
  *bytes = surr_layout(batch, nullptr).bytes;
  return OKR_OK;
}

extern "C" int okr_surrogate_grad(const float* params, const float* X, const float* t, int32_t B, float* grads,
                                  float* loss, void* work, size_t work_bytes, void* stream) {
  if (!params || !X || !t || !grads || B < 64 || B % 64 || !work) return OKR_E_ARG;
  const SurrWork w = surr_layout(B, work);
  if (work_bytes < w.bytes) return OKR_E_WORKSPACE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  surr_refresh(w, params, st);
  hipLaunchKernelGGL(k_zero_f32, dim3(1), dim3(64), 0, st, w.loss, 1);
  surr_forward(w, params, X, B, true, st);
  surr_backward(w, params, t, B, w.loss, st);
  if (hipMemcpyAsync(grads, w.grads, sizeof(float) * kSurrParams, hipMemcpyDeviceToDevice, st) != hipSuccess)
    return OKR_E_HIP;
  float l = 0.f;
  if (hipMemcpyAsync(&l, w.loss, sizeof(float), hipMemcpyDeviceToHost, st) != hipSuccess) return OKR_E_HIP;
  if (hipStreamSynchronize(st) != hipSuccess) return OKR_E_HIP;
  if (loss) *loss = l;
  return hipGetLastError() == hipSuccess ? OKR_OK : OKR_E_HIP;
}

extern "C" int okr_train_surrogate(const float* X, const float* t, int64_t n, int32_t epochs, int32_t batch, float lr,
                                   uint64_t seed, float* params, void* work, size_t work_bytes, void* stream,
                                   float* loss) {
  if (!X || !t || !params || !work || batch < 64 || batch % 64 || epochs < 1 || epochs > kMaxEpochs ||
      n < batch)
    return OKR_E_ARG;
  const SurrWork w = surr_layout(batch, work);
  if (work_bytes < w.bytes) return OKR_E_WORKSPACE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t nb = n / batch;
  hipLaunchKernelGGL(k_zero_f32, dim3((kSurrParams + 255) / 256), dim3(256), 0, st, w.m, kSurrParams);
  hipLaunchKernelGGL(k_zero_f32, dim3((kSurrParams + 255) / 256), dim3(256), 0, st, w.v, kSurrParams);
  hipLaunchKernelGGL(k_zero_f32, dim3((epochs + 255) / 256), dim3(256), 0, st, w.loss, epochs);
  std::vector<int64_t> order(nb);
  uint64_t rng = seed * 0x9E3779B97F4A7C15ull + 1;
  int64_t step = 0;
  for (int e = 0; e < epochs; ++e) {
    for (int64_t q = 0; q < nb; ++q) order[q] = q;
    for (int64_t q = nb - 1; q > 0; --q) {  // Fisher-Yates with a 64-bit LCG
      rng = rng * 6364136223846793005ull + 1442695040888963407ull;
      std::swap(order[q], order[(int64_t)((rng >> 33) % (uint64_t)(q + 1))]);
    }
    for (int64_t q = 0; q < nb; ++q) {
      const int64_t off = order[q] * batch;
      surr_refresh(w, params, st);
      surr_forward(w, params, X + off * kSurrF, batch, true, st);
      surr_backward(w, params, t + off, batch, w.loss + e, st);
      ++step;
      const float c1 = 1.f - std::pow(0.9f, (float)step), c2 = 1.f - std::pow(0.999f, (float)step);
      hipLaunchKernelGGL(k_adam, dim3((kSurrParams + 255) / 256), dim3(256), 0, st, params, (const float*)w.grads,
                         w.m, w.v, kSurrParams, lr, c1, c2);
    }
  }
  std::vector<float> lh(epochs);
  if (hipMemcpyAsync(lh.data(), w.loss, sizeof(float) * epochs, hipMemcpyDeviceToHost, st) != hipSuccess)
    return OKR_E_HIP;
  if (hipStreamSynchronize(st) != hipSuccess) return OKR_E_HIP;
  if (loss)
    for (int e = 0; e < epochs; ++e) loss[e] = lh[e] / (float)nb;
  return hipGetLastError() == hipSuccess ? OKR_OK : OKR_E_HIP;
}

extern "C" int okr_surrogate_forward(const float* params, const float* X, int64_t n, float* y, void* work,
                                     size_t work_bytes, void* stream) {
  if (!params || !X || !y || !work || n < 64 || n % 64) return OKR_E_ARG;
  const SurrWork w = surr_layout((int)n, work);
  if (work_bytes < w.bytes) return OKR_E_WORKSPACE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  surr_refresh(w, params, st);
  surr_forward(w, params, X, (int)n, false, st);
  if (hipMemcpyAsync(y, w.y, sizeof(float) * n, hipMemcpyDeviceToDevice, st) != hipSuccess) return OKR_E_HIP;
  if (hipStreamSynchronize(st) != hipSuccess) return OKR_E_HIP;
  return hipGetLastError() == hipSuccess ? OKR_OK : OKR_E_HIP;
}
