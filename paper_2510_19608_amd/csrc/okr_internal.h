// Internal tables shared by the host planner and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace okr {

constexpr int kMaxK = 24;                    // eligible nodes per segment
constexpr int kMaxPairs = kMaxK * (kMaxK + 1) / 2;  // (super slot, reduced slot) pairs
constexpr int kScoreBlock = 64;              // masks per tile record (one wave)
constexpr int kScoreThreads = 256;           // scoring block: 4 waves, one mask per lane

// Header of one segment's tables (one per segment, in device memory), written
// by the device-side builder; offsets index the int32 table buffer.
struct SegHdr {
  int g;          // segment id
  int valid;      // 0 if a structural invariant failed
  int k;          // eligible nodes in the segment
  int nchains;    // chains of the affected region
  int nslots;     // == k (every segment node is a slot of exactly one chain)
  int npairs;     // sum over chains of j(j+1)/2
  int nz;         // zone entries (kept target node, phase)
  int S;          // snapshots
  int nrange;     // preorder ranges whose union is Omega_g
  int nomega;     // nodes in Omega_g
  int o_chain;    // [nchains][kChainInts]
  int o_nest;     // nesting paths, outermost first, ending with the chain itself
  int o_slot;     // [nslots][kSlotInts]
  int o_pair;     // [npairs][kPairInts]
  int o_range;    // [nrange][3]: preorder start, end, cumulative node count
  int o_zent;     // [nz][3]: node, phase, chain
  int total_ints;
  int npat;       // chain patterns: sum over chains of 2^popcount(C_PMASK)
  int lanebits;   // the mask bits that vary across a scoring wave's 64 lanes
                  // (6 of them, all k when k < 6); a tile is the 64 masks
                  // sharing every other bit (tile_mask)
};

// Mask of scoring tile t, lane q: q's bits at the positions of the segment's
// lane bits L, t's bits at the other positions of the k mask bits.
// (lane_part: q's bits at L's positions; tile_part: t's bits at the others)
__host__ __device__ __forceinline__ uint32_t lane_part(uint32_t L, uint32_t q) {
  uint32_t m = 0;
  for (uint32_t l = L; l; l &= l - 1, q >>= 1) m |= (q & 1u) << __builtin_ctz(l);
  return m;
}
__host__ __device__ __forceinline__ uint32_t tile_part(uint32_t L, uint32_t t, int k) {
  uint32_t m = 0;
  for (uint32_t o = ((k >= 32 ? 0u : (1u << k)) - 1u) & ~L; o; o &= o - 1, t >>= 1) m |= (t & 1u) << __builtin_ctz(o);
  return m;
}
__host__ __device__ __forceinline__ uint32_t tile_mask(uint32_t L, uint32_t t, uint32_t q, int k) {
  return tile_part(L, t, k) | lane_part(L, q);
}

// A search step launched over a chunk of mutually independent segments:
// blockIdx.z picks the segment (segs[blockIdx.z]) and its scratch block; each
// per-segment scratch buffer of chunk position z lies z * lstride bytes after
// position 0's.
template <typename T>
__device__ __forceinline__ T* lane_ptr(T* p, size_t lstride) {
  return p ? (T*)((char*)p + (size_t)blockIdx.z * lstride) : p;
}

// Read-only int tables (segment structure) in the constant address space:
// kernels never write them while reading, so wave-uniform reads compile to
// scalar loads through the scalar cache instead of per-lane vector loads.
typedef __attribute__((address_space(4))) const int cint;
__device__ __forceinline__ const cint* as_cint(const int* p) { return (const cint*)p; }
// The header of the segment at chunk position blockIdx.z, by scalar loads
// (only for kernels that do not write headers or segment ids).
__device__ __forceinline__ SegHdr load_hdr_g(const SegHdr* hdrs, int g) {
  const cint* src = as_cint((const int*)(hdrs + g));
  SegHdr H;
  int* dst = (int*)&H;
#pragma unroll
  for (int q = 0; q < (int)(sizeof(SegHdr) / sizeof(int)); ++q) dst[q] = src[q];
  return H;
}
__device__ __forceinline__ SegHdr load_hdr(const SegHdr* hdrs, const int* segs) {
  return load_hdr_g(hdrs, *as_cint(segs + blockIdx.z));
}

// Static topology on the device.
struct Topo {
  int n;
  const int* parent;
  const uint8_t* phase;
  const int* segment;
  const int* pos;       // DFS preorder position
  const int* size;      // subtree size
  const int* pre;       // preorder -> node
  const int* ch_off;    // children CSR
  const int* ch;
  const int* seg_off;   // segment -> first index in seg_nodes
  const int* seg_nodes; // segment nodes in DFS preorder
  const int* seg_top;   // segment node -> highest ancestor reachable through its own segment's nodes
};

// Cumulative search state on the device.
struct State {
  uint8_t* kept;  // 1 while the node is kept
  int* sup;       // nearest kept ancestor (inclusive)
  int* slot_of;   // node -> slot of the segment being scored, -1 otherwise
  int* zent_of;   // node*3+phase -> zone entry of the segment being scored, -1 otherwise
};

// chain record
enum { C_HEAD = 0, C_NSLOT, C_SLOT0, C_NEST_OFF, C_NEST_LEN,
       C_ZOFF0, C_ZOFF1, C_ZOFF2, C_ZCNT0, C_ZCNT1, C_ZCNT2, C_OUTER, C_PHASE,
       C_BIT0,   // mask bit of the first slot; slot r has bit C_BIT0 + r
       C_PAIR0,  // first pair of the chain; slot r's pairs start at C_PAIR0 + r(r+1)/2
       C_PHW0, C_PHW1, C_PHW2,  // phase masks of slots 8w..8w+7, 3 bits each
       C_PMASK,  // mask bits the chain's terms depend on: its slots and those of its nesting path
       C_PBASE,  // first entry of the chain's patterns in the segment's pattern table
       kChainInts };
// slot record
enum { SL_NODE = 0, SL_BIT, SL_PHASE, SL_PAIRBASE, SL_CHAIN, kSlotInts };
// pair record: reduced slot node, its super-node for this pair, and the
// reduced slot's index
enum { PR_RNODE = 0, PR_SUPER, PR_RSLOT, kPairInts };

// Per-slot and per-zone-entry numeric data for one snapshot and phase.
struct TargetRec {
  double2 W;   // current voltage of the kept node the entry evaluates
  double lo;   // min |V^| over the cluster's members on that phase
  double hi;   // max |V^| over the cluster's members on that phase
};

// Decision written by the arg-min kernel.
struct DevDecision {
  uint32_t mask;
  int32_t popcount;
  double e_loc;
  double e_min;
  int32_t ambiguous;
  int32_t found;
  double key_gap;  // smallest key above the tie window at the chosen level, minus the smallest (inf if none)
  double smice_rise;  // with SMICE as the key: SMICE of the chosen mask minus SMICE of mask 0
};

// Per-mask partial score: max error and min band slack over a snapshot group.
struct MaskScore {
  double e;
  double slack;
};

// Chain-pattern score: max error and extreme kept squared magnitudes of one
// chain's terms (its slots and zone entries) over every snapshot, for one
// assignment of the mask bits in C_PMASK.
struct PatScore {
  double e, qmin, qmax;
};

// Per-tile (64 consecutive masks) summary written by the last scoring block
// of the tile: best feasible level, smallest error at that level, highest
// level of a near-boundary mask.
struct TileRec {
  int32_t best;   // max popcount of a feasible mask, -1 if none
  int32_t near;   // max popcount of a mask near the e_bar / band boundary, -1 if none
  double emin;    // min error among feasible masks at `best`
};

// Selection parameters shared by the scoring epilogue and the arg-min.
// delta bounds |e32 - e64| and |slack32 - slack64| of the FP32 screening pass.
struct SelParams {
  double e_bar, vmin, vmax, tie, amb, delta;
};

// ---- mixed precision (FP32 screening in difference form, FP64 refine) ----
// Every error term is (FP64 difference rounded to FP32) +/- d, where
// d = |W + S| - |W| = (2 Re(conj(W) S) + |S|^2) / (|W + S| + |W|) is the
// FP32 voltage-magnitude change; so FP32 rounding acts on small quantities.
struct Pair32 {      // per (snapshot, pair, phase)
  float2 P;          // Z(super -> reduced) A_reduced
  float a, b;        // |W_super| - lo_reduced, hi_reduced - |W_super|  (-inf on absent phases)
};
struct Rec32 {       // per (snapshot, slot or zone entry, phase)
  float2 W;          // current voltage
  float w;           // |W|
  float a, b;        // w - lo, hi - w of the node's own cluster (-inf on absent phases)
  float bmin, bmax;  // w - v_min, v_max - w (+inf on absent phases)
  float pad;
};
struct Head32 {      // per (snapshot, chain, phase)
  float2 W;
  float w;
  float pad;
};
struct MaskScore32 {
  float e, slack;
};
struct TileRec32 {   // max popcount of sure-feasible / possibly-feasible / uncertain masks
  int sure, poss, unc, pad;
};
// ---- surrogate ----
constexpr int kSurrF = 32;    // features per mask (16 used, zero padded)
constexpr int kSurrH = 256;   // hidden width
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kSurrH * kSurrF;
constexpr int kOffW2 = kOffB1 + kSurrH;
constexpr int kOffB2 = kOffW2 + kSurrH * kSurrH;
constexpr int kOffW3 = kOffB2 + kSurrH;
constexpr int kOffB3 = kOffW3 + kSurrH;
constexpr int kSurrParams = kOffB3 + 1;
struct SurrSlot {   // per slot of the segment being ranked
  float la;         // max over snapshots of the slot's aggregated load current
  float spread;     // max over snapshots and phases of its cluster's |V^| spread
  int nph;          // phases
  int pos;          // position in its chain
};

// SMICE prep table (int32, per segment): head count, zone-target count, head
// index of each chain, head nodes, head-inside-Omega flags, first zone target
// of each chain, then the zone targets [node, entry of phases 0..2 (-1 if
// absent), head index (-1 if not a head)].
enum { SM_NH = 0, SM_NZN = 1, SM_CHX = 2, SM_HNODE = SM_CHX + kMaxK, SM_HIN = SM_HNODE + kMaxK,
       SM_ZOFF = SM_HIN + kMaxK, SM_ZREC = SM_ZOFF + kMaxK + 1 };
constexpr int kZrecInts = 5;

struct MixedState {  // per segment: the screening levels and shortlist sizes
  int lo_level, hi_level, best, nA, nB, pad;
  double e_up;
  double max_dev;    // max |e32 - e64| over refined masks with e64 <= 2 e_bar
};

}  // namespace okr
