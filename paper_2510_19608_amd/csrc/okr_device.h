// Device helpers shared by the FP64 scoring and refine kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "okr_internal.h"

namespace okr {

// ---------------------------------------------------------------- complex --
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }
__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
  const double d = cabs2(b);
  const double2 t = cmul(a, cconj(b));
  return make_double2(t.x / d, t.y / d);
}
// Note: the bare v_sqrt_f64 instruction is accurate to only about 2^-27
// relative, far outside the 1e-13 decision window; magnitudes in the scoring
// use sqrt_nr() below, elsewhere the libm sqrt.

// ---------------------------------------------------------------- scoring --
// sqrt for arguments in the normal range (here |V|^2 of a bus voltage): the
// hardware reciprocal-square-root estimate refined by Newton-Raphson steps in
// Goldschmidt form (g -> sqrt(x), h -> 1/(2 sqrt(x))), two residual
// corrections at the end.  No range scaling: callers pass x in [2^-500, 2^500].
__device__ __forceinline__ double sqrt_nr(double x) {
  const double r = __builtin_amdgcn_rsq(x);
  double g = x * r, h = 0.5 * r;
  const double e = fma(-h, g, 0.5);
  g = fma(g, e, g);
  h = fma(h, e, h);
  double d = fma(-g, g, x);
  g = fma(d, h, g);
  d = fma(-g, g, x);
  return fma(d, h, g);
}
__device__ __forceinline__ double vmag(double2 a) { return sqrt_nr(a.x * a.x + a.y * a.y); }
// Magnitude of a chain head's voltage (mask-independent for chains that are
// not nested below another chain), one fixed evaluation order.
__device__ __forceinline__ double hmag(double2 a) { return sqrt_nr(fma(a.x, a.x, a.y * a.y)); }

// Walk one chain for one mask: super-node slots top to bottom; a reduced slot
// adds the voltage rise of moving its aggregated current to its current super
// (P from LDS); a kept slot becomes the super of the slots below it.  With
// ERR, every slot cluster's error against its super's magnitude is folded
// into el, and the squared magnitudes of kept slots into (qmin, qmax) for the
// band (the slack is formed once per mask: sqrt is monotone, so
// min(|V| - vmin) = sqrt(min |V|^2) - vmin exactly).  Structure records are
// wave-uniform (scalar loads, uniform phase branches); P entries depend on the
// lane's super slot.
template <bool ERR>
__device__ __forceinline__ void walk_chain(const int* __restrict__ cr, const int* __restrict__ slots,
                                           const double2* Ps, const TargetRec* Ss, const double2* Hs,
                                           const double* Hm, int c, uint32_t m, double2& B0, double2& B1,
                                           double2& B2, double& el, double& qmin, double& qmax) {
  double2 S0 = B0, S1 = B1, S2 = B2;
  double sm0 = 0.0, sm1 = 0.0, sm2 = 0.0;
  if (ERR) {
    const int hph = cr[C_PHASE];
    const double2* hv = Hs + c * 3;
    if (cr[C_OUTER] < 0) {  // head unaffected by the mask
      if (Hm) {
        sm0 = Hm[c * 3];
        sm1 = Hm[c * 3 + 1];
        sm2 = Hm[c * 3 + 2];
      } else {
        if (hph & 1) sm0 = hmag(hv[0]);
        if (hph & 2) sm1 = hmag(hv[1]);
        if (hph & 4) sm2 = hmag(hv[2]);
      }
    } else {
      if (hph & 1) sm0 = vmag(cadd(hv[0], B0));
      if (hph & 2) sm1 = vmag(cadd(hv[1], B1));
      if (hph & 4) sm2 = vmag(cadd(hv[2], B2));
    }
  }
  const int ns = cr[C_NSLOT], s0 = cr[C_SLOT0];
  int sidx = 0;
  for (int r = 0; r < ns; ++r) {
    const int* sr = slots + (s0 + r) * kSlotInts;
    const int bit = sr[SL_BIT], pb = sr[SL_PAIRBASE], ph = sr[SL_PHASE];
    const bool red = (m >> bit) & 1u;
    const double rf = red ? 1.0 : 0.0;
    const double2* pp = Ps + (pb + sidx) * 3;
    const TargetRec* tr = Ss + (s0 + r) * 3;
#define OKR_SLOT_PHASE(P_, S_, SM_)                                              \
    if (ph & (1 << P_)) {                                                        \
      const double2 pv = pp[P_];                                                 \
      S_.x = fma(rf, pv.x, S_.x);                                                \
      S_.y = fma(rf, pv.y, S_.y);                                                \
      if (ERR) {                                                                 \
        const TargetRec t = tr[P_];                                              \
        const double vx = t.W.x + S_.x, vy = t.W.y + S_.y;                       \
        const double q = fma(vx, vx, vy * vy);                                   \
        if (!red) SM_ = sqrt_nr(q);                                              \
        qmin = fmin(qmin, red ? INFINITY : q);                                   \
        qmax = fmax(qmax, red ? -INFINITY : q);                                  \
        el = fmax(el, fmax(SM_ - t.lo, t.hi - SM_));                             \
      }                                                                          \
    }
    OKR_SLOT_PHASE(0, S0, sm0)
    OKR_SLOT_PHASE(1, S1, sm1)
    OKR_SLOT_PHASE(2, S2, sm2)
#undef OKR_SLOT_PHASE
    sidx = red ? sidx : r + 1;
  }
  B0 = S0; B1 = S1; B2 = S2;
}

// Band slack of a mask from the extreme squared magnitudes of its kept
// node-phases: min(|V| - vmin, vmax - |V|) over them (+inf if there are none).
__device__ __forceinline__ double band_slack(double qmin, double qmax, double vmin, double vmax) {
  const double a = qmin < INFINITY ? sqrt_nr(qmin) - vmin : INFINITY;
  const double b = qmax > 0.0 ? vmax - sqrt_nr(qmax) : INFINITY;
  return fmin(a, b);
}

__device__ __forceinline__ bool feasible(const MaskScore& r, double e_bar) { return r.e <= e_bar && r.slack >= 0.0; }
__device__ __forceinline__ bool near_boundary(const MaskScore& r, double e_bar, double amb) {
  const bool rin = r.e <= e_bar - amb && r.slack >= amb;
  const bool rout = r.e > e_bar + amb || r.slack < -amb;
  return !rin && !rout;
}

// Error of one mask for one snapshot folded into el, kept squared magnitudes
// into (qmin, qmax): every chain walked with its nesting path recomputed, then
// the zone entries anchored below it.
__device__ __forceinline__ void score_snapshot(const SegHdr& H, const int* __restrict__ chains,
                                               const int* __restrict__ slots, const int* __restrict__ nest,
                                               const double2* Ps, const TargetRec* Ss, const double2* Hs,
                                               const double* Hm, const TargetRec* __restrict__ zrec_l, uint32_t m,
                                               double& el, double& qmin, double& qmax) {
  for (int c = 0; c < H.nchains; ++c) {
    const int* cr = chains + c * kChainInts;
    double2 B0 = make_double2(0.0, 0.0), B1 = B0, B2 = B0;
    const int nl = cr[C_NEST_LEN], no = cr[C_NEST_OFF];
    for (int q = 0; q + 1 < nl; ++q) {
      const int oc = nest[no + q];
      walk_chain<false>(chains + oc * kChainInts, slots, Ps, Ss, Hs, Hm, oc, m, B0, B1, B2, el, qmin, qmax);
    }
    walk_chain<true>(cr, slots, Ps, Ss, Hs, Hm, c, m, B0, B1, B2, el, qmin, qmax);
#define OKR_ZONE_PHASE(P_, B_)                                                   \
    for (int q = cr[C_ZOFF0 + P_], qe = q + cr[C_ZCNT0 + P_]; q < qe; ++q) {   \
      const TargetRec t = zrec_l[q];                                             \
      const double vx = t.W.x + B_.x, vy = t.W.y + B_.y;                         \
      const double q2 = fma(vx, vx, vy * vy);                                    \
      const double mag = sqrt_nr(q2);                                            \
      el = fmax(el, fmax(mag - t.lo, t.hi - mag));                               \
      qmin = fmin(qmin, q2);                                                     \
      qmax = fmax(qmax, q2);                                                     \
    }
    OKR_ZONE_PHASE(0, B0)
    OKR_ZONE_PHASE(1, B1)
    OKR_ZONE_PHASE(2, B2)
#undef OKR_ZONE_PHASE
  }
}

// ------------------------------------------------------------ block reduce --
template <typename T, typename Op>
__device__ T block_reduce(T v, Op op, T* sh) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  for (int o = 32; o > 0; o >>= 1) v = op(v, __shfl_xor(v, o, 64));
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  T r = sh[0];
  for (int w = 1; w < nw; ++w) r = op(r, sh[w]);
  __syncthreads();
  return r;
}

// Exclusive prefix sum of one int per thread over the block (Hillis-Steele in
// `sh`, which holds blockDim.x ints).
__device__ __forceinline__ int block_exclusive_scan(int v, int* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int o = 1; o < (int)blockDim.x; o <<= 1) {
    const int x = threadIdx.x >= (unsigned)o ? sh[threadIdx.x - o] : 0;
    __syncthreads();
    sh[threadIdx.x] += x;
    __syncthreads();
  }
  const int incl = sh[threadIdx.x];
  __syncthreads();
  return incl - v;
}

}  // namespace okr
