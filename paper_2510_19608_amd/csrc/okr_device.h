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
// hardware reciprocal-square-root estimate (relative error about 2^-24)
// refined by one Newton-Raphson step in Goldschmidt form (g -> sqrt(x),
// h -> 1/(2 sqrt(x)); error about 2^-48) and one residual correction
// g + (x - g^2) h, which leaves it within an ulp (the rounding test checks it
// against libm).  No range scaling: callers pass x in [2^-500, 2^500].
__device__ __forceinline__ double sqrt_nr(double x) {
  const double r = __builtin_amdgcn_rsq(x);
  double g = x * r, h = 0.5 * r;
  const double e = fma(-h, g, 0.5);
  g = fma(g, e, g);
  h = fma(h, e, h);
  const double d = fma(-g, g, x);
  return fma(d, h, g);
}
// |a|^2 in one fixed evaluation order (every magnitude of the scoring goes
// through it, so all scoring forms round alike).
__device__ __forceinline__ double mag2(double2 a) { return fma(a.x, a.x, a.y * a.y); }
__device__ __forceinline__ double vmag(double2 a) { return sqrt_nr(mag2(a)); }
// Magnitude of a chain head's voltage (mask-independent for chains that are
// not nested below another chain), one fixed evaluation order.
__device__ __forceinline__ double hmag(double2 a) { return sqrt_nr(fma(a.x, a.x, a.y * a.y)); }

// Walk one chain for M masks at once (one lane holds M masks; every
// wave-uniform quantity -- chain record, slot records, targets, head
// magnitude -- is shared by the M independent arithmetic chains): super-node
// slots top to bottom; a reduced slot adds the voltage rise of moving its
// aggregated current to its current super (P from LDS); a kept slot becomes
// the super of the slots below it.  With ERR, every slot cluster's error
// against its super's magnitude is folded into el, and the squared
// magnitudes of kept slots into (qmin, qmax) for the band (the slack is
// formed once per mask: sqrt is monotone, so min(|V| - vmin) =
// sqrt(min |V|^2) - vmin exactly).  Slot r of the chain has mask bit
// C_BIT0 + r, pairs from C_PAIR0 + r(r+1)/2 and its phases in the C_PHW
// words, so the slot loop issues no scalar loads.  The arithmetic of each
// mask is the same whatever M.
template <bool ERR, int M>
__device__ __forceinline__ void walk_chain(const int* __restrict__ cr, const double2* Ps, const TargetRec* Ss,
                                           const double2* Hs, const double* Hm, int c, const uint32_t (&m)[M],
                                           double2 (&B)[M][3], double (&el)[M], double (&qmin)[M],
                                           double (&qmax)[M]) {
  double2 S[M][3];
  double sm[M][3];
#pragma unroll
  for (int i = 0; i < M; ++i)
#pragma unroll
    for (int p = 0; p < 3; ++p) {
      S[i][p] = B[i][p];
      sm[i][p] = 0.0;
    }
  if (ERR) {
    const int hph = cr[C_PHASE];
    const double2* hv = Hs + c * 3;
    if (cr[C_OUTER] < 0) {  // head unaffected by the mask
#pragma unroll
      for (int p = 0; p < 3; ++p) {
        double h = 0.0;
        if (Hm) h = Hm[c * 3 + p];
        else if (hph >> p & 1) h = hmag(hv[p]);
#pragma unroll
        for (int i = 0; i < M; ++i) sm[i][p] = h;
      }
    } else {
#pragma unroll
      for (int p = 0; p < 3; ++p)
        if (hph >> p & 1) {
          const double2 h = hv[p];
#pragma unroll
          for (int i = 0; i < M; ++i) sm[i][p] = vmag(cadd(h, B[i][p]));
        }
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
    const TargetRec* tr = Ss + (s0 + r) * 3;
    bool red[M];
    double rf[M];
    const double2* pp[M];
#pragma unroll
    for (int i = 0; i < M; ++i) {
      red[i] = (m[i] >> (bit0 + r)) & 1u;
      rf[i] = red[i] ? 1.0 : 0.0;
      pp[i] = Ps + (prow + sidx[i]) * 3;
    }
#pragma unroll
    for (int p = 0; p < 3; ++p) {
      if (!(ph >> p & 1)) continue;
      TargetRec t;
      if (ERR) t = tr[p];
#pragma unroll
      for (int i = 0; i < M; ++i) {
        const double2 pv = pp[i][p];
        S[i][p].x = fma(rf[i], pv.x, S[i][p].x);
        S[i][p].y = fma(rf[i], pv.y, S[i][p].y);
        if (ERR) {
          const double vx = t.W.x + S[i][p].x, vy = t.W.y + S[i][p].y;
          const double q = fma(vx, vx, vy * vy);
          if (!red[i]) sm[i][p] = sqrt_nr(q);
          qmin[i] = fmin(qmin[i], red[i] ? INFINITY : q);
          qmax[i] = fmax(qmax[i], red[i] ? -INFINITY : q);
          el[i] = fmax(el[i], fmax(sm[i][p] - t.lo, t.hi - sm[i][p]));
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

// sqrt_nr of M independent values, step by step across them, so the M
// dependency chains interleave (each result equals sqrt_nr of its input).
template <int M>
__device__ __forceinline__ void sqrt_nr_v(const double (&x)[M], double (&y)[M]) {
  double g[M], h[M], e[M];
#pragma unroll
  for (int j = 0; j < M; ++j) {
    const double r = __builtin_amdgcn_rsq(x[j]);
    g[j] = x[j] * r;
    h[j] = 0.5 * r;
  }
#pragma unroll
  for (int j = 0; j < M; ++j) e[j] = fma(-h[j], g[j], 0.5);
#pragma unroll
  for (int j = 0; j < M; ++j) {
    g[j] = fma(g[j], e[j], g[j]);
    h[j] = fma(h[j], e[j], h[j]);
  }
#pragma unroll
  for (int j = 0; j < M; ++j) e[j] = fma(-g[j], g[j], x[j]);
#pragma unroll
  for (int j = 0; j < M; ++j) y[j] = fma(e[j], h[j], g[j]);
}

// Snapshot-vectorised chain walk: one mask, M snapshots at once, with the
// per-snapshot arithmetic of walk_chain.  The mask-dependent control (reduced
// or kept, current super) is shared by the M snapshots, so each side of the
// branch carries M independent chains, evaluated in lock-step, and on mask
// bits above the lane bits a whole wave takes one side.  el, qmin and qmax
// are per snapshot (folded later: max and min are exact).  LDS layout,
// snapshot fastest: P[(pair * 3 + p) * M + j], T[(slot * 3 + p) * M + j],
// H and Hm [(chain * 3 + p) * M + j].  With HM_FROM_H the magnitudes of
// heads no mask moves are formed from H here (as the LDS stage forms Hm)
// instead of read from Hm.
template <bool ERR, int M, bool HM_FROM_H = false>
__device__ __forceinline__ void walk_chain_sv(const cint* cr, const double2* Ps, const TargetRec* Ts,
                                              const double2* Hs, const double* Hm, int c, uint32_t m,
                                              double2 (&B)[M][3], double (&el)[M], double (&qmin)[M],
                                              double (&qmax)[M]) {
  double2 S[M][3];
  double sm[M][3];
#pragma unroll
  for (int j = 0; j < M; ++j)
#pragma unroll
    for (int p = 0; p < 3; ++p) {
      S[j][p] = B[j][p];
      sm[j][p] = 0.0;
    }
  if (ERR) {
    const int hph = cr[C_PHASE];
    if (cr[C_OUTER] < 0) {  // head unaffected by the mask: staged magnitude (0 on absent phases)
#pragma unroll
      for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int j = 0; j < M; ++j) {
          if (HM_FROM_H) {
            const double2 hv = Hs[(c * 3 + p) * M + j];
            sm[j][p] = (hv.x != 0.0 || hv.y != 0.0) ? hmag(hv) : 0.0;
          } else {
            sm[j][p] = Hm[(c * 3 + p) * M + j];
          }
        }
    } else {
#pragma unroll
      for (int p = 0; p < 3; ++p)
        if (hph >> p & 1) {
          double x[M], y[M];
#pragma unroll
          for (int j = 0; j < M; ++j) {
            x[j] = mag2(cadd(Hs[(c * 3 + p) * M + j], B[j][p]));
          }
          sqrt_nr_v<M>(x, y);
#pragma unroll
          for (int j = 0; j < M; ++j) sm[j][p] = y[j];
        }
    }
  }
  const int ns = cr[C_NSLOT], s0 = cr[C_SLOT0], pair0 = cr[C_PAIR0], bit0 = cr[C_BIT0];
  const int phw0 = cr[C_PHW0], phw1 = cr[C_PHW1], phw2 = cr[C_PHW2];
  int sidx = 0;
  for (int r = 0; r < ns; ++r) {
    const int w = r < 8 ? phw0 : (r < 16 ? phw1 : phw2);
    const int ph = __builtin_amdgcn_readfirstlane((w >> (3 * (r & 7))) & 7);  // same for every lane
    const int prow = pair0 + ((r * (r + 1)) >> 1);
    const TargetRec* tr = Ts + (s0 + r) * 3 * M;
    if ((m >> (bit0 + r)) & 1u) {  // reduced: the moved current's rise; cluster error against the super
      const double2* pr = Ps + (prow + sidx) * 3 * M;
#pragma unroll
      for (int p = 0; p < 3; ++p) {
        if (!(ph >> p & 1)) continue;
#pragma unroll
        for (int j = 0; j < M; ++j) {
          const double2 pv = pr[p * M + j];
          S[j][p].x += pv.x;
          S[j][p].y += pv.y;
          if (ERR) {
            const TargetRec t = tr[p * M + j];
            el[j] = fmax(el[j], fmax(sm[j][p] - t.lo, t.hi - sm[j][p]));
          }
        }
      }
    } else {  // kept: a new super
      if (ERR) {
#pragma unroll
        for (int p = 0; p < 3; ++p) {
          if (!(ph >> p & 1)) continue;
          double q[M], mg[M], lo[M], hi[M];
#pragma unroll
          for (int j = 0; j < M; ++j) {
            const TargetRec t = tr[p * M + j];
            const double vx = t.W.x + S[j][p].x, vy = t.W.y + S[j][p].y;
            q[j] = fma(vx, vx, vy * vy);
            lo[j] = t.lo;
            hi[j] = t.hi;
          }
          sqrt_nr_v<M>(q, mg);
#pragma unroll
          for (int j = 0; j < M; ++j) {
            sm[j][p] = mg[j];
            qmin[j] = fmin(qmin[j], q[j]);
            qmax[j] = fmax(qmax[j], q[j]);
            el[j] = fmax(el[j], fmax(mg[j] - lo[j], hi[j] - mg[j]));
          }
        }
      }
      sidx = r + 1;
    }
  }
#pragma unroll
  for (int j = 0; j < M; ++j)
#pragma unroll
    for (int p = 0; p < 3; ++p) B[j][p] = S[j][p];
}

// Terms of chain c for one mask over M snapshots (snapshot-vectorised
// score_chain): the nesting path, the chain, then its zone entries (the first
// zcap from the LDS stage Zs[q * M + j], the rest from global memory, where
// snapshot j's records start at zg[j]).
template <int M, bool HM_FROM_H = false>
__device__ __forceinline__ void score_chain_sv(const cint* chains, const cint* nest, int c,
                                               const double2* Ps, const TargetRec* Ts, const double2* Hs,
                                               const double* Hm, const TargetRec* Zs, int zcap,
                                               const TargetRec* const (&zg)[M], uint32_t m, double (&el)[M],
                                               double (&qmin)[M], double (&qmax)[M]) {
  const cint* cr = chains + c * kChainInts;
  double2 B[M][3];
#pragma unroll
  for (int j = 0; j < M; ++j)
#pragma unroll
    for (int p = 0; p < 3; ++p) B[j][p] = make_double2(0.0, 0.0);
  const int nl = cr[C_NEST_LEN], no = cr[C_NEST_OFF];
  for (int q = 0; q + 1 < nl; ++q) {
    const int oc = nest[no + q];
    walk_chain_sv<false, M, HM_FROM_H>(chains + oc * kChainInts, Ps, Ts, Hs, Hm, oc, m, B, el, qmin, qmax);
  }
  walk_chain_sv<true, M, HM_FROM_H>(cr, Ps, Ts, Hs, Hm, c, m, B, el, qmin, qmax);
#pragma unroll
  for (int p = 0; p < 3; ++p)
    for (int q = cr[C_ZOFF0 + p], qe = q + cr[C_ZCNT0 + p]; q < qe; ++q) {
      double q2[M], mag[M], lo[M], hi[M];
#pragma unroll
      for (int j = 0; j < M; ++j) {
        TargetRec t;
        if (q < zcap) t = Zs[q * M + j];
        else t = zg[j][q];
        const double vx = t.W.x + B[j][p].x, vy = t.W.y + B[j][p].y;
        q2[j] = fma(vx, vx, vy * vy);
        lo[j] = t.lo;
        hi[j] = t.hi;
      }
      sqrt_nr_v<M>(q2, mag);
#pragma unroll
      for (int j = 0; j < M; ++j) {
        el[j] = fmax(el[j], fmax(mag[j] - lo[j], hi[j] - mag[j]));
        qmin[j] = fmin(qmin[j], q2[j]);
        qmax[j] = fmax(qmax[j], q2[j]);
      }
    }
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

// Per-snapshot LDS stage of the scoring kernels, in 16-byte chunks: pair
// table, slot records (2 chunks each), chain heads, then the first kZoneLds
// zone records (2 chunks each; later ones are read from global memory).
constexpr int kZoneLds = 256;

struct Stage {
  int cP, cT, cH, cZ, total;
};

__device__ __forceinline__ Stage stage_sizes(const SegHdr& H) {
  Stage z;
  z.cP = H.npairs * 3;
  z.cT = H.nslots * 6;
  z.cH = H.nchains * 3;
  z.cZ = min(H.nz, kZoneLds) * 2;
  z.total = z.cP + z.cT + z.cH + z.cZ;
  return z;
}

__device__ __forceinline__ uint4 stage_src(const Stage& z, int i, const uint4* __restrict__ P_l,
                                           const uint4* __restrict__ S_l, const uint4* __restrict__ H_l,
                                           const uint4* __restrict__ Z_l) {
  if (i < z.cP) return P_l[i];
  i -= z.cP;
  if (i < z.cT) return S_l[i];
  i -= z.cT;
  if (i < z.cH) return H_l[i];
  return Z_l[i - z.cH];
}

// Store chunk i; with Hm (FP64 heads) also the head magnitude (absent phases 0).
__device__ __forceinline__ void stage_put(const Stage& z, int i, const uint4& v, uint4* Pd, uint4* Sd, uint4* Hd,
                                          double* Hm, uint4* Zd) {
  if (i < z.cP) {
    Pd[i] = v;
    return;
  }
  i -= z.cP;
  if (i < z.cT) {
    Sd[i] = v;
    return;
  }
  i -= z.cT;
  if (i < z.cH) {
    Hd[i] = v;
    if (Hm) {
      const double2 hv = make_double2(__hiloint2double((int)v.y, (int)v.x), __hiloint2double((int)v.w, (int)v.z));
      Hm[i] = (hv.x != 0.0 || hv.y != 0.0) ? hmag(hv) : 0.0;
    }
    return;
  }
  Zd[i - z.cH] = v;
}

// Terms of chain c for M masks and one snapshot folded into el, kept squared
// magnitudes into (qmin, qmax): the nesting path walked to the chain's head
// (voltage rises only), the chain's own slots, then the zone entries anchored
// below it (the first zcap of them from the LDS stage Zs when STAGED, the
// rest from global memory).  They depend on the mask bits in C_PMASK only.
template <bool STAGED, int M>
__device__ __forceinline__ void score_chain(const int* __restrict__ chains, const int* __restrict__ nest, int c,
                                            const double2* Ps, const TargetRec* Ss, const double2* Hs,
                                            const double* Hm, const TargetRec* Zs, int zcap,
                                            const TargetRec* __restrict__ zrec_l, const uint32_t (&m)[M],
                                            double (&el)[M], double (&qmin)[M], double (&qmax)[M]) {
  const int* cr = chains + c * kChainInts;
  double2 B[M][3];
#pragma unroll
  for (int i = 0; i < M; ++i)
#pragma unroll
    for (int p = 0; p < 3; ++p) B[i][p] = make_double2(0.0, 0.0);
  const int nl = cr[C_NEST_LEN], no = cr[C_NEST_OFF];
  for (int q = 0; q + 1 < nl; ++q) {
    const int oc = nest[no + q];
    walk_chain<false, M>(chains + oc * kChainInts, Ps, Ss, Hs, Hm, oc, m, B, el, qmin, qmax);
  }
  walk_chain<true, M>(cr, Ps, Ss, Hs, Hm, c, m, B, el, qmin, qmax);
#pragma unroll
  for (int p = 0; p < 3; ++p)
    for (int q = cr[C_ZOFF0 + p], qe = q + cr[C_ZCNT0 + p]; q < qe; ++q) {
      TargetRec t;
      if (STAGED && q < zcap) t = Zs[q];
      else t = zrec_l[q];
#pragma unroll
      for (int i = 0; i < M; ++i) {
        const double vx = t.W.x + B[i][p].x, vy = t.W.y + B[i][p].y;
        const double q2 = fma(vx, vx, vy * vy);
        const double mag = sqrt_nr(q2);
        el[i] = fmax(el[i], fmax(mag - t.lo, t.hi - mag));
        qmin[i] = fmin(qmin[i], q2);
        qmax[i] = fmax(qmax[i], q2);
      }
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
