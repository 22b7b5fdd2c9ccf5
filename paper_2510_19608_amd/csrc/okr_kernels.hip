// gfx950 kernels of the segment-exhaustive Kron-reduction search.
//
// Data layout in HBM (complex values as double2 = (re, im)):
//   z[n][9]            branch impedance of node i's upstream edge (restricted)
//   Vhat, Vcur, A      [S][n][3]: scenario voltages, current candidate-state
//                      voltages of kept nodes, aggregated load current of kept
//                      nodes (consumed current, = -I^ moved by the assignment)
//   absV[S][n][3]      |Vhat|
//   per segment        P[S][npairs][3], slot/zone TargetRec[S][..][3], headV
//   scores             MaskScore[snapshot group][2^k]
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "okr_internal.h"
#include "okr_device.h"

namespace okr {

// Restricted inverse of a 3x3 block on the phases in `mask` (zero-padded):
// for blocks supported on the present-phase principal submatrix this is the
// Moore-Penrose pseudo-inverse (Section II.B footnote).  Closed forms for
// 1x1, 2x2 (adjugate) and 3x3 (cofactors).  Returns false if singular.
__device__ bool inv_restricted(const double2* A, unsigned mask, double2* out) {
  int idx[3];
  int m = 0;
  for (int p = 0; p < 3; ++p)
    if (mask >> p & 1u) idx[m++] = p;
  for (int q = 0; q < 9; ++q) out[q] = make_double2(0.0, 0.0);
  if (m == 1) {
    const double2 a = A[idx[0] * 4];
    if (cabs2(a) == 0.0) return false;
    out[idx[0] * 4] = cdiv(make_double2(1.0, 0.0), a);
    return true;
  }
  if (m == 2) {
    const int i = idx[0], j = idx[1];
    const double2 a = A[i * 3 + i], b = A[i * 3 + j], c = A[j * 3 + i], d = A[j * 3 + j];
    const double2 det = csub(cmul(a, d), cmul(b, c));
    if (cabs2(det) == 0.0) return false;
    out[i * 3 + i] = cdiv(d, det);
    out[i * 3 + j] = cdiv(make_double2(-b.x, -b.y), det);
    out[j * 3 + i] = cdiv(make_double2(-c.x, -c.y), det);
    out[j * 3 + j] = cdiv(a, det);
    return true;
  }
  if (m == 3) {
    double2 cof[9];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        const int r1 = (r + 1) % 3, r2 = (r + 2) % 3, c1 = (c + 1) % 3, c2 = (c + 2) % 3;
        cof[r * 3 + c] = csub(cmul(A[r1 * 3 + c1], A[r2 * 3 + c2]), cmul(A[r1 * 3 + c2], A[r2 * 3 + c1]));
      }
    const double2 det = cadd(cadd(cmul(A[0], cof[0]), cmul(A[1], cof[1])), cmul(A[2], cof[2]));
    if (cabs2(det) == 0.0) return false;
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) out[r * 3 + c] = cdiv(cof[c * 3 + r], det);
    return true;
  }
  return m == 0;
}

__device__ __forceinline__ double blk_maxabs(const double2* A) {
  double mx = 0.0;
  for (int q = 0; q < 9; ++q) mx = fmax(mx, sqrt(cabs2(A[q])));
  return mx;
}

// ---------------------------------------------------------- validation + z --
// One thread per node: branch impedance z_i = (-Y_{i,parent})^+ and checks of
// the admittance input (symmetry, zero absent-phase entries, no shunts).
// status bits: 1 singular, 2 absent-phase entry, 4 asymmetric, 8 shunt.
__global__ void k_branch_z(int n, const int* __restrict__ parent, const uint8_t* __restrict__ phase,
                           const int* __restrict__ ch_off, const int* __restrict__ ch,
                           const double2* __restrict__ Ydiag, const double2* __restrict__ Yoff,
                           double2* __restrict__ z, int* __restrict__ status) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const unsigned ph = phase[i];
  int bad = 0;
  const double2* Yd = Ydiag + (size_t)i * 9;
  double dscale = blk_maxabs(Yd);
  // Laplacian row: Y_ii + Y_{i,p} + sum_c Y_{i,c} = 0, with Y_{i,c} = Y_{c,i}^T
  double2 acc[9];
  for (int q = 0; q < 9; ++q) acc[q] = Yd[q];
  if (i > 0) {
    const double2* Yo = Yoff + (size_t)i * 9;
    for (int q = 0; q < 9; ++q) acc[q] = cadd(acc[q], Yo[q]);
    const double oscale = blk_maxabs(Yo);
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        const double2 d = csub(Yo[r * 3 + c], Yo[c * 3 + r]);
        if (sqrt(cabs2(d)) > 1e-12 * oscale) bad |= 4;
        const bool absent = !((ph >> r) & 1u) || !((ph >> c) & 1u);
        if (absent && cabs2(Yo[r * 3 + c]) != 0.0) bad |= 2;
      }
    double2 y[9];
    for (int q = 0; q < 9; ++q) y[q] = make_double2(-Yo[q].x, -Yo[q].y);
    if (!inv_restricted(y, ph, z + (size_t)i * 9)) bad |= 1;
  } else {
    for (int q = 0; q < 9; ++q) z[q] = make_double2(0.0, 0.0);
  }
  for (int e = ch_off[i]; e < ch_off[i + 1]; ++e) {
    const double2* Yc = Yoff + (size_t)ch[e] * 9;
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) acc[r * 3 + c] = cadd(acc[r * 3 + c], Yc[c * 3 + r]);
  }
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      const bool absent = !((ph >> r) & 1u) || !((ph >> c) & 1u);
      if (absent && cabs2(Yd[r * 3 + c]) != 0.0) bad |= 2;
    }
  if (blk_maxabs(acc) > 1e-9 * fmax(dscale, 1e-300)) bad |= 8;
  if (bad) atomicOr(status, bad);
}

// ------------------------------------------------------------- load flow --
// Scenario library (Section III): constant-PQ wye loads, backward/forward
// sweep on the radial tree, one block per snapshot, level-synchronous.
// status bit 16: not converged; bit 32: base network outside the band.
// Forward-sweep update of node i: V(i) = V(parent) - z(i) J(i) on its
// present phases, and the largest change into dmax (NaN-propagating).
__device__ __forceinline__ void forward_node(int i, const int* __restrict__ parent, const uint8_t* __restrict__ phase,
                                             const double2 (&zi)[9], const double2* Jl, double2* Vl, double& dmax) {
  const int pv = parent[i];
  const double2 j0 = Jl[i * 3], j1 = Jl[i * 3 + 1], j2 = Jl[i * 3 + 2];
#pragma unroll
  for (int p = 0; p < 3; ++p) {
    if (!(phase[i] >> p & 1u)) continue;
    const double2 d = cadd(cadd(cmul(zi[p * 3], j0), cmul(zi[p * 3 + 1], j1)), cmul(zi[p * 3 + 2], j2));
    const double2 nv = csub(Vl[pv * 3 + p], d);
    const double dd = sqrt(cabs2(csub(nv, Vl[i * 3 + p])));
    dmax = (dd <= dmax) ? dmax : dd;
    Vl[i * 3 + p] = nv;
  }
}

// Where the sweep's data lives: kPfGlobal reads everything from global
// memory, kPfAll holds the iterates and the tree arrays in LDS.
enum { kPfGlobal = 0, kPfAll = 1 };

template <int MODE>
__device__ __forceinline__ void powerflow_body(
    int n, const int* __restrict__ gparent, const uint8_t* __restrict__ gphase,
    const int* __restrict__ glvl_off, const int* __restrict__ glvl_nodes, int nlev,
    const int* __restrict__ gch_off, const int* __restrict__ gch, const double2* __restrict__ z,
    const double2* __restrict__ Sload, double2 v0a, double2 v0b, double2 v0c, double tol, int maxit,
    double vmin, double vmax, double2* __restrict__ V, double2* __restrict__ J,
    double2* __restrict__ A, double* __restrict__ absV, int* __restrict__ iters, int* __restrict__ status,
    double2* sbuf, double* shd) {
  constexpr bool LDS = MODE == kPfAll;
  const int l = blockIdx.x;
  const size_t base = (size_t)l * n * 3;
  // (with LDS the iterates, and the tree arrays the sweeps index, live in
  // shared memory: every level step then waits on LDS instead of global
  // memory; only the branch impedances are read from global memory)
  double2* Vl = LDS ? sbuf : V + base;
  double2* Jl = LDS ? sbuf + (size_t)n * 3 : J + base;
  const int *parent, *lvl_nodes, *ch_off, *ch;
  const int* lvl_off;
  const uint8_t* phase;
  if constexpr (MODE == kPfGlobal) {
    parent = gparent;
    lvl_nodes = glvl_nodes;
    ch_off = gch_off;
    ch = gch;
    lvl_off = glvl_off;
    phase = gphase;
  } else {
    int* s_lvl_off = (int*)(sbuf + (LDS ? (size_t)n * 6 : 0));
    int* s_lvl_nodes = s_lvl_off + nlev + 1;
    int* s_ch_off = s_lvl_nodes + n;
    int* s_ch = s_ch_off + n + 1;
    int* s_parent = s_ch + n;
    uint8_t* s_phase = (uint8_t*)(s_parent + n);
    for (int i = threadIdx.x; i <= nlev; i += blockDim.x) s_lvl_off[i] = glvl_off[i];
    for (int i = threadIdx.x; i <= n; i += blockDim.x) s_ch_off[i] = gch_off[i];
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      s_lvl_nodes[i] = glvl_nodes[i];
      s_ch[i] = i < n - 1 ? gch[i] : 0;
      s_parent[i] = gparent[i];
      s_phase[i] = gphase[i];
    }
    lvl_off = s_lvl_off;
    lvl_nodes = s_lvl_nodes;
    ch_off = s_ch_off;
    ch = s_ch;
    parent = s_parent;
    phase = s_phase;
  }
  const double2* Sl = Sload + base;
  const double2 v0[3] = {v0a, v0b, v0c};
  for (int i = threadIdx.x; i < n; i += blockDim.x)
    for (int p = 0; p < 3; ++p) Vl[i * 3 + p] = (phase[i] >> p & 1u) ? v0[p] : make_double2(0.0, 0.0);
  __syncthreads();
  int it = 0;
  bool conv = false;
  const int tid = threadIdx.x, bd = blockDim.x;
  for (it = 1; it <= maxit; ++it) {
    // load currents conj(S/V) of every node in one pass (off the level
    // steps' latency chain), then the backward sweep adds each level's
    // children into their parents, deepest level first
    for (int i = tid; i < n; i += bd)
      for (int p = 0; p < 3; ++p)
        Jl[i * 3 + p] = (i > 0 && (phase[i] >> p & 1u)) ? cconj(cdiv(Sl[i * 3 + p], Vl[i * 3 + p]))
                                                        : make_double2(0.0, 0.0);
    __syncthreads();
    for (int lev = nlev - 2; lev >= 0; --lev) {
      for (int q = lvl_off[lev] + tid; q < lvl_off[lev + 1]; q += bd) {
        const int i = lvl_nodes[q];
        double2 s0 = Jl[i * 3], s1 = Jl[i * 3 + 1], s2 = Jl[i * 3 + 2];
        for (int e = ch_off[i]; e < ch_off[i + 1]; ++e) {
          const int c = ch[e];
          s0 = cadd(s0, Jl[c * 3]);
          s1 = cadd(s1, Jl[c * 3 + 1]);
          s2 = cadd(s2, Jl[c * 3 + 2]);
        }
        Jl[i * 3] = s0; Jl[i * 3 + 1] = s1; Jl[i * 3 + 2] = s2;
      }
      __syncthreads();
    }
    double dmax = 0.0;
    // the branch impedance of this thread's first node on the next level is
    // loaded while the current level is computed (the impedances are the
    // only global reads of the sweep; a thread with no node there loads the
    // root's, unused)
    double2 zn[9];
    {
      const int q1 = nlev > 1 ? lvl_off[1] + tid : 0;
      const double2* zz = z + (size_t)((nlev > 1 && q1 < lvl_off[2]) ? lvl_nodes[q1] : 0) * 9;
#pragma unroll
      for (int e = 0; e < 9; ++e) zn[e] = zz[e];
    }
    for (int lev = 1; lev < nlev; ++lev) {
      double2 zc[9];
#pragma unroll
      for (int e = 0; e < 9; ++e) zc[e] = zn[e];
      {
        const int qn = lev + 1 < nlev ? lvl_off[lev + 1] + tid : 0;
        const double2* zz = z + (size_t)((lev + 1 < nlev && qn < lvl_off[lev + 2]) ? lvl_nodes[qn] : 0) * 9;
#pragma unroll
        for (int e = 0; e < 9; ++e) zn[e] = zz[e];
      }
      const int q0 = lvl_off[lev] + tid, q1 = lvl_off[lev + 1];
      if (q0 < q1) forward_node(lvl_nodes[q0], parent, phase, zc, Jl, Vl, dmax);
      for (int q = q0 + bd; q < q1; q += bd) {  // (levels wider than the block)
        const int i = lvl_nodes[q];
        double2 zi[9];
#pragma unroll
        for (int e = 0; e < 9; ++e) zi[e] = z[(size_t)i * 9 + e];
        forward_node(i, parent, phase, zi, Jl, Vl, dmax);
      }
      if (LDS) {
        // the iterates are in LDS: order LDS only, so the next level's
        // impedance loads stay in flight across the barrier
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
        __builtin_amdgcn_s_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
      } else {
        __syncthreads();
      }
    }
    dmax = block_reduce(dmax, [](double a, double b) { return (b <= a) ? a : b; }, shd);
    if (!(dmax <= 1e3)) break;
    if (dmax <= tol) { conv = true; break; }
  }
  double vlo = 1e300, vhi = -1e300;
  for (int i = threadIdx.x; i < n; i += blockDim.x)
    for (int p = 0; p < 3; ++p) {
      const bool pr = (phase[i] >> p & 1u);
      const double2 v = Vl[i * 3 + p];
      if (LDS) V[base + i * 3 + p] = v;
      A[base + i * 3 + p] = (i > 0 && pr) ? cconj(cdiv(Sl[i * 3 + p], v)) : make_double2(0.0, 0.0);
      const double m = pr ? sqrt(cabs2(v)) : 0.0;
      absV[base + i * 3 + p] = m;
      if (pr) { vlo = fmin(vlo, m); vhi = fmax(vhi, m); }
    }
  vlo = block_reduce(vlo, [](double a, double b) { return fmin(a, b); }, shd);
  vhi = block_reduce(vhi, [](double a, double b) { return fmax(a, b); }, shd);
  if (threadIdx.x == 0) {
    iters[l] = it;
    if (!conv) atomicOr(status, 16);
    if (vlo < vmin || vhi > vmax) atomicOr(status, 32);
  }
}


__global__ __launch_bounds__(256) void k_powerflow(
    int n, const int* __restrict__ parent, const uint8_t* __restrict__ phase,
    const int* __restrict__ lvl_off, const int* __restrict__ lvl_nodes, int nlev,
    const int* __restrict__ ch_off, const int* __restrict__ ch, const double2* __restrict__ z,
    const double2* __restrict__ Sload, double2 v0a, double2 v0b, double2 v0c, double tol, int maxit,
    double vmin, double vmax, double2* __restrict__ V, double2* __restrict__ J,
    double2* __restrict__ A, double* __restrict__ absV, int* __restrict__ iters, int* __restrict__ status) {
  __shared__ double shd[16];
  powerflow_body<kPfGlobal>(n, parent, phase, lvl_off, lvl_nodes, nlev, ch_off, ch, z, Sload, v0a, v0b, v0c, tol, maxit,
                            vmin, vmax, V, J, A, absV, iters, status, nullptr, shd);
}

// The same with the voltage and current iterates in dynamic LDS (2 x n x 3
// double2), followed by the level offsets and nodes, child offsets and
// lists, parents and phases (for feeders small enough to fit).
__global__ __launch_bounds__(256) void k_powerflow_lds(
    int n, const int* __restrict__ parent, const uint8_t* __restrict__ phase,
    const int* __restrict__ lvl_off, const int* __restrict__ lvl_nodes, int nlev,
    const int* __restrict__ ch_off, const int* __restrict__ ch, const double2* __restrict__ z,
    const double2* __restrict__ Sload, double2 v0a, double2 v0b, double2 v0c, double tol, int maxit,
    double vmin, double vmax, double2* __restrict__ V, double2* __restrict__ J,
    double2* __restrict__ A, double* __restrict__ absV, int* __restrict__ iters, int* __restrict__ status) {
  extern __shared__ double2 pf_lds[];
  __shared__ double shd[16];
  powerflow_body<kPfAll>(n, parent, phase, lvl_off, lvl_nodes, nlev, ch_off, ch, z, Sload, v0a, v0b, v0c, tol, maxit,
                         vmin, vmax, V, J, A, absV, iters, status, pf_lds, shd);
}

// The same for feeders whose iterates do not fit in LDS (n < 65536): every
// per-node quantity of the sweep is stored by breadth-first queue position
// (each level a contiguous run, the children of position q at positions
// cf[q] .. cf[q+1]-1 in child-list order, pp[q] the parent's position), so
// each level step reads and writes contiguous records and a node's children
// are one contiguous run.  The queue tables (16-bit) sit in dynamic LDS; the
// snapshot's loads and voltages in queue order use the Vhat and A slices as
// scratch until the end, the branch currents the J slice.  Each node's
// arithmetic, and the order of every sum, is that of the node-order form.
__global__ __launch_bounds__(512) void k_powerflow_bfs(
    int n, const uint8_t* __restrict__ phase, const int* __restrict__ glvl_off, const int* __restrict__ glvl_nodes,
    int nlev, const int* __restrict__ gcf, const int* __restrict__ gpp, const double2* __restrict__ z,
    const double2* __restrict__ Sload, double2 v0a, double2 v0b, double2 v0c, double tol, int maxit,
    double vmin, double vmax, double2* __restrict__ V, double2* __restrict__ J,
    double2* __restrict__ A, double* __restrict__ absV, int* __restrict__ iters, int* __restrict__ status) {
  extern __shared__ double2 pf_lds[];
  __shared__ double shd[16];
  const int l = blockIdx.x, tid = threadIdx.x, bd = blockDim.x;
  const size_t base = (size_t)l * n * 3;
  int* lvl_off = (int*)pf_lds;
  uint16_t* node = (uint16_t*)(lvl_off + nlev + 1);
  uint16_t* cf = node + n;
  uint16_t* pp = cf + n + 1;
  uint8_t* ph = (uint8_t*)(pp + n);
  for (int i = tid; i <= nlev; i += bd) lvl_off[i] = glvl_off[i];
  for (int q = tid; q <= n; q += bd) cf[q] = (uint16_t)gcf[q];
  for (int q = tid; q < n; q += bd) {
    const int i = glvl_nodes[q];
    node[q] = (uint16_t)i;
    pp[q] = (uint16_t)gpp[q];
    ph[q] = phase[i];
  }
  const double2* Sl = Sload + base;
  double2* Sb = V + base;
  double2* Vb = A + base;
  double2* Jb = J + base;
  __syncthreads();
  const double2 v0[3] = {v0a, v0b, v0c};
  for (int q = tid; q < n; q += bd) {
    const int i = node[q];
    const unsigned m = ph[q];
#pragma unroll
    for (int p = 0; p < 3; ++p) {
      Sb[q * 3 + p] = Sl[i * 3 + p];
      Vb[q * 3 + p] = (m >> p & 1u) ? v0[p] : make_double2(0.0, 0.0);
    }
  }
  __syncthreads();
  int it = 0;
  bool conv = false;
  for (it = 1; it <= maxit; ++it) {
    // backward sweep, deepest level first: branch current = own load
    // current conj(S/V) on present phases + the children's branch currents
    // (finished on the previous step), added in child order after all of
    // them are loaded; the root's is never read and is not formed
    for (int lev = nlev - 1; lev >= 1; --lev) {
      for (int q = lvl_off[lev] + tid; q < lvl_off[lev + 1]; q += bd) {
        const unsigned m = ph[q];
        const int c0 = cf[q], c1 = cf[q + 1];
        double2 s[3], v[3], a[3];
#pragma unroll
        for (int p = 0; p < 3; ++p) { s[p] = Sb[q * 3 + p]; v[p] = Vb[q * 3 + p]; }
        for (int c = c0; c < c1; c += 2) {
          double2 t0[3], t1[3];
          const int cc = c + 1 < c1 ? c + 1 : c;
#pragma unroll
          for (int p = 0; p < 3; ++p) { t0[p] = Jb[c * 3 + p]; t1[p] = Jb[cc * 3 + p]; }
          if (c == c0) {
#pragma unroll
            for (int p = 0; p < 3; ++p) a[p] = (m >> p & 1u) ? cconj(cdiv(s[p], v[p])) : make_double2(0.0, 0.0);
          }
#pragma unroll
          for (int p = 0; p < 3; ++p) a[p] = cadd(a[p], t0[p]);
          if (c + 1 < c1) {
#pragma unroll
            for (int p = 0; p < 3; ++p) a[p] = cadd(a[p], t1[p]);
          }
        }
        if (c0 == c1) {
#pragma unroll
          for (int p = 0; p < 3; ++p) a[p] = (m >> p & 1u) ? cconj(cdiv(s[p], v[p])) : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int p = 0; p < 3; ++p) Jb[q * 3 + p] = a[p];
      }
      __syncthreads();
    }
    // forward sweep: V(q) = V(parent) - z J(q) on present phases, the
    // largest change into dmax (NaN-propagating)
    double dmax = 0.0;
    for (int lev = 1; lev < nlev; ++lev) {
      for (int q = lvl_off[lev] + tid; q < lvl_off[lev + 1]; q += bd) {
        const int i = node[q], pq = pp[q];
        const unsigned m = ph[q];
        double2 zi[9], j[3], vp[3], vo[3];
#pragma unroll
        for (int e = 0; e < 9; ++e) zi[e] = z[(size_t)i * 9 + e];
#pragma unroll
        for (int p = 0; p < 3; ++p) { j[p] = Jb[q * 3 + p]; vp[p] = Vb[pq * 3 + p]; vo[p] = Vb[q * 3 + p]; }
#pragma unroll
        for (int p = 0; p < 3; ++p) {
          if (!(m >> p & 1u)) continue;
          const double2 d = cadd(cadd(cmul(zi[p * 3], j[0]), cmul(zi[p * 3 + 1], j[1])), cmul(zi[p * 3 + 2], j[2]));
          const double2 nv = csub(vp[p], d);
          const double dd = sqrt(cabs2(csub(nv, vo[p])));
          dmax = (dd <= dmax) ? dmax : dd;
          Vb[q * 3 + p] = nv;
        }
      }
      __syncthreads();
    }
    dmax = block_reduce(dmax, [](double a, double b) { return (b <= a) ? a : b; }, shd);
    if (!(dmax <= 1e3)) break;
    if (dmax <= tol) { conv = true; break; }
  }
  // voltages back to node order (over the loads, no longer read), then the
  // load currents and magnitudes at the final voltages
  for (int q = tid; q < n; q += bd) {
    const int i = node[q];
#pragma unroll
    for (int p = 0; p < 3; ++p) V[base + i * 3 + p] = Vb[q * 3 + p];
  }
  __syncthreads();
  double vlo = 1e300, vhi = -1e300;
  for (int i = tid; i < n; i += bd)
    for (int p = 0; p < 3; ++p) {
      const bool pr = (phase[i] >> p & 1u);
      const double2 v = V[base + i * 3 + p];
      A[base + i * 3 + p] = (i > 0 && pr) ? cconj(cdiv(Sl[i * 3 + p], v)) : make_double2(0.0, 0.0);
      const double m = pr ? sqrt(cabs2(v)) : 0.0;
      absV[base + i * 3 + p] = m;
      if (pr) { vlo = fmin(vlo, m); vhi = fmax(vhi, m); }
    }
  vlo = block_reduce(vlo, [](double a, double b) { return fmin(a, b); }, shd);
  vhi = block_reduce(vhi, [](double a, double b) { return fmax(a, b); }, shd);
  if (tid == 0) {
    iters[l] = it;
    if (!conv) atomicOr(status, 16);
    if (vlo < vmin || vhi > vmax) atomicOr(status, 32);
  }
}

// Cumulative series impedance from the root, Zroot(v) = Zroot(parent) + z(v)
// (3x3 blocks, zero on absent phases), level by level; the impedance of the
// path between an ancestor s and r is Zroot(r) - Zroot(s).  One block.
__global__ __launch_bounds__(1024) void k_zroot(int n, const int* __restrict__ parent,
                                                const int* __restrict__ lvl_off, const int* __restrict__ lvl_nodes,
                                                int nlev, const double2* __restrict__ z, double2* __restrict__ Zroot) {
  for (int e = threadIdx.x; e < 9; e += blockDim.x) Zroot[e] = make_double2(0.0, 0.0);  // node 0, level 0
  __syncthreads();
  for (int L = 1; L < nlev; ++L) {
    const int a = lvl_off[L], b = lvl_off[L + 1];
    for (int t = a * 9 + threadIdx.x; t < b * 9; t += blockDim.x) {
      const int v = lvl_nodes[t / 9], e = t % 9;
      const double2 up = Zroot[(size_t)parent[v] * 9 + e], zv = z[(size_t)v * 9 + e];
      Zroot[(size_t)v * 9 + e] = make_double2(up.x + zv.x, up.y + zv.y);
    }
    __threadfence_block();
    __syncthreads();
  }
}

// Given V^ (caller supplied): load currents and magnitudes, band check.
__global__ void k_from_vhat(int n, int S, const uint8_t* __restrict__ phase, const double2* __restrict__ Sload,
                            const double2* __restrict__ V, double vmin, double vmax, double2* __restrict__ A,
                            double* __restrict__ absV, int* __restrict__ status) {
  const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (size_t)S * n * 3) return;
  const int p = q % 3, i = (q / 3) % n;
  const bool pr = (phase[i] >> p & 1u);
  A[q] = (i > 0 && pr) ? cconj(cdiv(Sload[q], V[q])) : make_double2(0.0, 0.0);
  const double m = pr ? sqrt(cabs2(V[q])) : 0.0;
  absV[q] = m;
  if (pr && (m < vmin || m > vmax)) atomicOr(status, 32);
}

// ----------------------------------------------------------------- argmin --
// Lexicographic selection over the tile records: most reduced nodes among
// feasible masks, then the smallest error, masks within tie_tol of that error
// tie and the lowest wins.  Only tiles whose record can hold the winner (or a
// mask within amb of the tie threshold) are rescanned mask by mask.
// Ambiguous when a mask at the chosen level or above lies within amb of the
// e_bar / band boundary, or a feasible mask at the chosen level lies within
// amb of e_min + tie_tol.
__global__ __launch_bounds__(1024) void k_argmin(const SegHdr* __restrict__ hdrs, const int* __restrict__ segs,
                                                 size_t lstride, const MaskScore* __restrict__ fin,
                                                 const TileRec* __restrict__ tiles, SelParams sp,
                                                 const int* __restrict__ status, DevDecision* __restrict__ decs,
                                                 const int* __restrict__ gates) {
  // one slot per wave for each reduction (each its own array, so no
  // reduction's slots are written while another's are still being read)
  __shared__ int s_best[16], s_amb[16], s_amb2[16];
  __shared__ double s_emin[16], s_run[16];
  __shared__ unsigned s_pick[16];
  __shared__ int ncand;
  __shared__ int cand[1024];
  const int g = segs[blockIdx.z];
  const SegHdr H = load_hdr_g(hdrs, g);
  if (gates && gates[g] == 0) return;  // decided without the full enumeration
  fin = lane_ptr(fin, lstride);
  tiles = lane_ptr(tiles, lstride);
  DevDecision* dec = decs + g;
  // nothing is reduced when the full network violates the band, the load
  // flow failed, or the segment's tables are inconsistent
  if (!H.valid || (*status & (16 | 32))) {
    if (threadIdx.x == 0) {
      DevDecision d;
      d.mask = 0; d.popcount = 0; d.e_loc = 0.0; d.e_min = 0.0; d.ambiguous = 0; d.found = 0;
      d.key_gap = INFINITY;
      d.smice_rise = 0.0;
      *dec = d;
    }
    return;
  }
  const int tid = threadIdx.x, bd = blockDim.x, lane = tid & 63, wv = tid >> 6, nw = bd >> 6;
  const int k = H.k;
  const uint32_t nm = 1u << k;
  const uint32_t L = (uint32_t)H.lanebits;  // tile t, lane q holds tile_mask(L, t, q, k)
  const int lb = __popc(L);
  const int ntiles = (int)(nm >> lb);
  // up to one tile per thread (segments of up to 16 nodes): its record is
  // read once and kept in registers
  const bool one = ntiles <= bd;
  TileRec r0;
  r0.best = -1;
  r0.near = -1;
  r0.emin = INFINITY;
  int best = -1;
  for (int t = tid; t < ntiles; t += bd) {
    const TileRec r = tiles[t];
    if (t == tid) r0 = r;
    best = max(best, r.best);
  }
  for (int o = 32; o > 0; o >>= 1) best = max(best, __shfl_xor(best, o, 64));
  if (lane == 0) s_best[wv] = best;
  __syncthreads();
  best = s_best[0];
  for (int w = 1; w < nw; ++w) best = max(best, s_best[w]);
  // the smallest error at the chosen level, and masks near the boundary
  double emin = INFINITY;
  int amb = 0;
  if (best >= 0)
    for (int t = tid; t < ntiles; t += bd) {
      const TileRec r = one ? r0 : tiles[t];
      if (r.best == best) emin = fmin(emin, r.emin);
      if (r.near >= best) amb = 1;
    }
  for (int o = 32; o > 0; o >>= 1) {
    emin = fmin(emin, __shfl_xor(emin, o, 64));
    amb |= __shfl_xor(amb, o, 64);
  }
  if (lane == 0) {
    s_emin[wv] = emin;
    s_amb[wv] = amb;
  }
  __syncthreads();
  emin = s_emin[0];
  amb = s_amb[0];
  for (int w = 1; w < nw; ++w) {
    emin = fmin(emin, s_emin[w]);
    amb |= s_amb[w];
  }
  unsigned pick = 0xffffffffu;
  const double thr = emin + sp.tie;
  // runner-up: the smallest error above the tie window at the chosen level
  // (a tile not rescanned holds it at its own minimum)
  double runner = INFINITY;
  // candidate tiles, processed in chunks of one tile per thread
  for (int base = 0; base < ntiles && best >= 0; base += bd) {
    if (tid == 0) ncand = 0;
    __syncthreads();
    const int t = base + tid;
    if (t < ntiles) {
      const TileRec r = one ? r0 : tiles[t];
      if (r.best == best && r.emin <= thr + sp.amb) cand[atomicAdd(&ncand, 1)] = t;
      else if (r.best == best) runner = fmin(runner, r.emin);
    }
    __syncthreads();
    const int nc = ncand;
    for (int q = tid; q < nc * 64; q += bd) {
      if ((q & 63) >> lb) continue;
      const uint32_t mm = tile_mask(L, (uint32_t)cand[q >> 6], (uint32_t)(q & 63), k);
      if (__popc(mm) != best) continue;  // (only these masks' scores are stored)
      const MaskScore r = fin[mm];
      if (!feasible(r, sp.e_bar)) continue;
      if (fabs(r.e - thr) <= sp.amb) amb = 1;
      if (r.e <= thr) pick = min(pick, mm);
      else runner = fmin(runner, r.e);
    }
    __syncthreads();
  }
  for (int o = 32; o > 0; o >>= 1) {
    pick = min(pick, (unsigned)__shfl_xor((int)pick, o, 64));
    amb |= __shfl_xor(amb, o, 64);
    runner = fmin(runner, __shfl_xor(runner, o, 64));
  }
  if (lane == 0) {
    s_pick[wv] = pick;
    s_amb2[wv] = amb;
    s_run[wv] = runner;
  }
  __syncthreads();
  if (tid == 0) {
    for (int w = 1; w < nw; ++w) {
      pick = min(pick, s_pick[w]);
      amb |= s_amb2[w];
      runner = fmin(runner, s_run[w]);
    }
    DevDecision d;
    if (best < 0) {
      d.mask = 0; d.popcount = 0; d.e_loc = fin[0].e; d.e_min = fin[0].e; d.ambiguous = 1; d.found = 0;
      d.key_gap = INFINITY;
      d.smice_rise = 0.0;
    } else {
      d.mask = pick; d.popcount = best; d.e_loc = fin[pick].e; d.e_min = emin; d.ambiguous = amb; d.found = 1;
      d.key_gap = runner - emin;
      d.smice_rise = 0.0;
    }
    *dec = d;
  }
}

// Self-test hook: sqrt_nr on an array (host compares with the libm result).
__global__ void k_sqrt_selftest(const double* __restrict__ x, double* __restrict__ y, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = sqrt_nr(x[i]);
}

// ------------------------------------------------------------ state update --
// Apply the chosen mask to the cumulative state (Algorithm 1 state update):
// aggregated currents move to the new super-nodes, kept slots and zone
// targets take their candidate voltages (same arithmetic as the scoring).
// Block 0 then updates the kept flags and super-nodes over Omega_g and clears
// the node -> slot / zone-entry maps for the next segment.
__global__ __launch_bounds__(64) void k_apply(const SegHdr* __restrict__ hdrs, const int* __restrict__ segs,
                                              size_t lstride, const int* __restrict__ tab,
                                              Topo T, State St, const DevDecision* __restrict__ decs,
                                              const double2* __restrict__ P, const TargetRec* __restrict__ srec,
                                              const TargetRec* __restrict__ zrec, double2* __restrict__ Vcur,
                                              double2* __restrict__ A) {
  __shared__ double2 Bs[kMaxK * 3];
  const int g = segs[blockIdx.z];
  const SegHdr H = load_hdr_g(hdrs, g);
  if (!H.valid) return;
  tab = lane_ptr(tab, lstride);
  P = lane_ptr(P, lstride);
  srec = lane_ptr(srec, lstride);
  zrec = lane_ptr(zrec, lstride);
  const int n = T.n;
  const int l = blockIdx.x;
  const uint32_t m = *as_cint((const int*)&decs[g].mask);
  const cint* chains = as_cint(tab + H.o_chain);
  const cint* slots = as_cint(tab + H.o_slot);
  if (threadIdx.x < 3) {  // phases are independent: one thread each
    const int p = threadIdx.x;
    const double2* Pl = P + (size_t)l * H.npairs * 3;
    const TargetRec* srec_l = srec + (size_t)l * H.nslots * 3;
    for (int c = 0; c < H.nchains; ++c) {
      const cint* cr = chains + c * kChainInts;
      const int outer = cr[C_OUTER];
      double2 S = outer >= 0 ? Bs[outer * 3 + p] : make_double2(0.0, 0.0);
      int sidx = 0;
      // the current super-node's aggregated current, kept in a register
      // while reduced slots add theirs (the same additions, in order)
      size_t a = ((size_t)l * n + cr[C_HEAD]) * 3 + p;
      double2 acc = A[a];
      const int ns = cr[C_NSLOT], s0 = cr[C_SLOT0];
      for (int r = 0; r < ns; ++r) {
        const cint* sr = slots + (s0 + r) * kSlotInts;
        const int node = sr[SL_NODE];
        if ((m >> sr[SL_BIT]) & 1u) {
          S = cadd(S, Pl[(sr[SL_PAIRBASE] + sidx) * 3 + p]);
          const size_t b = ((size_t)l * n + node) * 3 + p;
          acc = cadd(acc, A[b]);
          A[b] = make_double2(0.0, 0.0);
        } else {
          if (sr[SL_PHASE] >> p & 1) Vcur[((size_t)l * n + node) * 3 + p] = cadd(srec_l[(s0 + r) * 3 + p].W, S);
          sidx = r + 1;
          A[a] = acc;
          a = ((size_t)l * n + node) * 3 + p;
          acc = A[a];
        }
      }
      A[a] = acc;
      Bs[c * 3 + p] = S;
    }
  }
  __syncthreads();
  for (int q = threadIdx.x; q < H.nz; q += blockDim.x) {
    const int* ze = tab + H.o_zent + q * 3;
    const int node = ze[0], p = ze[1], c = ze[2];
    Vcur[((size_t)l * n + node) * 3 + p] = cadd(zrec[(size_t)l * H.nz + q].W, Bs[c * 3 + p]);
  }
  if (blockIdx.x != 0) return;
  __syncthreads();
  if (threadIdx.x < H.nslots) {
    const cint* sr = slots + threadIdx.x * kSlotInts;
    if ((m >> sr[SL_BIT]) & 1u) St.kept[sr[SL_NODE]] = 0;
    St.slot_of[sr[SL_NODE]] = -1;
  }
  for (int q = threadIdx.x; q < H.nz; q += blockDim.x) {
    const int* ze = tab + H.o_zent + q * 3;
    St.zent_of[ze[0] * 3 + ze[1]] = -1;
  }
  __syncthreads();
  const int* rg = tab + H.o_range;
  for (int q = threadIdx.x; q < H.nomega; q += blockDim.x) {
    int r = 0;
    while (r + 1 < H.nrange && rg[3 * (r + 1) + 2] <= q) ++r;
    const int i = T.pre[rg[3 * r] + (q - rg[3 * r + 2])];
    // up through reduced nodes; a reduced node's recorded super (before or
    // after this update) is an ancestor with only reduced nodes in between
    int v = i;
    while (!St.kept[v]) {
      const int s = St.sup[v];
      v = (s >= 0 && s != v) ? s : T.parent[v];
    }
    St.sup[i] = v;
  }
}

// Reset of the search state at the start of a call (no memset nodes, so the
// sequence can be captured in a graph).
__global__ void k_init_state(int n, State St, int* __restrict__ status, int nstatus, int* __restrict__ tickets,
                             int ntickets, int nlanes, size_t lstride) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    St.kept[i] = 1;
    St.sup[i] = i;
    St.slot_of[i] = -1;
    St.zent_of[3 * i] = St.zent_of[3 * i + 1] = St.zent_of[3 * i + 2] = -1;
  }
  if (i < nstatus) status[i] = 0;
  if (i < ntickets)  // every chunk position's ticket counters (position z: z * lstride bytes further)
    for (int z = 0; z < nlanes; ++z) ((int*)((char*)tickets + (size_t)z * lstride))[i] = 0;
}

__global__ void k_copy2(const double2* __restrict__ a, double2* __restrict__ b, size_t count) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
    b[i] = a[i];
}

// ---------------------------------------------------------- final outputs --
// Per-snapshot max error of the final reduction over every node-phase.
__global__ __launch_bounds__(256) void k_final_err(int n, const uint8_t* __restrict__ phase,
                                                   const int* __restrict__ sup, const double2* __restrict__ Vcur,
                                                   const double* __restrict__ absV, double* __restrict__ err) {
  __shared__ double shd[16];
  const int l = blockIdx.x;
  double e = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x)
    for (int p = 0; p < 3; ++p) {
      if (!(phase[i] >> p & 1u)) continue;
      const double m = sqrt(cabs2(Vcur[((size_t)l * n + sup[i]) * 3 + p]));
      e = fmax(e, fabs(m - absV[((size_t)l * n + i) * 3 + p]));
    }
  e = block_reduce(e, [](double a, double b) { return fmax(a, b); }, shd);
  if (threadIdx.x == 0) err[l] = e;
}

// Kron-reduced branch of every kept node: the eliminated path up to its kept
// parent is a series chain, so y_eq = (sum of z on the path, restricted to
// the node's phases)^-1 (eq. Y_kron for degree-2 and leaf eliminations).
__global__ void k_kron_yeq(Topo T, State St, const double2* __restrict__ z, double2* __restrict__ yeq,
                           double2* __restrict__ Yk_off, int* __restrict__ kp_out, int* __restrict__ status) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= T.n) return;
  double2* yo = Yk_off + (size_t)x * 9;
  double2* ye = yeq + (size_t)x * 9;
  for (int q = 0; q < 9; ++q) { yo[q] = make_double2(0.0, 0.0); ye[q] = yo[q]; }
  const int kp = (x > 0 && St.kept[x]) ? St.sup[T.parent[x]] : -1;
  kp_out[x] = kp;
  if (kp < 0) return;
  const unsigned ph = T.phase[x];
  double2 Z[9];
  for (int q = 0; q < 9; ++q) Z[q] = make_double2(0.0, 0.0);
  for (int v = x; v != kp; v = T.parent[v]) {
    const double2* zv = z + (size_t)v * 9;
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c)
        if ((ph >> r & 1u) && (ph >> c & 1u)) Z[r * 3 + c] = cadd(Z[r * 3 + c], zv[r * 3 + c]);
  }
  if (!inv_restricted(Z, ph, ye)) { atomicOr(status, 1); return; }
  for (int q = 0; q < 9; ++q) yo[q] = make_double2(-ye[q].x, -ye[q].y);
}

// Y_Kron(x,x) = y_eq of x's own branch plus those of its reduced-network
// children, found by following each tree child down through reduced nodes
// (which have at most one child) to the first kept node.
__global__ void k_kron_diag(Topo T, State St, const double2* __restrict__ yeq, double2* __restrict__ Yk_diag) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= T.n) return;
  double2 D[9];
  for (int q = 0; q < 9; ++q) D[q] = make_double2(0.0, 0.0);
  if (St.kept[x]) {
    if (x > 0)
      for (int q = 0; q < 9; ++q) D[q] = yeq[(size_t)x * 9 + q];
    for (int e = T.ch_off[x]; e < T.ch_off[x + 1]; ++e) {
      int v = T.ch[e];
      while (!St.kept[v] && T.ch_off[v + 1] > T.ch_off[v]) v = T.ch[T.ch_off[v]];
      if (St.kept[v])
        for (int q = 0; q < 9; ++q) D[q] = cadd(D[q], yeq[(size_t)v * 9 + q]);
    }
  }
  for (int q = 0; q < 9; ++q) Yk_diag[(size_t)x * 9 + q] = D[q];
}

}  // namespace okr
