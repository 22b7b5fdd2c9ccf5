// Learned pruning: a 3-layer MLP (F -> 256 -> 256 -> 1, GELU, BF16 operands,
// FP32 accumulation on MFMA) predicts y = ln(e_loc + 1e-12) of every mask of
// a segment from per-mask features; the top-k masks by (predicted feasible,
// most reduced, smallest predicted error) are rescored exactly in FP64, and
// the full enumeration runs when none of them is feasible with a reduction.
//
// Parameters (FP32, one contiguous buffer, [out][in] layout):
//   W1[256][32] b1[256] W2[256][256] b2[256] w3[256] b3[1]
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "okr_device.h"
#include "okr_internal.h"

namespace okr {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// ------------------------------------------------------ per-mask features --
// Per-pair and per-slot feature tables (maxima over the snapshots): one wave
// per pair or slot, lanes over the snapshots, a wave reduction.
__global__ __launch_bounds__(64) void k_surr_tables(const SegHdr* __restrict__ hdrs, int g,
                                                    const int* __restrict__ tab, int n,
                                                    const double2* __restrict__ Zroot, const double2* __restrict__ P,
                                                    const double2* __restrict__ A,
                                                    const TargetRec* __restrict__ srec, float* __restrict__ pz,
                                                    float* __restrict__ zs, SurrSlot* __restrict__ ss) {
  const SegHdr H = load_hdr_g(hdrs, g);
  if (!H.valid) return;
  const int t = blockIdx.x, lane = threadIdx.x;
  if (t < H.npairs) {
    const int* pr = tab + H.o_pair + t * kPairInts;
    double mx = 0.0;
    for (int l = lane; l < H.S; l += 64)
      for (int p = 0; p < 3; ++p) mx = fmax(mx, sqrt(cabs2(P[((size_t)l * H.npairs + t) * 3 + p])));
    for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
    if (lane == 0) {
      // sum of |Z(s -> r)| over the diagonal, Z(s -> r) = Zroot(r) - Zroot(s)
      double zsum = 0.0;
      const double2* zr = Zroot + (size_t)pr[PR_RNODE] * 9;
      const double2* zs0 = Zroot + (size_t)pr[PR_SUPER] * 9;
      for (int p = 0; p < 3; ++p) zsum += sqrt(cabs2(csub(zr[p * 4], zs0[p * 4])));
      pz[t] = (float)mx;
      zs[t] = (float)zsum;
    }
  } else if (t < H.npairs + H.nslots) {
    const int s = t - H.npairs;
    const int* sr = tab + H.o_slot + s * kSlotInts;
    const int node = sr[SL_NODE], ph = sr[SL_PHASE];
    double la = 0.0, sp = 0.0;
    for (int l = lane; l < H.S; l += 64) {
      double a = 0.0;
      for (int p = 0; p < 3; ++p) {
        a += sqrt(cabs2(A[((size_t)l * n + node) * 3 + p]));
        if (ph >> p & 1) {
          const TargetRec r = srec[((size_t)l * H.nslots + s) * 3 + p];
          sp = fmax(sp, r.hi - r.lo);
        }
      }
      la = fmax(la, a);
    }
    for (int o = 32; o > 0; o >>= 1) {
      la = fmax(la, __shfl_xor(la, o, 64));
      sp = fmax(sp, __shfl_xor(sp, o, 64));
    }
    if (lane == 0) {
      const int* cr = tab + H.o_chain + sr[SL_CHAIN] * kChainInts;
      SurrSlot o;
      o.la = (float)la;
      o.spread = (float)sp;
      o.nph = __popc(ph);
      o.pos = s - cr[C_SLOT0];
      ss[s] = o;
    }
  }
}

// Features of mask m from a snapshot-free walk of the chains (the moved
// currents' voltage rises, path impedance sums, load totals, phase counts,
// run lengths, depth), scaled to O(1); ec = the largest constant error over
// the snapshots.  Table pointers may point to global memory or to an LDS copy.
__device__ __forceinline__ void surr_features(const SegHdr& H, const int* chains, const int* slots, const float* pz,
                                              const float* zs, const SurrSlot* ss, double ec, uint32_t m,
                                              float (&f)[kSurrF]) {
  for (int q = 0; q < kSurrF; ++q) f[q] = 0.f;
  float sum_pz = 0.f, max_pz = 0.f, sum_z = 0.f, sum_la = 0.f, max_sp = 0.f, sum_pos = 0.f;
  int n1 = 0, n2 = 0, n3 = 0, maxrun = 0, touched = 0, pop = 0;
  for (int c = 0; c < H.nchains; ++c) {
    const int* cr = chains + c * kChainInts;
    int sidx = 0, run = 0, tc = 0;
    for (int r = 0; r < cr[C_NSLOT]; ++r) {
      const int s = cr[C_SLOT0] + r;
      const int* sr = slots + s * kSlotInts;
      if ((m >> sr[SL_BIT]) & 1u) {
        const int q = sr[SL_PAIRBASE] + sidx;
        const SurrSlot o = ss[s];
        sum_pz += pz[q];
        max_pz = fmaxf(max_pz, pz[q]);
        sum_z += zs[q];
        sum_la += o.la;
        max_sp = fmaxf(max_sp, o.spread);
        sum_pos += (float)o.pos;
        n1 += o.nph == 1;
        n2 += o.nph == 2;
        n3 += o.nph == 3;
        ++pop;
        maxrun = max(maxrun, ++run);
        tc = 1;
      } else {
        sidx = r + 1;
        run = 0;
      }
    }
    touched += tc;
  }
  const float k = (float)H.k;
  f[0] = pop / k;
  f[1] = sum_pz * 1e3f;
  f[2] = max_pz * 1e3f;
  f[3] = sum_z * 1e2f;
  f[4] = sum_la * 10.f;
  f[5] = n1 / k;
  f[6] = n2 / k;
  f[7] = n3 / k;
  f[8] = maxrun / k;
  f[9] = touched / (float)H.nchains;
  f[10] = sum_pos / k;
  f[11] = max_sp * 1e3f;
  f[12] = log10f(max_pz + 1e-9f) / 4.f;
  f[13] = log10f(sum_pz + 1e-9f) / 4.f;
  f[14] = (float)ec * 1e3f;
  f[15] = k / 24.f;
}

// Features of every listed mask (or mask = row); rows >= n or masks >= 2^k
// are zero padding.
__global__ void k_surr_features(const SegHdr* __restrict__ hdrs, int g, const int* __restrict__ tab,
                                const float* __restrict__ pz, const float* __restrict__ zs,
                                const SurrSlot* __restrict__ ss, const double* __restrict__ econst,
                                const uint32_t* __restrict__ masks, int n, int Mp, float* __restrict__ Xf,
                                __bf16* __restrict__ Xb, const int* __restrict__ flag, int skip_if) {
  const SegHdr H = load_hdr_g(hdrs, g);
  if (!H.valid || (flag && *flag == skip_if)) return;
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (uint32_t)Mp) return;
  const uint32_t m = (masks && i < (uint32_t)n) ? masks[i] : i;
  float f[kSurrF];
  for (int q = 0; q < kSurrF; ++q) f[q] = 0.f;
  if (i < (uint32_t)n && m < (1u << H.k)) {
    double ec = 0.0;
    for (int l = 0; l < H.S; ++l) ec = fmax(ec, econst[l]);
    surr_features(H, tab + H.o_chain, tab + H.o_slot, pz, zs, ss, ec, m, f);
  }
  if (Xf)
    for (int q = 0; q < kSurrF; ++q) Xf[(size_t)i * kSurrF + q] = f[q];
  if (Xb)
    for (int q = 0; q < kSurrF; ++q) Xb[(size_t)i * kSurrF + q] = (__bf16)f[q];
}

// Masks of popcount >= L1 over k bits, level by level from the top, each
// level in colexicographic order (combinatorial number system); rows
// [N1, M1) are padding.
struct BinomTable {
  uint32_t v[kMaxK + 1][kMaxK + 1];
};
constexpr BinomTable make_binom() {
  BinomTable t{};
  for (int n = 0; n <= kMaxK; ++n) {
    t.v[n][0] = 1u;
    for (int r = 1; r <= n; ++r) t.v[n][r] = t.v[n - 1][r - 1] + (r <= n - 1 ? t.v[n - 1][r] : 0u);
  }
  return t;
}
__constant__ BinomTable kBinom = make_binom();  // Pascal's triangle, C(n, r) for n <= 24

__device__ __forceinline__ uint32_t binom(int n, int r) { return (r < 0 || r > n) ? 0u : kBinom.v[n][r]; }

__global__ void k_level_masks(int k, int L1, int N1, int M1, uint32_t* __restrict__ masks) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M1) return;
  if (i >= N1) {
    masks[i] = 0u;
    return;
  }
  int j = k;
  uint32_t r = (uint32_t)i;
  while (j > L1 && r >= binom(k, j)) {
    r -= binom(k, j);
    --j;
  }
  uint32_t m = 0u;
  for (int pos = k - 1; pos >= 0 && j > 0; --pos) {
    const uint32_t c = binom(pos, j);
    if (c <= r) {
      m |= 1u << pos;
      r -= c;
      --j;
    }
  }
  masks[i] = m;
}

// Training target of every mask from the FP64 scores: y = ln(e + 1e-12).
__global__ void k_surr_target(const SegHdr* __restrict__ hdrs, int g, const MaskScore* __restrict__ fin,
                              float* __restrict__ t) {
  const SegHdr H = load_hdr_g(hdrs, g);
  const uint32_t m = blockIdx.x * blockDim.x + threadIdx.x;
  if (!H.valid || m >= (1u << H.k)) return;
  t[m] = (float)log(fin[m].e + 1e-12);
}

// --------------------------------------------------------------- BF16 GEMM --
__device__ __forceinline__ float gelu_f(float x) { return 0.5f * x * (1.f + erff(x * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad_f(float x) {
  const float cdf = 0.5f * (1.f + erff(x * 0.70710678118654752f));
  const float pdf = 0.39894228040143268f * expf(-0.5f * x * x);
  return cdf + x * pdf;
}

enum { EPI_STORE = 0, EPI_BIAS_GELU = 1, EPI_BIAS_GELU_DOT = 2 };

// C[M][N] = sum_k A[m][k] * B[n][k] (A, B BF16, K contiguous), FP32 results.
// 256 threads = 4 waves (2 x 2), block tile 64 x 64, K step 32 through LDS;
// each wave a 32 x 32 tile with v_mfma_f32_32x32x16_bf16.  M, N multiples of
// 64, K a multiple of 32.  Epilogues:
//   STORE          C (ldc)
//   BIAS_GELU      Z = C + bias (FP32, optional), H = gelu(Z) in BF16 [M][N]
//                  (optional) and transposed Ht [N][M] (optional)
//   BIAS_GELU_DOT  as BIAS_GELU, plus per-row partial dot products of
//                  gelu(Z) with w over each 32-column block: part[N/32][M]
template <int EPI>
__global__ __launch_bounds__(256) void k_gemm_nt(const __bf16* __restrict__ A, int lda, const __bf16* __restrict__ B,
                                                 int ldb, int K, float* __restrict__ C, int ldc,
                                                 const float* __restrict__ bias, float* __restrict__ Z,
                                                 __bf16* __restrict__ Hb, __bf16* __restrict__ Ht, int M,
                                                 const float* __restrict__ w, float* __restrict__ part,
                                                 const int* __restrict__ flag, int skip_if) {
  __shared__ __attribute__((aligned(16))) __bf16 As[64][40];
  if (flag && *flag == skip_if) return;
  __shared__ __attribute__((aligned(16))) __bf16 Bs[64][40];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  f32x16 acc;
  for (int v = 0; v < 16; ++v) acc[v] = 0.f;
  const int lr = tid >> 2, lc = (tid & 3) * 8;
  // split K over grid.z (STORE only): slice z writes its partial product to
  // C + z * M * ldc
  const int kspan = K / (int)gridDim.z, kb = (int)blockIdx.z * kspan;
  if (EPI == EPI_STORE) C += (size_t)blockIdx.z * M * ldc;
  for (int k0 = kb; k0 < kb + kspan; k0 += 32) {
    *(uint4*)&As[lr][lc] = *(const uint4*)&A[(size_t)(m0 + lr) * lda + k0 + lc];
    *(uint4*)&Bs[lr][lc] = *(const uint4*)&B[(size_t)(n0 + lr) * ldb + k0 + lc];
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 32; kk += 16) {
      const bf16x8 a = *(const bf16x8*)&As[wm * 32 + (lane & 31)][kk + 8 * (lane >> 5)];
      const bf16x8 b = *(const bf16x8*)&Bs[wn * 32 + (lane & 31)][kk + 8 * (lane >> 5)];
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
    }
    __syncthreads();
  }
  const int col = n0 + wn * 32 + (lane & 31);
  float dot[16];
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int row = m0 + wm * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
    float x = acc[v];
    if (EPI == EPI_STORE) {
      C[(size_t)row * ldc + col] = x;
    } else {
      x += bias[col];
      if (Z) Z[(size_t)row * ldc + col] = x;
      const float h = gelu_f(x);
      if (Hb) Hb[(size_t)row * ldc + col] = (__bf16)h;
      if (Ht) Ht[(size_t)col * M + row] = (__bf16)h;
      if (EPI == EPI_BIAS_GELU_DOT) dot[v] = h * w[col];
    }
  }
  if (EPI == EPI_BIAS_GELU_DOT) {
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      float s = dot[v];
      for (int o = 1; o < 32; o <<= 1) s += __shfl_xor(s, o, 64);
      const int row = m0 + wm * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
      if ((lane & 31) == 0) part[(size_t)((n0 + wn * 32) / 32) * M + row] = s;
    }
  }
}

#define OKR_GEMM_INST(E)                                                                                       \
  template __global__ void k_gemm_nt<E>(const __bf16*, int, const __bf16*, int, int, float*, int, const float*, \
                                        float*, __bf16*, __bf16*, int, const float*, float*, const int*, int);
OKR_GEMM_INST(EPI_STORE)
OKR_GEMM_INST(EPI_BIAS_GELU)
OKR_GEMM_INST(EPI_BIAS_GELU_DOT)
#undef OKR_GEMM_INST

// out[i] = sum over the K slices' partial products, in slice order.
__global__ void k_sum_splits(const float* __restrict__ part, int splits, int n, float* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float t = 0.f;
  for (int z = 0; z < splits; ++z) t += part[(size_t)z * n + i];
  out[i] = t;
}

// y[m] = b3 + sum over the column blocks' partial dots, in a fixed order.
__global__ void k_rowdot_finish(const float* __restrict__ part, int nblk, int M, const float* __restrict__ b3,
                                float* __restrict__ y, const int* __restrict__ flag, int skip_if) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= M || (flag && *flag == skip_if)) return;
  float s = b3[0];
  for (int j = 0; j < nblk; ++j) s += part[(size_t)j * M + m];
  y[m] = s;
}

// ------------------------------------------------------------- training --
// Batch rows (FP32 [B][F]) to BF16 [B][F] and the transposed [64][B] (rows
// F..63 zero) for the weight gradient of layer 1.
__global__ void k_batch_cast(const float* __restrict__ X, int B, __bf16* __restrict__ Xb, __bf16* __restrict__ Xt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= B * 64) return;
  const int b = i / 64, j = i % 64;
  const float v = j < kSurrF ? X[(size_t)b * kSurrF + j] : 0.f;
  if (j < kSurrF) Xb[(size_t)b * kSurrF + j] = (__bf16)v;
  Xt[(size_t)j * B + b] = (__bf16)v;
}

__global__ void k_loss_dy(const float* __restrict__ y, const float* __restrict__ t, int B, float* __restrict__ dy,
                          float* __restrict__ loss) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  float l = 0.f;
  if (b < B) {
    const float d = y[b] - t[b];
    dy[b] = 2.f * d / B;
    l = d * d / B;
  }
  for (int o = 32; o > 0; o >>= 1) l += __shfl_xor(l, o, 64);
  if ((threadIdx.x & 63) == 0) atomicAdd(loss, l);
}

// dZ2 = dy w3^T * gelu'(Z2) as BF16 [B][256] and transposed [256][B]
__global__ void k_dz2(const float* __restrict__ Z2, const float* __restrict__ dy, const float* __restrict__ w3, int B,
                      __bf16* __restrict__ dZ2b, __bf16* __restrict__ dZ2t) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= B * kSurrH) return;
  const int b = i / kSurrH, o = i % kSurrH;
  const float v = dy[b] * w3[o] * gelu_grad_f(Z2[i]);
  dZ2b[i] = (__bf16)v;
  dZ2t[(size_t)o * B + b] = (__bf16)v;
}

// dZ1 = dH1 * gelu'(Z1), transposed BF16 [256][B]
__global__ void k_dz1(const float* __restrict__ dH1, const float* __restrict__ Z1, int B, __bf16* __restrict__ dZ1t) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= B * kSurrH) return;
  const int b = i / kSurrH, o = i % kSurrH;
  dZ1t[(size_t)o * B + b] = (__bf16)(dH1[i] * gelu_grad_f(Z1[i]));
}

// Column reductions over the batch, in two passes with a fixed order (no
// atomics): partial sums over row chunks of kColChunk, then their sum.
//   gb2[o] = sum_b dy[b] w3[o] gelu'(Z2[b][o]);  gw3[o] = sum_b gelu(Z2[b][o]) dy[b]
//   gb1[o] = sum_b dH1[b][o] gelu'(Z1[b][o]);    gb3 = sum_b dy[b]
constexpr int kColChunk = 256;
constexpr int kColVals = 3 * kSurrH + 1;  // gb2, gw3, gb1 per column, then gb3

__global__ void k_colsums_part(const float* __restrict__ Z1, const float* __restrict__ dH1,
                               const float* __restrict__ Z2, const float* __restrict__ dy,
                               const float* __restrict__ w3, int B, float* __restrict__ part) {
  const int o = threadIdx.x;  // blockDim = kSurrH + 1
  const int b0 = blockIdx.x * kColChunk, b1 = min(B, b0 + kColChunk);
  float* out = part + (size_t)blockIdx.x * kColVals;
  if (o < kSurrH) {
    float a = 0.f, c = 0.f, d = 0.f;
    for (int b = b0; b < b1; ++b) {
      const float z2 = Z2[(size_t)b * kSurrH + o];
      a += dy[b] * w3[o] * gelu_grad_f(z2);
      c += gelu_f(z2) * dy[b];
      d += dH1[(size_t)b * kSurrH + o] * gelu_grad_f(Z1[(size_t)b * kSurrH + o]);
    }
    out[o] = a;
    out[kSurrH + o] = c;
    out[2 * kSurrH + o] = d;
  } else if (o == kSurrH) {
    float t = 0.f;
    for (int b = b0; b < b1; ++b) t += dy[b];
    out[3 * kSurrH] = t;
  }
}

__global__ void k_colsums_final(const float* __restrict__ part, int nchunk, float* __restrict__ gb1,
                                float* __restrict__ gb2, float* __restrict__ gw3, float* __restrict__ gb3) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= kColVals) return;
  float t = 0.f;
  for (int c = 0; c < nchunk; ++c) t += part[(size_t)c * kColVals + q];
  if (q < kSurrH) gb2[q] = t;
  else if (q < 2 * kSurrH) gw3[q - kSurrH] = t;
  else if (q < 3 * kSurrH) gb1[q - 2 * kSurrH] = t;
  else gb3[0] = t;
}

__global__ void k_copy_cols(const float* __restrict__ src, int lds, float* __restrict__ dst, int rows, int cols) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < rows * cols) dst[i] = src[(size_t)(i / cols) * lds + i % cols];
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ gr, float* __restrict__ m,
                       float* __restrict__ v, int n, float lr, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = gr[i];
  const float mi = 0.9f * m[i] + 0.1f * gi;
  const float vi = 0.999f * v[i] + 0.001f * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
}

// BF16 copies of the weights: W1 [256][32], W2 [256][256] and W2^T.
__global__ void k_refresh_weights(const float* __restrict__ prm, __bf16* __restrict__ W1b, __bf16* __restrict__ W2b,
                                  __bf16* __restrict__ W2tb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < kSurrH * kSurrF) W1b[i] = (__bf16)prm[kOffW1 + i];
  if (i < kSurrH * kSurrH) {
    const float v = prm[kOffW2 + i];
    W2b[i] = (__bf16)v;
    if (W2tb) W2tb[(size_t)(i % kSurrH) * kSurrH + i / kSurrH] = (__bf16)v;
  }
}

__global__ void k_zero_f32(float* __restrict__ a, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0.f;
}

// ---------------------------------------------------- top-k and decision --
__device__ __forceinline__ uint32_t ordered(float y) {
  const uint32_t u = __float_as_uint(y);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// Rank key of every mask: predicted feasible first, then most reduced, then
// smallest predicted error (26-bit monotone quantisation), ties by mask.

// Whether the first ranking stage (the top levels) holds at least K masks
// predicted feasible: then the K best keys overall are among them, since
// predicted-feasible masks rank by level first.
__global__ __launch_bounds__(256) void k_surr_stage(const SegHdr* __restrict__ hdrs, int g,
                                                    const uint32_t* __restrict__ keys, int n, int K,
                                                    int* __restrict__ flag) {
  __shared__ int shi[4];
  const SegHdr H = load_hdr_g(hdrs, g);
  int c = 0;
  if (H.valid)
    for (int i = threadIdx.x; i < n; i += blockDim.x) c += (keys[i] >> 31) == 0u;
  c = block_reduce(c, [](int a, int b) { return a + b; }, shi);
  if (threadIdx.x == 0) *flag = (H.valid && c >= K) ? 1 : 0;
}

// The K smallest keys, ties at the K-th key broken by the lowest mask index:
// a radix select of the K-th key, a radix select over the mask indices of
// the masks holding that key, then one collection pass (list order is not
// meaningful; its content is).  One block.
// Radix-select step, run by the first wave: the digit d holding the need-th
// smallest element of a 256-bin histogram, the count below it and its own
// count (lane l scans bins 4l..4l+3; a wave prefix sum and a ballot find d).
__device__ __forceinline__ void select_digit(const int* hist, int need, int& d, int& below, int& cnt) {
  const int lane = threadIdx.x & 63;
  const int h0 = hist[4 * lane], h1 = hist[4 * lane + 1], h2 = hist[4 * lane + 2], h3 = hist[4 * lane + 3];
  const int own = h0 + h1 + h2 + h3;
  int incl = own;
  for (int o = 1; o < 64; o <<= 1) {
    const int v = __shfl_up(incl, o, 64);
    if (lane >= o) incl += v;
  }
  const uint64_t hit = __ballot(incl >= need);
  const int src = hit ? __ffsll((unsigned long long)hit) - 1 : 63;
  int base = __shfl(incl - own, src, 64);
  const int c0 = __shfl(h0, src, 64), c1 = __shfl(h1, src, 64), c2 = __shfl(h2, src, 64),
            c3 = __shfl(h3, src, 64);
  int j = 0, c = c0;
  if (base + c0 < need) {
    base += c0;
    j = 1;
    c = c1;
    if (base + c1 < need) {
      base += c1;
      j = 2;
      c = c2;
      if (base + c2 < need) {
        base += c2;
        j = 3;
        c = c3;
      }
    }
  }
  d = 4 * src + j;
  below = base;
  cnt = c;
}

__global__ __launch_bounds__(1024) void k_topk(const SegHdr* __restrict__ hdrs, int g,
                                               const uint32_t* __restrict__ keys,
                                               const uint32_t* __restrict__ masks, int n, int topk,
                                               const int* __restrict__ status, uint32_t* __restrict__ list,
                                               int* __restrict__ count, const int* __restrict__ flag,
                                               int skip_if) {
  __shared__ int hist[256];
  __shared__ uint32_t s_prefix, s_maskbits, s_mprefix, s_mmaskbits;
  __shared__ int s_need, s_eq, s_n;
  if (flag && *flag == skip_if) return;
  const SegHdr H = load_hdr_g(hdrs, g);
  if (!H.valid || (*status & (16 | 32))) {
    if (threadIdx.x == 0) *count = 0;
    return;
  }
  const uint32_t nm = (uint32_t)n;
  const int K = (int)min((uint32_t)topk, nm);
  if (threadIdx.x == 0) { s_prefix = 0; s_maskbits = 0; s_need = K; s_eq = 0; s_n = 0; }
  __syncthreads();
  // K-th smallest key T; s_need = how many masks holding T belong to the top K
  for (int shift = 24; shift >= 0; shift -= 8) {
    for (int q = threadIdx.x; q < 256; q += blockDim.x) hist[q] = 0;
    __syncthreads();
    const uint32_t pre = s_prefix, mb = s_maskbits;
    for (uint32_t i = threadIdx.x; i < nm; i += blockDim.x) {
      const uint32_t key = keys[i];
      if ((key & mb) == pre) atomicAdd(&hist[(key >> shift) & 255u], 1);
    }
    __syncthreads();
    if (threadIdx.x < 64) {
      int d, below, cnt;
      select_digit(hist, s_need, d, below, cnt);
      if (threadIdx.x == 0) {
        s_need -= below;
        s_prefix = pre | ((uint32_t)d << shift);
        s_maskbits = mb | (255u << shift);
        if (shift == 0) s_eq = cnt;  // masks holding T
      }
    }
    __syncthreads();
  }
  const uint32_t T = s_prefix;
  // the s_need lowest mask indices among the s_eq masks holding T
  if (threadIdx.x == 0) { s_mprefix = 0; s_mmaskbits = 0; }
  __syncthreads();
  if (s_need < s_eq) {
    for (int shift = 16; shift >= 0; shift -= 8) {
      for (int q = threadIdx.x; q < 256; q += blockDim.x) hist[q] = 0;
      __syncthreads();
      const uint32_t pre = s_mprefix, mb = s_mmaskbits;
      for (uint32_t i = threadIdx.x; i < nm; i += blockDim.x) {
        const uint32_t m = masks ? masks[i] : i;
        if (keys[i] == T && (m & mb) == pre) atomicAdd(&hist[(m >> shift) & 255u], 1);
      }
      __syncthreads();
      if (threadIdx.x < 64) {
        int d, below, cnt;
        select_digit(hist, s_need, d, below, cnt);
        if (threadIdx.x == 0) {
          s_need -= below;
          s_mprefix = pre | ((uint32_t)d << shift);
          s_mmaskbits = mb | (255u << shift);
        }
      }
      __syncthreads();
    }
  } else if (threadIdx.x == 0) {
    s_mprefix = 0xffffffffu;  // every mask holding T
  }
  __syncthreads();
  const uint32_t Mt = s_mprefix;
  for (uint32_t i = threadIdx.x; i < nm; i += blockDim.x) {
    const uint32_t key = keys[i];
    const uint32_t m = masks ? masks[i] : i;
    if (key < T || (key == T && m <= Mt)) {
      const int pos = atomicAdd(&s_n, 1);
      if (pos < K) list[pos] = m;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) *count = min(s_n, K);
}

// Exact (FP64) selection among the top-k: most reduced feasible, smallest
// error, tie rule, lowest mask.  When no rescored mask is feasible with at
// least one reduced node, the full enumeration is enabled (gate = 1).
__global__ __launch_bounds__(1024) void k_surr_decide(const SegHdr* __restrict__ hdrs, int g, SelParams sp,
                                                      const int* __restrict__ status,
                                                      const uint32_t* __restrict__ list,
                                                      const int* __restrict__ count,
                                                      const MaskScore* __restrict__ sc, DevDecision* __restrict__ decs,
                                                      int* __restrict__ gate) {
  __shared__ double shd[16];
  __shared__ int shi[16];
  __shared__ unsigned shu[16];
  const SegHdr H = load_hdr_g(hdrs, g);
  if (!H.valid || (*status & (16 | 32))) {
    if (threadIdx.x == 0) *gate = 1;  // let the full path write its (null) decision
    return;
  }
  const int n = *count;
  int best = -1;
  for (int q = threadIdx.x; q < n; q += blockDim.x)
    if (feasible(sc[q], sp.e_bar)) best = max(best, __popc(list[q]));
  best = block_reduce(best, [](int a, int b) { return max(a, b); }, shi);
  if (best < 1) {
    if (threadIdx.x == 0) *gate = 1;
    return;
  }
  double emin = INFINITY;
  for (int q = threadIdx.x; q < n; q += blockDim.x)
    if (feasible(sc[q], sp.e_bar) && __popc(list[q]) == best) emin = fmin(emin, sc[q].e);
  emin = block_reduce(emin, [](double a, double b) { return fmin(a, b); }, shd);
  const double thr = emin + sp.tie;
  unsigned pick = 0xffffffffu;
  int amb = 0;
  double runner = INFINITY;  // among the rescored top-k
  for (int q = threadIdx.x; q < n; q += blockDim.x) {
    const MaskScore r = sc[q];
    const int pc = __popc(list[q]);
    if (pc >= best && near_boundary(r, sp.e_bar, sp.amb)) amb = 1;
    if (pc != best || !feasible(r, sp.e_bar)) continue;
    if (fabs(r.e - thr) <= sp.amb) amb = 1;
    if (r.e <= thr) pick = min(pick, list[q]);
    else runner = fmin(runner, r.e);
  }
  pick = block_reduce(pick, [](unsigned a, unsigned b) { return min(a, b); }, shu);
  amb = block_reduce(amb, [](int a, int b) { return a | b; }, shi);
  runner = block_reduce(runner, [](double a, double b) { return fmin(a, b); }, shd);
  for (int q = threadIdx.x; q < n; q += blockDim.x)  // masks in the list are distinct
    if (list[q] == pick) shd[0] = sc[q].e;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double epick = shd[0];
    DevDecision d;
    d.mask = pick;
    d.popcount = best;
    d.e_loc = epick;
    d.e_min = emin;
    d.ambiguous = amb;
    d.found = 1;
    d.key_gap = runner - emin;
    d.smice_rise = 0.0;
    decs[g] = d;
    *gate = 0;
  }
}

// ------------------------------------------------------- fused ranking --
// Ranking keys of 32 masks per block (masks[row], or mask = row), with the
// arithmetic of k_surr_features -> k_gemm_nt<1> -> k_gemm_nt<2> ->
// k_rowdot_finish -> k_surr_keys: the segment's feature tables are staged in
// LDS, the 64 feature rows, the first hidden layer (64 x 256, BF16) and the
// per-row partial products stay on chip, and both layers run on MFMA in the
// GEMM kernel's order (K in steps of 16, the same operand layouts), so the
// keys equal the unfused path's.  8 waves share the one row tile; wave w owns
// column tile w of each layer and fetches its W2 fragments before the first
// layer.
constexpr int kRankRows = 32;
constexpr int kRankThreads = 64 * (kSurrH / 32);
constexpr int kRankInts = kMaxK * kChainInts + kMaxK * kMaxK + kMaxK * kSlotInts;  // chains, nesting, slots
// LDS: H1 [32][256 + 8] BF16; the feature tables and rows.
constexpr int kRankH1 = kRankRows * (kSurrH + 8) * 2;
constexpr int kRankU = kRankInts * 4 + 2 * kMaxPairs * 4 + kMaxK * (int)sizeof(SurrSlot) + kRankRows * (kSurrF + 8) * 2;

__global__ __launch_bounds__(kRankThreads) void k_surr_rank(const SegHdr* __restrict__ hdrs, int g,
                                                   const int* __restrict__ tab, const float* __restrict__ pz,
                                                   const float* __restrict__ zs, const SurrSlot* __restrict__ ss,
                                                   const double* __restrict__ econst,
                                                   const uint32_t* __restrict__ masks, int n,
                                                   const __bf16* __restrict__ W1b, const __bf16* __restrict__ W2b,
                                                   const float* __restrict__ params, float ln_ebar,
                                                   uint32_t* __restrict__ keys, const int* __restrict__ flag,
                                                   int skip_if) {
  __shared__ __attribute__((aligned(16))) unsigned char lds_h1[kRankH1];
  __shared__ __attribute__((aligned(16))) unsigned char lds_u[kRankU];
  __shared__ float part[kSurrH / 32][kRankRows];
  __shared__ double s_ec;
  const SegHdr H = load_hdr_g(hdrs, g);
  if (!H.valid || (flag && *flag == skip_if)) return;
  const int i0 = blockIdx.x * kRankRows;
  if (i0 >= n) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  __bf16 (*H1)[kSurrH + 8] = (__bf16(*)[kSurrH + 8])lds_h1;
  int* s_int = (int*)lds_u;
  float* s_pz = (float*)(s_int + kRankInts);
  float* s_zs = s_pz + kMaxPairs;
  SurrSlot* s_ss = (SurrSlot*)(s_zs + kMaxPairs);
  __bf16 (*X)[kSurrF + 8] = (__bf16(*)[kSurrF + 8])(s_ss + kMaxK);
  const int ct = wave;
  const int arow = lane & 31, koff = 8 * (lane >> 5);
  const int bcol = ct * 32 + (lane & 31);
  // the W2 fragments of this wave's layer-2 tile, fetched first so the loads
  // overlap the features and the first layer
  bf16x8 bw[kSurrH / 16];
#pragma unroll
  for (int q = 0; q < kSurrH / 16; ++q) bw[q] = *(const bf16x8*)&W2b[(size_t)bcol * kSurrH + 16 * q + koff];
  // stage the feature tables (chains, nesting and slots: ints [0, o_pair))
  const int nint = min(H.o_pair, kRankInts);
  for (int q = tid; q < nint; q += blockDim.x) s_int[q] = tab[q];
  for (int q = tid; q < H.npairs; q += blockDim.x) {
    s_pz[q] = pz[q];
    s_zs[q] = zs[q];
  }
  for (int q = tid; q < H.nslots; q += blockDim.x) s_ss[q] = ss[q];
  if (wave == 0) {
    double ec = 0.0;
    for (int l = lane; l < H.S; l += 64) ec = fmax(ec, econst[l]);
    for (int o = 32; o > 0; o >>= 1) ec = fmax(ec, __shfl_xor(ec, o, 64));
    if (lane == 0) s_ec = ec;
  }
  __syncthreads();
  if (tid < kRankRows) {
    const int i = i0 + tid;
    const uint32_t m = (masks && i < n) ? masks[i] : (uint32_t)i;
    float f[kSurrF];
    for (int q = 0; q < kSurrF; ++q) f[q] = 0.f;
    if (i < n && m < (1u << H.k) && H.o_pair <= kRankInts)
      surr_features(H, s_int + H.o_chain, s_int + H.o_slot, s_pz, s_zs, s_ss, s_ec, m, f);
    for (int q = 0; q < kSurrF; ++q) X[tid][q] = (__bf16)f[q];
  }
  __syncthreads();
  // layer 1: H1 = gelu(X W1^T + b1), K = 32
  {
    f32x16 acc;
    for (int v = 0; v < 16; ++v) acc[v] = 0.f;
#pragma unroll
    for (int kk = 0; kk < kSurrF; kk += 16) {
      const bf16x8 a = *(const bf16x8*)&X[arow][kk + koff];
      const bf16x8 b = *(const bf16x8*)&W1b[(size_t)bcol * kSurrF + kk + koff];
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int row = 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
      H1[row][bcol] = (__bf16)gelu_f(acc[v] + params[kOffB1 + bcol]);
    }
  }
  __syncthreads();
  // layer 2: gelu(H1 W2^T + b2) . w3, K = 256
  {
    f32x16 acc;
    for (int v = 0; v < 16; ++v) acc[v] = 0.f;
#pragma unroll
    for (int q = 0; q < kSurrH / 16; ++q) {
      const bf16x8 a = *(const bf16x8*)&H1[arow][16 * q + koff];
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bw[q], acc, 0, 0, 0);
    }
    const float bias = params[kOffB2 + bcol], w3 = params[kOffW3 + bcol];
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      float sdot = gelu_f(acc[v] + bias) * w3;
      for (int o = 1; o < 32; o <<= 1) sdot += __shfl_xor(sdot, o, 64);
      const int row = 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
      if ((lane & 31) == 0) part[ct][row] = sdot;
    }
  }
  __syncthreads();
  if (tid < kRankRows && i0 + tid < n) {
    const int i = i0 + tid;
    float y = params[kOffB3];
    for (int j = 0; j < kSurrH / 32; ++j) y += part[j][tid];
    const uint32_t m = masks ? masks[i] : (uint32_t)i;
    const uint32_t pf = y <= ln_ebar ? 0u : 1u;
    const uint32_t lvl = (uint32_t)(H.k - __popc(m)) & 31u;
    keys[i] = (pf << 31) | (lvl << 26) | (ordered(y) >> 6);
  }
}

}  // namespace okr
