// Learned warm start: a message-passing network on the mesh edges that
// predicts the correction of the inertial guess for each step's first PD
// iterate.  Inference and training (forward, backward, Adam) run here.
//
// Every product of the network is a dense contraction with a 64-wide side, so
// it runs on the matrix cores: BF16 inputs, FP32 accumulation
// (v_mfma_f32_16x16x16_bf16), FP32 master weights; an FP32 build of the same
// kernels (plain FMA on the same tiles) serves as the precise reference path.
// A workgroup stages its operand tiles in LDS and each wave produces 16 x 16
// output tiles.  Sums over edges and vertices use fixed orders (edges sorted
// by destination; per-source edge lists; per-chunk partial products reduced in
// order), so training is bitwise reproducible.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <set>
#include <string>
#include <utility>
#include <vector>

#include "mpn_internal.h"

namespace pdhot {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short f2bf(float f) {
  // round to nearest even
  unsigned int u = __float_as_uint(f);
  const unsigned int lsb = (u >> 16) & 1u;
  u += 0x7FFFu + lsb;
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short b) { return __uint_as_float(((unsigned int)b) << 16); }

__device__ __forceinline__ float silu(float z) { return z / (1.0f + expf(-z)); }
__device__ __forceinline__ float dsilu(float z) {
  const float s = 1.0f / (1.0f + expf(-z));
  return s * (1.0f + z * (1.0f - s));
}

// LDS operand element: BF16 (stored as ushort) or FP32.
template <bool BF>
struct Lds;
template <>
struct Lds<true> {
  typedef unsigned short T;
  __device__ static T put(float f) { return f2bf(f); }
};
template <>
struct Lds<false> {
  typedef float T;
  __device__ static T put(float f) { return f; }
};

// One 16 x 16 output tile of a wave: acc += A(16 x K) B(K x 16).
// A(i, k) = a[i * sa_i + k * sa_k], B(k, n) = b[k * sb_k + n * sb_n] in LDS.
// Lane l owns D(4 (l / 16) + r, l % 16), r = 0..3 (the matrix-core layout);
// the FP32 path computes the same four entries with FMAs.
template <bool BF>
__device__ __forceinline__ void tile16(f32x4& acc, const typename Lds<BF>::T* a, int sa_i, int sa_k,
                                       const typename Lds<BF>::T* b, int sb_k, int sb_n, int K) {
  const int l = threadIdx.x & 63;
  const int i = l & 15, g = l >> 4;
  if constexpr (BF) {
    for (int k0 = 0; k0 < K; k0 += 16) {
      bf16x4 av, bv;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int k = k0 + 4 * g + j;
        av[j] = (short)a[i * sa_i + k * sa_k];
        bv[j] = (short)b[k * sb_k + i * sb_n];
      }
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc, 0, 0, 0);
    }
  } else {
#pragma unroll 2
    for (int k = 0; k < K; ++k) {
      const float bk = b[k * sb_k + i * sb_n];
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[r] += a[(4 * g + r) * sa_i + k * sa_k] * bk;
    }
  }
}

// ---------------------------------------------------------------- node features
__global__ void __launch_bounds__(256) k_mpn_feat(MpnArgs M, const double* __restrict__ qt, const double* __restrict__ vtm,
                                                  const double* __restrict__ vt, const double* __restrict__ f,
                                                  const double* __restrict__ logw) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M.nv) return;
  float* x = M.x0 + (size_t)i * kMpnF;
  const double il = 1.0 / M.ell;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double q = qt[3 * i + a], X = M.X[3 * i + a];
    x[a] = (float)((q - X) * il);
    x[3 + a] = (float)(M.h * (vt[3 * i + a] - vtm[3 * i + a]) / M.s_out);
    x[6 + a] = (float)(M.h * vt[3 * i + a] * il);
    x[9 + a] = (float)((f ? M.h * M.h * f[3 * i + a] / M.mass[i] : 0.0) / M.s_out);
    x[12 + a] = (float)((X - M.Xmin[a]) / M.L);
  }
  x[15] = (float)logw[i];
}

// ---------------------------------------------------------------- row providers
// Row r of each layer's input: the encoder's features (K = 16), a message's
// [h_dst, h_src, (q_src - q_dst)/ell, (X_src - X_dst)/ell] (K = 2H + 6), a node
// update's [h, a] (K = 2H).
enum { kEnc = 0, kMsg = 1, kNode = 2 };

template <int KIND>
__device__ __forceinline__ float row_val(const MpnArgs& M, const float* __restrict__ hin, int r, int k) {
  if (KIND == kEnc) return M.x0[(size_t)r * kMpnF + k];
  if (KIND == kNode) return k < kMpnH ? hin[(size_t)r * kMpnH + k] : M.agg[(size_t)r * kMpnH + (k - kMpnH)];
  const int i = M.dst[r], j = M.src[r];
  if (k < kMpnH) return hin[(size_t)i * kMpnH + k];
  if (k < 2 * kMpnH) return hin[(size_t)j * kMpnH + (k - kMpnH)];
  if (k < 2 * kMpnH + 3) {
    const int a = k - 2 * kMpnH;
    return (float)((M.qt[3 * j + a] - M.qt[3 * i + a]) / M.ell);
  }
  if (k < 2 * kMpnH + 6) {
    const int a = k - 2 * kMpnH - 3;
    return (float)((M.X[3 * j + a] - M.X[3 * i + a]) / M.ell);
  }
  return 0.0f;
}

template <int KIND>
constexpr int kin() { return KIND == kEnc ? kMpnF : (KIND == kMsg ? kMpnKM : 2 * kMpnH); }
template <int KIND>
constexpr int kpad() { return (kin<KIND>() + 15) / 16 * 16; }
// stages of 64 rows per weight-gradient workgroup: per-vertex layers (a few
// thousand rows) use one, so they spread over more workgroups; the per-edge
// layer uses two
template <int KIND>
constexpr int wstages() { return KIND == kMsg ? 2 : 1; }

// ---------------------------------------------------------------- forward layer
// Z = A W + b for 64 rows per workgroup; epilogue by kind:
//   encoder: z0, h0 = silu(z0); message: zm; node: zn, h_out = h_in + silu(zn).
template <bool BF, int KIND>
__global__ void __launch_bounds__(256) k_mpn_fwd(MpnArgs M, const float* __restrict__ W, const float* __restrict__ b,
                                                 const float* __restrict__ hin, float* __restrict__ zout,
                                                 float* __restrict__ hout, int rows) {
  typedef typename Lds<BF>::T T;
  constexpr int K = kin<KIND>(), KP = kpad<KIND>();
  __shared__ T sW[KP * kMpnH];
  __shared__ T sA[64 * KP];
  const int r0 = blockIdx.x * 64;
  for (int e = threadIdx.x; e < KP * kMpnH; e += blockDim.x) {
    const int k = e / kMpnH;
    sW[e] = Lds<BF>::put(k < K ? W[e] : 0.0f);
  }
  for (int e = threadIdx.x; e < 64 * KP; e += blockDim.x) {
    const int rr = e / KP, k = e % KP, r = r0 + rr;
    sA[e] = Lds<BF>::put((r < rows && k < K) ? row_val<KIND>(M, hin, r, k) : 0.0f);
  }
  __syncthreads();
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    tile16<BF>(acc, sA + (16 * w) * KP, KP, 1, sW + 16 * nt, kMpnH, 1, KP);
    const int col = 16 * nt + (l & 15);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = r0 + 16 * w + 4 * (l >> 4) + q;
      if (r >= rows) continue;
      const float z = acc[q] + b[col];
      const size_t o = (size_t)r * kMpnH + col;
      zout[o] = z;
      if (KIND == kEnc) hout[o] = silu(z);
      if (KIND == kNode) hout[o] = hin[o] + silu(z);
    }
  }
}

// a_i = sum over the in-edges of i of silu(zm) (edges sorted by destination)
__global__ void __launch_bounds__(256) k_mpn_agg(MpnArgs M, const float* __restrict__ zm) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = t / kMpnH, c = t % kMpnH;
  if (i >= M.nv) return;
  float s = 0.0f;
  for (int e = M.in_ptr[i]; e < M.in_ptr[i + 1]; ++e) s += silu(zm[(size_t)e * kMpnH + c]);
  M.agg[(size_t)i * kMpnH + c] = s;
}

// y = h W_dec + b_dec; q0 = q_t + h v_t + s_out y on free vertices (q_t on
// pinned).  With a target q_{t+h}: the residual r = y - (q_{t+h} - q_t - h v_t)/s_out
// on free vertices (zero on pinned), kept for the loss kernel.
__global__ void __launch_bounds__(256) k_mpn_dec(MpnArgs M, const float* __restrict__ hL, const float* __restrict__ Wd,
                                                 const float* __restrict__ bd, const double* __restrict__ vt,
                                                 const double* __restrict__ target, double* __restrict__ q0,
                                                 double* __restrict__ res) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M.nv) return;
  float y[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    float s = bd[c];
    for (int k = 0; k < kMpnH; ++k) s += hL[(size_t)i * kMpnH + k] * Wd[k * 3 + c];
    y[c] = s;
  }
  const bool fr = !M.pinned[i];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if (q0) q0[3 * i + c] = fr ? M.qt[3 * i + c] + M.h * vt[3 * i + c] + M.s_out * (double)y[c] : M.qt[3 * i + c];
    if (target) {
      const double ys = (target[3 * i + c] - M.qt[3 * i + c] - M.h * vt[3 * i + c]) / M.s_out;
      res[3 * i + c] = fr ? ((double)y[c] - ys) : 0.0;
    }
  }
}

// Training loss L = sum_free |r|^2 / (3 n_free) + kappa sum over directed edges
// |r_src - r_dst|^2 / (3 n_edges) (the second term weighs the correction's
// differences along edges, i.e. the strain it implies), its gradient dL/dy
// (zero on pinned vertices; both directions of an edge are listed, so
// dL_edge/dr_i = -4 kappa / (3 n_edges) sum_j (r_j - r_i) over i's in-edges)
// and the per-block partial loss.
__global__ void __launch_bounds__(256) k_mpn_loss(MpnArgs M, const double* __restrict__ res, float* __restrict__ dy,
                                                  double* __restrict__ lpart) {
  __shared__ double red[256];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double lsum = 0.0;
  if (i < M.nv) {
    const double cp = 1.0 / (3.0 * M.n_free), ce = M.kappa / (3.0 * M.ne);
    double ri[3], g[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      ri[c] = res[3 * i + c];
      lsum += cp * ri[c] * ri[c];
      g[c] = 2.0 * cp * ri[c];
    }
    if (M.kappa > 0.0)
      for (int e = M.in_ptr[i]; e < M.in_ptr[i + 1]; ++e) {
        const int j = M.src[e];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const double d = res[3 * j + c] - ri[c];
          lsum += ce * d * d;
          g[c] -= 4.0 * ce * d;
        }
      }
    const bool fr = !M.pinned[i];
#pragma unroll
    for (int c = 0; c < 3; ++c) dy[(size_t)i * 3 + c] = fr ? (float)g[c] : 0.0f;
  }
  red[threadIdx.x] = lsum;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) lpart[blockIdx.x] = red[0];
}

// ---------------------------------------------------------------- backward
// decoder: dh_L = dy W_dec^T; partial sums of dW_dec = h_L^T dy and db_dec per block
__global__ void __launch_bounds__(256) k_mpn_dec_bwd(MpnArgs M, const float* __restrict__ hL, const float* __restrict__ Wd,
                                                     const float* __restrict__ dy, float* __restrict__ dh,
                                                     float* __restrict__ part) {
  __shared__ float sdy[4 * 3];
  __shared__ float shl[4 * kMpnH];
  const int i0 = blockIdx.x * 4;
  const int t = threadIdx.x;
  // 4 vertices per block, one thread per (vertex, hidden unit)
  const int li = t / kMpnH, k = t % kMpnH, i = i0 + li;
  if (t < 12) sdy[t] = (i0 + t / 3 < M.nv) ? dy[(size_t)(i0 + t / 3) * 3 + t % 3] : 0.0f;
  shl[t] = (i < M.nv) ? hL[(size_t)i * kMpnH + k] : 0.0f;
  __syncthreads();
  if (i < M.nv) {
    float s = 0.0f;
#pragma unroll
    for (int c = 0; c < 3; ++c) s += sdy[li * 3 + c] * Wd[k * 3 + c];
    dh[(size_t)i * kMpnH + k] = s;
  }
  // dW_dec[k][c] and db_dec[c] partials of this block's 4 vertices
  if (t < kMpnH * 3 + 3) {
    float s = 0.0f;
    if (t < kMpnH * 3) {
      const int kk = t / 3, c = t % 3;
      for (int v = 0; v < 4; ++v) s += shl[v * kMpnH + kk] * sdy[v * 3 + c];
    } else {
      const int c = t - kMpnH * 3;
      for (int v = 0; v < 4; ++v) s += sdy[v * 3 + c];
    }
    part[(size_t)blockIdx.x * (kMpnH * 3 + 3) + t] = s;
  }
}

// Input gradient of a layer for 64 rows per workgroup.
//  node:    dzn = dh ⊙ silu'(zn); [dh_in, da] = dzn W_node^T; dh_in += dh (residual)
//  message: dzm = da[dst] ⊙ silu'(zm) (stored for the weight gradient);
//           dein[:, 0:2H] = dzm W_msg^T[:, 0:2H] (stored, scattered by k_mpn_scatter)
//  encoder: none (the inputs are data)
template <bool BF, int KIND>
__global__ void __launch_bounds__(256) k_mpn_bwd_in(MpnArgs M, const float* __restrict__ W, const float* __restrict__ z,
                                                    const float* __restrict__ dh, float* __restrict__ dz,
                                                    float* __restrict__ out, int rows) {
  typedef typename Lds<BF>::T T;
  constexpr int NO = 2 * kMpnH;  // output columns kept: [h, a] or [h_dst, h_src]
  __shared__ T sW[NO * kMpnH];   // W[k][n] for k < 2H, row-major
  __shared__ T sG[64 * kMpnH];   // dz rows
  const int r0 = blockIdx.x * 64;
  for (int e = threadIdx.x; e < NO * kMpnH; e += blockDim.x) sW[e] = Lds<BF>::put(W[e]);
  for (int e = threadIdx.x; e < 64 * kMpnH; e += blockDim.x) {
    const int rr = e / kMpnH, c = e % kMpnH, r = r0 + rr;
    float g = 0.0f;
    if (r < rows) {
      const size_t o = (size_t)r * kMpnH + c;
      const float up = (KIND == kNode) ? dh[o] : M.dagg[(size_t)M.dst[r] * kMpnH + c];
      g = up * dsilu(z[o]);
      dz[o] = g;
    }
    sG[e] = Lds<BF>::put(g);
  }
  __syncthreads();
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  for (int ct = 0; ct < NO / 16; ++ct) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    // D(r, k) = sum_n dz(r, n) W(k, n): B(n, k) = W[k][n] = sW[k * H + n]
    tile16<BF>(acc, sG + (16 * w) * kMpnH, kMpnH, 1, sW + 16 * ct * kMpnH, 1, kMpnH, kMpnH);
    const int col = 16 * ct + (l & 15);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = r0 + 16 * w + 4 * (l >> 4) + q;
      if (r >= rows) continue;
      if (KIND == kNode) {
        if (col < kMpnH) out[(size_t)r * kMpnH + col] = dh[(size_t)r * kMpnH + col] + acc[q];
        else M.dagg[(size_t)r * kMpnH + (col - kMpnH)] = acc[q];
      } else {
        out[(size_t)r * NO + col] = acc[q];
      }
    }
  }
}

// dh[i] += sum over in-edges of dein[:, 0:H] + sum over out-edges of dein[:, H:2H]
__global__ void __launch_bounds__(256) k_mpn_scatter(MpnArgs M, const float* __restrict__ dein, float* __restrict__ dh) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = t / kMpnH, c = t % kMpnH;
  if (i >= M.nv) return;
  float s = dh[(size_t)i * kMpnH + c];
  for (int e = M.in_ptr[i]; e < M.in_ptr[i + 1]; ++e) s += dein[(size_t)e * 2 * kMpnH + c];
  for (int p = M.out_ptr[i]; p < M.out_ptr[i + 1]; ++p) s += dein[(size_t)M.out_eid[p] * 2 * kMpnH + kMpnH + c];
  dh[(size_t)i * kMpnH + c] = s;
}

// Weight gradient partials: dW(k, n) = sum_r A(r, k) dz(r, n), db(n) = sum_r dz(r, n),
// over 64 wstages rows per workgroup (stages of 64), written to part[blk].
template <bool BF, int KIND>
__global__ void __launch_bounds__(256) k_mpn_wgrad(MpnArgs M, const float* __restrict__ hin, const float* __restrict__ dz,
                                                   float* __restrict__ part, int rows) {
  typedef typename Lds<BF>::T T;
  constexpr int K = kin<KIND>(), KP = kpad<KIND>();
  constexpr int NT = (KP / 16) * 4;  // output tiles
  __shared__ T sA[64 * KP];
  __shared__ T sG[64 * kMpnH];
  __shared__ float sb[4][kMpnH];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  f32x4 acc[(NT + 3) / 4];
#pragma unroll
  for (int j = 0; j < (NT + 3) / 4; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
  float bsum = 0.0f;  // thread c < 64: db partial of column c
  constexpr int NS = wstages<KIND>();
  for (int st = 0; st < NS; ++st) {
    const int r0 = blockIdx.x * (64 * NS) + st * 64;
    __syncthreads();
    for (int e = threadIdx.x; e < 64 * KP; e += blockDim.x) {
      const int rr = e / KP, k = e % KP, r = r0 + rr;
      sA[e] = Lds<BF>::put((r < rows && k < K) ? row_val<KIND>(M, hin, r, k) : 0.0f);
    }
    for (int e = threadIdx.x; e < 64 * kMpnH; e += blockDim.x) {
      const int rr = e / kMpnH, r = r0 + rr;
      sG[e] = Lds<BF>::put(r < rows ? dz[(size_t)r * kMpnH + (e % kMpnH)] : 0.0f);
    }
    __syncthreads();
    if (threadIdx.x < kMpnH) {
      for (int rr = 0; rr < 64; ++rr) {
        const int r = r0 + rr;
        if (r < rows) bsum += dz[(size_t)r * kMpnH + threadIdx.x];
      }
    }
#pragma unroll
    for (int j = 0; j < (NT + 3) / 4; ++j) {
      const int tile = w + 4 * j;
      if (tile < NT) {
        const int kt = tile / 4, nt = tile % 4;
        // D(k, n) = sum_r A(r, k) dz(r, n): A-operand(i = k, kk = r) = sA[r * KP + k]
        tile16<BF>(acc[j], sA + 16 * kt, 1, KP, sG + 16 * nt, kMpnH, 1, 64);
      }
    }
  }
  float* o = part + (size_t)blockIdx.x * (K * kMpnH + kMpnH);
#pragma unroll
  for (int j = 0; j < (NT + 3) / 4; ++j) {
    const int tile = w + 4 * j;
    if (tile < NT) {
      const int kt = tile / 4, nt = tile % 4;
      const int n = 16 * nt + (l & 15);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int k = 16 * kt + 4 * (l >> 4) + q;
        if (k < K) o[k * kMpnH + n] = acc[j][q];
      }
    }
  }
  if (threadIdx.x < kMpnH) o[K * kMpnH + threadIdx.x] = bsum;
  (void)sb;
}

// encoder: dz0 = dh0 ⊙ silu'(z0)
__global__ void __launch_bounds__(256) k_mpn_enc_dz(MpnArgs M, const float* __restrict__ z0, const float* __restrict__ dh,
                                                    float* __restrict__ dz) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= M.nv * kMpnH) return;
  dz[t] = dh[t] * dsilu(z0[t]);
}

// g[e] = sum over the partial rows part[b][e] in a fixed order: each of 8
// threads of an output sums the rows b = t, t + 8, t + 16, ... in order, then
// the 8 sums are added in t order (deterministic; 32 outputs per block, the
// threads of one t read consecutive outputs).
constexpr int kRedSplit = 8;
__global__ void __launch_bounds__(256) k_mpn_reduce(const float* __restrict__ part, int nblk, int width,
                                                    float* __restrict__ g) {
  __shared__ float acc[kRedSplit][32];
  const int el = threadIdx.x & 31, t = threadIdx.x >> 5;
  const int e = blockIdx.x * 32 + el;
  float s = 0.0f;
  if (e < width) {
#pragma unroll 4
    for (int b = t; b < nblk; b += kRedSplit) s += part[(size_t)b * width + e];
  }
  acc[t][el] = s;
  __syncthreads();
  if (t == 0 && e < width) {
    float r = acc[0][el];
#pragma unroll
    for (int k = 1; k < kRedSplit; ++k) r += acc[k][el];
    g[e] = r;
  }
}

// Adam on the FP32 master weights (bias-corrected), then the BF16 copy.
__global__ void __launch_bounds__(256) k_mpn_adam(float* __restrict__ p, const float* __restrict__ g,
                                                  float* __restrict__ m, float* __restrict__ v, int n, float lr,
                                                  float b1, float b2, float eps, float c1, float c2) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const float gg = g[e];
  const float mm = b1 * m[e] + (1.0f - b1) * gg;
  const float vv = b2 * v[e] + (1.0f - b2) * gg * gg;
  m[e] = mm;
  v[e] = vv;
  p[e] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

// ================================================================= host side
namespace {


#define MPN_HIP(x)                                                                    \
  do {                                                                                \
    hipError_t e_ = (x);                                                              \
    if (e_ != hipSuccess) throw MpnError{PD_ERR_HIP, std::string("HIP: ") + hipGetErrorString(e_)}; \
  } while (0)

struct MpnError {
  int code;
  std::string msg;
};

template <typename T>
T* dalloc(size_t n) {
  T* p = nullptr;
  MPN_HIP(hipMalloc((void**)&p, std::max<size_t>(1, n) * sizeof(T)));
  return p;
}
template <typename T>
void upload(T* d, const std::vector<T>& h) {
  if (!h.empty()) MPN_HIP(hipMemcpy(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
}
template <typename T>
void dfree(T*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

// parameter offsets in the flat vector
struct POff {
  size_t We, be, Wm[kMpnLayers], bm[kMpnLayers], Wn[kMpnLayers], bn[kMpnLayers], Wd, bd, n;
};
POff param_offsets() {
  POff o;
  size_t c = 0;
  o.We = c; c += kMpnF * kMpnH;
  o.be = c; c += kMpnH;
  for (int l = 0; l < kMpnLayers; ++l) {
    o.Wm[l] = c; c += (size_t)kMpnKM * kMpnH;
    o.bm[l] = c; c += kMpnH;
    o.Wn[l] = c; c += (size_t)2 * kMpnH * kMpnH;
    o.bn[l] = c; c += kMpnH;
  }
  o.Wd = c; c += kMpnH * 3;
  o.bd = c; c += 3;
  o.n = c;
  return o;
}

}  // namespace

struct MpnImpl {
  MpnArgs A{};
  int compute = 0;  // 0 BF16 matrix cores, 1 FP32
  int ne = 0;
  POff off{};
  float *P = nullptr, *G = nullptr, *Mo = nullptr, *Vo = nullptr;
  float* hbuf[kMpnLayers + 1] = {};
  float* zm[kMpnLayers] = {};
  float* zn[kMpnLayers] = {};
  float* aggl[kMpnLayers] = {};  // aggregated messages of each layer (kept for the backward pass)
  float* z0 = nullptr;
  float *dh = nullptr, *dh2 = nullptr, *dz = nullptr, *dein = nullptr, *dy = nullptr, *part = nullptr;
  double* lpart = nullptr;
  double* res = nullptr;
  double* hl = nullptr;
  size_t part_cap = 0;
  long long step = 0;
  std::vector<int> hpinned;
  bool shared = false;  // P, G, Mo, Vo belong to another instance (pd_mpn_share_params)
};

static int mpn_grid_rows(int rows, int per) { return (rows + per - 1) / per; }

static void mpn_forward(MpnImpl& N, const double* qt, const double* vtm, const double* vt, const double* f,
                        const double* logw, hipStream_t s) {
  MpnArgs& A = N.A;
  A.qt = qt;
  hipLaunchKernelGGL(k_mpn_feat, dim3(mpn_grid_rows(A.nv, 256)), dim3(256), 0, s, A, qt, vtm, vt, f, logw);
  const POff& o = N.off;
  const dim3 b(256);
#define FWD(BF, KIND, W, B, HIN, Z, HOUT, ROWS)                                                        \
  hipLaunchKernelGGL((k_mpn_fwd<BF, KIND>), dim3(mpn_grid_rows(ROWS, 64)), b, 0, s, A, N.P + (W), N.P + (B), \
                     HIN, Z, HOUT, ROWS)
  if (N.compute == 0) FWD(true, kEnc, o.We, o.be, nullptr, N.z0, N.hbuf[0], A.nv);
  else FWD(false, kEnc, o.We, o.be, nullptr, N.z0, N.hbuf[0], A.nv);
  for (int l = 0; l < kMpnLayers; ++l) {
    if (N.compute == 0) FWD(true, kMsg, o.Wm[l], o.bm[l], N.hbuf[l], N.zm[l], nullptr, N.ne);
    else FWD(false, kMsg, o.Wm[l], o.bm[l], N.hbuf[l], N.zm[l], nullptr, N.ne);
    A.agg = N.aggl[l];
    hipLaunchKernelGGL(k_mpn_agg, dim3(mpn_grid_rows(A.nv * kMpnH, 256)), b, 0, s, A, N.zm[l]);
    if (N.compute == 0) FWD(true, kNode, o.Wn[l], o.bn[l], N.hbuf[l], N.zn[l], N.hbuf[l + 1], A.nv);
    else FWD(false, kNode, o.Wn[l], o.bn[l], N.hbuf[l], N.zn[l], N.hbuf[l + 1], A.nv);
  }
#undef FWD
}

template <bool BF, int KIND>
static void mpn_wgrad(MpnImpl& N, const float* hin, const float* dz, int rows, size_t woff, size_t boff,
                      hipStream_t s) {
  constexpr int K = kin<KIND>();
  const int nblk = mpn_grid_rows(rows, 64 * wstages<KIND>());
  const int width = K * kMpnH + kMpnH;
  hipLaunchKernelGGL((k_mpn_wgrad<BF, KIND>), dim3(nblk), dim3(256), 0, s, N.A, hin, dz, N.part, rows);
  // the weight block and the bias block are contiguous in the partial rows but not in P:
  // reduce into G at the weight offset, and the bias columns follow it (b directly after W)
  hipLaunchKernelGGL(k_mpn_reduce, dim3(mpn_grid_rows(width, 32)), dim3(256), 0, s, N.part, nblk, width,
                     N.G + woff);
  (void)boff;
}

static void mpn_backward(MpnImpl& N, hipStream_t s) {
  MpnArgs& A = N.A;
  const POff& o = N.off;
  const dim3 b(256);
  const int nv = A.nv, ne = N.ne;
  const int ndb = mpn_grid_rows(nv, 4);
  hipLaunchKernelGGL(k_mpn_dec_bwd, dim3(ndb), b, 0, s, A, N.hbuf[kMpnLayers], N.P + o.Wd, N.dy, N.dh, N.part);
  hipLaunchKernelGGL(k_mpn_reduce, dim3(mpn_grid_rows(kMpnH * 3 + 3, 32)), b, 0, s, N.part, ndb, kMpnH * 3 + 3,
                     N.G + o.Wd);
  for (int l = kMpnLayers - 1; l >= 0; --l) {
    A.agg = N.aggl[l];  // the node update's input [h_l, a_l]
    // node update: dzn, [dh_prev, da]
    if (N.compute == 0) {
      hipLaunchKernelGGL((k_mpn_bwd_in<true, kNode>), dim3(mpn_grid_rows(nv, 64)), b, 0, s, A, N.P + o.Wn[l], N.zn[l],
                         N.dh, N.dz, N.dh2, nv);
      mpn_wgrad<true, kNode>(N, N.hbuf[l], N.dz, nv, o.Wn[l], o.bn[l], s);
      hipLaunchKernelGGL((k_mpn_bwd_in<true, kMsg>), dim3(mpn_grid_rows(ne, 64)), b, 0, s, A, N.P + o.Wm[l], N.zm[l],
                         nullptr, N.dz, N.dein, ne);
      mpn_wgrad<true, kMsg>(N, N.hbuf[l], N.dz, ne, o.Wm[l], o.bm[l], s);
    } else {
      hipLaunchKernelGGL((k_mpn_bwd_in<false, kNode>), dim3(mpn_grid_rows(nv, 64)), b, 0, s, A, N.P + o.Wn[l],
                         N.zn[l], N.dh, N.dz, N.dh2, nv);
      mpn_wgrad<false, kNode>(N, N.hbuf[l], N.dz, nv, o.Wn[l], o.bn[l], s);
      hipLaunchKernelGGL((k_mpn_bwd_in<false, kMsg>), dim3(mpn_grid_rows(ne, 64)), b, 0, s, A, N.P + o.Wm[l],
                         N.zm[l], nullptr, N.dz, N.dein, ne);
      mpn_wgrad<false, kMsg>(N, N.hbuf[l], N.dz, ne, o.Wm[l], o.bm[l], s);
    }
    hipLaunchKernelGGL(k_mpn_scatter, dim3(mpn_grid_rows(nv * kMpnH, 256)), b, 0, s, A, N.dein, N.dh2);
    std::swap(N.dh, N.dh2);
  }
  // encoder: dz0 = dh0 ⊙ silu'(z0), then its weight gradient
  hipLaunchKernelGGL(k_mpn_enc_dz, dim3(mpn_grid_rows(nv * kMpnH, 256)), b, 0, s, A, N.z0, N.dh, N.dz);
  if (N.compute == 0) mpn_wgrad<true, kEnc>(N, nullptr, N.dz, nv, o.We, o.be, s);
  else mpn_wgrad<false, kEnc>(N, nullptr, N.dz, nv, o.We, o.be, s);
}

}  // namespace pdhot

// ================================================================= C ABI
using namespace pdhot;

struct pd_mpn {
  MpnImpl N;
};

namespace {

#define MPN_TRY try {
#define MPN_CATCH                        \
  }                                      \
  catch (const MpnError& e) {            \
    set_last_error(e.msg);                   \
    return e.code;                       \
  }                                      \
  catch (const std::bad_alloc&) {        \
    set_last_error("host allocation failed"); \
    return PD_ERR_ALLOC;                 \
  }

void mpn_free(MpnImpl& N) {
  MpnArgs& A = N.A;
  dfree(const_cast<double*&>(A.X)); dfree(const_cast<double*&>(A.mass)); dfree(const_cast<uint8_t*&>(A.pinned));
  dfree(const_cast<int*&>(A.src)); dfree(const_cast<int*&>(A.dst)); dfree(const_cast<int*&>(A.in_ptr));
  dfree(const_cast<int*&>(A.out_ptr)); dfree(const_cast<int*&>(A.out_eid));
  dfree(A.x0); dfree(A.dagg);
  A.agg = nullptr;
  if (N.shared) N.P = N.G = N.Mo = N.Vo = nullptr;
  dfree(N.P); dfree(N.G); dfree(N.Mo); dfree(N.Vo);
  for (int l = 0; l <= kMpnLayers; ++l) dfree(N.hbuf[l]);
  for (int l = 0; l < kMpnLayers; ++l) { dfree(N.zm[l]); dfree(N.zn[l]); dfree(N.aggl[l]); }
  dfree(N.z0); dfree(N.dh); dfree(N.dh2); dfree(N.dz); dfree(N.dein); dfree(N.dy); dfree(N.part); dfree(N.lpart); dfree(N.res);
  if (N.hl) (void)hipHostFree(N.hl);
  N.hl = nullptr;
}

// splitmix64: the library's own seeded initialisation of the weights
uint64_t splitmix(uint64_t& x) {
  uint64_t z = (x += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

}  // namespace

extern "C" {

int pd_mpn_create(const pd_mesh_desc* mesh, const pd_mpn_desc* desc, pd_mpn** out) {
  if (!mesh || !desc || !out || mesh->n_verts <= 0 || mesh->n_tets <= 0 || !mesh->rest_xyz || !mesh->tets ||
      !mesh->pinned || !(desc->h > 0.0) || !(desc->rho > 0.0) || desc->compute < 0 || desc->compute > 1 ||
      !(desc->edge_weight >= 0.0)) {
    set_last_error("invalid argument");
    return PD_ERR_INVALID_ARG;
  }
  MPN_TRY
  pd_mpn* m = new pd_mpn();
  MpnImpl& N = m->N;
  try {
    const int nv = mesh->n_verts, nt = mesh->n_tets;
    const double* X = mesh->rest_xyz;
    // directed edges of the tets, both directions, sorted by (destination, source)
    std::set<std::pair<int, int>> es;  // (dst, src)
    std::vector<double> mass(nv, 0.0);
    for (int e = 0; e < nt; ++e) {
      const int* t = mesh->tets + 4 * (size_t)e;
      for (int a = 0; a < 4; ++a) {
        if (t[a] < 0 || t[a] >= nv) throw MpnError{PD_ERR_INVALID_ARG, "tet vertex index out of range"};
        for (int b = 0; b < 4; ++b)
          if (a != b) es.insert({t[a], t[b]});
      }
      double D[9];
      for (int a = 1; a < 4; ++a)
        for (int i = 0; i < 3; ++i) D[3 * i + a - 1] = X[3 * t[a] + i] - X[3 * t[0] + i];
      const double det = D[0] * (D[4] * D[8] - D[5] * D[7]) - D[1] * (D[3] * D[8] - D[5] * D[6]) +
                         D[2] * (D[3] * D[7] - D[4] * D[6]);
      for (int a = 0; a < 4; ++a) mass[t[a]] += desc->rho * std::fabs(det) / 6.0 / 4.0;
    }
    const int ne = (int)es.size();
    std::vector<int> src, dst, in_ptr(nv + 1, 0), out_ptr(nv + 1, 0), out_eid(ne);
    src.reserve(ne);
    dst.reserve(ne);
    double len = 0.0;
    for (const auto& p : es) {
      dst.push_back(p.first);
      src.push_back(p.second);
      in_ptr[p.first + 1]++;
      out_ptr[p.second + 1]++;
      double d2 = 0.0;
      for (int a = 0; a < 3; ++a) d2 += (X[3 * p.second + a] - X[3 * p.first + a]) * (X[3 * p.second + a] - X[3 * p.first + a]);
      len += std::sqrt(d2);
    }
    for (int i = 0; i < nv; ++i) {
      in_ptr[i + 1] += in_ptr[i];
      out_ptr[i + 1] += out_ptr[i];
    }
    std::vector<int> fill(out_ptr.begin(), out_ptr.end() - 1);
    for (int e = 0; e < ne; ++e) out_eid[fill[src[e]]++] = e;
    MpnArgs& A = N.A;
    A.nv = nv;
    A.n_free = 0;
    for (int i = 0; i < nv; ++i) A.n_free += mesh->pinned[i] ? 0 : 1;
    if (A.n_free == 0) throw MpnError{PD_ERR_INVALID_ARG, "no free vertex"};
    A.ell = len / std::max(1, ne);
    double lo[3], hi[3];
    for (int a = 0; a < 3; ++a) lo[a] = hi[a] = X[a];
    for (int i = 0; i < nv; ++i)
      for (int a = 0; a < 3; ++a) {
        lo[a] = std::min(lo[a], X[3 * i + a]);
        hi[a] = std::max(hi[a], X[3 * i + a]);
      }
    A.L = std::max(hi[0] - lo[0], std::max(hi[1] - lo[1], hi[2] - lo[2]));
    for (int a = 0; a < 3; ++a) A.Xmin[a] = lo[a];
    A.h = desc->h;
    A.s_out = 1.0;
    A.kappa = desc->edge_weight;
    A.ne = ne;
    N.compute = desc->compute;
    N.ne = ne;
    N.off = param_offsets();
    std::vector<double> Xv(X, X + 3 * (size_t)nv);
    std::vector<uint8_t> pin(mesh->pinned, mesh->pinned + nv);
    double* dX = dalloc<double>(Xv.size()); upload(dX, Xv); A.X = dX;
    double* dm = dalloc<double>(nv); upload(dm, mass); A.mass = dm;
    uint8_t* dp = dalloc<uint8_t>(nv); upload(dp, pin); A.pinned = dp;
    int* p;
    p = dalloc<int>(ne); upload(p, src); A.src = p;
    p = dalloc<int>(ne); upload(p, dst); A.dst = p;
    p = dalloc<int>(nv + 1); upload(p, in_ptr); A.in_ptr = p;
    p = dalloc<int>(nv + 1); upload(p, out_ptr); A.out_ptr = p;
    p = dalloc<int>(ne); upload(p, out_eid); A.out_eid = p;
    A.x0 = dalloc<float>((size_t)nv * kMpnF);
    A.agg = nullptr;  // points at the current layer's aggl
    A.dagg = dalloc<float>((size_t)nv * kMpnH);
    const size_t np = N.off.n;
    N.P = dalloc<float>(np); N.G = dalloc<float>(np); N.Mo = dalloc<float>(np); N.Vo = dalloc<float>(np);
    MPN_HIP(hipMemset(N.G, 0, np * sizeof(float)));
    MPN_HIP(hipMemset(N.Mo, 0, np * sizeof(float)));
    MPN_HIP(hipMemset(N.Vo, 0, np * sizeof(float)));
    for (int l = 0; l <= kMpnLayers; ++l) N.hbuf[l] = dalloc<float>((size_t)nv * kMpnH);
    for (int l = 0; l < kMpnLayers; ++l) {
      N.zm[l] = dalloc<float>((size_t)ne * kMpnH);
      N.zn[l] = dalloc<float>((size_t)nv * kMpnH);
      N.aggl[l] = dalloc<float>((size_t)nv * kMpnH);
    }
    const size_t rows = std::max(nv, ne);
    N.z0 = dalloc<float>((size_t)nv * kMpnH);
    N.dh = dalloc<float>((size_t)nv * kMpnH);
    N.dh2 = dalloc<float>((size_t)nv * kMpnH);
    N.dz = dalloc<float>(rows * kMpnH);
    N.dein = dalloc<float>((size_t)ne * 2 * kMpnH);
    N.dy = dalloc<float>((size_t)nv * 3);
    N.res = dalloc<double>((size_t)nv * 3);
    // weight-gradient partials: the widest layer over the most chunks
    const size_t chunks = (rows + 63) / 64 + (nv + 3) / 4;
    N.part_cap = chunks * (size_t)(kMpnKM * kMpnH + kMpnH);
    N.part = dalloc<float>(N.part_cap);
    N.lpart = dalloc<double>((nv + 255) / 256);
    MPN_HIP(hipHostMalloc((void**)&N.hl, sizeof(double) * ((nv + 255) / 256)));
  } catch (...) {
    mpn_free(N);
    delete m;
    throw;
  }
  *out = m;
  return PD_OK;
  MPN_CATCH
}

int pd_mpn_destroy(pd_mpn* m) {
  if (!m) return PD_OK;
  mpn_free(m->N);
  delete m;
  return PD_OK;
}

int pd_mpn_info(const pd_mpn* m, double* info) {
  if (!m || !info) {
    set_last_error("null argument");
    return PD_ERR_INVALID_ARG;
  }
  const MpnImpl& N = m->N;
  info[0] = N.A.nv; info[1] = N.ne; info[2] = N.A.ell; info[3] = N.A.L; info[4] = (double)N.off.n;
  info[5] = N.A.s_out; info[6] = N.compute;
  return PD_OK;
}

int pd_mpn_init_params(pd_mpn* m, uint64_t seed) {
  if (!m) {
    set_last_error("null argument");
    return PD_ERR_INVALID_ARG;
  }
  MPN_TRY
  MpnImpl& N = m->N;
  std::vector<float> h(N.off.n, 0.0f);
  uint64_t st = seed;
  auto uni = [&]() { return (double)(splitmix(st) >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0; };
  auto fill = [&](size_t off, int fan_in, int count, double scale) {
    for (int e = 0; e < count; ++e) h[off + e] = (float)(scale * uni() / std::sqrt((double)fan_in));
  };
  const POff& o = N.off;
  fill(o.We, kMpnF, kMpnF * kMpnH, 1.0);
  for (int l = 0; l < kMpnLayers; ++l) {
    fill(o.Wm[l], kMpnKM, kMpnKM * kMpnH, 1.0);
    fill(o.Wn[l], 2 * kMpnH, 2 * kMpnH * kMpnH, 1.0);
  }
  fill(o.Wd, kMpnH, kMpnH * 3, 0.1);
  upload(N.P, h);
  MPN_HIP(hipMemset(N.Mo, 0, N.off.n * sizeof(float)));
  MPN_HIP(hipMemset(N.Vo, 0, N.off.n * sizeof(float)));
  N.step = 0;
  return PD_OK;
  MPN_CATCH
}

int pd_mpn_set_params(pd_mpn* m, const float* host, int64_t n) {
  if (!m || !host || n != (int64_t)m->N.off.n) {
    set_last_error("null argument or wrong parameter count");
    return PD_ERR_INVALID_ARG;
  }
  MPN_TRY
  MPN_HIP(hipMemcpy(m->N.P, host, n * sizeof(float), hipMemcpyHostToDevice));
  MPN_HIP(hipMemset(m->N.Mo, 0, n * sizeof(float)));
  MPN_HIP(hipMemset(m->N.Vo, 0, n * sizeof(float)));
  m->N.step = 0;
  return PD_OK;
  MPN_CATCH
}

int pd_mpn_share_params(pd_mpn* dst, pd_mpn* src) {
  if (!dst || !src || dst == src || dst->N.off.n != src->N.off.n || dst->N.compute != src->N.compute) {
    set_last_error("null argument, the same network, or networks of different shapes");
    return PD_ERR_INVALID_ARG;
  }
  MPN_TRY
  MPN_HIP(hipDeviceSynchronize());  // kernels of dst may still use its own buffers
  MpnImpl& D = dst->N;
  if (!D.shared) {
    dfree(D.P); dfree(D.G); dfree(D.Mo); dfree(D.Vo);
  }
  D.P = src->N.P;
  D.G = src->N.G;
  D.Mo = src->N.Mo;
  D.Vo = src->N.Vo;
  D.shared = true;
  return PD_OK;
  MPN_CATCH
}

int pd_mpn_get_params(const pd_mpn* m, float* host, int64_t n) {
  if (!m || !host || n != (int64_t)m->N.off.n) {
    set_last_error("null argument or wrong parameter count");
    return PD_ERR_INVALID_ARG;
  }
  MPN_TRY
  MPN_HIP(hipMemcpy(host, m->N.P, n * sizeof(float), hipMemcpyDeviceToHost));
  return PD_OK;
  MPN_CATCH
}

int pd_mpn_get_grads(const pd_mpn* m, float* host, int64_t n) {
  if (!m || !host || n != (int64_t)m->N.off.n) {
    set_last_error("null argument or wrong parameter count");
    return PD_ERR_INVALID_ARG;
  }
  MPN_TRY
  MPN_HIP(hipMemcpy(host, m->N.G, n * sizeof(float), hipMemcpyDeviceToHost));
  return PD_OK;
  MPN_CATCH
}

int pd_mpn_set_output_scale(pd_mpn* m, double s_out) {
  if (!m || !(s_out > 0.0)) {
    set_last_error("invalid argument");
    return PD_ERR_INVALID_ARG;
  }
  m->N.A.s_out = s_out;
  return PD_OK;
}

int pd_mpn_forward(pd_mpn* m, const double* q_t, const double* v_tm1, const double* v_t, const double* f_ext,
                   const double* logw, double* q0, void* stream) {
  if (!m || !q_t || !v_tm1 || !v_t || !logw || !q0) {
    set_last_error("null argument");
    return PD_ERR_INVALID_ARG;
  }
  MPN_TRY
  MpnImpl& N = m->N;
  hipStream_t s = (hipStream_t)stream;
  mpn_forward(N, q_t, v_tm1, v_t, f_ext, logw, s);
  hipLaunchKernelGGL(k_mpn_dec, dim3(mpn_grid_rows(N.A.nv, 256)), dim3(256), 0, s, N.A, N.hbuf[kMpnLayers],
                     N.P + N.off.Wd, N.P + N.off.bd, v_t, nullptr, q0, nullptr);
  MPN_HIP(hipGetLastError());
  return PD_OK;
  MPN_CATCH
}

int pd_mpn_loss_grad(pd_mpn* m, const double* q_t, const double* v_tm1, const double* v_t, const double* f_ext,
                     const double* logw, const double* q_next, double* loss, void* stream) {
  if (!m || !q_t || !v_tm1 || !v_t || !logw || !q_next) {
    set_last_error("null argument");
    return PD_ERR_INVALID_ARG;
  }
  MPN_TRY
  MpnImpl& N = m->N;
  hipStream_t s = (hipStream_t)stream;
  mpn_forward(N, q_t, v_tm1, v_t, f_ext, logw, s);
  const int nb = mpn_grid_rows(N.A.nv, 256);
  hipLaunchKernelGGL(k_mpn_dec, dim3(nb), dim3(256), 0, s, N.A, N.hbuf[kMpnLayers], N.P + N.off.Wd,
                     N.P + N.off.bd, v_t, q_next, nullptr, N.res);
  hipLaunchKernelGGL(k_mpn_loss, dim3(nb), dim3(256), 0, s, N.A, N.res, N.dy, N.lpart);
  mpn_backward(N, s);
  MPN_HIP(hipGetLastError());
  if (loss) {
    MPN_HIP(hipMemcpyAsync(N.hl, N.lpart, sizeof(double) * nb, hipMemcpyDeviceToHost, s));
    MPN_HIP(hipStreamSynchronize(s));
    double t = 0.0;
    for (int b = 0; b < nb; ++b) t += N.hl[b];
    *loss = t;
  }
  return PD_OK;
  MPN_CATCH
}

int pd_mpn_adam_step(pd_mpn* m, double lr, double beta1, double beta2, double eps, void* stream) {
  if (!m || !(lr > 0.0) || !(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0) || !(eps > 0.0)) {
    set_last_error("invalid argument");
    return PD_ERR_INVALID_ARG;
  }
  MPN_TRY
  MpnImpl& N = m->N;
  N.step++;
  const float c1 = (float)(1.0 - std::pow(beta1, (double)N.step));
  const float c2 = (float)(1.0 - std::pow(beta2, (double)N.step));
  const int n = (int)N.off.n;
  hipLaunchKernelGGL(k_mpn_adam, dim3(mpn_grid_rows(n, 256)), dim3(256), 0, (hipStream_t)stream, N.P, N.G, N.Mo,
                     N.Vo, n, (float)lr, (float)beta1, (float)beta2, (float)eps, c1, c2);
  MPN_HIP(hipGetLastError());
  return PD_OK;
  MPN_CATCH
}

}  // extern "C"
