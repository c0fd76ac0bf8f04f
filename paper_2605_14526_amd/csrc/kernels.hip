// HIP kernels (gfx950) of the PD hot path.
//
// Launch-latency design: on this GPU a kernel boundary costs ~1.6 us inside a
// graph and a grid-wide barrier inside a persistent kernel ~30 us, so each PD
// iteration is a short fixed chain of wide kernels.  Element work runs one
// tet per lane; element contributions are written straight into the
// vertex-incidence order, so the right-hand-side gathers read contiguous
// memory with 8 lanes per vertex (no atomics, fixed summation order); every
// dense block product of the partitioned inverse runs one wave per row; block
// partial sums are reduced in a fixed order by the kernel that consumes them,
// so all results are bitwise reproducible.  The Anderson update
// of iteration k-1 is applied on the fly by the two kernels that start
// iteration k, and the conjugate-gradient direction update likewise by the two
// kernels that start the next adjoint iteration.  Each kernel requests every
// load that does not depend on another load (descriptors, own state, partial
// sums, the done flag) before it waits for any of them, so a stage costs about
// two dependent memory round trips.
//
// Vector layout: SoA over the library vertex order, x | y | z, stride nv.
// Per-tet arrays: SoA, stride ne.  Contributions: [axis][incidence position].
#include "kernels.h"

#include <hip/hip_ext.h>

#include "device_math.h"

namespace pdhot {

// ---------------------------------------------------------------- helpers
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// A value that every lane of the wave holds, moved to a scalar register (row
// descriptors of one-row-per-wave kernels), so that addresses built from it
// are scalar bases.
__device__ __forceinline__ int wave_uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ long long wave_uniform(long long x) {
  const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(x & 0xffffffffLL));
  const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)((unsigned long long)x >> 32));
  return (long long)(((unsigned long long)hi << 32) | lo);
}

// base[i] read through a 32-bit byte offset o = 8 i: with a scalar base the
// load keeps only o in a vector register
__device__ __forceinline__ double at_byte(const double* __restrict__ base, unsigned o) {
  return *reinterpret_cast<const double*>(reinterpret_cast<const char*>(base) + o);
}

// Workgroups are dealt to the chip's 8 XCDs round-robin (XCD = block id mod
// 8), each XCD with its own L2.  The element kernels renumber their blocks so
// that every XCD takes one contiguous range of tets: neighbouring tets share
// vertices, so their gathers and scattered contribution writes meet in one L2.
// A bijection on 0 .. n - 1 for any n.
__device__ __forceinline__ int xcd_block(int b, int n) {
  constexpr int kXcd = 8;
  const int x = b % kXcd, i = b / kXcd, q = n / kXcd, r = n % kXcd;
  return (x < r) ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

// sum within aligned groups of 8 lanes (every lane of the group gets it)
__device__ __forceinline__ double group8_sum(double v) {
  v += __shfl_xor(v, 4, 64);
  v += __shfl_xor(v, 2, 64);
  v += __shfl_xor(v, 1, 64);
  return v;
}

// block-wide sum of NV values per thread; result valid in thread 0.  With
// lane0 (block-uniform) only lane 0 of each wave holds nonzero values, and its
// values stand for the wave's sums: the butterfly would only add zeros.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* lds /* >= 16*NV */, bool lane0 = false) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (!lane0)
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] = wave_sum(v[i]);
  __syncthreads();
  if (lane == 0)
#pragma unroll
    for (int i = 0; i < NV; ++i) lds[wid * NV + i] = v[i];
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = blockDim.x >> 6;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      double s = 0.0;
      for (int w = 0; w < nw; ++w) s += lds[w * NV + i];
      v[i] = s;
    }
  }
  __syncthreads();
}

// Value j of every partial of `site`, indexed by the producing block: the
// values a consumer reads from consecutive partials are contiguous.
__device__ __forceinline__ double* part_value(const RedArgs& R, int site, int j) {
  return R.part + ((size_t)site * kRedWidth + j) * R.max_parts;
}

// Producer side: block sum of N values, written by thread 0 as partial `idx`
// of `site`.  Every thread of the block must call it.
template <int N>
__device__ __forceinline__ void write_partial(double (&v)[N], const RedArgs& R, int site, int idx,
                                              bool lane0 = false) {
  __shared__ double red[16 * N];
  block_sum<N>(v, red, lane0);
  if (threadIdx.x == 0)
#pragma unroll
    for (int j = 0; j < N; ++j) part_value(R, site, j)[idx] = v[j];
}

// Consumer side: the total of the first N values of every partial of `site`,
// returned to every thread; block 0 (bid) also stores it in fin.  Wave 0 does
// the sum in a fixed order that does not depend on the block size: lane l
// takes partials l, l + 64, l + 128, ... in that order, then the wave's
// butterfly.  The partials are requested a chunk at a time, each chunk before
// the previous one is summed, so two chunks cost one memory round trip.
// partials per lane in one chunk of the consumer wave (N values each)
template <int N>
constexpr int consume_chunk() { return N <= 4 ? 8 : (N <= 8 ? 4 : 1); }

template <int N>
__device__ __forceinline__ void consume_load(const RedArgs& R, int site, int width, int np, int first,
                                             double (&v)[consume_chunk<N>()][N]) {
  constexpr int kChunk = consume_chunk<N>();
#pragma unroll
  for (int c = 0; c < kChunk; ++c) {
    const int b = min(first + 64 * c, np - 1);  // past the end: a repeat of the last, not summed
#pragma unroll
    for (int j = 0; j < N; ++j) v[c][j] = (j < width) ? part_value(R, site, j)[b] : 0.0;
  }
}

template <int N>
__device__ __forceinline__ void consume_add(int np, int first, const double (&v)[consume_chunk<N>()][N],
                                            double (&acc)[N]) {
  constexpr int kChunk = consume_chunk<N>();
#pragma unroll
  for (int c = 0; c < kChunk; ++c)
    if (first + 64 * c < np)
#pragma unroll
      for (int j = 0; j < N; ++j) acc[j] += v[c][j];
}

template <int N>
__device__ __forceinline__ void consume(const RedArgs& R, int site, double (&tot)[N], int bid, int width = N) {
  constexpr int kChunk = consume_chunk<N>();
  constexpr int kStep = 64 * kChunk;
  __shared__ double bc[N];
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    const int np = R.nparts[site];
    double acc[N];
#pragma unroll
    for (int j = 0; j < N; ++j) acc[j] = 0.0;
    if (np > 0) {
      // two chunk buffers in turn: chunk i + 1 is requested before chunk i is added
      double v0[kChunk][N], v1[kChunk][N];
      consume_load<N>(R, site, width, np, lane, v0);
      for (int base = 0; base < np; base += 2 * kStep) {
        consume_load<N>(R, site, width, np, base + kStep + lane, v1);
        consume_add<N>(np, base + lane, v0, acc);
        consume_load<N>(R, site, width, np, base + 2 * kStep + lane, v0);  // unconditional: no wait on it below
        consume_add<N>(np, base + kStep + lane, v1, acc);
      }
    }
#pragma unroll
    for (int j = 0; j < N; ++j) acc[j] = wave_sum(acc[j]);
    if (lane == 0)
#pragma unroll
      for (int j = 0; j < N; ++j) {
        bc[j] = acc[j];
        if (bid == 0) R.fin[site * kFinStride + j] = acc[j];
      }
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < N; ++j) tot[j] = bc[j];
  __syncthreads();
}

__device__ __forceinline__ double* fin_site(const RedArgs& R, int site) { return R.fin + site * kFinStride; }

__device__ __forceinline__ void load_F(const ElemArgs& E, const double* __restrict__ q, int nv, int t, double F[9],
                                       int vi[4]) {
  vi[0] = E.tv[t];
  vi[1] = E.tv[E.ne + t];
  vi[2] = E.tv[2 * E.ne + t];
  vi[3] = E.tv[3 * E.ne + t];
  double Ds[9];
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    const double x0 = q[ax * nv + vi[0]];
    Ds[3 * ax + 0] = q[ax * nv + vi[1]] - x0;
    Ds[3 * ax + 1] = q[ax * nv + vi[2]] - x0;
    Ds[3 * ax + 2] = q[ax * nv + vi[3]] - x0;
  }
  double Bm[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) Bm[i] = E.Bm[i * E.ne + t];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) F[3 * i + j] = Ds[3 * i] * Bm[j] + Ds[3 * i + 1] * Bm[3 + j] + Ds[3 * i + 2] * Bm[6 + j];
}

// w G_e^T P written to the incidence positions of the tet's free vertices:
// vertex a (1..3) receives w P r_a (r_a = row a-1 of D_m^{-1}), vertex 0 minus
// their sum.
__device__ __forceinline__ void store_contrib(const ElemArgs& E, double* __restrict__ contrib, int t, double w,
                                              const double P[9]) {
  double Bm[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) Bm[i] = E.Bm[i * E.ne + t];
  double c0[3] = {0, 0, 0};
#pragma unroll
  for (int a = 1; a < 4; ++a) {
    const int pos = E.tinc[a * E.ne + t];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      const double v = w * (P[3 * ax] * Bm[3 * (a - 1)] + P[3 * ax + 1] * Bm[3 * (a - 1) + 1] +
                            P[3 * ax + 2] * Bm[3 * (a - 1) + 2]);
      if (pos >= 0) contrib[(size_t)ax * E.ninc + pos] = v;
      c0[ax] -= v;
    }
  }
  const int pos0 = E.tinc[t];
  if (pos0 >= 0)
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) contrib[(size_t)ax * E.ninc + pos0] = c0[ax];
}

// 8 lanes per vertex: the sum of the vertex's incidence entries k0 .. k1 - 1
// (contiguous, per axis).  Lane l adds entries k0 + l, k0 + l + 8, ... in
// that order, then the group's butterfly; a lane requests a chunk of its
// entries at once (a vertex has about 16), so the walk costs one memory round
// trip instead of one per entry.  The sums are those of the plain strided loop.
__device__ __forceinline__ void inc_sum8(const double* __restrict__ contrib, int ninc, int k0, int k1, int l,
                                         double out[3]) {
  constexpr int kChunk = 4;
  double s0 = 0, s1 = 0, s2 = 0;
  for (int base = k0; base < k1; base += 8 * kChunk) {
    double v[kChunk][3];
#pragma unroll
    for (int c = 0; c < kChunk; ++c) {
      const int kk = min(base + l + 8 * c, k1 - 1);
      v[c][0] = contrib[kk];
      v[c][1] = contrib[(size_t)ninc + kk];
      v[c][2] = contrib[2 * (size_t)ninc + kk];
    }
#pragma unroll
    for (int c = 0; c < kChunk; ++c)
      if (base + l + 8 * c < k1) {
        s0 += v[c][0];
        s1 += v[c][1];
        s2 += v[c][2];
      }
  }
  out[0] = group8_sum(s0);
  out[1] = group8_sum(s1);
  out[2] = group8_sum(s2);
}

__device__ __forceinline__ void gather8(const int* __restrict__ inc_ptr, const double* __restrict__ contrib, int ninc,
                                        int i, int l, double out[3]) {
  inc_sum8(contrib, ninc, inc_ptr[i], inc_ptr[i + 1], l, out);
}

// Element data of tet t: vertex ids, incidence positions, D_m^{-1}.
struct TetData {
  int vi[4], pos[4];
  double Bm[9];
};

__device__ __forceinline__ void load_tet(const ElemArgs& E, int t, TetData& T) {
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    T.vi[a] = E.tv[a * E.ne + t];
    T.pos[a] = E.tinc[a * E.ne + t];
  }
#pragma unroll
  for (int i = 0; i < 9; ++i) T.Bm[i] = E.Bm[i * E.ne + t];
}

__device__ __forceinline__ void grad_of(const TetData& T, const double xv[4][3], double F[9]) {
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    const double d1 = xv[1][ax] - xv[0][ax], d2 = xv[2][ax] - xv[0][ax], d3 = xv[3][ax] - xv[0][ax];
#pragma unroll
    for (int j = 0; j < 3; ++j) F[3 * ax + j] = d1 * T.Bm[j] + d2 * T.Bm[3 + j] + d3 * T.Bm[6 + j];
  }
}

// G_e^T P written to the incidence positions of the tet's free vertices.
__device__ __forceinline__ void store_GtP(const TetData& T, double* __restrict__ contrib, int ninc, const double P[9]) {
  double c0[3] = {0, 0, 0};
#pragma unroll
  for (int a = 1; a < 4; ++a)
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      const double v = P[3 * ax] * T.Bm[3 * (a - 1)] + P[3 * ax + 1] * T.Bm[3 * (a - 1) + 1] +
                       P[3 * ax + 2] * T.Bm[3 * (a - 1) + 2];
      if (T.pos[a] >= 0) contrib[(size_t)ax * ninc + T.pos[a]] = v;
      c0[ax] -= v;
    }
  if (T.pos[0] >= 0)
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) contrib[(size_t)ax * ninc + T.pos[0]] = c0[ax];
}

// The warm start of the tet's next SVD and prox Newton: the rotation V as a
// unit quaternion (4 doubles instead of 9; V is a proper rotation, so the
// quaternion holds it exactly up to rounding, and rebuilding it re-orthonormalises),
// and the ratios s*/sF.  The quaternion is taken from the largest of
// 1 + tr V, 1 + 2 V_ii - tr V (the numerically safe branch).
__device__ __forceinline__ void quat_of_rot(const double V[9], double q[4]) {
  const double tr = V[0] + V[4] + V[8];
  if (tr >= V[0] && tr >= V[4] && tr >= V[8]) {
    const double r = sqrt(fmax(1.0 + tr, 0.0)), f = 0.5 / r;
    q[0] = 0.5 * r; q[1] = (V[7] - V[5]) * f; q[2] = (V[2] - V[6]) * f; q[3] = (V[3] - V[1]) * f;
  } else if (V[0] >= V[4] && V[0] >= V[8]) {
    const double r = sqrt(fmax(1.0 + V[0] - V[4] - V[8], 0.0)), f = 0.5 / r;
    q[0] = (V[7] - V[5]) * f; q[1] = 0.5 * r; q[2] = (V[1] + V[3]) * f; q[3] = (V[2] + V[6]) * f;
  } else if (V[4] >= V[8]) {
    const double r = sqrt(fmax(1.0 - V[0] + V[4] - V[8], 0.0)), f = 0.5 / r;
    q[0] = (V[2] - V[6]) * f; q[1] = (V[1] + V[3]) * f; q[2] = 0.5 * r; q[3] = (V[5] + V[7]) * f;
  } else {
    const double r = sqrt(fmax(1.0 - V[0] - V[4] + V[8], 0.0)), f = 0.5 / r;
    q[0] = (V[3] - V[1]) * f; q[1] = (V[2] + V[6]) * f; q[2] = (V[5] + V[7]) * f; q[3] = 0.5 * r;
  }
}

__device__ __forceinline__ void store_rot(const ElemArgs& E, int t, const double V[9]) {
  double q[4];
  quat_of_rot(V, q);
#pragma unroll
  for (int j = 0; j < 4; ++j) E.Vw[(size_t)j * E.ne + t] = q[j];
}

// The rotation of a stored quaternion (false: none stored, start cold from
// the identity)
__device__ __forceinline__ bool rot_of_quat(const double q[4], double V[9]) {
  const double n2 = q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
  if (!(n2 > 0.5 && n2 < 2.0)) {  // also false for NaN
#pragma unroll
    for (int j = 0; j < 9; ++j) V[j] = (j % 4 == 0) ? 1.0 : 0.0;
    return false;
  }
  const double s = 2.0 / n2;
  const double w = q[0], x = q[1], y = q[2], z = q[3];
  V[0] = 1.0 - s * (y * y + z * z); V[1] = s * (x * y - w * z); V[2] = s * (x * z + w * y);
  V[3] = s * (x * y + w * z); V[4] = 1.0 - s * (x * x + z * z); V[5] = s * (y * z - w * x);
  V[6] = s * (x * z - w * y); V[7] = s * (y * z + w * x); V[8] = 1.0 - s * (x * x + y * y);
  return true;
}

__device__ __forceinline__ bool load_rot(const ElemArgs& E, int t, double V[9]) {
  double q[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) q[j] = E.Vw[(size_t)j * E.ne + t];
  return rot_of_quat(q, V);
}

// warm start of the next SVD and prox Newton of this tet: its rotation V and
// the stretch ratios s*/sF (Neo-Hookean prox), or the volume step's
// multiplier (corotated + volume composite)
__device__ __forceinline__ void store_warm(const ElemArgs& E, int t, const double V[9], const double sF[3],
                                           const double ss[3]) {
  store_rot(E, t, V);
#pragma unroll
  for (int j = 0; j < 3; ++j) E.rw[(size_t)j * E.ne + t] = (sF[j] > 1e-12) ? ss[j] / sF[j] : 0.0;
}

__device__ __forceinline__ void store_warm_nu(const ElemArgs& E, int t, const double V[9], double nu) {
  store_rot(E, t, V);
  E.rw[t] = nu;
}

// ---------------------------------------------------------------- muscle fibres
// A muscle tet carries the fibre constraint (w_m V_e / 2) dist^2(F m, S_l):
// the fibre image f = F m is projected onto the sphere of radius
// l = 1 - a_g (a_g the activation of the tet's group), p = l f/|f|, and
// w_m V_e G^T p joins b; its derivative (l/|f|)(I - f^ f^T) joins K and
// db/da_g = -w_m V_e G^T f^.  G^T (x m^T) gives vertex a the vector
// (Bhat_a . m) x, so every term enters the element's 3x3 matrix as x m^T.
__device__ __forceinline__ void fibre_of(const ElemArgs& E, int t, double m[3], double& wm) {
  const size_t ne = E.ne;
  m[0] = E.mus[t];
  m[1] = E.mus[ne + t];
  m[2] = E.mus[2 * ne + t];
  wm = E.mus[3 * ne + t];
}

__device__ __forceinline__ void mat_vec_m(const double F[9], const double m[3], double f[3]) {
#pragma unroll
  for (int i = 0; i < 3; ++i) f[i] = F[3 * i] * m[0] + F[3 * i + 1] * m[1] + F[3 * i + 2] * m[2];
}

// P += w_m V_e p m^T (local step)
__device__ __forceinline__ void muscle_local(const ElemArgs& E, int t, const double F[9], double P[9]) {
  double m[3], wm;
  fibre_of(E, t, m, wm);
  if (wm == 0.0) return;
  double f[3];
  mat_vec_m(F, m, f);
  const double nf = sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
  const double ell = 1.0 - E.act[E.mgrp[t]];
  double p[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) p[i] = (nf > 0.0) ? ell * f[i] / nf : ell * m[i];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) P[3 * i + j] += wm * p[i] * m[j];
}

// the fibre's energy (w_m V_e / 2)(|F m| - l)^2 (primal objective)
__device__ __forceinline__ double muscle_energy(const ElemArgs& E, int t, const double F[9]) {
  double m[3], wm;
  fibre_of(E, t, m, wm);
  if (wm == 0.0) return 0.0;
  double f[3];
  mat_vec_m(F, m, f);
  const double d = sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]) - (1.0 - E.act[E.mgrp[t]]);
  return 0.5 * wm * d * d;
}

// ---------------------------------------------------------------- Anderson mixing
struct AAMix {
  int stop;       // the loop has already stopped (done flag)
  int use;        // apply the mixing
  int reset;      // |gamma| > 10: history dropped
  int nc, head;   // columns after the append of iteration k-1
  int m;
  double gam[kMaxWindow];
};

__device__ __forceinline__ void aa_layout(const int* st, int m, int& nonempty, int& nc_after, int& head_after,
                                          int& slot_new) {
  nonempty = st[0];
  const int nc = st[1], head = st[2];
  slot_new = -1;
  nc_after = nc;
  head_after = head;
  if (m <= 0 || !nonempty) return;
  if (nc < m) {
    slot_new = (head + nc) % m;
    nc_after = nc + 1;
  } else {
    slot_new = head;
    head_after = (head + 1) % m;
  }
}

// gamma = (dG^T dG + rho I)^{-1} dG^T g with rho = max(1e-6 |dG|_F^2 / m_c, 1e-12)
// (Eq. aa_gamma) from the final Gram sums of iteration k-1; reliability guard
// |gamma|_2 > 10.  The window M is a compile-time constant, so the Gram sums
// and the M x M Cholesky stay in registers.  Computed by thread 0, broadcast
// through LDS together with the loop's done flag (read with the sums).  Every
// thread of the block must call it; loads issued before the call stay ahead
// of its barriers.
template <int M>
__device__ __forceinline__ void aa_prepare(const StepState& St, const RedArgs& R, int k, bool reduce, AAMix& out,
                                           int bid) {
  __shared__ AAMix mx;
  constexpr int NA = (M > 0) ? M * M + M : 1;
  int flag = 0;
  int st[4] = {0, 0, 0, 0};
  double tot[NA];
#pragma unroll
  for (int j = 0; j < NA; ++j) tot[j] = 0.0;
  if (threadIdx.x == 0) {
    flag = *St.done;
    if (M > 0 && k >= 1)
#pragma unroll
      for (int j = 0; j < 4; ++j) st[j] = St.ctl[kCtlAA + 4 * ((k - 1) & 1) + j];
  }
  if (M > 0 && k >= 1) {
    if (reduce) {
      consume<NA>(R, kRedAA, tot, bid);  // Gram sums of iteration k-1: G[j][l] at j*M + l, rhs[j] at M*M + j
    } else if (threadIdx.x == 0) {
#pragma unroll
      for (int j = 0; j < NA; ++j) tot[j] = R.fin[kRedAA * kFinStride + j];
    }
  }
  if (threadIdx.x == 0) {
    mx.stop = flag;
    mx.use = 0;
    mx.reset = 0;
    mx.m = M;
    mx.nc = 0;
    mx.head = 0;
#pragma unroll
    for (int j = 0; j < kMaxWindow; ++j) mx.gam[j] = 0.0;
    if constexpr (M > 0) {
      if (k >= 1 && !flag) {
        int nonempty, nc, head, slot_new;
        aa_layout(st, M, nonempty, nc, head, slot_new);
        mx.nc = nc;
        mx.head = head;
        if (nc >= 1) {
          // padded to M with identity rows (unused columns decouple)
          double G[M][M], rhs[M];
          double fro = 0.0;
#pragma unroll
          for (int j = 0; j < M; ++j) {
#pragma unroll
            for (int l = 0; l < M; ++l) {
              double g = (j == l) ? 1.0 : 0.0;
              if (j < nc && l < nc) g = (j <= l) ? tot[j * M + l] : tot[l * M + j];
              G[j][l] = g;
            }
            rhs[j] = (j < nc) ? tot[M * M + j] : 0.0;
            if (j < nc) fro += G[j][j];
          }
          const double rho = fmax(1e-6 * fro / nc, 1e-12);
#pragma unroll
          for (int j = 0; j < M; ++j)
            if (j < nc) G[j][j] += rho;
          bool ok = true;
#pragma unroll
          for (int j = 0; j < M; ++j) {
            double d = G[j][j];
#pragma unroll
            for (int l = 0; l < j; ++l) d -= G[j][l] * G[j][l];
            ok = ok && (d > 0.0);
            d = sqrt(fmax(d, 1e-300));
            G[j][j] = d;
#pragma unroll
            for (int i = j + 1; i < M; ++i) {
              double t = G[i][j];
#pragma unroll
              for (int l = 0; l < j; ++l) t -= G[i][l] * G[j][l];
              G[i][j] = t / d;
            }
          }
          double y[M], gam[M];
#pragma unroll
          for (int i = 0; i < M; ++i) {
            double t = rhs[i];
#pragma unroll
            for (int l = 0; l < i; ++l) t -= G[i][l] * y[l];
            y[i] = t / G[i][i];
          }
#pragma unroll
          for (int i = M - 1; i >= 0; --i) {
            double t = y[i];
#pragma unroll
            for (int l = i + 1; l < M; ++l) t -= G[l][i] * gam[l];
            gam[i] = t / G[i][i];
          }
          double nrm = 0.0;
#pragma unroll
          for (int i = 0; i < M; ++i) nrm += (i < nc) ? gam[i] * gam[i] : 0.0;
          nrm = ok ? sqrt(nrm) : INFINITY;
#pragma unroll
          for (int i = 0; i < M; ++i) mx.gam[i] = (i < nc) ? gam[i] : 0.0;
          mx.use = (nrm <= 10.0);
          mx.reset = !mx.use;
        }
      }
    }
  }
  __syncthreads();
  out = mx;
  __syncthreads();
}

// q^k of a free vertex: q^ - (dQ + dG) gamma (Eq. aa_update) or q^ (k >= 1);
// q_cur at k = 0 (the initial iterate)
template <int M>
__device__ __forceinline__ double aa_value(const StepState& St, const AAMix& mx, int nv, int a, int i, int k) {
  const int ix = a * nv + i;
  if (k == 0) return St.q_cur[ix];
  double q = St.qhat[ix];
  if (M > 0 && mx.use) {
#pragma unroll
    for (int j = 0; j < M; ++j)
      if (j < mx.nc) {
        int slot = mx.head + j;
        if (slot >= M) slot -= M;
        const size_t cix = ((size_t)slot * 3 + a) * nv + i;
        q -= (St.dQ[cix] + St.dG[cix]) * mx.gam[j];
      }
  }
  return q;
}

// ---------------------------------------------------------------- local step
// p*_e = U diag(s*) V^T of F_e = G_e q^k (Sec. 4.1 Eq. nh_prox) and its
// contribution w_e V_e G_e^T p*_e (Eq. A_basic).  The SVD and the prox Newton
// start from the tet's previous rotation and stretch ratios.
template <int M>
__device__ __forceinline__ void b_local(ElemArgs E, StepState St, RedArgs R, const double* __restrict__ q,
                                                  int nv, int nf, int k, int fwd, int* __restrict__ newton_cap, int bid) {
  const int t = bid * blockDim.x + threadIdx.x;
  const bool have = t < E.ne;
  // the tet's data and warm start, requested before the Anderson scalars
  TetData T;
  double q4[4], rt[3], wv = 0.0;
  if (have) {
    load_tet(E, t, T);
#pragma unroll
    for (int j = 0; j < 4; ++j) q4[j] = E.Vw[(size_t)j * E.ne + t];
#pragma unroll
    for (int j = 0; j < 3; ++j) rt[j] = E.rw[(size_t)j * E.ne + t];
    wv = E.wV[t];
  }
  AAMix mx;
  if (fwd) {
    aa_prepare<M>(St, R, k, true, mx, bid);
    if (mx.stop) return;
  }
  if (!have) return;
  double xv[4][3];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int ax = 0; ax < 3; ++ax)
      xv[a][ax] = (fwd && T.vi[a] < nf) ? aa_value<M>(St, mx, nv, ax, T.vi[a], k) : q[ax * nv + T.vi[a]];
  double F[9], U[9], V[9], sF[3], ss[3];
  grad_of(T, xv, F);
  const bool warm = rot_of_quat(q4, V);
  svd3(F, U, sF, V, warm);
  double P[9];
  if (E.energy >= 1) {
    // corotated + volume: 2 mu_e V_e R + lam_e V_e P_vol = U diag(2 mu_e V_e + lam_e V_e sv) V^T;
    // energy 2 takes the logarithmic barrier's stretch step (Eq. pd_log_volume: the prox Newton
    // without the I1 term, means mu_bar, lam_bar, penalty lam_bar) for the volume step
    double nu = rt[0], sv[3];
    if (E.energy == 1) {
      volume_project(sF, nu, sv);
    } else {
      const int nit = prox_stretch_g(sF, 0.0, E.mu_bar, E.lam_bar, E.lam_bar, sv, rt);
      if (newton_cap && nit >= kNewtonCap) *newton_cap = 1;
    }
    const double m2 = 2.0 * E.muV[t], lv = E.lamV[t];
    double sw[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) sw[j] = m2 + lv * sv[j];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j)
        P[3 * i + j] = U[3 * i] * sw[0] * V[3 * j] + U[3 * i + 1] * sw[1] * V[3 * j + 1] + U[3 * i + 2] * sw[2] * V[3 * j + 2];
    if (E.mus) muscle_local(E, t, F, P);
    store_GtP(T, St.contrib, E.ninc, P);
    if (E.energy == 1) store_warm_nu(E, t, V, nu);
    else store_warm(E, t, V, sF, sv);
    return;
  }
  const int nit = prox_stretch(sF, E.mu_bar, E.lam_bar, E.k_bar, ss, rt);
  // cap hit: every writer stores the same value, so plain stores suffice
  if (newton_cap && nit >= kNewtonCap) *newton_cap = 1;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      P[3 * i + j] =
          wv * (U[3 * i] * ss[0] * V[3 * j] + U[3 * i + 1] * ss[1] * V[3 * j + 1] + U[3 * i + 2] * ss[2] * V[3 * j + 2]);
  if (E.mus) muscle_local(E, t, F, P);
  store_GtP(T, St.contrib, E.ninc, P);
  store_warm(E, t, V, sF, ss);
}

template <int M>
__global__ void __launch_bounds__(kBlock) k_local(ElemArgs E, StepState St, RedArgs R, const double* __restrict__ q,
                                                  int nv, int nf, int k, int fwd, int* __restrict__ newton_cap) {
  b_local<M>(E, St, R, q, nv, nf, k, fwd, newton_cap, xcd_block(blockIdx.x, gridDim.x));
}

// The bodies of the kernels that run once per step exist once, called by the
// single-scene kernel and by its batched twin alike: compiled twice (inlined
// into each), the compiler may fuse multiply-adds differently in the two
// copies, and a scene of a batch would no longer match its run alone bit for
// bit.
#define PD_SHARED_BODY __attribute__((noinline))
// The vertex kernels' bodies stay inlined: their own arithmetic is not fused
// at all (they call nothing that multiplies), which settles the same question.
#define PD_VERT_BODY __forceinline__

// G_e^T (w G_e x): contributions of the symmetric element operator w V G^T G
// (B_beta q_t in the prologue).
__device__ PD_SHARED_BODY void b_elem_GtG(const ElemArgs& E, const double* __restrict__ x, int nv,
                                           const double* __restrict__ w, double* __restrict__ contrib, int bid) {
  const int t = bid * blockDim.x + threadIdx.x;
  if (t >= E.ne) return;
  double F[9];
  int vi[4];
  load_F(E, x, nv, t, F, vi);
  store_contrib(E, contrib, t, w[t], F);
}

__global__ void __launch_bounds__(kBlock) k_elem_GtG(ElemArgs E, const double* __restrict__ x, int nv,
                                                     const double* __restrict__ w, double* __restrict__ contrib) {
  b_elem_GtG(E, x, nv, w, contrib, blockIdx.x);
}

// ---------------------------------------------------------------- step prologue
// q~ = q_t + h v_t + h^2 (M^{-1} f_ext + g)   (Eq. freefall)
// c  = M/h^2 q~ + (alpha/h) M q_t + (1/h) B_beta q_t - A~_{fp} q_p
// (damping terms of the right-hand side derived from Eq. dynamics).
__device__ PD_VERT_BODY void b_prologue(const VertArgs& Vx, const double* __restrict__ q_t_user,
                                           const double* __restrict__ v_t_user, const double* __restrict__ f_user,
                                           const double* __restrict__ q0_user, int inertial, const StepState& St,
                                           int bid) {
#pragma clang fp contract(off)
  // the step's control words (done flag, counters, Anderson layout) start at
  // zero; nothing in this kernel reads them
  if (bid == 0 && threadIdx.x < kCtlSize) St.ctl[threadIdx.x] = 0;
  const int gtid = bid * blockDim.x + threadIdx.x;
  const int i = gtid >> 3, l = gtid & 7;
  const int nv = Vx.nv;
  if (i >= nv) return;  // whole groups of 8 leave together
  double bq[3] = {0, 0, 0};
  if (i < Vx.nf) gather8(Vx.inc_ptr, St.contrib, Vx.ninc, i, l, bq);
  if (l != 0) return;
  const int o = Vx.v_orig[i];
  if (i >= Vx.nf) {  // pinned: held at rest
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double r = Vx.rest[a * nv + i];
      St.qt[a * nv + i] = r;
      St.qtil[a * nv + i] = r;
      St.q_cur[a * nv + i] = r;
      St.q_prev[a * nv + i] = r;
      St.qhat[a * nv + i] = r;
      St.vt[a * nv + i] = 0.0;
    }
    return;
  }
  const double m = Vx.mass[i], h = Vx.h;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double qt = q_t_user[3 * o + a];
    const double vt = v_t_user[3 * o + a];
    const double f = f_user ? f_user[3 * o + a] : 0.0;
    const double qtil = qt + h * vt + h * h * (f / m + Vx.grav[a]);
    St.qt[a * nv + i] = qt;
    St.vt[a * nv + i] = vt;
    St.qtil[a * nv + i] = qtil;
    St.c[a * nv + i] = m / (h * h) * qtil + Vx.alpha / h * m * qt + bq[a] + Vx.cpin[a * nv + i];
    const double q0 = q0_user ? q0_user[3 * o + a] : (inertial ? qt + h * vt : qt);
    St.q_cur[a * nv + i] = q0;
    St.q_prev[a * nv + i] = q0;
  }
}

__global__ void __launch_bounds__(kBlock) k_prologue(VertArgs Vx, const double* __restrict__ q_t_user,
                                                     const double* __restrict__ v_t_user,
                                                     const double* __restrict__ f_user,
                                                     const double* __restrict__ q0_user, int inertial,
                                                     StepState St) {
  b_prologue(Vx, q_t_user, v_t_user, f_user, q0_user, inertial, St, blockIdx.x);
}

// ---------------------------------------------------------------- right-hand side
// b^k = c + gathered contributions; q^k (Anderson update of iteration k-1,
// written by the vertex's group); partial sums of the dual gate
// (Eq. convergence_dual): |q^k - q^{k-1}|^2, |q^{k-1}|^2, |b^k - b^{k-1}|^2,
// |b^{k-1}|^2.  Block 0 records the Anderson state of iteration k.
template <int M>
__device__ __forceinline__ void b_gather_fwd(VertArgs Vx, StepState St, RedArgs R, int k, int bid) {
  const int nv = Vx.nv;
  const int gtid = bid * blockDim.x + threadIdx.x;
  const int i = gtid >> 3, l = gtid & 7;
  const bool have = i < Vx.nf;
  const bool owner = have && l == 0;
  // the vertex's incidence range and state, requested before the Anderson scalars
  int k0 = 0, k1 = 0;
  if (have) {
    k0 = Vx.inc_ptr[i];
    k1 = Vx.inc_ptr[i + 1];
  }
  double qh[3] = {0, 0, 0}, qc[3] = {0, 0, 0}, qp0[3] = {0, 0, 0}, bo[3] = {0, 0, 0}, cc[3] = {0, 0, 0};
  if (owner)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int ix = a * nv + i;
      if (k >= 1) qh[a] = St.qhat[ix];
      else qp0[a] = St.q_prev[ix];
      qc[a] = St.q_cur[ix];
      bo[a] = St.b_cur[ix];
      cc[a] = St.c[ix];
    }
  AAMix mx;
  aa_prepare<M>(St, R, k, false, mx, bid);
  if (mx.stop) return;
  // the vertex's Anderson columns dQ + dG, requested with its incidence entries
  constexpr int MC = M > 0 ? M : 1;
  double dqg[3][MC];
  if (M > 0 && owner && k >= 1 && mx.use)
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int j = 0; j < MC; ++j) {
        int slot = mx.head + j;
        if (slot >= M) slot -= M;
        const size_t cix = ((size_t)slot * 3 + a) * nv + i;
        dqg[a][j] = (j < mx.nc) ? St.dQ[cix] + St.dG[cix] : 0.0;
      }
  double part[4] = {0, 0, 0, 0};
  if (have) {
    double bs[3];
    inc_sum8(St.contrib, Vx.ninc, k0, k1, l, bs);
    if (l == 0) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const int ix = a * nv + i;
        double qk = qc[a];
        if (k >= 1) {
          qk = qh[a];
          if (M > 0 && mx.use) {
#pragma unroll
            for (int j = 0; j < MC; ++j)
              if (j < mx.nc) qk -= dqg[a][j] * mx.gam[j];
          }
        }
        const double qp = (k == 0) ? qp0[a] : qc[a];
        if (k > 0) {
          St.q_prev[ix] = qp;
          St.q_cur[ix] = qk;
        }
        const double bn = bs[a] + cc[a];
        St.b_prev[ix] = bo[a];
        St.b_cur[ix] = bn;
        part[0] += (qk - qp) * (qk - qp);
        part[1] += qp * qp;
        part[2] += (bn - bo[a]) * (bn - bo[a]);
        part[3] += bo[a] * bo[a];
      }
    }
  }
  if (bid == 0 && threadIdx.x == 0 && k >= 1) {
    int* nxt = St.ctl + kCtlAA + 4 * (k & 1);
    if (M <= 0 || mx.reset) {
      nxt[0] = 0; nxt[1] = 0; nxt[2] = 0;
      if (mx.reset) St.ctl[kCtlResets] += 1;
    } else {
      nxt[0] = 1; nxt[1] = mx.nc; nxt[2] = mx.head;
    }
  }
  write_partial<4>(part, R, kRedGate, bid);
}

template <int M>
__global__ void __launch_bounds__(kBlock) k_gather_fwd(VertArgs Vx, StepState St, RedArgs R, int k) {
  b_gather_fwd<M>(Vx, St, R, k, blockIdx.x);
}

// b = sum of the incidence entries of every free vertex (diagnostics)
__global__ void __launch_bounds__(kBlock) k_gather_debug(VertArgs Vx, const double* __restrict__ contrib,
                                                         double* __restrict__ out) {
  const int gtid = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = gtid >> 3, l = gtid & 7;
  if (i >= Vx.nf) return;
  double bs[3];
  gather8(Vx.inc_ptr, contrib, Vx.ninc, i, l, bs);
  if (l == 0)
#pragma unroll
    for (int a = 0; a < 3; ++a) out[a * Vx.nv + i] = bs[a];
}

// ---------------------------------------------------------------- interface right-hand side
// One wave per interface row i: r_T[i] = rhs_T[i] - sum over the subdomains s
// coupled to i of E_s[p] . rhs_s (the Schur-complement right-hand side).  The
// forward mode first takes the dual-gate decision (Eq. convergence_dual; the
// gate holds for k >= 2, k == kmax - 1 ends the step unconverged).  The PCG
// mode forms the updated residual r - alpha w on the fly, alpha = (r.z)/(p.w).
// The row descriptors, the row's own entries and the partial sums are all
// requested before the first of them is needed.
__device__ __forceinline__ double* r_cur(const AdjState& A, int it) { return (it & 1) ? A.r1 : A.r0; }

template <int MODE>
__device__ __forceinline__ void b_Eb(VertArgs Vx, SolveArgs Sv, StepState St, AdjState A, RedArgs R,
                                               const double* __restrict__ rhs, int k, int bid) {
  constexpr int RW = kEbRowsPerWave;
  const int lane = threadIdx.x & 63;
  // rows row0 .. row0 + RW - 1 of this wave; lane j < RW owns row row0 + j
  const int row0 = ((bid * blockDim.x + threadIdx.x) >> 6) * RW;
  const int my = row0 + lane;
  const bool have = row0 < Sv.nT;  // wave-uniform
  const bool mine = lane < RW && my < Sv.nT;
  const int nv = Vx.nv, nB = Sv.nB;
  const double* __restrict__ src = (MODE == kModeFwd) ? St.b_cur : (MODE == kModePCG ? r_cur(A, k) : rhs);
  const double* __restrict__ wv = A.w;
  // lane j loads the row descriptor of row row0 + j, lane c + kMaxCoup j the
  // coupling c of that row
  Cpl cd = {0, 0, 0, 0};
  ERow er = {0, 0, 0};
  double own[3] = {0.0, 0.0, 0.0}, ownw[3] = {0.0, 0.0, 0.0};
  if (mine) {
    er = Sv.erow[my];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      own[a] = src[a * nv + nB + my];
      if (MODE == kModePCG) ownw[a] = wv[a * nv + nB + my];
    }
  }
  {
    const int rj = row0 + lane / kMaxCoup;
    if (lane < RW * kMaxCoup && rj < Sv.nT) cd = Sv.cpl[rj * kMaxCoup + lane % kMaxCoup];
  }
  __shared__ int stop;
  __shared__ double alpha_s;
  if (MODE == kModePCG) {
    int flag = 0;
    double rz = 0.0;
    if (threadIdx.x == 0) {
      flag = *A.done;
      rz = fin_site(R, kRedRZ0 + (k & 1))[0];
    }
    double pw[1] = {1.0};
    consume<1>(R, kRedPW, pw, bid);
    if (threadIdx.x == 0) {
      stop = flag;
      alpha_s = rz / pw[0];
    }
  } else if (MODE == kModeFwd) {
    int flag = 0;
    if (threadIdx.x == 0) flag = *St.done;
    double g[4] = {0, 0, 0, 0};
    if (k >= 1) consume<4>(R, kRedGate, g, bid);
    if (threadIdx.x == 0) {
      const double dq = sqrt(g[0]), nq = sqrt(g[1]), db = sqrt(g[2]), nb = sqrt(g[3]);
      // with contact rows the FB residual of the last contact solve is a third condition
      const bool fb_ok = !St.fb || St.fb[0] <= St.fb_tol;
      const bool pass = dq <= St.eps_rel * nq + St.eps_abs && db <= St.eps_rel * nb + St.eps_abs && fb_ok;
      const bool conv = (k >= 2) && pass;
      const bool cap = (k >= St.kmax - 1);
      stop = flag || conv || cap;
      if (!flag && (conv || cap) && bid == 0) {
        St.ctl[kCtlDone] = 1;
        St.ctl[kCtlIters] = k;
        St.ctl[kCtlStatus] = conv ? 0 : 1;
        St.dstat[0] = dq; St.dstat[1] = nq; St.dstat[2] = db; St.dstat[3] = nb;
        if (St.sig) {  // statistics first, then the sequence number (system-scope ordered)
          St.sigd[0] = dq; St.sigd[1] = nq; St.sigd[2] = db; St.sigd[3] = nb;
          St.sig[1] = k;
          St.sig[2] = conv ? 0 : 1;
          St.sig[3] = St.ctl[kCtlResets];
          St.sig[4] = St.ctl[kCtlNewton];
          __threadfence_system();
          St.sig[0] = St.seq;
        }
      }
    }
  } else {
    // the flag is written by earlier kernels only, so every thread reads the same value
    if (threadIdx.x == 0) stop = St.done ? *St.done : 0;
  }
  __syncthreads();
  if (stop || !have) return;
  const double alpha = (MODE == kModePCG) ? alpha_s : 0.0;
  // each row's couplings (first entry, row of its part) and length, wave-uniform
  int B[RW][kMaxCoup], P[RW][kMaxCoup], len[RW], ncp[RW];
  long long eoff[RW];
#pragma unroll
  for (int j = 0; j < RW; ++j) {
#pragma unroll
    for (int c = 0; c < kMaxCoup; ++c) {
      B[j][c] = wave_uniform(__shfl(cd.b0, j * kMaxCoup + c, 64));
      P[j][c] = wave_uniform(__shfl(cd.pre, j * kMaxCoup + c, 64));
    }
    len[j] = wave_uniform(__shfl(er.len, j, 64));  // 0 past nT
    ncp[j] = wave_uniform(__shfl(er.n, j, 64));
    eoff[j] = wave_uniform(__shfl(er.off, j, 64));
  }
  int lmax = 0;
#pragma unroll
  for (int j = 0; j < RW; ++j) lmax = max(lmax, len[j]);
  double acc[RW][3];
#pragma unroll
  for (int j = 0; j < RW; ++j) acc[j][0] = acc[j][1] = acc[j][2] = 0.0;
  // entries past the end repeat the last one with weight zero; every trip
  // requests the chunk of all the wave's rows before it adds any
  constexpr int kSpan = 64 * kEbChunk;
  for (int base = 0; base < lmax; base += kSpan) {
    double cf[RW][kEbChunk], y[RW][kEbChunk][3], w[RW][kEbChunk][3];
#pragma unroll
    for (int j = 0; j < RW; ++j) {
      if (base >= len[j]) continue;
      const double* __restrict__ Er = Sv.E + eoff[j];
#pragma unroll
      for (int i = 0; i < kEbChunk; ++i) {
        const int idx = min(base + lane + 64 * i, len[j] - 1);
        int col = B[j][0] + idx;
#pragma unroll
        for (int c = 1; c < kMaxCoup; ++c)
          if (c < ncp[j] && idx >= P[j][c]) col = B[j][c] + idx - P[j][c];
        const unsigned oc = 8u * (unsigned)col;
        cf[j][i] = at_byte(Er, 8u * (unsigned)idx);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          y[j][i][a] = at_byte(src + a * nv, oc);
          if (MODE == kModePCG) w[j][i][a] = at_byte(wv + a * nv, oc);
        }
      }
    }
#pragma unroll
    for (int j = 0; j < RW; ++j) {
      if (base >= len[j]) continue;
#pragma unroll
      for (int i = 0; i < kEbChunk; ++i) {
        const double c = (base + lane + 64 * i < len[j]) ? cf[j][i] : 0.0;
        acc[j][0] += c * (MODE == kModePCG ? y[j][i][0] - alpha * w[j][i][0] : y[j][i][0]);
        acc[j][1] += c * (MODE == kModePCG ? y[j][i][1] - alpha * w[j][i][1] : y[j][i][1]);
        acc[j][2] += c * (MODE == kModePCG ? y[j][i][2] - alpha * w[j][i][2] : y[j][i][2]);
      }
    }
  }
  double xr[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int j = 0; j < RW; ++j) {
    const double s0 = wave_sum(acc[j][0]), s1 = wave_sum(acc[j][1]), s2 = wave_sum(acc[j][2]);
    if (lane == j) {
      xr[0] = s0;
      xr[1] = s1;
      xr[2] = s2;
    }
  }
  if (mine) {
#pragma unroll
    for (int a = 0; a < 3; ++a) own[a] -= alpha * ownw[a];
    Sv.rT[my] = own[0] - xr[0];
    Sv.rT[Sv.nT + my] = own[1] - xr[1];
    Sv.rT[2 * Sv.nT + my] = own[2] - xr[2];
  }
}

template <int MODE>
__global__ void __launch_bounds__(kBlock) PD_ROW_WALK_EB k_Eb(VertArgs Vx, SolveArgs Sv, StepState St, AdjState A, RedArgs R,
                                               const double* __restrict__ rhs, int k) {
  b_Eb<MODE>(Vx, Sv, St, A, R, rhs, k, blockIdx.x);
}

// ---------------------------------------------------------------- interface solve
// S x_T = r_T over the separator tree, r_T already reduced by the subdomains
// (the interface right-hand side kernel).  Forward, level by level upward: a
// row of level l becomes y_i = r_i - sum_c E_c[m, :] y_c over the separator
// nodes c below it whose struct holds it (level 1 rows have none), in place in
// r_T.  Backward, level by level downward: the rows of node n become
// x = Z_n y_n - E_n^T x_struct(n), stored as the solution and copied to the
// slots of the subdomains and nodes that read them.  With a done flag
// (nullable) a launch after the loop has stopped exits at once.
__device__ __forceinline__ void b_sep_fwd(SolveArgs Sv, int lvl, int bid, const int* __restrict__ done) {
  __shared__ int stop_s;
  if (threadIdx.x == 0) stop_s = done ? *done : 0;
  __syncthreads();
  if (stop_s) return;
  const int lane = threadIdx.x & 63;
  const int r = Sv.lev_row[lvl - 1] + ((bid * (int)blockDim.x + (int)threadIdx.x) >> 6);
  if (r >= Sv.lev_row[lvl]) return;
  const int nT = Sv.nT;
  const FRow fr = Sv.frow[r];
  const int nseg = wave_uniform(fr.nseg);
  const double* __restrict__ Er = Sv.FE + wave_uniform(fr.off);
  // lane g < nseg holds segment g: where it starts in the concatenated row and
  // the shift from a row entry to its source row of y (lanes past the last
  // segment start at INT_MAX and are never chosen)
  int len = 0, shift = 0;
  if (lane < nseg) {
    const SSeg sg = Sv.sseg[fr.seg0 + lane];
    len = sg.len;
    shift = sg.src;
  }
  int end = len;  // inclusive prefix sum of the lengths
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int v = __shfl_up(end, d, 64);
    if (lane >= d) end += v;
  }
  const int total = wave_uniform(__shfl(end, 63, 64));
  const int beg = lane < nseg ? end - len : 0x7fffffff;
  shift -= end - len;
  double a0 = 0, a1 = 0, a2 = 0;
  constexpr int C = kSepFwdChunk;
  for (int base = 0; base < total; base += 64 * C) {
    double e[C], y[C][3];
    int q[C];
#pragma unroll
    for (int i = 0; i < C; ++i) {
      const int k = min(base + lane + 64 * i, total - 1);
      int g = 0;  // the last segment starting at or before k
#pragma unroll
      for (int st = 32; st >= 1; st >>= 1) {
        const int b = __shfl(beg, g + st, 64);
        if (b <= k) g += st;
      }
      q[i] = __shfl(shift, g, 64) + k;
      e[i] = Er[k];
    }
#pragma unroll
    for (int i = 0; i < C; ++i)
#pragma unroll
      for (int a = 0; a < 3; ++a) y[i][a] = Sv.rT[a * nT + q[i]];
#pragma unroll
    for (int i = 0; i < C; ++i) {
      const double c = (base + lane + 64 * i < total) ? e[i] : 0.0;
      a0 += c * y[i][0];
      a1 += c * y[i][1];
      a2 += c * y[i][2];
    }
  }
  a0 = wave_sum(a0);
  a1 = wave_sum(a1);
  a2 = wave_sum(a2);
  if (lane == 0) {
    Sv.rT[r] -= a0;
    Sv.rT[nT + r] -= a1;
    Sv.rT[2 * nT + r] -= a2;
  }
}

__device__ __forceinline__ void b_sep_back(VertArgs Vx, SolveArgs Sv, int lvl, double* __restrict__ out, int bid,
                                           const int* __restrict__ done) {
  __shared__ double ys[3 * kSepTile];
  __shared__ int stop_s;
  constexpr int RW = kSepRowsPerWave;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const SepBlk bk = Sv.sblk[Sv.lev_blk[lvl - 1] + bid];
  const SepNode nd = Sv.sep[bk.node];
  const int s = nd.s, L = nd.s + nd.b, nT = Sv.nT, ni = Sv.n_irows, nv = Vx.nv;
  const bool wide = bk.pad != 0;  // block-uniform
  // this wave's rows: RW consecutive rows in a narrow block, one in a wide one
  const int rw0 = wide ? bk.row0 + wave : bk.row0 + wave * RW;
  const int nrw = wide ? (wave < bk.nrows ? 1 : 0) : max(0, min(RW, bk.nrows - wave * RW));
  if (threadIdx.x == 0) stop_s = done ? *done : 0;
  // copy slots of the wave's rows, requested before the walk: lanes 0..7 the
  // row's subdomain couplings, lanes 8.. its separator segments (-1: none)
  int slot[RW];
#pragma unroll
  for (int j = 0; j < RW; ++j) {
    slot[j] = -1;
    if (j < nrw) {
      const int rj = rw0 + j;
      const int nc = Sv.erow[rj].n;
      const FRow fr = Sv.frow[rj];
      if (lane < kMaxCoup) {
        if (lane < nc) slot[j] = Sv.cpl[rj * kMaxCoup + lane].pos;
      } else if (lane - kMaxCoup < fr.nseg) {
        slot[j] = Sv.sseg[fr.seg0 + lane - kMaxCoup].slot;
      }
    }
  }
  const double* __restrict__ Zb = Sv.ZE + nd.zoff + (long long)(rw0 - nd.r0) * L;
  double acc[RW][3];
#pragma unroll
  for (int j = 0; j < RW; ++j) acc[j][0] = acc[j][1] = acc[j][2] = 0.0;
  for (int t0 = 0; t0 < L; t0 += kSepTile) {
    const int tl = min(kSepTile, L - t0);
    __syncthreads();
    for (int i = threadIdx.x; i < tl; i += blockDim.x) {
      const int k = t0 + i;
#pragma unroll
      for (int a = 0; a < 3; ++a)
        ys[a * kSepTile + i] = k < s ? Sv.rT[a * nT + nd.r0 + k] : Sv.xsT[a * ni + nd.xs0 + (k - s)];
    }
    __syncthreads();
    if (stop_s) return;
    if (wide) {
      if (nrw > 0) {
        constexpr int C = kTopChunk;
        for (int base = 0; base < tl; base += 64 * C) {
          double z[C];
#pragma unroll
          for (int i = 0; i < C; ++i) z[i] = Zb[t0 + min(base + lane + 64 * i, tl - 1)];
#pragma unroll
          for (int i = 0; i < C; ++i) {
            const int u = base + lane + 64 * i;
            const double c = u < tl ? z[i] : 0.0;
            const int q = min(u, tl - 1);
            acc[0][0] += c * ys[q];
            acc[0][1] += c * ys[kSepTile + q];
            acc[0][2] += c * ys[2 * kSepTile + q];
          }
        }
      }
    } else {
      // every trip requests the chunk of all the wave's rows before it adds any
      constexpr int C = kSepChunk;
      for (int base = 0; base < tl; base += 64 * C) {
        double z[RW][C];
#pragma unroll
        for (int j = 0; j < RW; ++j)
          if (j < nrw)
#pragma unroll
            for (int i = 0; i < C; ++i) z[j][i] = Zb[(long long)j * L + t0 + min(base + lane + 64 * i, tl - 1)];
#pragma unroll
        for (int j = 0; j < RW; ++j)
          if (j < nrw)
#pragma unroll
            for (int i = 0; i < C; ++i) {
              const int u = base + lane + 64 * i;
              const double c = u < tl ? z[j][i] : 0.0;
              const int q = min(u, tl - 1);
              acc[j][0] += c * ys[q];
              acc[j][1] += c * ys[kSepTile + q];
              acc[j][2] += c * ys[2 * kSepTile + q];
            }
      }
    }
  }
#pragma unroll
  for (int j = 0; j < RW; ++j) {
    if (j >= nrw) break;
    const double x0 = wave_sum(acc[j][0]), x1 = wave_sum(acc[j][1]), x2 = wave_sum(acc[j][2]);
    const int gi = Sv.nB + rw0 + j;
    if (lane == 0) {
      out[gi] = x0;
      out[nv + gi] = x1;
      out[2 * nv + gi] = x2;
    }
    if (slot[j] >= 0) {
      Sv.xsT[slot[j]] = x0;
      Sv.xsT[ni + slot[j]] = x1;
      Sv.xsT[2 * ni + slot[j]] = x2;
    }
  }
}

__global__ void __launch_bounds__(kBlock) k_sep_fwd(SolveArgs Sv, int lvl, const int* __restrict__ done) {
  b_sep_fwd(Sv, lvl, blockIdx.x, done);
}

__global__ void __launch_bounds__(kBlock) k_sep_back(VertArgs Vx, SolveArgs Sv, int lvl, double* __restrict__ out,
                                                     const int* __restrict__ done) {
  b_sep_back(Vx, Sv, lvl, out, blockIdx.x, done);
}

// Anderson append of one forward iteration for the free row my_row (-1: no
// row): g = q^ - q^k, the new difference columns (Eqs. aa_dG, aa_dQ) and the
// block's Gram partial sums.  xo = q^ of the row, u0 = q^k, u1 = g of the last
// iteration, u2 = q of the last iteration; aa = the ring state of parity k;
// lane0: only lane 0 of each wave has a row (block-uniform).  Every thread of
// the block calls it.
template <int M>
__device__ __forceinline__ void aa_append(const StepState& St, const RedArgs& R, int nv, int bid, int my_row,
                                          const double (&xo)[3], const double (&u0)[3], const double (&u1)[3],
                                          const double (&u2)[3], const int (&aa)[4], bool lane0 = false) {
  int nonempty, nc, head, slot_new;
  aa_layout(aa, M, nonempty, nc, head, slot_new);
  // Gram partial sums, compact layout: G[j][l] at j*M + l, rhs[j] at M*M + j
  constexpr int NA = M * M + M;
  double part[NA];
#pragma unroll
  for (int j = 0; j < NA; ++j) part[j] = 0.0;
  if (my_row >= 0) {
    const int i = my_row;
    double col[3][M];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int j = 0; j < M; ++j) {
        int slot = head + j;
        if (slot >= M) slot -= M;
        col[a][j] = (j < nc) ? St.dG[((size_t)slot * 3 + a) * nv + i] : 0.0;
      }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int ix = a * nv + i;
      const double qc = u0[a];
      const double g = xo[a] - qc;
      if (slot_new >= 0) {
        const size_t cix = ((size_t)slot_new * 3 + a) * nv + i;
        const double dg = g - u1[a];
        St.dG[cix] = dg;
        St.dQ[cix] = qc - u2[a];
        // the new column enters the Gram sums at its position in the window
#pragma unroll
        for (int j = 0; j < M; ++j) {
          int slot = head + j;
          if (slot >= M) slot -= M;
          if (j < nc && slot == slot_new) col[a][j] = dg;
        }
      }
      St.g_last[ix] = g;
      St.q_last[ix] = qc;
#pragma unroll
      for (int j = 0; j < M; ++j) {
#pragma unroll
        for (int l = 0; l < M; ++l)
          if (l >= j) part[j * M + l] += col[a][j] * col[a][l];
        part[M * M + j] += col[a][j] * g;
      }
    }
  }
  __shared__ double red[16 * NA];
  block_sum<NA>(part, red, lane0);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int j = 0; j < M; ++j) {
#pragma unroll
      for (int l = 0; l < M; ++l) part_value(R, kRedAA, j * M + l)[bid] = (j <= l) ? part[j * M + l] : part[l * M + j];
      part_value(R, kRedAA, M * M + j)[bid] = part[M * M + j];
    }
  }
}

// ---------------------------------------------------------------- subdomain solve
// x_s = Z_s rhs_s - E_s^T x_T on the subdomain rows (one wave per row), then
// the per-vertex work of each mode on every free row (the lane 0 of a
// subdomain row's wave, or one thread per interface row):
//  forward: g = q^ - q^k, the Anderson difference columns (Eqs. aa_dG, aa_dQ)
//           and the Gram partial sums of the mixing;
//  PCG:     the right-hand side is r - alpha w (formed on the fly); the
//           solution is z; r <- r - alpha w, mu <- mu + alpha p, partial
//           r.z, |z|^2, |mu|^2;
//  PCG start: partial r.z, |z|^2, |mu|^2 of the first solve;
//  fixed point: partial |z - mu|^2, |z|^2, then mu <- z.
// Everything a thread needs that does not depend on the row descriptors is
// requested together with them.
// The subdomain solve's LDS staging buffers (right-hand-side rows, then
// interface copies, three axes each): one allocation per kernel, shared by
// every instantiation a batched kernel dispatches between.
__device__ __forceinline__ double* bottom_stage_lds() {
  __shared__ double buf[3 * (kStageZ + kStageE)];
  return buf;
}

template <int MODE, int M>
__device__ __forceinline__ void b_bottom(VertArgs Vx, SolveArgs Sv, StepState St, AdjState A, RedArgs R,
                                                   const double* __restrict__ rhs, double* __restrict__ out, int k, int bid) {
  const int nv = Vx.nv, nB = Sv.nB, nf = Vx.nf;
  const int lane = threadIdx.x & 63;
  constexpr int RW = kBottomRowsPerWave;
  const int n_sub_blocks = (nB + kBottomRows - 1) / kBottomRows;
  const bool sub_block = (int)bid < n_sub_blocks;
  // rows v0 .. v0 + RW - 1 of this wave; lane j < RW owns row v0 + j
  const int v0 = bid * kBottomRows + (threadIdx.x >> 6) * RW;
  int my_row = -1;
  if (sub_block) {
    if (lane < RW && v0 + lane < nB) my_row = v0 + lane;
  } else {
    const int i = nB + (bid - n_sub_blocks) * blockDim.x + threadIdx.x;
    if (i < nf) my_row = i;
  }
  const bool have_row = sub_block && my_row >= 0;  // this lane owns a subdomain row
  const bool iface = my_row >= nB;
  constexpr bool kPCG = (MODE == kModePCG || MODE == kModePCGSolve);
  const double* __restrict__ src = (MODE == kModeFwd) ? St.b_cur : (kPCG ? r_cur(A, k) : rhs);
  const double* __restrict__ wv = A.w;
  double* dst = (MODE == kModeFwd) ? St.qhat : out;
  const int* done = (MODE == kModeFwd || MODE == kModePlain) ? St.done : A.done;
  // ---- first round of loads: lane j fetches the descriptors of row v0 + j
  BRow br = {0, 0, 0, 0};
  BOff bo = {0, 0};
  BStage bst = {0, 0, 0, 0};
  if (have_row) {
    br = Sv.brow[my_row];
    bo = Sv.boff[my_row];
  }
  if (sub_block) bst = Sv.bstage[bid];
  __shared__ int flag_s;
  if (threadIdx.x == 0) flag_s = done ? *done : 0;
  // per-vertex state of my_row (x_T of an interface row comes from k_top)
  double xo[3] = {0, 0, 0};
  double u0[3] = {0, 0, 0}, u1[3] = {0, 0, 0}, u2[3] = {0, 0, 0}, u3[3] = {0, 0, 0};
  int aa[4] = {0, 0, 0, 0};
  if (MODE == kModeFwd && M > 0)
#pragma unroll
    for (int j = 0; j < 4; ++j) aa[j] = St.ctl[kCtlAA + 4 * (k & 1) + j];
  if (my_row >= 0) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int ix = a * nv + my_row;
      if (iface) xo[a] = dst[ix];
      if (MODE == kModeFwd && M > 0) {
        u0[a] = St.q_cur[ix];
        u1[a] = St.g_last[ix];
        u2[a] = St.q_last[ix];
      } else if (kPCG) {
        u0[a] = src[ix];
        u1[a] = A.p[ix];
        u2[a] = wv[ix];
        u3[a] = A.mu[ix];
      } else if (MODE == kModePCGInit) {
        u0[a] = rhs[ix];
        u1[a] = A.mu[ix];
      } else if (MODE == kModeFixed) {
        u1[a] = A.mu[ix];
      }
    }
  }
  // alpha = (r.z)/(p.w): both totals were stored by k_Eb's block 0 and earlier
  const double rz = kPCG ? fin_site(R, kRedRZ0 + (k & 1))[0] : 0.0;
  const double pwt = kPCG ? fin_site(R, kRedPW)[0] : 1.0;
  __syncthreads();
  if (flag_s) return;
  const double alpha = rz / pwt;
  // the descriptors of the wave's rows, wave-uniform (ns = 0 for a row past nB)
  int ns[RW], nI[RW], b0[RW], ir0[RW];
  long long zs[RW], et[RW];
#pragma unroll
  for (int j = 0; j < RW; ++j) {
    ns[j] = wave_uniform(__shfl(br.ns, j, 64));
    nI[j] = wave_uniform(__shfl(br.nI, j, 64));
    b0[j] = wave_uniform(__shfl(br.b0, j, 64));
    ir0[j] = wave_uniform(__shfl(br.ir0, j, 64));
    zs[j] = wave_uniform(__shfl(bo.zs, j, 64));
    et[j] = wave_uniform(__shfl(bo.et, j, 64));
  }
  const int ni = Sv.n_irows;
  // each trip of a row walk takes 64 x kBottomChunk entries of Z_s[v, :]
  // (against the right-hand side) and 64 x kBottomChunkE of E_s^T[v, :]
  // (against x_T(s)); entries past a part's end repeat its last entry with
  // weight zero
  constexpr int kSpan = 64 * kBottomChunk, kSpanE = 64 * kBottomChunkE;
  int tz[RW], te[RW], tmax = 0;
#pragma unroll
  for (int j = 0; j < RW; ++j) {
    tz[j] = (ns[j] + kSpan - 1) / kSpan;
    te[j] = (nI[j] + kSpanE - 1) / kSpanE;
    tmax = max(tmax, max(tz[j], te[j]));
  }
  // ---- staging: the block's rows share one or a few subdomains, so it stages
  // their right-hand-side rows (r - alpha w in PCG) and interface copies in LDS
  // once instead of every row reading them from memory.  Blocks whose ranges
  // exceed the buffers (zn = 0) read them in the row walk instead.
  double* sz = bottom_stage_lds();
  double* se = sz + 3 * kStageZ;
  const bool staged = sub_block && bst.zn > 0;  // block-uniform
  if (staged) {
    constexpr int kPZ = (kStageZ + kBottomThreads - 1) / kBottomThreads;
    constexpr int kPE = (kStageE + kBottomThreads - 1) / kBottomThreads;
    double vz[kPZ][3], ve[kPE][3];
#pragma unroll
    for (int j = 0; j < kPZ; ++j) {
      const int i = min((int)threadIdx.x + j * kBottomThreads, bst.zn - 1);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const int ix = a * nv + bst.z0 + i;
        vz[j][a] = kPCG ? src[ix] - alpha * wv[ix] : src[ix];
      }
    }
    if (bst.en > 0)
#pragma unroll
      for (int j = 0; j < kPE; ++j) {
        const int i = min((int)threadIdx.x + j * kBottomThreads, bst.en - 1);
#pragma unroll
        for (int a = 0; a < 3; ++a) ve[j][a] = Sv.xsT[a * ni + bst.e0 + i];
      }
#pragma unroll
    for (int j = 0; j < kPZ; ++j) {
      const int i = (int)threadIdx.x + j * kBottomThreads;
      if (i < bst.zn)
#pragma unroll
        for (int a = 0; a < 3; ++a) sz[a * kStageZ + i] = vz[j][a];
    }
    if (bst.en > 0)
#pragma unroll
      for (int j = 0; j < kPE; ++j) {
        const int i = (int)threadIdx.x + j * kBottomThreads;
        if (i < bst.en)
#pragma unroll
          for (int a = 0; a < 3; ++a) se[a * kStageE + i] = ve[j][a];
      }
  }
  __syncthreads();
  // ---- the subdomain rows: x_v = Z_s[v, :] rhs_s - E_s^T[v, :] x_T(s)
  double acc[RW][3];
#pragma unroll
  for (int j = 0; j < RW; ++j) acc[j][0] = acc[j][1] = acc[j][2] = 0.0;
  if (sub_block && staged) {
    // every trip requests the chunk of all the wave's rows before it adds any
    // (per row the same per-lane order of terms as a walk of that row alone);
    // the right-hand side and x_T(s) come from LDS
    for (int t = 0; t < tmax; ++t) {
      double cz[RW][kBottomChunk], ce[RW][kBottomChunkE];
#pragma unroll
      for (int j = 0; j < RW; ++j) {
        const double* __restrict__ Zr = Sv.Zs + zs[j];
        const double* __restrict__ Er = Sv.Et + et[j];
        if (t < tz[j])
#pragma unroll
          for (int i = 0; i < kBottomChunk; ++i) cz[j][i] = Zr[min(t * kSpan + lane + 64 * i, ns[j] - 1)];
        if (t < te[j])
#pragma unroll
          for (int i = 0; i < kBottomChunkE; ++i) ce[j][i] = Er[min(t * kSpanE + lane + 64 * i, nI[j] - 1)];
      }
#pragma unroll
      for (int j = 0; j < RW; ++j) {
        const int zo = b0[j] - bst.z0, eo = ir0[j] - bst.e0;
        if (t < tz[j])
#pragma unroll
          for (int i = 0; i < kBottomChunk; ++i) {
            const int u = t * kSpan + lane + 64 * i;
            const double c = (u < ns[j]) ? cz[j][i] : 0.0;
            const int q = zo + min(u, ns[j] - 1);
            acc[j][0] += c * sz[q];
            acc[j][1] += c * sz[kStageZ + q];
            acc[j][2] += c * sz[2 * kStageZ + q];
          }
        if (t < te[j])
#pragma unroll
          for (int i = 0; i < kBottomChunkE; ++i) {
            const int p = t * kSpanE + lane + 64 * i;
            const double c = (p < nI[j]) ? ce[j][i] : 0.0;
            const int q = eo + min(p, nI[j] - 1);
            acc[j][0] -= c * se[q];
            acc[j][1] -= c * se[kStageE + q];
            acc[j][2] -= c * se[2 * kStageE + q];
          }
      }
    }
  } else if (sub_block) {
    // one row at a time, the right-hand side and x_T(s) read in the walk
#pragma unroll
    for (int j = 0; j < RW; ++j) {
      const double* __restrict__ Zr = Sv.Zs + zs[j];
      const double* __restrict__ Er = Sv.Et + et[j];
      const double* __restrict__ x0 = Sv.xsT + ir0[j];
      const double* __restrict__ s0 = src + b0[j];
      const double* __restrict__ w0 = wv + b0[j];
      const int nsj = ns[j], nIj = nI[j];
      double a0 = 0, a1 = 0, a2 = 0;
      double cz[kBottomChunk], yz[kBottomChunk][3], wz[kBottomChunk][3];
      double ce[kBottomChunkE], ye[kBottomChunkE][3];
      auto load_z = [&](int t) {
#pragma unroll
        for (int i = 0; i < kBottomChunk; ++i) {
          const unsigned o = 8u * (unsigned)min(t * kSpan + lane + 64 * i, nsj - 1);
          cz[i] = at_byte(Zr, o);
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            yz[i][a] = at_byte(s0 + a * nv, o);
            if (kPCG) wz[i][a] = at_byte(w0 + a * nv, o);
          }
        }
      };
      auto load_e = [&](int t) {
#pragma unroll
        for (int i = 0; i < kBottomChunkE; ++i) {
          const unsigned o = 8u * (unsigned)min(t * kSpanE + lane + 64 * i, nIj - 1);
          ce[i] = at_byte(Er, o);
#pragma unroll
          for (int a = 0; a < 3; ++a) ye[i][a] = at_byte(x0 + a * ni, o);
        }
      };
      auto add_z = [&](int t) {  // r - alpha w on the subdomain entries
#pragma unroll
        for (int i = 0; i < kBottomChunk; ++i) {
          const double c = (t * kSpan + lane + 64 * i < nsj) ? cz[i] : 0.0;
          a0 += c * (kPCG ? yz[i][0] - alpha * wz[i][0] : yz[i][0]);
          a1 += c * (kPCG ? yz[i][1] - alpha * wz[i][1] : yz[i][1]);
          a2 += c * (kPCG ? yz[i][2] - alpha * wz[i][2] : yz[i][2]);
        }
      };
      auto add_e = [&](int t) {
#pragma unroll
        for (int i = 0; i < kBottomChunkE; ++i) {
          const double c = (t * kSpanE + lane + 64 * i < nIj) ? ce[i] : 0.0;
          a0 -= c * ye[i][0];
          a1 -= c * ye[i][1];
          a2 -= c * ye[i][2];
        }
      };
      // trips over both parts (all loads of a trip before its arithmetic), then
      // the longer part alone; the trip counts are wave-uniform
      const int both = min(tz[j], te[j]);
      for (int t = 0; t < both; ++t) {
        load_z(t);
        load_e(t);
        add_z(t);
        add_e(t);
      }
      for (int t = both; t < tz[j]; ++t) {
        load_z(t);
        add_z(t);
      }
      for (int t = both; t < te[j]; ++t) {
        load_e(t);
        add_e(t);
      }
      acc[j][0] = a0;
      acc[j][1] = a1;
      acc[j][2] = a2;
    }
  }
  if (sub_block) {
#pragma unroll
    for (int j = 0; j < RW; ++j) {
      const double x0 = wave_sum(acc[j][0]), x1 = wave_sum(acc[j][1]), x2 = wave_sum(acc[j][2]);
      if (lane == j) {
        xo[0] = x0;
        xo[1] = x1;
        xo[2] = x2;
      }
    }
    if (have_row) {
      dst[my_row] = xo[0];
      dst[nv + my_row] = xo[1];
      dst[2 * nv + my_row] = xo[2];
    }
  }
  if (MODE == kModePlain) return;
  // ---- per-vertex work
  if (MODE == kModeFwd) {
    if constexpr (M > 0) aa_append<M>(St, R, nv, bid, my_row, xo, u0, u1, u2, aa, sub_block && RW == 1);
  } else {
    double v3[3] = {0, 0, 0};
    if (my_row >= 0) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const int ix = a * nv + my_row;
        const double x = xo[a];
        if (kPCG) {
          const double rn = u0[a] - alpha * u2[a];
          const double mn = u3[a] + alpha * u1[a];
          r_cur(A, k + 1)[ix] = rn;
          A.mu[ix] = mn;
          v3[0] += rn * x;
          v3[1] += x * x;
          v3[2] += mn * mn;
        } else if (MODE == kModePCGInit) {
          v3[0] += u0[a] * x;
          v3[1] += x * x;
          v3[2] += u1[a] * u1[a];
        } else {  // fixed point
          const double mo = u1[a];
          v3[0] += (x - mo) * (x - mo);
          v3[1] += x * x;
          A.mu[ix] = x;
        }
      }
    }
    if (MODE == kModeFixed) {
      write_partial<3>(v3, R, kRedFix, bid, sub_block && RW == 1);
    } else if (MODE != kModePCGSolve) {
      // PCG sums of iteration k land in the parity slot read by iteration k + 1
      const int slot = (MODE == kModePCGInit) ? 0 : ((k + 1) & 1);
      write_partial<3>(v3, R, kRedRZ0 + slot, bid, sub_block && RW == 1);
    }
  }
}

template <int MODE, int M>
__global__ void __launch_bounds__(kBottomThreads) PD_ROW_WALK k_bottom(VertArgs Vx, SolveArgs Sv, StepState St, AdjState A, RedArgs R,
                                                   const double* __restrict__ rhs, double* __restrict__ out, int k) {
  b_bottom<MODE, M>(Vx, Sv, St, A, R, rhs, out, k, blockIdx.x);
}


// ---------------------------------------------------------------- contact corrections
// The contact rows' correction of a solve, sum_c s_c a_{v_c}[row] per axis,
// with s_c = lam_c n_c (forward, Eq. q_update) or u_c n_c (adjoint
// projection); rows with s_c = 0 are skipped.  The row data sit in LDS.
struct ContactLds {
  double s[3 * kMaxAdjRows];
  int slot[kMaxAdjRows];
  int v[kMaxAdjRows];
};

__device__ __forceinline__ void contact_lds_load(const ContactArgs& C, ContactLds& L) {
  for (int c = threadIdx.x; c < C.K; c += blockDim.x) {
    L.s[3 * c] = C.s[3 * c];
    L.s[3 * c + 1] = C.s[3 * c + 1];
    L.s[3 * c + 2] = C.s[3 * c + 2];
    L.slot[c] = C.slot[c];
    L.v[c] = C.v[c];
  }
}

// The rows go in chunks: a chunk's column entries are requested together (rows
// past the end repeat the last one), then added in row order.
__device__ __forceinline__ void contact_correction(const ContactArgs& C, const ContactLds& L, int row, double (&x)[3]) {
  constexpr int kChunk = 8;
  const size_t nf = C.nf;
  for (int c0 = 0; c0 < C.K; c0 += kChunk) {
    double a[kChunk];
#pragma unroll
    for (int j = 0; j < kChunk; ++j) a[j] = C.cols[(size_t)L.slot[min(c0 + j, C.K - 1)] * nf + row];
#pragma unroll
    for (int j = 0; j < kChunk; ++j) {
      const int c = c0 + j;
      if (c >= C.K) continue;
      const double s0 = L.s[3 * c], s1 = L.s[3 * c + 1], s2 = L.s[3 * c + 2];
      if (s0 == 0.0 && s1 == 0.0 && s2 == 0.0) continue;
      x[0] += s0 * a[j];
      x[1] += s1 * a[j];
      x[2] += s2 * a[j];
    }
  }
}

// Forward: q^ += sum_c lam_c a_{v_c} n_c on every free row, then the Anderson
// append of the corrected q^ (one thread per free row).
template <int M>
__global__ void __launch_bounds__(kBlock) k_contact_apply_fwd(VertArgs Vx, StepState St, RedArgs R, ContactArgs C,
                                                              int k) {
  __shared__ ContactLds L;
  __shared__ int flag_s;
  const int nv = Vx.nv, nf = Vx.nf;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int my_row = i < nf ? i : -1;
  double xo[3] = {0, 0, 0}, u0[3] = {0, 0, 0}, u1[3] = {0, 0, 0}, u2[3] = {0, 0, 0};
  int aa[4] = {0, 0, 0, 0};
  if (M > 0)
#pragma unroll
    for (int j = 0; j < 4; ++j) aa[j] = St.ctl[kCtlAA + 4 * (k & 1) + j];
  if (my_row >= 0)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int ix = a * nv + my_row;
      xo[a] = St.qhat[ix];
      if (M > 0) {
        u0[a] = St.q_cur[ix];
        u1[a] = St.g_last[ix];
        u2[a] = St.q_last[ix];
      }
    }
  if (threadIdx.x == 0) flag_s = *St.done;
  contact_lds_load(C, L);
  __syncthreads();
  if (flag_s) return;
  if (my_row >= 0) {
    contact_correction(C, L, my_row, xo);
#pragma unroll
    for (int a = 0; a < 3; ++a) St.qhat[a * nv + my_row] = xo[a];
  }
  if constexpr (M > 0) aa_append<M>(St, R, nv, blockIdx.x, my_row, xo, u0, u1, u2, aa);
}

// Adjoint: z = P r = A~^{-1} r - sum_c u_c a_{v_c} n_c (the solve already in
// A.z), and the residual loses its constraint-force part, r <- r - J_A^T u,
// so that A~ z = r holds again (the conjugate-gradient recurrences rely on
// it; P J_A^T = 0 and J_A z = 0 leave every other quantity unchanged).  Then
// the per-row work of the mode, as in the subdomain solve: PCG (r of
// iteration k + 1 was written by the solve), PCG start (rhs = r0), fixed point.
template <int MODE>
__global__ void __launch_bounds__(kBlock) k_contact_apply_adj(VertArgs Vx, AdjState A, RedArgs R, ContactArgs C,
                                                              const double* __restrict__ rhs, int k) {
  __shared__ ContactLds L;
  __shared__ int flag_s;
  const int nv = Vx.nv, nf = Vx.nf;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int my_row = i < nf ? i : -1;
  double* rr = (MODE == kModePCG) ? r_cur(A, k + 1) : A.r0;
  double z[3] = {0, 0, 0}, r[3] = {0, 0, 0}, m[3] = {0, 0, 0};
  if (my_row >= 0)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int ix = a * nv + my_row;
      z[a] = A.z[ix];
      if (MODE != kModeFixed) r[a] = rr[ix];
      m[a] = A.mu[ix];
    }
  if (threadIdx.x == 0) flag_s = *A.done;
  contact_lds_load(C, L);
  __syncthreads();
  if (flag_s) return;
  double v3[3] = {0, 0, 0};
  if (my_row >= 0) {
    double corr[3] = {0, 0, 0};
    contact_correction(C, L, my_row, corr);
    bool on_contact = false;
    double f[3] = {0, 0, 0};
    for (int c = 0; c < C.K; ++c)
      if (L.v[c] == my_row) {
        on_contact = true;
        f[0] += L.s[3 * c];
        f[1] += L.s[3 * c + 1];
        f[2] += L.s[3 * c + 2];
      }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int ix = a * nv + my_row;
      const double x = z[a] - corr[a];
      A.z[ix] = x;
      if (MODE == kModeFixed) {
        v3[0] += (x - m[a]) * (x - m[a]);
        v3[1] += x * x;
        A.mu[ix] = x;
      } else {
        const double rn = r[a] - f[a];
        if (on_contact) rr[ix] = rn;
        v3[0] += rn * x;
        v3[1] += x * x;
        v3[2] += m[a] * m[a];
      }
    }
  }
  if (MODE == kModeFixed) write_partial<3>(v3, R, kRedFix, blockIdx.x);
  else write_partial<3>(v3, R, kRedRZ0 + ((MODE == kModePCGInit) ? 0 : ((k + 1) & 1)), blockIdx.x);
}

// ---------------------------------------------------------------- step epilogue
// q_{t+h} = q*, v_{t+h} = (q* - q_t) / h in the caller's order; checkpoint
// record {q_t, q~, q*, q*-1} in library order.
__device__ PD_VERT_BODY void b_epilogue(const VertArgs& Vx, const StepState& St, double* __restrict__ q_next,
                                           double* __restrict__ v_next, double* __restrict__ ckpt, int bid) {
  const int i = bid * blockDim.x + threadIdx.x;
  const int nv = Vx.nv;
  if (i >= nv) return;
  const int o = Vx.v_orig[i];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int ix = a * nv + i;
    const double q = St.q_cur[ix];
    const double qt = St.qt[ix];
    if (q_next) q_next[3 * o + a] = q;
    if (v_next) v_next[3 * o + a] = (i < Vx.nf) ? (q - qt) / Vx.h : 0.0;
    if (ckpt) {
      ckpt[ix] = qt;
      ckpt[3 * nv + ix] = St.qtil[ix];
      ckpt[6 * nv + ix] = q;
      ckpt[9 * nv + ix] = St.q_prev[ix];
    }
  }
}

__global__ void __launch_bounds__(kBlock) k_epilogue(VertArgs Vx, StepState St, double* __restrict__ q_next,
                                                     double* __restrict__ v_next, double* __restrict__ ckpt) {
  b_epilogue(Vx, St, q_next, v_next, ckpt, blockIdx.x);
}

// ---------------------------------------------------------------- layout conversion
__device__ PD_VERT_BODY void b_to_lib(const VertArgs& Vx, const double* __restrict__ user, double* __restrict__ lib,
                                         int free_only, int bid) {
  const int i = bid * blockDim.x + threadIdx.x;
  if (i >= Vx.nv) return;
  const int o = Vx.v_orig[i];
  const bool zero = free_only && i >= Vx.nf;
#pragma unroll
  for (int a = 0; a < 3; ++a) lib[a * Vx.nv + i] = zero ? 0.0 : user[3 * o + a];
}

__global__ void __launch_bounds__(kBlock) k_to_lib(VertArgs Vx, const double* __restrict__ user, double* __restrict__ lib,
                                                   int free_only) {
  b_to_lib(Vx, user, lib, free_only, blockIdx.x);
}

__global__ void __launch_bounds__(kBlock) k_from_lib(VertArgs Vx, const double* __restrict__ lib, double* __restrict__ user,
                                                     int free_only) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Vx.nv) return;
  const int o = Vx.v_orig[i];
  const bool zero = free_only && i >= Vx.nf;
#pragma unroll
  for (int a = 0; a < 3; ++a) user[3 * o + a] = zero ? 0.0 : lib[a * Vx.nv + i];
}

// ================================================================= backward
// Trust-region ratio sums (Eqs. tr_step, tr_decreases): per tet
// V_e (psi_e(F(q*-1)) - psi_e(F(q*))) and (w_e + beta_e/h) V_e |G_e dq|^2;
// per free vertex m/(2h^2) (a - b).(a + b - 2 q~) and (1 + alpha h) m/h^2 |dq|^2.
__device__ PD_SHARED_BODY void b_tr_partials(const ElemArgs& E, const VertArgs& Vx, const RedArgs& R,
                                              const double* __restrict__ ck, int n_tet_blocks, int bid) {
  const int nv = Vx.nv;
  const double* qtil = ck + 3 * nv;
  const double* qs = ck + 6 * nv;
  const double* qm = ck + 9 * nv;
  double v[2] = {0.0, 0.0};
  if ((int)bid < n_tet_blocks) {
    const int t = bid * blockDim.x + threadIdx.x;
    if (t < E.ne) {
      double Fa[9], Fb[9];
      int vi[4];
      load_F(E, qm, nv, t, Fa, vi);
      load_F(E, qs, nv, t, Fb, vi);
      const double Ja = Fa[0] * (Fa[4] * Fa[8] - Fa[5] * Fa[7]) - Fa[1] * (Fa[3] * Fa[8] - Fa[5] * Fa[6]) +
                        Fa[2] * (Fa[3] * Fa[7] - Fa[4] * Fa[6]);
      const double Jb = Fb[0] * (Fb[4] * Fb[8] - Fb[5] * Fb[7]) - Fb[1] * (Fb[3] * Fb[8] - Fb[5] * Fb[6]) +
                        Fb[2] * (Fb[3] * Fb[7] - Fb[4] * Fb[6]);
      double d = 0.0, gg = 0.0;
#pragma unroll
      for (int j = 0; j < 9; ++j) gg += (Fb[j] - Fa[j]) * (Fb[j] - Fa[j]);
      if (Ja > 0.0 && Jb > 0.0) {
        double Ia = 0.0, Ib = 0.0;
#pragma unroll
        for (int j = 0; j < 9; ++j) {
          Ia += Fa[j] * Fa[j];
          Ib += Fb[j] * Fb[j];
        }
        const double la = log(Ja), lb = log(Jb);
        d = 0.5 * E.muV[t] * (Ia - Ib) - E.muV[t] * (la - lb) + 0.5 * E.lamV[t] * (la * la - lb * lb);
      } else {
        d = (Ja > 0.0) ? -INFINITY : INFINITY;
      }
      v[0] = d;
      v[1] = (E.wV[t] + E.bV[t]) * gg;
      if (E.mus) {
        // the fibre's energy difference and its part of |dq|_A^2: w_m V_e |(Fb - Fa) m|^2
        double m[3], wm, dF[9], y[3];
        fibre_of(E, t, m, wm);
#pragma unroll
        for (int j = 0; j < 9; ++j) dF[j] = Fb[j] - Fa[j];
        mat_vec_m(dF, m, y);
        v[0] += muscle_energy(E, t, Fa) - muscle_energy(E, t, Fb);
        v[1] += wm * (y[0] * y[0] + y[1] * y[1] + y[2] * y[2]);
      }
    }
  } else {
    const int i = (bid - n_tet_blocks) * blockDim.x + threadIdx.x;
    if (i < Vx.nf) {
      const double m = Vx.mass[i], h = Vx.h;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const int ix = a * nv + i;
        const double Aq = qm[ix], Bq = qs[ix];
        v[0] += 0.5 / (h * h) * m * (Aq - Bq) * (Aq + Bq - 2.0 * qtil[ix]);
        v[1] += (1.0 + Vx.alpha * h) * m / (h * h) * (Bq - Aq) * (Bq - Aq);
      }
    }
  }
  write_partial<2>(v, R, kRedTR, bid);
}

__global__ void __launch_bounds__(kBlock) k_tr_partials(ElemArgs E, VertArgs Vx, RedArgs R, const double* __restrict__ ck,
                                                        int n_tet_blocks) {
  b_tr_partials(E, Vx, R, ck, n_tet_blocks, blockIdx.x);
}

// rho = dPhi_act / dPhi_mod (rho = 1 when dPhi_mod < 1e-12), tau* = 1/2 when
// |rho - 1| <= eps_TR else 1 (Eqs. tr_ratio, tr_rule); then per tet the
// recomputed SVD and prox stretches at q*, and the compact filtered prox
// differential {U, V, D, c1, c2, s*} (Alg. 2 element loop).
__device__ PD_SHARED_BODY void b_bwd_elem(const ElemArgs& E, const VertArgs& Vx, const RedArgs& R,
                                           const double* __restrict__ ck, double eps_tr, double tau_force,
                                           int use_partials, double* __restrict__ jac, double* __restrict__ bstat,
                                           int* __restrict__ zero, int nzero, int bid) {
  // words cleared for the kernels that follow (the adjoint's control words);
  // nothing in this kernel reads them
  if (zero && bid == 0 && threadIdx.x < nzero) zero[threadIdx.x] = 0;
  __shared__ double tau_s;
  double tr[2] = {0.0, 0.0};
  if (use_partials) consume<2>(R, kRedTR, tr, bid);
  if (threadIdx.x == 0) {
    const double act = tr[0], mod = 0.5 * fabs(tr[1]);
    const double rho = (mod < 1e-12) ? 1.0 : act / mod;
    double tau = (fabs(rho - 1.0) <= eps_tr) ? 0.5 : 1.0;
    if (tau_force >= 0.0) tau = tau_force;
    tau_s = tau;
    if (bid == 0) {
      bstat[0] = rho;
      bstat[1] = tau;
      bstat[2] = act;
      bstat[3] = mod;
    }
  }
  __syncthreads();
  const double tau = tau_s;
  const int t = bid * blockDim.x + threadIdx.x;
  if (t >= E.ne) return;
  const int nv = Vx.nv;
  const double* qs = ck + 6 * nv;
  double F[9], U[9], V[9], sF[3], ss[3], rt[3];
  int vi[4];
  load_F(E, qs, nv, t, F, vi);
  const bool warm = load_rot(E, t, V);
  svd3(F, U, sF, V, warm);
#pragma unroll
  for (int j = 0; j < 3; ++j) rt[j] = E.rw[(size_t)j * E.ne + t];
  double D[6], c1[3], c2[3];
  double nu = rt[0];
  double sv[3];  // the volume step's stretches (energies 1 and 2)
  if (E.energy >= 1) {
    // corotated + volume, per unit of w_e = 2 mu_e + lam_e: the stretch map
    // ss = th_r + th_v sv (th_r = 2 mu_e / w_e, th_v = lam_e / w_e), whose
    // Jacobian is th_v D_vol (the rotation's stretches are constant); no
    // trust-region filter (Alg. 2 applies it to the Neo-Hookean prox).  The
    // barrier's D_vol = lam_bar (H + lam_bar I)^{-1} from its stationarity.
    double Dv[6];
    if (E.energy == 1) {
      volume_project(sF, nu, sv);
      volume_diff(sF, sv, Dv);
    } else {
      double e1[3], e2[3];
      prox_stretch_g(sF, 0.0, E.mu_bar, E.lam_bar, E.lam_bar, sv, rt);
      prox_diff_g(sF, sv, 0.0, E.mu_bar, E.lam_bar, E.lam_bar, 0.0, Dv, e1, e2);
    }
    const double wv = E.wV[t], thr = 2.0 * E.muV[t] / wv, thv = E.lamV[t] / wv;
#pragma unroll
    for (int j = 0; j < 3; ++j) ss[j] = thr + thv * sv[j];
#pragma unroll
    for (int j = 0; j < 6; ++j) D[j] = thv * Dv[j];
    pair_coeffs(sF, ss, D, c1, c2);
  } else {
    prox_stretch(sF, E.mu_bar, E.lam_bar, E.k_bar, ss, rt);
    prox_diff(sF, ss, E.mu_bar, E.lam_bar, E.k_bar, tau, D, c1, c2);
  }
  // the compact differential, U and V as unit quaternions (both are proper
  // rotations): 23 doubles per tet
  const size_t ne = E.ne;
  double qU[4], qV[4];
  quat_of_rot(U, qU);
  quat_of_rot(V, qV);
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    jac[j * ne + t] = qU[j];
    jac[(kJacV + j) * ne + t] = qV[j];
  }
#pragma unroll
  for (int j = 0; j < 6; ++j) jac[(kJacD + j) * ne + t] = D[j];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    jac[(kJacC1 + j) * ne + t] = c1[j];
    jac[(kJacC2 + j) * ne + t] = c2[j];
    jac[(kJacS + j) * ne + t] = ss[j];
  }
  if (E.mus) {
    // the fibre's differential at q*: f^ and l/|f| (zero for a passive tet or f = 0)
    double m[3], wm, f[3];
    fibre_of(E, t, m, wm);
    mat_vec_m(F, m, f);
    const double nf = sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
    const bool on = wm != 0.0 && nf > 0.0;
#pragma unroll
    for (int j = 0; j < 3; ++j) E.mjac[j * ne + t] = on ? f[j] / nf : 0.0;
    E.mjac[3 * ne + t] = on ? (1.0 - E.act[E.mgrp[t]]) / nf : 0.0;
  }
  // a reverse sweep visits q* of neighbouring steps: start the next one from here
  if (E.energy == 1)
    store_warm_nu(E, t, V, nu);
  else if (E.energy == 2)
    store_warm(E, t, V, sF, sv);
  else
    store_warm(E, t, V, sF, ss);
}

__global__ void __launch_bounds__(kBlock) k_bwd_elem(ElemArgs E, VertArgs Vx, RedArgs R, const double* __restrict__ ck,
                                                     double eps_tr, double tau_force, int use_partials,
                                                     double* __restrict__ jac, double* __restrict__ bstat,
                                                     int* __restrict__ zero, int nzero) {
  b_bwd_elem(E, Vx, R, ck, eps_tr, tau_force, use_partials, jac, bstat, zero, nzero, blockIdx.x);
}

__device__ __forceinline__ void load_jac(const double* __restrict__ jac, int ne, int t, double U[9], double V[9],
                                         double D[6], double c1[3], double c2[3]) {
  double qU[4], qV[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    qU[j] = jac[(size_t)j * ne + t];
    qV[j] = jac[(size_t)(kJacV + j) * ne + t];
  }
#pragma unroll
  for (int j = 0; j < 6; ++j) D[j] = jac[(size_t)(kJacD + j) * ne + t];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    c1[j] = jac[(size_t)(kJacC1 + j) * ne + t];
    c2[j] = jac[(size_t)(kJacC2 + j) * ne + t];
  }
  rot_of_quat(qU, U);
  rot_of_quat(qV, V);
}

// PCG scalars at the start of adjoint iteration it: convergence of the
// previous solve (|z| <= eps |mu|, the relative preconditioned residual) and
// beta = (r.z)_{it} / (r.z)_{it-1} for the direction p = z + beta p.  The done
// flag of earlier iterations is read together with the partial sums; the
// decision is block-uniform.
struct PCGCtl {
  int stop;
  double beta;
};

template <int MODE>
__device__ __forceinline__ PCGCtl adj_control(const AdjState& A, const RedArgs& R, int it, int bid) {
  __shared__ PCGCtl c;
  int flag = 0;
  double prev = 1.0;
  if (threadIdx.x == 0) {
    flag = *A.done;
    if (MODE == kModePCG && it >= 1) prev = fin_site(R, kRedRZ0 + ((it - 1) & 1))[0];
  }
  double f[3] = {0.0, 0.0, 0.0};
  if (MODE == kModePCG) consume<3>(R, kRedRZ0 + (it & 1), f, bid);
  if (MODE == kModeFixed && it >= 1) consume<3>(R, kRedFix, f, bid);
  if (threadIdx.x == 0) {
    c.stop = 0;
    c.beta = 0.0;
    double res = INFINITY;
    bool conv = false;
    if (MODE == kModePCG) {
      const double rz = f[0], zz = f[1], mm = f[2];
      res = (zz == 0.0) ? 0.0 : sqrt(zz) / sqrt(mm);
      conv = res <= A.eps;
      if (it >= 1) c.beta = rz / prev;
    } else if (MODE == kModeFixed && it >= 1) {
      res = (f[1] == 0.0) ? 0.0 : sqrt(f[0]) / sqrt(f[1]);
      conv = res <= A.eps;
    }
    const bool cap = it >= A.kmax;
    c.stop = flag || conv || cap;
    if (!flag && bid == 0) {
      A.dstat[0] = res;
      if (conv || cap) {
        *A.done = 1;
        A.ctl[0] = it;
        A.ctl[1] = conv ? 0 : 1;
        if (A.sig) {  // statistics first, then the sequence number (system-scope ordered)
          A.sigd[8] = res;
          for (int j = 0; j < 4; ++j) A.sigd[4 + j] = A.trstat[j];
          A.sig[9] = it;
          A.sig[10] = conv ? 0 : 1;
          __threadfence_system();
          A.sig[8] = A.seq;
        }
      }
    }
  }
  __syncthreads();
  PCGCtl out = c;
  __syncthreads();
  return out;
}

// Element contributions on free vertices of
//   K x = sum_e w_e V_e G_e^T (dp*/dF) G_e x               (Eq. db_dq)
// and, in the warm-start mode, of (A~ - K) x without its mass term:
//   sum_e G_e^T [(w_e + beta_e / h) V_e G_e x - w_e V_e (dp*/dF) G_e x].
// PCG forms x = p = z + beta p on the fly.  The tet's data and its compact
// differential are requested together with the control sums.
template <int MODE>
__device__ __forceinline__ void b_apply_K(ElemArgs E, VertArgs Vx, AdjState A, RedArgs R,
                                                    const double* __restrict__ jac, const double* __restrict__ x, int it, int bid) {
  const int t = bid * blockDim.x + threadIdx.x;
  const bool have = t < E.ne;
  TetData T;
  double U[9], V[9], D[6], c1[3], c2[3], wv = 0.0, bv = 0.0;
  if (have) {
    load_tet(E, t, T);
    load_jac(jac, E.ne, t, U, V, D, c1, c2);
    wv = E.wV[t];
    if (MODE == kModeAmK) bv = E.bV[t];
  }
  PCGCtl c = {0, 0.0};
  if (MODE == kModePCG || MODE == kModeFixed) c = adj_control<MODE>(A, R, it, bid);
  if (c.stop || !have) return;
  const int nv = Vx.nv, nf = Vx.nf;
  double xv[4][3];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      const int ix = ax * nv + T.vi[a];
      double val = 0.0;
      if (T.vi[a] < nf) {
        if (MODE == kModePCG) val = A.z[ix] + c.beta * A.p[ix];
        else if (MODE == kModeFixed) val = A.mu[ix];
        else val = x[ix];
      }
      xv[a][ax] = val;
    }
  double dF[9], dP[9];
  grad_of(T, xv, dF);
  prox_diff_apply(U, V, D, c1, c2, dF, dP);
  double P[9];
#pragma unroll
  for (int j = 0; j < 9; ++j) P[j] = (MODE == kModeAmK) ? (wv + bv) * dF[j] - wv * dP[j] : wv * dP[j];
  if (E.mus) {
    // the fibre: K gains w_m V_e dp m^T, dp = (l/|f|)(y - f^ (f^ . y)), y = dF m; A~ gains w_m V_e y m^T
    double m[3], wm;
    fibre_of(E, t, m, wm);
    if (wm != 0.0) {
      const size_t ne = E.ne;
      const double fh[3] = {E.mjac[t], E.mjac[ne + t], E.mjac[2 * ne + t]}, r = E.mjac[3 * ne + t];
      double y[3], dp[3];
      mat_vec_m(dF, m, y);
      const double d = fh[0] * y[0] + fh[1] * y[1] + fh[2] * y[2];
#pragma unroll
      for (int i = 0; i < 3; ++i) dp[i] = r * (y[i] - fh[i] * d);
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) P[3 * i + j] += wm * ((MODE == kModeAmK) ? y[i] - dp[i] : dp[i]) * m[j];
    }
  }
  store_GtP(T, A.contrib, E.ninc, P);
}

template <int MODE>
__global__ void __launch_bounds__(kBlock) k_apply_K(ElemArgs E, VertArgs Vx, AdjState A, RedArgs R,
                                                    const double* __restrict__ jac, const double* __restrict__ x, int it) {
  b_apply_K<MODE>(E, Vx, A, R, jac, x, it, xcd_block(blockIdx.x, gridDim.x));
}

// Gathered contributions on free vertices (8 lanes per vertex).
//  PCG:   p = z + beta p, A p = r + beta A p (A z = r, so no product with A is
//         needed), w = A p - K p and the partial p.w;
//  fixed point: r = q bar + K mu;
//  warm start: r = q bar - (A~ - K) mu (mass term (1 + alpha h) m / h^2 added here);
//  debug: K x.
template <int MODE>
__device__ __forceinline__ void b_adj_gather(VertArgs Vx, AdjState A, RedArgs R, int it, int bid) {
  const int nv = Vx.nv;
  const int gtid = bid * blockDim.x + threadIdx.x;
  const int i = gtid >> 3, l = gtid & 7;
  const bool have = i < Vx.nf;
  const bool owner = have && l == 0;
  // first round: the vertex's incidence range, its own state and the scalars
  int k0 = 0, k1 = 0;
  if (have) {
    k0 = Vx.inc_ptr[i];
    k1 = Vx.inc_ptr[i + 1];
  }
  double u0[3] = {0, 0, 0}, u1[3] = {0, 0, 0}, u2[3] = {0, 0, 0}, u3[3] = {0, 0, 0};
  if (owner)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int ix = a * nv + i;
      if (MODE == kModePCG) {
        u0[a] = A.z[ix];
        u1[a] = A.p[ix];
        u2[a] = r_cur(A, it)[ix];
        u3[a] = A.Ap[ix];
      } else if (MODE == kModeFixed) {
        u0[a] = A.qbar[ix];
      } else if (MODE == kModeInit) {
        u0[a] = A.qbar[ix];
        u1[a] = A.mu[ix];
      }
    }
  double num = 0.0, den = 1.0, mass = 0.0;
  if (MODE == kModePCG && it >= 1) {
    num = fin_site(R, kRedRZ0 + (it & 1))[0];
    den = fin_site(R, kRedRZ0 + ((it - 1) & 1))[0];
  }
  if (MODE == kModeInit && owner) mass = Vx.mass[i];
  __shared__ int flag_s;
  if (threadIdx.x == 0) flag_s = (MODE == kModePCG || MODE == kModeFixed) ? *A.done : 0;
  __syncthreads();
  if (flag_s) return;
  const double beta = num / den;
  double v[1] = {0.0};
  if (have) {
    double kx[3];
    inc_sum8(A.contrib, Vx.ninc, k0, k1, l, kx);
    if (l == 0) {
      const double h = Vx.h;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const int ix = a * nv + i;
        if (MODE == kModePCG) {
          const double pn = u0[a] + beta * u1[a];
          const double apn = u2[a] + beta * u3[a];
          const double w = apn - kx[a];
          A.p[ix] = pn;
          A.Ap[ix] = apn;
          A.w[ix] = w;
          v[0] += pn * w;
        } else if (MODE == kModeFixed) {
          A.r0[ix] = u0[a] + kx[a];
        } else if (MODE == kModeInit) {
          A.r0[ix] = u0[a] - ((1.0 + Vx.alpha * h) * mass / (h * h) * u1[a] + kx[a]);
        } else {
          A.w[ix] = kx[a];
        }
      }
    }
  }
  if (MODE == kModePCG) write_partial<1>(v, R, kRedPW, bid);
}

template <int MODE>
__global__ void __launch_bounds__(kBlock) k_adj_gather(VertArgs Vx, AdjState A, RedArgs R, int it) {
  b_adj_gather<MODE>(Vx, A, R, it, blockIdx.x);
}

// q bar = gq_next + gv_next / h on free vertices (Alg. 2 first line), in
// library order; adjoint start mu0 (zero, the previous solution mu1 of the
// sweep, the linear extrapolation 2 mu1 - mu2 or the quadratic one
// 3 mu1 - 3 mu2 + mu3), r = q bar, p = A p = 0.
__device__ PD_VERT_BODY void b_bwd_prologue(const VertArgs& Vx, const AdjState& Ad, const double* __restrict__ gq,
                                               const double* __restrict__ gv, int warm, const double* __restrict__ h1,
                                               const double* __restrict__ h2, const double* __restrict__ h3, int bid) {
#pragma clang fp contract(off)
  const int i = bid * blockDim.x + threadIdx.x;
  if (i >= Vx.nv) return;
  const int nv = Vx.nv, o = Vx.v_orig[i];
  const bool fr = i < Vx.nf;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int ix = a * nv + i;
    const double qb = fr ? ((gq ? gq[3 * o + a] : 0.0) + (gv ? gv[3 * o + a] : 0.0) / Vx.h) : 0.0;
    double m0 = 0.0;
    if (fr && warm == 1) m0 = h1[ix];
    if (fr && warm == 2) m0 = 2.0 * h1[ix] - h2[ix];
    if (fr && warm == 3) m0 = 3.0 * (h1[ix] - h2[ix]) + h3[ix];
    Ad.qbar[ix] = qb;
    Ad.r0[ix] = qb;
    Ad.mu[ix] = m0;
    Ad.p[ix] = 0.0;
    Ad.Ap[ix] = 0.0;
  }
}

__global__ void __launch_bounds__(kBlock) k_bwd_prologue(VertArgs Vx, AdjState Ad, const double* __restrict__ gq,
                                                         const double* __restrict__ gv, int warm,
                                                         const double* __restrict__ h1, const double* __restrict__ h2,
                                                         const double* __restrict__ h3) {
  b_bwd_prologue(Vx, Ad, gq, gv, warm, h1, h2, h3, blockIdx.x);
}

// Gradient routing per tet (Eq. dl_dwe and its damping counterpart, chain
// rule through w_e and beta_e, both proportional to E_e):
// dL/dlogE_e += w_e V_e <G mu, p* - G q*> + (beta_e V_e / h) <G mu, G (q_t - q*)>,
// plus the contributions (beta_e V_e / h) G^T G mu for B_beta mu / h.
__device__ PD_SHARED_BODY void b_grad_elem(const ElemArgs& E, const VertArgs& Vx, const double* __restrict__ ck,
                                            const double* __restrict__ jac, const double* __restrict__ mu,
                                            double* __restrict__ contrib, double* __restrict__ g_logE, int bid) {
  const int t = bid * blockDim.x + threadIdx.x;
  if (t >= E.ne) return;
  const int nv = Vx.nv;
  double Gm[9], Fs[9], Ft[9];
  int vi[4];
  load_F(E, mu, nv, t, Gm, vi);  // mu is zero on pinned vertices
  load_F(E, ck + 6 * nv, nv, t, Fs, vi);
  load_F(E, ck, nv, t, Ft, vi);
  double U[9], V[9], ss[3], qU[4], qV[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    qU[j] = jac[(size_t)j * E.ne + t];
    qV[j] = jac[(size_t)(kJacV + j) * E.ne + t];
  }
#pragma unroll
  for (int j = 0; j < 3; ++j) ss[j] = jac[(size_t)(kJacS + j) * E.ne + t];
  rot_of_quat(qU, U);
  rot_of_quat(qV, V);
  double gw = 0.0, gb = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const double P = U[3 * i] * ss[0] * V[3 * j] + U[3 * i + 1] * ss[1] * V[3 * j + 1] + U[3 * i + 2] * ss[2] * V[3 * j + 2];
      gw += Gm[3 * i + j] * (P - Fs[3 * i + j]);
      gb += Gm[3 * i + j] * (Ft[3 * i + j] - Fs[3 * i + j]);
    }
  if (g_logE) g_logE[E.tet_orig[t]] += E.wV[t] * gw + E.bV[t] * gb;
  store_contrib(E, contrib, t, E.bV[t], Gm);
  if (E.mus) {
    // the tet's term of dL/da_g = -w_m V_e <G_m mu, f^> (summed per group afterwards)
    double m[3], wm, y[3];
    fibre_of(E, t, m, wm);
    mat_vec_m(Gm, m, y);
    const size_t ne = E.ne;
    E.mgt[t] = -wm * (y[0] * E.mjac[t] + y[1] * E.mjac[ne + t] + y[2] * E.mjac[2 * ne + t]);
  }
}

__global__ void __launch_bounds__(kBlock) k_grad_elem(ElemArgs E, VertArgs Vx, const double* __restrict__ ck,
                                                      const double* __restrict__ jac, const double* __restrict__ mu,
                                                      double* __restrict__ contrib, double* __restrict__ g_logE) {
  b_grad_elem(E, Vx, ck, jac, mu, contrib, g_logE, blockIdx.x);
}

// dL/da_g += the group's tet terms: one wave per group, lane l adds terms l,
// l + 64, ... of the group's list in order, then a fixed butterfly
__global__ void __launch_bounds__(64) k_muscle_grad(const double* __restrict__ mgt, const int* __restrict__ g_ptr,
                                                    const int* __restrict__ g_tets, double* __restrict__ g_act) {
  const int g = blockIdx.x, l = threadIdx.x;
  double s = 0.0;
  for (int k = g_ptr[g] + l; k < g_ptr[g + 1]; k += 64) s += mgt[g_tets[k]];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if (l == 0) g_act[g] += s;
}

// dL/dq_t = (M/h^2 + alpha M/h) mu + B_beta mu / h - v bar / h,
// dL/dv_t = M mu / h, dL/df_ext = mu (caller's order; zero on pinned).
// mu_copy (optional) receives a copy of mu (the adjoint history of a batch).
__device__ PD_VERT_BODY void b_grad_vert(const VertArgs& Vx, const double* __restrict__ mu,
                                            const double* __restrict__ contrib, const double* __restrict__ gv_next,
                                            double* __restrict__ gq_t, double* __restrict__ gv_t,
                                            double* __restrict__ gf, double* __restrict__ mu_copy, int bid) {
#pragma clang fp contract(off)
  const int gtid = bid * blockDim.x + threadIdx.x;
  const int i = gtid >> 3, l = gtid & 7;
  const int nv = Vx.nv;
  if (i >= nv) return;
  double bm[3] = {0, 0, 0};
  if (i < Vx.nf) gather8(Vx.inc_ptr, contrib, Vx.ninc, i, l, bm);
  if (l != 0) return;
  const int o = Vx.v_orig[i];
  if (mu_copy)
#pragma unroll
    for (int a = 0; a < 3; ++a) mu_copy[a * nv + i] = mu[a * nv + i];
  if (i >= Vx.nf) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (gq_t) gq_t[3 * o + a] = 0.0;
      if (gv_t) gv_t[3 * o + a] = 0.0;
      if (gf) gf[3 * o + a] = 0.0;
    }
    return;
  }
  const double m = Vx.mass[i], h = Vx.h;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double u = mu[a * nv + i];
    const double gvn = gv_next ? gv_next[3 * o + a] : 0.0;
    if (gq_t) gq_t[3 * o + a] = (m / (h * h) + Vx.alpha * m / h) * u + bm[a] - gvn / h;
    if (gv_t) gv_t[3 * o + a] = m / h * u;
    if (gf) gf[3 * o + a] = u;
  }
}

__global__ void __launch_bounds__(kBlock) k_grad_vert(VertArgs Vx, const double* __restrict__ mu,
                                                      const double* __restrict__ contrib,
                                                      const double* __restrict__ gv_next, double* __restrict__ gq_t,
                                                      double* __restrict__ gv_t, double* __restrict__ gf) {
  b_grad_vert(Vx, mu, contrib, gv_next, gq_t, gv_t, gf, nullptr, blockIdx.x);
}

__global__ void __launch_bounds__(kBlock) k_init_warm(ElemArgs E) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= E.ne) return;
#pragma unroll
  for (int j = 0; j < 4; ++j) E.Vw[(size_t)j * E.ne + t] = (j == 0) ? 1.0 : 0.0;
#pragma unroll
  for (int j = 0; j < 3; ++j) E.rw[(size_t)j * E.ne + t] = 0.0;
}

__global__ void __launch_bounds__(kBlock) k_zero_int(int* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// ================================================================= batched launches
// One launch per stage covers the scenes of a batch: block b belongs to the
// listed scene j with base[j] <= b < base[j+1] and runs as block b - base[j]
// of scene sid[j], with the scene's own arguments, reductions and done flag
// (a scene that converges within a chunk exits at once; the host drops it
// from the list at the next check).
__device__ __forceinline__ int scene_of(const BatchMap& M, int b) {
  int lo = 0, hi = M.ns - 1;  // the last s with base[s] <= b
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (M.base[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

#define PD_BATCH_PROLOGUE                      \
  const int s_ = scene_of(M, blockIdx.x);      \
  const int bid = blockIdx.x - M.base[s_];     \
  const SceneBundle& b = M.B[M.sid[s_]];

// per-step kernels of a batch (one launch over all scenes each)
#define PD_BATCH_IO(io)                        \
  const int s_ = scene_of(M, blockIdx.x);      \
  const int bid = blockIdx.x - M.base[s_];     \
  const SceneBundle& b = M.B[M.sid[s_]];       \
  const auto& x = io[M.sid[s_]];

__global__ void __launch_bounds__(kBlock) kb_fwd_to_lib(BatchMap M, const BFwdIO* __restrict__ io) {
  PD_BATCH_IO(io)
  b_to_lib(b.V, x.q_t, b.St.qt, 0, bid);
}

__global__ void __launch_bounds__(kBlock) kb_elem_GtG(BatchMap M) {
  PD_BATCH_PROLOGUE
  b_elem_GtG(b.E, b.St.qt, b.V.nv, b.E.bV, b.St.contrib, bid);
}

__global__ void __launch_bounds__(kBlock) kb_prologue(BatchMap M, const BFwdIO* __restrict__ io) {
  PD_BATCH_IO(io)
  b_prologue(b.V, x.q_t, x.v_t, x.f, x.q0, x.inertial, b.St, bid);
}

__global__ void __launch_bounds__(kBlock) kb_epilogue(BatchMap M, const BFwdIO* __restrict__ io) {
  PD_BATCH_IO(io)
  b_epilogue(b.V, b.St, x.q_next, x.v_next, x.ckpt, bid);
}

__global__ void __launch_bounds__(kBlock) kb_bwd_prologue(BatchMap M, const BBwdIO* __restrict__ io) {
  PD_BATCH_IO(io)
  b_bwd_prologue(b.V, b.A, x.gq, x.gv, x.warm, x.h1, x.h2, x.h3, bid);
}

__global__ void __launch_bounds__(kBlock) kb_tr_partials(BatchMap M, const BBwdIO* __restrict__ io) {
  PD_BATCH_IO(io)
  if (x.tr) b_tr_partials(b.E, b.V, b.R, x.ck, (b.E.ne + kBlock - 1) / kBlock, bid);
}

__global__ void __launch_bounds__(kBlock) kb_bwd_elem(BatchMap M, const BBwdIO* __restrict__ io) {
  PD_BATCH_IO(io)
  b_bwd_elem(b.E, b.V, b.R, x.ck, x.eps_tr, -1.0, x.tr, b.jac, b.St.dstat + 4, b.A.ctl, 4, bid);
}

__global__ void __launch_bounds__(kBlock) kb_grad_elem(BatchMap M, const BBwdIO* __restrict__ io) {
  PD_BATCH_IO(io)
  b_grad_elem(b.E, b.V, x.ck, b.jac, b.A.mu, b.A.contrib, x.g_logE, bid);
}

__global__ void __launch_bounds__(kBlock) kb_grad_vert(BatchMap M, const BBwdIO* __restrict__ io) {
  PD_BATCH_IO(io)
  b_grad_vert(b.V, b.A.mu, b.A.contrib, x.gv, x.gq_t, x.gv_t, x.gf, x.mu_copy, bid);
}

__global__ void __launch_bounds__(kBlock) kb_local(BatchMap M, int k) {
  PD_BATCH_PROLOGUE
  int* cap = b.St.ctl + kCtlNewton;
  switch (b.St.m) {
    case 1: b_local<1>(b.E, b.St, b.R, b.St.q_cur, b.V.nv, b.V.nf, k, 1, cap, bid); break;
    case 2: b_local<2>(b.E, b.St, b.R, b.St.q_cur, b.V.nv, b.V.nf, k, 1, cap, bid); break;
    case 3: b_local<3>(b.E, b.St, b.R, b.St.q_cur, b.V.nv, b.V.nf, k, 1, cap, bid); break;
    case 4: b_local<4>(b.E, b.St, b.R, b.St.q_cur, b.V.nv, b.V.nf, k, 1, cap, bid); break;
    case 5: b_local<5>(b.E, b.St, b.R, b.St.q_cur, b.V.nv, b.V.nf, k, 1, cap, bid); break;
    default: b_local<0>(b.E, b.St, b.R, b.St.q_cur, b.V.nv, b.V.nf, k, 1, cap, bid); break;
  }
}

__global__ void __launch_bounds__(kBlock) kb_gather_fwd(BatchMap M, int k) {
  PD_BATCH_PROLOGUE
  switch (b.St.m) {
    case 1: b_gather_fwd<1>(b.V, b.St, b.R, k, bid); break;
    case 2: b_gather_fwd<2>(b.V, b.St, b.R, k, bid); break;
    case 3: b_gather_fwd<3>(b.V, b.St, b.R, k, bid); break;
    case 4: b_gather_fwd<4>(b.V, b.St, b.R, k, bid); break;
    case 5: b_gather_fwd<5>(b.V, b.St, b.R, k, bid); break;
    default: b_gather_fwd<0>(b.V, b.St, b.R, k, bid); break;
  }
}

// forward (gate), PCG (alpha), or the adjoint's first solve (right-hand side r0)
template <int MODE>
__global__ void __launch_bounds__(kBlock) PD_ROW_WALK_EB kb_Eb(BatchMap M, int k) {
  PD_BATCH_PROLOGUE
  if (MODE == kModePlain) {
    StepState st = b.St;
    st.done = b.A.done;
    b_Eb<kModePlain>(b.V, b.S, st, b.A, b.R, b.A.r0, k, bid);
  } else {
    b_Eb<MODE>(b.V, b.S, b.St, b.A, b.R, nullptr, k, bid);
  }
}

// A block of a scene whose loop has stopped exits on that scene's flag.
__global__ void __launch_bounds__(kBlock) kb_sep_fwd(BatchMap M, int lvl, int adjoint) {
  PD_BATCH_PROLOGUE
  b_sep_fwd(b.S, lvl, bid, adjoint ? b.A.done : b.St.done);
}

__global__ void __launch_bounds__(kBlock) kb_sep_back(BatchMap M, int lvl, int adjoint) {
  PD_BATCH_PROLOGUE
  b_sep_back(b.V, b.S, lvl, adjoint ? b.A.z : b.St.qhat, bid, adjoint ? b.A.done : b.St.done);
}

template <int MODE>
__global__ void __launch_bounds__(kBottomThreads) PD_ROW_WALK kb_bottom(BatchMap M, int k) {
  PD_BATCH_PROLOGUE
  if (MODE == kModeFwd) {
    switch (b.St.m) {
      case 1: b_bottom<kModeFwd, 1>(b.V, b.S, b.St, b.A, b.R, nullptr, b.St.qhat, k, bid); break;
      case 2: b_bottom<kModeFwd, 2>(b.V, b.S, b.St, b.A, b.R, nullptr, b.St.qhat, k, bid); break;
      case 3: b_bottom<kModeFwd, 3>(b.V, b.S, b.St, b.A, b.R, nullptr, b.St.qhat, k, bid); break;
      case 4: b_bottom<kModeFwd, 4>(b.V, b.S, b.St, b.A, b.R, nullptr, b.St.qhat, k, bid); break;
      case 5: b_bottom<kModeFwd, 5>(b.V, b.S, b.St, b.A, b.R, nullptr, b.St.qhat, k, bid); break;
      default: b_bottom<kModeFwd, 0>(b.V, b.S, b.St, b.A, b.R, nullptr, b.St.qhat, k, bid); break;
    }
  } else if (MODE == kModePCGInit) {
    StepState st = b.St;
    st.done = b.A.done;
    b_bottom<kModePCGInit, 0>(b.V, b.S, st, b.A, b.R, b.A.r0, b.A.z, k, bid);
  } else {
    b_bottom<MODE, 0>(b.V, b.S, b.St, b.A, b.R, nullptr, b.A.z, k, bid);
  }
}

template <int MODE>
__global__ void __launch_bounds__(kBlock) kb_apply_K(BatchMap M, int it) {
  PD_BATCH_PROLOGUE
  b_apply_K<MODE>(b.E, b.V, b.A, b.R, b.jac, MODE == kModeAmK ? b.A.mu : nullptr, it, bid);
}

template <int MODE>
__global__ void __launch_bounds__(kBlock) kb_adj_gather(BatchMap M, int it) {
  PD_BATCH_PROLOGUE
  b_adj_gather<MODE>(b.V, b.A, b.R, it, bid);
}

// every scene's control block and statistics, gathered for one copy to the host
__global__ void __launch_bounds__(64) kb_flags(BatchMap M, int* __restrict__ ctl, double* __restrict__ dstat) {
  const int s = blockIdx.x;
  const SceneBundle& b = M.B[s];
  const int t = threadIdx.x;
  if (t < kCtlTotal) ctl[s * kCtlTotal + t] = b.St.ctl[t];
  if (t < 32) dstat[s * 32 + t] = b.St.dstat[t];
}
#undef PD_BATCH_PROLOGUE

// ================================================================= launchers
#define PD_GRID(n) dim3(((n) + kBlock - 1) / kBlock), dim3(kBlock)
#define PD_EGRID(n) dim3(((n) + kElemBlock - 1) / kElemBlock), dim3(kElemBlock)

// Every launch goes through the extended launch, which can stamp a start and
// a stop event from the dispatch itself (the kernel's own execution time, the
// figure a kernel trace reports).  The events are armed for one launch.
namespace {
thread_local hipEvent_t g_ev_start = nullptr, g_ev_stop = nullptr;
thread_local bool g_ev_used = false;

template <typename F, typename... Args>
void launch_ext(F kernel, const dim3& grid, const dim3& block, unsigned shmem, hipStream_t s, Args... args) {
  hipEvent_t e0 = g_ev_start, e1 = g_ev_stop;
  g_ev_start = g_ev_stop = nullptr;
  if (e0) g_ev_used = true;
  hipExtLaunchKernelGGL(kernel, grid, block, shmem, s, e0, e1, 0u, args...);
}
}  // namespace

void arm_launch_events(hipEvent_t start, hipEvent_t stop) {
  g_ev_start = start;
  g_ev_stop = stop;
  g_ev_used = false;
}

bool launch_events_used() {
  const bool u = g_ev_used;
  g_ev_start = g_ev_stop = nullptr;
  g_ev_used = false;
  return u;
}

int vert_group_blocks(int n) { return (8 * n + kBlock - 1) / kBlock; }
int eb_blocks(int nT) { return std::max(1, (nT + kEbRows - 1) / kEbRows); }
int bottom_blocks(int nB, int nT) {
  return (nB + kBottomRows - 1) / kBottomRows + (nT + kBottomThreads - 1) / kBottomThreads;
}
int tr_blocks(int ne, int nf) { return (ne + kBlock - 1) / kBlock + (nf + kBlock - 1) / kBlock; }
int contact_apply_blocks(int nf) { return (nf + kBlock - 1) / kBlock; }

void launch_contact_apply_fwd(const VertArgs& V, const StepState& St, const RedArgs& R, const ContactArgs& C, int k,
                              hipStream_t s) {
  const dim3 g(contact_apply_blocks(V.nf)), b(kBlock);
  switch (St.m) {
    case 1: launch_ext(k_contact_apply_fwd<1>, g, b, 0, s, V, St, R, C, k); break;
    case 2: launch_ext(k_contact_apply_fwd<2>, g, b, 0, s, V, St, R, C, k); break;
    case 3: launch_ext(k_contact_apply_fwd<3>, g, b, 0, s, V, St, R, C, k); break;
    case 4: launch_ext(k_contact_apply_fwd<4>, g, b, 0, s, V, St, R, C, k); break;
    case 5: launch_ext(k_contact_apply_fwd<5>, g, b, 0, s, V, St, R, C, k); break;
    default: launch_ext(k_contact_apply_fwd<0>, g, b, 0, s, V, St, R, C, k); break;
  }
}
void launch_contact_apply_adj(int mode, const VertArgs& V, const AdjState& A, const RedArgs& R,
                              const ContactArgs& C, const double* rhs, int k, hipStream_t s) {
  const dim3 g(contact_apply_blocks(V.nf)), b(kBlock);
  if (mode == kModePCG) launch_ext(k_contact_apply_adj<kModePCG>, g, b, 0, s, V, A, R, C, rhs, k);
  else if (mode == kModePCGInit) launch_ext(k_contact_apply_adj<kModePCGInit>, g, b, 0, s, V, A, R, C, rhs, k);
  else launch_ext(k_contact_apply_adj<kModeFixed>, g, b, 0, s, V, A, R, C, rhs, k);
}

void launch_local(const ElemArgs& E, const StepState& St, const RedArgs& R, const double* q, int nv, int nf,
                  int k, int fwd, hipStream_t s) {
  int* cap = fwd ? St.ctl + kCtlNewton : nullptr;
#define PD_LOCAL(M) launch_ext(k_local<M>, PD_EGRID(E.ne), 0, s, E, St, R, q, nv, nf, k, fwd, cap)
  switch (fwd ? St.m : 0) {
    case 1: PD_LOCAL(1); break;
    case 2: PD_LOCAL(2); break;
    case 3: PD_LOCAL(3); break;
    case 4: PD_LOCAL(4); break;
    case 5: PD_LOCAL(5); break;
    default: PD_LOCAL(0); break;
  }
#undef PD_LOCAL
}
void launch_elem_GtG(const ElemArgs& E, const double* x, int nv, const double* w, double* contrib, hipStream_t s) {
  launch_ext(k_elem_GtG, PD_GRID(E.ne), 0, s, E, x, nv, w, contrib);
}
void launch_prologue(const VertArgs& V, const double* qt, const double* vt, const double* f, const double* q0,
                     int inertial, const StepState& St, hipStream_t s) {
  launch_ext(k_prologue, dim3(vert_group_blocks(V.nv)), dim3(kBlock), 0, s, V, qt, vt, f, q0, inertial, St);
}
void launch_gather_fwd(const VertArgs& V, const StepState& St, const RedArgs& R, int k, hipStream_t s) {
  const dim3 g(vert_group_blocks(V.nf)), b(kBlock);
#define PD_GATHER(M) launch_ext(k_gather_fwd<M>, g, b, 0, s, V, St, R, k)
  switch (St.m) {
    case 1: PD_GATHER(1); break;
    case 2: PD_GATHER(2); break;
    case 3: PD_GATHER(3); break;
    case 4: PD_GATHER(4); break;
    case 5: PD_GATHER(5); break;
    default: PD_GATHER(0); break;
  }
#undef PD_GATHER
}
void launch_gather_debug(const VertArgs& V, const double* contrib, double* out, hipStream_t s) {
  launch_ext(k_gather_debug, dim3(vert_group_blocks(V.nf)), dim3(kBlock), 0, s, V, contrib, out);
}
void launch_Eb(int mode, const VertArgs& V, const SolveArgs& S, const StepState& St, const AdjState& A,
               const RedArgs& R, const double* rhs, int k, hipStream_t s) {
  // the forward mode (gate decision) and the PCG mode (alpha) always run, with at least one block
  const int nblk = eb_blocks(S.nT);
  if (mode == kModeFwd)
    launch_ext(k_Eb<kModeFwd>, dim3(nblk), dim3(kBlock), 0, s, V, S, St, A, R, rhs, k);
  else if (mode == kModePCG)
    launch_ext(k_Eb<kModePCG>, dim3(nblk), dim3(kBlock), 0, s, V, S, St, A, R, rhs, k);
  else if (S.nT > 0)
    launch_ext(k_Eb<kModePlain>, dim3(nblk), dim3(kBlock), 0, s, V, S, St, A, R, rhs, k);
}
// The interface solve is 2 nlev - 1 launches (forward levels 2..nlev, then
// backward levels nlev..1); armed launch events time it from the first
// launch's start to the last one's end.
void launch_top(const VertArgs& V, const SolveArgs& S, double* out, const int* done, hipStream_t s) {
  hipEvent_t e0 = g_ev_start, e1 = g_ev_stop;
  g_ev_start = g_ev_stop = nullptr;
  const int nl = S.nlev;
  if (S.nT == 0 || nl <= 0) return;
  if (e0) g_ev_used = true;
  const int last = 2 * nl - 2;
  int idx = 0;
  for (int l = 2; l <= nl; ++l, ++idx)
    hipExtLaunchKernelGGL(k_sep_fwd, dim3((S.lev_nrows[l - 1] + kBlock / 64 - 1) / (kBlock / 64)), dim3(kBlock), 0,
                          s, idx == 0 ? e0 : nullptr, idx == last ? e1 : nullptr, 0u, S, l, done);
  for (int l = nl; l >= 1; --l, ++idx)
    hipExtLaunchKernelGGL(k_sep_back, dim3(S.lev_nblk[l - 1]), dim3(kBlock), 0, s, idx == 0 ? e0 : nullptr,
                          idx == last ? e1 : nullptr, 0u, V, S, l, out, done);
}
void launch_bottom(int mode, const VertArgs& V, const SolveArgs& S, const StepState& St, const AdjState& A,
                   const RedArgs& R, const double* rhs, double* out, int k, hipStream_t s) {
  const int nblk = bottom_blocks(S.nB, S.nT);
  if (nblk == 0) return;
#define PD_BOTTOM(MODE, M) \
  launch_ext((k_bottom<MODE, M>), dim3(nblk), dim3(kBottomThreads), 0, s, V, S, St, A, R, rhs, out, k)
  switch (mode) {
    case kModeFwd:
      switch (St.m) {
        case 1: PD_BOTTOM(kModeFwd, 1); break;
        case 2: PD_BOTTOM(kModeFwd, 2); break;
        case 3: PD_BOTTOM(kModeFwd, 3); break;
        case 4: PD_BOTTOM(kModeFwd, 4); break;
        case 5: PD_BOTTOM(kModeFwd, 5); break;
        default: PD_BOTTOM(kModeFwd, 0); break;
      }
      break;
    case kModePCG: PD_BOTTOM(kModePCG, 0); break;
    case kModePCGSolve: PD_BOTTOM(kModePCGSolve, 0); break;
    case kModePCGInit: PD_BOTTOM(kModePCGInit, 0); break;
    case kModeFixed: PD_BOTTOM(kModeFixed, 0); break;
    default: PD_BOTTOM(kModePlain, 0); break;
  }
#undef PD_BOTTOM
}
void launch_epilogue(const VertArgs& V, const StepState& St, double* q_next, double* v_next, double* ckpt,
                     hipStream_t s) {
  launch_ext(k_epilogue, PD_GRID(V.nv), 0, s, V, St, q_next, v_next, ckpt);
}
void launch_to_lib(const VertArgs& V, const double* user, double* lib, int free_only, hipStream_t s) {
  launch_ext(k_to_lib, PD_GRID(V.nv), 0, s, V, user, lib, free_only);
}
void launch_from_lib(const VertArgs& V, const double* lib, double* user, int free_only, hipStream_t s) {
  launch_ext(k_from_lib, PD_GRID(V.nv), 0, s, V, lib, user, free_only);
}
void launch_tr_partials(const ElemArgs& E, const VertArgs& V, const RedArgs& R, const double* ck, hipStream_t s) {
  const int ntb = (E.ne + kBlock - 1) / kBlock;
  const int nblk = ntb + (V.nf + kBlock - 1) / kBlock;
  launch_ext(k_tr_partials, dim3(nblk), dim3(kBlock), 0, s, E, V, R, ck, ntb);
}
void launch_bwd_elem(const ElemArgs& E, const VertArgs& V, const RedArgs& R, const double* ck, double eps_tr,
                     double tau_force, int use_partials, double* jac, double* bstat, int* zero, int nzero,
                     hipStream_t s) {
  launch_ext(k_bwd_elem, PD_GRID(E.ne), 0, s, E, V, R, ck, eps_tr, tau_force, use_partials, jac, bstat, zero, nzero);
}
void launch_apply_K(int mode, const ElemArgs& E, const VertArgs& V, const AdjState& A, const RedArgs& R,
                    const double* jac, const double* x, int it, hipStream_t s) {
  if (mode == kModePCG) launch_ext(k_apply_K<kModePCG>, PD_EGRID(E.ne), 0, s, E, V, A, R, jac, x, it);
  else if (mode == kModeFixed) launch_ext(k_apply_K<kModeFixed>, PD_EGRID(E.ne), 0, s, E, V, A, R, jac, x, it);
  else if (mode == kModeAmK) launch_ext(k_apply_K<kModeAmK>, PD_EGRID(E.ne), 0, s, E, V, A, R, jac, x, it);
  else launch_ext(k_apply_K<kModeDebug>, PD_EGRID(E.ne), 0, s, E, V, A, R, jac, x, it);
}
void launch_adj_gather(int mode, const VertArgs& V, const AdjState& A, const RedArgs& R, int it, hipStream_t s) {
  const dim3 g(vert_group_blocks(V.nf)), b(kBlock);
  if (mode == kModePCG) launch_ext(k_adj_gather<kModePCG>, g, b, 0, s, V, A, R, it);
  else if (mode == kModeFixed) launch_ext(k_adj_gather<kModeFixed>, g, b, 0, s, V, A, R, it);
  else if (mode == kModeInit) launch_ext(k_adj_gather<kModeInit>, g, b, 0, s, V, A, R, it);
  else launch_ext(k_adj_gather<kModeDebug>, g, b, 0, s, V, A, R, it);
}
void launch_bwd_prologue(const VertArgs& V, const AdjState& A, const double* gq, const double* gv, int warm,
                         const double* h1, const double* h2, const double* h3, hipStream_t s) {
  launch_ext(k_bwd_prologue, PD_GRID(V.nv), 0, s, V, A, gq, gv, warm, h1, h2, h3);
}
void launch_grad_elem(const ElemArgs& E, const VertArgs& V, const double* ck, const double* jac, const double* mu,
                      double* contrib, double* g_logE, hipStream_t s) {
  launch_ext(k_grad_elem, PD_GRID(E.ne), 0, s, E, V, ck, jac, mu, contrib, g_logE);
}
void launch_grad_vert(const VertArgs& V, const double* mu, const double* contrib, const double* gv_next, double* gq_t,
                      double* gv_t, double* gf, hipStream_t s) {
  launch_ext(k_grad_vert, dim3(vert_group_blocks(V.nv)), dim3(kBlock), 0, s, V, mu, contrib, gv_next, gq_t,
                     gv_t, gf);
}
void launch_b_fwd_pre(const BatchMap& Mv, int nv_blk, const BatchMap& Me, int ne_blk, const BatchMap& Mv8,
                      int nv8_blk, const BFwdIO* io, hipStream_t s) {
  if (nv_blk > 0) launch_ext(kb_fwd_to_lib, dim3(nv_blk), dim3(kBlock), 0, s, Mv, io);
  if (ne_blk > 0) launch_ext(kb_elem_GtG, dim3(ne_blk), dim3(kBlock), 0, s, Me);
  if (nv8_blk > 0) launch_ext(kb_prologue, dim3(nv8_blk), dim3(kBlock), 0, s, Mv8, io);
}
void launch_b_fwd_post(const BatchMap& Mv, int nv_blk, const BFwdIO* io, hipStream_t s) {
  if (nv_blk > 0) launch_ext(kb_epilogue, dim3(nv_blk), dim3(kBlock), 0, s, Mv, io);
}
void launch_b_bwd_pre(const BatchMap& Mv, int nv_blk, const BatchMap& Mtr, int ntr_blk, const BatchMap& Me,
                      int ne_blk, const BBwdIO* io, hipStream_t s) {
  if (nv_blk > 0) launch_ext(kb_bwd_prologue, dim3(nv_blk), dim3(kBlock), 0, s, Mv, io);
  if (ntr_blk > 0) launch_ext(kb_tr_partials, dim3(ntr_blk), dim3(kBlock), 0, s, Mtr, io);
  if (ne_blk > 0) launch_ext(kb_bwd_elem, dim3(ne_blk), dim3(kBlock), 0, s, Me, io);
}
void launch_b_bwd_post(const BatchMap& Me, int ne_blk, const BatchMap& Mv8, int nv8_blk, const BBwdIO* io,
                       hipStream_t s) {
  if (ne_blk > 0) launch_ext(kb_grad_elem, dim3(ne_blk), dim3(kBlock), 0, s, Me, io);
  if (nv8_blk > 0) launch_ext(kb_grad_vert, dim3(nv8_blk), dim3(kBlock), 0, s, Mv8, io);
}
void launch_b_local(const BatchMap& M, int nblk, int block, int k, hipStream_t s) {
  if (nblk > 0) launch_ext(kb_local, dim3(nblk), dim3(block), 0, s, M, k);
}
void launch_b_gather_fwd(const BatchMap& M, int nblk, int k, hipStream_t s) {
  if (nblk > 0) launch_ext(kb_gather_fwd, dim3(nblk), dim3(kBlock), 0, s, M, k);
}
void launch_b_Eb(int mode, const BatchMap& M, int nblk, int k, hipStream_t s) {
  if (nblk <= 0) return;
  if (mode == kModeFwd) launch_ext(kb_Eb<kModeFwd>, dim3(nblk), dim3(kBlock), 0, s, M, k);
  else if (mode == kModePCG) launch_ext(kb_Eb<kModePCG>, dim3(nblk), dim3(kBlock), 0, s, M, k);
  else launch_ext(kb_Eb<kModePlain>, dim3(nblk), dim3(kBlock), 0, s, M, k);
}
void launch_b_sep(const BatchMap* Mf, const int* nblk_f, const BatchMap* Mb, const int* nblk_b, int nlev,
                  int adjoint, hipStream_t s) {
  hipEvent_t e0 = g_ev_start, e1 = g_ev_stop;
  g_ev_start = g_ev_stop = nullptr;
  // the non-empty launches in order: forward levels 2..nlev, backward nlev..1
  int kind[2 * kMaxLevels], lev[2 * kMaxLevels], n = 0;
  for (int l = 2; l <= nlev; ++l)
    if (nblk_f[l - 1] > 0) kind[n] = 0, lev[n++] = l;
  for (int l = nlev; l >= 1; --l)
    if (nblk_b[l - 1] > 0) kind[n] = 1, lev[n++] = l;
  if (n == 0) return;
  if (e0) g_ev_used = true;
  for (int i = 0; i < n; ++i) {
    const int l = lev[i];
    hipEvent_t a = i == 0 ? e0 : nullptr, b = i == n - 1 ? e1 : nullptr;
    if (kind[i] == 0)
      hipExtLaunchKernelGGL(kb_sep_fwd, dim3(nblk_f[l - 1]), dim3(kBlock), 0, s, a, b, 0u, Mf[l - 1], l, adjoint);
    else
      hipExtLaunchKernelGGL(kb_sep_back, dim3(nblk_b[l - 1]), dim3(kBlock), 0, s, a, b, 0u, Mb[l - 1], l, adjoint);
  }
}
void launch_b_bottom(int mode, const BatchMap& M, int nblk, int k, hipStream_t s) {
  if (nblk <= 0) return;
  if (mode == kModeFwd) launch_ext(kb_bottom<kModeFwd>, dim3(nblk), dim3(kBottomThreads), 0, s, M, k);
  else if (mode == kModePCG) launch_ext(kb_bottom<kModePCG>, dim3(nblk), dim3(kBottomThreads), 0, s, M, k);
  else launch_ext(kb_bottom<kModePCGInit>, dim3(nblk), dim3(kBottomThreads), 0, s, M, k);
}
void launch_b_apply_K(int mode, const BatchMap& M, int nblk, int block, int it, hipStream_t s) {
  if (nblk <= 0) return;
  if (mode == kModeAmK) launch_ext(kb_apply_K<kModeAmK>, dim3(nblk), dim3(block), 0, s, M, it);
  else launch_ext(kb_apply_K<kModePCG>, dim3(nblk), dim3(block), 0, s, M, it);
}
void launch_b_adj_gather(int mode, const BatchMap& M, int nblk, int it, hipStream_t s) {
  if (nblk <= 0) return;
  if (mode == kModeInit) launch_ext(kb_adj_gather<kModeInit>, dim3(nblk), dim3(kBlock), 0, s, M, it);
  else launch_ext(kb_adj_gather<kModePCG>, dim3(nblk), dim3(kBlock), 0, s, M, it);
}
void launch_b_flags(const BatchMap& M, int* ctl_out, double* dstat_out, hipStream_t s) {
  launch_ext(kb_flags, dim3(M.ns), dim3(64), 0, s, M, ctl_out, dstat_out);
}

void launch_muscle_grad(const ElemArgs& E, int n_groups, const int* g_ptr, const int* g_tets, double* g_act,
                        hipStream_t s) {
  if (n_groups > 0) hipLaunchKernelGGL(k_muscle_grad, dim3(n_groups), dim3(64), 0, s, E.mgt, g_ptr, g_tets, g_act);
}

void launch_init_warm(const ElemArgs& E, hipStream_t s) {
  launch_ext(k_init_warm, PD_GRID(E.ne), 0, s, E);
}
void launch_zero_int(int* p, int n, hipStream_t s) { launch_ext(k_zero_int, PD_GRID(n), 0, s, p, n); }

}  // namespace pdhot
