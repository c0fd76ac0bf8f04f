// Contact kernels (Sec. 4.7, frictionless reading): candidate detection
// against static obstacles, the columns a_v = A~^{-1} e_v of the contact
// vertices, the Delassus operator W = J A~^{-1} J^T from them, the per-PD-
// iteration Fischer-Burmeister Newton solve, and the projection that keeps
// the adjoint on the active constraints.
//
// A~ acts identically on the three axes, so one scalar column per contact
// vertex serves every axis and every row on that vertex: W_cd =
// (n_c . n_d) a_{v_c}[v_d], and an impulse lam_c along n_c moves the free
// vertices by lam_c a_{v_c} n_c.  The Newton systems are small (tens to a
// hundred and more rows), dense and SPD, so each is factored by one 1024-thread
// workgroup in LDS: the lower triangle is packed and the right-hand side rides
// along as an extra row, so the factorisation also produces L^{-1} rhs.
#include <hip/hip_ext.h>

#include "kernels.h"

namespace pdhot {

namespace {

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ double wmax(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

__host__ __device__ constexpr int tri(int i) { return i * (i + 1) / 2; }

// signed distance n.x - o without contraction (the same roundings as a plain
// left-to-right evaluation)
__device__ __forceinline__ double plane_dist(const double* P, double x, double y, double z) {
  double d = __dadd_rn(__dmul_rn(P[0], x), __dmul_rn(P[1], y));
  d = __dadd_rn(d, __dmul_rn(P[2], z));
  return __dsub_rn(d, P[3]);
}

// largest signed face distance of a box and the face attaining it (first on
// ties), faces in the order -x, +x, -y, +y, -z, +z
__device__ __forceinline__ double box_dist(const double* B, const double x[3], int& face) {
  double best = -INFINITY;
  face = 0;
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    const int a = f >> 1;
    const double d = (f & 1) ? __dsub_rn(x[a], B[3 + a]) : __dadd_rn(-x[a], B[a]);
    if (d > best) {
      best = d;
      face = f;
    }
  }
  return best;
}

}  // namespace

// ---------------------------------------------------------------- detection
// One workgroup walks the free vertices in library order, 1024 at a time; for
// each vertex and obstacle (planes, then boxes) the distance at x0 = q_t and
// at x1 = q_t + h v_t decides the row (min < d_c); the face that attains the
// distance at x0 gives its normal and offset.  Rows are compacted in
// (vertex, obstacle) order by a block prefix sum; flags[0] receives the total,
// rows past kmax are counted but not written.
__global__ void __launch_bounds__(kContactThreads) k_contact_detect(VertArgs Vx, const double* __restrict__ qt,
                                                                    const double* __restrict__ vt, ObsArgs O,
                                                                    int kmax, int* __restrict__ cv,
                                                                    double* __restrict__ cn, double* __restrict__ cg,
                                                                    int* __restrict__ flags) {
  __shared__ int wtot[kContactThreads / 64];
  __shared__ int base_s;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int nv = Vx.nv, nf = Vx.nf, nobs = O.n_planes + O.n_boxes;
  if (tid == 0) base_s = 0;
  __syncthreads();
  for (int c0 = 0; c0 < nf; c0 += kContactThreads) {
    const int i = c0 + tid;
    unsigned mask = 0;
    double best0 = 0.0;
    int faces[kMaxObstacles];
#pragma unroll
    for (int o = 0; o < kMaxObstacles; ++o) faces[o] = 0;
    if (i < nf) {
      double x0[3], x1[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        x0[a] = qt[a * nv + i];
        x1[a] = __dadd_rn(x0[a], __dmul_rn(O.h, vt[a * nv + i]));
      }
#pragma unroll
      for (int o = 0; o < kMaxObstacles; ++o) {
        if (o >= nobs) break;
        double d0, d1;
        int f = 0, f1 = 0;
        if (o < O.n_planes) {
          const double* P = O.planes + 4 * o;
          d0 = plane_dist(P, x0[0], x0[1], x0[2]);
          d1 = plane_dist(P, x1[0], x1[1], x1[2]);
        } else {
          const double* B = O.boxes + 6 * (o - O.n_planes);
          d0 = box_dist(B, x0, f);
          d1 = box_dist(B, x1, f1);
        }
        if (fmin(d0, d1) < O.d_c) {
          if (O.one_per_vertex) {
            // keep the qualifying obstacle with the smallest distance at x0 (the first on ties)
            if (mask == 0u || d0 < best0) {
              mask = 1u << o;
              best0 = d0;
            }
          } else {
            mask |= 1u << o;
          }
          faces[o] = f;
        }
      }
    }
    const int cnt = __popc(mask);
    // inclusive prefix within the wave, then across waves
    int inc = cnt;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int t = __shfl_up(inc, off, 64);
      if (lane >= off) inc += t;
    }
    if (lane == 63) wtot[wid] = inc;
    __syncthreads();
    int before = 0, total = 0;
    for (int w = 0; w < kContactThreads / 64; ++w) {
      if (w < wid) before += wtot[w];
      total += wtot[w];
    }
    int pos = base_s + before + inc - cnt;
#pragma unroll
    for (int o = 0; o < kMaxObstacles; ++o) {
      if (!(mask & (1u << o))) continue;
      if (pos < kmax) {
        cv[pos] = i;
        double nn[3] = {0, 0, 0}, off;
        if (o < O.n_planes) {
          const double* P = O.planes + 4 * o;
          nn[0] = P[0]; nn[1] = P[1]; nn[2] = P[2];
          off = P[3];
        } else {
          const double* B = O.boxes + 6 * (o - O.n_planes);
          const int f = faces[o], a = f >> 1;
          nn[a] = (f & 1) ? 1.0 : -1.0;
          off = (f & 1) ? B[3 + a] : -B[a];
        }
        cn[3 * pos] = nn[0];
        cn[3 * pos + 1] = nn[1];
        cn[3 * pos + 2] = nn[2];
        cg[pos] = off;
      }
      ++pos;
    }
    __syncthreads();
    if (tid == 0) base_s += total;
    __syncthreads();
  }
  if (tid == 0) flags[0] = base_s;
}

// ---------------------------------------------------------------- columns
// rhs = e_{v0} on axis 0, e_{v1} on axis 1, e_{v2} on axis 2 (v < 0: none), so
// one three-right-hand-side solve yields three columns.
__global__ void __launch_bounds__(kBlock) k_unit_rhs(int nv, double* __restrict__ rhs, int v0, int v1, int v2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nv) return;
  rhs[i] = (i == v0) ? 1.0 : 0.0;
  rhs[nv + i] = (i == v1) ? 1.0 : 0.0;
  rhs[2 * nv + i] = (i == v2) ? 1.0 : 0.0;
}

__global__ void __launch_bounds__(kBlock) k_store_cols(int nf, int nv, const double* __restrict__ x,
                                                       double* __restrict__ cols, int s0, int s1, int s2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nf) return;
  if (s0 >= 0) cols[(size_t)s0 * nf + i] = x[i];
  if (s1 >= 0) cols[(size_t)s1 * nf + i] = x[nv + i];
  if (s2 >= 0) cols[(size_t)s2 * nf + i] = x[2 * nv + i];
}

// W_cd = (n_c . n_d) a_{v_c}[v_d]; with friction the scalar block G_cd = a_{v_c}[v_d]
// (every row pair of two frames then couples by the product of their directions)
__global__ void __launch_bounds__(kBlock) k_contact_W(ContactArgs C, double* __restrict__ W) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int K = C.K;
  if (idx >= K * K) return;
  const int c = idx / K, d = idx - c * K;
  const double nn = C.mu > 0.0 ? 1.0
                               : C.n[3 * c] * C.n[3 * d] + C.n[3 * c + 1] * C.n[3 * d + 1] +
                                     C.n[3 * c + 2] * C.n[3 * d + 2];
  W[idx] = nn * C.cols[(size_t)C.slot[c] * C.nf + C.v[d]];
}

// impulses start at zero each step; s = 0, FB residual 0
__global__ void __launch_bounds__(kBlock) k_contact_start(ContactArgs C) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c == 0) {
    C.fb[0] = 0.0;
    C.fb[1] = 0.0;
    C.flags[1] = 0;
    C.flags[2] = 0;
  }
  if (c >= C.K) return;
  if (C.mu > 0.0) {
    C.lam[3 * c] = 0.0;
    C.lam[3 * c + 1] = 0.0;
    C.lam[3 * c + 2] = 0.0;
  } else {
    C.lam[c] = 0.0;
  }
  C.s[3 * c] = 0.0;
  C.s[3 * c + 1] = 0.0;
  C.s[3 * c + 2] = 0.0;
}

// ---------------------------------------------------------------- FB Newton
// Fischer-Burmeister values of every row at lam (Eqs. fb_n, omega_E_n with
// r_c = W_cc): one wave per row for delta = dfree + W lam; returns max |phi|.
__device__ void fb_rows(const ContactArgs& C, const double* dfree, const double* lam, double* phi, double* om,
                        double* E, double* red) {
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6, nw = blockDim.x >> 6;
  const int K = C.K;
  double mx = 0.0;
  for (int c = wid; c < K; c += nw) {
    const double* Wr = C.W + (size_t)c * K;
    double acc = 0.0;
    for (int d = lane; d < K; d += 64) acc += Wr[d] * lam[d];
    acc = wsum(acc);
    if (lane == 0) {
      const double delta = dfree[c] + acc;
      const double r = Wr[c], a = delta, b = r * lam[c];
      const double sq = sqrt(a * a + b * b);
      double p, w, e;
      if (C.kind && C.kind[c] == 1) {  // bilateral: the gap itself is the residual
        p = delta;
        w = 1.0;
        e = 0.0;
      } else if (sq == 0.0) {
        p = 0.0;
        w = 1.0 - 1.0 / sqrt(2.0);
        e = r * (1.0 - 1.0 / sqrt(2.0));
      } else {
        p = a + b - sq;
        w = 1.0 - a / sq;
        e = r * (1.0 - b / sq);
      }
      phi[c] = p;
      om[c] = w;
      E[c] = e;
      mx = fmax(mx, fabs(p));
    }
  }
  mx = wmax(mx);
  if (lane == 0) red[wid] = mx;
  __syncthreads();
  if (tid == 0) {
    double m = 0.0;
    for (int w = 0; w < nw; ++w) m = fmax(m, red[w]);
    red[16] = m;
  }
  __syncthreads();
}

// In-place Cholesky of the packed lower triangle L (rows 0..n-1) with the
// right-hand side as row n: afterwards row n holds L^{-1} rhs.  Returns false
// (uniformly) if a pivot is not positive.
__device__ bool chol_packed(double* L, int n, bool with_rhs, int* fail) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int last = with_rhs ? n : n - 1;  // last row updated
  for (int j = 0; j < n; ++j) {
    const double piv = L[tri(j) + j];
    if (!(piv > 0.0)) {
      if (tid == 0) *fail = 1;
      return false;
    }
    const double d = sqrt(piv);
    __syncthreads();
    if (tid == 0) L[tri(j) + j] = d;
    for (int i = j + 1 + tid; i <= last; i += nt) L[tri(i) + j] /= d;
    __syncthreads();
    // trailing update of rows i in (j, last], columns l in (j, min(i, n - 1)]
    const int R = last - j, Cn = n - 1 - j;
    if (Cn > 0) {
      const int cnt = R * Cn;
      for (int p = tid; p < cnt; p += nt) {
        const int i = j + 1 + p / Cn, l = j + 1 + p % Cn;
        if (l <= i) L[tri(i) + l] -= L[tri(i) + j] * L[tri(l) + j];
      }
    }
    __syncthreads();
  }
  return true;
}

// Newton on the FB residual of the rows whose weight omega exceeds 1e-12:
// (W_AA + diag(E / omega)) dlam = -phi / omega, lam <- max(lam + dlam, 0),
// the other rows at 0; at most kFBMaxIter steps, stopping at max |phi| <=
// 1e-14 (Eq. contact_system in role, READING symmetrised).  lam carries over
// between PD iterations.  Writes s = lam_c n_c and the residual.
__global__ void __launch_bounds__(kContactThreads) k_contact_fb(VertArgs Vx, ContactArgs C,
                                                                const double* __restrict__ qhat,
                                                                const int* __restrict__ done) {
  __shared__ double L[tri(kMaxNewtonRows + 1) + kMaxNewtonRows + 1];
  __shared__ double dfree[kMaxContactRows], lam[kMaxContactRows], phi[kMaxContactRows], om[kMaxContactRows],
      Ev[kMaxContactRows];
  __shared__ int act[kMaxContactRows];
  __shared__ double red[17];
  __shared__ int na_s, flag_s, fail_s;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int K = C.K, nv = Vx.nv;
  if (tid == 0) {
    flag_s = done ? *done : 0;
    fail_s = 0;
  }
  double q0 = 0, q1 = 0, q2 = 0, l0 = 0;
  if (tid < K) {
    const int v = C.v[tid];
    q0 = qhat[v];
    q1 = qhat[nv + v];
    q2 = qhat[2 * nv + v];
    l0 = C.lam[tid];
  }
  __syncthreads();
  if (flag_s) return;
  // K <= kMaxContactRows < blockDim (checked by the host): one row per thread
  if (tid < K) {
    dfree[tid] = C.n[3 * tid] * q0 + C.n[3 * tid + 1] * q1 + C.n[3 * tid + 2] * q2 - C.g[tid];
    lam[tid] = l0;
  }
  __syncthreads();
  fb_rows(C, dfree, lam, phi, om, Ev, red);
  double res = red[16];
  int it = 0;
  for (; it < kFBMaxIter && res > kFBTol; ++it) {
    if (tid == 0) {
      int na = 0;
      for (int c = 0; c < K; ++c) {
        if (om[c] > kOmegaMin) act[na++] = c;
        else lam[c] = 0.0;
      }
      na_s = na;
    }
    __syncthreads();
    const int na = na_s;
    // systems beyond the LDS size are factored in the global scratch (L2-resident)
    double* Lm = (na <= kMaxNewtonRows) ? L : C.Lg;
    if (na > 0) {
      // M = W_AA + diag(E / omega) (lower triangle) and rhs = -phi / omega as row na
      const int cntM = tri(na);
      for (int p = tid; p < cntM + na; p += nt) {
        if (p < cntM) {
          int i = (int)((sqrt(8.0 * p + 1.0) - 1.0) * 0.5);
          while (tri(i + 1) <= p) ++i;
          while (tri(i) > p) --i;
          const int j = p - tri(i);
          const int ci = act[i], cj = act[j];
          double m = C.W[(size_t)ci * K + cj];
          if (i == j) m += Ev[ci] / om[ci];
          Lm[p] = m;
        } else {
          const int j = p - cntM, cj = act[j];
          Lm[cntM + j] = -phi[cj] / om[cj];
        }
      }
      __syncthreads();
      if (!chol_packed(Lm, na, true, &fail_s)) break;
      // back substitution L^T x = y, y in row na
      double* y = Lm + tri(na);
      for (int i = na - 1; i >= 0; --i) {
        if (tid == 0) y[i] = y[i] / Lm[tri(i) + i];
        __syncthreads();
        const double xi = y[i];
        for (int j = tid; j < i; j += nt) y[j] -= Lm[tri(i) + j] * xi;
        __syncthreads();
      }
      for (int a = tid; a < na; a += nt) {
        const int c = act[a];
        const double l = lam[c] + y[a];
        lam[c] = (l > 0.0 || (C.kind && C.kind[c] == 1)) ? l : 0.0;
      }
    }
    __syncthreads();
    fb_rows(C, dfree, lam, phi, om, Ev, red);
    res = red[16];
  }
  for (int c = tid; c < K; c += nt) {
    const double l = lam[c];
    C.lam[c] = l;
    C.s[3 * c] = l * C.n[3 * c];
    C.s[3 * c + 1] = l * C.n[3 * c + 1];
    C.s[3 * c + 2] = l * C.n[3 * c + 2];
  }
  if (tid == 0) {
    C.fb[0] = res;
    C.fb[1] = (double)it;
    if (fail_s) C.flags[2] = 1;
  }
}


// The same Newton for at most 64 rows, one row per lane of a single wave:
// W is staged in LDS once; the FB values, the active compaction (ballot), the
// dense system, its left-looking Cholesky (lane i forms row i of each column
// from the finished columns, the pivot comes by shuffle) and both
// substitutions need no workgroup barrier beyond the single wave's own.
__global__ void __launch_bounds__(64) k_contact_fb_wave(VertArgs Vx, ContactArgs C, const double* __restrict__ qhat,
                                                        const int* __restrict__ done) {
  __shared__ double M[64 * 65];   // Newton matrix, row i at M[i * 65] (lower triangle, then L)
  __shared__ double Ws[64 * 65];  // W, row c at Ws[c * 65]
  __shared__ double lam_s[64];
  const int lane = threadIdx.x;
  const int K = C.K, nv = Vx.nv;
  const bool row = lane < K;
  int flag = done ? *done : 0;
  double q0 = 0, q1 = 0, q2 = 0, n0 = 0, n1 = 0, n2 = 0, g = 0, lam = 0;
  const bool bil = row && C.kind && C.kind[lane] == 1;  // bilateral row
  if (row) {
    const int v = C.v[lane];
    q0 = qhat[v];
    q1 = qhat[nv + v];
    q2 = qhat[2 * nv + v];
    n0 = C.n[3 * lane];
    n1 = C.n[3 * lane + 1];
    n2 = C.n[3 * lane + 2];
    g = C.g[lane];
    lam = C.lam[lane];
  }
  for (int idx = lane; idx < K * K; idx += 64) {
    const int c = idx / K, d = idx - c * K;
    Ws[c * 65 + d] = C.W[idx];
  }
  flag = __shfl(flag, 0, 64);
  if (flag) return;
  __syncthreads();
  const double dfree = n0 * q0 + n1 * q1 + n2 * q2 - g;
  const double* Wr = Ws + (row ? lane : 0) * 65;
  double phi = 0.0, om = 0.0, E = 0.0;
  auto evaluate = [&]() {
    lam_s[lane] = lam;
    __syncthreads();
    double delta = dfree;
    if (row)
      for (int d = 0; d < K; ++d) delta += Wr[d] * lam_s[d];
    double mx = 0.0;
    if (row) {
      const double r = Wr[lane], a = delta, b = r * lam;
      const double sq = sqrt(a * a + b * b);
      if (bil) {
        phi = delta;
        om = 1.0;
        E = 0.0;
      } else if (sq == 0.0) {
        phi = 0.0;
        om = 1.0 - 1.0 / sqrt(2.0);
        E = r * (1.0 - 1.0 / sqrt(2.0));
      } else {
        const double is = 1.0 / sq;  // one division on the serial path
        phi = a + b - sq;
        om = 1.0 - a * is;
        E = r * (1.0 - b * is);
      }
      mx = fabs(phi);
    }
    __syncthreads();
    return wmax(mx);
  };
  double res = evaluate();
  int it = 0, fail = 0;
  for (; it < kFBMaxIter && res > kFBTol; ++it) {
    const bool a_on = row && om > kOmegaMin;
    if (row && !a_on) lam = 0.0;
    const unsigned long long bal = __ballot(a_on);
    const int na = __popcll(bal);
    const int pos = a_on ? __popcll(bal & ((1ull << lane) - 1ull)) : -1;
    // row pos of the system: W restricted to the active rows, + E / omega on the diagonal
    double b = 0.0;
    if (a_on) {
      double* Mi = M + pos * 65;
      unsigned long long rest = bal;
      int j = 0;
      while (rest && j <= pos) {
        const int d = __ffsll((long long)rest) - 1;
        rest &= rest - 1ull;
        Mi[j] = Wr[d] + (d == lane ? E / om : 0.0);
        ++j;
      }
      b = -phi / om;
    }
    // lane p takes the rhs of system row p (the p-th active row)
    double y = 0.0;
    {
      unsigned long long rest = bal;
      int p = 0, src = 0;
      while (rest) {
        const int d = __ffsll((long long)rest) - 1;
        rest &= rest - 1ull;
        if (p == lane) src = d;
        ++p;
      }
      y = __shfl(b, src, 64);
      if (lane >= na) y = 0.0;
    }
    __syncthreads();
    // left-looking Cholesky, lane i owns row i
    bool ok = true;
    for (int j = 0; j < na; ++j) {
      double sv = 0.0;
      if (lane >= j && lane < na) {
        const double* Mi = M + lane * 65;
        const double* Mj = M + j * 65;
        sv = Mi[j];
        for (int k = 0; k < j; ++k) sv -= Mi[k] * Mj[k];
      }
      const double piv = __shfl(sv, j, 64);
      if (!(piv > 0.0)) {
        ok = false;
        break;
      }
      // the diagonal keeps 1 / L_jj, so neither substitution divides
      const double ij = 1.0 / sqrt(piv);
      if (lane == j) M[j * 65 + j] = ij;
      else if (lane > j && lane < na) M[lane * 65 + j] = sv * ij;
      __syncthreads();
    }
    if (!ok) {
      fail = 1;
      break;
    }
    // forward substitution L z = y, then back substitution L^T x = z (lane p holds entry p)
    for (int j = 0; j < na; ++j) {
      const double zj = __shfl(y, j, 64) * M[j * 65 + j];
      if (lane == j) y = zj;
      else if (lane > j && lane < na) y -= M[lane * 65 + j] * zj;
    }
    for (int i = na - 1; i >= 0; --i) {
      const double xi = __shfl(y, i, 64) * M[i * 65 + i];
      if (lane == i) y = xi;
      if (lane < i) y -= M[i * 65 + lane] * xi;
    }
    // dlam of active row pos sits in lane pos
    const double dl = __shfl(y, pos < 0 ? 0 : pos, 64);
    if (a_on) {
      const double l = lam + dl;
      lam = (l > 0.0 || bil) ? l : 0.0;
    }
    __syncthreads();
    res = evaluate();
  }
  if (row) {
    C.lam[lane] = lam;
    C.s[3 * lane] = lam * n0;
    C.s[3 * lane + 1] = lam * n1;
    C.s[3 * lane + 2] = lam * n2;
  }
  if (lane == 0) {
    C.fb[0] = res;
    C.fb[1] = (double)it;
    if (fail) C.flags[2] = 1;
  }
}

// ---------------------------------------------------------------- adjoint
// Inverse of W_AA (the active rows, K = n_active here) by Cholesky in LDS and
// one substitution pair per column (one thread per column).
__global__ void __launch_bounds__(kContactThreads) k_contact_winv(ContactArgs C, double* __restrict__ Winv) {
  __shared__ double Ls[tri(kMaxNewtonRows) + 1];
  __shared__ int fail_s;
  const int tid = threadIdx.x, nt = blockDim.x, na = C.K, nf = C.nf;
  double* L = (na <= kMaxNewtonRows) ? Ls : C.Lg;
  if (tid == 0) fail_s = 0;
  for (int p = tid; p < tri(na); p += nt) {
    int i = (int)((sqrt(8.0 * p + 1.0) - 1.0) * 0.5);
    while (tri(i + 1) <= p) ++i;
    while (tri(i) > p) --i;
    const int j = p - tri(i);
    const double nn = C.n[3 * i] * C.n[3 * j] + C.n[3 * i + 1] * C.n[3 * j + 1] + C.n[3 * i + 2] * C.n[3 * j + 2];
    L[p] = nn * C.cols[(size_t)C.slot[i] * nf + C.v[j]];
  }
  __syncthreads();
  if (!chol_packed(L, na, false, &fail_s)) {
    if (tid == 0) C.flags[2] = 1;
    return;
  }
  for (int j = tid; j < na; j += nt) {
    // column j: forward L y = e_j, back L^T x = y, stored in Winv[:, j]
    for (int i = 0; i < na; ++i) {
      double t = (i == j) ? 1.0 : 0.0;
      if (i > j)
        for (int k = j; k < i; ++k) t -= L[tri(i) + k] * Winv[(size_t)k * na + j];
      Winv[(size_t)i * na + j] = (i < j) ? 0.0 : t / L[tri(i) + i];
    }
    for (int i = na - 1; i >= 0; --i) {
      double t = Winv[(size_t)i * na + j];
      for (int k = i + 1; k < na; ++k) t -= L[tri(k) + i] * Winv[(size_t)k * na + j];
      Winv[(size_t)i * na + j] = t / L[tri(i) + i];
    }
  }
}

// u = W_AA^{-1} (J_A z), s = u_c n_c (z = A~^{-1} r, the unprojected solve);
// with friction the rows are measured along nb and act along n, and W holds
// the inverse of their coupling matrix
__global__ void __launch_bounds__(256) k_contact_proj(VertArgs Vx, ContactArgs C, const double* __restrict__ z,
                                                      const int* __restrict__ done) {
  __shared__ double y[kMaxAdjRows];
  __shared__ int flag_s;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6, nw = blockDim.x >> 6;
  const int na = C.K, nv = Vx.nv;
  const double* mb = C.nb ? C.nb : C.n;
  if (tid == 0) flag_s = done ? *done : 0;
  double yv[kMaxAdjRows / 256];
#pragma unroll
  for (int r = 0; r < kMaxAdjRows / 256; ++r) {
    const int c = tid + 256 * r;
    yv[r] = 0.0;
    if (c < na) {
      const int v = C.v[c];
      yv[r] = mb[3 * c] * z[v] + mb[3 * c + 1] * z[nv + v] + mb[3 * c + 2] * z[2 * nv + v];
    }
  }
  __syncthreads();
  if (flag_s) return;
#pragma unroll
  for (int r = 0; r < kMaxAdjRows / 256; ++r)
    if (tid + 256 * r < na) y[tid + 256 * r] = yv[r];
  __syncthreads();
  for (int c = wid; c < na; c += nw) {
    const double* Wr = C.W + (size_t)c * na;
    double acc = 0.0;
    for (int d = lane; d < na; d += 64) acc += Wr[d] * y[d];
    acc = wsum(acc);
    if (lane == 0) {
      C.s[3 * c] = acc * C.n[3 * c];
      C.s[3 * c + 1] = acc * C.n[3 * c + 1];
      C.s[3 * c + 2] = acc * C.n[3 * c + 2];
    }
  }
}

// checkpoint record of the step's rows: K, then v (as doubles), n (3 each),
// g, lam (with friction the tangential impulses, 2 each), the row kinds and
// the restitution flags, each block kmax long, then the restitution
// coefficient (negative: off)
__global__ void __launch_bounds__(kBlock) k_contact_ckpt(ContactArgs C, int kmax, double e_rest,
                                                          double* __restrict__ rec) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c == 0) {
    rec[0] = (double)C.K;
    rec[1 + 10 * kmax] = e_rest;
  }
  if (c >= C.K) return;
  rec[1 + c] = (double)C.v[c];
  rec[1 + kmax + 3 * c] = C.n[3 * c];
  rec[1 + kmax + 3 * c + 1] = C.n[3 * c + 1];
  rec[1 + kmax + 3 * c + 2] = C.n[3 * c + 2];
  rec[1 + 4 * kmax + c] = C.g[c];
  if (C.mu > 0.0) {
    rec[1 + 5 * kmax + c] = C.lam[3 * c];
    rec[1 + 6 * kmax + 2 * c] = C.lam[3 * c + 1];
    rec[1 + 6 * kmax + 2 * c + 1] = C.lam[3 * c + 2];
  } else {
    rec[1 + 5 * kmax + c] = C.lam[c];
  }
  rec[1 + 8 * kmax + c] = (C.kind && C.kind[c] == 1) ? 1.0 : 0.0;
  rec[1 + 9 * kmax + c] = 0.0;  // restitution flag, set by the restitution kernel
}

// ---------------------------------------------------------------- restitution
// Active unilateral rows (normal impulse above 1e-10 of the largest
// unilateral one) whose vertex approached (u = n . v_t < 0) set the vertex's
// outgoing normal velocity to -e u: v <- v + n (-e u - n . v).  Rows of one
// vertex are contiguous (detection order); the first row of each run applies
// them in order.  One workgroup; K <= kMaxContactRows.
__global__ void __launch_bounds__(kContactThreads) k_contact_restitution(VertArgs Vx, ContactArgs C,
                                                                         const double* __restrict__ v_t,
                                                                         double* __restrict__ v_next, double e,
                                                                         double* __restrict__ rec, int kmax) {
  __shared__ double red[16];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6, K = C.K;
  const int stride = C.mu > 0.0 ? 3 : 1;
  double m = 0.0;
  for (int c = tid; c < K; c += blockDim.x)
    if (!(C.kind && C.kind[c] == 1)) m = fmax(m, C.lam[stride * c]);
  m = wmax(m);
  if (lane == 0) red[wid] = m;
  __syncthreads();
  double lmax = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) lmax = fmax(lmax, red[w]);
  for (int c = tid; c < K; c += blockDim.x) {
    const int v = C.v[c];
    if (c > 0 && C.v[c - 1] == v) continue;
    const int o = Vx.v_orig[v];
    double vv[3] = {v_next[3 * o], v_next[3 * o + 1], v_next[3 * o + 2]};
    const double vi[3] = {v_t[3 * o], v_t[3 * o + 1], v_t[3 * o + 2]};
    bool any = false;
    for (int d = c; d < K && C.v[d] == v; ++d) {
      if ((C.kind && C.kind[d] == 1) || !(lmax > 0.0 && C.lam[stride * d] > 1e-10 * lmax)) continue;
      const double* n = C.n + 3 * d;
      const double u = n[0] * vi[0] + n[1] * vi[1] + n[2] * vi[2];
      if (!(u < 0.0)) continue;
      const double vn = n[0] * vv[0] + n[1] * vv[1] + n[2] * vv[2];
#pragma unroll
      for (int a = 0; a < 3; ++a) vv[a] += n[a] * (-e * u - vn);
      if (rec) rec[1 + 9 * kmax + d] = 1.0;
      any = true;
    }
    if (any)
#pragma unroll
      for (int a = 0; a < 3; ++a) v_next[3 * o + a] = vv[a];
  }
}

// the adjoint before the backward step: rows of a vertex in reverse order,
// v bar <- v bar - n (n . v bar), the product kept per row
__global__ void __launch_bounds__(kContactThreads) k_restitution_adj_pre(VertArgs Vx, const double* __restrict__ rec,
                                                                         int kmax, double* __restrict__ gv,
                                                                         double* __restrict__ s_row) {
  const int K = (int)rec[0];
  for (int c = threadIdx.x; c < K; c += blockDim.x) {
    const int v = (int)rec[1 + c];
    if (c < K - 1 && (int)rec[2 + c] == v) continue;  // the last row of the run walks it backwards
    const int o = Vx.v_orig[v];
    double g[3] = {gv[3 * o], gv[3 * o + 1], gv[3 * o + 2]};
    bool any = false;
    for (int d = c; d >= 0 && (int)rec[1 + d] == v; --d) {
      if (rec[1 + 9 * kmax + d] != 1.0) continue;
      const double* n = rec + 1 + kmax + 3 * d;
      const double p = n[0] * g[0] + n[1] * g[1] + n[2] * g[2];
      s_row[d] = p;
#pragma unroll
      for (int a = 0; a < 3; ++a) g[a] -= n[a] * p;
      any = true;
    }
    if (any)
#pragma unroll
      for (int a = 0; a < 3; ++a) gv[3 * o + a] = g[a];
  }
}

// after it: dL/dv_t += -e n s_row of every flagged row (rows of one vertex summed in order)
__global__ void __launch_bounds__(kContactThreads) k_restitution_adj_post(VertArgs Vx, const double* __restrict__ rec,
                                                                          int kmax, const double* __restrict__ s_row,
                                                                          double* __restrict__ gv_t) {
  const int K = (int)rec[0];
  const double e = rec[1 + 10 * kmax];
  for (int c = threadIdx.x; c < K; c += blockDim.x) {
    const int v = (int)rec[1 + c];
    if (c > 0 && (int)rec[c] == v) continue;
    const int o = Vx.v_orig[v];
    double g[3] = {0.0, 0.0, 0.0};
    bool any = false;
    for (int d = c; d < K && (int)rec[1 + d] == v; ++d) {
      if (rec[1 + 9 * kmax + d] != 1.0) continue;
      const double* n = rec + 1 + kmax + 3 * d;
#pragma unroll
      for (int a = 0; a < 3; ++a) g[a] += -e * n[a] * s_row[d];
      any = true;
    }
    if (any)
#pragma unroll
      for (int a = 0; a < 3; ++a) gv_t[3 * o + a] += g[a];
  }
}


// ---------------------------------------------------------------- friction
// Coulomb friction (Sec. 4.7 with the block projection onto the friction
// disk).  Contact c acts on vertex v_c through the frame (n, t1, t2) with
// t1 = (a - (a.n) n)/|a - (a.n) n| for a the coordinate axis of the smallest
// |n_i| (first on ties) and t2 = n x t1.  Its kinematics are the gap
// delta = n.q - g and the slip s = T^T (q - q_t) over the step; with
// G_cd = a_{v_c}[v_d] the rows of two frames couple by (e_r . e_s) G_cd, and
// every row of contact c has the diagonal w_c = G_cc.
__device__ __forceinline__ void contact_frame(const double n[3], double t1[3], double t2[3]) {
  int k = 0;
  if (fabs(n[1]) < fabs(n[k])) k = 1;
  if (fabs(n[2]) < fabs(n[k])) k = 2;
  const double an = n[k];
  double t[3], nrm = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    t[i] = (i == k ? 1.0 : 0.0) - an * n[i];
    nrm += t[i] * t[i];
  }
  nrm = sqrt(nrm);
#pragma unroll
  for (int i = 0; i < 3; ++i) t1[i] = t[i] / nrm;
  t2[0] = n[1] * t1[2] - n[2] * t1[1];
  t2[1] = n[2] * t1[0] - n[0] * t1[2];
  t2[2] = n[0] * t1[1] - n[1] * t1[0];
}

namespace {
// offsets (in units of K) of the friction scratch
enum { kFrE = 0, kFrU0 = 9, kFrU = 12, kFrRB = 15, kFrDiag = 24, kFrRhs = 27, kFrDl = 30, kFrRot = 33, kFrImp = 37,
       kFrY = 40 };
}  // namespace

// u = u0 + W lam for every row: the world impulse of each contact, then one
// wave per contact sums G_cd imp_d; returns max over contacts of the
// residual max(|phi_FB|, w |F_f|) (identical in every thread).
__device__ double fr_eval(const ContactArgs& C, double* red) {
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6, nw = blockDim.x >> 6, nt = blockDim.x;
  const int K = C.K;
  double* e = C.frw + kFrE * K;
  double* imp = C.frw + kFrImp * K;
  double* u0 = C.frw + kFrU0 * K;
  double* u = C.frw + kFrU * K;
  for (int c = tid; c < K; c += nt) {
    const double* l = C.lam + 3 * c;
    const double* ec = e + 9 * c;
#pragma unroll
    for (int a = 0; a < 3; ++a) imp[3 * c + a] = l[0] * ec[a] + l[1] * ec[3 + a] + l[2] * ec[6 + a];
  }
  __syncthreads();
  for (int c = wid; c < K; c += nw) {
    const double* Gr = C.W + (size_t)c * K;
    double y0 = 0.0, y1 = 0.0, y2 = 0.0;
    for (int d = lane; d < K; d += 64) {
      const double gcd = Gr[d];
      y0 += gcd * imp[3 * d];
      y1 += gcd * imp[3 * d + 1];
      y2 += gcd * imp[3 * d + 2];
    }
    y0 = wsum(y0);
    y1 = wsum(y1);
    y2 = wsum(y2);
    if (lane == 0) {
      const double* ec = e + 9 * c;
#pragma unroll
      for (int a = 0; a < 3; ++a)
        u[3 * c + a] = u0[3 * c + a] + (ec[3 * a] * y0 + ec[3 * a + 1] * y1 + ec[3 * a + 2] * y2);
    }
  }
  __syncthreads();
  double mx = 0.0;
  for (int c = tid; c < K; c += nt) {
    const double w = C.W[(size_t)c * K + c];
    const double* l = C.lam + 3 * c;
    const double a = u[3 * c], bb = w * l[0];
    const double phi = a + bb - sqrt(a * a + bb * bb);
    const double tau = C.mu * l[0];
    const double z1 = l[1] - u[3 * c + 1] / w, z2 = l[2] - u[3 * c + 2] / w;
    const double nz = sqrt(z1 * z1 + z2 * z2);
    double p1 = z1, p2 = z2;
    if (tau <= 0.0) {
      p1 = 0.0;
      p2 = 0.0;
    } else if (nz > tau) {
      p1 = tau * z1 / nz;
      p2 = tau * z2 / nz;
    }
    const double F1 = l[1] - p1, F2 = l[2] - p2;
    mx = fmax(mx, fmax(fabs(phi), w * sqrt(F1 * F1 + F2 * F2)));
  }
  mx = wmax(mx);
  if (lane == 0) red[wid] = mx;
  __syncthreads();
  if (tid == 0) {
    double m = 0.0;
    for (int w = 0; w < nw; ++w) m = fmax(m, red[w]);
    red[16] = m;
  }
  __syncthreads();
  return red[16];
}

// One frictional contact solve per PD iteration, one 1024-thread workgroup:
// semi-smooth Newton with the Fischer-Burmeister normal row (Eqs. fb_n,
// omega_E_n, r_c = w_c) and the natural map of the friction disk of radius
// tau = mu lam_n (tau at the current iterate).  Per step: a normal row is
// free if omega > 1e-12 (W_n dl + E/omega dl_n = -phi/omega), else fixed at
// dl_n = -lam_n; tau = 0 fixes both tangent rows at -lam_f; |z| <= tau (z =
// lam_f - s/w: stick) frees both with W_f dl = -s; |z| > tau (slide) turns the
// tangent basis to (z^, z^perp), fixes dl_z = tau - lam_f.z^ and frees the
// perpendicular row with the diagonal w (1 - kappa)/kappa and right-hand side
// -w F_perp/kappa (kappa = tau/|z|).  The free rows form W's principal block
// plus a non-negative diagonal (SPD), factored by Cholesky with the fixed
// increments moved to the right-hand side; then lam_n <- max(lam_n, 0) and
// lam_f is projected onto the disk.  At most kFrMaxIter steps, stop at a
// residual <= kFBTol; lam carries over between PD iterations.  Writes each
// contact's world impulse to s.
__global__ void __launch_bounds__(kContactThreads) k_contact_fr(VertArgs Vx, ContactArgs C,
                                                                const double* __restrict__ qhat,
                                                                const int* __restrict__ done) {
  __shared__ double L[tri(kMaxNewtonRows + 1) + kMaxNewtonRows + 1];
  __shared__ double red[17];
  __shared__ int nfr_s, flag_s, fail_s;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6, nw = blockDim.x >> 6, nt = blockDim.x;
  const int K = C.K, nv = Vx.nv;
  if (tid == 0) {
    flag_s = done ? *done : 0;
    fail_s = 0;
  }
  __syncthreads();
  if (flag_s) return;
  double* e = C.frw + kFrE * K;
  double* u0 = C.frw + kFrU0 * K;
  double* u = C.frw + kFrU * K;
  double* rb = C.frw + kFrRB * K;
  double* diag = C.frw + kFrDiag * K;
  double* rhs = C.frw + kFrRhs * K;
  double* dl = C.frw + kFrDl * K;
  double* rot = C.frw + kFrRot * K;
  double* imp = C.frw + kFrImp * K;
  int* isfree = C.fri;
  int* frl = C.fri + 3 * K;
  // frames and the free kinematics at qhat
  for (int c = tid; c < K; c += nt) {
    const int v = C.v[c];
    double n[3] = {C.n[3 * c], C.n[3 * c + 1], C.n[3 * c + 2]}, t1[3], t2[3];
    contact_frame(n, t1, t2);
    double* ec = e + 9 * c;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      ec[a] = n[a];
      ec[3 + a] = t1[a];
      ec[6 + a] = t2[a];
    }
    const double q[3] = {qhat[v], qhat[nv + v], qhat[2 * nv + v]};
    const double p[3] = {C.qt[v], C.qt[nv + v], C.qt[2 * nv + v]};
    u0[3 * c] = n[0] * q[0] + n[1] * q[1] + n[2] * q[2] - C.g[c];
    u0[3 * c + 1] = t1[0] * (q[0] - p[0]) + t1[1] * (q[1] - p[1]) + t1[2] * (q[2] - p[2]);
    u0[3 * c + 2] = t2[0] * (q[0] - p[0]) + t2[1] * (q[1] - p[1]) + t2[2] * (q[2] - p[2]);
  }
  __syncthreads();
  double res = fr_eval(C, red);
  int it = 0;
  for (; it < kFrMaxIter && res > kFBTol; ++it) {
    // classify every contact's rows
    for (int c = tid; c < K; c += nt) {
      const double w = C.W[(size_t)c * K + c];
      const double* l = C.lam + 3 * c;
      const double* ec = e + 9 * c;
      const double a = u[3 * c], bb = w * l[0], sq = sqrt(a * a + bb * bb);
      double phi, om, E;
      if (sq == 0.0) {
        phi = 0.0;
        om = 1.0 - 1.0 / sqrt(2.0);
        E = w * (1.0 - 1.0 / sqrt(2.0));
      } else {
        phi = a + bb - sq;
        om = 1.0 - a / sq;
        E = w * (1.0 - bb / sq);
      }
#pragma unroll
      for (int i = 0; i < 3; ++i) rb[9 * c + i] = ec[i];
      if (om > kOmegaMin) {
        isfree[3 * c] = 1;
        diag[3 * c] = E / om;
        rhs[3 * c] = -phi / om;
      } else {
        isfree[3 * c] = 0;
        dl[3 * c] = -l[0];
      }
      const double tau = C.mu * l[0];
      const double z1 = l[1] - u[3 * c + 1] / w, z2 = l[2] - u[3 * c + 2] / w;
      const double nz = sqrt(z1 * z1 + z2 * z2);
      double B0 = 1.0, B1 = 0.0, B2 = 0.0, B3 = 1.0;
      if (tau <= 0.0) {
        isfree[3 * c + 1] = 0;
        isfree[3 * c + 2] = 0;
        dl[3 * c + 1] = -l[1];
        dl[3 * c + 2] = -l[2];
      } else if (nz <= tau) {
        isfree[3 * c + 1] = 1;
        isfree[3 * c + 2] = 1;
        diag[3 * c + 1] = 0.0;
        diag[3 * c + 2] = 0.0;
        rhs[3 * c + 1] = -u[3 * c + 1];
        rhs[3 * c + 2] = -u[3 * c + 2];
      } else {
        const double h1 = z1 / nz, h2 = z2 / nz, kap = tau / nz;
        B0 = h1;
        B1 = h2;
        B2 = -h2;
        B3 = h1;
        const double lz = l[1] * h1 + l[2] * h2, lp = -l[1] * h2 + l[2] * h1;
        isfree[3 * c + 1] = 0;
        dl[3 * c + 1] = tau - lz;
        isfree[3 * c + 2] = 1;
        diag[3 * c + 2] = w * (1.0 - kap) / kap;
        rhs[3 * c + 2] = -w * lp / kap;
      }
      double* R = rot + 4 * c;
      R[0] = B0;
      R[1] = B1;
      R[2] = B2;
      R[3] = B3;
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        rb[9 * c + 3 + i] = B0 * ec[3 + i] + B1 * ec[6 + i];
        rb[9 * c + 6 + i] = B2 * ec[3 + i] + B3 * ec[6 + i];
      }
    }
    __syncthreads();
    if (tid == 0) {
      int nfr = 0;
      for (int r = 0; r < 3 * K; ++r)
        if (isfree[r]) frl[nfr++] = r;
      nfr_s = nfr;
    }
    // world increments of the fixed rows
    for (int c = tid; c < K; c += nt) {
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        double acc = 0.0;
#pragma unroll
        for (int a = 0; a < 3; ++a)
          if (!isfree[3 * c + a]) acc += dl[3 * c + a] * rb[9 * c + 3 * a + i];
        imp[3 * c + i] = acc;
      }
    }
    __syncthreads();
    // right-hand sides of the free rows lose the fixed rows' coupling
    for (int c = wid; c < K; c += nw) {
      const double* Gr = C.W + (size_t)c * K;
      double y0 = 0.0, y1 = 0.0, y2 = 0.0;
      for (int d = lane; d < K; d += 64) {
        const double gcd = Gr[d];
        y0 += gcd * imp[3 * d];
        y1 += gcd * imp[3 * d + 1];
        y2 += gcd * imp[3 * d + 2];
      }
      y0 = wsum(y0);
      y1 = wsum(y1);
      y2 = wsum(y2);
      if (lane < 3 && isfree[3 * c + lane]) {
        const double* r = rb + 9 * c + 3 * lane;
        rhs[3 * c + lane] -= r[0] * y0 + r[1] * y1 + r[2] * y2;
      }
    }
    __syncthreads();
    const int nfr = nfr_s;
    double* Lm = (nfr <= kMaxNewtonRows) ? L : C.Lg;
    if (nfr > 0) {
      const int cntM = tri(nfr);
      for (int p = tid; p < cntM + nfr; p += nt) {
        if (p < cntM) {
          int i = (int)((sqrt(8.0 * p + 1.0) - 1.0) * 0.5);
          while (tri(i + 1) <= p) ++i;
          while (tri(i) > p) --i;
          const int j = p - tri(i);
          const int ri = frl[i], rj = frl[j];
          const int ci = ri / 3, cj = rj / 3;
          const double* a = rb + 9 * ci + 3 * (ri - 3 * ci);
          const double* b = rb + 9 * cj + 3 * (rj - 3 * cj);
          double m = (a[0] * b[0] + a[1] * b[1] + a[2] * b[2]) * C.W[(size_t)ci * K + cj];
          if (i == j) m += diag[ri];
          Lm[p] = m;
        } else {
          Lm[p] = rhs[frl[p - cntM]];
        }
      }
      __syncthreads();
      if (!chol_packed(Lm, nfr, true, &fail_s)) break;
      double* y = Lm + tri(nfr);
      for (int i = nfr - 1; i >= 0; --i) {
        if (tid == 0) y[i] = y[i] / Lm[tri(i) + i];
        __syncthreads();
        const double xi = y[i];
        for (int j = tid; j < i; j += nt) y[j] -= Lm[tri(i) + j] * xi;
        __syncthreads();
      }
      for (int i = tid; i < nfr; i += nt) dl[frl[i]] = y[i];
    }
    __syncthreads();
    // update in the (t1, t2) frame, then the block projection
    for (int c = tid; c < K; c += nt) {
      double* l = C.lam + 3 * c;
      const double* R = rot + 4 * c;
      double ln = l[0] + dl[3 * c];
      double f1 = l[1] + R[0] * dl[3 * c + 1] + R[2] * dl[3 * c + 2];
      double f2 = l[2] + R[1] * dl[3 * c + 1] + R[3] * dl[3 * c + 2];
      ln = ln > 0.0 ? ln : 0.0;
      const double tau = C.mu * ln, nfv = sqrt(f1 * f1 + f2 * f2);
      if (tau <= 0.0) {
        f1 = 0.0;
        f2 = 0.0;
      } else if (nfv > tau) {
        f1 *= tau / nfv;
        f2 *= tau / nfv;
      }
      l[0] = ln;
      l[1] = f1;
      l[2] = f2;
    }
    __syncthreads();
    res = fr_eval(C, red);
  }
  // the world impulse of every contact at the final lam
  for (int c = tid; c < K; c += nt) {
    const double* l = C.lam + 3 * c;
    const double* ec = e + 9 * c;
#pragma unroll
    for (int a = 0; a < 3; ++a) C.s[3 * c + a] = l[0] * ec[a] + l[1] * ec[3 + a] + l[2] * ec[6 + a];
  }
  if (tid == 0) {
    C.fb[0] = res;
    C.fb[1] = (double)it;
    if (fail_s) C.flags[2] = 1;
  }
}

// Inverse of the adjoint rows' coupling matrix M_rq = (b_r . c_q) a_{v_r}[v_q]
// + d_r [r = q] (b = nb, c = n; unsymmetric where a sliding contact's friction
// follows its normal impulse): LU with partial pivoting in the global scratch,
// then one thread per column solves L U x = P e_j into Minv.
__global__ void __launch_bounds__(kContactThreads) k_contact_minv(ContactArgs C, double* __restrict__ Minv) {
  __shared__ double pv[kContactThreads / 64];
  __shared__ int pi[kContactThreads / 64];
  __shared__ int piv_s;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6, nw = blockDim.x >> 6, nt = blockDim.x;
  const int n = C.K, nf = C.nf;
  double* A = C.Lg;
  int* perm = C.fri;
  for (int p = tid; p < n * n; p += nt) {
    const int r = p / n, q = p - r * n;
    const double* b = C.nb + 3 * r;
    const double* c = C.n + 3 * q;
    double m = (b[0] * c[0] + b[1] * c[1] + b[2] * c[2]) * C.cols[(size_t)C.slot[q] * nf + C.v[r]];
    if (r == q && C.dg) m += C.dg[r];
    A[p] = m;
  }
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    // pivot: the largest |A_ik|, i >= k (the first on ties)
    double best = -1.0;
    int bi = k;
    for (int i = k + tid; i < n; i += nt) {
      const double a = fabs(A[(size_t)i * n + k]);
      if (a > best) {
        best = a;
        bi = i;
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double ob = __shfl_xor(best, off, 64);
      const int oi = __shfl_xor(bi, off, 64);
      if (ob > best || (ob == best && oi < bi)) {
        best = ob;
        bi = oi;
      }
    }
    if (lane == 0) {
      pv[wid] = best;
      pi[wid] = bi;
    }
    __syncthreads();
    if (tid == 0) {
      double b = pv[0];
      int i0 = pi[0];
      for (int w = 1; w < nw; ++w)
        if (pv[w] > b || (pv[w] == b && pi[w] < i0)) {
          b = pv[w];
          i0 = pi[w];
        }
      piv_s = (b > 0.0) ? i0 : -1;
      perm[k] = i0;
    }
    __syncthreads();
    const int p = piv_s;
    if (p < 0) {
      if (tid == 0) C.flags[2] = 1;
      return;
    }
    if (p != k)
      for (int j = tid; j < n; j += nt) {
        const double t = A[(size_t)k * n + j];
        A[(size_t)k * n + j] = A[(size_t)p * n + j];
        A[(size_t)p * n + j] = t;
      }
    __syncthreads();
    const double akk = A[(size_t)k * n + k];
    for (int i = k + 1 + tid; i < n; i += nt) A[(size_t)i * n + k] /= akk;
    __syncthreads();
    const int R = n - 1 - k;
    for (int q = tid; q < R * R; q += nt) {
      const int i = k + 1 + q / R, j = k + 1 + q % R;
      A[(size_t)i * n + j] -= A[(size_t)i * n + k] * A[(size_t)k * n + j];
    }
    __syncthreads();
  }
  for (int j = tid; j < n; j += nt) {
    // x = P e_j: apply the row swaps in order, then the two substitutions
    double* x = Minv;  // column j, stride n
    for (int i = 0; i < n; ++i) x[(size_t)i * n + j] = (i == j) ? 1.0 : 0.0;
    for (int k = 0; k < n; ++k) {
      const int p = perm[k];
      if (p != k) {
        const double t = x[(size_t)k * n + j];
        x[(size_t)k * n + j] = x[(size_t)p * n + j];
        x[(size_t)p * n + j] = t;
      }
    }
    for (int i = 1; i < n; ++i) {
      double t = x[(size_t)i * n + j];
      for (int k = 0; k < i; ++k) t -= A[(size_t)i * n + k] * x[(size_t)k * n + j];
      x[(size_t)i * n + j] = t;
    }
    for (int i = n - 1; i >= 0; --i) {
      double t = x[(size_t)i * n + j];
      for (int k = i + 1; k < n; ++k) t -= A[(size_t)i * n + k] * x[(size_t)k * n + j];
      x[(size_t)i * n + j] = t / A[(size_t)i * n + i];
    }
  }
}

// slip displacement q* - q_t and the diagonal a_{v_c}[v_c] of each listed
// contact vertex: out[4c .. 4c+3]
__global__ void __launch_bounds__(kBlock) k_contact_slip(VertArgs Vx, ContactArgs C, const double* __restrict__ qs,
                                                         const double* __restrict__ qt, double* __restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C.K) return;
  const int v = C.v[c], nv = Vx.nv;
#pragma unroll
  for (int a = 0; a < 3; ++a) out[4 * c + a] = qs[a * nv + v] - qt[a * nv + v];
  out[4 * c + 3] = C.cols[(size_t)C.slot[c] * C.nf + v];
}

// dL/dq_t += u_r c_r of the sticking and sliding rows (kind != 0), in the
// caller's order; one thread walks the rows (several rows share a vertex)
__global__ void __launch_bounds__(64) k_contact_route(VertArgs Vx, ContactArgs C, const int* __restrict__ kind,
                                                      double* __restrict__ gq_t) {
  if (threadIdx.x != 0) return;
  for (int r = 0; r < C.K; ++r) {
    if (kind[r] == 0) continue;
    const int o = Vx.v_orig[C.v[r]];
#pragma unroll
    for (int a = 0; a < 3; ++a) gq_t[3 * o + a] += C.s[3 * r + a];
  }
}

// ---------------------------------------------------------------- launchers
void launch_contact_detect(const VertArgs& V, const double* qt, const double* vt, const ObsArgs& O, int kmax,
                           int* v, double* n, double* g, int* flags, hipStream_t s) {
  hipLaunchKernelGGL(k_contact_detect, dim3(1), dim3(kContactThreads), 0, s, V, qt, vt, O, kmax, v, n, g, flags);
}
void launch_unit_rhs(int nv, double* rhs, int v0, int v1, int v2, hipStream_t s) {
  hipLaunchKernelGGL(k_unit_rhs, dim3((nv + kBlock - 1) / kBlock), dim3(kBlock), 0, s, nv, rhs, v0, v1, v2);
}
void launch_store_cols(int nf, int nv, const double* x, double* cols, int s0, int s1, int s2, hipStream_t s) {
  hipLaunchKernelGGL(k_store_cols, dim3((nf + kBlock - 1) / kBlock), dim3(kBlock), 0, s, nf, nv, x, cols, s0, s1,
                     s2);
}
void launch_contact_W(const ContactArgs& C, double* W, hipStream_t s) {
  const int n = C.K * C.K;
  if (n > 0) hipLaunchKernelGGL(k_contact_W, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, C, W);
}
void launch_contact_start(const ContactArgs& C, hipStream_t s) {
  hipLaunchKernelGGL(k_contact_start, dim3((std::max(C.K, 1) + kBlock - 1) / kBlock), dim3(kBlock), 0, s, C);
}
void launch_contact_fb(const VertArgs& V, const ContactArgs& C, const double* qhat, const int* done, hipStream_t s) {
  if (C.K <= 64) hipLaunchKernelGGL(k_contact_fb_wave, dim3(1), dim3(64), 0, s, V, C, qhat, done);
  else hipLaunchKernelGGL(k_contact_fb, dim3(1), dim3(kContactThreads), 0, s, V, C, qhat, done);
}
void launch_contact_winv(const ContactArgs& C, double* Winv, hipStream_t s) {
  hipLaunchKernelGGL(k_contact_winv, dim3(1), dim3(kContactThreads), 0, s, C, Winv);
}
void launch_contact_proj(const VertArgs& V, const ContactArgs& C, const double* z, const int* done, hipStream_t s) {
  hipLaunchKernelGGL(k_contact_proj, dim3(1), dim3(256), 0, s, V, C, z, done);
}
void launch_contact_fr(const VertArgs& V, const ContactArgs& C, const double* qhat, const int* done, hipStream_t s) {
  hipLaunchKernelGGL(k_contact_fr, dim3(1), dim3(kContactThreads), 0, s, V, C, qhat, done);
}
void launch_contact_minv(const ContactArgs& C, double* Minv, hipStream_t s) {
  hipLaunchKernelGGL(k_contact_minv, dim3(1), dim3(kContactThreads), 0, s, C, Minv);
}
void launch_contact_slip(const VertArgs& V, const ContactArgs& C, const double* qstar, const double* qt, double* out,
                         hipStream_t s) {
  if (C.K > 0)
    hipLaunchKernelGGL(k_contact_slip, dim3((C.K + kBlock - 1) / kBlock), dim3(kBlock), 0, s, V, C, qstar, qt, out);
}
void launch_contact_route(const VertArgs& V, const ContactArgs& C, const int* kind, double* gq_t, hipStream_t s) {
  if (C.K > 0 && gq_t) hipLaunchKernelGGL(k_contact_route, dim3(1), dim3(64), 0, s, V, C, kind, gq_t);
}
void launch_contact_restitution(const VertArgs& V, const ContactArgs& C, const double* v_t, double* v_next, double e,
                                double* rec, int kmax, hipStream_t s) {
  if (C.K > 0)
    hipLaunchKernelGGL(k_contact_restitution, dim3(1), dim3(kContactThreads), 0, s, V, C, v_t, v_next, e, rec, kmax);
}
void launch_restitution_adj_pre(const VertArgs& V, const double* rec, int kmax, double* gv, double* s_row,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_restitution_adj_pre, dim3(1), dim3(kContactThreads), 0, s, V, rec, kmax, gv, s_row);
}
void launch_restitution_adj_post(const VertArgs& V, const double* rec, int kmax, const double* s_row,
                                 double* gv_t, hipStream_t s) {
  hipLaunchKernelGGL(k_restitution_adj_post, dim3(1), dim3(kContactThreads), 0, s, V, rec, kmax, s_row, gv_t);
}
void launch_contact_ckpt(const ContactArgs& C, int kmax, double e_rest, double* rec, hipStream_t s) {
  hipLaunchKernelGGL(k_contact_ckpt, dim3((std::max(C.K, 1) + kBlock - 1) / kBlock), dim3(kBlock), 0, s, C, kmax,
                     e_rest, rec);
}

}  // namespace pdhot
