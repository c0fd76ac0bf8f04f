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
          mask |= 1u << o;
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

// W_cd = (n_c . n_d) a_{v_c}[v_d]
__global__ void __launch_bounds__(kBlock) k_contact_W(ContactArgs C, double* __restrict__ W) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int K = C.K;
  if (idx >= K * K) return;
  const int c = idx / K, d = idx - c * K;
  const double nn = C.n[3 * c] * C.n[3 * d] + C.n[3 * c + 1] * C.n[3 * d + 1] + C.n[3 * c + 2] * C.n[3 * d + 2];
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
  C.lam[c] = 0.0;
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
      if (sq == 0.0) {
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
        lam[c] = l > 0.0 ? l : 0.0;
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
      if (sq == 0.0) {
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
      lam = l > 0.0 ? l : 0.0;
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

// u = W_AA^{-1} (J_A z), s = u_c n_c (z = A~^{-1} r, the unprojected solve)
__global__ void __launch_bounds__(256) k_contact_proj(VertArgs Vx, ContactArgs C, const double* __restrict__ z,
                                                      const int* __restrict__ done) {
  __shared__ double y[kMaxContactRows];
  __shared__ int flag_s;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6, nw = blockDim.x >> 6;
  const int na = C.K, nv = Vx.nv;
  if (tid == 0) flag_s = done ? *done : 0;
  double yv[kMaxContactRows / 256];
#pragma unroll
  for (int r = 0; r < kMaxContactRows / 256; ++r) {
    const int c = tid + 256 * r;
    yv[r] = 0.0;
    if (c < na) {
      const int v = C.v[c];
      yv[r] = C.n[3 * c] * z[v] + C.n[3 * c + 1] * z[nv + v] + C.n[3 * c + 2] * z[2 * nv + v];
    }
  }
  __syncthreads();
  if (flag_s) return;
#pragma unroll
  for (int r = 0; r < kMaxContactRows / 256; ++r)
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
// g and lam, each block kmax long
__global__ void __launch_bounds__(kBlock) k_contact_ckpt(ContactArgs C, int kmax, double* __restrict__ rec) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c == 0) rec[0] = (double)C.K;
  if (c >= C.K) return;
  rec[1 + c] = (double)C.v[c];
  rec[1 + kmax + 3 * c] = C.n[3 * c];
  rec[1 + kmax + 3 * c + 1] = C.n[3 * c + 1];
  rec[1 + kmax + 3 * c + 2] = C.n[3 * c + 2];
  rec[1 + 4 * kmax + c] = C.g[c];
  rec[1 + 5 * kmax + c] = C.lam[c];
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
void launch_contact_ckpt(const ContactArgs& C, int kmax, double* rec, hipStream_t s) {
  hipLaunchKernelGGL(k_contact_ckpt, dim3((std::max(C.K, 1) + kBlock - 1) / kBlock), dim3(kBlock), 0, s, C, kmax,
                     rec);
}

}  // namespace pdhot
