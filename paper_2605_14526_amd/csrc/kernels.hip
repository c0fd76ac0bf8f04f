// HIP kernels (gfx950) of the PD hot path.  One lane per tetrahedron for the
// element work, deterministic gathers over a vertex -> (tet, slot) incidence
// list instead of atomics, dense blocks of the two-level partitioned inverse
// for the global solve, and block partial sums reduced in a fixed order by
// the next kernel (so every result is bitwise reproducible).
//
// Vector layout: SoA over the library vertex order, x | y | z, stride nv.
// Per-tet arrays: SoA, stride ne.  Contributions: [slot*3 + axis][tet].
#include "kernels.h"

#include "device_math.h"

namespace pdhot {

// ---------------------------------------------------------------- helpers
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// block-wide sum of NV values per thread; result valid in thread 0
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* lds /* >= 4*NV */) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
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

// The done flag read once per block (thread 0) and broadcast, so every wave of
// a block takes the same early exit even while another block sets the flag.
__device__ __forceinline__ bool block_done(const int* done) {
  __shared__ int flag;
  if (threadIdx.x == 0) flag = done ? __hip_atomic_load(done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0;
  __syncthreads();
  const bool r = flag != 0;
  __syncthreads();
  return r;
}

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

// G_e^T P scaled by w into the 12 contribution slots of tet t:
// vertex a (1..3) receives w P r_a (r_a = row a-1 of D_m^{-1}), vertex 0 minus their sum.
__device__ __forceinline__ void store_contrib(const ElemArgs& E, double* __restrict__ contrib, int t, double w,
                                              const double P[9]) {
  double Bm[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) Bm[i] = E.Bm[i * E.ne + t];
  double c0[3] = {0, 0, 0};
#pragma unroll
  for (int a = 1; a < 4; ++a) {
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      const double v = w * (P[3 * ax] * Bm[3 * (a - 1)] + P[3 * ax + 1] * Bm[3 * (a - 1) + 1] +
                            P[3 * ax + 2] * Bm[3 * (a - 1) + 2]);
      contrib[(a * 3 + ax) * E.ne + t] = v;
      c0[ax] -= v;
    }
  }
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) contrib[ax * E.ne + t] = c0[ax];
}

__device__ __forceinline__ void gather3(const int* __restrict__ inc_ptr, const int* __restrict__ inc_idx,
                                        const double* __restrict__ contrib, int ne, int i, double out[3]) {
  double s0 = 0, s1 = 0, s2 = 0;
  for (int k = inc_ptr[i]; k < inc_ptr[i + 1]; ++k) {
    const int ts = inc_idx[k];
    const int t = ts >> 2, slot = ts & 3;
    s0 += contrib[(slot * 3 + 0) * ne + t];
    s1 += contrib[(slot * 3 + 1) * ne + t];
    s2 += contrib[(slot * 3 + 2) * ne + t];
  }
  out[0] = s0;
  out[1] = s1;
  out[2] = s2;
}

// ---------------------------------------------------------------- local step
// p*_e = U diag(s*) V^T of F_e = G_e q (Sec. 4.1 Eq. nh_prox) and the
// contribution w_e V_e G_e^T p*_e of Eq. A_basic.
__global__ void __launch_bounds__(kBlock) k_local(ElemArgs E, const double* __restrict__ q, int nv,
                                                  double* __restrict__ contrib, const int* __restrict__ done,
                                                  int* __restrict__ newton_max) {
  if (done && *done) return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  int its = 0;
  if (t < E.ne) {
    double F[9], U[9], V[9], sF[3], ss[3];
    int vi[4];
    load_F(E, q, nv, t, F, vi);
    svd3(F, U, sF, V);
    its = prox_stretch(sF, E.mu_bar, E.lam_bar, E.k_bar, ss);
    double P[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j)
        P[3 * i + j] = U[3 * i] * ss[0] * V[3 * j] + U[3 * i + 1] * ss[1] * V[3 * j + 1] + U[3 * i + 2] * ss[2] * V[3 * j + 2];
    store_contrib(E, contrib, t, E.wV[t], P);
  }
  if (newton_max) {
    int m = its;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = max(m, __shfl_xor(m, off, 64));
    if ((threadIdx.x & 63) == 0 && m > 0) atomicMax(newton_max, m);
  }
}

// G_e^T (w G_e x): contributions of the symmetric element operator w V G^T G
// (used for B_beta q_t in the prologue and for B_beta mu in the gradient).
__global__ void __launch_bounds__(kBlock) k_elem_GtG(ElemArgs E, const double* __restrict__ x, int nv,
                                                     const double* __restrict__ w, double* __restrict__ contrib) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= E.ne) return;
  double F[9];
  int vi[4];
  load_F(E, x, nv, t, F, vi);
  store_contrib(E, contrib, t, w[t], F);
}

// ---------------------------------------------------------------- step prologue
// q~ = q_t + h v_t + h^2 (M^{-1} f_ext + g)   (Eq. freefall)
// c  = M/h^2 q~ + (alpha/h) M q_t + (1/h) B_beta q_t - A~_{fp} q_p
// (damping terms of the right-hand side derived from Eq. dynamics).
__global__ void __launch_bounds__(kBlock) k_prologue(VertArgs Vx, const double* __restrict__ q_t_user,
                                                     const double* __restrict__ v_t_user,
                                                     const double* __restrict__ f_user,
                                                     const double* __restrict__ q0_user,
                                                     const double* __restrict__ contrib, StepState St) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Vx.nv) return;
  const int nv = Vx.nv;
  const int o = Vx.v_orig[i];
  if (i >= Vx.nf) {  // pinned: held at rest
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double r = Vx.rest[a * nv + i];
      St.qt[a * nv + i] = r;
      St.qtil[a * nv + i] = r;
      St.q_cur[a * nv + i] = r;
      St.q_prev[a * nv + i] = r;
      St.vt[a * nv + i] = 0.0;
    }
    return;
  }
  double bq[3];
  gather3(Vx.inc_ptr, Vx.inc_idx, contrib, Vx.ne, i, bq);
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
    const double q0 = q0_user ? q0_user[3 * o + a] : qt;
    St.q_cur[a * nv + i] = q0;
    St.q_prev[a * nv + i] = q0;
  }
}

// ---------------------------------------------------------------- gather + E b
// Per subdomain block: b = c + gathered contributions for its vertices, the
// dual-gate partial norms, and t_s = E_s b_s for the interface rows it
// couples to.  Extra blocks gather the interface vertices.
template <int MODE>
__global__ void __launch_bounds__(kBlock) k_gather_E(VertArgs Vx, SolveArgs Sv, StepState St, const double* __restrict__ rhs_in,
                                                     double* __restrict__ rhs_out, int k) {
  extern __shared__ double lds[];
  if (block_done(St.done)) return;
  const int nv = Vx.nv;
  const int blk = blockIdx.x;
  int i0, i1, s = -1;
  if (blk < Sv.nsub) {
    s = blk;
    i0 = Sv.sub_begin[s];
    i1 = Sv.sub_begin[s + 1];
  } else {
    i0 = Sv.nB + (blk - Sv.nsub) * kBlock;
    i1 = min(i0 + kBlock, Vx.nf);
  }
  double part[4] = {0, 0, 0, 0};
  double* bl = lds;  // n_s x 3
  for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    double bn[3];
    if (MODE == kModeFwd) {
      gather3(Vx.inc_ptr, Vx.inc_idx, St.contrib, Vx.ne, i, bn);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        bn[a] += St.c[a * nv + i];
        const double bo = St.b_cur[a * nv + i];
        const double qc = St.q_cur[a * nv + i], qp = St.q_prev[a * nv + i];
        St.b_prev[a * nv + i] = bo;
        St.b_cur[a * nv + i] = bn[a];
        part[0] += (qc - qp) * (qc - qp);
        part[1] += qp * qp;
        part[2] += (bn[a] - bo) * (bn[a] - bo);
        part[3] += bo * bo;
      }
    } else if (MODE == kModeDebugGather) {
      gather3(Vx.inc_ptr, Vx.inc_idx, St.contrib, Vx.ne, i, bn);
#pragma unroll
      for (int a = 0; a < 3; ++a) rhs_out[a * nv + i] = bn[a];
    } else {  // plain right-hand side given
#pragma unroll
      for (int a = 0; a < 3; ++a) bn[a] = rhs_in[a * nv + i];
    }
    if (s >= 0)
#pragma unroll
      for (int a = 0; a < 3; ++a) bl[3 * (i - i0) + a] = bn[a];
  }
  if (MODE == kModeFwd) {
    block_sum<4>(part, lds + 3 * Vx.max_sub);
    if (threadIdx.x == 0)
#pragma unroll
      for (int j = 0; j < 4; ++j) St.gate_part[4 * blk + j] = part[j];
  }
  if (MODE == kModeDebugGather) return;
  if (s < 0) return;
  __syncthreads();
  const int ns = i1 - i0;
  const int nI = Sv.ir_off[s + 1] - Sv.ir_off[s];
  const double* __restrict__ Et = Sv.Et + Sv.et_off[s];
  for (int p = threadIdx.x; p < nI; p += blockDim.x) {
    double t0 = 0, t1 = 0, t2 = 0;
    for (int v = 0; v < ns; ++v) {
      const double e = Et[(long long)v * nI + p];
      t0 += e * bl[3 * v];
      t1 += e * bl[3 * v + 1];
      t2 += e * bl[3 * v + 2];
    }
    const int slot = Sv.slot_of[Sv.ir_off[s] + p];
    Sv.t_slots[3 * slot] = t0;
    Sv.t_slots[3 * slot + 1] = t1;
    Sv.t_slots[3 * slot + 2] = t2;
  }
}

// ---------------------------------------------------------------- top solve
// Forward mode first reduces the dual-gate partials (Eq. convergence_dual):
// the gate holds for k >= 2, and k == kmax - 1 ends the step unconverged.
// Then x_T = Z (b_T - sum_s t_s) over the interface rows of this block.
template <int MODE>
__global__ void __launch_bounds__(kBlock) k_top(VertArgs Vx, SolveArgs Sv, StepState St, const double* __restrict__ rhs,
                                                double* __restrict__ out, int k) {
  extern __shared__ double lds[];
  if (block_done(St.done)) return;
  const int nv = Vx.nv;
  if (MODE == kModeFwd && k >= 1) {
    double g[4] = {0, 0, 0, 0};
    // every block reduces the same partials in the same order
    for (int b = threadIdx.x; b < St.n_gate_blocks; b += blockDim.x)
#pragma unroll
      for (int j = 0; j < 4; ++j) g[j] += St.gate_part[4 * b + j];
    block_sum<4>(g, lds);
    __shared__ int stop;
    if (threadIdx.x == 0) {
      const double dq = sqrt(g[0]), nq = sqrt(g[1]), db = sqrt(g[2]), nb = sqrt(g[3]);
      const bool pass = dq <= St.eps_rel * nq + St.eps_abs && db <= St.eps_rel * nb + St.eps_abs;
      const bool conv = (k >= 2) && pass;
      const bool cap = (k >= St.kmax - 1);
      stop = conv || cap;
      if (stop && blockIdx.x == 0) {
        St.ctl[kCtlDone] = 1;
        St.ctl[kCtlIters] = k;
        St.ctl[kCtlStatus] = conv ? 0 : 1;
        St.dstat[0] = dq; St.dstat[1] = nq; St.dstat[2] = db; St.dstat[3] = nb;
      }
    }
    __syncthreads();
    if (stop) return;
  }
  const int nT = Sv.nT, nB = Sv.nB;
  const double* __restrict__ bsrc = (MODE == kModeFwd) ? St.b_cur : rhs;
  double* rT = lds;  // nT x 3
  for (int i = threadIdx.x; i < nT; i += blockDim.x) {
    double r0 = bsrc[nB + i], r1 = bsrc[nv + nB + i], r2 = bsrc[2 * nv + nB + i];
    for (int q = Sv.row_slot_ptr[i]; q < Sv.row_slot_ptr[i + 1]; ++q) {
      r0 -= Sv.t_slots[3 * q];
      r1 -= Sv.t_slots[3 * q + 1];
      r2 -= Sv.t_slots[3 * q + 2];
    }
    rT[3 * i] = r0;
    rT[3 * i + 1] = r1;
    rT[3 * i + 2] = r2;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int row0 = blockIdx.x * Sv.top_rows;
  const int row1 = min(row0 + Sv.top_rows, nT);
  double* dst = (MODE == kModeFwd) ? St.qhat : out;
  for (int i = row0 + wid; i < row1; i += nw) {
    const double* __restrict__ Zi = Sv.Z + (long long)i * nT;
    double a0 = 0, a1 = 0, a2 = 0;
    for (int j = lane; j < nT; j += 64) {
      const double z = Zi[j];
      a0 += z * rT[3 * j];
      a1 += z * rT[3 * j + 1];
      a2 += z * rT[3 * j + 2];
    }
    a0 = wave_sum(a0);
    a1 = wave_sum(a1);
    a2 = wave_sum(a2);
    if (lane == 0) {
      dst[nB + i] = a0;
      dst[nv + nB + i] = a1;
      dst[2 * nv + nB + i] = a2;
    }
  }
}

// ---------------------------------------------------------------- Anderson state
__device__ __forceinline__ void aa_layout(const int* ctl, int k, int m, int& nonempty, int& nc_after, int& head_after,
                                          int& slot_new) {
  const int* st = ctl + kCtlAA + 4 * (k & 1);
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

// ---------------------------------------------------------------- bottom solve
// x_s = Zs b_s - E_s^T x_T on subdomain rows (one wave per row); forward mode
// then forms g = q^ - q^k, appends the Anderson difference columns
// (Eqs. aa_dG, aa_dQ) and writes the Gram partial sums of this block.
template <int MODE>
__global__ void __launch_bounds__(kBlock) k_bottom(VertArgs Vx, SolveArgs Sv, StepState St, const double* __restrict__ rhs,
                                                   double* __restrict__ out, int k) {
  extern __shared__ double lds[];
  if (block_done(St.done)) return;
  const int nv = Vx.nv, nf = Vx.nf, nB = Sv.nB;
  const int blk = blockIdx.x;
  const double* __restrict__ bsrc = (MODE == kModeFwd) ? St.b_cur : rhs;
  double* dst = (MODE == kModeFwd) ? St.qhat : out;
  int r0, r1;  // library rows handled here
  if (blk < Sv.n_bottom_items) {
    const int s = Sv.bottom_items[3 * blk], lr0 = Sv.bottom_items[3 * blk + 1], lr1 = Sv.bottom_items[3 * blk + 2];
    const int i0 = Sv.sub_begin[s], ns = Sv.sub_begin[s + 1] - i0;
    const int nI = Sv.ir_off[s + 1] - Sv.ir_off[s];
    double* bl = lds;            // ns x 3
    double* xl = lds + 3 * ns;   // nI x 3
    for (int v = threadIdx.x; v < ns; v += blockDim.x)
#pragma unroll
      for (int a = 0; a < 3; ++a) bl[3 * v + a] = bsrc[a * nv + i0 + v];
    for (int p = threadIdx.x; p < nI; p += blockDim.x) {
      const int ri = nB + Sv.irows[Sv.ir_off[s] + p];
#pragma unroll
      for (int a = 0; a < 3; ++a) xl[3 * p + a] = dst[a * nv + ri];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const double* __restrict__ Zs = Sv.Zs + Sv.zs_off[s];
    const double* __restrict__ Et = Sv.Et + Sv.et_off[s];
    for (int v = lr0 + wid; v < lr1; v += nw) {
      double a0 = 0, a1 = 0, a2 = 0;
      const double* __restrict__ Zr = Zs + (long long)v * ns;
      for (int u = lane; u < ns; u += 64) {
        const double z = Zr[u];
        a0 += z * bl[3 * u];
        a1 += z * bl[3 * u + 1];
        a2 += z * bl[3 * u + 2];
      }
      const double* __restrict__ Er = Et + (long long)v * nI;
      for (int p = lane; p < nI; p += 64) {
        const double e = Er[p];
        a0 -= e * xl[3 * p];
        a1 -= e * xl[3 * p + 1];
        a2 -= e * xl[3 * p + 2];
      }
      a0 = wave_sum(a0);
      a1 = wave_sum(a1);
      a2 = wave_sum(a2);
      if (lane == 0) {
        dst[i0 + v] = a0;
        dst[nv + i0 + v] = a1;
        dst[2 * nv + i0 + v] = a2;
      }
    }
    r0 = i0 + lr0;
    r1 = i0 + lr1;
  } else {
    r0 = nB + (blk - Sv.n_bottom_items) * kBlock;
    r1 = min(r0 + kBlock, nf);
  }
  if (MODE != kModeFwd) return;
  __syncthreads();
  // Anderson acceleration: append and Gram partials
  const int m = St.m;
  int nonempty, nc, head, slot_new;
  aa_layout(St.ctl, k, m, nonempty, nc, head, slot_new);
  double part[kAAPart];
#pragma unroll
  for (int j = 0; j < kAAPart; ++j) part[j] = 0.0;
  if (m > 0) {
    for (int i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const int ix = a * nv + i;
        const double qc = St.q_cur[ix];
        const double g = St.qhat[ix] - qc;
        if (slot_new >= 0) {
          const long long cix = ((long long)slot_new * 3 + a) * nv + i;
          St.dG[cix] = g - St.g_last[ix];
          St.dQ[cix] = qc - St.q_last[ix];
        }
        St.g_last[ix] = g;
        St.q_last[ix] = qc;
        double col[kMaxWindow];
#pragma unroll
        for (int j = 0; j < kMaxWindow; ++j)
          col[j] = (j < nc) ? St.dG[((long long)((head + j) % m) * 3 + a) * nv + i] : 0.0;
#pragma unroll
        for (int j = 0; j < kMaxWindow; ++j) {
#pragma unroll
          for (int l = j; l < kMaxWindow; ++l) part[j * kMaxWindow + l] += col[j] * col[l];
          part[kMaxWindow * kMaxWindow + j] += col[j] * g;
        }
      }
    }
  }
  block_sum<kAAPart>(part, lds + 0);
  if (threadIdx.x == 0)
#pragma unroll
    for (int j = 0; j < kAAPart; ++j) St.aa_part[(long long)blk * kAAPart + j] = part[j];
}

// ---------------------------------------------------------------- Anderson update
// gamma = (dG^T dG + rho I)^{-1} dG^T g, rho = max(1e-6 |dG|_F^2 / m, 1e-12)
// (Eq. aa_gamma); q^{k+1} = q^ - (dQ + dG) gamma (Eq. aa_update), or q^ with
// the history dropped when |gamma|_2 > 10 (reliability guard).
__global__ void __launch_bounds__(kBlock) k_aa_update(VertArgs Vx, StepState St, int k) {
  if (block_done(St.done)) return;
  __shared__ double gam[kMaxWindow];
  __shared__ int use_aa;
  __shared__ double red[4 * kAAPart];
  const int nv = Vx.nv, m = St.m;
  int nonempty, nc, head, slot_new;
  aa_layout(St.ctl, k, m, nonempty, nc, head, slot_new);
  if (m > 0 && nc >= 1) {
    double part[kAAPart];
#pragma unroll
    for (int j = 0; j < kAAPart; ++j) part[j] = 0.0;
    for (int b = threadIdx.x; b < St.n_aa_blocks; b += blockDim.x)
#pragma unroll
      for (int j = 0; j < kAAPart; ++j) part[j] += St.aa_part[(long long)b * kAAPart + j];
    block_sum<kAAPart>(part, red);
    if (threadIdx.x == 0) {
      double G[kMaxWindow * kMaxWindow], rhs[kMaxWindow];
      double fro = 0.0;
      for (int j = 0; j < nc; ++j) {
        for (int l = 0; l < nc; ++l) G[j * nc + l] = (j <= l) ? part[j * kMaxWindow + l] : part[l * kMaxWindow + j];
        rhs[j] = part[kMaxWindow * kMaxWindow + j];
        fro += G[j * nc + j];
      }
      const double rho = fmax(1e-6 * fro / nc, 1e-12);
      for (int j = 0; j < nc; ++j) G[j * nc + j] += rho;
      // Cholesky solve
      bool ok = true;
      for (int j = 0; j < nc && ok; ++j) {
        double d = G[j * nc + j];
        for (int l = 0; l < j; ++l) d -= G[j * nc + l] * G[j * nc + l];
        if (!(d > 0.0)) { ok = false; break; }
        d = sqrt(d);
        G[j * nc + j] = d;
        for (int i = j + 1; i < nc; ++i) {
          double s = G[i * nc + j];
          for (int l = 0; l < j; ++l) s -= G[i * nc + l] * G[j * nc + l];
          G[i * nc + j] = s / d;
        }
      }
      double nrm = INFINITY;
      if (ok) {
        double y[kMaxWindow];
        for (int i = 0; i < nc; ++i) {
          double s = rhs[i];
          for (int l = 0; l < i; ++l) s -= G[i * nc + l] * y[l];
          y[i] = s / G[i * nc + i];
        }
        for (int i = nc - 1; i >= 0; --i) {
          double s = y[i];
          for (int l = i + 1; l < nc; ++l) s -= G[l * nc + i] * gam[l];
          gam[i] = s / G[i * nc + i];
        }
        nrm = 0.0;
        for (int i = 0; i < nc; ++i) nrm += gam[i] * gam[i];
        nrm = sqrt(nrm);
      }
      use_aa = (nrm <= 10.0);
    }
  } else if (threadIdx.x == 0) {
    use_aa = 0;
  }
  __syncthreads();
  const bool reset = (m > 0 && nc >= 1 && !use_aa);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    int* nxt = St.ctl + kCtlAA + 4 * ((k + 1) & 1);
    if (m <= 0) {
      nxt[0] = 0; nxt[1] = 0; nxt[2] = 0;
    } else if (reset) {
      nxt[0] = 0; nxt[1] = 0; nxt[2] = 0;
      St.ctl[kCtlResets] += 1;
    } else {
      nxt[0] = 1; nxt[1] = nc; nxt[2] = head;
    }
  }
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Vx.nf) return;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int ix = a * nv + i;
    double qn = St.qhat[ix];
    if (use_aa)
      for (int j = 0; j < nc; ++j) {
        const long long cix = ((long long)((head + j) % m) * 3 + a) * nv + i;
        qn -= (St.dQ[cix] + St.dG[cix]) * gam[j];
      }
    St.q_prev[ix] = St.q_cur[ix];
    St.q_cur[ix] = qn;
  }
}

// ---------------------------------------------------------------- step epilogue
// q_{t+h} = q*, v_{t+h} = (q* - q_t) / h in the caller's order; checkpoint
// record {q_t, q~, q*, q*-1} in library order.
__global__ void __launch_bounds__(kBlock) k_epilogue(VertArgs Vx, StepState St, double* __restrict__ q_next,
                                                     double* __restrict__ v_next, double* __restrict__ ckpt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
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

// ---------------------------------------------------------------- layout conversion
__global__ void __launch_bounds__(kBlock) k_to_lib(VertArgs Vx, const double* __restrict__ user, double* __restrict__ lib,
                                                   int free_only) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Vx.nv) return;
  const int o = Vx.v_orig[i];
  const bool zero = free_only && i >= Vx.nf;
#pragma unroll
  for (int a = 0; a < 3; ++a) lib[a * Vx.nv + i] = zero ? 0.0 : user[3 * o + a];
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
// Trust-region ratio partials (Eqs. tr_step, tr_decreases): per tet
// V_e (psi_e(F(q*-1)) - psi_e(F(q*))) and (w_e + beta_e/h) V_e |G_e dq|^2;
// per free vertex m/(2h^2) (a - b).(a + b - 2 q~) and (1 + alpha h) m/h^2 |dq|^2.
__global__ void __launch_bounds__(kBlock) k_tr_partials(ElemArgs E, VertArgs Vx, const double* __restrict__ ck,
                                                        double* __restrict__ part, int n_tet_blocks) {
  __shared__ double red[8];
  const int nv = Vx.nv;
  const double* qt = ck;
  const double* qtil = ck + 3 * nv;
  const double* qs = ck + 6 * nv;
  const double* qm = ck + 9 * nv;
  double v[2] = {0.0, 0.0};
  if ((int)blockIdx.x < n_tet_blocks) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
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
      if (Ja > 0.0 && Jb > 0.0) {
        double Ia = 0.0, Ib = 0.0;
#pragma unroll
        for (int j = 0; j < 9; ++j) {
          Ia += Fa[j] * Fa[j];
          Ib += Fb[j] * Fb[j];
          gg += (Fb[j] - Fa[j]) * (Fb[j] - Fa[j]);
        }
        const double la = log(Ja), lb = log(Jb);
        d = 0.5 * E.muV[t] * (Ia - Ib) - E.muV[t] * (la - lb) + 0.5 * E.lamV[t] * (la * la - lb * lb);
      } else {
        d = (Ja > 0.0) ? -INFINITY : INFINITY;
#pragma unroll
        for (int j = 0; j < 9; ++j) gg += (Fb[j] - Fa[j]) * (Fb[j] - Fa[j]);
      }
      v[0] = d;
      v[1] = (E.wV[t] + E.bV[t]) * gg;
    }
  } else {
    const int i = (blockIdx.x - n_tet_blocks) * blockDim.x + threadIdx.x;
    if (i < Vx.nf) {
      const double m = Vx.mass[i], h = Vx.h;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const int ix = a * nv + i;
        const double A = qm[ix], B = qs[ix];
        v[0] += 0.5 / (h * h) * m * (A - B) * (A + B - 2.0 * qtil[ix]);
        v[1] += (1.0 + Vx.alpha * h) * m / (h * h) * (B - A) * (B - A);
      }
    }
  }
  (void)qt;
  block_sum<2>(v, red);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = v[0];
    part[2 * blockIdx.x + 1] = v[1];
  }
}

// rho = dPhi_act / dPhi_mod (rho = 1 when dPhi_mod < 1e-12), tau* = 1/2 when
// |rho - 1| <= eps_TR else 1 (Eqs. tr_ratio, tr_rule); then per tet the
// recomputed SVD and prox stretches at q*, and the compact filtered prox
// differential {U, V, D, c1, c2, s*} (Alg. 2 element loop).
__global__ void __launch_bounds__(kBlock) k_bwd_elem(ElemArgs E, VertArgs Vx, const double* __restrict__ ck,
                                                     const double* __restrict__ part, int n_part, double eps_tr,
                                                     double tau_force, double* __restrict__ jac,
                                                     double* __restrict__ bstat) {
  __shared__ double red[8];
  __shared__ double tau_s;
  double v[2] = {0.0, 0.0};
  for (int b = threadIdx.x; b < n_part; b += blockDim.x) {
    v[0] += part[2 * b];
    v[1] += part[2 * b + 1];
  }
  block_sum<2>(v, red);
  if (threadIdx.x == 0) {
    const double act = v[0], mod = 0.5 * fabs(v[1]);
    const double rho = (mod < 1e-12) ? 1.0 : act / mod;
    double tau = (fabs(rho - 1.0) <= eps_tr) ? 0.5 : 1.0;
    if (tau_force >= 0.0) tau = tau_force;
    tau_s = tau;
    if (blockIdx.x == 0) {
      bstat[0] = rho;
      bstat[1] = tau;
      bstat[2] = act;
      bstat[3] = mod;
    }
  }
  __syncthreads();
  const double tau = tau_s;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= E.ne) return;
  const int nv = Vx.nv;
  const double* qs = ck + 6 * nv;
  double F[9], U[9], V[9], sF[3], ss[3];
  int vi[4];
  load_F(E, qs, nv, t, F, vi);
  svd3(F, U, sF, V);
  prox_stretch(sF, E.mu_bar, E.lam_bar, E.k_bar, ss);
  double D[6], c1[3], c2[3];
  prox_diff(sF, ss, E.mu_bar, E.lam_bar, E.k_bar, tau, D, c1, c2);
  const long long ne = E.ne;
#pragma unroll
  for (int j = 0; j < 9; ++j) {
    jac[j * ne + t] = U[j];
    jac[(9 + j) * ne + t] = V[j];
  }
#pragma unroll
  for (int j = 0; j < 6; ++j) jac[(18 + j) * ne + t] = D[j];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    jac[(24 + j) * ne + t] = c1[j];
    jac[(27 + j) * ne + t] = c2[j];
    jac[(30 + j) * ne + t] = ss[j];
  }
}

__device__ __forceinline__ void load_jac(const double* __restrict__ jac, int ne, int t, double U[9], double V[9],
                                         double D[6], double c1[3], double c2[3]) {
#pragma unroll
  for (int j = 0; j < 9; ++j) {
    U[j] = jac[(long long)j * ne + t];
    V[j] = jac[(long long)(9 + j) * ne + t];
  }
#pragma unroll
  for (int j = 0; j < 6; ++j) D[j] = jac[(long long)(18 + j) * ne + t];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    c1[j] = jac[(long long)(24 + j) * ne + t];
    c2[j] = jac[(long long)(27 + j) * ne + t];
  }
}

// K x element contributions: w_e V_e G_e^T (dp*/dF) G_e x (Eq. db_dq).
// x is read on free vertices only (pinned entries are treated as zero).
__global__ void __launch_bounds__(kBlock) k_apply_K(ElemArgs E, VertArgs Vx, const double* __restrict__ jac,
                                                    const double* __restrict__ x, double* __restrict__ contrib,
                                                    const int* __restrict__ done) {
  if (done && *done) return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= E.ne) return;
  const int nv = Vx.nv, nf = Vx.nf;
  int vi[4];
  vi[0] = E.tv[t];
  vi[1] = E.tv[E.ne + t];
  vi[2] = E.tv[2 * E.ne + t];
  vi[3] = E.tv[3 * E.ne + t];
  double xv[4][3];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) xv[a][ax] = vi[a] < nf ? x[ax * nv + vi[a]] : 0.0;
  double Bm[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) Bm[i] = E.Bm[i * E.ne + t];
  double dF[9];
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    const double d1 = xv[1][ax] - xv[0][ax], d2 = xv[2][ax] - xv[0][ax], d3 = xv[3][ax] - xv[0][ax];
#pragma unroll
    for (int j = 0; j < 3; ++j) dF[3 * ax + j] = d1 * Bm[j] + d2 * Bm[3 + j] + d3 * Bm[6 + j];
  }
  double U[9], V[9], D[6], c1[3], c2[3], dP[9];
  load_jac(jac, E.ne, t, U, V, D, c1, c2);
  prox_diff_apply(U, V, D, c1, c2, dF, dP);
  store_contrib(E, contrib, t, E.wV[t], dP);
}

// Gathered K x on free vertices; PCG: w = A p - K p and the partial p.w;
// fixed point: rhs = qbar + K mu.
template <int MODE>
__global__ void __launch_bounds__(kBlock) k_adj_gather(VertArgs Vx, AdjState Ad, int it) {
  __shared__ double red[8];
  if (block_done(Ad.done)) return;
  const int nv = Vx.nv;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double v[1] = {0.0};
  if (i < Vx.nf) {
    double kx[3];
    gather3(Vx.inc_ptr, Vx.inc_idx, Ad.contrib, Vx.ne, i, kx);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int ix = a * nv + i;
      if (MODE == kModePCG) {
        const double w = Ad.Ap[ix] - kx[a];
        Ad.w[ix] = w;
        v[0] += Ad.p[ix] * w;
      } else if (MODE == kModeFixed) {
        Ad.r[ix] = Ad.qbar[ix] + kx[a];
      } else {  // debug: K x
        Ad.w[ix] = kx[a];
      }
    }
  }
  if (MODE != kModePCG) return;
  block_sum<1>(v, red);
  if (threadIdx.x == 0) Ad.part[8 * blockIdx.x] = v[0];
}

// PCG: alpha = (r.z)/(p.w); mu += alpha p; r -= alpha w (done by every
// vertex block after an identical reduction of the p.w partials).
__global__ void __launch_bounds__(kBlock) k_pcg_alpha(VertArgs Vx, AdjState Ad, int it) {
  __shared__ double red[8];
  __shared__ double alpha_s;
  if (block_done(Ad.done)) return;
  double v[1] = {0.0};
  for (int b = threadIdx.x; b < Ad.n_vert_blocks; b += blockDim.x) v[0] += Ad.part[8 * b];
  block_sum<1>(v, red);
  if (threadIdx.x == 0) alpha_s = Ad.scal[(it & 1) * 4 + 0] / v[0];
  __syncthreads();
  const double alpha = alpha_s;
  const int nv = Vx.nv;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Vx.nf) return;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int ix = a * nv + i;
    Ad.mu[ix] += alpha * Ad.p[ix];
    Ad.r[ix] -= alpha * Ad.w[ix];
  }
}

// After z = A^{-1} r: partial sums of r.z, |z|^2, |mu|^2 (PCG) or of
// |mu_new - mu|^2, |mu_new|^2 (fixed point, which also moves mu_new into mu).
template <int MODE>
__global__ void __launch_bounds__(kBlock) k_adj_dots(VertArgs Vx, AdjState Ad, int it) {
  __shared__ double red[16];
  if (block_done(Ad.done)) return;
  const int nv = Vx.nv;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double v[3] = {0.0, 0.0, 0.0};
  if (i < Vx.nf) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int ix = a * nv + i;
      if (MODE == kModePCG) {
        const double z = Ad.z[ix];
        v[0] += Ad.r[ix] * z;
        v[1] += z * z;
        v[2] += Ad.mu[ix] * Ad.mu[ix];
      } else {
        const double mn = Ad.z[ix], mo = Ad.mu[ix];
        v[0] += (mn - mo) * (mn - mo);
        v[1] += mn * mn;
        Ad.mu[ix] = mn;
      }
    }
  }
  block_sum<3>(v, red);
  if (threadIdx.x == 0)
#pragma unroll
    for (int j = 0; j < 3; ++j) Ad.part[8 * blockIdx.x + 1 + j] = v[j];
}

// Convergence test and the next PCG direction: beta = (r.z)_new/(r.z)_old,
// p = z + beta p, A p = r + beta A p (A z = r, so no product with A is needed).
template <int MODE>
__global__ void __launch_bounds__(kBlock) k_adj_next(VertArgs Vx, AdjState Ad, int it) {
  __shared__ double red[16];
  __shared__ int stop;
  __shared__ double beta_s;
  if (block_done(Ad.done)) return;
  double v[3] = {0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < Ad.n_vert_blocks; b += blockDim.x)
#pragma unroll
    for (int j = 0; j < 3; ++j) v[j] += Ad.part[8 * b + 1 + j];
  block_sum<3>(v, red);
  if (threadIdx.x == 0) {
    double res;
    if (MODE == kModePCG) {
      res = sqrt(v[1]) / fmax(sqrt(v[2]), 1e-300);
      const double rz_old = Ad.scal[(it & 1) * 4 + 0];
      beta_s = v[0] / rz_old;
      if (blockIdx.x == 0) Ad.scal[((it + 1) & 1) * 4 + 0] = v[0];
    } else {
      res = sqrt(v[0]) / fmax(sqrt(v[1]), 1e-300);
      beta_s = 0.0;
    }
    const bool conv = res <= Ad.eps;
    const bool cap = it + 1 >= Ad.kmax;
    stop = conv || cap;
    if (blockIdx.x == 0) {
      Ad.dstat[0] = res;
      if (stop) {
        *Ad.done = 1;
        Ad.ctl[0] = it + 1;
        Ad.ctl[1] = conv ? 0 : 1;
      }
    }
  }
  __syncthreads();
  if (stop || MODE != kModePCG) return;
  const double beta = beta_s;
  const int nv = Vx.nv;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Vx.nf) return;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int ix = a * nv + i;
    Ad.p[ix] = Ad.z[ix] + beta * Ad.p[ix];
    Ad.Ap[ix] = Ad.r[ix] + beta * Ad.Ap[ix];
  }
}

// q bar = gq_next + gv_next / h on free vertices (Alg. 2 first line), in
// library order; PCG start: mu = 0, r = q bar.
__global__ void __launch_bounds__(kBlock) k_bwd_prologue(VertArgs Vx, AdjState Ad, const double* __restrict__ gq,
                                                         const double* __restrict__ gv) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Vx.nv) return;
  const int nv = Vx.nv, o = Vx.v_orig[i];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int ix = a * nv + i;
    const double qb = (i < Vx.nf) ? ((gq ? gq[3 * o + a] : 0.0) + (gv ? gv[3 * o + a] : 0.0) / Vx.h) : 0.0;
    Ad.qbar[ix] = qb;
    Ad.r[ix] = qb;
    Ad.mu[ix] = 0.0;
  }
}

// PCG after the first solve z0 = A^{-1} r0: p = z0, A p = r0, (r.z)_0.
__global__ void __launch_bounds__(kBlock) k_pcg_start(VertArgs Vx, AdjState Ad) {
  __shared__ double red[8];
  const int nv = Vx.nv;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double v[1] = {0.0};
  if (i < Vx.nf) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int ix = a * nv + i;
      const double z = Ad.z[ix];
      Ad.p[ix] = z;
      Ad.Ap[ix] = Ad.r[ix];
      v[0] += Ad.r[ix] * z;
    }
  }
  block_sum<1>(v, red);
  if (threadIdx.x == 0) Ad.part[8 * blockIdx.x] = v[0];
}

__global__ void __launch_bounds__(kBlock) k_pcg_start_reduce(AdjState Ad) {
  __shared__ double red[8];
  double v[1] = {0.0};
  for (int b = threadIdx.x; b < Ad.n_vert_blocks; b += blockDim.x) v[0] += Ad.part[8 * b];
  block_sum<1>(v, red);
  if (threadIdx.x == 0) Ad.scal[0] = v[0];
}

// Gradient routing per tet (Eq. dl_dwe and its damping counterpart, chain
// rule through w_e and beta_e, both proportional to E_e):
// dL/dlogE_e += w_e V_e <G mu, p* - G q*> + (beta_e V_e / h) <G mu, G (q_t - q*)>,
// plus the contributions (beta_e V_e / h) G^T G mu for B_beta mu / h.
__global__ void __launch_bounds__(kBlock) k_grad_elem(ElemArgs E, VertArgs Vx, const double* __restrict__ ck,
                                                      const double* __restrict__ jac, const double* __restrict__ mu,
                                                      double* __restrict__ contrib, double* __restrict__ g_logE) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= E.ne) return;
  const int nv = Vx.nv;
  double Gm[9], Fs[9], Ft[9];
  int vi[4];
  load_F(E, mu, nv, t, Gm, vi);  // mu is zero on pinned vertices
  load_F(E, ck + 6 * nv, nv, t, Fs, vi);
  load_F(E, ck, nv, t, Ft, vi);
  double U[9], V[9], ss[3];
#pragma unroll
  for (int j = 0; j < 9; ++j) {
    U[j] = jac[(long long)j * E.ne + t];
    V[j] = jac[(long long)(9 + j) * E.ne + t];
  }
#pragma unroll
  for (int j = 0; j < 3; ++j) ss[j] = jac[(long long)(30 + j) * E.ne + t];
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
}

// dL/dq_t = (M/h^2 + alpha M/h) mu + B_beta mu / h - v bar / h,
// dL/dv_t = M mu / h, dL/df_ext = mu (caller's order; zero on pinned).
__global__ void __launch_bounds__(kBlock) k_grad_vert(VertArgs Vx, const double* __restrict__ mu,
                                                      const double* __restrict__ contrib,
                                                      const double* __restrict__ gv_next, double* __restrict__ gq_t,
                                                      double* __restrict__ gv_t, double* __restrict__ gf) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int nv = Vx.nv;
  if (i >= nv) return;
  const int o = Vx.v_orig[i];
  if (i >= Vx.nf) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (gq_t) gq_t[3 * o + a] = 0.0;
      if (gv_t) gv_t[3 * o + a] = 0.0;
      if (gf) gf[3 * o + a] = 0.0;
    }
    return;
  }
  double bm[3];
  gather3(Vx.inc_ptr, Vx.inc_idx, contrib, Vx.ne, i, bm);
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

// ================================================================= launchers
#define PD_GRID(n) dim3(((n) + kBlock - 1) / kBlock), dim3(kBlock)

void launch_local(const ElemArgs& E, const double* q, int nv, double* contrib, const int* done, int* newton_max,
                  hipStream_t s) {
  hipLaunchKernelGGL(k_local, PD_GRID(E.ne), 0, s, E, q, nv, contrib, done, newton_max);
}
void launch_elem_GtG(const ElemArgs& E, const double* x, int nv, const double* w, double* contrib, hipStream_t s) {
  hipLaunchKernelGGL(k_elem_GtG, PD_GRID(E.ne), 0, s, E, x, nv, w, contrib);
}
void launch_prologue(const VertArgs& V, const double* qt, const double* vt, const double* f, const double* q0,
                     const double* contrib, const StepState& St, hipStream_t s) {
  hipLaunchKernelGGL(k_prologue, PD_GRID(V.nv), 0, s, V, qt, vt, f, q0, contrib, St);
}
static size_t lds_gather(const VertArgs& V) { return sizeof(double) * (3 * V.max_sub + 4 * 4 + 8); }
static size_t lds_top(const SolveArgs& S) { return sizeof(double) * std::max(3 * S.nT, 4 * 4 + 8); }
static size_t lds_bottom(const SolveArgs& S) {
  return sizeof(double) * std::max(3 * (S.max_ns + S.max_nI), 4 * kAAPart + 8);
}
void launch_gather_E(int mode, const VertArgs& V, const SolveArgs& S, const StepState& St, const double* rhs_in,
                     double* rhs_out, int k, hipStream_t s) {
  const int nblk = S.nsub + (S.nT + kBlock - 1) / kBlock;
  if (nblk == 0) return;
  if (mode == kModeFwd)
    hipLaunchKernelGGL(k_gather_E<kModeFwd>, dim3(nblk), dim3(kBlock), lds_gather(V), s, V, S, St, rhs_in, rhs_out, k);
  else if (mode == kModeDebugGather)
    hipLaunchKernelGGL(k_gather_E<kModeDebugGather>, dim3(nblk), dim3(kBlock), lds_gather(V), s, V, S, St, rhs_in,
                       rhs_out, k);
  else
    hipLaunchKernelGGL(k_gather_E<kModePlain>, dim3(nblk), dim3(kBlock), lds_gather(V), s, V, S, St, rhs_in, rhs_out,
                       k);
}
void launch_top(int mode, const VertArgs& V, const SolveArgs& S, const StepState& St, const double* rhs, double* out,
                int k, hipStream_t s) {
  // forward mode always runs: the dual-gate decision lives in this kernel
  if (mode == kModeFwd)
    hipLaunchKernelGGL(k_top<kModeFwd>, dim3(std::max(1, S.n_top_blocks)), dim3(kBlock), lds_top(S), s, V, S, St, rhs,
                       out, k);
  else if (S.nT == 0)
    return;
  else
    hipLaunchKernelGGL(k_top<kModePlain>, dim3(S.n_top_blocks), dim3(kBlock), lds_top(S), s, V, S, St, rhs, out, k);
}
void launch_bottom(int mode, const VertArgs& V, const SolveArgs& S, const StepState& St, const double* rhs,
                   double* out, int k, hipStream_t s) {
  const int nblk = S.n_bottom_items + (S.nT + kBlock - 1) / kBlock;
  if (nblk == 0) return;
  if (mode == kModeFwd)
    hipLaunchKernelGGL(k_bottom<kModeFwd>, dim3(nblk), dim3(kBlock), lds_bottom(S), s, V, S, St, rhs, out, k);
  else
    hipLaunchKernelGGL(k_bottom<kModePlain>, dim3(nblk), dim3(kBlock), lds_bottom(S), s, V, S, St, rhs, out, k);
}
void launch_aa_update(const VertArgs& V, const StepState& St, int k, hipStream_t s) {
  hipLaunchKernelGGL(k_aa_update, PD_GRID(V.nf), 0, s, V, St, k);
}
void launch_epilogue(const VertArgs& V, const StepState& St, double* q_next, double* v_next, double* ckpt,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_epilogue, PD_GRID(V.nv), 0, s, V, St, q_next, v_next, ckpt);
}
void launch_to_lib(const VertArgs& V, const double* user, double* lib, int free_only, hipStream_t s) {
  hipLaunchKernelGGL(k_to_lib, PD_GRID(V.nv), 0, s, V, user, lib, free_only);
}
void launch_from_lib(const VertArgs& V, const double* lib, double* user, int free_only, hipStream_t s) {
  hipLaunchKernelGGL(k_from_lib, PD_GRID(V.nv), 0, s, V, lib, user, free_only);
}
int tr_partial_blocks(const ElemArgs& E, const VertArgs& V) {
  return (E.ne + kBlock - 1) / kBlock + (V.nf + kBlock - 1) / kBlock;
}
void launch_tr_partials(const ElemArgs& E, const VertArgs& V, const double* ck, double* part, hipStream_t s) {
  const int ntb = (E.ne + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_tr_partials, dim3(tr_partial_blocks(E, V)), dim3(kBlock), 0, s, E, V, ck, part, ntb);
}
void launch_bwd_elem(const ElemArgs& E, const VertArgs& V, const double* ck, const double* part, int n_part,
                     double eps_tr, double tau_force, double* jac, double* bstat, hipStream_t s) {
  hipLaunchKernelGGL(k_bwd_elem, PD_GRID(E.ne), 0, s, E, V, ck, part, n_part, eps_tr, tau_force, jac, bstat);
}
void launch_apply_K(const ElemArgs& E, const VertArgs& V, const double* jac, const double* x, double* contrib,
                    const int* done, hipStream_t s) {
  hipLaunchKernelGGL(k_apply_K, PD_GRID(E.ne), 0, s, E, V, jac, x, contrib, done);
}
void launch_adj_gather(int mode, const VertArgs& V, const AdjState& A, int it, hipStream_t s) {
  if (mode == kModePCG) hipLaunchKernelGGL(k_adj_gather<kModePCG>, PD_GRID(V.nf), 0, s, V, A, it);
  else if (mode == kModeFixed) hipLaunchKernelGGL(k_adj_gather<kModeFixed>, PD_GRID(V.nf), 0, s, V, A, it);
  else hipLaunchKernelGGL(k_adj_gather<kModeDebugGather>, PD_GRID(V.nf), 0, s, V, A, it);
}
void launch_pcg_alpha(const VertArgs& V, const AdjState& A, int it, hipStream_t s) {
  hipLaunchKernelGGL(k_pcg_alpha, PD_GRID(V.nf), 0, s, V, A, it);
}
void launch_adj_dots(int mode, const VertArgs& V, const AdjState& A, int it, hipStream_t s) {
  if (mode == kModePCG) hipLaunchKernelGGL(k_adj_dots<kModePCG>, PD_GRID(V.nf), 0, s, V, A, it);
  else hipLaunchKernelGGL(k_adj_dots<kModeFixed>, PD_GRID(V.nf), 0, s, V, A, it);
}
void launch_adj_next(int mode, const VertArgs& V, const AdjState& A, int it, hipStream_t s) {
  if (mode == kModePCG) hipLaunchKernelGGL(k_adj_next<kModePCG>, PD_GRID(V.nf), 0, s, V, A, it);
  else hipLaunchKernelGGL(k_adj_next<kModeFixed>, PD_GRID(V.nf), 0, s, V, A, it);
}
void launch_bwd_prologue(const VertArgs& V, const AdjState& A, const double* gq, const double* gv, hipStream_t s) {
  hipLaunchKernelGGL(k_bwd_prologue, PD_GRID(V.nv), 0, s, V, A, gq, gv);
}
void launch_pcg_start(const VertArgs& V, const AdjState& A, hipStream_t s) {
  hipLaunchKernelGGL(k_pcg_start, PD_GRID(V.nf), 0, s, V, A);
  hipLaunchKernelGGL(k_pcg_start_reduce, dim3(1), dim3(kBlock), 0, s, A);
}
void launch_grad_elem(const ElemArgs& E, const VertArgs& V, const double* ck, const double* jac, const double* mu,
                      double* contrib, double* g_logE, hipStream_t s) {
  hipLaunchKernelGGL(k_grad_elem, PD_GRID(E.ne), 0, s, E, V, ck, jac, mu, contrib, g_logE);
}
void launch_grad_vert(const VertArgs& V, const double* mu, const double* contrib, const double* gv_next, double* gq_t,
                      double* gv_t, double* gf, hipStream_t s) {
  hipLaunchKernelGGL(k_grad_vert, PD_GRID(V.nv), 0, s, V, mu, contrib, gv_next, gq_t, gv_t, gf);
}

}  // namespace pdhot
