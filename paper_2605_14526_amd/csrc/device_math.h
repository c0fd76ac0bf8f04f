// Per-tetrahedron FP64 math for the local step and its differential:
// signed 3x3 SVD, the Neo-Hookean proximal stretches, the 3x3 symmetric
// eigendecomposition of the trust-region filter, and the filtered SVD
// differential.  All routines run in registers, one tet per lane.
#pragma once

#include <hip/hip_runtime.h>

namespace pdhot {

constexpr int kNewtonCap = 50;  // iteration cap of the prox Newton

// ---------------------------------------------------------------------------
// Symmetric 3x3 eigendecomposition by cyclic Jacobi rotations (the paper's
// closed-form Jacobi sweep of Sec. 4.4).  On entry a00..a22 hold the matrix;
// on exit the diagonal holds the eigenvalues and the columns of Q the
// eigenvectors (A = Q diag Q^T).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void jacobi_rotate(double& app, double& aqq, double& apq, double& apr, double& aqr,
                                              double* Q, int p, int q) {
  if (apq == 0.0) return;
  const double theta = (aqq - app) / (2.0 * apq);
  const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
  const double c = 1.0 / sqrt(t * t + 1.0);
  const double s = t * c;
  app -= t * apq;
  aqq += t * apq;
  apq = 0.0;
  const double r1 = apr, r2 = aqr;
  apr = c * r1 - s * r2;
  aqr = s * r1 + c * r2;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double qp = Q[3 * k + p], qq = Q[3 * k + q];
    Q[3 * k + p] = c * qp - s * qq;
    Q[3 * k + q] = s * qp + c * qq;
  }
}

// Jacobi sweeps that accumulate into the rotation Q given on entry.
__device__ __forceinline__ void jacobi_sweeps(double& a00, double& a11, double& a22, double& a01, double& a02,
                                              double& a12, double Q[9]) {
  for (int sweep = 0; sweep < 12; ++sweep) {
    const double off = a01 * a01 + a02 * a02 + a12 * a12;
    const double dia = a00 * a00 + a11 * a11 + a22 * a22;
    if (off <= 1e-32 * dia) break;
    jacobi_rotate(a00, a11, a01, a02, a12, Q, 0, 1);
    jacobi_rotate(a00, a22, a02, a01, a12, Q, 0, 2);
    jacobi_rotate(a11, a22, a12, a01, a02, Q, 1, 2);
  }
}

__device__ __forceinline__ void sym3_eig(double a00, double a11, double a22, double a01, double a02, double a12,
                                         double lam[3], double Q[9]) {
#pragma unroll
  for (int i = 0; i < 9; ++i) Q[i] = (i % 4 == 0) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 12; ++sweep) {
    const double off = a01 * a01 + a02 * a02 + a12 * a12;
    const double dia = a00 * a00 + a11 * a11 + a22 * a22;
    if (off <= 1e-32 * dia) break;
    // planes (0,1), (0,2), (1,2); the third index's couplings rotate along
    jacobi_rotate(a00, a11, a01, a02, a12, Q, 0, 1);
    jacobi_rotate(a00, a22, a02, a01, a12, Q, 0, 2);
    jacobi_rotate(a11, a22, a12, a01, a02, Q, 1, 2);
  }
  lam[0] = a00;
  lam[1] = a11;
  lam[2] = a22;
}

// ---------------------------------------------------------------------------
// Signed SVD F = U diag(s) V^T, U, V in SO(3), s0 >= s1 >= |s2| (the sign of
// det F on s2).  V diagonalises F^T F (Jacobi), then a Givens QR of B = F V
// gives U and the signed singular values on the diagonal of R.
// ---------------------------------------------------------------------------
// With warm = true, V holds on entry a rotation close to the answer (the
// previous iterate's): F^T F is first rotated into that frame, where it is
// nearly diagonal, so the Jacobi sweeps stop after one or two.
__device__ __forceinline__ void svd3(const double F[9], double U[9], double s[3], double V[9], bool warm = false) {
  // S = F^T F
  double a00 = 0, a11 = 0, a22 = 0, a01 = 0, a02 = 0, a12 = 0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double f0 = F[3 * k], f1 = F[3 * k + 1], f2 = F[3 * k + 2];
    a00 += f0 * f0; a11 += f1 * f1; a22 += f2 * f2;
    a01 += f0 * f1; a02 += f0 * f2; a12 += f1 * f2;
  }
  double lam[3];
  if (warm) {
    // S' = V^T S V
    double SV[9];
    const double Sm[9] = {a00, a01, a02, a01, a11, a12, a02, a12, a22};
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) SV[3 * i + j] = Sm[3 * i] * V[j] + Sm[3 * i + 1] * V[3 + j] + Sm[3 * i + 2] * V[6 + j];
    double Sp[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = i; j < 3; ++j) Sp[3 * i + j] = V[i] * SV[j] + V[3 + i] * SV[3 + j] + V[6 + i] * SV[6 + j];
    a00 = Sp[0]; a11 = Sp[4]; a22 = Sp[8]; a01 = Sp[1]; a02 = Sp[2]; a12 = Sp[5];
    jacobi_sweeps(a00, a11, a22, a01, a02, a12, V);
    lam[0] = a00; lam[1] = a11; lam[2] = a22;
  } else {
    sym3_eig(a00, a11, a22, a01, a02, a12, lam, V);
  }
  // sort eigenvalues descending; each swap negates one column to keep det V = +1
#define PD_SWAPCOL(i, j)                                               \
  {                                                                    \
    double tl = lam[i]; lam[i] = lam[j]; lam[j] = tl;                  \
    for (int k = 0; k < 3; ++k) {                                      \
      double tv = V[3 * k + i]; V[3 * k + i] = -V[3 * k + j]; V[3 * k + j] = tv; \
    }                                                                  \
  }
  if (lam[0] < lam[1]) PD_SWAPCOL(0, 1);
  if (lam[0] < lam[2]) PD_SWAPCOL(0, 2);
  if (lam[1] < lam[2]) PD_SWAPCOL(1, 2);
#undef PD_SWAPCOL
  // make V a proper rotation (Jacobi products already are; guard rounding)
  {
    const double d = V[0] * (V[4] * V[8] - V[5] * V[7]) - V[1] * (V[3] * V[8] - V[5] * V[6]) +
                     V[2] * (V[3] * V[7] - V[4] * V[6]);
    if (d < 0.0) { V[2] = -V[2]; V[5] = -V[5]; V[8] = -V[8]; }
  }
  // B = F V
  double B[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) B[3 * i + j] = F[3 * i] * V[j] + F[3 * i + 1] * V[3 + j] + F[3 * i + 2] * V[6 + j];
  // Givens QR: R = G3 G2 G1 B, U = (G3 G2 G1)^T
#pragma unroll
  for (int i = 0; i < 9; ++i) U[i] = (i % 4 == 0) ? 1.0 : 0.0;
  const int P[3] = {0, 0, 1}, Qr[3] = {1, 2, 2}, C[3] = {0, 0, 1};
#pragma unroll
  for (int g = 0; g < 3; ++g) {
    const int p = P[g], q = Qr[g], col = C[g];
    const double x = B[3 * p + col], y = B[3 * q + col];
    const double r = sqrt(x * x + y * y);
    double c = 1.0, sn = 0.0;
    if (r > 0.0) { c = x / r; sn = y / r; }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double bp = B[3 * p + k], bq = B[3 * q + k];
      B[3 * p + k] = c * bp + sn * bq;
      B[3 * q + k] = -sn * bp + c * bq;
      const double up = U[3 * k + p], uq = U[3 * k + q];  // U <- U G^T (columns p, q)
      U[3 * k + p] = c * up + sn * uq;
      U[3 * k + q] = -sn * up + c * uq;
    }
  }
  s[0] = B[0];
  s[1] = B[4];
  s[2] = B[8];
}

// ---------------------------------------------------------------------------
// Neo-Hookean stretch energy pieces (Sec. 3.2 Eq. neohookean in principal
// stretches, mesh means mu, lam) and the proximal objective
//   f(s) = k/2 |s - sF|^2 + mu/2 (sum s^2 - 3) - mu sum ln s + lam/2 (sum ln s)^2.
// ---------------------------------------------------------------------------
// mi is the weight of the I1 term: mu for the Neo-Hookean energy, 0 for the
// logarithmic volume barrier of Eq. pd_log_volume (-mu sum ln s + lam/2
// (sum ln s)^2, the same Newton on stretches without the I1 term).
__device__ __forceinline__ double prox_f(const double s[3], const double sF[3], double mi, double mu, double lam,
                                         double k) {
  const double l = log(s[0] * s[1] * s[2]);
  double q = 0.0, ss = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const double d = s[i] - sF[i];
    q += d * d;
    ss += s[i] * s[i];
  }
  return 0.5 * k * q + 0.5 * mi * (ss - 3.0) - mu * l + 0.5 * lam * l * l;
}

// Hessian of f: diag(k + mi + (mu - lam l + lam)/s_i^2) + lam u u^T with u_i = 1/s_i
// (Eq. nh_hessian_stretch with the diagonal read as mu (1 + s^-2)).
__device__ __forceinline__ void prox_hessian(const double s[3], double mi, double mu, double lam, double k, double l,
                                             double H[6]) {  // H00 H11 H22 H01 H02 H12
  const double u0 = 1.0 / s[0], u1 = 1.0 / s[1], u2 = 1.0 / s[2];
  const double dc = mu - lam * l + lam;
  H[0] = k + mi + dc * u0 * u0;
  H[1] = k + mi + dc * u1 * u1;
  H[2] = k + mi + dc * u2 * u2;
  H[3] = lam * u0 * u1;
  H[4] = lam * u0 * u2;
  H[5] = lam * u1 * u2;
}

// Proximal stretches s* = argmin f (Sec. 4.1 Eqs. nh_prox, nh_prox_normal).
// Damped Newton: Sherman-Morrison solve of (D + lam u u^T) d = -g when D > 0,
// otherwise a diagonally scaled gradient step; fraction-to-boundary 0.9 keeps
// s > 0; backtracking (Armijo) on f while the step is large; stops at
// |g|_inf <= 1e-13 k max(1, |sF|_inf).  Returns the Newton iteration count.
// ratio (may be null): per stretch, a previous s*/sF used as the start
// s = sF * ratio when both are positive.
__device__ __forceinline__ int prox_stretch_g(const double sF[3], double mi, double mu, double lam, double k,
                                              double s[3], const double* ratio) {
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    s[i] = fmax(sF[i], 0.1);
    if (ratio && sF[i] > 0.0 && ratio[i] > 0.0) s[i] = sF[i] * ratio[i];
  }
  const double sfmax = fmax(1.0, fmax(fabs(sF[0]), fmax(fabs(sF[1]), fabs(sF[2]))));
  const double gtol = 1e-13 * k * sfmax;
  int it = 0;
  for (; it < kNewtonCap; ++it) {
    const double l = log(s[0] * s[1] * s[2]);
    double g[3], u[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      u[i] = 1.0 / s[i];
      g[i] = k * (s[i] - sF[i]) + mi * s[i] - mu * u[i] + lam * l * u[i];
    }
    if (fmax(fabs(g[0]), fmax(fabs(g[1]), fabs(g[2]))) <= gtol) break;
    // Hessian = diag(D) + lam u u^T: the rank-one part carries lam / s_i^2 of
    // the diagonal, so D holds only the rest of it
    const double dc = mu - lam * l;
    double D[3], d[3];
    bool diag_pos = true;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      D[i] = k + mi + dc * u[i] * u[i];
      diag_pos = diag_pos && (D[i] > 0.0);
    }
    if (diag_pos) {
      // (D + lam u u^T)^{-1} g = D^{-1} g - D^{-1} u (lam u^T D^{-1} g) / (1 + lam u^T D^{-1} u)
      double ug = 0.0, uu = 0.0;
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        ug += u[i] * g[i] / D[i];
        uu += u[i] * u[i] / D[i];
      }
      const double f = lam * ug / (1.0 + lam * uu);
#pragma unroll
      for (int i = 0; i < 3; ++i) d[i] = -(g[i] - u[i] * f) / D[i];
    } else {
      // the diagonal part is not positive: the full 3x3 Hessian by Cholesky,
      // or, if it is indefinite too, its absolute-value filtered form
      double H[6];
      prox_hessian(s, mi, mu, lam, k, l, H);
      const double l00 = H[0];
      bool pd = l00 > 0.0;
      double L00 = 0, L10 = 0, L20 = 0, L11 = 0, L21 = 0, L22 = 0;
      if (pd) {
        L00 = sqrt(l00);
        L10 = H[3] / L00;
        L20 = H[4] / L00;
        const double a11 = H[1] - L10 * L10;
        pd = a11 > 0.0;
        if (pd) {
          L11 = sqrt(a11);
          L21 = (H[5] - L20 * L10) / L11;
          const double a22 = H[2] - L20 * L20 - L21 * L21;
          pd = a22 > 0.0;
          if (pd) L22 = sqrt(a22);
        }
      }
      if (pd) {
        const double y0 = -g[0] / L00, y1 = (-g[1] - L10 * y0) / L11, y2 = (-g[2] - L20 * y0 - L21 * y1) / L22;
        d[2] = y2 / L22;
        d[1] = (y1 - L21 * d[2]) / L11;
        d[0] = (y0 - L10 * d[1] - L20 * d[2]) / L00;
      } else {
        double ev[3], Q[9];
        sym3_eig(H[0], H[1], H[2], H[3], H[4], H[5], ev, Q);
        double t3[3];
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          const double a = -(Q[j] * g[0] + Q[3 + j] * g[1] + Q[6 + j] * g[2]);
          t3[j] = a / fmax(fabs(ev[j]), 1e-300);
        }
#pragma unroll
        for (int i = 0; i < 3; ++i) d[i] = Q[3 * i] * t3[0] + Q[3 * i + 1] * t3[1] + Q[3 * i + 2] * t3[2];
      }
    }
    double a = 1.0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
      if (d[i] < 0.0) a = fmin(a, 0.9 * s[i] / (-d[i]));
    const double dmax = fmax(fabs(d[0]), fmax(fabs(d[1]), fabs(d[2])));
    const double smax = fmax(s[0], fmax(s[1], s[2]));
    double sn[3];
    if (a == 1.0 && dmax <= 1e-4 * smax && diag_pos) {
      // close to the minimiser of a convex model: the full Newton step
#pragma unroll
      for (int i = 0; i < 3; ++i) sn[i] = s[i] + d[i];
    } else {
      const double f0 = prox_f(s, sF, mi, mu, lam, k);
      const double slope = g[0] * d[0] + g[1] * d[1] + g[2] * d[2];
      const double slack = 1e-13 * k * (1.0 + s[0] * s[0] + s[1] * s[1] + s[2] * s[2]);
      for (int ls = 0; ls < 40; ++ls) {
#pragma unroll
        for (int i = 0; i < 3; ++i) sn[i] = s[i] + a * d[i];
        if (prox_f(sn, sF, mi, mu, lam, k) <= f0 + 1e-4 * a * slope + slack) break;
        a *= 0.5;
      }
    }
    double step = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      step = fmax(step, fabs(sn[i] - s[i]));
      s[i] = sn[i];
    }
    if (step <= 1e-16 * smax) { ++it; break; }
  }
  return it;
}

__device__ __forceinline__ int prox_stretch(const double sF[3], double mu, double lam, double k, double s[3],
                                            const double* ratio = nullptr) {
  return prox_stretch_g(sF, mu, mu, lam, k, s, ratio);
}

// ---------------------------------------------------------------------------
// Filtered prox differential (Sec. 4.4 Eqs. Hprox, tr_blend, tr_ift):
//   D = k H~^+, H~ = (1 - tau) H_prox + tau |H_prox|, H_prox = H(s*) of f,
// pair coefficients c1 (symmetric part) and c2 (skew part) of the SVD
// differential.  D is returned packed: D00 D11 D22 D01 D02 D12.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void pair_coeffs(const double sF[3], const double ss[3], const double D[6], double c1[3],
                                            double c2[3]);

__device__ __forceinline__ void prox_diff_g(const double sF[3], const double ss[3], double mi, double mu, double lam,
                                            double k, double tau, double D[6], double c1[3], double c2[3]) {
  const double l = log(ss[0] * ss[1] * ss[2]);
  double H[6];
  prox_hessian(ss, mi, mu, lam, k, l, H);
  double ev[3], Q[9];
  sym3_eig(H[0], H[1], H[2], H[3], H[4], H[5], ev, Q);
  double kt[3];
  double kmax = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    kt[i] = (1.0 - tau) * ev[i] + tau * fabs(ev[i]);
    kmax = fmax(kmax, fabs(kt[i]));
  }
  double inv[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) inv[i] = (fabs(kt[i]) <= 1e-12 * kmax) ? 0.0 : k / kt[i];
  const int I0[6] = {0, 1, 2, 0, 0, 1}, I1[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
  for (int t = 0; t < 6; ++t) {
    const int i = I0[t], j = I1[t];
    D[t] = Q[3 * i] * inv[0] * Q[3 * j] + Q[3 * i + 1] * inv[1] * Q[3 * j + 1] + Q[3 * i + 2] * inv[2] * Q[3 * j + 2];
  }
  pair_coeffs(sF, ss, D, c1, c2);
}

__device__ __forceinline__ void prox_diff(const double sF[3], const double ss[3], double mu, double lam, double k,
                                          double tau, double D[6], double c1[3], double c2[3]) {
  prox_diff_g(sF, ss, mu, mu, lam, k, tau, D, c1, c2);
}

// Pair coefficients of the SVD differential of an isotropic stretch map
// sF -> ss with packed stretch Jacobian D: c1 = (ss_i - ss_j)/(sF_i - sF_j)
// (the symmetric limit (D_ii + D_jj)/2 - D_ij for coinciding stretches),
// c2 = (ss_i + ss_j)/(sF_i + sF_j) (denominator kept away from zero).
__device__ __forceinline__ void pair_coeffs(const double sF[3], const double ss[3], const double D[6], double c1[3],
                                            double c2[3]) {
  const double sfmax = fmax(1.0, fmax(fabs(sF[0]), fmax(fabs(sF[1]), fabs(sF[2]))));
  const int P0[3] = {0, 0, 1}, P1[3] = {1, 2, 2}, Dii[3] = {0, 0, 1}, Djj[3] = {1, 2, 2}, Dij[3] = {3, 4, 5};
#pragma unroll
  for (int pr = 0; pr < 3; ++pr) {
    const int i = P0[pr], j = P1[pr];
    const double dsf = sF[i] - sF[j];
    if (fabs(dsf) <= 1e-7 * sfmax)
      c1[pr] = 0.5 * (D[Dii[pr]] + D[Djj[pr]]) - D[Dij[pr]];
    else
      c1[pr] = (ss[i] - ss[j]) / dsf;
    double den = sF[i] + sF[j];
    if (fabs(den) < 1e-8) den = den < 0.0 ? -1e-8 : 1e-8;
    c2[pr] = (ss[i] + ss[j]) / den;
  }
}

// ---------------------------------------------------------------------------
// Volume step of the corotated + volume composite (Sec. 4.1, Sec. 7.2): the
// closest point sv of sF with sv1 sv2 sv3 = 1.  Stationarity gives
// sv_i (sv_i - sF_i) = nu, so sv_i = (sF_i +- sqrt(sF_i^2 + 4 nu)) / 2.  All
// roots take the plus sign unless even at the smallest admissible nu their
// product exceeds one; then the root of the smallest stretch takes the minus
// sign (nu between that bound and 0).  f(nu) = sum ln sv_i(nu) is brought to
// zero by Newton's method kept inside a sign-change bracket, starting from
// the tet's previous multiplier `nu` (updated on return).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double vol_eval(const double sF[3], double nu, int minus, double sv[3], double a[3]) {
  double f = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const double r = sqrt(fmax(sF[i] * sF[i] + 4.0 * nu, 0.0));
    const double sg = (i == minus) ? -1.0 : 1.0;
    sv[i] = 0.5 * (sF[i] + sg * r);
    a[i] = sg / fmax(r, 1e-300);  // d sv_i / d nu = 1 / (2 sv_i - sF_i)
    f += log(sv[i]);
  }
  return f;
}

__device__ __forceinline__ void volume_project(const double sF[3], double& nu, double sv[3]) {
  const bool pos = sF[0] > 0.0 && sF[1] > 0.0 && sF[2] > 0.0;
  int imin = 0;
#pragma unroll
  for (int i = 1; i < 3; ++i)
    if (fabs(sF[i]) < fabs(sF[imin])) imin = i;
  const double lo = pos ? -0.25 * sF[imin] * sF[imin] : 0.0;
  double a[3];
  int minus = -1;
  double l = lo, r;
  if (pos && vol_eval(sF, lo, -1, sv, a) > 0.0) {
    minus = imin;  // f decreases from f(lo) > 0 to -inf at nu = 0
    r = 0.0;
  } else {
    r = fmax(1.0, 2.0 * fabs(lo) + 1.0);
    for (int k = 0; k < 64 && vol_eval(sF, r, -1, sv, a) < 0.0; ++k) r *= 4.0;
  }
  // on either branch f(l) and f(r) have opposite signs; track them as "low" and "high"
  const double dir = (minus < 0) ? 1.0 : -1.0;  // f increasing (plus) or decreasing (mixed) in nu
  double x = (nu > l && nu < r) ? nu : 0.5 * (l + r);
  for (int it = 0; it < 80; ++it) {
    const double f = vol_eval(sF, x, minus, sv, a);
    if (f == 0.0) break;
    if (dir * f < 0.0) l = x; else r = x;
    double dfdnu = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) dfdnu += a[i] / sv[i];
    double xn = x - f / dfdnu;
    if (!(xn > l && xn < r)) xn = 0.5 * (l + r);
    if (xn == x || r - l <= 1e-16 * fmax(1.0, fabs(x))) { x = xn; break; }
    x = xn;
  }
  nu = x;
  vol_eval(sF, x, minus, sv, a);
}

// Stretch Jacobian of the volume step (packed D00 D11 D22 D01 D02 D12):
// D_ij = a_i sv_i delta_ij - a_i a_j / c, a_i = 1/(2 sv_i - sF_i),
// c = sum_k a_k / sv_k (from differentiating sv_i (sv_i - sF_i) = nu and
// sum ln sv_i = 0).
__device__ __forceinline__ void volume_diff(const double sF[3], const double sv[3], double D[6]) {
  double a[3], c = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    a[i] = 1.0 / (2.0 * sv[i] - sF[i]);
    c += a[i] / sv[i];
  }
  D[0] = a[0] * sv[0] - a[0] * a[0] / c;
  D[1] = a[1] * sv[1] - a[1] * a[1] / c;
  D[2] = a[2] * sv[2] - a[2] * a[2] / c;
  D[3] = -a[0] * a[1] / c;
  D[4] = -a[0] * a[2] / c;
  D[5] = -a[1] * a[2] / c;
}

// dP = U B V^T with B the differential of the stretches in the (U, V) frame
// of A = U^T dF V.
__device__ __forceinline__ void prox_diff_apply(const double U[9], const double V[9], const double D[6],
                                                const double c1[3], const double c2[3], const double dF[9],
                                                double dP[9]) {
  double T[9], A[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) T[3 * i + j] = U[i] * dF[j] + U[3 + i] * dF[3 + j] + U[6 + i] * dF[6 + j];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) A[3 * i + j] = T[3 * i] * V[j] + T[3 * i + 1] * V[3 + j] + T[3 * i + 2] * V[6 + j];
  double Bm[9];
  Bm[0] = D[0] * A[0] + D[3] * A[4] + D[4] * A[8];
  Bm[4] = D[3] * A[0] + D[1] * A[4] + D[5] * A[8];
  Bm[8] = D[4] * A[0] + D[5] * A[4] + D[2] * A[8];
  const int P0[3] = {0, 0, 1}, P1[3] = {1, 2, 2};
#pragma unroll
  for (int pr = 0; pr < 3; ++pr) {
    const int i = P0[pr], j = P1[pr];
    const double sy = 0.5 * (A[3 * i + j] + A[3 * j + i]);
    const double sk = 0.5 * (A[3 * i + j] - A[3 * j + i]);
    Bm[3 * i + j] = c1[pr] * sy + c2[pr] * sk;
    Bm[3 * j + i] = c1[pr] * sy - c2[pr] * sk;
  }
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) T[3 * i + j] = U[3 * i] * Bm[j] + U[3 * i + 1] * Bm[3 + j] + U[3 * i + 2] * Bm[6 + j];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) dP[3 * i + j] = T[3 * i] * V[3 * j] + T[3 * i + 1] * V[3 * j + 1] + T[3 * i + 2] * V[3 * j + 2];
}

}  // namespace pdhot
