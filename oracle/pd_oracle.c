/*
 * Plain FP64 CPU oracle: differentiable Projective Dynamics (PD) with the
 * Neo-Hookean proximal local step, stiffness-routed projective weights,
 * Rayleigh damping folded into the system matrix, bounded type-II Anderson
 * acceleration with the dual-gate stop, and the adjoint backward step with the
 * trust-region eigenvalue filter on the proximal-map Hessian.
 *
 * TEST INFRASTRUCTURE ONLY.  The GPU library never links, loads or calls this
 * file; only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark do.  Every routine is written for clarity, not speed: plain loops,
 * FP64, round-to-nearest, no fused multiply-add contraction (build with
 * -ffp-contract=off), serial.
 *
 * Citations name the paper's sections and equations (arXiv 2605.14526,
 * "DiffPhD").  Readings of places where the paper is silent or inconsistent are
 * marked READING and listed in the design notes of the repository.
 */
#include "pd_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* small dense helpers                                                       */
/* ------------------------------------------------------------------------ */

static void mat3_mul(const double A[9], const double B[9], double C[9]) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += A[3 * i + k] * B[3 * k + j];
      C[3 * i + j] = s;
    }
}

static void mat3_mul_tn(const double A[9], const double B[9], double C[9]) { /* A^T B */
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += A[3 * k + i] * B[3 * k + j];
      C[3 * i + j] = s;
    }
}

static void mat3_mul_nt(const double A[9], const double B[9], double C[9]) { /* A B^T */
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += A[3 * i + k] * B[3 * j + k];
      C[3 * i + j] = s;
    }
}

static double det3(const double A[9]) {
  return A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
         A[2] * (A[3] * A[7] - A[4] * A[6]);
}

static void inv3(const double A[9], double B[9]) {
  double d = det3(A);
  B[0] = (A[4] * A[8] - A[5] * A[7]) / d;
  B[1] = (A[2] * A[7] - A[1] * A[8]) / d;
  B[2] = (A[1] * A[5] - A[2] * A[4]) / d;
  B[3] = (A[5] * A[6] - A[3] * A[8]) / d;
  B[4] = (A[0] * A[8] - A[2] * A[6]) / d;
  B[5] = (A[2] * A[3] - A[0] * A[5]) / d;
  B[6] = (A[3] * A[7] - A[4] * A[6]) / d;
  B[7] = (A[1] * A[6] - A[0] * A[7]) / d;
  B[8] = (A[0] * A[4] - A[1] * A[3]) / d;
}

/* Cholesky of a small SPD matrix (n <= 8) in place (lower); returns 0 if not PD */
static int small_chol(double* A, int n) {
  for (int j = 0; j < n; ++j) {
    double d = A[j * n + j];
    for (int k = 0; k < j; ++k) d -= A[j * n + k] * A[j * n + k];
    if (!(d > 0.0)) return 0;
    d = sqrt(d);
    A[j * n + j] = d;
    for (int i = j + 1; i < n; ++i) {
      double s = A[i * n + j];
      for (int k = 0; k < j; ++k) s -= A[i * n + k] * A[j * n + k];
      A[i * n + j] = s / d;
    }
  }
  return 1;
}

static void small_chol_solve(const double* L, int n, const double* b, double* x) {
  double y[16];
  for (int i = 0; i < n; ++i) {
    double s = b[i];
    for (int k = 0; k < i; ++k) s -= L[i * n + k] * y[k];
    y[i] = s / L[i * n + i];
  }
  for (int i = n - 1; i >= 0; --i) {
    double s = y[i];
    for (int k = i + 1; k < n; ++k) s -= L[k * n + i] * x[k];
    x[i] = s / L[i * n + i];
  }
}

/* ------------------------------------------------------------------------ */
/* 3x3 symmetric eigendecomposition: cyclic Jacobi (used by the TR filter,   */
/* Sec. 4.4 "closed-form Jacobi sweep on 3x3 matrices")                      */
/* H = Q diag(kappa) Q^T, Q columns are eigenvectors.                         */
/* ------------------------------------------------------------------------ */
void or_sym3_eig(const double Hin[9], double kappa[3], double Q[9]) {
  double A[9];
  memcpy(A, Hin, sizeof(A));
  for (int i = 0; i < 9; ++i) Q[i] = (i % 4 == 0) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 50; ++sweep) {
    double off = A[1] * A[1] + A[2] * A[2] + A[5] * A[5];
    double diag = A[0] * A[0] + A[4] * A[4] + A[8] * A[8];
    if (off <= 1e-40 * diag || off == 0.0) break;
    for (int p = 0; p < 2; ++p)
      for (int r = p + 1; r < 3; ++r) {
        double apr = A[3 * p + r];
        if (apr == 0.0) continue;
        double theta = (A[3 * r + r] - A[3 * p + p]) / (2.0 * apr);
        double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        /* A <- J^T A J with J the rotation in plane (p, r) */
        for (int k = 0; k < 3; ++k) {
          double akp = A[3 * k + p], akr = A[3 * k + r];
          A[3 * k + p] = c * akp - s * akr;
          A[3 * k + r] = s * akp + c * akr;
        }
        for (int k = 0; k < 3; ++k) {
          double apk = A[3 * p + k], ark = A[3 * r + k];
          A[3 * p + k] = c * apk - s * ark;
          A[3 * r + k] = s * apk + c * ark;
        }
        for (int k = 0; k < 3; ++k) {
          double qkp = Q[3 * k + p], qkr = Q[3 * k + r];
          Q[3 * k + p] = c * qkp - s * qkr;
          Q[3 * k + r] = s * qkp + c * qkr;
        }
      }
  }
  for (int i = 0; i < 3; ++i) kappa[i] = A[4 * i];
}

/* ------------------------------------------------------------------------ */
/* Signed SVD of a 3x3 matrix (one-sided Jacobi, Hestenes).                  */
/* F = U diag(sig) V^T with U, V in SO(3), sig1 >= sig2 >= |sig3|, the sign  */
/* of det F carried by sig3 (used by the local step, Sec. 4.1 Eq. nh_prox).  */
/* ------------------------------------------------------------------------ */
void or_svd3(const double F[9], double U[9], double sig[3], double V[9]) {
  double W[9]; /* columns w_j = F v_j */
  memcpy(W, F, sizeof(W));
  for (int i = 0; i < 9; ++i) V[i] = (i % 4 == 0) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    int rotated = 0;
    for (int p = 0; p < 2; ++p)
      for (int r = p + 1; r < 3; ++r) {
        double a = 0, b = 0, g = 0;
        for (int k = 0; k < 3; ++k) {
          a += W[3 * k + p] * W[3 * k + p];
          b += W[3 * k + r] * W[3 * k + r];
          g += W[3 * k + p] * W[3 * k + r];
        }
        if (fabs(g) <= 1e-15 * sqrt(a * b) || g == 0.0) continue;
        rotated = 1;
        double zeta = (b - a) / (2.0 * g);
        double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
        for (int k = 0; k < 3; ++k) {
          double wp = W[3 * k + p], wr = W[3 * k + r];
          W[3 * k + p] = c * wp - s * wr;
          W[3 * k + r] = s * wp + c * wr;
          double vp = V[3 * k + p], vr = V[3 * k + r];
          V[3 * k + p] = c * vp - s * vr;
          V[3 * k + r] = s * vp + c * vr;
        }
      }
    if (!rotated) break;
  }
  /* sort columns by norm, descending */
  double nrm[3];
  for (int j = 0; j < 3; ++j) nrm[j] = sqrt(W[j] * W[j] + W[3 + j] * W[3 + j] + W[6 + j] * W[6 + j]);
  int ord[3] = {0, 1, 2};
  for (int i = 0; i < 3; ++i)
    for (int j = i + 1; j < 3; ++j)
      if (nrm[ord[j]] > nrm[ord[i]]) { int t = ord[i]; ord[i] = ord[j]; ord[j] = t; }
  double Ws[9], Vs[9], ns[3];
  for (int j = 0; j < 3; ++j) {
    ns[j] = nrm[ord[j]];
    for (int k = 0; k < 3; ++k) { Ws[3 * k + j] = W[3 * k + ord[j]]; Vs[3 * k + j] = V[3 * k + ord[j]]; }
  }
  /* make V a rotation: flipping v3 together with w3 leaves F unchanged */
  if (det3(Vs) < 0.0)
    for (int k = 0; k < 3; ++k) { Vs[3 * k + 2] = -Vs[3 * k + 2]; Ws[3 * k + 2] = -Ws[3 * k + 2]; }
  /* U: u1 = w1/|w1|, u2 = w2 orthogonalised, u3 = u1 x u2; sig3 = w3 . u3 (signed) */
  double u1[3], u2[3], u3[3];
  if (ns[0] > 0.0) {
    for (int k = 0; k < 3; ++k) u1[k] = Ws[3 * k] / ns[0];
  } else {
    u1[0] = 1; u1[1] = 0; u1[2] = 0;
  }
  double d12 = 0;
  for (int k = 0; k < 3; ++k) { u2[k] = Ws[3 * k + 1]; d12 += u1[k] * u2[k]; }
  for (int k = 0; k < 3; ++k) u2[k] -= d12 * u1[k];
  double n2 = sqrt(u2[0] * u2[0] + u2[1] * u2[1] + u2[2] * u2[2]);
  if (n2 <= 1e-300 || ns[1] <= 1e-14 * ns[0]) {
    /* rank <= 1: any unit vector orthogonal to u1 */
    double e[3] = {fabs(u1[0]) < 0.9 ? 1.0 : 0.0, fabs(u1[0]) < 0.9 ? 0.0 : 1.0, 0.0};
    double d = e[0] * u1[0] + e[1] * u1[1] + e[2] * u1[2];
    for (int k = 0; k < 3; ++k) u2[k] = e[k] - d * u1[k];
    n2 = sqrt(u2[0] * u2[0] + u2[1] * u2[1] + u2[2] * u2[2]);
  }
  for (int k = 0; k < 3; ++k) u2[k] /= n2;
  u3[0] = u1[1] * u2[2] - u1[2] * u2[1];
  u3[1] = u1[2] * u2[0] - u1[0] * u2[2];
  u3[2] = u1[0] * u2[1] - u1[1] * u2[0];
  for (int k = 0; k < 3; ++k) { U[3 * k] = u1[k]; U[3 * k + 1] = u2[k]; U[3 * k + 2] = u3[k]; }
  memcpy(V, Vs, sizeof(Vs));
  /* singular values as diagonal of U^T F V (exact up to rounding) */
  double T[9], S[9];
  mat3_mul_tn(U, F, T);
  mat3_mul(T, V, S);
  sig[0] = S[0];
  sig[1] = S[4];
  sig[2] = S[8];
}

/* ------------------------------------------------------------------------ */
/* Neo-Hookean energy, Sec. 3.2 Eq. neohookean:                               */
/* psi = mu/2 (|F|^2 - 3) - mu ln J + lam/2 (ln J)^2, +inf for J <= 0.        */
/* ------------------------------------------------------------------------ */
double or_psi_nh(const double F[9], double mu, double lam) {
  double J = det3(F);
  if (!(J > 0.0)) return INFINITY;
  double I1 = 0.0;
  for (int i = 0; i < 9; ++i) I1 += F[i] * F[i];
  double lj = log(J);
  return 0.5 * mu * (I1 - 3.0) - mu * lj + 0.5 * lam * lj * lj;
}

/* Stretch-space objective of the proximal step, Sec. 4.1 Eq. nh_prox reduced
 * by the SVD:  f(s) = k/2 |s - sF|^2 + psi(s),
 * psi(s) = mu/2 (sum s^2 - 3) - mu sum ln s + lam/2 (sum ln s)^2.
 * READING: V_e is dropped from the prox (the same stretch-space map in every
 * element, Sec. 4.2); the stationarity form grad f = 0 is solved (the printed
 * normal equation is its quadratic special case). */
/* mi: the weight of the I1 term (mu for the Neo-Hookean energy, 0 for the
 * logarithmic volume barrier of Eq. pd_log_volume) */
static double prox_obj(const double s[3], const double sF[3], double mi, double mu, double lam, double k) {
  if (!(s[0] > 0 && s[1] > 0 && s[2] > 0)) return INFINITY;
  double q = 0, ss = 0, sl = 0;
  for (int i = 0; i < 3; ++i) {
    q += (s[i] - sF[i]) * (s[i] - sF[i]);
    ss += s[i] * s[i];
    sl += log(s[i]);
  }
  return 0.5 * k * q + 0.5 * mi * (ss - 3.0) - mu * sl + 0.5 * lam * sl * sl;
}

/* gradient and Hessian of psi in stretch space.
 * READING of Eq. nh_hessian_stretch: the diagonal term is mu (1 + s^-2), the
 * exact second derivative of Eq. neohookean (the printed s^-4 is a typo). */
static void stretch_grad_hess(const double s[3], double mi, double mu, double lam, double g[3], double H[9]) {
  double l = log(s[0]) + log(s[1]) + log(s[2]);
  for (int i = 0; i < 3; ++i) g[i] = mi * s[i] - mu / s[i] + lam * l / s[i];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      if (i == j)
        H[3 * i + j] = (mi == mu ? mu * (1.0 + 1.0 / (s[i] * s[i])) : mi + mu / (s[i] * s[i])) +
                       lam * (1.0 - l) / (s[i] * s[i]);
      else
        H[3 * i + j] = lam / (s[i] * s[j]);
    }
}

static void psi_stretch_grad_hess(const double s[3], double mu, double lam, double g[3], double H[9]) {
  stretch_grad_hess(s, mu, mu, lam, g, H);
}

/* Proximal stretches, Sec. 4.1 Eqs. nh_prox / nh_prox_normal: Newton with
 * backtracking line search and positivity enforcement.
 * READING (constants the paper does not give): start max(sF, 0.1); direction
 * from a Cholesky of k I + H_psi, else of its absolute-value filtered form;
 * fraction-to-boundary step 0.9; Armijo c1 = 1e-4 with halving (<= 30) and a
 * rounding slack of 1e-13 k (1 + |s|^2);
 * stop at |g|_inf <= 1e-13 k max(1, |sF|_inf), a relative step <= 1e-15, or
 * 50 iterations.  Returns the iteration count (negative if the cap was hit). */
static int prox_newton(const double sF[3], double mi, double mu, double lam, double k, double s_out[3]) {
  double s[3];
  for (int i = 0; i < 3; ++i) s[i] = sF[i] > 0.1 ? sF[i] : 0.1;
  double sfmax = 1.0;
  for (int i = 0; i < 3; ++i) if (fabs(sF[i]) > sfmax) sfmax = fabs(sF[i]);
  double gtol = 1e-13 * k * sfmax;
  int it;
  for (it = 0; it < 50; ++it) {
    double gp[3], H[9], g[3];
    stretch_grad_hess(s, mi, mu, lam, gp, H);
    double gmax = 0;
    for (int i = 0; i < 3; ++i) {
      g[i] = k * (s[i] - sF[i]) + gp[i];
      H[4 * i] += k;
      if (fabs(g[i]) > gmax) gmax = fabs(g[i]);
    }
    if (gmax <= gtol) break;
    double L[9], d[3], mg[3] = {-g[0], -g[1], -g[2]};
    memcpy(L, H, sizeof(L));
    if (small_chol(L, 3)) {
      small_chol_solve(L, 3, mg, d);
    } else {
      double kap[3], Q[9], t[3];
      or_sym3_eig(H, kap, Q);
      for (int i = 0; i < 3; ++i) {
        double a = 0;
        for (int j = 0; j < 3; ++j) a += Q[3 * j + i] * mg[j];
        double ak = fabs(kap[i]) > 1e-300 ? fabs(kap[i]) : 1e-300;
        t[i] = a / ak;
      }
      for (int i = 0; i < 3; ++i) d[i] = Q[3 * i] * t[0] + Q[3 * i + 1] * t[1] + Q[3 * i + 2] * t[2];
    }
    double a0 = 1.0;
    for (int i = 0; i < 3; ++i)
      if (d[i] < 0.0) {
        double lim = 0.9 * s[i] / (-d[i]);
        if (lim < a0) a0 = lim;
      }
    double f0 = prox_obj(s, sF, mi, mu, lam, k);
    double slack = 1e-13 * k * (1.0 + s[0] * s[0] + s[1] * s[1] + s[2] * s[2]);
    double slope = g[0] * d[0] + g[1] * d[1] + g[2] * d[2];
    double a = a0, sn[3];
    int accepted = 0;
    for (int ls = 0; ls <= 30; ++ls) {
      for (int i = 0; i < 3; ++i) sn[i] = s[i] + a * d[i];
      double f1 = prox_obj(sn, sF, mi, mu, lam, k);
      /* the slack 1e-13 k (1 + |s|^2), the rounding level of the terms of f,
       * keeps the test meaningful once the decrease falls below what f can
       * resolve (close to the minimiser) */
      if (f1 <= f0 + 1e-4 * a * slope + slack) { accepted = 1; break; }
      a *= 0.5;
    }
    if (!accepted)
      for (int i = 0; i < 3; ++i) sn[i] = s[i] + a * d[i];
    double step = 0, nrm = 0;
    for (int i = 0; i < 3; ++i) {
      step += (sn[i] - s[i]) * (sn[i] - s[i]);
      nrm += sn[i] * sn[i];
      s[i] = sn[i];
    }
    if (sqrt(step) <= 1e-15 * sqrt(nrm)) { ++it; break; }
  }
  for (int i = 0; i < 3; ++i) s_out[i] = s[i];
  return it >= 50 ? -it : it;
}

int or_prox_stretch(const double sF[3], double mu, double lam, double k, double s_out[3]) {
  return prox_newton(sF, mu, mu, lam, k, s_out);
}

/* Volume step of the logarithmic barrier variant (Sec. 4.1 Eq. pd_log_volume):
 * the same Newton on stretches with the barrier -mu sum ln s + lam/2 (sum ln
 * s)^2 in place of psi (the I1 term dropped), Eq. nh_prox_normal's Hessian
 * replaced by the barrier's.  READING: like the Neo-Hookean prox it runs with
 * the mesh means, and its penalty is the mean of its weight, k = lam_bar (the
 * element's weight lam_e times the barrier with mu_e, lam_e has the same
 * minimiser, since mu_e / mu_bar = lam_e / lam_bar for a shared nu).  As
 * printed, the barrier's gradient at s = 1 is -mu, so the step is not the
 * identity at rest. */
int or_logvol_stretch(const double sF[3], double mu, double lam, double k, double s_out[3]) {
  return prox_newton(sF, 0.0, mu, lam, k, s_out);
}

/* stretch Jacobian of the barrier step: D = k (H + k I)^{-1} (the implicit
 * function theorem on its stationarity) */
static void logvol_diff(const double sv[3], double mu, double lam, double k, double D[9]) {
  double g[3], H[9];
  stretch_grad_hess(sv, 0.0, mu, lam, g, H);
  for (int i = 0; i < 3; ++i) H[4 * i] += k;
  or_tr_filter(H, 0.0, k, NULL, D);
}

/* p* = U diag(s*) V^T, Sec. 4.1 */
void or_prox_map(const double F[9], double mu, double lam, double k, double P[9]) {
  double U[9], V[9], sF[3], ss[3], T[9];
  or_svd3(F, U, sF, V);
  or_prox_stretch(sF, mu, lam, k, ss);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) T[3 * i + j] = U[3 * i + j] * ss[j];
  mat3_mul_nt(T, V, P);
}

/* Filtered proximal-map differential dp*_dF (9x9, row-major in (i,j) pairs):
 * Sec. 4.4 Eqs. Hprox, tr_blend, tr_ift and the SVD differential.
 * H_prox = H_psi(s*) + k I; H~ = (1 - tau) H_prox + tau |H_prox|;
 * D = k H~^+ (READING: pseudo-inverse, eigenvalues <= 1e-12 max are dropped);
 * in the (U, V) frame with A = U^T dF V: diagonal d p^_ii = sum_j D_ij A_jj;
 * for i < j with sym = (A_ij + A_ji)/2, skw = (A_ij - A_ji)/2:
 * d p^_ij = c1 sym + c2 skw, d p^_ji = c1 sym - c2 skw,
 * c1 = (s*_i - s*_j)/(sF_i - sF_j)  (limit (D_ii + D_jj)/2 - D_ij when the
 * two stretches coincide), c2 = (s*_i + s*_j)/(sF_i + sF_j) (denominator kept
 * away from zero by 1e-8 with its sign).  dp = U dp^ V^T. */
/* Trust-region blend of a symmetric 3x3 matrix, Eq. tr_blend:
 * H~(tau) = (1 - tau) H + tau |H| with |H| = Q diag(|kappa|) Q^T.
 * Returns H~ and, in Dinv, k times its pseudo-inverse (READING: eigenvalues
 * of H~ at most 1e-12 of the largest are treated as zero). */
void or_tr_filter(const double H[9], double tau, double k, double Ht[9], double Dinv[9]) {
  double kap[3], Q[9];
  or_sym3_eig(H, kap, Q);
  double kt[3], kmax = 0;
  for (int i = 0; i < 3; ++i) {
    kt[i] = (1.0 - tau) * kap[i] + tau * fabs(kap[i]);
    if (fabs(kt[i]) > kmax) kmax = fabs(kt[i]);
  }
  double inv[3];
  for (int i = 0; i < 3; ++i) inv[i] = (fabs(kt[i]) <= 1e-12 * kmax) ? 0.0 : 1.0 / kt[i];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0, t = 0;
      for (int l = 0; l < 3; ++l) {
        s += Q[3 * i + l] * inv[l] * Q[3 * j + l];
        t += Q[3 * i + l] * kt[l] * Q[3 * j + l];
      }
      if (Dinv) Dinv[3 * i + j] = k * s;
      if (Ht) Ht[3 * i + j] = t;
    }
}

/* pair coefficients of the SVD differential of an isotropic stretch map
 * sF -> ss with stretch Jacobian D (see above) */
static void pair_coeffs(const double sF[3], const double ss[3], const double D[9], double c1[3], double c2[3]) {
  const int P0[3] = {0, 0, 1}, P1[3] = {1, 2, 2};
  double sfmax = 1.0;
  for (int i = 0; i < 3; ++i) if (fabs(sF[i]) > sfmax) sfmax = fabs(sF[i]);
  for (int p = 0; p < 3; ++p) {
    int i = P0[p], j = P1[p];
    double dsf = sF[i] - sF[j];
    if (fabs(dsf) <= 1e-7 * sfmax)
      c1[p] = 0.5 * (D[3 * i + i] + D[3 * j + j]) - D[3 * i + j];
    else
      c1[p] = (ss[i] - ss[j]) / dsf;
    double den = sF[i] + sF[j];
    if (fabs(den) < 1e-8) den = den < 0 ? -1e-8 : 1e-8;
    c2[p] = (ss[i] + ss[j]) / den;
  }
}

static void prox_diff_coeffs(const double sF[3], const double ss[3], double mu, double lam, double k, double tau,
                             double D[9], double c1[3], double c2[3]) {
  double gp[3], H[9];
  psi_stretch_grad_hess(ss, mu, lam, gp, H);
  for (int i = 0; i < 3; ++i) H[4 * i] += k;
  /* H_prox = H_psi(s*) + k I (Eq. Hprox); D = k H~^+ solves Eq. tr_ift */
  or_tr_filter(H, tau, k, NULL, D);
  pair_coeffs(sF, ss, D, c1, c2);
}

static void prox_diff_apply(const double U[9], const double V[9], const double D[9], const double c1[3],
                            const double c2[3], const double dF[9], double dP[9]) {
  double T[9], A[9], B[9];
  mat3_mul_tn(U, dF, T);
  mat3_mul(T, V, A);
  for (int i = 0; i < 3; ++i) {
    double s = 0;
    for (int j = 0; j < 3; ++j) s += D[3 * i + j] * A[4 * j];
    B[4 * i] = s;
  }
  const int P0[3] = {0, 0, 1}, P1[3] = {1, 2, 2};
  for (int p = 0; p < 3; ++p) {
    int i = P0[p], j = P1[p];
    double sym = 0.5 * (A[3 * i + j] + A[3 * j + i]);
    double skw = 0.5 * (A[3 * i + j] - A[3 * j + i]);
    B[3 * i + j] = c1[p] * sym + c2[p] * skw;
    B[3 * j + i] = c1[p] * sym - c2[p] * skw;
  }
  mat3_mul(U, B, T);
  mat3_mul_nt(T, V, dP);
}

void or_prox_jacobian(const double F[9], double mu, double lam, double k, double tau, double J[81]) {
  double U[9], V[9], sF[3], ss[3], D[9], c1[3], c2[3];
  or_svd3(F, U, sF, V);
  or_prox_stretch(sF, mu, lam, k, ss);
  prox_diff_coeffs(sF, ss, mu, lam, k, tau, D, c1, c2);
  for (int col = 0; col < 9; ++col) {
    double dF[9] = {0}, dP[9];
    dF[col] = 1.0;
    prox_diff_apply(U, V, D, c1, c2, dF, dP);
    for (int r = 0; r < 9; ++r) J[9 * r + col] = dP[r];
  }
}

/* ------------------------------------------------------------------------ */
/* Corotated + volume composite (Sec. 4.1, volume-barrier paragraph: the     */
/* default heterogeneous PD assembly splits the projection into a corotated  */
/* rotation step and a volume step; Sec. 7.2: weights w0 = 2 mu_e for the    */
/* rotation, w1 = lam_e for the volume term).                                */
/* ------------------------------------------------------------------------ */

/* Volume step: the closest point of sF on {s > 0 : s1 s2 s3 = 1}, i.e. F
 * projected onto det F = 1 in stretch space (READING: the paper names the
 * step, not its constraint set).  Every stationary point of |s - sF|^2 on
 * the set has s_i (s_i - sF_i) = nu for one multiplier nu, so each s_i is a
 * root (sF_i +- sqrt(sF_i^2 + 4 nu)) / 2.  The candidates are the root choices
 * with at most one minus sign (two would leave the product below one); on
 * each, nu is found by bisection between sign changes of sum_i ln s_i(nu)
 * (located on a fine grid), and the candidate closest to sF is returned.
 * Returns the number of candidates. */
static int vol_roots(const double sF[3], double nu, int minus, double s[3]) {
  for (int i = 0; i < 3; ++i) {
    double d = sF[i] * sF[i] + 4.0 * nu;
    if (d < 0.0) return 0;
    s[i] = 0.5 * (sF[i] + (i == minus ? -sqrt(d) : sqrt(d)));
    if (!(s[i] > 0.0)) return 0;
  }
  return 1;
}

static double vol_phi(const double sF[3], double nu, int minus, int* ok) {
  double t[3];
  *ok = vol_roots(sF, nu, minus, t);
  return *ok ? log(t[0]) + log(t[1]) + log(t[2]) : 0.0;
}

int or_volume_project(const double sF[3], double s[3]) {
  double lo = -INFINITY;
  for (int i = 0; i < 3; ++i) if (-0.25 * sF[i] * sF[i] > lo) lo = -0.25 * sF[i] * sF[i];
  double best = INFINITY;
  int found = 0;
  for (int minus = -1; minus < 3; ++minus) {
    /* the nu range of this root choice: real roots above lo; a minus root needs nu < 0 */
    double a = lo, b;
    if (minus < 0) {
      b = 1.0;
      int ok;
      while (!(vol_phi(sF, b, minus, &ok) > 0.0) && b < 1e300) b *= 2.0;
    } else {
      if (!(sF[minus] > 0.0)) continue;
      b = 0.0;
    }
    const int N = 512;
    double prev_nu = 0.0, prev_phi = 0.0;
    int have_prev = 0;
    for (int k = 0; k <= N; ++k) {
      double nu = a + (b - a) * k / N;
      int ok;
      double ph = vol_phi(sF, nu, minus, &ok);
      if (!ok) { have_prev = 0; continue; }
      if (have_prev && ((prev_phi < 0.0) != (ph < 0.0) || ph == 0.0)) {
        double l = prev_nu, r = nu, pl = prev_phi;
        for (int it = 0; it < 200; ++it) {
          double mid = 0.5 * (l + r);
          if (mid <= l || mid >= r) break;
          int okm;
          double pm = vol_phi(sF, mid, minus, &okm);
          if (!okm) break;
          if ((pm < 0.0) == (pl < 0.0)) { l = mid; pl = pm; } else r = mid;
        }
        double c[3];
        if (vol_roots(sF, 0.5 * (l + r), minus, c)) {
          double dist = 0.0;
          for (int i = 0; i < 3; ++i) dist += (c[i] - sF[i]) * (c[i] - sF[i]);
          found++;
          if (dist < best) { best = dist; for (int i = 0; i < 3; ++i) s[i] = c[i]; }
        }
      }
      prev_nu = nu;
      prev_phi = ph;
      have_prev = 1;
    }
  }
  return found;
}

/* Stretch Jacobian of the volume step, from differentiating s_i (s_i - sF_i)
 * = nu and sum_i ln s_i = 0: with a_i = 1/(2 s_i - sF_i) and c = sum_k a_k/s_k,
 * D_ij = a_i s_i delta_ij - a_i a_j / c. */
static void volume_diff(const double sF[3], const double sv[3], double D[9]) {
  double a[3], c = 0.0;
  for (int i = 0; i < 3; ++i) { a[i] = 1.0 / (2.0 * sv[i] - sF[i]); c += a[i] / sv[i]; }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) D[3 * i + j] = (i == j ? a[i] * sv[i] : 0.0) - a[i] * a[j] / c;
}

/* The two projections at F: R = U V^T (the rotation of the signed polar
 * decomposition) and P_vol = U diag(s_vol) V^T, with their differentials in
 * the (U, V) frame: the rotation has D = 0 and the pair coefficients of the
 * constant map s = (1, 1, 1); the volume step has D from volume_diff. */
typedef struct {
  double U[9], V[9], sF[3], R[9], Pv[9], sv[3];
  double Dv[9], c1v[3], c2v[3], c1r[3], c2r[3];
} composite_parts;

/* kind 1: the volume projection; kind 2: the logarithmic barrier step with
 * the means mu_bar, lam_bar and penalty lam_bar */
static void composite_eval(const double F[9], composite_parts* c, int want_diff, int kind, double mu_bar,
                           double lam_bar) {
  double T[9];
  or_svd3(F, c->U, c->sF, c->V);
  mat3_mul_nt(c->U, c->V, c->R);
  if (kind == 2) or_logvol_stretch(c->sF, mu_bar, lam_bar, lam_bar, c->sv);
  else or_volume_project(c->sF, c->sv);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) T[3 * i + j] = c->U[3 * i + j] * c->sv[j];
  mat3_mul_nt(T, c->V, c->Pv);
  if (want_diff) {
    const double one[3] = {1.0, 1.0, 1.0}, zero[9] = {0};
    if (kind == 2) logvol_diff(c->sv, mu_bar, lam_bar, lam_bar, c->Dv);
    else volume_diff(c->sF, c->sv, c->Dv);
    pair_coeffs(c->sF, c->sv, c->Dv, c->c1v, c->c2v);
    pair_coeffs(c->sF, one, zero, c->c1r, c->c2r);
  }
}

static void composite_eval_s(const or_scene* s, const double F[9], composite_parts* c, int want_diff);

/* (2 mu R + lam P_vol) / (2 mu + lam): the composite's projection per unit of
 * its total weight w = 2 mu + lam (for element-level checks) */
void or_composite_map(const double F[9], double mu, double lam, double P[9]) {
  composite_parts c;
  composite_eval(F, &c, 0, 1, 0.0, 0.0);
  for (int i = 0; i < 9; ++i) P[i] = (2.0 * mu * c.R[i] + lam * c.Pv[i]) / (2.0 * mu + lam);
}

/* the same with the logarithmic barrier step (means mu_bar, lam_bar) */
void or_logvol_map(const double F[9], double mu_bar, double lam_bar, double mu, double lam, double P[9]) {
  composite_parts c;
  composite_eval(F, &c, 0, 2, mu_bar, lam_bar);
  for (int i = 0; i < 9; ++i) P[i] = (2.0 * mu * c.R[i] + lam * c.Pv[i]) / (2.0 * mu + lam);
}

void or_logvol_jacobian(const double F[9], double mu_bar, double lam_bar, double mu, double lam, double J[81]) {
  composite_parts c;
  const double zero[9] = {0};
  composite_eval(F, &c, 1, 2, mu_bar, lam_bar);
  for (int col = 0; col < 9; ++col) {
    double dF[9] = {0}, dR[9], dV[9];
    dF[col] = 1.0;
    prox_diff_apply(c.U, c.V, zero, c.c1r, c.c2r, dF, dR);
    prox_diff_apply(c.U, c.V, c.Dv, c.c1v, c.c2v, dF, dV);
    for (int r = 0; r < 9; ++r) J[9 * r + col] = (2.0 * mu * dR[r] + lam * dV[r]) / (2.0 * mu + lam);
  }
}

void or_composite_jacobian(const double F[9], double mu, double lam, double J[81]) {
  composite_parts c;
  const double zero[9] = {0};
  composite_eval(F, &c, 1, 1, 0.0, 0.0);
  for (int col = 0; col < 9; ++col) {
    double dF[9] = {0}, dR[9], dV[9];
    dF[col] = 1.0;
    prox_diff_apply(c.U, c.V, zero, c.c1r, c.c2r, dF, dR);
    prox_diff_apply(c.U, c.V, c.Dv, c.c1v, c.c2v, dF, dV);
    for (int r = 0; r < 9; ++r) J[9 * r + col] = (2.0 * mu * dR[r] + lam * dV[r]) / (2.0 * mu + lam);
  }
}

void or_volume_diff(const double sF[3], double D[9]) {
  double sv[3];
  or_volume_project(sF, sv);
  volume_diff(sF, sv, D);
}

/* ------------------------------------------------------------------------ */
/* scene                                                                     */
/* ------------------------------------------------------------------------ */
struct or_scene {
  int nv, ne, nf;
  double* X;
  int* tets;
  unsigned char* pinned;
  double* logE;
  double nu, rho, alpha, beta0, h, grav[3];
  int m, kmax_fwd, kmax_bwd;
  int energy; /* 0: Neo-Hookean proximal map; 1: corotated + volume composite; 2: corotated + log barrier */
  double eps_rel, eps_abs, eps_adj, eps_tr;
  /* derived (Sec. 3.1, 4.1, 4.2, 4.5) */
  double* Bhat;   /* ne x 4 x 3 shape gradients: F = sum_a x_a (x) Bhat_a */
  double* vol;    /* ne */
  double *mu, *lam, *w, *beta;
  double mu_bar, lam_bar, k_bar, mu_ref;
  double* mass; /* nv */
  int* fidx;    /* nv -> free index or -1 */
  int* fvert;   /* nf -> vertex */
  unsigned char* fmask3; /* 3 nv: 1 on the coordinates of free vertices */
  /* A~ restricted to free vertices, envelope (profile) storage */
  int* first;   /* nf: first column of row i */
  long* rowptr; /* nf+1: offset of row i's entries (columns first..i) */
  double* Aenv; /* assembled A~ (lower envelope) */
  double* Lenv; /* its Cholesky factor */
  /* muscle fibres (actuation; the reading is stated at or_scene_set_muscles):
   * group of each element (-1: passive), its unit fibre m_e in rest
   * coordinates, c_e[a] = Bhat_a . m_e (so F_e m_e = sum_a q_a c_e[a]), the
   * fibre weight w_m, the activations a_g, and the caller's accumulator of
   * dL/da_g that every backward step adds into (NULL: not formed) */
  int n_mg;
  double w_m;
  int* mgroup;
  double* mfib;  /* ne x 3 */
  double* mc;    /* ne x 4 */
  double* act;   /* n_mg */
  double* g_act; /* n_mg, caller-owned */
};

static void composite_eval_s(const or_scene* s, const double F[9], composite_parts* c, int want_diff) {
  composite_eval(F, c, want_diff, s->energy, s->mu_bar, s->lam_bar);
}

int or_scene_nfree(const or_scene* s) { return s->nf; }

void or_scene_info(const or_scene* s, double* vol, double* w, double* beta, double* mass, double* means4) {
  if (vol) memcpy(vol, s->vol, sizeof(double) * s->ne);
  if (w) memcpy(w, s->w, sizeof(double) * s->ne);
  if (beta) memcpy(beta, s->beta, sizeof(double) * s->ne);
  if (mass) memcpy(mass, s->mass, sizeof(double) * s->nv);
  if (means4) { means4[0] = s->mu_bar; means4[1] = s->lam_bar; means4[2] = s->k_bar; means4[3] = s->mu_ref; }
}

static double* env_at(double* env, const or_scene* s, int i, int j) { /* j <= i, j >= first[i] */
  return env + s->rowptr[i] + (j - s->first[i]);
}

/* deformation gradient F_e = sum_a q_a (x) Bhat_a (G_e q), Sec. 3.1 */
static void element_F(const or_scene* s, int e, const double* q, double F[9]) {
  for (int i = 0; i < 9; ++i) F[i] = 0.0;
  for (int a = 0; a < 4; ++a) {
    int v = s->tets[4 * e + a];
    const double* B = s->Bhat + 12 * e + 3 * a;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) F[3 * i + j] += q[3 * v + i] * B[j];
  }
}

/* The element loops below run in parallel (OpenMP over elements) and leave
 * each element's 12 contributions coef * (P Bhat_a)_i in a buffer; the
 * buffer is then added into y serially in element order, which is exactly
 * the order of a serial scatter, so results do not depend on the thread
 * count (bitwise). */
static void element_contrib(const or_scene* s, int e, double coef, const double P[9], double out[12]) {
  for (int a = 0; a < 4; ++a) {
    const double* B = s->Bhat + 12 * e + 3 * a;
    for (int i = 0; i < 3; ++i) {
      double t = 0;
      for (int j = 0; j < 3; ++j) t += P[3 * i + j] * B[j];
      out[3 * a + i] = coef * t;
    }
  }
}

/* Muscle of element e at deformation gradient F: the fibre image f = F m_e,
 * its length |f| and the fibre's target length l = 1 - a_g.  Returns 0 for a
 * passive element. */
static int muscle_eval(const or_scene* s, int e, const double F[9], double f[3], double* nf, double* ell) {
  if (!s->mgroup || s->mgroup[e] < 0) return 0;
  const double* m = s->mfib + 3 * e;
  for (int i = 0; i < 3; ++i) f[i] = F[3 * i] * m[0] + F[3 * i + 1] * m[1] + F[3 * i + 2] * m[2];
  *nf = sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
  *ell = 1.0 - s->act[s->mgroup[e]];
  return 1;
}

/* adds coef * G_e^T (x m_e^T) to out (12): the contribution of a fibre-space
 * vector x, since (x m^T) Bhat_a = (Bhat_a . m) x */
static void muscle_contrib_add(const or_scene* s, int e, double coef, const double x[3], double out[12]) {
  double P[9], cm[12];
  const double* m = s->mfib + 3 * e;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) P[3 * i + j] = x[i] * m[j];
  element_contrib(s, e, coef, P, cm);
  for (int i = 0; i < 12; ++i) out[i] += cm[i];
}

/* the fibre's projection onto the sphere of radius l: p = l f/|f| (l m_e for f = 0) */
static void muscle_project(const or_scene* s, int e, const double f[3], double nf, double ell, double p[3]) {
  for (int i = 0; i < 3; ++i) p[i] = nf > 0.0 ? ell * f[i] / nf : ell * s->mfib[3 * e + i];
}

/* its derivative applied to y: dp = (l/|f|)(y - f^ (f^ . y)) (zero for f = 0) */
static void muscle_dproj(const double f[3], double nf, double ell, const double y[3], double dp[3]) {
  if (!(nf > 0.0)) { dp[0] = dp[1] = dp[2] = 0.0; return; }
  double fh[3] = {f[0] / nf, f[1] / nf, f[2] / nf};
  double d = fh[0] * y[0] + fh[1] * y[1] + fh[2] * y[2];
  for (int i = 0; i < 3; ++i) dp[i] = ell / nf * (y[i] - fh[i] * d);
}

static void scatter_contribs(const or_scene* s, const double* ctb, double* y) {
  for (int e = 0; e < s->ne; ++e)
    for (int a = 0; a < 4; ++a) {
      int v = s->tets[4 * e + a];
      for (int i = 0; i < 3; ++i) y[3 * v + i] += ctb[12 * (size_t)e + 3 * a + i];
    }
}

/* thread count of the element loops (OpenMP); 0 leaves the runtime's default */
void or_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int or_get_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

static void assemble_factor(or_scene* s);

or_scene* or_scene_create(int nv, int ne, const double* X, const int* tets, const unsigned char* pinned,
                          const double* logE, const double* params, const double* solver) {
  or_scene* s = (or_scene*)calloc(1, sizeof(or_scene));
  s->nv = nv;
  s->ne = ne;
  s->X = (double*)malloc(sizeof(double) * 3 * nv);
  memcpy(s->X, X, sizeof(double) * 3 * nv);
  s->tets = (int*)malloc(sizeof(int) * 4 * ne);
  memcpy(s->tets, tets, sizeof(int) * 4 * ne);
  s->pinned = (unsigned char*)malloc(nv);
  memcpy(s->pinned, pinned, nv);
  s->logE = (double*)malloc(sizeof(double) * ne);
  memcpy(s->logE, logE, sizeof(double) * ne);
  s->nu = params[0]; s->rho = params[1]; s->alpha = params[2]; s->beta0 = params[3]; s->h = params[4];
  s->grav[0] = params[5]; s->grav[1] = params[6]; s->grav[2] = params[7];
  s->m = (int)solver[0]; s->eps_rel = solver[1]; s->eps_abs = solver[2];
  s->kmax_fwd = (int)solver[3]; s->kmax_bwd = (int)solver[4]; s->eps_adj = solver[5]; s->eps_tr = solver[6];
  s->energy = (int)solver[10];

  /* rest shape: tets reoriented to det D_m > 0; V_e = det/6; Bhat from D_m^-1 */
  s->Bhat = (double*)malloc(sizeof(double) * 12 * ne);
  s->vol = (double*)malloc(sizeof(double) * ne);
  for (int e = 0; e < ne; ++e) {
    int* t = s->tets + 4 * e;
    double Dm[9];
    for (int a = 1; a < 4; ++a)
      for (int i = 0; i < 3; ++i) Dm[3 * i + (a - 1)] = X[3 * t[a] + i] - X[3 * t[0] + i];
    if (det3(Dm) < 0.0) {
      int tmp = t[1]; t[1] = t[2]; t[2] = tmp;
      for (int a = 1; a < 4; ++a)
        for (int i = 0; i < 3; ++i) Dm[3 * i + (a - 1)] = X[3 * t[a] + i] - X[3 * t[0] + i];
    }
    double Bi[9];
    inv3(Dm, Bi);
    s->vol[e] = det3(Dm) / 6.0;
    double* B = s->Bhat + 12 * e;
    for (int j = 0; j < 3; ++j) {
      B[3 * 1 + j] = Bi[3 * 0 + j];
      B[3 * 2 + j] = Bi[3 * 1 + j];
      B[3 * 3 + j] = Bi[3 * 2 + j];
      B[j] = -(Bi[j] + Bi[3 + j] + Bi[6 + j]);
    }
  }
  /* Lame parameters, Eq. lame; weights w_e = 2 mu_e + lam_e (READING of Eq.
   * pd_weight: the rest tangent modulus of the Neo-Hookean energy, Sec. 7.2);
   * mesh means for the local prox (Sec. 4.2); beta_e = beta0 mu_e / mu_ref
   * with mu_ref = max mu_e (Sec. 4.5 Eq. rayleigh). */
  s->mu = (double*)malloc(sizeof(double) * ne);
  s->lam = (double*)malloc(sizeof(double) * ne);
  s->w = (double*)malloc(sizeof(double) * ne);
  s->beta = (double*)malloc(sizeof(double) * ne);
  double smu = 0, slam = 0, mref = 0;
  for (int e = 0; e < ne; ++e) {
    double E = exp(logE[e]);
    s->mu[e] = E / (2.0 * (1.0 + s->nu));
    s->lam[e] = E * s->nu / ((1.0 + s->nu) * (1.0 - 2.0 * s->nu));
    s->w[e] = 2.0 * s->mu[e] + s->lam[e];
    smu += s->mu[e];
    slam += s->lam[e];
    if (s->mu[e] > mref) mref = s->mu[e];
  }
  s->mu_bar = smu / ne;
  s->lam_bar = slam / ne;
  s->mu_ref = mref;
  /* optional frozen constants (finite-difference checks hold them fixed) */
  if (solver[7] > 0.0) { s->mu_bar = solver[7]; s->lam_bar = solver[8]; s->mu_ref = solver[9]; }
  s->k_bar = 2.0 * s->mu_bar + s->lam_bar;
  for (int e = 0; e < ne; ++e) s->beta[e] = s->beta0 * s->mu[e] / s->mu_ref;
  /* lumped mass m_v = sum_e rho V_e / 4 */
  s->mass = (double*)calloc(nv, sizeof(double));
  for (int e = 0; e < ne; ++e)
    for (int a = 0; a < 4; ++a) s->mass[s->tets[4 * e + a]] += s->rho * s->vol[e] / 4.0;
  /* free vertex numbering (original order) */
  s->fidx = (int*)malloc(sizeof(int) * nv);
  s->fvert = (int*)malloc(sizeof(int) * nv);
  s->nf = 0;
  for (int v = 0; v < nv; ++v) {
    if (pinned[v]) s->fidx[v] = -1;
    else { s->fidx[v] = s->nf; s->fvert[s->nf] = v; s->nf++; }
  }
  s->fmask3 = (unsigned char*)malloc(3 * (size_t)nv);
  for (int v = 0; v < nv; ++v) for (int ax = 0; ax < 3; ++ax) s->fmask3[3 * v + ax] = pinned[v] ? 0 : 1;
  assemble_factor(s);
  return s;
}

/* Envelope storage of A~ over the free vertices, its assembly and its
 * Cholesky factor (rebuilt when muscle fibres are set). */
static void assemble_factor(or_scene* s) {
  int nv = s->nv, ne = s->ne;
  (void)nv;
  free(s->first); free(s->rowptr); free(s->Aenv); free(s->Lenv);
  /* envelope of A~ */
  int nf = s->nf;
  s->first = (int*)malloc(sizeof(int) * (nf > 0 ? nf : 1));
  for (int i = 0; i < nf; ++i) s->first[i] = i;
  for (int e = 0; e < ne; ++e)
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) {
        int i = s->fidx[s->tets[4 * e + a]], j = s->fidx[s->tets[4 * e + b]];
        if (i >= 0 && j >= 0 && j < s->first[i]) s->first[i] = j;
      }
  s->rowptr = (long*)malloc(sizeof(long) * (nf + 1));
  s->rowptr[0] = 0;
  for (int i = 0; i < nf; ++i) s->rowptr[i + 1] = s->rowptr[i] + (i - s->first[i] + 1);
  s->Aenv = (double*)calloc(s->rowptr[nf] > 0 ? s->rowptr[nf] : 1, sizeof(double));
  s->Lenv = (double*)calloc(s->rowptr[nf] > 0 ? s->rowptr[nf] : 1, sizeof(double));
  /* A~ = (1 + alpha h) M / h^2 + sum_e (w_e + beta_e / h) V_e Bhat Bhat^T
   * (Sec. 4.5 Eq. A_damped; A = I_3 (x) A~ since |F|^2 separates by rows). */
  double h = s->h;
  for (int i = 0; i < nf; ++i) *env_at(s->Aenv, s, i, i) += (1.0 + s->alpha * h) * s->mass[s->fvert[i]] / (h * h);
  for (int e = 0; e < ne; ++e) {
    double c = (s->w[e] + s->beta[e] / h) * s->vol[e];
    const double* B = s->Bhat + 12 * e;
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) {
        int i = s->fidx[s->tets[4 * e + a]], j = s->fidx[s->tets[4 * e + b]];
        if (i < 0 || j < 0 || j > i) continue;
        double d = B[3 * a] * B[3 * b] + B[3 * a + 1] * B[3 * b + 1] + B[3 * a + 2] * B[3 * b + 2];
        *env_at(s->Aenv, s, i, j) += c * d;
      }
  }
  /* muscle fibres: w_m V_e G_m^T G_m = w_m V_e (c_e c_e^T) (x) I_3 */
  for (int e = 0; e < ne; ++e) {
    if (!s->mgroup || s->mgroup[e] < 0) continue;
    double c = s->w_m * s->vol[e];
    const double* mc = s->mc + 4 * e;
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) {
        int i = s->fidx[s->tets[4 * e + a]], j = s->fidx[s->tets[4 * e + b]];
        if (i < 0 || j < 0 || j > i) continue;
        *env_at(s->Aenv, s, i, j) += c * mc[a] * mc[b];
      }
  }
  /* envelope Cholesky A~ = L L^T (any ordering; the original one) */
  for (int i = 0; i < nf; ++i) {
    for (int j = s->first[i]; j <= i; ++j) {
      double sum = *env_at(s->Aenv, s, i, j);
      int k0 = s->first[i] > s->first[j] ? s->first[i] : s->first[j];
      for (int k = k0; k < j; ++k) sum -= *env_at(s->Lenv, s, i, k) * *env_at(s->Lenv, s, j, k);
      if (j < i) *env_at(s->Lenv, s, i, j) = sum / *env_at(s->Lenv, s, j, j);
      else *env_at(s->Lenv, s, i, i) = sqrt(sum);
    }
  }
}

/* READING (actuation; the paper's muscle-driven scenes route activations
 * through db/da but print no muscle energy): a muscle element carries the
 * fibre constraint (w_m V_e / 2) dist^2(F_e m_e, S_l) with S_l the sphere of
 * radius l = 1 - a_g in fibre space, a the activation of the element's group
 * (a > 0 shortens the fibre's rest length).  Its projection is p = l f/|f|
 * (f = F_e m_e); A~ gains w_m V_e (c_e c_e^T) (x) I_3 and b gains w_m V_e
 * G_m^T p, with G_m q = f; db/dq gains w_m V_e G_m^T (l/|f|)(I - f^ f^T) G_m
 * and db/da_g = -sum_{e in g} w_m V_e G_m^T f^.  Fibres must be unit vectors.
 * Setting muscles reassembles and refactors A~. */
void or_scene_set_muscles(or_scene* s, int n_groups, double w_m, const int* group, const double* fibre) {
  free(s->mgroup); free(s->mfib); free(s->mc); free(s->act);
  s->mgroup = NULL; s->mfib = NULL; s->mc = NULL; s->act = NULL;
  s->n_mg = n_groups;
  s->w_m = w_m;
  if (n_groups > 0 && group) {
    int ne = s->ne;
    s->mgroup = (int*)malloc(sizeof(int) * ne);
    s->mfib = (double*)malloc(sizeof(double) * 3 * ne);
    s->mc = (double*)calloc(4 * (size_t)ne, sizeof(double));
    s->act = (double*)calloc(n_groups, sizeof(double));
    memcpy(s->mgroup, group, sizeof(int) * ne);
    memcpy(s->mfib, fibre, sizeof(double) * 3 * ne);
    for (int e = 0; e < ne; ++e)
      for (int a = 0; a < 4; ++a) {
        const double* B = s->Bhat + 12 * e + 3 * a;
        const double* m = s->mfib + 3 * e;
        s->mc[4 * e + a] = B[0] * m[0] + B[1] * m[1] + B[2] * m[2];
      }
  }
  assemble_factor(s);
}

void or_scene_set_activation(or_scene* s, const double* a) {
  if (s->act) memcpy(s->act, a, sizeof(double) * s->n_mg);
}

void or_scene_set_act_grad(or_scene* s, double* g) { s->g_act = g; }

void or_scene_destroy(or_scene* s) {
  if (!s) return;
  free(s->X); free(s->tets); free(s->pinned); free(s->logE); free(s->Bhat); free(s->vol);
  free(s->mu); free(s->lam); free(s->w); free(s->beta); free(s->mass); free(s->fidx); free(s->fvert); free(s->fmask3);
  free(s->first); free(s->rowptr); free(s->Aenv); free(s->Lenv);
  free(s->mgroup); free(s->mfib); free(s->mc); free(s->act);
  free(s);
}

/* x = A~^{-1} r per axis, free rows only (Sec. 4.6: exact application of the
 * inverse from one factor; here an envelope Cholesky, forward + backward). */
void or_apply_Ainv(const or_scene* s, const double* r_all, double* x_all) {
  int nf = s->nf;
  for (int v = 0; v < s->nv; ++v)
    if (s->fidx[v] < 0) x_all[3 * v] = x_all[3 * v + 1] = x_all[3 * v + 2] = 0.0;
  /* the three axes are independent solves */
#pragma omp parallel for schedule(static, 1)
  for (int ax = 0; ax < 3; ++ax) {
    double* y = (double*)malloc(sizeof(double) * (nf > 0 ? nf : 1));
    for (int i = 0; i < nf; ++i) {
      double sum = r_all[3 * s->fvert[i] + ax];
      for (int k = s->first[i]; k < i; ++k) sum -= *env_at(s->Lenv, s, i, k) * y[k];
      y[i] = sum / *env_at(s->Lenv, s, i, i);
    }
    for (int i = nf - 1; i >= 0; --i) {
      double v = y[i] / *env_at(s->Lenv, s, i, i);
      y[i] = v;
      for (int k = s->first[i]; k < i; ++k) y[k] -= *env_at(s->Lenv, s, i, k) * v;
    }
    for (int i = 0; i < nf; ++i) x_all[3 * s->fvert[i] + ax] = y[i];
    free(y);
  }
}

void or_apply_A(const or_scene* s, const double* x_all, double* y_all) {
  for (int i = 0; i < 3 * s->nv; ++i) y_all[i] = 0.0;
  for (int i = 0; i < s->nf; ++i) {
    int vi = s->fvert[i];
    for (int j = s->first[i]; j <= i; ++j) {
      int vj = s->fvert[j];
      double a = *env_at(s->Aenv, s, i, j);
      for (int ax = 0; ax < 3; ++ax) {
        y_all[3 * vi + ax] += a * x_all[3 * vj + ax];
        if (j != i) y_all[3 * vj + ax] += a * x_all[3 * vi + ax];
      }
    }
  }
}

/* b(q) without its constant part: sum_e w_e V_e G_e^T p*_e(G_e q), Eq. A_basic */
static void local_rhs_stats(const or_scene* s, const double* q, double* b_all, int* capped, int* maxit) {
  for (int i = 0; i < 3 * s->nv; ++i) b_all[i] = 0.0;
  double* ctb = (double*)malloc(sizeof(double) * 12 * (size_t)(s->ne > 0 ? s->ne : 1));
  int ncap = 0, mit = 0;
#pragma omp parallel for schedule(static) reduction(+ : ncap) reduction(max : mit)
  for (int e = 0; e < s->ne; ++e) {
    double F[9], U[9], V[9], sF[3], ss[3], T[9], P[9];
    element_F(s, e, q, F);
    if (s->energy >= 1) {
      /* corotated + volume (or the barrier): 2 mu_e V_e G^T R + lam_e V_e G^T P_vol */
      composite_parts c;
      double cv[12];
      composite_eval_s(s, F, &c, 0);
      element_contrib(s, e, 2.0 * s->mu[e] * s->vol[e], c.R, ctb + 12 * (size_t)e);
      element_contrib(s, e, s->lam[e] * s->vol[e], c.Pv, cv);
      for (int i = 0; i < 12; ++i) ctb[12 * (size_t)e + i] += cv[i];
      continue;
    }
    or_svd3(F, U, sF, V);
    int it = or_prox_stretch(sF, s->mu_bar, s->lam_bar, s->k_bar, ss);
    if (it < 0) { ncap++; it = -it; }
    if (it > mit) mit = it;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) T[3 * i + j] = U[3 * i + j] * ss[j];
    mat3_mul_nt(T, V, P);
    element_contrib(s, e, s->w[e] * s->vol[e], P, ctb + 12 * (size_t)e);
  }
  /* muscle fibres: w_m V_e G_m^T p with p the fibre's projection */
  if (s->mgroup) {
#pragma omp parallel for schedule(static)
    for (int e = 0; e < s->ne; ++e) {
      double F[9], f[3], nf, ell, p[3];
      element_F(s, e, q, F);
      if (!muscle_eval(s, e, F, f, &nf, &ell)) continue;
      muscle_project(s, e, f, nf, ell, p);
      muscle_contrib_add(s, e, s->w_m * s->vol[e], p, ctb + 12 * (size_t)e);
    }
  }
  scatter_contribs(s, ctb, b_all);
  free(ctb);
  if (capped) *capped += ncap;
  if (maxit && mit > *maxit) *maxit = mit;
}

void or_local_rhs(const or_scene* s, const double* q, double* b_all) { local_rhs_stats(s, q, b_all, NULL, NULL); }

/* y = K x with K = db/dq = sum_e w_e V_e G_e^T (d p* / d F) G_e, Eq. db_dq */
void or_apply_K(const or_scene* s, const double* q, double tau, const double* x_all, double* y_all) {
  double* xf = (double*)malloc(sizeof(double) * 3 * s->nv);
  for (int v = 0; v < s->nv; ++v)
    for (int ax = 0; ax < 3; ++ax) xf[3 * v + ax] = s->fidx[v] >= 0 ? x_all[3 * v + ax] : 0.0;
  for (int i = 0; i < 3 * s->nv; ++i) y_all[i] = 0.0;
  double* ctb = (double*)malloc(sizeof(double) * 12 * (size_t)(s->ne > 0 ? s->ne : 1));
#pragma omp parallel for schedule(static)
  for (int e = 0; e < s->ne; ++e) {
    double F[9], U[9], V[9], sF[3], ss[3], D[9], c1[3], c2[3], dF[9], dP[9];
    element_F(s, e, q, F);
    if (s->energy >= 1) {
      composite_parts c;
      const double zero[9] = {0};
      double dR[9], cv[12];
      composite_eval_s(s, F, &c, 1);
      element_F(s, e, xf, dF);
      prox_diff_apply(c.U, c.V, zero, c.c1r, c.c2r, dF, dR);
      prox_diff_apply(c.U, c.V, c.Dv, c.c1v, c.c2v, dF, dP);
      element_contrib(s, e, 2.0 * s->mu[e] * s->vol[e], dR, ctb + 12 * (size_t)e);
      element_contrib(s, e, s->lam[e] * s->vol[e], dP, cv);
      for (int i = 0; i < 12; ++i) ctb[12 * (size_t)e + i] += cv[i];
      continue;
    }
    or_svd3(F, U, sF, V);
    or_prox_stretch(sF, s->mu_bar, s->lam_bar, s->k_bar, ss);
    prox_diff_coeffs(sF, ss, s->mu_bar, s->lam_bar, s->k_bar, tau, D, c1, c2);
    element_F(s, e, xf, dF);
    prox_diff_apply(U, V, D, c1, c2, dF, dP);
    element_contrib(s, e, s->w[e] * s->vol[e], dP, ctb + 12 * (size_t)e);
  }
  if (s->mgroup) {
#pragma omp parallel for schedule(static)
    for (int e = 0; e < s->ne; ++e) {
      double F[9], dF[9], f[3], nf, ell, y[3], dp[3];
      element_F(s, e, q, F);
      if (!muscle_eval(s, e, F, f, &nf, &ell)) continue;
      element_F(s, e, xf, dF);
      const double* m = s->mfib + 3 * e;
      for (int i = 0; i < 3; ++i) y[i] = dF[3 * i] * m[0] + dF[3 * i + 1] * m[1] + dF[3 * i + 2] * m[2];
      muscle_dproj(f, nf, ell, y, dp);
      muscle_contrib_add(s, e, s->w_m * s->vol[e], dp, ctb + 12 * (size_t)e);
    }
  }
  scatter_contribs(s, ctb, y_all);
  free(ctb);
  for (int v = 0; v < s->nv; ++v)
    if (s->fidx[v] < 0) y_all[3 * v] = y_all[3 * v + 1] = y_all[3 * v + 2] = 0.0;
  free(xf);
}

/* Per-element filtered prox differential at q (Alg. 2 element loop), stored
 * as U, V, D, c1, c2 (33 numbers per element) and applied to many vectors. */
#define KST 40 /* U, V, D, c1, c2 (33); the composite adds the rotation's c2; a muscle f = F m (3) and l */
static double* prox_diff_all(const or_scene* s, const double* q, double tau) {
  double* st = (double*)calloc(KST * (size_t)(s->ne > 0 ? s->ne : 1), sizeof(double));
#pragma omp parallel for schedule(static)
  for (int e = 0; e < s->ne; ++e) {
    double F[9], sF[3], ss[3];
    double* c = st + KST * (size_t)e;
    element_F(s, e, q, F);
    if (s->energy >= 1) {
      composite_parts p;
      composite_eval_s(s, F, &p, 1);
      memcpy(c, p.U, sizeof(p.U));
      memcpy(c + 9, p.V, sizeof(p.V));
      memcpy(c + 18, p.Dv, sizeof(p.Dv));
      memcpy(c + 27, p.c1v, sizeof(p.c1v));
      memcpy(c + 30, p.c2v, sizeof(p.c2v));
      memcpy(c + 33, p.c2r, sizeof(p.c2r));
      continue;
    }
    or_svd3(F, c, sF, c + 9);
    or_prox_stretch(sF, s->mu_bar, s->lam_bar, s->k_bar, ss);
    prox_diff_coeffs(sF, ss, s->mu_bar, s->lam_bar, s->k_bar, tau, c + 18, c + 27, c + 30);
  }
  if (s->mgroup) {
#pragma omp parallel for schedule(static)
    for (int e = 0; e < s->ne; ++e) {
      double F[9], nf;
      double* c = st + KST * (size_t)e;
      element_F(s, e, q, F);
      muscle_eval(s, e, F, c + 36, &nf, c + 39);
    }
  }
  return st;
}

static void apply_K_stored(const or_scene* s, const double* st, const double* x_all, double* y_all) {
  double* xf = (double*)malloc(sizeof(double) * 3 * s->nv);
  for (int v = 0; v < s->nv; ++v)
    for (int ax = 0; ax < 3; ++ax) xf[3 * v + ax] = s->fidx[v] >= 0 ? x_all[3 * v + ax] : 0.0;
  for (int i = 0; i < 3 * s->nv; ++i) y_all[i] = 0.0;
  double* ctb = (double*)malloc(sizeof(double) * 12 * (size_t)(s->ne > 0 ? s->ne : 1));
#pragma omp parallel for schedule(static)
  for (int e = 0; e < s->ne; ++e) {
    const double* c = st + KST * (size_t)e;
    double dF[9], dP[9];
    element_F(s, e, xf, dF);
    prox_diff_apply(c, c + 9, c + 18, c + 27, c + 30, dF, dP);
    if (s->energy >= 1) {
      /* 2 mu_e V_e G^T dR + lam_e V_e G^T dP_vol (the rotation's D and c1 vanish) */
      const double zero[9] = {0};
      double dR[9], cv[12];
      prox_diff_apply(c, c + 9, zero, zero, c + 33, dF, dR);
      element_contrib(s, e, 2.0 * s->mu[e] * s->vol[e], dR, ctb + 12 * (size_t)e);
      element_contrib(s, e, s->lam[e] * s->vol[e], dP, cv);
      for (int i = 0; i < 12; ++i) ctb[12 * (size_t)e + i] += cv[i];
      continue;
    }
    element_contrib(s, e, s->w[e] * s->vol[e], dP, ctb + 12 * (size_t)e);
  }
  if (s->mgroup) {
#pragma omp parallel for schedule(static)
    for (int e = 0; e < s->ne; ++e) {
      if (s->mgroup[e] < 0) continue;
      const double* c = st + KST * (size_t)e;
      const double* m = s->mfib + 3 * e;
      double dF[9], y[3], dp[3];
      const double* f = c + 36;
      double nf = sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
      element_F(s, e, xf, dF);
      for (int i = 0; i < 3; ++i) y[i] = dF[3 * i] * m[0] + dF[3 * i + 1] * m[1] + dF[3 * i + 2] * m[2];
      muscle_dproj(f, nf, c[39], y, dp);
      muscle_contrib_add(s, e, s->w_m * s->vol[e], dp, ctb + 12 * (size_t)e);
    }
  }
  scatter_contribs(s, ctb, y_all);
  free(ctb);
  for (int v = 0; v < s->nv; ++v)
    if (s->fidx[v] < 0) y_all[3 * v] = y_all[3 * v + 1] = y_all[3 * v + 2] = 0.0;
  free(xf);
}

/* the muscle energy of element e at F: (w_m V_e / 2)(|f| - l)^2 (dist^2 to the sphere), 0 if passive */
static double muscle_energy(const or_scene* s, int e, const double F[9]) {
  double f[3], nf, ell;
  if (!muscle_eval(s, e, F, f, &nf, &ell)) return 0.0;
  return 0.5 * s->w_m * s->vol[e] * (nf - ell) * (nf - ell);
}

/* Primal objective Phi, Eq. primal, with the true per-element mu_e, lam_e */
double or_primal_phi(const or_scene* s, const double* q, const double* qtilde) {
  double phi = 0.0, h = s->h;
  for (int v = 0; v < s->nv; ++v)
    for (int ax = 0; ax < 3; ++ax) {
      double d = q[3 * v + ax] - qtilde[3 * v + ax];
      phi += 0.5 / (h * h) * s->mass[v] * d * d;
    }
  double* pe = (double*)malloc(sizeof(double) * (s->ne > 0 ? s->ne : 1));
#pragma omp parallel for schedule(static)
  for (int e = 0; e < s->ne; ++e) {
    double F[9];
    element_F(s, e, q, F);
    pe[e] = s->vol[e] * or_psi_nh(F, s->mu[e], s->lam[e]) + muscle_energy(s, e, F);
  }
  for (int e = 0; e < s->ne; ++e) phi += pe[e];
  free(pe);
  return phi;
}

/* Constant part of the right-hand side (Alg. 1 prologue, Eq. freefall, and
 * READING of the damping terms from Eq. dynamics with v = (q - q_t)/h):
 * qtilde = q_t + h v_t + h^2 M^-1 f_ext + h^2 g,
 * c = M/h^2 qtilde + (alpha/h) M q_t + (1/h) B_beta q_t - A~_{free,pinned} q_pinned.
 * Pinned vertices are held at their rest positions. */
void or_const_rhs(const or_scene* s, const double* q_t, const double* v_t, const double* f_ext, double* c_all,
                  double* qtilde_all) {
  double h = s->h;
  for (int v = 0; v < s->nv; ++v)
    for (int ax = 0; ax < 3; ++ax) {
      double f = f_ext ? f_ext[3 * v + ax] : 0.0;
      double qt = q_t[3 * v + ax] + h * v_t[3 * v + ax] + h * h * (f / s->mass[v] + s->grav[ax]);
      if (qtilde_all) qtilde_all[3 * v + ax] = qt;
      c_all[3 * v + ax] = s->mass[v] / (h * h) * qt + s->alpha / h * s->mass[v] * q_t[3 * v + ax];
    }
  for (int e = 0; e < s->ne; ++e) {
    const double* B = s->Bhat + 12 * e;
    for (int a = 0; a < 4; ++a) {
      int va = s->tets[4 * e + a];
      for (int b = 0; b < 4; ++b) {
        int vb = s->tets[4 * e + b];
        double d = B[3 * a] * B[3 * b] + B[3 * a + 1] * B[3 * b + 1] + B[3 * a + 2] * B[3 * b + 2];
        double cb = s->beta[e] / h * s->vol[e] * d;                   /* (1/h) B_beta q_t */
        double cp = (s->w[e] + s->beta[e] / h) * s->vol[e] * d;       /* A~ coupling to pinned */
        if (s->mgroup && s->mgroup[e] >= 0) cp += s->w_m * s->vol[e] * s->mc[4 * e + a] * s->mc[4 * e + b];
        for (int ax = 0; ax < 3; ++ax) {
          c_all[3 * va + ax] += cb * q_t[3 * vb + ax];
          if (s->pinned[vb]) c_all[3 * va + ax] -= cp * s->X[3 * vb + ax];
        }
      }
    }
  }
  /* the pinned part of q is the rest position, so the A~ term on the pinned
   * block cancels the other pinned terms; pinned rows are never used. */
}

static double dot_free(const or_scene* s, const double* a, const double* b) {
  double r = 0.0;
  for (int v = 0; v < s->nv; ++v)
    if (s->fidx[v] >= 0)
      for (int ax = 0; ax < 3; ++ax) r += a[3 * v + ax] * b[3 * v + ax];
  return r;
}

/* One bounded type-II Anderson step on vectors of length n (Sec. 4.3, Eqs.
 * aa_dG, aa_dQ, aa_gamma, aa_update and the reliability guard).  The history
 * holds at most m+1 pairs (q^j, g^j), oldest first, in Hq, Hg (n x (m+1)), with
 * *hn pairs (READING: m+1 pairs give the m difference columns).  The pair
 * (q, g = qhat - q) is appended; with at least two pairs,
 *   gamma = (dG^T dG + rho I)^-1 dG^T g,  rho = max(1e-6 |dG|_F^2 / m_c, 1e-12),
 * m_c the current number of columns, and q_new = qhat - (dQ + dG) gamma; when
 * |gamma|_2 > 10 the history is dropped (the current pair included) and
 * q_new = qhat.  Inner products run over the entries with mask[i] != 0 (all if
 * mask is NULL).  gamma_out (may be NULL) receives gamma.  Returns 1 on a
 * reset, else 0. */
int or_aa_step(int n, int m, double* Hq, double* Hg, int* hn, const double* q, const double* qhat,
               const unsigned char* mask, double* qnew, double* gamma_out) {
  int hcap = m + 1, reset = 0;
  if (m <= 0) {
    memcpy(qnew, qhat, sizeof(double) * n);
    return 0;
  }
  if (*hn == hcap) {
    memmove(Hq, Hq + n, sizeof(double) * n * (hcap - 1));
    memmove(Hg, Hg + n, sizeof(double) * n * (hcap - 1));
    (*hn)--;
  }
  double* gq = Hq + (size_t)(*hn) * n;
  double* gg = Hg + (size_t)(*hn) * n;
  for (int i = 0; i < n; ++i) { gq[i] = q[i]; gg[i] = qhat[i] - q[i]; }
  (*hn)++;
  if (*hn < 2) {
    memcpy(qnew, qhat, sizeof(double) * n);
    return 0;
  }
  int mc = *hn - 1;
  double G[64], rhs[8], gam[8], L[64];
  const double* g = Hg + (size_t)mc * n;
  double* dG = (double*)malloc(sizeof(double) * n * mc);
  double* dQ = (double*)malloc(sizeof(double) * n * mc);
  for (int j = 0; j < mc; ++j)
    for (int i = 0; i < n; ++i) {
      dG[(size_t)j * n + i] = Hg[(size_t)(j + 1) * n + i] - Hg[(size_t)j * n + i];
      dQ[(size_t)j * n + i] = Hq[(size_t)(j + 1) * n + i] - Hq[(size_t)j * n + i];
    }
  double fro = 0;
  for (int a = 0; a < mc; ++a) {
    for (int c = 0; c < mc; ++c) {
      double d = 0;
      for (int i = 0; i < n; ++i) if (!mask || mask[i]) d += dG[(size_t)a * n + i] * dG[(size_t)c * n + i];
      G[a * mc + c] = d;
    }
    double d = 0;
    for (int i = 0; i < n; ++i) if (!mask || mask[i]) d += dG[(size_t)a * n + i] * g[i];
    rhs[a] = d;
    fro += G[a * mc + a];
  }
  double rho = 1e-6 * fro / mc;
  if (rho < 1e-12) rho = 1e-12;
  for (int a = 0; a < mc; ++a) G[a * mc + a] += rho;
  memcpy(L, G, sizeof(double) * mc * mc);
  double gn = INFINITY;
  if (small_chol(L, mc)) {
    small_chol_solve(L, mc, rhs, gam);
    gn = 0;
    for (int a = 0; a < mc; ++a) gn += gam[a] * gam[a];
    gn = sqrt(gn);
  }
  if (gn <= 10.0) {
    for (int i = 0; i < n; ++i) {
      double t = qhat[i];
      for (int j = 0; j < mc; ++j) t -= (dQ[(size_t)j * n + i] + dG[(size_t)j * n + i]) * gam[j];
      qnew[i] = t;
    }
    if (gamma_out) for (int a = 0; a < mc; ++a) gamma_out[a] = gam[a];
  } else {
    memcpy(qnew, qhat, sizeof(double) * n);
    *hn = 0;
    reset = 1;
  }
  free(dG);
  free(dQ);
  return reset;
}

/* ------------------------------------------------------------------------ */
/* forward step, Alg. 1 (no contact)                                         */
/* ------------------------------------------------------------------------ */

/* ------------------------------------------------------------------------ */
/* contact (Sec. 4.7), frictionless reading                                  */
/* ------------------------------------------------------------------------ */
/* READING (frictionless, per-step linearised obstacles): contact row c acts on
 * vertex v_c with unit normal n_c and gap delta_c = n_c . q_{v_c} - g_c (Sec. 4.7,
 * delta_{n,c}).  The impulse lambda_c >= 0 enters A~ q = b + J^T lambda, so
 * q = A~^{-1} b + sum_c lambda_c a_c n_c with a_c = A~^{-1} e_{v_c} (Eq. q_update)
 * and delta = delta_free + W lambda, W_cd = (n_c . n_d) [A~^{-1}]_{v_c v_d}
 * (the Delassus operator J A~^{-1} J^T).  Each PD iteration solves the
 * complementarity problem by Fischer-Burmeister semi-smooth Newton
 * (Eqs. fb_n, omega_E_n) with r_c = W_cc (READING: the paper's h^2 W_cc only
 * rescales lambda), restricted to rows with omega_c > 1e-12 and symmetrised as
 * (W_AA + diag(E/omega)) dlambda = -phi/omega (Eq. contact_system in role),
 * solved by dense Cholesky, then projected onto lambda >= 0; lambda carries
 * over between PD iterations. */
typedef struct or_contacts {
  int K;
  const int* v;
  const double* n;
  const double* g;
  double fb_tol;   /* third gate on the FB residual (READING: added to Eq. convergence_dual) */
  double* lambda;  /* K, warm start in, converged out */
  double* col;     /* K x nv: a_c (the axis-0 column of A~^{-1}, the same for every axis) */
  double* W;       /* K x K */
  double fb_res;
  int fb_iters;
  /* Coulomb friction (mu_f > 0): lambda holds 3 entries per contact (normal,
   * t1, t2), q_t gives the slip's start, e the frames, G the K x K block of
   * A~^{-1} between the contact vertices */
  double mu_f;
  const double* qt;
  double* e;
  double* G;
  /* bilateral rows (kind[c] = 1; NULL: every row unilateral) and the
   * restitution post-correction (rest_on, coefficient e_rest); backward: the
   * gradient of the loss w.r.t. each row's offset g_c (NULL: not formed) */
  const unsigned char* kind;
  int rest_on;
  double e_rest;
  double* g_gap;
} or_contacts;

/* READING (bilateral attachments, Sec. 4.7: the block projection leaves the
 * bilateral multipliers unconstrained): a bilateral row is the equality
 * n_c . q_{v_c} = g_c with a free multiplier; in the FB Newton its residual
 * is the gap itself (phi = delta, omega = 1, E = 0), it is always in the
 * Newton system and never projected, and the adjoint holds it as an
 * equality like an active unilateral row.  A full attachment of a vertex to a
 * point is three rows along the coordinate axes. */
static int row_bilateral(const or_contacts* con, int c) { return con->kind && con->kind[c] == 1; }

/* normal impulse of row c */
static double row_lam_n(const or_contacts* con, int c) { return con->mu_f > 0.0 ? con->lambda[3 * c] : con->lambda[c]; }

/* active rows of a converged step: every bilateral row, and the unilateral
 * rows whose normal impulse exceeds 1e-10 of the largest unilateral one */
static int row_active(const or_contacts* con, int c) {
  if (row_bilateral(con, c)) return 1;
  double lmax = 0.0;
  for (int d = 0; d < con->K; ++d)
    if (!row_bilateral(con, d) && row_lam_n(con, d) > lmax) lmax = row_lam_n(con, d);
  return lmax > 0.0 && row_lam_n(con, c) > 1e-10 * lmax;
}

/* READING (restitution; the paper states only that its velocity-level
 * post-correction fires while the normal velocity is negative and the
 * impulse positive): after the step, each active unilateral row c in row
 * order whose incoming normal velocity u = n_c . v_{t, v_c} is negative sets
 * the outgoing normal velocity of its vertex to -e u:
 * v <- v + n_c (-e u - n_c . v).  Positions are unchanged. */
static int restitution_rows(const or_contacts* con, const double* v_t, int* rows) {
  int n = 0;
  for (int c = 0; c < con->K; ++c) {
    if (row_bilateral(con, c) || !row_active(con, c)) continue;
    const double* nc = con->n + 3 * c;
    const double* v = v_t + 3 * con->v[c];
    if (nc[0] * v[0] + nc[1] * v[1] + nc[2] * v[2] < 0.0) rows[n++] = c;
  }
  return n;
}

static int chol_solve(double* A, int n, double* b) { /* SPD, in place (lower), returns 0 if not PD */
  for (int j = 0; j < n; ++j) {
    double d = A[(size_t)j * n + j];
    for (int k = 0; k < j; ++k) d -= A[(size_t)j * n + k] * A[(size_t)j * n + k];
    if (!(d > 0.0)) return 0;
    d = sqrt(d);
    A[(size_t)j * n + j] = d;
    for (int i = j + 1; i < n; ++i) {
      double t = A[(size_t)i * n + j];
      for (int k = 0; k < j; ++k) t -= A[(size_t)i * n + k] * A[(size_t)j * n + k];
      A[(size_t)i * n + j] = t / d;
    }
  }
  for (int i = 0; i < n; ++i) {
    double t = b[i];
    for (int k = 0; k < i; ++k) t -= A[(size_t)i * n + k] * b[k];
    b[i] = t / A[(size_t)i * n + i];
  }
  for (int i = n - 1; i >= 0; --i) {
    double t = b[i];
    for (int k = i + 1; k < n; ++k) t -= A[(size_t)k * n + i] * b[k];
    b[i] = t / A[(size_t)i * n + i];
  }
  return 1;
}

/* ------------------------------------------------------------------------ */
/* Coulomb friction (Sec. 4.7): three rows per contact                       */
/* ------------------------------------------------------------------------ */
/* READING (friction, Sec. 4.7 Eqs. fb_n, omega_E_n, contact_system, q_update
 * with the block projection onto the friction disk): contact c acts on vertex
 * v_c through the orthonormal frame (n_c, t1_c, t2_c) with impulse
 * lambda_c = (lambda_n, lambda_f1, lambda_f2).  Its kinematics are the
 * position-level normal gap delta_c = n_c . q_{v_c} - g_c and the slip
 * s_c = T_c^T (q_{v_c} - q_{t,v_c}) over the step (the tangential velocity
 * times h; Coulomb's law does not depend on that scale).  The law: delta >= 0,
 * lambda_n >= 0, delta lambda_n = 0; |lambda_f| <= mu lambda_n; s != 0 implies
 * lambda_f = -mu lambda_n s/|s|; |lambda_f| < mu lambda_n implies s = 0.  The
 * tangents: a = the coordinate axis of the smallest |n_i| (first on ties),
 * t1 = (a - (a.n) n)/|a - (a.n) n|, t2 = n x t1. */
void or_contact_frame(const double n[3], double t1[3], double t2[3]) {
  int k = 0;
  for (int i = 1; i < 3; ++i)
    if (fabs(n[i]) < fabs(n[k])) k = i;
  double a[3] = {0.0, 0.0, 0.0};
  a[k] = 1.0;
  double an = n[k];
  double t[3], nrm = 0.0;
  for (int i = 0; i < 3; ++i) {
    t[i] = a[i] - an * n[i];
    nrm += t[i] * t[i];
  }
  nrm = sqrt(nrm);
  for (int i = 0; i < 3; ++i) t1[i] = t[i] / nrm;
  t2[0] = n[1] * t1[2] - n[2] * t1[1];
  t2[1] = n[2] * t1[0] - n[0] * t1[2];
  t2[2] = n[0] * t1[1] - n[1] * t1[0];
}

/* frame rows of contact c: e[0..2] = n, e[3..5] = t1, e[6..8] = t2 */
static void frame_rows(const double* n, double e[9]) {
  e[0] = n[0]; e[1] = n[1]; e[2] = n[2];
  or_contact_frame(n, e + 3, e + 6);
}

/* The friction NCP of one PD iteration on u = u0 + W lambda (3K rows, W_rs =
 * (e_r . e_s) G_{c(r) c(s)} with G the K x K block of A~^{-1} between the
 * contact vertices, so every row of contact c has the diagonal w_c = G_cc).
 * READING (the per-iteration solve): semi-smooth Newton.  The normal row is
 * the Fischer-Burmeister function of Eq. fb_n with r_c = w_c and the weights
 * of Eq. omega_E_n; the tangent pair is the natural map F_f = lambda_f -
 * P_D(lambda_f - s/w_c) onto the disk D of radius tau_c = mu lambda_n (the
 * block projection of Sec. 4.7), tau taken at the current iterate.  Per
 * Newton step, with z = lambda_f - s/w:
 *   normal row: free if omega > 1e-12, equation W_n dl + (E/omega) dl_n =
 *     -phi/omega; otherwise fixed at dl_n = -lambda_n;
 *   tau = 0 (lambda_n = 0): both tangent rows fixed at dl_f = -lambda_f;
 *   |z| <= tau (stick): both rows free, W_f dl = -s;
 *   |z| > tau (slide): in the basis (z^, z^perp) the z^ row is fixed at
 *     dl_z = tau - lambda_f . z^ and the perp row is free with
 *     W_perp dl + w (1 - kappa)/kappa dl_perp = -w F_perp / kappa, kappa = tau/|z|.
 * The fixed rows' increments move to the right-hand side; the free rows form
 * a symmetric positive definite system (W's principal block plus a
 * non-negative diagonal), solved by dense Cholesky.  Then lambda_n <-
 * max(lambda_n, 0) and lambda_f <- its projection onto the disk of radius
 * mu lambda_n.  Stop at max_c max(|phi_c|, w_c |F_f,c|) <= 1e-14 (both in
 * displacement units) or after 50 steps; lambda carries over between PD
 * iterations. */
typedef struct fr_work {
  int K;
  const double* G;   /* K x K */
  const double* e;   /* K x 9 frame rows */
  double mu;
  const double* u0;  /* 3K: free gap and slip (lambda = 0) */
  double* lam;       /* 3K */
  double res;
  int iters;
} fr_work;

static void fr_u(const fr_work* f, const double* lam, double* u) {
  int K = f->K;
  for (int c = 0; c < K; ++c)
    for (int a = 0; a < 3; ++a) {
      double acc = f->u0[3 * c + a];
      const double* ea = f->e + 9 * c + 3 * a;
      for (int d = 0; d < K; ++d) {
        double g = f->G[(size_t)c * K + d];
        for (int b = 0; b < 3; ++b) {
          const double* eb = f->e + 9 * d + 3 * b;
          acc += (ea[0] * eb[0] + ea[1] * eb[1] + ea[2] * eb[2]) * g * lam[3 * d + b];
        }
      }
      u[3 * c + a] = acc;
    }
}

/* residual of every contact at lam; returns max */
static double fr_residual(const fr_work* f, const double* lam, const double* u) {
  double res = 0.0;
  for (int c = 0; c < f->K; ++c) {
    double w = f->G[(size_t)c * f->K + c];
    double a = u[3 * c], bb = w * lam[3 * c];
    double phi = a + bb - sqrt(a * a + bb * bb);
    double tau = f->mu * lam[3 * c];
    double z1 = lam[3 * c + 1] - u[3 * c + 1] / w, z2 = lam[3 * c + 2] - u[3 * c + 2] / w;
    double nz = sqrt(z1 * z1 + z2 * z2), p1 = z1, p2 = z2;
    if (tau <= 0.0) { p1 = 0.0; p2 = 0.0; }
    else if (nz > tau) { p1 = tau * z1 / nz; p2 = tau * z2 / nz; }
    double F1 = lam[3 * c + 1] - p1, F2 = lam[3 * c + 2] - p2;
    double rf = w * sqrt(F1 * F1 + F2 * F2);
    if (fabs(phi) > res) res = fabs(phi);
    if (rf > res) res = rf;
  }
  return res;
}

static void fr_newton(fr_work* f) {
  int K = f->K, R = 3 * K;
  double* u = (double*)malloc(sizeof(double) * R);
  double* dl = (double*)malloc(sizeof(double) * R);   /* increments in the row basis */
  double* rb = (double*)malloc(sizeof(double) * 9 * K); /* row directions (world) */
  int* isfree = (int*)malloc(sizeof(int) * R);
  double* diag = (double*)malloc(sizeof(double) * R);
  double* rhs = (double*)malloc(sizeof(double) * R);
  int* fr = (int*)malloc(sizeof(int) * R);
  double* M = (double*)malloc(sizeof(double) * (size_t)R * R);
  double* rot = (double*)malloc(sizeof(double) * 4 * K); /* 2x2 tangent basis per contact */
  fr_u(f, f->lam, u);
  double res = fr_residual(f, f->lam, u);
  int it = 0;
  for (; it < 50 && res > 1e-14; ++it) {
    for (int c = 0; c < K; ++c) {
      double w = f->G[(size_t)c * K + c];
      double* l = f->lam + 3 * c;
      const double* e = f->e + 9 * c;
      /* normal row */
      double a = u[3 * c], bb = w * l[0], sq = sqrt(a * a + bb * bb);
      double phi, om, E;
      if (sq == 0.0) { phi = 0.0; om = 1.0 - 1.0 / sqrt(2.0); E = w * (1.0 - 1.0 / sqrt(2.0)); }
      else { phi = a + bb - sq; om = 1.0 - a / sq; E = w * (1.0 - bb / sq); }
      for (int i = 0; i < 3; ++i) rb[9 * c + i] = e[i];
      if (om > 1e-12) { isfree[3 * c] = 1; diag[3 * c] = E / om; rhs[3 * c] = -phi / om; }
      else { isfree[3 * c] = 0; dl[3 * c] = -l[0]; }
      /* tangent rows */
      double tau = f->mu * l[0];
      double z1 = l[1] - u[3 * c + 1] / w, z2 = l[2] - u[3 * c + 2] / w;
      double nz = sqrt(z1 * z1 + z2 * z2);
      double* B = rot + 4 * c; /* rows: basis vectors in (t1, t2) coordinates */
      if (tau <= 0.0) {
        B[0] = 1.0; B[1] = 0.0; B[2] = 0.0; B[3] = 1.0;
        isfree[3 * c + 1] = 0; isfree[3 * c + 2] = 0;
        dl[3 * c + 1] = -l[1]; dl[3 * c + 2] = -l[2];
      } else if (nz <= tau) {
        B[0] = 1.0; B[1] = 0.0; B[2] = 0.0; B[3] = 1.0;
        isfree[3 * c + 1] = 1; isfree[3 * c + 2] = 1;
        diag[3 * c + 1] = 0.0; diag[3 * c + 2] = 0.0;
        rhs[3 * c + 1] = -u[3 * c + 1]; rhs[3 * c + 2] = -u[3 * c + 2];
      } else {
        double h1 = z1 / nz, h2 = z2 / nz, kap = tau / nz;
        B[0] = h1; B[1] = h2; B[2] = -h2; B[3] = h1;
        double lz = l[1] * h1 + l[2] * h2, lp = -l[1] * h2 + l[2] * h1;
        isfree[3 * c + 1] = 0; dl[3 * c + 1] = tau - lz;
        isfree[3 * c + 2] = 1; diag[3 * c + 2] = w * (1.0 - kap) / kap;
        /* F_perp = lambda_f . perp - P_perp = lp (P is along z^) */
        rhs[3 * c + 2] = -w * lp / kap;
      }
      for (int r = 0; r < 2; ++r)
        for (int i = 0; i < 3; ++i) rb[9 * c + 3 * (r + 1) + i] = B[2 * r] * e[3 + i] + B[2 * r + 1] * e[6 + i];
    }
    /* free rows, their system, fixed increments to the right-hand side */
    int nfr = 0;
    for (int r = 0; r < R; ++r) if (isfree[r]) fr[nfr++] = r;
    for (int i = 0; i < nfr; ++i) {
      int r = fr[i], c = r / 3;
      const double* er = rb + 9 * c + 3 * (r % 3);
      double t = rhs[r];
      for (int s2 = 0; s2 < R; ++s2) {
        if (isfree[s2]) continue;
        int d = s2 / 3;
        const double* es = rb + 9 * d + 3 * (s2 % 3);
        t -= (er[0] * es[0] + er[1] * es[1] + er[2] * es[2]) * f->G[(size_t)c * K + d] * dl[s2];
      }
      rhs[r] = t;
      for (int j = 0; j < nfr; ++j) {
        int s2 = fr[j], d = s2 / 3;
        const double* es = rb + 9 * d + 3 * (s2 % 3);
        M[(size_t)i * nfr + j] = (er[0] * es[0] + er[1] * es[1] + er[2] * es[2]) * f->G[(size_t)c * K + d];
      }
      M[(size_t)i * nfr + i] += diag[r];
    }
    double* x = (double*)malloc(sizeof(double) * (nfr > 0 ? nfr : 1));
    for (int i = 0; i < nfr; ++i) x[i] = rhs[fr[i]];
    int ok = nfr == 0 || chol_solve(M, nfr, x);
    if (!ok) { free(x); break; }
    for (int i = 0; i < nfr; ++i) dl[fr[i]] = x[i];
    free(x);
    /* update in the (t1, t2) frame, then the block projection */
    for (int c = 0; c < K; ++c) {
      double* l = f->lam + 3 * c;
      const double* B = rot + 4 * c;
      double ln = l[0] + dl[3 * c];
      double f1 = l[1] + B[0] * dl[3 * c + 1] + B[2] * dl[3 * c + 2];
      double f2 = l[2] + B[1] * dl[3 * c + 1] + B[3] * dl[3 * c + 2];
      ln = ln > 0.0 ? ln : 0.0;
      double tau = f->mu * ln, nf = sqrt(f1 * f1 + f2 * f2);
      if (tau <= 0.0) { f1 = 0.0; f2 = 0.0; }
      else if (nf > tau) { f1 *= tau / nf; f2 *= tau / nf; }
      l[0] = ln; l[1] = f1; l[2] = f2;
    }
    fr_u(f, f->lam, u);
    res = fr_residual(f, f->lam, u);
  }
  f->res = res;
  f->iters = it;
  free(u); free(dl); free(rb); free(isfree); free(diag); free(rhs); free(fr); free(M); free(rot);
}

/* the friction Newton alone on a given G (K x K), normals (K x 3) and free
 * kinematics u0 (3K: gap, slip along t1, t2), from lambda = 0; returns its
 * iterations */
int or_friction_ncp(int K, const double* G, const double* normals, const double* u0, double mu, double* lambda,
                    double* res) {
  double* e = (double*)malloc(sizeof(double) * 9 * (K > 0 ? K : 1));
  for (int c = 0; c < K; ++c) frame_rows(normals + 3 * c, e + 9 * c);
  for (int i = 0; i < 3 * K; ++i) lambda[i] = 0.0;
  fr_work f = {K, G, e, mu, u0, lambda, 0.0, 0};
  fr_newton(&f);
  if (res) *res = f.res;
  free(e);
  return f.iters;
}

static void contact_setup(const or_scene* s, or_contacts* con) {
  int nv = s->nv, n3 = 3 * nv, K = con->K;
  double* r = (double*)calloc(n3, sizeof(double));
  double* x = (double*)malloc(sizeof(double) * n3);
  con->col = (double*)malloc(sizeof(double) * (size_t)K * nv);
  con->W = (double*)malloc(sizeof(double) * (size_t)K * K);
  for (int c = 0; c < K; ++c) {
    r[3 * con->v[c]] = 1.0;
    or_apply_Ainv(s, r, x);
    r[3 * con->v[c]] = 0.0;
    for (int i = 0; i < nv; ++i) con->col[(size_t)c * nv + i] = x[3 * i];
  }
  for (int c = 0; c < K; ++c)
    for (int d = 0; d < K; ++d) {
      double nn = con->n[3 * c] * con->n[3 * d] + con->n[3 * c + 1] * con->n[3 * d + 1] +
                  con->n[3 * c + 2] * con->n[3 * d + 2];
      con->W[(size_t)c * K + d] = nn * con->col[(size_t)c * nv + con->v[d]];
    }
  if (con->mu_f > 0.0) {
    con->e = (double*)malloc(sizeof(double) * 9 * (size_t)(K > 0 ? K : 1));
    con->G = (double*)malloc(sizeof(double) * (size_t)(K > 0 ? K : 1) * (K > 0 ? K : 1));
    for (int c = 0; c < K; ++c) {
      frame_rows(con->n + 3 * c, con->e + 9 * c);
      for (int d = 0; d < K; ++d) con->G[(size_t)c * K + d] = con->col[(size_t)c * nv + con->v[d]];
    }
  }
  free(r);
  free(x);
}

static void contact_free(or_contacts* con) {
  free(con->col);
  free(con->W);
  free(con->e);
  free(con->G);
  con->col = NULL;
  con->W = NULL;
  con->e = NULL;
  con->G = NULL;
}

/* FB values of all rows at lambda; returns max |phi| */
static double fb_eval(const or_contacts* con, const double* dfree, const double* lam, double* phi, double* om,
                      double* E) {
  int K = con->K;
  double res = 0.0;
  for (int c = 0; c < K; ++c) {
    double delta = dfree[c];
    for (int d = 0; d < K; ++d) delta += con->W[(size_t)c * K + d] * lam[d];
    if (row_bilateral(con, c)) { /* equality row: the gap is the residual */
      phi[c] = delta;
      om[c] = 1.0;
      E[c] = 0.0;
      if (fabs(delta) > res) res = fabs(delta);
      continue;
    }
    double r = con->W[(size_t)c * K + c], a = delta, bb = r * lam[c];
    double sq = sqrt(a * a + bb * bb);
    if (sq == 0.0) {
      phi[c] = 0.0;
      om[c] = 1.0 - 1.0 / sqrt(2.0);
      E[c] = r * (1.0 - 1.0 / sqrt(2.0));
    } else {
      phi[c] = a + bb - sq;
      om[c] = 1.0 - a / sq;
      E[c] = r * (1.0 - bb / sq);
    }
    if (fabs(phi[c]) > res) res = fabs(phi[c]);
  }
  return res;
}

/* FB semi-smooth Newton on the LCP delta = dfree + W lambda (lambda warm in con->lambda) */
static void fb_newton(or_contacts* con, const double* dfree) {
  int K = con->K;
  double* phi = (double*)malloc(sizeof(double) * K);
  double* om = (double*)malloc(sizeof(double) * K);
  double* E = (double*)malloc(sizeof(double) * K);
  double* M = (double*)malloc(sizeof(double) * (size_t)K * K);
  double* rhs = (double*)malloc(sizeof(double) * K);
  int* act = (int*)malloc(sizeof(int) * K);
  double res = fb_eval(con, dfree, con->lambda, phi, om, E);
  int it = 0;
  for (; it < 30 && res > 1e-14; ++it) {
    int na = 0;
    for (int c = 0; c < K; ++c)
      if (om[c] > 1e-12) act[na++] = c;
      else con->lambda[c] = 0.0;
    for (int i = 0; i < na; ++i) {
      for (int j = 0; j < na; ++j) M[(size_t)i * na + j] = con->W[(size_t)act[i] * K + act[j]];
      M[(size_t)i * na + i] += E[act[i]] / om[act[i]];
      rhs[i] = -phi[act[i]] / om[act[i]];
    }
    if (na > 0 && !chol_solve(M, na, rhs)) break;
    for (int i = 0; i < na; ++i) {
      double l = con->lambda[act[i]] + rhs[i];
      con->lambda[act[i]] = (l > 0.0 || row_bilateral(con, act[i])) ? l : 0.0;
    }
    res = fb_eval(con, dfree, con->lambda, phi, om, E);
  }
  con->fb_res = res;
  con->fb_iters = it;
  free(phi); free(om); free(E); free(M); free(rhs); free(act);
}

/* the same with friction: kinematics of every contact at qhat, the friction
 * Newton, then qhat += sum_c a_c (lambda_n n + lambda_f1 t1 + lambda_f2 t2)
 * (Eq. q_update with the frame folded into lambda) */
static void contact_solve_fr(const or_scene* s, or_contacts* con, double* qhat) {
  int K = con->K, nv = s->nv;
  double* u0 = (double*)malloc(sizeof(double) * 3 * (size_t)K);
  for (int c = 0; c < K; ++c) {
    int v = con->v[c];
    const double* q = qhat + 3 * v;
    const double* p = con->qt + 3 * v;
    const double* e = con->e + 9 * c;
    u0[3 * c] = e[0] * q[0] + e[1] * q[1] + e[2] * q[2] - con->g[c];
    for (int a = 1; a < 3; ++a)
      u0[3 * c + a] = e[3 * a] * (q[0] - p[0]) + e[3 * a + 1] * (q[1] - p[1]) + e[3 * a + 2] * (q[2] - p[2]);
  }
  fr_work f = {K, con->G, con->e, con->mu_f, u0, con->lambda, 0.0, 0};
  fr_newton(&f);
  con->fb_res = f.res;
  con->fb_iters = f.iters;
  for (int c = 0; c < K; ++c) {
    const double* l = con->lambda + 3 * c;
    const double* e = con->e + 9 * c;
    double imp[3];
    for (int ax = 0; ax < 3; ++ax) imp[ax] = l[0] * e[ax] + l[1] * e[3 + ax] + l[2] * e[6 + ax];
    if (imp[0] == 0.0 && imp[1] == 0.0 && imp[2] == 0.0) continue;
    const double* a = con->col + (size_t)c * nv;
    for (int i = 0; i < nv; ++i) {
      if (s->fidx[i] < 0) continue;
      for (int ax = 0; ax < 3; ++ax) qhat[3 * i + ax] += a[i] * imp[ax];
    }
  }
  free(u0);
}

/* solve the contact problem at qhat (lambda warm) and add sum lambda_c a_c n_c to qhat */
static void contact_solve(const or_scene* s, or_contacts* con, double* qhat) {
  if (con->mu_f > 0.0) {
    contact_solve_fr(s, con, qhat);
    return;
  }
  int K = con->K, nv = s->nv;
  double* dfree = (double*)malloc(sizeof(double) * K);
  for (int c = 0; c < K; ++c) {
    const double* q = qhat + 3 * con->v[c];
    dfree[c] = con->n[3 * c] * q[0] + con->n[3 * c + 1] * q[1] + con->n[3 * c + 2] * q[2] - con->g[c];
  }
  fb_newton(con, dfree);
  for (int c = 0; c < K; ++c) {
    double l = con->lambda[c];
    if (l == 0.0) continue;
    const double* a = con->col + (size_t)c * nv;
    for (int i = 0; i < nv; ++i) {
      if (s->fidx[i] < 0) continue;
      for (int ax = 0; ax < 3; ++ax) qhat[3 * i + ax] += l * a[i] * con->n[3 * c + ax];
    }
  }
  free(dfree);
}

/* the FB Newton solve alone, on a given W and free gap (for checks); returns the Newton iterations */
int or_fb_lcp(int K, const double* W, const double* dfree, double* lambda, double* res) {
  or_contacts con = {K, NULL, NULL, NULL, 0.0, lambda, NULL, (double*)W, 0.0, 0};
  for (int c = 0; c < K; ++c) lambda[c] = 0.0;
  fb_newton(&con, dfree);
  if (res) *res = con.fb_res;
  return con.fb_iters;
}

static int step_forward_impl(const or_scene* s, const double* q_t, const double* v_t, const double* f_ext,
                             const double* q0, double* q_next, double* v_next, double* q_star_m1, int force_iters,
                             int m_override, int rec_max, double* rec, int* istats, double* dstats,
                             or_contacts* con) {
  int nv = s->nv, n3 = 3 * nv;
  int m = m_override >= 0 ? m_override : s->m;
  double* c = (double*)malloc(sizeof(double) * n3);
  double* q = (double*)malloc(sizeof(double) * n3);
  double* qprev = (double*)malloc(sizeof(double) * n3);
  double* b = (double*)malloc(sizeof(double) * n3);
  double* bprev = (double*)malloc(sizeof(double) * n3);
  double* qhat = (double*)malloc(sizeof(double) * n3);
  double* g = (double*)malloc(sizeof(double) * n3);
  /* history H of (q, g) pairs, at most m+1 entries (READING: m difference
   * columns), stored oldest first */
  int hcap = m + 1;
  double* Hq = (double*)malloc(sizeof(double) * n3 * (hcap > 0 ? hcap : 1));
  double* Hg = (double*)malloc(sizeof(double) * n3 * (hcap > 0 ? hcap : 1));
  int hn = 0;
  or_const_rhs(s, q_t, v_t, f_ext, c, NULL);
  /* q^0 = q_t (or the supplied warm start), pinned entries at rest */
  for (int v = 0; v < nv; ++v)
    for (int ax = 0; ax < 3; ++ax) {
      double x = q0 ? q0[3 * v + ax] : q_t[3 * v + ax];
      q[3 * v + ax] = s->pinned[v] ? s->X[3 * v + ax] : x;
    }
  memcpy(qprev, q, sizeof(double) * n3);
  int k, status = 1, resets = 0, capped = 0, maxit = 0;
  double gate[4] = {0, 0, 0, 0};
  if (con) {
    contact_setup(s, con);
    int nl = con->mu_f > 0.0 ? 3 * con->K : con->K;
    for (int c = 0; c < nl; ++c) con->lambda[c] = 0.0;
    con->fb_res = 0.0;
  }
  int kmax = force_iters > 0 ? force_iters + 1 : s->kmax_fwd;
  for (k = 0; k < kmax; ++k) {
    if (rec && k < rec_max) memcpy(rec + (size_t)k * n3, q, sizeof(double) * n3);
    /* local step and right-hand side, Alg. 1 */
    local_rhs_stats(s, q, b, &capped, &maxit);
    for (int i = 0; i < n3; ++i) b[i] += c[i];
    /* dual gate, Eq. convergence_dual, evaluated once b(q^k) exists: it
     * compares q^k with q^{k-1} and b^k with b^{k-1}; the paper's "k >= 1"
     * at loop index k-1 means k >= 2 here. */
    if (k >= 1) {
      double dq = 0, nq = 0, db = 0, nb = 0;
      for (int v = 0; v < nv; ++v) {
        if (s->fidx[v] < 0) continue;
        for (int ax = 0; ax < 3; ++ax) {
          int i = 3 * v + ax;
          dq += (q[i] - qprev[i]) * (q[i] - qprev[i]);
          nq += qprev[i] * qprev[i];
          db += (b[i] - bprev[i]) * (b[i] - bprev[i]);
          nb += bprev[i] * bprev[i];
        }
      }
      gate[0] = sqrt(dq); gate[1] = sqrt(nq); gate[2] = sqrt(db); gate[3] = sqrt(nb);
      int pass = gate[0] <= s->eps_rel * gate[1] + s->eps_abs && gate[2] <= s->eps_rel * gate[3] + s->eps_abs;
      if (con) pass = pass && con->fb_res <= con->fb_tol;
      if (force_iters <= 0 && k >= 2 && pass) { status = 0; break; }
    }
    if (force_iters > 0 && k == force_iters) { status = 0; break; }
    if (force_iters <= 0 && k == kmax - 1) break; /* not converged */
    /* global solve q^ = A^-1 b, Eq. two_spmv (role) */
    or_apply_Ainv(s, b, qhat);
    if (con) contact_solve(s, con, qhat);
    /* bounded type-II Anderson acceleration, Eqs. aa_dG..aa_update */
    memcpy(qprev, q, sizeof(double) * n3);
    memcpy(bprev, b, sizeof(double) * n3);
    memcpy(g, q, sizeof(double) * n3);
    if (or_aa_step(n3, m, Hq, Hg, &hn, g, qhat, s->fmask3, q, NULL)) resets++;
    /* Dirichlet vertices stay at rest */
    for (int v = 0; v < nv; ++v)
      if (s->pinned[v]) for (int ax = 0; ax < 3; ++ax) q[3 * v + ax] = s->X[3 * v + ax];
  }
  for (int i = 0; i < n3; ++i) {
    q_next[i] = q[i];
    v_next[i] = (q[i] - q_t[i]) / s->h;
    if (q_star_m1) q_star_m1[i] = qprev[i];
  }
  if (con && con->rest_on && con->K > 0) { /* restitution post-correction (reading at restitution_rows) */
    int* rows = (int*)malloc(sizeof(int) * con->K);
    int nr = restitution_rows(con, v_t, rows);
    for (int r = 0; r < nr; ++r) {
      int c = rows[r], vx = con->v[c];
      const double* nc = con->n + 3 * c;
      double* v = v_next + 3 * vx;
      const double* vi = v_t + 3 * vx;
      double u = nc[0] * vi[0] + nc[1] * vi[1] + nc[2] * vi[2];
      double vn = nc[0] * v[0] + nc[1] * v[1] + nc[2] * v[2];
      for (int ax = 0; ax < 3; ++ax) v[ax] += nc[ax] * (-con->e_rest * u - vn);
    }
    free(rows);
  }
  if (istats) { istats[0] = k; istats[1] = resets; istats[2] = capped; istats[3] = maxit; istats[4] = status; }
  if (dstats) for (int i = 0; i < 4; ++i) dstats[i] = gate[i];
  if (con) contact_free(con);
  free(c); free(q); free(qprev); free(b); free(bprev); free(qhat); free(g); free(Hq); free(Hg);
  return status;
}

int or_step_forward(const or_scene* s, const double* q_t, const double* v_t, const double* f_ext, const double* q0,
                    double* q_next, double* v_next, double* q_star_m1, int force_iters, int m_override,
                    int rec_max, double* rec, int* istats, double* dstats) {
  return step_forward_impl(s, q_t, v_t, f_ext, q0, q_next, v_next, q_star_m1, force_iters, m_override, rec_max, rec,
                           istats, dstats, NULL);
}

int or_step_forward_contact(const or_scene* s, const double* q_t, const double* v_t, const double* f_ext,
                            const double* q0, double* q_next, double* v_next, double* q_star_m1, int K,
                            const int* cv, const double* cn, const double* cg, double fb_tol, double* lambda,
                            int* istats, double* dstats) {
  or_contacts con = {K, cv, cn, cg, fb_tol, lambda, NULL, NULL, 0.0, 0};
  int st = step_forward_impl(s, q_t, v_t, f_ext, q0, q_next, v_next, q_star_m1, 0, -1, 0, NULL, istats, dstats,
                             K > 0 ? &con : NULL);
  if (dstats) dstats[4] = con.fb_res;
  return st;
}

int or_step_forward_friction(const or_scene* s, const double* q_t, const double* v_t, const double* f_ext,
                             const double* q0, double* q_next, double* v_next, double* q_star_m1, int K,
                             const int* cv, const double* cn, const double* cg, double mu_f, double fb_tol,
                             double* lambda3, int force_iters, int* istats, double* dstats) {
  or_contacts con = {K, cv, cn, cg, fb_tol, lambda3, NULL, NULL, 0.0, 0, mu_f, q_t, NULL, NULL};
  int st = step_forward_impl(s, q_t, v_t, f_ext, q0, q_next, v_next, q_star_m1, force_iters, -1, 0, NULL, istats,
                             dstats, K > 0 ? &con : NULL);
  if (dstats) { dstats[4] = con.fb_res; dstats[5] = con.fb_iters; }
  return st;
}

/* The contact step with bilateral rows and restitution: kind (K, 1 =
 * bilateral, may be NULL), rest_on / e_rest, friction mu_f (0: frictionless;
 * bilateral rows need mu_f = 0), impulses lambda (K, or 3K with friction). */
int or_step_forward_contact_ext(const or_scene* s, const double* q_t, const double* v_t, const double* f_ext,
                                const double* q0, double* q_next, double* v_next, double* q_star_m1, int K,
                                const int* cv, const double* cn, const double* cg, const unsigned char* kind,
                                int rest_on, double e_rest, double mu_f, double fb_tol, double* lambda,
                                int force_iters, int* istats, double* dstats) {
  or_contacts con = {K, cv, cn, cg, fb_tol, lambda, NULL, NULL, 0.0, 0, mu_f, q_t, NULL, NULL,
                     kind, rest_on, e_rest, NULL};
  int st = step_forward_impl(s, q_t, v_t, f_ext, q0, q_next, v_next, q_star_m1, force_iters, -1, 0, NULL, istats,
                             dstats, K > 0 ? &con : NULL);
  if (dstats) { dstats[4] = con.fb_res; dstats[5] = con.fb_iters; }
  return st;
}

/* dense LU with partial pivoting, in place; solves A x = b (n small) */
static int dense_lu_solve(double* A, int n, double* b) {
  for (int k = 0; k < n; ++k) {
    int p = k;
    for (int i = k + 1; i < n; ++i) if (fabs(A[(size_t)i * n + k]) > fabs(A[(size_t)p * n + k])) p = i;
    if (A[(size_t)p * n + k] == 0.0) return 0;
    if (p != k) {
      for (int j = 0; j < n; ++j) { double t = A[(size_t)k * n + j]; A[(size_t)k * n + j] = A[(size_t)p * n + j]; A[(size_t)p * n + j] = t; }
      double t = b[k]; b[k] = b[p]; b[p] = t;
    }
    for (int i = k + 1; i < n; ++i) {
      double f = A[(size_t)i * n + k] / A[(size_t)k * n + k];
      if (f == 0.0) continue;
      for (int j = k; j < n; ++j) A[(size_t)i * n + j] -= f * A[(size_t)k * n + j];
      b[i] -= f * b[k];
    }
  }
  for (int i = n - 1; i >= 0; --i) {
    double sum = b[i];
    for (int j = i + 1; j < n; ++j) sum -= A[(size_t)i * n + j] * b[j];
    b[i] = sum / A[(size_t)i * n + i];
  }
  return 1;
}

/* LU with partial pivoting in place (n x n, row-major) and its solve */
static int lu_factor(double* A, int n, int* piv) {
  for (int k = 0; k < n; ++k) {
    int p = k;
    for (int i = k + 1; i < n; ++i) if (fabs(A[(size_t)i * n + k]) > fabs(A[(size_t)p * n + k])) p = i;
    piv[k] = p;
    if (A[(size_t)p * n + k] == 0.0) return 0;
    if (p != k)
      for (int j = 0; j < n; ++j) { double t = A[(size_t)k * n + j]; A[(size_t)k * n + j] = A[(size_t)p * n + j]; A[(size_t)p * n + j] = t; }
    for (int i = k + 1; i < n; ++i) {
      double f = A[(size_t)i * n + k] / A[(size_t)k * n + k];
      A[(size_t)i * n + k] = f;
      for (int j = k + 1; j < n; ++j) A[(size_t)i * n + j] -= f * A[(size_t)k * n + j];
    }
  }
  return 1;
}

static void lu_solve(const double* A, int n, const int* piv, double* b) {
  for (int k = 0; k < n; ++k) {
    if (piv[k] != k) { double t = b[k]; b[k] = b[piv[k]]; b[piv[k]] = t; }
    for (int i = k + 1; i < n; ++i) b[i] -= A[(size_t)i * n + k] * b[k];
  }
  for (int i = n - 1; i >= 0; --i) {
    double sum = b[i];
    for (int j = i + 1; j < n; ++j) sum -= A[(size_t)i * n + j] * b[j];
    b[i] = sum / A[(size_t)i * n + i];
  }
}

/* Adjoint rows of the frictional contact set at a converged step.  READING
 * (Sec. 4.8 with the active set fixed, friction): with lambda_max the largest
 * normal impulse, contact c is active if lambda_n > 1e-10 lambda_max (else it
 * is dropped).  An active contact slides if |s| / w_c > 1e-8 mu lambda_n (s =
 * T^T (q* - q_t) at its vertex, w_c its diagonal of A~^{-1}), else it sticks.
 * Linearising the step's equations A q - b(q) - c - sum_c (impulse of c) = 0,
 * n.q = g (active), T^T (q - q_t) = 0 (stick), lambda_f = -mu lambda_n s^
 * (slide) gives the forward system [H, -B^T; C, 0] with H = A - K + D,
 * D = sum_slide (mu lambda_n / |s|) p p^T on the contact vertex (p the unit
 * tangent perpendicular to the slip), C the constraint rows (n; t1, t2 of
 * sticking contacts) and B the rows along which the multipliers act: n, or
 * n - mu s^_w for a sliding contact (the friction force follows lambda_n).
 * The adjoint therefore solves H mu + C^T nu = qbar, B mu = 0; the sticking
 * rows and D also route dL/dq_t += t nu (stick) + D mu (slide).  The fixed-point
 * form adds one row per sliding contact along p with diagonal |s|/(mu
 * lambda_n), which carries D mu = p eta. */
typedef struct fr_rows {
  int n;
  int* vert;
  int* kind;     /* 0 normal, 1 stick tangent, 2 slide perpendicular */
  double* b;     /* 3 per row */
  double* c;     /* 3 per row */
  double* d;     /* diagonal */
  double* dmat;  /* slide: the 3x3 D of the row's contact (kind 2 rows) */
} fr_rows;

static void fr_rows_build(const or_scene* s, const or_contacts* con, const double* q_star, const double* q_t,
                          fr_rows* R) {
  int K = con->K;
  R->n = 0;
  R->vert = (int*)malloc(sizeof(int) * 3 * (size_t)(K > 0 ? K : 1));
  R->kind = (int*)malloc(sizeof(int) * 3 * (size_t)(K > 0 ? K : 1));
  R->b = (double*)malloc(sizeof(double) * 9 * (size_t)(K > 0 ? K : 1));
  R->c = (double*)malloc(sizeof(double) * 9 * (size_t)(K > 0 ? K : 1));
  R->d = (double*)malloc(sizeof(double) * 3 * (size_t)(K > 0 ? K : 1));
  R->dmat = (double*)calloc(27 * (size_t)(K > 0 ? K : 1), sizeof(double));
  double lmax = 0.0;
  for (int c = 0; c < K; ++c) lmax = con->lambda[3 * c] > lmax ? con->lambda[3 * c] : lmax;
  for (int c = 0; c < K; ++c) {
    double ln = con->lambda[3 * c];
    if (!(lmax > 0.0 && ln > 1e-10 * lmax)) continue;
    int v = con->v[c];
    const double* e = con->e + 9 * c;
    double w = con->G[(size_t)c * K + c];
    double sl[2];
    for (int a = 0; a < 2; ++a) {
      const double* t = e + 3 * (a + 1);
      sl[a] = t[0] * (q_star[3 * v] - q_t[3 * v]) + t[1] * (q_star[3 * v + 1] - q_t[3 * v + 1]) +
              t[2] * (q_star[3 * v + 2] - q_t[3 * v + 2]);
    }
    double ns = sqrt(sl[0] * sl[0] + sl[1] * sl[1]);
    double tau = con->mu_f * ln;
    int r = R->n++;
    R->vert[r] = v;
    R->kind[r] = 0;
    R->d[r] = 0.0;
    for (int i = 0; i < 3; ++i) { R->b[3 * r + i] = e[i]; R->c[3 * r + i] = e[i]; }
    if (ns / w > 1e-8 * tau) {
      double h1 = sl[0] / ns, h2 = sl[1] / ns, sw[3], p[3];
      for (int i = 0; i < 3; ++i) {
        sw[i] = h1 * e[3 + i] + h2 * e[6 + i];
        p[i] = -h2 * e[3 + i] + h1 * e[6 + i];
        R->b[3 * r + i] = e[i] - con->mu_f * sw[i];
      }
      int r2 = R->n++;
      R->vert[r2] = v;
      R->kind[r2] = 2;
      R->d[r2] = ns / tau;
      for (int i = 0; i < 3; ++i) { R->b[3 * r2 + i] = p[i]; R->c[3 * r2 + i] = p[i]; }
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) R->dmat[9 * r2 + 3 * i + j] = tau / ns * p[i] * p[j];
    } else {
      for (int a = 1; a < 3; ++a) {
        int r2 = R->n++;
        R->vert[r2] = v;
        R->kind[r2] = 1;
        R->d[r2] = 0.0;
        for (int i = 0; i < 3; ++i) { R->b[3 * r2 + i] = e[3 * a + i]; R->c[3 * r2 + i] = e[3 * a + i]; }
      }
    }
  }
}

static void fr_rows_free(fr_rows* R) {
  free(R->vert); free(R->kind); free(R->b); free(R->c); free(R->d); free(R->dmat);
}

/* the frictional adjoint: mu (over all vertices) and the extra dL/dq_t of the
 * sticking and sliding contacts; adj_mode 1 = dense system, 0 = projected
 * fixed point; returns the status and writes the iterations */
static int fr_adjoint(const or_scene* s, const or_contacts* con, const double* kst, const double* qbar,
                      const double* q_star, const double* q_t, int adj_mode, double* mu, double* gqt_extra,
                      int* iters_out) {
  int nv = s->nv, n3 = 3 * nv, K = con->K;
  fr_rows R;
  fr_rows_build(s, con, q_star, q_t, &R);
  int status = 0, iters = 0;
  /* column of A~^{-1} for the contact vertex v: that of the first contact on v */
  int* colof = (int*)malloc(sizeof(int) * (R.n > 0 ? R.n : 1));
  for (int r = 0; r < R.n; ++r) {
    colof[r] = -1;
    for (int c = 0; c < K; ++c) if (con->v[c] == R.vert[r]) { colof[r] = c; break; }
  }
  for (int i = 0; i < n3; ++i) gqt_extra[i] = 0.0;
  if (adj_mode == 1) {
    /* [H, C^T; B, 0] [mu; nu] = [qbar; 0] over free coordinates and the
     * normal and sticking rows (D explicit in H) */
    int nf = s->nf;
    int* rr = (int*)malloc(sizeof(int) * (R.n > 0 ? R.n : 1));
    int nr = 0;
    for (int r = 0; r < R.n; ++r) if (R.kind[r] != 2) rr[nr++] = r;
    int N = 3 * nf + nr;
    double* Mat = (double*)calloc((size_t)N * N, sizeof(double));
    double* col = (double*)calloc(n3, sizeof(double));
    double* Ac = (double*)malloc(sizeof(double) * n3);
    double* Kc = (double*)malloc(sizeof(double) * n3);
    for (int j = 0; j < 3 * nf; ++j) {
      int vj = s->fvert[j / 3], aj = j % 3;
      col[3 * vj + aj] = 1.0;
      or_apply_A(s, col, Ac);
      apply_K_stored(s, kst, col, Kc);
      col[3 * vj + aj] = 0.0;
      for (int i = 0; i < 3 * nf; ++i) {
        int vi = s->fvert[i / 3], ai = i % 3;
        Mat[(size_t)i * N + j] = Ac[3 * vi + ai] - Kc[3 * vi + ai];
      }
    }
    for (int r = 0; r < R.n; ++r) {
      if (R.kind[r] != 2) continue;
      int fi = s->fidx[R.vert[r]];
      for (int a = 0; a < 3; ++a)
        for (int b2 = 0; b2 < 3; ++b2) Mat[(size_t)(3 * fi + a) * N + 3 * fi + b2] += R.dmat[9 * r + 3 * a + b2];
    }
    for (int k = 0; k < nr; ++k) {
      int r = rr[k], fi = s->fidx[R.vert[r]];
      for (int ax = 0; ax < 3; ++ax) {
        Mat[(size_t)(3 * fi + ax) * N + 3 * nf + k] = R.c[3 * r + ax];
        Mat[(size_t)(3 * nf + k) * N + 3 * fi + ax] = R.b[3 * r + ax];
      }
    }
    double* rhs = (double*)calloc(N, sizeof(double));
    for (int i = 0; i < 3 * nf; ++i) rhs[i] = qbar[3 * s->fvert[i / 3] + i % 3];
    if (!dense_lu_solve(Mat, N, rhs)) status = -1;
    for (int i = 0; i < 3 * nf; ++i) mu[3 * s->fvert[i / 3] + i % 3] = rhs[i];
    for (int k = 0; k < nr; ++k) {
      int r = rr[k];
      if (R.kind[r] != 1) continue;
      for (int ax = 0; ax < 3; ++ax) gqt_extra[3 * R.vert[r] + ax] += R.c[3 * r + ax] * rhs[3 * nf + k];
    }
    for (int r = 0; r < R.n; ++r) {
      if (R.kind[r] != 2) continue;
      int v = R.vert[r];
      for (int a = 0; a < 3; ++a)
        for (int b2 = 0; b2 < 3; ++b2) gqt_extra[3 * v + a] += R.dmat[9 * r + 3 * a + b2] * mu[3 * v + b2];
    }
    free(Mat); free(col); free(Ac); free(Kc); free(rhs); free(rr);
  } else {
    /* projected fixed point mu <- x - sum_r a_{v_r} c_r nu_r, x = A^-1 (qbar + K mu),
     * (B A^-1 C^T + diag(d)) nu = B x */
    int nr = R.n;
    double* Mf = (double*)malloc(sizeof(double) * (size_t)(nr > 0 ? nr : 1) * (nr > 0 ? nr : 1));
    int* piv = (int*)malloc(sizeof(int) * (nr > 0 ? nr : 1));
    for (int r = 0; r < nr; ++r)
      for (int q2 = 0; q2 < nr; ++q2) {
        const double* br = R.b + 3 * r;
        const double* cq = R.c + 3 * q2;
        double g = con->col[(size_t)colof[r] * nv + R.vert[q2]];
        Mf[(size_t)r * nr + q2] = (br[0] * cq[0] + br[1] * cq[1] + br[2] * cq[2]) * g + (r == q2 ? R.d[r] : 0.0);
      }
    if (nr > 0 && !lu_factor(Mf, nr, piv)) status = -1;
    double* t = (double*)malloc(sizeof(double) * n3);
    double* mun = (double*)malloc(sizeof(double) * n3);
    double* nu = (double*)calloc(nr > 0 ? nr : 1, sizeof(double));
    if (status == 0) {
      status = 1;
      for (iters = 1; iters <= s->kmax_bwd; ++iters) {
        apply_K_stored(s, kst, mu, t);
        for (int i = 0; i < n3; ++i) t[i] += qbar[i];
        or_apply_Ainv(s, t, mun);
        for (int r = 0; r < nr; ++r) {
          const double* z = mun + 3 * R.vert[r];
          nu[r] = R.b[3 * r] * z[0] + R.b[3 * r + 1] * z[1] + R.b[3 * r + 2] * z[2];
        }
        if (nr > 0) lu_solve(Mf, nr, piv, nu);
        for (int r = 0; r < nr; ++r) {
          const double* a = con->col + (size_t)colof[r] * nv;
          for (int i = 0; i < nv; ++i) {
            if (s->fidx[i] < 0) continue;
            for (int ax = 0; ax < 3; ++ax) mun[3 * i + ax] -= nu[r] * a[i] * R.c[3 * r + ax];
          }
        }
        double d = 0, nrm = 0;
        for (int i = 0; i < n3; ++i) {
          d += (mun[i] - mu[i]) * (mun[i] - mu[i]);
          nrm += mun[i] * mun[i];
        }
        memcpy(mu, mun, sizeof(double) * n3);
        if (sqrt(d) <= s->eps_adj * sqrt(nrm)) { status = 0; break; }
      }
      if (iters > s->kmax_bwd) iters = s->kmax_bwd;
      for (int r = 0; r < nr; ++r) {
        if (R.kind[r] == 0) continue;
        for (int ax = 0; ax < 3; ++ax) gqt_extra[3 * R.vert[r] + ax] += R.c[3 * r + ax] * nu[r];
      }
    }
    free(Mf); free(piv); free(t); free(mun); free(nu);
  }
  free(colof);
  fr_rows_free(&R);
  *iters_out = iters;
  return status;
}

/* ------------------------------------------------------------------------ */
/* backward step, Alg. 2 (no contact)                                        */
/* ------------------------------------------------------------------------ */
static int step_backward_impl(const or_scene* s, const double* q_t, const double* v_t, const double* f_ext,
                              const double* q_star, const double* q_star_m1, const double* gq_next,
                              const double* gv_next, double* gq_t, double* gv_t, double* gf_ext, double* g_logE,
                              int adj_mode, double tau_force, int* istats, double* dstats, or_contacts* con) {
  int nv = s->nv, n3 = 3 * nv;
  double h = s->h;
  double* qbar = (double*)malloc(sizeof(double) * n3);
  double* qtilde = (double*)malloc(sizeof(double) * n3);
  double* c = (double*)malloc(sizeof(double) * n3);
  double* dq = (double*)malloc(sizeof(double) * n3);
  double* Adq = (double*)malloc(sizeof(double) * n3);
  /* the restitution post-correction's adjoint, rows in reverse order: the
   * raw velocity (q* - q_t)/h keeps (I - n n^T) of the incoming v^bar and
   * v_t receives -e n (n . v^bar) */
  double* vbar = (double*)malloc(sizeof(double) * n3);
  double* gvt_rest = (double*)calloc(n3, sizeof(double));
  memcpy(vbar, gv_next, sizeof(double) * n3);
  if (con && con->rest_on && con->K > 0) {
    int* rows = (int*)malloc(sizeof(int) * con->K);
    int nr = restitution_rows(con, v_t, rows);
    for (int r = nr - 1; r >= 0; --r) {
      int c = rows[r], vx = con->v[c];
      const double* nc = con->n + 3 * c;
      double* vb = vbar + 3 * vx;
      double d = nc[0] * vb[0] + nc[1] * vb[1] + nc[2] * vb[2];
      for (int ax = 0; ax < 3; ++ax) {
        gvt_rest[3 * vx + ax] += -con->e_rest * nc[ax] * d;
        vb[ax] -= nc[ax] * d;
      }
    }
    free(rows);
  }
  /* q^bar = q^bar_{t+h} + v^bar_{t+h} / h on free vertices (Alg. 2) */
  for (int v = 0; v < nv; ++v)
    for (int ax = 0; ax < 3; ++ax) {
      int i = 3 * v + ax;
      qbar[i] = s->fidx[v] >= 0 ? gq_next[i] + vbar[i] / h : 0.0;
    }
  or_const_rhs(s, q_t, v_t, f_ext, c, qtilde);
  /* trust-region ratio on the last fixed-point increment, Eqs. tr_step,
   * tr_decreases, tr_ratio, tr_rule.  READING: Phi(q*-1) - Phi(q*) is summed as
   * per-vertex and per-element differences (the same sum, regrouped). */
  double dphi_act = 0.0, dphi_mod = 0.0, rho = 1.0, tau = 0.0;
  if (s->energy == 0) { /* Alg. 2: the ratio and its filter belong to the Neo-Hookean prox */
  for (int v = 0; v < nv; ++v)
    for (int ax = 0; ax < 3; ++ax) {
      int i = 3 * v + ax;
      double a = q_star_m1[i], b = q_star[i];
      dphi_act += 0.5 / (h * h) * s->mass[v] * (a - b) * (a + b - 2.0 * qtilde[i]);
    }
  double* pe = (double*)malloc(sizeof(double) * (s->ne > 0 ? s->ne : 1));
#pragma omp parallel for schedule(static)
  for (int e = 0; e < s->ne; ++e) {
    double Fa[9], Fb[9];
    element_F(s, e, q_star_m1, Fa);
    element_F(s, e, q_star, Fb);
    double pa = or_psi_nh(Fa, s->mu[e], s->lam[e]), pb = or_psi_nh(Fb, s->mu[e], s->lam[e]);
    pe[e] = s->vol[e] * (pa - pb) + (muscle_energy(s, e, Fa) - muscle_energy(s, e, Fb));
  }
  for (int e = 0; e < s->ne; ++e) dphi_act += pe[e];
  free(pe);
  for (int v = 0; v < nv; ++v)
    for (int ax = 0; ax < 3; ++ax) dq[3 * v + ax] = s->fidx[v] >= 0 ? q_star[3 * v + ax] - q_star_m1[3 * v + ax] : 0.0;
  or_apply_A(s, dq, Adq);
  dphi_mod = 0.5 * fabs(dot_free(s, dq, Adq));
  rho = dphi_mod < 1e-12 ? 1.0 : dphi_act / dphi_mod;
  tau = fabs(rho - 1.0) <= s->eps_tr ? 0.5 : 1.0;
  if (tau_force >= 0.0) tau = tau_force;
  }
  /* adjoint: (A - K) mu = q^bar (Eqs. adjoint_system, Rqq, db_dq with the
   * filtered prox differential; A, K symmetric).  READING: solved to
   * tolerance, by the fixed-point iteration mu <- A^-1 (q^bar + K mu), or, for
   * small meshes, by a dense direct solve. */
  double* mu = (double*)calloc(n3, sizeof(double));
  double* kst = prox_diff_all(s, q_star, tau);
  int iters = 0, status = 0;
  /* READING (contact adjoint, frictionless): the active set {c: lambda_c >
   * 1e-10 max lambda} is held fixed; active rows are equalities J_A dq = 0, so
   * (A - K) mu - J_A^T nu = q^bar, J_A mu = 0. */
  int na = 0;
  int* act = NULL;
  double* WA = NULL;
  double* gqt_fr = NULL;
  if (con && con->K > 0 && con->mu_f > 0.0) {
    contact_setup(s, con);
    gqt_fr = (double*)malloc(sizeof(double) * n3);
    status = fr_adjoint(s, con, kst, qbar, q_star, q_t, adj_mode, mu, gqt_fr, &iters);
  } else if (con && con->K > 0) {
    contact_setup(s, con);
    act = (int*)malloc(sizeof(int) * con->K);
    for (int c = 0; c < con->K; ++c)
      if (row_active(con, c)) act[na++] = c;
    WA = (double*)malloc(sizeof(double) * (size_t)(na > 0 ? na : 1) * (na > 0 ? na : 1));
    if (con->g_gap) for (int c = 0; c < con->K; ++c) con->g_gap[c] = 0.0;
  }
  if (gqt_fr) {
    /* solved above */
  } else if (na > 0 && adj_mode == 1) {
    /* dense saddle-point system */
    int nf = s->nf, N = 3 * nf + na;
    double* Mat = (double*)calloc((size_t)N * N, sizeof(double));
    double* col = (double*)calloc(n3, sizeof(double));
    double* Ac = (double*)malloc(sizeof(double) * n3);
    double* Kc = (double*)malloc(sizeof(double) * n3);
    for (int j = 0; j < 3 * nf; ++j) {
      int vj = s->fvert[j / 3], aj = j % 3;
      col[3 * vj + aj] = 1.0;
      or_apply_A(s, col, Ac);
      apply_K_stored(s, kst, col, Kc);
      col[3 * vj + aj] = 0.0;
      for (int i = 0; i < 3 * nf; ++i) {
        int vi = s->fvert[i / 3], ai = i % 3;
        Mat[(size_t)i * N + j] = Ac[3 * vi + ai] - Kc[3 * vi + ai];
      }
    }
    for (int a = 0; a < na; ++a) {
      int c = act[a], v = con->v[c];
      int fi = s->fidx[v];
      for (int ax = 0; ax < 3; ++ax) {
        int j = 3 * fi + ax;
        Mat[(size_t)j * N + 3 * nf + a] = -con->n[3 * c + ax];
        Mat[(size_t)(3 * nf + a) * N + j] = -con->n[3 * c + ax];
      }
    }
    double* rhs = (double*)calloc(N, sizeof(double));
    for (int i = 0; i < 3 * nf; ++i) rhs[i] = qbar[3 * s->fvert[i / 3] + i % 3];
    if (!dense_lu_solve(Mat, N, rhs)) status = -1;
    for (int i = 0; i < 3 * nf; ++i) mu[3 * s->fvert[i / 3] + i % 3] = rhs[i];
    /* dL/dg_c = -nu_c: the constraint n.q = g enters as J dq = dg */
    if (con->g_gap) for (int a = 0; a < na; ++a) con->g_gap[act[a]] = -rhs[3 * nf + a];
    free(Mat); free(col); free(Ac); free(Kc); free(rhs);
  } else if (na > 0) {
    /* projected fixed point mu <- P (q^bar + K mu), P = A^-1 - A^-1 J_A^T W_AA^-1 J_A A^-1 */
    double* t = (double*)malloc(sizeof(double) * n3);
    double* mun = (double*)malloc(sizeof(double) * n3);
    double* u = (double*)malloc(sizeof(double) * na);
    status = 1;
    for (iters = 1; iters <= s->kmax_bwd; ++iters) {
      apply_K_stored(s, kst, mu, t);
      for (int i = 0; i < n3; ++i) t[i] += qbar[i];
      or_apply_Ainv(s, t, mun);
      for (int a = 0; a < na; ++a) {
        int c = act[a];
        const double* z = mun + 3 * con->v[c];
        u[a] = con->n[3 * c] * z[0] + con->n[3 * c + 1] * z[1] + con->n[3 * c + 2] * z[2];
        for (int b2 = 0; b2 < na; ++b2) WA[(size_t)a * na + b2] = con->W[(size_t)c * con->K + act[b2]];
      }
      if (!chol_solve(WA, na, u)) { status = -1; break; }
      for (int a = 0; a < na; ++a) {
        int c = act[a];
        const double* col = con->col + (size_t)c * nv;
        for (int i = 0; i < nv; ++i) {
          if (s->fidx[i] < 0) continue;
          for (int ax = 0; ax < 3; ++ax) mun[3 * i + ax] -= u[a] * col[i] * con->n[3 * c + ax];
        }
      }
      double d = 0, nrm = 0;
      for (int i = 0; i < n3; ++i) {
        d += (mun[i] - mu[i]) * (mun[i] - mu[i]);
        nrm += mun[i] * mun[i];
      }
      memcpy(mu, mun, sizeof(double) * n3);
      /* the multipliers of the projection are -nu: dL/dg = u */
      if (con->g_gap) for (int a = 0; a < na; ++a) con->g_gap[act[a]] = u[a];
      if (sqrt(d) <= s->eps_adj * sqrt(nrm)) { status = 0; break; }
    }
    if (iters > s->kmax_bwd) iters = s->kmax_bwd;
    free(t); free(mun); free(u);
  } else if (adj_mode == 1) {
    int nf = s->nf, N = 3 * nf;
    double* Mat = (double*)malloc(sizeof(double) * (size_t)N * N);
    double* col = (double*)calloc(n3, sizeof(double));
    double* Ac = (double*)malloc(sizeof(double) * n3);
    double* Kc = (double*)malloc(sizeof(double) * n3);
    for (int j = 0; j < N; ++j) {
      int vj = s->fvert[j / 3], aj = j % 3;
      col[3 * vj + aj] = 1.0;
      or_apply_A(s, col, Ac);
      apply_K_stored(s, kst, col, Kc);
      col[3 * vj + aj] = 0.0;
      for (int i = 0; i < N; ++i) {
        int vi = s->fvert[i / 3], ai = i % 3;
        Mat[(size_t)i * N + j] = Ac[3 * vi + ai] - Kc[3 * vi + ai];
      }
    }
    double* rhs = (double*)malloc(sizeof(double) * N);
    for (int i = 0; i < N; ++i) rhs[i] = qbar[3 * s->fvert[i / 3] + i % 3];
    if (!dense_lu_solve(Mat, N, rhs)) status = -1;
    for (int i = 0; i < N; ++i) mu[3 * s->fvert[i / 3] + i % 3] = rhs[i];
    free(Mat); free(col); free(Ac); free(Kc); free(rhs);
  } else {
    double* t = (double*)malloc(sizeof(double) * n3);
    double* mun = (double*)malloc(sizeof(double) * n3);
    status = 1;
    for (iters = 1; iters <= s->kmax_bwd; ++iters) {
      apply_K_stored(s, kst, mu, t);
      for (int i = 0; i < n3; ++i) t[i] += qbar[i];
      or_apply_Ainv(s, t, mun);
      double d = 0, nrm = 0;
      for (int i = 0; i < n3; ++i) {
        d += (mun[i] - mu[i]) * (mun[i] - mu[i]);
        nrm += mun[i] * mun[i];
      }
      memcpy(mu, mun, sizeof(double) * n3);
      if (sqrt(d) <= s->eps_adj * sqrt(nrm)) { status = 0; break; }
    }
    if (iters > s->kmax_bwd) iters = s->kmax_bwd;
    free(t); free(mun);
  }
  /* gradient routing (Eqs. dl_dq, dl_dv_dfext, dl_dwe).  READING: the
   * implicit-function theorem on A q - b(q) - c(theta) = 0 gives
   * dL/dq_t = (M/h^2 + alpha M/h + B_beta/h) mu - v^bar/h, dL/dv_t = M mu / h,
   * dL/df_ext = mu; per element dL/dw_e = V_e <G mu, p* - G q*> and
   * dL/dbeta_e = (V_e/h) <G mu, G (q_t - q*)>; w_e and beta_e scale with E_e,
   * the mesh means and mu_ref are held fixed. */
  double* Bmu = (double*)calloc(n3, sizeof(double));
  double* ge = (double*)malloc(sizeof(double) * (s->ne > 0 ? s->ne : 1));
  double* ctb = (double*)malloc(sizeof(double) * 12 * (size_t)(s->ne > 0 ? s->ne : 1));
#pragma omp parallel for schedule(static)
  for (int e = 0; e < s->ne; ++e) {
    double Gm[9], F[9], Fd[9], P[9], U[9], V[9], sF[3], ss[3], T[9];
    double qd[12];
    element_F(s, e, mu, Gm);
    element_F(s, e, q_star, F);
    double gw = 0.0;
    if (s->energy >= 1) {
      /* dL/dlog E_e = 2 mu_e V_e <G mu, R - F> + lam_e V_e <G mu, P_vol - F> + the beta term */
      composite_parts c;
      composite_eval_s(s, F, &c, 0);
      double gr = 0.0, gv = 0.0;
      for (int i = 0; i < 9; ++i) {
        gr += Gm[i] * (c.R[i] - F[i]);
        gv += Gm[i] * (c.Pv[i] - F[i]);
      }
      gw = (2.0 * s->mu[e] * gr + s->lam[e] * gv) * s->vol[e];
    } else {
    or_svd3(F, U, sF, V);
    or_prox_stretch(sF, s->mu_bar, s->lam_bar, s->k_bar, ss);
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) T[3 * i + j] = U[3 * i + j] * ss[j];
    mat3_mul_nt(T, V, P);
    for (int i = 0; i < 9; ++i) gw += Gm[i] * (P[i] - F[i]);
    gw *= s->vol[e];
    gw = s->w[e] * gw;
    }
    /* G (q_t - q*) */
    for (int i = 0; i < 9; ++i) Fd[i] = 0.0;
    for (int a = 0; a < 4; ++a) {
      int v = s->tets[4 * e + a];
      for (int ax = 0; ax < 3; ++ax) qd[3 * a + ax] = q_t[3 * v + ax] - q_star[3 * v + ax];
      if (s->pinned[v]) for (int ax = 0; ax < 3; ++ax) qd[3 * a + ax] = 0.0;
      const double* B = s->Bhat + 12 * e + 3 * a;
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Fd[3 * i + j] += qd[3 * a + i] * B[j];
    }
    double gb = 0.0;
    for (int i = 0; i < 9; ++i) gb += Gm[i] * Fd[i];
    gb *= s->vol[e] / h;
    ge[e] = gw + s->beta[e] * gb;
    /* B_beta mu = sum_e beta_e V_e G^T G mu */
    element_contrib(s, e, s->beta[e] * s->vol[e], Gm, ctb + 12 * (size_t)e);
  }
  for (int e = 0; e < s->ne; ++e) g_logE[e] += ge[e];
  /* dL/da_g = mu^T db/da_g = -sum_{e in g} w_m V_e <G_m mu, f^> at q* (element order) */
  if (s->mgroup && s->g_act) {
#pragma omp parallel for schedule(static)
    for (int e = 0; e < s->ne; ++e) {
      double Gm[9], F[9], f[3], nf, ell, y[3];
      ge[e] = 0.0;
      element_F(s, e, q_star, F);
      if (!muscle_eval(s, e, F, f, &nf, &ell) || !(nf > 0.0)) continue;
      element_F(s, e, mu, Gm);
      const double* m = s->mfib + 3 * e;
      for (int i = 0; i < 3; ++i) y[i] = Gm[3 * i] * m[0] + Gm[3 * i + 1] * m[1] + Gm[3 * i + 2] * m[2];
      ge[e] = -s->w_m * s->vol[e] * (y[0] * f[0] + y[1] * f[1] + y[2] * f[2]) / nf;
    }
    for (int e = 0; e < s->ne; ++e)
      if (s->mgroup[e] >= 0) s->g_act[s->mgroup[e]] += ge[e];
  }
  scatter_contribs(s, ctb, Bmu);
  free(ge);
  free(ctb);
  for (int v = 0; v < nv; ++v)
    for (int ax = 0; ax < 3; ++ax) {
      int i = 3 * v + ax;
      if (s->fidx[v] < 0) { gq_t[i] = 0; gv_t[i] = 0; gf_ext[i] = 0; continue; }
      double m = s->mass[v];
      gq_t[i] = (m / (h * h) + s->alpha * m / h) * mu[i] + Bmu[i] / h - vbar[i] / h;
      if (gqt_fr) gq_t[i] += gqt_fr[i];
      gv_t[i] = m / h * mu[i] + gvt_rest[i];
      gf_ext[i] = mu[i];
    }
  if (istats) { istats[0] = iters; istats[1] = status; }
  if (dstats) { dstats[0] = rho; dstats[1] = tau; dstats[2] = dphi_act; dstats[3] = dphi_mod; }
  if (con && con->K > 0) contact_free(con);
  free(act); free(WA); free(gqt_fr); free(vbar); free(gvt_rest);
  free(qbar); free(qtilde); free(c); free(dq); free(Adq); free(mu); free(Bmu); free(kst);
  return status;
}

int or_step_backward(const or_scene* s, const double* q_t, const double* v_t, const double* f_ext,
                     const double* q_star, const double* q_star_m1, const double* gq_next, const double* gv_next,
                     double* gq_t, double* gv_t, double* gf_ext, double* g_logE, int adj_mode, double tau_force,
                     int* istats, double* dstats) {
  return step_backward_impl(s, q_t, v_t, f_ext, q_star, q_star_m1, gq_next, gv_next, gq_t, gv_t, gf_ext, g_logE,
                            adj_mode, tau_force, istats, dstats, NULL);
}

int or_step_backward_contact(const or_scene* s, const double* q_t, const double* v_t, const double* f_ext,
                             const double* q_star, const double* q_star_m1, const double* gq_next,
                             const double* gv_next, double* gq_t, double* gv_t, double* gf_ext, double* g_logE,
                             int adj_mode, double tau_force, int K, const int* cv, const double* cn,
                             const double* cg, const double* lambda, int* istats, double* dstats) {
  double* lam = (double*)malloc(sizeof(double) * (K > 0 ? K : 1));
  for (int c = 0; c < K; ++c) lam[c] = lambda[c];
  or_contacts con = {K, cv, cn, cg, 0.0, lam, NULL, NULL, 0.0, 0};
  int st = step_backward_impl(s, q_t, v_t, f_ext, q_star, q_star_m1, gq_next, gv_next, gq_t, gv_t, gf_ext, g_logE,
                              adj_mode, tau_force, istats, dstats, K > 0 ? &con : NULL);
  free(lam);
  return st;
}

int or_step_backward_friction(const or_scene* s, const double* q_t, const double* v_t, const double* f_ext,
                              const double* q_star, const double* q_star_m1, const double* gq_next,
                              const double* gv_next, double* gq_t, double* gv_t, double* gf_ext, double* g_logE,
                              int adj_mode, double tau_force, int K, const int* cv, const double* cn,
                              const double* cg, double mu_f, const double* lambda3, int* istats, double* dstats) {
  double* lam = (double*)malloc(sizeof(double) * 3 * (size_t)(K > 0 ? K : 1));
  for (int c = 0; c < 3 * K; ++c) lam[c] = lambda3[c];
  or_contacts con = {K, cv, cn, cg, 0.0, lam, NULL, NULL, 0.0, 0, mu_f, q_t, NULL, NULL};
  int st = step_backward_impl(s, q_t, v_t, f_ext, q_star, q_star_m1, gq_next, gv_next, gq_t, gv_t, gf_ext, g_logE,
                              adj_mode, tau_force, istats, dstats, K > 0 ? &con : NULL);
  free(lam);
  return st;
}

/* The backward of or_step_forward_contact_ext; g_gap (K, may be NULL; frictionless only) receives dL/dg_c
 * of each active row (0 for the others). */
int or_step_backward_contact_ext(const or_scene* s, const double* q_t, const double* v_t, const double* f_ext,
                                 const double* q_star, const double* q_star_m1, const double* gq_next,
                                 const double* gv_next, double* gq_t, double* gv_t, double* gf_ext, double* g_logE,
                                 int adj_mode, double tau_force, int K, const int* cv, const double* cn,
                                 const double* cg, const unsigned char* kind, int rest_on, double e_rest,
                                 double mu_f, const double* lambda, double* g_gap, int* istats, double* dstats) {
  size_t nl = (size_t)(mu_f > 0.0 ? 3 : 1) * (K > 0 ? K : 1);
  double* lam = (double*)malloc(sizeof(double) * nl);
  for (size_t c = 0; c < (size_t)(mu_f > 0.0 ? 3 : 1) * K; ++c) lam[c] = lambda[c];
  or_contacts con = {K, cv, cn, cg, 0.0, lam, NULL, NULL, 0.0, 0, mu_f, q_t, NULL, NULL,
                     kind, rest_on, e_rest, mu_f > 0.0 ? NULL : g_gap};
  int st = step_backward_impl(s, q_t, v_t, f_ext, q_star, q_star_m1, gq_next, gv_next, gq_t, gv_t, gf_ext, g_logE,
                              adj_mode, tau_force, istats, dstats, K > 0 ? &con : NULL);
  free(lam);
  return st;
}

/* Delassus operator of a contact set (for checks): W (K x K) */
void or_contact_W(const or_scene* s, int K, const int* cv, const double* cn, double* W_out) {
  double lam0 = 0.0;
  or_contacts con = {K, cv, cn, NULL, 0.0, &lam0, NULL, NULL, 0.0, 0};
  contact_setup(s, &con);
  memcpy(W_out, con.W, sizeof(double) * (size_t)K * K);
  contact_free(&con);
}
