// Host runtime of the pdhot library: scene setup, the factorization into the
// two-level partitioned inverse, and the forward / backward step drivers that
// issue the HIP kernels.  Implements the C ABI declared in include/pdhot.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <stdexcept>
#include <string>
#include <thread>
#include <vector>

#include "../../include/pdhot.h"
#include "kernels.h"
#include "pd_internal.h"

using namespace pdhot;

struct pd_scene {
  Scene S;
};

namespace pdhot {
thread_local std::string g_last_error;
void set_last_error(const std::string& m) { g_last_error = m; }
}  // namespace pdhot

namespace {


struct PdError {
  int code;
  std::string msg;
};

#define PD_HIP(x)                                                                                   \
  do {                                                                                              \
    hipError_t e_ = (x);                                                                            \
    if (e_ != hipSuccess) throw PdError{PD_ERR_HIP, std::string(#x) + ": " + hipGetErrorString(e_)}; \
  } while (0)

template <class T>
T* dalloc(size_t n) {
  if (n == 0) n = 1;
  void* p = nullptr;
  PD_HIP(hipMalloc(&p, n * sizeof(T)));
  return static_cast<T*>(p);
}

template <class T>
void upload(T* d, const std::vector<T>& h) {
  if (!h.empty()) PD_HIP(hipMemcpy(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
}

template <class T>
void dfree(T*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

// ---------------------------------------------------------------- dense SPD
// In-place inverse of a symmetric positive definite matrix (row-major, full):
// A = L L^T, W = L^{-1}, A^{-1} = W^T W.  Returns false if A is not SPD.
bool spd_inverse(std::vector<double>& A, int n) {
  std::vector<double> L(A);
  for (int j = 0; j < n; ++j) {
    double* Lj = &L[(size_t)j * n];
    double d = Lj[j];
    for (int k = 0; k < j; ++k) d -= Lj[k] * Lj[k];
    if (!(d > 0.0) || !std::isfinite(d)) return false;
    d = std::sqrt(d);
    Lj[j] = d;
    const double inv = 1.0 / d;
    for (int i = j + 1; i < n; ++i) {
      double* Li = &L[(size_t)i * n];
      double s = Li[j];
      for (int k = 0; k < j; ++k) s -= Li[k] * Lj[k];
      Li[j] = s * inv;
    }
  }
  std::vector<double> W((size_t)n * n, 0.0), acc(n);
  for (int i = 0; i < n; ++i) {
    const double* Li = &L[(size_t)i * n];
    std::fill(acc.begin(), acc.begin() + i, 0.0);
    for (int k = 0; k < i; ++k) {
      const double c = Li[k];
      const double* Wk = &W[(size_t)k * n];
      for (int j = 0; j <= k; ++j) acc[j] += c * Wk[j];
    }
    const double inv = 1.0 / Li[i];
    double* Wi = &W[(size_t)i * n];
    for (int j = 0; j < i; ++j) Wi[j] = -acc[j] * inv;
    Wi[i] = inv;
  }
  std::fill(A.begin(), A.end(), 0.0);
  for (int k = 0; k < n; ++k) {
    const double* Wk = &W[(size_t)k * n];
    for (int i = 0; i <= k; ++i) {
      const double c = Wk[i];
      if (c == 0.0) continue;
      double* Ai = &A[(size_t)i * n];
      for (int j = 0; j <= i; ++j) Ai[j] += c * Wk[j];
    }
  }
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) A[(size_t)i * n + j] = A[(size_t)j * n + i];
  return true;
}

// Host threads for the factorization: fn(t) for t = 0 .. T-1 with static
// work splits inside fn, so results do not depend on scheduling.
int host_threads() {
  static const int n = [] {
    const unsigned hw = std::thread::hardware_concurrency();
    return (int)std::max(1u, std::min(hw, 16u));
  }();
  return n;
}

template <class F>
void run_threads(int T, const F& fn) {
  if (T <= 1) {
    fn(0);
    return;
  }
  std::vector<std::thread> th;
  th.reserve(T - 1);
  for (int t = 1; t < T; ++t) th.emplace_back([&fn, t] { fn(t); });
  fn(0);
  for (auto& x : th) x.join();
}

// Threaded inverse of a large SPD matrix (row-major, full): blocked
// right-looking Cholesky A = L L^T (panel rows and trailing rows split over
// threads), W = L^{-1} column by column, A^{-1} = W^T W row by row.
bool spd_inverse_threaded(std::vector<double>& A, int n) {
  const int T = host_threads();
  if (n < 512 || T == 1) return spd_inverse(A, n);
  constexpr int kB = 64;
  std::vector<double>& L = A;  // lower triangle in place
  bool ok = true;
  for (int k0 = 0; k0 < n && ok; k0 += kB) {
    const int k1 = std::min(k0 + kB, n);
    // diagonal block
    for (int j = k0; j < k1 && ok; ++j) {
      double* Lj = &L[(size_t)j * n];
      double d = Lj[j];
      for (int k = k0; k < j; ++k) d -= Lj[k] * Lj[k];
      if (!(d > 0.0) || !std::isfinite(d)) {
        ok = false;
        break;
      }
      d = std::sqrt(d);
      Lj[j] = d;
      for (int i = j + 1; i < k1; ++i) {
        double* Li = &L[(size_t)i * n];
        double sum = Li[j];
        for (int k = k0; k < j; ++k) sum -= Li[k] * Lj[k];
        Li[j] = sum / d;
      }
    }
    if (!ok) break;
    // panel rows below the block, then the trailing update, rows split over threads
    run_threads(T, [&](int t) {
      for (int i = k1 + t; i < n; i += T) {
        double* Li = &L[(size_t)i * n];
        for (int j = k0; j < k1; ++j) {
          const double* Lj = &L[(size_t)j * n];
          double sum = Li[j];
          for (int k = k0; k < j; ++k) sum -= Li[k] * Lj[k];
          Li[j] = sum / Lj[j];
        }
      }
    });
    run_threads(T, [&](int t) {
      for (int i = k1 + t; i < n; i += T) {
        double* Li = &L[(size_t)i * n];
        for (int j = k1; j <= i; ++j) {
          const double* Lj = &L[(size_t)j * n];
          double sum = 0.0;
          for (int k = k0; k < k1; ++k) sum += Li[k] * Lj[k];
          Li[j] -= sum;
        }
      }
    });
  }
  if (!ok) return false;
  // W = L^{-1}, stored by columns: Wc[j][i] = W_ij (i >= j)
  std::vector<double> Wc((size_t)n * n, 0.0);
  run_threads(T, [&](int t) {
    for (int j = t; j < n; j += T) {
      double* y = &Wc[(size_t)j * n];
      y[j] = 1.0 / L[(size_t)j * n + j];
      for (int i = j + 1; i < n; ++i) {
        const double* Li = &L[(size_t)i * n];
        double sum = 0.0;
        for (int k = j; k < i; ++k) sum += Li[k] * y[k];
        y[i] = -sum / Li[i];
      }
    }
  });
  // A^{-1}_ij = sum_{k >= max(i, j)} W_ki W_kj
  run_threads(T, [&](int t) {
    for (int i = t; i < n; i += T) {
      const double* wi = &Wc[(size_t)i * n];
      double* Ai = &A[(size_t)i * n];
      for (int j = 0; j <= i; ++j) {
        const double* wj = &Wc[(size_t)j * n];
        double sum = 0.0;
        for (int k = i; k < n; ++k) sum += wi[k] * wj[k];
        Ai[j] = sum;
      }
    }
  });
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) A[(size_t)i * n + j] = A[(size_t)j * n + i];
  return true;
}

double det3(const double* A) {
  return A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) + A[2] * (A[3] * A[7] - A[4] * A[6]);
}

void contact_free(Scene& S) {
  dfree(S.obs); dfree(S.c_v); dfree(S.c_slot); dfree(S.c_flags); dfree(S.c_n); dfree(S.c_g); dfree(S.c_lam);
  dfree(S.c_s); dfree(S.c_W); dfree(S.c_fb); dfree(S.a_v); dfree(S.a_slot); dfree(S.a_n); dfree(S.a_s);
  dfree(S.a_Winv); dfree(S.c_Lg); dfree(S.cols);
  dfree(S.c_frw); dfree(S.c_fri); dfree(S.a_nb); dfree(S.a_dg); dfree(S.c_slip); dfree(S.a_kind);
  dfree(S.c_kind); dfree(S.gv_rest); dfree(S.rest_s);
  S.mu_f = 0.0;
  S.c_kmax = 0;
  S.n_planes = S.n_boxes = 0;
  S.a_fric = false;
  if (S.h_cbuf) (void)hipHostFree(S.h_cbuf);
  if (S.h_crec) (void)hipHostFree(S.h_crec);
  S.h_cbuf = nullptr;
  S.h_crec = nullptr;
  S.contact_on = false;
  S.col_cap = S.cols_used = 0;
  S.slot_of.clear();
  S.vert_of_slot.clear();
}

void free_solve(DeviceSolve& D) {
  dfree(D.Zs); dfree(D.Et); dfree(D.E); dfree(D.ZE); dfree(D.FE); dfree(D.sep); dfree(D.sblk); dfree(D.frow);
  dfree(D.sseg); dfree(D.lev_row); dfree(D.lev_blk); dfree(D.zs_off); dfree(D.e_off); dfree(D.sub_of);
  dfree(D.sub_begin); dfree(D.ir_off); dfree(D.irows); dfree(D.rl_ptr); dfree(D.rl_sub); dfree(D.rl_p); dfree(D.rT);
  dfree(D.cpl); dfree(D.erow); dfree(D.brow); dfree(D.boff); dfree(D.bstage); dfree(D.xsT);
}

void free_device(Scene& S) {
  dfree(S.tv); dfree(S.tinc); dfree(S.Bm); dfree(S.wV); dfree(S.bV); dfree(S.muV); dfree(S.lamV);
  dfree(S.tet_orig); dfree(S.Vw); dfree(S.rw);
  dfree(S.v_orig); dfree(S.mass); dfree(S.rest); dfree(S.cpin); dfree(S.inc_ptr);
  free_solve(S.S);
  dfree(S.contrib); dfree(S.qt); dfree(S.vt); dfree(S.qtil); dfree(S.c); dfree(S.q_cur); dfree(S.q_prev);
  dfree(S.b_cur); dfree(S.b_prev); dfree(S.qhat); dfree(S.q_last); dfree(S.g_last); dfree(S.dQ); dfree(S.dG);
  dfree(S.ctl); dfree(S.dstat); dfree(S.red_part); dfree(S.red_fin);
  dfree(S.jac); dfree(S.mu); dfree(S.r0); dfree(S.r1); dfree(S.z); dfree(S.p); dfree(S.Ap); dfree(S.wv);
  dfree(S.qbar); dfree(S.ck_scratch); dfree(S.mu_h1); dfree(S.mu_h2); dfree(S.mu_h3);
  dfree(S.mus); dfree(S.mgrp); dfree(S.act); dfree(S.mjac); dfree(S.mgt); dfree(S.mg_ptr); dfree(S.mg_tets);
  contact_free(S);
  if (S.hctl) (void)hipHostFree(S.hctl);
  if (S.hdstat) (void)hipHostFree(S.hdstat);
  if (S.sig_h) (void)hipHostFree(S.sig_h);
  if (S.sigd_h) (void)hipHostFree(S.sigd_h);
  S.sig_h = S.sig_d = nullptr;
  S.sigd_h = S.sigd_d = nullptr;
  S.hctl = nullptr;
  S.hdstat = nullptr;
  for (hipEvent_t e : S.kt.ev) (void)hipEventDestroy(e);
  S.kt.ev.clear();
}

// ---------------------------------------------------------------- kernel timer
enum { kKLocal = 0, kKGather = 1, kKTop = 2, kKBottom = 3, kKEb = 4, kKApplyK = 5, kKSolve = 6, kKCount = 7 };

// the timer of `which` takes launches of kernel `id` (kKSolve: the three
// stages of one global solve)
inline bool kt_match(int which, int id) {
  return which == id || (which == kKSolve && (id == kKEb || id == kKTop || id == kKBottom));
}
constexpr int kTimerPairs = 1024;
// the timer's events only stamp launches: no system-scope fence (cache
// writeback and invalidation) when they complete, which would otherwise slow
// the work they time
constexpr unsigned kTimerEventFlags = hipEventDisableSystemFence;

// Adds the durations of the pending event pairs in launch order; without
// `all`, it stops at the first pair whose kernel has not finished.
void kt_flush(KernelTimer& T, bool all = false) {
  while (T.used > 0) {
    const int i = T.head;
    if (!all) {
      const hipError_t q = hipEventQuery(T.ev[2 * i + 1]);
      if (q == hipErrorNotReady) break;
      PD_HIP(q);
    }
    float ms = 0.0f;
    PD_HIP(hipEventElapsedTime(&ms, T.ev[2 * i], T.ev[2 * i + 1]));
    T.total_ms += ms;
    T.launches++;
    T.head = (T.head + 1) % kTimerPairs;
    T.used--;
  }
}

void kt_flush(Scene& S, bool all = false) { kt_flush(S.kt, all); }

inline void kt_begin(KernelTimer& T, int id, hipStream_t st) {
  if (!kt_match(T.which, id)) return;
  if (T.used == kTimerPairs) {
    PD_HIP(hipStreamSynchronize(st));
    kt_flush(T, true);
  }
  const int i = (T.head + T.used) % kTimerPairs;
  arm_launch_events(T.ev[2 * i], T.ev[2 * i + 1]);
}

// Waits for the decision signal `seq` in slot `slot` of the mapped block, or
// for the stream to drain without it (the chunk of iterations ended before a
// decision).  Returns whether the signal arrived.
bool wait_signal(Scene& S, int slot, int seq, hipStream_t st) {
  volatile int* f = S.sig_h + slot;
  for (unsigned spin = 0;; ++spin) {
    if (*f == seq) {
      std::atomic_thread_fence(std::memory_order_acquire);
      return true;
    }
    if ((spin & 31u) == 31u) {
      const hipError_t q = hipStreamQuery(st);
      if (q == hipSuccess) {
        std::atomic_thread_fence(std::memory_order_acquire);
        return *f == seq;
      }
      if (q != hipErrorNotReady) PD_HIP(q);
    }
  }
}

inline void kt_end(KernelTimer& T, int id, hipStream_t st) {
  if (!kt_match(T.which, id)) return;
  (void)st;
  if (launch_events_used()) T.used++;  // the launcher may have skipped an empty launch
}

inline void kt_begin(Scene& S, int id, hipStream_t st) { kt_begin(S.kt, id, st); }
inline void kt_end(Scene& S, int id, hipStream_t st) { kt_end(S.kt, id, st); }

// working units of the timed kernel: launches that did work, or for kKSolve
// the solves (counted once, with the interface right-hand side stage)
inline void kt_work(Scene& S, int id, long long n) {
  if (S.kt.which == id || (S.kt.which == kKSolve && id == kKEb)) S.kt.working += n;
}

void kt_destroy(Scene& S) {
  for (hipEvent_t e : S.kt.ev) (void)hipEventDestroy(e);
  S.kt.ev.clear();
  S.kt.which = -1;
}

#define PD_TIMED(S, id, st, call) \
  do {                            \
    kt_begin(S, id, st);          \
    call;                         \
    kt_end(S, id, st);            \
  } while (0)

// ---------------------------------------------------------------- argument blocks
ElemArgs elem_args(const Scene& S) {
  ElemArgs E;
  E.ne = S.ne; E.ninc = S.ninc;
  E.tv = S.tv; E.tinc = S.tinc; E.Bm = S.Bm; E.wV = S.wV; E.bV = S.bV; E.muV = S.muV; E.lamV = S.lamV;
  E.tet_orig = S.tet_orig; E.Vw = S.Vw; E.rw = S.rw;
  E.mu_bar = S.mu_bar; E.lam_bar = S.lam_bar; E.k_bar = S.k_bar;
  E.energy = S.energy;
  E.mus = S.mus; E.mgrp = S.mgrp; E.act = S.act; E.mjac = S.mjac; E.mgt = S.mgt;
  return E;
}

VertArgs vert_args(const Scene& S) {
  VertArgs V;
  V.nv = S.nv; V.nf = S.L.nf; V.ne = S.ne; V.ninc = S.ninc;
  V.v_orig = S.v_orig; V.mass = S.mass; V.rest = S.rest; V.cpin = S.cpin; V.inc_ptr = S.inc_ptr;
  V.h = S.h; V.alpha = S.alpha;
  for (int a = 0; a < 3; ++a) V.grav[a] = S.grav[a];
  return V;
}

SolveArgs solve_args(const Scene& S) {
  SolveArgs A;
  const DeviceSolve& D = S.S;
  A.nsub = S.L.nsub; A.nB = S.L.nB; A.nT = S.L.nT;
  A.sub_of = D.sub_of; A.sub_begin = D.sub_begin; A.Zs = D.Zs; A.zs_off = D.zs_off; A.Et = D.Et; A.E = D.E;
  A.e_off = D.e_off; A.ir_off = D.ir_off; A.irows = D.irows; A.rl_ptr = D.rl_ptr; A.rl_sub = D.rl_sub;
  A.rl_p = D.rl_p; A.rT = D.rT;
  A.nlev = D.nlev; A.lev_row = D.lev_row; A.lev_blk = D.lev_blk; A.sep = D.sep; A.sblk = D.sblk; A.ZE = D.ZE;
  A.frow = D.frow; A.sseg = D.sseg; A.FE = D.FE;
  for (int l = 0; l < kMaxLevels; ++l) {
    A.lev_nrows[l] = l < D.nlev ? D.lev_row_h[l + 1] - D.lev_row_h[l] : 0;
    A.lev_nblk[l] = l < D.nlev ? D.lev_blk_h[l + 1] - D.lev_blk_h[l] : 0;
  }
  A.cpl = D.cpl; A.erow = D.erow; A.brow = D.brow; A.boff = D.boff; A.bstage = D.bstage; A.xsT = D.xsT;
  A.n_irows = D.n_irows;
  return A;
}

StepState step_state(Scene& S) {
  StepState T;
  T.m = S.m; T.kmax = S.kmax_fwd; T.eps_rel = S.eps_rel; T.eps_abs = S.eps_abs;
  T.contrib = S.contrib; T.qt = S.qt; T.vt = S.vt; T.qtil = S.qtil; T.c = S.c;
  T.q_cur = S.q_cur; T.q_prev = S.q_prev; T.b_cur = S.b_cur; T.b_prev = S.b_prev; T.qhat = S.qhat;
  T.q_last = S.q_last; T.g_last = S.g_last; T.dQ = S.dQ; T.dG = S.dG;
  T.ctl = S.ctl; T.done = S.ctl + kCtlDone; T.dstat = S.dstat;
  return T;
}

RedArgs red_args(const Scene& S) {
  RedArgs R;
  R.part = S.red_part; R.fin = S.red_fin; R.max_parts = S.red_max_parts;
  const int nb = bottom_blocks(S.L.nB, S.L.nT), ng = vert_group_blocks(S.L.nf);
  R.nparts[kRedGate] = ng;
  R.nparts[kRedAA] = nb;
  R.nparts[kRedPW] = ng;
  R.nparts[kRedRZ0] = nb;
  R.nparts[kRedRZ1] = nb;
  R.nparts[kRedTR] = tr_blocks(S.ne, S.L.nf);
  R.nparts[kRedFix] = nb;
  return R;
}

// ---------------------------------------------------------------- setup
void setup_scene(Scene& S, const pd_mesh_desc* mesh, const pd_material_desc* mat, const pd_solver_opts* o) {
  if (!mesh || !mat || !o) throw PdError{PD_ERR_INVALID_ARG, "null descriptor"};
  const int nv = mesh->n_verts, ne = mesh->n_tets;
  if (nv <= 0 || ne <= 0 || !mesh->rest_xyz || !mesh->tets || !mesh->pinned || !mat->log_E)
    throw PdError{PD_ERR_INVALID_ARG, "empty mesh or null array"};
  if (!(o->h > 0.0) || o->aa_window < 0 || o->aa_window > kMaxWindow || !(o->eps_rel >= 0.0) || o->kmax_fwd < 3 ||
      o->kmax_bwd < 1 || !(o->eps_adj > 0.0) || o->adj_method < 0 || o->adj_method > 1)
    throw PdError{PD_ERR_INVALID_ARG,
                  "invalid solver options (h > 0, 0 <= aa_window <= 5, kmax_fwd >= 3, adj_method 0 or 1)"};
  if (!(mat->nu > -1.0 && mat->nu < 0.5) || !(mat->rho > 0.0) || !(mat->alpha >= 0.0) || !(mat->beta0 >= 0.0))
    throw PdError{PD_ERR_INVALID_ARG, "invalid material constants"};
  S.nv = nv;
  S.ne = ne;
  S.X.assign(mesh->rest_xyz, mesh->rest_xyz + 3 * (size_t)nv);
  S.tets.assign(mesh->tets, mesh->tets + 4 * (size_t)ne);
  S.pinned.assign(mesh->pinned, mesh->pinned + nv);
  S.logE.assign(mat->log_E, mat->log_E + ne);
  for (double x : S.X)
    if (!std::isfinite(x)) throw PdError{PD_ERR_NONFINITE, "non-finite rest position"};
  for (double x : S.logE)
    if (!std::isfinite(x)) throw PdError{PD_ERR_NONFINITE, "non-finite log E"};
  for (int v : S.tets)
    if (v < 0 || v >= nv) throw PdError{PD_ERR_INVALID_ARG, "tet vertex index out of range"};
  S.nu = mat->nu; S.rho = mat->rho; S.alpha = mat->alpha; S.beta0 = mat->beta0;
  if (mat->energy < 0 || mat->energy > 2) throw PdError{PD_ERR_INVALID_ARG, "energy must be 0, 1 or 2"};
  S.energy = mat->energy;
  S.h = o->h;
  for (int a = 0; a < 3; ++a) S.grav[a] = o->gravity[a];
  S.m = o->aa_window; S.eps_rel = o->eps_rel; S.eps_abs = o->eps_abs; S.kmax_fwd = o->kmax_fwd;
  S.kmax_bwd = o->kmax_bwd; S.eps_adj = o->eps_adj; S.eps_tr = o->eps_tr; S.adj_method = o->adj_method;
  S.max_sub = o->max_sub > 0 ? o->max_sub : 256;
  if (o->iface_levels < 0 || o->iface_levels > kMaxLevels)
    throw PdError{PD_ERR_INVALID_ARG, "iface_levels must be 0 (default) or 1..8"};
  S.iface_levels = o->iface_levels > 0 ? o->iface_levels : kDefaultIfaceLevels;
  S.iters_per_check = o->iters_per_check;
  if (o->adj_warm < 0 || o->adj_warm > 3) throw PdError{PD_ERR_INVALID_ARG, "adj_warm must be 0, 1, 2 or 3"};
  if (o->fwd_start < 0 || o->fwd_start > 1) throw PdError{PD_ERR_INVALID_ARG, "fwd_start must be 0 or 1"};
  S.fwd_start = o->fwd_start;
  S.adj_warm = o->adj_warm;
  S.adj_hist = 0;
  // orientation (reorient negative tets), degenerate check
  for (int e = 0; e < ne; ++e) {
    int* t = &S.tets[4 * (size_t)e];
    if (t[0] == t[1] || t[0] == t[2] || t[0] == t[3] || t[1] == t[2] || t[1] == t[3] || t[2] == t[3])
      throw PdError{PD_ERR_DEGENERATE_TET, "repeated vertex in tet " + std::to_string(e)};
    double Dm[9];
    for (int a = 1; a < 4; ++a)
      for (int i = 0; i < 3; ++i) Dm[3 * i + a - 1] = S.X[3 * t[a] + i] - S.X[3 * t[0] + i];
    double d = det3(Dm);
    if (d < 0.0) std::swap(t[1], t[2]), d = -d;
    double scale = 0.0;
    for (int i = 0; i < 9; ++i) scale = std::max(scale, std::fabs(Dm[i]));
    if (!(d > 1e-14 * scale * scale * scale))
      throw PdError{PD_ERR_DEGENERATE_TET, "zero-volume tet " + std::to_string(e)};
  }
  build_layout(nv, ne, S.X.data(), S.tets.data(), S.pinned.data(), S.max_sub, S.iface_levels, S.L);
  if (S.L.nf == 0) throw PdError{PD_ERR_INVALID_ARG, "no free vertex"};
  S.nnz_L = factor_nnz_nd(nv, ne, S.X.data(), S.tets.data(), S.pinned.data());
  const Layout& L = S.L;
  // element geometry in library order
  std::vector<int>& tv = S.htv;
  std::vector<double>& Bm = S.hBm;
  tv.assign(4 * (size_t)ne, 0);
  Bm.assign(9 * (size_t)ne, 0.0);
  std::vector<int> tet_orig(ne);
  for (int t = 0; t < ne; ++t) {
    const int e = L.tet_lib2orig[t];
    tet_orig[t] = e;
    const int* tt = &S.tets[4 * (size_t)e];
    double Dm[9];
    for (int a = 1; a < 4; ++a)
      for (int i = 0; i < 3; ++i) Dm[3 * i + a - 1] = S.X[3 * tt[a] + i] - S.X[3 * tt[0] + i];
    const double d = det3(Dm);
    double Bi[9];
    Bi[0] = (Dm[4] * Dm[8] - Dm[5] * Dm[7]) / d;
    Bi[1] = (Dm[2] * Dm[7] - Dm[1] * Dm[8]) / d;
    Bi[2] = (Dm[1] * Dm[5] - Dm[2] * Dm[4]) / d;
    Bi[3] = (Dm[5] * Dm[6] - Dm[3] * Dm[8]) / d;
    Bi[4] = (Dm[0] * Dm[8] - Dm[2] * Dm[6]) / d;
    Bi[5] = (Dm[2] * Dm[3] - Dm[0] * Dm[5]) / d;
    Bi[6] = (Dm[3] * Dm[7] - Dm[4] * Dm[6]) / d;
    Bi[7] = (Dm[1] * Dm[6] - Dm[0] * Dm[7]) / d;
    Bi[8] = (Dm[0] * Dm[4] - Dm[1] * Dm[3]) / d;
    for (int i = 0; i < 9; ++i) Bm[(size_t)i * ne + t] = Bi[i];
    for (int a = 0; a < 4; ++a) tv[(size_t)a * ne + t] = L.orig2lib[tt[a]];
  }
  S.tv = dalloc<int>(4 * (size_t)ne);
  upload(S.tv, tv);
  S.Bm = dalloc<double>(9 * (size_t)ne);
  upload(S.Bm, Bm);
  S.tet_orig = dalloc<int>(ne);
  upload(S.tet_orig, tet_orig);
  // vertex arrays
  std::vector<int> v_orig(L.lib2orig.begin(), L.lib2orig.end());
  S.v_orig = dalloc<int>(nv);
  upload(S.v_orig, v_orig);
  std::vector<double> rest(3 * (size_t)nv);
  for (int i = 0; i < nv; ++i)
    for (int a = 0; a < 3; ++a) rest[(size_t)a * nv + i] = S.X[3 * (size_t)L.lib2orig[i] + a];
  S.rest = dalloc<double>(3 * (size_t)nv);
  upload(S.rest, rest);
  // incidence of free vertices: (tet, slot) in tet order; each tet slot knows
  // its position so element kernels write straight into vertex order
  const int nf = L.nf;
  std::vector<int> cnt(nf + 1, 0);
  for (int t = 0; t < ne; ++t)
    for (int a = 0; a < 4; ++a) {
      const int i = tv[(size_t)a * ne + t];
      if (i < nf) cnt[i + 1]++;
    }
  for (int i = 0; i < nf; ++i) cnt[i + 1] += cnt[i];
  S.ninc = cnt[nf];
  std::vector<int> fill(cnt.begin(), cnt.end() - 1), tinc(4 * (size_t)ne, -1);
  for (int t = 0; t < ne; ++t)
    for (int a = 0; a < 4; ++a) {
      const int i = tv[(size_t)a * ne + t];
      if (i < nf) tinc[(size_t)a * ne + t] = fill[i]++;
    }
  S.inc_ptr = dalloc<int>(nf + 1);
  upload(S.inc_ptr, cnt);
  S.tinc = dalloc<int>(4 * (size_t)ne);
  upload(S.tinc, tinc);
  // element-material arrays and iteration buffers (sized once)
  S.wV = dalloc<double>(ne); S.bV = dalloc<double>(ne); S.muV = dalloc<double>(ne); S.lamV = dalloc<double>(ne);
  S.Vw = dalloc<double>(4 * (size_t)ne);
  S.rw = dalloc<double>(3 * (size_t)ne);
  S.mass = dalloc<double>(nv);
  S.cpin = dalloc<double>(3 * (size_t)nv);
  const size_t V3 = 3 * (size_t)nv;
  S.contrib = dalloc<double>(3 * (size_t)std::max(1, S.ninc));
  S.qt = dalloc<double>(V3); S.vt = dalloc<double>(V3); S.qtil = dalloc<double>(V3); S.c = dalloc<double>(V3);
  S.q_cur = dalloc<double>(V3); S.q_prev = dalloc<double>(V3); S.b_cur = dalloc<double>(V3);
  S.b_prev = dalloc<double>(V3); S.qhat = dalloc<double>(V3); S.q_last = dalloc<double>(V3);
  S.g_last = dalloc<double>(V3);
  const int mm = std::max(1, S.m);
  S.dQ = dalloc<double>(mm * V3); S.dG = dalloc<double>(mm * V3);
  PD_HIP(hipMemset(S.b_cur, 0, V3 * sizeof(double)));
  S.ctl = dalloc<int>(kCtlTotal);
  PD_HIP(hipMemset(S.ctl, 0, kCtlTotal * sizeof(int)));
  S.dstat = dalloc<double>(32);
  PD_HIP(hipHostMalloc((void**)&S.hctl, kCtlTotal * sizeof(int)));
  PD_HIP(hipHostMalloc((void**)&S.hdstat, 32 * sizeof(double)));
  PD_HIP(hipHostMalloc((void**)&S.sig_h, 16 * sizeof(int), hipHostMallocMapped | hipHostMallocCoherent));
  PD_HIP(hipHostMalloc((void**)&S.sigd_h, 16 * sizeof(double), hipHostMallocMapped | hipHostMallocCoherent));
  std::memset(S.sig_h, 0, 16 * sizeof(int));
  std::memset(S.sigd_h, 0, 16 * sizeof(double));
  PD_HIP(hipHostGetDevicePointer((void**)&S.sig_d, S.sig_h, 0));
  PD_HIP(hipHostGetDevicePointer((void**)&S.sigd_d, S.sigd_h, 0));
  S.jac = dalloc<double>(kJacRows * (size_t)ne);
  S.mu = dalloc<double>(V3); S.r0 = dalloc<double>(V3); S.r1 = dalloc<double>(V3); S.z = dalloc<double>(V3);
  S.p = dalloc<double>(V3); S.Ap = dalloc<double>(V3); S.wv = dalloc<double>(V3); S.qbar = dalloc<double>(V3);
  S.ck_scratch = dalloc<double>(12 * (size_t)nv);
  S.mu_h1 = dalloc<double>(V3); S.mu_h2 = dalloc<double>(V3); S.mu_h3 = dalloc<double>(V3);
  PD_HIP(hipMemset(S.mu, 0, V3 * sizeof(double)));
  PD_HIP(hipMemset(S.z, 0, V3 * sizeof(double)));
  // reduction sites sized for the widest producing kernel
  S.red_max_parts = std::max({bottom_blocks(L.nB, L.nT), vert_group_blocks(nf), tr_blocks(ne, nf),
                               contact_apply_blocks(nf), 1});
  S.red_part = dalloc<double>((size_t)kRedSites * S.red_max_parts * kRedWidth);
  S.red_fin = dalloc<double>((size_t)kRedSites * kFinStride);
  PD_HIP(hipMemset(S.red_part, 0, (size_t)kRedSites * S.red_max_parts * kRedWidth * sizeof(double)));
  PD_HIP(hipMemset(S.red_fin, 0, (size_t)kRedSites * kFinStride * sizeof(double)));
  launch_init_warm(elem_args(S), nullptr);
  PD_HIP(hipDeviceSynchronize());
  S.stale = true;
}

// Block elimination of the interface Schur complement over the separator
// tree (levels ascending; the nodes of a level are independent).  Node n's
// frontal matrix F (its rows, then its struct) gets its children's updates;
// then Z_n = F_nn^{-1}, E_n = F_{struct,n} Z_n and the update
// F_{struct,struct} - E_n F_{n,struct} for its parent.  Returns per node the
// backward rows [Z_n[j, :], -E_n[:, j]] and E_n (forward rows).
struct SepFactor {
  std::vector<std::vector<double>> ZE, E;
};

SepFactor eliminate_separators(const Layout& L, std::vector<std::vector<double>>& Fr, const std::vector<int>& fs,
                               const std::vector<int>& fb, int T) {
  const int nsep = (int)fs.size();
  SepFactor R;
  R.ZE.resize(nsep);
  R.E.resize(nsep);
  std::vector<std::vector<int>> children(nsep);
  for (int n = 0; n < nsep; ++n)
    if (L.sep_parent[n] >= 0) children[L.sep_parent[n]].push_back(n);
  std::vector<std::vector<double>> U(nsep);
  std::vector<int> ok(nsep, 1);
  auto elim = [&](int n, int nth) {
    const int sn = fs[n], bn = fb[n];
    const size_t m = (size_t)sn + bn;
    std::vector<double>& F = Fr[n];
    for (int c : children[n]) {  // extend-add of the children's updates
      const auto& st = L.sep_struct[c];
      const int bc = (int)st.size();
      std::vector<int> at(bc);
      for (int p = 0; p < bc; ++p) {
        const int u = st[p];
        if (u >= L.sep_begin[n] && u < L.sep_begin[n + 1]) {
          at[p] = u - L.sep_begin[n];
        } else {
          const auto& sn_st = L.sep_struct[n];
          const auto it = std::lower_bound(sn_st.begin(), sn_st.end(), u);
          if (it == sn_st.end() || *it != u) {
            ok[n] = -1;  // a child's struct outside its parent's block: a layout error
            return;
          }
          at[p] = sn + (int)(it - sn_st.begin());
        }
      }
      for (int p = 0; p < bc; ++p)
        for (int q = 0; q < bc; ++q) F[(size_t)at[p] * m + at[q]] += U[c][(size_t)p * bc + q];
      std::vector<double>().swap(U[c]);
    }
    std::vector<double> Z((size_t)sn * sn);
    for (int i = 0; i < sn; ++i)
      for (int j = 0; j < sn; ++j) Z[(size_t)i * sn + j] = F[(size_t)i * m + j];
    if (!(nth > 1 ? spd_inverse_threaded(Z, sn) : spd_inverse(Z, sn))) {
      ok[n] = 0;
      return;
    }
    std::vector<double>& E = R.E[n];
    E.assign((size_t)bn * sn, 0.0);
    std::vector<double> Un((size_t)bn * bn);
    auto rows = [&](int t, int nt) {
      for (int p = t; p < bn; p += nt) {
        const double* f = &F[(size_t)(sn + p) * m];
        double* e = &E[(size_t)p * sn];
        for (int k = 0; k < sn; ++k) {
          if (f[k] == 0.0) continue;
          const double* z = &Z[(size_t)k * sn];
          for (int j = 0; j < sn; ++j) e[j] += f[k] * z[j];
        }
        for (int q = 0; q < bn; ++q) {
          double d = F[(size_t)(sn + p) * m + sn + q];
          for (int j = 0; j < sn; ++j) d -= e[j] * F[(size_t)j * m + sn + q];
          Un[(size_t)p * bn + q] = d;
        }
      }
    };
    if (nth > 1) run_threads(nth, [&](int t) { rows(t, nth); });
    else rows(0, 1);
    std::vector<double>& ZE = R.ZE[n];
    ZE.resize((size_t)sn * m);
    for (int j = 0; j < sn; ++j) {
      double* r = &ZE[(size_t)j * m];
      for (int k = 0; k < sn; ++k) r[k] = Z[(size_t)j * sn + k];
      for (int p = 0; p < bn; ++p) r[sn + p] = -E[(size_t)p * sn + j];
    }
    U[n] = std::move(Un);
    std::vector<double>().swap(F);
  };
  constexpr int kBigNode = 1024;  // rows above which a node is eliminated with all threads
  for (int lo = 0; lo < nsep;) {
    int hi = lo;
    while (hi < nsep && L.sep_level[hi] == L.sep_level[lo]) ++hi;
    std::vector<int> small, big;
    for (int n = lo; n < hi; ++n) (fs[n] < kBigNode ? small : big).push_back(n);
    run_threads(T, [&](int t) {
      for (size_t k = t; k < small.size(); k += T) elim(small[k], 1);
    });
    for (int n : big) elim(n, T);
    for (int n = lo; n < hi; ++n) {
      if (ok[n] < 0) throw PdError{PD_ERR_INVALID_ARG, "layout: separator blocks do not nest"};
      if (!ok[n]) throw PdError{PD_ERR_FACTOR_NOT_SPD, "interface Schur complement not SPD"};
    }
    lo = hi;
  }
  return R;
}

void factorize(Scene& S) {
  const Layout& L = S.L;
  const int nv = S.nv, ne = S.ne, nf = L.nf, nB = L.nB, nT = L.nT;
  const double h = S.h;
  // materials (Sec. 3.1 Eq. lame; Sec. 4.1 Eq. pd_weight read as the rest
  // tangent modulus w_e = 2 mu_e + lam_e; Sec. 4.2 mesh means; Sec. 4.5)
  std::vector<double> mu(ne), lam(ne), w(ne), beta(ne), vol(ne);
  double smu = 0.0, slam = 0.0, mref = 0.0;
  for (int e = 0; e < ne; ++e) {
    const double E = std::exp(S.logE[e]);
    mu[e] = E / (2.0 * (1.0 + S.nu));
    lam[e] = E * S.nu / ((1.0 + S.nu) * (1.0 - 2.0 * S.nu));
    w[e] = 2.0 * mu[e] + lam[e];
    smu += mu[e];
    slam += lam[e];
    mref = std::max(mref, mu[e]);
  }
  S.mu_bar = smu / ne;
  S.lam_bar = slam / ne;
  S.mu_ref = mref;
  if (S.frozen) {  // constants of the gradient held fixed (finite-difference checks)
    S.mu_bar = S.frozen_means[0];
    S.lam_bar = S.frozen_means[1];
    S.mu_ref = S.frozen_means[2];
  }
  S.k_bar = 2.0 * S.mu_bar + S.lam_bar;
  mref = S.mu_ref;
  for (int e = 0; e < ne; ++e) beta[e] = S.beta0 * mu[e] / mref;
  // per-tet data in library order
  const std::vector<double>& Bm = S.hBm;
  const std::vector<int>& tv = S.htv;
  std::vector<double> wV(ne), bV(ne), muV(ne), lamV(ne);
  std::vector<double> mass(nv, 0.0);
  for (int t = 0; t < ne; ++t) {
    const int e = L.tet_lib2orig[t];
    const int* tt = &S.tets[4 * (size_t)e];
    double Dm[9];
    for (int a = 1; a < 4; ++a)
      for (int i = 0; i < 3; ++i) Dm[3 * i + a - 1] = S.X[3 * tt[a] + i] - S.X[3 * tt[0] + i];
    vol[t] = det3(Dm) / 6.0;
    wV[t] = w[e] * vol[t];
    bV[t] = beta[e] * vol[t] / h;
    muV[t] = mu[e] * vol[t];
    lamV[t] = lam[e] * vol[t];
    for (int a = 0; a < 4; ++a) mass[tv[(size_t)a * ne + t]] += S.rho * vol[t] / 4.0;
  }
  upload(S.wV, wV); upload(S.bV, bV); upload(S.muV, muV); upload(S.lamV, lamV);
  upload(S.mass, mass);
  // muscle fibres in library order: m (3) and w_m V_e
  std::vector<double> mus;
  if (S.n_mg > 0) {
    mus.assign(4 * (size_t)ne, 0.0);
    for (int t = 0; t < ne; ++t) {
      const int e = L.tet_lib2orig[t];
      if (S.hmgroup[e] < 0) continue;
      for (int j = 0; j < 3; ++j) mus[(size_t)j * ne + t] = S.hmfib[3 * (size_t)e + j];
      mus[3 * (size_t)ne + t] = S.w_m * vol[t];
    }
    upload(S.mus, mus);
  }
  // assemble A~ (Sec. 4.5 Eq. A_damped) into the block structure
  const int nsub = L.nsub;
  std::vector<std::vector<double>> Ass(nsub), AIs(nsub);
  std::vector<int> sub_of(nf, -1);
  for (int s = 0; s < nsub; ++s) {
    const int ns = L.sub_begin[s + 1] - L.sub_begin[s];
    Ass[s].assign((size_t)ns * ns, 0.0);
    AIs[s].assign(L.Irows[s].size() * (size_t)ns, 0.0);
    for (int i = L.sub_begin[s]; i < L.sub_begin[s + 1]; ++i) sub_of[i] = s;
  }
  // frontal blocks of the separator tree: node n's rows, then its struct;
  // an entry of S between rows u and w is assembled at the lower of their
  // nodes (the other row is that node's own or in its struct)
  const int nsep = (int)L.sep_level.size();
  std::vector<int> node_of(std::max(1, nT), 0), fs(nsep), fb(nsep);
  for (int n = 0; n < nsep; ++n) {
    fs[n] = L.sep_begin[n + 1] - L.sep_begin[n];
    fb[n] = (int)L.sep_struct[n].size();
    for (int i = L.sep_begin[n]; i < L.sep_begin[n + 1]; ++i) node_of[i] = n;
    const size_t m = (size_t)fs[n] + fb[n];
    if (m * m > (size_t)1 << 28)
      throw PdError{PD_ERR_ALLOC, "a separator block is too large for its dense frontal matrix; use more levels"};
  }
  std::vector<std::vector<double>> Fr(nsep);
  for (int n = 0; n < nsep; ++n) Fr[n].assign(((size_t)fs[n] + fb[n]) * ((size_t)fs[n] + fb[n]), 0.0);
  auto fpos = [&](int n, int u) {
    if (node_of[u] == n) return u - L.sep_begin[n];
    const auto& st = L.sep_struct[n];
    const auto it = std::lower_bound(st.begin(), st.end(), u);
    if (it == st.end() || *it != u) throw PdError{PD_ERR_INVALID_ARG, "layout: entry outside the separator blocks"};
    return fs[n] + (int)(it - st.begin());
  };
  auto addS = [&](int u, int w, double val) {
    const int nu = node_of[u], nw = node_of[w];
    const int n = L.sep_level[nu] < L.sep_level[nw] ? nu : nw;
    if (L.sep_level[nu] == L.sep_level[nw] && nu != nw)
      throw PdError{PD_ERR_INVALID_ARG, "layout: coupled separators on one level"};
    const size_t m = (size_t)fs[n] + fb[n];
    Fr[n][(size_t)fpos(n, u) * m + fpos(n, w)] += val;
  };
  std::vector<double> cpin(3 * (size_t)nv, 0.0);
  auto ipos = [&](int s, int iface) {
    const auto& I = L.Irows[s];
    return (int)(std::lower_bound(I.begin(), I.end(), iface) - I.begin());
  };
  for (int i = 0; i < nf; ++i) {
    const double d = (1.0 + S.alpha * h) * mass[i] / (h * h);
    if (i < nB) {
      const int s = sub_of[i], b = L.sub_begin[s], ns = L.sub_begin[s + 1] - b;
      Ass[s][(size_t)(i - b) * ns + (i - b)] += d;
    } else {
      addS(i - nB, i - nB, d);
    }
  }
  for (int t = 0; t < ne; ++t) {
    const double cst = (wV[t] + bV[t]);
    double Bh[4][3];
    for (int j = 0; j < 3; ++j) {
      Bh[1][j] = Bm[(size_t)(0 + j) * ne + t];
      Bh[2][j] = Bm[(size_t)(3 + j) * ne + t];
      Bh[3][j] = Bm[(size_t)(6 + j) * ne + t];
      Bh[0][j] = -(Bh[1][j] + Bh[2][j] + Bh[3][j]);
    }
    // a muscle tet adds w_m V_e c c^T with c_a = Bhat_a . m (its fibre's G_m^T G_m)
    double mc[4] = {0, 0, 0, 0}, wm = 0.0;
    if (!mus.empty() && mus[3 * (size_t)ne + t] != 0.0) {
      wm = mus[3 * (size_t)ne + t];
      for (int a = 0; a < 4; ++a)
        for (int j = 0; j < 3; ++j) mc[a] += Bh[a][j] * mus[(size_t)j * ne + t];
    }
    for (int a = 0; a < 4; ++a) {
      const int i = tv[(size_t)a * ne + t];
      if (i >= nf) continue;
      for (int b = 0; b < 4; ++b) {
        const int j = tv[(size_t)b * ne + t];
        const double val = cst * (Bh[a][0] * Bh[b][0] + Bh[a][1] * Bh[b][1] + Bh[a][2] * Bh[b][2]) +
                           wm * mc[a] * mc[b];
        if (j >= nf) {  // coupling to a pinned vertex (held at rest)
          for (int ax = 0; ax < 3; ++ax) cpin[(size_t)ax * nv + i] -= val * S.X[3 * (size_t)L.lib2orig[j] + ax];
          continue;
        }
        if (i < nB && j < nB) {
          const int s = sub_of[i];
          if (sub_of[j] != s) throw PdError{PD_ERR_INVALID_ARG, "layout: coupled subdomains"};
          const int b0 = L.sub_begin[s], ns = L.sub_begin[s + 1] - b0;
          Ass[s][(size_t)(i - b0) * ns + (j - b0)] += val;
        } else if (i >= nB && j < nB) {
          const int s = sub_of[j], b0 = L.sub_begin[s], ns = L.sub_begin[s + 1] - b0;
          AIs[s][(size_t)ipos(s, i - nB) * ns + (j - b0)] += val;
        } else if (i >= nB && j >= nB) {
          addS(i - nB, j - nB, val);
        }
      }
    }
  }
  upload(S.cpin, cpin);
  // partitioned inverse: Zs = A_ss^{-1}, E_s = A_{I s} Zs, S = A_TT - sum E_s A_{s I}, Z = S^{-1}
  std::vector<long long> zs_off(nsub + 1, 0), e_off(nsub + 1, 0);
  for (int s = 0; s < nsub; ++s) {
    const long long ns = L.sub_begin[s + 1] - L.sub_begin[s];
    zs_off[s + 1] = zs_off[s] + ns * ns;
    e_off[s + 1] = e_off[s] + ns * (long long)L.Irows[s].size();
  }
  std::vector<double> Zs_all(zs_off[nsub]), Et_all(e_off[nsub]), E_all(e_off[nsub]);
  // subdomains in parallel (each writes only its own blocks and its Schur
  // contribution), then the contributions are added in subdomain order
  std::vector<std::vector<double>> schur(nsub);
  std::vector<int> sub_ok(nsub, 1);
  const int T = host_threads();
  run_threads(T, [&](int t) {
  for (int s = t; s < nsub; s += T) {
    const int ns = L.sub_begin[s + 1] - L.sub_begin[s];
    const int nI = (int)L.Irows[s].size();
    std::vector<double> Z = Ass[s];
    if (!spd_inverse(Z, ns)) {
      sub_ok[s] = 0;
      continue;
    }
    std::copy(Z.begin(), Z.end(), Zs_all.begin() + zs_off[s]);
    // E_s (nI x ns) = A_Is (nI x ns) Z (ns x ns)
    double* Es = &E_all[e_off[s]];
    for (int p = 0; p < nI; ++p) {
      const double* a = &AIs[s][(size_t)p * ns];
      double* e = Es + (size_t)p * ns;
      for (int u = 0; u < ns; ++u) {
        if (a[u] == 0.0) continue;
        const double* zr = &Z[(size_t)u * ns];
        for (int v = 0; v < ns; ++v) e[v] += a[u] * zr[v];
      }
    }
    for (int v = 0; v < ns; ++v)
      for (int p = 0; p < nI; ++p) Et_all[e_off[s] + (size_t)v * nI + p] = Es[(size_t)p * ns + v];
    // Schur contribution E_s A_{s I} on the interface rows of s
    std::vector<double>& sc = schur[s];
    sc.assign((size_t)nI * nI, 0.0);
    for (int p = 0; p < nI; ++p) {
      const double* e = Es + (size_t)p * ns;
      for (int q = 0; q < nI; ++q) {
        const double* a = &AIs[s][(size_t)q * ns];
        double d = 0.0;
        for (int v = 0; v < ns; ++v) d += e[v] * a[v];
        sc[(size_t)p * nI + q] = d;
      }
    }
  }
  });
  for (int s = 0; s < nsub; ++s) {
    if (!sub_ok[s]) throw PdError{PD_ERR_FACTOR_NOT_SPD, "subdomain block not SPD"};
    const int nI = (int)L.Irows[s].size();
    for (int p = 0; p < nI; ++p)
      for (int q = 0; q < nI; ++q) addS(L.Irows[s][p], L.Irows[s][q], -schur[s][(size_t)p * nI + q]);
  }
  schur.clear();
  SepFactor SF = eliminate_separators(L, Fr, fs, fb, T);
  Fr.clear();
  // couplings of each interface row: (subdomain, row of E_s), subdomains ascending
  std::vector<int> ir_off(nsub + 1, 0), irows;
  for (int s = 0; s < nsub; ++s) {
    ir_off[s + 1] = ir_off[s] + (int)L.Irows[s].size();
    irows.insert(irows.end(), L.Irows[s].begin(), L.Irows[s].end());
  }
  std::vector<int> rl_ptr(nT + 1, 0);
  for (int v : irows) rl_ptr[v + 1]++;
  for (int i = 0; i < nT; ++i) rl_ptr[i + 1] += rl_ptr[i];
  std::vector<int> rl_fill(rl_ptr.begin(), rl_ptr.end() - 1), rl_sub(irows.size()), rl_p(irows.size());
  for (int s = 0; s < nsub; ++s)
    for (int p = 0; p < (int)L.Irows[s].size(); ++p) {
      const int pos = rl_fill[L.Irows[s][p]]++;
      rl_sub[pos] = s;
      rl_p[pos] = p;
    }
  // descriptors of the kernels: per interface row its couplings, with E
  // re-stored row-concatenated; per subdomain row its blocks
  int max_coup = 0;
  std::vector<Cpl> cpl((size_t)std::max(1, nT) * kMaxCoup, Cpl{0, 0, 0, 0});
  std::vector<ERow> erow(std::max(1, nT), ERow{0, 0, 0});
  std::vector<double> E_flat(E_all.size());
  {
    long long off = 0;
    for (int i = 0; i < nT; ++i) {
      const int n = rl_ptr[i + 1] - rl_ptr[i];
      max_coup = std::max(max_coup, n);
      if (n > kMaxCoup)
        throw PdError{PD_ERR_INVALID_ARG, "an interface vertex borders more than 8 subdomains; lower max_sub"};
      int pre = 0;
      for (int c = 0; c < n; ++c) {
        const int s = rl_sub[rl_ptr[i] + c], pr = rl_p[rl_ptr[i] + c];
        const int b0 = L.sub_begin[s], ns = L.sub_begin[s + 1] - b0;
        cpl[(size_t)i * kMaxCoup + c] = Cpl{b0, pre, ir_off[s] + pr, 0};
        std::copy(&E_all[e_off[s] + (size_t)pr * ns], &E_all[e_off[s] + (size_t)(pr + 1) * ns],
                  E_flat.begin() + off + pre);
        pre += ns;
      }
      for (int c = n; c < kMaxCoup; ++c) cpl[(size_t)i * kMaxCoup + c] = Cpl{0, pre, 0, 0};
      erow[i] = ERow{off, pre, n};
      off += pre;
    }
    if (off != (long long)E_all.size()) throw PdError{PD_ERR_INVALID_ARG, "layout: coupling sizes disagree"};
  }
  std::vector<BRow> brow(std::max(1, nB), BRow{0, 0, 0, 0});
  std::vector<BOff> boff(std::max(1, nB), BOff{0, 0});
  for (int v = 0; v < nB; ++v) {
    const int s = sub_of[v], b0 = L.sub_begin[s], ns = L.sub_begin[s + 1] - b0, nI = (int)L.Irows[s].size();
    brow[v] = BRow{b0, ns, nI, ir_off[s]};
    boff[v] = BOff{zs_off[s] + (long long)(v - b0) * ns, e_off[s] + (long long)(v - b0) * nI};
  }
  // staged ranges of each subdomain-solve block (rows are in subdomain order, so
  // a block's rows span one contiguous range of right-hand-side rows and one of
  // interface copies)
  constexpr int kRowsPerBlock = kBottomRows;
  std::vector<BStage> bstage(std::max(1, (nB + kRowsPerBlock - 1) / kRowsPerBlock), BStage{0, 0, 0, 0});
  for (int b = 0; b * kRowsPerBlock < nB; ++b) {
    const BRow& f = brow[b * kRowsPerBlock];
    const BRow& l = brow[std::min(nB, (b + 1) * kRowsPerBlock) - 1];
    const int zn = l.b0 + l.ns - f.b0, en = l.ir0 + l.nI - f.ir0;
    if (zn <= kStageZ && en <= kStageE) bstage[b] = BStage{f.b0, zn, f.ir0, en};
  }
  // the separator tree's solve structure: backward rows per node, their
  // blocks per level, forward rows per interface row with their segments;
  // the gathered interface vectors hold the subdomains' slots, then every
  // node's struct
  const int n_leaf_slots = (int)irows.size();
  std::vector<SepNode> sep(std::max(1, nsep), SepNode{0, 0, 0, 0, 0});
  long long ze_total = 0;
  int slots = n_leaf_slots;
  for (int n = 0; n < nsep; ++n) {
    sep[n] = SepNode{ze_total, L.sep_begin[n], fs[n], fb[n], slots};
    ze_total += (long long)fs[n] * (fs[n] + fb[n]);
    slots += fb[n];
  }
  std::vector<double> ZE_all((size_t)std::max(1LL, ze_total));
  for (int n = 0; n < nsep; ++n) std::copy(SF.ZE[n].begin(), SF.ZE[n].end(), ZE_all.begin() + sep[n].zoff);
  std::vector<std::vector<std::pair<int, int>>> segs_of(std::max(1, nT));  // (node, struct position), nodes ascending
  for (int n = 0; n < nsep; ++n)
    for (int p = 0; p < fb[n]; ++p) segs_of[L.sep_struct[n][p]].push_back({n, p});
  std::vector<FRow> frow(std::max(1, nT), FRow{0, 0, 0});
  std::vector<SSeg> sseg;
  std::vector<double> FE_all;
  for (int i = 0; i < nT; ++i) {
    if ((int)segs_of[i].size() > kSepMaxSeg)
      throw PdError{PD_ERR_INVALID_ARG, "an interface vertex couples to more than 56 separator blocks; use fewer levels"};
    frow[i] = FRow{(long long)FE_all.size(), (int)sseg.size(), (int)segs_of[i].size()};
    for (const auto& cp : segs_of[i]) {
      const int c = cp.first, p = cp.second;
      sseg.push_back(SSeg{L.sep_begin[c], fs[c], sep[c].xs0 + p, 0});
      FE_all.insert(FE_all.end(), SF.E[c].begin() + (size_t)p * fs[c], SF.E[c].begin() + (size_t)(p + 1) * fs[c]);
    }
  }
  SF = SepFactor{};
  if (sseg.empty()) sseg.push_back(SSeg{0, 0, 0, 0});
  if (FE_all.empty()) FE_all.push_back(0.0);
  std::vector<SepBlk> sblk;
  std::vector<int> lev_blk(L.nlev + 1, 0);
  for (int n = 0; n < nsep; ++n) {
    if (n == 0 || L.sep_level[n] != L.sep_level[n - 1]) lev_blk[L.sep_level[n] - 1] = (int)sblk.size();
    // a wide node's rows go one per wave, the others kSepRowsPerWave per wave
    const bool wide = fs[n] + fb[n] >= kSepWide;
    const int per = wide ? kBlock / 64 : kSepRows;
    for (int r = 0; r < fs[n]; r += per)
      sblk.push_back(SepBlk{n, L.sep_begin[n] + r, std::min(per, fs[n] - r), wide ? 1 : 0});
  }
  if (L.nlev > 0) lev_blk[L.nlev] = (int)sblk.size();
  if (sblk.empty()) sblk.push_back(SepBlk{0, 0, 0, 0});
  // upload the solve structure
  DeviceSolve& D = S.S;
  free_solve(D);
  D.ZE = dalloc<double>(ZE_all.size()); upload(D.ZE, ZE_all);
  D.FE = dalloc<double>(FE_all.size()); upload(D.FE, FE_all);
  D.sep = dalloc<SepNode>(sep.size()); upload(D.sep, sep);
  D.sblk = dalloc<SepBlk>(sblk.size()); upload(D.sblk, sblk);
  D.frow = dalloc<FRow>(frow.size()); upload(D.frow, frow);
  D.sseg = dalloc<SSeg>(sseg.size()); upload(D.sseg, sseg);
  D.nlev = L.nlev;
  D.lev_row_h = L.lev_begin;
  D.lev_blk_h = lev_blk;
  D.lev_row = dalloc<int>(L.nlev + 1); upload(D.lev_row, L.lev_begin);
  D.lev_blk = dalloc<int>(L.nlev + 1); upload(D.lev_blk, lev_blk);
  D.Zs = dalloc<double>(Zs_all.size()); upload(D.Zs, Zs_all);
  D.Et = dalloc<double>(Et_all.size()); upload(D.Et, Et_all);
  D.E = dalloc<double>(E_flat.size()); upload(D.E, E_flat);
  D.cpl = dalloc<Cpl>(cpl.size()); upload(D.cpl, cpl);
  D.erow = dalloc<ERow>(erow.size()); upload(D.erow, erow);
  D.brow = dalloc<BRow>(brow.size()); upload(D.brow, brow);
  D.boff = dalloc<BOff>(boff.size()); upload(D.boff, boff);
  D.bstage = dalloc<BStage>(bstage.size()); upload(D.bstage, bstage);
  D.n_irows = slots;
  D.xsT = dalloc<double>(3 * (size_t)std::max(1, D.n_irows));
  D.max_coup = max_coup;
  D.zs_off = dalloc<long long>(nsub + 1); upload(D.zs_off, zs_off);
  D.e_off = dalloc<long long>(nsub + 1); upload(D.e_off, e_off);
  std::vector<int> sub_of_B(sub_of.begin(), sub_of.begin() + nB);
  D.sub_of = dalloc<int>(std::max(1, nB)); upload(D.sub_of, sub_of_B);
  D.sub_begin = dalloc<int>(nsub + 1); upload(D.sub_begin, L.sub_begin);
  D.ir_off = dalloc<int>(nsub + 1); upload(D.ir_off, ir_off);
  D.irows = dalloc<int>(irows.size()); upload(D.irows, irows);
  D.rl_ptr = dalloc<int>(nT + 1); upload(D.rl_ptr, rl_ptr);
  D.rl_sub = dalloc<int>(rl_sub.size()); upload(D.rl_sub, rl_sub);
  D.rl_p = dalloc<int>(rl_p.size()); upload(D.rl_p, rl_p);
  D.rT = dalloc<double>(3 * (size_t)std::max(1, nT));
  D.zs_entries = (double)Zs_all.size();
  D.e_entries = (double)E_all.size();
  D.ze_entries = (double)ze_total;
  D.fe_entries = (double)(FE_all.size() > 1 ? FE_all.size() : 0);
  D.bytes = (Zs_all.size() + Et_all.size() + E_all.size() + ZE_all.size() + FE_all.size()) * sizeof(double);
  PD_HIP(hipDeviceSynchronize());
  S.stale = false;
  S.fact_gen++;
  S.adj_hist = 0;
  // cached contact columns belong to the old factor
  for (int v : S.vert_of_slot) S.slot_of[v] = -1;
  S.vert_of_slot.clear();
  S.cols_used = 0;
}

AdjState adj_state(Scene& S) {
  AdjState A;
  A.kmax = S.kmax_bwd; A.eps = S.eps_adj;
  A.contrib = S.contrib; A.qbar = S.qbar; A.mu = S.mu; A.z = S.z; A.p = S.p; A.Ap = S.Ap; A.w = S.wv;
  A.r0 = S.r0; A.r1 = S.r1;
  A.ctl = S.ctl + kCtlAdj; A.done = S.ctl + kCtlAdj + 2; A.dstat = S.dstat + 16;
  return A;
}

// x = A~^{-1} rhs (plain mode: no reductions, `done` may be null)
void solve_plain(Scene& S, const double* rhs, double* out, int* done, hipStream_t st) {
  const VertArgs V = vert_args(S);
  const SolveArgs A = solve_args(S);
  const RedArgs R = red_args(S);
  StepState T = step_state(S);
  T.done = done;
  const AdjState Ad = adj_state(S);
  PD_TIMED(S, kKEb, st, launch_Eb(kModePlain, V, A, T, Ad, R, rhs, 0, st));
  PD_TIMED(S, kKTop, st, launch_top(V, A, out, done, st));
  PD_TIMED(S, kKBottom, st, launch_bottom(kModePlain, V, A, T, Ad, R, rhs, out, 0, st));
}


// ---------------------------------------------------------------- contact
constexpr int kErrContact = PD_ERR_CONTACT;

ContactArgs contact_args(Scene& S, int K, bool adjoint) {
  ContactArgs C;
  C.K = K;
  C.nf = S.L.nf;
  C.v = adjoint ? S.a_v : S.c_v;
  C.n = adjoint ? S.a_n : S.c_n;
  C.g = S.c_g;
  C.slot = adjoint ? S.a_slot : S.c_slot;
  C.cols = S.cols;
  C.W = adjoint ? S.a_Winv : S.c_W;
  C.lam = S.c_lam;
  C.s = adjoint ? S.a_s : S.c_s;
  C.fb = S.c_fb;
  C.flags = S.c_flags;
  C.Lg = S.c_Lg;
  C.mu = S.mu_f;
  C.qt = S.qt;
  C.frw = S.c_frw;
  C.fri = S.c_fri;
  C.kind = adjoint ? nullptr : S.c_kind;
  if (adjoint && S.a_fric) {
    C.nb = S.a_nb;
    C.dg = S.a_dg;
  }
  return C;
}

// Column a_v = A~^{-1} e_v of every listed vertex that the cache lacks (three
// per three-right-hand-side solve); slots receive each entry's column slot.
// A full cache is emptied first.
void ensure_columns(Scene& S, const int* verts, int n, int* slots, hipStream_t st) {
  std::vector<int> need;
  auto collect = [&]() {
    need.clear();
    for (int c = 0; c < n; ++c) {
      const int v = verts[c];
      if (S.slot_of[v] == -1) {
        S.slot_of[v] = -2;
        need.push_back(v);
      }
    }
  };
  collect();
  if (S.cols_used + (int)need.size() > S.col_cap) {
    for (int v : need) S.slot_of[v] = -1;
    for (int v : S.vert_of_slot) S.slot_of[v] = -1;
    S.vert_of_slot.clear();
    S.cols_used = 0;
    collect();
    if ((int)need.size() > S.col_cap) throw PdError{kErrContact, "contact vertices exceed the column cache"};
  }
  for (int v : need) {
    S.slot_of[v] = S.cols_used++;
    S.vert_of_slot.push_back(v);
  }
  const VertArgs V = vert_args(S);
  const SolveArgs A = solve_args(S);
  const RedArgs R = red_args(S);
  StepState T = step_state(S);
  T.done = nullptr;
  const AdjState Ad = adj_state(S);
  for (size_t j = 0; j < need.size(); j += 3) {
    int vv[3] = {-1, -1, -1}, ss[3] = {-1, -1, -1};
    for (int a = 0; a < 3 && j + a < need.size(); ++a) {
      vv[a] = need[j + a];
      ss[a] = S.slot_of[vv[a]];
    }
    launch_unit_rhs(S.nv, S.z, vv[0], vv[1], vv[2], st);
    launch_Eb(kModePlain, V, A, T, Ad, R, S.z, 0, st);
    launch_top(V, A, S.wv, nullptr, st);
    launch_bottom(kModePlain, V, A, T, Ad, R, S.z, S.wv, 0, st);
    launch_store_cols(S.L.nf, S.nv, S.wv, S.cols, ss[0], ss[1], ss[2], st);
  }
  S.c_cols_built += (int)need.size();
  for (int c = 0; c < n; ++c) slots[c] = S.slot_of[verts[c]];
}

// Candidate rows of this step (q_t, v_t already in library order), their
// columns and the Delassus operator; returns the row count.
int contact_rows(Scene& S, hipStream_t st) {
  const VertArgs V = vert_args(S);
  ObsArgs O;
  O.n_planes = S.n_planes;
  O.n_boxes = S.n_boxes;
  O.planes = S.obs;
  O.boxes = S.obs + 4 * S.n_planes;
  O.d_c = S.d_c;
  O.h = S.h;
  O.one_per_vertex = S.mu_f > 0.0 ? 1 : 0;
  int K = 0;
  if (S.n_planes + S.n_boxes > 0) {
    launch_contact_detect(V, S.qt, S.vt, O, S.c_kmax, S.c_v, S.c_n, S.c_g, S.c_flags, st);
    PD_HIP(hipMemcpyAsync(S.h_cbuf, S.c_flags, 4 * sizeof(int), hipMemcpyDeviceToHost, st));
    PD_HIP(hipStreamSynchronize(st));
    K = S.h_cbuf[0];
  }
  // the attachments' bilateral rows follow the detected ones
  const int nb = (int)S.att_v.size();
  if (K + nb > S.c_kmax)
    throw PdError{kErrContact, "contact rows (" + std::to_string(K + nb) + ") exceed max_contacts (" +
                                   std::to_string(S.c_kmax) + ")"};
  {
    std::vector<int> kind(std::max(K + nb, 1), 0);
    for (int c = K; c < K + nb; ++c) kind[c] = 1;
    if (nb > 0) {
      PD_HIP(hipMemcpy(S.c_v + K, S.att_v.data(), nb * sizeof(int), hipMemcpyHostToDevice));
      PD_HIP(hipMemcpy(S.c_n + 3 * (size_t)K, S.att_n.data(), 3 * nb * sizeof(double), hipMemcpyHostToDevice));
      PD_HIP(hipMemcpy(S.c_g + K, S.att_g.data(), nb * sizeof(double), hipMemcpyHostToDevice));
    }
    if (K + nb > 0) PD_HIP(hipMemcpy(S.c_kind, kind.data(), (K + nb) * sizeof(int), hipMemcpyHostToDevice));
  }
  K += nb;
  if (K == 0) return 0;
  int* hv = S.h_cbuf + 4;
  int* hs = hv + S.c_kmax;
  PD_HIP(hipMemcpyAsync(hv, S.c_v, K * sizeof(int), hipMemcpyDeviceToHost, st));
  PD_HIP(hipStreamSynchronize(st));
  ensure_columns(S, hv, K, hs, st);
  PD_HIP(hipMemcpyAsync(S.c_slot, hs, K * sizeof(int), hipMemcpyHostToDevice, st));
  const ContactArgs C = contact_args(S, K, false);
  launch_contact_W(C, S.c_W, st);
  launch_contact_start(C, st);
  PD_HIP(hipStreamSynchronize(st));
  return K;
}

// The adjoint rows of the active frictional contacts (Sec. 4.8 with the active
// set fixed): each keeps its normal row; a contact whose slip over the step
// |s| exceeds 1e-8 mu lam_n w_c (w_c = a_{v_c}[v_c]) slides and adds one row
// along p, the tangent perpendicular to the slip, with diagonal |s|/(mu
// lam_n), and its normal multiplier then acts along n - mu s^ (the friction
// force follows lam_n); a sticking contact adds its rows t1, t2.  The rows
// act along nb and constrain along n; the inverse of their coupling matrix
// goes to a_Winv.  Returns the row count.
static void host_frame(const double n[3], double t1[3], double t2[3]) {
  int k = 0;
  if (std::fabs(n[1]) < std::fabs(n[k])) k = 1;
  if (std::fabs(n[2]) < std::fabs(n[k])) k = 2;
  const double an = n[k];
  double t[3], nrm = 0.0;
  for (int i = 0; i < 3; ++i) {
    t[i] = (i == k ? 1.0 : 0.0) - an * n[i];
    nrm += t[i] * t[i];
  }
  nrm = std::sqrt(nrm);
  for (int i = 0; i < 3; ++i) t1[i] = t[i] / nrm;
  t2[0] = n[1] * t1[2] - n[2] * t1[1];
  t2[1] = n[2] * t1[0] - n[0] * t1[2];
  t2[2] = n[0] * t1[1] - n[1] * t1[0];
}

int contact_active_friction(Scene& S, const double* ck, const std::vector<int>& av, const std::vector<double>& an,
                            const std::vector<double>& al, const int* slots, hipStream_t st) {
  const int na = (int)av.size(), nv = S.nv;
  const VertArgs V = vert_args(S);
  // slip and diagonal of every active contact vertex
  PD_HIP(hipMemcpyAsync(S.a_v, av.data(), na * sizeof(int), hipMemcpyHostToDevice, st));
  PD_HIP(hipMemcpyAsync(S.a_slot, slots, na * sizeof(int), hipMemcpyHostToDevice, st));
  ContactArgs C0 = contact_args(S, na, true);
  launch_contact_slip(V, C0, ck + 6 * (size_t)nv, ck, S.c_slip, st);
  std::vector<double> sl(4 * (size_t)na);
  PD_HIP(hipMemcpyAsync(sl.data(), S.c_slip, 4 * (size_t)na * sizeof(double), hipMemcpyDeviceToHost, st));
  PD_HIP(hipStreamSynchronize(st));
  std::vector<int> rv, rs, kind;
  std::vector<double> rc, rb, rd;
  auto row = [&](int c, int k, const double* cdir, const double* bdir, double d) {
    rv.push_back(av[c]);
    rs.push_back(slots[c]);
    kind.push_back(k);
    rc.insert(rc.end(), cdir, cdir + 3);
    rb.insert(rb.end(), bdir, bdir + 3);
    rd.push_back(d);
  };
  for (int c = 0; c < na; ++c) {
    const double* n = an.data() + 3 * c;
    double t1[3], t2[3];
    host_frame(n, t1, t2);
    const double* dq = sl.data() + 4 * c;
    const double w = dq[3];
    const double s1 = t1[0] * dq[0] + t1[1] * dq[1] + t1[2] * dq[2];
    const double s2 = t2[0] * dq[0] + t2[1] * dq[1] + t2[2] * dq[2];
    const double ns = std::sqrt(s1 * s1 + s2 * s2), tau = S.mu_f * al[c];
    if (ns / w > 1e-8 * tau) {
      const double h1 = s1 / ns, h2 = s2 / ns;
      double b[3], p[3];
      for (int i = 0; i < 3; ++i) {
        b[i] = n[i] - S.mu_f * (h1 * t1[i] + h2 * t2[i]);
        p[i] = -h2 * t1[i] + h1 * t2[i];
      }
      row(c, 0, n, b, 0.0);
      row(c, 2, p, p, ns / tau);
    } else {
      row(c, 0, n, n, 0.0);
      row(c, 1, t1, t1, 0.0);
      row(c, 1, t2, t2, 0.0);
    }
  }
  const int nr = (int)rv.size();
  if (nr > kMaxAdjRows) throw PdError{kErrContact, "friction rows exceed the adjoint capacity"};
  PD_HIP(hipMemcpyAsync(S.a_v, rv.data(), nr * sizeof(int), hipMemcpyHostToDevice, st));
  PD_HIP(hipMemcpyAsync(S.a_slot, rs.data(), nr * sizeof(int), hipMemcpyHostToDevice, st));
  PD_HIP(hipMemcpyAsync(S.a_kind, kind.data(), nr * sizeof(int), hipMemcpyHostToDevice, st));
  PD_HIP(hipMemcpyAsync(S.a_n, rc.data(), 3 * nr * sizeof(double), hipMemcpyHostToDevice, st));
  PD_HIP(hipMemcpyAsync(S.a_nb, rb.data(), 3 * nr * sizeof(double), hipMemcpyHostToDevice, st));
  PD_HIP(hipMemcpyAsync(S.a_dg, rd.data(), nr * sizeof(double), hipMemcpyHostToDevice, st));
  launch_zero_int(S.c_flags + 2, 1, st);
  S.a_fric = true;
  const ContactArgs C = contact_args(S, nr, true);
  launch_contact_minv(C, S.a_Winv, st);
  PD_HIP(hipMemcpyAsync(S.h_cbuf, S.c_flags, 4 * sizeof(int), hipMemcpyDeviceToHost, st));
  PD_HIP(hipStreamSynchronize(st));
  if (S.h_cbuf[2]) throw PdError{kErrContact, "the adjoint's contact coupling matrix is singular"};
  return nr;
}

// Active rows of a checkpointed step (lam_c > 1e-10 max lam), their columns
// and the inverse of their Delassus block; returns the active count.
int contact_active(Scene& S, const double* ck, hipStream_t st) {
  const int kmax = S.c_kmax;
  const double* rec = ck + (size_t)kCheckpointVecs * 3 * S.nv;
  S.a_fric = false;
  PD_HIP(hipMemcpyAsync(S.h_crec, rec, (2 + 10 * (size_t)kmax) * sizeof(double), hipMemcpyDeviceToHost, st));
  PD_HIP(hipStreamSynchronize(st));
  const double* h = S.h_crec;
  const int K = (int)h[0];
  if (K < 0 || K > kmax) throw PdError{PD_ERR_INVALID_ARG, "checkpoint holds no valid contact record"};
  // active rows: every bilateral row, and the unilateral rows whose impulse
  // exceeds 1e-10 of the largest unilateral one
  auto bil = [&](int c) { return h[1 + 8 * kmax + c] == 1.0; };
  double lmax = 0.0;
  for (int c = 0; c < K; ++c)
    if (!bil(c)) lmax = std::max(lmax, h[1 + 5 * kmax + c]);
  auto active = [&](int c) { return bil(c) || (lmax > 0.0 && h[1 + 5 * kmax + c] > 1e-10 * lmax); };
  std::vector<int> av;
  std::vector<double> an;
  S.a_rows.clear();
  S.a_K = K;
  S.a_rest = false;
  for (int c = 0; c < K; ++c) {
    if (h[1 + 9 * kmax + c] == 1.0) S.a_rest = true;
    if (active(c)) {
      av.push_back((int)h[1 + c]);
      for (int a = 0; a < 3; ++a) an.push_back(h[1 + kmax + 3 * c + a]);
      S.a_rows.push_back(c);
    }
  }
  const int na = (int)av.size();
  S.c_last_active = na;
  if (na == 0) return 0;
  int* hs = S.h_cbuf + 4 + kmax;
  ensure_columns(S, av.data(), na, hs, st);
  if (S.mu_f > 0.0) {
    std::vector<double> al;
    for (int c = 0; c < K; ++c)
      if (active(c)) al.push_back(h[1 + 5 * kmax + c]);
    return contact_active_friction(S, ck, av, an, al, hs, st);
  }
  PD_HIP(hipMemcpyAsync(S.a_v, av.data(), na * sizeof(int), hipMemcpyHostToDevice, st));
  PD_HIP(hipMemcpyAsync(S.a_n, an.data(), 3 * na * sizeof(double), hipMemcpyHostToDevice, st));
  PD_HIP(hipMemcpyAsync(S.a_slot, hs, na * sizeof(int), hipMemcpyHostToDevice, st));
  launch_zero_int(S.c_flags + 2, 1, st);
  const ContactArgs C = contact_args(S, na, true);
  launch_contact_winv(C, S.a_Winv, st);
  PD_HIP(hipMemcpyAsync(S.h_cbuf, S.c_flags, 4 * sizeof(int), hipMemcpyDeviceToHost, st));
  PD_HIP(hipStreamSynchronize(st));
  if (S.h_cbuf[2]) throw PdError{kErrContact, "Delassus block of the active rows is not positive definite"};
  return na;
}

}  // namespace

// Algorithmic bytes of one working launch of each timed kernel: what the
// operation must read and write once (matrix blocks, element data, vectors),
// not what the implementation re-reads.
static double kernel_bytes(const Scene& S, int id) {
  const Layout& L = S.L;
  const double nf = L.nf, nT = L.nT, nB = L.nB, ne = S.ne, nv = S.nv, ninc = S.ninc;
  const double zs = S.S.zs_entries, et = S.S.e_entries;
  switch (id) {
    case kKLocal:  // tet indices, D_m^-1, weight per tet; positions in and right-hand side out per vertex
      return ne * (16.0 + 72.0 + 8.0) + 48.0 * nv;
    case kKGather:  // contributions and constant part in, b and q out
      return 24.0 * ninc + 24.0 * nf * 4;
    case kKEb:  // coupling blocks E_s, right-hand side in, interface right-hand side out
      return 8.0 * et + 24.0 * nf + 24.0 * nT;
    case kKTop:  // separator blocks (backward rows, forward rows), interface right-hand side in, solution out
      return 8.0 * (S.S.ze_entries + S.S.fe_entries) + 24.0 * nT * 2;
    case kKBottom:  // subdomain inverses and couplings, right-hand sides, solution out
      return 8.0 * (zs + et) + 24.0 * (nB * 2 + nT);
    case kKApplyK:  // tet indices, D_m^-1, weight, 30 Jacobian values per tet; x in and K x out per vertex
      return ne * (16.0 + 72.0 + 8.0 + 240.0) + 48.0 * nv;
    case kKSolve:  // one forward and one backward sweep of a sparse factor of A~, six vector passes
      return 16.0 * S.nnz_L + 6.0 * 24.0 * nf;
    default:
      return 0.0;
  }
}

// ================================================================= C ABI
#define PD_TRY try {
#define PD_CATCH                                   \
  }                                                \
  catch (const PdError& e) {                       \
    pdhot::g_last_error = e.msg;                                 \
    return e.code;                                 \
  }                                                \
  catch (const std::bad_alloc&) {                  \
    pdhot::g_last_error = "host allocation failed";              \
    return PD_ERR_ALLOC;                           \
  }                                                \
  catch (const std::exception& e) {                \
    pdhot::g_last_error = e.what();                              \
    return PD_ERR_INVALID_ARG;                     \
  }

extern "C" {

const char* pd_last_error(void) { return pdhot::g_last_error.c_str(); }

int pd_scene_vertex_logw(const pd_scene* scene, double* out) {
  if (!scene || !out) {
    pdhot::g_last_error = "null argument";
    return PD_ERR_INVALID_ARG;
  }
  PD_TRY
  const Scene& S = scene->S;
  std::vector<double> sum(S.nv, 0.0);
  std::vector<int> cnt(S.nv, 0);
  const double nu = S.nu;
  for (int e = 0; e < S.ne; ++e) {
    const double E = std::exp(S.logE[e]);
    const double mu = E / (2.0 * (1.0 + nu)), lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
    const double lw = std::log(2.0 * mu + lam);
    for (int a = 0; a < 4; ++a) {
      sum[S.tets[4 * (size_t)e + a]] += lw;
      cnt[S.tets[4 * (size_t)e + a]] += 1;
    }
  }
  double mean = 0.0;
  for (int i = 0; i < S.nv; ++i) {
    out[i] = sum[i] / std::max(1, cnt[i]);
    mean += out[i];
  }
  mean /= S.nv;
  for (int i = 0; i < S.nv; ++i) out[i] -= mean;
  return PD_OK;
  PD_CATCH
}

int pd_scene_create(const pd_mesh_desc* mesh, const pd_material_desc* mat, const pd_solver_opts* opts,
                    pd_scene** out) {
  if (!out) {
    pdhot::g_last_error = "null output pointer";
    return PD_ERR_INVALID_ARG;
  }
  *out = nullptr;
  pd_scene* sc = nullptr;
  PD_TRY
  sc = new pd_scene();
  setup_scene(sc->S, mesh, mat, opts);
  factorize(sc->S);
  *out = sc;
  pdhot::g_last_error.clear();
  return PD_OK;
  }
  catch (const PdError& e) {
    pdhot::g_last_error = e.msg;
    if (sc) { free_device(sc->S); delete sc; }
    return e.code;
  }
  catch (const std::exception& e) {
    pdhot::g_last_error = e.what();
    if (sc) { free_device(sc->S); delete sc; }
    return PD_ERR_INVALID_ARG;
  }
}

int pd_scene_destroy(pd_scene* scene) {
  if (!scene) return PD_OK;
  free_device(scene->S);
  delete scene;
  return PD_OK;
}

int pd_scene_set_material(pd_scene* scene, const double* log_E_host) {
  if (!scene || !log_E_host) {
    pdhot::g_last_error = "null argument";
    return PD_ERR_INVALID_ARG;
  }
  for (int e = 0; e < scene->S.ne; ++e)
    if (!std::isfinite(log_E_host[e])) {
      pdhot::g_last_error = "non-finite log E";
      return PD_ERR_NONFINITE;
    }
  scene->S.logE.assign(log_E_host, log_E_host + scene->S.ne);
  scene->S.stale = true;
  return PD_OK;
}

int pd_scene_factorize(pd_scene* scene, void* stream) {
  if (!scene) {
    pdhot::g_last_error = "null scene";
    return PD_ERR_INVALID_ARG;
  }
  PD_TRY
  // kernels of earlier steps (e.g. the gradient routing, which reads the
  // per-tet weights) may still run on the caller's stream or on a batch's
  // stream: the per-tet arrays and the factor are replaced only after all
  // device work has finished
  PD_HIP(hipStreamSynchronize((hipStream_t)stream));
  PD_HIP(hipDeviceSynchronize());
  factorize(scene->S);
  return PD_OK;
  PD_CATCH
}

int pd_scene_set_material_device(pd_scene* scene, const double* log_E_dev, void* stream) {
  if (!scene || !log_E_dev) {
    pdhot::g_last_error = "null argument";
    return PD_ERR_INVALID_ARG;
  }
  PD_TRY
  std::vector<double> h(scene->S.ne);
  PD_HIP(hipMemcpyAsync(h.data(), log_E_dev, h.size() * sizeof(double), hipMemcpyDeviceToHost,
                        (hipStream_t)stream));
  PD_HIP(hipStreamSynchronize((hipStream_t)stream));
  return pd_scene_set_material(scene, h.data());
  PD_CATCH
}

int pd_scene_set_muscles(pd_scene* scene, int n_groups, double w_m, const int32_t* group, const double* fibre) {
  if (!scene || n_groups < 0 || (n_groups > 0 && (!group || !fibre))) {
    pdhot::g_last_error = "null argument or negative group count";
    return PD_ERR_INVALID_ARG;
  }
  Scene& S = scene->S;
  const int ne = S.ne;
  if (n_groups > 0) {
    if (!(std::isfinite(w_m) && w_m > 0.0)) {
      pdhot::g_last_error = "the fibre weight must be positive and finite";
      return PD_ERR_INVALID_ARG;
    }
    for (int e = 0; e < ne; ++e) {
      if (group[e] < -1 || group[e] >= n_groups) {
        pdhot::g_last_error = "muscle group out of range";
        return PD_ERR_INVALID_ARG;
      }
      if (group[e] < 0) continue;
      const double* m = fibre + 3 * (size_t)e;
      const double n2 = m[0] * m[0] + m[1] * m[1] + m[2] * m[2];
      if (!std::isfinite(n2) || std::fabs(n2 - 1.0) > 1e-9) {
        pdhot::g_last_error = "muscle fibres must be unit vectors";
        return PD_ERR_INVALID_ARG;
      }
    }
  }
  PD_TRY
  PD_HIP(hipDeviceSynchronize());  // kernels of earlier steps may still read the fibre arrays
  dfree(S.mus); dfree(S.mgrp); dfree(S.act); dfree(S.mjac); dfree(S.mgt); dfree(S.mg_ptr); dfree(S.mg_tets);
  S.n_mg = n_groups;
  S.w_m = n_groups > 0 ? w_m : 0.0;
  S.hmgroup.clear();
  S.hmfib.clear();
  S.g_act = nullptr;
  if (n_groups > 0) {
    S.hmgroup.assign(group, group + ne);
    S.hmfib.assign(fibre, fibre + 3 * (size_t)ne);
    // each group's tets in library order, and the library-order group ids
    std::vector<int> cnt(n_groups + 1, 0), grp(ne, 0);
    for (int t = 0; t < ne; ++t) {
      const int g = group[S.L.tet_lib2orig[t]];
      if (g >= 0) {
        cnt[g + 1]++;
        grp[t] = g;
      }
    }
    for (int g = 0; g < n_groups; ++g) cnt[g + 1] += cnt[g];
    std::vector<int> list(std::max(1, cnt[n_groups])), fill(cnt.begin(), cnt.end() - 1);
    for (int t = 0; t < ne; ++t) {
      const int g = group[S.L.tet_lib2orig[t]];
      if (g >= 0) list[fill[g]++] = t;
    }
    S.mus = dalloc<double>(4 * (size_t)ne);
    S.mgrp = dalloc<int>(ne);
    upload(S.mgrp, grp);
    S.act = dalloc<double>(n_groups);
    PD_HIP(hipMemset(S.act, 0, sizeof(double) * n_groups));
    S.mjac = dalloc<double>(4 * (size_t)ne);
    S.mgt = dalloc<double>(ne);
    S.mg_ptr = dalloc<int>(n_groups + 1);
    upload(S.mg_ptr, cnt);
    S.mg_tets = dalloc<int>(list.size());
    upload(S.mg_tets, list);
  }
  S.stale = true;
  return PD_OK;
  PD_CATCH
}

int pd_scene_set_activation(pd_scene* scene, const double* a_dev, void* stream) {
  if (!scene || !a_dev || scene->S.n_mg <= 0) {
    pdhot::g_last_error = scene && scene->S.n_mg <= 0 ? "the scene has no muscles" : "null argument";
    return PD_ERR_INVALID_ARG;
  }
  PD_TRY
  PD_HIP(hipMemcpyAsync(scene->S.act, a_dev, sizeof(double) * scene->S.n_mg, hipMemcpyDeviceToDevice,
                        (hipStream_t)stream));
  return PD_OK;
  PD_CATCH
}

int pd_scene_set_activation_grad(pd_scene* scene, double* g_act_dev) {
  if (!scene || (g_act_dev && scene->S.n_mg <= 0)) {
    pdhot::g_last_error = scene ? "the scene has no muscles" : "null scene";
    return PD_ERR_INVALID_ARG;
  }
  scene->S.g_act = g_act_dev;
  return PD_OK;
}

int pd_scene_freeze_means(pd_scene* scene, const double* means3) {
  if (!scene) {
    pdhot::g_last_error = "null scene";
    return PD_ERR_INVALID_ARG;
  }
  if (means3 && !(means3[0] > 0.0 && std::isfinite(means3[0]) && std::isfinite(means3[1]) &&
                  means3[0] + means3[1] > 0.0 && means3[2] > 0.0 && std::isfinite(means3[2]))) {
    pdhot::g_last_error = "frozen means must be finite with mu_bar > 0, mu_ref > 0";
    return PD_ERR_INVALID_ARG;
  }
  Scene& S = scene->S;
  S.frozen = means3 != nullptr;
  if (means3)
    for (int i = 0; i < 3; ++i) S.frozen_means[i] = means3[i];
  S.stale = true;
  return PD_OK;
}

int pd_scene_factor_nnz(const pd_scene* scene, double* nnz) {
  if (!scene || !nnz) {
    pdhot::g_last_error = "null argument";
    return PD_ERR_INVALID_ARG;
  }
  *nnz = scene->S.nnz_L;
  return PD_OK;
}

int pd_scene_vertex_mass(const pd_scene* scene, double* out) {
  if (!scene || !out) {
    pdhot::g_last_error = "null argument";
    return PD_ERR_INVALID_ARG;
  }
  const Scene& S = scene->S;
  for (int v = 0; v < S.nv; ++v) out[v] = 0.0;
  for (int e = 0; e < S.ne; ++e) {
    const int* tt = &S.tets[4 * (size_t)e];
    double Dm[9];
    for (int a = 1; a < 4; ++a)
      for (int i = 0; i < 3; ++i) Dm[3 * i + a - 1] = S.X[3 * tt[a] + i] - S.X[3 * tt[0] + i];
    const double m4 = S.rho * det3(Dm) / 24.0;
    for (int a = 0; a < 4; ++a) out[tt[a]] += m4;
  }
  return PD_OK;
}

int pd_scene_info(const pd_scene* scene, double* info, double* means) {
  if (!scene) {
    pdhot::g_last_error = "null scene";
    return PD_ERR_INVALID_ARG;
  }
  const Scene& S = scene->S;
  if (info) {
    info[0] = S.nv; info[1] = S.ne; info[2] = S.L.nf; info[3] = S.L.nsub; info[4] = S.L.nT; info[5] = S.m;
    info[6] = (double)S.S.bytes;
    info[7] = S.S.max_coup;
  }
  if (means) { means[0] = S.mu_bar; means[1] = S.lam_bar; means[2] = S.k_bar; means[3] = S.mu_ref; }
  return PD_OK;
}

int pd_scene_get_permutation(const pd_scene* scene, int32_t* perm_out) {
  if (!scene || !perm_out) {
    pdhot::g_last_error = "null argument";
    return PD_ERR_INVALID_ARG;
  }
  const Scene& S = scene->S;
  for (int i = 0; i < S.nv; ++i) perm_out[i] = S.L.lib2orig[i];
  return PD_OK;
}

size_t pd_ckpt_bytes(const pd_scene* scene) {
  if (!scene) return 0;
  const Scene& S = scene->S;
  size_t n = (size_t)kCheckpointVecs * 3 * (size_t)S.nv;
  if (S.contact_on) n += 2 + 10 * (size_t)S.c_kmax;
  return n * sizeof(double);
}

int pd_scene_set_obstacles(pd_scene* scene, int n_planes, const double* planes, int n_boxes, const double* boxes,
                           double d_c, int max_contacts, double fb_tol) {
  if (!scene) {
    pdhot::g_last_error = "null scene";
    return PD_ERR_INVALID_ARG;
  }
  PD_TRY
  Scene& S = scene->S;
  if (n_planes < 0 || n_boxes < 0 || n_planes + n_boxes > kMaxObstacles)
    throw PdError{PD_ERR_INVALID_ARG, "at most " + std::to_string(kMaxObstacles) + " obstacles"};
  if ((n_planes > 0 && !planes) || (n_boxes > 0 && !boxes)) throw PdError{PD_ERR_INVALID_ARG, "null obstacle array"};
  contact_free(S);
  if (n_planes + n_boxes == 0 && S.att_v.empty()) return PD_OK;
  if (!(d_c > 0.0) || !(fb_tol > 0.0) || max_contacts < 1 || max_contacts > kMaxContactRows)
    throw PdError{PD_ERR_INVALID_ARG, "need d_c > 0, fb_tol > 0 and 1 <= max_contacts <= " +
                                          std::to_string(kMaxContactRows)};
  std::vector<double> obs;
  for (int i = 0; i < n_planes; ++i) {
    const double* P = planes + 4 * i;
    const double nn = std::sqrt(P[0] * P[0] + P[1] * P[1] + P[2] * P[2]);
    if (!(std::fabs(nn - 1.0) <= 1e-12)) throw PdError{PD_ERR_INVALID_ARG, "plane normals must be unit vectors"};
    obs.insert(obs.end(), P, P + 4);
  }
  for (int i = 0; i < n_boxes; ++i) {
    const double* B = boxes + 6 * i;
    if (!(B[0] < B[3] && B[1] < B[4] && B[2] < B[5])) throw PdError{PD_ERR_INVALID_ARG, "box needs lo < hi"};
    obs.insert(obs.end(), B, B + 6);
  }
  const int kmax = max_contacts, nf = S.L.nf;
  S.n_planes = n_planes;
  S.n_boxes = n_boxes;
  S.d_c = d_c;
  S.fb_tol = fb_tol;
  S.c_kmax = kmax;
  S.obs = dalloc<double>(obs.size());
  upload(S.obs, obs);
  S.c_v = dalloc<int>(kmax); S.c_slot = dalloc<int>(kmax); S.c_flags = dalloc<int>(4);
  // sized for friction (three rows per contact), which pd_scene_set_friction may turn on
  const size_t rmax = 3 * (size_t)kmax;
  S.c_n = dalloc<double>(3 * (size_t)kmax); S.c_g = dalloc<double>(kmax); S.c_lam = dalloc<double>(rmax);
  S.c_s = dalloc<double>(3 * (size_t)kmax); S.c_W = dalloc<double>((size_t)kmax * kmax);
  S.c_fb = dalloc<double>(2);
  S.a_v = dalloc<int>(rmax); S.a_slot = dalloc<int>(rmax);
  S.a_n = dalloc<double>(3 * rmax); S.a_s = dalloc<double>(3 * rmax);
  S.a_Winv = dalloc<double>(rmax * rmax);
  S.c_Lg = dalloc<double>(std::max(rmax * rmax, (rmax + 1) * (rmax + 2) / 2 + rmax + 1));
  S.c_frw = dalloc<double>((size_t)kFrWork * kmax); S.c_fri = dalloc<int>(2 * rmax);
  S.a_nb = dalloc<double>(3 * rmax); S.a_dg = dalloc<double>(rmax); S.a_kind = dalloc<int>(rmax);
  S.c_slip = dalloc<double>(4 * (size_t)kmax);
  S.c_kind = dalloc<int>(kmax); S.rest_s = dalloc<double>(kmax); S.gv_rest = dalloc<double>(3 * (size_t)S.nv);
  S.col_cap = 4 * kmax;
  S.cols = dalloc<double>((size_t)S.col_cap * std::max(nf, 1));
  S.cols_used = 0;
  S.slot_of.assign(std::max(nf, 1), -1);
  S.vert_of_slot.clear();
  PD_HIP(hipHostMalloc((void**)&S.h_cbuf, (4 + 2 * (size_t)kmax) * sizeof(int)));
  PD_HIP(hipHostMalloc((void**)&S.h_crec, (2 + 10 * (size_t)kmax) * sizeof(double)));
  PD_HIP(hipMemset(S.c_fb, 0, 2 * sizeof(double)));
  PD_HIP(hipMemset(S.c_flags, 0, 4 * sizeof(int)));
  S.contact_on = true;
  S.c_last_K = S.c_last_active = 0;
  return PD_OK;
  PD_CATCH
}

int pd_contact_rows(const pd_scene* scene, int* K, int32_t* vert, double* normals, double* offsets,
                    double* lambda, int capacity) {
  if (!scene || !K) {
    pdhot::g_last_error = "null argument";
    return PD_ERR_INVALID_ARG;
  }
  PD_TRY
  const Scene& S = scene->S;
  *K = S.contact_on ? S.c_last_K : 0;
  const int n = std::min(*K, std::max(capacity, 0));
  if (n > 0) {
    std::vector<int> v(n);
    PD_HIP(hipMemcpy(v.data(), S.c_v, n * sizeof(int), hipMemcpyDeviceToHost));
    if (vert)
      for (int c = 0; c < n; ++c) vert[c] = S.L.lib2orig[v[c]];
    if (normals) PD_HIP(hipMemcpy(normals, S.c_n, 3 * n * sizeof(double), hipMemcpyDeviceToHost));
    if (offsets) PD_HIP(hipMemcpy(offsets, S.c_g, n * sizeof(double), hipMemcpyDeviceToHost));
    if (lambda) {
      if (S.mu_f > 0.0) {
        std::vector<double> l3(3 * (size_t)n);
        PD_HIP(hipMemcpy(l3.data(), S.c_lam, 3 * n * sizeof(double), hipMemcpyDeviceToHost));
        for (int c = 0; c < n; ++c) lambda[c] = l3[3 * c];
      } else {
        PD_HIP(hipMemcpy(lambda, S.c_lam, n * sizeof(double), hipMemcpyDeviceToHost));
      }
    }
  }
  return PD_OK;
  PD_CATCH
}

int pd_scene_set_attachments(pd_scene* scene, int n_rows, const int32_t* vert, const double* normals,
                             const double* offsets) {
  if (!scene || n_rows < 0 || (n_rows > 0 && (!vert || !normals || !offsets))) {
    pdhot::g_last_error = "null argument or negative row count";
    return PD_ERR_INVALID_ARG;
  }
  PD_TRY
  Scene& S = scene->S;
  if (n_rows > 0 && S.mu_f > 0.0) throw PdError{PD_ERR_INVALID_ARG, "bilateral rows run with frictionless contact only"};
  if (n_rows > kMaxContactRows) throw PdError{PD_ERR_INVALID_ARG, "too many bilateral rows"};
  std::vector<int> av(n_rows);
  std::vector<double> an(3 * (size_t)n_rows), ag(n_rows);
  for (int c = 0; c < n_rows; ++c) {
    const int v = vert[c];
    if (v < 0 || v >= S.nv) throw PdError{PD_ERR_INVALID_ARG, "attachment vertex out of range"};
    if (S.pinned[v]) throw PdError{PD_ERR_INVALID_ARG, "attachment on a pinned vertex"};
    const double* n = normals + 3 * (size_t)c;
    const double nn = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    if (!(std::fabs(nn - 1.0) <= 1e-12) || !std::isfinite(offsets[c]))
      throw PdError{PD_ERR_INVALID_ARG, "attachment rows need unit directions and finite offsets"};
    av[c] = S.L.orig2lib[v];
    for (int a = 0; a < 3; ++a) an[3 * (size_t)c + a] = n[a];
    ag[c] = offsets[c];
  }
  if (S.contact_on && n_rows > S.c_kmax)
    throw PdError{PD_ERR_INVALID_ARG, "bilateral rows exceed max_contacts of the obstacles"};
  PD_HIP(hipDeviceSynchronize());  // earlier steps may still read the row buffers
  S.att_v = av;
  S.att_n = an;
  S.att_g = ag;
  S.c_last_K = S.c_last_active = 0;
  if (!S.contact_on && n_rows > 0) {
    // the rows run through the contact machinery: set it up without obstacles
    const int rc = pd_scene_set_obstacles(scene, 0, nullptr, 0, nullptr, 1.0, std::max(64, n_rows), 1e-10);
    if (rc != PD_OK) return rc;
  }
  return PD_OK;
  PD_CATCH
}

int pd_scene_set_restitution(pd_scene* scene, double e) {
  if (!scene || !std::isfinite(e)) {
    pdhot::g_last_error = "null scene or non-finite coefficient";
    return PD_ERR_INVALID_ARG;
  }
  scene->S.rest_e = e >= 0.0 ? e : -1.0;
  return PD_OK;
}

int pd_contact_gap_grad(pd_scene* scene, double* g_out, int capacity) {
  if (!scene || (capacity > 0 && !g_out)) {
    pdhot::g_last_error = "null argument";
    return PD_ERR_INVALID_ARG;
  }
  PD_TRY
  Scene& S = scene->S;
  if (!S.contact_on) throw PdError{PD_ERR_INVALID_ARG, "the scene has no contact rows"};
  if (S.mu_f > 0.0) throw PdError{PD_ERR_INVALID_ARG, "offset gradients are formed for frictionless rows only"};
  const int K = S.a_K;
  if (capacity < K) throw PdError{PD_ERR_INVALID_ARG, "capacity below the row count"};
  for (int c = 0; c < K; ++c) g_out[c] = 0.0;
  const int na = (int)S.a_rows.size();
  if (na == 0) return PD_OK;
  // dL/dg = W_AA^{-1} J_A A~^{-1} (q bar + K mu) from the last backward step's mu
  // (the backward step may still run on the caller's stream)
  PD_HIP(hipDeviceSynchronize());
  hipStream_t st = nullptr;
  const ElemArgs E = elem_args(S);
  const VertArgs V = vert_args(S);
  const AdjState Ad = adj_state(S);
  const RedArgs R = red_args(S);
  launch_apply_K(kModeDebug, E, V, Ad, R, S.jac, S.mu, 0, st);
  launch_adj_gather(kModeDebug, V, Ad, R, 0, st);
  const size_t n3 = 3 * (size_t)S.nv;
  std::vector<double> qb(n3), kx(n3), x(n3), Winv((size_t)na * na);
  std::vector<int> v(na);
  std::vector<double> nrm(3 * (size_t)na);
  PD_HIP(hipMemcpy(qb.data(), S.qbar, n3 * sizeof(double), hipMemcpyDeviceToHost));
  PD_HIP(hipMemcpy(kx.data(), S.wv, n3 * sizeof(double), hipMemcpyDeviceToHost));
  for (int a = 0; a < 3; ++a)
    for (int i = S.L.nf; i < S.nv; ++i) kx[(size_t)a * S.nv + i] = 0.0;
  for (size_t i = 0; i < n3; ++i) qb[i] += kx[i];
  PD_HIP(hipMemcpy(S.z, qb.data(), n3 * sizeof(double), hipMemcpyHostToDevice));
  solve_plain(S, S.z, S.p, nullptr, st);
  PD_HIP(hipMemcpy(x.data(), S.p, n3 * sizeof(double), hipMemcpyDeviceToHost));
  PD_HIP(hipMemcpy(Winv.data(), S.a_Winv, Winv.size() * sizeof(double), hipMemcpyDeviceToHost));
  PD_HIP(hipMemcpy(v.data(), S.a_v, na * sizeof(int), hipMemcpyDeviceToHost));
  PD_HIP(hipMemcpy(nrm.data(), S.a_n, nrm.size() * sizeof(double), hipMemcpyDeviceToHost));
  std::vector<double> y(na);
  for (int a = 0; a < na; ++a) {
    double t = 0.0;
    for (int ax = 0; ax < 3; ++ax) t += nrm[3 * (size_t)a + ax] * x[(size_t)ax * S.nv + v[a]];
    y[a] = t;
  }
  for (int a = 0; a < na; ++a) {
    double t = 0.0;
    for (int b = 0; b < na; ++b) t += Winv[(size_t)a * na + b] * y[b];
    g_out[S.a_rows[a]] = t;
  }
  return PD_OK;
  PD_CATCH
}

int pd_scene_set_friction(pd_scene* scene, double mu) {
  if (!scene) {
    pdhot::g_last_error = "null scene";
    return PD_ERR_INVALID_ARG;
  }
  PD_TRY
  Scene& S = scene->S;
  if (!S.contact_on) throw PdError{PD_ERR_INVALID_ARG, "friction needs obstacles (pd_scene_set_obstacles first)"};
  if (mu > 0.0 && !S.att_v.empty())
    throw PdError{PD_ERR_INVALID_ARG, "bilateral rows run with frictionless contact only"};
  if (!(mu >= 0.0) || !std::isfinite(mu)) throw PdError{PD_ERR_INVALID_ARG, "need a finite friction coefficient >= 0"};
  S.mu_f = mu;
  S.c_last_K = S.c_last_active = 0;
  return PD_OK;
  PD_CATCH
}

int pd_contact_impulses(const pd_scene* scene, double* lam3, int capacity) {
  if (!scene || !lam3) {
    pdhot::g_last_error = "null argument";
    return PD_ERR_INVALID_ARG;
  }
  PD_TRY
  const Scene& S = scene->S;
  const int K = S.contact_on ? S.c_last_K : 0;
  const int n = std::min(K, std::max(capacity, 0));
  if (n > 0) {
    if (S.mu_f > 0.0) {
      PD_HIP(hipMemcpy(lam3, S.c_lam, 3 * n * sizeof(double), hipMemcpyDeviceToHost));
    } else {
      std::vector<double> l(n);
      PD_HIP(hipMemcpy(l.data(), S.c_lam, n * sizeof(double), hipMemcpyDeviceToHost));
      for (int c = 0; c < n; ++c) {
        lam3[3 * c] = l[c];
        lam3[3 * c + 1] = 0.0;
        lam3[3 * c + 2] = 0.0;
      }
    }
  }
  return PD_OK;
  PD_CATCH
}

int pd_step_forward(pd_scene* scene, const double* q_t, const double* v_t, const double* f_ext, const double* q0,
                    double* q_next, double* v_next, void* ckpt, pd_fwd_stats* stats, void* stream) {
  if (!scene || !q_t || !v_t || !q_next || !v_next) {
    pdhot::g_last_error = "null argument";
    return PD_ERR_INVALID_ARG;
  }
  Scene& S = scene->S;
  if (S.stale) {
    pdhot::g_last_error = "factor is stale: call pd_scene_factorize after pd_scene_set_material";
    return PD_ERR_STALE_FACTOR;
  }
  PD_TRY
  hipStream_t st = (hipStream_t)stream;
  const ElemArgs E = elem_args(S);
  const VertArgs V = vert_args(S);
  const SolveArgs A = solve_args(S);
  StepState T = step_state(S);
  const AdjState Ad = adj_state(S);
  RedArgs R = red_args(S);
  // prologue: (1/h) B_beta q_t element terms, then q~, c, q^0
  launch_to_lib(V, q_t, S.qt, 0, st);
  launch_elem_GtG(E, S.qt, S.nv, S.bV, S.contrib, st);
  launch_prologue(V, q_t, v_t, f_ext, q0, S.fwd_start, T, st);  // also clears the control words
  // contact rows of this step (Sec. 4.7): with rows, every global solve is
  // followed by the FB Newton solve and the column correction, which also
  // appends the Anderson columns
  const int K = S.contact_on ? contact_rows(S, st) : 0;
  const ContactArgs C = contact_args(S, K, false);
  if (K > 0) {
    R.nparts[kRedAA] = contact_apply_blocks(V.nf);
    T.fb = S.c_fb;
    T.fb_tol = S.fb_tol;
  }
  T.sig = S.sig_d;
  T.sigd = S.sigd_d;
  T.seq = ++S.seq_fwd;
  int k = 0;
  int chunk = S.iters_per_check > 0 ? S.iters_per_check : std::max(3, S.last_fwd_iters + 1);
  for (;;) {
    const int kend = std::min(k + chunk, S.kmax_fwd);
    for (; k < kend; ++k) {
      PD_TIMED(S, kKLocal, st, launch_local(E, T, R, S.q_cur, S.nv, V.nf, k, 1, st));
      PD_TIMED(S, kKGather, st, launch_gather_fwd(V, T, R, k, st));
      PD_TIMED(S, kKEb, st, launch_Eb(kModeFwd, V, A, T, Ad, R, nullptr, k, st));
      PD_TIMED(S, kKTop, st, launch_top(V, A, S.qhat, T.done, st));
      if (K > 0) {
        PD_TIMED(S, kKBottom, st, launch_bottom(kModePlain, V, A, T, Ad, R, S.b_cur, S.qhat, k, st));
        if (S.mu_f > 0.0) launch_contact_fr(V, C, S.qhat, T.done, st);
        else launch_contact_fb(V, C, S.qhat, T.done, st);
        launch_contact_apply_fwd(V, T, R, C, k, st);
      } else {
        PD_TIMED(S, kKBottom, st, launch_bottom(kModeFwd, V, A, T, Ad, R, nullptr, S.qhat, k, st));
      }
    }
    // the deciding kernel signals with its statistics; kernels still queued
    // behind it exit at once, so the host does not wait for them
    const bool decided = wait_signal(S, 0, T.seq, st);
    S.hctl[kCtlDone] = decided ? 1 : 0;
    if (decided) {
      S.hctl[kCtlIters] = S.sig_h[1];
      S.hctl[kCtlStatus] = S.sig_h[2];
      S.hctl[kCtlResets] = S.sig_h[3];
      S.hctl[kCtlNewton] = S.sig_h[4];
      for (int j = 0; j < 4; ++j) S.hdstat[j] = S.sigd_h[j];
    }
    kt_flush(S);
    if (S.hctl[kCtlDone] || k >= S.kmax_fwd) break;
    chunk = S.iters_per_check > 0 ? S.iters_per_check : 2;
  }
  // the epilogue is stream-ordered: without contact rows nothing more is read back
  launch_epilogue(V, T, q_next, v_next, (double*)ckpt, st);
  double* rec = (S.contact_on && ckpt) ? (double*)ckpt + (size_t)kCheckpointVecs * 3 * S.nv : nullptr;
  if (rec) launch_contact_ckpt(C, S.c_kmax, S.rest_e, rec, st);
  // restitution post-correction of the outgoing velocities (flags the rows in the record)
  if (K > 0 && S.rest_e >= 0.0) launch_contact_restitution(V, C, v_t, v_next, S.rest_e, rec, S.c_kmax, st);
  int n_active = 0;
  double fb_res = 0.0;
  const int nl = S.mu_f > 0.0 ? 3 * K : K;  // impulse entries (three per contact with friction)
  if (K > 0) {
    PD_HIP(hipMemcpyAsync(S.h_crec, S.c_lam, nl * sizeof(double), hipMemcpyDeviceToHost, st));
    PD_HIP(hipMemcpyAsync(S.h_crec + nl, S.c_fb, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    PD_HIP(hipMemcpyAsync(S.h_cbuf, S.c_flags, 4 * sizeof(int), hipMemcpyDeviceToHost, st));
    PD_HIP(hipStreamSynchronize(st));
  }
  PD_HIP(hipGetLastError());
  if (K > 0) {
    const int stride = nl / K;
    for (int c = 0; c < K; ++c) n_active += S.h_crec[stride * c] > 0.0;
    fb_res = S.h_crec[nl];
    if (S.mu_f > 0.0 && S.h_cbuf[2]) throw PdError{kErrContact, "a frictional contact Newton system was not positive definite"};
  }
  S.c_last_K = K;
  S.c_last_active = n_active;
  S.c_last_fb = fb_res;
  const int iters = S.hctl[kCtlIters], status = S.hctl[kCtlStatus];
  if (S.hctl[kCtlDone]) S.last_fwd_iters = iters;
  // launches that did work: local step and gather at k = 0..iters, the
  // interface right-hand side, interface solve and subdomain solve at
  // k = 0..iters-1 (at k = iters the gate decision ends the step)
  kt_work(S, kKLocal, iters + 1);
  kt_work(S, kKGather, iters + 1);
  kt_work(S, kKEb, iters);
  kt_work(S, kKTop, iters);
  kt_work(S, kKBottom, iters);
  if (stats) {
    stats->iters = iters;
    stats->aa_resets = S.hctl[kCtlResets];
    stats->status = status;
    stats->newton_capped = S.hctl[kCtlNewton];
    for (int j = 0; j < 4; ++j) stats->gate[j] = S.hdstat[j];
    stats->n_contacts = K;
    stats->n_active = n_active;
    stats->fb_res = fb_res;
  }
  if (!S.hctl[kCtlDone]) throw PdError{PD_ERR_HIP, "forward loop ended without a decision"};
  return status == 0 ? PD_OK : PD_NOT_CONVERGED;
  PD_CATCH
}

// The adjoint solution just computed becomes the newest of the (up to three)
// kept for the next call's start; the buffers rotate, the oldest is overwritten.
// the oldest history buffer becomes the newest (its copy of mu is made by the caller)
static void rotate_adjoint_history(Scene& S) {
  double* newest = S.mu_h3;
  S.mu_h3 = S.mu_h2;
  S.mu_h2 = S.mu_h1;
  S.mu_h1 = newest;
  S.adj_hist = std::min(S.adj_hist + 1, 3);
}

static void push_adjoint_history(Scene& S, hipStream_t st) {
  PD_HIP(hipMemcpyAsync(S.mu_h3, S.mu, 3 * (size_t)S.nv * sizeof(double), hipMemcpyDeviceToDevice, st));
  rotate_adjoint_history(S);
}

static void adjoint_solve(Scene& S, hipStream_t st, double tau_force, double* bstat_host, const double* ck,
                          bool warm, int n_active) {
  const ElemArgs E = elem_args(S);
  const VertArgs V = vert_args(S);
  const SolveArgs Sv = solve_args(S);
  AdjState Ad = adj_state(S);
  Ad.sig = S.sig_d;
  Ad.sigd = S.sigd_d;
  Ad.trstat = S.dstat + 4;
  Ad.seq = ++S.seq_adj;
  RedArgs R = red_args(S);
  // with active contact rows every preconditioner solve is projected onto
  // J_A mu = 0 and the per-row work moves to the correction kernel
  const bool con = n_active > 0;
  const ContactArgs C = contact_args(S, n_active, true);
  if (con) {
    R.nparts[kRedRZ0] = R.nparts[kRedRZ1] = R.nparts[kRedFix] = contact_apply_blocks(V.nf);
  }
  StepState T = step_state(S);
  T.done = Ad.done;  // plain solves inside the adjoint stop with it
  // the trust-region ratio belongs to the Neo-Hookean prox (Alg. 2)
  const int tr = S.energy == 0;
  if (tr) launch_tr_partials(E, V, R, ck, st);
  launch_bwd_elem(E, V, R, ck, S.eps_tr, tau_force, tr, S.jac, S.dstat + 4, S.ctl + kCtlAdj, 4, st);
  // the frictional adjoint is unsymmetric (a sliding contact's friction follows
  // its normal impulse): it runs the projected fixed point
  const bool pcg = S.adj_method == 0 && !(con && S.a_fric);
  if (pcg) {
    if (warm) {  // r = q bar - (A~ - K) mu0
      launch_apply_K(kModeAmK, E, V, Ad, R, S.jac, S.mu, 0, st);
      launch_adj_gather(kModeInit, V, Ad, R, 0, st);
    }
    PD_TIMED(S, kKEb, st, launch_Eb(kModePlain, V, Sv, T, Ad, R, S.r0, 0, st));
    PD_TIMED(S, kKTop, st, launch_top(V, Sv, S.z, T.done, st));
    if (con) {
      PD_TIMED(S, kKBottom, st, launch_bottom(kModePlain, V, Sv, T, Ad, R, S.r0, S.z, 0, st));
      launch_contact_proj(V, C, S.z, Ad.done, st);
      launch_contact_apply_adj(kModePCGInit, V, Ad, R, C, S.r0, 0, st);
    } else {
      PD_TIMED(S, kKBottom, st, launch_bottom(kModePCGInit, V, Sv, T, Ad, R, S.r0, S.z, 0, st));
    }
  }
  int it = 0;
  int chunk = std::max(2, S.last_adj_iters + 1);
  for (;;) {
    const int iend = std::min(it + chunk, S.kmax_bwd + 1);
    for (; it < iend; ++it) {
      if (pcg) {
        PD_TIMED(S, kKApplyK, st, launch_apply_K(kModePCG, E, V, Ad, R, S.jac, nullptr, it, st));
        launch_adj_gather(kModePCG, V, Ad, R, it, st);
        PD_TIMED(S, kKEb, st, launch_Eb(kModePCG, V, Sv, T, Ad, R, nullptr, it, st));
        PD_TIMED(S, kKTop, st, launch_top(V, Sv, S.z, T.done, st));
        if (con) {
          PD_TIMED(S, kKBottom, st, launch_bottom(kModePCGSolve, V, Sv, T, Ad, R, nullptr, S.z, it, st));
          launch_contact_proj(V, C, S.z, Ad.done, st);
          launch_contact_apply_adj(kModePCG, V, Ad, R, C, nullptr, it, st);
        } else {
          PD_TIMED(S, kKBottom, st, launch_bottom(kModePCG, V, Sv, T, Ad, R, nullptr, S.z, it, st));
        }
      } else {
        PD_TIMED(S, kKApplyK, st, launch_apply_K(kModeFixed, E, V, Ad, R, S.jac, nullptr, it, st));
        launch_adj_gather(kModeFixed, V, Ad, R, it, st);
        PD_TIMED(S, kKEb, st, launch_Eb(kModePlain, V, Sv, T, Ad, R, S.r0, it, st));
        PD_TIMED(S, kKTop, st, launch_top(V, Sv, S.z, T.done, st));
        if (con) {
          PD_TIMED(S, kKBottom, st, launch_bottom(kModePlain, V, Sv, T, Ad, R, S.r0, S.z, it, st));
          launch_contact_proj(V, C, S.z, Ad.done, st);
          launch_contact_apply_adj(kModeFixed, V, Ad, R, C, S.r0, it, st);
        } else {
          PD_TIMED(S, kKBottom, st, launch_bottom(kModeFixed, V, Sv, T, Ad, R, S.r0, S.z, it, st));
        }
      }
    }
    // the deciding kernel signals with its statistics (see the forward loop)
    const bool decided = wait_signal(S, 8, Ad.seq, st);
    S.hctl[kCtlAdj + 2] = decided ? 1 : 0;
    if (decided) {
      S.hctl[kCtlAdj] = S.sig_h[9];
      S.hctl[kCtlAdj + 1] = S.sig_h[10];
      for (int j = 0; j < 4; ++j) S.hdstat[4 + j] = S.sigd_h[4 + j];
      S.hdstat[16] = S.sigd_h[8];
    }
    kt_flush(S);
    if (S.hctl[kCtlAdj + 2] || it > S.kmax_bwd) break;
    chunk = std::max(2, S.last_adj_iters / 4);  // more than predicted: short follow-up chunks
  }
  if (bstat_host) {
    for (int j = 0; j < 4; ++j) bstat_host[j] = S.hdstat[4 + j];
    bstat_host[4] = S.hdstat[16];
  }
  const int n_it = S.hctl[kCtlAdj];
  if (S.hctl[kCtlAdj + 2]) S.last_adj_iters = n_it;
  const int n_solves = pcg ? n_it + 1 : n_it;
  kt_work(S, kKApplyK, n_it);
  kt_work(S, kKEb, n_solves);
  kt_work(S, kKTop, n_solves);
  kt_work(S, kKBottom, n_solves);
  if (!S.hctl[kCtlAdj + 2]) throw PdError{PD_ERR_HIP, "adjoint loop ended without a decision"};
}

int pd_step_backward(pd_scene* scene, const void* ckpt, const double* gq_next, const double* gv_next, double* gq_t,
                     double* gv_t, double* gf_ext, double* g_logE_accum, pd_bwd_stats* stats, void* stream) {
  if (!scene || !ckpt) {
    pdhot::g_last_error = "null argument";
    return PD_ERR_INVALID_ARG;
  }
  Scene& S = scene->S;
  if (S.stale) {
    pdhot::g_last_error = "factor is stale: call pd_scene_factorize after pd_scene_set_material";
    return PD_ERR_STALE_FACTOR;
  }
  PD_TRY
  hipStream_t st = (hipStream_t)stream;
  const ElemArgs E = elem_args(S);
  const VertArgs V = vert_args(S);
  const AdjState Ad = adj_state(S);
  const double* ck = (const double*)ckpt;
  // active contact rows of the step (their columns are built before the
  // adjoint buffers are set up: the builder uses them as scratch)
  const int n_active = S.contact_on ? contact_active(S, ck, st) : 0;
  // adjoint start: zero, or from the last solutions of this backward sweep;
  // with active rows the start must satisfy J_A mu = 0, so it is zero
  const int warm = n_active > 0 ? 0 : std::min(S.adj_warm, S.adj_hist);
  // the restitution post-correction's adjoint: v bar of the corrected rows
  // loses its normal part before the step (and dL/dv_t gains it after)
  const double* rec = S.contact_on ? ck + (size_t)kCheckpointVecs * 3 * S.nv : nullptr;
  const bool rest = S.contact_on && S.a_rest && gv_next;
  if (rest) {
    PD_HIP(hipMemcpyAsync(S.gv_rest, gv_next, 3 * (size_t)S.nv * sizeof(double), hipMemcpyDeviceToDevice, st));
    launch_restitution_adj_pre(V, rec, S.c_kmax, S.gv_rest, S.rest_s, st);
    gv_next = S.gv_rest;
  }
  launch_bwd_prologue(V, Ad, gq_next, gv_next, warm, S.mu_h1, S.mu_h2, S.mu_h3, st);
  double bs[5] = {0, 0, 0, 0, 0};
  adjoint_solve(S, st, -1.0, bs, ck, warm > 0, n_active);
  if (S.adj_warm > 0) push_adjoint_history(S, st);
  // the gradient routing is stream-ordered; the statistics were read with the last check
  launch_grad_elem(E, V, ck, S.jac, S.mu, S.contrib, g_logE_accum, st);
  if (S.n_mg > 0 && S.g_act) launch_muscle_grad(E, S.n_mg, S.mg_ptr, S.mg_tets, S.g_act, st);
  launch_grad_vert(V, S.mu, S.contrib, gv_next, gq_t, gv_t, gf_ext, st);
  if (rest && gv_t) launch_restitution_adj_post(V, rec, S.c_kmax, S.rest_s, gv_t, st);
  // sticking rows constrain the slip from q_t and sliding rows' friction
  // depends on it: their multipliers reach dL/dq_t
  if (n_active > 0 && S.a_fric) launch_contact_route(V, contact_args(S, n_active, true), S.a_kind, gq_t, st);
  PD_HIP(hipGetLastError());
  const int status = S.hctl[kCtlAdj + 1];
  if (stats) {
    stats->adj_iters = S.hctl[kCtlAdj];
    stats->status = status;
    stats->rho = bs[0]; stats->tau = bs[1]; stats->dphi_act = bs[2]; stats->dphi_mod = bs[3];
    stats->residual = bs[4];
    stats->n_active = n_active > 0 ? S.c_last_active : 0;
  }
  return status == 0 ? PD_OK : PD_NOT_CONVERGED;
  PD_CATCH
}

int pd_adjoint_reset(pd_scene* scene) {
  if (!scene) {
    pdhot::g_last_error = "null scene";
    return PD_ERR_INVALID_ARG;
  }
  scene->S.adj_hist = 0;
  return PD_OK;
}

int pd_debug_local_rhs(pd_scene* scene, const double* q, double* b, void* stream) {
  if (!scene || !q || !b) {
    pdhot::g_last_error = "null argument";
    return PD_ERR_INVALID_ARG;
  }
  Scene& S = scene->S;
  if (S.stale) { pdhot::g_last_error = "factor is stale"; return PD_ERR_STALE_FACTOR; }
  PD_TRY
  hipStream_t st = (hipStream_t)stream;
  const ElemArgs E = elem_args(S);
  const VertArgs V = vert_args(S);
  const StepState T = step_state(S);
  const RedArgs R = red_args(S);
  launch_to_lib(V, q, S.z, 0, st);
  launch_local(E, T, R, S.z, S.nv, V.nf, 0, 0, st);
  launch_gather_debug(V, S.contrib, S.wv, st);
  launch_from_lib(V, S.wv, b, 1, st);
  PD_HIP(hipStreamSynchronize(st));
  PD_HIP(hipGetLastError());
  return PD_OK;
  PD_CATCH
}

int pd_debug_apply_Ainv(pd_scene* scene, const double* r, double* x, void* stream) {
  if (!scene || !r || !x) {
    pdhot::g_last_error = "null argument";
    return PD_ERR_INVALID_ARG;
  }
  Scene& S = scene->S;
  if (S.stale) { pdhot::g_last_error = "factor is stale"; return PD_ERR_STALE_FACTOR; }
  PD_TRY
  hipStream_t st = (hipStream_t)stream;
  const VertArgs V = vert_args(S);
  launch_to_lib(V, r, S.r1, 1, st);
  solve_plain(S, S.r1, S.z, nullptr, st);
  launch_from_lib(V, S.z, x, 1, st);
  PD_HIP(hipStreamSynchronize(st));
  PD_HIP(hipGetLastError());
  return PD_OK;
  PD_CATCH
}

}  // extern "C"

namespace pdhot {
size_t apply_Ainv_ws_doubles(const pd_scene* scene) {
  const Scene& S = scene->S;
  return 6 * (size_t)S.nv + 3 * (size_t)std::max(1, S.L.nT) + 3 * (size_t)std::max(1, S.S.n_irows);
}

// x = A~^{-1} r as pd_debug_apply_Ainv, with every scratch vector of the solve
// (both library-order staging vectors, the interface right-hand side and the
// gathered interface solution) taken from ws: nothing is allocated and the
// host does not wait (the result is ordered on the stream).  Each of those
// vectors is written in full before it is read, so ws needs no clearing.
int apply_Ainv_ws(pd_scene* scene, const double* r, double* x, double* ws, size_t ws_cap, void* stream) {
  if (!scene || !r || !x || !ws) {
    g_last_error = "null argument";
    return PD_ERR_INVALID_ARG;
  }
  Scene& S = scene->S;
  if (S.stale) {
    g_last_error = "factor is stale";
    return PD_ERR_STALE_FACTOR;
  }
  const size_t need = apply_Ainv_ws_doubles(scene);
  if (need > ws_cap) {
    g_last_error = "the solve needs " + std::to_string(need) + " doubles of scratch, more than the " +
                   std::to_string(ws_cap) + " of the static workspace";
    return PD_ERR_INVALID_ARG;
  }
  PD_TRY
  hipStream_t st = (hipStream_t)stream;
  const VertArgs V = vert_args(S);
  SolveArgs A = solve_args(S);
  double* rl = ws;
  double* xl = ws + 3 * (size_t)S.nv;
  A.rT = xl + 3 * (size_t)S.nv;
  A.xsT = A.rT + 3 * (size_t)std::max(1, S.L.nT);
  const RedArgs R = red_args(S);
  StepState T = step_state(S);
  T.done = nullptr;
  const AdjState Ad = adj_state(S);
  launch_to_lib(V, r, rl, 1, st);
  launch_Eb(kModePlain, V, A, T, Ad, R, rl, 0, st);
  launch_top(V, A, xl, nullptr, st);
  launch_bottom(kModePlain, V, A, T, Ad, R, rl, xl, 0, st);
  launch_from_lib(V, xl, x, 1, st);
  PD_HIP(hipGetLastError());
  return PD_OK;
  PD_CATCH
}
}  // namespace pdhot

extern "C" {

int pd_debug_apply_K(pd_scene* scene, const double* q, double tau, const double* x, double* y, void* stream) {
  if (!scene || !q || !x || !y) {
    pdhot::g_last_error = "null argument";
    return PD_ERR_INVALID_ARG;
  }
  Scene& S = scene->S;
  if (S.stale) { pdhot::g_last_error = "factor is stale"; return PD_ERR_STALE_FACTOR; }
  PD_TRY
  hipStream_t st = (hipStream_t)stream;
  const ElemArgs E = elem_args(S);
  const VertArgs V = vert_args(S);
  const AdjState Ad = adj_state(S);
  const RedArgs R = red_args(S);
  // a checkpoint-shaped scratch whose q* slot holds q
  double* ck = S.ck_scratch;
  launch_to_lib(V, q, ck + 6 * (size_t)S.nv, 0, st);
  launch_bwd_elem(E, V, R, ck, S.eps_tr, tau, 0, S.jac, S.dstat + 4, nullptr, 0, st);
  launch_to_lib(V, x, S.p, 1, st);
  launch_apply_K(kModeDebug, E, V, Ad, R, S.jac, S.p, 0, st);
  launch_adj_gather(kModeDebug, V, Ad, R, 0, st);
  launch_from_lib(V, S.wv, y, 1, st);
  PD_HIP(hipStreamSynchronize(st));
  PD_HIP(hipGetLastError());
  return PD_OK;
  PD_CATCH
}

int pd_kernel_timer(pd_scene* scene, int kernel) {
  if (!scene || kernel < -1 || kernel >= kKCount) {
    pdhot::g_last_error = "invalid scene or kernel id";
    return PD_ERR_INVALID_ARG;
  }
  PD_TRY
  KernelTimer& T = scene->S.kt;
  if (T.ev.empty() && kernel >= 0) {
    T.ev.resize(2 * kTimerPairs);
    for (auto& e : T.ev) PD_HIP(hipEventCreateWithFlags(&e, kTimerEventFlags));
  }
  PD_HIP(hipDeviceSynchronize());
  T.which = kernel;
  T.head = 0;
  T.used = 0;
  T.total_ms = 0.0;
  T.launches = 0;
  T.working = 0;
  return PD_OK;
  PD_CATCH
}

int pd_kernel_timer_read(pd_scene* scene, double* total_ms, int64_t* launches, int64_t* working,
                         double* bytes_per_launch) {
  if (!scene) {
    pdhot::g_last_error = "null scene";
    return PD_ERR_INVALID_ARG;
  }
  PD_TRY
  Scene& S = scene->S;
  PD_HIP(hipDeviceSynchronize());
  kt_flush(S, true);
  if (total_ms) *total_ms = S.kt.total_ms;
  if (launches) *launches = S.kt.launches;
  if (working) *working = S.kt.working;
  if (bytes_per_launch) *bytes_per_launch = S.kt.which >= 0 ? kernel_bytes(S, S.kt.which) : 0.0;
  return PD_OK;
  PD_CATCH
}

}  // extern "C"

// ================================================================= batches
// Many scenes stepped together: every iteration stage is one launch across
// all scenes (kb_* kernels), each scene keeps its own buffers, reductions,
// Anderson window and done flag, and the host checks all scenes' flags with
// one copy per chunk of iterations.  Chunks can be captured once into HIP
// graphs and replayed.
struct pd_batch {
  std::vector<pd_scene*> scenes;
  SceneBundle* dB = nullptr;
  int* dbase[kBKKinds] = {};
  int nblk[kBKKinds] = {};
  // block counts per kind and scene, and the maps over the scenes whose loop
  // still runs (rebuilt at each host check of an eager loop): kinds x (ns + 1)
  // prefix sums, then the scene list
  std::vector<std::vector<int>> cnt;
  int* dsid_all = nullptr;
  int* dlive = nullptr;
  std::vector<int> hlive;
  int nlive = 0;
  bool live_on = false;
  int nblk_live[kBKKinds] = {};
  int block_local = kBlock, block_applyK = kBlock;
  int chunk = 0;        // iterations per host check (0 = adaptive)
  int use_graph = 0;
  int nlev = 0;         // separator levels of the deepest scene
  int* dctl = nullptr;  // ns x kCtlTotal
  double* ddstat = nullptr;
  int* hctl = nullptr;
  double* hdstat = nullptr;
  int last_fwd = 4, last_adj = 8;
  // the fewest iterations any scene took in the last call: an eager loop
  // checks first there (no scene is expected to stop earlier), then every
  // few iterations, so stopped scenes leave the launches soon
  int first_fwd = 4, first_adj = 8;
  std::vector<std::pair<long long, hipGraphExec_t>> graphs;
  // graphs are captured and replayed on the batch's own stream (the caller's
  // may be the legacy default stream, which cannot be captured), ordered
  // after and before the caller's work with events
  hipStream_t gstream = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  // per-launch timing of one kernel kind (eager launches only, not graphs)
  // and the algorithmic bytes of the work those launches did
  KernelTimer kt;
  double bytes_done = 0.0;
  // per-call argument tables of the per-step kernels (host copies pinned; a
  // call rewrites a host table only once the previous copy from it is done)
  BFwdIO *dfio = nullptr, *hfio = nullptr;
  BBwdIO *dbio = nullptr, *hbio = nullptr;
  hipEvent_t ev_fio = nullptr, ev_bio = nullptr;
  // each scene's factorization count when the bundles were built: a scene
  // refactorized since (new factor arrays) makes the batch rebuild them
  std::vector<int> gen;
};

namespace {

void batch_free_graphs(pd_batch& B) {
  for (auto& g : B.graphs) (void)hipGraphExecDestroy(g.second);
  B.graphs.clear();
}

// per-scene block counts of each kind for the current launch shapes, and the
// prefix tables the kernels search
void batch_layout(pd_batch& B) {
  const int ns = (int)B.scenes.size();
  for (int kind = 0; kind < kBKKinds; ++kind) {
    std::vector<int> base(ns + 1, 0);
    for (int s = 0; s < ns; ++s) {
      const Scene& S = B.scenes[s]->S;
      int n = 0;
      switch (kind) {
        case kBKLocal: n = (S.ne + B.block_local - 1) / B.block_local; break;
        case kBKApplyK: n = (S.ne + B.block_applyK - 1) / B.block_applyK; break;
        case kBKGather: n = vert_group_blocks(S.L.nf); break;
        case kBKEb: n = eb_blocks(S.L.nT); break;
        case kBKBottom: n = bottom_blocks(S.L.nB, S.L.nT); break;
        case kBKVert: n = (S.nv + kBlock - 1) / kBlock; break;
        case kBKVert8: n = vert_group_blocks(S.nv); break;
        case kBKElem: n = (S.ne + kBlock - 1) / kBlock; break;
        case kBKTR: n = tr_blocks(S.ne, S.L.nf); break;
        default: {
          const bool fwd = kind < kBKSepB;
          const int l = kind - (fwd ? kBKSepF : kBKSepB);  // level l + 1
          const SolveArgs A = solve_args(S);
          n = !fwd ? A.lev_nblk[l] : l >= 1 ? (A.lev_nrows[l] + kBlock / 64 - 1) / (kBlock / 64) : 0;
          break;
        }
      }
      base[s + 1] = base[s] + n;
    }
    B.nblk[kind] = base[ns];
    dfree(B.dbase[kind]);
    B.dbase[kind] = dalloc<int>(ns + 1);
    upload(B.dbase[kind], base);
    B.cnt.resize(kBKKinds);
    B.cnt[kind].assign(ns, 0);
    for (int s = 0; s < ns; ++s) B.cnt[kind][s] = base[s + 1] - base[s];
  }
  std::vector<int> ident(ns);
  for (int s = 0; s < ns; ++s) ident[s] = s;
  dfree(B.dsid_all);
  B.dsid_all = dalloc<int>(ns);
  upload(B.dsid_all, ident);
  dfree(B.dlive);
  B.dlive = dalloc<int>((size_t)kBKKinds * (ns + 1) + ns);
  B.hlive.assign((size_t)kBKKinds * (ns + 1) + ns, 0);
  B.live_on = false;
  B.nlev = 0;
  for (pd_scene* p : B.scenes) B.nlev = std::max(B.nlev, p->S.S.nlev);
  batch_free_graphs(B);
}

void batch_bundles(pd_batch& B) {
  std::vector<SceneBundle> h;
  for (pd_scene* p : B.scenes) {
    Scene& S = p->S;
    SceneBundle b;
    b.E = elem_args(S);
    b.V = vert_args(S);
    b.S = solve_args(S);
    b.St = step_state(S);
    b.A = adj_state(S);
    b.R = red_args(S);
    b.jac = S.jac;
    h.push_back(b);
  }
  dfree(B.dB);
  B.dB = dalloc<SceneBundle>(h.size());
  PD_HIP(hipMemcpy(B.dB, h.data(), h.size() * sizeof(SceneBundle), hipMemcpyHostToDevice));
}

// Before a batched step: every scene still fits the batch, and scenes
// refactorized since the bundles were built get fresh bundles and maps.
void batch_refresh(pd_batch& B) {
  bool rebuild = false;
  for (size_t s = 0; s < B.scenes.size(); ++s) {
    const Scene& S = B.scenes[s]->S;
    if (S.stale) throw PdError{PD_ERR_STALE_FACTOR, "scene factor is stale"};
    if (S.contact_on) throw PdError{PD_ERR_INVALID_ARG, "batched scenes run without obstacles"};
    if (S.n_mg > 0) throw PdError{PD_ERR_INVALID_ARG, "batched scenes run without muscles"};
    if (S.adj_method != 0) throw PdError{PD_ERR_INVALID_ARG, "batches run the PCG adjoint"};
    rebuild = rebuild || S.fact_gen != B.gen[s];
  }
  if (!rebuild) return;
  batch_bundles(B);
  batch_layout(B);
  for (size_t s = 0; s < B.scenes.size(); ++s) B.gen[s] = B.scenes[s]->S.fact_gen;
}

BatchMap bmap(const pd_batch& B, int kind) {
  const int ns = (int)B.scenes.size();
  if (B.live_on) return BatchMap{B.dB, B.dlive + (size_t)kind * (ns + 1), B.nlive, B.dlive + (size_t)kBKKinds * (ns + 1)};
  return BatchMap{B.dB, B.dbase[kind], ns, B.dsid_all};
}

int bnblk(const pd_batch& B, int kind) { return B.live_on ? B.nblk_live[kind] : B.nblk[kind]; }

// the map of a kind over every scene of the batch
BatchMap full_map(const pd_batch& B, int kind) {
  return BatchMap{B.dB, B.dbase[kind], (int)B.scenes.size(), B.dsid_all};
}

// After a host check of an eager loop: list only the scenes whose loop still
// runs (`running(s)`), so later launches carry no blocks of stopped scenes.
// The stream is idle (the check synchronised it), so the tables are replaced
// with a plain copy.  Graph replays keep the full maps.
template <typename F>
void batch_compact(pd_batch& B, F running) {
  if (B.use_graph) return;
  const int ns = (int)B.scenes.size();
  std::vector<int> sid;
  for (int s = 0; s < ns; ++s)
    if (running(s)) sid.push_back(s);
  const int n = (int)sid.size();
  if (n == (B.live_on ? B.nlive : ns) || n == 0) return;
  for (int kind = 0; kind < kBKKinds; ++kind) {
    int* base = B.hlive.data() + (size_t)kind * (ns + 1);
    base[0] = 0;
    for (int j = 0; j < n; ++j) base[j + 1] = base[j] + B.cnt[kind][sid[j]];
    B.nblk_live[kind] = base[n];
  }
  std::copy(sid.begin(), sid.end(), B.hlive.begin() + (size_t)kBKKinds * (ns + 1));
  PD_HIP(hipMemcpy(B.dlive, B.hlive.data(), B.hlive.size() * sizeof(int), hipMemcpyHostToDevice));
  B.nlive = n;
  B.live_on = true;
}

// the interface solve of every scene, level by level
void batch_sep(const pd_batch& B, int adjoint, hipStream_t st) {
  BatchMap Mf[kMaxLevels], Mb[kMaxLevels];
  int nf[kMaxLevels], nb[kMaxLevels];
  for (int l = 0; l < kMaxLevels; ++l) {
    Mf[l] = bmap(B, kBKSepF + l);
    Mb[l] = bmap(B, kBKSepB + l);
    nf[l] = bnblk(B, kBKSepF + l);
    nb[l] = bnblk(B, kBKSepB + l);
  }
  launch_b_sep(Mf, nf, Mb, nb, B.nlev, adjoint, st);
}

#define PD_BTIMED(B, id, st, call)                     \
  do {                                                 \
    const bool tm_ = !(B).use_graph && (B).kt.which >= 0; \
    if (tm_) kt_begin((B).kt, id, st);                 \
    call;                                              \
    if (tm_) kt_end((B).kt, id, st);                   \
  } while (0)

void batch_fwd_iter(pd_batch& B, int k, hipStream_t st) {
  PD_BTIMED(B, kKLocal, st, launch_b_local(bmap(B, kBKLocal), bnblk(B, kBKLocal), B.block_local, k, st));
  PD_BTIMED(B, kKGather, st, launch_b_gather_fwd(bmap(B, kBKGather), bnblk(B, kBKGather), k, st));
  PD_BTIMED(B, kKEb, st, launch_b_Eb(kModeFwd, bmap(B, kBKEb), bnblk(B, kBKEb), k, st));
  PD_BTIMED(B, kKTop, st, batch_sep(B, 0, st));
  PD_BTIMED(B, kKBottom, st, launch_b_bottom(kModeFwd, bmap(B, kBKBottom), bnblk(B, kBKBottom), k, st));
}

void batch_adj_iter(pd_batch& B, int it, hipStream_t st) {
  PD_BTIMED(B, kKApplyK, st,
            launch_b_apply_K(kModePCG, bmap(B, kBKApplyK), bnblk(B, kBKApplyK), B.block_applyK, it, st));
  launch_b_adj_gather(kModePCG, bmap(B, kBKGather), bnblk(B, kBKGather), it, st);
  PD_BTIMED(B, kKEb, st, launch_b_Eb(kModePCG, bmap(B, kBKEb), bnblk(B, kBKEb), it, st));
  PD_BTIMED(B, kKTop, st, batch_sep(B, 1, st));
  PD_BTIMED(B, kKBottom, st, launch_b_bottom(kModePCG, bmap(B, kBKBottom), bnblk(B, kBKBottom), it, st));
}

// iterations k0 .. k1-1 of a loop, replayed from a graph when enabled
template <typename F>
void batch_chunk(pd_batch& B, int loop, int k0, int k1, hipStream_t st, F iter) {
  if (!B.use_graph) {
    for (int k = k0; k < k1; ++k) iter(B, k, st);
    return;
  }
  const long long key = ((long long)loop << 40) | ((long long)k0 << 20) | (long long)k1;
  hipGraphExec_t exec = nullptr;
  for (auto& g : B.graphs)
    if (g.first == key) exec = g.second;
  if (!exec) {
    hipGraph_t graph = nullptr;
    PD_HIP(hipStreamBeginCapture(B.gstream, hipStreamCaptureModeThreadLocal));
    for (int k = k0; k < k1; ++k) iter(B, k, B.gstream);
    PD_HIP(hipStreamEndCapture(B.gstream, &graph));
    PD_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
    (void)hipGraphDestroy(graph);
    B.graphs.push_back({key, exec});
  }
  PD_HIP(hipEventRecord(B.ev_in, st));
  PD_HIP(hipStreamWaitEvent(B.gstream, B.ev_in, 0));
  PD_HIP(hipGraphLaunch(exec, B.gstream));
  PD_HIP(hipEventRecord(B.ev_out, B.gstream));
  PD_HIP(hipStreamWaitEvent(st, B.ev_out, 0));
}

// all scenes' control blocks and statistics to the host
void batch_flags(pd_batch& B, hipStream_t st) {
  const int ns = (int)B.scenes.size();
  launch_b_flags(BatchMap{B.dB, B.dbase[0], ns, B.dsid_all}, B.dctl, B.ddstat, st);
  PD_HIP(hipMemcpyAsync(B.hctl, B.dctl, sizeof(int) * kCtlTotal * ns, hipMemcpyDeviceToHost, st));
  PD_HIP(hipMemcpyAsync(B.hdstat, B.ddstat, sizeof(double) * 32 * ns, hipMemcpyDeviceToHost, st));
  PD_HIP(hipStreamSynchronize(st));
}

}  // namespace

extern "C" {

int pd_batch_create(pd_scene* const* scenes, int n, pd_batch** out) {
  if (!scenes || n <= 0 || !out) {
    pdhot::g_last_error = "null argument or empty batch";
    return PD_ERR_INVALID_ARG;
  }
  PD_TRY
  pd_batch* B = new pd_batch();
  try {
    for (int s = 0; s < n; ++s) {
      if (!scenes[s]) throw PdError{PD_ERR_INVALID_ARG, "null scene in batch"};
      if (scenes[s]->S.stale) throw PdError{PD_ERR_STALE_FACTOR, "scene factor is stale"};
      if (scenes[s]->S.adj_method != 0) throw PdError{PD_ERR_INVALID_ARG, "batches run the PCG adjoint"};
      if (scenes[s]->S.contact_on) throw PdError{PD_ERR_INVALID_ARG, "batched scenes run without obstacles"};
      if (scenes[s]->S.n_mg > 0) throw PdError{PD_ERR_INVALID_ARG, "batched scenes run without muscles"};
      B->scenes.push_back(scenes[s]);
    }
    batch_bundles(*B);
    batch_layout(*B);
    for (int s = 0; s < n; ++s) B->gen.push_back(scenes[s]->S.fact_gen);
    B->dctl = dalloc<int>((size_t)kCtlTotal * n);
    B->ddstat = dalloc<double>((size_t)32 * n);
    PD_HIP(hipHostMalloc((void**)&B->hctl, sizeof(int) * kCtlTotal * n));
    PD_HIP(hipHostMalloc((void**)&B->hdstat, sizeof(double) * 32 * n));
    B->dfio = dalloc<BFwdIO>(n);
    B->dbio = dalloc<BBwdIO>(n);
    PD_HIP(hipHostMalloc((void**)&B->hfio, sizeof(BFwdIO) * n));
    PD_HIP(hipHostMalloc((void**)&B->hbio, sizeof(BBwdIO) * n));
    PD_HIP(hipEventCreateWithFlags(&B->ev_fio, hipEventDisableTiming));
    PD_HIP(hipEventCreateWithFlags(&B->ev_bio, hipEventDisableTiming));
    PD_HIP(hipStreamCreateWithFlags(&B->gstream, hipStreamNonBlocking));
    PD_HIP(hipEventCreateWithFlags(&B->ev_in, hipEventDisableTiming));
    PD_HIP(hipEventCreateWithFlags(&B->ev_out, hipEventDisableTiming));
  } catch (...) {
    pd_batch_destroy(B);
    throw;
  }
  *out = B;
  return PD_OK;
  PD_CATCH
}

int pd_batch_destroy(pd_batch* B) {
  if (!B) return PD_OK;
  batch_free_graphs(*B);
  for (hipEvent_t e : B->kt.ev) (void)hipEventDestroy(e);
  dfree(B->dB);
  for (int k = 0; k < kBKKinds; ++k) dfree(B->dbase[k]);
  dfree(B->dsid_all);
  dfree(B->dlive);
  dfree(B->dctl);
  dfree(B->ddstat);
  if (B->hctl) (void)hipHostFree(B->hctl);
  if (B->hdstat) (void)hipHostFree(B->hdstat);
  dfree(B->dfio);
  dfree(B->dbio);
  if (B->hfio) (void)hipHostFree(B->hfio);
  if (B->hbio) (void)hipHostFree(B->hbio);
  if (B->ev_fio) (void)hipEventDestroy(B->ev_fio);
  if (B->ev_bio) (void)hipEventDestroy(B->ev_bio);
  if (B->ev_in) (void)hipEventDestroy(B->ev_in);
  if (B->ev_out) (void)hipEventDestroy(B->ev_out);
  if (B->gstream) (void)hipStreamDestroy(B->gstream);
  delete B;
  return PD_OK;
}

int pd_batch_config(pd_batch* B, int block_local, int block_applyK, int iters_per_check, int use_graph) {
  auto ok = [](int b) { return b == 64 || b == 128 || b == 256; };
  if (!B || !ok(block_local) || !ok(block_applyK) || iters_per_check < 0 || use_graph < 0 || use_graph > 1) {
    pdhot::g_last_error = "invalid batch configuration (blocks 64, 128 or 256)";
    return PD_ERR_INVALID_ARG;
  }
  PD_TRY
  B->block_local = block_local;
  B->block_applyK = block_applyK;
  B->chunk = iters_per_check;
  B->use_graph = use_graph;
  batch_layout(*B);
  return PD_OK;
  PD_CATCH
}

int pd_batch_capture_graph(pd_batch* B, int iters_per_chunk) {
  if (!B || iters_per_chunk < 0) {
    pdhot::g_last_error = "null batch or negative chunk";
    return PD_ERR_INVALID_ARG;
  }
  return pd_batch_config(B, B->block_local, B->block_applyK, iters_per_chunk, iters_per_chunk > 0 ? 1 : 0);
}

int pd_batch_step_forward(pd_batch* B, const double* const* q_t, const double* const* v_t,
                          const double* const* f_ext, const double* const* q0, double* const* q_next,
                          double* const* v_next, void* const* ckpt, pd_fwd_stats* stats, void* stream) {
  if (!B || !q_t || !v_t || !q_next || !v_next) {
    pdhot::g_last_error = "null argument";
    return PD_ERR_INVALID_ARG;
  }
  PD_TRY
  hipStream_t st = (hipStream_t)stream;
  const int ns = (int)B->scenes.size();
  batch_refresh(*B);
  PD_HIP(hipEventSynchronize(B->ev_fio));  // the last copy from the host table is done
  int kmax = 0;
  for (int s = 0; s < ns; ++s) {
    Scene& S = B->scenes[s]->S;
    if (!q_t[s] || !v_t[s] || !q_next[s] || !v_next[s]) throw PdError{PD_ERR_INVALID_ARG, "null scene input"};
    B->hfio[s] = BFwdIO{q_t[s], v_t[s], f_ext ? f_ext[s] : nullptr, q0 ? q0[s] : nullptr, q_next[s], v_next[s],
                        ckpt ? (double*)ckpt[s] : nullptr, S.fwd_start};
    kmax = std::max(kmax, S.kmax_fwd);
  }
  // caller's q_t in library order, B_beta q_t, prologue: one launch each over all scenes
  PD_HIP(hipMemcpyAsync(B->dfio, B->hfio, sizeof(BFwdIO) * ns, hipMemcpyHostToDevice, st));
  PD_HIP(hipEventRecord(B->ev_fio, st));
  launch_b_fwd_pre(full_map(*B, kBKVert), B->nblk[kBKVert], full_map(*B, kBKElem), B->nblk[kBKElem],
                   full_map(*B, kBKVert8), B->nblk[kBKVert8], B->dfio, st);
  int k = 0;
  // graph replay wants fixed chunk boundaries (one graph per chunk start)
  const int fixed = B->chunk > 0 ? B->chunk : (B->use_graph ? 4 : 0);
  int chunk = fixed > 0 ? fixed : std::max(3, B->first_fwd + 1);
  bool all = false;
  B->live_on = false;
  for (;;) {
    const int kend = std::min(k + chunk, kmax);
    batch_chunk(*B, 0, k, kend, st, batch_fwd_iter);
    k = kend;
    batch_flags(*B, st);
    all = true;
    for (int s = 0; s < ns; ++s) all = all && B->hctl[s * kCtlTotal + kCtlDone];
    if (all || k >= kmax) break;
    batch_compact(*B, [&](int s) { return !B->hctl[s * kCtlTotal + kCtlDone]; });
    chunk = fixed > 0 ? fixed : 2;
  }
  B->live_on = false;
  int worst = 0, most = 0;
  launch_b_fwd_post(full_map(*B, kBKVert), B->nblk[kBKVert], B->dfio, st);
  for (int s = 0; s < ns; ++s) {
    Scene& S = B->scenes[s]->S;
    const int* c = B->hctl + s * kCtlTotal;
    if (stats) {
      stats[s].iters = c[kCtlIters];
      stats[s].aa_resets = c[kCtlResets];
      stats[s].status = c[kCtlStatus];
      stats[s].newton_capped = c[kCtlNewton];
      for (int j = 0; j < 4; ++j) stats[s].gate[j] = B->hdstat[s * 32 + j];
      stats[s].n_contacts = 0;
      stats[s].n_active = 0;
      stats[s].fb_res = 0.0;
    }
    if (!c[kCtlDone]) throw PdError{PD_ERR_HIP, "batched forward loop ended without a decision"};
    worst = std::max(worst, c[kCtlStatus]);
    most = std::max(most, c[kCtlIters]);
    if (B->kt.which == kKSolve) B->bytes_done += c[kCtlIters] * kernel_bytes(S, kKSolve);
    if (B->kt.which == kKLocal) B->bytes_done += (c[kCtlIters] + 1) * kernel_bytes(S, kKLocal);
  }
  if (B->kt.which >= 0 && !B->use_graph) kt_flush(B->kt);
  B->last_fwd = most;
  B->first_fwd = ns > 0 ? B->hctl[kCtlIters] : 4;
  for (int s = 0; s < ns; ++s) B->first_fwd = std::min(B->first_fwd, B->hctl[s * kCtlTotal + kCtlIters]);
  PD_HIP(hipStreamSynchronize(st));
  PD_HIP(hipGetLastError());
  return worst == 0 ? PD_OK : PD_NOT_CONVERGED;
  PD_CATCH
}

int pd_batch_step_backward(pd_batch* B, const void* const* ckpt, const double* const* gq_next,
                           const double* const* gv_next, double* const* gq_t, double* const* gv_t,
                           double* const* gf_ext, double* const* g_logE_accum, pd_bwd_stats* stats, void* stream) {
  if (!B || !ckpt) {
    pdhot::g_last_error = "null argument";
    return PD_ERR_INVALID_ARG;
  }
  PD_TRY
  hipStream_t st = (hipStream_t)stream;
  const int ns = (int)B->scenes.size();
  int kmax = 0;
  bool any_warm = false;
  std::vector<int> warm(ns, 0);
  batch_refresh(*B);
  PD_HIP(hipEventSynchronize(B->ev_bio));
  for (int s = 0; s < ns; ++s) {
    Scene& S = B->scenes[s]->S;
    if (!ckpt[s]) throw PdError{PD_ERR_INVALID_ARG, "null checkpoint"};
    warm[s] = std::min(S.adj_warm, S.adj_hist);
    any_warm = any_warm || warm[s] > 0;
    // this step's mu goes to the oldest history buffer (rotated to the front after the launches)
    B->hbio[s] = BBwdIO{gq_next ? gq_next[s] : nullptr, gv_next ? gv_next[s] : nullptr, (const double*)ckpt[s],
                        S.mu_h1, S.mu_h2, S.mu_h3, gq_t ? gq_t[s] : nullptr, gv_t ? gv_t[s] : nullptr,
                        gf_ext ? gf_ext[s] : nullptr, g_logE_accum ? g_logE_accum[s] : nullptr,
                        S.adj_warm > 0 ? S.mu_h3 : nullptr, S.eps_tr, warm[s], S.energy == 0 ? 1 : 0};
    kmax = std::max(kmax, S.kmax_bwd);
  }
  // adjoint start, trust-region partials, element differentials: one launch each over all scenes
  PD_HIP(hipMemcpyAsync(B->dbio, B->hbio, sizeof(BBwdIO) * ns, hipMemcpyHostToDevice, st));
  PD_HIP(hipEventRecord(B->ev_bio, st));
  launch_b_bwd_pre(full_map(*B, kBKVert), B->nblk[kBKVert], full_map(*B, kBKTR), B->nblk[kBKTR],
                   full_map(*B, kBKElem), B->nblk[kBKElem], B->dbio, st);
  B->live_on = false;
  if (any_warm) {  // r = q bar - (A~ - K) mu0 (a zero mu0 gives r = q bar again)
    launch_b_apply_K(kModeAmK, bmap(*B, kBKApplyK), B->nblk[kBKApplyK], B->block_applyK, 0, st);
    launch_b_adj_gather(kModeInit, bmap(*B, kBKGather), B->nblk[kBKGather], 0, st);
  }
  PD_BTIMED(*B, kKEb, st, launch_b_Eb(kModePlain, bmap(*B, kBKEb), B->nblk[kBKEb], 0, st));
  PD_BTIMED(*B, kKTop, st, batch_sep(*B, 1, st));
  PD_BTIMED(*B, kKBottom, st, launch_b_bottom(kModePCGInit, bmap(*B, kBKBottom), B->nblk[kBKBottom], 0, st));
  int it = 0;
  const int fixed = B->chunk > 0 ? B->chunk : (B->use_graph ? 4 : 0);
  int chunk = fixed > 0 ? fixed : std::max(4, B->first_adj + 1);
  for (;;) {
    const int iend = std::min(it + chunk, kmax + 1);
    batch_chunk(*B, 1, it, iend, st, batch_adj_iter);
    it = iend;
    batch_flags(*B, st);
    bool all = true;
    for (int s = 0; s < ns; ++s) all = all && B->hctl[s * kCtlTotal + kCtlAdj + 2];
    if (all || it > kmax) break;
    batch_compact(*B, [&](int s) { return !B->hctl[s * kCtlTotal + kCtlAdj + 2]; });
    chunk = fixed > 0 ? fixed : 4;
  }
  B->live_on = false;
  int worst = 0, most = 0;
  // gradient routing (and the copy of mu into the history): one launch each over all scenes
  launch_b_bwd_post(full_map(*B, kBKElem), B->nblk[kBKElem], full_map(*B, kBKVert8), B->nblk[kBKVert8], B->dbio, st);
  for (int s = 0; s < ns; ++s) {
    Scene& S = B->scenes[s]->S;
    if (S.adj_warm > 0) rotate_adjoint_history(S);
    const int* c = B->hctl + s * kCtlTotal;
    const double* d = B->hdstat + s * 32;
    if (!c[kCtlAdj + 2]) throw PdError{PD_ERR_HIP, "batched adjoint loop ended without a decision"};
    if (stats) {
      stats[s].adj_iters = c[kCtlAdj];
      stats[s].status = c[kCtlAdj + 1];
      stats[s].rho = d[4]; stats[s].tau = d[5]; stats[s].dphi_act = d[6]; stats[s].dphi_mod = d[7];
      stats[s].residual = d[16];
      stats[s].n_active = 0;
      stats[s].pad = 0;
    }
    worst = std::max(worst, c[kCtlAdj + 1]);
    most = std::max(most, c[kCtlAdj]);
    if (B->kt.which == kKSolve) B->bytes_done += (c[kCtlAdj] + 1) * kernel_bytes(S, kKSolve);
    if (B->kt.which == kKApplyK) B->bytes_done += c[kCtlAdj] * kernel_bytes(S, kKApplyK);
  }
  if (B->kt.which >= 0 && !B->use_graph) kt_flush(B->kt);
  B->last_adj = most;
  B->first_adj = ns > 0 ? B->hctl[kCtlAdj] : 8;
  for (int s = 0; s < ns; ++s) B->first_adj = std::min(B->first_adj, B->hctl[s * kCtlTotal + kCtlAdj]);
  PD_HIP(hipStreamSynchronize(st));
  PD_HIP(hipGetLastError());
  return worst == 0 ? PD_OK : PD_NOT_CONVERGED;
  PD_CATCH
}


int pd_batch_kernel_timer(pd_batch* B, int kernel) {
  if (!B || kernel < -1 || kernel >= kKCount) {
    pdhot::g_last_error = "invalid batch or kernel id";
    return PD_ERR_INVALID_ARG;
  }
  PD_TRY
  KernelTimer& T = B->kt;
  if (T.ev.empty() && kernel >= 0) {
    T.ev.resize(2 * kTimerPairs);
    for (auto& e : T.ev) PD_HIP(hipEventCreateWithFlags(&e, kTimerEventFlags));
  }
  PD_HIP(hipDeviceSynchronize());
  T.which = kernel;
  T.head = 0;
  T.used = 0;
  T.total_ms = 0.0;
  T.launches = 0;
  T.working = 0;
  B->bytes_done = 0.0;
  return PD_OK;
  PD_CATCH
}

int pd_batch_kernel_timer_read(pd_batch* B, double* total_ms, int64_t* launches, double* bytes_done) {
  if (!B) {
    pdhot::g_last_error = "null batch";
    return PD_ERR_INVALID_ARG;
  }
  PD_TRY
  PD_HIP(hipDeviceSynchronize());
  kt_flush(B->kt, true);
  if (total_ms) *total_ms = B->kt.total_ms;
  if (launches) *launches = B->kt.launches;
  if (bytes_done) *bytes_done = B->bytes_done;
  return PD_OK;
  PD_CATCH
}

}  // extern "C"
