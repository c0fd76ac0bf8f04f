// Internal declarations shared by the host runtime and the HIP kernels of the
// pdhot library.  Nothing here is part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

typedef struct pd_scene pd_scene;

namespace pdhot {

constexpr int kBlock = 256;      // threads per workgroup for every kernel
constexpr int kMaxWindow = 5;    // largest Anderson window supported
constexpr int kCheckpointVecs = 4;

// ---------------------------------------------------------------- host layout
// Library vertex order: free vertices in nested-dissection order, the
// subdomains first (contiguous ranges), then the interface (all separator
// vertices), then the pinned vertices.
struct Layout {
  int nv = 0, ne = 0, nf = 0;
  int nsub = 0, nB = 0, nT = 0;          // nB = first interface vertex, nT = nf - nB
  std::vector<int> lib2orig, orig2lib;   // vertices
  std::vector<int> tet_lib2orig;         // tets (sorted for locality)
  std::vector<int> sub_begin;            // nsub + 1
  std::vector<std::vector<int>> Irows;   // per subdomain: interface rows (relative, sorted)
  // separator tree over the interface: node n owns interface rows
  // sep_begin[n] .. sep_begin[n + 1] - 1; nodes are sorted by level (1 = only
  // subdomains below, levels grow toward the root; the nodes at or above
  // `levels` are merged into one top node), and every level's rows are
  // contiguous from lev_begin[level - 1] (interface rows, nlev + 1 entries)
  int nlev = 0;
  std::vector<int> sep_begin, sep_level, sep_parent;
  std::vector<int> lev_begin;
  // per node: the interface rows of its ancestors that its elimination
  // couples to (sorted); the tree's block structure
  std::vector<std::vector<int>> sep_struct;
};

// Nested dissection by coordinate bisection with vertex separators; the
// interface is split into separator-tree levels, at most `levels` of them
// (1: the whole interface is one block).
void build_layout(int nv, int ne, const double* X, const int32_t* tets, const uint8_t* pinned, int max_sub,
                  int levels, Layout& L);

// Entries (diagonal included) of the Cholesky factor of A~ over the free
// vertices under a deep nested-dissection order (the same coordinate
// bisection taken down to subdomains of a few vertices): the size of the
// sparse factor the method's triangular solves would sweep.
double factor_nnz_nd(int nv, int ne, const double* X, const int32_t* tets, const uint8_t* pinned);


// ---------------------------------------------------------------- device scene
// Couplings of interface row i with the subdomains s it borders (row p of
// E_s = A_Ts A_ss^{-1}).  E is stored row-concatenated: the rows E_s[p, :] of
// all couplings of i follow each other from off.  Coupling c starts at entry
// pre of that range, maps to the subdomain rows b0 .. b0 + ns - 1, and its
// interface value sits at pos = ir_off[s] + p of the per-subdomain interface
// vectors.  Unused entries (c >= n) repeat pre = len and are never read.
constexpr int kMaxCoup = 8;
struct alignas(16) Cpl {
  int b0, pre, pos, pad;
};
struct alignas(16) ERow {
  long long off;
  int len, n;
};
// A subdomain row: its subdomain's first row b0, size ns, interface count nI
// and interface offset ir0, and the offsets of its rows of Z_s and E_s^T.
struct alignas(16) BRow {
  int b0, ns, nI, ir0;
};
struct alignas(16) BOff {
  long long zs, et;
};
// The ranges a subdomain-solve block stages in LDS: the right-hand-side rows
// z0 .. z0 + zn - 1 that its rows' subdomains span and their interface copies
// e0 .. e0 + en - 1 (zn = 0: the ranges exceed the LDS buffers, no staging).
struct alignas(16) BStage {
  int z0, zn, e0, en;
};

// The interface Schur complement S is eliminated over the separator tree.
// Node n (interface rows r0 .. r0 + s - 1, b coupled rows of higher levels,
// its struct) keeps, per row j, Z_n[j, :] (Z_n = F_nn^{-1} of its frontal
// block) followed by -E_n[:, j] (E_n = F_{struct,n} Z_n), s + b entries from
// zoff + j (s + b), applied to [y_n ; x_struct]: the backward solve of its
// rows.  The values x_struct sit at xs0 .. xs0 + b - 1 of the gathered
// interface vectors.
struct alignas(16) SepNode {
  long long zoff;
  int r0, s, b, xs0;
};
// A block of the backward solve: rows row0 .. row0 + nrows - 1 of one node.
struct alignas(16) SepBlk {
  int node, row0, nrows, pad;
};
// Interface row i's part of the forward solve: for every separator node c
// below it whose struct holds i (at position m), the row E_c[m, :] against
// y_c (interface rows src .. src + len - 1); the rows are concatenated from
// off in the order of the segments seg0 .. seg0 + nseg - 1.  The segment's
// slot is where the backward solve copies x_i for node c.
struct alignas(16) FRow {
  long long off;
  int seg0, nseg;
};
struct alignas(16) SSeg {
  int src, len, slot, pad;
};
constexpr int kMaxLevels = 8;  // separator-tree levels of the interface solve
constexpr int kDefaultIfaceLevels = 4;

struct DeviceSolve {
  // partitioned inverse of A~ over free vertices: subdomain blocks, then the
  // interface Schur complement over the separator tree
  double* Zs = nullptr;         // per subdomain n_s x n_s (row-major), = A_ss^{-1}
  double* Et = nullptr;         // per subdomain n_s x |I_s| (row v holds E_s[:, v]), E_s = A_Ts A_ss^{-1}
  double* E = nullptr;          // per interface row: E_s[p, :] of its couplings, concatenated
  double* ZE = nullptr;         // per separator node: rows [Z_n[j, :], -E_n[:, j]]
  double* FE = nullptr;         // per interface row: its forward rows E_c[m, :], concatenated
  SepNode* sep = nullptr;
  SepBlk* sblk = nullptr;       // backward blocks, level by level
  FRow* frow = nullptr;         // nT
  SSeg* sseg = nullptr;
  int* lev_row = nullptr;       // nlev + 1: interface rows of each level
  int* lev_blk = nullptr;       // nlev + 1: backward blocks of each level
  int nlev = 0;
  std::vector<int> lev_row_h, lev_blk_h;
  long long* zs_off = nullptr;  // nsub + 1
  long long* e_off = nullptr;   // nsub + 1 (same offsets for E and Et)
  int* sub_of = nullptr;        // nB
  int* sub_begin = nullptr;     // nsub + 1
  int* ir_off = nullptr;        // nsub + 1
  int* irows = nullptr;         // concatenated I_s (relative interface rows)
  int* rl_ptr = nullptr;        // nT + 1
  int* rl_sub = nullptr;
  int* rl_p = nullptr;
  double* rT = nullptr;         // 3 x nT
  Cpl* cpl = nullptr;           // nT x kMaxCoup
  ERow* erow = nullptr;         // nT
  BRow* brow = nullptr;         // nB
  BOff* boff = nullptr;         // nB
  BStage* bstage = nullptr;     // one per subdomain-solve block of subdomain rows
  double* xsT = nullptr;        // 3 x n_irows: interface values gathered per subdomain, then per separator node
  int n_irows = 0;              // slots: the subdomains' couplings, then every node's struct
  int max_coup = 0;
  size_t bytes = 0;
  double zs_entries = 0, e_entries = 0, ze_entries = 0, fe_entries = 0;
};

// Per-launch timing of one kernel with HIP events (roofline instrumentation).
struct KernelTimer {
  int which = -1;
  std::vector<hipEvent_t> ev;  // begin/end pairs, a ring: pending pairs head .. head + used - 1
  int head = 0;
  int used = 0;
  double total_ms = 0.0;
  long long launches = 0, working = 0;
};

struct Scene {
  // --- host copies
  int nv = 0, ne = 0, ninc = 0;
  std::vector<double> X;
  std::vector<int32_t> tets;
  std::vector<uint8_t> pinned;
  std::vector<double> logE;
  double nu = 0, rho = 0, alpha = 0, beta0 = 0;
  int energy = 0;  // 0: Neo-Hookean proximal map; 1: corotated + volume composite
  double h = 0, grav[3] = {0, 0, 0};
  int m = 0, kmax_fwd = 1000, kmax_bwd = 1000, adj_method = 0, max_sub = 0, iters_per_check = 0;
  int iface_levels = 0;
  double eps_rel = 1e-6, eps_abs = 1e-12, eps_adj = 1e-6, eps_tr = 0.1;
  bool stale = true;
  int fact_gen = 0;  // counts factorizations (a batch rebuilds its argument bundles when it changes)
  int last_fwd_iters = 4, last_adj_iters = 8;
  Layout L;
  double mu_bar = 0, lam_bar = 0, k_bar = 0, mu_ref = 0;
  double nnz_L = 0;  // entries of a nested-dissection Cholesky factor of A~ (algorithmic solve bytes)
  // means held across refactorizations (pd_scene_freeze_means): mu_bar, lam_bar, mu_ref
  bool frozen = false;
  double frozen_means[3] = {0, 0, 0};
  std::vector<double> hBm;  // host copy of the per-tet D_m^{-1} (library order, SoA)
  std::vector<int> htv;     // host copy of the tet vertex ids

  // --- device: element arrays (library tet order, SoA)
  int* tv = nullptr;        // 4 x ne
  int* tinc = nullptr;      // 4 x ne incidence positions
  double* Bm = nullptr;     // 9 x ne  (D_m^{-1}, row-major per tet)
  double* wV = nullptr;     // ne: w_e V_e
  double* bV = nullptr;     // ne: beta_e V_e / h
  double* muV = nullptr;    // ne: mu_e V_e   (primal objective)
  double* lamV = nullptr;   // ne: lam_e V_e
  int* tet_orig = nullptr;  // ne
  double* Vw = nullptr;     // 4 x ne warm-start rotations (unit quaternions)
  double* rw = nullptr;     // 3 x ne warm-start stretch ratios
  // --- device: vertex arrays (library order)
  int* v_orig = nullptr;    // nv
  double* mass = nullptr;   // nv
  double* rest = nullptr;   // 3 x nv SoA
  double* cpin = nullptr;   // 3 x nv: -A~_{free,pinned} q_pinned
  int* inc_ptr = nullptr;   // nf + 1
  DeviceSolve S;
  // --- device: iteration state (3 x nv SoA)
  double* contrib = nullptr;  // 3 x ninc
  double *qt = nullptr, *vt = nullptr, *qtil = nullptr, *c = nullptr;
  double *q_cur = nullptr, *q_prev = nullptr, *b_cur = nullptr, *b_prev = nullptr, *qhat = nullptr;
  double *q_last = nullptr, *g_last = nullptr, *dQ = nullptr, *dG = nullptr;  // dQ, dG: m x 3 x nv
  int* ctl = nullptr;           // device control block (see kernels)
  double* dstat = nullptr;      // device statistics
  int* hctl = nullptr;          // pinned host mirror of ctl
  double* hdstat = nullptr;     // pinned host mirror of dstat
  // decision signals: the kernel that decides a loop writes its statistics and
  // then a sequence number into mapped host memory, so the host learns the
  // decision without draining the stream
  int* sig_h = nullptr;         // [0] forward sequence, [1..4] iters, status, resets, newton cap;
                                // [8] adjoint sequence, [9] iters, [10] status
  int* sig_d = nullptr;
  double* sigd_h = nullptr;     // [0..3] gate norms, [4..7] trust-region figures, [8] adjoint residual
  double* sigd_d = nullptr;
  int seq_fwd = 0, seq_adj = 0;
  // deterministic reductions
  double* red_part = nullptr;
  double* red_fin = nullptr;
  int red_max_parts = 0;
  // backward
  double* jac = nullptr;       // 23 x ne compact prox differential (rows kJac*)
  double *mu = nullptr, *r0 = nullptr, *r1 = nullptr, *z = nullptr, *p = nullptr, *Ap = nullptr, *wv = nullptr,
         *qbar = nullptr;
  // adjoint warm start: the last three adjoint solutions of a backward sweep (newest first)
  double *mu_h1 = nullptr, *mu_h2 = nullptr, *mu_h3 = nullptr;
  int adj_hist = 0, adj_warm = 0;
  int fwd_start = 0;  // 0: q0 = q_t; 1: q0 = q_t + h v_t (when the caller passes no q0)
  double* ck_scratch = nullptr;  // 12 x nv (diagnostic K apply)
  KernelTimer kt;
  // --- contact with static obstacles (off until obstacles are set)
  bool contact_on = false;
  int n_planes = 0, n_boxes = 0, c_kmax = 0;
  double d_c = 0.0, fb_tol = 1e-10;
  double* obs = nullptr;  // planes (4 each), then boxes (6 each)
  // rows of the current forward step
  int *c_v = nullptr, *c_slot = nullptr, *c_flags = nullptr;
  double *c_n = nullptr, *c_g = nullptr, *c_lam = nullptr, *c_s = nullptr, *c_W = nullptr, *c_fb = nullptr;
  // active rows of the current backward step and the inverse of their Delassus block
  int *a_v = nullptr, *a_slot = nullptr;
  double *a_n = nullptr, *a_s = nullptr, *a_Winv = nullptr;
  double* c_Lg = nullptr;  // dense factorizations beyond the LDS size
  // column cache: a_v = A~^{-1} e_v (free rows) for up to col_cap vertices
  double* cols = nullptr;
  int col_cap = 0, cols_used = 0;
  std::vector<int> slot_of, vert_of_slot;
  int* h_cbuf = nullptr;        // pinned: flags (4), vertex ids, slots
  double* h_crec = nullptr;     // pinned: one checkpoint contact record
  int c_last_K = 0, c_last_active = 0, c_cols_built = 0;
  double c_last_fb = 0.0;
  // Coulomb friction (mu_f > 0): scratch of the frictional Newton, and the
  // adjoint rows' multiplier directions, diagonals and kinds
  double mu_f = 0.0;
  double* c_frw = nullptr;
  int* c_fri = nullptr;
  double *a_nb = nullptr, *a_dg = nullptr, *c_slip = nullptr;
  int* a_kind = nullptr;
  bool a_fric = false;  // the current backward step has friction rows
  // bilateral rows (attachments; frictionless contact only): library vertex
  // ids, unit directions and offsets, appended to every step's rows
  std::vector<int> att_v;
  std::vector<double> att_n, att_g;
  int* c_kind = nullptr;       // kmax: 1 for a bilateral row of the current step
  // restitution post-correction (rest_e < 0: off)
  double rest_e = -1.0;
  double* gv_rest = nullptr;   // 3 x nv (caller order): v bar after the correction's adjoint
  double* rest_s = nullptr;    // kmax per-row products of that adjoint
  bool a_rest = false;         // the current backward step has corrected rows
  std::vector<int> a_rows;     // record indices of the current backward step's active rows
  int a_K = 0;                 // rows in that record
  // --- muscle fibres (off until pd_scene_set_muscles): host copies in the
  // caller's tet order, device arrays in library order
  int n_mg = 0;
  double w_m = 0.0;
  std::vector<int> hmgroup;
  std::vector<double> hmfib;
  double* mus = nullptr;     // 4 x ne: fibre (3), w_m V_e (0: passive)
  int* mgrp = nullptr;       // ne: group (0 for passive tets, whose w_m V_e is 0)
  double* act = nullptr;     // n_mg activations
  double* mjac = nullptr;    // 4 x ne fibre differential at q*
  double* mgt = nullptr;     // ne per-tet terms of dL/da
  int* mg_ptr = nullptr;     // n_mg + 1: each group's tets (library order)
  int* mg_tets = nullptr;
  double* g_act = nullptr;   // caller's accumulator of dL/da (may be null)
};

void set_last_error(const std::string& m);
// The global solve with caller-provided scratch (the allocation-free entry point)
size_t apply_Ainv_ws_doubles(const pd_scene* scene);
int apply_Ainv_ws(pd_scene* scene, const double* r, double* x, double* ws, size_t ws_cap, void* stream);

}  // namespace pdhot
