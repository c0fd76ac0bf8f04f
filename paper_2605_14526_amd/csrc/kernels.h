// Kernel argument blocks and launchers of the pdhot HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>

#include "pd_internal.h"

namespace pdhot {

enum {
  kModeFwd = 0,
  kModePlain = 1,
  kModeDebug = 2,
  kModePCG = 3,
  kModePCGInit = 4,
  kModeFixed = 5,
  kModeAmK = 6,   // (A~ - K) x element terms (adjoint warm start)
  kModeInit = 7,  // r = q bar - (A~ - K) mu (adjoint warm start)
  kModePCGSolve = 8  // PCG step whose preconditioned residual is corrected afterwards (contact projection)
};

// device control block (int): done flag, final iteration count, status,
// Anderson resets, Newton iteration maximum, then two Anderson states
// {nonempty, ncols, head, pad} selected by iteration parity; from kCtlAdj the
// adjoint's {iterations, status, done}.
enum { kCtlDone = 0, kCtlIters = 1, kCtlStatus = 2, kCtlResets = 3, kCtlNewton = 4, kCtlAA = 8, kCtlSize = 16,
       kCtlAdj = 16, kCtlTotal = 24 };

// Deterministic cross-block reductions without atomics: each producing block
// writes its partial vector; the first kernel that needs the total sums all
// partials in a fixed order (lane l of the first wave takes partials l,
// l + 64, ..., then the wave's butterfly) and its block 0 stores the total in
// `fin` for the kernels after it.
enum { kRedGate = 0, kRedAA = 1, kRedPW = 2, kRedRZ0 = 3, kRedRZ1 = 4, kRedTR = 5, kRedFix = 6, kRedSites = 7 };
constexpr int kRedWidth = 32;   // doubles per partial
constexpr int kFinStride = 64;  // doubles per site in the final buffer
#ifndef PD_BOTTOM_THREADS
#define PD_BOTTOM_THREADS 512
#endif
#ifndef PD_BOTTOM_CHUNK
#define PD_BOTTOM_CHUNK 1
#endif
#ifndef PD_BOTTOM_CHUNK_E
#define PD_BOTTOM_CHUNK_E 1
#endif
#ifndef PD_EB_CHUNK
#define PD_EB_CHUNK 2
#endif
#ifndef PD_EB_RPW
#define PD_EB_RPW 4
#endif
#ifndef PD_TOP_CHUNK
#define PD_TOP_CHUNK 8
#endif
#ifndef PD_ELEM_BLOCK
#define PD_ELEM_BLOCK 256
#endif
#ifndef PD_BOTTOM_RPW
#define PD_BOTTOM_RPW 4
#endif
constexpr int kBottomThreads = PD_BOTTOM_THREADS;  // subdomain solve: 64 threads per wave
// subdomain rows per wave: a wave walks kBottomRowsPerWave rows together (all
// their loads of a trip before the arithmetic), rows of one block are consecutive
constexpr int kBottomRowsPerWave = PD_BOTTOM_RPW;
constexpr int kBottomRows = (kBottomThreads / 64) * kBottomRowsPerWave;  // subdomain rows per block
// Row walks of the solve kernels: a wave takes its row in chunks of 64 x chunk
// entries and each lane requests all of its chunk's entries before it uses
// any, so a chunk costs one memory round trip.
constexpr int kBottomChunk = PD_BOTTOM_CHUNK;     // subdomain solve, Z_s rows
constexpr int kBottomChunkE = PD_BOTTOM_CHUNK_E;  // subdomain solve, E_s^T rows
constexpr int kEbChunk = PD_EB_CHUNK;          // interface right-hand side (E_s rows)
constexpr int kEbRowsPerWave = PD_EB_RPW;       // interface rows walked together by one wave
constexpr int kEbRows = (kBlock / 64) * kEbRowsPerWave;  // interface rows per block of that kernel
constexpr int kTopChunk = PD_TOP_CHUNK;        // interface solve, rows of wide separator blocks
// Interface solve over the separator tree: a backward block takes kSepRows
// rows of one node (kSepRowsPerWave per wave, chunks of 64 x kSepChunk), or
// for a wide node (s + b >= kSepWide) 4 rows, one per wave, in chunks of
// 64 x kTopChunk; the node's [y_n ; x_struct] is staged in LDS kSepTile
// entries at a time.  A forward row takes chunks of 64 x kSepFwdChunk.
// (2 rows per wave, chunks of 4: on the 64-scene identification batch 1842
// against 1778 scene-steps/s at 4 and 2, 1558 at 8 and 1, 1795-1830 with one
// row per wave)
#ifndef PD_SEP_RPW
#define PD_SEP_RPW 2
#endif
#ifndef PD_SEP_CHUNK
#define PD_SEP_CHUNK 4
#endif
#ifndef PD_SEP_FWD_CHUNK
#define PD_SEP_FWD_CHUNK 4
#endif
constexpr int kSepRowsPerWave = PD_SEP_RPW;
constexpr int kSepRows = (kBlock / 64) * kSepRowsPerWave;
constexpr int kSepChunk = PD_SEP_CHUNK;
constexpr int kSepFwdChunk = PD_SEP_FWD_CHUNK;
constexpr int kSepWide = 1536;
constexpr int kSepTile = 2048;
constexpr int kSepMaxSeg = 56;  // separator nodes whose struct may hold one interface row
// LDS buffers of the subdomain solve: right-hand-side rows and interface
// copies a block stages for its rows (three axes each)
constexpr int kStageZ = 768;
constexpr int kStageE = 640;
// Row-walking kernels ask for at most 4 waves per SIMD: the compiler may then
// spend up to 128 registers on a chunk's loads instead of trading them for
// occupancy by waiting between them (the grids need no more than 4 anyway).
// The interface right-hand side takes 3 and up to 168 registers: its PCG form
// holds 7 loads per entry and would spill at 128, and its grid (one wave per
// interface row) is the smallest of the three.
#define PD_ROW_WALK __attribute__((amdgpu_waves_per_eu(4, 4)))
#define PD_ROW_WALK_EB __attribute__((amdgpu_waves_per_eu(3, 3)))
constexpr int kElemBlock = PD_ELEM_BLOCK;  // tets per workgroup of the single-scene local step and K apply

struct RedArgs {
  double* part;    // per site: kRedWidth x max_parts (value j of partial b at [j][b])
  double* fin;     // per site: kFinStride doubles
  int max_parts;
  int nparts[kRedSites];  // producing blocks of each site
};

struct ElemArgs {
  int ne, ninc;
  const int* tv;      // 4 x ne library vertex ids
  const int* tinc;    // 4 x ne positions in the incidence order (-1 for pinned)
  const double* Bm;   // 9 x ne
  const double* wV;
  const double* bV;
  const double* muV;
  const double* lamV;
  const int* tet_orig;
  double* Vw;         // 4 x ne warm-start rotations as unit quaternions {w, x, y, z} (local step)
  double* rw;         // 3 x ne warm-start stretch ratios (the composite keeps its volume multiplier in row 0)
  double mu_bar, lam_bar, k_bar;
  int energy;         // 0: Neo-Hookean proximal map; 1: corotated + volume composite
  // muscle fibres (null when the scene has none): 4 x ne {m_x, m_y, m_z, w_m V_e} (w_m V_e = 0 for a
  // passive tet), the tet's group, the groups' activations, and 4 x ne {f^, l/|f|} at q* (backward)
  const double* mus;
  const int* mgrp;
  const double* act;
  double* mjac;
  double* mgt;        // ne: a muscle tet's term of dL/da (backward scratch)
};

struct VertArgs {
  int nv, nf, ne, ninc;
  const int* v_orig;
  const double* mass;
  const double* rest;
  const double* cpin;
  const int* inc_ptr;
  double h, alpha;
  double grav[3];
};

struct SolveArgs {
  int nsub, nB, nT;
  const int* sub_of;        // nB: subdomain of each subdomain row
  const int* sub_begin;     // nsub + 1
  const double* Zs;         // per subdomain ns x ns
  const long long* zs_off;
  const double* Et;         // per subdomain ns x nI (row v: E_s[:, v])
  const double* E;          // per interface row: E_s[p, :] of its couplings, concatenated
  const long long* e_off;
  const int* ir_off;        // nsub + 1
  const int* irows;         // concatenated interface rows of each subdomain
  const int* rl_ptr;        // nT + 1: couplings of each interface row
  const int* rl_sub;        // subdomain of each coupling
  const int* rl_p;          // row of E_s of each coupling
  int nlev;                 // separator-tree levels of the interface solve
  const int* lev_row;       // nlev + 1
  const int* lev_blk;       // nlev + 1
  const SepNode* sep;
  const SepBlk* sblk;
  const double* ZE;
  const FRow* frow;
  const SSeg* sseg;
  const double* FE;
  double* rT;               // 3 x nT interface right-hand side (the forward solve's y in place)
  int lev_nrows[kMaxLevels];  // host copies for the launchers: rows and backward blocks per level
  int lev_nblk[kMaxLevels];
  const Cpl* cpl;           // nT x kMaxCoup coupling descriptors
  const ERow* erow;         // nT: the row's couplings in E (row-concatenated)
  const BRow* brow;         // nB subdomain-row descriptors
  const BOff* boff;
  const BStage* bstage;     // per subdomain-solve block: the ranges it stages in LDS
  double* xsT;              // 3 x n_irows interface solution gathered per subdomain and separator node
  int n_irows;
};

struct StepState {
  int m, kmax;
  double eps_rel, eps_abs;
  double *contrib, *qt, *vt, *qtil, *c;
  double *q_cur, *q_prev, *b_cur, *b_prev, *qhat;
  double *q_last, *g_last, *dQ, *dG;
  int* ctl;
  int* done;
  double* dstat;
  const double* fb = nullptr;  // contact: FB residual of the last contact solve (null without contact rows)
  double fb_tol = 0.0;
  int* sig = nullptr;          // mapped host signal block (null: no signal)
  double* sigd = nullptr;
  int seq = 0;
};

struct AdjState {
  int kmax;
  double eps;
  double *contrib, *qbar, *mu, *z, *p, *Ap, *w;
  double *r0, *r1;  // residual, double-buffered by iteration parity (PCG reads r^k while writing r^{k+1});
                    // r0 also holds q bar + K mu (fixed point)
  int* ctl;       // [iters, status]
  int* done;
  double* dstat;  // [residual]
  int* sig = nullptr;             // mapped host signal block (null: no signal)
  double* sigd = nullptr;
  const double* trstat = nullptr;  // trust-region figures, copied into the signal
  int seq = 0;
};

// Contact rows of one step (forward: every candidate row; adjoint: the active
// rows) and the cached columns a = A~^{-1} e_v of their vertices.
constexpr int kContactThreads = 1024;
constexpr int kMaxContactRows = 512;  // candidate rows per step
constexpr int kMaxNewtonRows = 176;   // rows of one dense system factored in LDS (larger: global scratch)
constexpr int kMaxObstacles = 8;
constexpr int kFBMaxIter = 30;
constexpr double kFBTol = 1e-14;
constexpr double kOmegaMin = 1e-12;
constexpr int kFrMaxIter = 50;          // Newton steps of one frictional contact solve
constexpr int kMaxAdjRows = 3 * kMaxContactRows;  // adjoint rows with friction (at most three per contact)
constexpr int kFrWork = 48;             // doubles of friction scratch per contact
struct ContactArgs {
  int K;
  int nf;
  const int* v;        // K library vertex ids
  const double* n;     // 3K unit normals, row-major (n[3c + a]); adjoint: the rows' constraint directions
  const double* g;     // K offsets: gap = n . q_v - g
  const int* slot;     // K column slots
  const double* cols;  // columns: a_v at cols[slot * nf + row]
  const double* W;     // K x K Delassus operator (forward; with friction the scalar block G_cd = a_{v_c}[v_d])
                       // or the inverse of the adjoint rows' coupling matrix
  double* lam;         // K impulses (3K with friction: normal, t1, t2)
  double* s;           // 3K: the world impulse of each row (forward) or u_r c_r (adjoint projection)
  double* fb;          // [0] FB residual, [1] Newton iterations of the last solve
  int* flags;          // [0] candidate rows found, [1] unused, [2] factor not SPD / singular
  double* Lg;          // global scratch for dense factorizations larger than the LDS ones
  // Coulomb friction (mu > 0)
  double mu = 0.0;
  const double* qt = nullptr;   // q_t in library order (slip start)
  double* frw = nullptr;        // kFrWork x K doubles of scratch
  int* fri = nullptr;           // 6K ints of scratch
  const double* nb = nullptr;   // adjoint: 3 per row, the directions along which the multipliers act
                                // (null: n); with friction they differ from n on sliding normal rows
  const double* dg = nullptr;   // adjoint: per-row diagonal of the coupling matrix (null: none)
  const int* kind = nullptr;    // forward: K row kinds, 1 = bilateral (equality, free multiplier); null: none
};
struct ObsArgs {
  int n_planes, n_boxes;
  const double* planes;  // 4 per plane: unit normal, offset
  const double* boxes;   // 6 per box: lo xyz, hi xyz
  double d_c, h;
  int one_per_vertex = 0;  // keep only the closest qualifying obstacle of each vertex (friction)
};

// Everything a kernel needs about one scene, for launches that span many
// scenes (one device array entry per scene).
// Rows of the per-tet compact prox differential (SoA, stride n_e): U and V as
// unit quaternions, D (6), the pair coefficients c1, c2 (3 + 3) and s* (3)
enum { kJacV = 4, kJacD = 8, kJacC1 = 14, kJacC2 = 17, kJacS = 20, kJacRows = 23 };

struct SceneBundle {
  ElemArgs E;
  VertArgs V;
  SolveArgs S;
  StepState St;
  AdjState A;
  RedArgs R;
  double* jac;
};

// Per-call arguments of one scene of a batched step (a device table with one
// entry per scene, written by the host at the start of each call): the
// caller's arrays of the forward step ...
struct BFwdIO {
  const double *q_t, *v_t, *f, *q0;
  double *q_next, *v_next, *ckpt;
  int inertial;
};

// ... and of the backward step (h1..h3: the adjoint history the start is
// extrapolated from; mu_copy: where this step's mu is kept for the next one)
struct BBwdIO {
  const double *gq, *gv, *ck, *h1, *h2, *h3;
  double *gq_t, *gv_t, *gf, *g_logE, *mu_copy;
  double eps_tr;
  int warm, tr;
};

// Block-to-scene map of a batched launch over ns of the batch's scenes: the
// j-th of them (scene sid[j]) owns blocks base[j] .. base[j+1]-1 (empty
// ranges allowed).  Launches after a host check list only the scenes whose
// loop still runs.
struct BatchMap {
  const SceneBundle* B;
  const int* base;
  int ns;
  const int* sid;
};

// block-map kinds of a batch: the stages, then the forward (kBKSepF + l - 1)
// and backward (kBKSepB + l - 1) launches of interface-solve level l
// and (per step, not per iteration) one thread per vertex, eight per vertex,
// one per tet, and the trust-region partials' grid
enum { kBKLocal = 0, kBKGather = 1, kBKEb = 2, kBKBottom = 3, kBKApplyK = 4, kBKSepF = 5, kBKSepB = kBKSepF + kMaxLevels,
       kBKVert = kBKSepB + kMaxLevels, kBKVert8, kBKElem, kBKTR, kBKKinds };

void launch_b_local(const BatchMap& M, int nblk, int block, int k, hipStream_t s);
void launch_b_gather_fwd(const BatchMap& M, int nblk, int k, hipStream_t s);
void launch_b_Eb(int mode, const BatchMap& M, int nblk, int k, hipStream_t s);
// the interface solve over the separator tree: per level l (1..nlev) the
// maps and block counts of its forward (l >= 2) and backward launches
void launch_b_sep(const BatchMap* Mf, const int* nblk_f, const BatchMap* Mb, const int* nblk_b, int nlev,
                  int adjoint, hipStream_t s);
void launch_b_bottom(int mode, const BatchMap& M, int nblk, int k, hipStream_t s);
void launch_b_apply_K(int mode, const BatchMap& M, int nblk, int block, int it, hipStream_t s);
// the per-step kernels of a batch: before the forward loop (caller's q_t to
// library order, B_beta q_t, prologue), after it (epilogue), before the
// adjoint loop (adjoint start, trust-region partials, element differentials)
// and after it (gradient routing); maps of kinds kBKVert, kBKVert8, kBKElem,
// kBKTR with their block counts
void launch_b_fwd_pre(const BatchMap& Mv, int nv_blk, const BatchMap& Me, int ne_blk, const BatchMap& Mv8,
                      int nv8_blk, const BFwdIO* io, hipStream_t s);
void launch_b_fwd_post(const BatchMap& Mv, int nv_blk, const BFwdIO* io, hipStream_t s);
void launch_b_bwd_pre(const BatchMap& Mv, int nv_blk, const BatchMap& Mtr, int ntr_blk, const BatchMap& Me,
                      int ne_blk, const BBwdIO* io, hipStream_t s);
void launch_b_bwd_post(const BatchMap& Me, int ne_blk, const BatchMap& Mv8, int nv8_blk, const BBwdIO* io,
                       hipStream_t s);
void launch_b_adj_gather(int mode, const BatchMap& M, int nblk, int it, hipStream_t s);
void launch_b_flags(const BatchMap& M, int* ctl_out, double* dstat_out, hipStream_t s);

// Per-launch timing: arm a start/stop event pair for the next kernel launch of
// this thread (stamped by the dispatch itself); launch_events_used() tells
// whether a launch consumed them and disarms.
void arm_launch_events(hipEvent_t start, hipEvent_t stop);
bool launch_events_used();

int vert_group_blocks(int n);
int bottom_blocks(int nB, int nT);
int eb_blocks(int nT);  // blocks of the interface right-hand side (at least one)
int tr_blocks(int ne, int nf);
void launch_local(const ElemArgs& E, const StepState& St, const RedArgs& R, const double* q, int nv, int nf,
                  int k, int fwd, hipStream_t s);
void launch_elem_GtG(const ElemArgs& E, const double* x, int nv, const double* w, double* contrib, hipStream_t s);
void launch_prologue(const VertArgs& V, const double* qt, const double* vt, const double* f, const double* q0,
                     int inertial, const StepState& St, hipStream_t s);
void launch_gather_fwd(const VertArgs& V, const StepState& St, const RedArgs& R, int k, hipStream_t s);
void launch_gather_debug(const VertArgs& V, const double* contrib, double* out, hipStream_t s);
void launch_Eb(int mode, const VertArgs& V, const SolveArgs& S, const StepState& St, const AdjState& A,
               const RedArgs& R, const double* rhs, int k, hipStream_t s);
// done: the loop's done flag (nullptr: always solve)
void launch_top(const VertArgs& V, const SolveArgs& S, double* out, const int* done, hipStream_t s);
void launch_bottom(int mode, const VertArgs& V, const SolveArgs& S, const StepState& St, const AdjState& A,
                   const RedArgs& R, const double* rhs, double* out, int k, hipStream_t s);
void launch_epilogue(const VertArgs& V, const StepState& St, double* q_next, double* v_next, double* ckpt,
                     hipStream_t s);
void launch_to_lib(const VertArgs& V, const double* user, double* lib, int free_only, hipStream_t s);
void launch_from_lib(const VertArgs& V, const double* lib, double* user, int free_only, hipStream_t s);
void launch_tr_partials(const ElemArgs& E, const VertArgs& V, const RedArgs& R, const double* ck, hipStream_t s);
// also clears zero[0, nzero) (nullable; nzero at most one workgroup, kBlock) for the kernels that follow
void launch_bwd_elem(const ElemArgs& E, const VertArgs& V, const RedArgs& R, const double* ck, double eps_tr,
                     double tau_force, int use_partials, double* jac, double* bstat, int* zero, int nzero,
                     hipStream_t s);
void launch_apply_K(int mode, const ElemArgs& E, const VertArgs& V, const AdjState& A, const RedArgs& R,
                    const double* jac, const double* x, int it, hipStream_t s);
void launch_adj_gather(int mode, const VertArgs& V, const AdjState& A, const RedArgs& R, int it, hipStream_t s);
void launch_bwd_prologue(const VertArgs& V, const AdjState& A, const double* gq, const double* gv, int warm,
                         const double* h1, const double* h2, const double* h3, hipStream_t s);
void launch_grad_elem(const ElemArgs& E, const VertArgs& V, const double* ck, const double* jac, const double* mu,
                      double* contrib, double* g_logE, hipStream_t s);
void launch_grad_vert(const VertArgs& V, const double* mu, const double* contrib, const double* gv_next, double* gq_t,
                      double* gv_t, double* gf, hipStream_t s);
void launch_init_warm(const ElemArgs& E, hipStream_t s);
// dL/da_g += sum over the group's tets (g_ptr / g_tets, library tet order) of their terms E.mgt
void launch_muscle_grad(const ElemArgs& E, int n_groups, const int* g_ptr, const int* g_tets, double* g_act,
                        hipStream_t s);

// contact (contact.hip, and the apply kernels in kernels.hip)
void launch_contact_detect(const VertArgs& V, const double* qt, const double* vt, const ObsArgs& O, int kmax,
                           int* v, double* n, double* g, int* flags, hipStream_t s);
void launch_unit_rhs(int nv, double* rhs, int v0, int v1, int v2, hipStream_t s);
void launch_store_cols(int nf, int nv, const double* x, double* cols, int s0, int s1, int s2, hipStream_t s);
void launch_contact_W(const ContactArgs& C, double* W, hipStream_t s);
void launch_contact_start(const ContactArgs& C, hipStream_t s);
void launch_contact_fb(const VertArgs& V, const ContactArgs& C, const double* qhat, const int* done, hipStream_t s);
void launch_contact_winv(const ContactArgs& C, double* Winv, hipStream_t s);
void launch_contact_proj(const VertArgs& V, const ContactArgs& C, const double* z, const int* done, hipStream_t s);
void launch_contact_ckpt(const ContactArgs& C, int kmax, double e_rest, double* rec, hipStream_t s);
// restitution (forward): active unilateral rows whose vertex approached (n . v_t < 0) set its outgoing
// normal velocity to -e (n . v_t), rows of one vertex in order; flags the rows in the checkpoint record
void launch_contact_restitution(const VertArgs& V, const ContactArgs& C, const double* v_t, double* v_next, double e,
                                double* rec, int kmax, hipStream_t s);
// its adjoint from a checkpoint record: before the backward step v bar (caller order, copied to gv_out
// first) loses the normal part of flagged rows in reverse order, their values kept in s_row; after it
// dL/dv_t gains -e n s_row
void launch_restitution_adj_pre(const VertArgs& V, const double* rec, int kmax, double* gv, double* s_row,
                                hipStream_t s);
void launch_restitution_adj_post(const VertArgs& V, const double* rec, int kmax, const double* s_row,
                                 double* gv_t, hipStream_t s);
// friction: the per-iteration Newton (forward), the inverse of the adjoint rows' unsymmetric coupling
// matrix, the contact vertices' slip and diagonal for the adjoint's classification, and the routing of the
// sticking / sliding rows' multipliers to dL/dq_t (caller order; kind 0 rows skipped)
void launch_contact_fr(const VertArgs& V, const ContactArgs& C, const double* qhat, const int* done, hipStream_t s);
void launch_contact_minv(const ContactArgs& C, double* Minv, hipStream_t s);
void launch_contact_slip(const VertArgs& V, const ContactArgs& C, const double* qstar, const double* qt, double* out,
                         hipStream_t s);
void launch_contact_route(const VertArgs& V, const ContactArgs& C, const int* kind, double* gq_t, hipStream_t s);
int contact_apply_blocks(int nf);
void launch_contact_apply_fwd(const VertArgs& V, const StepState& St, const RedArgs& R, const ContactArgs& C, int k,
                              hipStream_t s);
void launch_contact_apply_adj(int mode, const VertArgs& V, const AdjState& A, const RedArgs& R,
                              const ContactArgs& C, const double* rhs, int k, hipStream_t s);
void launch_zero_int(int* p, int n, hipStream_t s);

}  // namespace pdhot
