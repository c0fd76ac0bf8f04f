// Kernel argument blocks and launchers of the pdhot HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>

#include "pd_internal.h"

namespace pdhot {

enum { kModeFwd = 0, kModePlain = 1, kModeDebugGather = 2, kModePCG = 3, kModeFixed = 4 };

// device control block (int): done flag, final iteration count, status,
// Anderson resets, Newton iteration maximum, then two Anderson states
// {nonempty, ncols, head, pad} selected by iteration parity; from kCtlAdj the
// adjoint's {iterations, status, done}.
enum { kCtlDone = 0, kCtlIters = 1, kCtlStatus = 2, kCtlResets = 3, kCtlNewton = 4, kCtlAA = 8, kCtlSize = 16,
       kCtlAdj = 16, kCtlTotal = 24 };

struct ElemArgs {
  int ne;
  const int* tv;
  const double* Bm;
  const double* wV;
  const double* bV;
  const double* muV;
  const double* lamV;
  const int* tet_orig;
  double mu_bar, lam_bar, k_bar;
};

struct VertArgs {
  int nv, nf, ne, max_sub;
  const int* v_orig;
  const double* mass;
  const double* rest;
  const double* cpin;
  const int* inc_ptr;
  const int* inc_idx;
  double h, alpha;
  double grav[3];
};

struct SolveArgs {
  int nsub, nB, nT, n_bottom_items, n_top_blocks, top_rows, max_ns, max_nI;
  const double* Zs;
  const double* Et;
  const double* Z;
  const long long* zs_off;
  const long long* et_off;
  const int* sub_begin;
  const int* ir_off;
  const int* irows;
  const int* slot_of;
  const int* row_slot_ptr;
  double* t_slots;
  const int* bottom_items;
};

struct StepState {
  int m, kmax;
  double eps_rel, eps_abs;
  int n_gate_blocks, n_aa_blocks;
  double *contrib, *qt, *vt, *qtil, *c;
  double *q_cur, *q_prev, *b_cur, *b_prev, *qhat;
  double *q_last, *g_last, *dQ, *dG;
  double *gate_part, *aa_part;
  int* ctl;
  int* done;
  double* dstat;
};

struct AdjState {
  int n_vert_blocks, kmax;
  double eps;
  double *contrib, *qbar, *mu, *r, *z, *p, *Ap, *w;
  double* part;   // per vertex block: 8 doubles
  double* scal;   // device scalars (2 x 4, by parity)
  int* ctl;       // [iters, status]
  int* done;
  double* dstat;  // [residual]
};

void launch_local(const ElemArgs& E, const double* q, int nv, double* contrib, const int* done, int* newton_max,
                  hipStream_t s);
void launch_elem_GtG(const ElemArgs& E, const double* x, int nv, const double* w, double* contrib, hipStream_t s);
void launch_prologue(const VertArgs& V, const double* qt, const double* vt, const double* f, const double* q0,
                     const double* contrib, const StepState& St, hipStream_t s);
void launch_gather_E(int mode, const VertArgs& V, const SolveArgs& S, const StepState& St, const double* rhs_in,
                     double* rhs_out, int k, hipStream_t s);
void launch_top(int mode, const VertArgs& V, const SolveArgs& S, const StepState& St, const double* rhs, double* out,
                int k, hipStream_t s);
void launch_bottom(int mode, const VertArgs& V, const SolveArgs& S, const StepState& St, const double* rhs,
                   double* out, int k, hipStream_t s);
void launch_aa_update(const VertArgs& V, const StepState& St, int k, hipStream_t s);
void launch_epilogue(const VertArgs& V, const StepState& St, double* q_next, double* v_next, double* ckpt,
                     hipStream_t s);
void launch_to_lib(const VertArgs& V, const double* user, double* lib, int free_only, hipStream_t s);
void launch_from_lib(const VertArgs& V, const double* lib, double* user, int free_only, hipStream_t s);
int tr_partial_blocks(const ElemArgs& E, const VertArgs& V);
void launch_tr_partials(const ElemArgs& E, const VertArgs& V, const double* ck, double* part, hipStream_t s);
void launch_bwd_elem(const ElemArgs& E, const VertArgs& V, const double* ck, const double* part, int n_part,
                     double eps_tr, double tau_force, double* jac, double* bstat, hipStream_t s);
void launch_apply_K(const ElemArgs& E, const VertArgs& V, const double* jac, const double* x, double* contrib,
                    const int* done, hipStream_t s);
void launch_adj_gather(int mode, const VertArgs& V, const AdjState& A, int it, hipStream_t s);
void launch_pcg_alpha(const VertArgs& V, const AdjState& A, int it, hipStream_t s);
void launch_adj_dots(int mode, const VertArgs& V, const AdjState& A, int it, hipStream_t s);
void launch_adj_next(int mode, const VertArgs& V, const AdjState& A, int it, hipStream_t s);
void launch_bwd_prologue(const VertArgs& V, const AdjState& A, const double* gq, const double* gv, hipStream_t s);
void launch_pcg_start(const VertArgs& V, const AdjState& A, hipStream_t s);
void launch_grad_elem(const ElemArgs& E, const VertArgs& V, const double* ck, const double* jac, const double* mu,
                      double* contrib, double* g_logE, hipStream_t s);
void launch_grad_vert(const VertArgs& V, const double* mu, const double* contrib, const double* gv_next, double* gq_t,
                      double* gv_t, double* gf, hipStream_t s);

}  // namespace pdhot
