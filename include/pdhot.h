/*
 * pdhot: MI355X (gfx950) library for the hot path of differentiable Projective
 * Dynamics (PD) on heterogeneous Neo-Hookean tetrahedral meshes
 * (arXiv 2605.14526, "DiffPhD").
 *
 * The library owns every internal buffer (factor blocks, element and vertex
 * arrays, Anderson history, scratch).  Per-step inputs and outputs are
 * caller-owned DEVICE buffers of doubles.  Every position-like vector is laid
 * out as n_verts x 3 (vertex-major, x y z per vertex) in the caller's vertex
 * numbering; the library reorders internally.
 *
 * Return values: PD_OK (0), PD_NOT_CONVERGED (1, a warning: results and
 * statistics are still written), or a negative error code.  No C++ exception
 * crosses this interface; pd_last_error() returns a message for the last
 * failing call of the calling thread.
 *
 * All entry points are synchronous with respect to the host on return unless
 * stated otherwise; `stream` is a hipStream_t passed as void* (NULL = the
 * default stream).  pd_step_forward and pd_step_backward return once their
 * convergence decision and statistics are on the host; the kernels that write
 * their outputs (positions and velocities and the checkpoint; the gradients)
 * may still be running on `stream`, ordered before any later work on it.
 */
#ifndef PDHOT_H
#define PDHOT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  PD_OK = 0,
  PD_NOT_CONVERGED = 1,
  PD_ERR_INVALID_ARG = -1,
  PD_ERR_DEGENERATE_TET = -2,
  PD_ERR_NONFINITE = -3,
  PD_ERR_STALE_FACTOR = -4,
  PD_ERR_FACTOR_NOT_SPD = -5,
  PD_ERR_HIP = -6,
  PD_ERR_ALLOC = -7,
  PD_ERR_CONTACT = -8  /* contact rows beyond max_contacts or the dense solve size, or a singular contact block */
};

typedef struct pd_scene pd_scene;

/* Mesh (host pointers, copied by pd_scene_create).
 * rest_xyz: n_verts x 3 rest positions.  tets: n_tets x 4 vertex indices; a
 * tet with negative rest volume is reoriented, one with zero volume is an
 * error (PD_ERR_DEGENERATE_TET).  pinned: n_verts flags, 1 = Dirichlet vertex
 * held at its rest position. */
typedef struct pd_mesh_desc {
  int32_t n_verts;
  int32_t n_tets;
  const double* rest_xyz;
  const int32_t* tets;
  const uint8_t* pinned;
} pd_mesh_desc;

/* Material (host pointers, copied).  Per-tet Young's modulus E_e = exp(log_E[e])
 * with a shared Poisson ratio nu gives the Lame parameters of Sec. 3.1
 * Eq. lame; rho is the density; alpha (1/s) and beta0 (Pa s) are the Rayleigh
 * coefficients of Sec. 4.5 Eq. rayleigh, beta_e = beta0 mu_e / max_e mu_e.
 * energy selects the local step (Sec. 4.1): 0 = the Neo-Hookean proximal map
 * with PD weight w_e = 2 mu_e + lam_e; 1 = the corotated + volume composite,
 * a rotation step p0 = R (signed polar rotation of F) with weight 2 mu_e and
 * a volume step p1 = F projected onto det = 1 (the closest unit-determinant
 * point in stretch space) with weight lam_e (Sec. 7.2); 2 = the rotation step
 * with the logarithmic volume barrier of Sec. 4.1 Eq. pd_log_volume (-mu sum
 * ln s + lam/2 (sum ln s)^2, solved on the stretches by the Neo-Hookean prox
 * Newton without its I1 term, with the mesh means and penalty lam_bar) as the
 * volume step of weight lam_e.  All give the same system matrix; the
 * trust-region filter of Sec. 4.4 applies to energy 0. */
typedef struct pd_material_desc {
  const double* log_E;
  double nu;
  double rho;
  double alpha;
  double beta0;
  int32_t energy;
} pd_material_desc;

/* Solver options.
 * h: time step (s).  gravity: acceleration added to every free vertex.
 * aa_window: Anderson window m (Sec. 4.3; 0 = plain local-global iteration).
 * eps_rel, eps_abs: dual-gate tolerances (Eq. convergence_dual).
 * kmax_fwd: PD iteration cap (PD_NOT_CONVERGED beyond it).
 * eps_adj, kmax_bwd: adjoint tolerance (relative preconditioned residual) and cap.
 * eps_tr: trust-region tolerance of Eq. tr_rule (0.1 in the paper).
 * adj_method: 0 = conjugate gradients preconditioned by the PD factor,
 *             1 = the fixed-point iteration mu <- A^-1 (qbar + K mu).
 * max_sub: largest subdomain (vertices) of the partitioned inverse
 *          (0 = library default).  The subdomains are the leaves of a nested
 *          dissection (Sec. 4.6's ordering); the separators above them form the
 *          interface.
 * iface_levels: levels of the separator tree that the interface solve keeps
 *          apart (1..8, 0 = library default 4): the separators at these levels
 *          are eliminated block by block (a dense frontal block per separator,
 *          two launches per extra level), the ones above merge into one dense
 *          top block; 1 is one dense inverse of the whole interface Schur
 *          complement.
 * iters_per_check: PD iterations issued between convergence checks of the
 *          host (0 = adaptive).
 * adj_warm: start of the adjoint iteration of pd_step_backward: 0 = zero
 *          (as in Alg. 2), 1 = the previous call's solution, 2 = the linear
 *          extrapolation 2 mu_{t+1} - mu_{t+2} of the two previous calls, 3 =
 *          the quadratic one 3 mu_{t+1} - 3 mu_{t+2} + mu_{t+3} of three (each
 *          uses as many previous solutions as the sweep has so far).  The
 *          history belongs to the scene; pd_adjoint_reset clears it (call it
 *          at the start of each reverse sweep); refactorization clears it too.
 *          The solve still runs to eps_adj, so only the iteration count
 *          depends on the start.
 * fwd_start: first PD iterate when pd_step_forward gets no q0: 0 = q_t (as in
 *          Alg. 1), 1 = the inertial guess q_t + h v_t.
 * Errors: PD_ERR_INVALID_ARG for an iface_levels outside 0..8. */
typedef struct pd_solver_opts {
  double h;
  double gravity[3];
  int32_t aa_window;
  double eps_rel;
  double eps_abs;
  int32_t kmax_fwd;
  int32_t kmax_bwd;
  double eps_adj;
  double eps_tr;
  int32_t adj_method;
  int32_t max_sub;
  int32_t iters_per_check;
  int32_t adj_warm;
  int32_t fwd_start;
  int32_t iface_levels;
} pd_solver_opts;

/* Forward statistics. gate[0..3] = |q^k - q^{k-1}|, |q^{k-1}|, |b^k - b^{k-1}|,
 * |b^{k-1}| at exit; iters = number of global solves. */
typedef struct pd_fwd_stats {
  int32_t iters;
  int32_t aa_resets;
  int32_t status;
  int32_t newton_capped;  /* 1 if a tet's prox Newton reached its 50-iteration cap */
  double gate[4];
  int32_t n_contacts;     /* candidate contact rows of the step */
  int32_t n_active;       /* rows with a positive impulse at exit */
  double fb_res;          /* Fischer-Burmeister residual max |phi| of the last contact solve */
} pd_fwd_stats;

/* Backward statistics: adjoint iterations, trust-region ratio rho and the
 * chosen tau (Eqs. tr_ratio, tr_rule), the two decreases of Eq. tr_decreases. */
typedef struct pd_bwd_stats {
  int32_t adj_iters;
  int32_t status;
  double rho;
  double tau;
  double dphi_act;
  double dphi_mod;
  double residual;
  int32_t n_active;  /* active contact rows held as equalities in the adjoint */
  int32_t pad;
} pd_bwd_stats;

/* Create a scene: validates and copies the mesh and material, builds the
 * library vertex order (nested-dissection subdomains, interface last, pinned
 * vertices at the end) and the element arrays, and factorizes (so a new scene
 * is ready to step).  Setup follows Alg. 1's stale-A branch (Secs. 4.1, 4.2,
 * 4.5, 4.6).  Allocates device memory on the current HIP device. */
int pd_scene_create(const pd_mesh_desc* mesh, const pd_material_desc* mat, const pd_solver_opts* opts,
                    pd_scene** out);
int pd_scene_destroy(pd_scene* scene);

/* Replace the per-tet log Young's moduli (host pointer, n_tets values).  The
 * factor becomes stale (refactorization policy, Sec. 4.6): stepping before
 * pd_scene_factorize returns PD_ERR_STALE_FACTOR. */
int pd_scene_set_material(pd_scene* scene, const double* log_E_host);
/* The same from a DEVICE buffer of n_tets doubles: the copy is ordered on
 * `stream` (the caller's producer of log E) and the call returns once the
 * values are on the host and checked (PD_ERR_NONFINITE for a non-finite
 * value, PD_ERR_HIP if the copy fails). */
int pd_scene_set_material_device(pd_scene* scene, const double* log_E_dev, void* stream);

/* Muscle actuation (the paper's muscle-driven scenes, Sec. 5, whose inverse
 * problems route through db/da; the paper prints no muscle energy, so the
 * reading is stated here).  A muscle tet e of group g carries the fibre
 * constraint (w_m V_e / 2) dist^2(F_e m_e, S_l), S_l the sphere of radius
 * l = 1 - a_g in fibre space: the local step projects f = F_e m_e to
 * p = l f/|f|, A~ gains w_m V_e G_m^T G_m (G_m q = f; it acts per axis like the
 * rest of A~), b gains w_m V_e G_m^T p, K gains w_m V_e G_m^T (l/|f|)(I - f^ f^T)
 * G_m, and dL/da_g = -sum_{e in g} w_m V_e <G_m mu, f^> at q*.
 * group: host, n_tets int32 in the caller's tet order, -1 for a passive tet,
 * else 0 .. n_groups - 1; fibre: host, n_tets x 3 unit vectors (|m|^2 within
 * 1e-9 of 1) in rest coordinates; w_m > 0 in Pa.  n_groups = 0 removes the
 * muscles.  Activations start at 0.  Marks the factor stale (A~ changes);
 * waits for all device work first.  Batches reject scenes with muscles.
 * Errors: PD_ERR_INVALID_ARG for a null array, a group out of range, a
 * non-unit fibre or w_m <= 0. */
int pd_scene_set_muscles(pd_scene* scene, int n_groups, double w_m, const int32_t* group, const double* fibre);

/* The groups' activations a (device, n_groups doubles), copied on `stream`
 * (stream-ordered with the steps).  They change b only, not A~, so no
 * refactorization is needed; a backward step uses the activations current
 * at its call, so keep them unchanged between a forward step and its
 * backward step.  Errors: PD_ERR_INVALID_ARG for a scene without muscles. */
int pd_scene_set_activation(pd_scene* scene, const double* a_dev, void* stream);

/* Register the caller's device buffer of n_groups doubles into which every
 * pd_step_backward ADDS dL/da (summed per group in a fixed order, no
 * atomics); NULL stops forming it.  The buffer stays caller-owned; clear it
 * before a sweep.  Setting muscles unregisters it. */
int pd_scene_set_activation_grad(pd_scene* scene, double* g_act_dev);

/* Hold the mesh means of the local prox and of Rayleigh damping fixed across
 * refactorizations.  The means mu_bar, lam_bar (Sec. 4.2) and mu_ref (Sec. 4.5
 * Eq. rayleigh) are constants of the gradient (the paper's gradient formulas
 * have no terms for them), so a finite-difference check of d/dlog E must keep
 * them fixed while it perturbs log E.  means3 (host) = {mu_bar, lam_bar,
 * mu_ref} with mu_bar > 0, mu_ref > 0; NULL returns to computing them from
 * the material at each factorization.  Marks the factor stale. */
int pd_scene_freeze_means(pd_scene* scene, const double* means3);

/* Lumped vertex masses m_v = sum_e rho V_e / 4 (Sec. 3.1), host output of
 * n_verts doubles in the caller's vertex order (e.g. the M-weighted
 * trajectory loss of an identification task).  No device work. */
int pd_scene_vertex_mass(const pd_scene* scene, double* out);

/* Assemble A = (1 + alpha h) M / h^2 + sum_e (w_e + beta_e / h) V_e G_e^T G_e
 * (Sec. 4.5 Eq. A_damped, Dirichlet vertices eliminated), freeze the mesh means
 * mu_bar, lam_bar, k_bar and mu_ref, and build the partitioned inverse used by
 * every solve (Sec. 4.6 Eq. Ainv_STS in role).  Host work plus one upload.
 * First waits for `stream` and then for the whole device, so kernels of
 * earlier steps that read the per-tet arrays finish before they change. */
int pd_scene_factorize(pd_scene* scene, void* stream);

/* Scene facts. info[0..7] = n_verts, n_tets, n_free, n_subdomains,
 * n_interface, aa_window, factor bytes on the device, most subdomains bordered
 * by one interface vertex (as double; info holds 8 values). means[0..3] =
 * mu_bar, lam_bar, k_bar, mu_ref (may be NULL). */
int pd_scene_info(const pd_scene* scene, double* info, double* means);

/* The library's vertex order (the ordering of the factorization, Sec. 4.6):
 * perm_out[i] = the caller's index of library vertex i, for i < n_verts (host
 * memory, int32).  Library order holds the subdomains' vertices first (one
 * contiguous range per subdomain), then the interface vertices, then the
 * pinned ones.  Every step entry point takes and returns caller order, so this
 * is for callers that want to lay their own data out like the factor.
 * Errors: PD_ERR_INVALID_ARG for a null argument. */
int pd_scene_get_permutation(const pd_scene* scene, int32_t* perm_out);

/* Bytes of one checkpoint record (q_t, q tilde, q*, q*-1 of one step; with
 * obstacles also the step's contact rows and impulses). */
size_t pd_ckpt_bytes(const pd_scene* scene);

/* One forward step (Alg. 1; contact rows as set by pd_scene_set_obstacles).
 * q_t, v_t: current state; f_ext: external force per vertex (NULL = none;
 * gravity from the options is added); q0: initial iterate, e.g. a learned
 * warm start (NULL = q_t, or q_t + h v_t with fwd_start = 1); outputs q_next,
 * v_next (may alias nothing else); ckpt: caller-allocated device buffer of
 * pd_ckpt_bytes() bytes or NULL.
 * Pinned vertices are held at their rest positions.  Runs the local step,
 * RHS assembly, dual gate, global solve and Anderson mixing until the gate
 * holds (Secs. 4.1-4.3). */
int pd_step_forward(pd_scene* scene, const double* q_t, const double* v_t, const double* f_ext,
                    const double* q0, double* q_next, double* v_next, void* ckpt, pd_fwd_stats* stats,
                    void* stream);

/* One backward step (Alg. 2, with the step's active contact rows) from a checkpoint written by
 * pd_step_forward.  gq_next, gv_next: dL/dq_{t+h}, dL/dv_{t+h}.  Outputs
 * dL/dq_t, dL/dv_t, dL/df_ext (overwritten; zero on pinned vertices) and
 * g_logE_accum += dL/dlog E_e (n_tets, caller's tet order).  Any output
 * pointer may be NULL.  Implements the trust-region selection (Sec. 4.4),
 * the filtered prox differential, the adjoint solve and the gradient routing
 * (Sec. 4.8). */
int pd_step_backward(pd_scene* scene, const void* ckpt, const double* gq_next, const double* gv_next,
                     double* gq_t, double* gv_t, double* gf_ext, double* g_logE_accum, pd_bwd_stats* stats,
                     void* stream);

/* ------------------------------------------------------------------------
 * Contact with static obstacles (Sec. 4.7, Eqs. fb_n, omega_E_n,
 * contact_system, q_update), read frictionless: each row c acts on one free
 * vertex v_c along a unit normal n_c with gap n_c . q_{v_c} - g_c >= 0 and
 * impulse lam_c >= 0, complementary.  At the start of every pd_step_forward
 * the library detects the rows: for each free vertex and each obstacle, the
 * obstacle's distance d (a plane's signed distance n.x - o; for a box the
 * largest signed distance over its faces -x, +x, -y, +y, -z, +z) is taken at
 * x0 = q_t and x1 = q_t + h v_t, and the pair is a row if min(d(x0), d(x1)) <
 * d_c, with the normal and offset of the face attaining d(x0).  Inside every
 * PD iteration the global solve is followed by a Fischer-Burmeister Newton
 * solve of the rows on the Delassus operator W = J A~^{-1} J^T (built from
 * cached columns A~^{-1} e_v, reused across steps: one factor serves the
 * forward, backward and contact stages) and the position correction
 * sum_c lam_c A~^{-1} e_{v_c} n_c; the dual gate also requires the FB
 * residual <= fb_tol.  pd_step_backward holds the active rows (lam > 1e-10
 * max lam) as equalities and projects the adjoint onto them.
 *
 * pd_scene_set_obstacles: planes n_planes x 4 (unit normal, offset o), boxes
 * n_boxes x 6 (lo xyz, hi xyz), host pointers, copied; at most 8 obstacles;
 * d_c > 0 the candidate distance; max_contacts (1..512) the row capacity per
 * step (PD_ERR_CONTACT beyond it); fb_tol > 0.  n_planes = n_boxes = 0 turns
 * contact off.  Checkpoints allocated before this call are too small
 * afterwards (pd_ckpt_bytes grows).  Scenes with obstacles cannot join a
 * batch.
 * pd_contact_rows: the rows of the last pd_step_forward (host buffers of
 * `capacity` entries, any may be NULL): caller's vertex ids, normals (3 per
 * row), offsets, impulses; *K receives the row count.
 * ------------------------------------------------------------------------ */
int pd_scene_set_obstacles(pd_scene* scene, int n_planes, const double* planes, int n_boxes, const double* boxes,
                           double d_c, int max_contacts, double fb_tol);
int pd_contact_rows(const pd_scene* scene, int* K, int32_t* vert, double* normals, double* offsets,
                    double* lambda, int capacity);

/* Bilateral rows (Sec. 4.7: attachments held as constraints; the block
 * projection leaves their multipliers free).  Row c is the equality
 * n_c . q_{v_c} = g_c with vertex vert[c] (caller order, not pinned), unit
 * direction normals[3c..3c+2] and offset offsets[c] (host arrays, copied); a
 * full attachment of a vertex to a point is three rows along x, y, z.  The
 * rows follow each step's detected contact rows (same Delassus operator and
 * column cache): in the FB Newton their residual is the gap (omega = 1,
 * E = 0) and they are never projected; the adjoint holds them as equalities.
 * Calling it again replaces the rows (offsets may change between steps: a
 * moving handle); n_rows = 0 removes them.  Without obstacles the contact
 * machinery is set up with room for max(64, n_rows) rows.  Frictionless
 * contact only.  Waits for all device work.  Errors: PD_ERR_INVALID_ARG for
 * a pinned or out-of-range vertex, a non-unit direction, more rows than the
 * obstacles' max_contacts, or a friction coefficient set. */
int pd_scene_set_attachments(pd_scene* scene, int n_rows, const int32_t* vert, const double* normals,
                             const double* offsets);

/* Restitution post-correction (the paper's velocity-level correction, which
 * fires while the normal velocity is negative and the impulse positive; the
 * reading): after each forward step, every active unilateral row (impulse
 * above 1e-10 of the largest) whose vertex approached (u = n . v_t < 0) sets
 * the vertex's outgoing normal velocity to -e u, rows of one vertex in order;
 * positions are unchanged.  The checkpoint records the corrected rows and e,
 * and the backward step applies the correction's adjoint.  e >= 0 turns it
 * on, e < 0 off (the default). */
int pd_scene_set_restitution(pd_scene* scene, double e);

/* The gradient of the loss w.r.t. the offsets g_c of the rows of the last
 * backward step's checkpoint (detected rows, then bilateral rows, as
 * pd_contact_rows lists them for that forward step): dL/dg =
 * W_AA^{-1} J_A A~^{-1} (q bar + K mu) on the active rows, 0 on the others.
 * Host output of at least that many doubles.  Frictionless rows only; it
 * waits for all device work.  Errors: PD_ERR_INVALID_ARG without contact, with
 * friction, or for a capacity below the row count. */
int pd_contact_gap_grad(pd_scene* scene, double* g_out, int capacity);

/* Coulomb friction on the obstacles (Sec. 4.7: the Signorini-Coulomb law
 * with the friction disk of radius mu lam_n; Sec. 4.8: its adjoint with the
 * active set fixed).  mu > 0 turns each contact row into a frame of three
 * rows: the normal n and the tangents t1 = (a - (a.n) n)/|a - (a.n) n| (a the
 * coordinate axis of the smallest |n_i|, the first on ties), t2 = n x t1.
 * The slip of a contact is s = T^T (q_{v_c} - q_{t,v_c}) over the step.
 * Detection then keeps one contact per vertex (the qualifying obstacle with
 * the smallest distance at q_t, the first on ties), since a frame already
 * spans the vertex's three directions.  Each PD iteration solves the contact
 * law by semi-smooth Newton: the Fischer-Burmeister normal row of Eq. fb_n
 * with the weights of Eq. omega_E_n, and the natural map lam_f -
 * P_D(lam_f - s/w) onto the disk D of radius mu lam_n for the tangent pair
 * (w = the contact vertex's diagonal of A~^{-1}); the free rows form a
 * symmetric positive definite system factored by dense Cholesky, then
 * lam_n >= 0 and the disk projection are enforced.  The gate's residual is
 * max(|phi_FB|, w |lam_f - P_D(.)|).  pd_step_backward holds the active
 * contacts fixed: sticking ones constrain the slip, sliding ones carry the
 * friction -mu lam_n s/|s| differentiated with respect to s and lam_n; this
 * adjoint is unsymmetric and runs the projected fixed point whatever
 * adj_method says.  mu = 0 returns to frictionless contact.  Call after
 * pd_scene_set_obstacles (which resets mu to 0); PD_ERR_INVALID_ARG without
 * obstacles or for a negative or non-finite mu. */
int pd_scene_set_friction(pd_scene* scene, double mu);
/* Impulses of the last pd_step_forward per contact row (host, 3 per row:
 * normal, t1, t2 components; tangents 0 without friction); capacity rows. */
int pd_contact_impulses(const pd_scene* scene, double* lam3, int capacity);

/* Forget the adjoint solutions kept for the warm start (adj_warm > 0), so the
 * next pd_step_backward starts from zero.  No device work. */
int pd_adjoint_reset(pd_scene* scene);

/* Diagnostic entry points (stage parity), all device pointers, n_verts x 3.
 * pd_debug_local_rhs: b = sum_e w_e V_e G_e^T p*_e(G_e q) (Eq. A_basic without
 *   its constant part), free rows (pinned rows zero).
 * pd_debug_apply_Ainv: x = A~^{-1} r per axis on free vertices (pinned zero).
 * pd_debug_apply_K: y = K x, K = sum_e w_e V_e G_e^T (d p* / d F)_tau G_e
 *   (Eq. db_dq with the filtered differential of Eq. tr_ift), free rows/cols. */
int pd_debug_local_rhs(pd_scene* scene, const double* q, double* b, void* stream);
int pd_debug_apply_Ainv(pd_scene* scene, const double* r, double* x, void* stream);
int pd_debug_apply_K(pd_scene* scene, const double* q, double tau, const double* x, double* y, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): x = A~^{-1} r
 * exactly as pd_debug_apply_Ainv (the same kernels and results), with the
 * solve's scratch (two staging vectors of 3 n_verts doubles, the interface
 * right-hand side and the gathered interface solution) in a static device
 * workspace of 2^21 doubles (16 MiB) that the library holds on each device it
 * runs on until the process ends.  Calls nothing that allocates and does not
 * wait: the result is ordered on `stream` (call with the scene's device
 * current).  Every call on a device shares that device's workspace, so calls
 * that overlap on one device (other streams, other threads) race; the
 * workspace keeps the last call's contents, and nothing in it needs to start
 * at zero.  PD_ERR_INVALID_ARG (before any device work) when the scene needs
 * more scratch than the workspace holds (6 n_verts + 3 n_interface + 3 times
 * the interface rows of all subdomains, about 300k vertices at most), for a
 * null argument; PD_ERR_STALE_FACTOR as the other solves; PD_ERR_HIP if the
 * workspace's address cannot be found. */
int pd_apply_Ainv_noalloc(pd_scene* scene, const double* r, double* x, void* stream);

/* Kernel timing for roofline reports: every launch of one kernel inside
 * pd_step_forward / pd_step_backward carries a start and a stop HIP event
 * stamped by the dispatch itself on the caller's stream, so the elapsed time
 * is the kernel's own execution time.  kernel: 0 local step, 1 right-hand-side
 * gather, 2 interface (Schur) solve, 3 subdomain solve, 4 interface
 * right-hand side (coupling products), 5 K apply, 6 the whole global solve
 * (the launches of 2, 3 and 4 together); -1 stops timing.  Resets the
 * totals.  Instrumentation only. */
int pd_kernel_timer(pd_scene* scene, int kernel);
/* Totals since pd_kernel_timer: summed launch durations (ms), launches timed,
 * working units (launches that did work, the others exit at once after
 * convergence; for kernel 6 the global solves) and the algorithmic bytes of
 * one unit: what the operation must move once (Sec. 4.1 local step: 96 B of
 * element data per tet and 48 B of vertex data per vertex; the global solve
 * of Sec. 4.6: one forward and one backward sweep of the sparse Cholesky
 * factor of A~ under nested dissection, 16 B per factor entry, plus six
 * passes over three-axis vectors of the free vertices), not what the
 * implementation re-reads. */
int pd_kernel_timer_read(pd_scene* scene, double* total_ms, int64_t* launches, int64_t* working,
                         double* bytes_per_launch);
/* Entries (diagonal included) of the sparse Cholesky factor of A~ over the
 * free vertices under a nested-dissection order (recursive coordinate
 * bisection with vertex separators): the factor that the method's triangular
 * solves would sweep (Sec. 4.6), used for the algorithmic bytes above. */
int pd_scene_factor_nnz(const pd_scene* scene, double* nnz);

/* ------------------------------------------------------------------------
 * Batches: many scenes (any sizes, materials and Anderson windows) stepped
 * together.  Every stage of a PD iteration and of an adjoint iteration is one
 * launch across all scenes; each scene keeps its own state, reductions and
 * convergence flag, so a converged scene idles while the others iterate.
 * Results are bitwise those of stepping each scene alone.  The scenes stay
 * owned by the caller and must outlive the batch; a batch runs the PCG
 * adjoint (adj_method 0) without obstacles, attachments or muscles (checked at
 * creation and at every step: PD_ERR_INVALID_ARG).  A scene refactorized after
 * the batch was made (pd_scene_set_material + pd_scene_factorize) is picked up
 * at the next batched step (the batch rebuilds its per-scene tables and drops
 * its captured graphs).  Array arguments hold one pointer per scene, in the
 * order given to pd_batch_create (device buffers as for the single-scene
 * calls; NULL entries where those calls allow NULL).
 * ------------------------------------------------------------------------ */
typedef struct pd_batch pd_batch;
int pd_batch_create(pd_scene* const* scenes, int n, pd_batch** out);
int pd_batch_destroy(pd_batch* batch);
/* Launch shapes and host checks: workgroup sizes (64, 128 or 256 threads) of
 * the local step and of the K apply, PD / adjoint iterations issued between
 * convergence checks (0 = adaptive; graphs use 4 then), and use_graph = 1 to
 * capture each chunk of iterations once into a HIP graph and replay it. */
int pd_batch_config(pd_batch* batch, int block_local, int block_applyK, int iters_per_check, int use_graph);
/* Graph replay of chunks of iters_per_chunk iterations (captured at first
 * use, one graph per chunk start); 0 returns to eager launches with adaptive
 * host checks.  The workgroup sizes stay as configured.  The same as
 * pd_batch_config with use_graph = (iters_per_chunk > 0). */
int pd_batch_capture_graph(pd_batch* batch, int iters_per_chunk);
/* pd_step_forward / pd_step_backward on every scene of the batch. stats: arrays
 * of n entries or NULL. Returns PD_NOT_CONVERGED if any scene did not converge. */
int pd_batch_step_forward(pd_batch* batch, const double* const* q_t, const double* const* v_t,
                          const double* const* f_ext, const double* const* q0, double* const* q_next,
                          double* const* v_next, void* const* ckpt, pd_fwd_stats* stats, void* stream);
int pd_batch_step_backward(pd_batch* batch, const void* const* ckpt, const double* const* gq_next,
                           const double* const* gv_next, double* const* gq_t, double* const* gv_t,
                           double* const* gf_ext, double* const* g_logE_accum, pd_bwd_stats* stats, void* stream);

/* Per-launch timing of one kernel kind inside the batched steps (as
 * pd_kernel_timer, eager launches only: nothing is timed while use_graph = 1)
 * and the algorithmic bytes of the work those launches did, summed over the
 * scenes (kernel 6, the global solve: each scene's solves times its bytes per
 * solve; 0: each scene's local steps; 5: each scene's K applies). */
int pd_batch_kernel_timer(pd_batch* batch, int kernel);
int pd_batch_kernel_timer_read(pd_batch* batch, double* total_ms, int64_t* launches, double* bytes_done);

/* Per-vertex material feature of the learned warm start: the mean of
 * log(2 mu_e + lam_e) over the vertex's tets (Eq. lame, the PD weight of
 * Sec. 4.2), minus its mean over the vertices.  out: host, n_verts doubles. */
int pd_scene_vertex_logw(const pd_scene* scene, double* out);

/* ------------------------------------------------------------------------
 * Learned warm start (an extension: the paper starts every step from q_t).
 * A message-passing network on the mesh edges predicts the correction of the
 * inertial guess; pd_step_forward takes its output as q0 and still iterates to
 * the same dual-gate tolerance.  Network: 16 node features
 * ((q_t - X)/l, h (v_t - v_{t-h})/s_out, h v_t/l, h^2 f/(m s_out),
 * (X - X_min)/L, vertex log w), encoder 16 -> 64 (SiLU), two message-passing layers
 * (m_ij = SiLU([h_i, h_j, (q_j - q_i)/l, (X_j - X_i)/l] W_msg + b_msg), sum over
 * in-edges, h_i += SiLU([h_i, a_i] W_node + b_node)), decoder 64 -> 3; q0 =
 * q_t + h v_t + s_out y on free vertices (l = mean edge length, L = largest
 * bounding-box extent).  Parameters: one FP32 vector, in the order W_enc
 * (16 x 64, row-major), b_enc, per layer W_msg (134 x 64), b_msg, W_node
 * (128 x 64), b_node, then W_dec (64 x 3), b_dec.
 * ------------------------------------------------------------------------ */
typedef struct pd_mpn pd_mpn;
typedef struct pd_mpn_desc {
  int32_t compute;  /* 0 = BF16 products on the matrix cores (FP32 accumulate), 1 = FP32 */
  double h;         /* time step of the scenes it serves */
  double rho;       /* density (lumped masses of the force feature) */
  double edge_weight; /* kappa of the training loss (edge-difference term, below) */
} pd_mpn_desc;

/* Build the network for a mesh (host arrays as in pd_scene_create; only the
 * topology, rest positions and pinned flags are used).  Weights are zero until
 * pd_mpn_init_params or pd_mpn_set_params. */
int pd_mpn_create(const pd_mesh_desc* mesh, const pd_mpn_desc* desc, pd_mpn** out);
int pd_mpn_destroy(pd_mpn* mpn);
/* info[0..6] = n_verts, directed edges, mean edge length, largest extent,
 * parameter count, output scale, compute mode. */
int pd_mpn_info(const pd_mpn* mpn, double* info);
/* Seeded initialisation: uniform(-1, 1)/sqrt(fan_in) weights (decoder x 0.1),
 * zero biases; resets the Adam moments. */
int pd_mpn_init_params(pd_mpn* mpn, uint64_t seed);
/* Host FP32 parameter vectors of exactly the parameter count. */
int pd_mpn_set_params(pd_mpn* mpn, const float* host, int64_t n);
int pd_mpn_get_params(const pd_mpn* mpn, float* host, int64_t n);
/* One network over several meshes (spec: one instance per mesh, shared
 * weights): dst drops its own parameters, gradient and Adam moments and uses
 * src's from now on, so a loss_grad on any mesh's instance writes the shared
 * gradient and an Adam step on src updates every instance.  Both must have
 * the same layer shapes and compute mode; src must outlive dst.  Waits for
 * all device work.  Errors: PD_ERR_INVALID_ARG for other shapes. */
int pd_mpn_share_params(pd_mpn* dst, pd_mpn* src);
/* Gradient of the last pd_mpn_loss_grad (host copy). */
int pd_mpn_get_grads(const pd_mpn* mpn, float* host, int64_t n);
/* s_out: the scale of the predicted correction (positions per unit output);
 * it also scales the correction-sized input features. */
int pd_mpn_set_output_scale(pd_mpn* mpn, double s_out);
/* q0 (device, n_verts x 3) for the step from (q_t, v_t) with the previous
 * step's velocity v_tm1 (v_t at the first step), the external force f_ext
 * (NULL = none) and the per-vertex
 * log w (device, n_verts, from pd_scene_vertex_logw).  Pinned vertices get q_t. */
int pd_mpn_forward(pd_mpn* mpn, const double* q_t, const double* v_tm1, const double* v_t, const double* f_ext,
                   const double* logw, double* q0, void* stream);
/* One training sample: forward, the loss
 *   sum_free |r|^2 / (3 n_free) + kappa sum_edges |r_j - r_i|^2 / (3 n_edges),
 *   r = y - (q_next - q_t - h v_t)/s_out on free vertices (0 on pinned),
 * summed over the directed edges (the second term weighs the strain that the
 * correction implies), and its gradient with respect to the parameters (kept
 * on the device).  loss: host pointer or NULL (NULL avoids a
 * synchronisation). */
int pd_mpn_loss_grad(pd_mpn* mpn, const double* q_t, const double* v_tm1, const double* v_t, const double* f_ext,
                     const double* logw, const double* q_next, double* loss, void* stream);
/* One Adam step on the FP32 master weights with the last gradient. */
int pd_mpn_adam_step(pd_mpn* mpn, double lr, double beta1, double beta2, double eps, void* stream);

/* Message of the last failing call on this thread ("" if none). */
const char* pd_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PDHOT_H */
