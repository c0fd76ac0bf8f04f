/*
 * Plain FP64 CPU oracle for differentiable Projective Dynamics with a
 * Neo-Hookean proximal local step (test infrastructure only).
 *
 * This library is the reference the HIP path is checked against.  Only the
 * test-suite, the smoke check and the CPU-baseline leg of the benchmark may
 * load it.  It shares no code with the GPU library.
 *
 * Vectors of positions are vertex-major: q[3*v + axis], original vertex order.
 */
#ifndef PD_ORACLE_H
#define PD_ORACLE_H
#ifdef __cplusplus
extern "C" {
#endif

typedef struct or_scene or_scene;

/* params: nu, rho, alpha, beta0, h, gx, gy, gz
 * solver: m (AA window), eps_rel, eps_abs, kmax_fwd, kmax_bwd, eps_adj, eps_tr,
 *         then mu_bar, lam_bar, mu_ref (frozen if mu_bar > 0, else computed),
 *         then the energy model (0: Neo-Hookean prox; 1: corotated + volume; 2: corotated + log barrier) */
or_scene* or_scene_create(int nv, int ne, const double* X, const int* tets, const unsigned char* pinned,
                          const double* logE, const double* params, const double* solver);
void or_scene_destroy(or_scene* s);
/* threads of the element loops and of the three per-axis solves (OpenMP);
 * results do not depend on it (fixed summation orders) */
void or_set_threads(int n);
int or_get_threads(void);
int or_scene_nfree(const or_scene* s);
/* muscle fibres (actuation; reading in pd_oracle.c): per element a group (-1: passive) and a unit fibre
 * (ne x 3, rest coordinates), fibre weight w_m; reassembles and refactors A~.  Activations a (n_groups)
 * default to 0.  g (n_groups, caller-owned, may be NULL) accumulates dL/da over backward steps. */
void or_scene_set_muscles(or_scene* s, int n_groups, double w_m, const int* group, const double* fibre);
void or_scene_set_activation(or_scene* s, const double* a);
void or_scene_set_act_grad(or_scene* s, double* g);
/* per-element / per-vertex quantities after setup (any may be NULL) */
void or_scene_info(const or_scene* s, double* vol, double* w, double* beta, double* mass, double* means4);

/* --- element level --- */
void or_svd3(const double F[9], double U[9], double sig[3], double V[9]);
int or_prox_stretch(const double sF[3], double mu, double lam, double k, double s_out[3]);
void or_prox_map(const double F[9], double mu, double lam, double k, double P[9]);
void or_prox_jacobian(const double F[9], double mu, double lam, double k, double tau, double J[81]);
double or_psi_nh(const double F[9], double mu, double lam);
/* corotated + volume composite (Sec. 4.1, Sec. 7.2): the volume step's stretches
 * (closest point with s1 s2 s3 = 1), its stretch Jacobian, and the composite
 * projection (2 mu R + lam P_vol) / (2 mu + lam) with its 9x9 Jacobian */
int or_volume_project(const double sF[3], double s[3]);
void or_volume_diff(const double sF[3], double D[9]);
void or_composite_map(const double F[9], double mu, double lam, double P[9]);
void or_composite_jacobian(const double F[9], double mu, double lam, double J[81]);
/* the logarithmic volume barrier variant (Sec. 4.1 Eq. pd_log_volume): its stretch step (the Newton of
 * or_prox_stretch without the I1 term), and the composite (2 mu R + lam P_log) / (2 mu + lam) whose
 * barrier step runs with the means mu_bar, lam_bar and penalty lam_bar, with its 9x9 Jacobian */
int or_logvol_stretch(const double sF[3], double mu, double lam, double k, double s_out[3]);
void or_logvol_map(const double F[9], double mu_bar, double lam_bar, double mu, double lam, double P[9]);
void or_logvol_jacobian(const double F[9], double mu_bar, double lam_bar, double mu, double lam, double J[81]);
void or_sym3_eig(const double H[9], double kappa[3], double Q[9]);
void or_tr_filter(const double H[9], double tau, double k, double Ht[9], double Dinv[9]);
int or_aa_step(int n, int m, double* Hq, double* Hg, int* hn, const double* q, const double* qhat,
               const unsigned char* mask, double* qnew, double* gamma_out);

/* --- global level --- */
/* b(q) over all vertices (3*nv), without the constant part c; pinned rows included */
void or_local_rhs(const or_scene* s, const double* q, double* b_all);
/* constant part of the right-hand side over all vertices (pinned rows meaningless) */
void or_const_rhs(const or_scene* s, const double* q_t, const double* v_t, const double* f_ext, double* c_all,
                  double* qtilde_all);
/* x = A~^{-1} r on free vertices, per axis (r, x over all vertices; pinned entries ignored / zeroed) */
void or_apply_Ainv(const or_scene* s, const double* r_all, double* x_all);
/* y = A~ x over all vertices (free rows and columns only) */
void or_apply_A(const or_scene* s, const double* x_all, double* y_all);
/* y = K x, K = db/dq at configuration q with TR parameter tau (free rows/cols only) */
void or_apply_K(const or_scene* s, const double* q, double tau, const double* x_all, double* y_all);
double or_primal_phi(const or_scene* s, const double* q, const double* qtilde);

/* istats: [0] iterations, [1] AA resets, [2] newton cap hits, [3] max newton iters, [4] status
 * dstats: [0..3] last gate norms (dq, q, db, b)
 * force_iters > 0 runs exactly that many PD iterations (gate ignored);
 * record: if non-NULL, iterates q^k (k = 0..rec_max-1) are stored there. */
int or_step_forward(const or_scene* s, const double* q_t, const double* v_t, const double* f_ext, const double* q0,
                    double* q_next, double* v_next, double* q_star_m1, int force_iters, int m_override,
                    int rec_max, double* rec, int* istats, double* dstats);

/* istats: [0] adjoint iterations, [1] status; dstats: [0] rho, [1] tau, [2] dphi_act, [3] dphi_mod
 * adj_mode 0: fixed-point iteration to eps_adj; 1: dense direct solve (small meshes) */
int or_step_backward(const or_scene* s, const double* q_t, const double* v_t, const double* f_ext,
                     const double* q_star, const double* q_star_m1, const double* gq_next, const double* gv_next,
                     double* gq_t, double* gv_t, double* gf_ext, double* g_logE, int adj_mode, double tau_force,
                     int* istats, double* dstats);

/* Contact (Sec. 4.7, frictionless reading): K rows, each on vertex cv[c] with unit normal cn[3c..3c+2] and
 * offset cg[c] (gap n.q - g).  Forward: lambda (K) receives the converged impulses, dstats[4] the final
 * FB residual; the dual gate also requires that residual <= fb_tol. */
int or_step_forward_contact(const or_scene* s, const double* q_t, const double* v_t, const double* f_ext,
                            const double* q0, double* q_next, double* v_next, double* q_star_m1, int K,
                            const int* cv, const double* cn, const double* cg, double fb_tol, double* lambda,
                            int* istats, double* dstats);
/* Backward with the forward's contact rows and impulses; the active set (lambda > 1e-10 max lambda) is held
 * fixed.  adj_mode 1 solves the dense saddle-point system, 0 the projected fixed point. */
int or_step_backward_contact(const or_scene* s, const double* q_t, const double* v_t, const double* f_ext,
                             const double* q_star, const double* q_star_m1, const double* gq_next,
                             const double* gv_next, double* gq_t, double* gv_t, double* gf_ext, double* g_logE,
                             int adj_mode, double tau_force, int K, const int* cv, const double* cn,
                             const double* cg, const double* lambda, int* istats, double* dstats);
/* Coulomb friction (Sec. 4.7; the reading is stated in pd_oracle.c): the same contact rows, each a frame
 * (n, t1, t2) with impulses lambda3[3c..3c+2] (normal, t1, t2) and friction coefficient mu_f > 0.
 * dstats[4] = final residual, dstats[5] = Newton steps of the last contact solve. */
int or_step_forward_friction(const or_scene* s, const double* q_t, const double* v_t, const double* f_ext,
                             const double* q0, double* q_next, double* v_next, double* q_star_m1, int K,
                             const int* cv, const double* cn, const double* cg, double mu_f, double fb_tol,
                             double* lambda3, int force_iters, int* istats, double* dstats);
int or_step_backward_friction(const or_scene* s, const double* q_t, const double* v_t, const double* f_ext,
                              const double* q_star, const double* q_star_m1, const double* gq_next,
                              const double* gv_next, double* gq_t, double* gv_t, double* gf_ext, double* g_logE,
                              int adj_mode, double tau_force, int K, const int* cv, const double* cn,
                              const double* cg, double mu_f, const double* lambda3, int* istats, double* dstats);
/* Bilateral rows and restitution (readings in pd_oracle.c): kind (K, 1 = bilateral equality row, NULL: all
 * unilateral), rest_on with coefficient e_rest, mu_f (0: frictionless; bilateral rows need mu_f = 0);
 * lambda has K (or 3K with friction) entries.  The backward's g_gap (K, frictionless) receives dL/dg_c. */
int or_step_forward_contact_ext(const or_scene* s, const double* q_t, const double* v_t, const double* f_ext,
                                const double* q0, double* q_next, double* v_next, double* q_star_m1, int K,
                                const int* cv, const double* cn, const double* cg, const unsigned char* kind,
                                int rest_on, double e_rest, double mu_f, double fb_tol, double* lambda,
                                int force_iters, int* istats, double* dstats);
int or_step_backward_contact_ext(const or_scene* s, const double* q_t, const double* v_t, const double* f_ext,
                                 const double* q_star, const double* q_star_m1, const double* gq_next,
                                 const double* gv_next, double* gq_t, double* gv_t, double* gf_ext, double* g_logE,
                                 int adj_mode, double tau_force, int K, const int* cv, const double* cn,
                                 const double* cg, const unsigned char* kind, int rest_on, double e_rest,
                                 double mu_f, const double* lambda, double* g_gap, int* istats, double* dstats);
/* the contact frame of a unit normal */
void or_contact_frame(const double n[3], double t1[3], double t2[3]);
/* the friction Newton alone: G (K x K block of A~^{-1}), normals (K x 3), free kinematics u0 (3K: gap and
 * the slip along t1, t2), from lambda = 0; returns its iterations */
int or_friction_ncp(int K, const double* G, const double* normals, const double* u0, double mu, double* lambda,
                    double* res);
/* Delassus operator W (K x K, row-major) of a contact set */
void or_contact_W(const or_scene* s, int K, const int* cv, const double* cn, double* W_out);
/* FB semi-smooth Newton on delta = dfree + W lambda, from lambda = 0; returns its iterations */
int or_fb_lcp(int K, const double* W, const double* dfree, double* lambda, double* res);

#ifdef __cplusplus
}
#endif
#endif
