/*
 * CPU oracle for the batched backward-Euler contact step -- TEST INFRASTRUCTURE.
 *
 * Plain single-threaded FP64 C++ written from the paper (Ostrich, Sec. III,
 * Eqs. (1)-(19)).  Only the tests, the smoke check and the benchmark's CPU
 * baseline may load it.  It shares no code or header with the GPU library.
 *
 * All pointers are HOST pointers.  Arrays are world-major and packed as
 * described by the scene generators (scenes/__init__.py).  Return value 0 on
 * success, negative on a malformed argument.
 */
#ifndef OSTRICH_REF_H
#define OSTRICH_REF_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t n_worlds;
  const int32_t* body_off;     /* [W+1] */
  const double*  body_mass;    /* [NB] */
  const double*  body_inertia; /* [NB*3] principal moments, body frame */
  const int32_t* joint_off;    /* [W+1] */
  const int32_t* joint_body;   /* [NJ*2] world-local (a, b) */
  const double*  joint_frame;  /* [NJ*18] anchor_a, anchor_b, axis_b, perp1_a, perp2_a, axis_a */
  const int32_t* joint_act;    /* [NJ] 0 none, 1 torque, 2 velocity servo, 3 torque + damping servo,
                                  4 position servo */
  const double*  joint_kp;     /* [NJ] servo gain */
  const int32_t* ctrl_off;     /* [W+1] */
  const int32_t* slot_off;     /* [W+1] */
  const int32_t* slot_int;     /* [NS*4] kind, body_a, body_b, feature */
  const double*  slot_real;    /* [NS*9] local offset(3), radius, mu, face half-height, rim-circle axis(3)
                                  (body frame, unit; all zero for a sphere or point proxy) */
  const int32_t* obs_off;      /* [W+1] */
  const double*  obs_box;      /* [NO*6] centre(3), half extents(3) */
  const int32_t* lam_off;      /* [W+1] */
  const int32_t* contact_cap;  /* [W] */
  const int32_t* world_hmap;   /* [W] heightmap index or -1 */
  int32_t hmap_n;              /* vertices per side */
  double hmap_spacing;
  const double* hmap_origin;   /* [NH*2] */
  const double* hmap_heights;  /* [NH*n*n], index i*n + j, i along x */
  const double* joint_kd;      /* [NJ] derivative gain of position servos */
} ostrich_ref_batch;

typedef struct {
  double h;
  double gravity[3];
  double tol;
  int32_t k_max;
  int32_t k_min;
  double eps;        /* FB / norm smoothing */
  double delta_g;    /* guarded denominators */
  double delta_reg;  /* relative Schur diagonal regularisation */
  double delta0;     /* contact activation margin */
  int32_t sigma_mode;/* 1: unit-scaled FB arguments, 0: sigma = 1 */
  int32_t n_feat;    /* heightmap features per proxy */
  int32_t newton_mode;/* 0: generalized Jacobian of the constraint rows, 1: W frozen (symmetric) */
  int32_t ls_max;    /* step halvings of the residual-decrease step length (0: full steps) */
  int32_t truncate;  /* 1: contact geometry held fixed within the step in the q- pull-back */
  double delta_reg_adj; /* relative regularisation of the adjoint's system (Eq. (16)): h delta_reg_adj
                          diag(J M~^-1 J^T) in its multiplier block; the Newton iterations use delta_reg */
} ostrich_ref_params;

/* status bits */
#define OSTRICH_REF_CONVERGED 1
#define OSTRICH_REF_BUDGET 2
#define OSTRICH_REF_NONFINITE 4
#define OSTRICH_REF_REGULARIZED 8
#define OSTRICH_REF_OVERFLOW 16

int ostrich_ref_step_forward(const ostrich_ref_batch* b, const ostrich_ref_params* p,
                             const double* q_prev, const double* u_prev, const double* lam_prev,
                             const double* ctrl, double* q_next, double* u_next, double* lam_next,
                             int32_t* act_slot, int32_t* n_act, int32_t* status, int32_t* iters,
                             double* resnorm);

/* mode 0: exact implicit-function-theorem adjoint; mode 1: the paper's lagged
 * Schur adjoint (Eqs. (18)-(19)) followed by the exact residual pull-back;
 * mode 2: the adjoint solved with the forward's own Newton matrix (the
 * generalized Jacobian of the rows without the geometric stiffness of
 * J^T lambda), the paper's reuse of the forward's matrix for this forward,
 * followed by the same pull-back.  Other modes: -1. */
int ostrich_ref_step_adjoint(const ostrich_ref_batch* b, const ostrich_ref_params* p,
                             const double* q_prev, const double* u_prev, const double* lam_prev,
                             const double* ctrl, const double* u_next, const double* lam_next,
                             const double* gq_next, const double* gu_next,
                             double* gq_prev, double* gu_prev, double* g_ctrl, int32_t mode);

/* The adjoint above and, by the same pull-back (Eq. (17)) with a model
 * parameter as xi, the cotangents of every body's mass (g_mass, per body),
 * every slot's friction coefficient (g_mu, per slot; zero for slots without an
 * active contact) and every joint's servo gain (g_kp, per joint; zero for
 * joints without a servo row).  All outputs are required. */
int ostrich_ref_step_adjoint_params(const ostrich_ref_batch* b, const ostrich_ref_params* p,
                                    const double* q_prev, const double* u_prev, const double* ctrl,
                                    const double* u_next, const double* lam_next, const double* gq_next,
                                    const double* gu_next, double* gq_prev, double* gu_prev, double* g_ctrl,
                                    double* g_mass, double* g_mu, double* g_kp, int32_t mode);

/* Natural cubic spline basis B[T*K]: control at step k is sum_j B[k,j] knot_j,
 * knots at t_j = j*T*h/(K-1), step k samples t = k*h. */
int ostrich_ref_spline_basis(int32_t T, int32_t K, double h, double* B);

/* T-step rollout with loss |xy(loss_body) - target|^2 at step T, and its
 * gradient by the per-step adjoint (mode as above).  knots [n_ctrl*K]. */
/* Shaped loss of the optimisation workloads; per world w, with p_k the xy,
 * psi_k the yaw (angle of the body x axis in the ground plane) and v_k the
 * linear velocity of the loss body in state k, a_k the controls of step k and
 * (r_k, rho_k) the reference of step k:
 *   L_w = w_pos |p_T - p*|^2 + w_head (1 - cos(psi_T - psi*)) + w_vel |v_T|^2
 *       + (w_ctrl / T) sum_{k<T} |a_k|^2 + (w_track / T) sum_{k=1..T} |p_k - r_k|^2
 *       + (w_yaw / T) sum_{k=1..T} (1 - cos(psi_k - rho_k)).
 * goal [W*3] (x*, y*, psi*); ref [T*W*3], entry (k - 1) W + w = (r_k, rho_k),
 * read only when w_track or w_yaw is not zero.  Host arrays. */
typedef struct {
  double w_pos, w_head, w_vel, w_ctrl, w_track, w_yaw;
  const double* goal;
  const double* ref;
} ostrich_ref_loss;

int ostrich_ref_rollout(const ostrich_ref_batch* b, const ostrich_ref_params* p,
                        const double* q0, const double* u0, const double* knots, int32_t K,
                        int32_t T, const int32_t* loss_body, const double* target,
                        double* loss, double* qT, double* uT, double* g_q0, double* g_u0,
                        double* g_knots, int32_t mode, int32_t* status_or);

/* The rollout above with the shaped loss in place of the final-xy loss. */
int ostrich_ref_rollout_shaped(const ostrich_ref_batch* b, const ostrich_ref_params* p, const double* q0,
                               const double* u0, const double* knots, int32_t K, int32_t T,
                               const int32_t* loss_body, const ostrich_ref_loss* spec, double* loss, double* qT,
                               double* uT, double* g_q0, double* g_u0, double* g_knots, int32_t mode,
                               int32_t* status_or);


/* Inspection of one world at a given iterate (u, lam in active-row order):
 * sizes, raw residual F [n_u+m], row scale D [n_u+m], constraint Jacobian
 * J [m*n_u], generalized Jacobian of the scaled constraint rows Gu [m*n_u]
 * and Gl [m*m], Newton Schur matrix A [m*m] and rhs [m], exact Jacobian of
 * the scaled residual H [(n_u+m)^2], FB scale of each row [m].  Output
 * pointers may be NULL. */
int ostrich_ref_inspect(const ostrich_ref_batch* b, const ostrich_ref_params* p, int32_t world,
                        const double* q_prev, const double* u_prev, const double* ctrl,
                        const double* u_it, const double* lam_it, int32_t* m_out, int32_t* nu_out,
                        double* F, double* J, double* D, double* Gu, double* Gl, double* A, double* rhs,
                        double* H, double* sigma, int32_t* act_slot);

#ifdef __cplusplus
}
#endif
#endif
