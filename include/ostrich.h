/*
 * ostrich.h -- C ABI of the MI355X (gfx950) implementation of the batched
 * backward-Euler contact step with implicit differentiation (Ostrich:
 * Kucera & Zimmermann, "Taking Large Strides Through Stiff Contact in
 * Differentiable Dynamics").
 *
 * The method (Sec. III of the paper):
 *   - Eqs. (1)-(2): backward Euler in maximal coordinates, q+ = q- + h G(q-) u+,
 *     M~ (u+ - u-) = h (f_ext + J(q+)^T lambda+), J implicit at q+, G at q-;
 *   - Eqs. (3)-(8): joints, Fischer-Burmeister normal contact, compliance-form
 *     Coulomb friction with the weight W >= 0 and the cone clamp, implicit
 *     servo rows;
 *   - Eqs. (9)-(13): the stacked residual solved by non-smooth Newton on the
 *     Schur system, with best-iterate selection over a fixed budget (Sec. III-C);
 *   - Eqs. (14)-(19): the implicit-function adjoint that reuses the forward
 *     Schur factor (Sec. III-D).
 *
 * Conventions.  All arrays are world-major and packed as the scene generators
 * describe them: per body q = (x, y, z, qx, qy, qz, qw) (unit quaternion, x y z
 * w order) and u = (v, w) (centre-of-mass velocity and angular velocity, both
 * in the world frame); lambda is stored per world as [5 per revolute joint]
 * [1 per servo row][3 per contact slot (normal, t1, t2)], slot-ordered, so a
 * warm start matches contacts by slot.  All numbers are FP64, indices int32.
 *
 * Ownership.  Every array pointer passed to ostrich_step_* and
 * ostrich_rollout is a DEVICE pointer owned by the caller; the library never
 * allocates on these paths.  ostrich_ctx_create copies the batch descriptor
 * (pointers only, the arrays stay the caller's and must outlive the context)
 * and reads a few offsets to the host once to size its launches.  Every call
 * is asynchronous on the given HIP stream.
 *
 * Errors.  Calls return 0 on success or a negative OSTRICH_E_* code; the
 * calling thread's last message is available from ostrich_last_error().
 * Per-world solver outcomes are status bits (OSTRICH_ST_*), not errors: a step
 * that does not reach the tolerance returns its best iterate and sets
 * OSTRICH_ST_BUDGET (Sec. III-C).
 */
#ifndef OSTRICH_H
#define OSTRICH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OSTRICH_E_ARG (-1)         /* malformed argument (checked on the host) */
#define OSTRICH_E_HIP (-2)         /* a HIP runtime call failed */
#define OSTRICH_E_WORKSPACE (-3)   /* workspace smaller than required */
#define OSTRICH_E_UNSUPPORTED (-4) /* world too large for the on-chip solver */

#define OSTRICH_ST_CONVERGED 1     /* residual norm <= tol */
#define OSTRICH_ST_BUDGET 2        /* budget exhausted: best iterate returned */
#define OSTRICH_ST_NONFINITE 4     /* non-finite residual or factor */
#define OSTRICH_ST_REGULARIZED 8   /* Schur regularisation had to be raised */
#define OSTRICH_ST_OVERFLOW 16     /* more active contacts than contact_cap */
#define OSTRICH_ST_ADJ_INEXACT 32  /* adjoint: the Krylov solve of the exact system ended above its stop
                                      (applications ran out or a value was not finite); the gradient is
                                      the last iterate's */
#define OSTRICH_ST_LOSS_BODY 64    /* rollout: loss_body[w] is not a body of world w (loss set to NaN,
                                      no cotangent written) */

/* Packed batch of worlds (device pointers).  Offsets have n_worlds+1 entries. */
typedef struct {
  int32_t n_worlds;
  const int32_t* body_off;     /* bodies of world w: [body_off[w], body_off[w+1]) */
  const double* body_mass;     /* [NB] */
  const double* body_inertia;  /* [NB*3] principal moments in the body frame */
  const int32_t* joint_off;
  const int32_t* joint_body;   /* [NJ*2] world-local body indices (parent a, child b) */
  const double* joint_frame;   /* [NJ*18] anchor_a, anchor_b, axis_b, perp1_a, perp2_a, axis_a (body frames) */
  const int32_t* joint_act;    /* [NJ] 0 none, 1 torque, 2 velocity servo, 3 torque + zero-speed servo,
                                  4 position servo (the control is the target angle) */
  const double* joint_kp;      /* [NJ] servo gain k_p (compliance 1/k_p of a velocity servo, Eq. (8)) */
  const int32_t* ctrl_off;     /* controls: one per actuated joint, in joint order */
  const int32_t* slot_off;     /* contact candidate slots */
  const int32_t* slot_int;     /* [NS*4] kind (0 plane, 1 static box, 2 face of body b, 3 heightmap mesh),
                                  body a, body b, obstacle (kind 1) or candidate rank (kind 3) */
  const double* slot_real;     /* [NS*9] proxy offset in body a (3), proxy radius, mu, face half-height,
                                  rim-circle axis in body a (3).  A zero axis makes the proxy a sphere
                                  (a point for radius 0).  A unit axis makes it the circle of that radius
                                  about the offset, normal to the axis: an edge of a cylindrical wheel
                                  (Sec. IV-D's wheels), which reaches r sqrt(1 - (n . a)^2) below its
                                  centre along a contact normal n; static features only (kinds 0, 1, 3).
                                  Context creation fails with OSTRICH_E_ARG for an axis that is not a
                                  unit vector, a rim circle of radius <= 0 or one on a kind-2 slot. */
  const int32_t* obs_off;
  const double* obs_box;       /* [NO*6] centre (3), half extents (3): axis-aligned static boxes */
  const int32_t* lam_off;      /* multiplier layout described above */
  const int32_t* contact_cap;  /* [W] maximum active contacts of the world */
  const int32_t* world_hmap;   /* [W] heightmap index or -1 */
  int32_t hmap_n;
  double hmap_spacing;
  const double* hmap_origin;
  const double* hmap_heights;
  const double* joint_kd;      /* [NJ] derivative gain k_d of position servos: compliance
                                  1 / (k_d + h k_p) and b_c = k_p (theta(q-) - theta*) / (k_d + h k_p),
                                  theta the angle of R_b perp1_a from R_a perp1_a about R_a axis_a
                                  (Eq. (8)); unused by other joints */
} ostrich_batch;

/* Solver parameters (host struct, copied at context creation). */
typedef struct {
  double h;            /* time step (s) */
  double gravity[3];
  double tol;          /* Newton tolerance on the residual norm */
  int32_t k_max;       /* Newton budget */
  int32_t k_min;       /* best-iterate floor (Sec. III-C) */
  double eps;          /* smoothing of the FB function and of norms */
  double delta_g;      /* guard of denominators */
  double delta_reg;    /* relative Schur diagonal regularisation of the Newton iterations (> 0) */
  double delta0;       /* contact activation margin (m) */
  int32_t ls_max;      /* step-length halvings of the residual-decrease test */
  int32_t refine;      /* most Krylov operator applications of the adjoint; 0: the stored factor alone, i.e.
                          the system with the forward's Newton matrix (without the geometric stiffness of
                          J^T lambda), the paper's reuse of the forward's factor (Sec. III-D); > 0: towards
                          the exact implicit-function system (OSTRICH_ST_ADJ_INEXACT if not reached) */
  int32_t team;        /* threads per world (64, 128 or 256) before autotuning; 0: 128, or 256 for a
                          bucket whose on-chip workspace fits only one 128-thread workgroup per CU */
  int32_t schedule;    /* OSTRICH_SCHED_FIXED or OSTRICH_SCHED_BUCKETED */
  int32_t truncate;    /* 1: the adjoint treats the contact geometry as a constant of the step, so no
                          derivative with respect to q- passes through a contact row or its force
                          (the truncated position pull-back of the terrain task, Sec. IV-D); 0: the
                          complete pull-back of Eq. (17) */
  int32_t linear_solver; /* Newton step: OSTRICH_LIN_LU (0) the banded LU of the Schur matrix;
                          OSTRICH_LIN_KRYLOV (1) the paper's iterative alternative, a
                          matrix-free Krylov solve (restarted GMRES, Jacobi preconditioner,
                          products with A from the row blocks), the matrix never formed.
                          OSTRICH_LIN_KRYLOV is switched off in this version: context creation
                          returns OSTRICH_E_UNSUPPORTED for it */
  int32_t krylov_iters; /* products with A per Newton step at most (0: 16, as the paper's 16
                          inner iterations); the solve stops earlier at 1e-12 of |rhs| */
  int32_t tier_contacts; /* tiered on-chip launches (a launch shape, not arithmetic: results are the
                          same bits either way).  A first launch carves each workgroup's LDS for
                          at most this many active contacts, so that more worlds share a CU, and
                          hands every world with more to a second, persistent launch with the full
                          carve.  The two launches run side by side: a planning pass counts each
                          world's active contacts at q- (the adjoint reads them from the tape;
                          a terrain slot, whose mesh search is the step's, counts with the
                          world's contacts of its previous step) and sends the worlds that exceed
                          the first carve to the second launch from the start; a world the first
                          launch still finds too large is taken by a last launch after both.
                          0: automatic, the largest count that raises the workgroups per CU
                          (two wavefronts per SIMD), if any; -1: never; n > 0: n, if below the
                          bucket's contact cap.  ostrich_autotune also times the untiered launch */
  double delta_reg_adj; /* relative regularisation (> 0) of the factor written to the tape, the one the
                          adjoint solves with: the multiplier block of the adjoint's system (Eq. (16))
                          carries h delta_reg_adj diag(J M~^-1 J^T), so the gradient differs from the
                          implicit-function derivative by O(delta_reg_adj).  The Newton iterations'
                          delta_reg does not change the root and need not be small; this one should be.
                          It cannot be arbitrarily small either: where a contact set is statically
                          indeterminate (a robot on four wheels) the multiplier block has a null
                          direction that only this term fixes, and the cotangents of q- that see it
                          lose digits as 1 / delta_reg_adj.  1e-8 keeps both below the 1e-6
                          gradient bar (bias about 4e-7, lost digits about 1e-7).  Cylindrical
                          wheels standing with both rim circles on flat ground make the rows
                          nearly dependent in the same way (two rims and the axle's hinge): there
                          the q- cotangents of those wheels' positions along their axles agree
                          between two implementations only to about 4e-4 at 1e-8 (1.6e-7 at 1e-6).
                          Raised tenfold while the factor's pivot test fails, the value used being
                          recorded in the tape */
} ostrich_params;

#define OSTRICH_LIN_LU 0
#define OSTRICH_LIN_KRYLOV 1

/* Launch schedules.  FIXED: every world in one launch shaped for the largest
 * world of the batch.  BUCKETED: worlds grouped by row capacity (edges 16, 32,
 * 64, 96, 128, 192, 256, 384), one launch per group, each shaped for its own
 * worlds and tunable by ostrich_autotune.  The per-world arithmetic, and so
 * every result, is identical under both. */
#define OSTRICH_SCHED_FIXED 0
#define OSTRICH_SCHED_BUCKETED 1

typedef struct ostrich_ctx ostrich_ctx;

/* Last error message of the calling thread (never NULL). */
const char* ostrich_last_error(void);

/* Create a context for a packed batch.  Reads body/joint/slot offsets,
 * joint_act and contact_cap to the host once to size the launches, and
 * allocates its own small tables (per-bucket world lists, per-world tape
 * offsets) and, for worlds whose Schur matrix does not fit on chip, one slice
 * of device memory per resident workgroup.  Fails with OSTRICH_E_ARG for an
 * empty batch (n_worlds < 1), a world without bodies or decreasing offsets,
 * and with OSTRICH_E_UNSUPPORTED if a world does not fit a workgroup even then. */
int ostrich_ctx_create(const ostrich_batch* batch, const ostrich_params* params, ostrich_ctx** out);
int ostrich_ctx_destroy(ostrich_ctx* ctx);

/* Bytes of device memory the context holds (its tables, the device scratch of
 * worlds kept off chip, the plain path's workspace and the measurement
 * counters), as allocated so far: ostrich_autotune and ostrich_ctx_timing may
 * add to it. */
size_t ostrich_ctx_device_bytes(const ostrich_ctx* ctx);

/* Sizes the caller allocates: the per-step tape of all worlds (bytes; world w
 * holds mr_w^2 + 4 doubles, mr_w its row capacity), and
 * the rollout workspace for horizon T and checkpoint interval k (0: keep every
 * state and tape; k >= 1: keep every k-th state and recompute segments). */
size_t ostrich_tape_bytes(const ostrich_ctx* ctx);
size_t ostrich_rollout_workspace_bytes(const ostrich_ctx* ctx, int32_t T, int32_t ckpt_every);

/* Capacities used for the launches: bodies, joints, slots, contacts, rows
 * per world (maxima over the batch), and the largest LDS bytes of one
 * workgroup.  out[6]. */
int ostrich_ctx_caps(const ostrich_ctx* ctx, int64_t* out);

/* Launch schedule: returns the number of buckets and, if out is not NULL,
 * writes for each of the first max_buckets buckets eight int32 (row capacity,
 * number of worlds, threads per world, storage split: 0 on chip / 1 Schur
 * matrix and Jacobian blocks in device memory, LDS bytes per workgroup of the
 * full carve, tuned flag, the contact capacity of a tiered first launch (0:
 * untiered), and that launch's LDS bytes per workgroup). */
int ostrich_ctx_schedule(const ostrich_ctx* ctx, int32_t* out, int32_t max_buckets);

/* Measurement of the forward and adjoint steps (a set-up facility, not for
 * the hot path).  mode 1: reset and start: every later ostrich_step_forward
 * call with n_act and iters, and every ostrich_step_adjoint call (including
 * those inside ostrich_rollout), is bracketed by a pair of HIP events on its
 * stream, and a one-workgroup kernel adds the step's algorithmic work to
 * device counters.  A forward step counts FP64 flops from each world's rows m
 * and Newton iteration count k (Sec. III-C, one Schur factor and solve per
 * iteration): the roofline count k (m^3/3 + 14 m^2 + 170 m), and this
 * implementation's finer count k (26 m^2 + 2 m^3 / 3 + 800 m) + 400 m, plus
 * 24 m^2 + 2 m^3 / 3 when a tape is written.  An adjoint step counts bytes
 * (Sec. III-D, one solve with the stored factor): the roofline count, states
 * read and written (2 x 13 doubles per body), multipliers read and a
 * triangular factor of m (m + 1) / 2 doubles; and the finer count, the band
 * the tape stores, m (2 bw + 1) - bw (bw + 1) doubles for the half band bw
 * recorded there, with the states, multipliers and cotangents read and
 * written.  mode 0: stop.  mode 2 (forward) and mode 3 (adjoint): synchronise
 * the device and write out[4] = (timed calls, their total duration in ms,
 * the roofline count, the finer count). */
int ostrich_ctx_timing(ostrich_ctx* ctx, int32_t mode, double* out);

/* Autotuner of the batching system: times `reps` forward steps of every bucket
 * from the given state (device pointers, as for ostrich_step_forward) under
 * each candidate launch (64, 128 or 256 threads per world; Schur matrix on
 * chip or in device memory) and keeps the fastest.  Synchronises the stream and
 * allocates temporary device memory: a set-up call, not for the hot path.
 * Results of later steps do not depend on the choice. */
int ostrich_autotune(ostrich_ctx* ctx, const double* q, const double* u, const double* lam, const double* ctrl,
                     int32_t reps, void* stream);

/* One backward-Euler step of every world (Sec. III-A..C, A1-A8 of the hot
 * path): contact refresh at q-, fused Newton loop, best iterate, q+.
 *   q_prev [NB*7], u_prev [NB*6], lam_prev [NL]: state s-;  ctrl [NCTRL]
 *   q_next, u_next, lam_next: state s+ (written)
 *   act_slot [NS]: per world the active slot ids in ascending order, -1 padded
 *   n_act, status, iters [W] int32;  resnorm [W] residual norm of s+
 *   tape: NULL or ostrich_tape_bytes() bytes; receives the Schur factor at s+. */
int ostrich_step_forward(ostrich_ctx* ctx, const double* q_prev, const double* u_prev, const double* lam_prev,
                         const double* ctrl, double* q_next, double* u_next, double* lam_next, int32_t* act_slot,
                         int32_t* n_act, int32_t* status, int32_t* iters, double* resnorm, void* tape,
                         void* stream);

/* ostrich_step_forward for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same arguments, kernels and results, but the device scratch
 * the launches need (the deferral queues of tiered buckets and the
 * per-workgroup slices of worlds kept in device memory) comes from a static
 * device array of 32 MiB inside the library (one per GPU, held until the
 * process ends) instead of the context's allocations.  The call allocates
 * nothing and records no timing.  A bucket kept in device memory runs on as
 * many persistent workgroups as its slices that fit (at least one), which
 * changes the time, not the results.  Errors: as ostrich_step_forward, and
 * OSTRICH_E_WORKSPACE when the batch needs more than the static scratch.
 * Every call on a GPU shares that GPU's array, so calls that overlap on one
 * GPU (other streams, other threads, other contexts) race: serialise them. */
int ostrich_step_forward_noalloc(ostrich_ctx* ctx, const double* q_prev, const double* u_prev,
                                 const double* lam_prev, const double* ctrl, double* q_next, double* u_next,
                                 double* lam_next, int32_t* act_slot, int32_t* n_act, int32_t* status,
                                 int32_t* iters, double* resnorm, void* tape, void* stream);

/* Adjoint of one step (Sec. III-D, Eqs. (16)-(19)): given s-, the controls,
 * s+ (u_next, lam_next) and the tape written by the forward call, map the
 * loss cotangents (gq_next [NB*7], gu_next [NB*6]) to gq_prev, gu_prev and
 * g_ctrl [NCTRL].  The stored factor is back-solved; with refine > 0 the
 * exact implicit-function Jacobian, whose velocity block adds the geometric
 * stiffness h K = h d(J(u)^T lambda)/du that the factor leaves out, is solved
 * by restarted GMRES on the 6 NB velocity unknowns, preconditioned by the
 * factor, with at most `refine` operator applications (params.refine if < 0)
 * and a stop at 1e-12 of the relative residual; refine = 0 keeps the factor's
 * solve alone.  The adjoint kernel's LDS adds the Krylov workspace,
 * 60 NB_cap + 106 doubles per world (NB_cap: most bodies of a world).
 * adj_status [W] int32 (device, may be NULL): OSTRICH_ST_ADJ_INEXACT is ORed
 * into entry w when world w's Krylov solve ends above its stop (other entries
 * and bits are left as they are). */
int ostrich_step_adjoint(ostrich_ctx* ctx, const double* q_prev, const double* u_prev, const double* ctrl,
                         const double* u_next, const double* lam_next, const void* tape, const double* gq_next,
                         const double* gu_next, double* gq_prev, double* gu_prev, double* g_ctrl, int32_t refine,
                         int32_t* adj_status, void* stream);

/* The adjoint of ostrich_step_adjoint together with the cotangents of the
 * model parameters (Eq. (17) with xi a parameter, the paper's system
 * identification use): g_mass [NB] of every body's mass, g_mu [NS] of every
 * slot's friction coefficient (zero for slots without an active contact at
 * q-), g_kp [NJ] of every joint's servo gain (zero for joints without a servo
 * row).  Device pointers, all required (OSTRICH_E_ARG otherwise); every entry
 * is written.  The FB scales and the Schur regularisation are held as in the
 * solve, so these are the derivatives of the solved, regularised step. */
int ostrich_step_adjoint_params(ostrich_ctx* ctx, const double* q_prev, const double* u_prev, const double* ctrl,
                                const double* u_next, const double* lam_next, const void* tape,
                                const double* gq_next, const double* gu_next, double* gq_prev, double* gu_prev,
                                double* g_ctrl, double* g_mass, double* g_mu, double* g_kp, int32_t refine,
                                int32_t* adj_status, void* stream);

/* The same two steps restricted to the worlds listed in `worlds` (device
 * int32 [n], distinct ids): only those worlds' entries of the state, status
 * and tape arrays are read or written.  The serving loop uses them to advance
 * the worlds of many requests, each at its own step, in one launch. */
int ostrich_step_forward_list(ostrich_ctx* ctx, const int32_t* worlds, int32_t n, const double* q_prev,
                              const double* u_prev, const double* lam_prev, const double* ctrl, double* q_next,
                              double* u_next, double* lam_next, int32_t* act_slot, int32_t* n_act, int32_t* status,
                              int32_t* iters, double* resnorm, void* tape, void* stream);
int ostrich_step_adjoint_list(ostrich_ctx* ctx, const int32_t* worlds, int32_t n, const double* q_prev,
                              const double* u_prev, const double* ctrl, const double* u_next, const double* lam_next,
                              const void* tape, const double* gq_next, const double* gu_next, double* gq_prev,
                              double* gu_prev, double* g_ctrl, int32_t refine, int32_t* adj_status, void* stream);

/* The plain path, a comparison baseline with the same arguments and the same
 * results (the same arithmetic, bit for bit): ostrich_step_forward_plain makes
 * one launch per world per Newton iteration (plus one set-up and one
 * finalisation launch per world, k_max + 2 in all), with the world's state in
 * device memory between launches; ostrich_step_adjoint_plain makes one launch
 * per world.  The plain forward steps with the banded LU only
 * (OSTRICH_E_UNSUPPORTED with linear_solver = OSTRICH_LIN_KRYLOV). */
int ostrich_step_forward_plain(ostrich_ctx* ctx, const double* q_prev, const double* u_prev, const double* lam_prev,
                               const double* ctrl, double* q_next, double* u_next, double* lam_next,
                               int32_t* act_slot, int32_t* n_act, int32_t* status, int32_t* iters, double* resnorm,
                               void* tape, void* stream);
int ostrich_step_adjoint_plain(ostrich_ctx* ctx, const double* q_prev, const double* u_prev, const double* ctrl,
                               const double* u_next, const double* lam_next, const void* tape, const double* gq_next,
                               const double* gu_next, double* gq_prev, double* gu_prev, double* g_ctrl,
                               int32_t refine, int32_t* adj_status, void* stream);

#define OSTRICH_FORWARD 1
#define OSTRICH_BACKWARD 2
#define OSTRICH_BOTH (OSTRICH_FORWARD | OSTRICH_BACKWARD) /* forward, then backward, in one call */

/* T-step rollout (the optimisation workload of Sec. IV: a rollout, its loss
 * and the adjoint of Sec. III-D over all steps) with controls from a spline
 * basis (ctrl_k = basis[k,:] . knots[c,:], basis [T*K] device, knots
 * [NCTRL*K]) and the loss |xy(loss_body) - target|^2 at step T (loss_body [W]
 * int32 device, loss_body[w] a body index of world w in [0, its body count):
 * read on the device, where an index outside that range gives loss[w] = NaN,
 * no cotangent, and OSTRICH_ST_LOSS_BODY in status_or[w]; target [W*2]).
 * FORWARD writes loss [W], qT, uT and checkpoints into the workspace;
 * BACKWARD (after a FORWARD with the same arguments and workspace) recomputes
 * each segment from its checkpoint and runs the adjoint steps in reverse,
 * writing g_q0, g_u0, g_knots: the gradients of sum_w loss_grad[w] loss[w]
 * (loss_grad [W] device, NULL for all ones).  status_or [W] (device, may be
 * NULL) is cleared by FORWARD and ORs the status bits of every forward step,
 * OSTRICH_ST_ADJ_INEXACT of every adjoint step and OSTRICH_ST_LOSS_BODY. */
int ostrich_rollout(ostrich_ctx* ctx, int32_t phase, const double* q0, const double* u0, const double* knots,
                    int32_t K, const double* basis, int32_t T, int32_t ckpt_every, const int32_t* loss_body,
                    const double* target, const double* loss_grad, double* loss, double* qT, double* uT,
                    double* g_q0, double* g_u0, double* g_knots, void* workspace, size_t workspace_bytes,
                    int32_t* status_or, void* stream);

/* Shaped loss of the optimisation workloads (Sec. IV-B: errors of the final
 * position and heading, the speed at the end, the size of the controls, and
 * the distance from a straight path at every step; Sec. IV-D: the distance from
 * and the yaw difference to a reference trajectory at every step, and the size
 * of the controls).  The paper lists the terms without their forms; per world
 * w, with p_k the xy, psi_k the yaw (the
 * heading of the body x axis in the ground plane) and v_k the linear velocity
 * of the loss body in state k, a_k the controls of step k, and (r_k, rho_k) the
 * reference of step k:
 *   L_w = w_pos |p_T - p*|^2 + w_head (1 - cos(psi_T - psi*)) + w_vel |v_T|^2
 *       + (w_ctrl / T) sum_{k=0}^{T-1} |a_k|^2
 *       + (w_track / T) sum_{k=1}^{T} |p_k - r_k|^2
 *       + (w_yaw / T) sum_{k=1}^{T} (1 - cos(psi_k - rho_k)).
 * goal [W*3] device: (x*, y*, psi*) per world.  ref [T*W*3] device: entry
 * (k - 1) W + w holds (r_k, rho_k); it is read only when w_track or w_yaw is
 * not zero (then it must not be NULL).  Weights must be finite. */
typedef struct {
  double w_pos, w_head, w_vel, w_ctrl, w_track, w_yaw;
  const double* goal;
  const double* ref;
} ostrich_loss;

/* ostrich_rollout with the shaped loss `spec` (host struct, device arrays;
 * read during the call) in place of the final-xy loss: the same phases,
 * workspace, checkpointing and outputs; loss [W] holds L_w, and the gradients
 * are those of sum_w loss_grad[w] L_w.  With P.truncate set every adjoint step
 * holds the contact geometry fixed (the terrain task of Sec. IV-D). */
int ostrich_rollout_shaped(ostrich_ctx* ctx, int32_t phase, const double* q0, const double* u0, const double* knots,
                           int32_t K, const double* basis, int32_t T, int32_t ckpt_every, const int32_t* loss_body,
                           const ostrich_loss* spec, const double* loss_grad, double* loss, double* qT, double* uT,
                           double* g_q0, double* g_u0, double* g_knots, void* workspace, size_t workspace_bytes,
                           int32_t* status_or, void* stream);

/* Device helpers of the trajectory-optimisation loop (Sec. IV: spline
 * controls, the final-position loss, Adam on the knots), all asynchronous on
 * `stream`, device pointers:
 *   ostrich_spline_controls: ctrl[k*nctrl + c] = sum_j basis[k*K + j] knots[c*K + j], k < T.
 *   ostrich_final_loss: for the n_worlds worlds whose body offsets start at
 *     body_off (n_worlds + 1 entries; body_off[i] indexes qT rows), loss[i] =
 *     |xy - target[i]|^2 of body loss_body[i] (loss may be NULL), and, if gq
 *     is not NULL, its cotangent 2 (xy - target) loss_grad[i] (loss_grad NULL:
 *     1) written into the x, y entries of gq (other entries untouched); a
 *     loss_body[i] outside [0, body_off[i+1] - body_off[i]) gives loss[i] = NaN
 *     and no cotangent.
 *   ostrich_knot_grad_accumulate: g_knots[c*K + j] += basis[k*K + j] g_ctrl[c].
 *   ostrich_adam: x -= lr mhat / (sqrt(vhat) + eps) with the moments m, v
 *     updated in place from g, bias corrections of step t >= 1; a non-finite
 *     entry of g (a rollout that diverged) counts as zero, so its moments
 *     decay instead of turning the knot into NaN. */
int ostrich_spline_controls(const double* basis, const double* knots, int32_t T, int32_t K, int32_t nctrl,
                            double* ctrl, void* stream);
int ostrich_final_loss(const int32_t* body_off, int32_t n_worlds, const double* qT, const int32_t* loss_body,
                       const double* target, const double* loss_grad, double* loss, double* gq, void* stream);
int ostrich_knot_grad_accumulate(const double* basis, const double* g_ctrl, int32_t k, int32_t K, int32_t nctrl,
                                 double* g_knots, void* stream);
int ostrich_adam(double* x, const double* g, double* m, double* v, int64_t n, double lr, double beta1, double beta2,
                 double eps, int32_t t, void* stream);

/* A contiguous copy of n doubles between device buffers. */
typedef struct {
  const double* src;
  double* dst;
  int64_t n;
} ostrich_copy_seg;

/* Moves of the serving loop (states, multipliers, tapes, controls and
 * cotangents between a request's arena and the pool's working arrays): copies
 * every segment segs[i] (n >= 0 doubles, device pointers; segments must not
 * overlap one another) asynchronously on `stream`, 32 segments per launch.
 * segs itself is host memory, read before the call returns.  Fails with
 * OSTRICH_E_ARG on n_segs < 0, a NULL segs with n_segs > 0, n < 0, or a NULL
 * pointer in a segment with n > 0 (then nothing is launched). */
int ostrich_copy_segments(const ostrich_copy_seg* segs, int32_t n_segs, void* stream);

/* Natural cubic spline basis on the host: B [T*K] (host), knots at
 * t_j = j T h / (K - 1), step k samples t = k h. */
int ostrich_spline_basis(int32_t T, int32_t K, double h, double* B);

#ifdef __cplusplus
}
#endif
#endif
