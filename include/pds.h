/*
 * pds.h -- C ABI of the MI355X (gfx950) library for Constrained SVGD over
 * simulation parameters by parallel differentiable simulation
 * (Heiden et al., "Probabilistic Inference of Simulation Parameters via
 * Parallel Differentiable Simulation").
 *
 * One CSVGD iteration (Algorithm 1) is
 *     sim_batch_adjoint -> svgd_phi -> svgd_step
 * over every particle of every job in a batch.  loglik_multishoot and
 * sim_batch_forward are the forward-only paths.
 *
 * Conventions shared by every call
 * --------------------------------
 * Jobs.  A call takes a batch of n_jobs problems as two arrays with the same
 *   contents: h_jobs in host memory (read during the call to size launches
 *   and validate) and d_jobs in device memory (read by the kernels).  Both
 *   are owned by the caller and must stay unchanged until the work queued by
 *   the call has finished.  One job is a batch of one; 1 <= n_jobs <=
 *   PDS_MAX_JOBS.
 * Memory.  Every pointer inside a pds_job is caller-owned device memory,
 *   row-major and contiguous with the shapes given below, 4-byte aligned for
 *   float/int32 and 8-byte aligned for double arrays.  The library never
 *   allocates or frees device memory and keeps no pointer after a call
 *   returns.  Scratch memory comes from the caller's workspace `ws` of
 *   `ws_bytes` bytes (256-byte aligned), sized by pds_workspace_size(); calls
 *   that need none accept ws = NULL.  (svgd_phi_noalloc instead uses a fixed
 *   array the library's code object holds on every device it is loaded on.)
 * Streams.  Work is queued on `stream` (a hipStream_t passed as void*; NULL
 *   is the default stream).  Calls are asynchronous: no host synchronisation
 *   and no host<->device copy happens inside them.  Calls are re-entrant;
 *   concurrent calls need disjoint outputs and workspaces.
 * Errors.  Every call returns PDS_OK (0) or a negative code; on error nothing
 *   has been queued and pds_last_error() returns a thread-local message.
 *   Numerical trouble is never an error: it is reported per particle in
 *   job.flags (PDS_FLAG_*: bit 0 a non-finite state, bit 1 a non-finite
 *   log-likelihood or gradient, bit 2 a parameter outside its limits, bit
 *   3 frozen).  flags are OR-ed into, never cleared, by the library.
 * Failed particles.  Simulators fail outside the range they were built for
 *   (Sec. III-D), and one non-finite score would make every phi of its job
 *   non-finite.  So a particle with bit 0, 1 or 3 set leaves the ensemble:
 *   svgd_phi (and svgd_phi_at_bandwidth) sums over the N' other particles
 *   only, divides by N', writes phi = 0 for it and the count N - N' to
 *   job.n_masked; svgd_step leaves all its variables as they are and sets
 *   bit 3.  The bandwidth median runs over the particles without bit 3,
 *   with log N' for their number: it reads theta and bit 3 only, which no
 *   call but svgd_step changes, so a bandwidth computed concurrently with
 *   sim_batch_adjoint equals one computed after it.  A particle that fails
 *   in an iteration therefore leaves the median in the next one.
 *
 * Notation: N particles, M parameters, K observed trajectories of T steps,
 * n_s shooting windows of h = T / n_s steps, n_dof joints, d_s = 2 n_dof
 * state components s = [q, qd], d_x observed components, U = N K n_s window
 * units.  Window j of trajectory k starts at step j h from s0[k] (j = 0) or
 * from the shooting state S[i,k,j-1] (j >= 1) and covers states
 * j h + 1 .. (j + 1) h, which it compares with the observations of the same
 * steps (Sec. III-C, eq. ms_likelihood).
 */
#ifndef PDS_H
#define PDS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PDS_OK 0
#define PDS_EINVAL (-1)        /* bad shape, pointer, alignment or scalar */
#define PDS_EUNSUPPORTED (-2)  /* model kind or size above compiled limits */
#define PDS_EWORKSPACE (-3)    /* workspace missing or too small */
#define PDS_ELAUNCH (-4)       /* the HIP runtime refused a launch */

#define PDS_MAX_JOBS 64
#define PDS_MAX_M 16
#define PDS_MAX_DOF 8
#define PDS_MAX_N 32768  /* particles per job */

/* Models.  PLANAR: chain of n_dof (1..5) revolute joints about z, link i a
 * massless rod of length l_i with a point mass m_i at its tip, q = 0 hanging
 * along the gravity direction; theta = (m_1..m_n, l_1..l_n), M = 2 n_dof;
 * observes x = q (d_x = n_dof) or the whole state x = (q, qd) (d_x =
 * 2 n_dof, one weight w_x per component); consts = [g_x, g_y, b_1..b_n]
 * (gravity in the plane, joint damping tau_i = -b_i qd_i).
 * ARM: 7 revolute arm joints about their local z axes after modified-DH
 * placements (Rot_x(alpha) Trans_x(a) Trans_z(d)), PD-controlled towards
 * q_d(t) = qc + amp sin(omega t + phase) (tau = kp (q_d - q) + kd (qd_d -
 * qd)), then a passive hinge about the flange x axis (offset flange_d along
 * the flange z axis, damping tau = -b_h qd) carrying a box and two equal
 * point masses at (x_a, y_a, z_m), (x_b, y_b, z_m) in the box frame;
 * n_dof = 8, theta = (x_a, y_a, x_b, y_b), M = 4, observes the hinge angle
 * (d_x = 1); consts (126 floats) = gravity[3], then for each arm joint
 * (a, alpha, d, m, c_x, c_y, c_z, I_xx, I_yy, I_zz, kp, kd, qc, amp,
 * omega, phase) with the link inertia diagonal about its centre of mass,
 * then flange_d, b_h, box m, box c[3], box I_xx, I_yy, I_zz, point-mass m,
 * z_m.  Arm jobs need a workspace in every call that rolls out windows.
 * A table with the Panda arm's kinematic structure -- twists (0, -pi/2,
 * pi/2, pi/2, -pi/2, pi/2, pi/2), each within 2e-7 rad (float rounding),
 * and a = 0 for joints 0, 1, 2, 5, d = 0 for joints 1, 3, 5, 6 -- runs
 * kernels compiled for that structure, which take those twists as exact
 * right angles; any other table runs the generic kernels.  Every value
 * stays a run-time input in both (all ARM* models). */
/* PLANAR_RIGID: the planar chain with rigid links, the parameterisation of
 * the paper's physical double pendulum (Sec. IV-B table of estimated
 * parameters): n_dof 1..2 revolute joints about z; link i has mass m_i,
 * rotational inertia I_i (> 0) about its centre of mass at (cx_i, cy_i) in
 * the link frame, joint friction tau_i = -b_i qd_i, and joint i sits at
 * (0, -L_i) in link i-1's frame; theta = (m_1, I_1, cx_1, cy_1, b_1, then
 * per further link L_i, m_i, I_i, cx_i, cy_i, b_i), M = 6 n_dof - 1 (11 for
 * the double pendulum); observes q or (q, qd) as PLANAR does (the
 * paper's pendulum experiment observes the whole state); consts = [g_x,
 * g_y]. */
#define PDS_MODEL_PLANAR 1
#define PDS_MODEL_ARM 2
#define PDS_MODEL_PLANAR_RIGID 3
/* ARM_UJOINT: the ARM model's 7 PD-controlled joints with the box on a
 * passive universal joint instead of the hinge, the mount of the paper's
 * Panda experiment (Sec. IV-C and its appendix, phase I): a massless ring
 * turns about the flange x axis (offset flange_d along the flange z axis),
 * the box about the ring's y axis through the same point; n_dof = 9;
 * theta = the box's inertia about its centre of mass (I_xx, I_yy, I_zz,
 * I_xy, I_xz, I_yz), its centre of mass (x, y, z) in the box frame and the
 * viscous friction of the two axes (tau = -b qd), M = 11; observes the box
 * frame, i.e. its origin and the points 1 m along its x, y and z axes in
 * world coordinates (d_x = 12, in that order); consts (117 floats) =
 * gravity[3], the 7 x 16 arm-joint table of ARM, flange_d, box mass. */
#define PDS_MODEL_ARM_UJOINT 4
/* ARM_UJOINT_WEIGHTS: the same universal-joint mount with the box's
 * phase-I values known and two equal point masses on the box floor to be
 * found (phase II of the paper's Panda experiment): theta = (x_a, y_a, x_b,
 * y_b), the in-plane positions of the masses at height z_m in the box
 * frame, M = 4; n_dof = 9; observes the box frame as ARM_UJOINT (d_x =
 * 12); consts (130 floats) = gravity[3], the 7 x 16 arm-joint table,
 * flange_d, box m, box c[3], box inertia about its centre of mass (I_xx,
 * I_yy, I_zz, I_xy, I_xz, I_yz), the damping of the two axes, point-mass
 * m, z_m. */
#define PDS_MODEL_ARM_UJOINT_WEIGHTS 5

#define PDS_COMBINE_SUM 0   /* equally weighted mixture over trajectories, eq. traj_likelihood */
#define PDS_COMBINE_PROD 1  /* product over trajectories, App. A-B eq. traj_likelihood_prod */

/* How the shooting defects enter (eq. likelihood-defect, eq. ms_likelihood).
 * MDMM: as equality constraints of Sec. III-E (CSVGD): the window
 *   log-likelihoods hold the observation terms only, the constraint
 *   channel carries (lam_def + c g_def) d g_def, and svgd_step ascends
 *   lam_def.
 * DEFECT: as Gaussian factors inside p_ms (eq. ms_likelihood, the form the
 *   paper gives its sampling baselines): window j < n_s-1 adds
 *   log N(S_{j+1} | s_end, sigma_def^2 / u^2) = -g_def / 2 + sum_d
 *   log(u_d / (sigma_def sqrt(2 pi))) to its log-likelihood, the defect
 *   gradients ride in the observation channel with the trajectory
 *   weights, the constraint channel's default defect seed is 0 (explicit
 *   seed_gdef still applies) and svgd_step leaves lam_def unchanged. */
#define PDS_LIK_MDMM 0
#define PDS_LIK_DEFECT 1

/* How svgd_step keeps theta inside [lo, hi] (Sec. III-D, III-E).
 * SOFT: only through the MDMM limit constraint g_lim = clamp(theta) -
 *   theta and its multiplier lam_lim, as the paper does; a particle may
 *   leave the box for a while.
 * PROJECT: additionally clamps every updated theta into [lo, hi], for
 *   models whose simulation is undefined outside the box (the rigid links'
 *   masses and inertias must stay positive); g_lim then stays 0. */
#define PDS_LIMITS_SOFT 0
#define PDS_LIMITS_PROJECT 1

#define PDS_OPT_SGD 0
#define PDS_OPT_ADAM 1

/* job.flags bits */
#define PDS_FLAG_STATE 1   /* a non-finite window state */
#define PDS_FLAG_GRAD 2    /* a non-finite log-likelihood or gradient */
#define PDS_FLAG_LIMIT 4   /* theta left outside [lo, hi] by svgd_step */
#define PDS_FLAG_FROZEN 8  /* left out of the ensemble by svgd_step */

/* which-call selector for pds_workspace_size */
#define PDS_CALL_FORWARD 0
#define PDS_CALL_LOGLIK 1
#define PDS_CALL_ADJOINT 2
#define PDS_CALL_PHI 3
#define PDS_CALL_STEP 4
#define PDS_CALL_ALL 5

typedef struct pds_job {
  /* ---- shape and scalars ---- */
  int32_t model;      /* PDS_MODEL_* */
  int32_t n_dof;
  int32_t M;          /* 1..PDS_MAX_M */
  int32_t d_x;
  int32_t N;          /* particles, 1..PDS_MAX_N */
  int32_t K;          /* trajectories, >= 1 */
  int32_t T;          /* steps per trajectory, T = n_s * h */
  int32_t n_s;        /* shooting windows, >= 1 */
  int32_t h;          /* steps per window, >= 1; N K n_s (2 n_dof + 1) at most
                       * 2e9 (else PDS_EUNSUPPORTED: flat 32-bit indexes) */
  int32_t combine;    /* PDS_COMBINE_* */
  int32_t lik;        /* PDS_LIK_* */
  int32_t limits;     /* PDS_LIMITS_* */
  float dt;           /* > 0 */
  float sigma_def;    /* > 0, defect scale of eq. likelihood-defect */
  float c;            /* >= 0, MDMM damping constant of eq. mdmm-loss */
  float eps_lam;      /* step size of the multiplier ascent */
  /* ---- constant inputs ---- */
  const float* consts;    /* model constants, layout per model kind */
  const float* lo;        /* [M] lower parameter limits (Sec. III-D) */
  const float* hi;        /* [M] upper parameter limits */
  const float* rho;       /* [M] kernel length scales (> 0) */
  const float* w_x;       /* [d_x] observation weights 1 / sigma_obs (> 0) */
  const float* u;         /* [d_s] defect state scales */
  const float* lr_theta;  /* [M] step sizes for theta */
  const float* lr_S;      /* [d_s] step sizes for shooting states */
  const float* s0;        /* [K, d_s] known start states */
  const float* obs;       /* [K, T, d_x]; row t-1 observes state t */
  const double* seed_logp;  /* [N] adjoint seed of log p, NULL = 1 */
  const double* seed_gdef;  /* [N, K, n_s-1] seed of g_def, NULL = lam_def + c g_def */
  /* ---- particle state (in/out) ---- */
  float* theta;     /* [N, M] */
  float* S;         /* [N, K, n_s-1, d_s] shooting states */
  float* lam_lim;   /* [N, M] */
  float* lam_def;   /* [N, K, n_s-1] */
  float* adam_m;    /* [N, M + K (n_s-1) d_s] */
  float* adam_v;    /* [N, M + K (n_s-1) d_s] */
  /* ---- outputs ---- */
  float* end_states;  /* [N, K, n_s, d_s] last state of each window */
  float* traj;        /* [N, K, T, d_s] visited states, or NULL (sim_batch_forward only) */
  double* ll_win;     /* [N, K, n_s] window log-likelihoods (with Gaussian constants; with
                         PDS_LIK_DEFECT window j < n_s-1 includes its defect's log density) */
  double* gdef;       /* [N, K, n_s-1] defects ||(S_{j+1} - s_end) u||^2 / sigma_def^2 */
  double* logp;       /* [N] log p_obs per particle */
  double* wk;         /* [N, K] d log p / d l_k (mixture responsibilities, or 1) */
  double* g_obs;      /* [N, M] seed_logp * d log p / d theta */
  double* g_con;      /* [N, M] sum seed_gdef * d g_def / d theta */
  float* S_dot;       /* [N, K, n_s-1, d_s] seed_logp d log p/dS - sum seed_gdef d g_def/dS */
  float* phi;         /* [N, M] SVGD direction */
  double* bandwidth;  /* [1] kernel bandwidth h used by phi */
  int32_t* flags;     /* [N] per-particle status bits */
  int32_t* iter_dev;  /* [2] Adam iteration counter in device memory, or NULL:
                         when set, svgd_step uses iter_dev[0] + 1 (ignoring
                         its `iter` argument) and then increments iter_dev[0],
                         so a captured graph can be replayed without new
                         arguments.  iter_dev[1] is the step's block count,
                         zero before and after every call: allocate both
                         zeroed, and never run two steps of one job at once */
  int32_t* n_masked;  /* [1] particles left out of the last phi (flag bit 0,
                         1 or 3), or NULL */
  /* ---- optional outputs and seeds ---- */
  float* traj_obs;    /* [N, K, T, d_x] the observed quantities f_obs of every
                         visited state, row t-1 for state t as in obs (PLANAR
                         and PLANAR_RIGID: the first d_x components of (q, qd);
                         ARM: the hinge angle; ARM_UJOINT*: the box frame), or
                         NULL (sim_batch_forward only) */
  double* g_theta;    /* [N, M] g_obs - g_con, the theta counterpart of S_dot
                         (sim_batch_adjoint), or NULL */
  const double* cot_gdef; /* [N, K, n_s-1] cotangent of g_def for a
                         vector-Jacobian product, or NULL.  When set (seed_gdef
                         must then be NULL) the constraint channel is seeded with
                         -cot_gdef, so that g_theta and S_dot are d/dtheta and
                         d/dS of seed_logp log p + sum cot_gdef g_def */
} pds_job;

/* Rolls out every window (a batched f_sim of Sec. II with the semi-implicit
 * Euler step of App. B-A eq. dynamics; forward dynamics by the Articulated
 * Body Algorithm).  Writes end_states and, where job.traj != NULL, every
 * visited state; where job.traj_obs != NULL, what the observation model of
 * eq. combinedlikelihood sees of every visited state (f_obs: for the
 * universal-joint arm the box frame's forward kinematics), so that observed
 * trajectories can be synthesised from a rollout.  Needs a workspace only
 * for arm jobs. */
int sim_batch_forward(const pds_job* h_jobs, const pds_job* d_jobs, int32_t n_jobs, void* ws,
                      size_t ws_bytes, void* stream);

/* Multiple-shooting log-likelihood (Sec. III-B/C): window rollouts, the
 * Gaussian observation terms of eq. combinedlikelihood summed in FP64 per
 * window (ll_win), the defects g_def of Sec. III-E, and the combination over
 * trajectories (logp, wk).  Writes end_states, ll_win, gdef, logp, wk.
 * Needs a workspace only for arm jobs. */
int loglik_multishoot(const pds_job* h_jobs, const pds_job* d_jobs, int32_t n_jobs, void* ws,
                      size_t ws_bytes, void* stream);

/* Reverse-mode gradient of the multiple-shooting likelihood and of the
 * defect terms (App. B-A: chain rule through f_step), recomputing each
 * window from its start state; assembled for the MDMM flow of Sec. III-E /
 * Algorithm 1.  Writes everything loglik_multishoot writes plus g_obs,
 * g_con, S_dot and, where job.g_theta != NULL, g_theta.  With cot_gdef
 * (and seed_logp) the call is the vector-Jacobian product of (log p, g_def)
 * with respect to (theta, S): g_theta and S_dot. */
int sim_batch_adjoint(const pds_job* h_jobs, const pds_job* d_jobs, int32_t n_jobs, void* ws,
                      size_t ws_bytes, void* stream);

/* SVGD direction of eq. svgd_update with the RBF kernel
 * k(a, b) = exp(-||(a - b) / rho||^2 / h) and the median heuristic
 * h = med^2 / log N (Sec. III-A), med the exact FP64 median of the
 * N (N - 1) / 2 scaled pair distances (mean of the two middle values for an
 * even count; h = 1 for N = 1), over the particles of the ensemble (see
 * Failed particles above).  Uses g_obs as the score.  Writes bandwidth,
 * phi and n_masked.  The workspace holds, per job, the selection state, one 8-byte
 * slot per pair when N (N - 1) / 2 > 16384, and the phi partial sums. */
int svgd_phi(const pds_job* h_jobs, const pds_job* d_jobs, int32_t n_jobs, void* ws, size_t ws_bytes,
             void* stream);

/* The two halves of svgd_phi, for callers that overlap the bandwidth with
 * the adjoint: svgd_bandwidth writes `bandwidth` only (the median
 * heuristic of Sec. III-A; reads theta and rho), svgd_phi_at_bandwidth
 * writes phi from the `bandwidth` already in device memory (eq.
 * svgd_update).  svgd_phi == svgd_bandwidth then svgd_phi_at_bandwidth on
 * one stream.  The bandwidth depends on theta alone and uses workspace
 * regions sim_batch_adjoint does not touch, so on a second stream it may
 * run concurrently with sim_batch_adjoint of the same batch and workspace
 * (nothing may write theta meanwhile).  svgd_bandwidth is meant for that
 * use: when the batch's window kernels leave SIMDs free (fewer than 1020
 * waves) and include an arm job with windows of at least 32 steps (long
 * enough to hide it), jobs above 256 particles get the median from blocks
 * of one wave each, which fit beside them (larger blocks would wait for
 * their end); the bandwidth is the same. */
int svgd_bandwidth(const pds_job* h_jobs, const pds_job* d_jobs, int32_t n_jobs, void* ws, size_t ws_bytes,
                   void* stream);
int svgd_phi_at_bandwidth(const pds_job* h_jobs, const pds_job* d_jobs, int32_t n_jobs, void* ws, size_t ws_bytes,
                          void* stream);

/* svgd_phi for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation):
 * the same bandwidth and phi, bitwise, with the workspace taken from a
 * fixed array of PDS_NOALLOC_SCRATCH_BYTES bytes that the library holds on
 * each device it runs on until the process ends (the device of `stream`,
 * or the current device for the NULL stream).  No allocation happens in
 * the call.  PDS_EWORKSPACE (nothing queued) when the batch needs more
 * than the array: pds_workspace_size(h_jobs, n_jobs, PDS_CALL_PHI) bytes,
 * e.g. about 29 MB for one job of 2048 particles with 30 windows of the
 * 8-body arm.  Every call on a device shares that device's array and
 * leaves its contents behind: calls that overlap on one device (on
 * concurrent streams) race and give undefined results; calls ordered on
 * one stream, or synchronised, are safe. */
#define PDS_NOALLOC_SCRATCH_BYTES (64ull << 20)
int svgd_phi_noalloc(const pds_job* h_jobs, const pds_job* d_jobs, int32_t n_jobs, void* stream);

/* MDMM update of Sec. III-E / Algorithm 1, simultaneous for all variables:
 * theta_dot = phi - (lam_lim + c g_lim) dg_lim/dtheta - g_con with
 * g_lim = clamp(theta, lo, hi) - theta; S_dot as computed; lam_lim += eps_lam
 * g_lim; lam_def += eps_lam g_def.  optimizer PDS_OPT_SGD: x += lr x_dot;
 * PDS_OPT_ADAM: Adam (0.9, 0.999, 1e-8) on (theta, S) with -x_dot as the
 * gradient, iteration `iter` >= 1 for bias correction.  Particles with flag
 * bit 0, 1 or 3 keep every variable and get bit 3.  Sets flags bit 2 for
 * particles left outside their limits.  Needs no workspace. */
int svgd_step(const pds_job* h_jobs, const pds_job* d_jobs, int32_t n_jobs, int32_t optimizer,
              int32_t iter, void* stream);

/* Workspace bytes the call `which` (PDS_CALL_*) needs for this batch;
 * PDS_CALL_ALL gives the maximum over all calls.  0 on invalid input (see
 * pds_last_error). */
size_t pds_workspace_size(const pds_job* h_jobs, int32_t n_jobs, int32_t which);

/* Device bytes one job occupies in a CSVGD iteration, for admission by
 * HBM footprint: every buffer the pds_job fields point to at the sizes
 * documented above (gdef and S_dot with at least one window, iter_dev with
 * 2 entries, n_masked with 1; traj, traj_obs, g_theta, seed_logp, seed_gdef
 * and cot_gdef only when non-NULL in *h_job) plus its workspace for all
 * calls.  Reads only shapes and those optional pointers; 0 on invalid
 * shapes (see pds_last_error). */
size_t pds_job_footprint(const pds_job* h_job);

/* ---- Posterior-consistency metrics (Sec. III-F, App. A-D) ----
 * Compares two sets of trajectories, each row one trajectory's
 * observations flattened to d floats (e.g. rollouts of the particles
 * against held-out trajectories):
 *   out[0] = d_KL(P || Q) by the k-nearest-neighbour estimate of eq. knn-kl,
 *            d/n sum_i log(nu_k(i) / rho_l(i)) + psi(l) - psi(k)
 *            + log(m / (n - 1)), nu_k(i) the Euclidean distance from P_i to
 *            its k-th nearest row of Q, rho_l(i) to its l-th nearest row of
 *            P other than itself (the paper takes k = l = 3);
 *   out[1] = d_KL(Q || P), the same with the roles swapped;
 *   out[2] = squared MMD (Sec. III-F), unbiased estimate with the Gaussian
 *            kernel exp(-||x - y||^2 / (2 sigma^2));
 *   out[3] = the sigma used: `sigma` if > 0, else the median Euclidean
 *            distance over all distinct pairs of P u Q (mean of the two
 *            middle ones for an even count; 1 if that median is 0).
 * P [n, d], Q [m, d]: row-major device floats; w [d] device floats
 * scaling each coordinate before the distances, or NULL for 1.  Rows must
 * be finite; a zero nearest-neighbour distance gives an infinite estimate,
 * as the formula does.  rows: NULL, or device doubles [n + m, 3] receiving
 * per pooled row r (P rows first) d/2 (log nu^2 - log rho^2) with nu over
 * the other set and rho over its own set, and the kernel sums over its own
 * set (j != r) and over the other set.  out: device doubles [4].  ws:
 * caller-owned device workspace of pds_traj_metrics_workspace(n, m, d)
 * bytes, 256-byte aligned.  Limits: 1 <= k, l <= PDS_METRICS_MAX_K,
 * n, m >= max(k, l + 1, 2), n + m <= PDS_METRICS_MAX_ROWS, d >= 1.
 * Returns PDS_OK or a negative code before anything is queued; the outputs
 * are ready when the stream reaches them.  The library allocates nothing. */
#define PDS_METRICS_MAX_K 8
#define PDS_METRICS_MAX_ROWS 16384
size_t pds_traj_metrics_workspace(int32_t n, int32_t m, int32_t d);
int pds_traj_metrics(const float* P, int32_t n, const float* Q, int32_t m, int32_t d, const float* w, int32_t k,
                     int32_t l, double sigma, double* out, double* rows, void* ws, size_t ws_bytes, void* stream);

/* Message for the last error on this thread ("" if none). */
const char* pds_last_error(void);

/* Library version (major * 10000 + minor * 100 + patch). */
int32_t pds_version(void);

/* ---- measurement helpers (not on the inference path) ---- */

/* Algorithmic FLOPs of one simulation step of the given model (ABA + Euler +
 * observation residual) and of one reverse step for one adjoint channel
 * (reverse of the same + observation seed + FP64 parameter accumulation),
 * counted by running the library's own step functions on the host with a
 * counting scalar type (add, sub, mul, div = 1 each); sin/cos evaluations
 * are returned separately.  In-window recomputation is not counted.  For the
 * arm models this is the generic kinematic structure's step (a given table's
 * own: pds_arm_algorithmic_flops).  Returns PDS_OK, PDS_EINVAL or
 * PDS_EUNSUPPORTED. */
int pds_algorithmic_flops(int32_t model, int32_t n_dof, double* fwd_step, double* rev_step,
                          double* transcendental);

/* The same for an arm model (PDS_MODEL_ARM*) with the job's raw constants
 * `consts` (HOST memory, the layout documented with the models): counts
 * the step functions of the kinematic structure the kernels run for that
 * table -- the Panda arm's (*panda = 1; the twists and zero offsets of its
 * modified-DH table, see the ARM model) or the generic one (*panda = 0).
 * panda may be NULL.  Returns PDS_OK or PDS_EINVAL. */
int pds_arm_algorithmic_flops(int32_t model, const float* consts, double* fwd_step, double* rev_step,
                              double* transcendental, int32_t* panda);

/* Kernel timing for benchmarks.  While enabled, every sim_batch_adjoint,
 * loglik_multishoot and traj_metrics call records a pair of HIP events on its
 * stream around its window-kernel (distance-kernel) launches (a ring of 4096
 * pairs).  pds_timing_enable(r), 1 <= r <= 64, clears the ring and turns
 * timing on with r back-to-back launches of those kernels inside each pair
 * (they rewrite the same outputs from the same inputs, so results are
 * unchanged): the dispatch latency an event pair adds is then paid once per
 * r launches.  pds_timing_enable(0) turns timing off; other values give
 * PDS_EINVAL.  pds_timing_read waits for the recorded events and writes up
 * to max_n times in milliseconds, each a pair's elapsed time divided by its
 * r, returning how many it wrote (or a negative error code). */
int pds_timing_enable(int32_t enable);
int pds_timing_read(float* ms, int32_t max_n);

#ifdef __cplusplus
}
#endif

#endif /* PDS_H */
