/* Batched differentiable rigid-body time step for MI355X (gfx950): C ABI.
 *
 * The library simulates E independent environments ("envs", robot models) at
 * once.  Each env is a set of rigid bodies with 6 DOF (position, rotation
 * matrix, linear and angular velocity), hinge joints, and collision spheres
 * that touch the ground plane z = 0 and each other.  One time step
 * x^{t+1} = f_ph(x^t, u^t) (paper, section 2.1 and eq. (L)) is:
 *   joint torques u and damping -> velocity prediction with gravity ->
 *   contact candidates and gap test -> constraint rows (Jacobians, effective
 *   masses, Baumgarte / speculative bias, restitution) -> warm start from the previous
 *   step's impulses -> a fixed number of projected Gauss-Seidel sweeps in a
 *   fixed colour-major order -> semi-implicit Euler and rotation
 *   renormalisation N(A) = (3A - A A^T A)/2 (eq. (1)).
 * `rollout` unrolls T steps and accumulates the loss L = sum_t l(x^t, p)
 * (eq. (L)); `rollout_grad` returns the exact reverse-mode derivative of the
 * unrolled discrete map (back-propagation through time, section 2.1.1) with
 * respect to the initial state, the control tape (or the controller's
 * weights) and the model parameters section 4 names, masses and lengths:
 * inverse masses and inertias, the hinge anchors (the link lengths), joint
 * damping and the friction coefficient.
 *
 * Conventions for every call:
 *  - Arrays marked (device) are device pointers (hipMalloc / torch CUDA
 *    tensors) owned by the caller; the library never frees them.  Arrays
 *    marked (host) are read synchronously during the call.
 *  - All floats are IEEE binary32; all arithmetic on the GPU is FP32.
 *  - State layout is struct-of-arrays: x[18][B] with component k of body b
 *    at x[k*B + b]; components p(0..2), R(3..11, row-major), v(12..14),
 *    omega(15..17).  B = total bodies over all envs, bodies of an env are
 *    contiguous (CSR offsets env_body_off).
 *  - Carried state besides x ("lambda"), per env a contiguous block of
 *    5*J_e + 4*G_e + 4*P_e warm-start impulses (6*J_e + ... with servo
 *    motors; then, with a recurrent controller, its mlp_rec units h^t) at the
 *    offset sim_info.lam_off[e]: 5 hinge rows per joint (point x, y, z,
 *    angular t1, t2; then the servo's motor row), then per ground
 *    sphere (sphere order) [lambda_n, Lambda_t.x, .y, .z], then per sphere
 *    pair candidate [lambda_n, Lambda_t(3)] in (body a, body b) lexicographic
 *    order of the env's local body indices; Lambda_t is the tangent impulse
 *    as a world vector.  Inactive candidates hold zeros.
 *  - Control tape u[T_max][J] (device), joint-major within a step.
 *  - Calls are asynchronous on the given HIP stream (NULL = default stream)
 *    and never synchronise the device.  Argument, shape and descriptor errors
 *    are detected on the host before any launch: they return a negative
 *    status and set a thread-local message (sim_last_error).  A device fault
 *    from an earlier launch surfaces as SIM_E_DEVICE.  Per-env numerical
 *    events are not errors: they are reported in env_flags.
 *  - A handle is not re-entrant: do not run two calls with one handle on
 *    different streams concurrently.
 *  - Results are bitwise deterministic for a given handle (no float atomics).
 */
#ifndef PAPER_1611_01652_SIM_H
#define PAPER_1611_01652_SIM_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SIM_ABI_VERSION 10

typedef struct sim_model* sim_handle;

typedef enum {
  SIM_OK = 0,
  SIM_E_ARG = -1,         /* null pointer or invalid scalar */
  SIM_E_SHAPE = -2,       /* inconsistent sizes / offsets / indices */
  SIM_E_UNSUPPORTED = -3, /* model exceeds a device limit (e.g. LDS per env) */
  SIM_E_NOMEM = -4,       /* device allocation failed, or workspace too small */
  SIM_E_DEVICE = -5,      /* a HIP call failed (includes earlier async faults) */
  SIM_E_STATE = -6        /* handle used in an invalid state */
} sim_status;

/* per-env flags written by rollout / rollout_grad / sim_step */
#define SIM_FLAG_NONFINITE 1u        /* a state component became NaN/Inf */
#define SIM_FLAG_CONTACT_OVERFLOW 2u /* more active contacts than the env's capacity */
#define SIM_FLAG_GRAD_NONFINITE 4u   /* rollout_grad: the env's adjoint overflowed; its gradient is zeroed */

/* loss kinds l(x^t, p) of eq. (L); p = the env's target and loss body */
#define SIM_LOSS_FINAL_SQDIST 0  /* sum_k mask_k (p_k(T_e) - target_k)^2                */
#define SIM_LOSS_MEAN_DIST 1     /* (1/T_e) sum_{t=1..T_e} |mask*(p(t) - target)|          */
#define SIM_LOSS_NEG_MEAN_VELX 2 /* -(p_x(T_e) - p_x(0)) / (T_e dt)  (mean forward speed) */
#define SIM_LOSS_FINAL_STATE 3   /* sum_k mask_k (p_k(T_e) - target_k)^2 + |v(T_e)|^2 + |omega(T_e)|^2
                                    (the ball of section 2.1.1: at rest on the target) */

/* control kinds (eq. (g) of section 2.2 without the recurrent state) */
#define SIM_CTRL_TAPE 0 /* open-loop torques u[T_max][J] */
#define SIM_CTRL_MLP 1  /* [u^t, a^t] = g(s(x^t), h^t) shared by all envs (eq. (g)): s = [joint angles
                           (J_e), joint rates (J_e), sin, cos of 2 pi f t dt]; h^t the controller's
                           mlp_rec recurrent units, h^0 = 0, h^{t+1} = tanh(a^t); tanh hidden layers,
                           linear outputs u^t (J_e) and a^t (mlp_rec); weights W1[h1][in] b1
                           W2[h2][h1] b2 W3[out][h2] b3 */

/* solver and warm-start kinds */
#define SIM_SOLVE_FIXED 0 /* n_iters sweeps per step */
#define SIM_SOLVE_TOL 1   /* sweeps until the residual is at most tol */
/* Reverse sweep memory modes (sim_model_desc.grad_store).  Rollouts keep a
   checkpoint every K_ck steps; rollout_grad then
   - REPLAY: recomputes one segment at a time keeping step-start states, and
     replays each step up to its sweeps before reversing it (least memory:
     K_ck states per env);
   - SEGMENT: recomputes one segment at a time saving each step's working set
     after its sweeps, which the reverse reloads (K_ck working sets per env);
   - TRAJECTORY: recomputes all segments of all envs at once in a separate
     launch, saving every step's working set, then reverses the whole
     trajectory from them (T working sets per env). */
#define SIM_GRAD_AUTO 0
#define SIM_GRAD_REPLAY 1
#define SIM_GRAD_SEGMENT 2
#define SIM_GRAD_TRAJECTORY 3

#define SIM_WS_PLAIN 0    /* warm start: the previous step's impulses times `warm` */
#define SIM_WS_LEARNED 1  /* contacts: the warm-start network, with fallback */

/* Model description (host memory, read during sim_init; the caller keeps
 * ownership).  Indices of bodies/joints/spheres are global (over all envs),
 * and each env's items must lie inside its own CSR range. */
typedef struct {
  int32_t n_envs;
  const int32_t* env_body_off;   /* [E+1] */
  const int32_t* env_joint_off;  /* [E+1] */
  const int32_t* env_sphere_off; /* [E+1] */
  const float* inv_mass;         /* [B] 1/m (> 0) */
  const float* inv_inertia;      /* [B][3] inverse diagonal body-frame inertia */
  const int32_t* sphere_body;    /* [S] body carrying the sphere */
  const float* sphere_offset;    /* [S][3] centre in the body frame */
  const float* sphere_radius;    /* [S] */
  const int32_t* sphere_flags;   /* [S] bit0 ground contact, bit1 sphere-sphere contact
                                    (at most one bit1 sphere per body) */
  const int32_t* joint_parent;   /* [J] body index or -1 (world) */
  const int32_t* joint_child;    /* [J] body index */
  const float* anchor_p;         /* [J][3] hinge point in the parent (world) frame */
  const float* anchor_c;         /* [J][3] hinge point in the child frame */
  const float* axis_p;           /* [J][3] unit hinge axis, parent (world) frame */
  const float* axis_c;           /* [J][3] unit hinge axis, child frame */
  const float* perp_p;           /* [J][3] unit vector normal to axis_p, parent frame */
  const float* perp_c;           /* [J][3] unit vector normal to axis_c, child frame */
  const float* damping;          /* [J] viscous damping about the hinge axis */
  const float* mu;               /* [E] Coulomb friction coefficient */
  const int32_t* loss_body;      /* [E] body whose centre enters the loss */
  const float* target;           /* [E][3] loss target */
  const int32_t* T_env;          /* [E] steps of each env, 0 <= T_e <= T_max */
  int32_t T_max;                 /* rows of the control tape */
  float dt;                      /* time step [s] (> 0) */
  float gravity[3];
  float beta;                    /* Baumgarte factor (softening of section 2.1) */
  float gamma;                   /* constraint force mixing (>= 0) */
  float spec_margin;             /* contact candidate is active iff gap < spec_margin */
  float warm;                    /* factor on carried impulses at the warm start */
  int32_t n_iters;               /* Gauss-Seidel sweeps per step (>= 0) */
  int32_t ground;                /* 1: ground plane z = 0 present */
  int32_t loss_kind;             /* SIM_LOSS_* */
  int32_t loss_mask;             /* bit k: coordinate k enters the loss */
  int32_t ckpt_every;            /* K_ck: rollout stores the state every K_ck steps */
  int32_t min_team;              /* 0: automatic; else lanes per env are at least this
                                    (power of two <= 64).  Results do not depend on it. */
  int32_t ctrl_kind;             /* SIM_CTRL_* */
  int32_t mlp_sizes[4];          /* in, h1, h2, out; every env has out = J_e + mlp_rec,
                                    in = 2 J_e + 2 + mlp_rec; h1, h2 <= 256 */
  float clock_hz;                /* clock frequency f of the controller inputs */
  /* Solve to a residual tolerance (forward only; rollout_grad refuses): after
     each sweep the residual is the largest |change of impulse| / effective
     mass over the active rows (a friction block: the norm of its tangent
     change over its mass), in m/s; sweeps stop at the first residual <= tol
     or after max_iters sweeps. */
  int32_t solve_mode;            /* SIM_SOLVE_FIXED (n_iters sweeps) or SIM_SOLVE_TOL */
  float tol;
  int32_t max_iters;
  /* Learned warm start of contacts (tolerance mode only): the warm-start
     network (SIM_WSN_*) maps a contact's features to corrections of its
     carried impulses (impulse over effective mass); the corrected impulses,
     projected onto lambda_n >= 0, |lambda_t| <= mu lambda_n, start the solve.
     If after fb_iters sweeps the solve has not converged and the residual of
     the contact rows exceeds fb_tol, that env's solve restarts from the plain
     warm start (fb_iters = 0: always). */
  int32_t ws_kind;               /* SIM_WS_PLAIN or SIM_WS_LEARNED */
  const float* ws_net;           /* host [SIM_WSN_PARAMS] FP32 weights (rounded to bfloat16 by sim_init) */
  int32_t fb_iters;
  float fb_tol;
  /* Reverse sweep memory (the rollout_grad workspace), one of SIM_GRAD_*.
     SIM_GRAD_AUTO takes the first of TRAJECTORY, SEGMENT, REPLAY whose
     buffers fit grad_mem_limit bytes (0: 32 GiB).  Every mode gives the same
     result bits; they trade memory for recomputation. */
  int32_t grad_store;
  int64_t grad_mem_limit;
  /* Gradient decay (section 3.2, a training aid against exploding gradients):
     with use_grad_decay != 0, rollout_grad multiplies the adjoints carried
     back from step t+1 to step t (the state's and the carried impulses') by
     grad_decay, in [0, 1], before reversing step t; the loss term of x^{t+1}
     enters undecayed.  The result is then not the exact derivative.
     use_grad_decay = 0 (a zero-initialised description): the exact
     derivative. */
  int32_t use_grad_decay;
  float grad_decay;
  /* SIM_CTRL_MLP: recurrent units of the controller (0: none); then
     mlp_sizes in = 2 J_e + 2 + mlp_rec and out = J_e + mlp_rec, and h^t rides
     at the end of each env's carried-state block */
  int32_t mlp_rec;
  /* Restitution (the ball of section 2.1.1 has e = 0.5): restitution[e] in
     [0, 1] per env (host, NULL: 0 everywhere).  A contact whose normal
     velocity at the predicted velocities v* (gravity and torques applied,
     before the warm start), v_n = J_n v*, is below -rest_threshold and would
     close its gap within the step (gap + dt v_n < 0) takes the normal-row
     bias min(b, e v_n), b its speculative or Baumgarte bias: it leaves at e
     times its approach speed unless the push-out is faster.  The threshold
     (m/s, >= 0) keeps resting contacts from bouncing. */
  const float* restitution;
  float rest_threshold;
  /* Servo motors (section 2.1: gain, maximal torque, maximal velocity; the
     arm of section 3.2 has 30 1/s, 30 N m, 45 deg/s).  servo = 1: every hinge
     is a velocity motor and the control u^t_j (tape or controller output) is
     its target angle theta*_j in rad, not a torque.  The motor is a sixth
     row of the joint, angular about the parent's world hinge axis n_a
     (J w = n_a . (w_b - w_a)), visited after the five hinge rows; it aims at
     the rate clip(servo_gain_j (theta*_j - theta_j), -servo_vmax_j,
     servo_vmax_j), theta_j the hinge angle (the controller's angle sensor),
     and its impulse is clamped to [-servo_torque_j dt, servo_torque_j dt].
     The joint's direct torque is then its viscous damping alone.  The
     carried state has 6 impulses per joint (the motor's last).  rollout_grad
     differentiates through the clip and the clamp (zero where active).
     Arrays [J] (host), finite and >= 0; servo = 0: plain torques. */
  int32_t servo;
  const float* servo_gain;
  const float* servo_torque;
  const float* servo_vmax;
} sim_model_desc;

/* Sizes derived by sim_init. */
typedef struct {
  int32_t n_envs, n_bodies, n_joints;
  int32_t lam_size;           /* total floats of the warm-start state */
  int32_t n_ckpt;             /* checkpoints per rollout: floor((T_max-1)/K_ck)+1 (1 if T_max=0) */
  int64_t ckpt_floats;        /* floats of the checkpoint buffer: n_ckpt*(18*B + lam_size) */
  int64_t workspace_bytes;    /* device workspace needed by rollout_grad */
  int32_t max_lds_bytes;      /* largest LDS allocation per workgroup among the tiles */
  int32_t n_tiles;            /* env tiles scheduled per rollout */
  int32_t n_params;           /* controller parameters (0 for a control tape) */
  int32_t grad_store;         /* reverse sweep memory mode chosen (SIM_GRAD_REPLAY, _SEGMENT or _TRAJECTORY) */
} sim_info;

int sim_abi_version(void);

/* Thread-local description of the last failure on this thread ("" if none). */
const char* sim_last_error(void);

/* Validate the description, build per-env topology (contact candidates,
 * colour-major sweep order), size-bucket and tile the envs, and upload all
 * constants to the current device (synchronous).  On success *out owns the
 * device copies; release with sim_destroy.
 * With several buckets, each call forks them onto streams of their own and
 * joins them back to the caller's stream.  HIP maps streams onto
 * GPU_MAX_HW_QUEUES hardware queues (4 unless the process sets it before HIP
 * starts) and runs the kernels of streams that share a queue one after
 * another: for the buckets to run at once, set it to at least the bucket
 * count (sim_get_teams). */
sim_status sim_init(const sim_model_desc* desc, sim_handle* out);
sim_status sim_destroy(sim_handle h);
sim_status sim_get_info(sim_handle h, sim_info* info);
/* lam_off[E+1] (host): start of each env's warm-start block. */
sim_status sim_lambda_offsets(sim_handle h, int32_t* lam_off);

/* Host only (touches no device): the canonical sweep order of env `env` of
 * a description.  Writes up to `cap` codes (kind << 24 | index; kind 0 =
 * joint (global index), 1 = ground contact (global sphere index), 2 = sphere
 * pair (local body a | local body b << 12)) and colour ids into codes[] and
 * colours[] (host, may be NULL) and returns the number of constraints, or a
 * negative sim_status.  Inside one colour no two constraints share a body. */
int32_t sim_describe_order(const sim_model_desc* desc, int32_t env, int32_t* codes, int32_t* colours,
                           int32_t cap);

/* One step for all envs: x_out = f_ph(x_in, u) (device pointers, x[18][B],
 * u[J] torques (servo targets with servo motors) or, for SIM_CTRL_MLP, the
 * controller weights [n_params];
 * lambda[lam_size]).  t is the step index (it selects the clock input of a
 * controller; 0 <= t < T_max then).  lam_in may equal lam_out; x_in must not
 * alias x_out.  env_flags[E] (device, may be NULL) is overwritten. */
sim_status sim_step(sim_handle h, const float* x_in, float* x_out, const float* u, const float* lam_in,
                    float* lam_out, int32_t t, uint32_t* env_flags, void* stream);

/* Forward rollout from x0 (device, x[18][B]) with the control tape u
 * (device, [T_max][J]) or, for SIM_CTRL_MLP, the controller weights
 * (device, [n_params]); warm-start impulses start at zero.  Writes
 * loss_env[E] (device), x_final[18][B] (device, may be NULL), lam_final
 * (device, may be NULL), the checkpoint buffer ckpt (device, sim_info
 * .ckpt_floats floats, may be NULL when no gradient will be asked for) and
 * env_flags[E] (device, may be NULL). */
sim_status rollout(sim_handle h, const float* x0, const float* u, float* loss_env, float* x_final,
                   float* lam_final, float* ckpt, uint32_t* env_flags, void* stream);

/* Forward rollout of a model in tolerance mode (solve_mode SIM_SOLVE_TOL),
 * as `rollout` without checkpoints, plus (each may be NULL, all device):
 *   iters_env[E]: Gauss-Seidel sweeps summed over the env's steps, counting
 *     the sweeps a rejected learned warm start cost;
 *   fallbacks_env[E]: steps whose learned warm start was rejected;
 *   records[rec_cap][SIM_REC_FLOATS]: one training record per placed contact
 *     of every step t with t % rec_every == 0 whose solve converged: floats
 *     0..6 the features (gap / dt, J v of the normal and both tangent rows at
 *     the velocities before the warm start, the plain warm-start impulses over
 *     their effective masses), 7..9 the converged impulses over their
 *     effective masses, 10 m_n, 11 m_t, then env, step and candidate code
 *     (kind << 24 | id; ground: index of the sphere among the env's ground
 *     spheres, pair: local body a | local body b << 12) as int32 bit
 *     patterns, 15 zero.  *rec_count (device,
 *     zeroed by the caller) is advanced atomically by the number of records
 *     wanted; only the first rec_cap are written, in no fixed order.
 * Returns SIM_E_STATE for a fixed-sweep model. */
sim_status rollout_solve(sim_handle h, const float* x0, const float* u, float* loss_env, float* x_final,
                         float* lam_final, uint32_t* env_flags, int32_t* iters_env, int32_t* fallbacks_env,
                         float* records, int64_t rec_cap, uint64_t* rec_count, int32_t rec_every, void* stream);

/* Reverse mode.  Given the checkpoints written by `rollout` with the same
 * x0 and u, and dL/dloss_env (device [E]), writes (each may be NULL):
 *   g_x0[18][B], g_u[T_max][J] (entries beyond an env's T_e are zero) or,
 *   for SIM_CTRL_MLP, dL/dW [n_params] summed over envs (the paper's dL/dW,
 *   section 2.2), g_inv_mass[B], g_inv_inertia[B][3], g_mu[E], g_damping[J],
 *   g_anchor_p[J][3] and g_anchor_c[J][3] (the hinge anchors in the parent,
 *   or world, frame and in the child frame: the link lengths of section 4)
 *   (device).
 * env_flags[E] (device, may be NULL) is overwritten: SIM_FLAG_GRAD_NONFINITE
 * for an env whose adjoint overflowed or exceeded 1e30 (the gradient of a
 * chaotic trajectory grows exponentially with its length; beyond 1e30 its sums
 * over env-steps are no longer representable); that env's gradients are
 * written as zeros and it contributes nothing to dL/dW.
 * workspace: device scratch of at least sim_info.workspace_bytes (the
 * per-env buffer of the checkpoint recompute, see SIM_GRAD_*, and, with a
 * controller, the per env-step activations and deltas plus the split-K
 * partial sums of the weight-gradient contraction).
 * In trajectory mode the call makes two launches per bucket: the recompute
 * of all segments (k_recompute), then the reverse sweep (k_rollout_grad). */
sim_status rollout_grad(sim_handle h, const float* x0, const float* u, const float* ckpt,
                        const float* dloss_env, float* g_x0, float* g_u, float* g_inv_mass,
                        float* g_inv_inertia, float* g_mu, float* g_damping, float* g_anchor_p,
                        float* g_anchor_c, void* workspace, size_t workspace_bytes, uint32_t* env_flags,
                        void* stream);

/* Forward rollout that keeps its working sets (trajectory mode only: the
 * model's sim_info.grad_store is SIM_GRAD_TRAJECTORY, else SIM_E_UNSUPPORTED;
 * fixed-sweep models).  As `rollout`, and it also writes every step's saved
 * working set into `workspace` (device, at least sim_info.workspace_bytes),
 * exactly what rollout_grad's recompute would write from the checkpoints, so
 * that rollout_grad_kept can skip that recompute.  ckpt may be NULL. */
sim_status rollout_keep(sim_handle h, const float* x0, const float* u, float* loss_env, float* x_final,
                        float* lam_final, float* ckpt, uint32_t* env_flags, void* workspace, size_t workspace_bytes,
                        void* stream);

/* Reverse mode after rollout_keep: as rollout_grad without its recompute,
 * reading the working sets that the last rollout_keep on this handle wrote to
 * `workspace` with the same x0 and u (the caller keeps the workspace
 * untouched in between).  The results are those of rollout_grad, bit for
 * bit. */
sim_status rollout_grad_kept(sim_handle h, const float* x0, const float* u, const float* dloss_env, float* g_x0,
                             float* g_u, float* g_inv_mass, float* g_inv_inertia, float* g_mu, float* g_damping,
                             float* g_anchor_p, float* g_anchor_c, void* workspace, size_t workspace_bytes,
                             uint32_t* env_flags, void* stream);

/* Forward and reverse mode in one call (trajectory mode, fixed-sweep
 * models): rollout_keep followed by rollout_grad_kept, with the same
 * arguments and the same results bit for bit, except that each size bucket's
 * reverse sweep starts as soon as that bucket's own forward has finished
 * instead of after the slowest bucket's (the buckets join once, at the end).
 * The upstream dL/dloss_env must therefore be known before the call (e.g. a
 * sum or mean of the envs' losses).  env_flags (nullable) receives the
 * forward's flags, grad_flags (nullable) the reverse's, as the two calls
 * write them.  While sim_time_grad events are set, the "reverse" pair spans
 * the whole call and the recompute pair is empty. */
sim_status rollout_and_grad(sim_handle h, const float* x0, const float* u, float* loss_env, float* x_final,
                            float* lam_final, float* ckpt, uint32_t* env_flags, const float* dloss_env, float* g_x0,
                            float* g_u, float* g_inv_mass, float* g_inv_inertia, float* g_mu, float* g_damping,
                            float* g_anchor_p, float* g_anchor_c, void* workspace, size_t workspace_bytes,
                            uint32_t* grad_flags, void* stream);

/* Allocation-free reverse mode, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving or training loops,
 * harnesses that forbid hipMalloc): rollout_grad with the same arguments and
 * results, except that its workspace is a scratch array of
 * SIM_NOALLOC_SCRATCH_BYTES in the library's own device memory, one per GPU,
 * set up by sim_init and held until the process ends.  The call itself
 * allocates and frees nothing.  Returns SIM_E_NOMEM, before any launch, when
 * the model's sim_info.workspace_bytes exceeds SIM_NOALLOC_SCRATCH_BYTES (pick
 * grad_store = SIM_GRAD_REPLAY or a grad_mem_limit that fits), and
 * SIM_E_STATE when the handle's device is not the current one.  Every call on
 * a GPU shares that GPU's scratch, which keeps the last call's contents
 * (nothing in it needs to start at zero): calls that overlap on one GPU,
 * from any handle, thread or stream, race and must be serialised by the
 * caller. */
#define SIM_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
sim_status rollout_grad_noalloc(sim_handle h, const float* x0, const float* u, const float* ckpt,
                                const float* dloss_env, float* g_x0, float* g_u, float* g_inv_mass,
                                float* g_inv_inertia, float* g_mu, float* g_damping, float* g_anchor_p,
                                float* g_anchor_c, uint32_t* env_flags, void* stream);

/* Device timing of rollout_grad's phases.  While set, every rollout_grad call
 * on h records, on its stream, ev[0] and ev[1] around the recompute of all
 * segments (back to back when the mode has no such phase) and ev[2] and ev[3]
 * around the reverse sweep (the weight-gradient contraction of a controller
 * comes after ev[3]).  ev: 4 hipEvent_t created by the caller, which keeps
 * them alive while they are set; ev = NULL stops the recording. */
sim_status sim_time_grad(sim_handle h, void* const* ev);

/* Device timing of each size bucket's reverse sweep.  While set, every
 * rollout_grad call records ev[2 i] and ev[2 i + 1] just before and after
 * bucket i's reverse sweep kernel, on the stream that kernel runs on.  ev:
 * 2 n hipEvent_t created by the caller, which keeps them alive while they
 * are set; n must be the bucket count (sim_get_teams); ev = NULL stops it. */
sim_status sim_time_buckets(sim_handle h, void* const* ev, int32_t n);
/* Host: the bucket (0 .. n-1, the order of sim_get_teams) that each env is
 * scheduled in; bucket_of_env[E]. */
sim_status sim_env_buckets(sim_handle h, int32_t* bucket_of_env);

/* ---- Replayable step sequences (HIP graphs). ----
 * Captures n_steps consecutive sim_step calls into a HIP graph, for callers
 * that step the simulation in a loop (a policy in the loop, serving): one
 * sim_graph_launch then costs one graph launch instead of n_steps x (queue
 * reset + kernel) launches per bucket.  Nothing runs at capture time.
 *   x: device [2][18][B]; step k reads x[k % 2] and writes x[(k + 1) % 2],
 *      so the result is in x[n_steps % 2].
 *   u: device control tape [n_steps][J] (step k uses row k) or, for
 *      SIM_CTRL_MLP, the controller weights [n_params].
 *   lam: device [lam_size], carried in place from step to step.
 *   t0: step index of the first step (the controller's clock input);
 *      with a controller t0 + n_steps <= T_max.
 *   env_flags: device [E] or NULL; holds the flags of the last step (a
 *      non-finite state stays non-finite, so it is still flagged).
 * The pointers are baked into the graph: every launch reads and writes the
 * same buffers.  A graph must not run concurrently with another call on the
 * same handle (they share the tile queues).  Release with sim_graph_destroy;
 * while graphs of a handle are alive, sim_destroy, sim_tune and
 * sim_set_teams refuse with SIM_E_STATE (the graphs use its tile lists). */
typedef struct sim_graph_s* sim_graph;
sim_status sim_step_graph(sim_handle h, int32_t n_steps, float* x, const float* u, float* lam, int32_t t0,
                          uint32_t* env_flags, sim_graph* out);
sim_status sim_graph_launch(sim_graph g, void* stream);
sim_status sim_graph_destroy(sim_graph g);

/* ---- The differentiable camera (paper section 3.4). ----
 * A pinhole camera at pos with axes (rows of axes: e_x right, e_y up, e_z the
 * optical axis) and its projection plane at distance focal; pixel (i, j) of a
 * width x height image (i to the right, j down) has its centre on the plane
 * at (u, v) = ((i + 1/2 - width/2) pitch, (height/2 - j - 1/2) pitch), and its
 * ray is pos + s d with d = focal e_z + u e_x + v e_y (the plane is s = 1).
 * The ray is intersected with every sphere of the env (the model's spheres:
 * centre p_b + R_b offset, the radius) and, when the model has a ground, the
 * plane z = 0; of all intersections the one closest in front of the
 * projection plane (the smallest s >= 1) is kept and its colour is a
 * bilinear sample of the object's texture (bilinear so that the image has
 * non-zero derivatives with respect to the state, as section 3.4 explains).
 * A sphere hit at h reads the sphere texture at texel coordinates
 * ((l_x + 1)(nx - 1)/2, (l_y + 1)(ny - 1)/2) for l = R_b^T (h - c) / r, its
 * direction in the body frame; the ground reads the ground texture at
 * (h_x, h_y) / ground_cell.  Texel (a, b) sits at integer coordinates
 * (texture[b * nx + a], row-major), indices wrap around.  A ray that hits
 * nothing has colour 0.  The camera and texture structs are read on the host
 * during the call (the caller keeps them); the textures stay on the device.
 * Both calls return SIM_E_ARG, before any launch, for a null pointer, a
 * width, height, focal length or pitch that is not positive, an image of more
 * than 2^28 pixels, a texture of fewer than 2 x 2 texels or a cell that is
 * not positive; SIM_E_DEVICE when a launch fails. */
typedef struct {
  float pos[3];
  float axes[9];       /* rows: right, up, optical axis (unit, orthogonal) */
  float focal, pitch;  /* > 0 */
  int32_t width, height;
} sim_camera;
typedef struct {
  const float* sphere;   /* device [sphere_ny][sphere_nx], nx, ny >= 2 */
  int32_t sphere_nx, sphere_ny;
  const float* ground;   /* device [ground_ny][ground_nx], nx, ny >= 2 */
  int32_t ground_nx, ground_ny;
  float ground_cell;     /* > 0 */
} sim_textures;
/* image (device [E][height][width], overwritten): every env seen by the
 * camera in the state x (device [18][B], as sim_step's).  Asynchronous on
 * stream. */
sim_status sim_render(sim_handle h, const float* x, const sim_camera* cam, const sim_textures* tex, float* image,
                      void* stream);
/* g_x (device [18][B], overwritten): dL/dx of every body's position (rows
 * 0..2) and rotation (rows 3..11) for L = sum of w * image, w device
 * [E][height][width]; the velocity rows are 0.  The hit object of each ray is
 * decided on the values (the silhouettes carry no derivative).  Every env
 * may hold at most SIM_RENDER_MAX_SPHERES spheres (else SIM_E_UNSUPPORTED).
 * Reduced per env in a fixed order: bitwise reproducible. */
#define SIM_RENDER_MAX_SPHERES 16
sim_status sim_render_grad(sim_handle h, const float* x, const sim_camera* cam, const sim_textures* tex,
                           const float* w, float* g_x, void* stream);

/* ---- Tile autotuning. ----
 * Envs are scheduled in buckets of equal team width (lanes per env) and LDS
 * class.  Results never depend on the width (the sweep order is fixed), only
 * the speed does.  sim_tune times, for each bucket, the forward rollout (and,
 * if with_grad, rollout_grad) of that bucket alone at each admissible width
 * (powers of two from the narrowest the bucket's envs allow whose tile fits
 * LDS; the first max_candidates of them), keeps the fastest, and writes the
 * chosen widths to teams[] (host, up to cap entries, may be NULL).  x0 and u
 * are as for rollout.  Synchronous; allocates and frees its own temporaries
 * (checkpoints, workspace).  Returns the number of buckets or a negative
 * sim_status.
 * sim_get_teams returns the bucket count and writes the current widths;
 * sim_set_teams applies widths (for instance cached from an earlier
 * sim_tune; each must be admissible), after synchronising the device. */
int32_t sim_tune(sim_handle h, const float* x0, const float* u, int32_t with_grad, int32_t max_candidates,
                 int32_t* teams, int32_t cap, void* stream);
int32_t sim_get_teams(sim_handle h, int32_t* teams, int32_t cap);
sim_status sim_set_teams(sim_handle h, const int32_t* teams, int32_t n);

/* ---- Learned warm start: the per-contact network. ----
 * 7 features -> 64 ReLU -> 64 ReLU -> 3 outputs; the 4,867 parameters are
 * packed W1[64][7] b1[64] W2[64][64] b2[64] W3[3][64] b3[3].  The kernels
 * use bfloat16 weights, inputs and hidden activations with FP32
 * accumulation on matrix cores.  Training records (SIM_REC_FLOATS floats,
 * written by rollout_solve) hold the features in floats 0..6 and the
 * targets in floats 7..9; see rollout_solve for their meaning.  All pointers
 * are device memory; calls are asynchronous on `stream`. */
#define SIM_WSN_IN 7
#define SIM_WSN_HID 64
#define SIM_WSN_OUT 3
#define SIM_WSN_PARAMS 4867
#define SIM_REC_FLOATS 16
/* w_bf16[p] = bfloat16(w[p]) (nearest, ties to even). */
sim_status wsn_to_bf16(const float* w, uint16_t* w_bf16, void* stream);
/* y[i][0..2] = net(x[i * stride + 0..6]) for i < n. */
sim_status wsn_forward(const uint16_t* w_bf16, const float* x, int64_t stride, int64_t n, float* y, void* stream);
/* Bytes of workspace wsn_loss_grad needs for n records. */
int64_t wsn_workspace_bytes(int64_t n);
/* Training loss over n records rec[i * stride + ...] (features x = floats
 * 0..6, targets t = floats 7..9, or, with relative != 0, floats 7..9 minus
 * floats 4..6: the correction to the carried impulses that the learned warm
 * start adds the network's output to):
 *   *loss = (1/n) sum_i sum_k rho(net(x_i)_k - t_ik),
 *   rho(e) = e^2 for |e| <= huber (every e when huber = 0), else
 *   2 huber |e| - huber^2,
 * and grad[4867] its gradient (either may be NULL).  Deterministic (fixed
 * reduction order). */
sim_status wsn_loss_grad(const uint16_t* w_bf16, const float* rec, int64_t stride, int64_t n, float huber,
                         int32_t relative, float* loss, float* grad, void* workspace, size_t workspace_bytes,
                         void* stream);
/* One Adam step (Kingma and Ba, with bias correction; step counts from 1) on
 * the FP32 master weights w, moments m and v, then w_bf16 = bfloat16(w). */
sim_status wsn_adam(float* w, uint16_t* w_bf16, const float* grad, float* m, float* v, int32_t step, float lr,
                    float beta1, float beta2, float eps, void* stream);

/* ---- Optimiser for the controller (section 2.2 policy search). ----
 * One Adam step (Kingma and Ba, with bias correction; step counts from 1) on
 * n FP32 parameters w with moments m and v, after scaling the gradient to a
 * norm of at most max_norm (0: no clipping).  A non-finite gradient norm
 * skips the step.  scratch: device, at least 513 floats (SIM_ADAM_SCRATCH);
 * grad_norm (device, may be NULL) receives the norm before clipping.  All
 * pointers are device memory; asynchronous on `stream`. */
#define SIM_ADAM_SCRATCH 513
sim_status sim_adam(float* w, const float* grad, float* m, float* v, int64_t n, int32_t step, float lr,
                    float beta1, float beta2, float eps, float max_norm, float* scratch, float* grad_norm,
                    void* stream);

#ifdef __cplusplus
}
#endif
#endif
