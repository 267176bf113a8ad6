/* FP64 CPU oracle: C interface used by the Python test harness (ctypes).
 *
 * TEST INFRASTRUCTURE ONLY: the product library never includes this header.
 * Arrays are host memory, float64, in the layouts of the seeded workload
 * generator (AoS per body/joint: x[B][18], inv_inertia[B][3], anchors [J][3]).
 */
#ifndef ORACLE_H
#define ORACLE_H
#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int n_envs;
  const int *env_body_off, *env_joint_off, *env_sphere_off; /* [E+1] */
  const double *inv_mass;     /* [B] */
  const double *inv_inertia;  /* [B][3] */
  const int *sphere_body;     /* [S] global body */
  const double *sphere_offset;/* [S][3] */
  const double *sphere_radius;/* [S] */
  const int *sphere_flags;    /* [S] bit0 ground, bit1 pair */
  const int *joint_parent, *joint_child; /* [J], parent -1 = world */
  const double *anchor_p, *anchor_c, *axis_p, *axis_c, *perp_p, *perp_c; /* [J][3] */
  const double *damping;      /* [J] */
  const double *mu;           /* [E] */
  const int *loss_body;       /* [E] global body */
  const double *target;       /* [E][3] */
  const int *T_env;           /* [E] */
  const double *u;            /* [T_max][u_stride] torque tape (ctrl_kind 0) */
  int u_stride, T_max;
  double dt, gravity[3], beta, gamma, spec_margin;
  int n_iters, ground, loss_kind, loss_mask;   /* loss_kind 3: final state: masked squared
                                                 position error + |v|^2 + |omega|^2 at T */
  int ctrl_kind;              /* 0 tape, 1 MLP controller shared by all envs */
  int mlp_in, mlp_h1, mlp_h2, mlp_out, mlp_n_params;
  const double *mlp_w;        /* W1[h1][in] b1 W2[h2][h1] b2 W3[out][h2] b3 */
  int mlp_rec;                /* recurrent state h^t of the controller (eq. (g)): the
                                 network reads [sensors, clock, h^t] (in = 2 J + 2 + rec)
                                 and emits [u^t, a] (out = J + rec), h^{t+1} = tanh(a),
                                 h^0 = 0; h^t is carried after the env's warm-start
                                 impulses in its carried-state block */
  double clock_hz;
  double warm;                /* warm-start factor applied to carried impulses */
  double noise;               /* test aid: relative rounding-sized noise added to the state after every step */
  int noise_seed;
  /* solve to a tolerance (forward only): after each sweep the residual is the
     largest |change of impulse| / effective mass over the active rows (for a
     friction block the norm of the tangent change over its mass), in m/s;
     sweeps stop at the first residual <= tol, or after max_iters sweeps. */
  int solve_mode;             /* 0 fixed n_iters sweeps, 1 to tolerance */
  double tol;
  int max_iters;
  /* learned warm start of contacts (tolerance mode): per-contact network
     7 -> 64 -> 64 -> 3 with ReLU, weights, inputs and hidden activations
     rounded to bfloat16, predicting the correction to the carried impulses
     (over their effective masses); if, after fb_iters sweeps, the solve has
     not converged and the residual of the contact rows exceeds fb_tol, the
     env's solve restarts from the plain warm start. */
  int ws_kind;                /* 0 plain, 1 learned */
  const double *ws_w;         /* W1[64][7] b1[64] W2[64][64] b2[64] W3[3][64] b3[3] */
  int fb_iters;
  double fb_tol;
  /* warm-start impulses at the start of a rollout ([lam_total], the layout
     of oracle_lambda_size's offsets); NULL: zeros.  A rollout started from a
     saved state and impulses continues the trajectory it was saved from. */
  const double *lam0;
  /* gradient decay (section 3.2): the adjoints carried back from step t+1
     to step t (state and warm-start impulses) are multiplied by grad_decay
     before step t is reversed; the loss term of x^{t+1} enters undecayed.
     1: the exact derivative. */
  double grad_decay;
  /* restitution (section 2.1.1's ball): per env e [E] or NULL (0).  A contact
     whose approach speed at the predicted velocities v* (before the warm
     start), v_n = J_n v* < -rest_threshold, would close its gap within the
     step (gap + dt v_n < 0) gets the normal-row bias min(b, e v_n), b the
     speculative or Baumgarte bias: it separates at e times its approach
     speed unless the push-out is faster. */
  const double *restitution;
  double rest_threshold;
  /* servo motors (section 2.1: gain, maximal torque, maximal velocity).  With
     servo != 0 every hinge is driven by a velocity motor and u^t_j is its
     target angle: a sixth row of the joint, angular about the parent's world
     hinge axis n_a (J w = n_a . (w_b - w_a)), aims at the rate
     clip(gain_j (u_j - theta_j), -vmax_j, vmax_j), theta_j the hinge angle
     (the controller's angle sensor), with its impulse clamped to
     [-torque_j dt, torque_j dt]; the joint's direct torque is then the
     viscous damping alone.  Arrays [J]. */
  int servo;
  const double *servo_gain, *servo_torque, *servo_vmax;
} oracle_model;

/* Warm-start network shape and training-record layout. */
#define ORACLE_WSN_IN 7
#define ORACLE_WSN_HID 64
#define ORACLE_WSN_OUT 3
#define ORACLE_WSN_PARAMS 4867
/* record: features f[7] (gap/dt, J_n v, J_t1 v, J_t2 v at the predicted
   velocities, plain warm-start impulses over their effective masses), target
   y[3] (converged impulses over their effective masses), m_n, m_t, env, step,
   candidate code (kind << 24 | id; ground: index of the sphere among the env's
   ground spheres, pair: local body a | local body b << 12), 0 */
#define ORACLE_REC 16

int oracle_lambda_size(const oracle_model* m, int* out_offsets /* [E+1] or NULL */);
int oracle_order(const oracle_model* m, int env, int* kinds, int* idx, int cap);
int oracle_step(const oracle_model* m, const double* x, const double* lam, const double* u, double* xn,
                double* lamn, int t);
int oracle_rollout(const oracle_model* m, const double* x0, double* loss_env, double* x_final,
                   double* lam_final, double* traj /* [T_max+1][B][18] or NULL */, int n_threads);
/* reverse mode: gradients of sum_e dloss[e] L_e with respect to x0, the
   torque tape (or the controller weights g_w), 1/m, 1/I, mu, damping and the
   hinge anchors in the parent and child frames (g_anchor_p, g_anchor_c [J][3]);
   any output may be NULL */
int oracle_rollout_grad(const oracle_model* m, const double* x0, const double* dloss, double* loss_env,
                        double* g_x0, double* g_u, double* g_inv_mass, double* g_inv_inertia,
                        double* g_mu, double* g_damping, double* g_w, double* g_anchor_p, double* g_anchor_c,
                        int n_threads);
/* Forward rollout with solver statistics: sweeps per env summed over its
   steps (sweeps discarded by a fallback included), fallbacks per env, and,
   with recs, one record per active contact of every converged step t with
   t % rec_every == 0 (envs in order).  Returns the number of records (only
   the first rec_cap are written). */
long long oracle_rollout_ex(const oracle_model* m, const double* x0, double* loss_env, double* x_final,
                            double* lam_final, int* iters_env, int* fallbacks_env, int rec_every, double* recs,
                            long long rec_cap, int n_threads);
/* controller outputs u^t (J_env values) of env `env` at state x [B][18] and
   step t; returns J_env, or -1 without a controller */
int oracle_controls(const oracle_model* m, int env, const double* x, int t, double* u_out);
/* bfloat16 rounding (nearest, ties to even) of a double */
double oracle_bf16(double x);
/* the warm-start network as used by the learned warm start (bfloat16
   weights, inputs and hidden activations): y[i][0..2] = net(x[i*stride..]) */
void oracle_wsn_forward(const double* w, const double* x, int stride, int n, double* y);

long long oracle_count_flops(const oracle_model* m, int env, const double* x, const double* lam,
                             const double* u, int t);

long long oracle_count_tape_edges(const oracle_model* m, int env, const double* x, const double* lam,
                                  const double* u, int t);

/* The differentiable camera (render.cpp; section 3.4).  axes: rows e_x
   (right), e_y (up), e_z (optical axis); focal: distance of the projection
   plane; pitch: pixel size on it. */
typedef struct {
  double pos[3], axes[9], focal, pitch;
  int width, height;
} oracle_camera;
/* grayscale textures, row-major: the spheres' (nx x ny) and the ground's,
   whose texel coordinates are the hit's (x, y) / cell */
typedef struct {
  const double* sphere;
  int sphere_nx, sphere_ny;
  const double* ground;
  int ground_nx, ground_ny;
  double ground_cell;
} oracle_textures;
/* image [E][H][W] of the state x [B][18] */
int oracle_render(const oracle_model* m, const double* x, const oracle_camera* cam, const oracle_textures* tex,
                  double* image);
/* g_x [B][18] = dL/dx for L = sum of w * image (w [E][H][W]) */
int oracle_render_grad(const oracle_model* m, const double* x, const oracle_camera* cam, const oracle_textures* tex,
                       const double* w, double* g_x);

#ifdef __cplusplus
}
#endif
#endif
