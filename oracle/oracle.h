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
  int n_iters, ground, loss_kind, loss_mask;
  int ctrl_kind;              /* 0 tape, 1 MLP controller shared by all envs */
  int mlp_in, mlp_h1, mlp_h2, mlp_out, mlp_n_params;
  const double *mlp_w;        /* W1[h1][in] b1 W2[h2][h1] b2 W3[out][h2] b3 */
  double clock_hz;
  double warm;                /* warm-start factor applied to carried impulses */
  double noise;               /* test aid: relative rounding-sized noise added to the state after every step */
  int noise_seed;
} oracle_model;

int oracle_lambda_size(const oracle_model* m, int* out_offsets /* [E+1] or NULL */);
int oracle_order(const oracle_model* m, int env, int* kinds, int* idx, int cap);
int oracle_step(const oracle_model* m, const double* x, const double* lam, const double* u, double* xn,
                double* lamn, int t);
int oracle_rollout(const oracle_model* m, const double* x0, double* loss_env, double* x_final,
                   double* lam_final, double* traj /* [T_max+1][B][18] or NULL */, int n_threads);
int oracle_rollout_grad(const oracle_model* m, const double* x0, const double* dloss, double* loss_env,
                        double* g_x0, double* g_u, double* g_inv_mass, double* g_inv_inertia,
                        double* g_mu, double* g_damping, double* g_w, int n_threads);
long long oracle_count_flops(const oracle_model* m, int env, const double* x, const double* lam,
                             const double* u, int t);

long long oracle_count_tape_edges(const oracle_model* m, int env, const double* x, const double* lam,
                                  const double* u, int t);

#ifdef __cplusplus
}
#endif
#endif
