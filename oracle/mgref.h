/* mgref.h -- FP64 CPU reference ("oracle") for the batched trajectory cost,
 * its gradient, the L-BFGS direction, the parallel noisy line search and the
 * solve loop of the motion optimizer in arXiv 2310.17274 (cuRobo).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  The product path
 * (the HIP library under paper_2310_17274_amd/) shares no code with it.
 *
 * Every array is host memory, double precision, row-major.  Conventions:
 *   pose      = x, y, z, qw, qx, qy, qz (unit quaternion, sign free)
 *   transform = 3x4 row-major [R | p]
 *   link l    = T(parent(l)) * fixed_tf[l] * Rz(q[joint[l]])   (Tab.6, F*J)
 */
#ifndef MGREF_H
#define MGREF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int n_links;              /* L; parent[l] < l (topological order) */
  int dof;                  /* D */
  const int *parent;        /* [L] parent link, -1 = base frame (identity) */
  const int *joint;         /* [L] joint index rotating the link about local z, -1 = fixed */
  const double *fixed_tf;   /* [L][12] joint frame in the parent frame */
  int n_spheres;            /* M */
  const int *sphere_link;   /* [M] */
  const double *sphere;     /* [M][4] center in link frame, radius */
  int n_ee;                 /* end effectors with a goal pose */
  const int *ee_link;       /* [n_ee] */
  const double *ee_tf;      /* [n_ee][12] tool frame in the link frame */
  const double *q_lo;       /* [D] */
  const double *q_hi;       /* [D] */
} mgref_robot;

typedef struct {
  double a0, a1, a2, a3;    /* pose reaching weights, Eq.(14) */
  double a6, a7, a8, a9;    /* smoothness weights, Eq.(16) */
  double w_bound, eta2;     /* joint-limit weight and band, Eq.(17) */
  double w_coll, eta;       /* world collision weight and activation distance, Eq.(10)/(11) */
  double dt;                /* waypoint spacing h of the five-point stencils */
  int vel_all;              /* 0: velocity logcosh term at t = T only; 1: at every t in [0,T] */
  int swept;                /* 1: continuous (swept) sphere collision, Sec. 'Continuous Collision Checking' */
  int sweep_steps;          /* maximum sphere-tracing samples per half segment */
  double w_self;            /* self-collision weight beta_1, Eq.(9) */
  int n_self;               /* sphere pairs checked for self-collision (the set S of Eq.(9)) */
  const int *self_pairs;    /* [n_self][2] sphere indices, or NULL */
  int speed;                /* 1: speed metric on the world collision term, Eq.(11) */
} mgref_params;

/* Forward kinematics of one configuration q[D] (Sec. 'Robot Kinematics', Alg.7, Tab.6).
 * Outputs (each may be NULL): link transforms [L][12], sphere centers [M][3],
 * end-effector poses [n_ee][7]. */
void mgref_fk(const mgref_robot *rb, const double *q, double *link_tf,
              double *spheres, double *ee_pose);

/* Rotation matrix -> unit quaternion (Shepperd's method), wxyz. */
void mgref_mat_to_quat(const double *R9, double *q4);

/* Exact signed distance from point c to a cuboid with pose (box->world) and
 * full side lengths dims: positive outside, minus the distance to the nearest
 * face inside.  grad (world frame, may be NULL) is d sdf / d c. */
double mgref_box_sdf(const double *pose7, const double *dims3, const double *c,
                     double *grad);

/* Collision activation profile d_c(d; eta) of Eq.(10) and its slope. */
double mgref_dc(double d, double eta, double *slope);

/* Joint-limit profile of Eq.(17) for one value and its slope. */
double mgref_bound(double x, double lo, double hi, double eta2, double *slope);

/* Five-point-stencil velocity, acceleration and jerk at t = 0..T of the
 * padded trajectory (start repeated three times, last waypoint repeated three
 * times).  q0[D], q[T][D]; v, a, j are [T+1][D] (each may be NULL). */
void mgref_derivatives(int T, int D, const double *q0, const double *q,
                       double dt, double *v, double *a, double *j);
/* Alg.4 retime: the spacing at which the largest |v|/vmax, |a|/amax or
 * |j|/jmax over t = 0..T reaches 1 (limits <= 0 are left out). */
double mgref_retime(int T, int D, const double *q0, const double *q, double dt,
                    const double *vmax, const double *amax, const double *jmax);

/* Total cost of one trajectory and its exact gradient.
 * q0[D] start, goal[n_ee][7], q[T][D].  T == 1 is the inverse-kinematics
 * problem (no start, no smoothness).  grad [T][D] may be NULL.
 * min_clear (may be NULL) = min over waypoints, spheres, cuboids of
 * min(sdf - r, eta): the trajectory is collision free iff it is >= 0.
 * terms (may be NULL) = {smooth, bound, collision, pose}. */
double mgref_traj_cost(const mgref_robot *rb, const mgref_params *pr,
                       int n_box, const double *box_pose, const double *box_dims,
                       const double *q0, const double *goal, int T,
                       const double *q, double *grad, double *min_clear,
                       double *terms);

/* Position error |p_g - p| and rotation angle 2 acos(min(1,|<q_g,q>|)) of
 * each end effector at configuration qT[D].  pos_err, rot_err: [n_ee]. */
void mgref_pose_error(const mgref_robot *rb, const double *qT, const double *goal,
                      double *pos_err, double *rot_err);

/* Batch of S trajectories of one problem: cost[S], grad[S][T][D] (or NULL),
 * min_clear[S] (or NULL).  nthreads > 1 evaluates seeds in parallel. */
void mgref_cost_grad_batch(const mgref_robot *rb, const mgref_params *pr,
                           int n_box, const double *box_pose, const double *box_dims,
                           const double *q0, const double *goal, int T, int S,
                           const double *q, double *cost, double *grad,
                           double *min_clear, int nthreads);

/* One L-BFGS direction (Alg.6; Nocedal & Wright Alg. 7.4) for a vector of
 * length n with history m.  State: count, head, S[m][n], Y[m][n], rho[m],
 * x_prev[n], g_prev[n].  reset != 0 clears the history.  dir = -H g. */
void mgref_lbfgs_step(int n, int m, int reset, int *count, int *head,
                      double *S, double *Y, double *rho, double *x_prev,
                      double *g_prev, const double *x, const double *g,
                      double *dir);

/* Selection rule of the parallel noisy line search (Alg.1): largest k whose
 * conditions hold, else 0.  mode 0 Armijo, 1 Armijo + weak Wolfe,
 * 2 Armijo + strong Wolfe.  c[K] costs, gd[K] = <g_k, d>, g0d = <g_0, d>. */
int mgref_ls_select(int K, const double *alpha, double c0, double g0d,
                    const double *c, const double *gd, int mode, double eta1,
                    double eta_w);

/* Parallel noisy line search of one trajectory (Alg.1).  Candidates
 * clip(x + alpha_k d) are costed with gradients; returns the chosen index and
 * writes x_out, g_out ([T][D]), *c_out and *mc_out (min clearance). */
int mgref_linesearch(const mgref_robot *rb, const mgref_params *pr,
                     int n_box, const double *box_pose, const double *box_dims,
                     const double *q0, const double *goal, int T,
                     const double *x, double c0, const double *g0, const double *dir,
                     int K, const double *alpha, int mode, double eta1, double eta_w,
                     double *x_out, double *c_out, double *g_out, double *mc_out);

/* Solve loop of one problem with S seeds (Sec. 'Parallel L-BFGS Optimization'): iters iterations of
 * L-BFGS direction + line search + best tracking per seed.  x[S][T][D] holds
 * the seeds on entry and the best iterate per seed on exit; best_cost[S].
 * trace (may be NULL) receives best_cost after each iteration [iters][S]. */
void mgref_solve(const mgref_robot *rb, const mgref_params *pr,
                 int n_box, const double *box_pose, const double *box_dims,
                 const double *q0, const double *goal, int T, int S, double *x,
                 int iters, int m, int K, const double *alpha, int mode,
                 double eta1, double eta_w, double *best_cost, double *trace,
                 int nthreads);

/* Particle-based optimization (Sec. 'Particle-Based Optimization', Alg.5,
 * Eq.(12)-(13)), update step of one seed with n elements and N particles:
 * weights w = softmax(-(C - min C) / beta) (exponential utility), then
 *   mu'  = (1 - k_mu) mu + k_mu sum_i w_i theta_i
 *   var' = (1 - k_sigma) var + k_sigma sum_i w_i (theta_i - mu)^2
 * with mu the mean before the update.  Readings: the printed variance update
 * lacks k_sigma and squares theta instead of the deviation; it is taken as
 * the weighted variance about the previous mean.  beta <= 0 selects
 * beta = 0.1 (max C - min C) + 1e-12.  theta[N][n]; w_out[N] may be NULL. */
void mgref_particle_update(int n, int N, const double *cost, const double *theta,
                           double *mu, double *var, double beta, double k_mu,
                           double k_sigma, double *w_out);

/* Particle stage of one problem with S seeds of T waypoints: n_iters rounds
 * of sampling theta_i = clip(mu + sqrt(var) * eps_i) (eps standard normal,
 * given: [n_iters][N][S][T][D]), costing every particle (cost only) and the
 * update above.  mu[S][T][D] holds the seeds on entry and the final means on
 * exit; var[S][T][D] the initial and final variances.  cost_out (may be
 * NULL) receives [n_iters][S][N] particle costs. */
void mgref_particles(const mgref_robot *rb, const mgref_params *pr,
                     int n_box, const double *box_pose, const double *box_dims,
                     const double *q0, const double *goal, int T, int S, double *mu,
                     double *var, int N, int n_iters, const double *eps, double beta,
                     double k_mu, double k_sigma, double *cost_out, int nthreads);

/* Counter-based normal draws of the particle stage (Alg.5 samples its
 * particles from a zero-mean Gaussian).  Philox-4x64 with 10 rounds (Salmon,
 * Moraes, Dror, Shaw, 'Parallel random numbers: as easy as 1, 2, 3', SC'11):
 * out = philox(ctr, key).  The draw of element e (= row * D + joint of the
 * batch's rows), particle k and round it under seed s takes word e mod 4 of
 * philox({e / 4, k, it, 0}, {s, 0}); its bits 41..63 and 9..31 give
 * u1, u2 = (23-bit integer + 1/2) / 2^23, and the draw is the Box-Muller
 * value sqrt(-2 ln u1) cos(2 pi u2). */
void mgref_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);
double mgref_philox_normal(uint64_t seed, int it, int k, int64_t e);
/* [n_iters][N][rows][D] draws of rounds 0..n_iters-1, particles 0..N-1. */
void mgref_philox_normals(uint64_t seed, int n_iters, int N, int rows, int D, double *out);

#ifdef __cplusplus
}
#endif
#endif
