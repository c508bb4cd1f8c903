/* mg.h -- C ABI of the MI355X (gfx950) batched trajectory-optimizer hot path.
 *
 * The library evaluates, for many seeds x waypoints x line-search candidates
 * at once, the motion-generation objective of arXiv 2310.17274 (cuRobo),
 * Sec. "Motion Generation as Optimization", Eq.(1) with its constraints
 * turned into costs:
 *   - forward kinematics of the robot's collision spheres (Sec. "Robot
 *     Kinematics", Tab.6) and of the end effector;
 *   - sphere-vs-cuboid world collision cost (Eq.(10), Eq.(11), Alg.10),
 *     summed over cuboids and spheres, optionally swept between waypoints
 *     (Sec. "Continuous Collision Checking");
 *   - joint-limit cost (Eq.(17));
 *   - five-point-stencil velocity / acceleration / jerk smoothness cost
 *     (Eq.(16), appendix "Finite Difference for State Derivatives");
 *   - pose-reaching cost at the last waypoint (Eq.(14));
 * with a hand-written gradient (adjoint) that recomputes kinematics, and the
 * solver built on it: the L-BFGS direction (Alg.6) and the parallel noisy
 * line search (Alg.1) with best-iterate tracking (Sec. "Parallel L-BFGS
 * Optimization").
 *
 * Conventions
 *   - All floating point is fp32, integers are int32.
 *   - A pose is 7 floats: x, y, z, qw, qx, qy, qz (unit quaternion).
 *   - A transform is a 3x4 row-major matrix [R | p].
 *   - Link l of the robot is T(parent(l)) * fixed_tf[l] * Rz(q[joint[l]]).
 *   - A trajectory of problem p is T_p waypoints x D joints, row-major; the
 *     trajectories of all seeds of all problems are concatenated in problem
 *     order, then seed order ("rows" = sum_p S_p * T_p waypoint rows).
 *   - "Device" pointers are HIP device memory; "host" pointers are host
 *     memory read during the call only.  The caller owns every buffer it
 *     passes; the library owns its context, batch tables and workspaces.
 *   - stream is a hipStream_t (NULL = the null stream).  Calls enqueue work
 *     and return; outputs are valid once the stream has executed it.
 *   - Every function returns MG_OK or a negative mg_status and then writes
 *     nothing; mg_last_error() describes the last failure of this thread.
 *     NaN inputs propagate to NaN outputs and are not detected.
 *   - A context is not thread safe; use one per thread or serialise calls.
 */
#ifndef MG_H
#define MG_H

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MG_OK = 0,
  MG_ERR_ARG = -1,          /* null or inconsistent argument */
  MG_ERR_SHAPE = -2,        /* a size outside the supported range */
  MG_ERR_HIP = -3,          /* a HIP runtime call failed */
  MG_ERR_OOM = -4,          /* device allocation failed */
  MG_ERR_UNSUPPORTED = -5,  /* valid request this build does not implement */
  MG_ERR_STATE = -6         /* call out of order (e.g. no world set) */
} mg_status;

typedef struct mg_ctx mg_ctx;       /* robot, cost parameters, worlds */
typedef struct mg_batch mg_batch;   /* problem layout and solver workspaces */

/* Robot description, all HOST pointers, copied by mg_create.
 * Links are in topological order (parent[l] < l).  1 <= dof <= 16,
 * n_links <= 16 along any root-to-link chain, 1 <= n_ee <= 2, radius > 0. */
typedef struct {
  int n_links;              /* L */
  int dof;                  /* D */
  int n_spheres;            /* M */
  int n_ee;                 /* end effectors with a goal pose */
  const int *parent;        /* [L] parent link or -1 (base frame = identity) */
  const int *joint;         /* [L] joint index 0..D-1 rotating the link about z, or -1 */
  const float *fixed_tf;    /* [L][12] joint frame in the parent link frame */
  const int *sphere_link;   /* [M] */
  const float *sphere;      /* [M][4] center in the link frame, radius */
  const int *ee_link;       /* [n_ee] */
  const float *ee_tf;       /* [n_ee][12] tool frame in the link frame */
  const float *q_lo;        /* [D] joint limits (Eq.(2)) */
  const float *q_hi;        /* [D] */
} mg_robot_desc;

/* Cost and solver parameters.  mg_default_params() fills the paper's values:
 * a0..a3 = 2000, 350, 100, 100 (Eq.(14)); a6..a9 = 5000, 50, 5000, 1
 * (Eq.(16)); w_bound = w_coll = 5000 and eta = 0.025 m (appendix "cuRobo
 * Parameters"); eta2 = 0.1 (Eq.(17)); dt = 0.25 s (Alg.4 first pass). */
typedef struct {
  float a0, a1, a2, a3;     /* pose: a0 logcosh(a2 |dp|) + a1 logcosh(a3 d_rot) */
  float a6, a7, a8, a9;     /* smoothness weights of Eq.(16) */
  float w_bound, eta2;      /* joint-limit weight and band */
  float w_coll, eta;        /* collision weight and activation distance */
  float dt;                 /* waypoint spacing of the stencils */
  int vel_all;              /* 0: velocity term at the last waypoint only; 1: all */
  int swept;                /* 1: swept-sphere (continuous) collision, Alg.11-12 */
  int sweep_steps;          /* max sphere-tracing samples per half segment, 0..64 */
  float ls_eta1;            /* Armijo constant (default 1e-4) */
  float ls_eta_w;           /* Wolfe constant (default 0.9) */
  float success_pos;        /* success: position error <= (default 0.005 m) */
  float success_rot;        /* success: rotation angle <= (default 0.05 rad) */
  float w_self;             /* self-collision weight beta_1 of Eq.(9) (default 5000) */
  int speed;                /* 1: speed metric of Eq.(11) (default 0): each sphere's world
                               collision cost times its speed |c(t+1) - c(t-1)| / (2 dt) on
                               the padded trajectory (start before waypoint 1, waypoint T
                               after T), with its exact gradient (the speed's gradient acts
                               on the neighbouring waypoints; a second launch adds it).
                               Evaluated by the wave-per-link layout only (robots of at
                               most 15 links), one workgroup per 64 evaluations; batches
                               keep a [K_max][rows][spheres] float4 buffer for it while it
                               is on (allocated by mg_batch_create / mg_set_params). */
} mg_params;

void mg_default_params(mg_params *out);

/* Create a context on the current HIP device.  Copies robot tables and
 * parameters to the device.  Not capturable (allocates, synchronises). */
mg_status mg_create(const mg_robot_desc *robot, const mg_params *params, mg_ctx **out);
void mg_destroy(mg_ctx *ctx);

/* Replace the parameters (same robot).  Host-only; affects later calls. */
mg_status mg_set_params(mg_ctx *ctx, const mg_params *params);

/* Set the cuboid worlds (Sec. "World Representation": oriented bounding
 * boxes).  offsets: HOST [n_worlds+1] prefix sums of cuboid counts;
 * pose: DEVICE [n][7] box-to-world poses; dims: DEVICE [n][3] full side
 * lengths (> 0).  The cuboids are converted on stream into the library's own
 * layout; pose/dims may be reused by the caller once the stream reaches this
 * point.  Reallocates (not capturable) only when n or n_worlds grow. */
mg_status mg_set_worlds(mg_ctx *ctx, int n_worlds, const int *offsets,
                        const float *pose, const float *dims, void *stream);

/* Describe a batch of P problems, all HOST arrays [P]: seeds per problem
 * (>= 1), horizon T (1..64; 1 = inverse kinematics), world index.  K_max
 * (1..16) bounds the line-search candidates and m_max (0..16) the L-BFGS
 * history of later calls.  Allocates tables and workspaces (not capturable). */
mg_status mg_batch_create(mg_ctx *ctx, int P, const int *seeds, const int *horizon,
                          const int *world, int K_max, int m_max, mg_batch **out);
void mg_batch_destroy(mg_batch *batch);
/* Totals of a batch: seeds and waypoint rows (floats per array = rows * D). */
int mg_batch_seeds(const mg_batch *batch);
int mg_batch_rows(const mg_batch *batch);

/* Cost (and gradient) of every seed's trajectory (Eq.(1) as soft costs).
 *   q_start DEVICE [P][D]   start configuration theta_0 (unused for T = 1)
 *   goal    DEVICE [P][n_ee][7]
 *   q       DEVICE [rows][D] trajectories
 *   cost    DEVICE [seeds]  total cost per seed
 *   grad    DEVICE [rows][D] d cost / d q, or NULL for cost only
 *   min_clear DEVICE [seeds] min over waypoints, spheres and cuboids of
 *           min(signed distance - radius, eta), or NULL; a trajectory is
 *           collision free iff its value is >= 0.  Capturable. */
mg_status mg_cost_grad(mg_ctx *ctx, mg_batch *batch, const float *q_start,
                       const float *goal, const float *q, float *cost, float *grad,
                       float *min_clear, void *stream);

/* L-BFGS direction (Alg.6; Nocedal & Wright two-loop recursion) for every
 * seed: dir = -H g with history m <= m_max kept in the batch.  reset != 0
 * starts a new history (first iteration).  x, g, dir: DEVICE [rows][D].
 * Pairs with <y,s> <= 1e-10 |s||y| are not stored; H0 = gamma I with gamma
 * = <s,y>/<y,y> of the newest pair, or min(1, 0.1/|g|_inf) without one.
 * Capturable. */
mg_status mg_lbfgs_step(mg_ctx *ctx, mg_batch *batch, int m, int reset,
                        const float *x, const float *g, float *dir, void *stream);

/* Parallel noisy line search (Alg.1) for every seed: candidates
 * clip(x + alpha_k dir, q_lo, q_hi), k < K, are costed with gradients in one
 * launch; the largest k meeting the conditions is chosen, else k = 0 (the
 * paper's 0.01 noisy step).  mode 0: Armijo c_k <= c0 + eta1 alpha_k <g0,d>;
 * 1: + weak Wolfe <g_k,d> >= eta_w <g0,d>; 2: + strong Wolfe
 * |<g_k,d>| <= eta_w |<g0,d>|.
 *   alpha   HOST [K], K <= K_max
 *   x, g0, dir DEVICE [rows][D]; c0 DEVICE [seeds]
 *   x_out, g_out DEVICE [rows][D]; c_out DEVICE [seeds] (may alias x, g0, c0)
 *   chosen  DEVICE [seeds] or NULL; min_clear DEVICE [seeds] or NULL.
 * Capturable. */
mg_status mg_linesearch(mg_ctx *ctx, mg_batch *batch, const float *q_start,
                        const float *goal, const float *x, const float *c0,
                        const float *g0, const float *dir, int K, const float *alpha,
                        int mode, float *x_out, float *c_out, float *g_out, int *chosen,
                        float *min_clear, void *stream);

/* The batched evaluation of the line-search candidates (Alg.1: every
 * candidate of every seed costed with its gradient in one launch), without
 * the choice: candidate k < K of a seed is clip(x + alpha_k dir, q_lo, q_hi)
 * and is evaluated by the same launch mg_linesearch and mg_solve make for
 * these K candidates (layout, workgroups and all).
 *   x, dir DEVICE [rows][D]; alpha HOST [K], K <= K_max
 *   cost DEVICE [K][seeds] total cost of each candidate
 *   gd   DEVICE [K][seeds] directional derivative <grad C(x_k), dir>
 *   grad DEVICE [K][rows][D] gradient of each candidate, or NULL
 *   min_clear DEVICE [K][seeds] clearance (as mg_cost_grad), or NULL.
 * Capturable. */
mg_status mg_linesearch_eval(mg_ctx *ctx, mg_batch *batch, const float *q_start, const float *goal,
                             const float *x, const float *dir, int K, const float *alpha, float *cost,
                             float *gd, float *grad, float *min_clear, void *stream);

/* mg_linesearch for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same arguments, checks and results as mg_linesearch, but the
 * per-(candidate, row) costs, directional derivatives, clearances and
 * gradients of the call live in a static device array of the library
 * (16 MiB per GPU, held until the process ends) instead of the batch's
 * workspace.  The call allocates nothing; K * rows * (3 + D) floats (each
 * of the first three parts rounded up to 64) must fit in 4 Mi floats, else
 * MG_ERR_SHAPE.  The wave-per-link layout runs with one workgroup per
 * chunk (no cuboid slices over workgroups); with the speed metric on it
 * returns MG_ERR_UNSUPPORTED.  Every call on one GPU shares
 * that GPU's array and overwrites it: calls that overlap on one GPU (other
 * streams, other threads, other contexts) race.  Nothing in the array needs
 * clearing between calls.  Capturable. */
mg_status mg_linesearch_noalloc(mg_ctx *ctx, mg_batch *batch, const float *q_start,
                                const float *goal, const float *x, const float *c0,
                                const float *g0, const float *dir, int K, const float *alpha,
                                int mode, float *x_out, float *c_out, float *g_out, int *chosen,
                                float *min_clear, void *stream);

/* Full solve (Sec. "Parallel L-BFGS Optimization"): iters iterations of
 * direction + line search + best tracking for every seed, in place.
 *   x        DEVICE [rows][D]: seeds on entry, best iterate per seed on exit
 *   best_cost DEVICE [seeds]; best_seed DEVICE [P] (argmin, lowest index on
 *            ties) or NULL; success DEVICE [P] (best seed within
 *            success_pos / success_rot of the goal and collision free) or NULL.
 * use_graph != 0 captures graph_inner iterations in a hipGraph and replays it
 * (the first call for a new argument set captures; later calls replay; when
 * the choices are folded into the evaluation launches, see
 * mg_batch_set_fusion, a graph holds graph_inner rounded up to even
 * iterations); use_graph == 0 launches every kernel directly.  The batch's
 * L-BFGS history and workspaces are the solve's: their contents after the
 * call are unspecified.  Not capturable itself. */
mg_status mg_solve(mg_ctx *ctx, mg_batch *batch, const float *q_start, const float *goal,
                   float *x, int iters, int m, int K, const float *alpha, int mode,
                   int graph_inner, int use_graph, float *best_cost, int *best_seed,
                   int *success, void *stream);

/* Self-collision (Sec. "Self-Collision Avoidance", Eq.(9)): at every
 * waypoint, w_self times the largest penetration r_i + r_j - |x_i - x_j|
 * over the listed sphere pairs (0 if none overlaps); its gradient acts on
 * the two spheres of the first listed pair reaching the maximum.
 *   pairs HOST [n_pairs][2] sphere indices (i != j); n_pairs = 0 turns the
 *   term off.  Copied to the device (not capturable).
 * The term is evaluated by the wave-per-link layout only: while pairs are
 * set, every evaluation uses it (robots of at most 15 links; otherwise
 * MG_ERR_UNSUPPORTED), mg_particles included (with the particle count of
 * the last mg_batch_reserve_particles, at least 2). */
mg_status mg_set_self_collision(mg_ctx *ctx, int n_pairs, const int *pairs);

/* Forward kinematics of the end effectors (Sec. "Robot Kinematics", Tab.6):
 * pose (x, y, z, qw, qx, qy, qz; Shepperd's quaternion, sign unspecified)
 * of every end effector at each of `rows` configurations.
 *   q DEVICE [rows][D]; pose DEVICE [rows][n_ee][7].  Capturable. */
mg_status mg_ee_pose(mg_ctx *ctx, int rows, const float *q, float *pose, void *stream);

/* Evaluation layouts.  Lane per link (layout 0): 8 or 16 lanes per
 * evaluation, one per link, with the world's cuboids split over 1, 2 or 4
 * waves ("slices").  Wave per link (layout 1): 64 evaluations per
 * workgroup, one wave per link plus one for the joint terms, each wave
 * skipping the cuboids that a ball around its link's spheres over all 64
 * lanes cannot reach (with swept collision, the ball grows by half the
 * longer segment); needs at most 15 links; the particle stage does not use it.
 * The wave-per-link layout can also split the cuboids over 2, 4, 8 or 16
 * workgroups per 64 evaluations (as many as the batch's 64 MB of slice
 * scratch holds); the last to finish adds the slices' sums in slice order
 * (the batch keeps the scratch and counters).
 * A robot of up to 8 links can also give each link two waves with half of
 * its spheres each (layout 2), the second also taking that link's joint
 * terms: shorter waves, no separate joint wave.  Layout 3 keeps one wave
 * per link but holds 32 evaluations per workgroup, each half of a wave
 * testing half of the link's sphere slots (twice the workgroups for the
 * same batch; no self-collision, at least 4 slots per link); layout 4 holds
 * 16 evaluations per workgroup, each quarter of a wave testing a quarter of
 * the slots (four times the workgroups; at least 8 slots per link).  In
 * both, two lane groups split each evaluation's kinematic chain in halves.
 * mg_batch_set_layout fixes a layout (-1: library default, 0 .. 4) and a
 * slice count (0: automatic; 1, 2 or 4, and for layout 1 also 8 or 16;
 * layouts 2, 3 and 4 take 0 or 1).
 * Host-only; affects later calls.
 *
 * Autotuner for a batch's launch shape: times the line-search evaluation
 * kernel for K candidates under every layout and slice count the library
 * offers for this robot (mg_time_eval with `launches` launches each) and
 * fixes the fastest for every later call on this batch.  *slices_out (may
 * be NULL) receives the slice count for the lane-per-link layout, minus
 * the workgroups per 64 evaluations for the wave-per-link layout, -8 for
 * two waves per link, -16 for two slot groups per wave or -32 for four.
 * Overwrites the batch's evaluation workspaces; not capturable.  With
 * swept collision the lane-per-link layout takes one slice. */
mg_status mg_batch_set_layout(mg_batch *batch, int layout, int slices);

/* Choice folded into the next evaluation (Alg.1 and Alg.6 inside the
 * iteration loop of Sec. "Parallel L-BFGS Optimization"): with enable != 0
 * (the default) mg_solve computes each iteration's line-search choice and
 * next L-BFGS direction at the start of the following iteration's
 * evaluation launch (every workgroup for its own seed, the seed's first one
 * storing them) instead of in a launch of its own, where the batch
 * qualifies: wave-per-link layout with one wave per link and at most 7
 * links (one, two or four slot groups), no swept collision or speed metric,
 * one horizon T with 128 < T * D <= 256 and T * D a multiple of 4, K <= 8,
 * m <= 4, and x 16-byte aligned.  The results are those of the separate
 * launches, bit for bit.  enable = 0 keeps the launches
 * separate.  Host-only; affects later calls.  Errors: MG_ERR_ARG (null
 * batch). */
mg_status mg_batch_set_fusion(mg_batch *batch, int enable);
/* 1 when mg_solve on this batch with K candidates, history m and iterate x
 * (device pointer, only its alignment is looked at) folds the choices into
 * the evaluation launches, else 0 (also for invalid arguments).  Host-only. */
int mg_solve_fuses(mg_ctx *ctx, mg_batch *batch, int K, int m, const float *x);
mg_status mg_autotune(mg_ctx *ctx, mg_batch *batch, const float *q_start, const float *goal,
                      const float *x, const float *dir, int K, const float *alpha, int launches,
                      int *slices_out, void *stream);

/* Particle-based optimization (Sec. "Particle-Based Optimization", Alg.5,
 * Eq.(12)-(13)), run before L-BFGS to move the seeds to a good region.
 * mg_batch_reserve_particles allocates the per-row particle costs for up to
 * n_particles (1..1024) particles per seed (not capturable).  mg_particles
 * runs n_iters rounds; each round, for every seed,
 *   theta_i = clip(mean + sqrt(var) * eps_i, q_lo, q_hi),  i < n_particles
 * is costed (cost only, one launch over all seeds and particles), then with
 * w = softmax(-(C - min C) / beta) (exponential utility)
 *   mean' = (1 - k_mu) mean + k_mu sum_i w_i theta_i
 *   var'  = (1 - k_sigma) var + k_sigma sum_i w_i (theta_i - mean)^2.
 * The printed variance update lacks k_sigma and squares theta rather than
 * its deviation; it is read as the weighted variance about the previous
 * mean.  beta <= 0 uses 0.1 (max C - min C) + 1e-12 per seed.
 *   mean, var DEVICE [rows][D] in/out (var per element, rad^2)
 *   eps       DEVICE [n_iters][n_particles][rows][D] standard normal draws
 *   costs_out DEVICE [n_iters][seeds][n_particles] particle costs, or NULL
 * The costing launch is wave per link (one slot group per wave, unless
 * mg_batch_set_layout chose two or four) when n_particles is the last reserved
 * count and the layout fits the robot, lane per link when
 * mg_batch_set_layout chose it (self-collision and the speed metric keep
 * wave per link); the autotuner's choice for line-search candidates is not
 * carried over.
 * MG_ERR_STATE if n_particles exceeds the reservation.  Capturable. */
mg_status mg_batch_reserve_particles(mg_batch *batch, int n_particles);
mg_status mg_particles(mg_ctx *ctx, mg_batch *batch, const float *q_start, const float *goal,
                       float *mean, float *var, int n_particles, int n_iters, const float *eps,
                       float beta, float k_mu, float k_sigma, float *costs_out, void *stream);

/* The particle stage with its noise drawn on the device: as mg_particles,
 * with round it's draws eps[k][row][j] the counter-based standard normals of
 * mg_philox_normals(seed, it, ...) (it = 0 .. n_iters - 1 <= 65535).  The
 * evaluation kernel makes each particle's draws where it forms the particle
 * and the update kernel makes them again (one Philox block per four
 * elements): no draw is stored, read back or uploaded.  Capturable. */
mg_status mg_particles_seeded(mg_ctx *ctx, mg_batch *batch, const float *q_start, const float *goal,
                              float *mean, float *var, int n_particles, int n_iters,
                              unsigned long long seed, float beta, float k_mu, float k_sigma,
                              float *costs_out, void *stream);

/* Counter-based standard normal draws (Alg.5 samples its particles from a
 * zero-mean Gaussian): out[i][k][e] for rounds it = it0 + i, particles k and
 * elements e = row * dof + joint is word e mod 4 of Philox-4x64-10 (Salmon,
 * Moraes, Dror, Shaw, SC'11) at counter {e / 4, k, it, 0} and key {seed, 0},
 * turned into a normal by Box-Muller: bits 41..63 and 9..31 give u1, u2 =
 * (23-bit integer + 1/2) / 2^23, draw = sqrt(-2 ln u1) cos(2 pi u2).
 *   out DEVICE [n_iters][n_particles][rows][dof], 16-byte aligned.
 * Capturable. */
mg_status mg_philox_normals(unsigned long long seed, int it0, int n_iters, int n_particles, int rows,
                            int dof, float *out, void *stream);

/* Retiming (Alg.4 retime, appendix "Time-step Descretization and Temporal
 * Weight Scaling"): for every seed, the waypoint spacing at which the
 * seed's largest joint velocity, acceleration or jerk reaches its limit.
 * The five-point stencils at the context's dt (start padded with q_start,
 * t = 0..T) give v, a, j; derivatives of order k scale as dt^-k, so the
 * result is dt times the largest of |v| / vmax, sqrt(|a| / amax),
 * cbrt(|j| / jmax) over waypoints and joints.
 *   q_start DEVICE [P][D]; x DEVICE [rows][D]
 *   vmax, amax, jmax HOST [D] per-joint limits (rad/s, rad/s^2, rad/s^3); a
 *     limit <= 0 leaves its kind out; NaN is MG_ERR_ARG
 *   dt_out DEVICE [seeds] (0 for a seed that never leaves its start)
 *   jerk_out DEVICE [seeds] or NULL: the seed's largest |jerk| read at its
 *     retimed spacing (the selection's jerk metric; 0 at rest).
 * Capturable. */
mg_status mg_retime(mg_ctx *ctx, mg_batch *batch, const float *q_start, const float *x,
                    const float *vmax, const float *amax, const float *jmax, float *dt_out,
                    float *jerk_out, void *stream);

/* Time-step optimization (Alg.4): two solves with the spacing re-chosen in
 * between.  (1) mg_solve for iters1 iterations at the context's dt with the
 * jerk weight a9 set to 0; (2) dt_opt = the largest mg_retime of the
 * problems' best seeds, at least dt_min (one spacing for the whole batch);
 * (3) with rho = dt_opt / dt the derivative weights become a7 rho, a8 rho^4
 * and a9 rho^6 (the paper's "scale weights by the new dt", read as keeping
 * the cost of the same waypoints unchanged, since v, a, j scale as rho^-1,
 * rho^-2, rho^-3), jerk back on; (4) mg_solve for iters2 iterations from the
 * first pass's best iterates at dt_opt; (5) dt_f = the largest retime of the
 * new best seeds.  The context's parameters are restored on return.
 *   x DEVICE [rows][D] seeds in, best iterates out; best_cost, best_seed,
 *   success as mg_solve (of the second pass); vmax, amax, jmax as mg_retime;
 *   dt_out HOST [2] = {dt_opt, dt_f}.
 * Not capturable (allocates two small buffers, reads the spacings on the
 * host between the passes). */
mg_status mg_solve_timestep(mg_ctx *ctx, mg_batch *batch, const float *q_start, const float *goal,
                            float *x, int iters1, int iters2, int m, int K, const float *alpha,
                            int mode, int graph_inner, int use_graph, const float *vmax,
                            const float *amax, const float *jmax, float dt_min, float *best_cost,
                            int *best_seed, int *success, float *dt_out, void *stream);

/* Seeds for trajectory optimization from collision-free IK (the paper's
 * global motion generation: IK, then seeds, then trajectory optimization;
 * App. "Evaluating Optimized Trajectories" for the ranking).  The IK seeds
 * x_ik are evaluated as given; per problem, those within success_pos /
 * success_rot of the goal and collision free are ranked by
 * pos_err + rot_err + w_dist |q - q_start| (the paper's weighted sum of pose
 * error and distance to the current configuration), ties to the lower
 * index; a problem with none ranks every seed by cost and reports
 * ik_ok = 0.  Trajectory seed i of the problem is the line from q_start to
 * the (i mod count)-th ranked solution: waypoint t = q_start + t/T (q - q_start).
 *   ik_batch: horizon 1 for every problem, at most 1024 seeds each; to_batch:
 *   the same problems (any seeds and horizons)
 *   x_ik DEVICE [ik rows][D]; x_to DEVICE [to rows][D] out; ik_ok DEVICE [P] or NULL.
 * Capturable. */
mg_status mg_ik_seeds(mg_ctx *ctx, mg_batch *ik_batch, mg_batch *to_batch, const float *q_start,
                      const float *goal, const float *x_ik, float w_dist, float *x_to, int *ik_ok,
                      void *stream);

/* Choice among the trajectory seeds of every problem (App. "Evaluating
 * Optimized Trajectories": a blend of pose error, largest jerk and motion
 * time).  The seeds x are evaluated; those that reach the goal within the
 * success tolerances and are collision free score
 *   pos_err + rot_err + w_jerk max|jerk| + w_time T dt_s
 * with dt_s the seed's retimed spacing (mg_retime) and max|jerk| read at it
 * (T dt_s is the motion time: T intervals from the start, waypoint 0, to
 * the last waypoint T);
 * the lowest wins (ties to the lower index).  A problem with no such seed
 * takes its lowest-cost seed and success = 0.
 *   best_seed DEVICE [P]; success, motion_time (T dt_s of the chosen
 *   seed) DEVICE [P] or NULL.  Capturable. */
mg_status mg_traj_select(mg_ctx *ctx, mg_batch *batch, const float *q_start, const float *goal,
                         const float *x, const float *vmax, const float *amax, const float *jmax,
                         float w_jerk, float w_time, int *best_seed, int *success,
                         float *motion_time, void *stream);

/* Motion generation for every problem: mg_solve on ik_batch (iters_ik
 * iterations from the seeds in x_ik), mg_ik_seeds into x_to,
 * mg_solve_timestep on to_batch (iters1, iters2), mg_traj_select.
 * Arguments as in those calls; x_ik and x_to hold the IK and trajectory
 * iterates on return.  The solves launch their kernels directly (each pass
 * runs once with its own parameters).  Not capturable (mg_solve_timestep). */
mg_status mg_motion_gen(mg_ctx *ctx, mg_batch *ik_batch, mg_batch *to_batch, const float *q_start,
                        const float *goal, float *x_ik, float *x_to, int iters_ik, int iters1,
                        int iters2, int m, int K, const float *alpha, int mode, const float *vmax,
                        const float *amax, const float *jmax, float dt_min, float w_dist,
                        float w_jerk, float w_time, int *ik_ok, int *best_seed, int *success,
                        float *motion_time, float *dt_out, void *stream);

/* Parallel steering (Sec. "Parallel Geometric Planner", Alg.3) of n_edges
 * graph edges at once.  Edge e from a = from[e] toward b = to[e] takes
 * n = floor(max_j |b_j - a_j| / res) + 1 steps; its samples
 * a + (i / n)(b - a), i = 0..n, are checked in one launch (joint limits,
 * clearance >= 0 against the batch's world; self-collision is not part of
 * the check).  The edge keeps the last sample before the first that
 * fails: last[e] = that index (n when none fails, -1 when the start fails:
 * reach = a, dist = 0; -2 when n > n_max: not checked, reach = a).
 *   batch: one problem of horizon 1 with n_edges (n_max + 1) seeds (the
 *   sample grid; its workspaces hold the samples)
 *   from, to DEVICE [n_edges][D]; reach DEVICE [n_edges][D];
 *   last DEVICE [n_edges]; dist DEVICE [n_edges] (|reach - a|) or NULL.
 * Capturable. */
mg_status mg_steer(mg_ctx *ctx, mg_batch *batch, int n_edges, const float *from, const float *to,
                   float res, int n_max, float *reach, int *last, float *dist, void *stream);

/* The k nearest graph nodes of every query configuration (the geometric
 * planner's neighbour search, Alg.2), one wavefront per query.  Distances
 * are squared Euclidean joint-space distances summed joint by joint in fp32,
 * each product and sum rounded (no fused multiply-add), so that an fp32
 * brute force reproduces them exactly; ties go to the lower node index.
 *   nodes DEVICE [n_nodes][dof]; queries DEVICE [n_queries][dof]
 *   idx DEVICE [n_queries][k] nearest first (-1 beyond n_nodes)
 *   d2 DEVICE [n_queries][k] their squared distances, or NULL.
 * 1 <= k <= 32.  Capturable. */
mg_status mg_knn(int dof, int n_nodes, const float *nodes, int n_queries, const float *queries, int k,
                 int *idx, float *d2, void *stream);

/* Geometric planning (Sec. "Parallel Geometric Planner", Alg.2) of several
 * start / goal queries in the batch's world on one shared roadmap, every
 * steering step a batched mg_steer launch.  The start and goal of each
 * query, and the (optional) retract configuration with every start and goal,
 * are steer-connected both ways.  While some query has no path, a round
 * picks one unsolved query at random and samples configurations uniformly
 * within the joint limits (after its first failed round, within its informed
 * region |q - start| + |q - goal| <= c_max); the samples in collision are
 * dropped (one horizon-1 evaluation launch per batch-full) and each kept one
 * is steered toward from its k nearest graph nodes (mg_knn on the device; an
 * edge that stops short adds its last valid sample as a node).  A failed
 * round widens the query's c_max by a quarter of its start-goal distance and
 * grows its sample and neighbour counts by a quarter (at most 4x n_samples,
 * 2x k_near).  Once every query has a path, refine_rounds more rounds each
 * pick a query at random and sample inside the ellipsoid bounded by its
 * current path length, so that shorter paths can appear.  Each query's
 * shortest path (Dijkstra) is then shortcut: from each waypoint, the
 * farthest later waypoint reachable directly.  At most max_rounds rounds in
 * all.
 *   batch: one problem of horizon 1 with a multiple of (n_max + 1) seeds
 *   (that multiple is the number of edges per launch)
 *   starts, goals HOST [n_queries][D]; retract HOST [D] or NULL; seed: host
 *   sampler; k_near <= 16
 *   paths HOST [n_queries][max_waypoints][D]; n_waypoints HOST [n_queries]:
 *   waypoints written (0: no path within max_rounds).
 * Not capturable (host graph, synchronises after every launch). */
mg_status mg_plan_batch(mg_ctx *ctx, mg_batch *batch, int n_queries, const float *starts, const float *goals,
                        const float *retract, float res, int n_max, int n_samples, int k_near, int max_rounds,
                        int refine_rounds, unsigned seed, int max_waypoints, float *paths, int *n_waypoints,
                        void *stream);

/* mg_plan_batch of one query with no refine rounds. */
mg_status mg_plan(mg_ctx *ctx, mg_batch *batch, const float *start, const float *goal, const float *retract,
                  float res, int n_max, int n_samples, int k_near, int max_rounds, unsigned seed,
                  int max_waypoints, float *path, int *n_waypoints, void *stream);

/* Measurement hooks.  mg_set_timing(batch, 1) clears the batch's timing
 * record and from then on brackets every direct evaluation-kernel launch
 * made for the batch with a pair of HIP events on the launch stream
 * (launches captured into a graph, and mg_solve's launches that fold in
 * the previous choice, are not timed); 0 turns it off.
 * mg_eval_time waits for the recorded events and returns the mean kernel
 * time in microseconds over the last <= 256 recorded launches and how many
 * that was.  Not capturable. */
mg_status mg_set_timing(mg_batch *batch, int enable);
mg_status mg_eval_time(mg_batch *batch, float *mean_us, int *count);
/* Launch the line-search evaluation kernel (the one mg_linesearch and
 * mg_solve use for these K candidates) `launches` times back to back on
 * stream between two HIP events, wait, and return the mean time per launch
 * in microseconds.  Overwrites the batch's evaluation workspaces.  Not
 * capturable (synchronises). */
mg_status mg_time_eval(mg_ctx *ctx, mg_batch *batch, const float *q_start, const float *goal,
                       const float *x, const float *dir, int K, const float *alpha,
                       int launches, float *mean_us, void *stream);

/* Message for the last non-OK status returned on this thread. */
const char *mg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
