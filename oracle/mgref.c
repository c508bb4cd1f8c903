/* mgref.c -- FP64 CPU reference of the trajectory optimizer's hot path
 * (arXiv 2310.17274).  TEST INFRASTRUCTURE ONLY: loaded by the tests, the
 * smoke check and the CPU-baseline leg of the benchmark, never by the product.
 *
 * Plain, slow and literal on purpose: every quantity is computed from its
 * definition in double precision, with no blocking or fusion.  Readings of
 * passages the paper leaves open are marked "Reading:".
 *
 * Parity unpinned (no value in the paper to check against; pinned only by
 * the written definition and by invariants): the swept trace's stopping
 * rule and its surrogate gradient, and the particle-stage constants
 * (initial variance, temperature, mixing rates).
 */
#include "mgref.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ */
/* Rigid transforms: 3x4 row-major [R | p]; the bottom row 0 0 0 1 is implied. */

static void tf_identity(double *M) {
  memset(M, 0, 12 * sizeof(double));
  M[0] = M[5] = M[10] = 1.0;
}

static void tf_mul(const double *A, const double *B, double *C) {
  double out[12];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 4; ++c) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += A[r * 4 + k] * B[k * 4 + c];
      if (c == 3) s += A[r * 4 + 3];
      out[r * 4 + c] = s;
    }
  memcpy(C, out, sizeof(out));
}

/* Revolute joint about local z (Tab.6, "Revolute Z" joint transformation). */
static void tf_rotz(double th, double *M) {
  tf_identity(M);
  M[0] = cos(th); M[1] = -sin(th);
  M[4] = sin(th); M[5] = cos(th);
}

static void tf_point(const double *M, const double *p, double *out) {
  for (int r = 0; r < 3; ++r)
    out[r] = M[r * 4 + 0] * p[0] + M[r * 4 + 1] * p[1] + M[r * 4 + 2] * p[2] + M[r * 4 + 3];
}

static void cross3(const double *a, const double *b, double *c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

static double dot3(const double *a, const double *b) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

/* Unit quaternion (wxyz, normalised here) -> rotation matrix R[3][3]. */
static void quat_to_mat(const double *q_in, double *R) {
  double n = sqrt(q_in[0] * q_in[0] + q_in[1] * q_in[1] + q_in[2] * q_in[2] + q_in[3] * q_in[3]);
  double w = q_in[0] / n, x = q_in[1] / n, y = q_in[2] / n, z = q_in[3] / n;
  R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
  R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
  R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

/* Shepperd's method: branch on the largest of trace and diagonal. */
void mgref_mat_to_quat(const double *R, double *q) {
  double tr = R[0] + R[4] + R[8];
  if (tr >= R[0] && tr >= R[4] && tr >= R[8]) {
    double w = 0.5 * sqrt(1.0 + tr);
    q[0] = w;
    q[1] = (R[7] - R[5]) / (4 * w);
    q[2] = (R[2] - R[6]) / (4 * w);
    q[3] = (R[3] - R[1]) / (4 * w);
  } else if (R[0] >= R[4] && R[0] >= R[8]) {
    double x = 0.5 * sqrt(1.0 + R[0] - R[4] - R[8]);
    q[1] = x;
    q[0] = (R[7] - R[5]) / (4 * x);
    q[2] = (R[1] + R[3]) / (4 * x);
    q[3] = (R[2] + R[6]) / (4 * x);
  } else if (R[4] >= R[8]) {
    double y = 0.5 * sqrt(1.0 - R[0] + R[4] - R[8]);
    q[2] = y;
    q[0] = (R[2] - R[6]) / (4 * y);
    q[1] = (R[1] + R[3]) / (4 * y);
    q[3] = (R[5] + R[7]) / (4 * y);
  } else {
    double z = 0.5 * sqrt(1.0 - R[0] - R[4] + R[8]);
    q[3] = z;
    q[0] = (R[3] - R[1]) / (4 * z);
    q[1] = (R[2] + R[6]) / (4 * z);
    q[2] = (R[5] + R[7]) / (4 * z);
  }
}

/* ------------------------------------------------------------------ */
/* Kinematics (Sec. 'Robot Kinematics'; Alg.7 computes the same link products). */

void mgref_fk(const mgref_robot *rb, const double *q, double *link_tf,
              double *spheres, double *ee_pose) {
  int L = rb->n_links;
  double *T = (double *)malloc((size_t)L * 12 * sizeof(double));
  for (int l = 0; l < L; ++l) {
    double P[12], J[12], Rz[12];
    if (rb->parent[l] < 0) tf_identity(P);
    else memcpy(P, T + rb->parent[l] * 12, sizeof(P));
    tf_mul(P, rb->fixed_tf + l * 12, J);
    if (rb->joint[l] >= 0) {
      tf_rotz(q[rb->joint[l]], Rz);
      tf_mul(J, Rz, J);
    }
    memcpy(T + l * 12, J, sizeof(J));
  }
  if (link_tf) memcpy(link_tf, T, (size_t)L * 12 * sizeof(double));
  if (spheres)
    for (int m = 0; m < rb->n_spheres; ++m)
      tf_point(T + rb->sphere_link[m] * 12, rb->sphere + m * 4, spheres + m * 3);
  if (ee_pose)
    for (int e = 0; e < rb->n_ee; ++e) {
      double E[12], R[9];
      tf_mul(T + rb->ee_link[e] * 12, rb->ee_tf + e * 12, E);
      for (int r = 0; r < 3; ++r) {
        ee_pose[e * 7 + r] = E[r * 4 + 3];
        for (int c = 0; c < 3; ++c) R[r * 3 + c] = E[r * 4 + c];
      }
      mgref_mat_to_quat(R, ee_pose + e * 7 + 3);
    }
  free(T);
}

/* ------------------------------------------------------------------ */
/* World: exact cuboid signed distance (Sec. 'World Representation', oriented bounding boxes).
 * Reading: the paper asks the world for the closest point and an inside /
 * outside sign; for a cuboid that defines the exact Euclidean signed
 * distance computed here. */

double mgref_box_sdf(const double *pose, const double *dims, const double *c,
                     double *grad) {
  double R[9], d[3], p[3], a[3], h[3];
  quat_to_mat(pose + 3, R);
  for (int i = 0; i < 3; ++i) d[i] = c[i] - pose[i];
  for (int i = 0; i < 3; ++i) p[i] = R[0 * 3 + i] * d[0] + R[1 * 3 + i] * d[1] + R[2 * 3 + i] * d[2];
  for (int i = 0; i < 3; ++i) {
    h[i] = 0.5 * dims[i];
    a[i] = fabs(p[i]) - h[i];
  }
  double out2 = 0.0;
  for (int i = 0; i < 3; ++i) out2 += a[i] > 0 ? a[i] * a[i] : 0.0;
  double outside = sqrt(out2);
  int imax = 0;
  for (int i = 1; i < 3; ++i) if (a[i] > a[imax]) imax = i;
  double inside = a[imax] < 0 ? a[imax] : 0.0;
  double sdf = outside + inside;
  if (grad) {
    double gp[3] = {0, 0, 0};
    if (outside > 0) {
      for (int i = 0; i < 3; ++i)
        gp[i] = (a[i] > 0 ? a[i] : 0.0) / outside * (p[i] >= 0 ? 1.0 : -1.0);
    } else {
      gp[imax] = p[imax] >= 0 ? 1.0 : -1.0;
    }
    for (int r = 0; r < 3; ++r) grad[r] = R[r * 3 + 0] * gp[0] + R[r * 3 + 1] * gp[1] + R[r * 3 + 2] * gp[2];
  }
  return sdf;
}

/* Eq.(10): linear in penetration beyond contact, quadratic within eta. */
double mgref_dc(double d, double eta, double *slope) {
  if (d > 0) { if (slope) *slope = 1.0; return d + 0.5 * eta; }
  if (d > -eta) { if (slope) *slope = (d + eta) / eta; return 0.5 / eta * (d + eta) * (d + eta); }
  if (slope) *slope = 0.0;
  return 0.0;
}

/* Eq.(17).  Reading: the lower and upper bands are separate terms and are
 * summed when they overlap. */
double mgref_bound(double x, double lo, double hi, double eta2, double *slope) {
  double c = 0.0, s = 0.0;
  if (x < lo) { c += lo - x + 0.5 * eta2; s += -1.0; }
  else if (x < lo + eta2) { double u = lo - x + eta2; c += 0.5 / eta2 * u * u; s += -u / eta2; }
  if (x > hi) { c += x - hi + 0.5 * eta2; s += 1.0; }
  else if (x > hi - eta2) { double u = x - hi + eta2; c += 0.5 / eta2 * u * u; s += u / eta2; }
  if (slope) *slope = s;
  return c;
}

/* Stable log(cosh(x)). */
static double logcosh(double x) {
  double ax = fabs(x);
  return ax + log1p(exp(-2.0 * ax)) - log(2.0);
}

/* tanh(k r) / r, with its limit k at r = 0. */
static double tanh_over(double k, double r) {
  return r > 0 ? tanh(k * r) / r : k;
}

/* ------------------------------------------------------------------ */
/* Time derivatives (appendix 'Finite Difference for State Derivatives'): five-point stencils on the padded trajectory
 * X(-2) = X(-1) = X(0) = q0, X(t) = q(t) for t = 1..T, X(T+1) = X(T+2) = q(T).
 * Reading: Tab.1's last row makes the first and last three states equal; the
 * stencil half-width 2 needs exactly those copies.  Coefficients are the
 * textbook central five-point formulas (Fornberg). */

static double padded(int T, int D, const double *q0, const double *q, int tau, int d) {
  if (tau <= 0) return q0[d];
  if (tau >= T) return q[(T - 1) * D + d];
  return q[(tau - 1) * D + d];
}

void mgref_derivatives(int T, int D, const double *q0, const double *q,
                       double dt, double *v, double *a, double *j) {
  double h = dt;
  for (int tau = 0; tau <= T; ++tau)
    for (int d = 0; d < D; ++d) {
      double xm2 = padded(T, D, q0, q, tau - 2, d), xm1 = padded(T, D, q0, q, tau - 1, d);
      double x0 = padded(T, D, q0, q, tau, d);
      double xp1 = padded(T, D, q0, q, tau + 1, d), xp2 = padded(T, D, q0, q, tau + 2, d);
      if (v) v[tau * D + d] = (xm2 - 8 * xm1 + 8 * xp1 - xp2) / (12 * h);
      if (a) a[tau * D + d] = (-xm2 + 16 * xm1 - 30 * x0 + 16 * xp1 - xp2) / (12 * h * h);
      if (j) j[tau * D + d] = (-xm2 + 2 * xm1 - 2 * xp1 + xp2) / (2 * h * h * h);
    }
}

/* Retiming (Alg.4, appendix 'Time-step Descretization and Temporal Weight
 * Scaling'): the waypoint spacing at which the trajectory's largest
 * velocity, acceleration or jerk reaches the robot's limit.  The stencil
 * derivatives of order k scale as dt^-k, so re-spacing the same waypoints
 * at dt' gives |v| dt / dt', |a| (dt / dt')^2, |j| (dt / dt')^3; each meets
 * its limit at dt' = dt |v| / vmax, dt sqrt(|a| / amax), dt cbrt(|j| / jmax).
 * The result is the largest of these over t = 0..T and every joint (the
 * first limit reached as dt' shrinks).  A limit <= 0 leaves its kind out. */
double mgref_retime(int T, int D, const double *q0, const double *q, double dt,
                    const double *vmax, const double *amax, const double *jmax) {
  double *v = (double *)malloc(sizeof(double) * (size_t)(T + 1) * D * 3);
  double *a = v + (size_t)(T + 1) * D, *j = a + (size_t)(T + 1) * D;
  mgref_derivatives(T, D, q0, q, dt, v, a, j);
  double r = 0.0;
  for (int tau = 0; tau <= T; ++tau)
    for (int d = 0; d < D; ++d) {
      const size_t i = (size_t)tau * D + d;
      if (vmax[d] > 0) r = fmax(r, fabs(v[i]) / vmax[d]);
      if (amax[d] > 0) r = fmax(r, sqrt(fabs(a[i]) / amax[d]));
      if (jmax[d] > 0) r = fmax(r, cbrt(fabs(j[i]) / jmax[d]));
    }
  free(v);
  return dt * r;
}

/* Eq.(16): alpha6 * sum_{t in Q} logcosh(alpha7 v_t) + sum_{t=0..T}
 * (alpha8 |a_t|^2 + alpha9 |j_t|^2).  Reading: Q is not defined in the
 * paper; Q = {T} (stop at the goal, Eq.(6)) unless vel_all is set. */
static double smooth_cost(const mgref_params *pr, int D, int T, const double *q0,
                          const double *q, double *grad) {
  int n = (T + 1) * D;
  double *v = (double *)malloc(3 * (size_t)n * sizeof(double));
  double *a = v + n, *jk = v + 2 * n;
  mgref_derivatives(T, D, q0, q, pr->dt, v, a, jk);
  double h = pr->dt, cv = 1.0 / (12 * h), ca = 1.0 / (12 * h * h), cj = 1.0 / (2 * h * h * h);
  /* dC/dX for X(tau), tau = -2..T+2 stored at index tau + 2 */
  double *dX = (double *)calloc((size_t)(T + 5) * D, sizeof(double));
  double cost = 0.0;
  for (int tau = 0; tau <= T; ++tau)
    for (int d = 0; d < D; ++d) {
      double vv = v[tau * D + d], aa = a[tau * D + d], jj = jk[tau * D + d];
      double gv = 0.0;
      if (tau == T || pr->vel_all) {
        cost += pr->a6 * logcosh(pr->a7 * vv);
        gv = pr->a6 * pr->a7 * tanh(pr->a7 * vv);
      }
      cost += pr->a8 * aa * aa + pr->a9 * jj * jj;
      double ga = 2 * pr->a8 * aa, gj = 2 * pr->a9 * jj;
      int i = tau + 2;
      dX[(i - 2) * D + d] += gv * cv * 1 + ga * ca * -1 + gj * cj * -1;
      dX[(i - 1) * D + d] += gv * cv * -8 + ga * ca * 16 + gj * cj * 2;
      dX[(i + 0) * D + d] += ga * ca * -30;
      dX[(i + 1) * D + d] += gv * cv * 8 + ga * ca * 16 + gj * cj * -2;
      dX[(i + 2) * D + d] += gv * cv * -1 + ga * ca * -1 + gj * cj * 1;
    }
  if (grad) {
    /* X(t) = q(t) for t = 1..T; the two pad copies after T are q(T) too;
     * the start copies are constant and drop out. */
    for (int t = 1; t <= T; ++t)
      for (int d = 0; d < D; ++d) grad[(t - 1) * D + d] += dX[(t + 2) * D + d];
    for (int d = 0; d < D; ++d)
      grad[(T - 1) * D + d] += dX[(T + 3) * D + d] + dX[(T + 4) * D + d];
  }
  free(dX);
  free(v);
  return cost;
}

/* ------------------------------------------------------------------ */
/* Pose reaching cost, Eq.(14).  Reading: the printed orientation term puts
 * q_g^T q_T inside logcosh, which is largest at the goal; the distance used
 * here is d = |q_g - s q_T| with s = sign(<q_g, q_T>) (s = +1 at 0), which
 * is zero at the goal and blind to the quaternion sign. */
static double pose_cost(const mgref_params *pr, const double *ee, const double *goal,
                        double *g_pos, double *g_quat) {
  double e[3], n2 = 0.0;
  for (int i = 0; i < 3; ++i) { e[i] = goal[i] - ee[i]; n2 += e[i] * e[i]; }
  double n = sqrt(n2);
  double c = pr->a0 * logcosh(pr->a2 * n);
  double f = pr->a0 * pr->a2 * tanh_over(pr->a2, n);
  for (int i = 0; i < 3; ++i) g_pos[i] = -f * e[i];
  const double *qg = goal + 3, *qt = ee + 3;
  double dqv = qg[0] * qt[0] + qg[1] * qt[1] + qg[2] * qt[2] + qg[3] * qt[3];
  double s = dqv >= 0 ? 1.0 : -1.0;
  double eq[4], r2 = 0.0;
  for (int i = 0; i < 4; ++i) { eq[i] = qg[i] - s * qt[i]; r2 += eq[i] * eq[i]; }
  double r = sqrt(r2);
  c += pr->a1 * logcosh(pr->a3 * r);
  double fr = pr->a1 * pr->a3 * tanh_over(pr->a3, r);
  for (int i = 0; i < 4; ++i) g_quat[i] = -s * fr * eq[i];
  return c;
}

void mgref_pose_error(const mgref_robot *rb, const double *qT, const double *goal,
                      double *pos_err, double *rot_err) {
  double *ee = (double *)malloc((size_t)rb->n_ee * 7 * sizeof(double));
  mgref_fk(rb, qT, NULL, NULL, ee);
  for (int e = 0; e < rb->n_ee; ++e) {
    const double *p = ee + e * 7, *g = goal + e * 7;
    double d2 = 0.0;
    for (int i = 0; i < 3; ++i) d2 += (g[i] - p[i]) * (g[i] - p[i]);
    pos_err[e] = sqrt(d2);
    double w = fabs(g[3] * p[3] + g[4] * p[4] + g[5] * p[5] + g[6] * p[6]);
    rot_err[e] = 2.0 * acos(w < 1.0 ? w : 1.0);
  }
  free(ee);
}

/* ------------------------------------------------------------------ */
/* One sphere against one cuboid, with the continuous sweep when enabled.
 * Returns the cost, accumulates d cost / d center into gc.
 *
 * Continuous collision (Sec. 'Continuous Collision Checking', Alg.11-12).  Reading: starting from the
 * waypoint, sphere tracing moves along the segment toward each neighbour by
 * the clearance (or by the inflated radius when the sphere is within the
 * band), costing every sample, until the half-way point; the samples'
 * gradients are attributed to this waypoint's sphere, as the paper does. */
static double sphere_box(const mgref_params *pr, const double *pose, const double *dims,
                         const double *c, double r, const double *prev, const double *next,
                         double *gc, double *mc) {
  double g[3];
  double sdf = mgref_box_sdf(pose, dims, c, g);
  if (sdf - r < *mc) *mc = sdf - r;
  double slope;
  double cost = pr->w_coll * mgref_dc(r - sdf, pr->eta, &slope);
  for (int i = 0; i < 3; ++i) gc[i] += -pr->w_coll * slope * g[i];
  if (!pr->swept) return cost;
  const double rho = r + pr->eta;
  const double *nb[2] = {prev, next};
  for (int side = 0; side < 2; ++side) {
    if (!nb[side]) continue;
    double u[3], len = 0.0;
    for (int i = 0; i < 3; ++i) { u[i] = nb[side][i] - c[i]; len += u[i] * u[i]; }
    len = sqrt(len);
    if (len <= 0) continue;
    for (int i = 0; i < 3; ++i) u[i] /= len;
    double j = sdf < rho ? rho : sdf - rho;
    for (int step = 0; step < pr->sweep_steps && j < 0.5 * len; ++step) {
      double p[3], gs[3];
      for (int i = 0; i < 3; ++i) p[i] = c[i] + j * u[i];
      double s2 = mgref_box_sdf(pose, dims, p, gs);
      double sl;
      cost += pr->w_coll * mgref_dc(r - s2, pr->eta, &sl);
      for (int i = 0; i < 3; ++i) gc[i] += -pr->w_coll * sl * gs[i];
      j += (s2 - rho > 0) ? s2 - rho : rho;
    }
  }
  return cost;
}

/* ------------------------------------------------------------------ */

/* Adds d cost / d q of a gradient g acting at world point c on link `link`:
 * Tab.7 revolute z, d c / d q_j = z_j x (c - o_j) for every joint on the
 * chain from the link to the base. */
static void project_point(const mgref_robot *rb, const double *T_t, int link, const double *c,
                          const double *g, double *gt) {
  for (int l = link; l >= 0; l = rb->parent[l]) {
    int j = rb->joint[l];
    if (j < 0) continue;
    const double *Tl = T_t + l * 12;
    double z[3] = {Tl[2], Tl[6], Tl[10]}, o[3] = {Tl[3], Tl[7], Tl[11]};
    double rel[3], dc[3];
    for (int i = 0; i < 3; ++i) rel[i] = c[i] - o[i];
    cross3(z, rel, dc);
    gt[j] += dot3(g, dc);
  }
}

/* Self-collision at one waypoint, Eq.(9): beta_1 times the largest
 * penetration r_i + r_j - |x_i - x_j| over the checked pairs (0 if none
 * overlaps); the gradient acts on the two spheres of the first pair reaching
 * the maximum. */
static double self_collision(const mgref_robot *rb, const mgref_params *pr, const double *T_t,
                             const double *sp, double *gt) {
  if (pr->n_self <= 0 || !pr->self_pairs) return 0.0;
  double best = 0.0;
  int bk = -1;
  for (int k = 0; k < pr->n_self; ++k) {
    const int i = pr->self_pairs[2 * k], j = pr->self_pairs[2 * k + 1];
    double d2 = 0.0;
    for (int a = 0; a < 3; ++a) d2 += (sp[i * 3 + a] - sp[j * 3 + a]) * (sp[i * 3 + a] - sp[j * 3 + a]);
    const double pen = rb->sphere[i * 4 + 3] + rb->sphere[j * 4 + 3] - sqrt(d2);
    if (pen > best) { best = pen; bk = k; }
  }
  if (gt && bk >= 0) {
    const int i = pr->self_pairs[2 * bk], j = pr->self_pairs[2 * bk + 1];
    double u[3], d2 = 0.0;
    for (int a = 0; a < 3; ++a) { u[a] = sp[i * 3 + a] - sp[j * 3 + a]; d2 += u[a] * u[a]; }
    const double d = sqrt(d2);
    if (d > 0.0) {
      double gi[3], gj[3];
      for (int a = 0; a < 3; ++a) { gi[a] = -pr->w_self * u[a] / d; gj[a] = -gi[a]; }
      project_point(rb, T_t, rb->sphere_link[i], sp + i * 3, gi, gt);
      project_point(rb, T_t, rb->sphere_link[j], sp + j * 3, gj, gt);
    }
  }
  return pr->w_self * best;
}

double mgref_traj_cost(const mgref_robot *rb, const mgref_params *pr,
                       int n_box, const double *box_pose, const double *box_dims,
                       const double *q0, const double *goal, int T,
                       const double *q, double *grad, double *min_clear,
                       double *terms) {
  const int D = rb->dof, L = rb->n_links, M = rb->n_spheres, E = rb->n_ee;
  double c_smooth = 0.0, c_bound = 0.0, c_coll = 0.0, c_pose = 0.0, c_self = 0.0;
  double mc = pr->eta;
  if (grad) memset(grad, 0, (size_t)T * D * sizeof(double));
  if (T > 1) c_smooth = smooth_cost(pr, D, T, q0, q, grad);

  /* kinematics of every waypoint; slot 0 holds the start (swept neighbour) */
  double *tf = (double *)malloc((size_t)(T + 1) * L * 12 * sizeof(double));
  double *sp = (double *)malloc((size_t)(T + 1) * M * 3 * sizeof(double));
  double *ee = (double *)malloc((size_t)(T + 1) * (E > 0 ? E : 1) * 7 * sizeof(double));
  if (T > 1 || pr->speed) mgref_fk(rb, q0, tf, sp, ee);
  for (int t = 1; t <= T; ++t)
    mgref_fk(rb, q + (t - 1) * D, tf + t * L * 12, sp + t * M * 3, ee + t * E * 7);

  for (int t = 1; t <= T; ++t) {
    const double *qt = q + (t - 1) * D;
    double *gt = grad ? grad + (t - 1) * D : NULL;
    const double *T_t = tf + t * L * 12;
    /* joint-limit cost, Eq.(17), weight 5000 like every soft constraint */
    for (int d = 0; d < D; ++d) {
      double s;
      c_bound += pr->w_bound * mgref_bound(qt[d], rb->q_lo[d], rb->q_hi[d], pr->eta2, &s);
      if (gt) gt[d] += pr->w_bound * s;
    }
    /* world collision, Eq.(11); summed over cuboids (Alg.10 accumulates
     * every cuboid) and spheres.  The speed factor (Sec. 'Speeding through
     * obstacles'), when on, scales the sphere's collision cost by the
     * sphere's speed from the central difference of its neighbouring
     * positions, |c(t+1) - c(t-1)| / (2 dt), on the padded trajectory (the
     * start before waypoint 1, waypoint T repeated after it).  The gradient
     * is the derivative of that product: the speed times the collision
     * gradient at c(t), plus the collision cost times the speed's gradient,
     * which acts on the two neighbouring positions (the unit chord / (2 dt)
     * on c(t+1), or on c(t) itself at t = T, and its negative on c(t-1),
     * none on the constant start). */
    for (int m = 0; m < M; ++m) {
      const double *c = sp + (t * M + m) * 3;
      double r = rb->sphere[m * 4 + 3];
      const double *prev = (pr->swept && T > 1) ? sp + ((t - 1) * M + m) * 3 : NULL;
      const double *next = (pr->swept && T > 1 && t < T) ? sp + ((t + 1) * M + m) * 3 : NULL;
      double gc[3] = {0, 0, 0};
      double cm = 0.0;
      for (int k = 0; k < n_box; ++k)
        cm += sphere_box(pr, box_pose + k * 7, box_dims + k * 3, c, r, prev, next, gc, &mc);
      if (pr->speed) {
        const double *cp = sp + ((t - 1) * M + m) * 3, *cn = t < T ? sp + ((t + 1) * M + m) * 3 : c;
        double u[3] = {cn[0] - cp[0], cn[1] - cp[1], cn[2] - cp[2]};
        const double un = sqrt(dot3(u, u));
        const double speed = un / (2.0 * pr->dt);
        if (grad && cm != 0.0 && un > 0.0) {
          /* d speed / d cn = u / (|u| 2 dt), d speed / d cp = -u / (|u| 2 dt) */
          double gs[3];
          for (int i = 0; i < 3; ++i) gs[i] = cm * u[i] / (un * 2.0 * pr->dt);
          const int tn = t < T ? t + 1 : t;
          project_point(rb, tf + tn * L * 12, rb->sphere_link[m], cn, gs, grad + (tn - 1) * D);
          if (t >= 2) {
            for (int i = 0; i < 3; ++i) gs[i] = -gs[i];
            project_point(rb, tf + (t - 1) * L * 12, rb->sphere_link[m], cp, gs, grad + (t - 2) * D);
          }
        }
        cm *= speed;
        for (int i = 0; i < 3; ++i) gc[i] *= speed;
      }
      c_coll += cm;
      if (gt && (gc[0] != 0 || gc[1] != 0 || gc[2] != 0)) {
        /* Tab.7 revolute-z: d c / d q_j = z_j x (c - o_j) for every joint on
         * the chain from the sphere's link to the base */
        for (int l = rb->sphere_link[m]; l >= 0; l = rb->parent[l]) {
          int j = rb->joint[l];
          if (j < 0) continue;
          const double *Tl = T_t + l * 12;
          double z[3] = {Tl[2], Tl[6], Tl[10]}, o[3] = {Tl[3], Tl[7], Tl[11]};
          double rel[3], dc[3];
          for (int i = 0; i < 3; ++i) rel[i] = c[i] - o[i];
          cross3(z, rel, dc);
          gt[j] += dot3(gc, dc);
        }
      }
    }
    /* self-collision, Eq.(9) */
    c_self += self_collision(rb, pr, T_t, sp + t * M * 3, gt);
    /* pose reaching cost at the last waypoint */
    if (t == T)
      for (int e = 0; e < E; ++e) {
        const double *pe = ee + (t * E + e) * 7;
        double gp[3], gq[4];
        c_pose += pose_cost(pr, pe, goal + e * 7, gp, gq);
        if (!gt) continue;
        for (int l = rb->ee_link[e]; l >= 0; l = rb->parent[l]) {
          int j = rb->joint[l];
          if (j < 0) continue;
          const double *Tl = T_t + l * 12;
          double z[3] = {Tl[2], Tl[6], Tl[10]}, o[3] = {Tl[3], Tl[7], Tl[11]};
          double rel[3], dp[3];
          for (int i = 0; i < 3; ++i) rel[i] = pe[i] - o[i];
          cross3(z, rel, dp);
          /* orientation rate: d quat = 1/2 (0, z) (x) quat */
          const double *qt4 = pe + 3;
          double zxv[3];
          cross3(z, qt4 + 1, zxv);
          double dq[4] = {-0.5 * dot3(z, qt4 + 1),
                          0.5 * (qt4[0] * z[0] + zxv[0]),
                          0.5 * (qt4[0] * z[1] + zxv[1]),
                          0.5 * (qt4[0] * z[2] + zxv[2])};
          gt[j] += dot3(gp, dp) + gq[0] * dq[0] + gq[1] * dq[1] + gq[2] * dq[2] + gq[3] * dq[3];
        }
      }
  }
  free(tf);
  free(sp);
  free(ee);
  if (min_clear) *min_clear = mc;
  if (terms) {
    terms[0] = c_smooth; terms[1] = c_bound; terms[2] = c_coll; terms[3] = c_pose; terms[4] = c_self;
  }
  return c_smooth + c_bound + c_coll + c_pose + c_self;
}

void mgref_cost_grad_batch(const mgref_robot *rb, const mgref_params *pr,
                           int n_box, const double *box_pose, const double *box_dims,
                           const double *q0, const double *goal, int T, int S,
                           const double *q, double *cost, double *grad,
                           double *min_clear, int nthreads) {
  const int n = T * rb->dof;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads > 0 ? nthreads : 1)
#endif
  for (int s = 0; s < S; ++s) {
    double mc;
    cost[s] = mgref_traj_cost(rb, pr, n_box, box_pose, box_dims, q0, goal, T, q + (size_t)s * n,
                              grad ? grad + (size_t)s * n : NULL, &mc, NULL);
    if (min_clear) min_clear[s] = mc;
  }
  (void)nthreads;
}

/* ------------------------------------------------------------------ */
/* L-BFGS direction (Alg.6, the two-loop recursion of Nocedal & Wright).
 * Readings: (1) a pair enters the history only when <y,s> > 1e-10 |s||y|,
 * since a noisy step can give <y,s> <= 0 and a negative rho would make an
 * ascent direction; (2) H0 = gamma I with gamma = <s,y>/<y,y> of the newest
 * pair (N&W eq. 7.20), and gamma = min(1, 0.1 / |g|_inf) with no pair;
 * (3) the returned direction is -H g (Alg.1 adds alpha * direction). */
void mgref_lbfgs_step(int n, int m, int reset, int *count, int *head,
                      double *S, double *Y, double *rho, double *x_prev,
                      double *g_prev, const double *x, const double *g,
                      double *dir) {
  if (reset) { *count = 0; *head = 0; }
  else if (m > 0) {
    double *s = S + (size_t)(*head) * n, *y = Y + (size_t)(*head) * n;
    double sy = 0.0, ss = 0.0, yy = 0.0;
    for (int i = 0; i < n; ++i) {
      double si = x[i] - x_prev[i], yi = g[i] - g_prev[i];
      sy += si * yi; ss += si * si; yy += yi * yi;
    }
    if (sy > 1e-10 * sqrt(ss) * sqrt(yy) && sy > 0) {
      for (int i = 0; i < n; ++i) { s[i] = x[i] - x_prev[i]; y[i] = g[i] - g_prev[i]; }
      rho[*head] = 1.0 / sy;
      *head = (*head + 1) % m;
      if (*count < m) *count += 1;
    }
  }
  double *qv = (double *)malloc((size_t)n * sizeof(double));
  double *al = (double *)malloc((size_t)(m > 0 ? m : 1) * sizeof(double));
  memcpy(qv, g, (size_t)n * sizeof(double));
  for (int k = 0; k < *count; ++k) {              /* newest -> oldest */
    int i = ((*head - 1 - k) % m + m) % m;
    double a = 0.0;
    for (int e = 0; e < n; ++e) a += S[(size_t)i * n + e] * qv[e];
    a *= rho[i];
    al[i] = a;
    for (int e = 0; e < n; ++e) qv[e] -= a * Y[(size_t)i * n + e];
  }
  double gamma;
  if (*count > 0) {
    int i = ((*head - 1) % m + m) % m;
    double sy = 0.0, yy = 0.0;
    for (int e = 0; e < n; ++e) { sy += S[(size_t)i * n + e] * Y[(size_t)i * n + e]; yy += Y[(size_t)i * n + e] * Y[(size_t)i * n + e]; }
    gamma = sy / yy;
  } else {
    double gi = 0.0;
    for (int e = 0; e < n; ++e) if (fabs(g[e]) > gi) gi = fabs(g[e]);
    gamma = gi > 0 ? fmin(1.0, 0.1 / gi) : 1.0;
  }
  for (int e = 0; e < n; ++e) qv[e] *= gamma;
  for (int k = *count - 1; k >= 0; --k) {         /* oldest -> newest */
    int i = ((*head - 1 - k) % m + m) % m;
    double b = 0.0;
    for (int e = 0; e < n; ++e) b += Y[(size_t)i * n + e] * qv[e];
    b *= rho[i];
    for (int e = 0; e < n; ++e) qv[e] += S[(size_t)i * n + e] * (al[i] - b);
  }
  for (int e = 0; e < n; ++e) dir[e] = -qv[e];
  memcpy(x_prev, x, (size_t)n * sizeof(double));
  memcpy(g_prev, g, (size_t)n * sizeof(double));
  free(qv);
  free(al);
}

/* Alg.1 selection.  Reading: the printed Armijo test omits the inner product;
 * it is c_k <= c_0 + eta1 alpha_k <g_0, d>; weak Wolfe <g_k,d> >= eta_w <g_0,d>,
 * strong Wolfe |<g_k,d>| <= eta_w |<g_0,d>| (Nocedal & Wright eq. 3.6-3.7). */
int mgref_ls_select(int K, const double *alpha, double c0, double g0d,
                    const double *c, const double *gd, int mode, double eta1,
                    double eta_w) {
  int best = 0;
  for (int k = 0; k < K; ++k) {
    int ok = c[k] <= c0 + eta1 * alpha[k] * g0d;
    if (mode == 1) ok = ok && (gd[k] >= eta_w * g0d);
    if (mode == 2) ok = ok && (fabs(gd[k]) <= eta_w * fabs(g0d));
    if (ok) best = k;
  }
  return best;
}

int mgref_linesearch(const mgref_robot *rb, const mgref_params *pr,
                     int n_box, const double *box_pose, const double *box_dims,
                     const double *q0, const double *goal, int T,
                     const double *x, double c0, const double *g0, const double *dir,
                     int K, const double *alpha, int mode, double eta1, double eta_w,
                     double *x_out, double *c_out, double *g_out, double *mc_out) {
  const int D = rb->dof, n = T * D;
  double *xs = (double *)malloc((size_t)K * n * sizeof(double));
  double *gs = (double *)malloc((size_t)K * n * sizeof(double));
  double *cs = (double *)malloc((size_t)K * sizeof(double));
  double *gd = (double *)malloc((size_t)K * sizeof(double));
  double *mcs = (double *)malloc((size_t)K * sizeof(double));
  double g0d = 0.0;
  for (int e = 0; e < n; ++e) g0d += g0[e] * dir[e];
  for (int k = 0; k < K; ++k) {
    double *xk = xs + (size_t)k * n;
    for (int e = 0; e < n; ++e) {                 /* bounded variables */
      double v = x[e] + alpha[k] * dir[e];
      int d = e % D;
      if (v < rb->q_lo[d]) v = rb->q_lo[d];
      if (v > rb->q_hi[d]) v = rb->q_hi[d];
      xk[e] = v;
    }
    cs[k] = mgref_traj_cost(rb, pr, n_box, box_pose, box_dims, q0, goal, T, xk,
                            gs + (size_t)k * n, mcs + k, NULL);
    gd[k] = 0.0;
    for (int e = 0; e < n; ++e) gd[k] += gs[(size_t)k * n + e] * dir[e];
  }
  int i = mgref_ls_select(K, alpha, c0, g0d, cs, gd, mode, eta1, eta_w);
  memcpy(x_out, xs + (size_t)i * n, (size_t)n * sizeof(double));
  memcpy(g_out, gs + (size_t)i * n, (size_t)n * sizeof(double));
  *c_out = cs[i];
  if (mc_out) *mc_out = mcs[i];
  free(xs); free(gs); free(cs); free(gd); free(mcs);
  return i;
}

/* Sec. 'Parallel L-BFGS Optimization': L-BFGS direction, noisy line search and best-iterate tracking
 * (strictly lower cost replaces the best) for every seed independently. */
void mgref_solve(const mgref_robot *rb, const mgref_params *pr,
                 int n_box, const double *box_pose, const double *box_dims,
                 const double *q0, const double *goal, int T, int S, double *x,
                 int iters, int m, int K, const double *alpha, int mode,
                 double eta1, double eta_w, double *best_cost, double *trace,
                 int nthreads) {
  const int n = T * rb->dof;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads > 0 ? nthreads : 1)
#endif
  for (int s = 0; s < S; ++s) {
    int mm = m > 0 ? m : 1;
    double *buf = (double *)calloc((size_t)(2 * mm + 8) * n + mm, sizeof(double));
    double *Sh = buf, *Yh = Sh + (size_t)mm * n, *xp = Yh + (size_t)mm * n, *gp = xp + n;
    double *xc = gp + n, *gc = xc + n, *dir = gc + n, *xn = dir + n, *best = xn + n;
    double *gn = best + n, *rho = gn + n;
    int count = 0, head = 0;
    memcpy(xc, x + (size_t)s * n, (size_t)n * sizeof(double));
    double c = mgref_traj_cost(rb, pr, n_box, box_pose, box_dims, q0, goal, T, xc, gc, NULL, NULL);
    double bc = c;
    memcpy(best, xc, (size_t)n * sizeof(double));
    for (int it = 0; it < iters; ++it) {
      mgref_lbfgs_step(n, m, it == 0, &count, &head, Sh, Yh, rho, xp, gp, xc, gc, dir);
      double cn;
      mgref_linesearch(rb, pr, n_box, box_pose, box_dims, q0, goal, T, xc, c, gc, dir,
                       K, alpha, mode, eta1, eta_w, xn, &cn, gn, NULL);
      memcpy(xc, xn, (size_t)n * sizeof(double));
      memcpy(gc, gn, (size_t)n * sizeof(double));
      c = cn;
      if (c < bc) { bc = c; memcpy(best, xc, (size_t)n * sizeof(double)); }
      if (trace) trace[(size_t)it * S + s] = bc;
    }
    memcpy(x + (size_t)s * n, best, (size_t)n * sizeof(double));
    best_cost[s] = bc;
    free(buf);
  }
  (void)nthreads;
}

/* ------------------------------------------------------------------ */
/* Particle-based optimization (Alg.5, Eq.(12)-(13)). */

void mgref_particle_update(int n, int N, const double *cost, const double *theta,
                           double *mu, double *var, double beta, double k_mu,
                           double k_sigma, double *w_out) {
  double cmin = cost[0], cmax = cost[0];
  for (int i = 1; i < N; ++i) {
    if (cost[i] < cmin) cmin = cost[i];
    if (cost[i] > cmax) cmax = cost[i];
  }
  if (beta <= 0) beta = 0.1 * (cmax - cmin) + 1e-12;
  double *w = (double *)malloc((size_t)N * sizeof(double));
  double z = 0.0;
  for (int i = 0; i < N; ++i) {
    w[i] = exp(-(cost[i] - cmin) / beta);
    z += w[i];
  }
  for (int i = 0; i < N; ++i) w[i] /= z;
  for (int e = 0; e < n; ++e) {
    double m1 = 0.0, m2 = 0.0;
    for (int i = 0; i < N; ++i) {
      const double th = theta[(size_t)i * n + e];
      m1 += w[i] * th;
      m2 += w[i] * (th - mu[e]) * (th - mu[e]);
    }
    var[e] = (1.0 - k_sigma) * var[e] + k_sigma * m2;
    mu[e] = (1.0 - k_mu) * mu[e] + k_mu * m1;
  }
  if (w_out) memcpy(w_out, w, (size_t)N * sizeof(double));
  free(w);
}

void mgref_particles(const mgref_robot *rb, const mgref_params *pr,
                     int n_box, const double *box_pose, const double *box_dims,
                     const double *q0, const double *goal, int T, int S, double *mu,
                     double *var, int N, int n_iters, const double *eps, double beta,
                     double k_mu, double k_sigma, double *cost_out, int nthreads) {
  const int D = rb->dof, n = T * D;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads > 0 ? nthreads : 1)
#endif
  for (int s = 0; s < S; ++s) {
    double *theta = (double *)malloc((size_t)N * n * sizeof(double));
    double *c = (double *)malloc((size_t)N * sizeof(double));
    double *m = mu + (size_t)s * n, *v = var + (size_t)s * n;
    for (int it = 0; it < n_iters; ++it) {
      for (int i = 0; i < N; ++i) {
        const double *z = eps + (((size_t)it * N + i) * S + s) * n;
        double *th = theta + (size_t)i * n;
        for (int e = 0; e < n; ++e) {
          const int d = e % D;
          double x = m[e] + sqrt(v[e]) * z[e];
          th[e] = x < rb->q_lo[d] ? rb->q_lo[d] : (x > rb->q_hi[d] ? rb->q_hi[d] : x);
        }
        c[i] = mgref_traj_cost(rb, pr, n_box, box_pose, box_dims, q0, goal, T, th, NULL, NULL, NULL);
        if (cost_out) cost_out[((size_t)it * S + s) * N + i] = c[i];
      }
      mgref_particle_update(n, N, c, theta, m, v, beta, k_mu, k_sigma, NULL);
    }
    free(theta);
    free(c);
  }
  (void)nthreads;
}

/* ------------------------------------------------------------------ */
/* Philox-4x64-10 (Salmon et al., SC'11): ten rounds of the S-box that
 * multiplies counter words 0 and 2 by the two round multipliers (high and
 * low 64-bit halves of the 128-bit products), mixes in the key and swaps the
 * words; the key is bumped by the two Weyl constants between rounds. */
static void mul64(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo) {
  const unsigned __int128 p = (unsigned __int128)a * b;
  *hi = (uint64_t)(p >> 64);
  *lo = (uint64_t)p;
}

void mgref_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
  const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
  uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3], k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    uint64_t hi0, lo0, hi1, lo1;
    mul64(c0, M0, &hi0, &lo0);
    mul64(c2, M1, &hi1, &lo1);
    const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    k0 += W0;
    k1 += W1;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

double mgref_philox_normal(uint64_t seed, int it, int k, int64_t e) {
  const uint64_t ctr[4] = {(uint64_t)(e >> 2), (uint64_t)(uint32_t)k, (uint64_t)(uint32_t)it, 0};
  const uint64_t key[2] = {seed, 0};
  uint64_t w[4];
  mgref_philox4x64(ctr, key, w);
  const uint64_t x = w[e & 3];
  const double u1 = ((double)(x >> 41) + 0.5) / 8388608.0;
  const double u2 = ((double)((x >> 9) & 0x7FFFFFULL) + 0.5) / 8388608.0;
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586476925287 * u2);   /* 2 pi */
}

void mgref_philox_normals(uint64_t seed, int n_iters, int N, int rows, int D, double *out) {
  const int64_t n = (int64_t)rows * D;
  for (int it = 0; it < n_iters; ++it)
    for (int k = 0; k < N; ++k)
      for (int64_t e = 0; e < n; ++e) out[((int64_t)it * N + k) * n + e] = mgref_philox_normal(seed, it, k, e);
}
