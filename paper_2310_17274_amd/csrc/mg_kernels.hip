// mg_kernels.hip -- gfx950 kernels of the batched trajectory-optimizer hot path.
//
// eval_kernel      one launch evaluates cost (and gradient) of every
//                  (candidate k, waypoint row): FK in registers, sphere-vs-
//                  cuboid cost with cuboids read as wave-uniform scalar
//                  loads, joint-limit, smoothness and pose costs, and the
//                  hand-written adjoint with the chain transforms recomputed.
// reduce_kernel    per-seed sums of a single evaluation.
// (select_kernel and lbfgs_kernel, the line-search choice with best
//  tracking and the two-loop L-BFGS direction, are in mg_solver.h)
// particle_update_kernel  particle-stage weights, mean and variance update.
// final_kernel     per-problem best seed and success verdict.
// retime_kernel    per-seed spacing that puts the trajectory on its limits.
// ik_seed_kernel   IK seeds ranked per problem, linear trajectory seeds.
// traj_select_kernel  per-problem choice among trajectory seeds.
// steer_points_kernel, steer_scan_kernel  parallel steering of graph edges.
#include <climits>

#include "mg_device.h"
#include "mg_eval.h"

namespace mg {
namespace {

// --------------------------------------------------------------------------
// Per-seed totals of one evaluation (K = 1).
__global__ __launch_bounds__(kBlock) void reduce_kernel(const ReduceArgs a) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= a.n_seeds) return;
  const SeedInfo si = a.seeds[s];
  float c = 0.0f, m = 3.0e38f;
  for (int t = 0; t < si.T; ++t) {
    c += a.cost_e[si.row0 + t];
    m = fminf(m, a.mc_e[si.row0 + t]);
  }
  a.cost[s] = c;
  if (a.min_clear) a.min_clear[s] = m;
}

// --------------------------------------------------------------------------
// The speed metric's gradient on the neighbouring waypoints (Eq.(11)).  The
// evaluation kernel left, per (candidate k, row, sphere m), h = C_m u / (|u|
// 2 dt): the sphere's collision cost times its unit chord between the
// neighbouring positions.  The speed at waypoint t is |c(t+1) - c(t-1)| /
// (2 dt) (the start before waypoint 1, waypoint T repeated after T), so
// sphere m at row t feels h(t-1) from its left neighbour's speed, -h(t+1)
// from its right neighbour's, and h(t) itself at the last waypoint.  One
// wave per (seed, candidate), lane = waypoint: the link frames (Tab.6, in
// LDS), each link's wrench of those forces, and joint j's derivative
// z_j . (M - o_j x F) over the links below it (Tab.7), added to the
// evaluation's gradient and directional derivative.
__global__ __launch_bounds__(kWave) void speed_adjoint_kernel(const SpeedAdjArgs a) {
  extern __shared__ float s_tf[];   // [lane][L][12]
  const int seed = blockIdx.x, k = blockIdx.y, t = threadIdx.x;
  const SeedInfo si = a.seeds[seed];
  if (t >= si.T) return;
  const int D = a.dof, L = a.n_links, M = a.n_spheres;
  const int row = si.row0 + t;
  float* tf = s_tf + (size_t)t * L * 12;
  const float al = a.alpha[k];
  // link frames at the evaluation's configuration (the candidate exactly
  // as the evaluation kernel formed it)
  for (int l = 0; l < L; ++l) {
    float q = a.x[(size_t)row * D + l];
    if (a.cand) q = fminf(fmaxf(fmaf(al, a.d[(size_t)row * D + l], q), a.q_lo[l]), a.q_hi[l]);
    float sn, cs;
    sincosf(q, &sn, &cs);
    const float* F = a.fixed_tf + l * 12;
    float P[12];
    if (a.info[l].x > 1) {
      for (int e = 0; e < 12; ++e) P[e] = tf[(l - 1) * 12 + e];
    } else {
      identity(P);
    }
    float* To = tf + l * 12;
    for (int r = 0; r < 3; ++r) {
      const float t0 = P[r * 4 + 0], t1 = P[r * 4 + 1], t2 = P[r * 4 + 2], t3 = P[r * 4 + 3];
      const float u0 = t0 * F[0] + t1 * F[4] + t2 * F[8];
      const float u1 = t0 * F[1] + t1 * F[5] + t2 * F[9];
      To[r * 4 + 2] = t0 * F[2] + t1 * F[6] + t2 * F[10];
      To[r * 4 + 3] = t0 * F[3] + t1 * F[7] + t2 * F[11] + t3;
      To[r * 4 + 0] = u0 * cs + u1 * sn;
      To[r * 4 + 1] = u1 * cs - u0 * sn;
    }
  }
  const float4* hb = a.sp_h + ((size_t)k * a.rows + row) * M;
  const bool has_prev = t >= 1, has_next = t + 1 < si.T, last = t + 1 == si.T;
  // links from the last to the first: wrench sums over each arm's tail
  float SF[3] = {0.0f, 0.0f, 0.0f}, SM[3] = {0.0f, 0.0f, 0.0f};
  float gd = 0.0f;
  float* g = a.grad_e + ((size_t)k * a.rows + row) * D;
  for (int l = L - 1; l >= 0; --l) {
    const float* T = tf + l * 12;
    const int ns = a.info[l].y;
    for (int s = 0; s < ns; ++s) {
      const float4 ls = a.sphere[l * a.maxs + s];
      const int m = a.slot_sphere[l * a.maxs + s];
      float fx = 0.0f, fy = 0.0f, fz = 0.0f;
      if (has_prev) { const float4 h = hb[m - M]; fx += h.x; fy += h.y; fz += h.z; }
      if (has_next) { const float4 h = hb[m + M]; fx -= h.x; fy -= h.y; fz -= h.z; }
      if (last) { const float4 h = hb[m]; fx += h.x; fy += h.y; fz += h.z; }
      if (fx == 0.0f && fy == 0.0f && fz == 0.0f) continue;
      const float cx = T[0] * ls.x + T[1] * ls.y + T[2] * ls.z + T[3];
      const float cy = T[4] * ls.x + T[5] * ls.y + T[6] * ls.z + T[7];
      const float cz = T[8] * ls.x + T[9] * ls.y + T[10] * ls.z + T[11];
      SF[0] += fx; SF[1] += fy; SF[2] += fz;
      SM[0] += cy * fz - cz * fy; SM[1] += cz * fx - cx * fz; SM[2] += cx * fy - cy * fx;
    }
    const float zx = T[2], zy = T[6], zz = T[10], ox = T[3], oy = T[7], oz = T[11];
    const float dg = zx * (SM[0] - (oy * SF[2] - oz * SF[1])) + zy * (SM[1] - (oz * SF[0] - ox * SF[2])) +
                     zz * (SM[2] - (ox * SF[1] - oy * SF[0]));
    if (l < D) {
      g[l] += dg;
      if (a.cand) gd = fmaf(dg, a.d[(size_t)row * D + l], gd);
    }
    if (a.info[l].x <= 1) {   // the root of an arm: the next arm's sums start afresh
      SF[0] = SF[1] = SF[2] = 0.0f;
      SM[0] = SM[1] = SM[2] = 0.0f;
    }
  }
  if (a.cand) a.gd_e[(size_t)k * a.rows + row] += gd;
}

// --------------------------------------------------------------------------
// Standard normal draws of the particle stage, one thread per four
// consecutive elements of a (round, particle): one Philox block gives the
// four words (float4 stores where the row block allows).
__global__ __launch_bounds__(kBlock) void philox_normals_kernel(unsigned long long seed, int it0, int N,
                                                                long long n, float* out) {
  const long long q = (long long)blockIdx.x * kBlock + threadIdx.x;   // group of four elements
  const int k = blockIdx.y, it = it0 + blockIdx.z;
  if (4 * q >= n) return;
  uint64_t w[4];
  philox4x64((uint64_t)q, (uint64_t)(unsigned)k, (uint64_t)(unsigned)it, 0, seed, 0, w);
  float* o = out + ((size_t)blockIdx.z * N + k) * n + 4 * q;
  if ((n & 3) == 0) {
    *reinterpret_cast<float4*>(o) = float4{box_muller(w[0]), box_muller(w[1]), box_muller(w[2]), box_muller(w[3])};
  } else {
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (4 * q + i < n) o[i] = box_muller(w[i]);
  }
}

// --------------------------------------------------------------------------
// Particle-based optimization update (Alg.5, Eq.(12)-(13)) of one seed per
// workgroup: particle costs from the per-row sums, exponential-utility
// weights w = softmax(-(C - min C) / beta), then per element
//   mean' = (1 - k_mu) mean + k_mu sum_i w_i theta_i
//   var'  = (1 - k_sigma) var + k_sigma sum_i w_i (theta_i - mean)^2
// with theta_i = clip(mean + sqrt(var) eps_i) formed exactly as the
// evaluation kernel formed it.  Fixed-order reductions: deterministic.
template <typename Op>
__device__ __forceinline__ float block_reduce(float v, float* s_red, Op op) {
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
#pragma unroll
  for (int o = kWave / 2; o >= 1; o >>= 1) v = op(v, __shfl_xor(v, o, kWave));
  __syncthreads();
  if (lane == 0) s_red[wave] = v;
  __syncthreads();
  float r = s_red[0];
  for (int w = 1; w < kBlock / kWave; ++w) r = op(r, s_red[w]);
  return r;
}

__global__ __launch_bounds__(kBlock) void particle_update_kernel(const ParticleArgs a) {
  __shared__ float s_w[kMaxParticles];
  __shared__ float s_red[kBlock / kWave];
  warm_kernargs<sizeof(ParticleArgs)>();
  const int seed = blockIdx.x;
  const SeedInfo si = a.seeds[seed];
  const int D = a.dof, N = a.N;
  float cmin = 3.0e38f, cmax = -3.0e38f;
  for (int i = threadIdx.x; i < N; i += kBlock) {
    const float* ce = a.cost_e + (size_t)i * a.rows + si.row0;
    float c = 0.0f;
    for (int t = 0; t < si.T; ++t) c += ce[t];
    s_w[i] = c;
    if (a.costs_out) a.costs_out[(size_t)seed * N + i] = c;
    cmin = fminf(cmin, c);
    cmax = fmaxf(cmax, c);
  }
  cmin = block_reduce(cmin, s_red, [](float x, float y) { return fminf(x, y); });
  cmax = block_reduce(cmax, s_red, [](float x, float y) { return fmaxf(x, y); });
  const float beta = a.beta > 0.0f ? a.beta : 0.1f * (cmax - cmin) + 1e-12f;
  const float inv_beta = 1.0f / beta;
  float z = 0.0f;
  for (int i = threadIdx.x; i < N; i += kBlock) {
    const float w = expf(-(s_w[i] - cmin) * inv_beta);
    s_w[i] = w;
    z += w;
  }
  z = block_reduce(z, s_red, [](float x, float y) { return x + y; });
  const float inv_z = 1.0f / z;
  __syncthreads();
  const int n = si.T * D;
  const size_t base = (size_t)si.row0 * D, stride = (size_t)a.rows * D;
  if (!a.eps) {
    // draws re-made as the evaluation made them, a Philox block (four
    // consecutive elements) per thread and particle
    const size_t q0 = base >> 2, nq = ((base + n + 3) >> 2) - q0;
    for (size_t qi = threadIdx.x; qi < nq; qi += kBlock) {
      const size_t e0 = 4 * (q0 + qi);
      float mu[4], v[4], sd[4], lo[4], hi[4], m1[4], m2[4];
      bool in[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        in[u] = e0 + u >= base && e0 + u < base + n;
        const size_t e = in[u] ? e0 + u : base;
        const int j = (int)(e % D);
        mu[u] = a.mean[e];
        v[u] = a.var[e];
        sd[u] = sqrtf(v[u]);
        lo[u] = a.q_lo[j];
        hi[u] = a.q_hi[j];
        m1[u] = 0.0f;
        m2[u] = 0.0f;
      }
      for (int i = 0; i < N; ++i) {
        float ep[4];
        philox_draws4(a.seed, i, a.it, q0 + qi, ep);
        const float w = s_w[i];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const float th = fminf(fmaxf(fmaf(sd[u], ep[u], mu[u]), lo[u]), hi[u]);
          const float dv = th - mu[u];
          m1[u] = fmaf(w, th, m1[u]);
          m2[u] = fmaf(w, dv * dv, m2[u]);
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (!in[u]) continue;
        const size_t e = e0 + u;
        a.var[e] = (1.0f - a.k_sigma) * v[u] + a.k_sigma * (m2[u] * inv_z);
        a.mean[e] = (1.0f - a.k_mu) * mu[u] + a.k_mu * (m1[u] * inv_z);
      }
    }
    return;
  }
  for (int e = threadIdx.x; e < n; e += kBlock) {
    const float mu = a.mean[base + e], v = a.var[base + e], sd = sqrtf(v);
    const int j = e % D;
    const float lo = a.q_lo[j], hi = a.q_hi[j];
    float m1 = 0.0f, m2 = 0.0f;
    const float* ep = a.eps + base + e;
    for (int i = 0; i < N; ++i) {
      const float th = fminf(fmaxf(fmaf(sd, ep[(size_t)i * stride], mu), lo), hi);
      const float w = s_w[i];
      const float dv = th - mu;
      m1 = fmaf(w, th, m1);
      m2 = fmaf(w, dv * dv, m2);
    }
    a.var[base + e] = (1.0f - a.k_sigma) * v + a.k_sigma * (m2 * inv_z);
    a.mean[base + e] = (1.0f - a.k_mu) * mu + a.k_mu * (m1 * inv_z);
  }
}

// --------------------------------------------------------------------------
// Per problem: best seed (lowest index on ties) and success verdict.
// --------------------------------------------------------------------------
// Retiming (Alg.4), one wave per seed.  Read at spacing h, the five-point
// stencils of the padded trajectory (start copied below t = 1, the last
// waypoint above T) give v, a, j at t = 0..T; derivatives of order k scale
// as h^-k, so the spacing that puts each on its limit is h |v| / vmax,
// h sqrt(|a| / amax), h cbrt(|j| / jmax), and the seed's result is the
// largest over waypoints and joints (the first limit met as h shrinks).
__global__ __launch_bounds__(kWave) void retime_kernel(const RetimeArgs a) {
  const int seed = blockIdx.x, lane = threadIdx.x;
  const SeedInfo si = a.seeds[seed];
  const int D = a.dof, T = si.T;
  const float* q0 = a.q_start + (size_t)si.prob * D;
  const float* q = a.x + (size_t)si.row0 * D;
  auto X = [&](int tau, int d) { return tau <= 0 ? q0[d] : q[(size_t)(min(tau, T) - 1) * D + d]; };
  const float h = a.dt;
  const float kv = 1.0f / (12.0f * h), ka = 1.0f / (12.0f * h * h), kj = 1.0f / (2.0f * h * h * h);
  float r = 0.0f, jm = 0.0f;
  for (int i = lane; i < (T + 1) * D; i += kWave) {
    const int tau = i / D, d = i - tau * D;
    // offsets from the centre value (the stencil weights sum to zero for
    // a, so it drops out): exactly zero where the trajectory rests
    const float x0 = X(tau, d);
    const float m2 = X(tau - 2, d) - x0, m1 = X(tau - 1, d) - x0, p1 = X(tau + 1, d) - x0, p2 = X(tau + 2, d) - x0;
    const float v = ((m2 - p2) + 8.0f * (p1 - m1)) * kv;
    const float ac = (16.0f * (m1 + p1) - (m2 + p2)) * ka;
    const float jk = ((p2 - m2) + 2.0f * (m1 - p1)) * kj;
    r = fmaxf(r, fabsf(v) * a.inv_v[d]);
    r = fmaxf(r, sqrtf(fabsf(ac) * a.inv_a[d]));
    r = fmaxf(r, cbrtf(fabsf(jk) * a.inv_j[d]));
    jm = fmaxf(jm, fabsf(jk));
  }
#pragma unroll
  for (int o = kWave / 2; o >= 1; o >>= 1) {
    r = fmaxf(r, __shfl_xor(r, o, kWave));
    jm = fmaxf(jm, __shfl_xor(jm, o, kWave));
  }
  if (lane == 0) {
    a.dt_out[seed] = h * r;
    // jerk read at spacing h r is jerk at h over r^3
    if (a.jerk_out) a.jerk_out[seed] = r > 0.0f ? jm / (r * r * r) : 0.0f;
  }
}

// --------------------------------------------------------------------------
// Seeds for trajectory optimization from collision-free IK (the overview of
// global motion generation; App. 'Evaluating Optimized Trajectories').  Per
// problem: the IK seeds within the success tolerances and collision free,
// ranked by pos_err + rot_err + w_dist |q - q_start| (ties to the lower
// index); with none, every seed ranked by cost.  Trajectory seed i runs on
// the line from the start to the (i mod count)-th ranked IK solution.
__global__ __launch_bounds__(kBlock) void ik_seed_kernel(const IkSeedArgs a) {
  __shared__ float s_key[kMaxIkSeeds];
  __shared__ int s_ok[kMaxIkSeeds];
  __shared__ int s_order[kMaxIkSeeds];
  __shared__ int s_nvalid;
  const int p = blockIdx.x, D = a.dof;
  const Problem ik = a.ik[p], to = a.to[p];
  const float* q0 = a.q_start + (size_t)p * D;
  if (threadIdx.x == 0) s_nvalid = 0;
  __syncthreads();
  for (int s = threadIdx.x; s < ik.S; s += kBlock) {
    const int r = ik.row0 + s;
    const bool ok = a.pe_e[2 * r] <= a.pos_tol && a.pe_e[2 * r + 1] <= a.rot_tol && a.mc_e[r] >= 0.0f;
    float d2 = 0.0f;
    for (int j = 0; j < D; ++j) {
      const float u = a.x_ik[(size_t)r * D + j] - q0[j];
      d2 = fmaf(u, u, d2);
    }
    const float key = ok ? a.pe_e[2 * r] + a.pe_e[2 * r + 1] + a.w_dist * sqrtf(d2) : a.cost_e[r];
    s_ok[s] = ok;
    // a NaN key (a NaN cost or seed) ranks last: the order stays total
    s_key[s] = key == key ? key : INFINITY;
    s_order[s] = s;
    if (ok) atomicAdd(&s_nvalid, 1);
  }
  __syncthreads();
  const int nv = s_nvalid;
  // rank among the eligible seeds: smaller key, then lower index (a
  // permutation of 0 .. eligible - 1, so every used slot is written)
  for (int s = threadIdx.x; s < ik.S; s += kBlock) {
    if (nv > 0 && !s_ok[s]) continue;
    const float k = s_key[s];
    int rank = 0;
    for (int u = 0; u < ik.S; ++u)
      rank += (nv == 0 || s_ok[u]) && (s_key[u] < k || (s_key[u] == k && u < s));
    s_order[rank] = s;
  }
  __syncthreads();
  const int n_use = nv > 0 ? nv : ik.S;
  const float inv_T = 1.0f / (float)to.T;
  for (int e = threadIdx.x; e < to.S * to.T * D; e += kBlock) {
    const int i = e / (to.T * D), rem = e - i * (to.T * D), t = rem / D, j = rem - t * D;
    const int g = min(max(s_order[i % n_use], 0), ik.S - 1);
    const float qs = q0[j], qg = a.x_ik[(size_t)(ik.row0 + g) * D + j];
    a.x_to[(size_t)(to.row0 + i * to.T + t) * D + j] = fmaf((float)(t + 1) * inv_T, qg - qs, qs);
  }
  if (a.ik_ok && threadIdx.x == 0) a.ik_ok[p] = nv > 0;
}

// Choice among the trajectory seeds of a problem: the seeds that reach the
// goal within the success tolerances collision free, by pos_err + rot_err +
// w_jerk max|jerk| + w_time T dt (motion time: T intervals from the start
// at t = 0 to the last waypoint at the seed's retimed spacing dt), ties to
// the lower index; with none, the lowest cost.
__global__ __launch_bounds__(kBlock) void traj_select_kernel(const TrajSelectArgs a) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= a.P) return;
  const Problem pb = a.prob[p];
  int best_v = -1, best_c = 0;
  float sv = 3.0e38f, sc = 3.0e38f;
  for (int s = 0; s < pb.S; ++s) {
    const int r0 = pb.row0 + s * pb.T, rl = r0 + pb.T - 1;
    float c = 0.0f, m = 3.0e38f;
    for (int t = 0; t < pb.T; ++t) {
      c += a.cost_e[r0 + t];
      m = fminf(m, a.mc_e[r0 + t]);
    }
    const float pe = a.pe_e[2 * rl], re = a.pe_e[2 * rl + 1];
    if (c < sc) { sc = c; best_c = s; }
    if (pe <= a.pos_tol && re <= a.rot_tol && m >= 0.0f) {
      const int seed = pb.seed0 + s;
      const float v = pe + re + a.w_jerk * a.jerk_s[seed] + a.w_time * (float)pb.T * a.dt_s[seed];
      if (v < sv) { sv = v; best_v = s; }
    }
  }
  const int b = best_v >= 0 ? best_v : best_c;
  a.best_seed[p] = b;
  if (a.success) a.success[p] = best_v >= 0;
  if (a.motion_time) a.motion_time[p] = (float)pb.T * a.dt_s[pb.seed0 + b];
}

__global__ __launch_bounds__(kBlock) void final_kernel(const FinalArgs a) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= a.P) return;
  const Problem pb = a.prob[p];
  int bs = 0;
  float bc = a.best_c[pb.seed0];
  for (int s = 1; s < pb.S; ++s) {
    const float c = a.best_c[pb.seed0 + s];
    if (c < bc) { bc = c; bs = s; }
  }
  if (a.best_seed) a.best_seed[p] = bs;
  if (a.success) {
    const int r0 = pb.row0 + bs * pb.T;
    float m = 3.0e38f;
    for (int t = 0; t < pb.T; ++t) m = fminf(m, a.mc_e[r0 + t]);
    const int rl = r0 + pb.T - 1;
    const bool ok = a.pe_e[(size_t)rl * 2 + 0] <= a.success_pos &&
                    a.pe_e[(size_t)rl * 2 + 1] <= a.success_rot && m >= 0.0f;
    a.success[p] = ok ? 1 : 0;
  }
}

// End-effector poses, one thread per (row, end effector): the chain from
// the root (Tab.6 F * Rz per joint), the tool transform, Shepperd's
// quaternion.
__global__ __launch_bounds__(kBlock) void ee_pose_kernel(const EePoseArgs a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.rows * a.n_ee) return;
  const int r = i / a.n_ee, e = i - r * a.n_ee;
  const int l = a.ee_link[e];
  const int depth = a.info[l].x;
  float T[12];
  identity(T);
  for (int c = 0; c < depth; ++c) {
    const int u = a.chain[l * kMaxDof + c];
    const float q = a.q[(size_t)r * a.dof + u];
    compose(T, a.fixed_tf + u * 12);
    rotz(T, __sinf(q), __cosf(q));
  }
  compose(T, a.ee_tf + e * 12);
  float qw, qx, qy, qz;
  mat_to_quat(T, qw, qx, qy, qz);
  float* o = a.pose + (size_t)i * 7;
  o[0] = T[3]; o[1] = T[7]; o[2] = T[11];
  o[3] = qw; o[4] = qx; o[5] = qy; o[6] = qz;
}

// Cuboid pose (xyz + wxyz) and full sides -> library layout.
__global__ __launch_bounds__(kBlock) void boxes_kernel(const float* __restrict__ pose,
                                                       const float* __restrict__ dims, int n,
                                                       Box* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float* pz = pose + 7 * i;
  float w = pz[3], x = pz[4], y = pz[5], z = pz[6];
  const float inv = 1.0f / sqrtf(w * w + x * x + y * y + z * z);
  w *= inv; x *= inv; y *= inv; z *= inv;
  // R (box -> world)
  const float r00 = 1 - 2 * (y * y + z * z), r01 = 2 * (x * y - w * z), r02 = 2 * (x * z + w * y);
  const float r10 = 2 * (x * y + w * z), r11 = 1 - 2 * (x * x + z * z), r12 = 2 * (y * z - w * x);
  const float r20 = 2 * (x * z - w * y), r21 = 2 * (y * z + w * x), r22 = 1 - 2 * (x * x + y * y);
  const float tx = pz[0], ty = pz[1], tz = pz[2];
  Box b;
  // A = R^T, b = -R^T t
  b.q[0] = make_float4(r00, r10, r20, -(r00 * tx + r10 * ty + r20 * tz));
  b.q[1] = make_float4(r01, r11, r21, -(r01 * tx + r11 * ty + r21 * tz));
  b.q[2] = make_float4(r02, r12, r22, -(r02 * tx + r12 * ty + r22 * tz));
  b.q[3] = make_float4(0.5f * dims[3 * i + 0], 0.5f * dims[3 * i + 1], 0.5f * dims[3 * i + 2], 0.0f);
  out[i] = b;
}

__global__ __launch_bounds__(kBlock) void copy_kernel(const float* __restrict__ src,
                                                      float* __restrict__ dst, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

__global__ __launch_bounds__(kBlock) void fill_i32_kernel(int* __restrict__ dst, int v, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    dst[i] = v;
}

int blocks_for(size_t n) {
  size_t b = (n + kBlock - 1) / kBlock;
  if (b < 1) b = 1;
  if (b > 65535) b = 65535;
  return (int)b;
}

}  // namespace

hipError_t launch_eval(const EvalArgs& a, int grid_x, bool cand, bool grad, hipStream_t s) {
  if (a.pr.speed) return hipErrorInvalidValue;   // evaluated by the wave-per-link layout only
  const int L = a.ln.lpe, S = a.ln.maxs;
  if (L == 8 && S == 4) return launch_eval_l8s4(a, grid_x, cand, grad, s);
  if (L == 8 && S == 8) return launch_eval_l8s8(a, grid_x, cand, grad, s);
  if (L == 8 && S == 16) return launch_eval_l8s16(a, grid_x, cand, grad, s);
  if (L == 16 && S == 4) return launch_eval_l16s4(a, grid_x, cand, grad, s);
  if (L == 16 && S == 8) return launch_eval_l16s8(a, grid_x, cand, grad, s);
  if (L == 16 && S == 16) return launch_eval_l16s16(a, grid_x, cand, grad, s);
  return hipErrorInvalidValue;
}

hipError_t launch_reduce(const ReduceArgs& a, hipStream_t s) {
  reduce_kernel<<<(a.n_seeds + kBlock - 1) / kBlock, kBlock, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_speed_adjoint(const SpeedAdjArgs& a, hipStream_t s) {
  if (a.n_links < 1 || a.n_links > kMaxDof || a.K < 1 || a.K > kMaxK || !a.sp_h || !a.grad_e ||
      (a.cand && (!a.d || !a.gd_e)))
    return hipErrorInvalidValue;
  const size_t lds = (size_t)kWave * a.n_links * 12 * sizeof(float);
  speed_adjoint_kernel<<<dim3(a.n_seeds, a.K), kWave, lds, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_philox_normals(unsigned long long seed, int it0, int n_iters, int N, long long n, float* out,
                                 hipStream_t s) {
  if (n_iters < 1 || N < 1 || n < 1 || N > 65535 || n_iters > 65535 || (((uintptr_t)out) & 15)) return hipErrorInvalidValue;
  const long long groups = (n + 3) / 4;
  const dim3 grid((unsigned)((groups + kBlock - 1) / kBlock), N, n_iters);
  philox_normals_kernel<<<grid, kBlock, 0, s>>>(seed, it0, N, n, out);
  return hipGetLastError();
}

hipError_t launch_particle_update(const ParticleArgs& a, hipStream_t s) {
  if (a.N < 1 || a.N > kMaxParticles) return hipErrorInvalidValue;
  particle_update_kernel<<<a.n_seeds, kBlock, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_retime(const RetimeArgs& a, hipStream_t s) {
  if (a.n_seeds == 0) return hipSuccess;
  if (a.dof < 1 || a.dof > kMaxDof || !(a.dt > 0.0f)) return hipErrorInvalidValue;
  retime_kernel<<<a.n_seeds, kWave, 0, s>>>(a);
  return hipGetLastError();
}

// --------------------------------------------------------------------------
// Parallel steering (Alg.3).  Edge e from a to b takes n = floor(max_j
// |b_j - a_j| / res) + 1 steps; sample i (0..n) is a + (i / n)(b - a).  An
// edge needing more than n_max steps is not checked.  Samples past n repeat
// the end so every slot of the fixed sample grid holds a configuration.
__device__ __forceinline__ int steer_steps(const SteerArgs& a, int e) {
  float gm = 0.0f;
  for (int j = 0; j < a.dof; ++j)
    gm = fmaxf(gm, fabsf(a.to[(size_t)e * a.dof + j] - a.from[(size_t)e * a.dof + j]));
  return (int)floorf(gm / a.res) + 1;
}

__global__ __launch_bounds__(kBlock) void steer_points_kernel(const SteerArgs a) {
  const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int per = a.n_max + 1;
  if (k >= (long)a.n_edges * per) return;
  const int e = (int)(k / per), i = (int)(k - (long)e * per);
  const int n = steer_steps(a, e);
  const float f = n <= a.n_max ? (float)min(i, n) / (float)n : 0.0f;
  for (int j = 0; j < a.dof; ++j) {
    const float q0 = a.from[(size_t)e * a.dof + j];
    a.pts[(size_t)k * a.dof + j] = fmaf(f, a.to[(size_t)e * a.dof + j] - q0, q0);
  }
}

// The first sample outside the joint limits or in collision (clearance < 0)
// ends the edge: it keeps the sample before (h = n when none fails, -1 when
// the start fails: no progress; -2: the edge needs more than n_max steps).
__global__ __launch_bounds__(kBlock) void steer_scan_kernel(const SteerArgs a) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= a.n_edges) return;
  const int n = steer_steps(a, e), per = a.n_max + 1, D = a.dof;
  int h = -2;
  if (n <= a.n_max) {
    h = n;
    for (int i = 0; i <= n; ++i) {
      const size_t k = (size_t)e * per + i;
      bool ok = a.mc[k] >= 0.0f;
      for (int j = 0; j < D; ++j) {
        const float q = a.pts[k * D + j];
        ok = ok && q >= a.q_lo[j] && q <= a.q_hi[j];
      }
      if (!ok) { h = i - 1; break; }
    }
  }
  const size_t src = (size_t)e * per + (h >= 0 ? h : 0);
  float d2 = 0.0f;
  for (int j = 0; j < D; ++j) {
    const float q = h >= 0 ? a.pts[src * D + j] : a.from[(size_t)e * D + j];
    const float u = q - a.from[(size_t)e * D + j];
    d2 = fmaf(u, u, d2);
    a.reach[(size_t)e * D + j] = q;
  }
  a.last[e] = h;
  if (a.dist) a.dist[e] = sqrtf(d2);
}

hipError_t launch_steer_points(const SteerArgs& a, hipStream_t s) {
  const long n = (long)a.n_edges * (a.n_max + 1);
  steer_points_kernel<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, s>>>(a);
  return hipGetLastError();
}

// --------------------------------------------------------------------------
// The k nearest graph nodes of every query (the geometric planner's
// neighbour search, Alg.2).  Squared Euclidean distances summed joint by
// joint in fp32 without fused multiply-add (each product and sum rounded, so
// a host brute force in fp32 reproduces them bit for bit); ties go to the
// lower node index.  One wave per query: each lane keeps the KMAX nearest of
// its strided share of the nodes in a sorted register list, then k
// wave-wide minimum rounds take the overall nearest in order, the owning
// lane popping its head each round.
template <int KMAX>
__global__ __launch_bounds__(kWave) void knn_kernel(const KnnArgs a) {
#pragma clang fp contract(off)
  const int qi = blockIdx.x, lane = threadIdx.x, D = a.dof;
  float q[kMaxDof];
#pragma unroll
  for (int j = 0; j < kMaxDof; ++j) q[j] = j < D ? a.queries[(size_t)qi * D + j] : 0.0f;
  float bd[KMAX];
  int bi[KMAX];
#pragma unroll
  for (int r = 0; r < KMAX; ++r) { bd[r] = INFINITY; bi[r] = INT_MAX; }
  for (int i = lane; i < a.n_nodes; i += kWave) {
    const float* nd = a.nodes + (size_t)i * D;
    float d2 = 0.0f;
#pragma unroll
    for (int j = 0; j < kMaxDof; ++j)
      if (j < D) {
        const float u = nd[j] - q[j];
        d2 = d2 + u * u;
      }
    if (d2 < bd[KMAX - 1]) {   // (a lane's indices increase: ties keep the earlier)
      float cd = d2;
      int ci = i;
#pragma unroll
      for (int r = 0; r < KMAX; ++r) {
        const bool sw = cd < bd[r];
        const float td = bd[r];
        const int ti = bi[r];
        bd[r] = sw ? cd : td;
        bi[r] = sw ? ci : ti;
        cd = sw ? td : cd;
        ci = sw ? ti : ci;
      }
    }
  }
  for (int r = 0; r < a.k; ++r) {
    float md = bd[0];
    int mi = bi[0];
#pragma unroll
    for (int o = kWave / 2; o >= 1; o >>= 1) {
      const float od = __shfl_xor(md, o, kWave);
      const int oi = __shfl_xor(mi, o, kWave);
      const bool take = od < md || (od == md && oi < mi);
      md = take ? od : md;
      mi = take ? oi : mi;
    }
    if (lane == 0) {
      a.idx[(size_t)qi * a.k + r] = mi == INT_MAX ? -1 : mi;
      if (a.d2) a.d2[(size_t)qi * a.k + r] = md;
    }
    if (bi[0] == mi && mi != INT_MAX) {   // the owner pops its head
#pragma unroll
      for (int u = 0; u + 1 < KMAX; ++u) { bd[u] = bd[u + 1]; bi[u] = bi[u + 1]; }
      bd[KMAX - 1] = INFINITY;
      bi[KMAX - 1] = INT_MAX;
    }
  }
}

hipError_t launch_knn(const KnnArgs& a, hipStream_t s) {
  if (a.n_queries < 1) return hipSuccess;
  if (a.k < 1 || a.k > 32 || a.dof < 1 || a.dof > kMaxDof || a.n_nodes < 0) return hipErrorInvalidValue;
  if (a.k <= 8) knn_kernel<8><<<a.n_queries, kWave, 0, s>>>(a);
  else if (a.k <= 16) knn_kernel<16><<<a.n_queries, kWave, 0, s>>>(a);
  else knn_kernel<32><<<a.n_queries, kWave, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_steer_scan(const SteerArgs& a, hipStream_t s) {
  steer_scan_kernel<<<(a.n_edges + kBlock - 1) / kBlock, kBlock, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_ik_seeds(const IkSeedArgs& a, hipStream_t s) {
  if (a.P == 0) return hipSuccess;
  ik_seed_kernel<<<a.P, kBlock, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_traj_select(const TrajSelectArgs& a, hipStream_t s) {
  if (a.P == 0) return hipSuccess;
  traj_select_kernel<<<(a.P + kBlock - 1) / kBlock, kBlock, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_ee_pose(const EePoseArgs& a, hipStream_t s) {
  const int n = a.rows * a.n_ee;
  if (n == 0) return hipSuccess;
  ee_pose_kernel<<<(n + kBlock - 1) / kBlock, kBlock, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_final(const FinalArgs& a, hipStream_t s) {
  final_kernel<<<(a.P + kBlock - 1) / kBlock, kBlock, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_boxes(const float* pose, const float* dims, int n, Box* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  boxes_kernel<<<(n + kBlock - 1) / kBlock, kBlock, 0, s>>>(pose, dims, n, out);
  return hipGetLastError();
}

hipError_t launch_copy(const float* src, float* dst, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  copy_kernel<<<blocks_for(n), kBlock, 0, s>>>(src, dst, n);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int* dst, int v, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  fill_i32_kernel<<<blocks_for(n), kBlock, 0, s>>>(dst, v, n);
  return hipGetLastError();
}

}  // namespace mg
