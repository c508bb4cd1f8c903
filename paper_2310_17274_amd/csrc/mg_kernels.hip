// mg_kernels.hip -- gfx950 kernels of the batched trajectory-optimizer hot path.
//
// eval_kernel      one launch evaluates cost (and gradient) of every
//                  (candidate k, waypoint row): FK in registers, sphere-vs-
//                  cuboid cost with cuboids read as wave-uniform scalar
//                  loads, joint-limit, smoothness and pose costs, and the
//                  hand-written adjoint with the chain transforms recomputed.
// reduce_kernel    per-seed sums of a single evaluation.
// select_kernel    parallel noisy line-search choice and best tracking.
// lbfgs_kernel     two-loop L-BFGS direction, one wavefront per seed.
// particle_update_kernel  particle-stage weights, mean and variance update.
// final_kernel     per-problem best seed and success verdict.
// retime_kernel    per-seed spacing that puts the trajectory on its limits.
// ik_seed_kernel   IK seeds ranked per problem, linear trajectory seeds.
// traj_select_kernel  per-problem choice among trajectory seeds.
// steer_points_kernel, steer_scan_kernel  parallel steering of graph edges.
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
// Seed s's first row and horizon: from the table, or arithmetic when every
// seed has the same horizon (one dependent memory round trip less).
__device__ __forceinline__ SeedInfo seed_info(const SeedInfo* seeds, int uniform_T, int s) {
  if (uniform_T > 0) return SeedInfo{s * uniform_T, uniform_T, 0, 0};
  return seeds[s];
}

// A seed's row block of n = T*D floats held PL per lane: element u of a
// lane is lane + 64 u (strided), or with V4 lane PL + u (contiguous, moved
// as float4: the block is a multiple of 4 floats and 16-byte aligned).
template <int PL, bool V4>
__device__ __forceinline__ int el_idx(int lane, int u) {
  return V4 ? lane * PL + u : lane + u * kWave;
}
// Loads at clamped (always valid) addresses, masked afterwards (zero
// outside the block).
template <int PL, bool V4>
__device__ __forceinline__ void ld_row(const float* p, int n, int lane, float* v) {
  if constexpr (V4) {
#pragma unroll
    for (int c = 0; c < PL / 4; ++c) {
      const int e = lane * PL + 4 * c;
      const float4 q = *reinterpret_cast<const float4*>(p + min(e, n - 4));
      const bool in = e < n;
      v[4 * c + 0] = in ? q.x : 0.0f;
      v[4 * c + 1] = in ? q.y : 0.0f;
      v[4 * c + 2] = in ? q.z : 0.0f;
      v[4 * c + 3] = in ? q.w : 0.0f;
    }
  } else {
#pragma unroll
    for (int u = 0; u < PL; ++u) {
      const int e = lane + u * kWave;
      v[u] = p[min(e, n - 1)];
      v[u] = e < n ? v[u] : 0.0f;
    }
  }
}
template <int PL, bool V4>
__device__ __forceinline__ void st_row(float* p, int n, int lane, const float* v) {
  if constexpr (V4) {
#pragma unroll
    for (int c = 0; c < PL / 4; ++c) {
      const int e = lane * PL + 4 * c;
      if (e < n) *reinterpret_cast<float4*>(p + e) = make_float4(v[4 * c], v[4 * c + 1], v[4 * c + 2], v[4 * c + 3]);
    }
  } else {
#pragma unroll
    for (int u = 0; u < PL; ++u) {
      const int e = lane + u * kWave;
      if (e < n) p[e] = v[u];
    }
  }
}

// L-BFGS state of one seed in registers: history (newest first), the
// previous iterate and gradient.  Loaded before anything it does not depend
// on is computed, so the loads' latency overlaps that work.  Memory holds
// the history as a ring (slot (head - 1 - c) mod m is the c-th newest);
// every ring slot is read without waiting for the head and the count, and
// the newest-first order is formed in registers once they arrive.
template <int PL, int MH>
struct LbfgsRegs {
  int count, head;
  bool reset;
  float xp[PL], gp[PL];
  float Sh[MH][PL], Yh[MH][PL], rh[MH];
};

template <int PL, int MH, bool V4>
__device__ __forceinline__ void lbfgs_load(const LbfgsArgs& a, int s, int lane, const SeedInfo& si,
                                           LbfgsRegs<PL, MH>& h) {
  const int n = si.T * a.dof;
  const size_t base = (size_t)si.row0 * a.dof;
  const size_t stride = (size_t)a.rows * a.dof;
  const int m = a.m;
  // Every load is unconditional, at a clamped (always valid) address, and
  // masked afterwards: a guarded load becomes a branch around it, which
  // costs more than the load.  (Per-seed scalars go through the constant
  // address space: scalar loads, waited for where first used.)
  const int first = ((cint*)a.first)[s];
  int count = ((cint*)a.meta)[2 * s + 0];
  int head = ((cint*)a.meta)[2 * s + 1];
  ld_row<PL, V4>(a.x_prev + base, n, lane, h.xp);
  ld_row<PL, V4>(a.g_prev + base, n, lane, h.gp);
  float RS[MH][PL], RY[MH][PL], Rr[MH];
#pragma unroll
  for (int r = 0; r < MH; ++r) {
    const int rc = min(r, max(m - 1, 0));   // (the history holds at least one slot)
    Rr[r] = ((cfloat*)a.rho)[(size_t)s * a.m_max + rc];
    ld_row<PL, V4>(a.S + (size_t)rc * stride + base, n, lane, RS[r]);
    ld_row<PL, V4>(a.Y + (size_t)rc * stride + base, n, lane, RY[r]);
  }
  const bool reset = a.reset != 0 || (a.use_first && first != 0);
  if (reset) { count = 0; head = 0; }
  count = min(count, m);
  h.count = count;
  h.head = head;
  h.reset = reset;
#pragma unroll
  for (int u = 0; u < PL; ++u) {
    h.xp[u] = reset ? 0.0f : h.xp[u];
    h.gp[u] = reset ? 0.0f : h.gp[u];
  }
  // newest first: slot c is ring slot (head - 1 - c) mod m (a uniform
  // index; selected, since registers cannot be indexed)
#pragma unroll
  for (int c = 0; c < MH; ++c) {
    const bool live = c < count;
    int i = head - 1 - c;
    i += i < 0 ? m : 0;
    i += i < 0 ? m : 0;
    float rv = Rr[0];
#pragma unroll
    for (int r = 1; r < MH; ++r) rv = i == r ? Rr[r] : rv;
    h.rh[c] = live ? rv : 0.0f;
#pragma unroll
    for (int u = 0; u < PL; ++u) {
      float sv = RS[0][u], yv = RY[0][u];
#pragma unroll
      for (int r = 1; r < MH; ++r) {
        sv = i == r ? RS[r][u] : sv;
        yv = i == r ? RY[r][u] : yv;
      }
      const bool in = live && el_idx<PL, V4>(lane, u) < n;
      h.Sh[c][u] = in ? sv : 0.0f;
      h.Yh[c][u] = in ? yv : 0.0f;
    }
  }
}

// L-BFGS direction (Alg.6) of one seed held by one wavefront, from its
// state in registers and the new iterate xv and gradient gv (lane-strided,
// n = T*D <= 64*PL): stores the last step's pair in the ring when its
// curvature passes the guard, runs the two loops on registers and DPP sums,
// and writes dir and x/g_prev.
template <int PL, int MH, bool V4>
__device__ __forceinline__ void lbfgs_finish(const LbfgsArgs& a, int s, int lane, const SeedInfo& si,
                                             const float* xv, const float* gv, LbfgsRegs<PL, MH>& h) {
  const int n = si.T * a.dof;
  const size_t base = (size_t)si.row0 * a.dof;
  const size_t stride = (size_t)a.rows * a.dof;
  const int m = a.m;
  int count = h.count, head = h.head;
  float sv[PL], yv[PL];
#pragma unroll
  for (int u = 0; u < PL; ++u) {
    const bool in = el_idx<PL, V4>(lane, u) < n && !h.reset;
    sv[u] = in ? xv[u] - h.xp[u] : 0.0f;
    yv[u] = in ? gv[u] - h.gp[u] : 0.0f;
  }
  // curvature pair of the last step
  if (!h.reset && m > 0) {
    float sy = 0.0f, ss = 0.0f, yy = 0.0f;
#pragma unroll
    for (int u = 0; u < PL; ++u) {
      sy = fmaf(sv[u], yv[u], sy);
      ss = fmaf(sv[u], sv[u], ss);
      yy = fmaf(yv[u], yv[u], yy);
    }
    sy = wave_sum(sy); ss = wave_sum(ss); yy = wave_sum(yy);
    if (sy > 1e-10f * sqrtf(ss) * sqrtf(yy) && sy > 0.0f) {
      st_row<PL, V4>(a.S + (size_t)head * stride + base, n, lane, sv);
      st_row<PL, V4>(a.Y + (size_t)head * stride + base, n, lane, yv);
      if (lane == 0) a.rho[(size_t)s * a.m_max + head] = 1.0f / sy;
      // shift the register copy: the new pair becomes slot 0
#pragma unroll
      for (int c = MH - 1; c > 0; --c) {
        h.rh[c] = h.rh[c - 1];
#pragma unroll
        for (int u = 0; u < PL; ++u) { h.Sh[c][u] = h.Sh[c - 1][u]; h.Yh[c][u] = h.Yh[c - 1][u]; }
      }
      h.rh[0] = 1.0f / sy;
#pragma unroll
      for (int u = 0; u < PL; ++u) { h.Sh[0][u] = sv[u]; h.Yh[0][u] = yv[u]; }
      head = (head + 1) % m;
      count = count < m ? count + 1 : m;
    }
  }
  // two-loop recursion
  float q[PL];
#pragma unroll
  for (int u = 0; u < PL; ++u) q[u] = gv[u];
  float al[MH];
#pragma unroll
  for (int c = 0; c < MH; ++c) {
    al[c] = 0.0f;
    if (c < count) {
      float dsq = 0.0f;
#pragma unroll
      for (int u = 0; u < PL; ++u) dsq = fmaf(h.Sh[c][u], q[u], dsq);
      const float ai = h.rh[c] * wave_sum(dsq);
      al[c] = ai;
#pragma unroll
      for (int u = 0; u < PL; ++u) q[u] = fmaf(-ai, h.Yh[c][u], q[u]);
    }
  }
  float gamma;
  if (count > 0) {
    float sy = 0.0f, yy = 0.0f;
#pragma unroll
    for (int u = 0; u < PL; ++u) { sy = fmaf(h.Sh[0][u], h.Yh[0][u], sy); yy = fmaf(h.Yh[0][u], h.Yh[0][u], yy); }
    gamma = wave_sum(sy) / wave_sum(yy);
  } else {
    float gi = 0.0f;
#pragma unroll
    for (int u = 0; u < PL; ++u) gi = fmaxf(gi, fabsf(gv[u]));
    gi = -wave_min(-gi);
    gamma = gi > 0.0f ? fminf(1.0f, 0.1f / gi) : 1.0f;
  }
#pragma unroll
  for (int u = 0; u < PL; ++u) q[u] *= gamma;
#pragma unroll
  for (int c = MH - 1; c >= 0; --c) {
    if (c < count) {
      float dyr = 0.0f;
#pragma unroll
      for (int u = 0; u < PL; ++u) dyr = fmaf(h.Yh[c][u], q[u], dyr);
      const float b = h.rh[c] * wave_sum(dyr);
#pragma unroll
      for (int u = 0; u < PL; ++u) q[u] = fmaf(al[c] - b, h.Sh[c][u], q[u]);
    }
  }
#pragma unroll
  for (int u = 0; u < PL; ++u) q[u] = -q[u];
  st_row<PL, V4>(a.dir + base, n, lane, q);
  st_row<PL, V4>(a.x_prev + base, n, lane, xv);
  st_row<PL, V4>(a.g_prev + base, n, lane, gv);
  if (lane == 0) {
    a.meta[2 * s + 0] = count;
    a.meta[2 * s + 1] = head;
    if (a.use_first) a.first[s] = 0;
  }
}

template <int PL, int MH, bool V4>
__global__ __launch_bounds__(kWave) void lbfgs_kernel(const LbfgsArgs a) {
  const int s = blockIdx.x;          // one wavefront (and workgroup) per seed
  const int lane = threadIdx.x;
  warm_kernargs<sizeof(LbfgsArgs)>();

  const SeedInfo si = seed_info(a.seeds, a.uniform_T, s);
  const int n = si.T * a.dof;
  const size_t base = (size_t)si.row0 * a.dof;
  float xv[PL], gv[PL];
  ld_row<PL, V4>(a.x + base, n, lane, xv);
  ld_row<PL, V4>(a.g + base, n, lane, gv);
  LbfgsRegs<PL, MH> h;
  lbfgs_load<PL, MH, V4>(a, s, lane, si, h);
  lbfgs_finish<PL, MH, V4>(a, s, lane, si, xv, gv, h);
}

// --------------------------------------------------------------------------
// Line-search choice (Alg.1), one wavefront (and workgroup, so the seeds
// spread over the CUs) per seed; lane t holds waypoint t of every
// candidate, all loads issued before the reductions.  KP: the candidate
// count padded to 4, 8 or 16, so the candidates' sums run unrolled and
// overlap.  With FUSED the same wavefront then computes the next L-BFGS
// direction from the chosen iterate, which is still in its registers.
template <int PL, int MH, bool FUSED, int KP, bool V4>
__global__ __launch_bounds__(kWave) void select_kernel(const SelectArgs a, const LbfgsArgs la) {
  const int s = blockIdx.x;            // (the grid is exactly one workgroup per seed)
  const int lane = threadIdx.x;
  warm_kernargs<sizeof(SelectArgs) + (FUSED ? sizeof(LbfgsArgs) + 8 : 0)>();
  const SeedInfo si = seed_info(a.seeds, a.uniform_T, s);
  const int D = a.dof, n = si.T * D;
  const size_t base = (size_t)si.row0 * D;

  // everything that does not depend on the choice is loaded first: the
  // L-BFGS state, the joint limits, and for up to 8 candidates every
  // candidate's gradient
  LbfgsRegs<PL, FUSED ? MH : 1> h;
  if constexpr (FUSED) lbfgs_load<PL, MH, V4>(la, s, lane, si, h);
  constexpr int KG = (PL <= 4 && KP <= 8) ? KP : 1;
  const bool pre = KG > 1;
  float gall[KG][PL];
#pragma unroll
  for (int k = 0; k < KG; ++k) {
    if (pre) ld_row<PL, V4>(a.grad_e + ((size_t)min(k, a.K - 1) * a.rows + si.row0) * D, n, lane, gall[k]);
  }
  float qlo[PL], qhi[PL];
#pragma unroll
  for (int u = 0; u < PL; ++u) {
    const int j = el_idx<PL, V4>(lane, u) % D;
    qlo[u] = a.q_lo[j];
    qhi[u] = a.q_hi[j];
  }
  const float best_prev = ((cfloat*)a.best_c)[s];
  const float c0 = ((cfloat*)a.c0)[s];

  // candidate sums with the lanes split over the candidates: lane kq * G
  // + jq takes waypoints jq, jq + G, ... of candidate kq, then a reduction
  // over its G lanes leaves candidate kq's sums in all of them
  constexpr int G = kWave / KP;
  const int kq = lane / G, jq = lane % G;
  const bool kin = kq < a.K;
  const size_t erow = (size_t)min(kq, a.K - 1) * a.rows + si.row0;
  float cq[KP], gq[KP], mq[KP];
#pragma unroll
  for (int i = 0; i < KP; ++i) {
    const int t = jq + G * i;
    const size_t e = erow + min(t, si.T - 1);
    cq[i] = a.cost_e[e];
    gq[i] = a.gd_e[e];
    mq[i] = a.mc_e[e];
  }
  float gdv[PL], xv[PL], dv[PL], g0v[PL];
  ld_row<PL, V4>(a.x + base, n, lane, xv);
  ld_row<PL, V4>(a.d + base, n, lane, dv);
  ld_row<PL, V4>(a.g0 + base, n, lane, g0v);
  float g0d = 0.0f;
#pragma unroll
  for (int u = 0; u < PL; ++u) {
    gdv[u] = 0.0f;
    g0d = fmaf(g0v[u], dv[u], g0d);
  }
  g0d = wave_sum(g0d);
  float cs = 0.0f, gs = 0.0f, ms = 3.0e38f;
#pragma unroll
  for (int i = 0; i < KP; ++i) {
    const bool in = kin && jq + G * i < si.T;
    cs += in ? cq[i] : 0.0f;
    gs += in ? gq[i] : 0.0f;
    ms = fminf(ms, in ? mq[i] : 3.0e38f);
  }
  cs = group_sum<G>(cs);
  gs = group_sum<G>(gs);
  ms = group_min<G>(ms);
  // Armijo (and Wolfe) test of every candidate; the choice is the last
  // candidate that passes, else the first
  float ak = a.alpha[0];
#pragma unroll
  for (int k = 1; k < KP; ++k) ak = kq == k ? a.alpha[k] : ak;
  bool ok = kin && cs <= c0 + a.eta1 * ak * g0d;
  if (a.mode == 1) ok = ok && (gs >= a.eta_w * g0d);
  if (a.mode == 2) ok = ok && (fabsf(gs) <= a.eta_w * fabsf(g0d));
  const uint64_t okm = __ballot(ok && jq == 0 && kq > 0);
  const int best = okm ? (63 - __builtin_clzll(okm)) / G : 0;
  const float cb = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(cs), best * G));
  const float mcb = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(ms), best * G));
  float al = a.alpha[0];
#pragma unroll
  for (int k = 1; k < KP; ++k) al = best == k ? a.alpha[k] : al;
  const bool improve = a.track && cb < best_prev;
  if (pre) {
#pragma unroll
    for (int k = 0; k < KG; ++k)
#pragma unroll
      for (int u = 0; u < PL; ++u) gdv[u] = k == best ? gall[k][u] : gdv[u];
  } else {
    ld_row<PL, V4>(a.grad_e + ((size_t)best * a.rows + si.row0) * D, n, lane, gdv);
  }
#pragma unroll
  for (int u = 0; u < PL; ++u) {
    const int e = el_idx<PL, V4>(lane, u);
    xv[u] = e < n ? fminf(fmaxf(fmaf(al, dv[u], xv[u]), qlo[u]), qhi[u]) : 0.0f;
  }
  st_row<PL, V4>(a.x_out + base, n, lane, xv);
  st_row<PL, V4>(a.g_out + base, n, lane, gdv);
  if (improve) st_row<PL, V4>(a.best_x + base, n, lane, xv);
  if (lane == 0) {
    a.c_out[s] = cb;
    if (a.chosen) a.chosen[s] = best;
    if (a.mc_out) a.mc_out[s] = mcb;
    if (improve) a.best_c[s] = cb;
  }
  if constexpr (FUSED) lbfgs_finish<PL, MH, V4>(la, s, lane, si, xv, gdv, h);
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

template <int PL, int KP, bool V4>
hipError_t launch_select_k(const SelectArgs& a, const LbfgsArgs* la, hipStream_t s) {
  const dim3 grid(a.n_seeds);
  if (!la) select_kernel<PL, 4, false, KP, V4><<<grid, kWave, 0, s>>>(a, LbfgsArgs{});
  else if (la->m <= 4) select_kernel<PL, 4, true, KP, V4><<<grid, kWave, 0, s>>>(a, *la);
  else select_kernel<PL, kMaxHist, true, KP, V4><<<grid, kWave, 0, s>>>(a, *la);
  return hipGetLastError();
}

// Row blocks move as float4 when every seed's block is a multiple of 4
// floats and every array is 16-byte aligned.
bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }
bool rows_v4(int uniform_T, int dof) { return uniform_T > 0 && (uniform_T * dof) % 4 == 0; }
bool select_v4(const SelectArgs& a, const LbfgsArgs* la) {
  bool ok = rows_v4(a.uniform_T, a.dof) && aligned16(a.x) && aligned16(a.d) && aligned16(a.g0) &&
            aligned16(a.x_out) && aligned16(a.g_out) && aligned16(a.best_x) && aligned16(a.grad_e);
  if (la)
    ok = ok && aligned16(la->S) && aligned16(la->Y) && aligned16(la->x_prev) && aligned16(la->g_prev) &&
         aligned16(la->dir) && (la->rows * la->dof) % 4 == 0;
  return ok;
}

template <int PL>
hipError_t launch_select_pl(const SelectArgs& a, const LbfgsArgs* la, hipStream_t s) {
  if (a.K < 1 || a.K > kMaxK) return hipErrorInvalidValue;
  if constexpr (PL >= 4) {
    if (select_v4(a, la)) {
      if (a.K <= 4) return launch_select_k<PL, 4, true>(a, la, s);
      if (a.K <= 8) return launch_select_k<PL, 8, true>(a, la, s);
      return launch_select_k<PL, 16, true>(a, la, s);
    }
  }
  if (a.K <= 4) return launch_select_k<PL, 4, false>(a, la, s);
  if (a.K <= 8) return launch_select_k<PL, 8, false>(a, la, s);
  return launch_select_k<PL, 16, false>(a, la, s);
}

hipError_t launch_select(const SelectArgs& a, int max_n, const LbfgsArgs* fuse, hipStream_t s) {
  if (max_n <= 64) return launch_select_pl<1>(a, fuse, s);
  if (max_n <= 128) return launch_select_pl<2>(a, fuse, s);
  if (max_n <= 256) return launch_select_pl<4>(a, fuse, s);
  if (max_n <= 512) return launch_select_pl<8>(a, fuse, s);
  return launch_select_pl<16>(a, fuse, s);
}

template <int MH>
hipError_t launch_lbfgs_h(const LbfgsArgs& a, int max_n, hipStream_t s) {
  const dim3 grid(a.n_seeds);
  const bool v4 = rows_v4(a.uniform_T, a.dof) && (a.rows * a.dof) % 4 == 0 && aligned16(a.x) && aligned16(a.g) &&
                  aligned16(a.S) && aligned16(a.Y) && aligned16(a.x_prev) && aligned16(a.g_prev) && aligned16(a.dir);
  if (max_n <= 64) lbfgs_kernel<1, MH, false><<<grid, kWave, 0, s>>>(a);
  else if (max_n <= 128) lbfgs_kernel<2, MH, false><<<grid, kWave, 0, s>>>(a);
  else if (max_n <= 256 && v4) lbfgs_kernel<4, MH, true><<<grid, kWave, 0, s>>>(a);
  else if (max_n <= 256) lbfgs_kernel<4, MH, false><<<grid, kWave, 0, s>>>(a);
  else if (max_n <= 512 && v4) lbfgs_kernel<8, MH, true><<<grid, kWave, 0, s>>>(a);
  else if (max_n <= 512) lbfgs_kernel<8, MH, false><<<grid, kWave, 0, s>>>(a);
  else if (v4) lbfgs_kernel<16, MH, true><<<grid, kWave, 0, s>>>(a);
  else lbfgs_kernel<16, MH, false><<<grid, kWave, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_lbfgs(const LbfgsArgs& a, int max_n, hipStream_t s) {
  if (a.m <= 4) return launch_lbfgs_h<4>(a, max_n, s);
  return launch_lbfgs_h<kMaxHist>(a, max_n, s);
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
