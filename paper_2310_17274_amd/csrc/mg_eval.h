// mg_eval.h -- the evaluation kernel: cost and adjoint of every (candidate,
// waypoint row) of a batch in one launch.  Instantiated per lane layout in
// mg_eval_*.hip so the variants compile in parallel.
#pragma once

#include "mg_device.h"

namespace mg {
namespace {

// Copy of a lane's 3x4 transform from the lane `OFF` below (row_shr) or
// above (row_shl) within the 16-lane DPP row.
template <int CTRL>
__device__ __forceinline__ void dpp12(const float* src, float* dst) {
#pragma unroll
  for (int e = 0; e < 12; ++e) dst[e] = dpp<CTRL>(src[e]);
}

// One Hillis-Steele step of the prefix product along a chain:
// P <- P(lane - OFF) * P for lanes at least OFF past their chain start.
template <int OFF>
__device__ __forceinline__ void scan_step(float* P, bool active) {
  float Q[12];
  dpp12<0x110 + OFF>(P, Q);          // row_shr:OFF
  float R[12];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const float q0 = Q[r * 4 + 0], q1 = Q[r * 4 + 1], q2 = Q[r * 4 + 2], q3 = Q[r * 4 + 3];
    R[r * 4 + 0] = q0 * P[0] + q1 * P[4] + q2 * P[8];
    R[r * 4 + 1] = q0 * P[1] + q1 * P[5] + q2 * P[9];
    R[r * 4 + 2] = q0 * P[2] + q1 * P[6] + q2 * P[10];
    R[r * 4 + 3] = q0 * P[3] + q1 * P[7] + q2 * P[11] + q3;
  }
#pragma unroll
  for (int e = 0; e < 12; ++e) P[e] = active ? R[e] : P[e];
}

// One step of the suffix sum of a 6-vector along a chain (row_shl:OFF).
template <int OFF>
__device__ __forceinline__ void suffix_step(float* W, bool active) {
#pragma unroll
  for (int e = 0; e < 6; ++e) {
    const float v = dpp<0x100 + OFF>(W[e]);
    W[e] = active ? W[e] + v : W[e];
  }
}

// Pose reaching cost (Eq.(14)) of end effector ee whose link pose is T
// (3x4): position term a0 logcosh(a2 |p_g - p|), rotation term
// a1 logcosh(a3 |q_g - s q|) with s the sign of <q_g, q>.  The gradient
// enters as a wrench on the link: force d cost / d p at the tool point and
// the moment conjugate to a world-frame rotation.  pe_row >= 0 (and ee 0)
// records the position and angle errors of that row.
// etf: the tool transform (3x4), gl: the goal (position, quaternion w x y z).
__device__ __forceinline__ void pose_term_at(const EvalArgs& a, const float* etf, const float* gl, int ee,
                                             const float* T, int pe_row, float& cost, float& Fx, float& Fy,
                                             float& Fz, float& Mx, float& My, float& Mz) {
  float E[12];
#pragma unroll
  for (int i = 0; i < 12; ++i) E[i] = T[i];
  compose(E, etf);
  float qw, qx, qy, qz;
  mat_to_quat(E, qw, qx, qy, qz);
  const float px = E[3], py = E[7], pz = E[11];
  const float ex = gl[0] - px, ey = gl[1] - py, ez = gl[2] - pz;
  const float n = sqrtf(ex * ex + ey * ey + ez * ez);
  cost += a.pr.a0 * logcosh_f(a.pr.a2 * n);
  const float fp = -a.pr.a0 * a.pr.a2 * tanh_over(a.pr.a2, n);
  const float gpx = fp * ex, gpy = fp * ey, gpz = fp * ez;     // d cost / d p
  const float dot = gl[3] * qw + gl[4] * qx + gl[5] * qy + gl[6] * qz;
  const float sg = dot >= 0.0f ? 1.0f : -1.0f;
  const float e0 = gl[3] - sg * qw, e1 = gl[4] - sg * qx;
  const float e2 = gl[5] - sg * qy, e3 = gl[6] - sg * qz;
  const float dr = sqrtf(e0 * e0 + e1 * e1 + e2 * e2 + e3 * e3);
  cost += a.pr.a1 * logcosh_f(a.pr.a3 * dr);
  // d cost / d quaternion, then the moment conjugate to a world-frame
  // rotation omega: d quat = 1/2 (0, omega) (x) quat
  const float fq = -sg * a.pr.a1 * a.pr.a3 * tanh_over(a.pr.a3, dr);
  const float gw = fq * e0, gvx = fq * e1, gvy = fq * e2, gvz = fq * e3;
  const float tx = 0.5f * (qw * gvx - gw * qx + (qy * gvz - qz * gvy));
  const float ty = 0.5f * (qw * gvy - gw * qy + (qz * gvx - qx * gvz));
  const float tz = 0.5f * (qw * gvz - gw * qz + (qx * gvy - qy * gvx));
  Fx += gpx; Fy += gpy; Fz += gpz;
  Mx += py * gpz - pz * gpy + tx;
  My += pz * gpx - px * gpz + ty;
  Mz += px * gpy - py * gpx + tz;
  if (a.pe_e && pe_row >= 0 && ee == 0) {
    a.pe_e[(size_t)pe_row * 2 + 0] = n;
    a.pe_e[(size_t)pe_row * 2 + 1] = 2.0f * acosf(fminf(fabsf(dot), 1.0f));
  }
}

__device__ __forceinline__ void pose_term(const EvalArgs& a, int p, int ee, const float* T, int pe_row,
                                          float& cost, float& Fx, float& Fy, float& Fz, float& Mx,
                                          float& My, float& Mz) {
  pose_term_at(a, a.rb.ee_tf + ee * 12, a.goal + ((size_t)p * a.rb.n_ee + ee) * 7, ee, T, pe_row, cost, Fx,
               Fy, Fz, Mx, My, Mz);
}

// Joint j at waypoint row `row` (waypoint t+1 of its seed): joint-limit cost
// (Eq.(17), weight w_bound, band eta2) and the smoothness terms of Eq.(16)
// whose five-point stencils (centred at t-1..t+3 on the padded trajectory:
// the start before waypoint 1, the last waypoint after T) touch this state.
// jc receives the terms this waypoint owns, js d cost / d q_j.  qj is the
// (candidate) value at row, qval(r, j) the value at another row; lo_, hi_
// are joint j's limits and q0 its start value.
template <typename QV>
__device__ __forceinline__ void joint_terms(const EvalArgs& a, const Problem& pb, int row, int t, int j,
                                            float qj, float lo_, float hi_, float q0, QV&& qval,
                                            float& jc, float& js) {
  const float e2 = a.pr.eta2, wb = a.pr.w_bound;
  const float inv_e2 = 1.0f / e2;
  float bc = 0.0f, bs = 0.0f;
  if (qj < lo_) { bc += lo_ - qj + 0.5f * e2; bs -= 1.0f; }
  else if (qj < lo_ + e2) { const float u = lo_ - qj + e2; bc += 0.5f * u * u * inv_e2; bs -= u * inv_e2; }
  if (qj > hi_) { bc += qj - hi_ + 0.5f * e2; bs += 1.0f; }
  else if (qj > hi_ - e2) { const float u = qj - hi_ + e2; bc += 0.5f * u * u * inv_e2; bs += u * inv_e2; }
  jc += wb * bc;
  js += wb * bs;
  if (pb.T <= 1) return;
  // padded states X(s), s = w-4..w+4 around this waypoint w = t+1
  const int w1 = t + 1, Tn = pb.T;
  float X[9];
#pragma unroll
  for (int u = 0; u < 9; ++u) {
    const int sgi = w1 - 4 + u;
    const int wv = sgi < 1 ? 1 : (sgi < Tn ? sgi : Tn);
    const float v = u == 4 ? qj : qval(row - t + wv - 1, j);
    X[u] = sgi <= 0 ? q0 : v;
  }
  const float h = a.pr.dt;
  const float cv = 1.0f / (12.0f * h), ca = 1.0f / (12.0f * h * h), cj = 1.0f / (2.0f * h * h * h);
  const float kv[5] = {1.0f, -8.0f, 0.0f, 8.0f, -1.0f};
  const float ka[5] = {-1.0f, 16.0f, -30.0f, 16.0f, -1.0f};
  const float kj[5] = {-1.0f, 2.0f, 0.0f, -2.0f, 1.0f};
#pragma unroll
  for (int c = 0; c < 5; ++c) {
    const int tau = w1 - 2 + c;          // stencil centre, states X[c..c+4]
    float v = 0.0f, ac = 0.0f, jk = 0.0f;
#pragma unroll
    for (int i = 0; i < 5; ++i) {
      v = fmaf(kv[i], X[c + i], v);
      ac = fmaf(ka[i], X[c + i], ac);
      jk = fmaf(kj[i], X[c + i], jk);
    }
    v *= cv; ac *= ca; jk *= cj;
    const bool in = tau >= 0 && tau <= Tn;
    const bool mine = in && (tau == w1 || (tau == 0 && w1 == 1));   // cost owner
    const bool vel = in && (a.pr.vel_all || tau == Tn);
    float gv = 0.0f;
    if (vel) {   // transcendentals only where the velocity term applies
      gv = a.pr.a6 * a.pr.a7 * tanhf(a.pr.a7 * v) * cv;
      if (mine) jc += a.pr.a6 * logcosh_f(a.pr.a7 * v);
    }
    if (mine) jc += a.pr.a8 * ac * ac + a.pr.a9 * jk * jk;
    const float ga = 2.0f * a.pr.a8 * ac * ca, gjk = 2.0f * a.pr.a9 * jk * cj;
    // stencil entry i touches padded state tau - 2 + i; this waypoint's
    // state is entry 4 - c alone, or, for the last waypoint, every entry
    // from 4 - c on (the padding after it repeats it)
    float wv = 0.0f, wa = 0.0f, wj = 0.0f;
#pragma unroll
    for (int i = 4 - c; i < 5; ++i) { wv += kv[i]; wa += ka[i]; wj += kj[i]; }
    const bool last = w1 == Tn;
    const float ev = last ? wv : kv[4 - c], ea = last ? wa : ka[4 - c], ej = last ? wj : kj[4 - c];
    js += in ? gv * ev + ga * ea + gjk * ej : 0.0f;
  }
}

// Pose of this lane's link at its joint value q: the local transform
// F_l Rz(q) from the Tab.6 closed form (columns 0 and 1 mix, 2 and 3 are
// F's), then the prefix product along the chain (pos = lanes past the chain
// start).  Lanes without a link hold the identity.
template <int LPE>
__device__ __forceinline__ void link_pose(const float* __restrict__ fixed_tf, int lj, bool on, int pos,
                                          float q, float* T) {
  const float sn = __sinf(q), cs = __cosf(q);
  const float4 f0 = *reinterpret_cast<const float4*>(fixed_tf + lj * 12 + 0);
  const float4 f1 = *reinterpret_cast<const float4*>(fixed_tf + lj * 12 + 4);
  const float4 f2 = *reinterpret_cast<const float4*>(fixed_tf + lj * 12 + 8);
  T[0] = f0.x * cs + f0.y * sn;  T[1] = f0.y * cs - f0.x * sn;  T[2] = f0.z;  T[3] = f0.w;
  T[4] = f1.x * cs + f1.y * sn;  T[5] = f1.y * cs - f1.x * sn;  T[6] = f1.z;  T[7] = f1.w;
  T[8] = f2.x * cs + f2.y * sn;  T[9] = f2.y * cs - f2.x * sn;  T[10] = f2.z; T[11] = f2.w;
  if (!on) identity(T);
  scan_step<1>(T, pos >= 1);
  scan_step<2>(T, pos >= 2);
  scan_step<4>(T, pos >= 4);
  if (LPE > 8) scan_step<8>(T, pos >= 8);
}

// Continuous collision of one sphere against one cuboid (Alg.11-12 sphere
// tracing): from the centre c toward the neighbouring waypoint's centre,
// step by the clearance (by r + eta inside the band) while short of the
// half-way point, at most sweep_steps samples per side, each costed with the
// Eq.(10) profile.  (px, py, pz) is c in the box frame, sdf its distance.
// ls: the sphere in its link's frame; Tp, Tn: the link's poses at the
// neighbouring waypoints.
__device__ __forceinline__ void sweep_pair_ls(const float4 ls, int steps, const float* Tp, const float* Tn,
                                              bool has_next, float cx, float cy, float cz, const v4f& A0,
                                              const v4f& A1, const v4f& A2, const v4f& Hh, float px, float py,
                                              float pz, float sdf, float r, float w, float eta, float inv_eta,
                                              float& cost, float& gx, float& gy, float& gz) {
  const float rh = r + eta;
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    const float* Tb = side == 0 ? Tp : Tn;
    if (side == 1 && !has_next) break;
    float ux = Tb[0] * ls.x + Tb[1] * ls.y + Tb[2] * ls.z + Tb[3] - cx;
    float uy = Tb[4] * ls.x + Tb[5] * ls.y + Tb[6] * ls.z + Tb[7] - cy;
    float uz = Tb[8] * ls.x + Tb[9] * ls.y + Tb[10] * ls.z + Tb[11] - cz;
    const float len = sqrtf(ux * ux + uy * uy + uz * uz);
    if (!(len > 0.0f)) continue;
    const float il = 1.0f / len;
    ux *= il; uy *= il; uz *= il;
    // unit direction in the box frame
    const float vx = A0.x * ux + A0.y * uy + A0.z * uz;
    const float vy = A1.x * ux + A1.y * uy + A1.z * uz;
    const float vz = A2.x * ux + A2.y * uy + A2.z * uz;
    const float half = 0.5f * len;
    float j = sdf < rh ? rh : sdf - rh;
    for (int st = 0; st < steps && j < half; ++st) {
      const float qx = fmaf(j, vx, px), qy = fmaf(j, vy, py), qz = fmaf(j, vz, pz);
      float gpx, gpy, gpz;
      const float s2 = box_sdf(qx, qy, qz, fabsf(qx) - Hh.x, fabsf(qy) - Hh.y, fabsf(qz) - Hh.z,
                               gpx, gpy, gpz);
      dc_term(A0, A1, A2, s2, gpx, gpy, gpz, r, w, eta, inv_eta, cost, gx, gy, gz);
      j += s2 - rh > 0.0f ? s2 - rh : rh;
    }
  }
}

// sweep_pair_ls with the samples' gradients left in the box frame (added to
// b; the caller rotates the pair's sum back to the world once).
__device__ __forceinline__ void sweep_pair_box(const float4 ls, int steps, const float* Tp, const float* Tn,
                                               bool has_next, float cx, float cy, float cz, const v4f& A0,
                                               const v4f& A1, const v4f& A2, const v4f& Hh, float px, float py,
                                               float pz, float sdf, float r, float w, float eta, float inv_eta,
                                               float& cost, float& bx, float& by, float& bz) {
  const float rh = r + eta;
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    const float* Tb = side == 0 ? Tp : Tn;
    if (side == 1 && !has_next) break;
    float ux = Tb[0] * ls.x + Tb[1] * ls.y + Tb[2] * ls.z + Tb[3] - cx;
    float uy = Tb[4] * ls.x + Tb[5] * ls.y + Tb[6] * ls.z + Tb[7] - cy;
    float uz = Tb[8] * ls.x + Tb[9] * ls.y + Tb[10] * ls.z + Tb[11] - cz;
    const float len = sqrtf(ux * ux + uy * uy + uz * uz);
    if (!(len > 0.0f)) continue;
    const float il = 1.0f / len;
    ux *= il; uy *= il; uz *= il;
    const float vx = A0.x * ux + A0.y * uy + A0.z * uz;
    const float vy = A1.x * ux + A1.y * uy + A1.z * uz;
    const float vz = A2.x * ux + A2.y * uy + A2.z * uz;
    const float half = 0.5f * len;
    float j = sdf < rh ? rh : sdf - rh;
    for (int st = 0; st < steps && j < half; ++st) {
      const float qx = fmaf(j, vx, px), qy = fmaf(j, vy, py), qz = fmaf(j, vz, pz);
      float gpx, gpy, gpz;
      const float s2 = box_sdf(qx, qy, qz, fabsf(qx) - Hh.x, fabsf(qy) - Hh.y, fabsf(qz) - Hh.z,
                               gpx, gpy, gpz);
      dc_term_box(s2, gpx, gpy, gpz, r, w, eta, inv_eta, cost, bx, by, bz);
      j += s2 - rh > 0.0f ? s2 - rh : rh;
    }
  }
}

// sweep_pair_box for cost-only evaluations: the trace samples' costs alone.
__device__ __forceinline__ void sweep_pair_cost(const float4 ls, int steps, const float* Tp, const float* Tn,
                                                bool has_next, float cx, float cy, float cz, const v4f& A0,
                                                const v4f& A1, const v4f& A2, const v4f& Hh, float px, float py,
                                                float pz, float sdf, float r, float w, float eta, float inv_eta,
                                                float& cost) {
  const float rh = r + eta;
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    const float* Tb = side == 0 ? Tp : Tn;
    if (side == 1 && !has_next) break;
    float ux = Tb[0] * ls.x + Tb[1] * ls.y + Tb[2] * ls.z + Tb[3] - cx;
    float uy = Tb[4] * ls.x + Tb[5] * ls.y + Tb[6] * ls.z + Tb[7] - cy;
    float uz = Tb[8] * ls.x + Tb[9] * ls.y + Tb[10] * ls.z + Tb[11] - cz;
    const float len = sqrtf(ux * ux + uy * uy + uz * uz);
    if (!(len > 0.0f)) continue;
    const float il = 1.0f / len;
    ux *= il; uy *= il; uz *= il;
    const float vx = A0.x * ux + A0.y * uy + A0.z * uz;
    const float vy = A1.x * ux + A1.y * uy + A1.z * uz;
    const float vz = A2.x * ux + A2.y * uy + A2.z * uz;
    const float half = 0.5f * len;
    float j = sdf < rh ? rh : sdf - rh;
    for (int st = 0; st < steps && j < half; ++st) {
      const float qx = fmaf(j, vx, px), qy = fmaf(j, vy, py), qz = fmaf(j, vz, pz);
      const float s2 = box_dist(fabsf(qx) - Hh.x, fabsf(qy) - Hh.y, fabsf(qz) - Hh.z);
      dc_cost(s2, r, w, eta, inv_eta, cost);
      j += s2 - rh > 0.0f ? s2 - rh : rh;
    }
  }
}

__device__ __forceinline__ void sweep_pair(const EvalArgs& a, int slot, const float* Tp,
                                           const float* Tn, bool has_next, float cx, float cy,
                                           float cz, const v4f& A0, const v4f& A1, const v4f& A2,
                                           const v4f& Hh, float px, float py, float pz, float sdf,
                                           float r, float w, float eta, float inv_eta, float& cost,
                                           float& gx, float& gy, float& gz) {
  sweep_pair_ls(a.ln.sphere[slot], a.pr.sweep_steps, Tp, Tn, has_next, cx, cy, cz, A0, A1, A2, Hh, px, py,
                pz, sdf, r, w, eta, inv_eta, cost, gx, gy, gz);
}

// Lane layout: lane l of an evaluation owns link l.  A wave holds 64/LPE
// evaluations (consecutive waypoint rows of one problem, candidate k =
// blockIdx.y); the 4 waves of a workgroup hold 4/H evaluation groups, each
// group spread over H waves that split the world's cuboids (H slices).
//
// Kinematics: lane l forms its link's local transform F_l Rz(q_l) (Tab.6
// closed form) and a log-depth prefix product along the chain gives the link
// pose.  Adjoint: lane l's link wrench (force and moment of the cost
// gradients at its spheres and end effector) is summed over the links below
// it by a suffix scan; joint l's derivative is z_l . (M - o_l x F) (Tab.7).
//
// SW (continuous collision, Sec. continuous collision checking, Alg.11-12):
// the lane also forms its link pose at the neighbouring waypoints (the start
// configuration before waypoint 1), and each sphere is traced from its
// centre toward the half-way point of both segments; the samples' cost
// gradients act on the centre, as in the paper.
template <int LPE, int MAXS, int H, bool CAND, bool GRAD, bool SW>
__global__ __launch_bounds__(kBlock) void eval_kernel(const EvalArgs a) {
  constexpr int EPW = kWave / LPE;                 // evaluations per wave
  constexpr int GROUPS = (kBlock / kWave) / H;     // evaluation groups per workgroup
  constexpr int EPB = GROUPS * EPW;                // evaluations per workgroup
  __shared__ float s_part[H > 1 ? 8 * kBlock : 1];
  warm_kernargs<sizeof(EvalArgs)>();

  // wave index as a scalar: the cuboid slice of a wave must be provably
  // uniform for its loads to stay scalar
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int lane = threadIdx.x % kWave;
  const int grp = wave / H, slice = wave % H;
  const int l = lane % LPE;
  const int k = blockIdx.y;
  const int bx = blockIdx.x;
  // problem of this workgroup: last p with chunk_prefix[p] <= bx
  int lo = 0, hi = a.P;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (a.chunk_prefix[mid] <= bx) lo = mid; else hi = mid;
  }
  const int p = lo;
  const Problem pb = a.prob[p];
  const int D = a.rb.dof, L = a.rb.n_links;
  const int nrows = pb.S * pb.T;
  const int rloc = (bx - a.chunk_prefix[p]) * EPB + grp * EPW + lane / LPE;
  const bool valid = rloc < nrows;
  const int rl = valid ? rloc : nrows - 1;
  const int t = rl % pb.T;          // waypoint t+1 of its seed
  const int row = pb.row0 + rl;
  const float alpha = CAND ? a.alpha[k < kMaxK ? k : 0] : 0.0f;
  const float* dk = CAND && a.d ? a.d + (size_t)k * a.d_stride : nullptr;

  // candidate value of joint j at waypoint row r: clip(x + alpha d) for a
  // line-search candidate, clip(x + sqrt(var) d_k) for a particle
  auto qval = [&](int r, int j) -> float {
    const size_t e = (size_t)r * D + j;
    float v = a.x[e];
    if (CAND) {
      if (a.var) v = fmaf(sqrtf(a.var[e]), dk ? dk[e] : philox_draw(a.pm_seed, k, a.pm_it, e), v);
      else v = fmaf(alpha, dk[e], v);
      v = fminf(fmaxf(v, a.rb.q_lo[j]), a.rb.q_hi[j]);
    }
    return v;
  };

  const int4 li = a.ln.info[l];     // chain start lane, chain end lane, spheres, end effector
  const bool on = l < L;
  const int lj = on ? l : 0;
  const float ql = qval(row, lj);

  // ---- forward kinematics ----
  float T[12];
  link_pose<LPE>(a.rb.fixed_tf, lj, on, l - li.x, ql, T);

  // link poses at the neighbouring waypoints (swept collision; one waypoint
  // alone has no segments to trace)
  float Tp[SW ? 12 : 1], Tn[SW ? 12 : 1];
  const bool sweep = SW && pb.T > 1;
  const bool has_next = sweep && t + 1 < pb.T;
  if constexpr (SW) {
    if (sweep) {
      const float qp = t >= 1 ? qval(row - 1, lj) : a.q_start[(size_t)p * D + lj];
      const float qn = has_next ? qval(row + 1, lj) : ql;
      link_pose<LPE>(a.rb.fixed_tf, lj, on, l - li.x, qp, Tp);
      link_pose<LPE>(a.rb.fixed_tf, lj, on, l - li.x, qn, Tn);
    }
  }

  float cost = 0.0f;
  float mc = a.pr.eta;
  // wrench of this link about the world origin: F = sum of d cost / d point,
  // M = sum of point x (d cost / d point) (+ pure moments of the pose term)
  float Fx = 0.0f, Fy = 0.0f, Fz = 0.0f, Mx = 0.0f, My = 0.0f, Mz = 0.0f;

  // ---- terms that do not involve the world, first slice of each group only:
  //      pose at the last waypoint, joint limits and smoothness ----
  float gsm = 0.0f;
  if (slice == 0) {
    // ---- pose reaching cost at the last waypoint (Eq.(14)) ----
    if (li.w >= 0 && t == pb.T - 1)
      pose_term(a, p, li.w, T, valid ? row : -1, cost, Fx, Fy, Fz, Mx, My, Mz);
    // ---- joint l: limit cost (Eq.(17)) and smoothness (Eq.(16)); every lane
    //      computes (clamped joint), lanes l >= D discard the result ----
    float jc = 0.0f, js = 0.0f;
    joint_terms(a, pb, row, t, lj, ql, a.rb.q_lo[lj], a.rb.q_hi[lj], a.q_start[(size_t)p * D + lj], qval,
                jc, js);
    cost += l < D ? jc : 0.0f;
    gsm = l < D ? js : 0.0f;
  }

  // ---- world collision (Eq.(10)/(11) without the speed factor, summed over
  //      cuboids and spheres); cuboid loop outside, this link's spheres inside
  {
    const float w = a.pr.w_coll, eta = a.pr.eta, inv_eta = 1.0f / fmaxf(eta, 1e-30f);
    float cx[MAXS], cy[MAXS], cz[MAXS], rr[MAXS], rho[MAXS];
#pragma unroll
    for (int s = 0; s < MAXS; ++s) {
      const float4 ls = a.ln.sphere[l * MAXS + s];
      const bool used = s < li.z;
      // unused slots sit far away and never pass the face test
      cx[s] = used ? T[0] * ls.x + T[1] * ls.y + T[2] * ls.z + T[3] : 1e18f;
      cy[s] = used ? T[4] * ls.x + T[5] * ls.y + T[6] * ls.z + T[7] : 1e18f;
      cz[s] = used ? T[8] * ls.x + T[9] * ls.y + T[10] * ls.z + T[11] : 1e18f;
      rr[s] = used ? ls.w : 0.0f;
      rho[s] = rr[s] + eta;
      if constexpr (SW) {
        // every trace sample lies within half a segment of the centre and the
        // distance is 1-Lipschitz, so r + eta + L/2 bounds the cull
        if (sweep && used) {
          const float bx = Tp[0] * ls.x + Tp[1] * ls.y + Tp[2] * ls.z + Tp[3] - cx[s];
          const float by = Tp[4] * ls.x + Tp[5] * ls.y + Tp[6] * ls.z + Tp[7] - cy[s];
          const float bz = Tp[8] * ls.x + Tp[9] * ls.y + Tp[10] * ls.z + Tp[11] - cz[s];
          float l2 = bx * bx + by * by + bz * bz;
          if (has_next) {
            const float fx = Tn[0] * ls.x + Tn[1] * ls.y + Tn[2] * ls.z + Tn[3] - cx[s];
            const float fy = Tn[4] * ls.x + Tn[5] * ls.y + Tn[6] * ls.z + Tn[7] - cy[s];
            const float fz = Tn[8] * ls.x + Tn[9] * ls.y + Tn[10] * ls.z + Tn[11] - cz[s];
            l2 = fmaxf(l2, fx * fx + fy * fy + fz * fz);
          }
          // (slightly widened so rounding never culls a sample the trace takes)
          rho[s] += 0.5f * sqrtf(l2) * 1.0001f + 1e-6f;
        }
      }
    }
    const int w0 = a.world_off[pb.world], w1 = a.world_off[pb.world + 1];
    const int per = (w1 - w0 + H - 1) / H;
    const int o0 = w0 + slice * per;
    const int o1 = min(w1, o0 + per);
    cv4f* boxes = (cv4f*)(a.box);
    // the next cuboid's scalar loads are issued one iteration ahead
    v4f nA0 = {}, nA1 = {}, nA2 = {}, nH = {};
    if (o0 < o1) {
      nA0 = boxes[4 * o0 + 0]; nA1 = boxes[4 * o0 + 1];
      nA2 = boxes[4 * o0 + 2]; nH = boxes[4 * o0 + 3];
    }
    for (int o = o0; o < o1; ++o) {
      const v4f A0 = nA0, A1 = nA1, A2 = nA2, Hh = nH;
      if (o + 1 < o1) {
        nA0 = boxes[4 * o + 4]; nA1 = boxes[4 * o + 5];
        nA2 = boxes[4 * o + 6]; nH = boxes[4 * o + 7];
      }
      // face test of every slot; the box-frame point is recomputed on the
      // rare near path instead of being kept live
      float m3[MAXS];
      bool any = false;
#pragma unroll
      for (int s = 0; s < MAXS; ++s) {
        const float px = fmaf(A0.x, cx[s], fmaf(A0.y, cy[s], fmaf(A0.z, cz[s], A0.w)));
        const float py = fmaf(A1.x, cx[s], fmaf(A1.y, cy[s], fmaf(A1.z, cz[s], A1.w)));
        const float pz = fmaf(A2.x, cx[s], fmaf(A2.y, cy[s], fmaf(A2.z, cz[s], A2.w)));
        m3[s] = fmaxf(fabsf(px) - Hh.x, fmaxf(fabsf(py) - Hh.y, fabsf(pz) - Hh.z));
        // |max(a,0)| >= max(a): a cuboid whose face distance exceeds r + eta
        // adds no cost and cannot lower the clearance clamped at eta
        any |= m3[s] < rho[s];
      }
      if (any) {
#pragma unroll
        for (int s = 0; s < MAXS; ++s)
          if (m3[s] < rho[s]) {
            const float px = fmaf(A0.x, cx[s], fmaf(A0.y, cy[s], fmaf(A0.z, cz[s], A0.w)));
            const float py = fmaf(A1.x, cx[s], fmaf(A1.y, cy[s], fmaf(A1.z, cz[s], A1.w)));
            const float pz = fmaf(A2.x, cx[s], fmaf(A2.y, cy[s], fmaf(A2.z, cz[s], A2.w)));
            float gx = 0.0f, gy = 0.0f, gz = 0.0f;
            const float sdf = near_pair(A0, A1, A2, px, py, pz, fabsf(px) - Hh.x, fabsf(py) - Hh.y,
                                        fabsf(pz) - Hh.z, rr[s], w, eta, inv_eta, cost, mc, gx, gy, gz);
            if constexpr (SW) {
              if (sweep) sweep_pair(a, l * MAXS + s, Tp, Tn, has_next, cx[s], cy[s], cz[s], A0, A1,
                                    A2, Hh, px, py, pz, sdf, rr[s], w, eta, inv_eta, cost, gx, gy, gz);
            }
            Fx += gx; Fy += gy; Fz += gz;
            Mx += cy[s] * gz - cz[s] * gy;
            My += cz[s] * gx - cx[s] * gz;
            Mz += cx[s] * gy - cy[s] * gx;
          }
      }
    }
  }

  // the adjoint only needs this link's joint axis and origin
  const float zx = T[2], zy = T[6], zz = T[10], ox = T[3], oy = T[7], oz = T[11];

  // ---- combine the cuboid slices of an evaluation group (fixed order) ----
  if constexpr (H > 1) {
    float part[8] = {cost, mc, Fx, Fy, Fz, Mx, My, Mz};
#pragma unroll
    for (int q = 0; q < 8; ++q) s_part[q * kBlock + threadIdx.x] = part[q];
    __syncthreads();
    if (slice != 0) return;            // the first wave of the group finishes the row
#pragma unroll
    for (int h = 1; h < H; ++h) {
      const int src = threadIdx.x + h * kWave;
#pragma unroll
      for (int q = 0; q < 8; ++q) part[q] = q == 1 ? fminf(part[q], s_part[q * kBlock + src])
                                                   : part[q] + s_part[q * kBlock + src];
    }
    cost = part[0]; mc = part[1];
    Fx = part[2]; Fy = part[3]; Fz = part[4]; Mx = part[5]; My = part[6]; Mz = part[7];
  }

  // ---- adjoint: suffix sum of link wrenches, projection on joint l's axis ----
  float gradj = 0.0f;
  if (GRAD) {
    float W[6] = {Fx, Fy, Fz, Mx, My, Mz};
    const int left = li.y - 1 - l;     // links after this one on its chain
    suffix_step<1>(W, left >= 1);
    suffix_step<2>(W, left >= 2);
    suffix_step<4>(W, left >= 4);
    if (LPE > 8) suffix_step<8>(W, left >= 8);
    // revolute z (Tab.7): joint axis z and origin o are columns 2 and 3 of the
    // link pose; d/dq = z . (M - o x F)
    const float ux = W[3] - (oy * W[2] - oz * W[1]);
    const float uy = W[4] - (oz * W[0] - ox * W[2]);
    const float uz = W[5] - (ox * W[1] - oy * W[0]);
    gradj = l < D ? zx * ux + zy * uy + zz * uz + gsm : 0.0f;
  }

  const float csum = group_sum<LPE>(cost);
  const float mcmin = group_min<LPE>(mc);
  float gd = 0.0f;
  if (CAND && GRAD && l < D) gd = gradj * a.d[(size_t)row * D + l];
  gd = group_sum<LPE>(gd);
  if (valid) {
    const size_t e = (size_t)k * a.rows + row;
    if (l == 0) {
      a.cost_e[e] = csum;
      if (a.mc_e) a.mc_e[e] = mcmin;
      if (CAND && GRAD) a.gd_e[e] = gd;
    }
    if (GRAD && l < D) a.grad_e[e * D + l] = gradj;
  }
}

template <int LPE, int MAXS, int H, bool SW>
hipError_t launch_eval_hs(const EvalArgs& a, int grid_x, bool cand, bool grad, hipStream_t s) {
  const dim3 grid(grid_x, cand ? a.K : 1), block(kBlock);
  if (cand && grad) eval_kernel<LPE, MAXS, H, true, true, SW><<<grid, block, 0, s>>>(a);
  else if (grad) eval_kernel<LPE, MAXS, H, false, true, SW><<<grid, block, 0, s>>>(a);
  else if (!cand) eval_kernel<LPE, MAXS, H, false, false, SW><<<grid, block, 0, s>>>(a);
  else eval_kernel<LPE, MAXS, H, true, false, SW><<<grid, block, 0, s>>>(a);   // particle costs
  return hipGetLastError();
}

// Swept collision is built for whole-world waves only (one slice).
template <int LPE, int MAXS, int H>
hipError_t launch_eval_h(const EvalArgs& a, int grid_x, bool cand, bool grad, hipStream_t s) {
  if constexpr (H == 1) {
    if (a.pr.swept) return launch_eval_hs<LPE, MAXS, 1, true>(a, grid_x, cand, grad, s);
  } else {
    if (a.pr.swept) return hipErrorInvalidValue;
  }
  return launch_eval_hs<LPE, MAXS, H, false>(a, grid_x, cand, grad, s);
}

template <int LPE, int MAXS>
hipError_t launch_eval_shape(const EvalArgs& a, int grid_x, bool cand, bool grad, hipStream_t s) {
  if (a.slices == 1) return launch_eval_h<LPE, MAXS, 1>(a, grid_x, cand, grad, s);
  if (a.slices == 2) return launch_eval_h<LPE, MAXS, 2>(a, grid_x, cand, grad, s);
  if (a.slices == 4) return launch_eval_h<LPE, MAXS, 4>(a, grid_x, cand, grad, s);
  return hipErrorInvalidValue;
}

}  // namespace

// One translation unit per (lanes per evaluation, sphere slots) pair.
hipError_t launch_eval_l8s4(const EvalArgs& a, int grid_x, bool cand, bool grad, hipStream_t s);
hipError_t launch_eval_l8s8(const EvalArgs& a, int grid_x, bool cand, bool grad, hipStream_t s);
hipError_t launch_eval_l8s16(const EvalArgs& a, int grid_x, bool cand, bool grad, hipStream_t s);
hipError_t launch_eval_l16s4(const EvalArgs& a, int grid_x, bool cand, bool grad, hipStream_t s);
hipError_t launch_eval_l16s8(const EvalArgs& a, int grid_x, bool cand, bool grad, hipStream_t s);
hipError_t launch_eval_l16s16(const EvalArgs& a, int grid_x, bool cand, bool grad, hipStream_t s);

}  // namespace mg
