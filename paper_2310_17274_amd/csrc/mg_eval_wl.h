// mg_eval_wl.h -- the evaluation kernel in the wave-per-link layout.
//
// A workgroup holds 64 evaluations (lanes; candidates of consecutive
// waypoint rows of one seed side by side, so the lanes of a wave sit close
// together in configuration space).  Wave l owns link l: it runs the
// kinematic chain from the root to l (Tab.6 closed form per joint), places
// the link's spheres, and tests them against the world's cuboids; the last
// wave owns the joint-limit and smoothness terms of every joint (or, with
// two waves per link, each link's second wave owns its joint's).
//
// The workgroups of one launch run side by side once, on cold caches, so
// every dependent read of memory costs a full round trip.  The kernel
// therefore reads memory in two dependent rounds only: the chunk's record
// (problem, rows, cuboid range) with this wave's tables, then one staging
// pass that brings the rows, limits, start, goals, tool transforms, chain
// records, sphere slots and the first cuboid tile into LDS.  After that
// every read is from LDS (later cuboid tiles are read a tile ahead).
//
// Per cuboid, one test of a ball enclosing the wave's spheres over all 64
// lanes decides whether the wave looks at that cuboid at all (the distance
// is 1-Lipschitz, so a cuboid farther than the ball radius + eta from the
// ball's centre adds no cost and cannot lower the clamped clearance for any
// lane); for a cuboid that passes, each lane tests a ball around its own
// copy of the spheres, and the wave skips the cuboid when none reaches it.
// The adjoint recomputes the chain (Alg.8: no stored transforms) and
// projects the link's wrench on every joint above it (Tab.7); each link
// wave also forms its share of the directional derivative.  The waves'
// partial sums meet in LDS in a fixed order: wave j gathers joint j's
// derivative, the last wave the cost, clearance and directional derivative.
// The world's cuboids can also be split over gridDim.y workgroups of the
// same 64 evaluations; the last of them to finish adds the slices' sums in
// slice order.
#pragma once

#include "mg_eval.h"
#include "mg_solver.h"

namespace mg {
namespace {

__device__ __forceinline__ float wave_max(float v) { return -wave_min(-v); }

// Rows staged per workgroup: 64 evaluations cover at most 64 rows, plus the
// stencils' reach of four rows on either side.
constexpr int kStageRows = kWlStageRows;

__device__ __forceinline__ void part_store(float* p, float v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ float part_load(const float* p) {
  return __hip_atomic_load(const_cast<float*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Self-collision (Eq.(9)), shared by every wave of the workgroup.  The
// link waves have parked their sphere centres in s_sph[(m * 3 + c) * 64 +
// lane]; wave w takes the pairs k = w, w + W, ... and parks its largest
// penetration (first such pair) in s_best; every wave then reads the same
// winner: the largest penetration over all pairs, the first pair on ties.
__device__ __forceinline__ void self_pairs_phase(const EvalArgs& a, int w, int W, const float* s_sph,
                                                 float* s_best, int lane) {
  float bv = 0.0f;
  int bk = -1;
  cv4i* pairs = (cv4i*)(a.wl.self_pairs);
  for (int k = w; k < a.pr.n_self; k += W) {
    const v4i pr = pairs[k];
    const float dx = s_sph[(pr.x * 3 + 0) * kWave + lane] - s_sph[(pr.y * 3 + 0) * kWave + lane];
    const float dy = s_sph[(pr.x * 3 + 1) * kWave + lane] - s_sph[(pr.y * 3 + 1) * kWave + lane];
    const float dz = s_sph[(pr.x * 3 + 2) * kWave + lane] - s_sph[(pr.y * 3 + 2) * kWave + lane];
    const float pen = __int_as_float(pr.w) - sqrtf(dx * dx + dy * dy + dz * dz);
    if (pen > bv) { bv = pen; bk = k; }
  }
  s_best[(w * 2 + 0) * kWave + lane] = bv;
  s_best[(w * 2 + 1) * kWave + lane] = __int_as_float(bk);
}

__device__ __forceinline__ void self_winner(int W, const float* s_best, int lane, float& bv, int& bk) {
  bv = 0.0f;
  bk = -1;
  for (int w = 0; w < W; ++w) {
    const float v = s_best[(w * 2 + 0) * kWave + lane];
    const int k = __float_as_int(s_best[(w * 2 + 1) * kWave + lane]);
    if (v > bv || (v == bv && k >= 0 && (bk < 0 || k < bk))) { bv = v; bk = k; }
  }
}

// Pose of link l: the chain from the root, joint by joint (Tab.6: fixed
// transform, then the rotation about z), from the chain records staged in
// LDS.  The next joint's record and joint value are read while the current
// joint's arithmetic runs.  visit(i, c, T) sees the pose after chain
// position i, whose joint is c.
template <typename QV, typename VIS>
__device__ __forceinline__ void chain_fk(const float4* rec, int depth, int row, QV&& qval, float* T,
                                         VIS&& visit) {
  identity(T);
  if (depth <= 0) return;
  float4 f0 = rec[0], f1 = rec[1], f2 = rec[2];
  int c = __float_as_int(rec[3].x);
  float q = qval(row, c);
  for (int i = 0; i < depth; ++i) {
    float4 g0 = f0, g1 = f1, g2 = f2;
    int cn = c;
    float qn = q;
    if (i + 1 < depth) {
      const float4* r = rec + 4 * (i + 1);
      g0 = r[0]; g1 = r[1]; g2 = r[2];
      cn = __float_as_int(r[3].x);
      qn = qval(row, cn);
    }
    const float sn = __sinf(q), cs = __cosf(q);
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const float t0 = T[r * 4 + 0], t1 = T[r * 4 + 1], t2 = T[r * 4 + 2], t3 = T[r * 4 + 3];
      const float u0 = t0 * f0.x + t1 * f1.x + t2 * f2.x;
      const float u1 = t0 * f0.y + t1 * f1.y + t2 * f2.y;
      T[r * 4 + 2] = t0 * f0.z + t1 * f1.z + t2 * f2.z;
      T[r * 4 + 3] = t0 * f0.w + t1 * f1.w + t2 * f2.w + t3;
      // then Rz(q): the first two columns mix
      T[r * 4 + 0] = u0 * cs + u1 * sn;
      T[r * 4 + 1] = u1 * cs - u0 * sn;
    }
    visit(i, c, T);
    f0 = g0; f1 = g1; f2 = g2;
    c = cn;
    q = qn;
  }
}

// World collision of one link wave's spheres against a staged tile of nb
// cuboids (Eq.(10)/(11), summed over cuboids and spheres).  Per cuboid, the
// wave's ball (centre cw, radius Rw, scalar) decides whether the wave looks
// at it; for one that passes, each lane's own ball (centre b, radius rl)
// must reach it; then the slots' face tests and, where one passes, the near
// path.  rho: each slot's cull radius (r + eta, plus half the longer
// segment with swept collision).
//
// Swept collision (SW): the lane's link poses at the neighbouring waypoints
// and its slots' spheres in the link frame (for the trace, Alg.11-12).
// ws: each slot's collision weight (w_coll, times the sphere's speed under
// the speed metric of Eq.(11)).
struct SweepCtx {
  const float* Tp;
  const float* Tn;
  const float4* sl;        // this lane's first slot (LDS)
  int steps;
  bool on, has_next;
};

// SP (speed metric): ws holds each slot's speed; the pair's cost and
// gradient are formed at weight w0 (w_coll), summed per slot into dsl (the
// slot's collision cost before the speed) and scaled by the speed.
// GRAD = false (cost-only launches): distances and costs alone, no gradient.
template <int MAXS, bool SW, bool SP, bool GRAD>
__device__ __forceinline__ void world_tile(const float4* tile, int nb, int lane, float cwx, float cwy,
                                           float cwz, float Rw, float bx, float by, float bz, float rl,
                                           const float* cx, const float* cy, const float* cz,
                                           const float* rr, const float* rho, const SweepCtx& sw, const float* ws,
                                           float w0, float* dsl, float eta, float inv_eta, float& cost, float& mc,
                                           float& Fx, float& Fy, float& Fz, float& Mx, float& My, float& Mz) {
  // lane j tests cuboid j of the tile against the wave's ball
  bool cand = false;
  if (lane < nb) {
    const float4 B0 = tile[4 * lane + 0], B1 = tile[4 * lane + 1];
    const float4 B2 = tile[4 * lane + 2], BH = tile[4 * lane + 3];
    const float px = fmaf(B0.x, cwx, fmaf(B0.y, cwy, fmaf(B0.z, cwz, B0.w)));
    const float py = fmaf(B1.x, cwx, fmaf(B1.y, cwy, fmaf(B1.z, cwz, B1.w)));
    const float pz = fmaf(B2.x, cwx, fmaf(B2.y, cwy, fmaf(B2.z, cwz, B2.w)));
    const float m3 = fmaxf(fabsf(px) - BH.x, fmaxf(fabsf(py) - BH.y, fabsf(pz) - BH.z));
    cand = m3 < Rw;
  }
  // (the mask made scalar, so the candidate index is too)
  const uint64_t bal = __ballot(cand);
  uint64_t mask = ((uint64_t)__builtin_amdgcn_readfirstlane((unsigned)(bal >> 32)) << 32) |
                  (unsigned)__builtin_amdgcn_readfirstlane((unsigned)bal);
  if (!mask) return;
  // the next candidate is read one iteration ahead
  int ob = __builtin_ctzll(mask);
  mask &= mask - 1;
  v4f nA0, nA1, nA2, nH;
  {
    const float4 q0 = tile[4 * ob + 0], q1 = tile[4 * ob + 1], q2 = tile[4 * ob + 2], q3 = tile[4 * ob + 3];
    nA0 = {q0.x, q0.y, q0.z, q0.w}; nA1 = {q1.x, q1.y, q1.z, q1.w};
    nA2 = {q2.x, q2.y, q2.z, q2.w}; nH = {q3.x, q3.y, q3.z, q3.w};
  }
  bool more = true;
  while (more) {
    const v4f A0 = nA0, A1 = nA1, A2 = nA2, Hh = nH;
    more = mask != 0;
    if (more) {
      ob = __builtin_ctzll(mask);
      mask &= mask - 1;
      const float4 q0 = tile[4 * ob + 0], q1 = tile[4 * ob + 1], q2 = tile[4 * ob + 2], q3 = tile[4 * ob + 3];
      nA0 = {q0.x, q0.y, q0.z, q0.w}; nA1 = {q1.x, q1.y, q1.z, q1.w};
      nA2 = {q2.x, q2.y, q2.z, q2.w}; nH = {q3.x, q3.y, q3.z, q3.w};
    }
    // second level: this lane's own ball; the wave skips the cuboid when no
    // lane's ball reaches it
    {
      const float px = fmaf(A0.x, bx, fmaf(A0.y, by, fmaf(A0.z, bz, A0.w)));
      const float py = fmaf(A1.x, bx, fmaf(A1.y, by, fmaf(A1.z, bz, A1.w)));
      const float pz = fmaf(A2.x, bx, fmaf(A2.y, by, fmaf(A2.z, bz, A2.w)));
      const float mb = fmaxf(fabsf(px) - Hh.x, fmaxf(fabsf(py) - Hh.y, fabsf(pz) - Hh.z));
      if (__ballot(mb < rl) == 0) continue;
    }
    // slots in groups of at most 8: face tests, then the near path of the
    // group (bounds the live face-test results)
    // (the box-frame points of the group stay live for the near path)
    constexpr int G = MAXS < 8 ? MAXS : 8;
#pragma unroll
    for (int g0 = 0; g0 < MAXS; g0 += G) {
      float m3[G], ppx[G], ppy[G], ppz[G];
      bool any = false;
#pragma unroll
      for (int u = 0; u < G; ++u) {
        const int s = g0 + u;
        ppx[u] = fmaf(A0.x, cx[s], fmaf(A0.y, cy[s], fmaf(A0.z, cz[s], A0.w)));
        ppy[u] = fmaf(A1.x, cx[s], fmaf(A1.y, cy[s], fmaf(A1.z, cz[s], A1.w)));
        ppz[u] = fmaf(A2.x, cx[s], fmaf(A2.y, cy[s], fmaf(A2.z, cz[s], A2.w)));
        m3[u] = fmaxf(fabsf(ppx[u]) - Hh.x, fmaxf(fabsf(ppy[u]) - Hh.y, fabsf(ppz[u]) - Hh.z));
        any |= m3[u] < rho[s];
      }
      if (any) {
#pragma unroll
        for (int u = 0; u < G; ++u) {
          const int s = g0 + u;
          if (!GRAD && m3[u] < rho[s]) {
            // cost only: the distance, the profile, the clearance
            const float px = ppx[u], py = ppy[u], pz = ppz[u];
            float cs = 0.0f;
            float& cacc = SP ? cs : cost;
            const float wp = SP ? w0 : ws[s];
            const float sdf = box_dist(fabsf(px) - Hh.x, fabsf(py) - Hh.y, fabsf(pz) - Hh.z);
            mc = fminf(mc, sdf - rr[s]);
            dc_cost(sdf, rr[s], wp, eta, inv_eta, cacc);
            // (every trace sample lies within the slot's half segment of its
            // centre: beyond the cull radius none reaches the band)
            if (SW && sw.on && sdf < rho[s])
              sweep_pair_cost(sw.sl[s], sw.steps, sw.Tp, sw.Tn, sw.has_next, cx[s], cy[s], cz[s], A0, A1, A2, Hh,
                              px, py, pz, sdf, rr[s], wp, eta, inv_eta, cacc);
            if constexpr (SP) {
              dsl[s] += cs;
              cost = fmaf(ws[s], cs, cost);
            }
          } else if (GRAD && m3[u] < rho[s]) {
            const float px = ppx[u], py = ppy[u], pz = ppz[u];
            float gx = 0.0f, gy = 0.0f, gz = 0.0f;
            float cs = 0.0f;
            float& cacc = SP ? cs : cost;
            const float wp = SP ? w0 : ws[s];
            if constexpr (SW) {
              // the pair's samples (its own and the trace's) sum their
              // gradients in the box frame, rotated back to the world once
              float gpx, gpy, gpz, bgx = 0.0f, bgy = 0.0f, bgz = 0.0f;
              const float sdf = box_sdf(px, py, pz, fabsf(px) - Hh.x, fabsf(py) - Hh.y, fabsf(pz) - Hh.z, gpx,
                                        gpy, gpz);
              mc = fminf(mc, sdf - rr[s]);
              dc_term_box(sdf, gpx, gpy, gpz, rr[s], wp, eta, inv_eta, cacc, bgx, bgy, bgz);
              if (sw.on && sdf < rho[s])
                sweep_pair_box(sw.sl[s], sw.steps, sw.Tp, sw.Tn, sw.has_next, cx[s], cy[s], cz[s], A0, A1, A2,
                               Hh, px, py, pz, sdf, rr[s], wp, eta, inv_eta, cacc, bgx, bgy, bgz);
              gx = A0.x * bgx + A1.x * bgy + A2.x * bgz;
              gy = A0.y * bgx + A1.y * bgy + A2.y * bgz;
              gz = A0.z * bgx + A1.z * bgy + A2.z * bgz;
            } else {
              near_pair(A0, A1, A2, px, py, pz, fabsf(px) - Hh.x, fabsf(py) - Hh.y, fabsf(pz) - Hh.z, rr[s], wp,
                        eta, inv_eta, cacc, mc, gx, gy, gz);
            }
            if constexpr (SP) {
              dsl[s] += cs;
              cost = fmaf(ws[s], cs, cost);
              gx *= ws[s]; gy *= ws[s]; gz *= ws[s];
            }
            Fx += gx; Fy += gy; Fz += gz;
            Mx += cy[s] * gz - cz[s] * gy;
            My += cz[s] * gx - cx[s] * gz;
            Mz += cx[s] * gy - cy[s] * gx;
          }
        }
      }
    }
  }
}

// The value of the lane that holds the other half of this lane's chain: lane
// i +- 32 with two slot groups, i +- 16 with four (groups g and g ^ 1 split
// one evaluation's chain).  Every lane takes part in the swap.
template <int G>
__device__ __forceinline__ float chain_partner(float v, int lane) {
  if constexpr (G == 4) {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_int(v), __float_as_int(v), false, false);
    return __int_as_float((lane & 16) ? (int)r[0] : (int)r[1]);
  } else {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_int(v), __float_as_int(v), false, false);
    return __int_as_float(lane < 32 ? (int)r[1] : (int)r[0]);
  }
}
// This lane's slot-group ball among a link's kWlBalls.
template <int G>
__device__ __forceinline__ int group_ball(int g) {
  return G == 4 ? 3 + g : G == 2 ? 1 + g : 0;
}

// Sum / minimum over the G slot groups of a wave (lanes e, e + E, ...).
template <int G>
__device__ __forceinline__ float groups_sum(float v) {
  if (G >= 4) v = swap16_sum(v);
  if (G >= 2) v = swap32_sum(v);
  return v;
}
template <int G>
__device__ __forceinline__ float groups_min(float v) {
  if (G >= 4) v = swap16_min(v);
  if (G >= 2) v = swap32_min(v);
  return v;
}

// NT: launch bound, 512 threads for robots of up to 7 links (register
// budget of two waves per SIMD), else 1024.  G: slot groups per wave; a
// workgroup holds E = 64 / G evaluations and lane g * E + e tests group g
// of the link's sphere slots for evaluation e (G = 2, 4: G times the
// workgroups for the same batch; groups g and g ^ 1 split the chain).
// SW: the chain also runs at the neighbouring waypoints, for swept
// collision and the speed metric; SP: the speed metric (Eq.(11)).
// LP: link passes (HS = 1, more links than link waves); without it the
// pass loop runs once and compiles away (the register budget of the
// one-pass kernel stays what it was).
struct NoFuse {};

// FS > 0 (cost and gradient of candidates, link waves alone, no swept
// collision or speed metric): the previous iteration's line-search choice
// and next L-BFGS direction (FA = SelFuse) are computed first, by the joint
// wave while the others stage, for the seed of the workgroup's rows (whose
// chunk lies within one seed); the new iterate and direction become the
// staged rows.  FS is the candidate count padded to 4 or 8.
template <int MAXS, bool CAND, bool GRAD, int NT, int G, bool SW, bool SP, bool LP, int FS, typename FA>
__device__ __forceinline__ void eval_wl_body(const EvalArgs& a, const FA& fa) {
  static_assert(FS == 0 || (CAND && GRAD && !SW && !SP && !LP), "the choice folds into line-search evaluations");
  constexpr int E = kWave / G;
  extern __shared__ float s_mem[];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int lane = threadIdx.x % kWave;
  const int g = lane / E, el = lane % E;
  warm_kernargs<sizeof(EvalArgs)>();
  // (FS: the choice's arguments follow; brought in with the same round)
  constexpr int fs_off = (int)((sizeof(EvalArgs) + alignof(SelFuse) - 1) / alignof(SelFuse) * alignof(SelFuse));
  static_assert(sizeof(SelFuse) <= 512, "the choice's arguments fit one warm-up");
  if constexpr (FS > 0) warm_kernargs<(int)sizeof(SelFuse), fs_off>();
  const int tid = threadIdx.x;
  const int L = a.rb.n_links, D = a.rb.dof, K = a.K, n_ee = a.rb.n_ee;
  const int maxd = a.wl.max_depth, maxs = a.wl.maxs;
  // (FS: chunks in XCD-sized runs -- workgroups go to the 8 XCDs in turn,
  // so workgroup b takes chunk (b mod 8) n/8 + b/8 and a seed's chunks share
  // one XCD's L2 for the choice's reads; any permutation is correct)
  const int nbx = gridDim.x;
  const int bx = FS > 0 && nbx % 8 == 0 ? (int)(blockIdx.x % 8) * (nbx / 8) + (int)(blockIdx.x / 8) : (int)blockIdx.x;
  // cuboid slice of this workgroup (gridDim.y slices share a chunk)
  const int h = __builtin_amdgcn_readfirstlane(blockIdx.y), H = __builtin_amdgcn_readfirstlane(gridDim.y);
  // waves: link waves and one for the joint terms (HS = 1), or two per link
  // with half of its spheres each (HS = 2, robots of up to 8 links).  With
  // HS = 1 there are LW <= L link waves: link wave w takes links w, w + LW,
  // ... in passes (a workgroup of at most 8 waves keeps the register budget
  // of two waves per SIMD for a longer robot)
  const int HS = a.wl.halves;
  const int LW = HS == 2 ? 2 * L : (LP ? a.wl.link_waves : L);
  const int W = HS == 2 ? 2 * L : LW + 1;
  const int npass = LP ? (L + LW - 1) / LW : 1;
  const int nthreads = W * kWave;   // (the launch's block: no read of the dispatch packet)
  const bool joint_w = HS == 1 && wave == W - 1;
  const bool sel_w = FS > 0 && joint_w;    // (the joint wave computes the choice)

  // ---- everything is read from memory in two dependent rounds: the
  //      chunk's record and this wave's tables (scalar loads), then the
  //      workgroup's staging into LDS; after that only LDS is read ----
  // (one problem: the record follows from the workgroup index, one memory
  // round fewer)
  v4i c0, c1;
  if (a.wl.one.S > 0) {
    c0 = v4i{0, bx * E, a.wl.one.S, a.wl.one.T};
    c1 = v4i{a.wl.one.box_lo, a.wl.one.box_hi, 0, a.wl.one.n_e};
  } else {
    c0 = ((cv4i*)(a.wl.chunk + bx))[0];
    c1 = ((cv4i*)(a.wl.chunk + bx))[1];
  }
  const int p = c0.x, e_first = c0.y;
  Problem pb;
  pb.S = c0.z; pb.T = c0.w; pb.world = 0; pb.row0 = c1.z;
  pb.seed0 = 0; pb.pad0 = 0; pb.pad1 = 0; pb.pad2 = 0;
  const int box_lo = c1.x, box_hi = c1.y, n_e = c1.w;
  // (this wave's first link: its tables are read with the chunk record)
  const int l0 = HS == 2 ? wave >> 1 : min(wave, L - 1);
  v4i info = *(cv4i*)(a.wl.info + l0);
  // (the ball of this lane's slot group: all slots, or half of them)
  v4f bl = *(cv4f*)(a.wl.ball + l0 * kWlBalls + (HS == 2 ? 1 + (wave & 1) : group_ball<G>(g)));
  // subtree masks of the joints this wave gathers (wave and wave + W), read
  // with the first round
  const int jsub0 = ((cint*)a.wl.joint_rec)[2 * min(wave, D - 1) + 1];
  const int jsub1 = LP ? ((cint*)a.wl.joint_rec)[2 * min(wave + W, D - 1) + 1] : 0;

  const int e0 = e_first + el;
  const bool valid = e0 < n_e;
  const int e = valid ? e0 : n_e - 1;
  const int rl = e / K, k = e - rl * K;       // candidates of a row side by side
  const int t = rl % pb.T;
  const int row = pb.row0 + rl;
  const float alpha = CAND ? a.alpha[k < kMaxK ? k : 0] : 0.0f;

  // particle mode (cost only): candidate k of row r is clip(x + sqrt(var) eps_k)
  // with the draws eps_k = d + k d_stride (Alg.5); var is staged in d's place
  const bool pm = CAND && !GRAD && a.var != nullptr;
  const int pm_rows = pm ? a.wl.pm_rows : 0;
  const WlLds o = wl_lds_layout(L, D, maxd, a.rb.n_spheres, a.pr.n_self > 0, HS, maxs, E, pm_rows);
  float* s_x = s_mem + o.x;
  float* s_d = s_mem + o.d;
  float* s_lim = s_mem + o.lim;               // lower, upper, start
  float* s_goal = s_mem + o.goal;
  float* s_etf = s_mem + o.etf;
  float4* s_chain = reinterpret_cast<float4*>(s_mem + o.chain);
  float4* s_slot = reinterpret_cast<float4*>(s_mem + o.slot);
  float4* s_box = reinterpret_cast<float4*>(s_mem + o.box);   // two tiles
  int* s_tick = reinterpret_cast<int*>(s_mem + o.tick);
  float* s_eps = s_mem + o.eps;

  // the workgroup's rows and the four on either side (the stencils' reach)
  const int e_last = min(n_e, e_first + E) - 1;
  const int p_end = pb.row0 + pb.S * pb.T;
  const int r_lo = max(pb.row0, pb.row0 + e_first / K - 4);
  const int r_hi = min(p_end - 1, pb.row0 + e_last / K + 4);
  const int n_st = (r_hi - r_lo + 1) * D;
  // this workgroup's cuboids, staged a tile at a time
  const int per = (box_hi - box_lo + H - 1) / H;
  const int w0 = min(box_hi, box_lo + h * per), w1 = min(box_hi, w0 + per);
  {
    // scalars: rows of x (and d, or var), limits, start, goals, tool
    // transforms, and in particle mode each lane's draws over the rows
    const int nxd = FS > 0 ? 0 : (CAND ? 2 * n_st : n_st);
    const int n_eps = pm && a.d ? min(r_hi - r_lo + 1, pm_rows) * E * D : 0;
    const int nf = nxd + 3 * D + n_ee * 19 + n_eps;
    const float* dsrc = pm ? a.var : a.d;
    auto fsrc = [&](int i, float*& dst) -> const float* {
      if (i < (FS > 0 ? 0 : n_st)) { dst = s_x + i; return a.x + (size_t)r_lo * D + i; }
      if (i < nxd) { dst = s_d + (i - n_st); return dsrc + (size_t)r_lo * D + (i - n_st); }
      i -= nxd;
      if (i < n_eps) {
        // item (row rr, lane ee, joint j): lane ee's particle at row r_lo + rr
        dst = s_eps + i;
        const int rr = i / (E * D), rem = i - rr * (E * D), ee = rem / D, j = rem - ee * D;
        const int ke = min(e_first + ee, n_e - 1) % K;
        return a.d + (size_t)ke * a.d_stride + (size_t)(r_lo + rr) * D + j;
      }
      i -= n_eps;
      if (i < D) { dst = s_lim + i; return a.rb.q_lo + i; }
      if (i < 2 * D) { dst = s_lim + i; return a.rb.q_hi + (i - D); }
      if (i < 3 * D) { dst = s_lim + i; return a.q_start + (size_t)p * D + (i - 2 * D); }
      i -= 3 * D;
      if (i < n_ee * 7) { dst = s_goal + i; return a.goal + (size_t)p * n_ee * 7 + i; }
      i -= n_ee * 7;
      dst = s_etf + i;
      return a.rb.ee_tf + i;
    };
    // float4: chain records (the first maxd of every link), sphere slots,
    // the first cuboid tile
    const int nch = L * maxd * 4, nsl = L * maxs;
    const int nb0 = min(kWlBoxTile, w1 - w0);
    const int n4 = nch + nsl + 4 * max(nb0, 0);
    auto f4src = [&](int i) -> const float4* {
      if (i < nch) {
        const int lk = i / (maxd * 4), rem = i - lk * (maxd * 4);
        return a.wl.chain_rec + (size_t)lk * kMaxDof * 4 + rem;
      }
      if (i < nch + nsl) return a.wl.sphere + (i - nch);
      return reinterpret_cast<const float4*>(a.box + w0) + (i - nch - nsl);
    };
    // every load of a pass is issued before its LDS stores (with FS the
    // joint wave stages nothing: it is the last wave)
    const int st_n = FS > 0 ? nthreads - kWave : nthreads;
    for (int b0 = 0; !sel_w && (b0 < nf || b0 < n4); b0 += 2 * st_n) {
      const int i0 = b0 + tid, i1 = i0 + st_n;
      float* d0 = nullptr;
      float* d1 = nullptr;
      const float v0 = i0 < nf ? *fsrc(i0, d0) : 0.0f;
      const float v1 = i1 < nf ? *fsrc(i1, d1) : 0.0f;
      const float4 u0 = i0 < n4 ? *f4src(i0) : float4{};
      const float4 u1 = i1 < n4 ? *f4src(i1) : float4{};
      if (i0 < nf) *d0 = v0;
      if (i1 < nf) *d1 = v1;
      if (i0 < n4) s_chain[i0] = u0;
      if (i1 < n4) s_chain[i1] = u1;
    }
    if (pm && !a.d) {
      // each lane's draws over the staged rows, made here: one Philox block
      // gives elements 4q .. 4q + 3 of the flattened [rows][D] range
      const int nr = min(r_hi - r_lo + 1, pm_rows);
      const long long e_lo = (long long)r_lo * D, e_hi = e_lo + (long long)nr * D;
      const long long q_lo = e_lo >> 2, nq = ((e_hi + 3) >> 2) - q_lo;
      for (long long i = tid; i < nq * E; i += nthreads) {
        const int ee = (int)(i / nq);
        const long long q = q_lo + (i - (long long)ee * nq);
        const int ke = min(e_first + ee, n_e - 1) % K;
        float w4[4];
        philox_draws4(a.pm_seed, ke, a.pm_it, (uint64_t)q, w4);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const long long e = 4 * q + u;
          if (e < e_lo || e >= e_hi) continue;
          const int rr = (int)((e - e_lo) / D), j = (int)(e - e_lo - (long long)rr * D);
          s_eps[(rr * E + ee) * D + j] = w4[u];
        }
      }
    }
    if constexpr (FS > 0) {
      if (sel_w) {
        const int T = pb.T;
        const int rl0 = e_first / K;                  // (the chunk's first row in its problem)
        const int srow0 = pb.row0 + rl0 - rl0 % T;    // the seed's first row
        const bool writer = rl0 % T == 0 && h == 0;   // the seed's first workgroup stores
        float xo[4], qo[4];
        select_seed<4, 4, true, FS, true, kWave>(fa.sa, fa.la, srow0 / T, lane, 0, writer, xo, qo);
        const int n = T * D, sh = (r_lo - srow0) * D;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int e = lane * 4 + u, i = e - sh;
          if (e < n && i >= 0 && i < n_st) {
            s_x[i] = xo[u];
            s_d[i] = qo[u];
          }
        }
      }
    }
  }
  __syncthreads();
  auto qval = [&](int r, int j) -> float {
    const int i = (r - r_lo) * D + j;
    float v = s_x[i];
    if (CAND) {
      if (pm) v = fmaf(sqrtf(s_d[i]), s_eps[((r - r_lo) * E + el) * D + j], v);
      else v = fmaf(alpha, s_d[i], v);
      v = fminf(fmaxf(v, s_lim[j]), s_lim[D + j]);
    }
    return v;
  };

  // parts: quantity q of evaluation el at part[q * E + el]; per link
  // cost, clearance, directional derivative, own joint's terms, the wrench
  // (F, M about the world origin) and the link frame's z axis and origin
  float* s_part = s_mem;
  constexpr int NPL = kWlPartsPerLink;
  float* s_joint = s_part + (size_t)L * NPL * E;
  float* s_ex = s_joint + (size_t)(3 + D) * E;

  // one pass over this wave's link (LP: one per link of the wave in turn)
  auto link_pass = [&](const int pass) {
  const int lp = HS == 2 ? wave >> 1 : wave + pass * LW;
  const bool link_w = HS == 2 ? wave < 2 * L : (LP ? wave < LW && lp < L : wave < L);
  const int l = link_w ? lp : 0, hs = HS == 2 ? wave & 1 : 0;
  if (LP && pass > 0 && link_w) {
    info = *(cv4i*)(a.wl.info + l);
    bl = *(cv4f*)(a.wl.ball + l * kWlBalls + group_ball<G>(g));
  }
  float* part = link_w ? s_part + (size_t)l * NPL * E : s_joint;
  if (LP && pass > 0) {
    // the first cuboid tile again (the previous pass's tiles overwrote it)
    __syncthreads();
    const int nb0 = min(kWlBoxTile, w1 - w0);
    for (int i = tid; i < 4 * nb0; i += nthreads) s_box[i] = reinterpret_cast<const float4*>(a.box + w0)[i];
    __syncthreads();
  }

  // ---- link waves: forward kinematics along the chain, the pose term,
  //      this wave's sphere slots ----
  const int depth = info.x, ee = info.z;
  const int sg = HS == 2 ? hs : g;                        // this lane's slot group
  const int ns = min(max(info.y - sg * MAXS, 0), MAXS);   // and its slots
  const float4* rec = s_chain + (size_t)l * maxd * 4;
  float T[12];
  float cost = 0.0f, mc = a.pr.eta;
  float Fx = 0.0f, Fy = 0.0f, Fz = 0.0f, Mx = 0.0f, My = 0.0f, Mz = 0.0f;
  float cx[MAXS], cy[MAXS], cz[MAXS], rr[MAXS], rho[MAXS];
  float wx = 0.0f, wy = 0.0f, wz = 0.0f, vx = 0.0f, vy = 0.0f, vz = 0.0f;
  // swept collision: the link's poses at the neighbouring waypoints (the
  // start before waypoint 1; one waypoint alone has no segments)
  // SW also carries the speed metric (Eq.(11)): each sphere's collision
  // cost times |c(t+1) - c(t-1)| / (2 dt), the start before waypoint 1 and
  // waypoint T after T; the speed's own gradient, on the neighbouring
  // waypoints, is added by speed_adjoint_kernel from the per-sphere terms
  // written below (sp_h)
  float Tp[SW ? 12 : 1], Tn[SW ? 12 : 1];
  const bool sweep = SW && a.pr.swept && pb.T > 1;
  const bool spd = SP && a.pr.speed;
  const bool nxt = t + 1 < pb.T;
  const bool has_next = sweep && nxt;
  float ws[MAXS];    // each slot's collision weight (SP: its speed)
  float dsl[SP ? MAXS : 1];   // SP: each slot's collision cost before the speed
#pragma unroll
  for (int s = 0; s < MAXS; ++s) ws[s] = SP ? 0.0f : a.pr.w_coll;
#pragma unroll
  for (int s = 0; s < (SP ? MAXS : 1); ++s) dsl[s] = 0.0f;
  float ext = 0.0f;   // the largest half segment over this lane's slots
  if (link_w) {
    // With CAND and GRAD the pass also forms the link's velocity under the
    // joint rates d (omega = sum d_c z_c, v = sum d_c o_c x z_c over its
    // chain): its share of the directional derivative is M . omega + F . v.
    const int xr = (row - r_lo) * D;
    auto twist = [&](int, int c, const float* P) {
      if (CAND && GRAD) {
        const float dc = s_d[xr + c];
        const float zx = P[2], zy = P[6], zz = P[10], ox = P[3], oy = P[7], oz = P[11];
        wx = fmaf(dc, zx, wx); wy = fmaf(dc, zy, wy); wz = fmaf(dc, zz, wz);
        vx = fmaf(dc, oy * zz - oz * zy, vx);
        vy = fmaf(dc, oz * zx - ox * zz, vy);
        vz = fmaf(dc, ox * zy - oy * zx, vz);
      }
    };
    auto none = [](int, int, const float*) {};
    // the link's pose at joint values qv into To; with G > 1 the slot groups
    // g and g ^ 1 split the chain: the even one composes its first half
    // (world frame), the odd one the rest from the identity; the halves are
    // swapped and both form the same product P0 P1 (tw: the velocity is
    // formed as well)
    auto link_fk = [&](auto&& qv, float* To, auto&& vis, bool tw) {
      if constexpr (G >= 2) {
        const int odd = g & 1;
        const int split = (depth + 1) >> 1;
        float Pp[12];
        chain_fk(rec + (odd ? 4 * split : 0), odd ? depth - split : split, row, qv, Pp, vis);
        float Po[12];
#pragma unroll
        for (int e = 0; e < 12; ++e) Po[e] = chain_partner<G>(Pp[e], lane);
        const float* P0 = odd ? Po : Pp;
        const float* P1 = odd ? Pp : Po;
#pragma unroll
        for (int r = 0; r < 3; ++r) {
          const float a0 = P0[r * 4 + 0], a1 = P0[r * 4 + 1], a2 = P0[r * 4 + 2], a3 = P0[r * 4 + 3];
          To[r * 4 + 0] = a0 * P1[0] + a1 * P1[4] + a2 * P1[8];
          To[r * 4 + 1] = a0 * P1[1] + a1 * P1[5] + a2 * P1[9];
          To[r * 4 + 2] = a0 * P1[2] + a1 * P1[6] + a2 * P1[10];
          To[r * 4 + 3] = a0 * P1[3] + a1 * P1[7] + a2 * P1[11] + a3;
        }
        if (CAND && GRAD && tw) {
          // group 1's velocity is in P0's frame: omega_1 = R0 omega_1',
          // v_1 = R0 v_1' + p0 x omega_1
          // (the other group's values are fetched by every lane first: a
          // conditional operator evaluates only the operand it selects, and
          // a lane swap inside one would run with half the wave inactive)
          const float ox_[6] = {chain_partner<G>(wx, lane), chain_partner<G>(wy, lane), chain_partner<G>(wz, lane),
                                chain_partner<G>(vx, lane), chain_partner<G>(vy, lane), chain_partner<G>(vz, lane)};
          float w1[3] = {odd ? wx : ox_[0], odd ? wy : ox_[1], odd ? wz : ox_[2]};
          float u1[3] = {odd ? vx : ox_[3], odd ? vy : ox_[4], odd ? vz : ox_[5]};
          float w0[3] = {odd ? ox_[0] : wx, odd ? ox_[1] : wy, odd ? ox_[2] : wz};
          float u0[3] = {odd ? ox_[3] : vx, odd ? ox_[4] : vy, odd ? ox_[5] : vz};
          float Rw[3], Ru[3];
#pragma unroll
          for (int r = 0; r < 3; ++r) {
            Rw[r] = P0[r * 4 + 0] * w1[0] + P0[r * 4 + 1] * w1[1] + P0[r * 4 + 2] * w1[2];
            Ru[r] = P0[r * 4 + 0] * u1[0] + P0[r * 4 + 1] * u1[1] + P0[r * 4 + 2] * u1[2];
          }
          const float px = P0[3], py = P0[7], pz = P0[11];
          wx = w0[0] + Rw[0]; wy = w0[1] + Rw[1]; wz = w0[2] + Rw[2];
          vx = u0[0] + Ru[0] + (py * Rw[2] - pz * Rw[1]);
          vy = u0[1] + Ru[1] + (pz * Rw[0] - px * Rw[2]);
          vz = u0[2] + Ru[2] + (px * Rw[1] - py * Rw[0]);
        }
      } else {
        chain_fk(rec, depth, row, qv, To, vis);
      }
    };
    link_fk(qval, T, twist, true);
    if constexpr (SW) {
      if (sweep || spd) {
        auto qprev = [&](int r, int j) -> float { return t >= 1 ? qval(r - 1, j) : s_lim[2 * D + j]; };
        auto qnext = [&](int r, int j) -> float { return nxt ? qval(r + 1, j) : qval(r, j); };
        link_fk(qprev, Tp, none, false);
        link_fk(qnext, Tn, none, false);
      }
    }
    if (ee >= 0 && sg == 0 && h == 0 && t == pb.T - 1)
      pose_term_at(a, s_etf + ee * 12, s_goal + ee * 7, ee, T, valid ? row : -1, cost, Fx, Fy, Fz, Mx, My, Mz);
    const float eta = a.pr.eta;
#pragma unroll
    for (int s = 0; s < MAXS; ++s) {
      const float4 ls = s_slot[l * maxs + sg * MAXS + (s < ns ? s : 0)];
      const bool used = s < ns;
      // unused slots sit far away and never pass the face test
      cx[s] = used ? T[0] * ls.x + T[1] * ls.y + T[2] * ls.z + T[3] : 1e18f;
      cy[s] = used ? T[4] * ls.x + T[5] * ls.y + T[6] * ls.z + T[7] : 1e18f;
      cz[s] = used ? T[8] * ls.x + T[9] * ls.y + T[10] * ls.z + T[11] : 1e18f;
      rr[s] = used ? ls.w : 0.0f;
      rho[s] = rr[s] + eta;
      if constexpr (SW) {
        if (spd && used) {
          const float ux = (Tn[0] - Tp[0]) * ls.x + (Tn[1] - Tp[1]) * ls.y + (Tn[2] - Tp[2]) * ls.z + (Tn[3] - Tp[3]);
          const float uy = (Tn[4] - Tp[4]) * ls.x + (Tn[5] - Tp[5]) * ls.y + (Tn[6] - Tp[6]) * ls.z + (Tn[7] - Tp[7]);
          const float uz = (Tn[8] - Tp[8]) * ls.x + (Tn[9] - Tp[9]) * ls.y + (Tn[10] - Tp[10]) * ls.z + (Tn[11] - Tp[11]);
          ws[s] = sqrtf(ux * ux + uy * uy + uz * uz) * (0.5f / a.pr.dt);
        }
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
          const float e = 0.5f * sqrtf(l2) * 1.0001f + 1e-6f;
          rho[s] += e;
          ext = fmaxf(ext, e);
        }
      }
    }
  }

  // ---- self-collision (Eq.(9)), first slice only: sphere centres and
  //      per-wave winners share the parts' space ----
  float jc = 0.0f;    // the joint wave's cost
  if (G == 1 && a.pr.n_self > 0 && h == 0) {
    float* s_sph = s_part;
    float* s_best = s_sph + (size_t)a.rb.n_spheres * 3 * kWave;
    if (link_w) {
      cint* sm = (cint*)(a.wl.slot_sphere + l * maxs + hs * MAXS);
#pragma unroll
      for (int s = 0; s < MAXS; ++s)
        if (s < ns) {
          const int m = sm[s];
          s_sph[(m * 3 + 0) * kWave + lane] = cx[s];
          s_sph[(m * 3 + 1) * kWave + lane] = cy[s];
          s_sph[(m * 3 + 2) * kWave + lane] = cz[s];
        }
    }
    __syncthreads();
    self_pairs_phase(a, wave, W, s_sph, s_best, lane);
    __syncthreads();
    float bv;
    int bk;
    self_winner(W, s_best, lane, bv, bk);
    if (!link_w) jc += a.pr.w_self * bv;                        // the joint wave (one pass)
    if (HS == 2 && l == 0 && hs == 1) cost += a.pr.w_self * bv;  // (no joint wave)
    if (link_w && bk >= 0) {
      const int4 pr = reinterpret_cast<const int4*>(a.wl.self_pairs)[bk];
      // owners: link and slot position of each sphere (this wave holds
      // positions hs * MAXS .. hs * MAXS + MAXS - 1 of its link)
      const int li = pr.z & 0xff, lj = (pr.z >> 8) & 0xff;
      const bool own_i = li == l && ((pr.z >> 16) & 0xff) / MAXS == hs;
      const bool own_j = lj == l && ((pr.z >> 24) & 0xff) / MAXS == hs;
      if (own_i || own_j) {
        const float xi = s_sph[(pr.x * 3 + 0) * kWave + lane], yi = s_sph[(pr.x * 3 + 1) * kWave + lane];
        const float zi = s_sph[(pr.x * 3 + 2) * kWave + lane];
        const float xj = s_sph[(pr.y * 3 + 0) * kWave + lane], yj = s_sph[(pr.y * 3 + 1) * kWave + lane];
        const float zj = s_sph[(pr.y * 3 + 2) * kWave + lane];
        const float ux = xi - xj, uy = yi - yj, uz = zi - zj;
        const float d = sqrtf(ux * ux + uy * uy + uz * uz);
        if (d > 0.0f) {
          // d cost / d x_i = -w (x_i - x_j) / d, the opposite on x_j
          const float f = -a.pr.w_self / d;
          const float fx = f * ux, fy = f * uy, fz = f * uz;
          if (own_i) {
            Fx += fx; Fy += fy; Fz += fz;
            Mx += yi * fz - zi * fy; My += zi * fx - xi * fz; Mz += xi * fy - yi * fx;
          }
          if (own_j) {
            Fx -= fx; Fy -= fy; Fz -= fz;
            Mx -= yj * fz - zj * fy; My -= zj * fx - xj * fz; Mz -= xj * fy - yj * fx;
          }
        }
      }
    }
    __syncthreads();   // the spheres' space becomes the parts' space
  }

  // ---- the joint wave (HS = 1): joint limits (Eq.(17)) and smoothness
  //      (Eq.(16)) of joints j = h mod H ----
  //      (slot group g takes joints g, g + G, ...)
  // (written as !link_w so that the compiler sees the link-wave and
  // joint-wave paths exclude each other and shares their registers)
  if (!link_w && (!LP || (joint_w && pass == 0))) {
    float gdj = 0.0f;
    for (int j0 = 0; j0 < D; j0 += G) {
      const int j = j0 + g;
      if (j < D) {
        float js = 0.0f;
        if (j % H == h)
          joint_terms(a, pb, row, t, j, qval(row, j), s_lim[j], s_lim[D + j], s_lim[2 * D + j], qval, jc, js);
        part[(3 + j) * E + el] = js;
        if (CAND) gdj = fmaf(js, s_d[(row - r_lo) * D + j], gdj);
      }
    }
    jc = groups_sum<G>(jc);
    gdj = groups_sum<G>(gdj);
    if (g == 0) {
      part[0 * E + el] = jc;
      part[1 * E + el] = a.pr.eta;
      part[2 * E + el] = gdj;
    }
  }

  // ---- world collision, a staged tile of cuboids at a time; the next
  //      tile is read into registers while this one is tested ----
  const float eta = a.pr.eta, inv_eta = 1.0f / fmaxf(eta, 1e-30f);
  float cwx = 0.0f, cwy = 0.0f, cwz = 0.0f, Rw = 0.0f, bxl = 0.0f, byl = 0.0f, bzl = 0.0f, rlb = 0.0f;
  // (wave-uniform: the wave has a sphere in some slot group; a lane whose
  // group has none tests unused slots, which never pass)
  const bool wave_sph = link_w && (HS == 2 ? ns > 0 : info.y > 0);
  if (wave_sph) {
    // ball around the wave's spheres of every lane: centre of the lanes'
    // bounding box of ball centres, radius half its diagonal + ball radius
    bxl = T[0] * bl.x + T[1] * bl.y + T[2] * bl.z + T[3];
    byl = T[4] * bl.x + T[5] * bl.y + T[6] * bl.z + T[7];
    bzl = T[8] * bl.x + T[9] * bl.y + T[10] * bl.z + T[11];
    const float lx = wave_min(bxl), ux = wave_max(bxl);
    const float ly = wave_min(byl), uy = wave_max(byl);
    const float lz = wave_min(bzl), uz = wave_max(bzl);
    cwx = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(0.5f * (lx + ux))));
    cwy = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(0.5f * (ly + uy))));
    cwz = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(0.5f * (lz + uz))));
    const float hx = ux - lx, hy = uy - ly, hz = uz - lz;
    // (widened slightly so rounding never drops a cuboid that matters)
    const float rb = bl.w + ext;   // (ext: the sweep's reach, 0 without)
    const float rw = (0.5f * sqrtf(hx * hx + hy * hy + hz * hz) + (G > 1 || SW ? wave_max(rb) : rb) + eta) * 1.0001f +
                     1e-6f;
    Rw = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(rw)));
    rlb = (bl.w + eta) * 1.0001f + 1e-6f + ext;   // one lane's ball
  }
  SweepCtx swc;
  swc.Tp = Tp;
  swc.Tn = Tn;
  swc.sl = s_slot + l * maxs + sg * MAXS;
  swc.steps = a.pr.sweep_steps;
  swc.on = sweep;
  swc.has_next = has_next;
  for (int tl = w0, buf = 0; tl < w1; tl += kWlBoxTile, buf ^= 1) {
    const int nb = min(kWlBoxTile, w1 - tl);
    const int nn = min(kWlBoxTile, w1 - tl - kWlBoxTile);   // next tile (<= 0: none)
    const float4* nsrc = reinterpret_cast<const float4*>(a.box + tl + kWlBoxTile);
    const int i0 = tid, i1 = tid + nthreads;   // 2 x 64 threads cover a tile
    const float4 u0 = i0 < 4 * nn ? nsrc[i0] : float4{};
    const float4 u1 = i1 < 4 * nn ? nsrc[i1] : float4{};
    if (wave_sph)
      world_tile<MAXS, SW, SP, GRAD>(s_box + buf * kWlBoxTile * 4, nb, lane, cwx, cwy, cwz, Rw, bxl, byl, bzl, rlb, cx,
                               cy, cz, rr, rho, swc, ws, a.pr.w_coll, dsl, eta, inv_eta, cost, mc, Fx, Fy, Fz, Mx, My,
                               Mz);
    if (nn <= 0) break;
    float4* nxt = s_box + (buf ^ 1) * kWlBoxTile * 4;
    if (i0 < 4 * nn) nxt[i0] = u0;
    if (i1 < 4 * nn) nxt[i1] = u1;
    __syncthreads();
  }

  if constexpr (SP && GRAD) {
    // the speed's gradient acts on the neighbouring waypoints: each sphere's
    // collision cost times its unit chord / (2 dt), for speed_adjoint_kernel
    // (every sphere has one slot, so the sums are whole; one slice only)
    if (spd && link_w && valid && a.sp_h) {
      const size_t hb = ((size_t)k * a.rows + row) * a.rb.n_spheres;
#pragma unroll
      for (int s = 0; s < MAXS; ++s)
        if (s < ns) {
          const float4 ls = s_slot[l * maxs + sg * MAXS + s];
          const float ux = (Tn[0] - Tp[0]) * ls.x + (Tn[1] - Tp[1]) * ls.y + (Tn[2] - Tp[2]) * ls.z + (Tn[3] - Tp[3]);
          const float uy = (Tn[4] - Tp[4]) * ls.x + (Tn[5] - Tp[5]) * ls.y + (Tn[6] - Tp[6]) * ls.z + (Tn[7] - Tp[7]);
          const float uz = (Tn[8] - Tp[8]) * ls.x + (Tn[9] - Tp[9]) * ls.y + (Tn[10] - Tp[10]) * ls.z + (Tn[11] - Tp[11]);
          const float un = sqrtf(ux * ux + uy * uy + uz * uz);
          const float f = un > 0.0f ? dsl[s] * (0.5f / a.pr.dt) / un : 0.0f;
          const int m = a.wl.slot_sphere[l * maxs + sg * MAXS + s];
          a.sp_h[hb + m] = float4{f * ux, f * uy, f * uz, 0.0f};
        }
    }
  }

  if (G > 1 && link_w) {
    // the slot groups' sums meet in every lane of the evaluation
    cost = groups_sum<G>(cost);
    mc = groups_min<G>(mc);
    Fx = groups_sum<G>(Fx); Fy = groups_sum<G>(Fy); Fz = groups_sum<G>(Fz);
    Mx = groups_sum<G>(Mx); My = groups_sum<G>(My); Mz = groups_sum<G>(Mz);
  }

  // ---- two waves per link: the second adds joint l's own terms (l < D)
  //      and hands its sums to the first ----
  float own_js = 0.0f;
  if (HS == 2) {
    float* ex = s_ex + (size_t)l * 9 * E;
    if (hs == 1) {
      float js = 0.0f;
      if (l < D)
        joint_terms(a, pb, row, t, l, qval(row, l), s_lim[l], s_lim[D + l], s_lim[2 * D + l], qval, cost, js);
      ex[0 * E + el] = cost;
      ex[1 * E + el] = mc;
      ex[2 * E + el] = Fx; ex[3 * E + el] = Fy; ex[4 * E + el] = Fz;
      ex[5 * E + el] = Mx; ex[6 * E + el] = My; ex[7 * E + el] = Mz;
      ex[8 * E + el] = js;
    }
    __syncthreads();
    if (hs == 0) {
      cost += ex[0 * E + el];
      mc = fminf(mc, ex[1 * E + el]);
      Fx += ex[2 * E + el]; Fy += ex[3 * E + el]; Fz += ex[4 * E + el];
      Mx += ex[5 * E + el]; My += ex[6 * E + el]; Mz += ex[7 * E + el];
      own_js = ex[8 * E + el];
    }
  }

  // ---- the link's sums, wrench and frame (Alg.8 without a second pass
  //      along the chain: joint c's derivative is z_c . (M - o_c x F)
  //      summed over the links below it, formed by the gathering wave) ----
  if (link_w && hs == 0 && g == 0) {
    float gdp = 0.0f;
    if (CAND && GRAD) {
      gdp = Mx * wx + My * wy + Mz * wz + (Fx * vx + Fy * vy + Fz * vz);
      if (HS == 2 && l < D) gdp = fmaf(own_js, s_d[(row - r_lo) * D + l], gdp);
    }
    part[0 * E + el] = cost;
    part[1 * E + el] = mc;
    part[2 * E + el] = gdp;
    part[3 * E + el] = own_js;
    if (GRAD) {
      part[4 * E + el] = Fx; part[5 * E + el] = Fy; part[6 * E + el] = Fz;
      part[7 * E + el] = Mx; part[8 * E + el] = My; part[9 * E + el] = Mz;
      part[10 * E + el] = T[2]; part[11 * E + el] = T[6]; part[12 * E + el] = T[10];
      part[13 * E + el] = T[3]; part[14 * E + el] = T[7]; part[15 * E + el] = T[11];
    }
  }
  };
  if constexpr (LP) {
    for (int pass = 0; pass < npass; ++pass) link_pass(pass);
  } else {
    link_pass(0);
  }
  __syncthreads();

  // ---- combine: wave j < D forms joint j's derivative from the wrenches
  //      of the links whose chain holds it (summed in link order) and link
  //      j's frame; the last wave sums cost, clearance and directional
  //      derivative over the links in order, then the joint wave's ----
  //      (wave w gathers joints w, w + W: a workgroup of W >= D / 2 waves)
  const size_t eo = (size_t)k * a.rows + row;
  constexpr int NJ = LP ? 2 : 1;   // joints gathered per wave
  float gsv[2] = {0.0f, 0.0f};
#pragma unroll
  for (int qj = 0; qj < NJ; ++qj) {
    const int jj = wave + qj * W;
    if (!GRAD || jj >= D) continue;
    const int jsub = qj == 0 ? jsub0 : jsub1;
    const float* pj = s_part + (size_t)jj * NPL * E + el;
    float gsum = HS == 1 ? s_joint[(3 + jj) * E + el] : pj[3 * E];
    float sF[3] = {0.0f, 0.0f, 0.0f}, sM[3] = {0.0f, 0.0f, 0.0f};
    for (int v = 0; v < L; ++v) {
      const float* pv = s_part + (size_t)v * NPL * E + el;
      const bool in = (jsub >> v) & 1;
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const float f = pv[(4 + q) * E], m = pv[(7 + q) * E];
        sF[q] += in ? f : 0.0f;
        sM[q] += in ? m : 0.0f;
      }
    }
    const float zx = pj[10 * E], zy = pj[11 * E], zz = pj[12 * E];
    const float ox = pj[13 * E], oy = pj[14 * E], oz = pj[15 * E];
    const float ux = sM[0] - (oy * sF[2] - oz * sF[1]);
    const float uy = sM[1] - (oz * sF[0] - ox * sF[2]);
    const float uz = sM[2] - (ox * sF[1] - oy * sF[0]);
    gsv[qj] = gsum + (zx * ux + zy * uy + zz * uz);
  }
  float tc = 0.0f, tm = 3.0e38f, tg = 0.0f;
  if (wave == W - 1) {
    for (int v = 0; v < L; ++v) {
      tc += s_part[((size_t)v * NPL + 0) * E + el];
      tm = fminf(tm, s_part[((size_t)v * NPL + 1) * E + el]);
      tg += s_part[((size_t)v * NPL + 2) * E + el];
    }
    if (HS == 1) {
      tc += s_joint[0 * E + el];
      tm = fminf(tm, s_joint[1 * E + el]);
      tg += s_joint[2 * E + el];
    }
  }
  if (G == 1 && H > 1) {
    // park this slice's sums; the last workgroup of the chunk to arrive
    // adds the slices in slice order (deterministic whatever the arrival
    // order) and finishes the evaluation.  (Agent-scope atomic accesses:
    // the slices may run on different XCDs, whose L2 caches are not
    // coherent with each other.)
    const int NP = 3 + D;
    const size_t cbase = (size_t)bx * H * NP * kWave;
    float* mine = a.wl.part + cbase + (size_t)h * NP * kWave;
#pragma unroll
    for (int qj = 0; qj < NJ; ++qj)
      if (GRAD && wave + qj * W < D) part_store(mine + (3 + wave + qj * W) * kWave + lane, gsv[qj]);
    if (wave == W - 1) {
      part_store(mine + 0 * kWave + lane, tc);
      part_store(mine + 1 * kWave + lane, tm);
      part_store(mine + 2 * kWave + lane, tg);
    }
    __threadfence();
    __syncthreads();
    if (wave == 0) {
      int ticket = 0;
      if (lane == 0) ticket = atomicAdd(a.wl.count + bx, 1);
      ticket = __shfl(ticket, 0, kWave);
      if (lane == 0) s_tick[0] = ticket;
    }
    __syncthreads();
    const int ticket = __builtin_amdgcn_readfirstlane(s_tick[0]);
    if (ticket != H - 1) return;
    __threadfence();
    if (wave == 0 && lane == 0) __hip_atomic_store(a.wl.count + bx, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
    for (int qj = 0; qj < NJ; ++qj)
      if (GRAD && wave + qj * W < D) {
        float gsum = 0.0f;
        for (int u = 0; u < H; ++u)
          gsum += part_load(a.wl.part + cbase + ((size_t)u * NP + 3 + wave + qj * W) * kWave + lane);
        gsv[qj] = gsum;
      }
    if (wave == W - 1) {
      tc = 0.0f; tm = 3.0e38f; tg = 0.0f;
      for (int u = 0; u < H; ++u) {
        const float* pu = a.wl.part + cbase + (size_t)u * NP * kWave;
        tc += part_load(pu + 0 * kWave + lane);
        tm = fminf(tm, part_load(pu + 1 * kWave + lane));
        tg += part_load(pu + 2 * kWave + lane);
      }
    }
  }
  if (!valid || g != 0) return;
#pragma unroll
  for (int qj = 0; qj < NJ; ++qj)
    if (GRAD && wave + qj * W < D) a.grad_e[eo * D + wave + qj * W] = gsv[qj];
  if (wave == W - 1) {
    a.cost_e[eo] = tc;
    if (a.mc_e) a.mc_e[eo] = tm;
    if (CAND && GRAD) a.gd_e[eo] = tg;
  }
}

template <int MAXS, bool CAND, bool GRAD, int NT, int G, bool SW, bool SP, bool LP>
__global__ __launch_bounds__(NT) void eval_wl_kernel(const EvalArgs a) {
  eval_wl_body<MAXS, CAND, GRAD, NT, G, SW, SP, LP, 0>(a, NoFuse{});
}

template <int MAXS, int G, int FS>
__global__ __launch_bounds__(512) void eval_wl_fs_kernel(const EvalArgs a, const SelFuse f) {
  eval_wl_body<MAXS, true, true, 512, G, false, false, false, FS>(a, f);
}

// Launch one instantiation; more than 64 KB of LDS needs the kernel's
// dynamic-LDS limit raised first.
template <typename KF, typename... Args>
hipError_t wl_launch(KF kern, dim3 grid, dim3 block, size_t lds, hipStream_t s, const Args&... args) {
  if (lds > 64 * 1024) {
    const hipError_t e =
        hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  kern<<<grid, block, lds, s>>>(args...);
  return hipGetLastError();
}

template <int MAXS, int G, bool SW, bool SP>
hipError_t wl_pick(const EvalArgs& a, dim3 grid, dim3 block, size_t lds, int waves, bool cand, bool grad,
                   hipStream_t s, const SelFuse* fs) {
  if (fs) {
    if constexpr (MAXS <= 8 && !SW && !SP) {
      if (a.wl.halves != 1 || a.wl.link_waves < a.rb.n_links || waves > 8 || !cand || !grad)
        return hipErrorInvalidValue;
      if (fs->sa.K <= 4) return wl_launch(eval_wl_fs_kernel<MAXS, G, 4>, grid, block, lds, s, a, *fs);
      return wl_launch(eval_wl_fs_kernel<MAXS, G, 8>, grid, block, lds, s, a, *fs);
    }
    return hipErrorInvalidValue;
  }
  if (a.wl.halves == 1 && a.wl.link_waves < a.rb.n_links) {
    // link passes: at most 8 waves by construction
    if (waves > 8) return hipErrorInvalidValue;
    if (cand && grad) return wl_launch(eval_wl_kernel<MAXS, true, true, 512, G, SW, SP, true>, grid, block, lds, s, a);
    if (grad) return wl_launch(eval_wl_kernel<MAXS, false, true, 512, G, SW, SP, true>, grid, block, lds, s, a);
    if (!cand) return wl_launch(eval_wl_kernel<MAXS, false, false, 512, G, SW, SP, true>, grid, block, lds, s, a);
    return wl_launch(eval_wl_kernel<MAXS, true, false, 512, G, SW, SP, true>, grid, block, lds, s, a);
  }
  if (waves <= 8) {
    if (cand && grad) return wl_launch(eval_wl_kernel<MAXS, true, true, 512, G, SW, SP, false>, grid, block, lds, s, a);
    if (grad) return wl_launch(eval_wl_kernel<MAXS, false, true, 512, G, SW, SP, false>, grid, block, lds, s, a);
    if (!cand) return wl_launch(eval_wl_kernel<MAXS, false, false, 512, G, SW, SP, false>, grid, block, lds, s, a);
    return wl_launch(eval_wl_kernel<MAXS, true, false, 512, G, SW, SP, false>, grid, block, lds, s, a);
  }
  if (cand && grad) return wl_launch(eval_wl_kernel<MAXS, true, true, 1024, G, SW, SP, false>, grid, block, lds, s, a);
  if (grad) return wl_launch(eval_wl_kernel<MAXS, false, true, 1024, G, SW, SP, false>, grid, block, lds, s, a);
  if (!cand) return wl_launch(eval_wl_kernel<MAXS, false, false, 1024, G, SW, SP, false>, grid, block, lds, s, a);
  return wl_launch(eval_wl_kernel<MAXS, true, false, 1024, G, SW, SP, false>, grid, block, lds, s, a);
}

template <int MAXS, int G>
hipError_t launch_eval_wl_g(const EvalArgs& a, int grid_x, int slices, bool cand, bool grad, hipStream_t s,
                            const SelFuse* fs) {
  const int HS = a.wl.halves;
  const int L = a.rb.n_links;
  const int LW = a.wl.link_waves;
  const int waves = HS == 2 ? 2 * L : LW + 1;
  if (waves * kWave > 1024 || slices < 1 || ((HS == 2 || G > 1) && slices > 1)) return hipErrorInvalidValue;
  // link passes: every link covered, every joint gathered (two per wave at
  // most), self-collision in one pass only
  if (HS == 1 && (LW < 1 || LW > L || (LW < L ? 2 * waves : waves) < a.rb.dof || (a.pr.n_self > 0 && LW != L)))
    return hipErrorInvalidValue;
  if (G > 1 && (HS != 1 || a.pr.n_self > 0)) return hipErrorInvalidValue;
  if (slices > 1 && (!a.wl.part || !a.wl.count)) return hipErrorInvalidValue;
  // particle mode (per-candidate draws): cost only, draws staged per row
  const bool pm = a.var != nullptr;
  if (pm && (!cand || grad || a.K < 1 || a.wl.pm_rows < (kWave / G - 1) / a.K + 10 || a.wl.pm_rows > kWlStageRows))
    return hipErrorInvalidValue;
  // the joint gathers fit (two per wave), and two 64-thread passes cover a
  // cuboid tile
  if (a.rb.dof > 2 * waves || waves < 2 || !a.wl.chunk) return hipErrorInvalidValue;
  const size_t lds = wl_lds_bytes(a.rb.n_links, a.rb.dof, a.wl.max_depth, a.rb.n_spheres, a.pr.n_self > 0, HS,
                                  a.wl.maxs, kWave / G, pm ? a.wl.pm_rows : 0);
  if (lds > kWlLdsMax) return hipErrorInvalidValue;
  if (fs) {
    // the choice: uniform horizons, blocks of 129 to 256 floats moved as
    // float4 (four per lane), at most 8 candidates and 4 history pairs, and
    // every chunk of E / K rows inside one seed
    const SelectArgs& sa = fs->sa;
    const int T = sa.uniform_T, E = kWave / G, n = T * a.rb.dof;
    if (T < 1 || n <= 2 * kWave || n > 4 * kWave || n % 4 || sa.K != a.K || sa.K > 8 || E % sa.K || T % (E / sa.K) ||
        fs->la.m > 4 || fs->la.use_first || !fs->la.keep_prev || !fs->la.meta_out)
      return hipErrorInvalidValue;
  }
  const dim3 grid(grid_x, slices), block(waves * kWave);
  // SW: poses at the neighbouring waypoints (swept collision, the speed
  // metric); SP: the speed metric
  if (a.pr.speed) return wl_pick<MAXS, G, true, true>(a, grid, block, lds, waves, cand, grad, s, fs);
  if (a.pr.swept) return wl_pick<MAXS, G, true, false>(a, grid, block, lds, waves, cand, grad, s, fs);
  return wl_pick<MAXS, G, false, false>(a, grid, block, lds, waves, cand, grad, s, fs);
}

}  // namespace

// One compilation unit per (slots per lane, slot groups) so the variants
// compile in parallel: mg_eval_wl_s<MAXS>g<G>.hip.
#define MG_WL_LAUNCHER(S, G)                                                                         \
  hipError_t launch_eval_wl_s##S##g##G(const EvalArgs& a, int grid_x, int slices, bool cand, bool grad, \
                                       hipStream_t s, const SelFuse* fs)
MG_WL_LAUNCHER(2, 1);
MG_WL_LAUNCHER(4, 1);
MG_WL_LAUNCHER(8, 1);
MG_WL_LAUNCHER(16, 1);
MG_WL_LAUNCHER(2, 2);
MG_WL_LAUNCHER(4, 2);
MG_WL_LAUNCHER(8, 2);
MG_WL_LAUNCHER(2, 4);
MG_WL_LAUNCHER(4, 4);
}  // namespace mg
