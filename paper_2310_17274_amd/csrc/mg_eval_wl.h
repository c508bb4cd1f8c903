// mg_eval_wl.h -- the evaluation kernel in the wave-per-link layout.
//
// A workgroup holds 64 evaluations (lanes; candidates of consecutive
// waypoint rows of one seed side by side, so the lanes of a wave sit close
// together in configuration space).  Wave l owns link l: it runs the
// kinematic chain from the root to l (Tab.6 closed form per joint), places
// the link's spheres, and tests them against the world's cuboids; the last
// wave owns the joint-limit and smoothness terms of every joint.  Per
// cuboid, one test of a ball enclosing the link's spheres over all 64 lanes
// decides whether the wave looks at that cuboid at all (the distance is
// 1-Lipschitz, so a cuboid farther than the ball radius + eta from the
// ball's centre adds no cost and cannot lower the clamped clearance for any
// lane); for a cuboid that passes, each lane tests a ball around its own
// copy of the link's spheres, and the wave skips the cuboid when none
// reaches it.  The adjoint recomputes the chain (Alg.8: no stored transforms)
// and projects the link's wrench on every joint above it (Tab.7); the waves'
// partial sums meet in LDS in a fixed order.  The world's cuboids can also
// be split over gridDim.y workgroups of the same 64 evaluations (more
// workgroups for small batches); the last of them to finish adds the slices'
// sums in slice order.
#pragma once

#include "mg_eval.h"

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
// transform, then the rotation about z).  Each joint's record (fixed
// transform rows and joint index) is loaded one joint ahead, so the scalar
// loads overlap the previous joint's arithmetic.  visit(i, T) sees the pose
// after chain position i.
template <typename QV, typename VIS>
__device__ __forceinline__ void chain_fk(const EvalArgs& a, int l, int depth, int row, QV&& qval,
                                         float* T, VIS&& visit) {
  cv4f* rec = (cv4f*)(a.wl.chain_rec + (size_t)l * kMaxDof * 4);
  identity(T);
  v4f n0 = rec[0], n1 = rec[1], n2 = rec[2], n3 = rec[3];
  for (int i = 0; i < depth; ++i) {
    const v4f f0 = n0, f1 = n1, f2 = n2;
    const int c = __float_as_int(n3.x);
    if (i + 1 < depth) {
      n0 = rec[4 * (i + 1) + 0]; n1 = rec[4 * (i + 1) + 1];
      n2 = rec[4 * (i + 1) + 2]; n3 = rec[4 * (i + 1) + 3];
    }
    const float q = qval(row, c);
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
    visit(i, T);
  }
}

// Collision, pose and adjoint of link l for this lane's evaluation.
// part[q * kWave + lane]: q = 0 cost, 1 clearance, 2 + i d cost / d q of the
// joint at chain position i (root first).
// With HS = 2 a link has two waves, each with half of its sphere slots
// (hs = 0, 1); the second also owns joint l's limit and smoothness terms and
// hands its sums to the first (s_ex), which runs the adjoint.  Returns false
// for a wave whose part is handed over.
template <int MAXS, bool GRAD, typename QV>
__device__ __forceinline__ bool link_wave(const EvalArgs& a, int l, int hs, int HS, int p,
                                          const Problem& pb, int row, int t, bool valid, int h, int H,
                                          QV&& qval, float* part, int lane, bool self_on, float* s_sph,
                                          float* s_best, int W, float* s_ex, const float* s_lim) {
  // per-link tables through the constant address space (wave-uniform)
  const v4i info = *(cv4i*)(a.wl.info + l);
  const int depth = info.x, ee = info.z;
  const int sbase = l * a.wl.maxs + hs * MAXS;          // this wave's first slot
  const int ns = min(max(info.y - hs * MAXS, 0), MAXS);  // and how many it has

  // ---- forward kinematics along the chain ----
  float T[12];
  chain_fk(a, l, depth, row, qval, T, [](int, const float*) {});

  float cost = 0.0f, mc = a.pr.eta;
  float Fx = 0.0f, Fy = 0.0f, Fz = 0.0f, Mx = 0.0f, My = 0.0f, Mz = 0.0f;
  if (ee >= 0 && hs == 0 && h == 0 && t == pb.T - 1)
    pose_term(a, p, ee, T, valid ? row : -1, cost, Fx, Fy, Fz, Mx, My, Mz);

  // ---- the link's spheres (this wave's share) ----
  cv4f* sph = (cv4f*)(a.wl.sphere + sbase);
  float cx[MAXS], cy[MAXS], cz[MAXS], rr[MAXS];
#pragma unroll
  for (int s = 0; s < MAXS; ++s) {
    const v4f ls = sph[s];
    const bool used = s < ns;
    // unused slots sit far away and never pass the face test
    cx[s] = used ? T[0] * ls.x + T[1] * ls.y + T[2] * ls.z + T[3] : 1e18f;
    cy[s] = used ? T[4] * ls.x + T[5] * ls.y + T[6] * ls.z + T[7] : 1e18f;
    cz[s] = used ? T[8] * ls.x + T[9] * ls.y + T[10] * ls.z + T[11] : 1e18f;
    rr[s] = used ? ls.w : 0.0f;
  }

  // ---- self-collision (Eq.(9)): the winning pair's forces on this link ----
  if (self_on) {
    cint* sm = (cint*)(a.wl.slot_sphere + sbase);
#pragma unroll
    for (int s = 0; s < MAXS; ++s)
      if (s < ns) {
        const int m = sm[s];
        s_sph[(m * 3 + 0) * kWave + lane] = cx[s];
        s_sph[(m * 3 + 1) * kWave + lane] = cy[s];
        s_sph[(m * 3 + 2) * kWave + lane] = cz[s];
      }
    __syncthreads();
    self_pairs_phase(a, l * HS + hs, W, s_sph, s_best, lane);
    __syncthreads();
    float bv;
    int bk;
    self_winner(W, s_best, lane, bv, bk);
    if (HS == 2 && l == 0 && hs == 1) cost += a.pr.w_self * bv;   // (no joint wave)
    if (bk >= 0) {
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

  // ---- world collision of the link's spheres, cuboid slice h of H ----
  const int wa = ((cint*)a.world_off)[pb.world], wb = ((cint*)a.world_off)[pb.world + 1];
  const int per = (wb - wa + H - 1) / H;
  const int w0 = min(wb, wa + h * per), w1 = min(wb, w0 + per);
  if (ns > 0 && w1 > w0) {
    const float w = a.pr.w_coll, eta = a.pr.eta, inv_eta = 1.0f / fmaxf(eta, 1e-30f);
    // ball around the link's spheres of every lane: centre of the lanes'
    // bounding box of ball centres, radius half its diagonal + ball radius
    const v4f bl = *(cv4f*)(a.wl.ball + l * 3 + (HS == 2 ? 1 + hs : 0));
    const float bx = T[0] * bl.x + T[1] * bl.y + T[2] * bl.z + T[3];
    const float by = T[4] * bl.x + T[5] * bl.y + T[6] * bl.z + T[7];
    const float bz = T[8] * bl.x + T[9] * bl.y + T[10] * bl.z + T[11];
    const float lx = wave_min(bx), ux = wave_max(bx);
    const float ly = wave_min(by), uy = wave_max(by);
    const float lz = wave_min(bz), uz = wave_max(bz);
    const float cwx = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(0.5f * (lx + ux))));
    const float cwy = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(0.5f * (ly + uy))));
    const float cwz = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(0.5f * (lz + uz))));
    const float hx = ux - lx, hy = uy - ly, hz = uz - lz;
    // (widened slightly so rounding never drops a cuboid that matters)
    const float rw = (0.5f * sqrtf(hx * hx + hy * hy + hz * hz) + bl.w + eta) * 1.0001f + 1e-6f;
    const float Rw = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(rw)));
    const float rl = (bl.w + eta) * 1.0001f + 1e-6f;   // one lane's ball

    cv4f* boxes = (cv4f*)(a.box);
    for (int base = w0; base < w1; base += kWave) {
      // lane j tests cuboid base + j against the wave's ball
      const int o = base + lane;
      bool cand = false;
      if (o < w1) {
        const float4* bq = reinterpret_cast<const float4*>(a.box + o);
        const float4 B0 = bq[0], B1 = bq[1], B2 = bq[2], BH = bq[3];
        const float px = fmaf(B0.x, cwx, fmaf(B0.y, cwy, fmaf(B0.z, cwz, B0.w)));
        const float py = fmaf(B1.x, cwx, fmaf(B1.y, cwy, fmaf(B1.z, cwz, B1.w)));
        const float pz = fmaf(B2.x, cwx, fmaf(B2.y, cwy, fmaf(B2.z, cwz, B2.w)));
        const float m3 = fmaxf(fabsf(px) - BH.x, fmaxf(fabsf(py) - BH.y, fabsf(pz) - BH.z));
        cand = m3 < Rw;
      }
      // (the mask made scalar, so the candidate index and its loads are too)
      const uint64_t bal = __ballot(cand);
      uint64_t mask = ((uint64_t)__builtin_amdgcn_readfirstlane((unsigned)(bal >> 32)) << 32) |
                      (unsigned)__builtin_amdgcn_readfirstlane((unsigned)bal);
      // the next candidate's scalar loads are issued one iteration ahead
      v4f nA0 = {}, nA1 = {}, nA2 = {}, nH = {};
      if (mask) {
        const int ob = base + __builtin_ctzll(mask);
        nA0 = boxes[4 * ob + 0]; nA1 = boxes[4 * ob + 1];
        nA2 = boxes[4 * ob + 2]; nH = boxes[4 * ob + 3];
        mask &= mask - 1;
      }
      bool more = bal != 0;
      while (more) {
        const v4f A0 = nA0, A1 = nA1, A2 = nA2, Hh = nH;
        more = mask != 0;
        if (more) {
          const int ob = base + __builtin_ctzll(mask);
          nA0 = boxes[4 * ob + 0]; nA1 = boxes[4 * ob + 1];
          nA2 = boxes[4 * ob + 2]; nH = boxes[4 * ob + 3];
          mask &= mask - 1;
        }
        // second level: this lane's own ball; the wave skips the cuboid
        // when no lane's ball reaches it
        {
          const float px = fmaf(A0.x, bx, fmaf(A0.y, by, fmaf(A0.z, bz, A0.w)));
          const float py = fmaf(A1.x, bx, fmaf(A1.y, by, fmaf(A1.z, bz, A1.w)));
          const float pz = fmaf(A2.x, bx, fmaf(A2.y, by, fmaf(A2.z, bz, A2.w)));
          const float mb = fmaxf(fabsf(px) - Hh.x, fmaxf(fabsf(py) - Hh.y, fabsf(pz) - Hh.z));
          if (__ballot(mb < rl) == 0) continue;
        }
        // slots in groups of at most 8: face tests, then the near path of
        // the group (bounds the live face-test results)
        constexpr int G = MAXS < 8 ? MAXS : 8;
#pragma unroll
        for (int g0 = 0; g0 < MAXS; g0 += G) {
        float m3[G];
        bool any = false;
#pragma unroll
        for (int u = 0; u < G; ++u) {
          const int s = g0 + u;
          const float px = fmaf(A0.x, cx[s], fmaf(A0.y, cy[s], fmaf(A0.z, cz[s], A0.w)));
          const float py = fmaf(A1.x, cx[s], fmaf(A1.y, cy[s], fmaf(A1.z, cz[s], A1.w)));
          const float pz = fmaf(A2.x, cx[s], fmaf(A2.y, cy[s], fmaf(A2.z, cz[s], A2.w)));
          m3[u] = fmaxf(fabsf(px) - Hh.x, fmaxf(fabsf(py) - Hh.y, fabsf(pz) - Hh.z));
          any |= m3[u] < rr[s] + eta;
        }
        if (any) {
#pragma unroll
          for (int u = 0; u < G; ++u) {
            const int s = g0 + u;
            if (m3[u] < rr[s] + eta) {
              const float px = fmaf(A0.x, cx[s], fmaf(A0.y, cy[s], fmaf(A0.z, cz[s], A0.w)));
              const float py = fmaf(A1.x, cx[s], fmaf(A1.y, cy[s], fmaf(A1.z, cz[s], A1.w)));
              const float pz = fmaf(A2.x, cx[s], fmaf(A2.y, cy[s], fmaf(A2.z, cz[s], A2.w)));
              float gx = 0.0f, gy = 0.0f, gz = 0.0f;
              near_pair(A0, A1, A2, px, py, pz, fabsf(px) - Hh.x, fabsf(py) - Hh.y, fabsf(pz) - Hh.z,
                        rr[s], w, eta, inv_eta, cost, mc, gx, gy, gz);
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
  }
  float own_js = 0.0f;
  if (HS == 2) {
    // the second wave adds joint l's own terms and hands its sums over
    float* ex = s_ex + (size_t)l * 9 * kWave;
    if (hs == 1) {
      float jc = 0.0f, js = 0.0f;
      joint_terms(a, pb, row, t, l, qval(row, l), s_lim[l], s_lim[a.rb.dof + l], s_lim[2 * a.rb.dof + l],
                  qval, jc, js);
      ex[0 * kWave + lane] = cost + jc;
      ex[1 * kWave + lane] = mc;
      ex[2 * kWave + lane] = Fx; ex[3 * kWave + lane] = Fy; ex[4 * kWave + lane] = Fz;
      ex[5 * kWave + lane] = Mx; ex[6 * kWave + lane] = My; ex[7 * kWave + lane] = Mz;
      ex[8 * kWave + lane] = js;
    }
    __syncthreads();
    if (hs == 1) return false;
    cost += ex[0 * kWave + lane];
    mc = fminf(mc, ex[1 * kWave + lane]);
    Fx += ex[2 * kWave + lane]; Fy += ex[3 * kWave + lane]; Fz += ex[4 * kWave + lane];
    Mx += ex[5 * kWave + lane]; My += ex[6 * kWave + lane]; Mz += ex[7 * kWave + lane];
    own_js = ex[8 * kWave + lane];
  }
  part[0 * kWave + lane] = cost;
  part[1 * kWave + lane] = mc;
  part[(2 + a.wl.max_depth) * kWave + lane] = own_js;

  // ---- adjoint: the chain again, joint c's derivative z_c . (M - o_c x F) ----
  if (GRAD) {
    chain_fk(a, l, depth, row, qval, T, [&](int i, const float* P) {
      const float zx = P[2], zy = P[6], zz = P[10], ox = P[3], oy = P[7], oz = P[11];
      const float vx = Mx - (oy * Fz - oz * Fy);
      const float vy = My - (oz * Fx - ox * Fz);
      const float vz = Mz - (ox * Fy - oy * Fx);
      part[(2 + i) * kWave + lane] = zx * vx + zy * vy + zz * vz;
    });
  }
  return true;
}

// NT: launch bound, 512 threads for robots of up to 7 links (register
// budget of two waves per SIMD), else 1024.
template <int MAXS, bool CAND, bool GRAD, int NT>
__global__ __launch_bounds__(NT) void eval_wl_kernel(const EvalArgs a) {
  extern __shared__ float s_part[];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int lane = threadIdx.x % kWave;
  const int L = a.rb.n_links, D = a.rb.dof, K = a.K;
  const int bx = blockIdx.x;
  int lo = 0, hi = a.P;
  cint* chunk_prefix = (cint*)a.chunk_prefix;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (chunk_prefix[mid] <= bx) lo = mid; else hi = mid;
  }
  // (the problem, its table row and everything derived from them are wave
  // uniform; reading them through the constant address space keeps them in
  // scalar registers, so the cuboid loop below runs on scalar loads)
  const int p = __builtin_amdgcn_readfirstlane(lo);
  Problem pb;
  {
    const v4i p0 = ((cv4i*)(a.prob + p))[0], p1 = ((cv4i*)(a.prob + p))[1];
    pb.S = p0.x; pb.T = p0.y; pb.world = p0.z; pb.row0 = p0.w;
    pb.seed0 = p1.x; pb.pad0 = p1.y; pb.pad1 = p1.z; pb.pad2 = p1.w;
  }
  const int n_e = pb.S * pb.T * K;
  const int e0 = (bx - chunk_prefix[p]) * kWave + lane;
  const bool valid = e0 < n_e;
  const int e = valid ? e0 : n_e - 1;
  const int rl = e / K, k = e - rl * K;       // candidates of a row side by side
  const int t = rl % pb.T;
  const int row = pb.row0 + rl;
  const float alpha = CAND ? a.alpha[k < kMaxK ? k : 0] : 0.0f;
  const float* dk = CAND ? a.d : nullptr;     // one direction for every candidate

  // waves: one per link and one for the joint terms (HS = 1), or two per
  // link with half of its spheres each (HS = 2, robots of up to 8 links)
  const int HS = a.wl.halves;
  const int W = HS == 2 ? 2 * L : L + 1;
  // LDS: the link parts (3 + deepest chain each: cost, clearance, the
  // chain's derivatives, the own joint's terms), the joint part (2 + D), the
  // halves' hand-over (9 per link), or, during the self-collision phase, the
  // sphere centres and winners; then the staged rows
  const int NP = 2 + D;
  const int NPL = 3 + a.wl.max_depth;
  float* s_joint = s_part + (size_t)L * NPL * kWave;
  float* s_ex = s_joint + (size_t)NP * kWave;

  // the workgroup's rows and the four on either side (the stencils' reach)
  // are staged in LDS once: every wave reads its joint values from there
  const int e_first = (bx - chunk_prefix[p]) * kWave;
  const int e_last = min(n_e, e_first + kWave) - 1;
  const int p_end = pb.row0 + pb.S * pb.T;
  const int r_lo = max(pb.row0, pb.row0 + e_first / K - 4);
  const int r_hi = min(p_end - 1, pb.row0 + e_last / K + 4);
  const int n_st = (r_hi - r_lo + 1) * D;
  float* s_x = s_part + wl_region_floats(L, D, a.wl.max_depth, a.rb.n_spheres, a.pr.n_self > 0, HS);
  float* s_d = s_x + kStageRows * D;
  // and the joint limits and the problem's start (lower, upper, start)
  float* s_lim = s_d + kStageRows * D;
  for (int i = threadIdx.x; i < n_st; i += blockDim.x) {
    s_x[i] = a.x[(size_t)r_lo * D + i];
    if (CAND) s_d[i] = dk[(size_t)r_lo * D + i];
  }
  for (int i = threadIdx.x; i < D; i += blockDim.x) {
    s_lim[i] = a.rb.q_lo[i];
    s_lim[D + i] = a.rb.q_hi[i];
    s_lim[2 * D + i] = a.q_start[(size_t)p * D + i];
  }
  __syncthreads();
  auto qval = [&](int r, int j) -> float {
    const int i = (r - r_lo) * D + j;
    float v = s_x[i];
    if (CAND) {
      v = fmaf(alpha, s_d[i], v);
      v = fminf(fmaxf(v, s_lim[j]), s_lim[D + j]);
    }
    return v;
  };

  // cuboid slice of this workgroup (gridDim.y slices share a chunk)
  const int h = __builtin_amdgcn_readfirstlane(blockIdx.y), H = __builtin_amdgcn_readfirstlane(gridDim.y);
  const int n_link_waves = L * HS;
  float* part = wave < n_link_waves ? s_part + (size_t)(wave / HS) * NPL * kWave : s_joint;
  // self-collision in the first slice: sphere centres and per-wave winners
  // follow the wave parts in LDS
  const bool self_on = a.pr.n_self > 0 && h == 0;
  float* s_sph = s_part;     // (shares the parts' space, see link_wave)
  float* s_best = s_sph + (size_t)a.rb.n_spheres * 3 * kWave;
  if (wave < n_link_waves) {
    link_wave<MAXS, GRAD>(a, wave / HS, wave % HS, HS, p, pb, row, t, valid, h, H, qval, part, lane,
                          self_on, s_sph, s_best, W, s_ex, s_lim);
  } else {
    float jc = 0.0f;
    if (self_on) {
      __syncthreads();
      self_pairs_phase(a, wave, W, s_sph, s_best, lane);
      __syncthreads();
      float bv;
      int bk;
      self_winner(W, s_best, lane, bv, bk);
      jc += a.pr.w_self * bv;
      __syncthreads();   // the spheres' space becomes the parts' space
    }
    // joint limits (Eq.(17)) and smoothness (Eq.(16)): joints j = h mod H
    for (int j = 0; j < D; ++j) {
      float js = 0.0f;
      if (j % H == h)
        joint_terms(a, pb, row, t, j, qval(row, j), s_lim[j], s_lim[D + j], s_lim[2 * D + j], qval, jc, js);
      part[(2 + j) * kWave + lane] = js;
    }
    part[0 * kWave + lane] = jc;
    part[1 * kWave + lane] = a.pr.eta;
  }
  __syncthreads();
  if (wave != W - 1) return;

  // ---- the last wave sums the waves' parts in a fixed order: links in
  //      order, then its own; joint derivatives gather into its part ----
  float cost = 0.0f, mc = 3.0e38f;
  for (int v = 0; v < L; ++v) {
    cost += s_part[(v * NPL + 0) * kWave + lane];
    mc = fminf(mc, s_part[(v * NPL + 1) * kWave + lane]);
  }
  if (HS == 1) {
    cost += s_joint[lane];
    mc = fminf(mc, s_joint[kWave + lane]);
  }
  if (GRAD) {
    // joint j sits at chain position pos_j of every link in its subtree;
    // its own terms come from the joint part (HS = 1) or link j's part
    cint* jrec = (cint*)(a.wl.joint_rec);
    for (int j = 0; j < D; ++j) {
      const int pos = jrec[2 * j], sub = jrec[2 * j + 1];
      float g = HS == 1 ? s_joint[(2 + j) * kWave + lane]
                        : s_part[(j * NPL + 2 + a.wl.max_depth) * kWave + lane];
#pragma unroll
      for (int v = 0; v < 15; ++v)
        if (v < L && ((sub >> v) & 1)) g += s_part[(v * NPL + 2 + pos) * kWave + lane];
      s_joint[(2 + j) * kWave + lane] = g;
    }
  }
  if (H > 1) {
    // park this slice's sums; the last workgroup of the chunk to arrive
    // adds the slices in slice order (deterministic whatever the arrival
    // order) and finishes the evaluation
    const size_t cbase = (size_t)bx * H * NP * kWave;
    float* mine = a.wl.part + cbase + (size_t)h * NP * kWave;
    // (agent-scope atomic accesses: the slices may run on different XCDs,
    // whose L2 caches are not coherent with each other)
    part_store(mine + 0 * kWave + lane, cost);
    part_store(mine + 1 * kWave + lane, mc);
    if (GRAD)
      for (int j = 0; j < D; ++j) part_store(mine + (2 + j) * kWave + lane, s_joint[(2 + j) * kWave + lane]);
    __threadfence();
    int ticket = 0;
    if (lane == 0) ticket = atomicAdd(a.wl.count + bx, 1);
    ticket = __shfl(ticket, 0, kWave);
    if (ticket != H - 1) return;
    __threadfence();
    if (lane == 0) __hip_atomic_store(a.wl.count + bx, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    cost = 0.0f;
    mc = 3.0e38f;
    for (int u = 0; u < H; ++u) {
      const float* pu = a.wl.part + cbase + (size_t)u * NP * kWave;
      cost += part_load(pu + lane);
      mc = fminf(mc, part_load(pu + kWave + lane));
    }
  }
  const size_t eo = (size_t)k * a.rows + row;
  float gd = 0.0f;
  if (GRAD) {
    for (int j = 0; j < D; ++j) {
      float g = 0.0f;
      if (H > 1) {
        const size_t cbase = (size_t)bx * H * NP * kWave;
        for (int u = 0; u < H; ++u)
          g += part_load(a.wl.part + cbase + ((size_t)u * NP + 2 + j) * kWave + lane);
      } else {
        g = s_joint[(2 + j) * kWave + lane];
      }
      if (valid) a.grad_e[eo * D + j] = g;
      if (CAND) gd = fmaf(g, s_d[(row - r_lo) * D + j], gd);
    }
  }
  if (valid) {
    a.cost_e[eo] = cost;
    if (a.mc_e) a.mc_e[eo] = mc;
    if (CAND && GRAD) a.gd_e[eo] = gd;
  }
}

template <int MAXS>
hipError_t launch_eval_wl_s(const EvalArgs& a, int grid_x, int slices, bool cand, bool grad, hipStream_t s) {
  const int HS = a.wl.halves;
  const int waves = HS == 2 ? 2 * a.rb.n_links : a.rb.n_links + 1;
  if (waves * kWave > 1024 || slices < 1 || (HS == 2 && slices > 1)) return hipErrorInvalidValue;
  if (slices > 1 && (!a.wl.part || !a.wl.count)) return hipErrorInvalidValue;
  // particle mode (per-candidate draws) is not staged in this layout
  if (a.var || a.d_stride) return hipErrorInvalidValue;
  const size_t lds = wl_lds_bytes(a.rb.n_links, a.rb.dof, a.wl.max_depth, a.rb.n_spheres, a.pr.n_self > 0, HS);
  if (lds > kWlLdsMax) return hipErrorInvalidValue;
  const dim3 grid(grid_x, slices), block(waves * kWave);
  if (waves <= 8) {
    if (cand && grad) eval_wl_kernel<MAXS, true, true, 512><<<grid, block, lds, s>>>(a);
    else if (grad) eval_wl_kernel<MAXS, false, true, 512><<<grid, block, lds, s>>>(a);
    else if (!cand) eval_wl_kernel<MAXS, false, false, 512><<<grid, block, lds, s>>>(a);
    else eval_wl_kernel<MAXS, true, false, 512><<<grid, block, lds, s>>>(a);
  } else {
    if (cand && grad) eval_wl_kernel<MAXS, true, true, 1024><<<grid, block, lds, s>>>(a);
    else if (grad) eval_wl_kernel<MAXS, false, true, 1024><<<grid, block, lds, s>>>(a);
    else if (!cand) eval_wl_kernel<MAXS, false, false, 1024><<<grid, block, lds, s>>>(a);
    else eval_wl_kernel<MAXS, true, false, 1024><<<grid, block, lds, s>>>(a);
  }
  return hipGetLastError();
}

}  // namespace
}  // namespace mg
