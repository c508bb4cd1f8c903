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

__device__ __forceinline__ void part_store(float* p, float v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ float part_load(const float* p) {
  return __hip_atomic_load(const_cast<float*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Collision, pose and adjoint of link l for this lane's evaluation.
// part[q * kWave + lane]: q = 0 cost, 1 clearance, 2 + j d cost / d q_j.
template <int MAXS, bool GRAD, typename QV>
__device__ __forceinline__ void link_wave(const EvalArgs& a, int l, int p, const Problem& pb, int row,
                                          int t, bool valid, int h, int H, QV&& qval, float* part,
                                          int lane) {
  const int D = a.rb.dof;
  // per-link tables through the constant address space (wave-uniform)
  const v4i info = *(cv4i*)(a.wl.info + l);
  const int depth = info.x, ns = info.y, ee = info.z;
  cint* chain = (cint*)(a.wl.chain + l * kMaxDof);

  // ---- forward kinematics along the chain ----
  float T[12];
  identity(T);
  for (int i = 0; i < depth; ++i) {
    const int c = chain[i];
    const float q = qval(row, c);
    compose_u(T, (cfloat*)(a.rb.fixed_tf + c * 12));
    rotz(T, __sinf(q), __cosf(q));
  }

  float cost = 0.0f, mc = a.pr.eta;
  float Fx = 0.0f, Fy = 0.0f, Fz = 0.0f, Mx = 0.0f, My = 0.0f, Mz = 0.0f;
  if (ee >= 0 && h == 0 && t == pb.T - 1)
    pose_term(a, p, ee, T, valid ? row : -1, cost, Fx, Fy, Fz, Mx, My, Mz);

  // ---- world collision of the link's spheres, cuboid slice h of H ----
  const int wa = a.world_off[pb.world], wb = a.world_off[pb.world + 1];
  const int per = (wb - wa + H - 1) / H;
  const int w0 = min(wb, wa + h * per), w1 = min(wb, w0 + per);
  if (ns > 0 && w1 > w0) {
    const float w = a.pr.w_coll, eta = a.pr.eta, inv_eta = 1.0f / fmaxf(eta, 1e-30f);
    cv4f* sph = (cv4f*)(a.wl.sphere + l * MAXS);
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
    // ball around the link's spheres of every lane: centre of the lanes'
    // bounding box of ball centres, radius half its diagonal + ball radius
    const v4f bl = *(cv4f*)(a.wl.ball + l);
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
      uint64_t mask = __ballot(cand);
      while (mask) {
        const int kk = __builtin_ctzll(mask);
        mask &= mask - 1;
        const int ob = base + kk;
        const v4f A0 = boxes[4 * ob + 0], A1 = boxes[4 * ob + 1];
        const v4f A2 = boxes[4 * ob + 2], Hh = boxes[4 * ob + 3];
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
  part[0 * kWave + lane] = cost;
  part[1 * kWave + lane] = mc;

  // ---- adjoint: the chain again, joint c's derivative z_c . (M - o_c x F) ----
  if (GRAD) {
    for (int j = 0; j < D; ++j) part[(2 + j) * kWave + lane] = 0.0f;
    identity(T);
    for (int i = 0; i < depth; ++i) {
      const int c = chain[i];
      const float q = qval(row, c);
      compose_u(T, (cfloat*)(a.rb.fixed_tf + c * 12));
      rotz(T, __sinf(q), __cosf(q));
      const float zx = T[2], zy = T[6], zz = T[10], ox = T[3], oy = T[7], oz = T[11];
      const float vx = Mx - (oy * Fz - oz * Fy);
      const float vy = My - (oz * Fx - ox * Fz);
      const float vz = Mz - (ox * Fy - oy * Fx);
      part[(2 + c) * kWave + lane] = zx * vx + zy * vy + zz * vz;
    }
  }
}

template <int MAXS, bool CAND, bool GRAD>
__global__ __launch_bounds__(1024) void eval_wl_kernel(const EvalArgs a) {
  extern __shared__ float s_part[];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int lane = threadIdx.x % kWave;
  const int L = a.rb.n_links, D = a.rb.dof, K = a.K;
  const int bx = blockIdx.x;
  int lo = 0, hi = a.P;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (a.chunk_prefix[mid] <= bx) lo = mid; else hi = mid;
  }
  const int p = lo;
  const Problem pb = a.prob[p];
  const int n_e = pb.S * pb.T * K;
  const int e0 = (bx - a.chunk_prefix[p]) * kWave + lane;
  const bool valid = e0 < n_e;
  const int e = valid ? e0 : n_e - 1;
  const int rl = e / K, k = e - rl * K;       // candidates of a row side by side
  const int t = rl % pb.T;
  const int row = pb.row0 + rl;
  const float alpha = CAND ? a.alpha[k < kMaxK ? k : 0] : 0.0f;
  const float* dk = CAND ? a.d + (size_t)k * a.d_stride : nullptr;
  auto qval = [&](int r, int j) -> float {
    const size_t i = (size_t)r * D + j;
    float v = a.x[i];
    if (CAND) {
      v = a.var ? fmaf(sqrtf(a.var[i]), dk[i], v) : fmaf(alpha, dk[i], v);
      v = fminf(fmaxf(v, a.rb.q_lo[j]), a.rb.q_hi[j]);
    }
    return v;
  };

  // cuboid slice of this workgroup (gridDim.y slices share a chunk)
  const int h = blockIdx.y, H = gridDim.y;
  const int NP = 2 + D;
  float* part = s_part + (size_t)wave * NP * kWave;
  if (wave < L) {
    link_wave<MAXS, GRAD>(a, wave, p, pb, row, t, valid, h, H, qval, part, lane);
  } else {
    // joint limits (Eq.(17)) and smoothness (Eq.(16)): joints j = h mod H
    float jc = 0.0f;
    for (int j = 0; j < D; ++j) {
      float js = 0.0f;
      if (j % H == h) joint_terms(a, pb, p, row, t, j, qval(row, j), qval, jc, js);
      part[(2 + j) * kWave + lane] = js;
    }
    part[0 * kWave + lane] = jc;
    part[1 * kWave + lane] = a.pr.eta;
  }
  __syncthreads();
  if (wave != L) return;

  // ---- the last wave sums the waves' parts in a fixed order ----
  float cost = 0.0f, mc = 3.0e38f;
  for (int v = 0; v <= L; ++v) {
    cost += s_part[(v * NP + 0) * kWave + lane];
    mc = fminf(mc, s_part[(v * NP + 1) * kWave + lane]);
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
      for (int j = 0; j < D; ++j) {
        float g = 0.0f;
        for (int v = 0; v <= L; ++v) g += s_part[(v * NP + 2 + j) * kWave + lane];
        part_store(mine + (2 + j) * kWave + lane, g);
      }
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
        for (int v = 0; v <= L; ++v) g += s_part[(v * NP + 2 + j) * kWave + lane];
      }
      if (valid) a.grad_e[eo * D + j] = g;
      if (CAND) gd = fmaf(g, dk[(size_t)row * D + j], gd);
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
  const int waves = a.rb.n_links + 1;
  if (waves * kWave > 1024 || slices < 1) return hipErrorInvalidValue;
  if (slices > 1 && (!a.wl.part || !a.wl.count)) return hipErrorInvalidValue;
  const size_t lds = (size_t)waves * (2 + a.rb.dof) * kWave * sizeof(float);
  const dim3 grid(grid_x, slices), block(waves * kWave);
  if (cand && grad) eval_wl_kernel<MAXS, true, true><<<grid, block, lds, s>>>(a);
  else if (grad) eval_wl_kernel<MAXS, false, true><<<grid, block, lds, s>>>(a);
  else if (!cand) eval_wl_kernel<MAXS, false, false><<<grid, block, lds, s>>>(a);
  else eval_wl_kernel<MAXS, true, false><<<grid, block, lds, s>>>(a);
  return hipGetLastError();
}

}  // namespace
}  // namespace mg
