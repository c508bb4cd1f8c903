// mg_solver.h -- line-search choice, best tracking and L-BFGS kernels (one
// wavefront per seed), shared by their instantiation units
// (mg_select_p<PL>.hip, mg_lbfgs.hip).
#pragma once

#include "mg_device.h"

namespace mg {
namespace {

// --------------------------------------------------------------------------
// Seed s's first row and horizon: from the table, or arithmetic when every
// seed has the same horizon (one dependent memory round trip less).
__device__ __forceinline__ SeedInfo seed_info(const SeedInfo* seeds, int uniform_T, int s) {
  if (uniform_T > 0) return SeedInfo{s * uniform_T, uniform_T, 0, 0};
  return seeds[s];
}

// A seed's row block of n = T*D floats held PL per lane of its W lanes
// (one wavefront, or W = 8, 16, 32 lanes of one when several seeds share
// it): element u of a lane is lane + W u (strided), or with V4 lane PL + u
// (contiguous, moved as float4: the block is a multiple of 4 floats and
// 16-byte aligned).
template <int PL, bool V4, int W = kWave>
__device__ __forceinline__ int el_idx(int lane, int u) {
  return V4 ? lane * PL + u : lane + u * W;
}
// A per-seed scalar: through the scalar cache when the seed is the
// wavefront's own (W = 64), else a vector load.
template <int W, typename Tv>
__device__ __forceinline__ Tv ld_seed(const Tv* p) {
  if constexpr (W == kWave) return *(const __attribute__((address_space(4))) Tv*)p;
  else return *p;
}
// Loads at clamped (always valid) addresses, masked afterwards (zero
// outside the block).
template <int PL, bool V4, int W = kWave>
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
      const int e = lane + u * W;
      v[u] = p[min(e, n - 1)];
      v[u] = e < n ? v[u] : 0.0f;
    }
  }
}
template <int PL, bool V4, int W = kWave>
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
      const int e = lane + u * W;
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

template <int PL, int MH, bool V4, int W = kWave>
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
  const int first = ld_seed<W>(a.first + s);
  int count = ld_seed<W>(a.meta + 2 * s + 0);
  int head = ld_seed<W>(a.meta + 2 * s + 1);
  ld_row<PL, V4, W>(a.x_prev + base, n, lane, h.xp);
  ld_row<PL, V4, W>(a.g_prev + base, n, lane, h.gp);
  float RS[MH][PL], RY[MH][PL], Rr[MH];
#pragma unroll
  for (int r = 0; r < MH; ++r) {
    const int rc = min(r, max(m - 1, 0));   // (the history holds at least one slot)
    Rr[r] = ld_seed<W>(a.rho + (size_t)s * a.m_max + rc);
    ld_row<PL, V4, W>(a.S + (size_t)rc * stride + base, n, lane, RS[r]);
    ld_row<PL, V4, W>(a.Y + (size_t)rc * stride + base, n, lane, RY[r]);
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
      const bool in = live && el_idx<PL, V4, W>(lane, u) < n;
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
// (st_ok false: a lane group that only pads the last wavefront, or a
// workgroup that is not its seed's first, computes but stores nothing;
// q_out, or null, receives the direction)
template <int PL, int MH, bool V4, int W = kWave>
__device__ __forceinline__ void lbfgs_finish(const LbfgsArgs& a, int s, int lane, const SeedInfo& si,
                                             const float* xv, const float* gv, LbfgsRegs<PL, MH>& h,
                                             bool st_ok = true, float* q_out = nullptr) {
  const int n = si.T * a.dof;
  const size_t base = (size_t)si.row0 * a.dof;
  const size_t stride = (size_t)a.rows * a.dof;
  const int m = a.m;
  int count = h.count, head = h.head;
  float sv[PL], yv[PL];
#pragma unroll
  for (int u = 0; u < PL; ++u) {
    const bool in = el_idx<PL, V4, W>(lane, u) < n && !h.reset;
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
    sy = group_sum<W>(sy); ss = group_sum<W>(ss); yy = group_sum<W>(yy);
    if (sy > 1e-10f * sqrtf(ss) * sqrtf(yy) && sy > 0.0f) {
      if (st_ok) {
        st_row<PL, V4, W>(a.S + (size_t)head * stride + base, n, lane, sv);
        st_row<PL, V4, W>(a.Y + (size_t)head * stride + base, n, lane, yv);
        if (lane == 0) a.rho[(size_t)s * a.m_max + head] = 1.0f / sy;
      }
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
      const float ai = h.rh[c] * group_sum<W>(dsq);
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
    gamma = group_sum<W>(sy) / group_sum<W>(yy);
  } else {
    float gi = 0.0f;
#pragma unroll
    for (int u = 0; u < PL; ++u) gi = fmaxf(gi, fabsf(gv[u]));
    gi = -group_min<W>(-gi);
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
      const float b = h.rh[c] * group_sum<W>(dyr);
#pragma unroll
      for (int u = 0; u < PL; ++u) q[u] = fmaf(al[c] - b, h.Sh[c][u], q[u]);
    }
  }
#pragma unroll
  for (int u = 0; u < PL; ++u) q[u] = -q[u];
  if (q_out) {
#pragma unroll
    for (int u = 0; u < PL; ++u) q_out[u] = q[u];
  }
  if (!st_ok) return;
  st_row<PL, V4, W>(a.dir + base, n, lane, q);
  if (!a.keep_prev) {
    st_row<PL, V4, W>(a.x_prev + base, n, lane, xv);
    st_row<PL, V4, W>(a.g_prev + base, n, lane, gv);
  }
  if (lane == 0) {
    int* mo = a.meta_out ? a.meta_out : a.meta;
    mo[2 * s + 0] = count;
    mo[2 * s + 1] = head;
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
// W < 64 packs 64 / W seeds into a wavefront, W lanes each, for row blocks
// of at most W floats (inverse kinematics: T = 1); control flow then
// diverges between the lane groups but never inside one, so every group
// reduction sees only its own, active, lanes.
// Seed s's choice by the W lanes of group sub of a wavefront (lane: the
// lane within the group); the body of select_kernel, and the prologue of an
// evaluation launch that folds the choice in.  st_ok false: compute, store
// nothing.  xo / qo (or null): the new iterate and direction, element
// el_idx(lane, u) in xo[u] / qo[u].
template <int PL, int MH, bool FUSED, int KP, bool V4, int W>
__device__ __forceinline__ void select_seed(const SelectArgs& a, const LbfgsArgs& la, int s, int lane, int sub,
                                            bool st_ok, float* xo = nullptr, float* qo = nullptr) {
  static_assert(KP <= W && kWave % W == 0, "a candidate needs a lane of its seed's group");
  constexpr int SPW = kWave / W;       // seeds per wavefront
  const SeedInfo si = seed_info(a.seeds, a.uniform_T, s);
  const int D = a.dof, n = si.T * D;
  const size_t base = (size_t)si.row0 * D;

  // everything that does not depend on the choice is loaded first: for up
  // to 8 candidates every candidate's gradient, the joint limits, the
  // candidates' sums, the rows, then the L-BFGS state (whose per-seed
  // scalars are waited for inside lbfgs_load, after every load is issued)
  constexpr int KG = (PL <= 4 && KP <= 8) ? KP : 1;
  const bool pre = KG > 1;
  float gall[KG][PL];
#pragma unroll
  for (int k = 0; k < KG; ++k) {
    if (pre) ld_row<PL, V4, W>(a.grad_e + ((size_t)min(k, a.K - 1) * a.rows + si.row0) * D, n, lane, gall[k]);
  }
  float qlo[PL], qhi[PL];
#pragma unroll
  for (int u = 0; u < PL; ++u) {
    const int j = el_idx<PL, V4, W>(lane, u) % D;
    qlo[u] = a.q_lo[j];
    qhi[u] = a.q_hi[j];
  }
  const float best_prev = ld_seed<W>(a.best_c + s);
  const float c0 = ld_seed<W>(a.c0 + s);

  // candidate sums with the lanes split over the candidates: lane kq * G
  // + jq takes waypoints jq, jq + G, ... of candidate kq, then a reduction
  // over its G lanes leaves candidate kq's sums in all of them
  constexpr int G = W / KP;
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
  ld_row<PL, V4, W>(a.x + base, n, lane, xv);
  ld_row<PL, V4, W>(a.d + base, n, lane, dv);
  ld_row<PL, V4, W>(a.g0 + base, n, lane, g0v);
  LbfgsRegs<PL, FUSED ? MH : 1> h;
  if constexpr (FUSED) lbfgs_load<PL, MH, V4, W>(la, s, lane, si, h);
  float g0d = 0.0f;
#pragma unroll
  for (int u = 0; u < PL; ++u) {
    gdv[u] = 0.0f;
    g0d = fmaf(g0v[u], dv[u], g0d);
  }
  g0d = group_sum<W>(g0d);
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
  uint64_t okm = __ballot(ok && jq == 0 && kq > 0);
  if constexpr (SPW > 1) okm = (okm >> (sub * W)) & ((1ull << W) - 1);   // this seed's group
  const int best = okm ? (63 - __builtin_clzll(okm)) / G : 0;
  float cb, mcb;
  if constexpr (SPW == 1) {
    cb = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(cs), best * G));
    mcb = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(ms), best * G));
  } else {
    cb = __shfl(cs, sub * W + best * G);
    mcb = __shfl(ms, sub * W + best * G);
  }
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
    ld_row<PL, V4, W>(a.grad_e + ((size_t)best * a.rows + si.row0) * D, n, lane, gdv);
  }
#pragma unroll
  for (int u = 0; u < PL; ++u) {
    const int e = el_idx<PL, V4, W>(lane, u);
    xv[u] = e < n ? fminf(fmaxf(fmaf(al, dv[u], xv[u]), qlo[u]), qhi[u]) : 0.0f;
  }
  if (st_ok) {
    st_row<PL, V4, W>(a.x_out + base, n, lane, xv);
    st_row<PL, V4, W>(a.g_out + base, n, lane, gdv);
    if (improve) st_row<PL, V4, W>(a.best_x + base, n, lane, xv);
  }
  if (lane == 0 && st_ok) {
    a.c_out[s] = cb;
    if (a.chosen) a.chosen[s] = best;
    if (a.mc_out) a.mc_out[s] = mcb;
    if (improve) a.best_c[s] = cb;
  }
  if (xo) {
#pragma unroll
    for (int u = 0; u < PL; ++u) xo[u] = xv[u];
  }
  if constexpr (FUSED) lbfgs_finish<PL, MH, V4, W>(la, s, lane, si, xv, gdv, h, st_ok, qo);
}

template <int PL, int MH, bool FUSED, int KP, bool V4, int W = kWave>
__global__ __launch_bounds__(kWave) void select_kernel(const SelectArgs a, const LbfgsArgs la) {
  constexpr int SPW = kWave / W;       // seeds per wavefront
  const int sub = SPW > 1 ? (int)threadIdx.x / W : 0;
  const int lane = SPW > 1 ? (int)threadIdx.x % W : (int)threadIdx.x;
  // (the grid is exactly one workgroup per SPW seeds; the last one's spare
  // groups take the last seed and store nothing)
  const int s_raw = (int)blockIdx.x * SPW + sub;
  const bool st_ok = SPW == 1 || s_raw < a.n_seeds;
  const int s = SPW == 1 ? s_raw : min(s_raw, a.n_seeds - 1);
  warm_kernargs<sizeof(SelectArgs) + (FUSED ? sizeof(LbfgsArgs) + 8 : 0)>();
  select_seed<PL, MH, FUSED, KP, V4, W>(a, la, s, lane, sub, st_ok);
}

// Row blocks move as float4 when every seed's block is a multiple of 4
// floats and every array is 16-byte aligned.
inline bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }
inline bool rows_v4(int uniform_T, int dof) { return uniform_T > 0 && (uniform_T * dof) % 4 == 0; }

}  // namespace

// select_kernel launchers for PL vector elements per lane (one unit each)
hipError_t launch_select_p1(const SelectArgs& a, const LbfgsArgs* la, hipStream_t s);
// several seeds per wavefront: row blocks of at most 32 floats
hipError_t launch_select_packed(const SelectArgs& a, int max_n, const LbfgsArgs* la, hipStream_t s);
hipError_t launch_select_p2(const SelectArgs& a, const LbfgsArgs* la, hipStream_t s);
hipError_t launch_select_p4(const SelectArgs& a, const LbfgsArgs* la, hipStream_t s);
hipError_t launch_select_p8(const SelectArgs& a, const LbfgsArgs* la, hipStream_t s);
hipError_t launch_select_p16(const SelectArgs& a, const LbfgsArgs* la, hipStream_t s);
// PL = 16 with the fused L-BFGS step over more than 4 history pairs
hipError_t launch_select_p16_long(const SelectArgs& a, const LbfgsArgs& la, int KP, bool V4, hipStream_t s);
}  // namespace mg
