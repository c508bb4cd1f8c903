// mg_eval.h -- the evaluation kernel: cost and adjoint of every (candidate,
// waypoint row) of a batch in one launch.  Instantiated per kinematic shape
// in mg_eval_*.hip so the variants compile in parallel.
#pragma once

#include "mg_device.h"

namespace mg {
namespace {

// Lane layout: a workgroup of 256 lanes handles 256/G consecutive waypoint
// rows of one problem for one line-search candidate k (blockIdx.y); the G
// lanes of a row split the robot's spheres into G groups (<= MAXS spheres,
// one link each).  Lanes g < D also own joint g of the row: its limit and
// smoothness terms and the final gradient entry.
//
// SERIAL robots (link l has parent l-1 and joint l) walk one shared chain:
// every lane composes the same fixed transforms, read as scalar loads, and
// keeps the transform of its own link; joint gradients are summed across the
// row's lanes with DPP.  Other kinematic trees use per-group chain tables
// padded with identities and sum joint gradients through LDS lists.
template <int G, int MAXS, int DEPTH, bool SERIAL, bool CAND, bool GRAD>
__global__ __launch_bounds__(kBlock) void eval_kernel(const EvalArgs a) {
  constexpr int EPW = kBlock / G;
  constexpr bool USE_LDS = GRAD && !SERIAL;
  __shared__ float s_dq[USE_LDS ? DEPTH * kBlock : 1];

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
  const int D = a.rb.dof;
  const int ev = threadIdx.x / G;
  const int g = threadIdx.x % G;
  const int nrows = pb.S * pb.T;
  const int rloc = (bx - a.chunk_prefix[p]) * EPW + ev;
  const bool valid = rloc < nrows;
  const int rl = valid ? rloc : nrows - 1;
  const int t = rl % pb.T;          // waypoint t+1 of its seed
  const int row = pb.row0 + rl;
  const float alpha = CAND ? a.alpha[k] : 0.0f;

  // candidate value of joint j at waypoint row r: clip(x + alpha d)
  auto qval = [&](int r, int j) -> float {
    float v = a.x[(size_t)r * D + j];
    if (CAND) {
      v = fmaf(alpha, a.d[(size_t)r * D + j], v);
      v = fminf(fmaxf(v, a.rb.q_lo[j]), a.rb.q_hi[j]);
    }
    return v;
  };

  const int4 gi = a.gr.info[g];     // chain length, -, spheres, end effector
  cfloat* ftf_u = (cfloat*)a.rb.fixed_tf;

  // ---- forward kinematics of the group's link ----
  float sn[DEPTH], cs[DEPTH];
  float T[12];
  identity(T);
  if constexpr (SERIAL) {
    const int L = a.rb.n_links;
    float qr[DEPTH];
#pragma unroll
    for (int i = 0; i < DEPTH; ++i) qr[i] = qval(row, i < L ? i : L - 1);
    float U[12];
    identity(U);
#pragma unroll
    for (int i = 0; i < DEPTH; ++i) {
      sn[i] = 0.0f;
      cs[i] = 1.0f;
      if (i < L) {
        sn[i] = __sinf(qr[i]);
        cs[i] = __cosf(qr[i]);
        compose_u(U, ftf_u + i * 12);
        rotz(U, sn[i], cs[i]);
        const bool mine = i < gi.x;
#pragma unroll
        for (int e = 0; e < 12; ++e) T[e] = mine ? U[e] : T[e];
      }
    }
  } else {
    const int* jidx = a.gr.jidx + g * DEPTH;
    const float* ftf = a.gr.ftf + (size_t)g * DEPTH * 12;
    float qc[DEPTH];
    int jc[DEPTH];
#pragma unroll
    for (int i = 0; i < DEPTH; ++i) {
      jc[i] = jidx[i];
      qc[i] = qval(row, jc[i] >= 0 ? jc[i] : 0);
    }
#pragma unroll
    for (int i = 0; i < DEPTH; ++i) {
      sn[i] = jc[i] >= 0 ? __sinf(qc[i]) : 0.0f;
      cs[i] = jc[i] >= 0 ? __cosf(qc[i]) : 1.0f;
      compose(T, ftf + i * 12);      // unused slots hold identities
      rotz(T, sn[i], cs[i]);
    }
  }

  float cost = 0.0f;
  float mc = a.pr.eta;
  // wrench of this group about the world origin: F = sum of d cost / d point,
  // M = sum of point x (d cost / d point) (+ pure moments of the pose term)
  float Fx = 0.0f, Fy = 0.0f, Fz = 0.0f, Mx = 0.0f, My = 0.0f, Mz = 0.0f;

  // ---- world collision (Eq.(10)/(11) without the speed factor, summed over
  //      cuboids and spheres); cuboid loop outside, this lane's spheres inside
  {
    const float w = a.pr.w_coll, eta = a.pr.eta, inv_eta = 1.0f / fmaxf(eta, 1e-30f);
    float cx[MAXS], cy[MAXS], cz[MAXS], rr[MAXS], rho[MAXS], gx[MAXS], gy[MAXS], gz[MAXS];
#pragma unroll
    for (int s = 0; s < MAXS; ++s) {
      const float4 ls = a.gr.sphere[g * MAXS + s];
      const bool on = s < gi.z;
      // unused slots sit far away and never pass the face test
      cx[s] = on ? T[0] * ls.x + T[1] * ls.y + T[2] * ls.z + T[3] : 1e18f;
      cy[s] = on ? T[4] * ls.x + T[5] * ls.y + T[6] * ls.z + T[7] : 1e18f;
      cz[s] = on ? T[8] * ls.x + T[9] * ls.y + T[10] * ls.z + T[11] : 1e18f;
      rr[s] = on ? ls.w : 0.0f;
      rho[s] = rr[s] + eta;
      gx[s] = gy[s] = gz[s] = 0.0f;
    }
    const int o0 = a.world_off[pb.world], o1 = a.world_off[pb.world + 1];
    cv4f* boxes = (cv4f*)(a.box);
    // the next cuboid's scalar loads are issued one iteration ahead
    v4f nA0 = {}, nA1 = {}, nA2 = {}, nH = {};
    if (o0 < o1) {
      nA0 = boxes[4 * o0 + 0]; nA1 = boxes[4 * o0 + 1];
      nA2 = boxes[4 * o0 + 2]; nH = boxes[4 * o0 + 3];
    }
    for (int o = o0; o < o1; ++o) {
      const v4f A0 = nA0, A1 = nA1, A2 = nA2, H = nH;
      if (o + 1 < o1) {
        nA0 = boxes[4 * o + 4]; nA1 = boxes[4 * o + 5];
        nA2 = boxes[4 * o + 6]; nH = boxes[4 * o + 7];
      }
      float px[MAXS], py[MAXS], pz[MAXS], ax[MAXS], ay[MAXS], az[MAXS], m3[MAXS];
      bool any = false;
#pragma unroll
      for (int s = 0; s < MAXS; ++s) {
        px[s] = fmaf(A0.x, cx[s], fmaf(A0.y, cy[s], fmaf(A0.z, cz[s], A0.w)));
        py[s] = fmaf(A1.x, cx[s], fmaf(A1.y, cy[s], fmaf(A1.z, cz[s], A1.w)));
        pz[s] = fmaf(A2.x, cx[s], fmaf(A2.y, cy[s], fmaf(A2.z, cz[s], A2.w)));
        ax[s] = fabsf(px[s]) - H.x;
        ay[s] = fabsf(py[s]) - H.y;
        az[s] = fabsf(pz[s]) - H.z;
        m3[s] = fmaxf(ax[s], fmaxf(ay[s], az[s]));
        // |max(a,0)| >= max(a): a cuboid whose face distance exceeds r + eta
        // adds no cost and cannot lower the clearance clamped at eta
        any |= m3[s] < rho[s];
      }
      if (any) {
#pragma unroll
        for (int s = 0; s < MAXS; ++s)
          if (m3[s] < rho[s])
            near_pair(A0, A1, A2, px[s], py[s], pz[s], ax[s], ay[s], az[s], m3[s], rr[s], w, eta,
                      inv_eta, cost, mc, gx[s], gy[s], gz[s]);
      }
    }
#pragma unroll
    for (int s = 0; s < MAXS; ++s) {
      Fx += gx[s]; Fy += gy[s]; Fz += gz[s];
      Mx += cy[s] * gz[s] - cz[s] * gy[s];
      My += cz[s] * gx[s] - cx[s] * gz[s];
      Mz += cx[s] * gy[s] - cy[s] * gx[s];
    }
  }

  // ---- pose reaching cost at the last waypoint (Eq.(14)) ----
  if (gi.w >= 0 && t == pb.T - 1) {
    float E[12];
#pragma unroll
    for (int i = 0; i < 12; ++i) E[i] = T[i];
    compose(E, a.rb.ee_tf + gi.w * 12);
    float qt[4];
    mat_to_quat(E, qt[0], qt[1], qt[2], qt[3]);
    const float* gl = a.goal + ((size_t)p * a.rb.n_ee + gi.w) * 7;
    const float px = E[3], py = E[7], pz = E[11];
    const float ex = gl[0] - px, ey = gl[1] - py, ez = gl[2] - pz;
    const float n = sqrtf(ex * ex + ey * ey + ez * ez);
    cost += a.pr.a0 * logcosh_f(a.pr.a2 * n);
    const float fp = -a.pr.a0 * a.pr.a2 * tanh_over(a.pr.a2, n);
    const float gpx = fp * ex, gpy = fp * ey, gpz = fp * ez;     // d cost / d p
    const float dot = gl[3] * qt[0] + gl[4] * qt[1] + gl[5] * qt[2] + gl[6] * qt[3];
    const float sg = dot >= 0.0f ? 1.0f : -1.0f;
    const float e0 = gl[3] - sg * qt[0], e1 = gl[4] - sg * qt[1];
    const float e2 = gl[5] - sg * qt[2], e3 = gl[6] - sg * qt[3];
    const float dr = sqrtf(e0 * e0 + e1 * e1 + e2 * e2 + e3 * e3);
    cost += a.pr.a1 * logcosh_f(a.pr.a3 * dr);
    // d cost / d quaternion, then the moment conjugate to a world-frame
    // rotation omega: d quat = 1/2 (0, omega) (x) quat
    const float fq = -sg * a.pr.a1 * a.pr.a3 * tanh_over(a.pr.a3, dr);
    const float gw = fq * e0, gvx = fq * e1, gvy = fq * e2, gvz = fq * e3;
    const float w = qt[0], vx = qt[1], vy = qt[2], vz = qt[3];
    const float tx = 0.5f * (w * gvx - gw * vx + (vy * gvz - vz * gvy));
    const float ty = 0.5f * (w * gvy - gw * vy + (vz * gvx - vx * gvz));
    const float tz = 0.5f * (w * gvz - gw * vz + (vx * gvy - vy * gvx));
    Fx += gpx; Fy += gpy; Fz += gpz;
    Mx += py * gpz - pz * gpy + tx;
    My += pz * gpx - px * gpz + ty;
    Mz += px * gpy - py * gpx + tz;
    if (a.pe_e && valid && gi.w == 0) {
      a.pe_e[(size_t)row * 2 + 0] = n;
      a.pe_e[(size_t)row * 2 + 1] = 2.0f * acosf(fminf(fabsf(dot), 1.0f));
    }
  }

  // ---- joint g: limit cost (Eq.(17)) and smoothness (Eq.(16)); every lane
  //      loads (clamped index), lanes g >= D discard the result ----
  float gsm = 0.0f;
  {
    const int gj = g < D ? g : D - 1;
    const bool own = g < D;
    float jc = 0.0f;
    const float xq = qval(row, gj);
    const float lo_ = a.rb.q_lo[gj], hi_ = a.rb.q_hi[gj], e2 = a.pr.eta2, wb = a.pr.w_bound;
    const float inv_e2 = 1.0f / e2;
    float bc = 0.0f, bs = 0.0f;
    if (xq < lo_) { bc += lo_ - xq + 0.5f * e2; bs -= 1.0f; }
    else if (xq < lo_ + e2) { const float u = lo_ - xq + e2; bc += 0.5f * u * u * inv_e2; bs -= u * inv_e2; }
    if (xq > hi_) { bc += xq - hi_ + 0.5f * e2; bs += 1.0f; }
    else if (xq > hi_ - e2) { const float u = xq - hi_ + e2; bc += 0.5f * u * u * inv_e2; bs += u * inv_e2; }
    jc += wb * bc;
    float js = wb * bs;

    if (pb.T > 1) {
      // padded states X(s), s = w-4..w+4 around this waypoint w = t+1:
      // start for s <= 0, last waypoint for s >= T
      const int w1 = t + 1, Tn = pb.T;
      const float q0 = a.q_start[(size_t)p * D + gj];
      float X[9];
#pragma unroll
      for (int u = 0; u < 9; ++u) {
        const int sgi = w1 - 4 + u;
        const int wv = sgi < 1 ? 1 : (sgi < Tn ? sgi : Tn);
        const float v = qval(row - t + wv - 1, gj);
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
        const bool vel = a.pr.vel_all || tau == Tn;
        // this centre's cost belongs to waypoint tau (the start's to waypoint 1)
        if (in && (tau == w1 || (tau == 0 && w1 == 1)))
          jc += (vel ? a.pr.a6 * logcosh_f(a.pr.a7 * v) : 0.0f) + a.pr.a8 * ac * ac + a.pr.a9 * jk * jk;
        const float gv = vel ? a.pr.a6 * a.pr.a7 * tanhf(a.pr.a7 * v) * cv : 0.0f;
        const float ga = 2.0f * a.pr.a8 * ac * ca, gjk = 2.0f * a.pr.a9 * jk * cj;
#pragma unroll
        for (int i = 0; i < 5; ++i) {
          const int s = tau - 2 + i;         // state touched by stencil entry i
          if (in && s >= 1 && (s < Tn ? s : Tn) == w1) js += gv * kv[i] + ga * ka[i] + gjk * kj[i];
        }
      }
    }
    cost += own ? jc : 0.0f;
    gsm = own ? js : 0.0f;
  }

  // ---- adjoint: project the group's wrench on the joint axes of its chain,
  //      recomputing the chain's transforms instead of storing them ----
  float gradj = 0.0f;
  if (GRAD) {
    float R[12];
    identity(R);
    if constexpr (SERIAL) {
      const int L = a.rb.n_links;
      float dq[DEPTH];
#pragma unroll
      for (int i = 0; i < DEPTH; ++i) {
        dq[i] = 0.0f;
        if (i < L) {
          compose_u(R, ftf_u + i * 12);
          // revolute z (Tab.7): d/dq = z . (M - o x F) with axis z and origin o
          // of the joint frame; only joints on this group's chain
          const float zx = R[2], zy = R[6], zz = R[10], ox = R[3], oy = R[7], oz = R[11];
          const float ux = Mx - (oy * Fz - oz * Fy);
          const float uy = My - (oz * Fx - ox * Fz);
          const float uz = Mz - (ox * Fy - oy * Fx);
          dq[i] = i < gi.x ? zx * ux + zy * uy + zz * uz : 0.0f;
          rotz(R, sn[i], cs[i]);
          dq[i] = group_sum<G>(dq[i]);
          gradj = g == i ? dq[i] : gradj;
        }
      }
      gradj += gsm;
    } else {
      const int* jidx = a.gr.jidx + g * DEPTH;
      const float* ftf = a.gr.ftf + (size_t)g * DEPTH * 12;
#pragma unroll
      for (int i = 0; i < DEPTH; ++i) {
        compose(R, ftf + i * 12);
        const float zx = R[2], zy = R[6], zz = R[10], ox = R[3], oy = R[7], oz = R[11];
        const float ux = Mx - (oy * Fz - oz * Fy);
        const float uy = My - (oz * Fx - ox * Fz);
        const float uz = Mz - (ox * Fy - oy * Fx);
        s_dq[i * kBlock + threadIdx.x] = jidx[i] >= 0 ? zx * ux + zy * uy + zz * uz : 0.0f;
        rotz(R, sn[i], cs[i]);
      }
      __syncthreads();
      if (g < D) {
        const int b0 = a.gr.red[g], b1 = a.gr.red[g + 1];
        float acc = 0.0f;
        for (int u = b0; u < b1; ++u) {
          const int slot = a.gr.red[D + 1 + u];
          acc += s_dq[(slot % DEPTH) * kBlock + ev * G + slot / DEPTH];
        }
        gradj = acc + gsm;
      }
    }
  }

  const float csum = group_sum<G>(cost);
  const float mcmin = group_min<G>(mc);
  float gd = 0.0f;
  if (CAND && GRAD && g < D) gd = gradj * a.d[(size_t)row * D + g];
  gd = group_sum<G>(gd);
  if (valid) {
    const size_t e = (size_t)k * a.rows + row;
    if (g == 0) {
      a.cost_e[e] = csum;
      a.mc_e[e] = mcmin;
      if (CAND && GRAD) a.gd_e[e] = gd;
    }
    if (GRAD && g < D) a.grad_e[e * D + g] = gradj;
  }
}

template <int G, int MAXS, int DEPTH, bool SERIAL>
hipError_t launch_eval_g(const EvalArgs& a, int grid_x, bool cand, bool grad, hipStream_t s) {
  const dim3 grid(grid_x, cand ? a.K : 1), block(kBlock);
  if (cand && grad) eval_kernel<G, MAXS, DEPTH, SERIAL, true, true><<<grid, block, 0, s>>>(a);
  else if (grad) eval_kernel<G, MAXS, DEPTH, SERIAL, false, true><<<grid, block, 0, s>>>(a);
  else if (!cand) eval_kernel<G, MAXS, DEPTH, SERIAL, false, false><<<grid, block, 0, s>>>(a);
  else return hipErrorInvalidValue;   // candidates without gradients are not used
  return hipGetLastError();
}

template <int DEPTH, bool SERIAL>
hipError_t launch_eval_shape(const EvalArgs& a, int grid_x, bool cand, bool grad, hipStream_t s) {
  const int G = a.gr.G, S = a.gr.maxs;
  if (G == 8 && S == 8) return launch_eval_g<8, 8, DEPTH, SERIAL>(a, grid_x, cand, grad, s);
  if (G == 8 && S == 16) return launch_eval_g<8, 16, DEPTH, SERIAL>(a, grid_x, cand, grad, s);
  if (G == 16 && S == 4) return launch_eval_g<16, 4, DEPTH, SERIAL>(a, grid_x, cand, grad, s);
  if (G == 16 && S == 8) return launch_eval_g<16, 8, DEPTH, SERIAL>(a, grid_x, cand, grad, s);
  if (G == 16 && S == 16) return launch_eval_g<16, 16, DEPTH, SERIAL>(a, grid_x, cand, grad, s);
  if (G == 32 && S == 2) return launch_eval_g<32, 2, DEPTH, SERIAL>(a, grid_x, cand, grad, s);
  if (G == 32 && S == 4) return launch_eval_g<32, 4, DEPTH, SERIAL>(a, grid_x, cand, grad, s);
  if (G == 32 && S == 8) return launch_eval_g<32, 8, DEPTH, SERIAL>(a, grid_x, cand, grad, s);
  return hipErrorInvalidValue;
}

}  // namespace

// One translation unit per (DEPTH, SERIAL) pair defines its launcher.
hipError_t launch_eval_d8s(const EvalArgs& a, int grid_x, bool cand, bool grad, hipStream_t s);
hipError_t launch_eval_d16s(const EvalArgs& a, int grid_x, bool cand, bool grad, hipStream_t s);
hipError_t launch_eval_d8t(const EvalArgs& a, int grid_x, bool cand, bool grad, hipStream_t s);
hipError_t launch_eval_d16t(const EvalArgs& a, int grid_x, bool cand, bool grad, hipStream_t s);

}  // namespace mg
