// mg_device.h -- device helpers shared by the gfx950 kernels of libmg:
// cuboid loads through the constant address space, stable logcosh,
// DPP / lane-swap reductions, 3x4 transform algebra, Shepperd quaternions
// and the exact sphere-cuboid term of the collision cost.
#pragma once

#include "mg_internal.h"

namespace mg {
namespace {


// Cuboids are read through the constant address space: every lane of a wave
// reads the same cuboid, so the loads become scalar loads into SGPRs and the
// cuboid reaches the whole wave as instruction operands.
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(4))) const v4f cv4f;
typedef __attribute__((address_space(4))) const float cfloat;
typedef int v4i __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(4))) const v4i cv4i;
typedef __attribute__((address_space(4))) const int cint;

__device__ __forceinline__ float logcosh_f(float x) {
  const float ax = fabsf(x);
  if (ax < 1.0f) {
    // log(cosh x) = log1p(2 sinh^2(x/2)): no cancellation for small x
    const float s = sinhf(0.5f * ax);
    return log1pf(2.0f * s * s);
  }
  return ax + log1pf(expf(-2.0f * ax)) - 0.693147180559945f;
}

// tanh(k r) / r with its limit k at r = 0.
__device__ __forceinline__ float tanh_over(float k, float r) {
  return r > 0.0f ? tanhf(k * r) / r : k;
}

// ---- cross-lane reductions (DPP within rows of 16, lane swaps across rows) ----
template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}

__device__ __forceinline__ float swap16_sum(float v) {
  const auto r = __builtin_amdgcn_permlane16_swap(__builtin_bit_cast(int, v), __builtin_bit_cast(int, v), false, false);
  return __builtin_bit_cast(float, (int)r[0]) + __builtin_bit_cast(float, (int)r[1]);
}

__device__ __forceinline__ float swap32_sum(float v) {
  const auto r = __builtin_amdgcn_permlane32_swap(__builtin_bit_cast(int, v), __builtin_bit_cast(int, v), false, false);
  return __builtin_bit_cast(float, (int)r[0]) + __builtin_bit_cast(float, (int)r[1]);
}

__device__ __forceinline__ float swap16_min(float v) {
  const auto r = __builtin_amdgcn_permlane16_swap(__builtin_bit_cast(int, v), __builtin_bit_cast(int, v), false, false);
  return fminf(__builtin_bit_cast(float, (int)r[0]), __builtin_bit_cast(float, (int)r[1]));
}

__device__ __forceinline__ float swap32_min(float v) {
  const auto r = __builtin_amdgcn_permlane32_swap(__builtin_bit_cast(int, v), __builtin_bit_cast(int, v), false, false);
  return fminf(__builtin_bit_cast(float, (int)r[0]), __builtin_bit_cast(float, (int)r[1]));
}

// Sum over aligned groups of WIDTH lanes; every lane of a group gets the same
// bits (each step adds the same two partial sums in either order).
template <int WIDTH>
__device__ __forceinline__ float group_sum(float v) {
  if (WIDTH >= 2) v += dpp<0xB1>(v);      // quad_perm [1,0,3,2]
  if (WIDTH >= 4) v += dpp<0x4E>(v);      // quad_perm [2,3,0,1]
  if (WIDTH >= 8) v += dpp<0x141>(v);     // row_half_mirror
  if (WIDTH >= 16) v += dpp<0x140>(v);    // row_mirror
  if (WIDTH >= 32) v = swap16_sum(v);
  if (WIDTH >= 64) v = swap32_sum(v);
  return v;
}

template <int WIDTH>
__device__ __forceinline__ float group_min(float v) {
  if (WIDTH >= 2) v = fminf(v, dpp<0xB1>(v));
  if (WIDTH >= 4) v = fminf(v, dpp<0x4E>(v));
  if (WIDTH >= 8) v = fminf(v, dpp<0x141>(v));
  if (WIDTH >= 16) v = fminf(v, dpp<0x140>(v));
  if (WIDTH >= 32) v = swap16_min(v);
  if (WIDTH >= 64) v = swap32_min(v);
  return v;
}

// The kernel arguments sit in memory that each launch reads cold, and the
// compiler fetches a field (a scalar load) where it is first used, behind
// the branches and waits before it, which chains round trips.  Touching
// every 64-byte line of the argument block at once at the start brings it
// all into the scalar cache in one round trip.
// (OFF: the range starts OFF bytes into the block, a multiple of 4)
template <int BYTES, int OFF = 0>
__device__ __forceinline__ void warm_kernargs() {
  static_assert(BYTES <= 512, "one load per line, at most 8 lines");
  static_assert(OFF % 4 == 0, "dword aligned");
  const cint* kp = (const cint*)__builtin_amdgcn_kernarg_segment_ptr() + OFF / 4;
  constexpr int last = (BYTES - 4) / 4;
  const int v0 = kp[0], v1 = kp[16 < last ? 16 : last], v2 = kp[32 < last ? 32 : last];
  const int v3 = kp[48 < last ? 48 : last], v4 = kp[64 < last ? 64 : last], v5 = kp[80 < last ? 80 : last];
  const int v6 = kp[96 < last ? 96 : last], v7 = kp[112 < last ? 112 : last];
  asm volatile("" ::"s"(v0), "s"(v1), "s"(v2), "s"(v3), "s"(v4), "s"(v5), "s"(v6), "s"(v7));
}

__device__ __forceinline__ float wave_sum(float v) { return group_sum<kWave>(v); }
__device__ __forceinline__ float wave_min(float v) { return group_min<kWave>(v); }

// T <- T * F for 3x4 row-major affine transforms (F read from memory).
__device__ __forceinline__ void compose(float* T, const float* __restrict__ F) {
  const float4 f0 = *reinterpret_cast<const float4*>(F + 0);
  const float4 f1 = *reinterpret_cast<const float4*>(F + 4);
  const float4 f2 = *reinterpret_cast<const float4*>(F + 8);
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const float t0 = T[r * 4 + 0], t1 = T[r * 4 + 1], t2 = T[r * 4 + 2], t3 = T[r * 4 + 3];
    T[r * 4 + 0] = t0 * f0.x + t1 * f1.x + t2 * f2.x;
    T[r * 4 + 1] = t0 * f0.y + t1 * f1.y + t2 * f2.y;
    T[r * 4 + 2] = t0 * f0.z + t1 * f1.z + t2 * f2.z;
    T[r * 4 + 3] = t0 * f0.w + t1 * f1.w + t2 * f2.w + t3;
  }
}

// T <- T * F with F read through the constant address space (wave-uniform
// address: scalar loads).
__device__ __forceinline__ void compose_u(float* T, cfloat* F) {
  const v4f f0 = *(cv4f*)(F + 0);
  const v4f f1 = *(cv4f*)(F + 4);
  const v4f f2 = *(cv4f*)(F + 8);
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const float t0 = T[r * 4 + 0], t1 = T[r * 4 + 1], t2 = T[r * 4 + 2], t3 = T[r * 4 + 3];
    T[r * 4 + 0] = t0 * f0.x + t1 * f1.x + t2 * f2.x;
    T[r * 4 + 1] = t0 * f0.y + t1 * f1.y + t2 * f2.y;
    T[r * 4 + 2] = t0 * f0.z + t1 * f1.z + t2 * f2.z;
    T[r * 4 + 3] = t0 * f0.w + t1 * f1.w + t2 * f2.w + t3;
  }
}

// T <- T * Rz: mixes the first two columns (Tab.6, revolute z) given sin, cos.
__device__ __forceinline__ void rotz(float* T, float s, float c) {
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const float a = T[r * 4 + 0], b = T[r * 4 + 1];
    T[r * 4 + 0] = a * c + b * s;
    T[r * 4 + 1] = b * c - a * s;
  }
}

__device__ __forceinline__ void identity(float* T) {
#pragma unroll
  for (int i = 0; i < 12; ++i) T[i] = 0.0f;
  T[0] = T[5] = T[10] = 1.0f;
}

// Rotation matrix (row-major 3x3 inside a 3x4) -> unit quaternion wxyz,
// Shepperd's method.
__device__ __forceinline__ void mat_to_quat(const float* T, float& qw, float& qx, float& qy, float& qz) {
  const float r00 = T[0], r01 = T[1], r02 = T[2];
  const float r10 = T[4], r11 = T[5], r12 = T[6];
  const float r20 = T[8], r21 = T[9], r22 = T[10];
  const float tr = r00 + r11 + r22;
  if (tr >= r00 && tr >= r11 && tr >= r22) {
    const float w = 0.5f * sqrtf(1.0f + tr), f = 0.25f * __builtin_amdgcn_rcpf(w);
    qw = w; qx = (r21 - r12) * f; qy = (r02 - r20) * f; qz = (r10 - r01) * f;
  } else if (r00 >= r11 && r00 >= r22) {
    const float x = 0.5f * sqrtf(1.0f + r00 - r11 - r22), f = 0.25f * __builtin_amdgcn_rcpf(x);
    qx = x; qw = (r21 - r12) * f; qy = (r01 + r10) * f; qz = (r02 + r20) * f;
  } else if (r11 >= r22) {
    const float y = 0.5f * sqrtf(1.0f - r00 + r11 - r22), f = 0.25f * __builtin_amdgcn_rcpf(y);
    qy = y; qw = (r02 - r20) * f; qx = (r01 + r10) * f; qz = (r12 + r21) * f;
  } else {
    const float z = 0.5f * sqrtf(1.0f - r00 - r11 + r22), f = 0.25f * __builtin_amdgcn_rcpf(z);
    qz = z; qw = (r10 - r01) * f; qx = (r02 + r20) * f; qy = (r12 + r21) * f;
  }
}

// Exact signed distance of a box-frame point p to a box with half extents h,
// given a = |p| - h componentwise (Sec. world collision: closest point and
// inside/outside sign), and its gradient in the box frame.  Inside, the
// gradient is the outward normal of the nearest face, lowest axis on ties.
// Branch-free: the outside and inside forms are both formed and selected
// (the lanes of a wave differ), with the hardware square root.
__device__ __forceinline__ float box_sdf(float px, float py, float pz, float ax, float ay, float az,
                                         float& gpx, float& gpy, float& gpz) {
  const float qx = fmaxf(ax, 0.0f), qy = fmaxf(ay, 0.0f), qz = fmaxf(az, 0.0f);
  const float n2 = qx * qx + qy * qy + qz * qz;
  const bool out = n2 > 0.0f;
  const float n = __builtin_amdgcn_sqrtf(n2);
  const float inv = __builtin_amdgcn_rcpf(out ? n : 1.0f);
  const float sx = px >= 0.0f ? 1.0f : -1.0f, sy = py >= 0.0f ? 1.0f : -1.0f, sz = pz >= 0.0f ? 1.0f : -1.0f;
  const bool ix = ax >= ay && ax >= az, iy = !ix && ay >= az, iz = !ix && !iy;
  gpx = out ? sx * qx * inv : (ix ? sx : 0.0f);
  gpy = out ? sy * qy * inv : (iy ? sy : 0.0f);
  gpz = out ? sz * qz * inv : (iz ? sz : 0.0f);
  return out ? n : fmaxf(ax, fmaxf(ay, az));
}

// box_sdf without the gradient (cost-only evaluations).
__device__ __forceinline__ float box_dist(float ax, float ay, float az) {
  const float qx = fmaxf(ax, 0.0f), qy = fmaxf(ay, 0.0f), qz = fmaxf(az, 0.0f);
  const float n2 = qx * qx + qy * qy + qz * qz;
  return n2 > 0.0f ? __builtin_amdgcn_sqrtf(n2) : fmaxf(ax, fmaxf(ay, az));
}

// Eq.(10) smoothed penetration cost w d_c(r - sdf) alone.
__device__ __forceinline__ void dc_cost(float sdf, float r, float w, float eta, float inv_eta, float& cost) {
  const float pen = r - sdf;
  const float u = pen + eta;
  const float dcv = pen > 0.0f ? pen + 0.5f * eta : 0.5f * u * u * inv_eta;
  cost += pen > -eta ? w * dcv : 0.0f;
}

// Eq.(10) smoothed penetration cost w d_c(r - sdf) added to cost; the box-frame
// gradient (gpx, gpy, gpz) of sdf is rotated back to the world and
// d cost / d point is accumulated into g.  Outside the band (r - sdf <=
// -eta) both are zero.  Branch-free.
__device__ __forceinline__ void dc_term(const v4f& A0, const v4f& A1, const v4f& A2, float sdf,
                                        float gpx, float gpy, float gpz, float r, float w,
                                        float eta, float inv_eta, float& cost, float& gx, float& gy,
                                        float& gz) {
  const float pen = r - sdf;
  const float u = pen + eta;
  const bool deep = pen > 0.0f, band = pen > -eta;
  float dcv = deep ? pen + 0.5f * eta : 0.5f * u * u * inv_eta;
  float slope = deep ? 1.0f : u * inv_eta;
  dcv = band ? dcv : 0.0f;
  slope = band ? slope : 0.0f;
  cost += w * dcv;
  // d cost / d c = -w slope A^T grad_p
  const float f = -w * slope;
  gx = fmaf(f, A0.x * gpx + A1.x * gpy + A2.x * gpz, gx);
  gy = fmaf(f, A0.y * gpx + A1.y * gpy + A2.y * gpz, gy);
  gz = fmaf(f, A0.z * gpx + A1.z * gpy + A2.z * gpz, gz);
}

// dc_term with the gradient left in the box frame: f grad_p accumulated into
// b (f = -w slope), for several samples against one cuboid that are rotated
// back to the world once (A^T b).
__device__ __forceinline__ void dc_term_box(float sdf, float gpx, float gpy, float gpz, float r, float w, float eta,
                                            float inv_eta, float& cost, float& bx, float& by, float& bz) {
  const float pen = r - sdf;
  const float u = pen + eta;
  const bool deep = pen > 0.0f, band = pen > -eta;
  float dcv = deep ? pen + 0.5f * eta : 0.5f * u * u * inv_eta;
  float slope = deep ? 1.0f : u * inv_eta;
  dcv = band ? dcv : 0.0f;
  slope = band ? slope : 0.0f;
  cost += w * dcv;
  const float f = -w * slope;
  bx = fmaf(f, gpx, bx);
  by = fmaf(f, gpy, by);
  bz = fmaf(f, gpz, bz);
}

// One sphere against one cuboid, taken only when the cheap face test says
// the sphere may be within r + eta: exact signed distance, Eq.(10) profile,
// clearance, and d cost / d centre accumulated into g.  Returns the distance.
__device__ __forceinline__ float near_pair(const v4f& A0, const v4f& A1, const v4f& A2, float px,
                                           float py, float pz, float ax, float ay, float az,
                                           float r, float w, float eta, float inv_eta, float& cost,
                                           float& mc, float& gx, float& gy, float& gz) {
  float gpx, gpy, gpz;
  const float sdf = box_sdf(px, py, pz, ax, ay, az, gpx, gpy, gpz);
  mc = fminf(mc, sdf - r);
  dc_term(A0, A1, A2, sdf, gpx, gpy, gpz, r, w, eta, inv_eta, cost, gx, gy, gz);
  return sdf;
}

// Counter-based normal draws of the particle stage: Philox-4x64 with 10
// rounds (Salmon et al., SC'11) and Box-Muller.  Element e (= row * D +
// joint), particle k and round it under seed s take word e mod 4 of
// philox({e / 4, k, it, 0}, {s, 0}); bits 41..63 and 9..31 give the
// uniforms u1, u2 = (23-bit integer + 1/2) / 2^23 and the draw is
// sqrt(-2 ln u1) cos(2 pi u2).
__device__ __forceinline__ void philox4x64(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0,
                                           uint64_t k1, uint64_t* out) {
  constexpr uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
  constexpr uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t hi0 = __umul64hi(c0, M0), lo0 = c0 * M0;
    const uint64_t hi1 = __umul64hi(c2, M1), lo1 = c2 * M1;
    const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    k0 += W0;
    k1 += W1;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

__device__ __forceinline__ float box_muller(uint64_t w) {
  const float u1 = ((float)(unsigned)(w >> 41) + 0.5f) * (1.0f / 8388608.0f);
  const float u2 = ((float)(unsigned)((w >> 9) & 0x7FFFFFu) + 0.5f) * (1.0f / 8388608.0f);
  // (cos(2 pi u2) as cospi(2 u2): no rounding of the angle)
  return sqrtf(-2.0f * logf(u1)) * cospif(2.0f * u2);
}

// The four standard normal draws of particle k, round it, elements 4q ..
// 4q + 3 (one Philox block at counter {q, k, it, 0}, key {seed, 0}).
__device__ __forceinline__ void philox_draws4(uint64_t seed, int k, int it, uint64_t q, float* out4) {
  uint64_t w[4];
  philox4x64(q, (uint64_t)(unsigned)k, (uint64_t)(unsigned)it, 0, seed, 0, w);
#pragma unroll
  for (int i = 0; i < 4; ++i) out4[i] = box_muller(w[i]);
}

// The draw of particle k, round it, element e alone (word e mod 4).
__device__ __forceinline__ float philox_draw(uint64_t seed, int k, int it, uint64_t e) {
  uint64_t w[4];
  philox4x64(e >> 2, (uint64_t)(unsigned)k, (uint64_t)(unsigned)it, 0, seed, 0, w);
  const int i = (int)(e & 3);
  return box_muller(i == 0 ? w[0] : i == 1 ? w[1] : i == 2 ? w[2] : w[3]);
}

}  // namespace
}  // namespace mg
