// mg_internal.h -- device-side tables and launch interfaces of libmg.
//
// Shared by the C ABI (mg_api.hip) and the kernels (mg_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace mg {

constexpr int kBlock = 256;      // threads per workgroup of the per-evaluation kernels
constexpr int kWave = 64;        // CDNA wavefront
constexpr int kMaxK = 16;        // line-search candidates per call
constexpr int kMaxDof = 16;
constexpr int kMaxT = 64;        // waypoints per trajectory
constexpr int kMaxEE = 2;
constexpr int kMaxHist = 16;     // L-BFGS history
constexpr int kMaxParticles = 1024;   // particles per seed of the particle stage
constexpr int kPerLane = kMaxT * kMaxDof / kWave;   // vector elements per lane in the solver kernels

// Cost parameters (see mg_params in mg.h).
struct Params {
  float a0, a1, a2, a3;
  float a6, a7, a8, a9;
  float w_bound, eta2;
  float w_coll, eta;
  float dt;
  int vel_all;
  int swept;
  int sweep_steps;
  float ls_eta1, ls_eta_w;
  float success_pos, success_rot;
  float w_self;
  int n_self;              // self-collision pairs (wave-per-link layout only)
  int speed;               // speed metric (wave-per-link layout only)
};

// One motion problem of a batch.  Rows are waypoints: seed s of problem p
// owns rows row0 + s*T .. row0 + (s+1)*T - 1.
struct Problem {
  int S, T, world, row0, seed0, pad0, pad1, pad2;
};

// Per seed: first row, horizon, problem.
struct SeedInfo {
  int row0, T, prob, pad;
};

// Robot tables on the device.  Link l is driven by joint l and its parent is
// link l-1 or the base, so the links form chains that start at the base
// (a serial arm, or several arms on one base).
struct Robot {
  int dof, n_links, n_ee, n_spheres;
  const float* fixed_tf;   // [L][12]
  const float* q_lo;       // [D]
  const float* q_hi;       // [D]
  const float* ee_tf;      // [n_ee][12]
};

// Lane layout of the evaluation kernel: lane l of an evaluation owns link l,
// its spheres and (if l < D) joint l.
struct Lanes {
  int lpe;                 // lanes per evaluation: 8 or 16
  int maxs;                // sphere slots per link: 4, 8 or 16
  const int4* info;        // [lpe]: chain start lane, chain end lane, spheres, end effector or -1
  const float4* sphere;    // [lpe][maxs] center in link frame + radius
};

// One 64-evaluation chunk of the wave-per-link layout: its problem, its
// first evaluation within the problem, the problem's seeds, horizon, first
// row and evaluation count, and its world's cuboid range.
struct WlChunk {
  int p, e_first, S, T;
  int box_lo, box_hi, row0, n_e;
};

// Wave-per-link layout of the evaluation kernel: a workgroup holds 64
// evaluations; wave l owns link l (its kinematic chain, spheres and end
// effector) for all 64, the last wave owns the joint terms.
struct WaveLinks {
  const WlChunk* chunk;    // [workgroups along x] (per candidate count K)
  // one problem (one.S > 0): chunk x is {0, x E, one.S, one.T, one.box_lo,
  // one.box_hi, 0, one.n_e}, formed without reading the table
  struct {
    int S, T, box_lo, box_hi, n_e;
  } one;
  const int4* info;        // [L]: chain depth, spheres, end effector or -1, 0
  const int* chain;        // [L][kMaxDof]: links from the root down to l
  const int* joint_rec;    // [D][2]: chain position of joint j (its link's depth - 1) and
                           //   the bit mask of the links whose chain contains it
  const float4* chain_rec; // [L][kMaxDof][4]: fixed transform rows of chain[i], then
                           //   {joint index (int bits), 0, 0, 0}
  const float4* sphere;    // [L][maxs] centre in link frame + radius
  const float4* ball;      // [L][kWlBalls] balls bounding the link's spheres (link frame):
                           //   centre, radius; all slots, each half, each quarter
  int maxs;
  int max_depth;           // deepest chain (joints from the root)
  int halves;              // waves per link: 1, or 2 (each with half of the slots)
  int link_waves;          // halves == 1: link waves (<= n_links); wave w takes links w,
                           //   w + link_waves, ... in passes
  int groups;              // slot groups per wave: 1, 2 or 4 (64 / groups evaluations per
                           //   workgroup, each lane group with its share of the slots;
                           //   halves == 1)
  int pm_rows;             // particle mode: rows of draws staged per workgroup (else 0)
  // cuboid slices over workgroups (gridDim.y > 1): per-slice partial sums
  // [chunk][slice][3 + D][64] and one arrival counter per chunk (zero
  // between launches; the last workgroup of a chunk resets it)
  float* part;
  int* count;
  // self-collision: [n_self] pairs {sphere i, sphere j, link_i | link_j << 16,
  // bits of r_i + r_j}, and the sphere index of every slot [L][maxs]
  const int4* self_pairs;
  const int* slot_sphere;
};

// LDS of a wave-per-link workgroup.  First a region that holds, in turn,
// the self-collision phase's sphere centres and per-wave winners, then the
// waves' parts: per link 16 floats per evaluation (cost, clearance,
// directional derivative, own joint's terms, wrench, frame z axis and
// origin), the joint wave's 3 + D (cost, clearance, directional
// derivative, joint terms), and with two waves per link the halves'
// hand-over (9 per link).  Then what the workgroup stages once: rows of x
// and d, joint limits and start, goal poses and tool transforms, the chain
// records, sphere slots and two cuboid tiles (float4 aligned), and the
// slice ticket.
constexpr size_t kWlLdsMax = 160 * 1024;   // LDS of a gfx950 CU (the device may report less)
constexpr int kWlStageRows = kWave + 8;
constexpr int kWlBoxTile = 64;   // cuboids per staged tile
// bounding balls per link (link frame): all its slots, each half of them,
// each quarter (the slot groups of two and four groups per wave)
constexpr int kWlBalls = 7;
// E: evaluations per workgroup (64 / slot groups per wave).
constexpr int kWlPartsPerLink = 16;
__host__ __device__ inline size_t wl_region_floats(int L, int D, int max_depth, int n_spheres, bool self,
                                                   int halves, int E) {
  const size_t parts = ((size_t)L * kWlPartsPerLink + 3 + D + (halves == 2 ? 9 * (size_t)L : 0)) * E;
  const size_t waves = halves == 2 ? 2 * (size_t)L : (size_t)L + 1;
  const size_t selfb = self ? ((size_t)n_spheres * 3 + 2 * waves) * kWave : 0;
  return parts > selfb ? parts : selfb;
}
// float offsets of the staged tables
struct WlLds {
  size_t x, d, lim, goal, etf, chain, slot, box, tick, eps, total;
};
// pm_rows > 0 (particle mode): the draws of every lane's particle over the
// staged rows, [pm_rows][E][D]
__host__ __device__ inline WlLds wl_lds_layout(int L, int D, int max_depth, int n_spheres, bool self,
                                               int halves, int maxs, int E, int pm_rows = 0) {
  WlLds o;
  size_t at = wl_region_floats(L, D, max_depth, n_spheres, self, halves, E);
  auto take = [&at](size_t n) {
    const size_t r = at;
    at += (n + 3) & ~(size_t)3;
    return r;
  };
  o.x = take((size_t)kWlStageRows * D);
  o.d = take((size_t)kWlStageRows * D);
  o.lim = take(3 * (size_t)D);
  o.goal = take((size_t)kMaxEE * 7);
  o.etf = take((size_t)kMaxEE * 12);
  // chain records, sphere slots and the cuboid tiles are contiguous (float4)
  o.chain = take((size_t)L * max_depth * 16);
  o.slot = take((size_t)L * maxs * 4);
  o.box = take(2 * (size_t)kWlBoxTile * 16);
  o.tick = take(4);
  o.eps = take((size_t)pm_rows * E * D);
  o.total = at;
  return o;
}
__host__ __device__ inline size_t wl_lds_bytes(int L, int D, int max_depth, int n_spheres, bool self,
                                               int halves, int maxs, int E, int pm_rows = 0) {
  return wl_lds_layout(L, D, max_depth, n_spheres, self, halves, maxs, E, pm_rows).total * sizeof(float);
}

// Cuboid in the library layout: p = A c + b maps a world point into the box
// frame (A = R^T, b = -R^T t); h = half side lengths.
//   q[0] = A00 A01 A02 b0, q[1] = A10 A11 A12 b1, q[2] = A20 A21 A22 b2, q[3] = h0 h1 h2 0
struct Box {
  float4 q[4];
};

struct EvalArgs {
  Robot rb;
  Lanes ln;
  WaveLinks wl;
  Params pr;
  int slices;              // waves that split one evaluation group's cuboids: 1, 2 or 4
  const Problem* prob;     // [P]
  const int* chunk_prefix; // [P+1] workgroups before problem p (for this lane layout)
  int P;
  int rows;
  const Box* box;          // all worlds' cuboids
  const int* world_off;    // [W+1]
  const float* q_start;    // [P][D]
  const float* goal;       // [P][n_ee][7]
  const float* x;          // [rows][D]
  const float* d;          // [rows][D] direction (candidate mode) or null
  // particle mode (var != null): candidate k is clip(x + sqrt(var) d_k) with
  // d_k = d + k * d_stride standard normal draws; alpha is not used.  With
  // d null the kernel makes the draws itself: particle k's draw of element
  // e = row * D + j is the Philox-4x64-10 normal at counter {e / 4, k,
  // pm_it, 0}, key {pm_seed, 0}, word e mod 4
  const float* var;        // [rows][D] per-element variance or null
  union {
    size_t d_stride;               // d != null
    unsigned long long pm_seed;    // d == null
  };
  float alpha[kMaxK];
  int K;
  int pm_it;
  float* cost_e;           // [K][rows]
  float* gd_e;             // [K][rows] (candidate mode)
  float* mc_e;             // [K][rows]
  float* grad_e;           // [K][rows][D] (gradient mode)
  float* pe_e;             // [rows][2] position / rotation error at the last waypoint, or null
  // speed metric with gradients: per (candidate, row, sphere) the sphere's
  // collision cost times its unit chord / (2 dt), for the speed's gradient on
  // the neighbouring waypoints (speed_adjoint_kernel), or null
  float4* sp_h;            // [K][rows][M]
};

// The speed metric's gradient on the neighbouring waypoints (Eq.(11)): for
// every (candidate, row) the force h(t-1) - h(t+1) (+ h(t) at the last
// waypoint) on each sphere, projected on the joints and added to the
// evaluation's gradient (and directional derivative).
struct SpeedAdjArgs {
  const SeedInfo* seeds;
  int n_seeds, rows, dof, n_links, n_spheres, K, maxs;
  float alpha[kMaxK];
  int cand;                // candidates clip(x + alpha_k d) (else x itself)
  const float* fixed_tf;   // [L][12]
  const float* q_lo;
  const float* q_hi;
  const int4* info;        // [L]: chain depth, spheres, ...
  const float4* sphere;    // [L][maxs] centre in link frame + radius
  const int* slot_sphere;  // [L][maxs]
  const float* x;          // [rows][D]
  const float* d;          // [rows][D] or null
  const float4* sp_h;      // [K][rows][M]
  float* grad_e;           // [K][rows][D]
  float* gd_e;             // [K][rows] (candidates)
};

struct ReduceArgs {
  const SeedInfo* seeds;
  int n_seeds;
  const float* cost_e;     // [rows]
  const float* mc_e;       // [rows]
  float* cost;             // [seeds]
  float* min_clear;        // [seeds] or null
};

struct SelectArgs {
  const SeedInfo* seeds;
  int uniform_T;           // > 0: every seed has this horizon (seed s starts at row s T)
  int n_seeds, rows, dof, K, mode;
  float alpha[kMaxK];
  float eta1, eta_w;
  const float* q_lo;
  const float* q_hi;
  const float* x;          // [rows][D]
  const float* c0;         // [seeds]
  const float* g0;         // [rows][D]
  const float* d;          // [rows][D]
  const float* cost_e;     // [K][rows]
  const float* gd_e;
  const float* mc_e;
  const float* grad_e;     // [K][rows][D]
  float* x_out;            // may alias x
  float* c_out;            // may alias c0
  float* g_out;            // may alias g0
  int* chosen;             // or null
  float* mc_out;           // or null
  int track;               // best tracking: best_c / best_x updated when the cost improves
  float* best_c;           // [seeds] (read even without tracking)
  float* best_x;
};

struct LbfgsArgs {
  const SeedInfo* seeds;
  int uniform_T;           // > 0: every seed has this horizon (seed s starts at row s T)
  int n_seeds, rows, dof, m, reset;
  const float* x;
  const float* g;
  float* dir;
  float* S;                // [m_max][rows*D] history pairs, a ring
  float* Y;
  float* x_prev;           // [rows*D]
  float* g_prev;
  float* rho;              // [seeds][m_max]
  int* meta;               // [seeds][2]: count, head (next ring slot)
  int use_first;           // first[] is honoured (and cleared)
  int* first;              // [seeds] (read even when not used): 1 forces a reset for that seed
  int m_max;
  // the choice folded into the next evaluation launch: meta is read from
  // meta and written to meta_out (null: meta), and with keep_prev x_prev /
  // g_prev are only read (they are the iterate and gradient the choice
  // started from, which other workgroups of the launch still read)
  int* meta_out;
  int keep_prev;
};

// The line-search choice of the previous iteration and the next L-BFGS
// direction, computed at the start of an evaluation launch of the solve
// (every workgroup of a seed computes them; the seed's first workgroup
// stores them).  sa / la read one set of the solver's state and write the
// other.
struct SelFuse {
  SelectArgs sa;
  LbfgsArgs la;
};

// Particle stage update (Eq.(12)-(13)) of every seed after its particles
// were costed.
struct ParticleArgs {
  const SeedInfo* seeds;
  int n_seeds, rows, dof, N;
  float beta, k_mu, k_sigma;   // beta <= 0: 0.1 x the seed's cost range
  const float* q_lo;
  const float* q_hi;
  const float* cost_e;     // [N][rows] per-row particle costs
  const float* eps;        // [N][rows][D] this round's draws, or null: drawn
                           // here as the evaluation drew them (seed, it)
  unsigned long long seed;
  int it;
  float* mean;             // [rows][D] in/out
  float* var;              // [rows][D] in/out
  float* costs_out;        // [n_seeds][N] or null
};

// Retiming (Alg.4) of every seed: the spacing at which the seed's largest
// velocity, acceleration or jerk ratio to its limit reaches 1.
struct RetimeArgs {
  const SeedInfo* seeds;
  int n_seeds, dof;
  float dt;                // the spacing the trajectories are read at
  float inv_v[kMaxDof];    // 1 / limit per joint; 0 leaves the kind out
  float inv_a[kMaxDof];
  float inv_j[kMaxDof];
  const float* q_start;    // [P][D]
  const float* x;          // [rows][D]
  float* dt_out;           // [n_seeds]
  float* jerk_out;         // [n_seeds] largest |jerk| at the retimed spacing, or null
};

// Motion generation: IK seeds of every problem ranked, trajectory seeds on
// the line from the start to them (one workgroup per problem).
constexpr int kMaxIkSeeds = 1024;
struct IkSeedArgs {
  const Problem* ik;       // [P] (T = 1: one row per seed)
  const Problem* to;       // [P]
  int P, dof;
  const float* q_start;    // [P][D]
  const float* x_ik;       // [ik rows][D]
  const float* cost_e;     // [ik rows] cost of each IK seed
  const float* mc_e;       // [ik rows] clearance
  const float* pe_e;       // [ik rows][2] position / rotation error
  float pos_tol, rot_tol, w_dist;
  float* x_to;             // [to rows][D]
  int* ik_ok;              // [P] or null
};

// Parallel steering (Alg.3): samples of every edge, then the last valid one.
struct SteerArgs {
  int n_edges, n_max, dof;
  float res;               // largest joint step between samples
  const float* from;       // [n_edges][D]
  const float* to;         // [n_edges][D]
  const float* q_lo;
  const float* q_hi;
  float* pts;              // [n_edges][n_max + 1][D] samples
  const float* mc;         // [n_edges][n_max + 1] clearance of every sample
  float* reach;            // [n_edges][D]
  int* last;               // [n_edges]
  float* dist;             // [n_edges] or null
};

// k nearest nodes of every query (the planner's neighbour search).
struct KnnArgs {
  int n_nodes, n_queries, dof, k;
  const float* nodes;      // [n_nodes][D]
  const float* queries;    // [n_queries][D]
  int* idx;                // [n_queries][k] (-1 past the node count)
  float* d2;               // [n_queries][k] squared distances, or null
};

// Trajectory selection among the seeds of every problem (one thread each).
struct TrajSelectArgs {
  const Problem* prob;
  int P;
  const float* cost_e;     // [rows]
  const float* mc_e;       // [rows]
  const float* pe_e;       // [rows][2]
  const float* dt_s;       // [seeds] retimed spacing
  const float* jerk_s;     // [seeds] largest |jerk| at that spacing
  float pos_tol, rot_tol, w_jerk, w_time;
  int* best_seed;          // [P]
  int* success;            // [P] or null
  float* motion_time;      // [P] or null
};

// End-effector poses of every row (forward kinematics only).
struct EePoseArgs {
  int rows, dof, n_ee;
  int ee_link[kMaxEE];
  const float* fixed_tf;   // [L][12]
  const float* ee_tf;      // [n_ee][12]
  const int* chain;        // [L][kMaxDof] links from the root down to l
  const int4* info;        // [L]: chain depth, ...
  const float* q;          // [rows][D]
  float* pose;             // [rows][n_ee][7]
};

struct FinalArgs {
  const Problem* prob;
  int P, rows;
  const float* best_c;     // [seeds]
  const float* pe_e;       // [rows][2]
  const float* mc_e;       // [rows]
  float success_pos, success_rot;
  int* best_seed;          // [P] or null
  int* success;            // [P] or null
};

// Launchers (mg_kernels.hip).  Each returns the hipError_t of the launch.
hipError_t launch_eval(const EvalArgs& a, int grid_x, bool cand, bool grad, hipStream_t s);
// wave-per-link layout: grid_x workgroups of 64 evaluations (chunk_prefix
// counts 64-evaluation chunks of rows x K per problem)
// fs (or null): the previous choice folded into this launch (cost and
// gradient of candidates, the wave-per-link layout with one joint wave and
// link waves alone, no swept collision or speed metric)
hipError_t launch_eval_wl(const EvalArgs& a, int grid_x, int slices, bool cand, bool grad, hipStream_t s,
                          const SelFuse* fs = nullptr);
hipError_t launch_reduce(const ReduceArgs& a, hipStream_t s);
hipError_t launch_speed_adjoint(const SpeedAdjArgs& a, hipStream_t s);
// fuse (optional): compute the next L-BFGS direction from the chosen iterate
hipError_t launch_select(const SelectArgs& a, int max_n, const LbfgsArgs* fuse, hipStream_t s);
hipError_t launch_lbfgs(const LbfgsArgs& a, int max_n, hipStream_t s);

hipError_t launch_particle_update(const ParticleArgs& a, hipStream_t s);
// standard normal draws [n_iters][N][n] of rounds it0 .. it0 + n_iters - 1
// (Philox-4x64-10 + Box-Muller, mg_device.h)
hipError_t launch_philox_normals(unsigned long long seed, int it0, int n_iters, int N, long long n, float* out,
                                 hipStream_t s);
hipError_t launch_retime(const RetimeArgs& a, hipStream_t s);
hipError_t launch_ik_seeds(const IkSeedArgs& a, hipStream_t s);
hipError_t launch_traj_select(const TrajSelectArgs& a, hipStream_t s);
hipError_t launch_steer_points(const SteerArgs& a, hipStream_t s);
hipError_t launch_steer_scan(const SteerArgs& a, hipStream_t s);
hipError_t launch_knn(const KnnArgs& a, hipStream_t s);
hipError_t launch_final(const FinalArgs& a, hipStream_t s);
hipError_t launch_ee_pose(const EePoseArgs& a, hipStream_t s);
hipError_t launch_boxes(const float* pose, const float* dims, int n, Box* out, hipStream_t s);
hipError_t launch_copy(const float* src, float* dst, size_t n, hipStream_t s);
hipError_t launch_fill_i32(int* dst, int v, size_t n, hipStream_t s);

}  // namespace mg
