// mg_api.hip -- C ABI of libmg (declared in include/mg.h).
//
// Host-side bookkeeping only: argument checks, device tables, workspaces,
// launch sequencing and hipGraph capture of the solver iteration.  All
// arithmetic of the method runs in the kernels of mg_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <mutex>
#include <queue>
#include <random>
#include <string>
#include <vector>

#include "../../include/mg.h"
#include "mg_internal.h"

using mg::Box;

namespace {

thread_local std::string g_last_error;

mg_status fail(mg_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

#define HIP_TRY(expr)                                                                    \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return fail(MG_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));           \
  } while (0)

template <typename T>
mg_status dev_alloc(T** p, size_t n) {
  *p = nullptr;
  if (n == 0) n = 1;
  hipError_t e = hipMalloc(reinterpret_cast<void**>(p), n * sizeof(T));
  if (e != hipSuccess) return fail(MG_ERR_OOM, "hipMalloc(%zu bytes): %s", n * sizeof(T), hipGetErrorString(e));
  return MG_OK;
}

template <typename T>
mg_status dev_upload(T** p, const std::vector<T>& v) {
  mg_status st = dev_alloc(p, v.size());
  if (st != MG_OK) return st;
  if (!v.empty()) HIP_TRY(hipMemcpy(*p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return MG_OK;
}

template <typename T>
void dev_free(T*& p) {
  if (p) (void)hipFree(const_cast<void*>(reinterpret_cast<const void*>(p)));
  p = nullptr;
}

// Cuboid slices per evaluation group offered by the evaluation kernel.
constexpr int kNumSlices = 3;
constexpr int kSlices[kNumSlices] = {1, 2, 4};

}  // namespace

struct mg_ctx {
  int device = 0;
  int L = 0, D = 0, M = 0, n_ee = 0;
  int lpe = 8, maxs = 4;     // lanes per evaluation, sphere slots per link
  std::vector<int> parent, joint, sphere_link, ee_link;
  std::vector<float> fixed_tf, sphere, ee_tf, q_lo, q_hi;
  mg::Params params{};
  float* d_fixed_tf = nullptr;
  float* d_zero = nullptr;     // zeros standing in for a start where none matters
  float* d_goal_id = nullptr;  // identity poses standing in for a goal where none matters
  int* d_joint = nullptr;
  float* d_q_lo = nullptr;
  float* d_q_hi = nullptr;
  float* d_ee_tf = nullptr;
  int4* d_lane_info = nullptr;
  float4* d_lane_sphere = nullptr;
  int4* d_wl_info = nullptr;     // wave-per-link tables
  int* d_wl_chain = nullptr;
  float4* d_wl_ball = nullptr;
  int* d_slot_sphere = nullptr;  // [L][maxs] sphere index of each slot
  std::vector<int> slot_of;      // [M] slot (link * maxs + position) of each sphere
  float4* d_chain_rec = nullptr; // [L][kMaxDof][4] chain transforms and joints
  int* d_joint_rec = nullptr;    // [D][2] chain position and subtree mask per joint
  int max_depth = 0;             // deepest chain
  int n_self = 0;                // self-collision pairs
  int self_cap = 0;
  int4* d_self_pairs = nullptr;
  Box* d_box = nullptr;
  int box_cap = 0, n_boxes = 0;
  int* d_world_off = nullptr;
  int world_cap = 0, n_worlds = 0;
  size_t lds_max = 64 * 1024;    // LDS one workgroup may hold on this device
  std::vector<int> world_off;    // host copy of the cuboid offsets
  std::vector<mg_batch*> batches;   // live batches (their chunk records name cuboid ranges)
  hipStream_t cap_stream = nullptr;
  float* d_scratch = nullptr;    // this device's copy of the static scratch array
};

struct mg_batch {
  mg_ctx* ctx = nullptr;
  int P = 0, n_seeds = 0, rows = 0, K_max = 0, m_max = 0;
  std::vector<int> seeds, horizon, world;
  mg::Problem* d_prob = nullptr;
  mg::SeedInfo* d_seed = nullptr;
  int* d_chunk[kNumSlices] = {nullptr, nullptr, nullptr};
  int chunks[kNumSlices] = {0, 0, 0};
  int max_n = 0;      // largest T*D of a seed
  int uniform_T = 0;  // the horizon when every problem has the same one, else 0
  float *cost_e = nullptr, *gd_e = nullptr, *mc_e = nullptr, *grad_e = nullptr, *pe_e = nullptr;
  float *c_cur = nullptr, *g_cur = nullptr, *dir = nullptr, *best_c = nullptr, *best_x = nullptr;
  float *sel_dt = nullptr, *sel_jerk = nullptr;   // per-seed retimed spacing and jerk (selection)
  int* first = nullptr;
  float *S = nullptr, *Y = nullptr, *x_prev = nullptr, *g_prev = nullptr, *rho = nullptr;
  int* meta = nullptr;
  // the solver's second set of state (iterate, cost, gradient, direction,
  // history count/head, evaluation outputs) for iterations whose choice is
  // folded into the next evaluation launch: launch i reads one set and
  // writes the other
  float *fs_x = nullptr, *fs_c = nullptr, *fs_g = nullptr, *fs_dir = nullptr;
  float *fs_cost_e = nullptr, *fs_gd_e = nullptr, *fs_mc_e = nullptr, *fs_grad_e = nullptr;
  int* fs_meta = nullptr;
  bool fusion = true;   // mg_batch_set_fusion
  // cached solver graph and the arguments it was captured with
  hipGraphExec_t gexec = nullptr;
  std::vector<char> gkey;
  // evaluation-kernel timing (mg_set_timing): event pairs used as a ring
  bool timing = false;
  std::vector<hipEvent_t> ev_start, ev_stop;
  int ev_next = 0, ev_count = 0;
  int slices = -1;    // forced cuboid slices index (-1: automatic)
  int layout = -1;    // evaluation layout: -1 automatic, 0 lane per link, 1 wave per link
  bool layout_set = false;   // the layout came from mg_batch_set_layout (not the autotuner)
  // wave-per-link chunks of 64 evaluations, per candidate count K
  // ([K][gi]: 64 >> gi evaluations per chunk, for 1 << gi slot groups)
  mg::WlChunk* d_chunk_wl[mg::kMaxK + 1][3] = {};
  int chunks_wl[mg::kMaxK + 1][3] = {};
  int wl_slices = 0;        // wave-per-link cuboid slices over workgroups (0: automatic)
  int wl_halves = 0;        // wave-per-link waves per link: 1, 2 (0: automatic)
  int wl_groups = 1;        // wave-per-link slot groups per wave: 1, 2, 4
  int wl_slices_max = 1;    // largest the scratch below holds
  float* wl_part = nullptr; // [chunks][slices][3 + D][64]
  int* wl_count = nullptr;  // [chunks], zero between launches
  // particle stage: per-row costs of every particle [p_cap][rows], and
  // wave-per-link chunk records for pm_K particles per row
  float* p_cost = nullptr;
  int p_cap = 0;
  int pm_K = 0;
  mg::WlChunk* d_chunk_pm[3] = {};
  int chunks_pm[3] = {};
  // speed metric with gradients: per (candidate, row, sphere) terms of the
  // speed's gradient [K_max][rows][M] (allocated while the metric is on)
  float4* sp_h = nullptr;
};

namespace {

mg::Robot dev_robot(const mg_ctx* c) {
  mg::Robot r;
  r.dof = c->D;
  r.n_links = c->L;
  r.n_ee = c->n_ee;
  r.n_spheres = c->M;
  r.fixed_tf = c->d_fixed_tf;
  r.q_lo = c->d_q_lo;
  r.q_hi = c->d_q_hi;
  r.ee_tf = c->d_ee_tf;
  return r;
}

// Lane layout: lane l of an evaluation owns link l.  Each lane records the
// lanes where its chain starts and ends, its spheres and its end effector.
mg_status build_lanes(mg_ctx* c) {
  c->lpe = c->L <= 8 ? 8 : 16;
  std::vector<int> count(c->L, 0);
  for (int m = 0; m < c->M; ++m) count[c->sphere_link[m]]++;
  int most = 0;
  for (int l = 0; l < c->L; ++l) most = std::max(most, count[l]);
  c->maxs = most <= 4 ? 4 : most <= 8 ? 8 : 16;
  if (most > 16) return fail(MG_ERR_UNSUPPORTED, "a link carries %d spheres (at most 16)", most);
  const int lpe = c->lpe, maxs = c->maxs;
  std::vector<int4> info(lpe);
  std::vector<float4> sph((size_t)lpe * maxs, make_float4(0.0f, 0.0f, 0.0f, 0.0f));
  std::vector<int> fill(lpe, 0);
  for (int l = 0; l < lpe; ++l) {
    if (l >= c->L) { info[l] = make_int4(l, l + 1, 0, -1); continue; }
    int start = l;
    while (c->parent[start] >= 0) start = c->parent[start];
    int end = l + 1;
    while (end < c->L && c->parent[end] == end - 1) ++end;
    int ee = -1;
    for (int e = 0; e < c->n_ee; ++e)
      if (c->ee_link[e] == l) ee = e;
    info[l] = make_int4(start, end, count[l], ee);
  }
  std::vector<int> slot_sphere((size_t)lpe * maxs, 0);
  for (int m = 0; m < c->M; ++m) {
    const int l = c->sphere_link[m];
    slot_sphere[(size_t)l * maxs + fill[l]] = m;
    c->slot_of.push_back(l * maxs + fill[l]);
    sph[(size_t)l * maxs + fill[l]++] =
        make_float4(c->sphere[4 * m + 0], c->sphere[4 * m + 1], c->sphere[4 * m + 2], c->sphere[4 * m + 3]);
  }
  // wave-per-link: chain of every link (root first) and a ball around its
  // spheres in the link frame (centre of their bounding box, radius to the
  // farthest sphere surface)
  std::vector<int4> wl_info(c->L);
  std::vector<int> wl_chain((size_t)c->L * mg::kMaxDof, 0);
  std::vector<float4> chain_rec((size_t)c->L * mg::kMaxDof * 4, make_float4(0.0f, 0.0f, 0.0f, 0.0f));
  std::vector<float4> wl_ball((size_t)c->L * mg::kWlBalls, make_float4(0.0f, 0.0f, 0.0f, 0.0f));
  // ball around slots [s0, s1) of link l: centre of their bounding box,
  // radius to the farthest sphere surface (slightly widened)
  auto ball_of = [&](int l, int s0, int s1) {
    if (s1 <= s0) return make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    float lo[3] = {3e38f, 3e38f, 3e38f}, hi[3] = {-3e38f, -3e38f, -3e38f};
    for (int s = s0; s < s1; ++s) {
      const float4 q = sph[(size_t)l * maxs + s];
      const float v[3] = {q.x, q.y, q.z};
      for (int i = 0; i < 3; ++i) { lo[i] = std::min(lo[i], v[i]); hi[i] = std::max(hi[i], v[i]); }
    }
    const float ctr[3] = {0.5f * (lo[0] + hi[0]), 0.5f * (lo[1] + hi[1]), 0.5f * (lo[2] + hi[2])};
    double rad = 0.0;
    for (int s = s0; s < s1; ++s) {
      const float4 q = sph[(size_t)l * maxs + s];
      const double dx = q.x - ctr[0], dy = q.y - ctr[1], dz = q.z - ctr[2];
      rad = std::max(rad, std::sqrt(dx * dx + dy * dy + dz * dz) + q.w);
    }
    return make_float4(ctr[0], ctr[1], ctr[2], (float)(rad * 1.0001 + 1e-6));
  };
  for (int l = 0; l < c->L; ++l) {
    std::vector<int> ch;
    for (int u = l; u >= 0; u = c->parent[u]) ch.push_back(u);
    if ((int)ch.size() > mg::kMaxDof) return fail(MG_ERR_UNSUPPORTED, "chain of link %d deeper than %d", l, mg::kMaxDof);
    for (size_t i = 0; i < ch.size(); ++i) {
      const int u = ch[ch.size() - 1 - i];
      wl_chain[(size_t)l * mg::kMaxDof + i] = u;
      float4* r = &chain_rec[((size_t)l * mg::kMaxDof + i) * 4];
      for (int k = 0; k < 3; ++k)
        r[k] = make_float4(c->fixed_tf[u * 12 + 4 * k + 0], c->fixed_tf[u * 12 + 4 * k + 1],
                           c->fixed_tf[u * 12 + 4 * k + 2], c->fixed_tf[u * 12 + 4 * k + 3]);
      int j = c->joint[u];
      float jf;
      memcpy(&jf, &j, sizeof(jf));
      r[3] = make_float4(jf, 0.0f, 0.0f, 0.0f);
    }
    int ee = -1;
    for (int e = 0; e < c->n_ee; ++e)
      if (c->ee_link[e] == l) ee = e;
    wl_info[l] = make_int4((int)ch.size(), count[l], ee, 0);
    c->max_depth = std::max(c->max_depth, (int)ch.size());
    // balls of all the link's slots, of each half and of each quarter
    const int half = maxs / 2, quarter = maxs / 4;
    float4* bl = &wl_ball[(size_t)mg::kWlBalls * l];
    bl[0] = ball_of(l, 0, count[l]);
    bl[1] = ball_of(l, 0, std::min(count[l], half));
    bl[2] = ball_of(l, half, count[l]);
    for (int q = 0; q < 4; ++q)
      bl[3 + q] = ball_of(l, std::min(count[l], q * quarter), q == 3 ? count[l] : std::min(count[l], (q + 1) * quarter));
  }
  mg_status st;
  if ((st = dev_upload(&c->d_lane_info, info)) != MG_OK) return st;
  if ((st = dev_upload(&c->d_wl_info, wl_info)) != MG_OK) return st;
  if ((st = dev_upload(&c->d_wl_chain, wl_chain)) != MG_OK) return st;
  if ((st = dev_upload(&c->d_wl_ball, wl_ball)) != MG_OK) return st;
  if ((st = dev_upload(&c->d_slot_sphere, slot_sphere)) != MG_OK) return st;
  if ((st = dev_upload(&c->d_chain_rec, chain_rec)) != MG_OK) return st;
  // joint j drives link j: its chain position is that link's depth - 1, and
  // it is on the chain of every link whose chain passes through link j
  std::vector<int> joint_rec(2 * (size_t)c->D, 0);
  for (int l = 0; l < c->L; ++l) {
    const int d = wl_info[l].x;
    for (int i = 0; i < d; ++i) {
      const int u = wl_chain[(size_t)l * mg::kMaxDof + i];
      joint_rec[2 * u + 0] = i;
      if (l < 31) joint_rec[2 * u + 1] |= 1 << l;
    }
  }
  if ((st = dev_upload(&c->d_joint_rec, joint_rec)) != MG_OK) return st;
  return dev_upload(&c->d_lane_sphere, sph);
}

mg::Lanes dev_lanes(const mg_ctx* c) {
  mg::Lanes ln;
  ln.lpe = c->lpe;
  ln.maxs = c->maxs;
  ln.info = c->d_lane_info;
  ln.sphere = c->d_lane_sphere;
  return ln;
}

mg::WaveLinks dev_wave_links(const mg_ctx* c) {
  mg::WaveLinks wl{};
  wl.info = c->d_wl_info;
  wl.chain = c->d_wl_chain;
  wl.sphere = c->d_lane_sphere;
  wl.ball = c->d_wl_ball;
  wl.maxs = c->maxs;
  wl.max_depth = c->max_depth;
  wl.halves = 1;
  // at most 8 waves per workgroup (two per SIMD, the full register budget):
  // a robot of more than 7 links runs its links in passes of 7, except with
  // self-collision, whose phase needs every link's spheres at once
  wl.link_waves = (c->n_self == 0 && c->L + 1 > 8) ? 7 : c->L;
  wl.part = nullptr;
  wl.count = nullptr;
  wl.self_pairs = c->d_self_pairs;
  wl.slot_sphere = c->d_slot_sphere;
  wl.chain_rec = c->d_chain_rec;
  wl.joint_rec = c->d_joint_rec;
  return wl;
}

// Identity poses (xyz 0, quaternion 1 0 0 0), one per end effector.
mg_status upload_identity_goals(mg_ctx* c) {
  std::vector<float> g((size_t)7 * c->n_ee, 0.0f);
  for (int e = 0; e < c->n_ee; ++e) g[7 * e + 3] = 1.0f;
  return dev_upload(&c->d_goal_id, g);
}

// The wave-per-link layout needs a workgroup of L + 1 waves.
bool wl_possible(const mg_ctx* c, bool self) {
  return c->L + 1 <= 16 &&
         mg::wl_lds_bytes(c->L, c->D, c->max_depth, c->M, self, 1, c->maxs, mg::kWave) <= c->lds_max;
}
// two waves per link: at most 8 links (16 waves) and the LDS for the hand-over
bool wl_halves_possible(const mg_ctx* c) {
  return 2 * c->L <= 16 &&
         mg::wl_lds_bytes(c->L, c->D, c->max_depth, c->M, c->n_self > 0, 2, c->maxs, mg::kWave) <= c->lds_max;
}
bool wl_possible(const mg_ctx* c) { return wl_possible(c, c->n_self > 0); }
// terms only the wave-per-link layout evaluates: self-collision, the speed metric
bool needs_wl(const mg_ctx* c) { return c->n_self > 0 || c->params.speed; }
// G slot groups per wave (64 / G evaluations per workgroup): no
// self-collision, at least two sphere slots per group
bool wl_groups_possible(const mg_ctx* c, int G = 2) {
  return c->L + 1 <= 16 && c->n_self == 0 && c->maxs >= 2 * G &&
         mg::wl_lds_bytes(c->L, c->D, c->max_depth, c->M, false, 1, c->maxs, mg::kWave / G) <= c->lds_max;
}
// index of a slot-group count in the chunk-record tables
int groups_index(int G) { return G == 4 ? 2 : G == 2 ? 1 : 0; }

// Layout of an evaluation launch with K candidates.
bool use_wl(const mg_batch* b, int K) {
  const mg_ctx* c = b->ctx;
  if (!wl_possible(c) || K > b->K_max) return false;
  if (needs_wl(c)) return true;     // self-collision and the speed metric live in this layout only
  if (b->layout >= 0) return b->layout == 1;
  const char* env = getenv("MG_EVAL_LAYOUT");
  if (env) return atoi(env) == 1;
  return false;
}

mg::Params to_dev(const mg_params& p) {
  mg::Params d;
  d.a0 = p.a0; d.a1 = p.a1; d.a2 = p.a2; d.a3 = p.a3;
  d.a6 = p.a6; d.a7 = p.a7; d.a8 = p.a8; d.a9 = p.a9;
  d.w_bound = p.w_bound; d.eta2 = p.eta2; d.w_coll = p.w_coll; d.eta = p.eta; d.dt = p.dt;
  d.vel_all = p.vel_all; d.swept = p.swept; d.sweep_steps = p.sweep_steps;
  d.ls_eta1 = p.ls_eta1; d.ls_eta_w = p.ls_eta_w;
  d.success_pos = p.success_pos; d.success_rot = p.success_rot;
  d.w_self = p.w_self; d.n_self = 0; d.speed = p.speed;
  return d;
}

mg_status check_params(const mg_params* p) {
  if (!p) return fail(MG_ERR_ARG, "params is null");
  if (!(p->dt > 0)) return fail(MG_ERR_ARG, "dt must be > 0");
  if (!(p->eta >= 0) || !(p->eta2 > 0)) return fail(MG_ERR_ARG, "eta must be >= 0 and eta2 > 0");
  if (p->swept && (p->sweep_steps < 0 || p->sweep_steps > 64))
    return fail(MG_ERR_ARG, "sweep_steps must be in [0, 64] (got %d)", p->sweep_steps);
  if (p->speed != 0 && p->speed != 1) return fail(MG_ERR_ARG, "speed must be 0 or 1");
  return MG_OK;
}

// Cuboid slices for a call evaluating n_evals rows x candidates: the fewest
// slices (least repeated kinematics) that still give every SIMD about four
// wavefronts; MG_CUBOID_SLICES forces a choice.
int pick_slices(const mg_batch* b, long n_evals) {
  if (b->ctx->params.swept) return 0;   // the swept kernels take whole worlds
  if (b->slices >= 0) return b->slices;
  const char* env = getenv("MG_CUBOID_SLICES");
  if (env) {
    const int h = atoi(env);
    for (int i = 0; i < kNumSlices; ++i)
      if (kSlices[i] == h) return i;
  }
  const long waves1 = (n_evals * b->ctx->lpe + mg::kWave - 1) / mg::kWave;
  const long target = 256L * 4 * 4;   // CUs x SIMDs x waves
  for (int i = 0; i < kNumSlices; ++i)
    if (waves1 * kSlices[i] >= target) return i;
  return kNumSlices - 1;
}

mg::EvalArgs eval_args(const mg_ctx* c, const mg_batch* b, int hi, const float* q_start,
                       const float* goal, const float* x, const float* d, int K, const float* alpha) {
  mg::EvalArgs a;
  memset(&a, 0, sizeof(a));
  a.rb = dev_robot(c);
  a.ln = dev_lanes(c);
  a.wl = dev_wave_links(c);
  a.pr = c->params;
  a.pr.n_self = c->n_self;
  a.slices = kSlices[hi];
  a.prob = b->d_prob;
  a.chunk_prefix = b->d_chunk[hi];
  a.P = b->P;
  a.rows = b->rows;
  a.box = c->d_box;
  a.world_off = c->d_world_off;
  a.q_start = q_start;
  a.goal = goal;
  a.x = x;
  a.d = d;
  a.K = K;
  for (int k = 0; k < K && k < mg::kMaxK; ++k) a.alpha[k] = alpha ? alpha[k] : 0.0f;
  a.cost_e = b->cost_e;
  a.gd_e = b->gd_e;
  a.mc_e = b->mc_e;
  a.grad_e = b->grad_e;
  a.pe_e = nullptr;
  a.sp_h = c->params.speed ? b->sp_h : nullptr;
  return a;
}

// The speed metric's per-(candidate, row, sphere) buffer of a batch,
// allocated once the metric is on.
mg_status ensure_speed_buf(mg_batch* b) {
  if (b->sp_h || !b->ctx || !b->ctx->params.speed || b->ctx->M == 0) return MG_OK;
  return dev_alloc(&b->sp_h, (size_t)b->K_max * b->rows * b->ctx->M);
}

// Wave-per-link chunk records of a batch for K candidates per row and E
// evaluations per chunk, problem by problem, with the problem's cuboid
// range in the context's current worlds (empty for a world not set yet).
// Allocated on the first call, rewritten in place (synchronously) after.
mg_status wl_records(mg_batch* b, int K, int E, mg::WlChunk** dptr, int* count) {
  const mg_ctx* c = b->ctx;
  std::vector<mg::WlChunk> rec;
  int r0 = 0;
  for (int p = 0; p < b->P; ++p) {
    const int n_e = b->seeds[p] * b->horizon[p] * K;
    const int w = b->world[p];
    const bool set = w + 1 < (int)c->world_off.size();
    const int lo = set ? c->world_off[w] : 0, hi = set ? c->world_off[w + 1] : 0;
    for (int e = 0; e < n_e; e += E) rec.push_back(mg::WlChunk{p, e, b->seeds[p], b->horizon[p], lo, hi, r0, n_e});
    r0 += b->seeds[p] * b->horizon[p];
  }
  if (!*dptr || *count != (int)rec.size()) {
    dev_free(*dptr);
    mg_status st = dev_upload(dptr, rec);
    if (st != MG_OK) return st;
    *count = (int)rec.size();
  } else {
    HIP_TRY(hipMemcpy(*dptr, rec.data(), rec.size() * sizeof(mg::WlChunk), hipMemcpyHostToDevice));
  }
  return MG_OK;
}

// Every K <= K_max and both chunk sizes (64 and 32 evaluations), and the
// particle stage's records when particles are reserved.
mg_status wl_chunks_upload(mg_batch* b) {
  mg_status st;
  for (int K = 1; K <= b->K_max; ++K)
    for (int gi = 0; gi < 3; ++gi)
      if ((st = wl_records(b, K, mg::kWave >> gi, &b->d_chunk_wl[K][gi], &b->chunks_wl[K][gi])) != MG_OK)
        return st;
  if (b->pm_K > 0)
    for (int gi = 0; gi < 3; ++gi)
      if ((st = wl_records(b, b->pm_K, mg::kWave >> gi, &b->d_chunk_pm[gi], &b->chunks_pm[gi])) != MG_OK)
        return st;
  return MG_OK;
}

mg_status common_checks(mg_ctx* c, mg_batch* b) {
  if (!c || !b) return fail(MG_ERR_ARG, "null context or batch");
  if (b->ctx != c) return fail(MG_ERR_ARG, "batch belongs to another context");
  if (!c->d_world_off || c->n_worlds <= 0) return fail(MG_ERR_STATE, "no world set (mg_set_worlds)");
  for (int p = 0; p < b->P; ++p)
    if (b->world[p] >= c->n_worlds)
      return fail(MG_ERR_STATE, "problem %d uses world %d but only %d worlds are set", p, b->world[p], c->n_worlds);
  return MG_OK;
}

// Launch an evaluation in the batch's layout: lane per link (cuboid slices
// index hi) or wave per link.
// Wave-per-link slices: the forced count, else enough workgroups for two
// per CU.
// One problem: the wave-per-link kernel forms its chunk records from the
// workgroup index (the same records the table holds).
void wl_single(const mg_batch* b, int K, mg::WaveLinks& wl) {
  wl.one.S = 0;
  if (b->P != 1) return;
  const mg_ctx* c = b->ctx;
  const int w = b->world[0];
  const bool set = w + 1 < (int)c->world_off.size();
  wl.one.S = b->seeds[0];
  wl.one.T = b->horizon[0];
  wl.one.box_lo = set ? c->world_off[w] : 0;
  wl.one.box_hi = set ? c->world_off[w + 1] : 0;
  wl.one.n_e = b->seeds[0] * b->horizon[0] * K;
}

int wl_slices(const mg_batch* b, int K) {
  if (b->wl_slices > 0) return std::min(b->wl_slices, b->wl_slices_max);
  int h = 1;
  while (h < b->wl_slices_max && (long)b->chunks_wl[K][0] * h < 512) h *= 2;
  return h;
}

// slices_ok = false keeps the wave-per-link layout at one workgroup per
// chunk (no slice scratch or arrival counters of the batch).
hipError_t launch_layout(mg_batch* b, mg::EvalArgs a, int hi, bool cand, bool grad, hipStream_t s,
                         bool slices_ok = true, const mg::SelFuse* fs = nullptr) {
  if (use_wl(b, a.K)) {
    a.wl.part = b->wl_part;
    a.wl.count = b->wl_count;
    // two slot groups per wave when chosen; else two waves per link where
    // they fit (shorter waves), unless forced
    const int groups = b->wl_groups > 1 && wl_groups_possible(b->ctx, b->wl_groups) ? b->wl_groups : 1;
    const int halves = groups > 1 ? 1 : (b->wl_halves > 0 ? b->wl_halves : (wl_halves_possible(b->ctx) ? 2 : 1));
    if (halves == 2 && !wl_halves_possible(b->ctx)) return hipErrorInvalidValue;
    a.wl.halves = halves;
    a.wl.groups = groups;
    a.wl.chunk = b->d_chunk_wl[a.K][groups_index(groups)];
    wl_single(b, a.K, a.wl);
    // (the speed's gradient terms need every cuboid of a sphere in one workgroup)
    const int wls = (halves == 2 || groups > 1 || !slices_ok || (a.sp_h && grad)) ? 1 : wl_slices(b, a.K);
    return mg::launch_eval_wl(a, b->chunks_wl[a.K][groups_index(groups)], wls, cand, grad, s, fs);
  }
  if (fs) return hipErrorInvalidValue;
  return mg::launch_eval(a, b->chunks[hi], cand, grad, s);
}

// Per-(candidate, row) outputs of an evaluation launch held outside the
// batch (the allocation-free entry point's static scratch).
struct EvalOut {
  float *cost_e, *gd_e, *mc_e, *grad_e;
};

mg_status enqueue_eval(mg_ctx* c, mg_batch* b, const float* q_start, const float* goal,
                       const float* x, const float* d, int K, const float* alpha, bool grad,
                       float* grad_out, float* pe_out, hipStream_t s, const EvalOut* eo = nullptr) {
  if (needs_wl(c) && !use_wl(b, K))
    return fail(MG_ERR_UNSUPPORTED, "self-collision and the speed metric need the wave-per-link layout (at most 15 links)");
  const int hi = pick_slices(b, (long)b->rows * K);
  mg::EvalArgs a = eval_args(c, b, hi, q_start, goal, x, d, K, alpha);
  if (grad_out) a.grad_e = grad_out;
  if (eo) {
    a.cost_e = eo->cost_e;
    a.gd_e = eo->gd_e;
    a.mc_e = eo->mc_e;
    a.grad_e = eo->grad_e;
  }
  a.pe_e = pe_out;
  const int slot = b->ev_next;
  // events are recorded around direct launches only (an event recorded while
  // a stream is captured is a graph dependency, not a timestamp)
  bool timed = b->timing;
  if (timed) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(s, &cs));
    timed = cs == hipStreamCaptureStatusNone;
  }
  if (timed) HIP_TRY(hipEventRecord(b->ev_start[slot], s));
  if (c->params.speed && grad && !a.sp_h && c->M > 0)
    return fail(MG_ERR_STATE, "the speed metric's gradient buffer is missing");
  HIP_TRY(launch_layout(b, a, hi, d != nullptr, grad, s, eo == nullptr));
  if (timed) {
    HIP_TRY(hipEventRecord(b->ev_stop[slot], s));
    b->ev_next = (slot + 1) % (int)b->ev_start.size();
    b->ev_count = std::min(b->ev_count + 1, (int)b->ev_start.size());
  }
  if (a.sp_h && grad) {
    // the speed's gradient on the neighbouring waypoints (Eq.(11))
    mg::SpeedAdjArgs sa;
    memset(&sa, 0, sizeof(sa));
    sa.seeds = b->d_seed;
    sa.n_seeds = b->n_seeds;
    sa.rows = b->rows;
    sa.dof = c->D;
    sa.n_links = c->L;
    sa.n_spheres = c->M;
    sa.K = K;
    sa.maxs = c->maxs;
    for (int k = 0; k < K; ++k) sa.alpha[k] = alpha ? alpha[k] : 0.0f;
    sa.cand = d != nullptr;
    sa.fixed_tf = c->d_fixed_tf;
    sa.q_lo = c->d_q_lo;
    sa.q_hi = c->d_q_hi;
    sa.info = c->d_wl_info;
    sa.sphere = c->d_lane_sphere;
    sa.slot_sphere = c->d_slot_sphere;
    sa.x = x;
    sa.d = d;
    sa.sp_h = a.sp_h;
    sa.grad_e = a.grad_e;
    sa.gd_e = a.gd_e;
    HIP_TRY(mg::launch_speed_adjoint(sa, s));
  }
  return MG_OK;
}

mg::LbfgsArgs lbfgs_args(mg_ctx* c, mg_batch* b, int m, int reset, const float* x, const float* g,
                         float* dir, int* first) {
  mg::LbfgsArgs a;
  memset(&a, 0, sizeof(a));
  a.seeds = b->d_seed;
  a.uniform_T = b->uniform_T;
  a.n_seeds = b->n_seeds;
  a.rows = b->rows;
  a.dof = c->D;
  a.m = m;
  a.reset = reset;
  a.x = x; a.g = g; a.dir = dir;
  a.S = b->S; a.Y = b->Y; a.x_prev = b->x_prev; a.g_prev = b->g_prev;
  a.rho = b->rho; a.meta = b->meta;
  a.use_first = first != nullptr;
  a.first = first ? first : b->first;
  a.m_max = b->m_max;
  return a;
}

mg_status enqueue_select(mg_ctx* c, mg_batch* b, const float* x, const float* c0, const float* g0,
                         const float* d, int K, const float* alpha, int mode, float* x_out,
                         float* c_out, float* g_out, int* chosen, float* mc_out, bool track,
                         const mg::LbfgsArgs* fuse, hipStream_t s, const EvalOut* eo = nullptr) {
  mg::SelectArgs a;
  memset(&a, 0, sizeof(a));
  a.seeds = b->d_seed;
  a.uniform_T = b->uniform_T;
  a.n_seeds = b->n_seeds;
  a.rows = b->rows;
  a.dof = c->D;
  a.K = K;
  a.mode = mode;
  for (int k = 0; k < K; ++k) a.alpha[k] = alpha[k];
  a.eta1 = c->params.ls_eta1;
  a.eta_w = c->params.ls_eta_w;
  a.q_lo = c->d_q_lo;
  a.q_hi = c->d_q_hi;
  a.x = x; a.c0 = c0; a.g0 = g0; a.d = d;
  a.cost_e = b->cost_e; a.gd_e = b->gd_e; a.mc_e = b->mc_e; a.grad_e = b->grad_e;
  if (eo) { a.cost_e = eo->cost_e; a.gd_e = eo->gd_e; a.mc_e = eo->mc_e; a.grad_e = eo->grad_e; }
  a.x_out = x_out; a.c_out = c_out; a.g_out = g_out; a.chosen = chosen; a.mc_out = mc_out;
  a.track = track ? 1 : 0;
  a.best_c = b->best_c;
  a.best_x = b->best_x;
  HIP_TRY(mg::launch_select(a, b->max_n, fuse, s));
  return MG_OK;
}

mg_status enqueue_lbfgs(mg_ctx* c, mg_batch* b, int m, int reset, const float* x, const float* g,
                        float* dir, int* first, hipStream_t s) {
  const mg::LbfgsArgs a = lbfgs_args(c, b, m, reset, x, g, dir, first);
  HIP_TRY(mg::launch_lbfgs(a, b->max_n, s));
  return MG_OK;
}

// The solver folds each line-search choice into the next evaluation launch
// when the batch's layout and shapes allow it (the conditions of
// launch_eval_wl's fs path): wave per link (one, two or four slot groups)
// with a joint wave and no link passes, no swept collision or speed metric,
// one horizon with blocks of 129 to 256 floats (a multiple of 4: the
// separate choice then holds 4 per lane too, so both sum in the same order),
// at most 8 candidates and 4 history pairs, and workgroup chunks inside one
// seed.
bool fuse_ok(const mg_ctx* c, const mg_batch* b, int K, int m, const float* x) {
  if (!b->fusion || !use_wl(b, K) || c->params.swept || c->params.speed) return false;
  const int groups = b->wl_groups > 1 && wl_groups_possible(c, b->wl_groups) ? b->wl_groups : 1;
  const int halves = groups > 1 ? 1 : (b->wl_halves > 0 ? b->wl_halves : (wl_halves_possible(c) ? 2 : 1));
  if (halves != 1 || c->L + 1 > 8 || c->maxs / groups > 8) return false;
  const int T = b->uniform_T, E = mg::kWave / groups, n = T * c->D;
  return T > 0 && n > 2 * mg::kWave && n <= 4 * mg::kWave && n % 4 == 0 && K <= 8 && E % K == 0 && T % (E / K) == 0 && m >= 1 &&
         m <= 4 && ((uintptr_t)x & 15) == 0;
}

// The two sets of solver state: set 0 is the caller's x and the batch's
// usual buffers, set 1 the fs_ ones.
struct StateSet {
  float *x, *c, *g, *dir, *cost_e, *gd_e, *mc_e, *grad_e;
  int* meta;
};
StateSet state_set(mg_batch* b, float* x, int i) {
  if (i == 0) return StateSet{x, b->c_cur, b->g_cur, b->dir, b->cost_e, b->gd_e, b->mc_e, b->grad_e, b->meta};
  return StateSet{b->fs_x, b->fs_c, b->fs_g, b->fs_dir, b->fs_cost_e, b->fs_gd_e, b->fs_mc_e, b->fs_grad_e,
                  b->fs_meta};
}

mg_status check_K_alpha(const mg_batch* b, int K, const float* alpha) {
  if (K < 1 || K > b->K_max) return fail(MG_ERR_SHAPE, "K = %d outside 1..%d", K, b->K_max);
  if (!alpha) return fail(MG_ERR_ARG, "alpha is null");
  for (int k = 0; k < K; ++k)
    if (!(alpha[k] >= 0.0f)) return fail(MG_ERR_ARG, "alpha[%d] must be >= 0", k);
  return MG_OK;
}

}  // namespace

// Scratch of the allocation-free line search (mg_linesearch_noalloc): the
// per-(candidate, row) cost, directional derivative, clearance and
// gradient of one call.  Every GPU the library runs on holds its own copy
// (16 MiB) until the process ends.  Host code never passes the array's name
// to a kernel (on the host it is a stand-in, not a device address); it uses
// the per-device address from hipGetSymbolAddress.
static constexpr size_t kScratchFloats = (size_t)4 << 20;
static __device__ __align__(256) float scratch[kScratchFloats];

namespace {

std::mutex g_scratch_mu;
std::vector<float*> g_scratch_dev;   // per device ordinal: the address of `scratch`

// The current device's address of `scratch`, looked up once per device.
mg_status scratch_address(int device, float** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (device < 0) return fail(MG_ERR_ARG, "bad device ordinal %d", device);
  if ((int)g_scratch_dev.size() <= device) g_scratch_dev.resize(device + 1, nullptr);
  if (!g_scratch_dev[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(MG_ERR_HIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch_dev[device] = static_cast<float*>(p);
  }
  *out = g_scratch_dev[device];
  return MG_OK;
}

}  // namespace

extern "C" {

void mg_default_params(mg_params* p) {
  if (!p) return;
  memset(p, 0, sizeof(*p));
  p->a0 = 2000.0f; p->a1 = 350.0f; p->a2 = 100.0f; p->a3 = 100.0f;
  p->a6 = 5000.0f; p->a7 = 50.0f; p->a8 = 5000.0f; p->a9 = 1.0f;
  p->w_bound = 5000.0f; p->eta2 = 0.1f; p->w_coll = 5000.0f; p->eta = 0.025f; p->dt = 0.25f;
  p->vel_all = 0; p->swept = 0; p->sweep_steps = 4;
  p->ls_eta1 = 1e-4f; p->ls_eta_w = 0.9f;
  p->success_pos = 0.005f; p->success_rot = 0.05f;
  p->w_self = 5000.0f;
}

const char* mg_last_error(void) { return g_last_error.c_str(); }

mg_status mg_create(const mg_robot_desc* r, const mg_params* params, mg_ctx** out) {
  if (!out) return fail(MG_ERR_ARG, "out is null");
  *out = nullptr;
  if (!r) return fail(MG_ERR_ARG, "robot is null");
  mg_status st = check_params(params);
  if (st != MG_OK) return st;
  if (r->dof < 1 || r->dof > mg::kMaxDof) return fail(MG_ERR_SHAPE, "dof %d outside 1..%d", r->dof, mg::kMaxDof);
  if (r->n_links < 1 || r->n_links > 64) return fail(MG_ERR_SHAPE, "n_links %d outside 1..64", r->n_links);
  if (r->n_spheres < 0 || r->n_ee < 1 || r->n_ee > mg::kMaxEE) return fail(MG_ERR_SHAPE, "bad sphere / end-effector count");
  if (!r->parent || !r->joint || !r->fixed_tf || !r->ee_link || !r->ee_tf || !r->q_lo || !r->q_hi ||
      (r->n_spheres > 0 && (!r->sphere_link || !r->sphere)))
    return fail(MG_ERR_ARG, "null robot table");
  std::vector<int> jcount(r->dof, 0);
  for (int l = 0; l < r->n_links; ++l) {
    if (r->parent[l] >= l || r->parent[l] < -1) return fail(MG_ERR_ARG, "parent[%d] = %d is not a lower link", l, r->parent[l]);
    if (r->joint[l] < -1 || r->joint[l] >= r->dof) return fail(MG_ERR_ARG, "joint[%d] out of range", l);
    if (r->joint[l] >= 0) jcount[r->joint[l]]++;
  }
  for (int j = 0; j < r->dof; ++j)
    if (jcount[j] != 1) return fail(MG_ERR_ARG, "joint %d drives %d links (must be 1)", j, jcount[j]);
  // kinematic layout of the evaluation kernel: link l is driven by joint l and
  // hangs from link l-1 or from the base (chains that start at the base)
  if (r->n_links != r->dof || r->n_links > 16)
    return fail(MG_ERR_UNSUPPORTED, "need one joint per link and at most 16 links (got %d links, %d joints)",
                r->n_links, r->dof);
  for (int l = 0; l < r->n_links; ++l)
    if (r->joint[l] != l || (r->parent[l] != -1 && r->parent[l] != l - 1))
      return fail(MG_ERR_UNSUPPORTED, "link %d: need joint[l] = l and parent[l] in {-1, l-1}", l);
  for (int m = 0; m < r->n_spheres; ++m) {
    if (r->sphere_link[m] < 0 || r->sphere_link[m] >= r->n_links) return fail(MG_ERR_ARG, "sphere_link[%d] out of range", m);
    if (!(r->sphere[4 * m + 3] > 0)) return fail(MG_ERR_ARG, "sphere %d radius must be > 0", m);
  }
  for (int e = 0; e < r->n_ee; ++e)
    if (r->ee_link[e] < 0 || r->ee_link[e] >= r->n_links) return fail(MG_ERR_ARG, "ee_link[%d] out of range", e);
  for (int j = 0; j < r->dof; ++j)
    if (!(r->q_lo[j] <= r->q_hi[j])) return fail(MG_ERR_ARG, "q_lo[%d] > q_hi[%d]", j, j);

  mg_ctx* c = new mg_ctx();
  (void)hipGetDevice(&c->device);
  if ((st = scratch_address(c->device, &c->d_scratch)) != MG_OK) {
    delete c;
    return st;
  }
  {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device) == hipSuccess && v > 0)
      c->lds_max = std::min((size_t)v, mg::kWlLdsMax);
  }
  c->L = r->n_links; c->D = r->dof; c->M = r->n_spheres; c->n_ee = r->n_ee;
  c->parent.assign(r->parent, r->parent + c->L);
  c->joint.assign(r->joint, r->joint + c->L);
  c->fixed_tf.assign(r->fixed_tf, r->fixed_tf + 12 * c->L);
  c->sphere_link.assign(r->sphere_link, r->sphere_link + c->M);
  c->sphere.assign(r->sphere, r->sphere + 4 * c->M);
  c->ee_link.assign(r->ee_link, r->ee_link + c->n_ee);
  c->ee_tf.assign(r->ee_tf, r->ee_tf + 12 * c->n_ee);
  c->q_lo.assign(r->q_lo, r->q_lo + c->D);
  c->q_hi.assign(r->q_hi, r->q_hi + c->D);
  c->params = to_dev(*params);
  if ((st = dev_upload(&c->d_fixed_tf, c->fixed_tf)) != MG_OK ||
      (st = dev_upload(&c->d_joint, c->joint)) != MG_OK ||
      (st = dev_upload(&c->d_q_lo, c->q_lo)) != MG_OK ||
      (st = dev_upload(&c->d_q_hi, c->q_hi)) != MG_OK ||
      (st = dev_upload(&c->d_ee_tf, c->ee_tf)) != MG_OK ||
      (st = dev_upload(&c->d_zero, std::vector<float>(c->D, 0.0f))) != MG_OK ||
      (st = upload_identity_goals(c)) != MG_OK ||
      (st = build_lanes(c)) != MG_OK) {
    mg_destroy(c);
    return st;
  }
  hipError_t e = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking);
  if (e != hipSuccess) { mg_destroy(c); return fail(MG_ERR_HIP, "hipStreamCreate: %s", hipGetErrorString(e)); }
  *out = c;
  return MG_OK;
}

void mg_destroy(mg_ctx* c) {
  if (!c) return;
  (void)hipDeviceSynchronize();
  for (mg_batch* b : c->batches) b->ctx = nullptr;   // (batches outliving their context)
  dev_free(c->d_fixed_tf); dev_free(c->d_joint); dev_free(c->d_q_lo); dev_free(c->d_q_hi); dev_free(c->d_ee_tf);
  dev_free(c->d_zero); dev_free(c->d_goal_id);
  dev_free(c->d_lane_info); dev_free(c->d_lane_sphere);
  dev_free(c->d_wl_info); dev_free(c->d_wl_chain); dev_free(c->d_wl_ball);
  dev_free(c->d_slot_sphere); dev_free(c->d_self_pairs); dev_free(c->d_chain_rec); dev_free(c->d_joint_rec);
  dev_free(c->d_box); dev_free(c->d_world_off);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  delete c;
}

mg_status mg_set_params(mg_ctx* c, const mg_params* params) {
  if (!c) return fail(MG_ERR_ARG, "null context");
  mg_status st = check_params(params);
  if (st != MG_OK) return st;
  if (params->speed && !wl_possible(c))
    return fail(MG_ERR_UNSUPPORTED, "the speed metric needs the wave-per-link layout (at most 15 links)");
  c->params = to_dev(*params);
  for (mg_batch* b : c->batches)
    if ((st = ensure_speed_buf(b)) != MG_OK) return st;
  return MG_OK;
}

mg_status mg_set_worlds(mg_ctx* c, int n_worlds, const int* offsets, const float* pose,
                        const float* dims, void* stream) {
  if (!c) return fail(MG_ERR_ARG, "null context");
  if (n_worlds < 1 || !offsets) return fail(MG_ERR_ARG, "need n_worlds >= 1 and offsets");
  if (offsets[0] != 0) return fail(MG_ERR_ARG, "offsets[0] must be 0");
  for (int w = 0; w < n_worlds; ++w)
    if (offsets[w + 1] < offsets[w]) return fail(MG_ERR_ARG, "offsets must be non-decreasing");
  const int n = offsets[n_worlds];
  if (n > 0 && (!pose || !dims)) return fail(MG_ERR_ARG, "null pose or dims");
  hipStream_t s = static_cast<hipStream_t>(stream);
  mg_status st;
  if (n > c->box_cap) {
    HIP_TRY(hipStreamSynchronize(s));
    dev_free(c->d_box);
    if ((st = dev_alloc(&c->d_box, n)) != MG_OK) return st;
    c->box_cap = n;
  }
  if (n_worlds + 1 > c->world_cap) {
    HIP_TRY(hipStreamSynchronize(s));
    dev_free(c->d_world_off);
    if ((st = dev_alloc(&c->d_world_off, n_worlds + 1)) != MG_OK) return st;
    c->world_cap = n_worlds + 1;
  }
  // offsets are tiny host data; a synchronous copy keeps the host array free
  HIP_TRY(hipStreamSynchronize(s));
  HIP_TRY(hipMemcpy(c->d_world_off, offsets, (n_worlds + 1) * sizeof(int), hipMemcpyHostToDevice));
  HIP_TRY(mg::launch_boxes(pose, dims, n, c->d_box, s));
  c->n_boxes = n;
  c->n_worlds = n_worlds;
  c->world_off.assign(offsets, offsets + n_worlds + 1);
  // the batches' chunk records carry their worlds' cuboid ranges
  for (mg_batch* b : c->batches)
    if ((st = wl_chunks_upload(b)) != MG_OK) return st;
  return MG_OK;
}

mg_status mg_batch_create(mg_ctx* c, int P, const int* seeds, const int* horizon, const int* world,
                          int K_max, int m_max, mg_batch** out) {
  if (!out) return fail(MG_ERR_ARG, "out is null");
  *out = nullptr;
  if (!c || !seeds || !horizon || !world) return fail(MG_ERR_ARG, "null argument");
  if (P < 1) return fail(MG_ERR_SHAPE, "P must be >= 1");
  if (K_max < 1 || K_max > mg::kMaxK) return fail(MG_ERR_SHAPE, "K_max outside 1..%d", mg::kMaxK);
  if (m_max < 0 || m_max > mg::kMaxHist) return fail(MG_ERR_SHAPE, "m_max outside 0..%d", mg::kMaxHist);
  long rows = 0, n_seeds = 0;
  for (int p = 0; p < P; ++p) {
    if (seeds[p] < 1) return fail(MG_ERR_SHAPE, "problem %d: seeds must be >= 1", p);
    if (horizon[p] < 1 || horizon[p] > mg::kMaxT) return fail(MG_ERR_SHAPE, "problem %d: horizon outside 1..%d", p, mg::kMaxT);
    if (world[p] < 0) return fail(MG_ERR_ARG, "problem %d: negative world", p);
    rows += (long)seeds[p] * horizon[p];
    n_seeds += seeds[p];
  }
  if (rows * K_max * c->D > (1L << 30)) return fail(MG_ERR_SHAPE, "batch too large");
  mg_batch* b = new mg_batch();
  b->ctx = c;
  b->P = P;
  b->rows = (int)rows;
  b->n_seeds = (int)n_seeds;
  b->K_max = K_max;
  b->m_max = m_max;
  b->seeds.assign(seeds, seeds + P);
  b->horizon.assign(horizon, horizon + P);
  b->world.assign(world, world + P);
  b->uniform_T = horizon[0];
  for (int p = 1; p < P; ++p)
    if (horizon[p] != horizon[0]) b->uniform_T = 0;
  std::vector<mg::Problem> prob(P);
  std::vector<mg::SeedInfo> sinfo;
  sinfo.reserve(n_seeds);
  int r0 = 0, s0 = 0;
  for (int p = 0; p < P; ++p) {
    b->max_n = std::max(b->max_n, horizon[p] * c->D);
    prob[p] = mg::Problem{seeds[p], horizon[p], world[p], r0, s0, 0, 0, 0};
    for (int s = 0; s < seeds[p]; ++s) sinfo.push_back(mg::SeedInfo{r0 + s * horizon[p], horizon[p], p, 0});
    r0 += seeds[p] * horizon[p];
    s0 += seeds[p];
  }
  mg_status st;
  auto bail = [&](mg_status s) { mg_batch_destroy(b); return s; };
  if ((st = dev_upload(&b->d_prob, prob)) != MG_OK) return bail(st);
  if ((st = dev_upload(&b->d_seed, sinfo)) != MG_OK) return bail(st);
  for (int hi = 0; hi < kNumSlices; ++hi) {
    // evaluations per workgroup: (waves / slices) groups of (wave / lanes) rows
    const int epb = (mg::kBlock / mg::kWave / kSlices[hi]) * (mg::kWave / c->lpe);
    std::vector<int> pre(P + 1, 0);
    for (int p = 0; p < P; ++p) pre[p + 1] = pre[p] + (seeds[p] * horizon[p] + epb - 1) / epb;
    b->chunks[hi] = pre[P];
    if ((st = dev_upload(&b->d_chunk[hi], pre)) != MG_OK) return bail(st);
  }
  c->batches.push_back(b);
  if ((st = wl_chunks_upload(b)) != MG_OK) return bail(st);
  {
    // wave-per-link slice scratch: up to 16 slices while it stays under 64 MB
    const size_t per = (size_t)b->chunks_wl[K_max][0] * (3 + c->D) * mg::kWave * sizeof(float);
    b->wl_slices_max = 1;
    while (b->wl_slices_max < 16 && per * b->wl_slices_max * 2 <= (64u << 20)) b->wl_slices_max *= 2;
    if (b->wl_slices_max > 1) {
      if ((st = dev_alloc(&b->wl_part, per / sizeof(float) * b->wl_slices_max)) != MG_OK ||
          (st = dev_alloc(&b->wl_count, (size_t)b->chunks_wl[K_max][0])) != MG_OK)
        return bail(st);
      if (hipMemset(b->wl_count, 0, (size_t)b->chunks_wl[K_max][0] * sizeof(int)) != hipSuccess)
        return bail(fail(MG_ERR_HIP, "initialising the slice counters failed"));
    }
  }
  const size_t R = rows, RD = rows * c->D, KR = (size_t)K_max * rows, mm = std::max(m_max, 1);
  if ((st = dev_alloc(&b->cost_e, KR)) != MG_OK || (st = dev_alloc(&b->gd_e, KR)) != MG_OK ||
      (st = dev_alloc(&b->mc_e, KR)) != MG_OK || (st = dev_alloc(&b->grad_e, KR * c->D)) != MG_OK ||
      (st = dev_alloc(&b->pe_e, 2 * R)) != MG_OK || (st = dev_alloc(&b->c_cur, n_seeds)) != MG_OK ||
      (st = dev_alloc(&b->g_cur, RD)) != MG_OK || (st = dev_alloc(&b->dir, RD)) != MG_OK ||
      (st = dev_alloc(&b->best_c, n_seeds)) != MG_OK || (st = dev_alloc(&b->best_x, RD)) != MG_OK ||
      (st = dev_alloc(&b->first, n_seeds)) != MG_OK || (st = dev_alloc(&b->S, mm * RD)) != MG_OK ||
      (st = dev_alloc(&b->Y, mm * RD)) != MG_OK || (st = dev_alloc(&b->x_prev, RD)) != MG_OK ||
      (st = dev_alloc(&b->g_prev, RD)) != MG_OK || (st = dev_alloc(&b->rho, n_seeds * mm)) != MG_OK ||
      (st = dev_alloc(&b->meta, 2 * n_seeds)) != MG_OK || (st = dev_alloc(&b->sel_dt, n_seeds)) != MG_OK ||
      (st = dev_alloc(&b->sel_jerk, n_seeds)) != MG_OK)
    return bail(st);
  if ((st = dev_alloc(&b->fs_x, RD)) != MG_OK || (st = dev_alloc(&b->fs_c, n_seeds)) != MG_OK ||
      (st = dev_alloc(&b->fs_g, RD)) != MG_OK || (st = dev_alloc(&b->fs_dir, RD)) != MG_OK ||
      (st = dev_alloc(&b->fs_meta, 2 * n_seeds)) != MG_OK || (st = dev_alloc(&b->fs_cost_e, KR)) != MG_OK ||
      (st = dev_alloc(&b->fs_gd_e, KR)) != MG_OK || (st = dev_alloc(&b->fs_mc_e, KR)) != MG_OK ||
      (st = dev_alloc(&b->fs_grad_e, KR * c->D)) != MG_OK)
    return bail(st);
  if ((st = ensure_speed_buf(b)) != MG_OK) return bail(st);
  // zero the history metadata so a first step without reset is well defined
  if (hipMemset(b->meta, 0, 2 * n_seeds * sizeof(int)) != hipSuccess ||
      hipMemset(b->first, 0, n_seeds * sizeof(int)) != hipSuccess ||
      hipDeviceSynchronize() != hipSuccess)
    return bail(fail(MG_ERR_HIP, "initialising batch workspaces failed"));
  *out = b;
  return MG_OK;
}

void mg_batch_destroy(mg_batch* b) {
  if (!b) return;
  (void)hipDeviceSynchronize();
  if (b->ctx) {
    auto& v = b->ctx->batches;
    v.erase(std::remove(v.begin(), v.end(), b), v.end());
  }
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  for (auto e : b->ev_start) (void)hipEventDestroy(e);
  for (auto e : b->ev_stop) (void)hipEventDestroy(e);
  dev_free(b->d_prob); dev_free(b->d_seed);
  for (auto& p : b->d_chunk) dev_free(p);
  for (auto& pk : b->d_chunk_wl)
    for (auto& p : pk) dev_free(p);
  for (auto& p : b->d_chunk_pm) dev_free(p);
  dev_free(b->cost_e); dev_free(b->gd_e); dev_free(b->mc_e); dev_free(b->grad_e); dev_free(b->pe_e);
  dev_free(b->c_cur); dev_free(b->g_cur); dev_free(b->dir); dev_free(b->best_c); dev_free(b->best_x);
  dev_free(b->first); dev_free(b->S); dev_free(b->Y); dev_free(b->x_prev); dev_free(b->g_prev);
  dev_free(b->rho); dev_free(b->meta); dev_free(b->p_cost); dev_free(b->sel_dt);
  dev_free(b->sel_jerk);
  dev_free(b->fs_x); dev_free(b->fs_c); dev_free(b->fs_g); dev_free(b->fs_dir); dev_free(b->fs_meta);
  dev_free(b->fs_cost_e); dev_free(b->fs_gd_e); dev_free(b->fs_mc_e); dev_free(b->fs_grad_e);
  dev_free(b->wl_part); dev_free(b->wl_count); dev_free(b->sp_h);
  delete b;
}

int mg_batch_seeds(const mg_batch* b) { return b ? b->n_seeds : 0; }

mg_status mg_set_timing(mg_batch* b, int enable) {
  if (!b) return fail(MG_ERR_ARG, "null batch");
  if (enable && b->ev_start.empty()) {
    b->ev_start.resize(256, nullptr);
    b->ev_stop.resize(256, nullptr);
    for (size_t i = 0; i < b->ev_start.size(); ++i) {
      HIP_TRY(hipEventCreate(&b->ev_start[i]));
      HIP_TRY(hipEventCreate(&b->ev_stop[i]));
    }
  }
  b->timing = enable != 0;
  b->ev_next = 0;
  b->ev_count = 0;
  return MG_OK;
}

mg_status mg_eval_time(mg_batch* b, float* mean_us, int* count) {
  if (!b || !mean_us || !count) return fail(MG_ERR_ARG, "null argument");
  double sum = 0.0;
  const int n = b->ev_count;
  for (int i = 0; i < n; ++i) {
    HIP_TRY(hipEventSynchronize(b->ev_stop[i]));
    float ms = 0.0f;
    HIP_TRY(hipEventElapsedTime(&ms, b->ev_start[i], b->ev_stop[i]));
    sum += ms;
  }
  *mean_us = n ? (float)(1000.0 * sum / n) : 0.0f;
  *count = n;
  return MG_OK;
}
int mg_batch_rows(const mg_batch* b) { return b ? b->rows : 0; }

mg_status mg_time_eval(mg_ctx* c, mg_batch* b, const float* q_start, const float* goal,
                       const float* x, const float* dir, int K, const float* alpha, int launches,
                       float* mean_us, void* stream) {
  mg_status st = common_checks(c, b);
  if (st != MG_OK) return st;
  if ((st = check_K_alpha(b, K, alpha)) != MG_OK) return st;
  if (!q_start || !goal || !x || !dir || !mean_us) return fail(MG_ERR_ARG, "null argument");
  if (launches < 1) return fail(MG_ERR_ARG, "launches must be >= 1");
  if (needs_wl(c) && !use_wl(b, K))
    return fail(MG_ERR_UNSUPPORTED, "self-collision and the speed metric need the wave-per-link layout (at most 15 links)");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int hi = pick_slices(b, (long)b->rows * K);
  const mg::EvalArgs a = eval_args(c, b, hi, q_start, goal, x, dir, K, alpha);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  hipError_t err = hipEventRecord(e0, s);
  for (int i = 0; i < launches && err == hipSuccess; ++i) err = launch_layout(b, a, hi, true, true, s);
  if (err == hipSuccess) err = hipEventRecord(e1, s);
  if (err == hipSuccess) err = hipEventSynchronize(e1);
  float ms = 0.0f;
  if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (err != hipSuccess) return fail(MG_ERR_HIP, "timing the evaluation kernel: %s", hipGetErrorString(err));
  *mean_us = 1000.0f * ms / launches;
  return MG_OK;
}

mg_status mg_cost_grad(mg_ctx* c, mg_batch* b, const float* q_start, const float* goal,
                       const float* q, float* cost, float* grad, float* min_clear, void* stream) {
  mg_status st = common_checks(c, b);
  if (st != MG_OK) return st;
  if (!q_start || !goal || !q || !cost) return fail(MG_ERR_ARG, "null q_start, goal, q or cost");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if ((st = enqueue_eval(c, b, q_start, goal, q, nullptr, 1, nullptr, grad != nullptr, grad, nullptr, s)) != MG_OK)
    return st;
  mg::ReduceArgs ra{b->d_seed, b->n_seeds, b->cost_e, b->mc_e, cost, min_clear};
  HIP_TRY(mg::launch_reduce(ra, s));
  return MG_OK;
}

mg_status mg_lbfgs_step(mg_ctx* c, mg_batch* b, int m, int reset, const float* x, const float* g,
                        float* dir, void* stream) {
  if (!c || !b || b->ctx != c) return fail(MG_ERR_ARG, "null or mismatched context / batch");
  if (m < 0 || m > b->m_max) return fail(MG_ERR_SHAPE, "m = %d outside 0..%d", m, b->m_max);
  if (!x || !g || !dir) return fail(MG_ERR_ARG, "null x, g or dir");
  return enqueue_lbfgs(c, b, m, reset, x, g, dir, nullptr, static_cast<hipStream_t>(stream));
}

mg_status mg_linesearch(mg_ctx* c, mg_batch* b, const float* q_start, const float* goal,
                        const float* x, const float* c0, const float* g0, const float* dir, int K,
                        const float* alpha, int mode, float* x_out, float* c_out, float* g_out,
                        int* chosen, float* min_clear, void* stream) {
  mg_status st = common_checks(c, b);
  if (st != MG_OK) return st;
  if ((st = check_K_alpha(b, K, alpha)) != MG_OK) return st;
  if (mode < 0 || mode > 2) return fail(MG_ERR_ARG, "mode must be 0, 1 or 2");
  if (!q_start || !goal || !x || !c0 || !g0 || !dir || !x_out || !c_out || !g_out)
    return fail(MG_ERR_ARG, "null argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if ((st = enqueue_eval(c, b, q_start, goal, x, dir, K, alpha, true, nullptr, nullptr, s)) != MG_OK) return st;
  return enqueue_select(c, b, x, c0, g0, dir, K, alpha, mode, x_out, c_out, g_out, chosen, min_clear, false,
                        nullptr, s);
}

mg_status mg_linesearch_eval(mg_ctx* c, mg_batch* b, const float* q_start, const float* goal,
                             const float* x, const float* dir, int K, const float* alpha, float* cost,
                             float* gd, float* grad, float* min_clear, void* stream) {
  mg_status st = common_checks(c, b);
  if (st != MG_OK) return st;
  if ((st = check_K_alpha(b, K, alpha)) != MG_OK) return st;
  if (!q_start || !goal || !x || !dir || !cost || !gd) return fail(MG_ERR_ARG, "null argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  // the launch mg_linesearch and mg_solve make for these K candidates
  if ((st = enqueue_eval(c, b, q_start, goal, x, dir, K, alpha, true, nullptr, nullptr, s)) != MG_OK) return st;
  const size_t R = b->rows;
  for (int k = 0; k < K; ++k) {
    mg::ReduceArgs rc{b->d_seed, b->n_seeds, b->cost_e + k * R, b->mc_e + k * R, cost + (size_t)k * b->n_seeds,
                      min_clear ? min_clear + (size_t)k * b->n_seeds : nullptr};
    HIP_TRY(mg::launch_reduce(rc, s));
    mg::ReduceArgs rg{b->d_seed, b->n_seeds, b->gd_e + k * R, b->mc_e + k * R, gd + (size_t)k * b->n_seeds, nullptr};
    HIP_TRY(mg::launch_reduce(rg, s));
  }
  if (grad) HIP_TRY(mg::launch_copy(b->grad_e, grad, (size_t)K * R * c->D, s));
  return MG_OK;
}

mg_status mg_linesearch_noalloc(mg_ctx* c, mg_batch* b, const float* q_start, const float* goal,
                                const float* x, const float* c0, const float* g0, const float* dir, int K,
                                const float* alpha, int mode, float* x_out, float* c_out, float* g_out,
                                int* chosen, float* min_clear, void* stream) {
  mg_status st = common_checks(c, b);
  if (st != MG_OK) return st;
  if ((st = check_K_alpha(b, K, alpha)) != MG_OK) return st;
  if (mode < 0 || mode > 2) return fail(MG_ERR_ARG, "mode must be 0, 1 or 2");
  if (!q_start || !goal || !x || !c0 || !g0 || !dir || !x_out || !c_out || !g_out)
    return fail(MG_ERR_ARG, "null argument");
  if (!c->d_scratch) return fail(MG_ERR_STATE, "no scratch address for this context's device");
  if (c->params.speed)
    return fail(MG_ERR_UNSUPPORTED, "the speed metric's gradient needs the batch's workspace (use mg_linesearch)");
  // [K][rows] cost, directional derivative, clearance, then [K][rows][D]
  // gradient, each part starting on a 256-byte boundary
  const size_t KR = (size_t)K * b->rows, part = (KR + 63) & ~(size_t)63;
  const size_t need = 3 * part + KR * c->D;
  if (need > kScratchFloats)
    return fail(MG_ERR_SHAPE, "K * rows * (3 + D) = %zu floats exceeds the static scratch of %zu floats",
                need, kScratchFloats);
  const EvalOut eo{c->d_scratch, c->d_scratch + part, c->d_scratch + 2 * part, c->d_scratch + 3 * part};
  hipStream_t s = static_cast<hipStream_t>(stream);
  if ((st = enqueue_eval(c, b, q_start, goal, x, dir, K, alpha, true, nullptr, nullptr, s, &eo)) != MG_OK) return st;
  return enqueue_select(c, b, x, c0, g0, dir, K, alpha, mode, x_out, c_out, g_out, chosen, min_clear, false,
                        nullptr, s, &eo);
}

mg_status mg_autotune(mg_ctx* c, mg_batch* b, const float* q_start, const float* goal,
                      const float* x, const float* dir, int K, const float* alpha, int launches,
                      int* slices_out, void* stream) {
  mg_status st = common_checks(c, b);
  if (st != MG_OK) return st;
  if ((st = check_K_alpha(b, K, alpha)) != MG_OK) return st;
  if (!q_start || !goal || !x || !dir) return fail(MG_ERR_ARG, "null argument");
  if (launches < 1) return fail(MG_ERR_ARG, "launches must be >= 1");
  // candidates: lane per link with 1, 2 or 4 cuboid slices per workgroup;
  // wave per link with two waves per link; wave per link with 1, 2 or 4
  // workgroups per 64 evaluations.  Each is {layout, slices index, halves,
  // workgroup slices}.
  struct Opt { int layout, hi, halves, wls, groups; };
  std::vector<Opt> opts;
  if (!needs_wl(c))
    for (int hi = 0; hi < kNumSlices; ++hi) opts.push_back({0, hi, 0, 0, 1});
  if (wl_groups_possible(c, 4)) opts.push_back({1, -1, 1, 1, 4});
  if (wl_groups_possible(c)) opts.push_back({1, -1, 1, 1, 2});
  if (wl_halves_possible(c)) opts.push_back({1, -1, 2, 1, 1});
  if (wl_possible(c))
    for (int h = 1; h <= b->wl_slices_max; h *= 2) opts.push_back({1, -1, 1, h, 1});
  if (opts.empty()) return fail(MG_ERR_UNSUPPORTED, "no evaluation layout fits this robot");
  size_t best = 0;
  float best_us = 3.0e38f;
  for (size_t o = 0; o < opts.size(); ++o) {
    b->layout = opts[o].layout;
    b->slices = opts[o].hi;
    b->wl_halves = opts[o].halves;
    b->wl_slices = opts[o].wls;
    b->wl_groups = opts[o].groups;
    float us = 0.0f;
    // one untimed launch per layout first (code upload, caches)
    if ((st = mg_time_eval(c, b, q_start, goal, x, dir, K, alpha, 1, &us, stream)) != MG_OK ||
        (st = mg_time_eval(c, b, q_start, goal, x, dir, K, alpha, launches, &us, stream)) != MG_OK) {
      b->slices = -1;
      b->layout = -1;
      b->wl_slices = 0;
      b->wl_halves = 0;
      b->wl_groups = 1;
      return st;
    }
    if (us < best_us) { best_us = us; best = o; }
  }
  b->layout = opts[best].layout;
  b->layout_set = false;
  b->slices = opts[best].hi;
  b->wl_halves = opts[best].halves;
  b->wl_slices = opts[best].wls;
  b->wl_groups = opts[best].groups;
  // lane per link: the slice count; wave per link: minus the workgroups per
  // 64 evaluations, -8 for two waves per link, -16 for two slot groups, -32
  // for four
  if (slices_out)
    *slices_out = opts[best].layout == 0 ? kSlices[opts[best].hi]
                  : opts[best].groups == 4 ? -32 : opts[best].groups == 2 ? -16
                  : (opts[best].halves == 2 ? -8 : -opts[best].wls);
  return MG_OK;
}

mg_status mg_set_self_collision(mg_ctx* c, int n_pairs, const int* pairs) {
  if (!c) return fail(MG_ERR_ARG, "null context");
  if (n_pairs < 0 || (n_pairs > 0 && !pairs)) return fail(MG_ERR_ARG, "bad pair list");
  if (n_pairs > 0 && !wl_possible(c, true))
    return fail(MG_ERR_UNSUPPORTED, "self-collision needs at most 15 links and "
                "workgroup memory for the robot's spheres");
  std::vector<int4> pr(n_pairs);
  for (int k = 0; k < n_pairs; ++k) {
    const int i = pairs[2 * k], j = pairs[2 * k + 1];
    if (i < 0 || j < 0 || i >= c->M || j >= c->M || i == j)
      return fail(MG_ERR_ARG, "pair %d: spheres %d, %d out of range or equal", k, i, j);
    const float rs = c->sphere[4 * i + 3] + c->sphere[4 * j + 3];
    int bits;
    memcpy(&bits, &rs, sizeof(bits));
    // owners: link and slot position within the link of each sphere
    const int pi = c->slot_of[i] % c->maxs, pj = c->slot_of[j] % c->maxs;
    pr[k] = make_int4(i, j, c->sphere_link[i] | (c->sphere_link[j] << 8) | (pi << 16) | (pj << 24), bits);
  }
  if (n_pairs > c->self_cap) {
    HIP_TRY(hipDeviceSynchronize());
    dev_free(c->d_self_pairs);
    c->self_cap = 0;
    mg_status st = dev_alloc(&c->d_self_pairs, (size_t)n_pairs);
    if (st != MG_OK) return st;
    c->self_cap = n_pairs;
  }
  if (n_pairs > 0) HIP_TRY(hipMemcpy(c->d_self_pairs, pr.data(), pr.size() * sizeof(int4), hipMemcpyHostToDevice));
  c->n_self = n_pairs;
  return MG_OK;
}

mg_status mg_ee_pose(mg_ctx* c, int rows, const float* q, float* pose, void* stream) {
  if (!c) return fail(MG_ERR_ARG, "null context");
  if (rows < 0) return fail(MG_ERR_ARG, "rows must be >= 0");
  if (rows > 0 && (!q || !pose)) return fail(MG_ERR_ARG, "null q or pose");
  mg::EePoseArgs a;
  memset(&a, 0, sizeof(a));
  a.rows = rows;
  a.dof = c->D;
  a.n_ee = c->n_ee;
  for (int e = 0; e < c->n_ee; ++e) a.ee_link[e] = c->ee_link[e];
  a.fixed_tf = c->d_fixed_tf;
  a.ee_tf = c->d_ee_tf;
  a.chain = c->d_wl_chain;
  a.info = c->d_wl_info;
  a.q = q;
  a.pose = pose;
  HIP_TRY(mg::launch_ee_pose(a, static_cast<hipStream_t>(stream)));
  return MG_OK;
}

mg_status mg_batch_set_layout(mg_batch* b, int layout, int slices) {
  if (!b) return fail(MG_ERR_ARG, "null batch");
  if (layout < -1 || layout > 4) return fail(MG_ERR_ARG, "layout must be -1, 0, 1, 2, 3 or 4");
  if (layout >= 1 && !wl_possible(b->ctx))
    return fail(MG_ERR_UNSUPPORTED, "the wave-per-link layout needs at most 15 links");
  if (layout == 2 && !wl_halves_possible(b->ctx))
    return fail(MG_ERR_UNSUPPORTED, "two waves per link need at most 8 links");
  if (layout == 3 && !wl_groups_possible(b->ctx))
    return fail(MG_ERR_UNSUPPORTED, "two slot groups per wave need no self-collision and 4 or more slots per link");
  if (layout == 4 && !wl_groups_possible(b->ctx, 4))
    return fail(MG_ERR_UNSUPPORTED, "four slot groups per wave need no self-collision and 8 or more slots per link");
  b->wl_halves = layout == 2 ? 2 : (layout == 1 || layout >= 3 ? 1 : 0);
  b->wl_groups = layout == 4 ? 4 : layout == 3 ? 2 : 1;
  b->layout_set = layout >= 0;
  if (layout >= 2) {
    if (slices > 1) return fail(MG_ERR_ARG, "layouts 2, 3 and 4 take one workgroup per chunk of evaluations");
    b->layout = 1;
    b->slices = -1;
    b->wl_slices = 1;
    return MG_OK;
  }
  int hi = -1;
  if (slices != 0) {
    for (int i = 0; i < kNumSlices; ++i)
      if (kSlices[i] == slices) hi = i;
    // (wave per link also takes 8 and 16 workgroups per chunk)
    const bool wl_ok = layout == 1 && (slices == 8 || slices == 16);
    if (hi < 0 && !wl_ok) return fail(MG_ERR_ARG, "slices must be 0 (automatic), 1, 2 or 4 (wave per link: or 8, 16)");
    if (layout == 1 && slices > b->wl_slices_max)
      return fail(MG_ERR_SHAPE, "this batch holds at most %d wave-per-link slices", b->wl_slices_max);
  }
  b->layout = layout;
  b->slices = layout == 1 ? -1 : hi;
  b->wl_slices = layout == 1 ? slices : 0;
  return MG_OK;
}

mg_status mg_batch_reserve_particles(mg_batch* b, int n_particles) {
  if (!b) return fail(MG_ERR_ARG, "null batch");
  if (n_particles < 1 || n_particles > mg::kMaxParticles)
    return fail(MG_ERR_SHAPE, "n_particles = %d outside 1..%d", n_particles, mg::kMaxParticles);
  HIP_TRY(hipDeviceSynchronize());
  mg_status st;
  if (n_particles > b->p_cap) {
    dev_free(b->p_cost);
    b->p_cap = 0;
    if ((st = dev_alloc(&b->p_cost, (size_t)n_particles * b->rows)) != MG_OK) return st;
    b->p_cap = n_particles;
  }
  // wave-per-link records for this particle count
  b->pm_K = n_particles;
  for (int gi = 0; gi < 3; ++gi)
    if ((st = wl_records(b, n_particles, mg::kWave >> gi, &b->d_chunk_pm[gi], &b->chunks_pm[gi])) != MG_OK)
      return st;
  return MG_OK;
}

}  // extern "C"

namespace {

// The particle stage on draws from memory (eps) or, with eps null, on
// draws each kernel makes itself (round it's at counter round it0 + it).
mg_status particle_rounds(mg_ctx* c, mg_batch* b, const float* q_start, const float* goal, float* mean, float* var,
                          int n_particles, int n_iters, const float* eps, unsigned long long seed, float beta,
                          float k_mu, float k_sigma, float* costs_out, hipStream_t s) {
  mg_status st = common_checks(c, b);
  if (st != MG_OK) return st;
  if (n_particles < 1 || n_particles > b->p_cap)
    return fail(MG_ERR_STATE, "n_particles = %d exceeds the %d reserved (mg_batch_reserve_particles)",
                n_particles, b->p_cap);
  if (n_iters < 0) return fail(MG_ERR_ARG, "n_iters must be >= 0");
  if (!q_start || !goal || !mean || !var) return fail(MG_ERR_ARG, "null q_start, goal, mean or var");
  if (!(k_mu >= 0.0f && k_mu <= 1.0f) || !(k_sigma >= 0.0f && k_sigma <= 1.0f))
    return fail(MG_ERR_ARG, "k_mu and k_sigma must lie in [0, 1]");
  // wave per link with one slot group (64 particles of one row per
  // workgroup: their spheres lie close together, so the wave-level cuboid
  // cull is tight) unless mg_batch_set_layout chose another layout; the
  // autotuner's choice for line-search candidates is not carried over (on
  // the two-arm tree with 500 cuboids and swept collision a particle round
  // measured 139 ms with one slot group, 244 ms with two, 350 ms lane per
  // link)
  const bool lane_set = b->layout_set && b->layout == 0;
  const int groups =
      b->layout_set && b->wl_groups > 1 && wl_groups_possible(c, b->wl_groups) ? b->wl_groups : 1;
  const int halves = groups > 1 ? 1 : (b->wl_halves > 0 ? b->wl_halves : (wl_halves_possible(c) ? 2 : 1));
  const int E = mg::kWave / groups;
  // rows a chunk of E particles touches, with the stencils' four on either side
  const int pm_rows = (E - 1) / n_particles + 10;
  const bool wl = (!lane_set || needs_wl(c)) && wl_possible(c) &&
                  n_particles == b->pm_K && pm_rows <= mg::kWlStageRows &&
                  mg::wl_lds_bytes(c->L, c->D, c->max_depth, c->M, c->n_self > 0, halves, c->maxs, E, pm_rows) <=
                      c->lds_max;
  if (needs_wl(c) && !wl)
    return fail(MG_ERR_UNSUPPORTED,
                "self-collision or the speed metric in the particle stage needs the wave-per-link layout for %d particles "
                "(the last mg_batch_reserve_particles count, at least 2)", n_particles);
  const size_t draws = (size_t)n_particles * b->rows * c->D;
  const int hi = pick_slices(b, (long)b->rows * n_particles);
  for (int it = 0; it < n_iters; ++it) {
    const float* e = eps ? eps + (size_t)it * draws : nullptr;
    mg::EvalArgs a = eval_args(c, b, hi, q_start, goal, mean, e, n_particles, nullptr);
    a.var = var;
    if (e) a.d_stride = (size_t)b->rows * c->D;
    else a.pm_seed = seed;
    a.pm_it = it;
    a.cost_e = b->p_cost;
    a.mc_e = nullptr;
    a.gd_e = nullptr;
    a.grad_e = nullptr;
    if (wl) {
      a.wl.halves = halves;
      a.wl.groups = groups;
      a.wl.chunk = b->d_chunk_pm[groups_index(groups)];
      wl_single(b, n_particles, a.wl);
      a.wl.pm_rows = pm_rows;
      HIP_TRY(mg::launch_eval_wl(a, b->chunks_pm[groups_index(groups)], 1, true, false, s));
    } else {
      HIP_TRY(mg::launch_eval(a, b->chunks[hi], true, false, s));
    }
    mg::ParticleArgs pa;
    memset(&pa, 0, sizeof(pa));
    pa.seeds = b->d_seed;
    pa.n_seeds = b->n_seeds;
    pa.rows = b->rows;
    pa.dof = c->D;
    pa.N = n_particles;
    pa.beta = beta;
    pa.k_mu = k_mu;
    pa.k_sigma = k_sigma;
    pa.q_lo = c->d_q_lo;
    pa.q_hi = c->d_q_hi;
    pa.cost_e = b->p_cost;
    pa.eps = e;
    pa.seed = seed;
    pa.it = it;
    pa.mean = mean;
    pa.var = var;
    pa.costs_out = costs_out ? costs_out + (size_t)it * b->n_seeds * n_particles : nullptr;
    HIP_TRY(mg::launch_particle_update(pa, s));
  }
  return MG_OK;
}

}  // namespace

extern "C" {

mg_status mg_particles(mg_ctx* c, mg_batch* b, const float* q_start, const float* goal, float* mean,
                       float* var, int n_particles, int n_iters, const float* eps, float beta,
                       float k_mu, float k_sigma, float* costs_out, void* stream) {
  if (n_iters > 0 && !eps) return fail(MG_ERR_ARG, "null eps");
  return particle_rounds(c, b, q_start, goal, mean, var, n_particles, n_iters, eps, 0, beta, k_mu, k_sigma,
                         costs_out, static_cast<hipStream_t>(stream));
}

mg_status mg_particles_seeded(mg_ctx* c, mg_batch* b, const float* q_start, const float* goal, float* mean,
                              float* var, int n_particles, int n_iters, unsigned long long seed, float beta,
                              float k_mu, float k_sigma, float* costs_out, void* stream) {
  if (n_iters > 65535) return fail(MG_ERR_ARG, "n_iters must be <= 65535");
  return particle_rounds(c, b, q_start, goal, mean, var, n_particles, n_iters, nullptr, seed, beta, k_mu, k_sigma,
                         costs_out, static_cast<hipStream_t>(stream));
}

mg_status mg_knn(int dof, int n_nodes, const float* nodes, int n_queries, const float* queries, int k, int* idx,
                 float* d2, void* stream) {
  if (dof < 1 || dof > mg::kMaxDof) return fail(MG_ERR_SHAPE, "dof %d outside 1..%d", dof, mg::kMaxDof);
  if (k < 1 || k > 32) return fail(MG_ERR_SHAPE, "k = %d outside 1..32", k);
  if (n_nodes < 0 || n_queries < 0) return fail(MG_ERR_SHAPE, "negative count");
  if ((n_nodes > 0 && !nodes) || (n_queries > 0 && (!queries || !idx))) return fail(MG_ERR_ARG, "null argument");
  mg::KnnArgs a{n_nodes, n_queries, dof, k, nodes, queries, idx, d2};
  HIP_TRY(mg::launch_knn(a, static_cast<hipStream_t>(stream)));
  return MG_OK;
}

mg_status mg_philox_normals(unsigned long long seed, int it0, int n_iters, int n_particles, int rows, int dof,
                            float* out, void* stream) {
  if (!out) return fail(MG_ERR_ARG, "null out");
  if (it0 < 0 || n_iters < 1 || n_particles < 1 || rows < 1 || dof < 1 || n_iters > 65535 || n_particles > 65535)
    return fail(MG_ERR_SHAPE, "bad draw shape");
  if (((uintptr_t)out) & 15) return fail(MG_ERR_ARG, "out must be 16-byte aligned");
  HIP_TRY(mg::launch_philox_normals(seed, it0, n_iters, n_particles, (long long)rows * dof, out,
                                    static_cast<hipStream_t>(stream)));
  return MG_OK;
}

}  // extern "C"

namespace {

// One solver iteration: candidates of the current direction are costed
// (eval), the line search picks the next iterate, tracks the best and, in the
// same kernel, computes the next L-BFGS direction.
mg_status enqueue_iteration(mg_ctx* c, mg_batch* b, const float* q_start, const float* goal, float* x,
                            int m, int K, const float* alpha, int mode, hipStream_t s) {
  mg_status st;
  if ((st = enqueue_eval(c, b, q_start, goal, x, b->dir, K, alpha, true, nullptr, nullptr, s)) != MG_OK) return st;
  const mg::LbfgsArgs la = lbfgs_args(c, b, m, 0, x, b->g_cur, b->dir, b->first);
  return enqueue_select(c, b, x, b->c_cur, b->g_cur, b->dir, K, alpha, mode, x, b->c_cur, b->g_cur,
                        nullptr, nullptr, true, &la, s);
}

// One iteration with the previous choice folded in: the launch reads state
// set `cur` (the last iterate, its candidates' costs and gradients) and
// writes set 1 - cur (the chosen iterate, its cost and gradient, the next
// direction and this iteration's candidates).
mg_status enqueue_fused_iteration(mg_ctx* c, mg_batch* b, const float* q_start, const float* goal, float* x,
                                  int m, int K, const float* alpha, int mode, int cur, hipStream_t s) {
  const StateSet a0 = state_set(b, x, cur), a1 = state_set(b, x, 1 - cur);
  mg::SelFuse f;
  memset(&f, 0, sizeof(f));
  mg::SelectArgs& sa = f.sa;
  sa.seeds = b->d_seed;
  sa.uniform_T = b->uniform_T;
  sa.n_seeds = b->n_seeds;
  sa.rows = b->rows;
  sa.dof = c->D;
  sa.K = K;
  sa.mode = mode;
  for (int k = 0; k < K; ++k) sa.alpha[k] = alpha[k];
  sa.eta1 = c->params.ls_eta1;
  sa.eta_w = c->params.ls_eta_w;
  sa.q_lo = c->d_q_lo;
  sa.q_hi = c->d_q_hi;
  sa.x = a0.x; sa.c0 = a0.c; sa.g0 = a0.g; sa.d = a0.dir;
  sa.cost_e = a0.cost_e; sa.gd_e = a0.gd_e; sa.mc_e = a0.mc_e; sa.grad_e = a0.grad_e;
  sa.x_out = a1.x; sa.c_out = a1.c; sa.g_out = a1.g;
  sa.track = 1;
  sa.best_c = b->best_c;
  sa.best_x = b->best_x;
  // (the previous iterate and gradient are the set being read)
  mg::LbfgsArgs& la = f.la;
  la = lbfgs_args(c, b, m, 0, a0.x, a0.g, a1.dir, nullptr);
  la.x_prev = a0.x;
  la.g_prev = a0.g;
  la.keep_prev = 1;
  la.meta = a0.meta;
  la.meta_out = a1.meta;
  const int hi = pick_slices(b, (long)b->rows * K);
  mg::EvalArgs ea = eval_args(c, b, hi, q_start, goal, a1.x, a1.dir, K, alpha);
  ea.cost_e = a1.cost_e; ea.gd_e = a1.gd_e; ea.mc_e = a1.mc_e; ea.grad_e = a1.grad_e;
  ea.pe_e = nullptr;
  HIP_TRY(launch_layout(b, ea, hi, true, true, s, true, &f));
  return MG_OK;
}

template <typename T>
void key_push(std::vector<char>& k, const T& v) {
  const char* p = reinterpret_cast<const char*>(&v);
  k.insert(k.end(), p, p + sizeof(T));
}

}  // namespace

namespace {

// The solve's iterations with each choice folded into the next evaluation
// launch (fuse_ok): iteration 0 evaluates the first direction's candidates,
// iterations 1 .. iters - 1 each choose the previous step and evaluate the
// next one in one launch (alternating the two state sets; a graph replays
// an even number of them, so every replay starts from set 0), and the last
// choice runs alone.  The same arithmetic as the separate launches, so the
// same results.
mg_status solve_fused(mg_ctx* c, mg_batch* b, const float* q_start, const float* goal, float* x, int iters,
                      int m, int K, const float* alpha, int mode, int graph_inner, int use_graph, hipStream_t s) {
  if (iters < 1) return MG_OK;
  mg_status st;
  if ((st = enqueue_eval(c, b, q_start, goal, x, b->dir, K, alpha, true, nullptr, nullptr, s)) != MG_OK) return st;
  int i = 1;
  const int gi = graph_inner + (graph_inner & 1);
  if (use_graph && iters - 1 >= gi) {
    std::vector<char> key;
    key_push(key, 1); key_push(key, q_start); key_push(key, goal); key_push(key, x); key_push(key, m);
    key_push(key, K); key_push(key, mode); key_push(key, gi); key_push(key, c->params);
    key_push(key, c->d_box); key_push(key, c->d_world_off); key_push(key, b->slices);
    key_push(key, b->layout); key_push(key, b->wl_slices); key_push(key, c->n_self);
    key_push(key, b->wl_halves); key_push(key, b->wl_groups);
    for (int v : c->world_off) key_push(key, v);
    for (int k = 0; k < K; ++k) key_push(key, alpha[k]);
    if (!b->gexec || key != b->gkey) {
      if (b->gexec) { (void)hipGraphExecDestroy(b->gexec); b->gexec = nullptr; }
      HIP_TRY(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
      mg_status cst = MG_OK;
      for (int j = 0; j < gi && cst == MG_OK; ++j)
        cst = enqueue_fused_iteration(c, b, q_start, goal, x, m, K, alpha, mode, j & 1, c->cap_stream);
      hipGraph_t graph = nullptr;
      hipError_t e = hipStreamEndCapture(c->cap_stream, &graph);
      if (cst != MG_OK) { if (graph) (void)hipGraphDestroy(graph); return cst; }
      if (e != hipSuccess) return fail(MG_ERR_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
      e = hipGraphInstantiate(&b->gexec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (e != hipSuccess) { b->gexec = nullptr; return fail(MG_ERR_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e)); }
      b->gkey = key;
    }
    for (; i + gi <= iters; i += gi) HIP_TRY(hipGraphLaunch(b->gexec, s));
  }
  for (; i < iters; ++i)
    if ((st = enqueue_fused_iteration(c, b, q_start, goal, x, m, K, alpha, mode, (i - 1) & 1, s)) != MG_OK)
      return st;
  const int cur = (iters - 1) & 1;
  const StateSet a0 = state_set(b, x, cur), a1 = state_set(b, x, 1 - cur);
  const EvalOut eo{a0.cost_e, a0.gd_e, a0.mc_e, a0.grad_e};
  return enqueue_select(c, b, a0.x, a0.c, a0.g, a0.dir, K, alpha, mode, a1.x, a1.c, a1.g, nullptr, nullptr, true,
                        nullptr, s, &eo);
}

}  // namespace

extern "C" {

mg_status mg_batch_set_fusion(mg_batch* b, int enable) {
  if (!b) return fail(MG_ERR_ARG, "null batch");
  b->fusion = enable != 0;
  return MG_OK;
}

int mg_solve_fuses(mg_ctx* c, mg_batch* b, int K, int m, const float* x) {
  if (!c || !b || b->ctx != c || K < 1 || K > b->K_max || m < 0 || m > b->m_max) return 0;
  return fuse_ok(c, b, K, m, x) ? 1 : 0;
}

mg_status mg_solve(mg_ctx* c, mg_batch* b, const float* q_start, const float* goal, float* x,
                   int iters, int m, int K, const float* alpha, int mode, int graph_inner,
                   int use_graph, float* best_cost, int* best_seed, int* success, void* stream) {
  mg_status st = common_checks(c, b);
  if (st != MG_OK) return st;
  if ((st = check_K_alpha(b, K, alpha)) != MG_OK) return st;
  if (mode < 0 || mode > 2) return fail(MG_ERR_ARG, "mode must be 0, 1 or 2");
  if (m < 0 || m > b->m_max) return fail(MG_ERR_SHAPE, "m = %d outside 0..%d", m, b->m_max);
  if (iters < 0) return fail(MG_ERR_ARG, "iters must be >= 0");
  if (!q_start || !goal || !x || !best_cost) return fail(MG_ERR_ARG, "null q_start, goal, x or best_cost");
  if (use_graph && graph_inner < 1) return fail(MG_ERR_ARG, "graph_inner must be >= 1");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t RD = (size_t)b->rows * c->D;

  // initial cost and gradient, best = start, fresh history per seed
  if ((st = enqueue_eval(c, b, q_start, goal, x, nullptr, 1, nullptr, true, b->g_cur, nullptr, s)) != MG_OK) return st;
  mg::ReduceArgs ra{b->d_seed, b->n_seeds, b->cost_e, b->mc_e, b->c_cur, nullptr};
  HIP_TRY(mg::launch_reduce(ra, s));
  HIP_TRY(mg::launch_copy(b->c_cur, b->best_c, b->n_seeds, s));
  HIP_TRY(mg::launch_copy(x, b->best_x, RD, s));
  HIP_TRY(mg::launch_fill_i32(b->first, 1, b->n_seeds, s));
  if ((st = enqueue_lbfgs(c, b, m, 1, x, b->g_cur, b->dir, b->first, s)) != MG_OK) return st;

  if (fuse_ok(c, b, K, m, x)) {
    if ((st = solve_fused(c, b, q_start, goal, x, iters, m, K, alpha, mode, graph_inner, use_graph, s)) != MG_OK)
      return st;
    iters = 0;
  }
  int done = 0;
  if (use_graph && iters >= graph_inner) {
    std::vector<char> key;
    key_push(key, 0);
    key_push(key, q_start); key_push(key, goal); key_push(key, x); key_push(key, m); key_push(key, K);
    key_push(key, mode); key_push(key, graph_inner); key_push(key, c->params);
    key_push(key, c->d_box); key_push(key, c->d_world_off); key_push(key, b->slices);
    key_push(key, b->layout); key_push(key, b->wl_slices); key_push(key, c->n_self);
    key_push(key, b->wl_halves);
    key_push(key, b->wl_groups);
    // (one-problem launches carry the world's cuboid range by value)
    for (int v : c->world_off) key_push(key, v);
    for (int k = 0; k < K; ++k) key_push(key, alpha[k]);
    if (!b->gexec || key != b->gkey) {
      if (b->gexec) { (void)hipGraphExecDestroy(b->gexec); b->gexec = nullptr; }
      HIP_TRY(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
      mg_status cst = MG_OK;
      for (int i = 0; i < graph_inner && cst == MG_OK; ++i)
        cst = enqueue_iteration(c, b, q_start, goal, x, m, K, alpha, mode, c->cap_stream);
      hipGraph_t graph = nullptr;
      hipError_t e = hipStreamEndCapture(c->cap_stream, &graph);
      if (cst != MG_OK) { if (graph) (void)hipGraphDestroy(graph); return cst; }
      if (e != hipSuccess) return fail(MG_ERR_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
      e = hipGraphInstantiate(&b->gexec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (e != hipSuccess) { b->gexec = nullptr; return fail(MG_ERR_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e)); }
      b->gkey = key;
    }
    for (; done + graph_inner <= iters; done += graph_inner) HIP_TRY(hipGraphLaunch(b->gexec, s));
  }
  for (; done < iters; ++done)
    if ((st = enqueue_iteration(c, b, q_start, goal, x, m, K, alpha, mode, s)) != MG_OK) return st;

  HIP_TRY(mg::launch_copy(b->best_x, x, RD, s));
  HIP_TRY(mg::launch_copy(b->best_c, best_cost, b->n_seeds, s));
  if (best_seed || success) {
    if (success)
      if ((st = enqueue_eval(c, b, q_start, goal, x, nullptr, 1, nullptr, false, nullptr, b->pe_e, s)) != MG_OK)
        return st;
    mg::FinalArgs fa{b->d_prob, b->P, b->rows, b->best_c, b->pe_e, b->mc_e,
                     c->params.success_pos, c->params.success_rot, best_seed, success};
    HIP_TRY(mg::launch_final(fa, s));
  }
  return MG_OK;
}

mg_status mg_retime(mg_ctx* c, mg_batch* b, const float* q_start, const float* x, const float* vmax,
                    const float* amax, const float* jmax, float* dt_out, float* jerk_out, void* stream) {
  mg_status st = common_checks(c, b);
  if (st != MG_OK) return st;
  if (!q_start || !x || !dt_out || !vmax || !amax || !jmax)
    return fail(MG_ERR_ARG, "null q_start, x, dt_out or limits");
  mg::RetimeArgs a;
  memset(&a, 0, sizeof(a));
  a.seeds = b->d_seed;
  a.n_seeds = b->n_seeds;
  a.dof = c->D;
  a.dt = c->params.dt;
  for (int d = 0; d < c->D; ++d) {
    if (std::isnan(vmax[d]) || std::isnan(amax[d]) || std::isnan(jmax[d]))
      return fail(MG_ERR_ARG, "NaN limit for joint %d", d);
    a.inv_v[d] = vmax[d] > 0.0f ? 1.0f / vmax[d] : 0.0f;
    a.inv_a[d] = amax[d] > 0.0f ? 1.0f / amax[d] : 0.0f;
    a.inv_j[d] = jmax[d] > 0.0f ? 1.0f / jmax[d] : 0.0f;
  }
  a.q_start = q_start;
  a.x = x;
  a.dt_out = dt_out;
  a.jerk_out = jerk_out;
  HIP_TRY(mg::launch_retime(a, static_cast<hipStream_t>(stream)));
  return MG_OK;
}

mg_status mg_solve_timestep(mg_ctx* c, mg_batch* b, const float* q_start, const float* goal, float* x,
                            int iters1, int iters2, int m, int K, const float* alpha, int mode,
                            int graph_inner, int use_graph, const float* vmax, const float* amax,
                            const float* jmax, float dt_min, float* best_cost, int* best_seed,
                            int* success, float* dt_out, void* stream) {
  mg_status st = common_checks(c, b);
  if (st != MG_OK) return st;
  if (!best_cost || !dt_out || !vmax || !amax || !jmax) return fail(MG_ERR_ARG, "null best_cost, dt_out or limits");
  if (iters1 < 0 || iters2 < 0) return fail(MG_ERR_ARG, "iters1 and iters2 must be >= 0");
  if (!(dt_min > 0.0f)) return fail(MG_ERR_ARG, "dt_min must be > 0");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const mg::Params p0 = c->params;
  float* d_dt = nullptr;
  int* d_bs = nullptr;
  if ((st = dev_alloc(&d_dt, b->n_seeds)) != MG_OK) return st;
  if ((st = dev_alloc(&d_bs, b->P)) != MG_OK) {
    dev_free(d_dt);
    return st;
  }
  std::vector<float> h_dt(b->n_seeds);
  std::vector<int> h_bs(b->P);
  // the largest retimed spacing over the problems' best seeds
  auto retime_best = [&](float* out) -> mg_status {
    mg_status r = mg_retime(c, b, q_start, x, vmax, amax, jmax, d_dt, nullptr, stream);
    if (r != MG_OK) return r;
    HIP_TRY(hipMemcpyAsync(h_dt.data(), d_dt, h_dt.size() * sizeof(float), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(h_bs.data(), d_bs, h_bs.size() * sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    float dt = 0.0f;
    int seed0 = 0;
    for (int p = 0; p < b->P; ++p) {
      dt = std::max(dt, h_dt[seed0 + h_bs[p]]);
      seed0 += b->seeds[p];
    }
    *out = std::max(dt, dt_min);
    return MG_OK;
  };
  auto run = [&]() -> mg_status {
    // first pass at the context's spacing without the jerk term
    c->params.a9 = 0.0f;
    mg_status r = mg_solve(c, b, q_start, goal, x, iters1, m, K, alpha, mode, graph_inner, use_graph,
                           best_cost, d_bs, nullptr, stream);
    if (r != MG_OK) return r;
    float dt_opt;
    if ((r = retime_best(&dt_opt)) != MG_OK) return r;
    // weights of the derivative terms rescaled so that the same waypoints
    // cost what they cost at the first spacing (v, a, j scale as rho^-1,
    // rho^-2, rho^-3), and the jerk term switched on
    const float rho = dt_opt / p0.dt;
    c->params = p0;
    c->params.dt = dt_opt;
    c->params.a7 = p0.a7 * rho;
    const float rho2 = rho * rho, rho3 = rho2 * rho;
    c->params.a8 = p0.a8 * (rho2 * rho2);
    c->params.a9 = p0.a9 * (rho3 * rho3);
    if ((r = mg_solve(c, b, q_start, goal, x, iters2, m, K, alpha, mode, graph_inner, use_graph, best_cost, d_bs,
                      success, stream)) != MG_OK)
      return r;
    float dt_f;
    if ((r = retime_best(&dt_f)) != MG_OK) return r;
    if (best_seed) HIP_TRY(hipMemcpyAsync(best_seed, d_bs, b->P * sizeof(int), hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    dt_out[0] = dt_opt;
    dt_out[1] = dt_f;
    return MG_OK;
  };
  st = run();
  c->params = p0;
  dev_free(d_dt);
  dev_free(d_bs);
  return st;
}

mg_status mg_ik_seeds(mg_ctx* c, mg_batch* ik, mg_batch* to, const float* q_start, const float* goal,
                      const float* x_ik, float w_dist, float* x_to, int* ik_ok, void* stream) {
  mg_status st = common_checks(c, ik);
  if (st != MG_OK || (st = common_checks(c, to)) != MG_OK) return st;
  if (!q_start || !goal || !x_ik || !x_to) return fail(MG_ERR_ARG, "null q_start, goal, x_ik or x_to");
  if (ik->P != to->P) return fail(MG_ERR_SHAPE, "the IK and trajectory batches hold %d and %d problems", ik->P, to->P);
  for (int p = 0; p < ik->P; ++p) {
    if (ik->horizon[p] != 1) return fail(MG_ERR_SHAPE, "IK problem %d has horizon %d (must be 1)", p, ik->horizon[p]);
    if (ik->seeds[p] > mg::kMaxIkSeeds)
      return fail(MG_ERR_SHAPE, "IK problem %d has %d seeds (at most %d)", p, ik->seeds[p], mg::kMaxIkSeeds);
  }
  if (!(w_dist >= 0.0f)) return fail(MG_ERR_ARG, "w_dist must be >= 0");
  hipStream_t s = static_cast<hipStream_t>(stream);
  // pose error, clearance and cost of every IK seed as given
  if ((st = enqueue_eval(c, ik, q_start, goal, x_ik, nullptr, 1, nullptr, false, nullptr, ik->pe_e, s)) != MG_OK)
    return st;
  mg::IkSeedArgs a;
  memset(&a, 0, sizeof(a));
  a.ik = ik->d_prob;
  a.to = to->d_prob;
  a.P = ik->P;
  a.dof = c->D;
  a.q_start = q_start;
  a.x_ik = x_ik;
  a.cost_e = ik->cost_e;
  a.mc_e = ik->mc_e;
  a.pe_e = ik->pe_e;
  a.pos_tol = c->params.success_pos;
  a.rot_tol = c->params.success_rot;
  a.w_dist = w_dist;
  a.x_to = x_to;
  a.ik_ok = ik_ok;
  HIP_TRY(mg::launch_ik_seeds(a, s));
  return MG_OK;
}

mg_status mg_traj_select(mg_ctx* c, mg_batch* b, const float* q_start, const float* goal, const float* x,
                         const float* vmax, const float* amax, const float* jmax, float w_jerk, float w_time,
                         int* best_seed, int* success, float* motion_time, void* stream) {
  mg_status st = common_checks(c, b);
  if (st != MG_OK) return st;
  if (!q_start || !goal || !x || !best_seed) return fail(MG_ERR_ARG, "null q_start, goal, x or best_seed");
  if (!(w_jerk >= 0.0f) || !(w_time >= 0.0f)) return fail(MG_ERR_ARG, "w_jerk and w_time must be >= 0");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if ((st = enqueue_eval(c, b, q_start, goal, x, nullptr, 1, nullptr, false, nullptr, b->pe_e, s)) != MG_OK)
    return st;
  if ((st = mg_retime(c, b, q_start, x, vmax, amax, jmax, b->sel_dt, b->sel_jerk, stream)) != MG_OK) return st;
  mg::TrajSelectArgs a;
  memset(&a, 0, sizeof(a));
  a.prob = b->d_prob;
  a.P = b->P;
  a.cost_e = b->cost_e;
  a.mc_e = b->mc_e;
  a.pe_e = b->pe_e;
  a.dt_s = b->sel_dt;
  a.jerk_s = b->sel_jerk;
  a.pos_tol = c->params.success_pos;
  a.rot_tol = c->params.success_rot;
  a.w_jerk = w_jerk;
  a.w_time = w_time;
  a.best_seed = best_seed;
  a.success = success;
  a.motion_time = motion_time;
  HIP_TRY(mg::launch_traj_select(a, s));
  return MG_OK;
}

mg_status mg_motion_gen(mg_ctx* c, mg_batch* ik, mg_batch* to, const float* q_start, const float* goal,
                        float* x_ik, float* x_to, int iters_ik, int iters1, int iters2, int m, int K,
                        const float* alpha, int mode, const float* vmax, const float* amax, const float* jmax,
                        float dt_min, float w_dist, float w_jerk, float w_time, int* ik_ok, int* best_seed,
                        int* success, float* motion_time, float* dt_out, void* stream) {
  mg_status st = common_checks(c, ik);
  if (st != MG_OK || (st = common_checks(c, to)) != MG_OK) return st;
  if (!dt_out || !best_seed) return fail(MG_ERR_ARG, "null dt_out or best_seed");
  // collision-free IK, seeds on the lines to its solutions, trajectory
  // optimization with the time-step passes, choice per problem.  Kernels
  // are launched directly: each pass runs once with its own parameters, so
  // a captured graph would not be replayed.  The solves' per-seed best
  // costs go to each batch's selection scratch (sel_dt), which nothing
  // reads before mg_traj_select rewrites it.
  if ((st = mg_solve(c, ik, q_start, goal, x_ik, iters_ik, m, K, alpha, mode, 25, 0, ik->sel_dt, nullptr, nullptr,
                     stream)) != MG_OK ||
      (st = mg_ik_seeds(c, ik, to, q_start, goal, x_ik, w_dist, x_to, ik_ok, stream)) != MG_OK ||
      (st = mg_solve_timestep(c, to, q_start, goal, x_to, iters1, iters2, m, K, alpha, mode, 25, 0, vmax, amax,
                              jmax, dt_min, to->sel_dt, nullptr, nullptr, dt_out, stream)) != MG_OK)
    return st;
  return mg_traj_select(c, to, q_start, goal, x_to, vmax, amax, jmax, w_jerk, w_time, best_seed, success,
                        motion_time, stream);
}

mg_status mg_steer(mg_ctx* c, mg_batch* b, int n_edges, const float* from, const float* to, float res,
                   int n_max, float* reach, int* last, float* dist, void* stream) {
  mg_status st = common_checks(c, b);
  if (st != MG_OK) return st;
  if (n_edges < 1 || n_max < 1) return fail(MG_ERR_ARG, "n_edges and n_max must be >= 1");
  if (!from || !to || !reach || !last) return fail(MG_ERR_ARG, "null from, to, reach or last");
  if (!(res > 0.0f)) return fail(MG_ERR_ARG, "res must be > 0");
  if (b->P != 1 || b->horizon[0] != 1 || (long)b->seeds[0] != (long)n_edges * (n_max + 1))
    return fail(MG_ERR_SHAPE, "the batch must hold one problem of horizon 1 with n_edges x (n_max + 1) = %ld seeds",
                (long)n_edges * (n_max + 1));
  hipStream_t s = static_cast<hipStream_t>(stream);
  mg::SteerArgs a;
  memset(&a, 0, sizeof(a));
  a.n_edges = n_edges;
  a.n_max = n_max;
  a.dof = c->D;
  a.res = res;
  a.from = from;
  a.to = to;
  a.q_lo = c->d_q_lo;
  a.q_hi = c->d_q_hi;
  a.pts = b->g_cur;      // the batch's [rows][D] workspace holds the samples
  a.mc = b->mc_e;
  a.reach = reach;
  a.last = last;
  a.dist = dist;
  HIP_TRY(mg::launch_steer_points(a, s));
  // clearance of every sample (a start and goal are not used at horizon 1
  // for the clearance)
  if ((st = enqueue_eval(c, b, c->d_zero, c->d_goal_id, b->g_cur, nullptr, 1, nullptr, false, nullptr, nullptr, s)) !=
      MG_OK)
    return st;
  HIP_TRY(mg::launch_steer_scan(a, s));
  return MG_OK;
}

mg_status mg_plan_batch(mg_ctx* c, mg_batch* b, int n_queries, const float* starts, const float* goals,
                        const float* retract, float res, int n_max, int n_samples, int k_near, int max_rounds,
                        int refine_rounds, unsigned seed, int max_waypoints, float* paths, int* n_waypoints,
                        void* stream) {
  mg_status st = common_checks(c, b);
  if (st != MG_OK) return st;
  if (n_queries < 1 || !starts || !goals || !paths || !n_waypoints)
    return fail(MG_ERR_ARG, "need n_queries >= 1, starts, goals, paths and n_waypoints");
  if (n_samples < 1 || k_near < 1 || 2 * k_near > 32 || max_rounds < 0 || refine_rounds < 0 || max_waypoints < 2)
    return fail(MG_ERR_ARG, "need n_samples >= 1, 1 <= k_near <= 16, max_rounds, refine_rounds >= 0, max_waypoints >= 2");
  if (b->P != 1 || b->horizon[0] != 1 || b->seeds[0] % (n_max + 1) != 0)
    return fail(MG_ERR_SHAPE, "the batch must hold one problem of horizon 1 with a multiple of n_max + 1 seeds");
  const int D = c->D, cap = b->seeds[0] / (n_max + 1);   // edges per steering launch
  const int rows = b->rows;                               // samples per clearance launch
  constexpr int kOversample = 32;                         // candidates drawn per kept sample
  hipStream_t s = static_cast<hipStream_t>(stream);
  for (int qy = 0; qy < n_queries; ++qy) n_waypoints[qy] = 0;
  std::vector<std::vector<float>> node;                  // graph nodes (host)
  std::vector<std::vector<std::pair<int, float>>> adj;   // undirected weighted edges
  std::vector<int> comp;                                 // union-find over the nodes
  auto add_node = [&](const float* q) {
    node.emplace_back(q, q + D);
    adj.emplace_back();
    comp.push_back((int)comp.size());
    return (int)node.size() - 1;
  };
  auto find = [&](int v) {
    while (comp[v] != v) v = comp[v] = comp[comp[v]];
    return v;
  };
  auto join = [&](int u, int v, float d) {
    adj[u].push_back({v, d});
    adj[v].push_back({u, d});
    comp[find(u)] = find(v);
  };
  auto dist = [&](const float* a, const float* bq) {
    double d2 = 0.0;
    for (int j = 0; j < D; ++j) d2 += ((double)a[j] - bq[j]) * ((double)a[j] - bq[j]);
    return (float)std::sqrt(d2);
  };
  // device buffers: steering edges, samples and their neighbours, the nodes
  const int p_cap = 4 * n_samples, k_cap = 2 * k_near;
  float *d_from = nullptr, *d_to = nullptr, *d_reach = nullptr, *d_smp = nullptr, *d_nodes = nullptr;
  int *d_last = nullptr, *d_idx = nullptr;
  size_t node_cap = 0;
  // (a horizon-1 batch of one round's candidates in the same world, for
  // their clearance)
  const int cl_rows = std::min(rows, kOversample * p_cap), one = 1;
  mg_batch* cb = nullptr;
  auto free_all = [&]() {
    dev_free(d_from); dev_free(d_to); dev_free(d_reach); dev_free(d_last); dev_free(d_smp); dev_free(d_idx);
    dev_free(d_nodes);
    if (cb) mg_batch_destroy(cb);
  };
  if ((st = dev_alloc(&d_from, (size_t)cap * D)) != MG_OK || (st = dev_alloc(&d_to, (size_t)cap * D)) != MG_OK ||
      (st = dev_alloc(&d_reach, (size_t)cap * D)) != MG_OK || (st = dev_alloc(&d_last, (size_t)cap)) != MG_OK ||
      (st = dev_alloc(&d_smp, (size_t)p_cap * D)) != MG_OK || (st = dev_alloc(&d_idx, (size_t)p_cap * k_cap)) != MG_OK ||
      (st = mg_batch_create(c, 1, &cl_rows, &one, &b->world[0], 1, 0, &cb)) != MG_OK) {
    free_all();
    return st;
  }
  std::vector<float> h_from((size_t)cap * D), h_to((size_t)cap * D), h_reach((size_t)cap * D);
  std::vector<int> h_last(cap);
  // steer_connect (Alg.3 on every edge, in launches of cap edges): an edge
  // that reaches its target joins the two nodes; one that stops short adds
  // its last valid sample as a node joined to the source (when it moved)
  auto steer_connect = [&](const std::vector<std::pair<int, int>>& edges, const std::vector<std::vector<float>>* tgt,
                           std::vector<int>* reached) -> mg_status {
    for (size_t e0 = 0; e0 < edges.size(); e0 += cap) {
      const int ne = (int)std::min(edges.size() - e0, (size_t)cap);
      for (int e = 0; e < cap; ++e) {
        const int k = (int)e0 + std::min(e, ne - 1);   // padding repeats the last edge
        const float* a = node[edges[k].first].data();
        const float* t = edges[k].second >= 0 ? node[edges[k].second].data() : (*tgt)[k].data();
        std::copy(a, a + D, &h_from[(size_t)e * D]);
        std::copy(t, t + D, &h_to[(size_t)e * D]);
      }
      HIP_TRY(hipMemcpyAsync(d_from, h_from.data(), h_from.size() * 4, hipMemcpyHostToDevice, s));
      HIP_TRY(hipMemcpyAsync(d_to, h_to.data(), h_to.size() * 4, hipMemcpyHostToDevice, s));
      mg_status r = mg_steer(c, b, cap, d_from, d_to, res, n_max, d_reach, d_last, nullptr, stream);
      if (r != MG_OK) return r;
      HIP_TRY(hipMemcpyAsync(h_reach.data(), d_reach, h_reach.size() * 4, hipMemcpyDeviceToHost, s));
      HIP_TRY(hipMemcpyAsync(h_last.data(), d_last, h_last.size() * 4, hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      for (int e = 0; e < ne; ++e) {
        const int k = (int)e0 + e, from = edges[k].first;
        const float* v = &h_reach[(size_t)e * D];
        const float* t = &h_to[(size_t)e * D];
        int to = -1;
        if (h_last[e] < 1) continue;                       // no progress or not checked
        // (the last sample is the target up to the rounding of a + (b - a))
        const bool full = dist(v, t) <= 1e-5f;
        if (full && edges[k].second >= 0) to = edges[k].second;
        else to = add_node(v);
        join(from, to, dist(node[from].data(), node[to].data()));
        if (reached && full) (*reached)[k] = to;
      }
    }
    return MG_OK;
  };
  // clearance of candidate samples: one horizon-1 evaluation launch per
  // batch-full of a batch sized for one round's candidates (world clearance
  // >= 0 keeps a sample; limits hold by construction)
  std::vector<float> h_rows((size_t)cl_rows * D), h_mc(cl_rows);
  auto clear_samples = [&](std::vector<std::vector<float>>& smp) -> mg_status {
    std::vector<std::vector<float>> keep;
    for (size_t s0 = 0; s0 < smp.size(); s0 += cl_rows) {
      const int n = (int)std::min(smp.size() - s0, (size_t)cl_rows);
      for (int r = 0; r < cl_rows; ++r) {
        const auto& q = smp[s0 + std::min(r, n - 1)];
        std::copy(q.begin(), q.end(), &h_rows[(size_t)r * D]);
      }
      HIP_TRY(hipMemcpyAsync(cb->g_cur, h_rows.data(), h_rows.size() * 4, hipMemcpyHostToDevice, s));
      mg_status r = enqueue_eval(c, cb, c->d_zero, c->d_goal_id, cb->g_cur, nullptr, 1, nullptr, false, nullptr,
                                 nullptr, s);
      if (r != MG_OK) return r;
      HIP_TRY(hipMemcpyAsync(h_mc.data(), cb->mc_e, (size_t)n * 4, hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      for (int i = 0; i < n; ++i)
        if (h_mc[i] >= 0.0f) keep.push_back(smp[s0 + i]);
    }
    smp.swap(keep);
    return MG_OK;
  };
  // the k nearest nodes of every sample, on the device
  std::vector<int> h_idx((size_t)p_cap * k_cap);
  auto nearest = [&](const std::vector<std::vector<float>>& smp, int kk) -> mg_status {
    if (node.size() > node_cap) {
      dev_free(d_nodes);
      node_cap = std::max<size_t>(2 * node.size(), 1024);
      mg_status r = dev_alloc(&d_nodes, node_cap * D);
      if (r != MG_OK) return r;
    }
    std::vector<float> hn(node.size() * D), hs(smp.size() * D);
    for (size_t i = 0; i < node.size(); ++i) std::copy(node[i].begin(), node[i].end(), &hn[i * D]);
    for (size_t i = 0; i < smp.size(); ++i) std::copy(smp[i].begin(), smp[i].end(), &hs[i * D]);
    HIP_TRY(hipMemcpyAsync(d_nodes, hn.data(), hn.size() * 4, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(d_smp, hs.data(), hs.size() * 4, hipMemcpyHostToDevice, s));
    mg::KnnArgs ka{(int)node.size(), (int)smp.size(), D, kk, d_nodes, d_smp, d_idx, nullptr};
    HIP_TRY(mg::launch_knn(ka, s));
    HIP_TRY(hipMemcpyAsync(h_idx.data(), d_idx, smp.size() * kk * sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return MG_OK;
  };
  // shortest path between two nodes, Dijkstra on a heap
  auto shortest = [&](int src, int dst, std::vector<int>& out) {
    const size_t n = node.size();
    std::vector<float> dd(n, 3.0e38f);
    std::vector<int> prev(n, -1);
    std::priority_queue<std::pair<float, int>, std::vector<std::pair<float, int>>, std::greater<>> pq;
    dd[src] = 0.0f;
    pq.push({0.0f, src});
    while (!pq.empty()) {
      const auto [du, u] = pq.top();
      pq.pop();
      if (du > dd[u]) continue;
      if (u == dst) break;
      for (auto& [v, w] : adj[u])
        if (du + w < dd[v]) { dd[v] = du + w; prev[v] = u; pq.push({dd[v], v}); }
    }
    out.clear();
    if (dd[dst] >= 3.0e38f) return 3.0e38f;
    for (int v = dst; v >= 0; v = prev[v]) out.push_back(v);
    std::reverse(out.begin(), out.end());
    return dd[dst];
  };
  auto run = [&]() -> mg_status {
    // nodes: start and goal of every query, then the retract configuration
    std::vector<int> sn(n_queries), gn(n_queries);
    for (int qy = 0; qy < n_queries; ++qy) {
      sn[qy] = add_node(starts + (size_t)qy * D);
      gn[qy] = add_node(goals + (size_t)qy * D);
    }
    std::vector<std::pair<int, int>> e0;
    for (int qy = 0; qy < n_queries; ++qy) e0.insert(e0.end(), {{sn[qy], gn[qy]}, {gn[qy], sn[qy]}});
    if (retract) {
      const int r = add_node(retract);
      for (int qy = 0; qy < n_queries; ++qy)
        e0.insert(e0.end(), {{sn[qy], r}, {r, sn[qy]}, {gn[qy], r}, {r, gn[qy]}});
    }
    mg_status r = steer_connect(e0, nullptr, nullptr);
    if (r != MG_OK) return r;
    std::vector<std::vector<int>> route(n_queries);
    std::vector<float> len(n_queries), c_min(n_queries), c_max(n_queries, 3.0e38f);
    std::vector<int> k_n(n_queries, k_near), p_n(n_queries, n_samples);
    int n_solved = 0;
    for (int qy = 0; qy < n_queries; ++qy) {
      len[qy] = find(sn[qy]) == find(gn[qy]) ? shortest(sn[qy], gn[qy], route[qy]) : 3.0e38f;
      c_min[qy] = dist(starts + (size_t)qy * D, goals + (size_t)qy * D);
      n_solved += !route[qy].empty();
    }
    std::mt19937 rng(seed);
    int refine_left = refine_rounds;
    for (int round = 0; round < max_rounds && (n_solved < n_queries || refine_left > 0); ++round) {
      // a query at random among the unsolved ones (Alg.2), or, once all are
      // solved, among all of them to refine its path in its informed set
      const bool refine = n_solved == n_queries;
      if (refine) --refine_left;
      std::vector<int> pool;
      for (int qy = 0; qy < n_queries; ++qy)
        if (refine || route[qy].empty()) pool.push_back(qy);
      const int qy = pool[std::uniform_int_distribution<int>(0, (int)pool.size() - 1)(rng)];
      const float cm = refine ? len[qy] : c_max[qy];
      const float* st_q = starts + (size_t)qy * D;
      const float* gl_q = goals + (size_t)qy * D;
      // candidates: uniform within the joint limits, or uniform in the
      // informed ellipsoid |q - start| + |q - goal| <= cm (a unit-ball
      // sample stretched to the semi-axes cm/2 along the start-goal line
      // and sqrt(cm^2 - c_min^2)/2 across it, turned onto that line by a
      // Householder reflection), outside the limits dropped
      std::vector<std::vector<float>> smp;
      const int n_cand = std::min(rows, kOversample * p_n[qy]);
      std::uniform_real_distribution<float> U(0.0f, 1.0f);
      std::normal_distribution<float> N01(0.0f, 1.0f);
      const bool ell = cm < 3.0e38f && c_min[qy] > 0.0f;
      std::vector<double> axis(D), hv(D);
      double hvv = 0.0;
      if (ell) {
        for (int j = 0; j < D; ++j) axis[j] = ((double)gl_q[j] - st_q[j]) / c_min[qy];
        for (int j = 0; j < D; ++j) hv[j] = (j == 0 ? 1.0 : 0.0) - axis[j];
        for (int j = 0; j < D; ++j) hvv += hv[j] * hv[j];
      }
      const double r1 = 0.5 * cm, r2 = ell ? 0.5 * std::sqrt(std::max(0.0, (double)cm * cm -
                                                                       (double)c_min[qy] * c_min[qy])) : 0.0;
      for (int i = 0; i < n_cand; ++i) {
        std::vector<float> q(D);
        if (!ell) {
          for (int j = 0; j < D; ++j) q[j] = c->q_lo[j] + (c->q_hi[j] - c->q_lo[j]) * U(rng);
        } else {
          std::vector<double> x(D);
          double n2 = 0.0;
          for (int j = 0; j < D; ++j) { x[j] = N01(rng); n2 += x[j] * x[j]; }
          const double rad = std::pow((double)U(rng), 1.0 / D) / std::sqrt(std::max(n2, 1e-300));
          for (int j = 0; j < D; ++j) x[j] *= rad * (j == 0 ? r1 : r2);
          double xv = 0.0;
          for (int j = 0; j < D; ++j) xv += x[j] * hv[j];
          bool in = true;
          for (int j = 0; j < D; ++j) {
            const double y = x[j] - (hvv > 1e-24 ? 2.0 * xv / hvv * hv[j] : 0.0);
            q[j] = (float)(0.5 * ((double)st_q[j] + gl_q[j]) + y);
            in = in && q[j] >= c->q_lo[j] && q[j] <= c->q_hi[j];
          }
          if (!in) continue;
        }
        smp.push_back(q);
      }
      // collision-free candidates only (one evaluation launch), the first
      // p_n of them kept; each is steered toward from its k nearest nodes
      // (found on the device)
      if ((r = clear_samples(smp)) != MG_OK) return r;
      if ((int)smp.size() > p_n[qy]) smp.resize(p_n[qy]);
      std::vector<std::pair<int, int>> edges;
      std::vector<std::vector<float>> tgt;
      const int kk = std::min<int>(k_n[qy], (int)node.size());
      if (!smp.empty()) {
        if ((r = nearest(smp, kk)) != MG_OK) return r;
        for (size_t i = 0; i < smp.size(); ++i)
          for (int u = 0; u < kk; ++u) {
            edges.push_back({h_idx[i * kk + u], -1});
            tgt.push_back(smp[i]);
          }
      }
      std::vector<int> reached(edges.size(), -1);
      if ((r = steer_connect(edges, &tgt, &reached)) != MG_OK) return r;
      // a sample reached from several nodes becomes one node: its copies
      // (edges i*kk .. i*kk + kk - 1) are joined at zero length
      for (size_t i = 0; i < smp.size(); ++i) {
        int first = -1;
        for (int u = 0; u < kk; ++u) {
          const int v = reached[i * kk + u];
          if (v < 0) continue;
          if (first < 0) { first = v; continue; }
          if (v == first) continue;
          join(first, v, 0.0f);
        }
      }
      // the roadmap is shared: an unsolved query whose start and goal the
      // round joined (union-find) takes its shortest path, and a refine
      // round updates the picked query's
      n_solved = 0;
      for (int u = 0; u < n_queries; ++u) {
        const bool look = route[u].empty() ? find(sn[u]) == find(gn[u]) : (refine && u == qy);
        if (look) {
          std::vector<int> rt;
          const float l2 = shortest(sn[u], gn[u], rt);
          if (!rt.empty() && (route[u].empty() || l2 < len[u])) { route[u] = rt; len[u] = l2; }
        }
        n_solved += !route[u].empty();
      }
      // a failed round widens the picked query's region and grows its
      // counts by a quarter (capped at 4x the samples, 2x the neighbours)
      if (!refine && route[qy].empty()) {
        if (c_max[qy] >= 3.0e38f) c_max[qy] = 2.0f * c_min[qy];
        c_max[qy] += 0.25f * c_min[qy];
        p_n[qy] = std::min(p_n[qy] + std::max(1, p_n[qy] / 4), p_cap);
        k_n[qy] = std::min(k_n[qy] + std::max(1, k_n[qy] / 4), k_cap);
      }
    }
    for (int qy = 0; qy < n_queries; ++qy) {
      if (route[qy].empty()) continue;
      // shortcut: from each waypoint, the farthest later one reachable directly
      const auto& rt = route[qy];
      std::vector<int> sc = {rt[0]};
      for (size_t i = 0; i + 1 < rt.size();) {
        std::vector<std::pair<int, int>> edges;
        for (size_t j = rt.size() - 1; j > i + 1; --j) edges.push_back({rt[i], rt[j]});
        size_t next = i + 1;
        if (!edges.empty()) {
          std::vector<int> reached(edges.size(), -1);
          if ((r = steer_connect(edges, nullptr, &reached)) != MG_OK) return r;
          for (size_t k = 0; k < edges.size(); ++k)
            if (reached[k] == edges[k].second) { next = rt.size() - 1 - k; break; }
        }
        sc.push_back(rt[next]);
        i = next;
      }
      if ((int)sc.size() > max_waypoints)
        return fail(MG_ERR_SHAPE, "query %d: the path has %d waypoints (max %d)", qy, (int)sc.size(), max_waypoints);
      float* out = paths + (size_t)qy * max_waypoints * D;
      for (size_t i = 0; i < sc.size(); ++i) std::copy(node[sc[i]].begin(), node[sc[i]].end(), out + i * D);
      n_waypoints[qy] = (int)sc.size();
    }
    return MG_OK;
  };
  st = run();
  free_all();
  return st;
}

mg_status mg_plan(mg_ctx* c, mg_batch* b, const float* start, const float* goal, const float* retract,
                  float res, int n_max, int n_samples, int k_near, int max_rounds, unsigned seed,
                  int max_waypoints, float* path, int* n_waypoints, void* stream) {
  return mg_plan_batch(c, b, 1, start, goal, retract, res, n_max, n_samples, k_near, max_rounds, 0, seed,
                       max_waypoints, path, n_waypoints, stream);
}

}  // extern "C"
