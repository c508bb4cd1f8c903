// mg_api.hip -- C ABI of libmg (declared in include/mg.h).
//
// Host-side bookkeeping only: argument checks, device tables, workspaces,
// launch sequencing and hipGraph capture of the solver iteration.  All
// arithmetic of the method runs in the kernels of mg_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
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

// Sphere groups for G lanes per evaluation (see mg::Groups).
struct GroupVariant {
  int G = 0, maxs = 0;
  bool ok = false;
  float* ftf = nullptr;
  int* jidx = nullptr;
  int4* info = nullptr;
  float4* sphere = nullptr;
  int* red = nullptr;
};

constexpr int kNumVariants = 3;
constexpr int kVariantG[kNumVariants] = {8, 16, 32};

}  // namespace

struct mg_ctx {
  int device = 0;
  int L = 0, D = 0, M = 0, n_ee = 0, depth = 8;
  bool serial = false;   // link l has parent l-1 and joint l
  std::vector<int> parent, joint, sphere_link, ee_link;
  std::vector<float> fixed_tf, sphere, ee_tf, q_lo, q_hi;
  mg::Params params{};
  float* d_fixed_tf = nullptr;
  int* d_joint = nullptr;
  float* d_q_lo = nullptr;
  float* d_q_hi = nullptr;
  float* d_ee_tf = nullptr;
  GroupVariant var[kNumVariants];
  Box* d_box = nullptr;
  int box_cap = 0, n_boxes = 0;
  int* d_world_off = nullptr;
  int world_cap = 0, n_worlds = 0;
  hipStream_t cap_stream = nullptr;
};

struct mg_batch {
  mg_ctx* ctx = nullptr;
  int P = 0, n_seeds = 0, rows = 0, K_max = 0, m_max = 0;
  std::vector<int> seeds, horizon, world;
  mg::Problem* d_prob = nullptr;
  mg::SeedInfo* d_seed = nullptr;
  int* d_chunk[kNumVariants] = {nullptr, nullptr, nullptr};
  int chunks[kNumVariants] = {0, 0, 0};
  int max_n = 0;      // largest T*D of a seed
  float *cost_e = nullptr, *gd_e = nullptr, *mc_e = nullptr, *grad_e = nullptr, *pe_e = nullptr;
  float *c_cur = nullptr, *g_cur = nullptr, *dir = nullptr, *best_c = nullptr, *best_x = nullptr;
  int* first = nullptr;
  float *S = nullptr, *Y = nullptr, *x_prev = nullptr, *g_prev = nullptr, *rho = nullptr;
  int* meta = nullptr;
  // cached solver graph and the arguments it was captured with
  hipGraphExec_t gexec = nullptr;
  std::vector<char> gkey;
  // evaluation-kernel timing (mg_set_timing): event pairs used as a ring
  bool timing = false;
  std::vector<hipEvent_t> ev_start, ev_stop;
  int ev_next = 0, ev_count = 0;
  int variant = -1;   // forced G variant (-1: automatic)
};

namespace {

mg::Robot dev_robot(const mg_ctx* c) {
  mg::Robot r;
  r.dof = c->D;
  r.serial = c->serial ? 1 : 0;
  r.n_links = c->L;
  r.n_ee = c->n_ee;
  r.n_spheres = c->M;
  r.fixed_tf = c->d_fixed_tf;
  r.joint = c->d_joint;
  r.q_lo = c->d_q_lo;
  r.q_hi = c->d_q_hi;
  r.ee_tf = c->d_ee_tf;
  return r;
}

// Partition the spheres into G groups, each on a single link, so that the
// largest group is as small as possible; every end-effector link gets a
// group (possibly without spheres) that evaluates its pose term.
mg_status build_groups(mg_ctx* c, int vi) {
  GroupVariant& v = c->var[vi];
  const int G = kVariantG[vi];
  v.G = G;
  v.ok = false;
  std::vector<int> count(c->L, 0);
  for (int m = 0; m < c->M; ++m) count[c->sphere_link[m]]++;
  std::vector<int> need(c->L, 0);
  for (int l = 0; l < c->L; ++l) need[l] = count[l] > 0 ? 1 : 0;
  for (int e = 0; e < c->n_ee; ++e) need[c->ee_link[e]] = 1;
  int used = 0;
  for (int l = 0; l < c->L; ++l) used += need[l];
  if (used > G) return MG_OK;  // infeasible for this G
  std::vector<int> ng = need;
  for (int extra = G - used; extra > 0; --extra) {
    int best = -1, best_load = 0;
    for (int l = 0; l < c->L; ++l) {
      if (!ng[l] || count[l] == 0) continue;
      const int load = (count[l] + ng[l] - 1) / ng[l];
      if (load > best_load) { best_load = load; best = l; }
    }
    if (best < 0 || best_load <= 1) break;
    ng[best]++;
  }
  int largest = 0;
  for (int l = 0; l < c->L; ++l)
    if (ng[l]) largest = std::max(largest, (count[l] + ng[l] - 1) / ng[l]);
  int maxs = 0;
  for (int cand : {2, 4, 8, 16})
    if (largest <= cand && mg::eval_shape_supported(G, cand)) { maxs = cand; break; }
  if (maxs == 0) return MG_OK;  // groups too large for this G
  v.maxs = maxs;
  const int depth = c->depth;
  // spheres of each link in input order
  std::vector<std::vector<int>> by_link(c->L);
  for (int m = 0; m < c->M; ++m) by_link[c->sphere_link[m]].push_back(m);
  // unused chain slots hold identity transforms with no joint
  std::vector<float> ftf((size_t)G * depth * 12, 0.0f);
  for (size_t q = 0; q < (size_t)G * depth; ++q) ftf[q * 12 + 0] = ftf[q * 12 + 5] = ftf[q * 12 + 10] = 1.0f;
  std::vector<int> jidx((size_t)G * depth, -1), chain((size_t)G * depth, -1);
  std::vector<int4> info(G, make_int4(0, 0, 0, -1));
  std::vector<float4> sph((size_t)G * maxs, make_float4(0.0f, 0.0f, 0.0f, 0.0f));
  int g = 0;
  for (int l = 0; l < c->L; ++l) {
    if (!ng[l]) continue;
    std::vector<int> path;   // base .. l
    for (int x = l; x >= 0; x = c->parent[x]) path.push_back(x);
    std::reverse(path.begin(), path.end());
    if ((int)path.size() > depth)
      return fail(MG_ERR_SHAPE, "chain of link %d has %zu links > %d", l, path.size(), depth);
    const int n = count[l];
    for (int part = 0; part < ng[l]; ++part) {
      const int b = n * part / ng[l], e = n * (part + 1) / ng[l];
      for (size_t i = 0; i < path.size(); ++i) {
        chain[g * depth + i] = path[i];
        jidx[g * depth + i] = c->joint[path[i]];
        for (int q = 0; q < 12; ++q) ftf[((size_t)g * depth + i) * 12 + q] = c->fixed_tf[path[i] * 12 + q];
      }
      int ee = -1;
      if (part == 0)
        for (int k = 0; k < c->n_ee; ++k)
          if (c->ee_link[k] == l) ee = k;
      info[g] = make_int4((int)path.size(), 0, e - b, ee);
      for (int i = b; i < e; ++i) {
        const int m = by_link[l][i];
        sph[(size_t)g * maxs + (i - b)] =
            make_float4(c->sphere[4 * m + 0], c->sphere[4 * m + 1], c->sphere[4 * m + 2], c->sphere[4 * m + 3]);
      }
      ++g;
    }
  }
  // unused lanes keep empty groups (no chain, no spheres)
  // reduction lists: joint j sums slots (g, i) whose chain link carries j
  std::vector<int> off(c->D + 1, 0), slots;
  for (int j = 0; j < c->D; ++j) {
    off[j] = (int)slots.size();
    for (int gg = 0; gg < G; ++gg)
      for (int i = 0; i < info[gg].x; ++i)
        if (jidx[gg * depth + i] == j) slots.push_back(gg * depth + i);
  }
  off[c->D] = (int)slots.size();
  std::vector<int> red = off;
  red.insert(red.end(), slots.begin(), slots.end());
  mg_status st;
  if ((st = dev_upload(&v.ftf, ftf)) != MG_OK) return st;
  if ((st = dev_upload(&v.jidx, jidx)) != MG_OK) return st;
  if ((st = dev_upload(&v.info, info)) != MG_OK) return st;
  if ((st = dev_upload(&v.sphere, sph)) != MG_OK) return st;
  if ((st = dev_upload(&v.red, red)) != MG_OK) return st;
  v.ok = true;
  return MG_OK;
}

mg::Groups dev_groups(const mg_ctx* c, int vi) {
  mg::Groups g;
  g.G = c->var[vi].G;
  g.depth = c->depth;
  g.maxs = c->var[vi].maxs;
  g.ftf = c->var[vi].ftf;
  g.jidx = c->var[vi].jidx;
  g.info = c->var[vi].info;
  g.sphere = c->var[vi].sphere;
  g.red = c->var[vi].red;
  return g;
}

mg::Params to_dev(const mg_params& p) {
  mg::Params d;
  d.a0 = p.a0; d.a1 = p.a1; d.a2 = p.a2; d.a3 = p.a3;
  d.a6 = p.a6; d.a7 = p.a7; d.a8 = p.a8; d.a9 = p.a9;
  d.w_bound = p.w_bound; d.eta2 = p.eta2; d.w_coll = p.w_coll; d.eta = p.eta; d.dt = p.dt;
  d.vel_all = p.vel_all; d.swept = p.swept; d.sweep_steps = p.sweep_steps;
  d.ls_eta1 = p.ls_eta1; d.ls_eta_w = p.ls_eta_w;
  d.success_pos = p.success_pos; d.success_rot = p.success_rot;
  return d;
}

mg_status check_params(const mg_params* p) {
  if (!p) return fail(MG_ERR_ARG, "params is null");
  if (!(p->dt > 0)) return fail(MG_ERR_ARG, "dt must be > 0");
  if (!(p->eta >= 0) || !(p->eta2 > 0)) return fail(MG_ERR_ARG, "eta must be >= 0 and eta2 > 0");
  if (p->swept) return fail(MG_ERR_UNSUPPORTED, "swept collision is not implemented in this build");
  return MG_OK;
}

// G variant for a call evaluating n_evals rows x candidates: the fewest
// lanes per evaluation (least repeated kinematics) that still gives every
// SIMD about four wavefronts; MG_LANES_PER_EVAL forces a choice.
int pick_variant(const mg_batch* b, long n_evals) {
  const mg_ctx* c = b->ctx;
  if (b->variant >= 0 && c->var[b->variant].ok) return b->variant;
  const char* env = getenv("MG_LANES_PER_EVAL");
  if (env) {
    const int G = atoi(env);
    for (int i = 0; i < kNumVariants; ++i)
      if (kVariantG[i] == G && c->var[i].ok) return i;
  }
  const long target_lanes = 256L * 4 * 4 * mg::kWave;   // CUs x SIMDs x waves x lanes
  int pick = -1;
  for (int i = 0; i < kNumVariants; ++i) {
    if (!c->var[i].ok) continue;
    pick = i;
    if (n_evals * kVariantG[i] >= target_lanes) break;
  }
  return pick;
}

mg::EvalArgs eval_args(const mg_ctx* c, const mg_batch* b, int vi, const float* q_start,
                       const float* goal, const float* x, const float* d, int K, const float* alpha) {
  mg::EvalArgs a;
  memset(&a, 0, sizeof(a));
  a.rb = dev_robot(c);
  a.gr = dev_groups(c, vi);
  a.pr = c->params;
  a.prob = b->d_prob;
  a.chunk_prefix = b->d_chunk[vi];
  a.P = b->P;
  a.rows = b->rows;
  a.box = c->d_box;
  a.world_off = c->d_world_off;
  a.q_start = q_start;
  a.goal = goal;
  a.x = x;
  a.d = d;
  a.K = K;
  for (int k = 0; k < K; ++k) a.alpha[k] = alpha ? alpha[k] : 0.0f;
  a.cost_e = b->cost_e;
  a.gd_e = b->gd_e;
  a.mc_e = b->mc_e;
  a.grad_e = b->grad_e;
  a.pe_e = nullptr;
  return a;
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

mg_status enqueue_eval(mg_ctx* c, mg_batch* b, const float* q_start, const float* goal,
                       const float* x, const float* d, int K, const float* alpha, bool grad,
                       float* grad_out, float* pe_out, hipStream_t s) {
  const int vi = pick_variant(b, (long)b->rows * K);
  if (vi < 0) return fail(MG_ERR_UNSUPPORTED, "robot needs more sphere groups than lanes per evaluation");
  mg::EvalArgs a = eval_args(c, b, vi, q_start, goal, x, d, K, alpha);
  if (grad_out) a.grad_e = grad_out;
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
  HIP_TRY(mg::launch_eval(a, b->chunks[vi], d != nullptr, grad, s));
  if (timed) {
    HIP_TRY(hipEventRecord(b->ev_stop[slot], s));
    b->ev_next = (slot + 1) % (int)b->ev_start.size();
    b->ev_count = std::min(b->ev_count + 1, (int)b->ev_start.size());
  }
  return MG_OK;
}

mg_status enqueue_select(mg_ctx* c, mg_batch* b, const float* x, const float* c0, const float* g0,
                         const float* d, int K, const float* alpha, int mode, float* x_out,
                         float* c_out, float* g_out, int* chosen, float* mc_out, bool track,
                         hipStream_t s) {
  mg::SelectArgs a;
  memset(&a, 0, sizeof(a));
  a.seeds = b->d_seed;
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
  a.x_out = x_out; a.c_out = c_out; a.g_out = g_out; a.chosen = chosen; a.mc_out = mc_out;
  a.best_c = track ? b->best_c : nullptr;
  a.best_x = track ? b->best_x : nullptr;
  HIP_TRY(mg::launch_select(a, b->max_n, s));
  return MG_OK;
}

mg_status enqueue_lbfgs(mg_ctx* c, mg_batch* b, int m, int reset, const float* x, const float* g,
                        float* dir, int* first, hipStream_t s) {
  mg::LbfgsArgs a;
  memset(&a, 0, sizeof(a));
  a.seeds = b->d_seed;
  a.n_seeds = b->n_seeds;
  a.rows = b->rows;
  a.dof = c->D;
  a.m = m;
  a.reset = reset;
  a.x = x; a.g = g; a.dir = dir;
  a.S = b->S; a.Y = b->Y; a.x_prev = b->x_prev; a.g_prev = b->g_prev;
  a.rho = b->rho; a.meta = b->meta; a.first = first;
  a.m_max = b->m_max;
  HIP_TRY(mg::launch_lbfgs(a, b->max_n, s));
  return MG_OK;
}

mg_status check_K_alpha(const mg_batch* b, int K, const float* alpha) {
  if (K < 1 || K > b->K_max) return fail(MG_ERR_SHAPE, "K = %d outside 1..%d", K, b->K_max);
  if (!alpha) return fail(MG_ERR_ARG, "alpha is null");
  for (int k = 0; k < K; ++k)
    if (!(alpha[k] >= 0.0f)) return fail(MG_ERR_ARG, "alpha[%d] must be >= 0", k);
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
  int maxdepth = 0;
  for (int l = 0; l < c->L; ++l) {
    int dpt = 0;
    for (int x = l; x >= 0; x = c->parent[x]) ++dpt;
    maxdepth = std::max(maxdepth, dpt);
  }
  if (maxdepth > 16) { delete c; return fail(MG_ERR_SHAPE, "kinematic chain deeper than 16 links"); }
  c->depth = maxdepth <= 8 ? 8 : 16;
  c->serial = c->L == c->D;
  for (int l = 0; l < c->L; ++l) c->serial = c->serial && c->parent[l] == l - 1 && c->joint[l] == l;
  if ((st = dev_upload(&c->d_fixed_tf, c->fixed_tf)) != MG_OK ||
      (st = dev_upload(&c->d_joint, c->joint)) != MG_OK ||
      (st = dev_upload(&c->d_q_lo, c->q_lo)) != MG_OK ||
      (st = dev_upload(&c->d_q_hi, c->q_hi)) != MG_OK ||
      (st = dev_upload(&c->d_ee_tf, c->ee_tf)) != MG_OK) {
    mg_destroy(c);
    return st;
  }
  bool any = false;
  for (int vi = 0; vi < kNumVariants; ++vi) {
    if ((st = build_groups(c, vi)) != MG_OK) { mg_destroy(c); return st; }
    any = any || c->var[vi].ok;
  }
  if (!any) {
    mg_destroy(c);
    return fail(MG_ERR_UNSUPPORTED, "robot spheres do not fit 32 groups of at most 4 (or 16 of 8, 8 of 16)");
  }
  hipError_t e = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking);
  if (e != hipSuccess) { mg_destroy(c); return fail(MG_ERR_HIP, "hipStreamCreate: %s", hipGetErrorString(e)); }
  *out = c;
  return MG_OK;
}

void mg_destroy(mg_ctx* c) {
  if (!c) return;
  (void)hipDeviceSynchronize();
  dev_free(c->d_fixed_tf); dev_free(c->d_joint); dev_free(c->d_q_lo); dev_free(c->d_q_hi); dev_free(c->d_ee_tf);
  for (auto& v : c->var) { dev_free(v.ftf); dev_free(v.jidx); dev_free(v.info); dev_free(v.sphere); dev_free(v.red); }
  dev_free(c->d_box); dev_free(c->d_world_off);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  delete c;
}

mg_status mg_set_params(mg_ctx* c, const mg_params* params) {
  if (!c) return fail(MG_ERR_ARG, "null context");
  mg_status st = check_params(params);
  if (st != MG_OK) return st;
  c->params = to_dev(*params);
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
  for (int vi = 0; vi < kNumVariants; ++vi) {
    const int epw = mg::kBlock / kVariantG[vi];
    std::vector<int> pre(P + 1, 0);
    for (int p = 0; p < P; ++p) pre[p + 1] = pre[p] + (seeds[p] * horizon[p] + epw - 1) / epw;
    b->chunks[vi] = pre[P];
    if ((st = dev_upload(&b->d_chunk[vi], pre)) != MG_OK) return bail(st);
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
      (st = dev_alloc(&b->meta, 2 * n_seeds)) != MG_OK)
    return bail(st);
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
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  for (auto e : b->ev_start) (void)hipEventDestroy(e);
  for (auto e : b->ev_stop) (void)hipEventDestroy(e);
  dev_free(b->d_prob); dev_free(b->d_seed);
  for (auto& p : b->d_chunk) dev_free(p);
  dev_free(b->cost_e); dev_free(b->gd_e); dev_free(b->mc_e); dev_free(b->grad_e); dev_free(b->pe_e);
  dev_free(b->c_cur); dev_free(b->g_cur); dev_free(b->dir); dev_free(b->best_c); dev_free(b->best_x);
  dev_free(b->first); dev_free(b->S); dev_free(b->Y); dev_free(b->x_prev); dev_free(b->g_prev);
  dev_free(b->rho); dev_free(b->meta);
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
  return enqueue_select(c, b, x, c0, g0, dir, K, alpha, mode, x_out, c_out, g_out, chosen, min_clear, false, s);
}

}  // extern "C"

namespace {

mg_status enqueue_iteration(mg_ctx* c, mg_batch* b, const float* q_start, const float* goal, float* x,
                            int m, int K, const float* alpha, int mode, hipStream_t s) {
  mg_status st;
  if ((st = enqueue_lbfgs(c, b, m, 0, x, b->g_cur, b->dir, b->first, s)) != MG_OK) return st;
  if ((st = enqueue_eval(c, b, q_start, goal, x, b->dir, K, alpha, true, nullptr, nullptr, s)) != MG_OK) return st;
  return enqueue_select(c, b, x, b->c_cur, b->g_cur, b->dir, K, alpha, mode, x, b->c_cur, b->g_cur,
                        nullptr, nullptr, true, s);
}

template <typename T>
void key_push(std::vector<char>& k, const T& v) {
  const char* p = reinterpret_cast<const char*>(&v);
  k.insert(k.end(), p, p + sizeof(T));
}

}  // namespace

extern "C" {

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

  int done = 0;
  if (use_graph && iters >= graph_inner) {
    std::vector<char> key;
    key_push(key, q_start); key_push(key, goal); key_push(key, x); key_push(key, m); key_push(key, K);
    key_push(key, mode); key_push(key, graph_inner); key_push(key, c->params);
    key_push(key, c->d_box); key_push(key, c->d_world_off);
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

}  // extern "C"
