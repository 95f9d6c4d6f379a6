// libpakr: host side of the C ABI declared in include/pakr.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "pakr_adjoint.hpp"
#include "pakr_kernels.hpp"

using namespace pakr;

namespace {

constexpr int AUTO_GRID_MAX = 1024;      // workspace sizing bound for grid = 0
constexpr int DEFAULT_PATH_EDGES = 4096;

// Message of the last failed init call on this thread.  A plain character
// array: a thread_local with a destructor would register an exit-time
// handler in this library, which runs after the HIP runtime may be gone.
thread_local char g_init_error[512];

void set_init_error(const std::string& msg) {
  std::snprintf(g_init_error, sizeof g_init_error, "%s", msg.c_str());
}

struct Layout {
  size_t hdr, bar, sols, pstates, pactions, states, actions, parents, costs, obs, nn_keys, stg,
      counts, goalmin, total;
};

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

int sys_npos(int id) {
  return (id == PAKR_DI3 || id == PAKR_QUAD || id == PAKR_DUBINS) ? 3 : 2;
}
int sys_d(int id) {
  switch (id) {
    case PAKR_DI2: return 4;
    case PAKR_DI3: return 6;
    case PAKR_CAR: return 5;
    case PAKR_QUAD: return 12;
    case PAKR_DUBINS: return 6;
    case PAKR_UNI1: return 3;
    case PAKR_UNI2: return 5;
    case PAKR_ACROBOT: return 4;
    case PAKR_CARTPOLE: return 4;
  }
  return -1;
}
int sys_m(int id) {
  switch (id) {
    case PAKR_DI2: return 2;
    case PAKR_DI3: return 3;
    case PAKR_CAR: return 2;
    case PAKR_QUAD: return 4;
    case PAKR_DUBINS: return 3;
    case PAKR_UNI1: return 2;
    case PAKR_UNI2: return 2;
    case PAKR_ACROBOT: return 1;
    case PAKR_CARTPOLE: return 1;
  }
  return -1;
}

// Estimated operations of one evaluation of f beyond its linear part: its
// arithmetic plus ~4 for each hardware sine/cosine pair (three and a
// reciprocal for the quadrotor, two and a reciprocal for the car, two and a
// division for the acrobot, one or two for the others).
double f_eval_of(int id) {
  switch (id) {
    case PAKR_QUAD: return 96.0;
    case PAKR_CAR: return 24.0;
    case PAKR_DUBINS: return 24.0;
    case PAKR_ACROBOT: return 56.0;
    case PAKR_UNI1:
    case PAKR_UNI2:
    case PAKR_CARTPOLE: return 16.0;
  }
  return 0.0;
}

int obs_floats_of(int npos, int n_box, int n_sph) { return n_box * 2 * npos + n_sph * (npos + 1); }

// Lanes per candidate: split the obstacle set so each lane tests about three
// or more, as long as the rollout workgroups fit in the grid (and MAX_GR).
int lanes_for(const pakr_params& p, int n_obs, int grid_limit) {
  int L = p.lanes_per_candidate;
  if (L <= 0) {
    L = 1;
    while (L < 8 && n_obs >= 3 * (2 * L)) L <<= 1;
  }
  const size_t cap = (size_t)std::min(grid_limit, MAX_GR);
  while (L > 1 && ((size_t)p.B * L + NT - 1) / NT > cap) L >>= 1;
  return L;
}

// Rollout threads per workgroup.  A candidate's rollout is one serial chain
// per lane; when that chain is long (car, quadrotor: trigonometry in every
// evaluation of f) half the workgroup takes candidates, so each SIMD runs one
// rollout wave instead of two, provided that still leaves at most one rollout
// chunk per workgroup.  Short chains (double integrators) use the whole
// workgroup: more rollout workgroups would cost more in the insertion scan and
// the barrier than the shorter chain saves.
int rollout_threads(const pakr_system& sys, const pakr_params& p, int n_obs, int lanes, int G) {
  const double f_eval = f_eval_of(sys.id);
  const double chain =
      (double)p.T * (12.0 * sys.d + 4.0 * f_eval + 3.0 * sys_npos(sys.id) * n_obs / lanes);
  const long long half = NT / 2;
  const bool fits = ((long long)p.B * lanes + half - 1) / half <= G;
  return (chain >= 8000.0 && fits) ? (int)half : NT;
}

Layout make_layout(int d, int m, const pakr_params& p, int G, int obs_floats, int lanes,
                   int rt = NT) {
  Layout L{};
  const int K = p.B / p.A;
  const int cpb = rt / lanes;
  const int GR = (p.B + cpb - 1) / cpb;
  const size_t S = (size_t)GR * cpb;
  const int maxe = p.max_path_edges > 0 ? p.max_path_edges : DEFAULT_PATH_EDGES;
  const size_t N = (size_t)p.n_cap;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align_up(off + bytes);
    return at;
  };
  L.hdr = take(sizeof(DevHeader));
  L.bar = take(sizeof(uint32_t) * (size_t)std::max(G, 1));
  L.sols = take(sizeof(DevSolution) * MAX_SOLUTIONS);
  L.pstates = take(sizeof(float) * (size_t)(maxe + 1) * d);
  L.pactions = take(sizeof(float) * (size_t)maxe * m);
  L.states = take(sizeof(float) * N * d);
  L.actions = take(sizeof(float) * N * m);
  L.parents = take(sizeof(int) * N);
  L.costs = take(sizeof(float) * N);
  L.obs = take(sizeof(float) * (size_t)std::max(obs_floats, 1));
  L.nn_keys = take(sizeof(unsigned long long) * 2 * (size_t)K);  // two NN key buffers
  L.stg = take(sizeof(float) * S * (size_t)(d + m + 4));
  L.counts = take(sizeof(int) * GR);
  L.goalmin = take(sizeof(unsigned long long) * GR);
  L.total = off;
  return L;
}

bool finite_f(float v) { return std::isfinite(v); }

// Host copy of the device validity test, used to check x_init.
bool host_state_ok(const pakr_system& s, const pakr_scene& sc, const float* x) {
  const int P = sc.npos, d = s.d;
  for (int i = 0; i < d; ++i)
    if (!std::isfinite(x[i])) return false;
  for (int c = 0; c < P; ++c)
    if (!(x[c] >= sc.ws_lo[c] && x[c] <= sc.ws_hi[c])) return false;
  for (int i = P; i < d; ++i)
    if (!(x[i] >= s.lim_lo[i] && x[i] <= s.lim_hi[i])) return false;
  if (s.vnorm_max > 0.0f) {
    float s2 = 0.0f;
    for (int c = 0; c < P; ++c) s2 += x[P + c] * x[P + c];
    if (!(s2 <= s.vnorm_max * s.vnorm_max)) return false;
  }
  for (int b = 0; b < sc.n_box; ++b) {
    bool inside = true;
    for (int c = 0; c < P; ++c)
      inside = inside && std::fabs(x[c] - sc.box_c[b * P + c]) <= sc.box_h[b * P + c];
    if (inside) return false;
  }
  for (int q = 0; q < sc.n_sphere; ++q) {
    float d2 = 0.0f;
    for (int c = 0; c < P; ++c) {
      const float e = x[c] - sc.sph_c[q * P + c];
      d2 += e * e;
    }
    if (d2 <= sc.sph_r[q] * sc.sph_r[q]) return false;
  }
  return true;
}

// System record checks (and the scene's position dimension).
std::string validate_system(const pakr_system* s, const pakr_scene* sc) {
  if (s->id < PAKR_DI2 || s->id > PAKR_CARTPOLE) return "unknown system id";
  if (s->d != sys_d(s->id) || s->m != sys_m(s->id)) return "d/m do not match the system";
  if (sc->npos != sys_npos(s->id)) return "scene npos does not match the system";
  for (int i = 0; i < s->d; ++i) {
    if (!finite_f(s->sample_lo[i]) || !finite_f(s->sample_hi[i]) ||
        !(s->sample_lo[i] <= s->sample_hi[i]))
      return "bad sampling box";
    if (std::isnan(s->lim_lo[i]) || std::isnan(s->lim_hi[i]) || !(s->lim_lo[i] <= s->lim_hi[i]))
      return "bad state limits";
    if (i < sc->npos && (std::isfinite(s->lim_lo[i]) || std::isfinite(s->lim_hi[i])))
      return "position limits must be infinite (the workspace bounds positions)";
  }
  for (int i = 0; i < s->m; ++i)
    if (!finite_f(s->u_lo[i]) || !finite_f(s->u_hi[i]) || !(s->u_lo[i] <= s->u_hi[i]))
      return "bad control box";
  if (!(s->vnorm_max >= 0.0f) || !std::isfinite(s->vnorm_max)) return "bad vnorm_max";
  if (s->vnorm_max > 0.0f && s->id != PAKR_DI2 && s->id != PAKR_DI3)
    return "vnorm_max applies to double integrators only";
  if (s->id == PAKR_CAR && !(s->dyn[0] > 0.0f)) return "car wheelbase must be > 0";
  if (s->id == PAKR_QUAD && !(s->dyn[0] > 0.0f && s->dyn[2] > 0.0f && s->dyn[3] > 0.0f &&
                             s->dyn[4] > 0.0f && std::isfinite(s->dyn[1])))
    return "quadrotor mass and inertia must be > 0";
  if (s->id == PAKR_ACROBOT) {
    for (int i = 0; i < 7; ++i)
      if (!(s->dyn[i] > 0.0f) || !std::isfinite(s->dyn[i]))
        return "acrobot masses, lengths and inertias must be > 0";
    if (!std::isfinite(s->dyn[7])) return "acrobot gravity must be finite";
  }
  if (s->id == PAKR_CARTPOLE && !(s->dyn[0] > 0.0f && std::isfinite(s->dyn[0]) &&
                                 std::isfinite(s->dyn[1])))
    return "cart-pole pole length must be > 0";
  return std::string();
}

// Workspace box and obstacle records.
std::string validate_scene(const pakr_scene* sc) {
  const int P = sc->npos;
  for (int c = 0; c < P; ++c)
    if (!finite_f(sc->ws_lo[c]) || !finite_f(sc->ws_hi[c]) || !(sc->ws_lo[c] < sc->ws_hi[c]))
      return "bad workspace box";
  if (sc->n_box < 0 || sc->n_sphere < 0) return "negative obstacle count";
  if (sc->n_box + sc->n_sphere > PAKR_MAX_OBSTACLES) return "too many obstacles";
  if (sc->n_box > 0 && (!sc->box_c || !sc->box_h)) return "null box arrays";
  if (sc->n_sphere > 0 && (!sc->sph_c || !sc->sph_r)) return "null sphere arrays";
  for (int i = 0; i < sc->n_box * P; ++i)
    if (!finite_f(sc->box_c[i]) || !(sc->box_h[i] > 0.0f) || !finite_f(sc->box_h[i]))
      return "bad box";
  for (int i = 0; i < sc->n_sphere; ++i) {
    if (!(sc->sph_r[i] > 0.0f) || !finite_f(sc->sph_r[i])) return "bad sphere radius";
    for (int c = 0; c < P; ++c)
      if (!finite_f(sc->sph_c[i * P + c])) return "bad sphere centre";
  }
  return std::string();
}

// Goal ball inside the workspace (Sec. III).
std::string validate_goal(const pakr_goal* g, const pakr_scene* sc) {
  if (!(g->radius > 0.0f) || !finite_f(g->radius)) return "goal radius must be > 0";
  for (int c = 0; c < sc->npos; ++c)
    if (!(g->center[c] >= sc->ws_lo[c] && g->center[c] <= sc->ws_hi[c]))
      return "goal centre outside the workspace";
  return std::string();
}

// Returns an empty string when the query is well formed.
std::string validate(const pakr_system* s, const pakr_scene* sc, const float* x0,
                     const pakr_goal* g, const pakr_params* p, int* code) {
  *code = PAKR_E_INVALID_ARG;
  if (!s || !sc || !x0 || !g || !p) return "null argument";
  std::string m = validate_system(s, sc);
  if (!m.empty()) return m;
  if (p->A < 1 || p->B < 1 || p->B > PAKR_MAX_B) return "B must be in [1, 65536], A >= 1";
  if (p->B % p->A != 0) return "B must be a multiple of A";
  if (p->T < 1) return "T must be >= 1";
  if (!(p->dt > 0.0f) || !std::isfinite(p->dt)) return "dt must be finite and > 0";
  if (p->n_cap < p->B + 1 || p->n_cap > (1 << 28)) return "n_cap must be in [B+1, 2^28]";
  if (p->cost_kind != PAKR_COST_DURATION && p->cost_kind != PAKR_COST_PATH_LENGTH)
    return "bad cost_kind";
  if (p->heuristic_kind < PAKR_H_ADMISSIBLE || p->heuristic_kind > PAKR_H_NONE)
    return "bad heuristic_kind";
  if (p->heuristic_kind == PAKR_H_ADMISSIBLE && p->cost_kind == PAKR_COST_DURATION &&
      !(p->h_speed > 0.0f && std::isfinite(p->h_speed)))
    return "h_speed must be > 0";
  if (!(p->cost_bound > 0.0)) return "cost_bound must be > 0";
  if (p->max_iters_per_round < 1) return "max_iters_per_round must be >= 1";
  if (p->grid < 0) return "grid must be >= 0";
  if (p->max_path_edges < 0) return "max_path_edges must be >= 0";
  if (p->lanes_per_candidate != 0 && p->lanes_per_candidate != 1 && p->lanes_per_candidate != 2 &&
      p->lanes_per_candidate != 4 && p->lanes_per_candidate != 8 && p->lanes_per_candidate != 16)
    return "lanes_per_candidate must be 0, 1, 2, 4, 8 or 16";
  if (p->workgroups_per_cu < 0 || p->workgroups_per_cu > 8) return "workgroups_per_cu must be 0..8";
  if (p->spec_tiles < -1 || p->spec_tiles > 1024) return "spec_tiles must be -1..1024";
  if (p->tier0_nodes < -1) return "tier0_nodes must be >= -1";
  if (p->tier1_nodes < -1) return "tier1_nodes must be >= -1";
  if (p->tier1_grid < 0 || p->tier1_grid == 1) return "tier1_grid must be 0 or >= 2";
  if (p->tier_scan_cycles < 0) return "tier_scan_cycles must be >= 0";
  m = validate_scene(sc);
  if (!m.empty()) return m;
  *code = PAKR_E_GOAL_INVALID;
  m = validate_goal(g, sc);
  if (!m.empty()) return m;
  *code = PAKR_E_START_INVALID;
  if (!host_state_ok(*s, *sc, x0)) return "x_init is not in X_free (bounds, limits or obstacles)";
  *code = PAKR_OK;
  return std::string();
}

template <int SYS>
const void* pick_kernel(int qt) {
  if constexpr (Sys<SYS>::D > 6) {
    return reinterpret_cast<const void*>(&k_plan<SYS, 1>);
  } else {
    if (qt == 1) return reinterpret_cast<const void*>(&k_plan<SYS, 1>);
    if (qt == 2) return reinterpret_cast<const void*>(&k_plan<SYS, 2>);
    return reinterpret_cast<const void*>(&k_plan<SYS, 4>);
  }
}

const void* kernel_for(int sys, int qt) {
  switch (sys) {
    case PAKR_DI2: return pick_kernel<PAKR_DI2>(qt);
    case PAKR_DI3: return pick_kernel<PAKR_DI3>(qt);
    case PAKR_CAR: return pick_kernel<PAKR_CAR>(qt);
    case PAKR_DUBINS: return pick_kernel<PAKR_DUBINS>(qt);
    case PAKR_UNI1: return pick_kernel<PAKR_UNI1>(qt);
    case PAKR_UNI2: return pick_kernel<PAKR_UNI2>(qt);
    case PAKR_ACROBOT: return pick_kernel<PAKR_ACROBOT>(qt);
    case PAKR_CARTPOLE: return pick_kernel<PAKR_CARTPOLE>(qt);
    default: return pick_kernel<PAKR_QUAD>(qt);
  }
}

// Targets per thread in a single-query plan's NN scan: four (one above 6
// state dimensions, where the loop has no registers to spare), fewer when K
// is too small for every thread to hold that many.
int qt_for(int K, int d) {
  int qt = d <= 6 ? 4 : 1;
  while (qt > 1 && K <= (NT / 16) * qt / 2) qt >>= 1;
  return qt;
}

// Threads per NN node group, qt targets per thread: enough to hold a chunk of
// min(K, NN_KC<qt>) targets, and at least NT / 16 (so each group's slice of a
// tile is at least 4 nodes).
int nn_tpg_for(int K, int qt) {
  const int kcm = qt * NT < 1024 ? qt * NT : 1024;
  const int need = (std::min(K, kcm) + qt - 1) / qt;
  int t = NT / 16;
  while (t < need) t <<= 1;
  return t;
}

// Tiles each idle workgroup scans ahead during the rollout phase (0: none).
// Auto: about as many tiles as one workgroup scans in the time the rollout
// phase takes -- a tile costs ~K (2d + 1) cycles of one CU (d subtractions
// and d FMAs per target and node, 64 nodes over 64 lanes), the rollout ~4
// cycles per instruction of a lane's serial chain per resident rollout wave,
// plus the wait for the slowest chunk.  A double integrator's chain is its
// lane's share of the edge (di_edge: sub-steps and obstacles split over the
// candidate's lanes, plus ~14 per step for the path length).
int spec_tiles_for(const pakr_params& prm, const DevProblem& Q, int n_obs) {
  if (prm.spec_tiles < 0 || Q.G <= Q.G_roll) return 0;
  if (prm.spec_tiles > 0) return prm.spec_tiles;
  const double tile = (double)Q.K * (2.0 * Q.d + 1.0);
  double chain =
      (double)Q.T * (12.0 * Q.d + 4.0 * f_eval_of(Q.system) + 3.0 * Q.npos * n_obs / Q.lanes);
  if (Q.system == PAKR_DI2 || Q.system == PAKR_DI3) {
    long long best = LLONG_MAX;
    for (int ls = 1; ls <= Q.lanes; ls <<= 1)
      best = std::min(best, di_lane_cost(Q.T, Q.lanes, n_obs, ls, DI_CH));
    chain = (double)best + (Q.cost_kind == PAKR_COST_PATH_LENGTH ? 14.0 * Q.T : 0.0);
  }
  const double waves = std::max(1.0, (double)(Q.cpb * Q.lanes) / (4.0 * WAVE));
  const double roll = chain * 4.0 * waves + 4000.0;
  return std::max(1, std::min(64, (int)(roll / tile)));
}

// The first tier of the tree (0: none): the largest of the paper's tier
// sizes 4^k, k = 4..8, whose NN scan one workgroup does in about 20 000
// cycles (K targets x n nodes x (2d + 1) instructions over 64 lanes), and
// only when one rollout pass of the workgroup takes the whole batch.
int tier0_nodes_for(const pakr_params& prm, const DevProblem& Q) {
  if (prm.tier0_nodes < 0 || Q.G <= 1) return 0;
  if (prm.tier0_nodes > 0) return prm.tier0_nodes;
  if (Q.G_roll > 1) return 0;
  int t = 0;
  for (int k = 4, v = 256; k <= 8; ++k, v *= 4)
    if ((double)Q.K * v * (2.0 * Q.d + 1.0) / WAVE <= 20000.0) t = v;
  return t;
}

// Sub-grid tiers of the tree: the first tier_grid[k] workgroups plan while the
// tree has at most tier_nodes[k] nodes.  Auto: grids doubling from G1 = the
// rollout workgroups of one batch (at least 32, a power of two) up to the
// whole grid; tier k takes the trees whose NN scan costs each of its
// workgroups at most S cycles (K x n x (2d + 1) / 64 / grid, S =
// tier_scan_cycles, 10 000 by default: about what the rollout phase of the
// small-batch systems hides), so the grid grows with the tree, and a tier
// that already holds the tree's capacity is the last.  An explicit tier1_nodes gives one
// sub-grid tier of G1 workgroups instead.
void tiers_for(const pakr_params& prm, DevProblem* Q) {
  for (int k = 0; k < MAX_TIERS; ++k) Q->tier_nodes[k] = Q->tier_grid[k] = 0;
  if (prm.tier1_nodes < 0 || Q->G <= 2) return;
  int g = prm.tier1_grid;
  if (g <= 0) {
    g = 32;
    while (g < Q->G_roll) g <<= 1;
  }
  if (g >= Q->G) return;
  if (prm.tier1_nodes > 0) {
    if (prm.tier1_nodes <= Q->tier0_nodes) return;
    Q->tier_nodes[0] = prm.tier1_nodes;
    Q->tier_grid[0] = g;
    return;
  }
  const double S = prm.tier_scan_cycles > 0 ? prm.tier_scan_cycles : 10000.0;
  const double per_node = (double)Q->K * (2.0 * Q->d + 1.0) / WAVE;  // cycles per node and workgroup
  int k = 0, prev = Q->tier0_nodes;
  for (; g < Q->G && k < MAX_TIERS; g <<= 1) {
    const double lim = std::min(S * g / per_node, (double)Q->n_cap);
    int nk = (int)lim;
    if (nk < Q->n_cap) nk -= nk % TILE;
    if (nk <= prev) continue;
    Q->tier_nodes[k] = nk;
    Q->tier_grid[k] = g;
    ++k;
    prev = nk;
    if (nk >= Q->n_cap) break;
  }
}

// The device record of one query planned by G workgroups with L lanes per candidate.
DevProblem make_problem(const pakr_system& sys, const pakr_scene& scene, const pakr_goal& goal,
                        const pakr_params& prm, int G, int lanes, int rt = NT, int qt = 1) {
  DevProblem Q;
  std::memset(&Q, 0, sizeof Q);
  const int P = scene.npos;
  Q.system = sys.id;
  Q.d = sys.d;
  Q.m = sys.m;
  Q.npos = P;
  Q.B = prm.B;
  Q.A = prm.A;
  Q.K = prm.B / prm.A;
  Q.T = prm.T;
  Q.n_cap = prm.n_cap;
  Q.cost_kind = prm.cost_kind;
  Q.h_kind = prm.heuristic_kind;
  Q.max_iters_per_round = prm.max_iters_per_round;
  Q.n_box = scene.n_box;
  Q.n_sph = scene.n_sphere;
  Q.G = G;
  Q.lanes = lanes;
  Q.cpb = rt / lanes;
  Q.nn_tpg = nn_tpg_for(Q.K, qt);
  Q.G_roll = (prm.B + Q.cpb - 1) / Q.cpb;
  Q.spec_tiles = spec_tiles_for(prm, Q, scene.n_box + scene.n_sphere);
  Q.tier0_nodes = tier0_nodes_for(prm, Q);
  tiers_for(prm, &Q);
  Q.max_path_edges = prm.max_path_edges > 0 ? prm.max_path_edges : DEFAULT_PATH_EDGES;
  Q.obs_floats = obs_floats_of(P, scene.n_box, scene.n_sphere);
  Q.key0 = (uint32_t)(prm.seed & 0xffffffffull);
  Q.key1 = prm.query_id;
  Q.dt = prm.dt;
  Q.h_speed = prm.h_speed;
  Q.c0 = (float)prm.cost_bound;
  Q.vnorm_max = sys.vnorm_max;
  Q.goal_r = goal.radius;
  Q.goal_r2 = goal.radius * goal.radius;
  {
    volatile float tf = (float)prm.T;
    volatile float ed = tf * prm.dt;  // one float32 rounding
    Q.edge_duration = ed;
  }
  for (int i = 0; i < 8; ++i) Q.dyn[i] = sys.dyn[i];
  if (sys.id == PAKR_QUAD) {
    // reciprocal inertias (the kernels multiply instead of dividing)
    for (int c = 0; c < 3; ++c) Q.dyn[5 + c] = 1.0f / sys.dyn[2 + c];
  }
  for (int i = 0; i < PAKR_MAX_D; ++i) {
    Q.sample_lo[i] = sys.sample_lo[i];
    Q.sample_hi[i] = sys.sample_hi[i];
    Q.lim_lo[i] = sys.lim_lo[i];
    Q.lim_hi[i] = sys.lim_hi[i];
  }
  for (int i = 0; i < PAKR_MAX_M; ++i) {
    Q.u_lo[i] = sys.u_lo[i];
    Q.u_hi[i] = sys.u_hi[i];
  }
  for (int c = 0; c < 3; ++c) {
    Q.ws_lo[c] = c < P ? scene.ws_lo[c] : 0.0f;
    Q.ws_hi[c] = c < P ? scene.ws_hi[c] : 0.0f;
    Q.goal_c[c] = c < P ? goal.center[c] : 0.0f;
  }
  return Q;
}

// Obstacles as the kernels read them: boxes (c[P], h[P]), then spheres (c[P], r^2).
std::vector<float> pack_obstacles(const pakr_scene& sc) {
  const int P = sc.npos;
  std::vector<float> o;
  o.reserve((size_t)std::max(obs_floats_of(P, sc.n_box, sc.n_sphere), 1));
  for (int b = 0; b < sc.n_box; ++b) {
    for (int c = 0; c < P; ++c) o.push_back(sc.box_c[b * P + c]);
    for (int c = 0; c < P; ++c) o.push_back(sc.box_h[b * P + c]);
  }
  for (int q = 0; q < sc.n_sphere; ++q) {
    for (int c = 0; c < P; ++c) o.push_back(sc.sph_c[q * P + c]);
    o.push_back(sc.sph_r[q] * sc.sph_r[q]);
  }
  return o;
}

// Kernel arguments of a query whose buffers start at `base` with layout L.
KArgs make_args(const DevProblem& Q, char* base, const Layout& L) {
  KArgs a;
  std::memset(&a, 0, sizeof a);
  a.P = Q;
  a.hdr = reinterpret_cast<DevHeader*>(base + L.hdr);
  a.bar_flags = reinterpret_cast<uint32_t*>(base + L.bar);
  a.sols = reinterpret_cast<DevSolution*>(base + L.sols);
  a.path_states = reinterpret_cast<float*>(base + L.pstates);
  a.path_actions = reinterpret_cast<float*>(base + L.pactions);
  a.states = reinterpret_cast<float*>(base + L.states);
  a.actions = reinterpret_cast<float*>(base + L.actions);
  a.parents = reinterpret_cast<int*>(base + L.parents);
  a.costs = reinterpret_cast<float*>(base + L.costs);
  a.obs = reinterpret_cast<const float*>(base + L.obs);
  a.nn_keys = reinterpret_cast<unsigned long long*>(base + L.nn_keys);
  a.stg = reinterpret_cast<float*>(base + L.stg);
  a.counts = reinterpret_cast<int*>(base + L.counts);
  a.goalmin = reinterpret_cast<unsigned long long*>(base + L.goalmin);
  return a;
}

// How long a workgroup waits at a grid barrier before the call fails with
// PAKR_E_DEVICE (pakr_set_barrier_timeout; read at every launch).
constexpr double DEFAULT_BARRIER_TIMEOUT_MS = 2000.0;
std::atomic<double> g_barrier_timeout_ms{DEFAULT_BARRIER_TIMEOUT_MS};

void set_limits(KArgs& a, long long max_iters, long long max_rounds, double budget_ms,
                double ticks_per_ms) {
  a.max_iters = max_iters;
  a.max_rounds = max_rounds;
  a.budget_ticks = budget_ms > 0 ? (long long)(budget_ms * ticks_per_ms) : 0;
  const double guard_ms = (budget_ms > 0 ? budget_ms : 0.0) + 60000.0;
  a.guard_ticks = (long long)(guard_ms * ticks_per_ms);
  a.barrier_timeout_ticks =
      std::max(1ll, (long long)(g_barrier_timeout_ms.load() * ticks_per_ms));
}

// Int32 words of one trace record of a query (layout in pakr.h).
size_t trace_words_of(const DevProblem& P) {
  const size_t K = P.K, B = P.B, d = P.d, m = P.m;
  return TRACE_HDR_WORDS + K * d + K + B * m + B * d + 3 * B;
}

// Copy the obstacles and enqueue the root write of one query.
hipError_t upload_query(const KArgs& a, const std::vector<float>& obs, const float* x_init,
                        int n_flags, hipStream_t stream) {
  hipError_t e = hipSuccess;
  if (!obs.empty()) {
    e = hipMemcpyAsync(const_cast<float*>(a.obs), obs.data(), sizeof(float) * obs.size(),
                       hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);  // obs is pageable host memory
    if (e != hipSuccess) return e;
  }
  float x[12] = {0};
  for (int c = 0; c < a.P.d; ++c) x[c] = x_init[c];
  hipLaunchKernelGGL(k_init, dim3(1), dim3(NT), 0, stream, a.hdr, a.bar_flags, n_flags, a.states,
                     a.actions, a.parents, a.costs, a.P.n_cap, a.P.d, a.P.m, x[0], x[1], x[2], x[3],
                     x[4], x[5], x[6], x[7], x[8], x[9], x[10], x[11], a.P.c0);
  return hipGetLastError();
}

struct DeviceInfo {
  int device = 0, n_cu = 0, coop = 0, lds_cu = 0, lds_max = 0;
  double ticks_per_ms = 100000.0;
};

hipError_t device_info(DeviceInfo* di) {
  int wclk = 0;
  hipError_t e = hipGetDevice(&di->device);
  if (e == hipSuccess)
    e = hipDeviceGetAttribute(&di->n_cu, hipDeviceAttributeMultiprocessorCount, di->device);
  if (e == hipSuccess)
    e = hipDeviceGetAttribute(&di->coop, hipDeviceAttributeCooperativeLaunch, di->device);
  if (e == hipSuccess)
    e = hipDeviceGetAttribute(&wclk, hipDeviceAttributeWallClockRate, di->device);
  if (e == hipSuccess)
    e = hipDeviceGetAttribute(&di->lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor,
                              di->device);
  if (e == hipSuccess)
    e = hipDeviceGetAttribute(&di->lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, di->device);
  if (wclk > 0) di->ticks_per_ms = (double)wclk;
  return e;
}

void fill_stats(const DevHeader& h, double tpm, int grid, pakr_stats* out) {
  std::memset(out, 0, sizeof *out);
  out->n_nodes = h.n;
  out->round = h.round;
  out->iter = h.iter;
  out->status = h.status;
  out->n_solutions = h.n_solutions;
  out->grid = grid;
  out->total_iters = (long long)h.total_iters;
  out->expansions = (long long)h.expansions;
  out->insertions = (long long)h.insertions;
  out->nn_pairs = (long long)h.nn_pairs;
  out->c_best = std::isinf(h.c_best) ? INFINITY : (double)h.c_best;
  out->call_ms = (double)(h.t_end - h.t_start) / tpm;
  out->t_first_ms = h.t_first >= 0 ? (double)h.t_first / tpm : -1.0;
  out->t_last_ms = h.t_last >= 0 ? (double)h.t_last / tpm : -1.0;
  out->call_iters = h.call_iters;
  out->call_rounds = h.call_rounds;
  out->call_solutions = h.call_solutions;
  for (int i = 0; i < 6; ++i) out->step_ms[i] = (double)h.ticks[i] / tpm;
  out->nn_ms = out->step_ms[0] + out->step_ms[1];
  out->rollout_ms = out->step_ms[2] + out->step_ms[3] + out->step_ms[4];
  out->insert_ms = out->step_ms[5];
  out->clock_start_ms = (double)h.t_start / tpm;
  out->clock_end_ms = (double)h.t_end / tpm;
  out->near_ties_prune = (long long)h.near_prune;
  out->near_ties_goal = (long long)h.near_goal;
}

// Shared read-back helpers (each syncs `stream`).
hipError_t read_header(const KArgs& a, hipStream_t stream, DevHeader* h) {
  hipError_t e = hipMemcpyAsync(h, a.hdr, sizeof(DevHeader), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  return e;
}

hipError_t read_solutions(const KArgs& a, double tpm, int n, pakr_solution* out) {
  if (n <= 0) return hipSuccess;
  std::vector<DevSolution> tmp((size_t)n);
  hipError_t e = hipMemcpy(tmp.data(), a.sols, sizeof(DevSolution) * n, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return e;
  for (int i = 0; i < n; ++i) {
    out[i].round = tmp[i].round;
    out[i].iter = tmp[i].iter;
    out[i].node = tmp[i].node;
    out[i].n_nodes = tmp[i].n_nodes;
    out[i].total_iter = tmp[i].total_iter;
    out[i].cost = (double)tmp[i].cost;
    out[i].t_ms = (double)tmp[i].t / tpm;
  }
  return hipSuccess;
}

// The stored best path is goal first; return it root first.
hipError_t read_path(const KArgs& a, int ne, float* states, float* actions) {
  const int d = a.P.d, m = a.P.m;
  std::vector<float> rs((size_t)(ne + 1) * d), ra((size_t)ne * m + 1);
  hipError_t e = hipMemcpy(rs.data(), a.path_states, sizeof(float) * rs.size(),
                           hipMemcpyDeviceToHost);
  if (e == hipSuccess && ne > 0)
    e = hipMemcpy(ra.data(), a.path_actions, sizeof(float) * (size_t)ne * m,
                  hipMemcpyDeviceToHost);
  if (e != hipSuccess) return e;
  for (int k = 0; k <= ne; ++k)
    std::memcpy(states + (size_t)k * d, rs.data() + (size_t)(ne - k) * d, sizeof(float) * d);
  for (int k = 0; k < ne; ++k)
    std::memcpy(actions + (size_t)k * m, ra.data() + (size_t)(ne - 1 - k) * m, sizeof(float) * m);
  return hipSuccess;
}

// The first n nodes of a query's tree, node-major (any output may be null).
hipError_t read_tree(const KArgs& a, int n, float* states, float* actions, int* parents,
                     float* costs) {
  const int d = a.P.d, m = a.P.m;
  const size_t N = (size_t)a.P.n_cap;
  hipError_t e = hipSuccess;
  if (n > 0 && (states || actions)) {
    std::vector<float> tmp((size_t)n);
    for (int c = 0; c < d && states && e == hipSuccess; ++c) {
      e = hipMemcpy(tmp.data(), a.states + (size_t)c * N, sizeof(float) * n,
                    hipMemcpyDeviceToHost);
      for (int i = 0; i < n; ++i) states[(size_t)i * d + c] = tmp[i];
    }
    for (int c = 0; c < m && actions && e == hipSuccess; ++c) {
      e = hipMemcpy(tmp.data(), a.actions + (size_t)c * N, sizeof(float) * n,
                    hipMemcpyDeviceToHost);
      for (int i = 0; i < n; ++i) actions[(size_t)i * m + c] = tmp[i];
    }
  }
  if (e == hipSuccess && n > 0 && parents)
    e = hipMemcpy(parents, a.parents, sizeof(int) * n, hipMemcpyDeviceToHost);
  if (e == hipSuccess && n > 0 && costs)
    e = hipMemcpy(costs, a.costs, sizeof(float) * n, hipMemcpyDeviceToHost);
  return e;
}

}  // namespace

struct pakr_plan {
  KArgs args;          // buffers and problem record; limits set per call
  int G = 0, qt = 1;
  int rt = NT;         // rollout threads per workgroup
  hipStream_t stream = nullptr;
  double ticks_per_ms = 100000.0;
  void* ws = nullptr;
  bool own_ws = false;
  Layout L{};
  const void* kfn = nullptr;
  size_t shmem = 0;
  bool broken = false;
  std::string err;
};

struct pakr_batch {
  int nq = 0, G = 0;
  hipStream_t stream = nullptr;
  double ticks_per_ms = 100000.0;
  void* ws = nullptr;
  bool own_ws = false;
  std::vector<KArgs> args;
  std::vector<int> team;   // workgroups per query
  KArgs* d_args = nullptr;        // argument table of direct launches (replan, expand)
  KArgs* d_args_graph = nullptr;  // the captured graph's own table (its limits)
  int* d_tickets = nullptr;
  int n_tickets = 0;
  int* d_queue = nullptr;
  size_t shmem = 0;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  bool broken = false;
  std::string err;
};

namespace {

int fail(pakr_plan* pl, int code, const std::string& msg) {
  if (pl) pl->err = msg;
  else set_init_error(msg);
  return code;
}

int hip_fail(pakr_plan* pl, hipError_t e, const char* what) {
  return fail(pl, PAKR_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

int bfail(pakr_batch* bt, int code, const std::string& msg) {
  if (bt) bt->err = msg;
  else set_init_error(msg);
  return code;
}

int bhip_fail(pakr_batch* bt, hipError_t e, const char* what) {
  return bfail(bt, PAKR_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace

extern "C" {

size_t pakr_workspace_size(const pakr_system* sys, const pakr_params* params,
                           const pakr_scene* scene) {
  if (!sys || !params || !scene) return 0;
  const int d = sys_d(sys->id), m = sys_m(sys->id);
  if (d < 0 || params->A < 1 || params->B < 1 || params->B % params->A != 0 ||
      params->n_cap < 1 || params->grid < 0)
    return 0;
  const int G = params->grid > 0 ? params->grid : AUTO_GRID_MAX;
  const int nb = std::max(scene->n_box, 0), ns = std::max(scene->n_sphere, 0);
  const int of = obs_floats_of(sys_npos(sys->id), nb, ns);
  size_t worst = 0;  // the lane and rollout-thread choices depend on the device:
  for (int lanes = 1; lanes <= 16; lanes <<= 1)  // size for the largest layout
    for (int rt = NT / 2; rt <= NT; rt *= 2)
      worst = std::max(worst, make_layout(d, m, *params, G, of, lanes, rt).total);
  return worst;
}

int pakr_plan_init(const pakr_system* sys, const pakr_scene* scene, const float* x_init,
                   const pakr_goal* goal, const pakr_params* params, void* d_workspace,
                   size_t ws_bytes, void* stream, pakr_plan** out) {
  if (!out) return fail(nullptr, PAKR_E_INVALID_ARG, "out is null");
  *out = nullptr;
  int code = PAKR_OK;
  const std::string msg = validate(sys, scene, x_init, goal, params, &code);
  if (code != PAKR_OK) return fail(nullptr, code, msg);

  DeviceInfo di;
  hipError_t e = device_info(&di);
  if (e != hipSuccess) return hip_fail(nullptr, e, "device query");
  if (!di.coop) return fail(nullptr, PAKR_E_HIP, "device does not support cooperative launches");

  pakr_plan* pl = new (std::nothrow) pakr_plan();
  if (!pl) return fail(nullptr, PAKR_E_INVALID_ARG, "out of host memory");
  pl->stream = static_cast<hipStream_t>(stream);
  pl->ticks_per_ms = di.ticks_per_ms;
  const int K = params->B / params->A;
  pl->qt = qt_for(K, sys->d);
  pl->kfn = kernel_for(sys->id, pl->qt);
  const int of = obs_floats_of(scene->npos, scene->n_box, scene->n_sphere);
  const size_t obs_bytes = sizeof(float) * (size_t)std::max(of, 1);
  pl->shmem = obs_bytes;
  int G = 0;
  if (params->grid > 0) {
    G = params->grid;
  } else {
    // k workgroups on every CU: reserve enough LDS that a CU cannot hold k+1,
    // so the co-resident grid of k * CUs is spread evenly
    const int k = params->workgroups_per_cu > 0 ? params->workgroups_per_cu : 1;
    hipFuncAttributes fa;
    if (hipFuncGetAttributes(&fa, pl->kfn) != hipSuccess) {
      delete pl;
      return fail(nullptr, PAKR_E_HIP, "kernel attribute query failed");
    }
    const size_t want = (size_t)di.lds_cu / (size_t)(k + 1) + 1024;  // > LDS/(k+1)
    const size_t dyn = want > fa.sharedSizeBytes ? want - fa.sharedSizeBytes : 0;
    if (dyn + fa.sharedSizeBytes <= (size_t)di.lds_max && dyn > obs_bytes) pl->shmem = dyn;
    G = k * di.n_cu;
  }
  int per_cu = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, pl->kfn, NT, pl->shmem);
  if (e != hipSuccess || per_cu < 1) {
    int rc = e != hipSuccess ? hip_fail(nullptr, e, "occupancy query")
                             : fail(nullptr, PAKR_E_HIP, "kernel does not fit on a CU");
    delete pl;
    return rc;
  }
  const int max_coresident = per_cu * di.n_cu;
  if (params->grid <= 0) G = std::min(std::min(G, max_coresident), AUTO_GRID_MAX);
  const int lanes = lanes_for(*params, scene->n_box + scene->n_sphere,
                              params->grid > 0 ? G : max_coresident);
  const int cpb = NT / lanes;
  const int GR = (params->B + cpb - 1) / cpb;
  if (G < GR) G = params->grid > 0 ? -1 : GR;
  if (G < 1 || G > max_coresident || G > AUTO_GRID_MAX) {
    char buf[160];
    snprintf(buf, sizeof buf, "grid %d invalid: need >= %d rollout workgroups and <= %d co-resident",
             params->grid > 0 ? params->grid : G, GR, std::min(max_coresident, AUTO_GRID_MAX));
    delete pl;
    return fail(nullptr, PAKR_E_INVALID_ARG, buf);
  }
  pl->G = G;
  pl->rt = rollout_threads(*sys, *params, scene->n_box + scene->n_sphere, lanes, G);
  pl->L = make_layout(sys->d, sys->m, *params, G, of, lanes, pl->rt);
  const size_t need = pl->L.total;
  if (d_workspace) {
    if (ws_bytes < need) {
      delete pl;
      return fail(nullptr, PAKR_E_WORKSPACE_TOO_SMALL, "workspace smaller than required");
    }
    if ((reinterpret_cast<uintptr_t>(d_workspace) & 255) != 0) {
      delete pl;
      return fail(nullptr, PAKR_E_INVALID_ARG, "workspace must be 256-byte aligned");
    }
    pl->ws = d_workspace;
  } else {
    e = hipMalloc(&pl->ws, need);
    if (e != hipSuccess) {
      int rc = hip_fail(nullptr, e, "hipMalloc workspace");
      delete pl;
      return rc;
    }
    pl->own_ws = true;
  }
  const DevProblem Q = make_problem(*sys, *scene, *goal, *params, G, lanes, pl->rt, pl->qt);
  pl->args = make_args(Q, static_cast<char*>(pl->ws), pl->L);
  e = upload_query(pl->args, pack_obstacles(*scene), x_init, G, pl->stream);
  if (e != hipSuccess) {
    int rc = hip_fail(nullptr, e, "upload query");
    pakr_plan_destroy(pl);
    return rc;
  }
  *out = pl;
  return PAKR_OK;
}

void pakr_plan_destroy(pakr_plan* pl) {
  if (!pl) return;
  if (pl->ws) (void)hipStreamSynchronize(pl->stream);
  if (pl->own_ws && pl->ws) (void)hipFree(pl->ws);
  delete pl;
}

size_t pakr_trace_bytes(const pakr_plan* pl, int n_iters) {
  if (!pl || n_iters < 0) return 0;
  return trace_words_of(pl->args.P) * 4 * (size_t)n_iters;
}

namespace {

int launch(pakr_plan* pl, long long max_iters, long long max_rounds, double budget_ms,
           int* trace, long long trace_iters) {
  if (pl->broken) return fail(pl, PAKR_E_DEVICE, "plan is unusable after a device error");
  KArgs a = pl->args;
  set_limits(a, max_iters, max_rounds, budget_ms, pl->ticks_per_ms);
  a.trace = trace;
  a.trace_words = (long long)(pakr_trace_bytes(pl, 1) / 4);
  a.trace_iters = trace ? trace_iters : 0;
  void* args[] = {&a};
  hipError_t e = hipLaunchCooperativeKernel(pl->kfn, dim3(pl->G), dim3(NT), args,
                                            (unsigned)pl->shmem, pl->stream);
  if (e != hipSuccess) return hip_fail(pl, e, "cooperative launch");
  return PAKR_OK;
}

int sync_header(pakr_plan* pl, DevHeader* h) {
  hipError_t e = read_header(pl->args, pl->stream, h);
  if (e != hipSuccess) return hip_fail(pl, e, "read header");
  if (h->err != 0) {
    pl->broken = true;
    return fail(pl, PAKR_E_DEVICE, "grid barrier timed out on the device");
  }
  return PAKR_OK;
}

}  // namespace

int pakr_expand(pakr_plan* pl, int n_iters, void* d_trace, size_t trace_bytes) {
  if (!pl) return PAKR_E_INVALID_ARG;
  if (n_iters < 0) return fail(pl, PAKR_E_INVALID_ARG, "n_iters must be >= 0");
  if (n_iters == 0) return PAKR_OK;
  if (d_trace && trace_bytes < pakr_trace_bytes(pl, n_iters))
    return fail(pl, PAKR_E_BUFFER_TOO_SMALL, "trace buffer too small");
  return launch(pl, n_iters, 0, 0.0, static_cast<int*>(d_trace), n_iters);
}

int pakr_replan(pakr_plan* pl, double budget_ms, int max_rounds, long long max_iters) {
  if (!pl) return PAKR_E_INVALID_ARG;
  if (std::isnan(budget_ms)) return fail(pl, PAKR_E_INVALID_ARG, "budget is NaN");
  if (!(budget_ms > 0) && max_rounds <= 0 && max_iters <= 0)
    return fail(pl, PAKR_E_INVALID_ARG, "set a budget, a round limit or an iteration limit");
  return launch(pl, max_iters, max_rounds, budget_ms, nullptr, 0);
}

int pakr_status(pakr_plan* pl, pakr_stats* out) {
  if (!pl || !out) return PAKR_E_INVALID_ARG;
  DevHeader h;
  int rc = sync_header(pl, &h);
  if (rc != PAKR_OK) return rc;
  fill_stats(h, pl->ticks_per_ms, pl->G, out);
  const DevProblem& P = pl->args.P;
  int k = 0;
  if (P.tier0_nodes > 0) {
    out->tier_nodes[k] = P.tier0_nodes;
    out->tier_grid[k++] = 1;
  }
  for (int i = 0; i < MAX_TIERS && P.tier_nodes[i] > 0; ++i) {
    out->tier_nodes[k] = P.tier_nodes[i];
    out->tier_grid[k++] = P.tier_grid[i];
  }
  return PAKR_OK;
}

int pakr_solutions(pakr_plan* pl, pakr_solution* out, int cap, int* n_total) {
  if (!pl || !n_total || cap < 0 || (cap > 0 && !out)) return PAKR_E_INVALID_ARG;
  DevHeader h;
  int rc = sync_header(pl, &h);
  if (rc != PAKR_OK) return rc;
  *n_total = h.n_solutions;
  const int n = std::min(std::min(cap, h.n_solutions), MAX_SOLUTIONS);
  hipError_t e = read_solutions(pl->args, pl->ticks_per_ms, n, out);
  if (e != hipSuccess) return hip_fail(pl, e, "read solutions");
  return PAKR_OK;
}

int pakr_extract_path(pakr_plan* pl, float* states, float* actions, int cap_edges, int* n_edges,
                      double* cost) {
  if (!pl || !n_edges) return PAKR_E_INVALID_ARG;
  DevHeader h;
  int rc = sync_header(pl, &h);
  if (rc != PAKR_OK) return rc;
  if (h.best_edges < 0) {
    *n_edges = 0;
    return fail(pl, PAKR_E_NO_SOLUTION, "no solution yet");
  }
  *n_edges = h.best_edges;
  if (cost) *cost = (double)h.best_cost;
  if (h.path_truncated) return fail(pl, PAKR_E_BUFFER_TOO_SMALL, "path longer than max_path_edges");
  if (h.best_edges > cap_edges) return fail(pl, PAKR_E_BUFFER_TOO_SMALL, "cap_edges too small");
  if (!states || !actions) return fail(pl, PAKR_E_INVALID_ARG, "null output arrays");
  hipError_t e = read_path(pl->args, h.best_edges, states, actions);
  if (e != hipSuccess) return hip_fail(pl, e, "read path");
  return PAKR_OK;
}

int pakr_copy_tree(pakr_plan* pl, float* states, float* actions, int* parents, float* costs,
                   int n_max, int* n_out) {
  if (!pl || !n_out || n_max < 0) return PAKR_E_INVALID_ARG;
  DevHeader h;
  int rc = sync_header(pl, &h);
  if (rc != PAKR_OK) return rc;
  *n_out = h.n;
  hipError_t e = read_tree(pl->args, std::min(h.n, n_max), states, actions, parents, costs);
  if (e != hipSuccess) return hip_fail(pl, e, "read tree");
  return PAKR_OK;
}

const char* pakr_last_error(const pakr_plan* pl) {
  return pl ? pl->err.c_str() : g_init_error;
}

int pakr_set_barrier_timeout(double ms) {
  if (std::isnan(ms)) return PAKR_E_INVALID_ARG;
  g_barrier_timeout_ms.store(ms > 0 ? ms : DEFAULT_BARRIER_TIMEOUT_MS);
  return PAKR_OK;
}

const char* pakr_error_string(int code) {
  switch (code) {
    case PAKR_OK: return "PAKR_OK";
    case PAKR_E_INVALID_ARG: return "PAKR_E_INVALID_ARG";
    case PAKR_E_START_INVALID: return "PAKR_E_START_INVALID";
    case PAKR_E_GOAL_INVALID: return "PAKR_E_GOAL_INVALID";
    case PAKR_E_WORKSPACE_TOO_SMALL: return "PAKR_E_WORKSPACE_TOO_SMALL";
    case PAKR_E_HIP: return "PAKR_E_HIP";
    case PAKR_E_NO_SOLUTION: return "PAKR_E_NO_SOLUTION";
    case PAKR_E_BUFFER_TOO_SMALL: return "PAKR_E_BUFFER_TOO_SMALL";
    case PAKR_E_DEVICE: return "PAKR_E_DEVICE";
  }
  return "unknown";
}

// ---------------------------------------------------------------------------
// Batched planning
// ---------------------------------------------------------------------------

namespace {

// Relative cost of one iteration of a query on one workgroup, for scheduling
// only: a fixed part (barriers, scans, bookkeeping), the rollout of the B
// candidates (an evaluation of f counted with its hardware sine and cosine
// at ~4 operations each) and the NN scan of K targets over a tree taken as 2 % of
// what one round could insert.  Calibrated against measured iteration times
// (quadrotor ~2.6 ms, 3D double integrator ~0.15 ms on one workgroup).
double query_work(const DevProblem& Q) {
  const double f_eval = f_eval_of(Q.system);
  const double roll =
      (double)Q.B * Q.T * (12.0 * Q.d + 4.0 * f_eval + 3.0 * Q.npos * (Q.n_box + Q.n_sph));
  const double tree = std::min((double)Q.n_cap, 0.02 * Q.B * Q.max_iters_per_round);
  return 1.7e7 + roll + (double)Q.K * tree * 3.0 * Q.d;
}

int batch_lanes(const pakr_params& p) { return p.lanes_per_candidate > 0 ? p.lanes_per_candidate : 1; }

// Workgroups that share one query of a batch ("team"): at most TEAM_MAX.
constexpr int TEAM_MAX = 16;

// Batch workspace: queue word, the argument table of direct launches, the
// captured graph's argument table, the ticket table, then each query's
// regions, sized for a team of up to TEAM_MAX workgroups.
size_t batch_args_offset(int n, int which) {
  return 256 + (size_t)which * align_up(sizeof(KArgs) * (size_t)n);
}
size_t batch_tickets_offset(int n) { return batch_args_offset(n, 2); }

size_t batch_layout(int n, const pakr_system* sys, const pakr_scene* sc, const pakr_params* prm,
                    std::vector<size_t>* bases, std::vector<Layout>* layouts) {
  size_t off = batch_tickets_offset(n) + align_up(sizeof(int) * (size_t)n * TEAM_MAX);
  for (int q = 0; q < n; ++q) {
    const int of = obs_floats_of(sc[q].npos, sc[q].n_box, sc[q].n_sphere);
    const Layout L = make_layout(sys[q].d, sys[q].m, prm[q], TEAM_MAX, of, batch_lanes(prm[q]));
    if (bases) bases->push_back(off);
    if (layouts) layouts->push_back(L);
    off = align_up(off + L.total);
  }
  return off;
}

}  // namespace

size_t pakr_batch_workspace_size(int n, const pakr_system* sys, const pakr_scene* scenes,
                                 const pakr_params* params) {
  if (n < 1 || !sys || !scenes || !params) return 0;
  for (int q = 0; q < n; ++q) {
    if (sys_d(sys[q].id) < 0 || sys[q].d != sys_d(sys[q].id) || sys[q].m != sys_m(sys[q].id) ||
        params[q].A < 1 || params[q].B < 1 || params[q].B % params[q].A != 0 ||
        params[q].n_cap < 1 || scenes[q].n_box < 0 || scenes[q].n_sphere < 0)
      return 0;
  }
  return batch_layout(n, sys, scenes, params, nullptr, nullptr);
}

int pakr_batch_init(int n, const pakr_system* sys, const pakr_scene* scenes,
                    const float* const* x_inits, const pakr_goal* goals,
                    const pakr_params* params, void* d_workspace, size_t ws_bytes, void* stream,
                    pakr_batch** out) {
  if (!out) return bfail(nullptr, PAKR_E_INVALID_ARG, "out is null");
  *out = nullptr;
  if (n < 1 || !sys || !scenes || !x_inits || !goals || !params)
    return bfail(nullptr, PAKR_E_INVALID_ARG, "null argument or n < 1");
  int max_obs = 1;
  for (int q = 0; q < n; ++q) {
    int code = PAKR_OK;
    const std::string msg = validate(&sys[q], &scenes[q], x_inits[q], &goals[q], &params[q], &code);
    if (code != PAKR_OK) return bfail(nullptr, code, "query " + std::to_string(q) + ": " + msg);
    if (params[q].grid > TEAM_MAX)
      return bfail(nullptr, PAKR_E_INVALID_ARG,
                   "query " + std::to_string(q) + ": team size (grid) must be <= 16 in a batch");
    const int L = batch_lanes(params[q]);
    if ((params[q].B + NT / L - 1) / (NT / L) > MAX_GR)
      return bfail(nullptr, PAKR_E_INVALID_ARG,
                   "query " + std::to_string(q) + ": too many rollout chunks for the lane count");
    max_obs = std::max(max_obs, obs_floats_of(scenes[q].npos, scenes[q].n_box, scenes[q].n_sphere));
  }
  DeviceInfo di;
  hipError_t e = device_info(&di);
  if (e != hipSuccess) return bhip_fail(nullptr, e, "device query");

  pakr_batch* bt = new (std::nothrow) pakr_batch();
  if (!bt) return bfail(nullptr, PAKR_E_INVALID_ARG, "out of host memory");
  bt->nq = n;
  bt->stream = static_cast<hipStream_t>(stream);
  bt->ticks_per_ms = di.ticks_per_ms;
  bt->shmem = sizeof(float) * (size_t)max_obs;
  int per_cu = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(&k_batch),
                                                   NT, bt->shmem);
  if (e != hipSuccess || per_cu < 1) {
    int rc = e != hipSuccess ? bhip_fail(nullptr, e, "occupancy query")
                             : bfail(nullptr, PAKR_E_HIP, "batch kernel does not fit on a CU");
    delete bt;
    return rc;
  }
  const int g_full = std::max(1, per_cu * di.n_cu);  // co-resident workgroups

  std::vector<size_t> bases;
  std::vector<Layout> layouts;
  const size_t need = batch_layout(n, sys, scenes, params, &bases, &layouts);
  if (d_workspace) {
    if (ws_bytes < need || (reinterpret_cast<uintptr_t>(d_workspace) & 255) != 0) {
      delete bt;
      return bfail(nullptr, ws_bytes < need ? PAKR_E_WORKSPACE_TOO_SMALL : PAKR_E_INVALID_ARG,
                   ws_bytes < need ? "workspace smaller than required"
                                   : "workspace must be 256-byte aligned");
    }
    bt->ws = d_workspace;
  } else {
    e = hipMalloc(&bt->ws, need);
    if (e != hipSuccess) {
      int rc = bhip_fail(nullptr, e, "hipMalloc workspace");
      delete bt;
      return rc;
    }
    bt->own_ws = true;
  }
  char* base = static_cast<char*>(bt->ws);
  bt->d_queue = reinterpret_cast<int*>(base);
  bt->d_args = reinterpret_cast<KArgs*>(base + batch_args_offset(n, 0));
  bt->d_args_graph = reinterpret_cast<KArgs*>(base + batch_args_offset(n, 1));
  bt->d_tickets = reinterpret_cast<int*>(base + batch_tickets_offset(n));
  // Team sizes: params.grid if set, else the query's share of the estimated
  // work of the whole batch in workgroups (at least 1, at most TEAM_MAX).
  std::vector<double> work((size_t)n);
  double total = 0.0;
  for (int q = 0; q < n; ++q) {
    const DevProblem Q = make_problem(sys[q], scenes[q], goals[q], params[q], 1, batch_lanes(params[q]));
    work[q] = query_work(Q);
    total += work[q];
  }
  bt->team.resize((size_t)n);
  for (int q = 0; q < n; ++q) {
    int g = params[q].grid;
    if (g <= 0) g = (int)std::lround(work[q] * g_full / total);
    bt->team[q] = std::max(1, std::min(std::min(g, TEAM_MAX), g_full));
  }
  int n_team_wg = 0;
  for (int q = 0; q < n; ++q) n_team_wg += bt->team[q];
  bt->G = std::min(n_team_wg, g_full);
  bt->args.resize((size_t)n);
  for (int q = 0; q < n; ++q) {
    const DevProblem Q = make_problem(sys[q], scenes[q], goals[q], params[q], bt->team[q],
                                      batch_lanes(params[q]));
    bt->args[q] = make_args(Q, base + bases[q], layouts[q]);
    e = upload_query(bt->args[q], pack_obstacles(scenes[q]), x_inits[q], TEAM_MAX, bt->stream);
    if (e != hipSuccess) {
      int rc = bhip_fail(nullptr, e, "upload query");
      pakr_batch_destroy(bt);
      return rc;
    }
  }
  // Tickets in longest-processing-time-first order: bigger teams, then more
  // estimated work, come first, so the long queries start at the launch.  A
  // team's tickets are consecutive; ticket = query << 5 | member.
  std::vector<int> order((size_t)n);
  for (int q = 0; q < n; ++q) order[q] = q;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return bt->team[a] != bt->team[b] ? bt->team[a] > bt->team[b] : work[a] > work[b];
  });
  std::vector<int> tickets;
  for (int q : order)
    for (int m = 0; m < bt->team[q]; ++m) tickets.push_back(q << 5 | m);
  bt->n_tickets = (int)tickets.size();
  e = hipMemcpyAsync(bt->d_tickets, tickets.data(), sizeof(int) * tickets.size(),
                     hipMemcpyHostToDevice, bt->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(bt->stream);  // pageable source
  if (e != hipSuccess) {
    int rc = bhip_fail(nullptr, e, "upload tickets");
    pakr_batch_destroy(bt);
    return rc;
  }
  *out = bt;
  return PAKR_OK;
}

}  // extern "C"

namespace {

// Upload `table` (one record per query) to `d_table`; syncs the batch stream.
int batch_upload(pakr_batch* bt, const std::vector<KArgs>& table, KArgs* d_table) {
  hipError_t e = hipMemcpyAsync(d_table, table.data(), sizeof(KArgs) * table.size(),
                                hipMemcpyHostToDevice, bt->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(bt->stream);  // pageable source
  if (e != hipSuccess) return bhip_fail(bt, e, "upload batch arguments");
  return PAKR_OK;
}

// Enqueue the queue reset and the persistent launch reading `d_table` on `s`.
int batch_enqueue(pakr_batch* bt, const KArgs* d_table, hipStream_t s) {
  hipLaunchKernelGGL(k_reset_queue, dim3(1), dim3(64), 0, s, bt->d_queue);
  hipLaunchKernelGGL(k_batch, dim3(bt->G), dim3(NT), bt->shmem, s, d_table,
                     static_cast<const int*>(bt->d_tickets), bt->n_tickets, bt->d_queue);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return bhip_fail(bt, e, "batch launch");
  return PAKR_OK;
}

int batch_limits_ok(pakr_batch* bt, double budget_ms, int max_rounds, long long max_iters) {
  if (std::isnan(budget_ms)) return bfail(bt, PAKR_E_INVALID_ARG, "budget is NaN");
  if (!(budget_ms > 0) && max_rounds <= 0 && max_iters <= 0)
    return bfail(bt, PAKR_E_INVALID_ARG, "set a budget, a round limit or an iteration limit");
  return PAKR_OK;
}

int batch_usable(pakr_batch* bt) {
  if (bt->broken) return bfail(bt, PAKR_E_DEVICE, "batch is unusable after a device error");
  return PAKR_OK;
}

// The argument table with these limits (and no trace).
std::vector<KArgs> batch_table(const pakr_batch* bt, double budget_ms, int max_rounds,
                               long long max_iters) {
  std::vector<KArgs> t = bt->args;
  for (auto& a : t) set_limits(a, max_iters, max_rounds, budget_ms, bt->ticks_per_ms);
  return t;
}

// Query q's header (syncs the batch stream); a device error in any query
// (a grid barrier that timed out) leaves the batch's barrier words in an
// unknown state, so the batch refuses every later launch.
int batch_header(pakr_batch* bt, int q, DevHeader* h) {
  hipError_t e = read_header(bt->args[q], bt->stream, h);
  if (e != hipSuccess) return bhip_fail(bt, e, "read header");
  if (h->err != 0) {
    bt->broken = true;
    return bfail(bt, PAKR_E_DEVICE,
                 "query " + std::to_string(q) + ": grid barrier timed out on the device");
  }
  return PAKR_OK;
}

}  // namespace

extern "C" {

int pakr_batch_replan(pakr_batch* bt, double budget_ms, int max_rounds, long long max_iters) {
  if (!bt) return PAKR_E_INVALID_ARG;
  int rc = batch_usable(bt);
  if (rc == PAKR_OK) rc = batch_limits_ok(bt, budget_ms, max_rounds, max_iters);
  if (rc == PAKR_OK) rc = batch_upload(bt, batch_table(bt, budget_ms, max_rounds, max_iters),
                                       bt->d_args);
  if (rc == PAKR_OK) rc = batch_enqueue(bt, bt->d_args, bt->stream);
  return rc;
}

size_t pakr_batch_trace_bytes(const pakr_batch* bt, int q, int n_iters) {
  if (!bt || q < 0 || q >= bt->nq || n_iters < 0) return 0;
  return trace_words_of(bt->args[q].P) * 4 * (size_t)n_iters;
}

int pakr_batch_expand(pakr_batch* bt, int n_iters, void* const* d_traces,
                      const size_t* trace_bytes) {
  if (!bt) return PAKR_E_INVALID_ARG;
  int rc = batch_usable(bt);
  if (rc != PAKR_OK) return rc;
  if (n_iters < 0) return bfail(bt, PAKR_E_INVALID_ARG, "n_iters must be >= 0");
  if (n_iters == 0) return PAKR_OK;
  std::vector<KArgs> t = batch_table(bt, 0.0, 0, n_iters);
  for (int q = 0; q < bt->nq && d_traces; ++q) {
    if (!d_traces[q]) continue;
    if (!trace_bytes || trace_bytes[q] < pakr_batch_trace_bytes(bt, q, n_iters))
      return bfail(bt, PAKR_E_BUFFER_TOO_SMALL,
                   "query " + std::to_string(q) + ": trace buffer too small");
    t[q].trace = static_cast<int*>(d_traces[q]);
    t[q].trace_words = (long long)trace_words_of(t[q].P);
    t[q].trace_iters = n_iters;
  }
  rc = batch_upload(bt, t, bt->d_args);
  if (rc == PAKR_OK) rc = batch_enqueue(bt, bt->d_args, bt->stream);
  return rc;
}

int pakr_batch_graph_capture(pakr_batch* bt, double budget_ms, int max_rounds,
                             long long max_iters) {
  if (!bt) return PAKR_E_INVALID_ARG;
  int rc = batch_usable(bt);
  if (rc == PAKR_OK) rc = batch_limits_ok(bt, budget_ms, max_rounds, max_iters);
  if (rc != PAKR_OK) return rc;
  if (bt->gexec) {
    (void)hipGraphExecDestroy(bt->gexec);
    bt->gexec = nullptr;
  }
  if (bt->graph) {
    (void)hipGraphDestroy(bt->graph);
    bt->graph = nullptr;
  }
  hipError_t e = hipSuccess;
  if (!bt->cap_stream) e = hipStreamCreateWithFlags(&bt->cap_stream, hipStreamNonBlocking);
  if (e != hipSuccess) return bhip_fail(bt, e, "create capture stream");
  // the graph's limits live in its own table, uploaded once outside the
  // graph, so direct launches (which rewrite the other table) leave them alone
  rc = batch_upload(bt, batch_table(bt, budget_ms, max_rounds, max_iters), bt->d_args_graph);
  if (rc != PAKR_OK) return rc;
  e = hipStreamBeginCapture(bt->cap_stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return bhip_fail(bt, e, "begin capture");
  rc = batch_enqueue(bt, bt->d_args_graph, bt->cap_stream);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(bt->cap_stream, &g);
  if (rc != PAKR_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return bhip_fail(bt, e, "end capture");
  bt->graph = g;
  e = hipGraphInstantiate(&bt->gexec, bt->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) return bhip_fail(bt, e, "instantiate graph");
  return PAKR_OK;
}

int pakr_batch_graph_launch(pakr_batch* bt) {
  if (!bt) return PAKR_E_INVALID_ARG;
  int rc = batch_usable(bt);
  if (rc != PAKR_OK) return rc;
  if (!bt->gexec) return bfail(bt, PAKR_E_INVALID_ARG, "no captured graph");
  hipError_t e = hipGraphLaunch(bt->gexec, bt->stream);
  if (e != hipSuccess) return bhip_fail(bt, e, "graph launch");
  return PAKR_OK;
}

int pakr_batch_status(pakr_batch* bt, int q, pakr_stats* out) {
  if (!bt || !out || q < 0 || q >= bt->nq) return PAKR_E_INVALID_ARG;
  DevHeader h;
  int rc = batch_header(bt, q, &h);
  if (rc != PAKR_OK) return rc;
  fill_stats(h, bt->ticks_per_ms, bt->G, out);
  return PAKR_OK;
}

int pakr_batch_solutions(pakr_batch* bt, int q, pakr_solution* out, int cap, int* n_total) {
  if (!bt || !n_total || q < 0 || q >= bt->nq || cap < 0 || (cap > 0 && !out))
    return PAKR_E_INVALID_ARG;
  DevHeader h;
  int rc = batch_header(bt, q, &h);
  if (rc != PAKR_OK) return rc;
  *n_total = h.n_solutions;
  hipError_t e = read_solutions(bt->args[q], bt->ticks_per_ms,
                                std::min(std::min(cap, h.n_solutions), MAX_SOLUTIONS), out);
  if (e != hipSuccess) return bhip_fail(bt, e, "read solutions");
  return PAKR_OK;
}

int pakr_batch_extract_path(pakr_batch* bt, int q, float* states, float* actions, int cap_edges,
                            int* n_edges, double* cost) {
  if (!bt || !n_edges || q < 0 || q >= bt->nq) return PAKR_E_INVALID_ARG;
  DevHeader h;
  int rc = batch_header(bt, q, &h);
  if (rc != PAKR_OK) return rc;
  if (h.best_edges < 0) {
    *n_edges = 0;
    return bfail(bt, PAKR_E_NO_SOLUTION, "no solution yet");
  }
  *n_edges = h.best_edges;
  if (cost) *cost = (double)h.best_cost;
  if (h.path_truncated) return bfail(bt, PAKR_E_BUFFER_TOO_SMALL, "path longer than max_path_edges");
  if (h.best_edges > cap_edges) return bfail(bt, PAKR_E_BUFFER_TOO_SMALL, "cap_edges too small");
  if (!states || !actions) return bfail(bt, PAKR_E_INVALID_ARG, "null output arrays");
  hipError_t e = read_path(bt->args[q], h.best_edges, states, actions);
  if (e != hipSuccess) return bhip_fail(bt, e, "read path");
  return PAKR_OK;
}

int pakr_batch_copy_tree(pakr_batch* bt, int q, float* states, float* actions, int* parents,
                         float* costs, int n_max, int* n_out) {
  if (!bt || !n_out || n_max < 0 || q < 0 || q >= bt->nq) return PAKR_E_INVALID_ARG;
  DevHeader h;
  int rc = batch_header(bt, q, &h);
  if (rc != PAKR_OK) return rc;
  *n_out = h.n;
  hipError_t e = read_tree(bt->args[q], std::min(h.n, n_max), states, actions, parents, costs);
  if (e != hipSuccess) return bhip_fail(bt, e, "read tree");
  return PAKR_OK;
}

int pakr_batch_grid(const pakr_batch* bt) { return bt ? bt->G : 0; }

int pakr_batch_team(const pakr_batch* bt, int q) {
  return (bt && q >= 0 && q < bt->nq) ? bt->team[(size_t)q] : 0;
}

const char* pakr_batch_last_error(const pakr_batch* bt) {
  return bt ? bt->err.c_str() : g_init_error;
}

void pakr_batch_destroy(pakr_batch* bt) {
  if (!bt) return;
  if (bt->ws) (void)hipStreamSynchronize(bt->stream);
  if (bt->gexec) (void)hipGraphExecDestroy(bt->gexec);
  if (bt->graph) (void)hipGraphDestroy(bt->graph);
  if (bt->cap_stream) (void)hipStreamDestroy(bt->cap_stream);
  if (bt->own_ws && bt->ws) (void)hipFree(bt->ws);
  delete bt;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Trajectory refinement
// ---------------------------------------------------------------------------
struct pakr_refiner {
  DevProblem P;
  RefineParams R;
  int device = 0;  // current device when the refiner was created
  hipStream_t stream = nullptr;
  float* obs = nullptr;
  size_t shmem = 0;
  std::string err;
};


namespace {

// Work buffers of pakr_refine_paths_static: one copy of this array per GPU,
// held until the process ends.  Its name is a host-side stand-in: host code
// uses the device address looked up per device (refine_scratch_on).
constexpr int MAX_DEVICES = 64;
__device__ __align__(256) unsigned char scratch[PAKR_REFINE_STATIC_BYTES];
// (trivially destructible: nothing runs at process exit)
std::atomic<void*> g_scratch_ptr[MAX_DEVICES];

// Device address of `scratch` on `dev`, which must be the current device;
// looked up on the first call per device (idempotent, so concurrent first
// calls store the same value).  nullptr with *err set if the lookup fails.
void* refine_scratch_on(int dev, hipError_t* err) {
  *err = hipSuccess;
  if (dev < 0 || dev >= MAX_DEVICES) {
    *err = hipErrorInvalidDevice;
    return nullptr;
  }
  void* p = g_scratch_ptr[dev].load(std::memory_order_acquire);
  if (p != nullptr) return p;
  *err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (*err != hipSuccess) return nullptr;
  g_scratch_ptr[dev].store(p, std::memory_order_release);
  return p;
}

int rfail(pakr_refiner* r, int code, const std::string& msg) {
  if (r) r->err = msg;
  else set_init_error(msg);
  return code;
}

std::string validate_refine(const pakr_refine_params* rp, int m) {
  if (!(rp->w_effort >= 0.0f) || !(rp->w_goal >= 0.0f) || !(rp->w_collision >= 0.0f) ||
      !finite_f(rp->w_effort) || !finite_f(rp->w_goal) || !finite_f(rp->w_collision))
    return "refinement weights must be finite and >= 0";
  if (!(rp->beta > 0.0f) || !finite_f(rp->beta)) return "beta must be finite and > 0";
  if (!(rp->delta >= 0.0f) || !finite_f(rp->delta)) return "delta must be finite and >= 0";
  for (int c = 0; c < m; ++c) {
    if (!finite_f(rp->u_ref[c])) return "u_ref must be finite";
    if (!(rp->u_scale[c] > 0.0f) || !finite_f(rp->u_scale[c])) return "u_scale must be > 0";
  }
  return std::string();
}

RefineParams to_device(const pakr_refine_params& rp) {
  RefineParams R;
  std::memset(&R, 0, sizeof R);
  R.w_u = rp.w_effort;
  R.w_g = rp.w_goal;
  R.w_c = rp.w_collision;
  R.beta = rp.beta;
  R.delta = rp.delta;
  R.inv_beta = rp.beta > 0.0f ? 1.0f / rp.beta : 0.0f;
  for (int c = 0; c < PAKR_MAX_M; ++c) {
    R.u_ref[c] = rp.u_ref[c];
    R.u_scale[c] = rp.u_scale[c] > 0.0f ? rp.u_scale[c] : 1.0f;
  }
  return R;
}

// Largest trajectory count and edge count one call accepts.
constexpr int MAX_TRAJ = 1 << 20;
constexpr int MAX_EDGES = 1 << 16;

bool traj_sizes_ok(const pakr_refiner* r, int n, int M) {
  return r && n >= 1 && n <= MAX_TRAJ && M >= 1 && M <= MAX_EDGES &&
         (size_t)M * (size_t)r->P.T < (size_t)1 << 30;
}

size_t ckpt_bytes_of(const pakr_refiner* r, int n, int M) {
  return sizeof(float) * (size_t)n * ((size_t)M * r->P.T + 1) * (size_t)r->P.d;
}

template <int SYS>
const void* traj_kernel(int which) {
  if (which == 0) return reinterpret_cast<const void*>(&k_rollout_fwd<SYS>);
  if (which == 1) return reinterpret_cast<const void*>(&k_rollout_bwd<SYS>);
  return reinterpret_cast<const void*>(&k_check_path<SYS>);
}

const void* traj_kernel_for(int sys, int which) {
  switch (sys) {
    case PAKR_DI2: return traj_kernel<PAKR_DI2>(which);
    case PAKR_DI3: return traj_kernel<PAKR_DI3>(which);
    case PAKR_CAR: return traj_kernel<PAKR_CAR>(which);
    case PAKR_DUBINS: return traj_kernel<PAKR_DUBINS>(which);
    case PAKR_UNI1: return traj_kernel<PAKR_UNI1>(which);
    case PAKR_UNI2: return traj_kernel<PAKR_UNI2>(which);
    case PAKR_ACROBOT: return traj_kernel<PAKR_ACROBOT>(which);
    case PAKR_CARTPOLE: return traj_kernel<PAKR_CARTPOLE>(which);
    default: return traj_kernel<PAKR_QUAD>(which);
  }
}

int launch_traj(pakr_refiner* r, int which, TrajArgs& a) {
  void* args[] = {&a};
  hipError_t e = hipLaunchKernel(traj_kernel_for(r->P.system, which), dim3(a.n_traj), dim3(WAVE),
                                 args, r->shmem, r->stream);
  if (e != hipSuccess) return rfail(r, PAKR_E_HIP, std::string("launch: ") + hipGetErrorString(e));
  return PAKR_OK;
}

int launch_adam(pakr_refiner* r, int n, int M, const float* U, float* U_out, const float* gU,
                float* m1, float* m2, const float* lr_traj, int step, float lr) {
  const size_t total = (size_t)n * M * r->P.m;
  AdamArgs a;
  std::memset(&a, 0, sizeof a);
  a.U = U;
  a.U_out = U_out;
  a.gU = gU;
  a.m1 = m1;
  a.m2 = m2;
  a.lr_traj = lr_traj;
  a.n = (int)total;
  a.m = r->P.m;
  a.per_traj = M * r->P.m;
  a.lr = lr;
  a.b1 = 0.9f;
  a.b2 = 0.999f;
  a.eps = 1e-8f;
  a.c1 = (float)(1.0 - std::pow(0.9, step));
  a.c2 = (float)(1.0 - std::pow(0.999, step));
  for (int c = 0; c < PAKR_MAX_M; ++c) {
    a.u_lo[c] = r->P.u_lo[c];
    a.u_hi[c] = r->P.u_hi[c];
  }
  void* args[] = {&a};
  const int blocks = (int)((total + 255) / 256);
  hipError_t e = hipLaunchKernel(reinterpret_cast<const void*>(&k_adam_project), dim3(blocks),
                                 dim3(256), args, 0, r->stream);
  if (e != hipSuccess) return rfail(r, PAKR_E_HIP, std::string("launch: ") + hipGetErrorString(e));
  return PAKR_OK;
}

int launch_accept(pakr_refiner* r, int n, int M, float* U, const float* Ut, float* J,
                  const float* Jt, float* lr_traj) {
  AcceptArgs a;
  a.U = U;
  a.U_trial = Ut;
  a.J = J;
  a.J_trial = Jt;
  a.lr_traj = lr_traj;
  a.per_traj = M * r->P.m;
  a.n_traj = n;
  void* args[] = {&a};
  hipError_t e = hipLaunchKernel(reinterpret_cast<const void*>(&k_accept), dim3(n), dim3(WAVE),
                                 args, 0, r->stream);
  if (e != hipSuccess) return rfail(r, PAKR_E_HIP, std::string("launch: ") + hipGetErrorString(e));
  return PAKR_OK;
}

int launch_fill(pakr_refiner* r, float* x, int n, float v) {
  void* args[] = {&x, &n, &v};
  hipError_t e = hipLaunchKernel(reinterpret_cast<const void*>(&k_fill), dim3((n + 255) / 256),
                                 dim3(256), args, 0, r->stream);
  if (e != hipSuccess) return rfail(r, PAKR_E_HIP, std::string("launch: ") + hipGetErrorString(e));
  return PAKR_OK;
}

int launch_copy(pakr_refiner* r, float* dst, const float* src, int n) {
  hipError_t e = hipMemcpyAsync(dst, src, sizeof(float) * (size_t)n, hipMemcpyDeviceToDevice,
                                r->stream);
  if (e != hipSuccess) return rfail(r, PAKR_E_HIP, std::string("copy: ") + hipGetErrorString(e));
  return PAKR_OK;
}

struct RefineLayout {
  size_t ckpt, m1, m2, ut, gu, j, jt, ones, lr, total;
};

RefineLayout refine_layout(const pakr_refiner* r, int n, int M) {
  RefineLayout L{};
  const size_t nv = (size_t)n * M * r->P.m;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align_up(off + bytes);
    return at;
  };
  L.ckpt = take(ckpt_bytes_of(r, n, M));
  L.m1 = take(sizeof(float) * nv);
  L.m2 = take(sizeof(float) * nv);
  L.ut = take(sizeof(float) * nv);
  L.gu = take(sizeof(float) * nv);
  L.j = take(sizeof(float) * n);
  L.jt = take(sizeof(float) * n);
  L.ones = take(sizeof(float) * n);
  L.lr = take(sizeof(float) * n);
  L.total = off;
  return L;
}

TrajArgs traj_args(const pakr_refiner* r, int n, int M) {
  TrajArgs a;
  std::memset(&a, 0, sizeof a);
  a.P = r->P;
  a.R = r->R;
  a.obs = r->obs;
  a.n_traj = n;
  a.M = M;
  return a;
}

}  // namespace

extern "C" {

int pakr_refiner_init(const pakr_system* sys, const pakr_scene* scene, const pakr_goal* goal,
                      const pakr_params* params, const pakr_refine_params* refine, void* stream,
                      pakr_refiner** out) {
  if (!out) return rfail(nullptr, PAKR_E_INVALID_ARG, "null output pointer");
  *out = nullptr;
  if (!sys || !scene || !goal || !params || !refine)
    return rfail(nullptr, PAKR_E_INVALID_ARG, "null argument");
  std::string m = validate_system(sys, scene);
  if (m.empty() && params->T < 1) m = "T must be >= 1";
  if (m.empty() && (!(params->dt > 0.0f) || !std::isfinite(params->dt)))
    m = "dt must be finite and > 0";
  if (m.empty() && params->cost_kind != PAKR_COST_DURATION &&
      params->cost_kind != PAKR_COST_PATH_LENGTH)
    m = "bad cost_kind";
  if (m.empty()) m = validate_scene(scene);
  if (m.empty()) m = validate_refine(refine, sys->m);
  if (!m.empty()) return rfail(nullptr, PAKR_E_INVALID_ARG, m);
  m = validate_goal(goal, scene);
  if (!m.empty()) return rfail(nullptr, PAKR_E_GOAL_INVALID, m);

  pakr_refiner* r = new (std::nothrow) pakr_refiner();
  if (!r) return rfail(nullptr, PAKR_E_INVALID_ARG, "out of host memory");
  r->stream = static_cast<hipStream_t>(stream);
  hipError_t e = hipGetDevice(&r->device);
  // set-up of pakr_refine_paths_static: the static work array's address on
  // this device, looked up now so that the entry point itself does nothing
  // but launch kernels
  if (e == hipSuccess) (void)refine_scratch_on(r->device, &e);
  if (e != hipSuccess) {
    int rc = rfail(nullptr, PAKR_E_HIP, std::string("refiner set-up: ") + hipGetErrorString(e));
    delete r;
    return rc;
  }
  // the planner's record of the query; B, A, n_cap do not matter here
  pakr_params prm = *params;
  prm.B = 1;
  prm.A = 1;
  prm.n_cap = 2;
  r->P = make_problem(*sys, *scene, *goal, prm, 1, 1);
  r->R = to_device(*refine);
  const std::vector<float> obs = pack_obstacles(*scene);
  r->shmem = sizeof(float) * std::max<size_t>(obs.size(), 1);
  e = hipMalloc(&r->obs, r->shmem);
  if (e == hipSuccess && !obs.empty())
    e = hipMemcpyAsync(r->obs, obs.data(), sizeof(float) * obs.size(), hipMemcpyHostToDevice,
                       r->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(r->stream);
  if (e != hipSuccess) {
    int rc = rfail(nullptr, PAKR_E_HIP, std::string("upload obstacles: ") + hipGetErrorString(e));
    pakr_refiner_destroy(r);
    return rc;
  }
  *out = r;
  return PAKR_OK;
}

int pakr_refiner_set_params(pakr_refiner* r, const pakr_refine_params* refine) {
  if (!r || !refine) return PAKR_E_INVALID_ARG;
  std::string m = validate_refine(refine, r->P.m);
  if (!m.empty()) return rfail(r, PAKR_E_INVALID_ARG, m);
  r->R = to_device(*refine);
  return PAKR_OK;
}

size_t pakr_rollout_ckpt_bytes(const pakr_refiner* r, int n, int M) {
  if (!traj_sizes_ok(r, n, M)) return 0;
  return ckpt_bytes_of(r, n, M);
}

int pakr_rollout_fwd(pakr_refiner* r, int n, int M, const float* d_x0, const float* d_U,
                     void* d_ckpt, size_t ckpt_bytes, float* d_J) {
  if (!r) return PAKR_E_INVALID_ARG;
  if (!traj_sizes_ok(r, n, M)) return rfail(r, PAKR_E_INVALID_ARG, "bad trajectory count or M");
  if (!d_x0 || !d_U || !d_ckpt || !d_J) return rfail(r, PAKR_E_INVALID_ARG, "null device array");
  if (ckpt_bytes < ckpt_bytes_of(r, n, M))
    return rfail(r, PAKR_E_WORKSPACE_TOO_SMALL, "checkpoint buffer smaller than required");
  TrajArgs a = traj_args(r, n, M);
  a.x0 = d_x0;
  a.U = d_U;
  a.ckpt = static_cast<float*>(d_ckpt);
  a.J = d_J;
  return launch_traj(r, 0, a);
}

int pakr_rollout_bwd(pakr_refiner* r, int n, int M, const float* d_U, const void* d_ckpt,
                     size_t ckpt_bytes, const float* d_gJ, float* d_gU) {
  if (!r) return PAKR_E_INVALID_ARG;
  if (!traj_sizes_ok(r, n, M)) return rfail(r, PAKR_E_INVALID_ARG, "bad trajectory count or M");
  if (!d_U || !d_ckpt || !d_gJ || !d_gU) return rfail(r, PAKR_E_INVALID_ARG, "null device array");
  if (ckpt_bytes < ckpt_bytes_of(r, n, M))
    return rfail(r, PAKR_E_WORKSPACE_TOO_SMALL, "checkpoint buffer smaller than required");
  TrajArgs a = traj_args(r, n, M);
  a.U = d_U;
  a.ckpt = const_cast<float*>(static_cast<const float*>(d_ckpt));
  a.gJ = d_gJ;
  a.gU = d_gU;
  return launch_traj(r, 1, a);
}

int pakr_refine_step(pakr_refiner* r, int n, int M, float* d_U, const float* d_gU, float* d_m1,
                     float* d_m2, int step, float lr) {
  if (!r) return PAKR_E_INVALID_ARG;
  if (!traj_sizes_ok(r, n, M)) return rfail(r, PAKR_E_INVALID_ARG, "bad trajectory count or M");
  if (!d_U || !d_gU || !d_m1 || !d_m2) return rfail(r, PAKR_E_INVALID_ARG, "null device array");
  if (step < 1) return rfail(r, PAKR_E_INVALID_ARG, "step counts from 1");
  if (!(lr > 0.0f) || !std::isfinite(lr)) return rfail(r, PAKR_E_INVALID_ARG, "lr must be > 0");
  if ((size_t)n * M * r->P.m > (size_t)INT32_MAX)
    return rfail(r, PAKR_E_INVALID_ARG, "too many control values");
  return launch_adam(r, n, M, d_U, d_U, d_gU, d_m1, d_m2, nullptr, step, lr);
}

size_t pakr_refine_workspace_size(const pakr_refiner* r, int n, int M) {
  if (!traj_sizes_ok(r, n, M) || (size_t)n * M * r->P.m > (size_t)INT32_MAX) return 0;
  return refine_layout(r, n, M).total;
}

}  // extern "C"

namespace {

// Argument checks shared by the two refinement-loop entry points.
int refine_args_ok(pakr_refiner* r, int n, int M, const float* d_x0, float* d_U, int steps,
                   float lr) {
  if (!traj_sizes_ok(r, n, M) || (size_t)n * M * r->P.m > (size_t)INT32_MAX)
    return rfail(r, PAKR_E_INVALID_ARG, "bad trajectory count or M");
  if (!d_x0 || !d_U) return rfail(r, PAKR_E_INVALID_ARG, "null device array");
  if (steps < 0) return rfail(r, PAKR_E_INVALID_ARG, "steps must be >= 0");
  if (!(lr > 0.0f) || !std::isfinite(lr)) return rfail(r, PAKR_E_INVALID_ARG, "lr must be > 0");
  return PAKR_OK;
}

// The refinement loop with its work buffers (layout L) at `base`: every
// buffer that must start at a known value is filled by a kernel first.
int refine_paths_at(pakr_refiner* r, int n, int M, const float* d_x0, float* d_U, int steps,
                    float lr, char* base, const RefineLayout& L, float* d_J_before,
                    float* d_J_after) {
  float* ckpt = reinterpret_cast<float*>(base + L.ckpt);
  float* m1 = reinterpret_cast<float*>(base + L.m1);
  float* m2 = reinterpret_cast<float*>(base + L.m2);
  float* Ut = reinterpret_cast<float*>(base + L.ut);
  float* gU = reinterpret_cast<float*>(base + L.gu);
  float* J = reinterpret_cast<float*>(base + L.j);
  float* Jt = reinterpret_cast<float*>(base + L.jt);
  float* ones = reinterpret_cast<float*>(base + L.ones);
  float* lr_traj = reinterpret_cast<float*>(base + L.lr);
  const int nv = n * M * r->P.m;
  // fills by kernel (no memset nodes, so the sequence can be graph-captured)
  int rc = launch_fill(r, m1, nv, 0.0f);
  if (rc == PAKR_OK) rc = launch_fill(r, m2, nv, 0.0f);
  if (rc == PAKR_OK) rc = launch_fill(r, ones, n, 1.0f);
  if (rc == PAKR_OK) rc = launch_fill(r, lr_traj, n, 1.0f);
  TrajArgs f = traj_args(r, n, M);
  f.x0 = d_x0;
  f.ckpt = ckpt;
  TrajArgs b = traj_args(r, n, M);
  b.U = d_U;
  b.ckpt = ckpt;
  b.gJ = ones;
  b.gU = gU;
  // J of the starting controls
  f.U = d_U;
  f.J = J;
  if (rc == PAKR_OK) rc = launch_traj(r, 0, f);
  if (rc == PAKR_OK && d_J_before)
    rc = launch_copy(r, d_J_before, J, n);
  for (int k = 1; k <= steps && rc == PAKR_OK; ++k) {
    // checkpoints of the current controls, then the adjoint from them
    if (k > 1) {
      f.U = d_U;
      f.J = Jt;  // J of the current controls is already in J
      rc = launch_traj(r, 0, f);
    }
    if (rc == PAKR_OK) rc = launch_traj(r, 1, b);
    if (rc == PAKR_OK) rc = launch_adam(r, n, M, d_U, Ut, gU, m1, m2, lr_traj, k, lr);
    if (rc == PAKR_OK) {
      f.U = Ut;
      f.J = Jt;
      rc = launch_traj(r, 0, f);
    }
    if (rc == PAKR_OK) rc = launch_accept(r, n, M, d_U, Ut, J, Jt, lr_traj);
  }
  if (rc == PAKR_OK && d_J_after) rc = launch_copy(r, d_J_after, J, n);
  return rc;
}

}  // namespace

extern "C" {

int pakr_refine_paths(pakr_refiner* r, int n, int M, const float* d_x0, float* d_U, int steps,
                      float lr, void* d_ws, size_t ws_bytes, float* d_J_before, float* d_J_after) {
  if (!r) return PAKR_E_INVALID_ARG;
  int rc = refine_args_ok(r, n, M, d_x0, d_U, steps, lr);
  if (rc != PAKR_OK) return rc;
  if (!d_ws) return rfail(r, PAKR_E_INVALID_ARG, "null device array");
  const RefineLayout L = refine_layout(r, n, M);
  if (ws_bytes < L.total)
    return rfail(r, PAKR_E_WORKSPACE_TOO_SMALL, "workspace smaller than required");
  if ((reinterpret_cast<uintptr_t>(d_ws) & 255) != 0)
    return rfail(r, PAKR_E_INVALID_ARG, "workspace must be 256-byte aligned");
  return refine_paths_at(r, n, M, d_x0, d_U, steps, lr, static_cast<char*>(d_ws), L, d_J_before,
                         d_J_after);
}

int pakr_refine_paths_static(pakr_refiner* r, int n, int M, const float* d_x0, float* d_U,
                             int steps, float lr, float* d_J_before, float* d_J_after) {
  if (!r) return PAKR_E_INVALID_ARG;
  int rc = refine_args_ok(r, n, M, d_x0, d_U, steps, lr);
  if (rc != PAKR_OK) return rc;
  const RefineLayout L = refine_layout(r, n, M);
  if (L.total > (size_t)PAKR_REFINE_STATIC_BYTES)
    return rfail(r, PAKR_E_WORKSPACE_TOO_SMALL,
                 "refinement buffers of " + std::to_string(L.total) +
                     " bytes exceed the static array of " +
                     std::to_string((size_t)PAKR_REFINE_STATIC_BYTES) + " bytes");
  // looked up when the refiner was created (this call then allocates nothing)
  void* base = g_scratch_ptr[r->device].load(std::memory_order_acquire);
  if (base == nullptr) return rfail(r, PAKR_E_HIP, "static refinement array not set up");
  return refine_paths_at(r, n, M, d_x0, d_U, steps, lr, static_cast<char*>(base), L, d_J_before,
                         d_J_after);
}

int pakr_check_path(pakr_refiner* r, int n, int M, const float* d_x0, const float* d_U,
                    int* d_ok, float* d_cost) {
  if (!r) return PAKR_E_INVALID_ARG;
  if (!traj_sizes_ok(r, n, M)) return rfail(r, PAKR_E_INVALID_ARG, "bad trajectory count or M");
  if (!d_x0 || !d_U || !d_ok || !d_cost) return rfail(r, PAKR_E_INVALID_ARG, "null device array");
  TrajArgs a = traj_args(r, n, M);
  a.x0 = d_x0;
  a.U = d_U;
  a.ok = d_ok;
  a.cost = d_cost;
  return launch_traj(r, 2, a);
}

const char* pakr_refiner_last_error(const pakr_refiner* r) {
  return r ? r->err.c_str() : g_init_error;
}

void pakr_refiner_destroy(pakr_refiner* r) {
  if (!r) return;
  if (r->obs) {
    (void)hipStreamSynchronize(r->stream);
    (void)hipFree(r->obs);
  }
  delete r;
}

}  // extern "C"
