// libpakr: host side of the C ABI declared in include/pakr.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "pakr_kernels.hpp"

using namespace pakr;

namespace {

constexpr int AUTO_GRID_MAX = 1024;      // workspace sizing bound for grid = 0
constexpr int DEFAULT_PATH_EDGES = 4096;

thread_local std::string g_init_error;

struct Layout {
  size_t hdr, bar, sols, pstates, pactions, states, actions, parents, costs, obs, partial, stg,
      counts, goalmin, total;
};

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

int sys_npos(int id) { return (id == PAKR_DI2 || id == PAKR_CAR) ? 2 : 3; }
int sys_d(int id) {
  switch (id) {
    case PAKR_DI2: return 4;
    case PAKR_DI3: return 6;
    case PAKR_CAR: return 5;
    case PAKR_QUAD: return 12;
  }
  return -1;
}
int sys_m(int id) {
  switch (id) {
    case PAKR_DI2: return 2;
    case PAKR_DI3: return 3;
    case PAKR_CAR: return 2;
    case PAKR_QUAD: return 4;
  }
  return -1;
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

Layout make_layout(int d, int m, const pakr_params& p, int G, int obs_floats, int lanes) {
  Layout L{};
  const int K = p.B / p.A;
  const int cpb = NT / lanes;
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
  L.partial = take(sizeof(unsigned long long) * (size_t)G * K);
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

// Returns an empty string when the query is well formed.
std::string validate(const pakr_system* s, const pakr_scene* sc, const float* x0,
                     const pakr_goal* g, const pakr_params* p, int* code) {
  *code = PAKR_E_INVALID_ARG;
  if (!s || !sc || !x0 || !g || !p) return "null argument";
  if (s->id < PAKR_DI2 || s->id > PAKR_QUAD) return "unknown system id";
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
      p->lanes_per_candidate != 4 && p->lanes_per_candidate != 8)
    return "lanes_per_candidate must be 0, 1, 2, 4 or 8";
  if (p->workgroups_per_cu < 0 || p->workgroups_per_cu > 8) return "workgroups_per_cu must be 0..8";
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
  *code = PAKR_E_GOAL_INVALID;
  if (!(g->radius > 0.0f) || !finite_f(g->radius)) return "goal radius must be > 0";
  for (int c = 0; c < P; ++c)
    if (!(g->center[c] >= sc->ws_lo[c] && g->center[c] <= sc->ws_hi[c]))
      return "goal centre outside the workspace";
  *code = PAKR_E_START_INVALID;
  if (!host_state_ok(*s, *sc, x0)) return "x_init is not in X_free (bounds, limits or obstacles)";
  *code = PAKR_OK;
  return std::string();
}

typedef void (*kernel_fn)(KArgs);

template <int SYS>
const void* pick_kernel(int qt) {
  if (qt == 1) return reinterpret_cast<const void*>(&k_plan<SYS, 1>);
  if (qt == 2) return reinterpret_cast<const void*>(&k_plan<SYS, 2>);
  return reinterpret_cast<const void*>(&k_plan<SYS, 4>);
}

const void* kernel_for(int sys, int qt) {
  switch (sys) {
    case PAKR_DI2: return pick_kernel<PAKR_DI2>(qt);
    case PAKR_DI3: return pick_kernel<PAKR_DI3>(qt);
    case PAKR_CAR: return pick_kernel<PAKR_CAR>(qt);
    default: return pick_kernel<PAKR_QUAD>(qt);
  }
}

}  // namespace

struct pakr_plan {
  pakr_system sys;
  pakr_params prm;
  DevProblem P;
  int G = 0, qt = 1;
  int device = 0;
  hipStream_t stream = nullptr;
  double ticks_per_ms = 100000.0;
  void* ws = nullptr;
  bool own_ws = false;
  size_t ws_bytes = 0;
  Layout L{};
  const void* kfn = nullptr;
  size_t shmem = 0;
  bool broken = false;
  std::string err;
  template <typename T>
  T* at(size_t off) const {
    return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
  }
};

namespace {

int fail(pakr_plan* pl, int code, const std::string& msg) {
  if (pl) pl->err = msg;
  else g_init_error = msg;
  return code;
}

int hip_fail(pakr_plan* pl, hipError_t e, const char* what) {
  std::string m = std::string(what) + ": " + hipGetErrorString(e);
  return fail(pl, PAKR_E_HIP, m);
}

int qt_for(int K) { return K <= NT ? 1 : (K <= 2 * NT ? 2 : 4); }

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
  size_t worst = 0;  // the auto lane choice may differ; size for the largest layout
  for (int lanes = 1; lanes <= 8; lanes <<= 1) {
    pakr_params q = *params;
    q.lanes_per_candidate = lanes;
    worst = std::max(worst, make_layout(d, m, q, G, of, lanes).total);
  }
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

  pakr_plan* pl = new (std::nothrow) pakr_plan();
  if (!pl) return fail(nullptr, PAKR_E_INVALID_ARG, "out of host memory");
  pl->sys = *sys;
  pl->prm = *params;
  pl->stream = static_cast<hipStream_t>(stream);
  hipError_t e = hipGetDevice(&pl->device);
  if (e != hipSuccess) {
    int rc = hip_fail(nullptr, e, "hipGetDevice");
    delete pl;
    return rc;
  }
  int n_cu = 0, coop = 0, wclk_khz = 0;
  if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, pl->device) != hipSuccess ||
      hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, pl->device) != hipSuccess ||
      hipDeviceGetAttribute(&wclk_khz, hipDeviceAttributeWallClockRate, pl->device) != hipSuccess) {
    delete pl;
    return fail(nullptr, PAKR_E_HIP, "device attribute query failed");
  }
  if (wclk_khz > 0) pl->ticks_per_ms = (double)wclk_khz;
  if (!coop) {
    delete pl;
    return fail(nullptr, PAKR_E_HIP, "device does not support cooperative launches");
  }

  const int d = sys->d, m = sys->m, P = scene->npos;
  const int K = params->B / params->A;
  pl->qt = qt_for(K);
  pl->kfn = kernel_for(sys->id, pl->qt);
  const int of = obs_floats_of(P, scene->n_box, scene->n_sphere);
  const size_t obs_bytes = sizeof(float) * (size_t)std::max(of, 1);
  pl->shmem = obs_bytes;
  int G = 0;
  if (params->grid > 0) {
    G = params->grid;
  } else {
    // k workgroups on every CU: reserve enough LDS that a CU cannot hold k+1,
    // so the co-resident grid of k * CUs is spread evenly
    const int k = params->workgroups_per_cu > 0 ? params->workgroups_per_cu : 1;
    int lds_cu = 0, lds_max = 0;
    hipFuncAttributes fa;
    if (hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor,
                              pl->device) != hipSuccess ||
        hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, pl->device) !=
            hipSuccess ||
        hipFuncGetAttributes(&fa, pl->kfn) != hipSuccess) {
      delete pl;
      return fail(nullptr, PAKR_E_HIP, "LDS attribute query failed");
    }
    const size_t want = (size_t)lds_cu / (size_t)(k + 1) + 1024;  // > LDS/(k+1) per workgroup
    const size_t dyn = want > fa.sharedSizeBytes ? want - fa.sharedSizeBytes : 0;
    if (dyn + fa.sharedSizeBytes <= (size_t)lds_max && dyn > obs_bytes) pl->shmem = dyn;
    G = k * n_cu;
  }
  int per_cu = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, pl->kfn, NT, pl->shmem);
  if (e != hipSuccess || per_cu < 1) {
    int rc = e != hipSuccess ? hip_fail(nullptr, e, "occupancy query")
                             : fail(nullptr, PAKR_E_HIP, "kernel does not fit on a CU");
    delete pl;
    return rc;
  }
  const int max_coresident = per_cu * n_cu;
  if (params->grid <= 0) G = std::min(G, max_coresident);
  const int lanes = lanes_for(*params, scene->n_box + scene->n_sphere,
                              params->grid > 0 ? G : max_coresident);
  const int cpb = NT / lanes;
  const int GR = (params->B + cpb - 1) / cpb;
  if (G < GR) G = params->grid > 0 ? -1 : GR;
  if (G < 1 || G > max_coresident) {
    char buf[160];
    snprintf(buf, sizeof buf, "grid %d invalid: need >= %d rollout workgroups and <= %d co-resident",
             params->grid > 0 ? params->grid : G, GR, max_coresident);
    delete pl;
    return fail(nullptr, PAKR_E_INVALID_ARG, buf);
  }
  pl->G = G;

  pl->L = make_layout(d, m, *params, G, of, lanes);
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
    pl->ws_bytes = ws_bytes;
  } else {
    e = hipMalloc(&pl->ws, need);
    if (e != hipSuccess) {
      int rc = hip_fail(nullptr, e, "hipMalloc workspace");
      delete pl;
      return rc;
    }
    pl->own_ws = true;
    pl->ws_bytes = need;
  }

  DevProblem& Q = pl->P;
  std::memset(&Q, 0, sizeof Q);
  Q.system = sys->id;
  Q.d = d;
  Q.m = m;
  Q.npos = P;
  Q.B = params->B;
  Q.A = params->A;
  Q.K = K;
  Q.T = params->T;
  Q.n_cap = params->n_cap;
  Q.cost_kind = params->cost_kind;
  Q.h_kind = params->heuristic_kind;
  Q.max_iters_per_round = params->max_iters_per_round;
  Q.n_box = scene->n_box;
  Q.n_sph = scene->n_sphere;
  Q.G = G;
  Q.G_roll = GR;
  Q.lanes = lanes;
  Q.cpb = cpb;
  Q.max_path_edges = params->max_path_edges > 0 ? params->max_path_edges : DEFAULT_PATH_EDGES;
  Q.obs_floats = of;
  Q.key0 = (uint32_t)(params->seed & 0xffffffffull);
  Q.key1 = params->query_id;
  Q.dt = params->dt;
  Q.h_speed = params->h_speed;
  Q.c0 = (float)params->cost_bound;
  Q.vnorm_max = sys->vnorm_max;
  Q.goal_r = goal->radius;
  Q.goal_r2 = goal->radius * goal->radius;
  {
    volatile float tf = (float)params->T;
    volatile float ed = tf * params->dt;  // one float32 rounding
    Q.edge_duration = ed;
  }
  for (int i = 0; i < 8; ++i) Q.dyn[i] = sys->dyn[i];
  for (int i = 0; i < PAKR_MAX_D; ++i) {
    Q.sample_lo[i] = sys->sample_lo[i];
    Q.sample_hi[i] = sys->sample_hi[i];
    Q.lim_lo[i] = sys->lim_lo[i];
    Q.lim_hi[i] = sys->lim_hi[i];
  }
  for (int i = 0; i < PAKR_MAX_M; ++i) {
    Q.u_lo[i] = sys->u_lo[i];
    Q.u_hi[i] = sys->u_hi[i];
  }
  for (int c = 0; c < 3; ++c) {
    Q.ws_lo[c] = c < P ? scene->ws_lo[c] : 0.0f;
    Q.ws_hi[c] = c < P ? scene->ws_hi[c] : 0.0f;
    Q.goal_c[c] = c < P ? goal->center[c] : 0.0f;
  }

  // pack obstacles: boxes (c[P], h[P]) then spheres (c[P], r^2)
  float* obs_h = static_cast<float*>(std::malloc(sizeof(float) * (size_t)std::max(of, 1)));
  if (!obs_h) {
    pakr_plan_destroy(pl);
    return fail(nullptr, PAKR_E_INVALID_ARG, "out of host memory");
  }
  int w = 0;
  for (int b = 0; b < scene->n_box; ++b) {
    for (int c = 0; c < P; ++c) obs_h[w++] = scene->box_c[b * P + c];
    for (int c = 0; c < P; ++c) obs_h[w++] = scene->box_h[b * P + c];
  }
  for (int q = 0; q < scene->n_sphere; ++q) {
    for (int c = 0; c < P; ++c) obs_h[w++] = scene->sph_c[q * P + c];
    obs_h[w++] = scene->sph_r[q] * scene->sph_r[q];
  }
  if (of > 0) {
    e = hipMemcpyAsync(pl->at<float>(pl->L.obs), obs_h, sizeof(float) * of,
                       hipMemcpyHostToDevice, pl->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(pl->stream);  // obs_h is pageable, freed below
  }
  std::free(obs_h);
  if (e != hipSuccess) {
    int rc = hip_fail(nullptr, e, "copy obstacles");
    pakr_plan_destroy(pl);
    return rc;
  }
  float x[12] = {0};
  for (int c = 0; c < d; ++c) x[c] = x_init[c];
  hipLaunchKernelGGL(k_init, dim3(1), dim3(NT), 0, pl->stream, pl->at<DevHeader>(pl->L.hdr),
                     pl->at<uint32_t>(pl->L.bar), G, pl->at<float>(pl->L.states),
                     pl->at<float>(pl->L.actions), pl->at<int>(pl->L.parents),
                     pl->at<float>(pl->L.costs), params->n_cap, d, m, x[0], x[1], x[2], x[3], x[4],
                     x[5], x[6], x[7], x[8], x[9], x[10], x[11], Q.c0);
  e = hipGetLastError();
  if (e != hipSuccess) {
    int rc = hip_fail(nullptr, e, "launch k_init");
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
  const size_t K = pl->P.K, B = pl->P.B, d = pl->P.d, m = pl->P.m;
  const size_t words = TRACE_HDR_WORDS + K * d + K + B * m + B * d + 3 * B;
  return words * 4 * (size_t)n_iters;
}

namespace {

int launch(pakr_plan* pl, long long max_iters, long long max_rounds, double budget_ms,
           int* trace, long long trace_iters) {
  if (pl->broken) return fail(pl, PAKR_E_DEVICE, "plan is unusable after a device error");
  KArgs a;
  std::memset(&a, 0, sizeof a);
  a.P = pl->P;
  a.hdr = pl->at<DevHeader>(pl->L.hdr);
  a.bar_flags = pl->at<uint32_t>(pl->L.bar);
  a.sols = pl->at<DevSolution>(pl->L.sols);
  a.path_states = pl->at<float>(pl->L.pstates);
  a.path_actions = pl->at<float>(pl->L.pactions);
  a.states = pl->at<float>(pl->L.states);
  a.actions = pl->at<float>(pl->L.actions);
  a.parents = pl->at<int>(pl->L.parents);
  a.costs = pl->at<float>(pl->L.costs);
  a.obs = pl->at<float>(pl->L.obs);
  a.partial = pl->at<unsigned long long>(pl->L.partial);
  a.stg = pl->at<float>(pl->L.stg);
  a.counts = pl->at<int>(pl->L.counts);
  a.goalmin = pl->at<unsigned long long>(pl->L.goalmin);
  a.trace = trace;
  a.trace_words = (long long)(pakr_trace_bytes(pl, 1) / 4);
  a.trace_iters = trace ? trace_iters : 0;
  a.max_iters = max_iters;
  a.max_rounds = max_rounds;
  a.budget_ticks = budget_ms > 0 ? (long long)(budget_ms * pl->ticks_per_ms) : 0;
  const double guard_ms = (budget_ms > 0 ? budget_ms : 0.0) + 60000.0;
  a.guard_ticks = (long long)(guard_ms * pl->ticks_per_ms);
  a.barrier_timeout_ticks = (long long)(2000.0 * pl->ticks_per_ms);
  void* args[] = {&a};
  hipError_t e = hipLaunchCooperativeKernel(pl->kfn, dim3(pl->G), dim3(NT), args,
                                            (unsigned)pl->shmem, pl->stream);
  if (e != hipSuccess) return hip_fail(pl, e, "cooperative launch");
  return PAKR_OK;
}

int sync_header(pakr_plan* pl, DevHeader* h) {
  hipError_t e = hipMemcpyAsync(h, pl->at<DevHeader>(pl->L.hdr), sizeof(DevHeader),
                                hipMemcpyDeviceToHost, pl->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(pl->stream);
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
  if (!(budget_ms > 0) && max_rounds <= 0 && max_iters <= 0)
    return fail(pl, PAKR_E_INVALID_ARG, "set a budget, a round limit or an iteration limit");
  if (std::isnan(budget_ms)) return fail(pl, PAKR_E_INVALID_ARG, "budget is NaN");
  return launch(pl, max_iters, max_rounds, budget_ms, nullptr, 0);
}

int pakr_status(pakr_plan* pl, pakr_stats* out) {
  if (!pl || !out) return PAKR_E_INVALID_ARG;
  DevHeader h;
  int rc = sync_header(pl, &h);
  if (rc != PAKR_OK) return rc;
  std::memset(out, 0, sizeof *out);
  out->n_nodes = h.n;
  out->round = h.round;
  out->iter = h.iter;
  out->status = h.status;
  out->n_solutions = h.n_solutions;
  out->grid = pl->G;
  out->total_iters = (long long)h.total_iters;
  out->expansions = (long long)h.expansions;
  out->insertions = (long long)h.insertions;
  out->nn_pairs = (long long)h.nn_pairs;
  out->c_best = std::isinf(h.c_best) ? INFINITY : (double)h.c_best;
  out->call_ms = (double)(h.t_end - h.t_start) / pl->ticks_per_ms;
  out->t_first_ms = h.t_first >= 0 ? (double)h.t_first / pl->ticks_per_ms : -1.0;
  out->t_last_ms = h.t_last >= 0 ? (double)h.t_last / pl->ticks_per_ms : -1.0;
  out->call_iters = h.call_iters;
  out->call_rounds = h.call_rounds;
  out->call_solutions = h.call_solutions;
  for (int i = 0; i < 6; ++i) out->step_ms[i] = (double)h.ticks[i] / pl->ticks_per_ms;
  out->nn_ms = out->step_ms[0] + out->step_ms[1];
  out->rollout_ms = out->step_ms[2] + out->step_ms[3] + out->step_ms[4];
  out->insert_ms = out->step_ms[5];
  return PAKR_OK;
}

int pakr_solutions(pakr_plan* pl, pakr_solution* out, int cap, int* n_total) {
  if (!pl || !n_total || cap < 0 || (cap > 0 && !out)) return PAKR_E_INVALID_ARG;
  DevHeader h;
  int rc = sync_header(pl, &h);
  if (rc != PAKR_OK) return rc;
  *n_total = h.n_solutions;
  const int n = std::min(std::min(cap, h.n_solutions), MAX_SOLUTIONS);
  if (n <= 0) return PAKR_OK;
  DevSolution* tmp = new (std::nothrow) DevSolution[n];
  if (!tmp) return fail(pl, PAKR_E_INVALID_ARG, "out of host memory");
  hipError_t e = hipMemcpy(tmp, pl->at<DevSolution>(pl->L.sols), sizeof(DevSolution) * n,
                           hipMemcpyDeviceToHost);
  if (e != hipSuccess) {
    delete[] tmp;
    return hip_fail(pl, e, "read solutions");
  }
  for (int i = 0; i < n; ++i) {
    out[i].round = tmp[i].round;
    out[i].iter = tmp[i].iter;
    out[i].node = tmp[i].node;
    out[i].n_nodes = tmp[i].n_nodes;
    out[i].total_iter = tmp[i].total_iter;
    out[i].cost = (double)tmp[i].cost;
    out[i].t_ms = (double)tmp[i].t / pl->ticks_per_ms;
  }
  delete[] tmp;
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
  const int ne = h.best_edges, d = pl->P.d, m = pl->P.m;
  *n_edges = ne;
  if (cost) *cost = (double)h.best_cost;
  if (h.path_truncated) return fail(pl, PAKR_E_BUFFER_TOO_SMALL, "path longer than max_path_edges");
  if (ne > cap_edges) return fail(pl, PAKR_E_BUFFER_TOO_SMALL, "cap_edges too small");
  if (!states || !actions) return fail(pl, PAKR_E_INVALID_ARG, "null output arrays");
  float* rs = new (std::nothrow) float[(size_t)(ne + 1) * d];
  float* ra = new (std::nothrow) float[(size_t)ne * m + 1];
  if (!rs || !ra) {
    delete[] rs;
    delete[] ra;
    return fail(pl, PAKR_E_INVALID_ARG, "out of host memory");
  }
  hipError_t e = hipMemcpy(rs, pl->at<float>(pl->L.pstates), sizeof(float) * (size_t)(ne + 1) * d,
                           hipMemcpyDeviceToHost);
  if (e == hipSuccess)
    e = hipMemcpy(ra, pl->at<float>(pl->L.pactions), sizeof(float) * (size_t)ne * m,
                  hipMemcpyDeviceToHost);
  if (e != hipSuccess) {
    delete[] rs;
    delete[] ra;
    return hip_fail(pl, e, "read path");
  }
  // stored goal first; return root first
  for (int k = 0; k <= ne; ++k)
    std::memcpy(states + (size_t)k * d, rs + (size_t)(ne - k) * d, sizeof(float) * d);
  for (int k = 0; k < ne; ++k)
    std::memcpy(actions + (size_t)k * m, ra + (size_t)(ne - 1 - k) * m, sizeof(float) * m);
  delete[] rs;
  delete[] ra;
  return PAKR_OK;
}

int pakr_copy_tree(pakr_plan* pl, float* states, float* actions, int* parents, float* costs,
                   int n_max, int* n_out) {
  if (!pl || !n_out || n_max < 0) return PAKR_E_INVALID_ARG;
  DevHeader h;
  int rc = sync_header(pl, &h);
  if (rc != PAKR_OK) return rc;
  *n_out = h.n;
  const int n = std::min(h.n, n_max);
  const int d = pl->P.d, m = pl->P.m;
  const size_t N = (size_t)pl->P.n_cap;
  hipError_t e = hipSuccess;
  if (n > 0 && (states || actions)) {
    float* tmp = new (std::nothrow) float[(size_t)n];
    if (!tmp) return fail(pl, PAKR_E_INVALID_ARG, "out of host memory");
    for (int c = 0; c < d && states && e == hipSuccess; ++c) {
      e = hipMemcpy(tmp, pl->at<float>(pl->L.states) + (size_t)c * N, sizeof(float) * n,
                    hipMemcpyDeviceToHost);
      for (int i = 0; i < n; ++i) states[(size_t)i * d + c] = tmp[i];
    }
    for (int c = 0; c < m && actions && e == hipSuccess; ++c) {
      e = hipMemcpy(tmp, pl->at<float>(pl->L.actions) + (size_t)c * N, sizeof(float) * n,
                    hipMemcpyDeviceToHost);
      for (int i = 0; i < n; ++i) actions[(size_t)i * m + c] = tmp[i];
    }
    delete[] tmp;
  }
  if (e == hipSuccess && n > 0 && parents)
    e = hipMemcpy(parents, pl->at<int>(pl->L.parents), sizeof(int) * n, hipMemcpyDeviceToHost);
  if (e == hipSuccess && n > 0 && costs)
    e = hipMemcpy(costs, pl->at<float>(pl->L.costs), sizeof(float) * n, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(pl, e, "read tree");
  return PAKR_OK;
}

const char* pakr_last_error(const pakr_plan* pl) {
  return pl ? pl->err.c_str() : g_init_error.c_str();
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

}  // extern "C"
