// Device-side building blocks of the PAKR planner for gfx950: the problem
// record, Philox draws, system dynamics, RK4 and the per-state validity test.
// float32 throughout.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/pakr.h"

namespace pakr {

constexpr int NT = 512;          // threads per workgroup (eight wave64s)
constexpr int TILE = 64;         // tree nodes per NN tile (unit of ownership)
// Targets per NN chunk: QT per thread in TPG = NT / NG threads, at most 1024.
template <int QT>
constexpr int NN_KC = QT * NT < 1024 ? QT * NT : 1024;
constexpr int WAVE = 64;
// Decision margins at or below this (relative to max(1, bound) for the prune,
// absolute for the goal radius) are counted as near ties.
constexpr float NEAR_TIE = 1e-5f;
constexpr int MAX_SOLUTIONS = 1024;
constexpr int MAX_GR = 1024;     // rollout workgroups per iteration
constexpr int MAX_TIERS = 6;     // sub-grid tiers of the tree (grids 32 .. 1024 doubling)
constexpr int VAL_FLOATS = 32;   // validity record held in LDS (see load_validity)

enum : int { F_VALID = 1, F_PRUNE_OK = 2, F_KEEP = 4, F_GOAL = 8 };
enum : int { END_NONE = 0, END_GOAL = 1, END_TREE_FULL = 2, END_ITER_CAP = 3 };
constexpr int TRACE_HDR_WORDS = 16;

// Everything a kernel needs to know about one query; passed by value.
struct DevProblem {
  int system, d, m, npos;
  int B, A, K, T;
  int n_cap, cost_kind, h_kind, max_iters_per_round;
  int n_box, n_sph, G, G_roll;
  int max_path_edges, obs_floats;
  int lanes, cpb;                  // lanes per candidate, candidates per rollout workgroup
  int nn_tpg;                     // NN: threads per node group (NT / TPG groups)
  int spec_tiles;                 // tiles each idle workgroup scans ahead in phase 2 (0: none)
  int tier0_nodes;                // workgroup 0 plans alone while the tree has <= this many nodes
  // then the first tier_grid[k] workgroups while it has <= tier_nodes[k] (both ascending;
  // unused entries 0); beyond the last bound the whole grid
  int tier_nodes[MAX_TIERS];
  int tier_grid[MAX_TIERS];
  int pad_t;
  uint32_t key0, key1;
  float dt, h_speed, c0, vnorm_max;
  float goal_r, goal_r2, edge_duration, pad0;
  float dyn[8];
  float sample_lo[PAKR_MAX_D], sample_hi[PAKR_MAX_D];
  float lim_lo[PAKR_MAX_D], lim_hi[PAKR_MAX_D];
  float u_lo[PAKR_MAX_M], u_hi[PAKR_MAX_M];
  float ws_lo[3], ws_hi[3], goal_c[3], pad1[3];
};

// Loop state and per-call results; lives at the start of the workspace.
struct DevHeader {
  int n, round, iter, n_solutions;           // persistent loop state
  float c_best;
  int status;                                // pakr_status_bits of the last call
  uint32_t bar_gen;                          // grid-barrier generation counter
  int err;                                   // nonzero after a barrier timeout
  unsigned long long total_iters, expansions, insertions, nn_pairs;
  long long t_start, t_end, t_first, t_last; // device wall-clock ticks of the last call
  int call_iters, call_rounds, call_solutions, path_truncated;
  int best_edges, best_node, pad0, pad1;
  float best_cost, pad2, pad3, pad4;
  uint32_t release;                          // barrier release word
  // hand-off of the loop from workgroup 0 (alone while the tree is in the
  // first tier) to the grid: word ((iterations done + 1) << 1 | call ended),
  // then the loop state that the resuming workgroups adopt
  // ((iterations done + 1) << 32 | workgroups of the tier that starts << 1 | call ended)
  unsigned long long join;
  int ho_rounds, ho_status;
  uint32_t ho_gen;
  long long ticks[8];                        // per-step device time of the last call
  // candidates whose prune or goal decision lay within the near-tie band
  // (since initialisation; added by the rollout waves that saw one)
  unsigned long long near_prune, near_goal;
};

struct DevSolution {
  int round, iter, node, n_nodes;
  long long total_iter;
  float cost;
  int pad;
  long long t;
};

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                              uint32_t k0, uint32_t k1, uint32_t out[4]) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t hi0 = __umulhi(0xD2511F53u, c0), lo0 = 0xD2511F53u * c0;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2), lo1 = 0xCD9E8D57u * c2;
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

// u32 -> [lo, hi]: top 24 bits scaled exactly to [0,1), then lo + (hi-lo)*u
// with one float32 rounding per operation (no contraction into an FMA).
__device__ __forceinline__ float draw_range(uint32_t x, float lo, float hi) {
#pragma clang fp contract(off)
  const float u = (float)(x >> 8) * 5.9604644775390625e-08f;
  const float w = hi - lo;
  const float p = w * u;
  return lo + p;
}

enum : uint32_t { TAG_STATE = 0u, TAG_CONTROL = 1u };

// SampleStates: target k of iteration `it` of round `rd`.
template <int D>
__device__ __forceinline__ void sample_state(const DevProblem& P, uint32_t k, uint32_t it,
                                             uint32_t rd, float* q) {
#pragma unroll
  for (int blk = 0; blk * 4 < D; ++blk) {
    uint32_t r[4];
    philox4x32_10(k, it, rd, (TAG_STATE << 16) | (uint32_t)blk, P.key0, P.key1, r);
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      const int c = blk * 4 + w;
      if (c < D) q[c] = draw_range(r[w], P.sample_lo[c], P.sample_hi[c]);
    }
  }
}

// SampleControls: branch a of parent query k.
template <int M>
__device__ __forceinline__ void sample_control(const DevProblem& P, uint32_t k, uint32_t a,
                                               uint32_t it, uint32_t rd, float* u) {
  uint32_t r[4];
  philox4x32_10(k, it, rd, (TAG_CONTROL << 16) | a, P.key0, P.key1, r);
#pragma unroll
  for (int c = 0; c < M; ++c) u[c] = draw_range(r[c], P.u_lo[c], P.u_hi[c]);
}

// ---------------------------------------------------------------------------
// Systems.  Sizes are compile-time so every state lives in registers.
// ---------------------------------------------------------------------------
template <int SYS> struct Sys;
// D state dims, M controls, P position dims, CH steps per collision sweep
// (4 where f takes two or more sincos: a longer sweep spills in the batched
// kernel, which holds every system's loop).
template <> struct Sys<PAKR_DI2> { static constexpr int D = 4, M = 2, P = 2, CH = 8; };
template <> struct Sys<PAKR_DI3> { static constexpr int D = 6, M = 3, P = 3, CH = 8; };
template <> struct Sys<PAKR_CAR> { static constexpr int D = 5, M = 2, P = 2, CH = 8; };
template <> struct Sys<PAKR_QUAD> { static constexpr int D = 12, M = 4, P = 3, CH = 4; };
template <> struct Sys<PAKR_DUBINS> { static constexpr int D = 6, M = 3, P = 3, CH = 4; };
template <> struct Sys<PAKR_UNI1> { static constexpr int D = 3, M = 2, P = 2, CH = 8; };
template <> struct Sys<PAKR_UNI2> { static constexpr int D = 5, M = 2, P = 2, CH = 8; };
template <> struct Sys<PAKR_ACROBOT> { static constexpr int D = 4, M = 1, P = 2, CH = 8; };
template <> struct Sys<PAKR_CARTPOLE> { static constexpr int D = 4, M = 1, P = 2, CH = 8; };

// The trigonometric values f needs at one state: the car's heading sine and
// cosine and steering tangent, the quadrotor's roll, pitch and yaw sines and
// cosines, the Dubins airplane's yaw and pitch sines and cosines, the
// unicycles' heading and the cart-pole's pole angle sine and cosine, the
// acrobot's two joint angles and their sum.  Computed once per evaluation (and, in the adjoint, shared between
// an RK4 stage's evaluation of f and its vector-Jacobian product).
struct Trig {
  float s[3], c[3], t;
};

// The planner's sines and cosines come from the hardware v_sin_f32 /
// v_cos_f32 (the angle scaled to revolutions; absolute error about 1e-6 at
// these angles, a few 1e-6 m in an edge's end position against the FP64
// reference, below the 1e-5 decision band and the 1e-4 state bar) rather
// than the correctly rounded library sincos, whose range reduction makes the
// rollout's serial chain several times longer on the trigonometric systems.
__device__ __forceinline__ void hw_sincos(float a, float* s, float* c) {
  *s = __sinf(a);
  *c = __cosf(a);
}

template <int SYS>
__device__ __forceinline__ Trig trig_of(const float* x) {
  Trig g;
  if constexpr (SYS == PAKR_CAR) {
    hw_sincos(x[2], &g.s[0], &g.c[0]);
    float sp, cp;
    hw_sincos(x[4], &sp, &cp);
    g.t = sp * __builtin_amdgcn_rcpf(cp);  // tan of the steering angle (|phi| <= 0.6)
  } else if constexpr (SYS == PAKR_QUAD) {
#pragma unroll
    for (int k = 0; k < 3; ++k) hw_sincos(x[3 + k], &g.s[k], &g.c[k]);
  } else if constexpr (SYS == PAKR_DUBINS) {
    hw_sincos(x[3], &g.s[0], &g.c[0]);
    hw_sincos(x[4], &g.s[1], &g.c[1]);
  } else if constexpr (SYS == PAKR_UNI1 || SYS == PAKR_UNI2) {
    hw_sincos(x[2], &g.s[0], &g.c[0]);
  } else if constexpr (SYS == PAKR_CARTPOLE) {
    hw_sincos(x[1], &g.s[0], &g.c[0]);
  } else if constexpr (SYS == PAKR_ACROBOT) {
    hw_sincos(x[0], &g.s[0], &g.c[0]);
    hw_sincos(x[1], &g.s[1], &g.c[1]);
    g.s[2] = g.s[0] * g.c[1] + g.c[0] * g.s[1];  // angle sum
    g.c[2] = g.c[0] * g.c[1] - g.s[0] * g.s[1];
  }
  return g;
}

// The acrobot's mass matrix (symmetric, a function of the elbow angle), the
// right-hand side r = (0, tau) - c - g and the joint accelerations M^-1 r;
// dyn = (m1, m2, l1, lc1, lc2, I1, I2, gravity).
struct AcrobotTerms {
  float m00, m01, m11, inv_det, r0, r1, a1, a2;
};

__device__ __forceinline__ AcrobotTerms acrobot_terms(const DevProblem& P, const float* x,
                                                      float tau, const Trig& tg) {
  const float m1 = P.dyn[0], m2 = P.dyn[1], l1 = P.dyn[2], lc1 = P.dyn[3];
  const float lc2 = P.dyn[4], I1 = P.dyn[5], I2 = P.dyn[6], g = P.dyn[7];
  const float k = m2 * l1 * lc2;
  const float b = m2 * lc2 * lc2 + I2;
  const float v1 = x[2], v2 = x[3];
  AcrobotTerms t;
  t.m00 = m1 * lc1 * lc1 + m2 * l1 * l1 + b + I1 + 2.0f * k * tg.c[1];
  t.m01 = b + k * tg.c[1];
  t.m11 = b;
  const float g2 = m2 * lc2 * g * tg.s[2];
  const float g1 = (m1 * lc1 + m2 * l1) * g * tg.s[0] + g2;
  t.r0 = k * tg.s[1] * (v2 * v2 + 2.0f * v1 * v2) - g1;
  t.r1 = tau - k * tg.s[1] * v1 * v1 - g2;
  t.inv_det = 1.0f / (t.m00 * t.m11 - t.m01 * t.m01);
  t.a1 = (t.m11 * t.r0 - t.m01 * t.r1) * t.inv_det;
  t.a2 = (t.m00 * t.r1 - t.m01 * t.r0) * t.inv_det;
  return t;
}

// x' = f(x, u), Eq. (1), given the state's trigonometric values.
template <int SYS>
__device__ __forceinline__ void dynamics_trig(const DevProblem& P, const float* x, const float* u,
                                              const Trig& tg, float* xd) {
  if constexpr (SYS == PAKR_DI2 || SYS == PAKR_DI3) {
    constexpr int Dp = Sys<SYS>::P;
#pragma unroll
    for (int a = 0; a < Dp; ++a) {
      xd[a] = x[Dp + a];
      xd[Dp + a] = u[a];
    }
  } else if constexpr (SYS == PAKR_CAR) {
    const float s = tg.s[0], c = tg.c[0];
    const float v = x[3];
    xd[0] = v * c;
    xd[1] = v * s;
    xd[2] = v * tg.t * (1.0f / P.dyn[0]);
    xd[3] = u[0];
    xd[4] = u[1];
  } else if constexpr (SYS == PAKR_DUBINS) {
    // state (p, yaw, pitch, speed); the controls drive yaw, pitch and speed
    const float v = x[5];
    const float vc = v * tg.c[1];
    xd[0] = vc * tg.c[0];
    xd[1] = vc * tg.s[0];
    xd[2] = v * tg.s[1];
    xd[3] = u[0];
    xd[4] = u[1];
    xd[5] = u[2];
  } else if constexpr (SYS == PAKR_UNI1) {
    // state (p, heading); controls (speed, turn rate)
    xd[0] = u[0] * tg.c[0];
    xd[1] = u[0] * tg.s[0];
    xd[2] = u[1];
  } else if constexpr (SYS == PAKR_UNI2) {
    // state (p, heading, speed, turn rate); controls accelerate both
    xd[0] = x[3] * tg.c[0];
    xd[1] = x[3] * tg.s[0];
    xd[2] = x[4];
    xd[3] = u[0];
    xd[4] = u[1];
  } else if constexpr (SYS == PAKR_ACROBOT) {
    // M(q) q'' = (0, tau) - c(q, q') - g(q): two rigid links, elbow torque
    const AcrobotTerms t = acrobot_terms(P, x, u[0], tg);
    xd[0] = x[2];
    xd[1] = x[3];
    xd[2] = t.a1;
    xd[3] = t.a2;
  } else if constexpr (SYS == PAKR_CARTPOLE) {
    // point-mass pole on a cart whose acceleration is the control
    const float l = P.dyn[0], g = P.dyn[1];
    xd[0] = x[2];
    xd[1] = x[3];
    xd[2] = u[0];
    xd[3] = (g * tg.s[0] - u[0] * tg.c[0]) / l;
  } else {
    static_assert(SYS == PAKR_QUAD, "unknown system");
    // quadrotor, Z-Y-X Euler angles; body-frame velocity (ub,vb,wb), rates (p,q,r)
    const float inv_m = 1.0f / P.dyn[0], g = P.dyn[1];
    const float Ix = P.dyn[2], Iy = P.dyn[3], Iz = P.dyn[4];
    const float iIx = P.dyn[5], iIy = P.dyn[6], iIz = P.dyn[7];  // 1 / inertia
    const float sph = tg.s[0], cph = tg.c[0], sth = tg.s[1], cth = tg.c[1];
    const float sps = tg.s[2], cps = tg.c[2];
    const float ub = x[6], vb = x[7], wb = x[8];
    const float p = x[9], q = x[10], r = x[11];
    // rotation body -> world, R = Rz(yaw) Ry(pitch) Rx(roll)
    const float r00 = cps * cth, r01 = cps * sth * sph - sps * cph, r02 = cps * sth * cph + sps * sph;
    const float r10 = sps * cth, r11 = sps * sth * sph + cps * cph, r12 = sps * sth * cph - cps * sph;
    const float r20 = -sth, r21 = cth * sph, r22 = cth * cph;
    xd[0] = r00 * ub + r01 * vb + r02 * wb;
    xd[1] = r10 * ub + r11 * vb + r12 * wb;
    xd[2] = r20 * ub + r21 * vb + r22 * wb;
    const float inv_cth = __builtin_amdgcn_rcpf(cth);  // hardware reciprocal, 1 ulp
    const float qs_rc = q * sph + r * cph;
    xd[3] = p + qs_rc * sth * inv_cth;
    xd[4] = q * cph - r * sph;
    xd[5] = qs_rc * inv_cth;
    // v_b' = -w x v_b + R^T (0,0,-g) + (0,0,thrust/m)
    xd[6] = -(q * wb - r * vb) - g * r20;
    xd[7] = -(r * ub - p * wb) - g * r21;
    xd[8] = -(p * vb - q * ub) - g * r22 + u[0] * inv_m;
    // w' = I^-1 (tau - w x I w)
    xd[9] = (u[1] - (Iz - Iy) * q * r) * iIx;
    xd[10] = (u[2] - (Ix - Iz) * r * p) * iIy;
    xd[11] = (u[3] - (Iy - Ix) * p * q) * iIz;
  }
}

// x' = f(x, u), Eq. (1).
template <int SYS>
__device__ __forceinline__ void dynamics(const DevProblem& P, const float* x, const float* u,
                                         float* xd) {
  dynamics_trig<SYS>(P, x, u, trig_of<SYS>(x), xd);
}

// One classical RK4 step with the control held (Sec. IV-A).
template <int SYS>
__device__ __forceinline__ void rk4_step(const DevProblem& P, float* x, const float* u, float h) {
  constexpr int D = Sys<SYS>::D;
  if constexpr (SYS == PAKR_DI2 || SYS == PAKR_DI3) {
    // Double integrator: x' = A x + B u with A nilpotent (A^2 = 0), so the
    // four stages combine to p + h v + (h^2/2) u, v + h u -- the RK4 map
    // written out (RK4 reproduces the quadratic flow exactly), 3 FMAs per axis
    // instead of the stage sums.
    constexpr int NP = D / 2;
    const float h2 = 0.5f * h * h;
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      x[i] = x[i] + h * x[NP + i] + h2 * u[i];
      x[NP + i] = x[NP + i] + h * u[i];
    }
    return;
  }
  float k1[D], k2[D], k3[D], k4[D], t[D];
  const float hh = 0.5f * h;
  dynamics<SYS>(P, x, u, k1);
#pragma unroll
  for (int i = 0; i < D; ++i) t[i] = x[i] + hh * k1[i];
  dynamics<SYS>(P, t, u, k2);
#pragma unroll
  for (int i = 0; i < D; ++i) t[i] = x[i] + hh * k2[i];
  dynamics<SYS>(P, t, u, k3);
#pragma unroll
  for (int i = 0; i < D; ++i) t[i] = x[i] + h * k3[i];
  dynamics<SYS>(P, t, u, k4);
  const float h6 = h * (1.0f / 6.0f);
#pragma unroll
  for (int i = 0; i < D; ++i) x[i] = x[i] + h6 * (k1[i] + 2.0f * (k2[i] + k3[i]) + k4[i]);
}

// The validity constants of a query, copied to LDS once per launch:
// [0,3) workspace lo, [3,6) workspace hi, [6,18) state lower limits,
// [18,30) upper limits, [30] squared speed bound (+inf when none).
__device__ __forceinline__ void load_validity(const DevProblem& P, float* s_val, int tid) {
  if (tid < 3) {
    s_val[tid] = P.ws_lo[tid];
    s_val[3 + tid] = P.ws_hi[tid];
  }
  if (tid < PAKR_MAX_D) {
    s_val[6 + tid] = P.lim_lo[tid];
    s_val[18 + tid] = P.lim_hi[tid];
  }
  if (tid == 0) s_val[30] = P.vnorm_max > 0.0f ? P.vnorm_max * P.vnorm_max : INFINITY;
}

// Workspace box and state limits of one state (no obstacles); branch free.
// NaN compares false and so is invalid.
template <int SYS>
__device__ __forceinline__ bool limits_ok(const float* s_val, const float* x) {
  constexpr int D = Sys<SYS>::D, NP = Sys<SYS>::P;
  bool ok = true;
#pragma unroll
  for (int c = 0; c < NP; ++c) ok = ok & (x[c] >= s_val[c]) & (x[c] <= s_val[3 + c]);
#pragma unroll
  for (int i = NP; i < D; ++i) ok = ok & (x[i] >= s_val[6 + i]) & (x[i] <= s_val[18 + i]);
  if constexpr (SYS == PAKR_DI2 || SYS == PAKR_DI3) {
    float s2 = 0.0f;
#pragma unroll
    for (int c = 0; c < NP; ++c) s2 += x[NP + c] * x[NP + c];
    ok = ok & (s2 <= s_val[30]);
  }
  return ok;
}

// True if any of CH positions lies in a closed obstacle.  Obstacles sit in
// LDS: boxes first as (c[NP], h[NP]) records, then spheres as (c[NP], r^2).
// This lane tests obstacles first, first + stride, ...; NaN coordinates
// never hit (limits_ok rejects them).
template <int NP, int CH>
__device__ __forceinline__ bool any_obstacle_hit(const float (&pos)[CH][NP], const float* s_obs,
                                                 int nb, int ns, int first, int stride) {
  bool hit = false;
  for (int b = first; b < nb; b += stride) {
    const float* o = s_obs + b * (2 * NP);
    float oc[NP], oh[NP];
#pragma unroll
    for (int c = 0; c < NP; ++c) {
      oc[c] = o[c];
      oh[c] = o[NP + c];
    }
#pragma unroll
    for (int s = 0; s < CH; ++s) {
      bool inside = true;
#pragma unroll
      for (int c = 0; c < NP; ++c) inside = inside & (fabsf(pos[s][c] - oc[c]) <= oh[c]);
      hit = hit | inside;
    }
  }
  const float* sp = s_obs + nb * (2 * NP);
  for (int q = first; q < ns; q += stride) {
    const float* o = sp + q * (NP + 1);
    float oc[NP];
#pragma unroll
    for (int c = 0; c < NP; ++c) oc[c] = o[c];
    const float r2 = o[NP];
#pragma unroll
    for (int s = 0; s < CH; ++s) {
      float d2 = 0.0f;
#pragma unroll
      for (int c = 0; c < NP; ++c) {
        const float e = pos[s][c] - oc[c];
        d2 += e * e;
      }
      hit = hit | (d2 <= r2);
    }
  }
  return hit;
}

// One double-integrator edge shared by the L lanes of its candidate.  The RK4
// map of these systems is their exact flow (rk4_step), so the state after s
// steps is p0 + t v0 + (t^2/2) u, v0 + t u at t = s h: any lane can evaluate
// any sub-step directly, and the same expression gives the same bits in every
// lane.  Lane lg takes sub-steps s = 1 + (lg mod LS), then every LS-th, in
// chunks of CH (a chunk past T repeats its first sub-step), and tests them
// against obstacles lg / LS, then every (L / LS)-th; the caller ORs the lanes'
// verdicts.  With the path-length cost every lane sums all T segment lengths
// in step order, so neither the cost nor the verdict depends on the split.
// On return x holds the state after T steps; `bad` is set if a tested
// sub-step leaves the limits or hits an obstacle.
template <int SYS, int CH>
__device__ __forceinline__ void di_edge(const DevProblem& P, const float* s_val, const float* s_obs,
                                        float* x, const float* u, int lg, int L, int LS,
                                        bool path_len, float& len, bool& bad) {
  constexpr int D = Sys<SYS>::D, NP = D / 2;
  const float h = P.dt;
  const int T = P.T;
  auto state_at = [&](int s, float* xs) {
    const float t = (float)s * h, th = 0.5f * t * t;
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      xs[i] = x[i] + t * x[NP + i] + th * u[i];
      xs[NP + i] = x[NP + i] + t * u[i];
    }
  };
  const int ls = lg & (LS - 1), lo = lg / LS, LO = L / LS;
  bool ok = true, hit = false;
  for (int s0 = ls + 1; s0 <= T; s0 += CH * LS) {
    float pos[CH][NP];
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int s = s0 + c * LS <= T ? s0 + c * LS : s0;
      float xs[D];
      state_at(s, xs);
      ok = ok & limits_ok<SYS>(s_val, xs);
#pragma unroll
      for (int k = 0; k < NP; ++k) pos[c][k] = xs[k];
    }
    hit = hit | any_obstacle_hit<NP, CH>(pos, s_obs, P.n_box, P.n_sph, lo, LO);
  }
  if (path_len) {
    float prev[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) prev[k] = x[k];
    for (int s = 1; s <= T; ++s) {
      float xs[D];
      state_at(s, xs);
      float s2 = 0.0f;
#pragma unroll
      for (int k = 0; k < NP; ++k) {
        const float e = xs[k] - prev[k];
        s2 += e * e;
        prev[k] = xs[k];
      }
      len += __builtin_amdgcn_sqrtf(s2);  // v_sqrt_f32 (1 ulp)
    }
  }
  float xe[D];
  state_at(T, xe);
#pragma unroll
  for (int i = 0; i < D; ++i) x[i] = xe[i];
  bad = hit | !ok;
}

constexpr int DI_CH = 5;  // sub-steps per lane and obstacle sweep in di_edge

// Per-lane work of di_edge with LS sub-step groups (instructions, roughly:
// each evaluated sub-step ~16 for its state and limits, each obstacle test
// ~11, chunks of ch sub-steps counted whole).  The kernel picks the LS with
// the least; the host prices the rollout phase with it.
__host__ __device__ inline long long di_lane_cost(int T, int L, int n_obs, int ls, int ch) {
  const int lo = L / ls;
  const long long steps = (long long)(((T + ls - 1) / ls + ch - 1) / ch) * ch;
  return steps * (16 + 11 * ((n_obs + lo - 1) / lo));
}

// Sub-step groups LS (a power of two dividing L) for di_edge.
template <int CH>
__device__ __forceinline__ int di_step_groups(const DevProblem& P, int L) {
  int best_ls = 1;
  long long best = LLONG_MAX;
  for (int ls = 1; ls <= L; ls <<= 1) {
    const long long c = di_lane_cost(P.T, L, P.n_box + P.n_sph, ls, CH);
    if (c < best) {
      best = c;
      best_ls = ls;
    }
  }
  return best_ls;
}

template <int SYS>
__device__ __forceinline__ float goal_dist2(const DevProblem& P, const float* x) {
  constexpr int NP = Sys<SYS>::P;
  float s2 = 0.0f;
#pragma unroll
  for (int c = 0; c < NP; ++c) {
    const float e = x[c] - P.goal_c[c];
    s2 += e * e;
  }
  return s2;
}

// h(x) of the prune test.
template <int SYS>
__device__ __forceinline__ float heuristic(const DevProblem& P, float dist) {
  if (P.h_kind == PAKR_H_NONE) return 0.0f;
  if (P.h_kind == PAKR_H_PAPER_LITERAL) return dist;
  float gap = fmaxf(dist - P.goal_r, 0.0f);
  if (P.cost_kind == PAKR_COST_DURATION) gap = gap / P.h_speed;
  return gap;
}

}  // namespace pakr
