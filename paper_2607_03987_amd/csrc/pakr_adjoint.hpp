// Trajectory refinement on gfx950: a float32 rollout of a piecewise-constant
// control sequence (one control per tree edge, held for T RK4 steps as in the
// planner, Sec. IV-A) with a smooth objective, and its hand-written adjoint.
//
//   J = w_u * sum_e T*dt * |(u_e - u_ref) / u_scale|^2
//     + w_g * |pos(x_N) - goal|^2
//     + w_c * sum_{n=1..N} pen(x_n),
//   pen(x) = sum_obstacles sp(delta - sd(pos)) + sp over the workspace box,
//            the finite state limits and the speed bound,
//   sp(z)  = log(1 + exp(beta z)) / beta.
//
// The forward pass stores every step's state (per-step checkpoints); the
// backward pass walks the steps in reverse, recomputes that step's four RK4
// stages from its checkpoint and pushes the adjoint through them with the
// vector-Jacobian products of f written out per system.
//
// One wavefront per trajectory: the rollout itself is a serial chain, so every
// lane integrates the same state, and the obstacle terms (the bulk of each
// step) are split across the 64 lanes and summed with a wave reduction.
#pragma once

#include "pakr_device.hpp"

namespace pakr {

struct RefineParams {
  float w_u, w_g, w_c, beta, delta, inv_beta;
  float u_ref[PAKR_MAX_M], u_scale[PAKR_MAX_M];
};

struct TrajArgs {
  DevProblem P;        // system, scene sizes, T, dt, goal, limits (the planner's record)
  RefineParams R;
  const float* obs;    // packed obstacles, as for the planner
  int n_traj, M;       // trajectories, edges per trajectory
  const float* x0;     // [n_traj][d]
  const float* U;      // [n_traj][M][m]
  float* ckpt;         // [n_traj][M*T + 1][d]
  float* J;            // [n_traj]
  const float* gJ;     // [n_traj]
  float* gU;           // [n_traj][M][m]
  int* ok;             // [n_traj] bit 0: every sub-step valid, bit 1: final state in the goal
  float* cost;         // [n_traj] the planner's cost of the trajectory
};

// softplus_beta(z) = log(1 + exp(beta z)) / beta and its derivative
// sigmoid(beta z).  A term with beta z < SP_CUT is taken as zero (its value is
// below e^-30 / beta), so inactive terms cost a compare: for the state-bound
// terms, which every lane evaluates on the same state, the branch is uniform.
// The hardware exp2 / log2 (v_exp_f32, v_log_f32, a few ulp) stand in for the
// library exp / log1p: log(1 + e) loses e's last bits only when e is below the
// float epsilon, i.e. for terms under 1e-7 / beta, and these penalties sit on
// the rollout's serial chain.  For the same reason the signed distances use
// the hardware square root and reciprocal (v_sqrt_f32, v_rcp_f32, 1 ulp).
constexpr float SP_CUT = -30.0f;

__device__ __forceinline__ float softplus_b(float z, const RefineParams& R) {
  const float bz = R.beta * z;
  if (bz < SP_CUT) return 0.0f;
  return bz > 0.0f ? z + __logf(1.0f + __expf(-bz)) * R.inv_beta
                    : __logf(1.0f + __expf(bz)) * R.inv_beta;
}

__device__ __forceinline__ float sigmoid_b(float z, const RefineParams& R) {
  const float bz = R.beta * z;
  if (bz < SP_CUT) return 0.0f;
  return __frcp_rn(1.0f + __expf(-bz));
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Obstacle part of pen(x) over obstacles first, first+stride, ... and, with
// grad != nullptr, its gradient with respect to the position (added to grad).
template <int NP>
__device__ __forceinline__ float obstacle_penalty(const DevProblem& P, const RefineParams& R,
                                                  const float* s_obs, const float* x, float* grad,
                                                  int first, int stride) {
  float pen = 0.0f;
  for (int b = first; b < P.n_box; b += stride) {
    const float* o = s_obs + b * (2 * NP);
    float q[NP], sg[NP], outside = 0.0f, inner = 0.0f;
    int arg = 0;
#pragma unroll
    for (int c = 0; c < NP; ++c) {
      const float e = x[c] - o[c];
      sg[c] = e >= 0.0f ? 1.0f : -1.0f;
      q[c] = fabsf(e) - o[NP + c];
      const float qp = q[c] >= 0.0f ? q[c] : 0.0f;
      outside += qp * qp;
      if (c == 0 || q[c] > inner) {
        inner = q[c];
        arg = c;
      }
    }
    // signed distance to the box: outside part plus (inside) the largest face gap
    const float so = outside > 0.0f ? __builtin_amdgcn_sqrtf(outside) : 0.0f;
    const float sd = so + (inner < 0.0f ? inner : 0.0f);
    pen += softplus_b(R.delta - sd, R);
    if (grad) {
      const float dsd = -sigmoid_b(R.delta - sd, R);
#pragma unroll
      for (int c = 0; c < NP; ++c) {
        float dq = 0.0f;
        if (so > 0.0f && q[c] > 0.0f) dq += q[c] * __builtin_amdgcn_rcpf(so);
        if (inner < 0.0f && c == arg) dq += 1.0f;
        grad[c] += dsd * dq * sg[c];
      }
    }
  }
  const float* sp = s_obs + P.n_box * (2 * NP);
  for (int s = first; s < P.n_sph; s += stride) {
    const float* o = sp + s * (NP + 1);
    float e[NP], r2 = 0.0f;
#pragma unroll
    for (int c = 0; c < NP; ++c) {
      e[c] = x[c] - o[c];
      r2 += e[c] * e[c];
    }
    const float dist = __builtin_amdgcn_sqrtf(r2);
    const float sd = dist - __builtin_amdgcn_sqrtf(o[NP]);  // the record holds r^2
    pen += softplus_b(R.delta - sd, R);
    if (grad && dist > 0.0f) {
      const float dsd = -sigmoid_b(R.delta - sd, R) * __builtin_amdgcn_rcpf(dist);
#pragma unroll
      for (int c = 0; c < NP; ++c) grad[c] += dsd * e[c];
    }
  }
  return pen;
}

// Bound part of pen(x): workspace box, finite state limits, speed bound.
template <int SYS>
__device__ __forceinline__ float bound_penalty(const DevProblem& P, const RefineParams& R,
                                               const float* s_val, const float* x, float* grad) {
  constexpr int D = Sys<SYS>::D, NP = Sys<SYS>::P;
  float pen = 0.0f;
#pragma unroll
  for (int c = 0; c < NP; ++c) {
    pen += softplus_b(x[c] - s_val[3 + c], R) + softplus_b(s_val[c] - x[c], R);
    if (grad) grad[c] += sigmoid_b(x[c] - s_val[3 + c], R) - sigmoid_b(s_val[c] - x[c], R);
  }
#pragma unroll
  for (int i = NP; i < D; ++i) {
    const float lo = s_val[6 + i], hi = s_val[18 + i];
    if (hi < INFINITY) {
      pen += softplus_b(x[i] - hi, R);
      if (grad) grad[i] += sigmoid_b(x[i] - hi, R);
    }
    if (lo > -INFINITY) {
      pen += softplus_b(lo - x[i], R);
      if (grad) grad[i] -= sigmoid_b(lo - x[i], R);
    }
  }
  if constexpr (SYS == PAKR_DI2 || SYS == PAKR_DI3) {
    if (P.vnorm_max > 0.0f) {
      float v2 = 0.0f;
#pragma unroll
      for (int c = 0; c < NP; ++c) v2 += x[NP + c] * x[NP + c];
      const float vn = __builtin_amdgcn_sqrtf(v2);
      pen += softplus_b(vn - P.vnorm_max, R);
      if (grad && vn > 0.0f) {
        const float g = sigmoid_b(vn - P.vnorm_max, R) * __builtin_amdgcn_rcpf(vn);
#pragma unroll
        for (int c = 0; c < NP; ++c) grad[NP + c] += g * x[NP + c];
      }
    }
  }
  return pen;
}

// pen(x) for the whole wave (every lane receives the total).
template <int SYS>
__device__ __forceinline__ float wave_penalty(const DevProblem& P, const RefineParams& R,
                                              const float* s_obs, const float* s_val,
                                              const float* x, int lane) {
  constexpr int NP = Sys<SYS>::P;
  const float part = obstacle_penalty<NP>(P, R, s_obs, x, nullptr, lane, WAVE);
  const float obs = __ballot(part != 0.0f) != 0ull ? wave_sum(part) : 0.0f;
  return obs + bound_penalty<SYS>(P, R, s_val, x, nullptr);
}

// d pen / dx for the whole wave, added to g on every lane.
template <int SYS>
__device__ __forceinline__ void wave_penalty_grad(const DevProblem& P, const RefineParams& R,
                                                  const float* s_obs, const float* s_val,
                                                  const float* x, int lane, float* g) {
  constexpr int NP = Sys<SYS>::P;
  float gp[NP];
#pragma unroll
  for (int c = 0; c < NP; ++c) gp[c] = 0.0f;
  const float part = obstacle_penalty<NP>(P, R, s_obs, x, gp, lane, WAVE);
  if (__ballot(part != 0.0f) != 0ull) {  // some lane has an active obstacle term
#pragma unroll
    for (int c = 0; c < NP; ++c) g[c] += wave_sum(gp[c]);
  }
  bound_penalty<SYS>(P, R, s_val, x, g);
}

// Vector-Jacobian products of f (Eq. (1)): gx += (df/dx)^T w, gu += (df/du)^T w,
// at a state x (trigonometric values tg) under control u.
template <int SYS>
__device__ __forceinline__ void dynamics_vjp(const DevProblem& P, const float* x, const float* u,
                                             const Trig& tg, const float* w, float* gx,
                                             float* gu) {
  if constexpr (SYS == PAKR_DI2 || SYS == PAKR_DI3) {
    constexpr int Dp = Sys<SYS>::P;
#pragma unroll
    for (int a = 0; a < Dp; ++a) {
      gx[Dp + a] += w[a];  // position' = velocity
      gu[a] += w[Dp + a];  // velocity' = control
    }
  } else if constexpr (SYS == PAKR_CAR) {
    const float s = tg.s[0], c = tg.c[0];
    const float v = x[3], t = tg.t, invL = 1.0f / P.dyn[0];
    gx[2] += -v * s * w[0] + v * c * w[1];
    gx[3] += c * w[0] + s * w[1] + t * invL * w[2];
    gx[4] += v * (1.0f + t * t) * invL * w[2];
    gu[0] += w[3];
    gu[1] += w[4];
  } else if constexpr (SYS == PAKR_DUBINS) {
    const float sy = tg.s[0], cy = tg.c[0], sp = tg.s[1], cp = tg.c[1];
    const float v = x[5];
    const float wh = cy * w[0] + sy * w[1];  // w along the horizontal heading
    gx[3] += v * cp * (cy * w[1] - sy * w[0]);
    gx[4] += v * (cp * w[2] - sp * wh);
    gx[5] += cp * wh + sp * w[2];
    gu[0] += w[3];
    gu[1] += w[4];
    gu[2] += w[5];
  } else if constexpr (SYS == PAKR_UNI1) {
    const float s = tg.s[0], c = tg.c[0];
    gx[2] += u[0] * (c * w[1] - s * w[0]);
    gu[0] += c * w[0] + s * w[1];
    gu[1] += w[2];
  } else if constexpr (SYS == PAKR_UNI2) {
    const float s = tg.s[0], c = tg.c[0];
    gx[2] += x[3] * (c * w[1] - s * w[0]);
    gx[3] += c * w[0] + s * w[1];
    gx[4] += w[2];
    gu[0] += w[3];
    gu[1] += w[4];
  } else if constexpr (SYS == PAKR_CARTPOLE) {
    const float l = P.dyn[0], g = P.dyn[1];
    const float s = tg.s[0], c = tg.c[0];
    gx[1] += w[3] * (g * c + u[0] * s) / l;
    gx[2] += w[0];
    gx[3] += w[1];
    gu[0] += w[2] - w[3] * c / l;
  } else if constexpr (SYS == PAKR_ACROBOT) {
    // q'' = M^-1 r: with lambda = M^-1 (w2, w3) (M symmetric), the weights
    // reach r as lambda and M as -lambda q''^T; M depends on the elbow angle
    // only, r on both angles, both rates and the torque
    const float m1 = P.dyn[0], m2 = P.dyn[1], l1 = P.dyn[2], lc1 = P.dyn[3];
    const float lc2 = P.dyn[4], g = P.dyn[7];
    const float k = m2 * l1 * lc2, gm2 = m2 * lc2 * g, gm1 = (m1 * lc1 + m2 * l1) * g;
    const AcrobotTerms t = acrobot_terms(P, x, u[0], tg);
    const float v1 = x[2], v2 = x[3];
    const float s2 = tg.s[1], c2 = tg.c[1];
    const float l0 = (t.m11 * w[2] - t.m01 * w[3]) * t.inv_det;
    const float lm = (t.m00 * w[3] - t.m01 * w[2]) * t.inv_det;
    // dM/d(elbow) = -k s2 [[2, 1], [1, 0]]
    const float dM = l0 * (2.0f * t.a1 + t.a2) + lm * t.a1;
    gx[0] += -l0 * (gm1 * tg.c[0] + gm2 * tg.c[2]) - lm * gm2 * tg.c[2];
    gx[1] += l0 * (k * c2 * (v2 * v2 + 2.0f * v1 * v2) - gm2 * tg.c[2]) -
             lm * (k * c2 * v1 * v1 + gm2 * tg.c[2]) + k * s2 * dM;
    gx[2] += w[0] + 2.0f * k * s2 * (l0 * v2 - lm * v1);
    gx[3] += w[1] + 2.0f * k * s2 * l0 * (v2 + v1);
    gu[0] += lm;
  } else {
    static_assert(SYS == PAKR_QUAD, "unknown system");
    const float inv_m = 1.0f / P.dyn[0], g = P.dyn[1];
    const float Ix = P.dyn[2], Iy = P.dyn[3], Iz = P.dyn[4];
    const float iIx = P.dyn[5], iIy = P.dyn[6], iIz = P.dyn[7];  // 1 / inertia
    const float sph = tg.s[0], cph = tg.c[0], sth = tg.s[1], cth = tg.c[1];
    const float sps = tg.s[2], cps = tg.c[2];
    const float v0 = x[6], v1 = x[7], v2 = x[8];
    const float p = x[9], q = x[10], r = x[11];
    const float r00 = cps * cth, r01 = cps * sth * sph - sps * cph, r02 = cps * sth * cph + sps * sph;
    const float r10 = sps * cth, r11 = sps * sth * sph + cps * cph, r12 = sps * sth * cph - cps * sph;
    const float r20 = -sth, r21 = cth * sph, r22 = cth * cph;
    const float wp0 = w[0], wp1 = w[1], wp2 = w[2];
    const float wf = w[3], wt = w[4], ws = w[5];
    const float W0 = w[6], W1 = w[7], W2 = w[8];
    const float Z0 = w[9], Z1 = w[10], Z2 = w[11];
    // position' = R v: d/dv is R^T; d/droll turns column 1 into column 2 and
    // column 2 into minus column 1; d/dyaw rotates R v by +90 degrees about z
    gx[6] += r00 * wp0 + r10 * wp1 + r20 * wp2;
    gx[7] += r01 * wp0 + r11 * wp1 + r21 * wp2;
    gx[8] += r02 * wp0 + r12 * wp1 + r22 * wp2;
    gx[3] += wp0 * (r02 * v1 - r01 * v2) + wp1 * (r12 * v1 - r11 * v2) + wp2 * (r22 * v1 - r21 * v2);
    const float s1 = sph * v1 + cph * v2;
    const float brk = -sth * v0 + cth * s1;
    gx[4] += wp0 * cps * brk + wp1 * sps * brk + wp2 * (-cth * v0 - sth * s1);
    const float Rv0 = r00 * v0 + r01 * v1 + r02 * v2, Rv1 = r10 * v0 + r11 * v1 + r12 * v2;
    gx[5] += -wp0 * Rv1 + wp1 * Rv0;
    // Euler-angle rates
    const float ict = __builtin_amdgcn_rcpf(cth), tth = sth * ict;  // as in f
    const float a = q * sph + r * cph, bq = q * cph - r * sph;
    gx[9] += wf;
    gx[10] += wf * sph * tth + wt * cph + ws * sph * ict;
    gx[11] += wf * cph * tth - wt * sph + ws * cph * ict;
    gx[3] += wf * bq * tth - wt * a + ws * bq * ict;
    gx[4] += wf * a * (1.0f + tth * tth) + ws * a * sth * ict * ict;
    // body velocity' = -w x v - g R[2,:] + (0, 0, thrust / m)
    gx[6] += q * W2 - r * W1;  // w x W
    gx[7] += r * W0 - p * W2;
    gx[8] += p * W1 - q * W0;
    gx[9] += W1 * v2 - W2 * v1;  // W x v
    gx[10] += W2 * v0 - W0 * v2;
    gx[11] += W0 * v1 - W1 * v0;
    gx[3] += -g * (W1 * cth * cph - W2 * cth * sph);
    gx[4] += g * (W0 * cth + W1 * sth * sph + W2 * sth * cph);
    gu[0] += W2 * inv_m;
    // body rates' = I^-1 (tau - w x I w)
    gu[1] += Z0 * iIx;
    gu[2] += Z1 * iIy;
    gu[3] += Z2 * iIz;
    gx[9] += -Z1 * (Ix - Iz) * r * iIy - Z2 * (Iy - Ix) * q * iIz;
    gx[10] += -Z0 * (Iz - Iy) * r * iIx - Z2 * (Iy - Ix) * p * iIz;
    gx[11] += -Z0 * (Iz - Iy) * q * iIx - Z1 * (Ix - Iz) * p * iIy;
  }
}

// Trigonometric values for the refinement's rollouts, from the hardware sine
// and cosine (v_sin_f32 / v_cos_f32 after scaling to revolutions; absolute
// error about 1e-6 at these angles) rather than the correctly rounded
// library sincos: the rollout is one serial chain per path, and its length
// sets the refinement's latency.  The objective's f and its VJP take the same
// values, so the gradient is exact for the objective as evaluated; the
// planner's own check of a refined path (k_check_path) integrates with the
// planner's f.
__device__ __forceinline__ void fast_sincos(float a, float* s, float* c) {
  *s = __sinf(a);
  *c = __cosf(a);
}

template <int SYS>
__device__ __forceinline__ Trig wave_trig(const float* x, int /*lane*/) {
  Trig g;
  g.s[0] = g.s[1] = g.s[2] = 0.0f;
  g.c[0] = g.c[1] = g.c[2] = 0.0f;
  g.t = 0.0f;
  if constexpr (SYS == PAKR_CAR) {
    fast_sincos(x[2], &g.s[0], &g.c[0]);
    float sp, cp;
    fast_sincos(x[4], &sp, &cp);
    g.t = sp / cp;
  } else if constexpr (SYS == PAKR_QUAD) {
#pragma unroll
    for (int k = 0; k < 3; ++k) fast_sincos(x[3 + k], &g.s[k], &g.c[k]);
  } else if constexpr (SYS == PAKR_DUBINS) {
    fast_sincos(x[3], &g.s[0], &g.c[0]);
    fast_sincos(x[4], &g.s[1], &g.c[1]);
  } else if constexpr (SYS == PAKR_UNI1 || SYS == PAKR_UNI2) {
    fast_sincos(x[2], &g.s[0], &g.c[0]);
  } else if constexpr (SYS == PAKR_CARTPOLE) {
    fast_sincos(x[1], &g.s[0], &g.c[0]);
  } else if constexpr (SYS == PAKR_ACROBOT) {
    fast_sincos(x[0], &g.s[0], &g.c[0]);
    fast_sincos(x[1], &g.s[1], &g.c[1]);
    g.s[2] = g.s[0] * g.c[1] + g.c[0] * g.s[1];  // angle sum
    g.c[2] = g.c[0] * g.c[1] - g.s[0] * g.s[1];
  }
  return g;
}

// One RK4 step (as the planner takes it) on a state the whole wave holds.
template <int SYS>
__device__ __forceinline__ void rk4_step_wave(const DevProblem& P, float* x, const float* u,
                                              float h, int lane) {
  constexpr int D = Sys<SYS>::D;
  float k1[D], k2[D], k3[D], k4[D], t[D];
  const float hh = 0.5f * h;
  dynamics_trig<SYS>(P, x, u, wave_trig<SYS>(x, lane), k1);
#pragma unroll
  for (int i = 0; i < D; ++i) t[i] = x[i] + hh * k1[i];
  dynamics_trig<SYS>(P, t, u, wave_trig<SYS>(t, lane), k2);
#pragma unroll
  for (int i = 0; i < D; ++i) t[i] = x[i] + hh * k2[i];
  dynamics_trig<SYS>(P, t, u, wave_trig<SYS>(t, lane), k3);
#pragma unroll
  for (int i = 0; i < D; ++i) t[i] = x[i] + h * k3[i];
  dynamics_trig<SYS>(P, t, u, wave_trig<SYS>(t, lane), k4);
  const float h6 = h * (1.0f / 6.0f);
#pragma unroll
  for (int i = 0; i < D; ++i) x[i] = x[i] + h6 * (k1[i] + 2.0f * (k2[i] + k3[i]) + k4[i]);
}

// Reverse of one RK4 step taken from x under control u: lam holds dJ/dx_{n+1}
// on entry and the part of dJ/dx_n that flows through the step on exit;
// gu accumulates dJ/du.  The four stage states are recomputed from x.
template <int SYS>
__device__ __forceinline__ void rk4_step_vjp(const DevProblem& P, const float* x, const float* u,
                                             float h, float* lam, float* gu, int lane) {
  constexpr int D = Sys<SYS>::D;
  float k[3][D], xs[4][D];
  Trig tg[4];
  const float hh = 0.5f * h;
#pragma unroll
  for (int i = 0; i < D; ++i) xs[0][i] = x[i];
  tg[0] = wave_trig<SYS>(xs[0], lane);
  dynamics_trig<SYS>(P, xs[0], u, tg[0], k[0]);
#pragma unroll
  for (int i = 0; i < D; ++i) xs[1][i] = x[i] + hh * k[0][i];
  tg[1] = wave_trig<SYS>(xs[1], lane);
  dynamics_trig<SYS>(P, xs[1], u, tg[1], k[1]);
#pragma unroll
  for (int i = 0; i < D; ++i) xs[2][i] = x[i] + hh * k[1][i];
  tg[2] = wave_trig<SYS>(xs[2], lane);
  dynamics_trig<SYS>(P, xs[2], u, tg[2], k[2]);
#pragma unroll
  for (int i = 0; i < D; ++i) xs[3][i] = x[i] + h * k[2][i];
  tg[3] = wave_trig<SYS>(xs[3], lane);
  // x_{n+1} = x + h/6 (k1 + 2 k2 + 2 k3 + k4); stage s (0-based) evaluates f
  // at x + c_s k_{s-1} with c = (h/2, h/2, h)
  const float h6 = h * (1.0f / 6.0f);
  const float wk[4] = {h6, 2.0f * h6, 2.0f * h6, h6};
  const float cs[3] = {hh, hh, h};
  float lam_out[D], carry[D];
#pragma unroll
  for (int i = 0; i < D; ++i) {
    lam_out[i] = lam[i];
    carry[i] = 0.0f;
  }
#pragma unroll
  for (int s = 3; s >= 0; --s) {
    float gk[D], gxs[D];
#pragma unroll
    for (int i = 0; i < D; ++i) {
      gk[i] = wk[s] * lam[i] + carry[i];
      gxs[i] = 0.0f;
    }
    dynamics_vjp<SYS>(P, xs[s], u, tg[s], gk, gxs, gu);
#pragma unroll
    for (int i = 0; i < D; ++i) {
      carry[i] = s > 0 ? cs[s - 1] * gxs[i] : 0.0f;
      lam_out[i] += gxs[i];
    }
  }
#pragma unroll
  for (int i = 0; i < D; ++i) lam[i] = lam_out[i];
}

__device__ __forceinline__ void load_traj_lds(const TrajArgs& a, float* s_obs, float* s_val) {
  for (int i = threadIdx.x; i < a.P.obs_floats; i += blockDim.x) s_obs[i] = a.obs[i];
  load_validity(a.P, s_val, threadIdx.x);
  __syncthreads();
}

// Forward rollout: J per trajectory and the checkpoints x_0 .. x_N.
// Launch: one 64-lane workgroup per trajectory.
template <int SYS>
__global__ __launch_bounds__(WAVE) void k_rollout_fwd(TrajArgs a) {
  constexpr int D = Sys<SYS>::D, M = Sys<SYS>::M, NP = Sys<SYS>::P;
  extern __shared__ float s_obs[];
  __shared__ float s_val[VAL_FLOATS];
  load_traj_lds(a, s_obs, s_val);
  const int p = blockIdx.x, lane = threadIdx.x;
  const DevProblem& P = a.P;
  const size_t N = (size_t)a.M * P.T;
  float* ck = a.ckpt + (size_t)p * (N + 1) * D;
  const float* Up = a.U + (size_t)p * a.M * M;
  float x[D];
#pragma unroll
  for (int c = 0; c < D; ++c) x[c] = a.x0[(size_t)p * D + c];
  if (lane < D) ck[lane] = a.x0[(size_t)p * D + lane];
  const float edge_t = P.edge_duration;
  float J = 0.0f;
  for (int e = 0; e < a.M; ++e) {
    float u[M];
#pragma unroll
    for (int c = 0; c < M; ++c) {
      u[c] = Up[e * M + c];
      const float z = (u[c] - a.R.u_ref[c]) / a.R.u_scale[c];
      J += a.R.w_u * edge_t * z * z;
    }
    for (int t = 0; t < P.T; ++t) {
      rk4_step_wave<SYS>(P, x, u, P.dt, lane);
      const size_t n = (size_t)e * P.T + t + 1;
      if (lane == 0) {
#pragma unroll
        for (int c = 0; c < D; ++c) ck[n * D + c] = x[c];
      }
      J += a.R.w_c * wave_penalty<SYS>(P, a.R, s_obs, s_val, x, lane);
    }
  }
#pragma unroll
  for (int c = 0; c < NP; ++c) {
    const float e = x[c] - P.goal_c[c];
    J += a.R.w_g * e * e;
  }
  if (lane == 0) a.J[p] = J;
}

// Adjoint: gU = gJ * dJ/dU from the checkpoints of the forward pass.
// Launch: one 64-lane workgroup per trajectory.
template <int SYS>
__global__ __launch_bounds__(WAVE) void k_rollout_bwd(TrajArgs a) {
  constexpr int D = Sys<SYS>::D, M = Sys<SYS>::M, NP = Sys<SYS>::P;
  extern __shared__ float s_obs[];
  __shared__ float s_val[VAL_FLOATS];
  load_traj_lds(a, s_obs, s_val);
  const int p = blockIdx.x, lane = threadIdx.x;
  const DevProblem& P = a.P;
  const size_t N = (size_t)a.M * P.T;
  const float* ck = a.ckpt + (size_t)p * (N + 1) * D;
  const float* Up = a.U + (size_t)p * a.M * M;
  float* gUp = a.gU + (size_t)p * a.M * M;
  const float gJ = a.gJ[p];
  float x[D], lam[D];
#pragma unroll
  for (int c = 0; c < D; ++c) {
    x[c] = ck[N * D + c];
    lam[c] = 0.0f;
  }
  // terminal goal term and the penalty of x_N
#pragma unroll
  for (int c = 0; c < NP; ++c) lam[c] = 2.0f * a.R.w_g * (x[c] - P.goal_c[c]);
  {
    float g[D];
#pragma unroll
    for (int c = 0; c < D; ++c) g[c] = 0.0f;
    wave_penalty_grad<SYS>(P, a.R, s_obs, s_val, x, lane, g);
#pragma unroll
    for (int c = 0; c < D; ++c) lam[c] += a.R.w_c * g[c];
  }
  const float edge_t = P.edge_duration;
  for (int e = a.M - 1; e >= 0; --e) {
    float u[M], gu[M];
#pragma unroll
    for (int c = 0; c < M; ++c) {
      u[c] = Up[e * M + c];
      gu[c] = 0.0f;
    }
    for (int t = P.T - 1; t >= 0; --t) {
      const size_t n = (size_t)e * P.T + t;  // step n takes x_n to x_{n+1}
#pragma unroll
      for (int c = 0; c < D; ++c) x[c] = ck[n * D + c];
      rk4_step_vjp<SYS>(P, x, u, P.dt, lam, gu, lane);
      if (n > 0) {
        float g[D];
#pragma unroll
        for (int c = 0; c < D; ++c) g[c] = 0.0f;
        wave_penalty_grad<SYS>(P, a.R, s_obs, s_val, x, lane, g);
#pragma unroll
        for (int c = 0; c < D; ++c) lam[c] += a.R.w_c * g[c];
      }
    }
    if (lane == 0) {
#pragma unroll
      for (int c = 0; c < M; ++c) {
        const float z = (u[c] - a.R.u_ref[c]) / a.R.u_scale[c];
        gUp[e * M + c] = gJ * (gu[c] + 2.0f * a.R.w_u * edge_t * z / a.R.u_scale[c]);
      }
    }
  }
}

// The planner's acceptance test of each trajectory: every sub-step valid
// (workspace, limits, obstacles, as an edge rollout tests it), the final
// position in the goal ball, and the trajectory's cost.
// Launch: one 64-lane workgroup per trajectory.
template <int SYS>
__global__ __launch_bounds__(WAVE) void k_check_path(TrajArgs a) {
  constexpr int D = Sys<SYS>::D, M = Sys<SYS>::M, NP = Sys<SYS>::P;
  extern __shared__ float s_obs[];
  __shared__ float s_val[VAL_FLOATS];
  load_traj_lds(a, s_obs, s_val);
  const int p = blockIdx.x, lane = threadIdx.x;
  const DevProblem& P = a.P;
  const float* Up = a.U + (size_t)p * a.M * M;
  float x[D];
#pragma unroll
  for (int c = 0; c < D; ++c) x[c] = a.x0[(size_t)p * D + c];
  bool ok = true;
  float cost = 0.0f;
  for (int e = 0; e < a.M; ++e) {
    float u[M];
#pragma unroll
    for (int c = 0; c < M; ++c) u[c] = Up[e * M + c];
    float len = 0.0f;
    for (int t = 0; t < P.T; ++t) {
      float xp[NP];
#pragma unroll
      for (int c = 0; c < NP; ++c) xp[c] = x[c];
      rk4_step<SYS>(P, x, u, P.dt);
      float s2 = 0.0f;
#pragma unroll
      for (int c = 0; c < NP; ++c) {
        const float d = x[c] - xp[c];
        s2 += d * d;
      }
      len += __builtin_amdgcn_sqrtf(s2);  // as the planner's rollout
      float pos[1][NP];
#pragma unroll
      for (int c = 0; c < NP; ++c) pos[0][c] = x[c];
      const bool hit = any_obstacle_hit<NP, 1>(pos, s_obs, P.n_box, P.n_sph, lane, WAVE);
      // every lane takes part in the ballot, whatever its own verdict so far
      const bool clear = __ballot(hit) == 0ull;
      const bool lim = limits_ok<SYS>(s_val, x);
      ok = ok && lim && clear;
    }
    cost += P.cost_kind == PAKR_COST_PATH_LENGTH ? len : P.edge_duration;
  }
  const float dist = sqrtf(goal_dist2<SYS>(P, x));
  if (lane == 0) {
    a.ok[p] = (ok ? 1 : 0) | (dist <= P.goal_r ? 2 : 0);
    a.cost[p] = cost;
  }
}

// One projected Adam step on the controls, taken in the normalised variables
// z = (u - mid) / half_range so that every control moves on the same scale,
// then clipped to the control box.  One lane per control value.  With
// lr_traj set, each trajectory uses its own step size lr * lr_traj[p].
struct AdamArgs {
  const float* U;                 // controls the step starts from
  float* U_out;                   // result (may alias U)
  const float* gU;
  float* m1;
  float* m2;
  const float* lr_traj;           // [n_traj] step-size factors, or null
  int n, m, per_traj;             // values, controls per edge, values per trajectory
  float lr, b1, b2, eps, c1, c2;  // c1 = 1 - b1^t, c2 = 1 - b2^t
  float u_lo[PAKR_MAX_M], u_hi[PAKR_MAX_M];
};

__global__ __launch_bounds__(256) void k_adam_project(AdamArgs a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const int c = i % a.m;
  const float half = 0.5f * (a.u_hi[c] - a.u_lo[c]);
  const float g = a.gU[i] * half;  // gradient in z
  const float m1 = a.b1 * a.m1[i] + (1.0f - a.b1) * g;
  const float m2 = a.b2 * a.m2[i] + (1.0f - a.b2) * g * g;
  a.m1[i] = m1;
  a.m2[i] = m2;
  const float lr = a.lr_traj ? a.lr * a.lr_traj[i / a.per_traj] : a.lr;
  const float step = lr * (m1 / a.c1) / (sqrtf(m2 / a.c2) + a.eps);
  const float u = a.U[i] - half * step;
  a.U_out[i] = fminf(fmaxf(u, a.u_lo[c]), a.u_hi[c]);
}

// Safeguard of the refinement loop: a trial that lowers J replaces the
// current controls and lets its trajectory's step grow (up to the base
// step); a trial that does not is dropped and the step is halved.
// One 64-lane workgroup per trajectory: every lane reads J and J_trial, all
// of them copy the trial controls if it is taken, and only after a workgroup
// barrier does lane 0 overwrite J (so no lane can see the updated J and take
// a different decision).
struct AcceptArgs {
  float* U;
  const float* U_trial;
  float* J;                       // J of U; becomes min(J, J_trial)
  const float* J_trial;
  float* lr_traj;
  int n_traj, per_traj;
};

__global__ __launch_bounds__(WAVE) void k_accept(AcceptArgs a) {
  const int p = blockIdx.x;
  if (p >= a.n_traj) return;
  const float J = a.J[p], Jt = a.J_trial[p];
  const bool take = Jt < J;  // NaN trials are never taken
  if (take) {
    const size_t base = (size_t)p * a.per_traj;
    for (int i = threadIdx.x; i < a.per_traj; i += blockDim.x) a.U[base + i] = a.U_trial[base + i];
  }
  __syncthreads();  // every lane has read J before it changes
  if (threadIdx.x == 0) {
    a.lr_traj[p] = take ? fminf(a.lr_traj[p] * 1.25f, 1.0f) : a.lr_traj[p] * 0.5f;
    if (take) a.J[p] = Jt;
  }
}

__global__ __launch_bounds__(256) void k_fill(float* x, int n, float v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}

}  // namespace pakr
