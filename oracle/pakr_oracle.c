/*
 * FP64 reference planner for PAKR -- TEST INFRASTRUCTURE ONLY (see
 * pakr_oracle.h).  Plain, slow, sequential C.  Build with
 *   gcc -O2 -std=c99 -ffp-contract=off -fno-fast-math -shared -fPIC
 * so that the float32 sample conversion below is evaluated exactly as written
 * (two round-to-nearest operations, no fused multiply-add).
 */
#include "pakr_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define MAXD 12
#define MAXM 4
#define PI_D 3.14159265358979323846

/* ------------------------------------------------------------------------ */
/* Philox4x32-10, from its published definition (Salmon, Moraes, Dror and   */
/* Shaw, "Parallel Random Numbers: As Easy as 1, 2, 3", SC'11): ten rounds  */
/* of two 32x32->64 multiplies, the high halves xored with the other words  */
/* and the round key, the key bumped by the Weyl constants between rounds.  */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t prod0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
    uint64_t prod1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
    uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
    uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
    uint32_t y0 = hi1 ^ x1 ^ k0;
    uint32_t y1 = lo1;
    uint32_t y2 = hi0 ^ x3 ^ k1;
    uint32_t y3 = lo0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* The uniform draw on [lo, hi] used by SampleStates / SampleControls (Alg. 1):
 * the top 24 bits give u in [0,1) exactly; the value is lo + (hi - lo) * u
 * evaluated in float32 with one rounding per operation. */
float orc_u32_to_range(uint32_t x, float lo, float hi) {
  volatile float u = (float)(x >> 8) * 5.9604644775390625e-08f; /* 2^-24, exact */
  volatile float w = hi - lo;
  volatile float prod = w * u;
  volatile float val = lo + prod;
  return val;
}

void orc_u32_to_range_n(const uint32_t* x, int n, float lo, float hi, float* out) {
  for (int i = 0; i < n; ++i) out[i] = orc_u32_to_range(x[i], lo, hi);
}

enum { TAG_STATE = 0, TAG_CONTROL = 1 };

/* Counter layout: (index, iteration in round, round, tag << 16 | sub), key
 * (low word of the seed, query id).  For states the index is the target k and
 * sub the block of four dimensions; for controls the index is the parent
 * query k and sub the branch a, so branch a = 0 of every query draws the same
 * control whatever the branching factor. */
static void draw(const orc_problem* p, uint32_t idx, uint32_t sub, uint32_t iter, uint32_t round,
                 uint32_t tag, int n, const float* lo, const float* hi, float* out) {
  uint32_t key[2] = {(uint32_t)(p->seed & 0xffffffffu), p->qid};
  for (int blk = 0; blk * 4 < n; ++blk) {
    uint32_t ctr[4] = {idx, iter, round, (tag << 16) | (sub + (uint32_t)blk)};
    uint32_t r[4];
    orc_philox4x32_10(ctr, key, r);
    for (int w = 0; w < 4 && blk * 4 + w < n; ++w) {
      int c = blk * 4 + w;
      out[c] = orc_u32_to_range(r[w], lo[c], hi[c]);
    }
  }
}

/* SampleStates(B/A), Alg. 1: one uniform target per NN query, no goal bias. */
void orc_sample_state(const orc_problem* p, uint32_t k, uint32_t iter, uint32_t round, float* out) {
  draw(p, k, 0, iter, round, TAG_STATE, p->d, p->sample_lo, p->sample_hi, out);
}

/* SampleControls(B/A, A), Alg. 1: one uniform control per (parent query k,
 * branch a); candidate j = k*A + a.  m <= 4, so one Philox block suffices. */
void orc_sample_control(const orc_problem* p, uint32_t k, uint32_t a, uint32_t iter,
                        uint32_t round, float* out) {
  draw(p, k, a, iter, round, TAG_CONTROL, p->m, p->u_lo, p->u_hi, out);
}

/* ------------------------------------------------------------------------ */
/* Dynamics x' = f(x, u), Eq. (1).  The paper names the systems (Sec. V-A)  */
/* but does not print their equations; these are the textbook forms.        */
/* ------------------------------------------------------------------------ */
static void f_double_integrator(int D, const double* x, const double* u, double* xd) {
  for (int a = 0; a < D; ++a) {
    xd[a] = x[D + a];   /* position' = velocity */
    xd[D + a] = u[a];   /* velocity' = acceleration */
  }
}

/* Second-order car: (x, y, theta, v, phi), controls (a, steering rate). */
static void f_car(const orc_problem* p, const double* x, const double* u, double* xd) {
  double L = (double)p->dyn[0];
  double th = x[2], v = x[3], ph = x[4];
  xd[0] = v * cos(th);
  xd[1] = v * sin(th);
  xd[2] = v * tan(ph) / L;
  xd[3] = u[0];
  xd[4] = u[1];
}

/* Quadrotor, Z-Y-X Euler angles, body-frame velocities and rates (Sec. V-A):
 *   p'      = R(roll, pitch, yaw) v_b
 *   angles' = W(roll, pitch) w
 *   v_b'    = -w x v_b + R^T (0, 0, -g) + (0, 0, thrust / mass)
 *   w'      = I^-1 (tau - w x I w),  I = diag(Ixx, Iyy, Izz). */
static void f_quad(const orc_problem* p, const double* x, const double* u, double* xd) {
  double mass = p->dyn[0], g = p->dyn[1];
  double Ix = p->dyn[2], Iy = p->dyn[3], Iz = p->dyn[4];
  double ph = x[3], th = x[4], ps = x[5];
  double ub = x[6], vb = x[7], wb = x[8];
  double pr = x[9], qr = x[10], rr = x[11];
  double cph = cos(ph), sph = sin(ph), cth = cos(th), sth = sin(th), cps = cos(ps), sps = sin(ps);
  double R[3][3];
  /* R = Rz(yaw) * Ry(pitch) * Rx(roll) */
  double Rx[3][3] = {{1, 0, 0}, {0, cph, -sph}, {0, sph, cph}};
  double Ry[3][3] = {{cth, 0, sth}, {0, 1, 0}, {-sth, 0, cth}};
  double Rz[3][3] = {{cps, -sps, 0}, {sps, cps, 0}, {0, 0, 1}};
  double Ryx[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      Ryx[i][j] = 0;
      for (int k = 0; k < 3; ++k) Ryx[i][j] += Ry[i][k] * Rx[k][j];
    }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      R[i][j] = 0;
      for (int k = 0; k < 3; ++k) R[i][j] += Rz[i][k] * Ryx[k][j];
    }
  double v[3] = {ub, vb, wb};
  for (int i = 0; i < 3; ++i) xd[i] = R[i][0] * v[0] + R[i][1] * v[1] + R[i][2] * v[2];
  /* Euler-angle rates from body rates */
  double tth = sth / cth;
  xd[3] = pr + (qr * sph + rr * cph) * tth;
  xd[4] = qr * cph - rr * sph;
  xd[5] = (qr * sph + rr * cph) / cth;
  /* translational: -w x v + R^T g_world + thrust */
  double w[3] = {pr, qr, rr};
  double wxv[3] = {w[1] * v[2] - w[2] * v[1], w[2] * v[0] - w[0] * v[2],
                   w[0] * v[1] - w[1] * v[0]};
  double gw[3] = {0.0, 0.0, -g};
  double gb[3];
  for (int i = 0; i < 3; ++i) gb[i] = R[0][i] * gw[0] + R[1][i] * gw[1] + R[2][i] * gw[2];
  double thrust = u[0];
  xd[6] = -wxv[0] + gb[0];
  xd[7] = -wxv[1] + gb[1];
  xd[8] = -wxv[2] + gb[2] + thrust / mass;
  /* rotational: I^-1 (tau - w x (I w)) */
  double Iw[3] = {Ix * pr, Iy * qr, Iz * rr};
  double wxIw[3] = {w[1] * Iw[2] - w[2] * Iw[1], w[2] * Iw[0] - w[0] * Iw[2],
                    w[0] * Iw[1] - w[1] * Iw[0]};
  xd[9] = (u[1] - wxIw[0]) / Ix;
  xd[10] = (u[2] - wxIw[1]) / Iy;
  xd[11] = (u[3] - wxIw[2]) / Iz;
}

/* Dubins airplane (Sec. V-A): state (x, y, z, yaw, pitch, speed), controls
 * (yaw rate, pitch rate, acceleration); the speed acts along the heading
 * given by yaw and pitch. */
static void f_dubins(const double* x, const double* u, double* xd) {
  double ps = x[3], th = x[4], v = x[5];
  xd[0] = v * cos(ps) * cos(th);
  xd[1] = v * sin(ps) * cos(th);
  xd[2] = v * sin(th);
  xd[3] = u[0];
  xd[4] = u[1];
  xd[5] = u[2];
}

/* Unicycle 1 (Sec. V-C): state (x, y, heading), controls (speed, turn rate). */
static void f_uni1(const double* x, const double* u, double* xd) {
  xd[0] = u[0] * cos(x[2]);
  xd[1] = u[0] * sin(x[2]);
  xd[2] = u[1];
}

/* Unicycle 2 (Sec. V-C): state (x, y, heading, speed, turn rate), controls
 * (acceleration, angular acceleration). */
static void f_uni2(const double* x, const double* u, double* xd) {
  xd[0] = x[3] * cos(x[2]);
  xd[1] = x[3] * sin(x[2]);
  xd[2] = x[4];
  xd[3] = u[0];
  xd[4] = u[1];
}

/* Acrobot (Sec. V-C): two links hanging from a fixed pivot, angles measured
 * from the downward vertical, the second relative to the first; torque at the
 * elbow only.  The paper names states and control only; these are the
 * Euler-Lagrange equations of two rigid links: M(q) q'' + c(q, q') + g(q) =
 * (0, tau), dyn = (m1, m2, l1, lc1, lc2, I1, I2, gravity), I about each centre
 * of mass. */
static void acrobot_terms(const orc_problem* p, const double* x, double M[2][2], double r[2],
                          double tau) {
  const double m1 = p->dyn[0], m2 = p->dyn[1], l1 = p->dyn[2], lc1 = p->dyn[3];
  const double lc2 = p->dyn[4], I1 = p->dyn[5], I2 = p->dyn[6], g = p->dyn[7];
  const double q1 = x[0], q2 = x[1], w1 = x[2], w2 = x[3];
  const double k = m2 * l1 * lc2;
  M[0][0] = m1 * lc1 * lc1 + m2 * (l1 * l1 + lc2 * lc2) + I1 + I2 + 2.0 * k * cos(q2);
  M[0][1] = M[1][0] = m2 * lc2 * lc2 + I2 + k * cos(q2);
  M[1][1] = m2 * lc2 * lc2 + I2;
  const double c1 = -k * sin(q2) * (w2 * w2 + 2.0 * w1 * w2);
  const double c2 = k * sin(q2) * w1 * w1;
  const double g2 = m2 * lc2 * g * sin(q1 + q2);
  const double g1 = (m1 * lc1 + m2 * l1) * g * sin(q1) + g2;
  r[0] = -c1 - g1;
  r[1] = tau - c2 - g2;
}

static void f_acrobot(const orc_problem* p, const double* x, const double* u, double* xd) {
  double M[2][2], r[2];
  acrobot_terms(p, x, M, r, u[0]);
  const double det = M[0][0] * M[1][1] - M[0][1] * M[1][0];
  xd[0] = x[2];
  xd[1] = x[3];
  xd[2] = (M[1][1] * r[0] - M[0][1] * r[1]) / det;
  xd[3] = (M[0][0] * r[1] - M[1][0] * r[0]) / det;
}

/* Cart-pole (Sec. V-E lists it with an acceleration control): state (cart
 * position, pole angle from the upward vertical, cart speed, pole rate),
 * control the cart's acceleration; the pole is a point mass at distance
 * dyn[0] from the pivot, dyn[1] gravity.  With the cart's acceleration
 * prescribed the pole obeys l theta'' = g sin(theta) - a cos(theta). */
static void f_cartpole(const orc_problem* p, const double* x, const double* u, double* xd) {
  const double l = p->dyn[0], g = p->dyn[1];
  xd[0] = x[2];
  xd[1] = x[3];
  xd[2] = u[0];
  xd[3] = (g * sin(x[1]) - u[0] * cos(x[1])) / l;
}

void orc_dynamics(const orc_problem* p, const double* x, const double* u, double* xd) {
  switch (p->system) {
    case ORC_DI2: f_double_integrator(2, x, u, xd); break;
    case ORC_DI3: f_double_integrator(3, x, u, xd); break;
    case ORC_CAR: f_car(p, x, u, xd); break;
    case ORC_QUAD: f_quad(p, x, u, xd); break;
    case ORC_DUBINS: f_dubins(x, u, xd); break;
    case ORC_UNI1: f_uni1(x, u, xd); break;
    case ORC_UNI2: f_uni2(x, u, xd); break;
    case ORC_ACROBOT: f_acrobot(p, x, u, xd); break;
    case ORC_CARTPOLE: f_cartpole(p, x, u, xd); break;
    default: for (int i = 0; i < p->d; ++i) xd[i] = NAN;
  }
}

/* Propagate, Sec. IV-A: classical fourth-order Runge-Kutta, control held. */
void orc_rk4_step(const orc_problem* p, const double* x, const double* u, double h, double* out) {
  int d = p->d;
  double k1[MAXD], k2[MAXD], k3[MAXD], k4[MAXD], tmp[MAXD];
  orc_dynamics(p, x, u, k1);
  for (int i = 0; i < d; ++i) tmp[i] = x[i] + 0.5 * h * k1[i];
  orc_dynamics(p, tmp, u, k2);
  for (int i = 0; i < d; ++i) tmp[i] = x[i] + 0.5 * h * k2[i];
  orc_dynamics(p, tmp, u, k3);
  for (int i = 0; i < d; ++i) tmp[i] = x[i] + h * k3[i];
  orc_dynamics(p, tmp, u, k4);
  for (int i = 0; i < d; ++i) out[i] = x[i] + h / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
}

void orc_rollout(const orc_problem* p, const double* x0, const double* u, int T, double h,
                 double* states) {
  int d = p->d;
  memcpy(states, x0, sizeof(double) * d);
  for (int t = 0; t < T; ++t) orc_rk4_step(p, states + t * d, u, h, states + (t + 1) * d);
}

/* ------------------------------------------------------------------------ */
/* State validity, "validity checked at each step" (Sec. IV-A) and the      */
/* feasibility definition of Sec. III: a point robot at the position        */
/* coordinates must lie in the closed workspace and outside every closed    */
/* obstacle, and the state must respect the system's limits.               */
/* ------------------------------------------------------------------------ */
typedef struct {
  int violated;   /* some check fails by more than eps */
  int near;       /* some check lies within eps */
  int valid;      /* exact decision */
  double margin;  /* closest signed margin (>0 on the valid side) */
} check_acc;

static void acc_check(check_acc* a, double m, int ok, double eps) {
  if (isnan(m)) { a->violated = 1; a->valid = 0; a->margin = NAN; return; }
  if (!ok) a->valid = 0;
  if (fabs(m) <= eps) a->near = 1;
  else if (!ok) a->violated = 1;
  if (!isnan(a->margin) && fabs(m) < fabs(a->margin)) a->margin = m;
}

static void check_state(const orc_problem* p, const double* x, double eps, check_acc* a) {
  int P = p->npos;
  for (int i = 0; i < p->d; ++i) {
    if (isnan(x[i])) { a->violated = 1; a->valid = 0; a->margin = NAN; return; }
  }
  /* closed workspace box: valid iff lo <= p <= hi */
  for (int c = 0; c < P; ++c) {
    double lo = x[c] - (double)p->ws_lo[c];
    double hi = (double)p->ws_hi[c] - x[c];
    double m = lo < hi ? lo : hi;
    acc_check(a, m, m >= 0.0, eps);
  }
  /* per-dimension limits: valid iff lim_lo <= x <= lim_hi */
  for (int i = 0; i < p->d; ++i) {
    double lo = (double)p->lim_lo[i], hi = (double)p->lim_hi[i];
    if (isinf(lo) && isinf(hi)) continue;
    double m = x[i] - lo;
    if (hi - x[i] < m) m = hi - x[i];
    acc_check(a, m, m >= 0.0, eps);
  }
  /* speed-norm limit on the velocity block (double integrators) */
  if (p->vnorm_max > 0.0f) {
    double s2 = 0.0;
    for (int c = 0; c < P; ++c) s2 += x[P + c] * x[P + c];
    double m = (double)p->vnorm_max - sqrt(s2);
    acc_check(a, m, m >= 0.0, eps);
  }
  /* closed axis-aligned boxes: collision iff |p - c| <= h on every axis */
  for (int b = 0; b < p->n_box; ++b) {
    double m = -INFINITY;
    for (int c = 0; c < P; ++c) {
      double e = fabs(x[c] - (double)p->box_c[b * P + c]) - (double)p->box_h[b * P + c];
      if (e > m) m = e;
    }
    acc_check(a, m, m > 0.0, eps);
  }
  /* closed spheres / discs: collision iff |p - c| <= r */
  for (int s = 0; s < p->n_sph; ++s) {
    double s2 = 0.0;
    for (int c = 0; c < P; ++c) {
      double e = x[c] - (double)p->sph_c[s * P + c];
      s2 += e * e;
    }
    double m = sqrt(s2) - (double)p->sph_r[s];
    acc_check(a, m, m > 0.0, eps);
  }
}

int orc_state_valid(const orc_problem* p, const double* x, double eps, int* near, double* margin) {
  check_acc a = {0, 0, 1, INFINITY};
  check_state(p, x, eps, &a);
  if (near) *near = a.near && !a.violated;
  if (margin) *margin = a.margin;
  return a.valid;
}

/* Propagate + CollisionFree for one candidate (Alg. 1; Sec. IV-A): T RK4 steps
 * with the control held, every sub-step state t = 1..T checked, the edge cost
 * added to the parent's cost-to-come. */
int orc_edge(const orc_problem* p, const double* x0, double c0, const double* u, double* xT,
             double* cost, int* amb) {
  int d = p->d, P = p->npos;
  double x[MAXD], xn[MAXD];
  double h = (double)p->dt;
  memcpy(x, x0, sizeof(double) * d);
  check_acc acc = {0, 0, 1, INFINITY};
  double edge = 0.0;
  for (int t = 1; t <= p->T; ++t) {
    orc_rk4_step(p, x, u, h, xn);
    if (p->cost_kind == ORC_COST_PATH_LENGTH) {
      double s2 = 0.0;
      for (int c = 0; c < P; ++c) s2 += (xn[c] - x[c]) * (xn[c] - x[c]);
      edge += sqrt(s2);
    }
    check_state(p, xn, p->eps, &acc);
    memcpy(x, xn, sizeof(double) * d);
  }
  if (p->cost_kind == ORC_COST_DURATION) edge = (double)p->T * h;
  memcpy(xT, x, sizeof(double) * d);
  *cost = c0 + edge;
  if (amb) *amb = acc.near && !acc.violated;
  return acc.valid;
}

/* h(n) of the prune test in Alg. 1.  The paper writes the Euclidean distance
 * to the goal; the default reading measures it from the goal region and
 * divides by the maximum speed for a duration cost, which keeps it a lower
 * bound on cost-to-go. */
double orc_heuristic(const orc_problem* p, const double* x) {
  int P = p->npos;
  double s2 = 0.0;
  for (int c = 0; c < P; ++c) {
    double e = x[c] - (double)p->goal_c[c];
    s2 += e * e;
  }
  double dist = sqrt(s2);
  if (p->h_kind == ORC_H_NONE) return 0.0;
  if (p->h_kind == ORC_H_PAPER_LITERAL) return dist;
  double gap = dist - (double)p->goal_r;
  if (gap < 0.0) gap = 0.0;
  if (p->cost_kind == ORC_COST_DURATION) gap /= (double)p->h_speed;
  return gap;
}

/* NearestNeighbor(T, X_rand): brute force over the frozen tree [0, n), plain
 * squared Euclidean distance over all state dimensions, ties to the lowest
 * index.  Also reports the second-best distance for the near-tie test. */
int orc_nearest(const double* states, int n, int d, const double* q, double* d2_best,
                double* d2_second) {
  int best = -1;
  double b1 = INFINITY, b2 = INFINITY;
  for (int i = 0; i < n; ++i) {
    double s = 0.0;
    for (int c = 0; c < d; ++c) {
      double e = q[c] - states[(size_t)i * d + c];
      s += e * e;
    }
    if (s < b1) {
      b2 = b1;
      b1 = s;
      best = i;
    } else if (s < b2) {
      b2 = s;
    }
  }
  if (d2_best) *d2_best = b1;
  if (d2_second) *d2_second = b2;
  return best;
}

static double dist_to_goal(const orc_problem* p, const double* x) {
  double s2 = 0.0;
  for (int c = 0; c < p->npos; ++c) {
    double e = x[c] - (double)p->goal_c[c];
    s2 += e * e;
  }
  return sqrt(s2);
}

/* ------------------------------------------------------------------------ */
/* The planner state: one tree (Sec. IV-A: states, actions, parents, costs   */
/* and a node counter), the AO-x bound and the solutions found so far.      */
/* ------------------------------------------------------------------------ */
struct orc_plan {
  orc_problem p;
  /* owned copies of the problem arrays */
  float *dyn, *slo, *shi, *ulo, *uhi, *llo, *lhi, *wlo, *whi, *bc, *bh, *sc, *sr, *gc, *xi;
  double* states;   /* [n_cap][d] */
  double* actions;  /* [n_cap][m] */
  int* parents;     /* [n_cap] */
  double* costs;    /* [n_cap] */
  int n, round, iter, last_end;
  long total_iters, expansions, insertions;
  double c_best;
  orc_solution* sols;
  int n_sols, cap_sols;
  double* best_states;  /* [(n_edges+1)][d] */
  double* best_actions; /* [n_edges][m] */
  int best_edges;
  double best_cost;
  /* scratch */
  double *xnew, *cnew, *hval, *dbest, *dsecond;
  float *targets, *controls;
  int *par, *flags, *amb, *slots, *nntie;
};

static float* dup_f(const float* src, size_t n) {
  float* dst = (float*)malloc(sizeof(float) * (n ? n : 1));
  if (n && src) memcpy(dst, src, sizeof(float) * n);
  return dst;
}

static void reset_round(orc_plan* pl) {
  /* T <- {(x_init, none, 0)}  (Alg. 1, start of each outer iteration) */
  int d = pl->p.d, m = pl->p.m;
  for (int c = 0; c < d; ++c) pl->states[c] = (double)pl->p.x_init[c];
  for (int c = 0; c < m; ++c) pl->actions[c] = 0.0;
  pl->parents[0] = -1;
  pl->costs[0] = 0.0;
  pl->n = 1;
  pl->iter = 0;
}

orc_plan* orc_plan_create(const orc_problem* src) {
  orc_plan* pl = (orc_plan*)calloc(1, sizeof(orc_plan));
  pl->p = *src;
  orc_problem* p = &pl->p;
  int d = p->d, m = p->m, P = p->npos;
  pl->dyn = dup_f(src->dyn, 8);
  pl->slo = dup_f(src->sample_lo, d);
  pl->shi = dup_f(src->sample_hi, d);
  pl->ulo = dup_f(src->u_lo, m);
  pl->uhi = dup_f(src->u_hi, m);
  pl->llo = dup_f(src->lim_lo, d);
  pl->lhi = dup_f(src->lim_hi, d);
  pl->wlo = dup_f(src->ws_lo, P);
  pl->whi = dup_f(src->ws_hi, P);
  pl->bc = dup_f(src->box_c, (size_t)src->n_box * P);
  pl->bh = dup_f(src->box_h, (size_t)src->n_box * P);
  pl->sc = dup_f(src->sph_c, (size_t)src->n_sph * P);
  pl->sr = dup_f(src->sph_r, src->n_sph);
  pl->gc = dup_f(src->goal_c, P);
  pl->xi = dup_f(src->x_init, d);
  p->dyn = pl->dyn; p->sample_lo = pl->slo; p->sample_hi = pl->shi;
  p->u_lo = pl->ulo; p->u_hi = pl->uhi; p->lim_lo = pl->llo; p->lim_hi = pl->lhi;
  p->ws_lo = pl->wlo; p->ws_hi = pl->whi; p->box_c = pl->bc; p->box_h = pl->bh;
  p->sph_c = pl->sc; p->sph_r = pl->sr; p->goal_c = pl->gc; p->x_init = pl->xi;
  if (p->eps <= 0.0) p->eps = 1e-5;
  size_t N = (size_t)p->n_cap;
  pl->states = (double*)malloc(sizeof(double) * N * d);
  pl->actions = (double*)malloc(sizeof(double) * N * m);
  pl->parents = (int*)malloc(sizeof(int) * N);
  pl->costs = (double*)malloc(sizeof(double) * N);
  int B = p->B, K = p->B / p->A;
  pl->xnew = (double*)malloc(sizeof(double) * (size_t)B * d);
  pl->cnew = (double*)malloc(sizeof(double) * B);
  pl->hval = (double*)malloc(sizeof(double) * B);
  pl->dbest = (double*)malloc(sizeof(double) * K);
  pl->dsecond = (double*)malloc(sizeof(double) * K);
  pl->targets = (float*)malloc(sizeof(float) * (size_t)K * d);
  pl->controls = (float*)malloc(sizeof(float) * (size_t)B * m);
  pl->par = (int*)malloc(sizeof(int) * K);
  pl->nntie = (int*)malloc(sizeof(int) * K);
  pl->flags = (int*)malloc(sizeof(int) * B);
  pl->amb = (int*)malloc(sizeof(int) * B);
  pl->slots = (int*)malloc(sizeof(int) * B);
  pl->cap_sols = 64;
  pl->sols = (orc_solution*)malloc(sizeof(orc_solution) * pl->cap_sols);
  pl->c_best = p->c0;          /* c_best <- infinity (Alg. 1), or a given bound */
  pl->round = 0;
  pl->best_edges = -1;
  pl->best_cost = INFINITY;
  reset_round(pl);
  return pl;
}

void orc_plan_destroy(orc_plan* pl) {
  if (!pl) return;
  float* fs[] = {pl->dyn, pl->slo, pl->shi, pl->ulo, pl->uhi, pl->llo, pl->lhi, pl->wlo,
                 pl->whi, pl->bc, pl->bh, pl->sc, pl->sr, pl->gc, pl->xi, pl->targets,
                 pl->controls};
  for (size_t i = 0; i < sizeof(fs) / sizeof(fs[0]); ++i) free(fs[i]);
  free(pl->states); free(pl->actions); free(pl->parents); free(pl->costs);
  free(pl->xnew); free(pl->cnew); free(pl->hval); free(pl->dbest); free(pl->dsecond);
  free(pl->par); free(pl->nntie); free(pl->flags); free(pl->amb); free(pl->slots);
  free(pl->sols); free(pl->best_states); free(pl->best_actions);
  free(pl);
}

/* ExtractPath(T, x_new), Alg. 1: follow parent indices back to the root. */
static void save_path(orc_plan* pl, int node, double cost) {
  int d = pl->p.d, m = pl->p.m;
  int depth = 0;
  for (int s = node; pl->parents[s] >= 0; s = pl->parents[s]) ++depth;
  free(pl->best_states);
  free(pl->best_actions);
  pl->best_states = (double*)malloc(sizeof(double) * (size_t)(depth + 1) * d);
  pl->best_actions = (double*)malloc(sizeof(double) * (size_t)(depth ? depth : 1) * m);
  int s = node;
  for (int k = depth; k >= 0; --k) {
    memcpy(pl->best_states + (size_t)k * d, pl->states + (size_t)s * d, sizeof(double) * d);
    if (k > 0) memcpy(pl->best_actions + (size_t)(k - 1) * m, pl->actions + (size_t)s * m,
                      sizeof(double) * m);
    s = pl->parents[s];
  }
  pl->best_edges = depth;
  pl->best_cost = cost;
}

static int near_tie_nn(double d2a, double d2b, double eps) {
  double a = sqrt(d2a), b = sqrt(d2b);
  double scale = a > 1.0 ? a : 1.0;
  return fabs(b - a) <= eps * scale;
}

/* One inner iteration of Alg. 1 (sample, nearest neighbour, controls,
 * propagate, prune, collision check, insert, goal test) followed by the
 * outer-loop bookkeeping when the round ends. */
int orc_plan_iterate(orc_plan* pl, const orc_steer* steer, orc_report* rep) {
  orc_problem* p = &pl->p;
  int d = p->d, m = p->m, B = p->B, A = p->A, K = B / A;
  double eps = p->eps;
  int n0 = pl->n;
  double c_best = pl->c_best;  /* frozen for the whole batch */
  int n_steered = 0, n_mismatch = 0;

  /* X_rand <- SampleStates(B/A); X_near <- NearestNeighbor(T, X_rand) against
   * the tree as it stood at the start of the iteration (Sec. IV-B). */
  for (int k = 0; k < K; ++k) {
    float* q = pl->targets + (size_t)k * d;
    orc_sample_state(p, (uint32_t)k, (uint32_t)pl->iter, (uint32_t)pl->round, q);
    double qd[MAXD];
    for (int c = 0; c < d; ++c) qd[c] = (double)q[c];
    double b1, b2;
    int best = orc_nearest(pl->states, n0, d, qd, &b1, &b2);
    int tie = (n0 > 1) && near_tie_nn(b1, b2, eps);
    pl->nntie[k] = tie;
    if (steer && steer->parents) {
      int g = steer->parents[k];
      if (g != best) {
        int ok = 0;
        if (tie && g >= 0 && g < n0) {
          double s = 0.0;
          for (int c = 0; c < d; ++c) {
            double e = qd[c] - pl->states[(size_t)g * d + c];
            s += e * e;
          }
          ok = near_tie_nn(b1, s, eps);
          if (ok) b1 = s;
        }
        if (ok) { best = g; ++n_steered; } else { ++n_mismatch; }
      }
    }
    pl->par[k] = best;
    pl->dbest[k] = b1;
    pl->dsecond[k] = b2;
  }

  /* U <- SampleControls(B/A, A); Propagate; prune; CollisionFree. */
  for (int j = 0; j < B; ++j) {
    int k = j / A;
    float* uf = pl->controls + (size_t)j * m;
    orc_sample_control(p, (uint32_t)k, (uint32_t)(j - k * A), (uint32_t)pl->iter,
                       (uint32_t)pl->round, uf);
    double u[MAXM];
    for (int c = 0; c < m; ++c) u[c] = (double)uf[c];
    int par = pl->par[k];
    double* xT = pl->xnew + (size_t)j * d;
    int amb_valid = 0;
    int valid = orc_edge(p, pl->states + (size_t)par * d, pl->costs[par], u, xT, &pl->cnew[j],
                         &amb_valid);
    double h = orc_heuristic(p, xT);
    pl->hval[j] = h;
    /* cost-bounded pruning: keep iff g + h < c_best (strict) */
    double f = pl->cnew[j] + h;
    int prune_ok = f < c_best;
    int amb_prune = 0;
    if (isfinite(c_best)) {
      double scale = fabs(c_best) > 1.0 ? fabs(c_best) : 1.0;
      amb_prune = fabs(f - c_best) <= eps * scale;
    }
    /* goal test on the final state: closed ball around the goal centre */
    double dg = dist_to_goal(p, xT);
    int in_goal = dg <= (double)p->goal_r;
    int amb_goal = fabs(dg - (double)p->goal_r) <= eps;
    if (steer && steer->flags) {
      int gf = steer->flags[j];
      int gv = (gf & ORC_F_VALID) != 0;
      if (gv != valid) {
        if (amb_valid) { valid = gv; ++n_steered; } else { ++n_mismatch; }
      }
      if (valid) {
        int gp = (gf & ORC_F_PRUNE_OK) != 0, gg = (gf & ORC_F_GOAL) != 0;
        if (gp != prune_ok) {
          if (amb_prune) { prune_ok = gp; ++n_steered; } else { ++n_mismatch; }
        }
        if (gg != in_goal) {
          if (amb_goal) { in_goal = gg; ++n_steered; } else { ++n_mismatch; }
        }
      }
    }
    int fl = 0;
    if (valid) fl |= ORC_F_VALID;
    if (prune_ok) fl |= ORC_F_PRUNE_OK;
    if (valid && prune_ok) fl |= ORC_F_KEEP;
    if (in_goal) fl |= ORC_F_GOAL;
    pl->flags[j] = fl;
    pl->amb[j] = (amb_valid ? ORC_A_VALID : 0) | (amb_prune ? ORC_A_PRUNE : 0) |
                 (amb_goal ? ORC_A_GOAL : 0);
  }

  /* T <- T u {(x_new, u, c_new)}: survivors take consecutive slots at the
   * tree frontier in candidate order, up to the capacity (Sec. IV-A). */
  int n = n0, inserted = 0;
  for (int j = 0; j < B; ++j) {
    pl->slots[j] = -1;
    if (!(pl->flags[j] & ORC_F_KEEP)) continue;
    if (n >= p->n_cap) continue;
    int s = n++;
    pl->slots[j] = s;
    pl->flags[j] |= ORC_F_INSERTED;
    memcpy(pl->states + (size_t)s * d, pl->xnew + (size_t)j * d, sizeof(double) * d);
    for (int c = 0; c < m; ++c) pl->actions[(size_t)s * m + c] = (double)pl->controls[(size_t)j * m + c];
    pl->parents[s] = pl->par[j / A];
    pl->costs[s] = pl->cnew[j];
    ++inserted;
  }

  /* Goal reached: the cheapest inserted goal candidate (ties to the lowest j)
   * sets c_best and ends the round (the whole batch has been inserted). */
  int goal_j = -1, goal_tie = 0;
  for (int j = 0; j < B; ++j) {
    if ((pl->flags[j] & ORC_F_INSERTED) && (pl->flags[j] & ORC_F_GOAL)) {
      if (goal_j < 0 || pl->cnew[j] < pl->cnew[goal_j]) goal_j = j;
    }
  }
  if (goal_j >= 0) {
    double cg = pl->cnew[goal_j];
    double scale = fabs(cg) > 1.0 ? fabs(cg) : 1.0;
    for (int j = 0; j < B; ++j) {
      if (j == goal_j) continue;
      if ((pl->flags[j] & ORC_F_INSERTED) && (pl->flags[j] & ORC_F_GOAL) &&
          fabs(pl->cnew[j] - cg) <= eps * scale)
        goal_tie = 1;
    }
    if (steer && steer->goal_j != goal_j) {
      int g = steer->goal_j;
      if (goal_tie && g >= 0 && g < B && (pl->flags[g] & ORC_F_INSERTED) &&
          (pl->flags[g] & ORC_F_GOAL) && fabs(pl->cnew[g] - cg) <= eps * scale) {
        goal_j = g;
        ++n_steered;
      } else {
        ++n_mismatch;
      }
    }
  } else if (steer && steer->goal_j >= 0) {
    ++n_mismatch;
  }

  pl->n = n;
  pl->expansions += B;
  pl->insertions += inserted;
  pl->total_iters += 1;

  if (rep) {
    if (rep->targets) memcpy(rep->targets, pl->targets, sizeof(float) * (size_t)K * d);
    if (rep->parents) memcpy(rep->parents, pl->par, sizeof(int) * K);
    if (rep->nn_d2) memcpy(rep->nn_d2, pl->dbest, sizeof(double) * K);
    if (rep->nn_tie) memcpy(rep->nn_tie, pl->nntie, sizeof(int) * K);
    if (rep->controls) memcpy(rep->controls, pl->controls, sizeof(float) * (size_t)B * m);
    if (rep->xnew) memcpy(rep->xnew, pl->xnew, sizeof(double) * (size_t)B * d);
    if (rep->cnew) memcpy(rep->cnew, pl->cnew, sizeof(double) * B);
    if (rep->hval) memcpy(rep->hval, pl->hval, sizeof(double) * B);
    if (rep->flags) memcpy(rep->flags, pl->flags, sizeof(int) * B);
    if (rep->amb) memcpy(rep->amb, pl->amb, sizeof(int) * B);
    if (rep->slots) memcpy(rep->slots, pl->slots, sizeof(int) * B);
    rep->n0 = n0;
    rep->n1 = n;
    rep->round = pl->round;
    rep->iter = pl->iter;
    rep->goal_j = goal_j;
    rep->goal_slot = goal_j >= 0 ? pl->slots[goal_j] : -1;
    rep->c_best_before = c_best;
    rep->goal_tie = goal_tie;
  }

  int end = ORC_END_NONE;
  if (goal_j >= 0) {
    /* c_best <- c_new; sigma* <- ExtractPath; break to a fresh, tighter round */
    int s = pl->slots[goal_j];
    pl->c_best = pl->cnew[goal_j];
    save_path(pl, s, pl->c_best);
    if (pl->n_sols == pl->cap_sols) {
      pl->cap_sols *= 2;
      pl->sols = (orc_solution*)realloc(pl->sols, sizeof(orc_solution) * pl->cap_sols);
    }
    orc_solution* so = &pl->sols[pl->n_sols++];
    so->round = pl->round;
    so->iter = pl->iter;
    so->node = s;
    so->n_nodes = n;
    so->total_iter = pl->total_iters;
    so->cost = pl->c_best;
    end = ORC_END_GOAL;
  } else if (n >= p->n_cap) {
    end = ORC_END_TREE_FULL;
  } else if (pl->iter + 1 >= p->max_iters_per_round) {
    end = ORC_END_ITER_CAP;
  }
  if (rep) {
    rep->end_reason = end;
    rep->c_best_after = pl->c_best;
    rep->n_steered = n_steered;
    rep->n_mismatch = n_mismatch;
  }
  pl->last_end = end;
  if (end != ORC_END_NONE) {
    pl->round += 1;
    reset_round(pl);
  } else {
    pl->iter += 1;
  }
  return end;
}

/* Outer loop of Alg. 1 with a deterministic budget (rounds, iterations)
 * standing in for the wall-clock budget. */
int orc_plan_run(orc_plan* pl, int max_rounds, long max_iters) {
  long it = 0;
  int r0 = pl->round;
  while ((max_rounds <= 0 || pl->round - r0 < max_rounds) && (max_iters <= 0 || it < max_iters)) {
    orc_plan_iterate(pl, NULL, NULL);
    ++it;
  }
  return pl->n_sols;
}

void orc_plan_get(const orc_plan* pl, orc_state* out) {
  out->n = pl->n;
  out->round = pl->round;
  out->iter = pl->iter;
  out->n_solutions = pl->n_sols;
  out->last_end = pl->last_end;
  out->total_iters = pl->total_iters;
  out->expansions = pl->expansions;
  out->insertions = pl->insertions;
  out->c_best = pl->c_best;
}

int orc_plan_tree(const orc_plan* pl, double* states, double* actions, int* parents,
                  double* costs, int n_max) {
  int n = pl->n < n_max ? pl->n : n_max;
  int d = pl->p.d, m = pl->p.m;
  if (states) memcpy(states, pl->states, sizeof(double) * (size_t)n * d);
  if (actions) memcpy(actions, pl->actions, sizeof(double) * (size_t)n * m);
  if (parents) memcpy(parents, pl->parents, sizeof(int) * n);
  if (costs) memcpy(costs, pl->costs, sizeof(double) * n);
  return n;
}

/* Replace the tree by a float32 snapshot (node-major) and set the loop state,
 * so that a single iteration can be recomputed from another implementation's
 * tree. */
int orc_plan_load_tree(orc_plan* pl, const float* states, const float* actions,
                       const int* parents, const float* costs, int n, int round, int iter,
                       double c_best) {
  int d = pl->p.d, m = pl->p.m;
  if (n < 1 || n > pl->p.n_cap) return -1;
  for (size_t i = 0; i < (size_t)n * d; ++i) pl->states[i] = (double)states[i];
  for (size_t i = 0; i < (size_t)n * m; ++i) pl->actions[i] = actions ? (double)actions[i] : 0.0;
  for (int i = 0; i < n; ++i) {
    pl->parents[i] = parents ? parents[i] : -1;
    pl->costs[i] = (double)costs[i];
  }
  pl->n = n;
  pl->round = round;
  pl->iter = iter;
  pl->c_best = c_best;
  return 0;
}

int orc_plan_solutions(const orc_plan* pl, orc_solution* out, int cap) {
  int n = pl->n_sols < cap ? pl->n_sols : cap;
  if (out) memcpy(out, pl->sols, sizeof(orc_solution) * n);
  return pl->n_sols;
}

int orc_plan_best_path(const orc_plan* pl, double* states, double* actions, int cap_edges,
                       int* n_edges, double* cost) {
  if (pl->best_edges < 0) {
    *n_edges = 0;
    return -1;
  }
  *n_edges = pl->best_edges;
  if (cost) *cost = pl->best_cost;
  if (pl->best_edges > cap_edges) return -2;
  int d = pl->p.d, m = pl->p.m;
  if (states) memcpy(states, pl->best_states, sizeof(double) * (size_t)(pl->best_edges + 1) * d);
  if (actions) memcpy(actions, pl->best_actions, sizeof(double) * (size_t)pl->best_edges * m);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Trajectory refinement objective, evaluated in complex arithmetic so that  */
/* the complex-step method gives its exact gradient.  For a real input the   */
/* imaginary parts stay zero and this is the plain FP64 objective.  The      */
/* dynamics are written again here over complex numbers (no shared code      */
/* with the real-valued planner functions above).                           */
/* ------------------------------------------------------------------------ */
#include <complex.h>

typedef double complex cplx;

/* branch on the real part, keep the derivative of the active branch */
static cplx c_abs(cplx z) { return creal(z) >= 0.0 ? z : -z; }
static cplx c_max(cplx a, cplx b) { return creal(a) >= creal(b) ? a : b; }
static cplx c_min(cplx a, cplx b) { return creal(a) <= creal(b) ? a : b; }

static cplx c_softplus(cplx z, double beta) {
  /* log(1 + exp(beta z)) / beta, evaluated without overflow */
  cplx bz = beta * z;
  if (creal(bz) > 0.0) return (bz + clog(1.0 + cexp(-bz))) / beta;
  return clog(1.0 + cexp(bz)) / beta;
}

static void c_dynamics(const orc_problem* p, const cplx* x, const cplx* u, cplx* xd) {
  if (p->system == ORC_DI2 || p->system == ORC_DI3) {
    int D = p->npos;
    for (int a = 0; a < D; ++a) {
      xd[a] = x[D + a];
      xd[D + a] = u[a];
    }
  } else if (p->system == ORC_CAR) {
    double L = (double)p->dyn[0];
    xd[0] = x[3] * ccos(x[2]);
    xd[1] = x[3] * csin(x[2]);
    xd[2] = x[3] * ctan(x[4]) / L;
    xd[3] = u[0];
    xd[4] = u[1];
  } else if (p->system == ORC_DUBINS) {
    xd[0] = x[5] * ccos(x[3]) * ccos(x[4]);
    xd[1] = x[5] * csin(x[3]) * ccos(x[4]);
    xd[2] = x[5] * csin(x[4]);
    xd[3] = u[0];
    xd[4] = u[1];
    xd[5] = u[2];
  } else if (p->system == ORC_UNI1) {
    xd[0] = u[0] * ccos(x[2]);
    xd[1] = u[0] * csin(x[2]);
    xd[2] = u[1];
  } else if (p->system == ORC_UNI2) {
    xd[0] = x[3] * ccos(x[2]);
    xd[1] = x[3] * csin(x[2]);
    xd[2] = x[4];
    xd[3] = u[0];
    xd[4] = u[1];
  } else if (p->system == ORC_ACROBOT) {
    const double m1 = p->dyn[0], m2 = p->dyn[1], l1 = p->dyn[2], lc1 = p->dyn[3];
    const double lc2 = p->dyn[4], I1 = p->dyn[5], I2 = p->dyn[6], g = p->dyn[7];
    const double k = m2 * l1 * lc2;
    const cplx q1 = x[0], q2 = x[1], w1 = x[2], w2 = x[3];
    const cplx M00 = m1 * lc1 * lc1 + m2 * (l1 * l1 + lc2 * lc2) + I1 + I2 + 2.0 * k * ccos(q2);
    const cplx M01 = m2 * lc2 * lc2 + I2 + k * ccos(q2);
    const cplx M11 = m2 * lc2 * lc2 + I2;
    const cplx c1 = -k * csin(q2) * (w2 * w2 + 2.0 * w1 * w2);
    const cplx c2 = k * csin(q2) * w1 * w1;
    const cplx g2 = m2 * lc2 * g * csin(q1 + q2);
    const cplx g1 = (m1 * lc1 + m2 * l1) * g * csin(q1) + g2;
    const cplx r0 = -c1 - g1, r1 = u[0] - c2 - g2;
    const cplx det = M00 * M11 - M01 * M01;
    xd[0] = w1;
    xd[1] = w2;
    xd[2] = (M11 * r0 - M01 * r1) / det;
    xd[3] = (M00 * r1 - M01 * r0) / det;
  } else if (p->system == ORC_CARTPOLE) {
    const double l = p->dyn[0], g = p->dyn[1];
    xd[0] = x[2];
    xd[1] = x[3];
    xd[2] = u[0];
    xd[3] = (g * csin(x[1]) - u[0] * ccos(x[1])) / l;
  } else {
    double mass = p->dyn[0], g = p->dyn[1], Ix = p->dyn[2], Iy = p->dyn[3], Iz = p->dyn[4];
    cplx cph = ccos(x[3]), sph = csin(x[3]), cth = ccos(x[4]), sth = csin(x[4]);
    cplx cps = ccos(x[5]), sps = csin(x[5]);
    cplx R[3][3] = {{cps * cth, cps * sth * sph - sps * cph, cps * sth * cph + sps * sph},
                    {sps * cth, sps * sth * sph + cps * cph, sps * sth * cph - cps * sph},
                    {-sth, cth * sph, cth * cph}};
    cplx v[3] = {x[6], x[7], x[8]}, w[3] = {x[9], x[10], x[11]};
    for (int i = 0; i < 3; ++i) xd[i] = R[i][0] * v[0] + R[i][1] * v[1] + R[i][2] * v[2];
    cplx a = w[1] * sph + w[2] * cph;
    xd[3] = w[0] + a * sth / cth;
    xd[4] = w[1] * cph - w[2] * sph;
    xd[5] = a / cth;
    cplx wxv[3] = {w[1] * v[2] - w[2] * v[1], w[2] * v[0] - w[0] * v[2], w[0] * v[1] - w[1] * v[0]};
    for (int i = 0; i < 3; ++i) xd[6 + i] = -wxv[i] - g * R[2][i];
    xd[8] += u[0] / mass;
    xd[9] = (u[1] - (Iz - Iy) * w[1] * w[2]) / Ix;
    xd[10] = (u[2] - (Ix - Iz) * w[2] * w[0]) / Iy;
    xd[11] = (u[3] - (Iy - Ix) * w[0] * w[1]) / Iz;
  }
}

static void c_rk4(const orc_problem* p, cplx* x, const cplx* u, double h) {
  int d = p->d;
  cplx k1[MAXD], k2[MAXD], k3[MAXD], k4[MAXD], t[MAXD];
  c_dynamics(p, x, u, k1);
  for (int i = 0; i < d; ++i) t[i] = x[i] + 0.5 * h * k1[i];
  c_dynamics(p, t, u, k2);
  for (int i = 0; i < d; ++i) t[i] = x[i] + 0.5 * h * k2[i];
  c_dynamics(p, t, u, k3);
  for (int i = 0; i < d; ++i) t[i] = x[i] + h * k3[i];
  c_dynamics(p, t, u, k4);
  for (int i = 0; i < d; ++i) x[i] = x[i] + h / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
}

/* smooth penalty of one state: obstacles, workspace, limits, speed norm */
static cplx c_state_penalty(const orc_problem* p, const orc_refine* rp, const cplx* x) {
  int P = p->npos;
  double beta = rp->beta;
  cplx pen = 0.0;
  for (int b = 0; b < p->n_box; ++b) {
    cplx q[3], outside = 0.0, inner = -INFINITY;
    for (int c = 0; c < P; ++c) {
      q[c] = c_abs(x[c] - (double)p->box_c[b * P + c]) - (double)p->box_h[b * P + c];
      cplx qp = c_max(q[c], 0.0);
      outside += qp * qp;
      inner = c == 0 ? q[c] : c_max(inner, q[c]);
    }
    cplx sd = (creal(outside) > 0.0 ? csqrt(outside) : 0.0) + c_min(inner, 0.0);
    pen += c_softplus(rp->delta - sd, beta);
  }
  for (int s = 0; s < p->n_sph; ++s) {
    cplx r2 = 0.0;
    for (int c = 0; c < P; ++c) {
      cplx e = x[c] - (double)p->sph_c[s * P + c];
      r2 += e * e;
    }
    pen += c_softplus(rp->delta - (csqrt(r2) - (double)p->sph_r[s]), beta);
  }
  for (int c = 0; c < P; ++c) {
    pen += c_softplus(x[c] - (double)p->ws_hi[c], beta);
    pen += c_softplus((double)p->ws_lo[c] - x[c], beta);
  }
  for (int i = P; i < p->d; ++i) {
    if (!isinf(p->lim_hi[i])) pen += c_softplus(x[i] - (double)p->lim_hi[i], beta);
    if (!isinf(p->lim_lo[i])) pen += c_softplus((double)p->lim_lo[i] - x[i], beta);
  }
  if (p->vnorm_max > 0.0f) {
    cplx v2 = 0.0;
    for (int c = 0; c < P; ++c) v2 += x[P + c] * x[P + c];
    pen += c_softplus(csqrt(v2) - (double)p->vnorm_max, beta);
  }
  return pen;
}

static cplx c_traj_cost(const orc_problem* p, const orc_refine* rp, const double* x0,
                        const cplx* U, int M) {
  int d = p->d, m = p->m, P = p->npos;
  double h = (double)p->dt, edge_t = (double)p->T * h;
  cplx x[MAXD];
  for (int i = 0; i < d; ++i) x[i] = x0[i];
  cplx J = 0.0;
  for (int e = 0; e < M; ++e) {
    const cplx* u = U + (size_t)e * m;
    for (int c = 0; c < m; ++c) {
      cplx z = (u[c] - rp->u_ref[c]) / rp->u_scale[c];
      J += rp->w_u * edge_t * z * z;
    }
    for (int t = 0; t < p->T; ++t) {
      c_rk4(p, x, u, h);
      J += rp->w_c * c_state_penalty(p, rp, x);
    }
  }
  for (int c = 0; c < P; ++c) {
    cplx e = x[c] - (double)p->goal_c[c];
    J += rp->w_g * e * e;
  }
  return J;
}

double orc_traj_cost(const orc_problem* p, const orc_refine* rp, const double* x0,
                     const double* U, int M) {
  int n = M * p->m;
  cplx* Uc = (cplx*)malloc(sizeof(cplx) * (size_t)(n ? n : 1));
  for (int i = 0; i < n; ++i) Uc[i] = U[i];
  double J = creal(c_traj_cost(p, rp, x0, Uc, M));
  free(Uc);
  return J;
}

void orc_traj_grad(const orc_problem* p, const orc_refine* rp, const double* x0,
                   const double* U, int M, double* grad) {
  const double hstep = 1e-30;
  int n = M * p->m;
  cplx* Uc = (cplx*)malloc(sizeof(cplx) * (size_t)(n ? n : 1));
  for (int i = 0; i < n; ++i) Uc[i] = U[i];
  for (int i = 0; i < n; ++i) {
    Uc[i] = U[i] + I * hstep;
    grad[i] = cimag(c_traj_cost(p, rp, x0, Uc, M)) / hstep;
    Uc[i] = U[i];
  }
  free(Uc);
}
