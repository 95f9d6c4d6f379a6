/*
 * FP64 reference planner for PAKR (parallel AO kinodynamic RRT) -- TEST
 * INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library; the product path never
 * does.  It shares no code with the HIP implementation.
 *
 * What it computes: Alg. 1 of the paper (AO-x outer loop around a batched
 * kinodynamic RRT) step by step, in double precision, with the sampled
 * values (targets and controls) defined as float32 results of a
 * Philox4x32-10 stream so that both implementations draw identical samples.
 *
 * Near-tie handling: every decision (nearest neighbour, edge validity, cost
 * bound prune, goal test, goal arg-min) reports whether it lies within eps of
 * flipping.  When an optional "steer" record is supplied (the decisions of
 * another implementation), the reference adopts that record's choice for
 * near-tie decisions only, counts the adoptions, and counts every
 * disagreement on a decision that is not a near tie as a mismatch.
 *
 * Every real input is given as float32 (the planner is defined on those exact
 * values) and is read here as an exact double.
 */
#ifndef PAKR_ORACLE_H
#define PAKR_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_DI2 = 0, ORC_DI3 = 1, ORC_CAR = 2, ORC_QUAD = 3, ORC_DUBINS = 4, ORC_UNI1 = 5,
       ORC_UNI2 = 6, ORC_ACROBOT = 7, ORC_CARTPOLE = 8 };
enum { ORC_COST_DURATION = 0, ORC_COST_PATH_LENGTH = 1 };
enum { ORC_H_ADMISSIBLE = 0, ORC_H_PAPER_LITERAL = 1, ORC_H_NONE = 2 };

/* candidate flag bits */
enum { ORC_F_VALID = 1, ORC_F_PRUNE_OK = 2, ORC_F_KEEP = 4, ORC_F_GOAL = 8, ORC_F_INSERTED = 16 };
/* near-tie bits per candidate */
enum { ORC_A_VALID = 1, ORC_A_PRUNE = 2, ORC_A_GOAL = 4 };
/* why a round ended */
enum { ORC_END_NONE = 0, ORC_END_GOAL = 1, ORC_END_TREE_FULL = 2, ORC_END_ITER_CAP = 3 };

typedef struct {
  int system, d, m, npos;
  const float* dyn;          /* [8]  CAR: wheelbase; QUAD: mass, g, Ixx, Iyy, Izz */
  const float* sample_lo;    /* [d] */
  const float* sample_hi;    /* [d] */
  const float* u_lo;         /* [m] */
  const float* u_hi;         /* [m] */
  const float* lim_lo;       /* [d]  +-inf: no limit */
  const float* lim_hi;       /* [d] */
  float vnorm_max;           /* speed-norm limit (0: none) */
  const float* ws_lo;        /* [npos] */
  const float* ws_hi;        /* [npos] */
  int n_box;
  const float* box_c;        /* [n_box][npos] */
  const float* box_h;        /* [n_box][npos] */
  int n_sph;
  const float* sph_c;        /* [n_sph][npos] */
  const float* sph_r;        /* [n_sph] */
  const float* goal_c;       /* [npos] */
  float goal_r;
  const float* x_init;       /* [d] */
  int B, A, T;
  float dt;
  int n_cap;
  int cost_kind, h_kind;
  float h_speed;
  double c0;                 /* initial cost bound (+inf: none) */
  uint64_t seed;
  uint32_t qid;
  int max_iters_per_round;
  double eps;                /* near-tie band, 1e-5 */
} orc_problem;

/* Decisions of another implementation for one iteration (all nullable). */
typedef struct {
  const int* parents;        /* [K] */
  const int* flags;          /* [B] ORC_F_VALID / ORC_F_PRUNE_OK / ORC_F_GOAL bits used */
  int goal_j;                /* chosen goal candidate, -1 none */
} orc_steer;

/* Per-iteration report; every array is caller-owned and nullable. */
typedef struct {
  float* targets;            /* [K][d] */
  int* parents;              /* [K] */
  double* nn_d2;             /* [K] squared distance to the chosen parent */
  int* nn_tie;               /* [K] 1 if the arg-min is a near tie */
  float* controls;           /* [B][m] */
  double* xnew;              /* [B][d] */
  double* cnew;              /* [B] */
  double* hval;              /* [B] */
  int* flags;                /* [B] ORC_F_* */
  int* amb;                  /* [B] ORC_A_* */
  int* slots;                /* [B] tree slot of inserted candidates, else -1 */
  int n0, n1, round, iter, goal_j, goal_slot, end_reason;
  double c_best_before, c_best_after;
  int n_steered, n_mismatch, goal_tie;
} orc_report;

typedef struct {
  int round, iter, node, n_nodes;
  long total_iter;
  double cost;
} orc_solution;

typedef struct {
  int n, round, iter, n_solutions, last_end;
  long total_iters, expansions, insertions;
  double c_best;
} orc_state;

typedef struct orc_plan orc_plan;

/* --- primitives --------------------------------------------------------- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
float orc_u32_to_range(uint32_t x, float lo, float hi);
void orc_sample_state(const orc_problem* p, uint32_t k, uint32_t iter, uint32_t round, float* out);
void orc_sample_control(const orc_problem* p, uint32_t k, uint32_t a, uint32_t iter,
                        uint32_t round, float* out);
void orc_u32_to_range_n(const uint32_t* x, int n, float lo, float hi, float* out);
void orc_dynamics(const orc_problem* p, const double* x, const double* u, double* xdot);
void orc_rk4_step(const orc_problem* p, const double* x, const double* u, double h, double* out);
void orc_rollout(const orc_problem* p, const double* x0, const double* u, int T, double h,
                 double* states /* [(T+1)][d] */);
/* 1 valid, 0 invalid; *near set to 1 if any check lies within eps of flipping;
 * *margin receives the signed margin of the closest check (>0 valid side). */
int orc_state_valid(const orc_problem* p, const double* x, double eps, int* near,
                    double* margin);
/* One edge: T RK4 steps from (x0, c0) under held control u.  Returns the
 * validity decision; *amb is 1 when it is a near tie. */
int orc_edge(const orc_problem* p, const double* x0, double c0, const double* u, double* xT,
             double* cost, int* amb);
double orc_heuristic(const orc_problem* p, const double* x);
int orc_nearest(const double* states, int n, int d, const double* q, double* d2_best,
                double* d2_second);

/* --- planner ------------------------------------------------------------ */
orc_plan* orc_plan_create(const orc_problem* p);
void orc_plan_destroy(orc_plan* pl);
int orc_plan_iterate(orc_plan* pl, const orc_steer* steer, orc_report* rep);
int orc_plan_run(orc_plan* pl, int max_rounds, long max_iters);
void orc_plan_get(const orc_plan* pl, orc_state* out);
int orc_plan_tree(const orc_plan* pl, double* states, double* actions, int* parents,
                  double* costs, int n_max);
int orc_plan_load_tree(orc_plan* pl, const float* states, const float* actions,
                       const int* parents, const float* costs, int n, int round, int iter,
                       double c_best);
int orc_plan_solutions(const orc_plan* pl, orc_solution* out, int cap);
int orc_plan_best_path(const orc_plan* pl, double* states, double* actions, int cap_edges,
                       int* n_edges, double* cost);

/* --- trajectory refinement objective ----------------------------------
 * A trajectory holds control U[e] (e < M) for T steps of dt each from x0.
 * J = w_u * sum_e T*dt * sum_c ((U[e][c] - u_ref[c]) / u_scale[c])^2
 *   + w_g * |pos(x_N) - goal|^2
 *   + w_c * sum_{n=1..N} [ sum_obstacles sp(delta - sd(pos(x_n)))
 *                          + sum_{bounded dims} sp(x - hi) + sp(lo - x)
 *                          + (double integrators) sp(|v| - vmax) ]
 * with N = M*T, sp(z) = log(1 + exp(beta z)) / beta and sd the signed
 * distance to a sphere (|p-c| - r) or a box (outside: |max(|p-c|-h, 0)|;
 * inside: max_i(|p-c|_i - h_i)); the workspace box counts as bounds on the
 * position dimensions. */
typedef struct {
  double w_u, w_g, w_c, beta, delta;
  double u_ref[4], u_scale[4];
} orc_refine;

double orc_traj_cost(const orc_problem* p, const orc_refine* rp, const double* x0,
                     const double* U, int M);
/* dJ/dU by the complex-step method (step 1e-30): exact to rounding, and
 * independent of any adjoint. */
void orc_traj_grad(const orc_problem* p, const orc_refine* rp, const double* x0,
                   const double* U, int M, double* grad);

#ifdef __cplusplus
}
#endif
#endif
