/*
 * pakr.h -- C ABI of the MI355X (gfx950) PAKR planner library (libpakr.so).
 *
 * PAKR is the parallel asymptotically optimal kinodynamic RRT of
 * "Fast Asymptotically Optimal Kinodynamic Planning via Vectorization"
 * (Gao, Lu, Kingston).  The library runs Alg. 1 of the paper on one GPU:
 * an AO-x outer loop (restart with a tighter cost bound c_best after every
 * solution) around a batched kinodynamic RRT whose inner iteration samples
 * K = B/A target states, finds each target's nearest tree node, samples A
 * controls per selected parent, rolls all B candidates out with RK4 for T
 * steps of dt with the control held, checks every sub-step for validity,
 * prunes candidates whose cost-to-come plus heuristic is not below c_best,
 * and appends the survivors to the tree in candidate order.
 *
 * The problem statement (Sec. III) fixes the inputs: dynamics f, start
 * x_init in X_free, goal region X_goal, cost J, control space U; Alg. 1 adds
 * the batch size B and branching factor A; Sec. IV-A adds the step dt, the
 * step count T and the static tree capacity N.
 *
 * Conventions
 *  - All entry points return int: PAKR_OK (0) or a negative pakr_error.
 *    No C++ exception crosses the ABI.  pakr_last_error() gives a message.
 *  - Host pointers (marked "host") are read during the call only; the caller
 *    keeps ownership.  Device pointers (marked "device") must stay valid for
 *    as long as the plan uses them.
 *  - `stream` is a hipStream_t passed as void*.  Calls marked "async" only
 *    enqueue work on that stream; calls marked "syncs" wait for it.
 *  - Real-valued inputs are float32: the planner is defined on those exact
 *    values.  The device path computes in float32.
 *  - Random draws use Philox4x32-10 (Salmon et al., SC'11) with key
 *    (low 32 bits of seed, query_id) and counter (index, iteration in round,
 *    round, tag << 16 | sub): tag 0 draws targets (index = target k, sub =
 *    block of four state dimensions), tag 1 draws controls (index = parent
 *    query k, sub = branch a).  A u32 word x maps to [lo, hi] as
 *    lo + (hi - lo) * ((x >> 8) * 2^-24) with one float32 rounding per
 *    operation and no fused multiply-add.
 */
#ifndef PAKR_H
#define PAKR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PAKR_MAX_D 12          /* largest state dimension (quadrotor) */
#define PAKR_MAX_M 4           /* largest control dimension */
#define PAKR_MAX_OBSTACLES 1024 /* boxes + spheres per scene (held in LDS) */
#define PAKR_MAX_B 65536       /* rollouts per iteration */

/* Systems (Sec. V-A names the double integrator and the quadcopter; the
 * second-order car is a unicycle-2-like model with steering). */
enum pakr_system_id {
  PAKR_DI2 = 0,  /* 2D double integrator: x=(px,py,vx,vy), u=(ax,ay)        */
  PAKR_DI3 = 1,  /* 3D double integrator: x=(p, v) in R^6, u=a in R^3       */
  PAKR_CAR = 2,  /* car: x=(px,py,theta,v,phi), u=(accel, steering rate)     */
  PAKR_QUAD = 3, /* quadrotor: x=(p, roll,pitch,yaw, body vel, body rates),
                    u=(thrust, tau_x, tau_y, tau_z)                          */
  PAKR_DUBINS = 4, /* Dubins airplane (Sec. V-A): x=(p in R^3, yaw, pitch,
                      speed), u=(yaw rate, pitch rate, acceleration)         */
  PAKR_UNI1 = 5, /* unicycle 1 (Sec. V-C): x=(px,py,heading),
                    u=(speed, turn rate)                                     */
  PAKR_UNI2 = 6, /* unicycle 2 (Sec. V-C): x=(px,py,heading,speed,turn rate),
                    u=(acceleration, angular acceleration)                   */
  PAKR_ACROBOT = 7, /* acrobot (Sec. V-C): x=(shoulder angle from hanging,
                       elbow angle, their rates), u=(elbow torque)           */
  PAKR_CARTPOLE = 8 /* cart-pole (Sec. V-E): x=(cart position, pole angle from
                       upright, cart speed, pole rate), u=(cart acceleration) */
};

/* Cost J (Sec. III): trajectory duration or path length of the positions. */
enum pakr_cost_kind { PAKR_COST_DURATION = 0, PAKR_COST_PATH_LENGTH = 1 };

/* Heuristic h of the prune g + h < c_best (Alg. 1).  ADMISSIBLE measures the
 * position distance to the goal ball and divides it by h_speed for a duration
 * cost; PAPER_LITERAL is the Euclidean position distance to the goal centre;
 * NONE is 0. */
enum pakr_heuristic_kind { PAKR_H_ADMISSIBLE = 0, PAKR_H_PAPER_LITERAL = 1, PAKR_H_NONE = 2 };

enum pakr_error {
  PAKR_OK = 0,
  PAKR_E_INVALID_ARG = -1,          /* malformed sizes, pointers or parameters   */
  PAKR_E_START_INVALID = -2,        /* x_init outside X_free or its limits       */
  PAKR_E_GOAL_INVALID = -3,         /* goal centre outside the workspace, r <= 0 */
  PAKR_E_WORKSPACE_TOO_SMALL = -4,  /* ws_bytes < pakr_workspace_size()          */
  PAKR_E_HIP = -5,                  /* a HIP runtime call failed                 */
  PAKR_E_NO_SOLUTION = -6,          /* no solution found yet                     */
  PAKR_E_BUFFER_TOO_SMALL = -7,     /* caller buffer cannot hold the result      */
  PAKR_E_DEVICE = -8                /* a grid barrier timed out on the device; the plan
                                       or batch refuses every later launch          */
};

/* Status bits reported in pakr_stats.status (why the last call stopped). */
enum pakr_status_bits {
  PAKR_S_SOLVED = 1,          /* at least one solution exists               */
  PAKR_S_BUDGET_EXPIRED = 2,  /* the device-clock budget ran out            */
  PAKR_S_ROUNDS_DONE = 4,     /* max_rounds rounds completed                */
  PAKR_S_ITERS_DONE = 8,      /* the iteration budget of the call was used  */
  PAKR_S_TREE_FULL = 16,      /* some round ended with a full tree          */
  PAKR_S_ITER_CAP = 32,       /* some round hit max_iters_per_round         */
  PAKR_S_DEVICE_ERROR = 64    /* the call's guard time (its budget + 60 s of device
                                 clock) ran out; a grid barrier that times out is
                                 reported as PAKR_E_DEVICE instead             */
};

/* Dynamics and limits of one system.  Every field is required; the Python
 * package fills it from a per-system table. */
typedef struct pakr_system {
  int id;                          /* pakr_system_id                                  */
  int d, m;                        /* state / control dimension, must match id        */
  float dyn[8];                    /* CAR: [0]=wheelbase; QUAD: mass, g, Ixx, Iyy, Izz;
                                      ACROBOT: m1, m2, l1, lc1, lc2, I1, I2, g (lc: pivot
                                      to centre of mass, I about it); CARTPOLE: pole
                                      length, g                                       */
  float sample_lo[PAKR_MAX_D];     /* SampleStates box per state dimension            */
  float sample_hi[PAKR_MAX_D];
  float u_lo[PAKR_MAX_M];          /* control box U                                   */
  float u_hi[PAKR_MAX_M];
  float lim_lo[PAKR_MAX_D];        /* state limits, valid iff lim_lo <= x <= lim_hi;   */
  float lim_hi[PAKR_MAX_D];        /*   use -/+INFINITY for "no limit"                */
  float vnorm_max;                 /* |velocity| <= vnorm_max (double integrators); 0 = none */
} pakr_system;

/* Workspace and obstacles (host arrays, copied by pakr_plan_init).  A point
 * robot at the first npos state coordinates must lie in the closed box
 * [ws_lo, ws_hi] and outside every closed obstacle. */
typedef struct pakr_scene {
  int npos;                        /* 2 (DI2, CAR) or 3 (DI3, QUAD)                    */
  float ws_lo[3], ws_hi[3];
  int n_box;                       /* axis-aligned boxes                              */
  const float* box_c;              /* host [n_box][npos] centres                      */
  const float* box_h;              /* host [n_box][npos] half extents (> 0)           */
  int n_sphere;                    /* spheres (discs when npos = 2)                   */
  const float* sph_c;              /* host [n_sphere][npos] centres                   */
  const float* sph_r;              /* host [n_sphere] radii (> 0)                     */
} pakr_scene;

/* Goal region: closed ball of `radius` around `center` in position space. */
typedef struct pakr_goal {
  float center[3];
  float radius;
} pakr_goal;

typedef struct pakr_params {
  int B;                           /* rollouts per iteration, 1..PAKR_MAX_B, B % A == 0 */
  int A;                           /* branching factor, controls per selected parent    */
  int T;                           /* RK4 steps per edge (>= 1)                          */
  float dt;                        /* step length (> 0)                                 */
  int n_cap;                       /* tree capacity N (root included), > B              */
  int cost_kind;                   /* pakr_cost_kind                                    */
  int heuristic_kind;              /* pakr_heuristic_kind                               */
  float h_speed;                   /* speed bound used by PAKR_H_ADMISSIBLE + duration  */
  double cost_bound;               /* initial c_best, +INFINITY for none (> 0)          */
  uint64_t seed;                   /* Philox key word 0 = low 32 bits                   */
  uint32_t query_id;               /* Philox key word 1                                 */
  int max_iters_per_round;         /* a round with no solution ends after this many     */
  int grid;                        /* workgroups of the persistent launch, 0 = auto     */
  int max_path_edges;              /* capacity of the stored best path, 0 = 4096        */
  int lanes_per_candidate;         /* 1, 2, 4, 8 or 16 lanes share one rollout and split its
                                      obstacle tests; 0 = auto (from the obstacle count) */
  int workgroups_per_cu;           /* with grid = 0: launch this many workgroups per CU
                                      and reserve LDS so that no CU holds more; 0 = 1    */
  int spec_tiles;                  /* NN tiles each workgroup without a rollout chunk scans
                                      ahead for the next iteration while the others roll
                                      out (the tree is frozen then; results do not depend
                                      on it): 0 = auto, -1 = none, else 1..1024          */
  int tier0_nodes;                 /* first tier of the tree (Sec. IV-A's memory tiers): while
                                      a round's tree has at most this many nodes, one
                                      workgroup runs each iteration alone and the grid takes
                                      over beyond it (results do not depend on it); 0 = auto
                                      (a power of 4 from the query's sizes), -1 = none.
                                      Single-query plans only: a batch's team always plans
                                      together                                            */
  int tier1_nodes;                 /* sub-grid tiers beyond the first: while a round's tree
                                      has more than tier0_nodes nodes and fits a sub-grid
                                      tier, only that tier's first workgroups run each
                                      iteration (their barriers are cheaper; results do not
                                      depend on it).  0 = auto: grids doubling from
                                      tier1_grid up to the whole grid, each taking the trees
                                      whose NN scan costs each of its workgroups at most
                                      tier_scan_cycles; > 0 = one sub-grid tier of
                                      tier1_grid workgroups up to this many nodes; -1 =
                                      none.  Single-query plans only                      */
  int tier1_grid;                  /* workgroups of the first sub-grid tier, 0 = auto (at
                                      least the rollout workgroups of one batch and 32, a
                                      power of two), else 2..grid                         */
  int tier_scan_cycles;            /* auto sub-grid tiers: the NN scan cycles per workgroup
                                      and iteration (K x nodes x (2d + 1) / 64 / workgroups)
                                      up to which a tier keeps the tree; 0 = 10000        */
} pakr_params;

typedef struct pakr_stats {
  int n_nodes;                     /* nodes in the current round's tree                 */
  int round;                       /* current AO-x round (0-based)                      */
  int iter;                        /* iteration within the current round                */
  int status;                      /* pakr_status_bits of the last call                 */
  int n_solutions;                 /* solutions found since pakr_plan_init              */
  int grid;                        /* workgroups used by the persistent launch          */
  long long total_iters;           /* inner iterations since pakr_plan_init             */
  long long expansions;            /* candidates rolled out (B per iteration)           */
  long long insertions;            /* nodes inserted                                    */
  long long nn_pairs;              /* (query, node) distance evaluations                */
  double c_best;                   /* current bound (+INFINITY before the first solution) */
  double call_ms;                  /* device-clock duration of the last call            */
  double t_first_ms;               /* device time of the first solution of the last call, -1 */
  double t_last_ms;                /* device time of its last solution, -1              */
  int call_iters;                  /* iterations run by the last call                   */
  int call_rounds;                 /* rounds completed by the last call                 */
  int call_solutions;              /* solutions found by the last call                  */
  int reserved;
  double nn_ms;                    /* last call, device time in SampleStates + NN       */
  double rollout_ms;               /* ... in controls, rollout, validity and prune      */
  double insert_ms;                /* ... in insertion, goal test and bookkeeping       */
  double step_ms[6];               /* finer split, seen by workgroup 0: NN scan, wait at the
                                      first grid barrier, parent reduction, rollout, wait at
                                      the second barrier, insertion + bookkeeping        */
  double clock_start_ms;           /* device clock (ms) when the last call started this query */
  double clock_end_ms;             /* ... and when it finished it                        */
  /* Near ties since pakr_plan_init: valid candidates whose prune decision
   * c + h < c_best had |c + h - c_best| <= 1e-5 * max(1, c_best), and whose
   * goal test had | |pos - g| - r | <= 1e-5 -- decisions that float32 and an
   * FP64 evaluation may take differently.  (Nearest-neighbour and obstacle-
   * margin ties would need the second-best distance and every sub-step's
   * signed margin; they are not counted here.) */
  long long near_ties_prune;
  long long near_ties_goal;
  /* The plan's tiers of the tree: while a round's tree has at most tier_nodes[k]
   * nodes, only the first tier_grid[k] workgroups run an iteration (ascending;
   * unused entries 0; larger trees use all `grid` workgroups).  A first tier
   * has tier_grid 1.  All 0 for a batch's queries. */
  int tier_nodes[8];
  int tier_grid[8];
} pakr_stats;

typedef struct pakr_solution {
  int round, iter;                 /* when it was found                                 */
  int node;                        /* tree slot of the goal node                        */
  int n_nodes;                     /* tree size at that iteration                       */
  long long total_iter;            /* global iteration index                            */
  double cost;                     /* its cost, the new c_best                          */
  double t_ms;                     /* device time since the start of the call that found it */
} pakr_solution;

typedef struct pakr_plan pakr_plan;

/* Device bytes needed by a plan (tree, work buffers, trace-free).  Pure host
 * function; returns 0 for invalid sizes. */
size_t pakr_workspace_size(const pakr_system* sys, const pakr_params* params,
                           const pakr_scene* scene);

/* Validate the query (Sec. III: x_init in X_free, goal region in the
 * workspace; Alg. 1: B/A integral), copy the scene to the device and write
 * the root (x_init, no action, cost 0).  `d_workspace` (device, caller-owned,
 * >= pakr_workspace_size bytes, 256-byte aligned) holds every device buffer of
 * the plan; if NULL the library allocates and owns it.  Enqueues on `stream`;
 * the host arrays are copied before return.  *out is freed with
 * pakr_plan_destroy. */
int pakr_plan_init(const pakr_system* sys, const pakr_scene* scene, const float* x_init,
                   const pakr_goal* goal, const pakr_params* params, void* d_workspace,
                   size_t ws_bytes, void* stream, pakr_plan** out);

/* Free the plan (and the workspace if the library allocated it).  Syncs. */
void pakr_plan_destroy(pakr_plan* plan);

/* Bytes of a trace buffer holding n_iters iteration records (layout below). */
size_t pakr_trace_bytes(const pakr_plan* plan, int n_iters);

/* Run exactly n_iters inner iterations of Alg. 1 (rounds end and restart as
 * the algorithm says), recording each into `d_trace` (device, nullable,
 * >= pakr_trace_bytes(plan, n_iters)).  Async.
 *
 * Trace record i, int32 words at d_trace + i * pakr_trace_bytes(plan, 1):
 *   [0] round [1] iter [2] n0 (tree size at start) [3] n1 (at end)
 *   [4] goal candidate j or -1 [5] its slot or -1 [6] end reason
 *       (0 none, 1 goal, 2 tree full, 3 iteration cap)
 *   [7] c_best before (float bits) [8] c_best after (float bits)
 *   [9] survivors [10..15] reserved
 *   then targets K*d floats, parents K ints, controls B*m floats,
 *   final states B*d floats, costs B floats, flags B ints
 *   (1 valid, 2 under the bound, 4 kept, 8 final state in the goal), and
 *   slots B ints (tree slot, or -1 if not inserted). */
int pakr_expand(pakr_plan* plan, int n_iters, void* d_trace, size_t trace_bytes);

/* Run the AO-x loop on the device until the device-clock budget (ms, > 0)
 * runs out, `max_rounds` (> 0) rounds complete, or `max_iters` (> 0)
 * iterations have run -- whichever comes first; a value <= 0 disables that
 * limit, and at least one must be set.  Async. */
int pakr_replan(pakr_plan* plan, double budget_ms, int max_rounds, long long max_iters);

/* Counters and timings (syncs). */
int pakr_status(pakr_plan* plan, pakr_stats* out);

/* Solutions found so far (syncs).  Writes min(cap, count) records, *n_total
 * receives the count. */
int pakr_solutions(pakr_plan* plan, pakr_solution* out, int cap, int* n_total);

/* ExtractPath (Alg. 1): the best trajectory found, root first (syncs).
 * states: host [(n_edges + 1)][d]; actions: host [n_edges][m], the control
 * held on each edge.  PAKR_E_NO_SOLUTION with *n_edges = 0 if none yet;
 * PAKR_E_BUFFER_TOO_SMALL with *n_edges set if cap_edges is too small. */
int pakr_extract_path(pakr_plan* plan, float* states, float* actions, int cap_edges,
                      int* n_edges, double* cost);

/* Copy the current round's tree to host arrays, node-major (syncs):
 * states [n][d], actions [n][m], parents [n] (root -1), costs [n]; any may be
 * NULL.  At most n_max nodes; *n receives the tree size. */
int pakr_copy_tree(pakr_plan* plan, float* states, float* actions, int* parents, float* costs,
                   int n_max, int* n);

/* Message for the last error of `plan` (or of the last failed
 * pakr_plan_init / pakr_batch_init when plan is NULL).  Valid until the next
 * call. */
const char* pakr_last_error(const pakr_plan* plan);

/* ---------------------------------------------------------------------------
 * Batched planning: many independent queries (mixed systems, uneven tree
 * capacities) in one persistent launch.  Each workgroup takes the next ticket
 * (query, team member) from a device work queue and runs its part of that
 * query's AO-x loop together with the other members of the query's team (the
 * same iteration as a single-query plan, so every query's results are
 * identical to planning it alone with the same parameters), then takes the
 * next ticket.  Tickets go out largest team and most estimated work first.
 * ------------------------------------------------------------------------- */
typedef struct pakr_batch pakr_batch;

/* Device bytes for n queries (arrays of n entries, host).  0 if invalid. */
size_t pakr_batch_workspace_size(int n, const pakr_system* sys, const pakr_scene* scenes,
                                 const pakr_params* params);

/* Validate and set up n queries: query q uses sys[q], scenes[q], x_inits[q]
 * (host pointer to d floats), goals[q], params[q] (here `grid` is the query's
 * team size: the workgroups of the batch launch that plan it together, 1..16,
 * 0 = its share of the batch's estimated work; workgroups_per_cu is ignored;
 * lanes_per_candidate 0 means 1).  The
 * workspace rules are those of pakr_plan_init.  On a validation error the
 * message names the query.  Enqueues on `stream`. */
int pakr_batch_init(int n, const pakr_system* sys, const pakr_scene* scenes,
                    const float* const* x_inits, const pakr_goal* goals,
                    const pakr_params* params, void* d_workspace, size_t ws_bytes, void* stream,
                    pakr_batch** out);

/* One launch: every query runs its AO-x loop under the same limits as
 * pakr_replan (budget measured from the moment its workgroup starts it).
 * Async. */
int pakr_batch_replan(pakr_batch* batch, double budget_ms, int max_rounds, long long max_iters);

/* Capture (work-queue reset + batch launch with these limits) into a
 * hipGraph, replayed by pakr_batch_graph_launch on the batch's stream.
 * Captured on an internal stream; replaces any earlier capture.  The graph
 * keeps its own device copy of the limits, so later pakr_batch_replan or
 * pakr_batch_expand calls do not change what a replay runs.  Syncs. */
int pakr_batch_graph_capture(pakr_batch* batch, double budget_ms, int max_rounds,
                             long long max_iters);
int pakr_batch_graph_launch(pakr_batch* batch);

/* One launch that runs exactly n_iters inner iterations of Alg. 1 for every
 * query (rounds end and restart as for pakr_expand), recording query q's
 * iterations into d_traces[q] (device, >= pakr_batch_trace_bytes(batch, q,
 * n_iters), record layout as for pakr_expand).  d_traces and trace_bytes
 * are host arrays of n entries; d_traces or any entry may be NULL (no trace
 * for that query).  Async. */
size_t pakr_batch_trace_bytes(const pakr_batch* batch, int q, int n_iters);
int pakr_batch_expand(pakr_batch* batch, int n_iters, void* const* d_traces,
                      const size_t* trace_bytes);

/* Per-query results (sync); same meaning as the single-query calls.  After a
 * grid barrier timed out in any query they return PAKR_E_DEVICE, and the
 * batch refuses every later launch. */
int pakr_batch_status(pakr_batch* batch, int q, pakr_stats* out);
int pakr_batch_solutions(pakr_batch* batch, int q, pakr_solution* out, int cap, int* n_total);
int pakr_batch_extract_path(pakr_batch* batch, int q, float* states, float* actions,
                            int cap_edges, int* n_edges, double* cost);
int pakr_batch_copy_tree(pakr_batch* batch, int q, float* states, float* actions, int* parents,
                         float* costs, int n_max, int* n);

/* Workgroups of the batch launch (queries run concurrently). */
int pakr_batch_grid(const pakr_batch* batch);

/* Team size of query q (workgroups that plan it together); 0 if q is invalid. */
int pakr_batch_team(const pakr_batch* batch, int q);

/* Message for the last error of `batch`. */
const char* pakr_batch_last_error(const pakr_batch* batch);

void pakr_batch_destroy(pakr_batch* batch);

/* ---------------------------------------------------------------------------
 * Trajectory refinement (extension of the planner's output; the paper notes
 * only that a differentiable simulator could be used this way).  A path is a
 * start state and M piecewise-constant controls, each held for one edge of T
 * RK4 steps of dt (Sec. IV-A).  Its smooth objective is
 *
 *   J(U) = w_effort    * sum_e T*dt * sum_c ((u_e,c - u_ref_c) / u_scale_c)^2
 *        + w_goal      * |pos(x_N) - goal centre|^2
 *        + w_collision * sum_{n=1..N} pen(x_n),          N = M*T,
 *
 * where pen(x) sums softplus_beta(delta - sd) over the obstacles (sd: signed
 * distance of the position to the box or sphere) and softplus_beta of the
 * violation of the workspace box, of every finite state limit and of the
 * speed bound, softplus_beta(z) = log(1 + exp(beta z)) / beta.
 * pakr_rollout_fwd evaluates J and stores the N+1 states; pakr_rollout_bwd is
 * its hand-written reverse (adjoint) through the RK4 stages; pakr_check_path
 * is the planner's own hard acceptance test of a path.
 *
 * Device arrays, many trajectories per call (one workgroup each):
 *   x0 [n][d], U [n][M][m], J [n], gJ [n], gU [n][M][m], ok [n], cost [n],
 *   ckpt: pakr_rollout_ckpt_bytes(r, n, M) bytes, 256-byte aligned.
 * ------------------------------------------------------------------------- */
typedef struct pakr_refine_params {
  float w_effort;                  /* >= 0 */
  float w_goal;                    /* >= 0 */
  float w_collision;               /* >= 0 */
  float beta;                      /* softplus sharpness, > 0 */
  float delta;                     /* obstacle clearance margin, >= 0 */
  float u_ref[PAKR_MAX_M];         /* effort reference control */
  float u_scale[PAKR_MAX_M];       /* effort scale per control, > 0 */
} pakr_refine_params;

typedef struct pakr_refiner pakr_refiner;

/* Validate and upload one scene for refinement: sys, scene and goal as for
 * pakr_plan_init; of params only T, dt and cost_kind are read.  The library
 * allocates the (small) obstacle buffer.  Enqueues on `stream`. */
int pakr_refiner_init(const pakr_system* sys, const pakr_scene* scene, const pakr_goal* goal,
                      const pakr_params* params, const pakr_refine_params* refine, void* stream,
                      pakr_refiner** out);

/* Replace the objective's weights (e.g. for a continuation in beta). */
int pakr_refiner_set_params(pakr_refiner* r, const pakr_refine_params* refine);

/* Checkpoint bytes for n trajectories of M edges: (M*T + 1) * d floats each.
 * 0 if invalid. */
size_t pakr_rollout_ckpt_bytes(const pakr_refiner* r, int n, int M);

/* J of n trajectories; writes the states x_0..x_N of each into d_ckpt.  Async. */
int pakr_rollout_fwd(pakr_refiner* r, int n, int M, const float* d_x0, const float* d_U,
                     void* d_ckpt, size_t ckpt_bytes, float* d_J);

/* gU = gJ * dJ/dU, reading the checkpoints that pakr_rollout_fwd wrote for
 * the same U.  Async. */
int pakr_rollout_bwd(pakr_refiner* r, int n, int M, const float* d_U, const void* d_ckpt,
                     size_t ckpt_bytes, const float* d_gJ, float* d_gU);

/* One projected Adam step (moments d_m1, d_m2 of n*M*m floats, zero before
 * step 1; step counts from 1) taken in the controls normalised to [-1, 1] by
 * the control box, then clipped to the box.  Async. */
int pakr_refine_step(pakr_refiner* r, int n, int M, float* d_U, const float* d_gU, float* d_m1,
                     float* d_m2, int step, float lr);

/* Device bytes of the pakr_refine_paths workspace for n paths of M edges. */
size_t pakr_refine_workspace_size(const pakr_refiner* r, int n, int M);

/* Refine n paths in place: `steps` iterations of [J and its adjoint at U;
 * trial = projected Adam step (as pakr_refine_step, with a per-path step
 * size); J of the trial; the trial replaces U only if it lowers J, and the
 * path's step size then grows by 1.25 (up to lr) -- otherwise it halves].
 * J therefore never increases.  d_U [n][M][m] is read and overwritten;
 * d_J_before / d_J_after [n] (nullable) receive J before and after.
 * d_ws: pakr_refine_workspace_size bytes, 256-byte aligned.  Async. */
int pakr_refine_paths(pakr_refiner* r, int n, int M, const float* d_x0, float* d_U, int steps,
                      float lr, void* d_ws, size_t ws_bytes, float* d_J_before, float* d_J_after);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * refinement as pakr_refine_paths, with its work buffers (checkpoints, Adam
 * moments, trial controls, per-path J and step sizes) in a library-owned
 * static device array of PAKR_REFINE_STATIC_BYTES per GPU instead of a
 * caller workspace.  The array's address on a GPU is looked up once, when
 * the first refiner is created with that GPU current; the call itself
 * allocates nothing.  Sizes whose pakr_refine_workspace_size exceeds the
 * array fail with PAKR_E_WORKSPACE_TOO_SMALL.  Every call on one GPU shares
 * its array, so calls that may overlap on a GPU (different streams, or
 * refiners on different streams) race: order them.  Results equal
 * pakr_refine_paths' bit for bit.  Async on the refiner's stream. */
#define PAKR_REFINE_STATIC_BYTES (16u << 20)
int pakr_refine_paths_static(pakr_refiner* r, int n, int M, const float* d_x0, float* d_U,
                             int steps, float lr, float* d_J_before, float* d_J_after);

/* The planner's acceptance test of each path: ok bit 0 = every sub-step
 * state valid (workspace, limits, obstacles), bit 1 = final position in the
 * goal ball; cost = the path's cost under cost_kind.  Async. */
int pakr_check_path(pakr_refiner* r, int n, int M, const float* d_x0, const float* d_U,
                    int* d_ok, float* d_cost);

const char* pakr_refiner_last_error(const pakr_refiner* r);
void pakr_refiner_destroy(pakr_refiner* r);

/* How long a workgroup of any later launch waits at a grid barrier before
 * the call fails (every workgroup then leaves the kernel, and the next
 * status or read-back call returns PAKR_E_DEVICE).  Process-wide; ms <= 0
 * restores the default of 2000 ms.  A tiny value forces that failure path
 * from the host (failure-handling tests).  PAKR_E_INVALID_ARG for NaN. */
int pakr_set_barrier_timeout(double ms);

/* Static name of an error code. */
const char* pakr_error_string(int code);

#ifdef __cplusplus
}
#endif
#endif /* PAKR_H */
