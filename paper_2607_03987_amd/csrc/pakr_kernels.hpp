// The PAKR planner kernel for gfx950.
//
// One cooperative launch of G workgroups runs the AO-x loop of Alg. 1 on the
// device with no host round-trip.  Each inner iteration has three phases
// separated by two grid barriers:
//
//   1. SampleStates + NearestNeighbor.  Every workgroup draws the K targets
//      (Philox), stages them in LDS, and scans the tree tiles it owns -- tile t
//      (64 nodes) belongs to workgroup t mod G -- staging each tile through
//      LDS; threads hold several targets and scan a slice of each tile.  Each
//      workgroup folds its per-target (distance, index) minima, packed into
//      u64 keys, into the iteration's key buffer with a device-scope atomic min.
//   2. SampleControls + Propagate + CollisionFree + prune.  Rollout workgroup w
//      owns a chunk of consecutive candidates j (L lanes per candidate): it
//      reads its parents' keys, rolls each candidate out with RK4 (the L lanes
//      share the obstacle tests, obstacles in LDS), and compacts the survivors
//      in candidate order into a staging area with a wave ballot + prefix count.
//   3. Insert + bookkeeping.  All workgroups read the survivor counts, take an
//      exclusive prefix, and copy the survivors that land in their own tiles
//      from staging into the tree (so the next phase 1 reads only slots its
//      workgroup wrote itself, and needs no extra barrier).  The goal test, the
//      bound update and the round end are computed identically by every
//      workgroup; workgroup 0 records solutions and walks the parent chain.
//
// Survivor slots are n + (number of survivors before j): insertion order is
// deterministic and equal to the sequential order of Alg. 1.
#pragma once

#include <limits.h>

#include "pakr_device.hpp"

namespace pakr {

struct KArgs {
  DevProblem P;
  DevHeader* hdr;
  uint32_t* bar_flags;              // [G] arrival generation per workgroup
  DevSolution* sols;                // [MAX_SOLUTIONS]
  float* path_states;               // [(max_path_edges+1)][d], goal first
  float* path_actions;              // [max_path_edges][m]
  float* states;                    // [d][n_cap]  component-major
  float* actions;                   // [m][n_cap]
  int* parents;                     // [n_cap]
  float* costs;                     // [n_cap]
  const float* obs;                 // packed obstacles (see any_obstacle_hit)
  unsigned long long* nn_keys;      // [2][K] packed (d2 bits << 32 | node), alternate iterations
  float* stg;                       // survivor staging, S = G_roll*cpb entries
  int* counts;                      // [G_roll] survivors per rollout workgroup
  unsigned long long* goalmin;      // [G_roll] packed (cost bits << 32 | j)
  int* trace;                       // nullable: per-iteration records
  long long trace_words;            // int32 words per record
  long long trace_iters;            // records available
  long long max_iters;              // <= 0: no limit
  long long max_rounds;             // <= 0: no limit
  long long budget_ticks;           // <= 0: no budget
  long long guard_ticks;            // hard limit on the call's device time
  long long barrier_timeout_ticks;  // give up on a grid barrier after this long
};

__device__ __forceinline__ unsigned long long pack_key(float v, uint32_t idx) {
  return ((unsigned long long)__float_as_uint(v) << 32) | (unsigned long long)idx;
}

// A store that goes through to device-coherent memory (an agent-scope relaxed
// atomic store: the L2 keeps no dirty copy), so a grid barrier's release (an
// L2 write-back on this multi-XCD GPU) has less to flush.  Used to clear the
// NN key buffers, which the workgroups then fold their minima into with
// device-scope atomics (also performed past the L2).
template <typename T>
__device__ __forceinline__ void store_through(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Grid-wide barrier with a bounded wait.  Workgroup 0 collects the other
// workgroups' arrival flags and publishes a release word (generation << 3 |
// note << 1 | failed), where note (0..3) is a value workgroup 0's thread 0
// left in *s_note before the barrier; every workgroup finds it there after the
// barrier, with no extra memory round trip.  Returns false if any wait timed
// out; every workgroup then leaves the kernel.
//
// Every workgroup makes its own writes visible (agent-scope release: L2
// write-back) before raising its flag, so the collecting workgroup publishes
// the release word as soon as it has seen all flags and only then takes its own acquire
// (L2 invalidate) for the reads that follow.  One wave per workgroup runs the
// acquire; the workgroup barrier after it orders the other waves' reads.
template <typename Work>
__device__ __forceinline__ bool grid_barrier_with(const KArgs& a, uint32_t& gen, int* s_fail,
                                                  int wg, int G, int* s_note, Work&& work);

__device__ __forceinline__ bool grid_barrier(const KArgs& a, uint32_t& gen, int* s_fail, int wg,
                                             int G, int* s_note = nullptr) {
  return grid_barrier_with(a, gen, s_fail, wg, G, s_note, [](uint32_t) {});
}

// The barrier above; a workgroup other than the collector runs work(target)
// (every thread) after raising its flag and before it waits for the release
// (target: the generation the release word will carry).
template <typename Work>
__device__ __forceinline__ bool grid_barrier_with(const KArgs& a, uint32_t& gen, int* s_fail,
                                                  int wg, int G, int* s_note, Work&& work) {
  ++gen;
  __syncthreads();
  if (G == 1) return true;
  const uint32_t target = gen & 0x1fffffffu;
  // workgroup 0 owns the most NN tiles and the first rollout chunk, so it is
  // usually the last to arrive and finds the other flags already raised
  const int master = 0;
  if (wg == master) {
    if (threadIdx.x == 0) *s_fail = 0;
    __syncthreads();
    for (int i = threadIdx.x + 1; i < G; i += NT) {
      long long limit = 0;
      while (__hip_atomic_load(&a.bar_flags[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) !=
             target) {
        const long long now = wall_clock64();
        if (limit == 0) {
          limit = now + a.barrier_timeout_ticks;
        } else if (now > limit) {
          *s_fail = 1;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      const uint32_t note = s_note != nullptr ? (uint32_t)*s_note & 3u : 0u;
      __hip_atomic_store(&a.hdr->release, (target << 3) | (note << 1) | (uint32_t)(*s_fail != 0),
                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
  } else {
    if (threadIdx.x == 0) {
      *s_fail = 0;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      __hip_atomic_store(&a.bar_flags[wg], target, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    work(target);
    if (threadIdx.x == 0) {
      const long long limit = wall_clock64() + a.barrier_timeout_ticks;
      while (true) {
        const uint32_t v = __hip_atomic_load(&a.hdr->release, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
        if ((v >> 3) == target) {
          *s_fail = (int)(v & 1u);
          if (s_note != nullptr) *s_note = (int)((v >> 1) & 3u);
          break;
        }
        if (wall_clock64() > limit) {
          *s_fail = 1;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
  }
  __syncthreads();
  return *s_fail == 0;
}

// Offsets of the trace record fields (int32 words).
struct TraceView {
  int* hdr;
  float* targets;
  int* parents;
  float* controls;
  float* xnew;
  float* cnew;
  int* flags;
  int* slots;
  __device__ TraceView(int* base, int K, int B, int D, int M) {
    hdr = base;
    targets = reinterpret_cast<float*>(base + TRACE_HDR_WORDS);
    parents = reinterpret_cast<int*>(targets + (size_t)K * D);
    controls = reinterpret_cast<float*>(parents + K);
    xnew = controls + (size_t)B * M;
    cnew = xnew + (size_t)B * D;
    flags = reinterpret_cast<int*>(cnew + B);
    slots = flags + B;
  }
};

// Exclusive prefix sum of cnt[0..n) into off[0..n], off[n] = total; n <= 4*NT.
// Every thread of the workgroup must call it; ends with a barrier.
__device__ __forceinline__ void block_exclusive_scan(const int* cnt, int* off, int n, int* s_wave) {
  const int tid = threadIdx.x, lane = tid & (WAVE - 1), wv = tid / WAVE;
  int v[4];
  int sum = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int idx = tid * 4 + i;
    v[i] = idx < n ? cnt[idx] : 0;
    sum += v[i];
  }
  int incl = sum;  // inclusive scan of the per-thread sums within the wave
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) {
    const int t = __shfl_up(incl, o);
    if (lane >= o) incl += t;
  }
  if (lane == WAVE - 1) s_wave[wv] = incl;
  __syncthreads();
  int wbase = 0, total = 0;
#pragma unroll
  for (int w = 0; w < NT / WAVE; ++w) {
    wbase += (w < wv) ? s_wave[w] : 0;
    total += s_wave[w];
  }
  int run = wbase + incl - sum;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int idx = tid * 4 + i;
    if (idx < n) off[idx] = run;
    run += v[i];
  }
  if (tid == 0) off[n] = total;
  __syncthreads();
}

// Per-call bookkeeping of workgroup 0, touched by its thread 0 only: device
// clock marks (start, budget deadline, barrier-wait guard, first and last
// solution), ticks per step of the iteration (0 NN scan, 1 wait at barrier A,
// 2 parent reduction, 3 rollout, 4 wait at barrier B, 5 insertion and
// bookkeeping) and counters.  In LDS rather than registers, which the
// rollout needs.
struct Books {
  long long t0, deadline, guard, t_first, t_last, tk_mark;
  long long tk[6];
  unsigned long long c_exp, c_ins, c_nn;
  int c_sol;
};

struct LoopState;

// LDS used by one query's loop; each kernel that runs plan_loop declares it.
struct Smem {
  float* obs;                  // dynamic: obstacles (see any_obstacle_hit)
  float* tile;                 // [D][TILE] NN tile, 16-byte aligned
  float* targets;              // [D][NN_KC<QT>] the NN chunk's targets
  unsigned long long* keys;    // [NN_KC<QT>] their best keys over the node slices
  int* cnt;                    // [MAX_GR] survivors per rollout chunk
  int* off;                    // [MAX_GR + 1] their exclusive prefix
  int* wave;                   // [NT / WAVE]
  float* val;                  // [VAL_FLOATS] validity constants
  unsigned long long* goal;
  int* fail;
  int* misc;                   // [2]
  Books* books;
  LoopState* state;            // hand-off state read by waiting workgroups
};

// Loop state handed from workgroup 0 to workgroups that join when the tree
// grows into a tier with more workgroups (see plan_loop).
struct LoopState {
  int n, round, iter, n_sol, rounds_done, status;
  float c_best;
  uint32_t gen;
  long long it_done;
  int ended;
  int grid;  // workgroups of the tier that starts
};

// Workgroup 0 publishes the loop state; the workgroups below st.grid that
// wait take the next iteration (iterations done = it_done) from it, and all
// waiting workgroups leave if `ended`.  Every thread of the workgroup calls it.
__device__ __forceinline__ void publish_handoff(const KArgs& a, const LoopState& st) {
  __syncthreads();  // the whole workgroup's writes precede the release below
  if (threadIdx.x == 0) {
    DevHeader* h = a.hdr;
    h->n = st.n;
    h->round = st.round;
    h->iter = st.iter;
    h->n_solutions = st.n_sol;
    h->c_best = st.c_best;
    h->ho_rounds = st.rounds_done;
    h->ho_status = st.status;
    h->ho_gen = st.gen;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const unsigned long long w = ((unsigned long long)(st.it_done + 1) << 32) |
                                 ((unsigned long long)(uint32_t)st.grid << 1) |
                                 (unsigned long long)(st.ended != 0);
    __hip_atomic_store(&h->join, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Workgroup `b`, outside the tier of the iteration after `waited_at`
// iterations, waits until workgroup 0 publishes a hand-off made at or after
// it that starts a tier including b (or ends the call), and adopts its state.
// Hand-offs to tiers that still exclude b are skipped without reading the
// state (workgroup 0 may publish the next one meanwhile; a workgroup that
// joins takes part in the next iteration's barriers, so no newer hand-off can
// overwrite the state while it reads).  Returns false if the wait passed
// `deadline` (device clock).
__device__ __forceinline__ bool await_handoff(const KArgs& a, int b, long long waited_at,
                                              long long deadline, LoopState* s_st) {
  if (threadIdx.x == 0) {
    bool ok = true;
    unsigned long long w, skipped = 0ull;
    while (true) {
      w = __hip_atomic_load(&a.hdr->join, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      // (the call's end may be published at the same iteration count as a
      // hand-off this workgroup skipped: only that exact word is skipped)
      if ((long long)(w >> 32) > waited_at && w != skipped) {
        if ((w & 1ull) != 0ull || b < (int)((w >> 1) & 0x7fffffffull)) break;
        skipped = w;  // a tier without this workgroup: wait for a later one
      }
      if (wall_clock64() > deadline) {
        ok = false;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (ok) {
      const DevHeader* h = a.hdr;
      s_st->n = h->n;
      s_st->round = h->round;
      s_st->iter = h->iter;
      s_st->n_sol = h->n_solutions;
      s_st->c_best = h->c_best;
      s_st->rounds_done = h->ho_rounds;
      s_st->status = h->ho_status;
      s_st->gen = h->ho_gen;
      s_st->it_done = (long long)(w >> 32) - 1;
      s_st->ended = (int)(w & 1ull);
    } else {
      s_st->ended = -1;
    }
  }
  __syncthreads();
  return s_st->ended >= 0;
}

// The AO-x loop of one query, run by workgroup `b` of the `G_all` workgroups
// that share the query (G_all = 1 when a workgroup plans a query alone).  QT
// targets per thread in the NN scan; GROUPED: the scan may split tiles into
// node slices (P.nn_tpg threads per slice), else one target per thread.
//
// Tiers (the paper's memory tiers of the tree, Sec. IV-A): the number of
// workgroups that run an iteration grows with the round's tree -- workgroup 0
// alone while it has at most P.tier0_nodes nodes (no grid barrier at all),
// the first P.tier_grid[k] workgroups while it has at most P.tier_nodes[k]
// (barriers among fewer workgroups are cheaper, and a small tree's NN scan
// needs few), then all of them.  Workgroups outside the tier wait for a
// hand-off.  When the tree grows into a larger tier, the tier's workgroups
// meet at a barrier (their writes reach memory) and workgroup 0 publishes the
// loop state; at a round end that returns to a smaller tier, a barrier of the
// larger one first puts every participant's writes in memory, so fewer
// workgroups can reuse the tree's slots.
template <int SYS, int QT, bool GROUPED, bool TIERED>
__device__ __forceinline__ void plan_loop(const KArgs& a, const int b, const int G_all,
                                          const Smem& sm) {
  static_assert(GROUPED || QT == 1, "an ungrouped scan holds one target per thread");
  constexpr int D = Sys<SYS>::D, M = Sys<SYS>::M, NP = Sys<SYS>::P;
  const DevProblem& P = a.P;
  float* const s_obs = sm.obs;
  float (*const s_tile)[TILE] = reinterpret_cast<float (*)[TILE]>(sm.tile);
  float* const s_q = sm.targets;
  unsigned long long* const s_key = sm.keys;
  constexpr int KCM = NN_KC<QT>;
  int* const s_cnt = sm.cnt;
  int* const s_off = sm.off;
  int* const s_wave = sm.wave;
  float* const s_val = sm.val;
  unsigned long long& s_goal = *sm.goal;
  int& s_fail = *sm.fail;
  int* const s_misc = sm.misc;

  const int tid = threadIdx.x;
  const int B = P.B, A = P.A, K = P.K, GR = P.G_roll;
  const int L = P.lanes, CPB = P.cpb;   // lanes per candidate, candidates per rollout workgroup
  const int S = GR * CPB;
  // double integrators: a candidate's lanes split its sub-steps (LS groups)
  // and the obstacles (L / LS groups) instead of each integrating the edge
  constexpr bool DI = SYS == PAKR_DI2 || SYS == PAKR_DI3;
  const int LS = DI ? di_step_groups<DI_CH>(P, L) : 1;
  const size_t NC = (size_t)P.n_cap;

  float* stg_x = a.stg;
  float* stg_u = stg_x + (size_t)D * S;
  float* stg_c = stg_u + (size_t)M * S;
  int* stg_par = reinterpret_cast<int*>(stg_c + S);
  int* stg_j = stg_par + S;
  int* stg_f = stg_j + S;

  for (int i = tid; i < P.obs_floats; i += NT) s_obs[i] = a.obs[i];
  load_validity(P, s_val, tid);

  // loop state: identical in every workgroup
  int n = a.hdr->n, round = a.hdr->round, iter = a.hdr->iter;
  float c_best = a.hdr->c_best;
  uint32_t gen = a.hdr->bar_gen;
  int n_sol = a.hdr->n_solutions;
  long long it_done = 0, rounds_done = 0;
  int status = 0;
  int spec_lo = 0;  // tiles [0, spec_lo) already scanned for this iteration's targets
  // this workgroup's first pre_n own tiles of this iteration's scan were
  // scanned while it waited at the previous iteration's second barrier
  int pre_n = 0;
  // this workgroup's share of the last insertion, when its copy waits for
  // the next iteration's NN scan: slots [pend_n0, pend_n1) (see nn_scan)
  int pend_n0 = 0, pend_n1 = 0;
  int* pend_trace = nullptr;

  // workgroup-0 bookkeeping, kept by its thread 0 in LDS
  Books& bk = *sm.books;
  const bool keeper = b == 0 && tid == 0;
  auto mark = [&](int slot) {
    if (keeper) {
      const long long now = wall_clock64();
      bk.tk[slot] += now - bk.tk_mark;
      bk.tk_mark = now;
    }
  };
  if (keeper) {
    bk.t0 = wall_clock64();
    bk.deadline = a.budget_ticks > 0 ? bk.t0 + a.budget_ticks : LLONG_MAX;
    bk.guard = bk.t0 + a.guard_ticks;
    bk.t_first = -1;
    bk.t_last = -1;
    bk.tk_mark = 0;
    for (int i = 0; i < 6; ++i) bk.tk[i] = 0;
    bk.c_exp = bk.c_ins = bk.c_nn = 0;
    bk.c_sol = 0;
  }
  // both NN key buffers start cleared, and no hand-off is pending
  for (int k = b * NT + tid; k < 2 * K; k += G_all * NT) store_through(&a.nn_keys[k], ~0ull);
  if (b == 0 && tid == 0) store_through(&a.hdr->join, 0ull);
  if (!grid_barrier(a, gen, &s_fail, b, G_all)) {
    if (tid == 0) __hip_atomic_store(&a.hdr->err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return;
  }
  const int tier0 = (TIERED && G_all > 1) ? P.tier0_nodes : 0;
  // workgroups that run an iteration whose tree has nn nodes (same in all)
  auto tier_grid = [&](int nn) {
    if (nn <= tier0) return 1;
#pragma unroll
    for (int k = 0; k < MAX_TIERS; ++k)
      if (nn <= P.tier_nodes[k]) return min(P.tier_grid[k], G_all);
    return G_all;
  };
  // a waiting workgroup gives up at the call's guard time
  const long long wait_deadline = wall_clock64() + a.guard_ticks;
  LoopState* const s_st = sm.state;
  bool failed = false;  // a grid barrier of the loop timed out

  while (true) {
    if (a.max_iters > 0 && it_done >= a.max_iters) { status |= PAKR_S_ITERS_DONE; break; }
    if (a.max_rounds > 0 && rounds_done >= a.max_rounds) { status |= PAKR_S_ROUNDS_DONE; break; }
    // the tree's tier decides who runs this iteration (identical in every workgroup)
    const int G = TIERED ? tier_grid(n) : G_all;
    if (b >= G) {
      if (!await_handoff(a, b, it_done, wait_deadline, s_st)) {
        if (tid == 0) __hip_atomic_store(&a.hdr->err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return;
      }
      if (s_st->ended) return;  // workgroup 0 writes the call's results
      // the same values in every lane: keep the loop state in scalar registers
      auto uni = [](int v) { return __builtin_amdgcn_readfirstlane(v); };
      n = uni(s_st->n);
      round = uni(s_st->round);
      iter = uni(s_st->iter);
      n_sol = uni(s_st->n_sol);
      c_best = __int_as_float(uni(__float_as_int(s_st->c_best)));
      rounds_done = uni(s_st->rounds_done);
      status = uni(s_st->status);
      gen = (uint32_t)uni((int)s_st->gen);
      it_done = (long long)uni((int)s_st->it_done);
      spec_lo = 0;
      pre_n = 0;
      continue;
    }
    int* trace = (a.trace != nullptr && it_done < a.trace_iters) ? a.trace + it_done * a.trace_words
                                                                 : nullptr;
    const int n0 = n;
    const int ntiles = (n0 + TILE - 1) / TILE;
    // this iteration's NN keys: every scanning workgroup folds its minima in
    // by device-scope atomic min; two buffers alternate, each cleared during
    // the insertion phase of the iteration that consumed it
    unsigned long long* const nnk = a.nn_keys + (size_t)(it_done & 1) * K;
    unsigned long long* const nnk_next = a.nn_keys + (size_t)((it_done + 1) & 1) * K;
    if (keeper) bk.tk_mark = wall_clock64();

    // ---------------- NN scan (phase 1, and speculatively in phase 2) -----
    // Scans tiles t0, t0 + tstep, ... (at most tcount of them, t < t_end) of
    // the tree's first n0 nodes for the K targets of iteration it_q of this
    // round.  Targets are drawn once per chunk of kc <= TPG * QT and staged in
    // LDS; thread (grp, tl) holds the chunk's targets tl, tl + TPG, ... (QT of
    // them, so every node read from LDS serves QT targets) and scans node
    // slice grp (TILE / NG consecutive nodes) of each tile; the NG groups'
    // keys meet in LDS by atomic min and each workgroup's per-target minimum
    // is folded into `keys` by device-scope atomic min.  With trace_q set,
    // workgroup 0 records the targets (drawn even if it scans nothing).
    const int TPG = GROUPED ? P.nn_tpg : NT, NG = NT / TPG, SL = TILE / NG;
    // With stop_word set (one target chunk only), the scan also ends before a
    // tile once that word carries generation stop_gen in its upper bits (the
    // word is read one tile ahead); returns the tiles it scanned.
    // With do_copy, the scan first completes this workgroup's pending copy of
    // the last insertion: each of its new slots (one per thread) is loaded
    // from the staging area before the targets are drawn and stored just
    // before the first scanned tile that holds new slots is fetched, so the
    // loads' latency passes behind the target draw and the earlier tiles.
    auto nn_scan = [&](uint32_t it_q, int t0, int tstep, int tcount, int t_end,
                       unsigned long long* keys, int* trace_q,
                       const uint32_t* stop_word = nullptr, uint32_t stop_gen = 0,
                       bool do_copy = false) -> int {
      int cp_s = -1, cp_par = 0, cp_j = 0;
      float cp_x[D], cp_u[M], cp_c = 0.0f;
      int kt = 0;  // index of the first scanned tile that holds new slots
      if (do_copy) {
        const int t_lo = pend_n0 / TILE, t_hi = (pend_n1 - 1) / TILE;
        const int t_f = t_lo + ((b - t_lo % G) % G + G) % G;
        const int n_my = t_f <= t_hi ? (t_hi - t_f) / G + 1 : 0;
        if (tid < n_my * TILE) {
          const int sl = (t_f + (tid / TILE) * G) * TILE + (tid % TILE);
          if (sl >= pend_n0 && sl < pend_n1) {
            const int r = sl - pend_n0;
            int lo = 0, hi = GR - 1;
            while (lo < hi) {
              const int mid = (lo + hi + 1) >> 1;
              if (s_off[mid] <= r) lo = mid; else hi = mid - 1;
            }
            const int e = lo * CPB + (r - s_off[lo]);
#pragma unroll
            for (int c = 0; c < D; ++c) cp_x[c] = stg_x[(size_t)c * S + e];
#pragma unroll
            for (int c = 0; c < M; ++c) cp_u[c] = stg_u[(size_t)c * S + e];
            cp_par = stg_par[e];
            cp_c = stg_c[e];
            if (pend_trace != nullptr) cp_j = stg_j[e];
            cp_s = sl;
          }
        }
        kt = t_lo <= t0 ? 0 : (t_lo - t0 + tstep - 1) / tstep;
      }
      bool copied = !do_copy;
      auto store_copy = [&]() {
        if (cp_s >= 0) {
#pragma unroll
          for (int c = 0; c < D; ++c) a.states[(size_t)c * NC + cp_s] = cp_x[c];
#pragma unroll
          for (int c = 0; c < M; ++c) a.actions[(size_t)c * NC + cp_s] = cp_u[c];
          a.parents[cp_s] = cp_par;
          a.costs[cp_s] = cp_c;
          if (pend_trace != nullptr) {
            TraceView tv(pend_trace, K, B, D, M);
            tv.slots[cp_j] = cp_s;
          }
        }
        __syncthreads();  // the workgroup's reads of these slots come after
        copied = true;
      };
      const bool scans = tcount > 0 && t0 < t_end;
      const bool record = trace_q != nullptr && b == 0;
      if (!scans && !record) {
        if (!copied) store_copy();
        return 0;
      }
      if (stop_word != nullptr) {  // (released already: draw no targets)
        if (tid == 0) {
          const uint32_t w =
              __hip_atomic_load(stop_word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          s_misc[1] = (w >> 3) == stop_gen;
        }
        __syncthreads();
        if (s_misc[1]) return 0;
      }
      int done = 0;
      int tid_nn = tid;
      asm volatile("" : "+v"(tid_nn));  // derived per call, not held across the loop
      const int grp = tid_nn / TPG, tl = tid_nn - grp * TPG;
      // (one target per thread and one group: the target is drawn straight
      // into registers and the key written straight out)
      const bool direct = !GROUPED || (QT == 1 && NG == 1);
      for (int base = 0; base < K; base += TPG * QT) {
        const int kc = min(K - base, TPG * QT);
        if (!direct) __syncthreads();  // the previous chunk's readers of s_q and s_key are done
        for (int k = tid; k < kc && !direct; k += NT) {
          float qs[D];
          sample_state<D>(P, (uint32_t)(base + k), it_q, (uint32_t)round, qs);
#pragma unroll
          for (int c = 0; c < D; ++c) s_q[c * KCM + k] = qs[c];
          if (record) {
            TraceView tv(trace_q, K, B, D, M);
#pragma unroll
            for (int c = 0; c < D; ++c) tv.targets[(size_t)(base + k) * D + c] = qs[c];
          }
          s_key[k] = ~0ull;
        }
        if (!direct) __syncthreads();
        float q[QT][D];
        if (direct) {
          if (tid < kc) {
            sample_state<D>(P, (uint32_t)(base + tid), it_q, (uint32_t)round, q[0]);
            if (record) {
              TraceView tv(trace_q, K, B, D, M);
#pragma unroll
              for (int c = 0; c < D; ++c) tv.targets[(size_t)(base + tid) * D + c] = q[0][c];
            }
          } else {
#pragma unroll
            for (int c = 0; c < D; ++c) q[0][c] = 0.0f;
          }
        }
        if (!scans) {
          if (!copied) store_copy();
          continue;
        }
        float bd[QT];
        int bi[QT];
#pragma unroll
        for (int qq = 0; qq < QT; ++qq) {
          const int k = qq * TPG + tl;
          if (!direct) {
#pragma unroll
            for (int c = 0; c < D; ++c) q[qq][c] = k < kc ? s_q[c * KCM + k] : 0.0f;
          }
          bd[qq] = INFINITY;
          bi[qq] = 0;
        }
        // software pipeline: the next tile is fetched into registers while
        // the current one is scanned from LDS.  Slots past the tree end get a
        // coordinate whose squared distance overflows to +inf.
        constexpr int PF = (D * TILE + NT - 1) / NT;
        float pre[PF];
        auto fetch = [&](int t) {
          const int node0 = t * TILE;
#pragma unroll
          for (int r = 0; r < PF; ++r) {
            const int idx = tid + r * NT;
            const int c = idx / TILE, i = idx - c * TILE;
            pre[r] = (idx < D * TILE && node0 + i < n0) ? a.states[(size_t)c * NC + node0 + i]
                                                        : 3.0e38f;
          }
        };
        if (!copied && kt == 0) store_copy();
        fetch(t0);
        const int i0 = grp * SL;
        int t = t0;
        const int done0 = done;
        uint32_t seen = 0u;  // the stop word as thread 0 last read it
        if (stop_word != nullptr && tid == 0)
          seen = __hip_atomic_load(stop_word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        for (int cnt = 0; cnt < tcount && t < t_end; ++cnt, t += tstep) {
          const int node0 = t * TILE;
          __syncthreads();
          if (stop_word != nullptr) {
            if (tid == 0) s_misc[1] = (seen >> 3) == stop_gen;
            __syncthreads();
            if (s_misc[1]) break;
          }
#pragma unroll
          for (int r = 0; r < PF; ++r) {
            const int idx = tid + r * NT;
            if (idx < D * TILE) (&s_tile[0][0])[idx] = pre[r];
          }
          __syncthreads();
          if (!copied && cnt + 1 == kt) store_copy();
          if (cnt + 1 < tcount && t + tstep < t_end) fetch(t + tstep);
          if (stop_word != nullptr && tid == 0)
            seen = __hip_atomic_load(stop_word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ++done;
#pragma unroll 2
          for (int i = i0; i < i0 + SL; i += 4) {
            float4 pc[D];
#pragma unroll
            for (int c = 0; c < D; ++c) pc[c] = *reinterpret_cast<const float4*>(&s_tile[c][i]);
#pragma unroll
            for (int qq = 0; qq < QT; ++qq) {
              float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f, s3 = 0.0f;
#pragma unroll
              for (int c = 0; c < D; ++c) {
                const float e0 = q[qq][c] - pc[c].x, e1 = q[qq][c] - pc[c].y;
                const float e2 = q[qq][c] - pc[c].z, e3 = q[qq][c] - pc[c].w;
                s0 = fmaf(e0, e0, s0);
                s1 = fmaf(e1, e1, s1);
                s2 = fmaf(e2, e2, s2);
                s3 = fmaf(e3, e3, s3);
              }
              // only a strictly smaller distance replaces the best, and among
              // equal ones the lowest node index wins (the sequential rule;
              // across slices the packed key's index decides)
              const float m = fminf(fminf(s0, s1), fminf(s2, s3));
              if (m < bd[qq]) {
                bd[qq] = m;
                bi[qq] = node0 + i + (s0 == m ? 0 : (s1 == m ? 1 : (s2 == m ? 2 : 3)));
              }
            }
          }
        }
        if (!copied) store_copy();  // (no scanned tile holds new slots)
        if (done == done0) continue;  // stopped before any tile: nothing to fold
        if (direct) {
          if (tid < kc) atomicMin(&keys[base + tid], pack_key(bd[0], (uint32_t)bi[0]));
        } else {
#pragma unroll
          for (int qq = 0; qq < QT; ++qq) {
            const int k = qq * TPG + tl;
            if (k < kc) {
              const unsigned long long key = pack_key(bd[qq], (uint32_t)bi[qq]);
              if (NG == 1) s_key[k] = key;
              else atomicMin(&s_key[k], key);
            }
          }
          __syncthreads();
          for (int k = tid; k < kc; k += NT) atomicMin(&keys[base + k], s_key[k]);
        }
      }
      return done;
    };

    // ---------------- phase 1: targets + nearest neighbour -----------------
    // Tile t (64 nodes) belongs to workgroup t mod G, which writes it in the
    // insertion phase and scans it here.  Tiles [0, spec_lo) were already
    // scanned for these targets by the previous iteration's idle workgroups,
    // and this workgroup's next pre_n own tiles by itself while it waited at
    // the previous barrier; a tree of the root alone needs no scan (its only
    // node is the parent).
    if (n0 > 1) {
      const int t_first = spec_lo + ((b - spec_lo) % G + G) % G + pre_n * G;
      nn_scan((uint32_t)iter, t_first, G, INT_MAX, ntiles, nnk, trace, nullptr, 0,
              pend_n1 > pend_n0);
      pend_n0 = pend_n1 = 0;
    } else {
      nn_scan((uint32_t)iter, 0, G, 0, 0, nnk, trace);
    }
    mark(0);
    // workgroup 0 decides whether the call stops here (1: budget spent,
    // 2: guard time exceeded) and the barrier's release word carries it
    if (keeper) {
      const long long now = wall_clock64();
      s_misc[0] = now >= bk.deadline ? 1 : (now >= bk.guard ? 2 : 0);
    }
    if (!grid_barrier(a, gen, &s_fail, b, G, &s_misc[0])) {
      failed = true;
      break;
    }
    if (s_misc[0] != 0) {
      status |= (s_misc[0] == 1) ? PAKR_S_BUDGET_EXPIRED : PAKR_S_DEVICE_ERROR;
      break;
    }
    mark(1);

    // ---------------- phase 2: controls, rollout, validity, prune ---------
    for (int rb = b; rb < GR; rb += G) {
      const int j0 = rb * CPB;
      __syncthreads();  // the previous chunk's readers of s_goal are done
      if (tid == 0) s_goal = ~0ull;
      mark(2);

      // L consecutive lanes share candidate j: each integrates the edge and
      // tests every L-th obstacle (double integrators: di_edge's split of
      // sub-steps and obstacles); the group ORs its hits
      // (only the first L * CPB threads take candidates: with half the
      // workgroup, each SIMD runs one rollout wave)
      const int lg = tid % L;
      const int j = j0 + tid / L;
      const bool active = tid < L * CPB && j < B;
      float x[D], u[M];
      float cost = 0.0f;
      bool valid = false, prune_ok = false, in_goal = false;
      int parent = 0, k = 0, br = 0;
      bool hit = false;
      float margin_p = INFINITY, margin_g = INFINITY;  // prune and goal decision margins
      if (active) {
        k = j / A;
        br = j - k * A;
        // the lanes of a candidate and the A candidates of a target read the
        // same key: one cache line serves a wave
        parent = n0 > 1 ? (int)(uint32_t)(nnk[k] & 0xffffffffull) : 0;
        sample_control<M>(P, (uint32_t)k, (uint32_t)br, (uint32_t)iter, (uint32_t)round, u);
#pragma unroll
        for (int c = 0; c < D; ++c) x[c] = a.states[(size_t)c * NC + parent];
        const float c_par = a.costs[parent];
        float len = 0.0f;
        const bool path_len = P.cost_kind == PAKR_COST_PATH_LENGTH;
        constexpr int CH = Sys<SYS>::CH;
        bool lim_ok = true;
        if constexpr (DI) {
          bool bad = false;
          di_edge<SYS, DI_CH>(P, s_val, s_obs, x, u, lg, L, LS, path_len, len, bad);
          lim_ok = !bad;
        } else {
          // integrate CH steps, then test their CH positions against this
          // lane's obstacles in one sweep (each obstacle read once per chunk)
          for (int t0 = 0; t0 < P.T; t0 += CH) {
            float pos[CH][NP];
#pragma unroll
            for (int s = 0; s < CH; ++s) {
              if (t0 + s < P.T) {
                float xp[NP];
#pragma unroll
                for (int c = 0; c < NP; ++c) xp[c] = x[c];
                rk4_step<SYS>(P, x, u, P.dt);
                if (path_len) {
                  float s2 = 0.0f;
#pragma unroll
                  for (int c = 0; c < NP; ++c) {
                    const float e = x[c] - xp[c];
                    s2 += e * e;
                  }
                  len += __builtin_amdgcn_sqrtf(s2);  // v_sqrt_f32 (1 ulp)
                }
                lim_ok = lim_ok & limits_ok<SYS>(s_val, x);
              }
#pragma unroll
              for (int c = 0; c < NP; ++c) pos[s][c] = x[c];  // past T: repeats the last state
            }
            hit = hit | any_obstacle_hit<NP, CH>(pos, s_obs, P.n_box, P.n_sph, lg, L);
          }
        }
        hit = hit | !lim_ok;
        cost = c_par + (path_len ? len : P.edge_duration);
        const float dist = sqrtf(goal_dist2<SYS>(P, x));
        const float ch = cost + heuristic<SYS>(P, dist);
        prune_ok = ch < c_best;
        in_goal = dist <= P.goal_r;
        if (!__builtin_isinf(c_best)) margin_p = fabsf(ch - c_best) / fmaxf(1.0f, c_best);
        margin_g = fabsf(dist - P.goal_r);
      }
      int hi = hit ? 1 : 0;
      for (int o = 1; o < L; o <<= 1) hi |= __shfl_xor(hi, o);
      valid = active && hi == 0;
      const bool lead = lg == 0;
      const bool keep = lead && active && valid && prune_ok;
      // near ties (decisions within 1e-5 of their threshold, where float32
      // and FP64 evaluations may decide differently), counted per wave
      const unsigned long long tie_p = __ballot(lead && valid && margin_p <= NEAR_TIE);
      const unsigned long long tie_g = __ballot(lead && valid && margin_g <= NEAR_TIE);
      if ((tid & (WAVE - 1)) == 0 && (tie_p | tie_g) != 0ull) {
        if (tie_p) atomicAdd(&a.hdr->near_prune, (unsigned long long)__popcll(tie_p));
        if (tie_g) atomicAdd(&a.hdr->near_goal, (unsigned long long)__popcll(tie_g));
      }
      const unsigned long long mask = __ballot(keep);
      const int lane = tid & (WAVE - 1), wv = tid / WAVE;
      const int wrank = __popcll(mask & ((1ull << lane) - 1ull));
      if (lane == 0) s_wave[wv] = __popcll(mask);
      __syncthreads();
      int base_r = 0, total = 0;
#pragma unroll
      for (int w = 0; w < NT / WAVE; ++w) {
        base_r += (w < wv) ? s_wave[w] : 0;
        total += s_wave[w];
      }
      if (keep) {
        const int e = rb * CPB + base_r + wrank;
#pragma unroll
        for (int c = 0; c < D; ++c) stg_x[(size_t)c * S + e] = x[c];
#pragma unroll
        for (int c = 0; c < M; ++c) stg_u[(size_t)c * S + e] = u[c];
        stg_c[e] = cost;
        stg_par[e] = parent;
        stg_j[e] = j;
        stg_f[e] = in_goal ? F_GOAL : 0;
        if (in_goal) atomicMin(&s_goal, pack_key(cost, (uint32_t)j));
      }
      __syncthreads();
      if (tid == 0) {
        a.counts[rb] = total;
        a.goalmin[rb] = s_goal;
      }
      if (trace != nullptr && active && lead) {
        TraceView tv(trace, K, B, D, M);
        if (br == 0) tv.parents[k] = parent;
#pragma unroll
        for (int c = 0; c < M; ++c) tv.controls[(size_t)j * M + c] = u[c];
#pragma unroll
        for (int c = 0; c < D; ++c) tv.xnew[(size_t)j * D + c] = x[c];
        tv.cnew[j] = cost;
        tv.flags[j] = (valid ? F_VALID : 0) | (prune_ok ? F_PRUNE_OK : 0) | (keep ? F_KEEP : 0) |
                      (in_goal ? F_GOAL : 0);
        tv.slots[j] = -1;
      }
      mark(3);
    }
    // Workgroups without a rollout chunk scan ahead: the tree is frozen until
    // the insertion phase, and the next iteration's targets are fixed by their
    // counters, so idle workgroup j scans full tiles j, j + I, ... (spec_tiles
    // of them, I idle workgroups) for iteration iter + 1.  Together they cover
    // the prefix [0, min(spec_tiles * I, full tiles)) of the tree, which the
    // next phase 1 skips.  The minimum is idempotent, so results do not depend
    // on how much is scanned ahead; if this iteration ends the round, the next
    // one starts from the root and reads no keys.
    const int n_idle = G - GR;
    const bool spec_on = n_idle > 0 && P.spec_tiles > 0 && iter + 1 < P.max_iters_per_round;
    if (spec_on && b >= GR) nn_scan((uint32_t)(iter + 1), b - GR, n_idle, P.spec_tiles,
                                    n0 / TILE, nnk_next, nullptr);
    mark(3);
    // While it waits at this barrier, a workgroup other than the collector
    // scans its own full tiles for the next iteration's targets, in the order
    // the next phase 1 would, until the release arrives: those tiles do not
    // change in the insertion phase, and the next phase 1 starts after them.
    // (The minimum is idempotent: how far it gets changes no result.)
    const int spec_next = spec_on ? min(P.spec_tiles * n_idle, n0 / TILE) : 0;
    const bool pre_ok = b != 0 && n0 > 1 && iter + 1 < P.max_iters_per_round && K <= TPG * QT;
    int pre_done = 0;
    auto prescan = [&](uint32_t target) {
      if (!pre_ok) return;
      const int t_next = spec_next + ((b - spec_next) % G + G) % G;
      pre_done = nn_scan((uint32_t)(iter + 1), t_next, G, INT_MAX, n0 / TILE, nnk_next, nullptr,
                         &a.hdr->release, target);
    };
    if (!grid_barrier_with(a, gen, &s_fail, b, G, nullptr, prescan)) {
      failed = true;
      break;
    }

    mark(4);
    for (int k = b * NT + tid; k < K; k += G * NT) store_through(&nnk[k], ~0ull);

    // ---------------- phase 3: insert + goal + round bookkeeping ----------
    // The goal keys load together with the counts, so that their round trip
    // overlaps the scan and the copy; their minimum is the iteration's goal
    // candidate unless the tree fills up part-way through the survivors.
    unsigned long long gall = ~0ull;
    for (int w = tid; w < GR; w += NT) {
      s_cnt[w] = a.counts[w];
      const unsigned long long kk = a.goalmin[w];
      gall = kk < gall ? kk : gall;
    }
    __syncthreads();
    block_exclusive_scan(s_cnt, s_off, GR, s_wave);
    const int survivors = s_off[GR];
    const int n_ins = min(survivors, P.n_cap - n0);
    const int n1 = n0 + n_ins;
    // cheapest inserted goal candidate, ties to the lowest j
    unsigned long long key = n_ins == survivors ? gall : ~0ull;
    for (int w = n_ins == survivors ? GR : tid; w < GR; w += NT) {
      const int off = s_off[w], cnt = s_cnt[w];
      if (off + cnt <= n_ins) {
        const unsigned long long kk = a.goalmin[w];
        key = kk < key ? kk : key;
      } else if (off < n_ins) {
        for (int l = 0; l < n_ins - off; ++l) {
          const int e = w * CPB + l;
          if (stg_f[e] & F_GOAL) {
            const unsigned long long kk = pack_key(stg_c[e], (uint32_t)stg_j[e]);
            key = kk < key ? kk : key;
          }
        }
      }
    }
    if (tid == 0) {
      s_goal = ~0ull;
      s_misc[1] = -1;
    }
    __syncthreads();
    if (key != ~0ull) atomicMin(&s_goal, key);
    __syncthreads();
    const unsigned long long gk = s_goal;
    const bool goal = gk != ~0ull;
    int goal_j = -1, goal_e = -1, goal_slot = -1;
    float goal_cost = 0.0f;
    if (goal) {
      goal_j = (int)(uint32_t)(gk & 0xffffffffull);
      goal_cost = __uint_as_float((uint32_t)(gk >> 32));
      const int wg = goal_j / CPB;
      if (tid < s_cnt[wg] && stg_j[wg * CPB + tid] == goal_j) s_misc[1] = tid;
      __syncthreads();
      goal_e = wg * CPB + s_misc[1];
      goal_slot = n0 + s_off[wg] + s_misc[1];
    }
    int end = END_NONE;
    if (goal) end = END_GOAL;
    else if (n1 >= P.n_cap) end = END_TREE_FULL;
    else if (iter + 1 >= P.max_iters_per_round) end = END_ITER_CAP;

    if (n_ins > 0) {
      // this workgroup owns tiles t = b (mod G); copy the survivors that land
      // there -- now, or during the next iteration's NN scan when this
      // workgroup runs that iteration on the same tiles of the same round
      // and has at most one new slot per thread
      const int t_lo = n0 / TILE, t_hi = (n1 - 1) / TILE;
      const int t_first = t_lo + ((b - t_lo % G) % G + G) % G;
      const int n_my = t_first <= t_hi ? (t_hi - t_first) / G + 1 : 0;
      const bool defer = n_my * TILE <= NT && end == END_NONE &&
                         !(a.max_iters > 0 && it_done + 1 >= a.max_iters) &&
                         (!TIERED || tier_grid(n1) == G);
      if (defer) {
        if (n_my > 0) {
          pend_n0 = n0;
          pend_n1 = n1;
          pend_trace = trace;
        }
      } else {
        for (int idx = tid; idx < n_my * TILE; idx += NT) {
          const int s = (t_first + (idx / TILE) * G) * TILE + (idx % TILE);
          if (s >= n0 && s < n1) {
            const int r = s - n0;
            int lo = 0, hi = GR - 1;
            while (lo < hi) {
              const int mid = (lo + hi + 1) >> 1;
              if (s_off[mid] <= r) lo = mid; else hi = mid - 1;
            }
            const int e = lo * CPB + (r - s_off[lo]);
#pragma unroll
            for (int c = 0; c < D; ++c) a.states[(size_t)c * NC + s] = stg_x[(size_t)c * S + e];
#pragma unroll
            for (int c = 0; c < M; ++c) a.actions[(size_t)c * NC + s] = stg_u[(size_t)c * S + e];
            a.parents[s] = stg_par[e];
            a.costs[s] = stg_c[e];
            if (trace != nullptr) {
              TraceView tv(trace, K, B, D, M);
              tv.slots[stg_j[e]] = s;
            }
          }
        }
      }
    }

    if (b == 0 && tid == 0) {
      bk.c_exp += (unsigned long long)B;
      bk.c_ins += (unsigned long long)n_ins;
      bk.c_nn += (unsigned long long)K * (unsigned long long)n0;
      if (trace != nullptr) {
        int* h = trace;
        h[0] = round;
        h[1] = iter;
        h[2] = n0;
        h[3] = n1;
        h[4] = goal_j;
        h[5] = goal_slot;
        h[6] = end;
        h[7] = __float_as_int(c_best);
        h[8] = __float_as_int(goal ? goal_cost : c_best);
        h[9] = survivors;
      }
      if (goal) {
        const long long tnow = wall_clock64() - bk.t0;
        if (bk.t_first < 0) bk.t_first = tnow;
        bk.t_last = tnow;
        if (n_sol < MAX_SOLUTIONS) {
          DevSolution& so = a.sols[n_sol];
          so.round = round;
          so.iter = iter;
          so.node = goal_slot;
          so.n_nodes = n1;
          so.total_iter = (long long)a.hdr->total_iters + it_done;
          so.cost = goal_cost;
          so.t = tnow;
        }
        ++n_sol;
        ++bk.c_sol;
        // ExtractPath: walk the parent chain, goal first
        float* ps = a.path_states;
        float* pa = a.path_actions;
#pragma unroll
        for (int c = 0; c < D; ++c) ps[c] = stg_x[(size_t)c * S + goal_e];
#pragma unroll
        for (int c = 0; c < M; ++c) pa[c] = stg_u[(size_t)c * S + goal_e];
        int p = stg_par[goal_e];
        int ne = 1;
        int trunc = 0;
        while (p > 0) {
          if (ne >= P.max_path_edges) {
            trunc = 1;
            break;
          }
#pragma unroll
          for (int c = 0; c < D; ++c) ps[(size_t)ne * D + c] = a.states[(size_t)c * NC + p];
#pragma unroll
          for (int c = 0; c < M; ++c) pa[(size_t)ne * M + c] = a.actions[(size_t)c * NC + p];
          p = a.parents[p];
          ++ne;
        }
#pragma unroll
        for (int c = 0; c < D; ++c) ps[(size_t)ne * D + c] = a.states[(size_t)c * NC];
        a.hdr->best_edges = ne;
        a.hdr->best_node = goal_slot;
        a.hdr->best_cost = goal_cost;
        a.hdr->path_truncated = trunc;
      }
    }

    mark(5);
    if (goal) c_best = goal_cost;
    if (end == END_TREE_FULL) status |= PAKR_S_TREE_FULL;
    if (end == END_ITER_CAP) status |= PAKR_S_ITER_CAP;
    if (end != END_NONE) {
      ++round;
      iter = 0;
      n = 1;
      ++rounds_done;
      spec_lo = 0;
      pre_n = 0;
    } else {
      ++iter;
      n = n1;
      spec_lo = spec_next;
      pre_n = pre_done;
    }
    ++it_done;
    if (TIERED) {
      const int G_next = tier_grid(n);
      if (G_next != G) {
        pre_n = 0;  // (the tiles' owners change with the grid)
        // a larger tier: this tier's writes reach memory (a barrier of its
        // workgroups), then workgroup 0 wakes the workgroups that join; a
        // smaller one (a new round): every participant's writes reach memory
        // before fewer workgroups reuse the tree's slots
        if (G > 1 && !grid_barrier(a, gen, &s_fail, b, G)) {
          failed = true;
          break;
        }
        if (G_next > G && b == 0) {
          const LoopState st = {n, round, iter, n_sol, (int)rounds_done, status, c_best, gen,
                                it_done, 0, G_next};
          publish_handoff(a, st);
        }
      }
    }
  }
  if (failed) {
    // every participant leaves; workgroup 0 also releases the workgroups that
    // wait outside the tier (the plan is unusable: nothing more is written)
    if (tid == 0) __hip_atomic_store(&a.hdr->err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (TIERED && b == 0) {
      const LoopState st = {n, round, iter, n_sol, (int)rounds_done, status, c_best, gen, it_done,
                            1, G_all};
      publish_handoff(a, st);
    }
    return;
  }
  // workgroups outside the last tier may be waiting for a hand-off: the call has ended
  if (TIERED && b == 0 && tier_grid(n) < G_all) {
    const LoopState st = {n, round, iter, n_sol, (int)rounds_done, status, c_best, gen, it_done, 1,
                          G_all};
    publish_handoff(a, st);
  }

  if (b == 0 && tid == 0) {
    DevHeader* h = a.hdr;
    h->n = n;
    h->round = round;
    h->iter = iter;
    h->c_best = c_best;
    h->n_solutions = n_sol;
    h->bar_gen = gen;
    h->total_iters += (unsigned long long)it_done;
    h->expansions += bk.c_exp;
    h->insertions += bk.c_ins;
    h->nn_pairs += bk.c_nn;
    h->t_start = bk.t0;
    h->t_end = wall_clock64();
    h->t_first = bk.t_first;
    h->t_last = bk.t_last;
    h->call_iters = (int)it_done;
    h->call_rounds = (int)rounds_done;
    h->call_solutions = bk.c_sol;
    h->status = status | (n_sol > 0 ? PAKR_S_SOLVED : 0);
    for (int i = 0; i < 6; ++i) h->ticks[i] = bk.tk[i];
  }
}

__device__ __forceinline__ Smem make_smem(float* obs, float* tile, float* targets,
                                          unsigned long long* keys, int* cnt, int* off, int* wave, float* val,
                                          unsigned long long* goal, int* fail, int* misc,
                                          Books* books, LoopState* state) {
  Smem m;
  m.obs = obs;
  m.tile = tile;
  m.targets = targets;
  m.keys = keys;
  m.cnt = cnt;
  m.off = off;
  m.wave = wave;
  m.val = val;
  m.goal = goal;
  m.fail = fail;
  m.misc = misc;
  m.books = books;
  m.state = state;
  return m;
}

// One query planned by the whole (cooperative) grid.
template <int SYS, int QT>
__global__ __launch_bounds__(NT) void k_plan(KArgs a) {
  extern __shared__ float s_obs[];
  __shared__ __align__(16) float s_tile[Sys<SYS>::D * TILE];
  __shared__ float s_targets[Sys<SYS>::D * NN_KC<QT>];
  __shared__ unsigned long long s_keys[NN_KC<QT>];
  __shared__ int s_cnt[MAX_GR];
  __shared__ int s_off[MAX_GR + 1];
  __shared__ int s_wave[NT / WAVE];
  __shared__ float s_val[VAL_FLOATS];
  __shared__ unsigned long long s_goal;
  __shared__ int s_fail;
  __shared__ int s_misc[2];
  __shared__ Books s_books;
  __shared__ LoopState s_state;
  const Smem sm = make_smem(s_obs, s_tile, s_targets, s_keys, s_cnt, s_off, s_wave, s_val,
                            &s_goal, &s_fail, s_misc, &s_books, &s_state);
  // (above 6 state dimensions the plan keeps the plain scan: the node-slice
  // form costs the quadrotor's rollout code more than it saves)
  plan_loop<SYS, QT, (Sys<SYS>::D <= 6), true>(a, blockIdx.x, gridDim.x, sm);
}

// Many queries in one launch: each workgroup takes the next query from a
// device work queue and plans it alone (no grid barrier), until the queue is
// empty.  Queries may mix systems and tree capacities.
// Persistent batch: each workgroup takes the next ticket (query, member) from
// the device queue and runs that member's part of the query's AO-x loop with
// its teammates (consecutive tickets), then takes the next ticket.  Only
// running workgroups take tickets, so a team's members are co-resident, and
// every team below the first untaken ticket is complete and can progress.
__global__ __launch_bounds__(NT) void k_batch(const KArgs* __restrict__ qs,
                                              const int* __restrict__ tickets, int n_tickets,
                                              int* queue) {
  extern __shared__ float s_obs[];
  __shared__ __align__(16) float s_tile[PAKR_MAX_D * TILE];
  __shared__ float s_targets[PAKR_MAX_D * NN_KC<1>];
  __shared__ unsigned long long s_keys[NN_KC<1>];
  __shared__ int s_cnt[MAX_GR];
  __shared__ int s_off[MAX_GR + 1];
  __shared__ int s_wave[NT / WAVE];
  __shared__ float s_val[VAL_FLOATS];
  __shared__ unsigned long long s_goal;
  __shared__ int s_fail;
  __shared__ int s_misc[2];
  __shared__ int s_ticket;
  __shared__ Books s_books;
  __shared__ LoopState s_state;
  const Smem sm = make_smem(s_obs, s_tile, s_targets, s_keys, s_cnt, s_off, s_wave, s_val,
                            &s_goal, &s_fail, s_misc, &s_books, &s_state);
  while (true) {
    __syncthreads();  // everyone has read the previous s_ticket
    if (threadIdx.x == 0) {
      const int t = atomicAdd(queue, 1);
      s_ticket = t < n_tickets ? tickets[t] : -1;
    }
    __syncthreads();
    const int ticket = __builtin_amdgcn_readfirstlane(s_ticket);
    if (ticket < 0) break;
    const KArgs& a = qs[ticket >> 5];
    const int member = ticket & 31, team = a.P.G;
    switch (a.P.system) {
      case PAKR_DI2: plan_loop<PAKR_DI2, 1, true, false>(a, member, team, sm); break;
      case PAKR_DI3: plan_loop<PAKR_DI3, 1, true, false>(a, member, team, sm); break;
      case PAKR_CAR: plan_loop<PAKR_CAR, 1, true, false>(a, member, team, sm); break;
      case PAKR_DUBINS: plan_loop<PAKR_DUBINS, 1, true, false>(a, member, team, sm); break;
      case PAKR_UNI1: plan_loop<PAKR_UNI1, 1, true, false>(a, member, team, sm); break;
      case PAKR_UNI2: plan_loop<PAKR_UNI2, 1, true, false>(a, member, team, sm); break;
      case PAKR_ACROBOT: plan_loop<PAKR_ACROBOT, 1, true, false>(a, member, team, sm); break;
      case PAKR_CARTPOLE: plan_loop<PAKR_CARTPOLE, 1, true, false>(a, member, team, sm); break;
      default: plan_loop<PAKR_QUAD, 1, true, false>(a, member, team, sm); break;
    }
  }
}

__global__ void k_reset_queue(int* queue) {
  if (threadIdx.x == 0) *queue = 0;
}

// Writes the root (x_init, no action, cost 0) and resets the loop state.
__global__ void k_init(DevHeader* hdr, uint32_t* bar_flags, int n_flags, float* states,
                       float* actions, int* parents, float* costs, int n_cap, int d, int m,
                       float x0, float x1, float x2, float x3, float x4, float x5, float x6,
                       float x7, float x8, float x9, float x10, float x11, float c0) {
  const int tid = threadIdx.x;
  for (int i = tid; i < n_flags; i += blockDim.x) bar_flags[i] = 0u;
  if (tid == 0) {
    const float xi[12] = {x0, x1, x2, x3, x4, x5, x6, x7, x8, x9, x10, x11};
    for (int c = 0; c < d; ++c) states[(size_t)c * n_cap] = xi[c];
    for (int c = 0; c < m; ++c) actions[(size_t)c * n_cap] = 0.0f;
    parents[0] = -1;
    costs[0] = 0.0f;
    DevHeader z = {};
    z.n = 1;
    z.c_best = c0;
    z.best_edges = -1;
    z.best_node = -1;
    z.t_first = -1;
    z.t_last = -1;
    *hdr = z;
  }
}

}  // namespace pakr
