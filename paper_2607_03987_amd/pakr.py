"""Python binding of libpakr (include/pakr.h): argument marshalling only.

Every step of the planner runs in the HIP kernels of libpakr.so.  PyTorch
provides device memory (the plan workspace and trace buffers are torch
tensors) and the HIP stream.  There is no fallback: if the library is not
built, or no GPU is present, the calls raise.

The function names follow the C ABI: ``workspace_size``, ``plan_init``,
``expand``, ``replan``, ``status``, ``solutions``, ``extract_path``,
``copy_tree``; ``Plan`` bundles them.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from typing import Optional

import numpy as np

from . import workloads as W

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libpakr.so")

MAX_D, MAX_M = 12, 4
PAKR_OK = 0
ERRORS = {0: "PAKR_OK", -1: "PAKR_E_INVALID_ARG", -2: "PAKR_E_START_INVALID",
          -3: "PAKR_E_GOAL_INVALID", -4: "PAKR_E_WORKSPACE_TOO_SMALL", -5: "PAKR_E_HIP",
          -6: "PAKR_E_NO_SOLUTION", -7: "PAKR_E_BUFFER_TOO_SMALL", -8: "PAKR_E_DEVICE"}
S_SOLVED, S_BUDGET_EXPIRED, S_ROUNDS_DONE, S_ITERS_DONE = 1, 2, 4, 8
S_TREE_FULL, S_ITER_CAP, S_DEVICE_ERROR = 16, 32, 64
F_VALID, F_PRUNE_OK, F_KEEP, F_GOAL = 1, 2, 4, 8
TRACE_HDR_WORDS = 16

EXPORTED = ["pakr_workspace_size", "pakr_plan_init", "pakr_plan_destroy", "pakr_trace_bytes",
            "pakr_expand", "pakr_replan", "pakr_status", "pakr_solutions", "pakr_extract_path",
            "pakr_copy_tree", "pakr_last_error", "pakr_error_string",
            "pakr_batch_workspace_size", "pakr_batch_init", "pakr_batch_replan",
            "pakr_batch_graph_capture", "pakr_batch_graph_launch", "pakr_batch_status",
            "pakr_batch_solutions", "pakr_batch_extract_path", "pakr_batch_grid",
            "pakr_batch_team", "pakr_batch_trace_bytes", "pakr_batch_expand",
            "pakr_batch_copy_tree", "pakr_set_barrier_timeout",
            "pakr_batch_last_error", "pakr_batch_destroy",
            "pakr_refiner_init", "pakr_refiner_set_params", "pakr_rollout_ckpt_bytes",
            "pakr_rollout_fwd", "pakr_rollout_bwd", "pakr_refine_step", "pakr_check_path",
            "pakr_refine_workspace_size", "pakr_refine_paths", "pakr_refine_paths_static",
            "pakr_refiner_last_error", "pakr_refiner_destroy"]


class PakrError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class System(C.Structure):
    _fields_ = [("id", C.c_int), ("d", C.c_int), ("m", C.c_int), ("dyn", C.c_float * 8),
                ("sample_lo", C.c_float * MAX_D), ("sample_hi", C.c_float * MAX_D),
                ("u_lo", C.c_float * MAX_M), ("u_hi", C.c_float * MAX_M),
                ("lim_lo", C.c_float * MAX_D), ("lim_hi", C.c_float * MAX_D),
                ("vnorm_max", C.c_float)]


class Scene(C.Structure):
    _fields_ = [("npos", C.c_int), ("ws_lo", C.c_float * 3), ("ws_hi", C.c_float * 3),
                ("n_box", C.c_int), ("box_c", C.POINTER(C.c_float)), ("box_h", C.POINTER(C.c_float)),
                ("n_sphere", C.c_int), ("sph_c", C.POINTER(C.c_float)),
                ("sph_r", C.POINTER(C.c_float))]


class Goal(C.Structure):
    _fields_ = [("center", C.c_float * 3), ("radius", C.c_float)]


class Params(C.Structure):
    _fields_ = [("B", C.c_int), ("A", C.c_int), ("T", C.c_int), ("dt", C.c_float),
                ("n_cap", C.c_int), ("cost_kind", C.c_int), ("heuristic_kind", C.c_int),
                ("h_speed", C.c_float), ("cost_bound", C.c_double), ("seed", C.c_uint64),
                ("query_id", C.c_uint32), ("max_iters_per_round", C.c_int), ("grid", C.c_int),
                ("max_path_edges", C.c_int), ("lanes_per_candidate", C.c_int),
                ("workgroups_per_cu", C.c_int), ("spec_tiles", C.c_int),
                ("tier0_nodes", C.c_int), ("tier1_nodes", C.c_int), ("tier1_grid", C.c_int),
                ("tier_scan_cycles", C.c_int)]


class Stats(C.Structure):
    _fields_ = [("n_nodes", C.c_int), ("round", C.c_int), ("iter", C.c_int), ("status", C.c_int),
                ("n_solutions", C.c_int), ("grid", C.c_int), ("total_iters", C.c_longlong),
                ("expansions", C.c_longlong), ("insertions", C.c_longlong),
                ("nn_pairs", C.c_longlong), ("c_best", C.c_double), ("call_ms", C.c_double),
                ("t_first_ms", C.c_double), ("t_last_ms", C.c_double), ("call_iters", C.c_int),
                ("call_rounds", C.c_int), ("call_solutions", C.c_int), ("reserved", C.c_int),
                ("nn_ms", C.c_double), ("rollout_ms", C.c_double), ("insert_ms", C.c_double),
                ("step_ms", C.c_double * 6), ("clock_start_ms", C.c_double),
                ("clock_end_ms", C.c_double), ("near_ties_prune", C.c_longlong),
                ("near_ties_goal", C.c_longlong), ("tier_nodes", C.c_int * 8),
                ("tier_grid", C.c_int * 8)]


class Solution(C.Structure):
    _fields_ = [("round", C.c_int), ("iter", C.c_int), ("node", C.c_int), ("n_nodes", C.c_int),
                ("total_iter", C.c_longlong), ("cost", C.c_double), ("t_ms", C.c_double)]


class RefineParams(C.Structure):
    _fields_ = [("w_effort", C.c_float), ("w_goal", C.c_float), ("w_collision", C.c_float),
                ("beta", C.c_float), ("delta", C.c_float), ("u_ref", C.c_float * MAX_M),
                ("u_scale", C.c_float * MAX_M)]


_lib = None


def load():
    """Load libpakr.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run __graft_entry__.build() first")
        import torch  # noqa: F401  -- the HIP runtime comes from torch's process image
        L = C.CDLL(LIB_PATH, mode=C.RTLD_GLOBAL)
        vp, sz = C.c_void_p, C.c_size_t
        L.pakr_workspace_size.argtypes = [C.POINTER(System), C.POINTER(Params), C.POINTER(Scene)]
        L.pakr_workspace_size.restype = sz
        L.pakr_plan_init.argtypes = [C.POINTER(System), C.POINTER(Scene), C.POINTER(C.c_float),
                                     C.POINTER(Goal), C.POINTER(Params), vp, sz, vp,
                                     C.POINTER(vp)]
        L.pakr_plan_init.restype = C.c_int
        L.pakr_plan_destroy.argtypes = [vp]
        L.pakr_plan_destroy.restype = None
        L.pakr_trace_bytes.argtypes = [vp, C.c_int]
        L.pakr_trace_bytes.restype = sz
        L.pakr_expand.argtypes = [vp, C.c_int, vp, sz]
        L.pakr_expand.restype = C.c_int
        L.pakr_replan.argtypes = [vp, C.c_double, C.c_int, C.c_longlong]
        L.pakr_replan.restype = C.c_int
        L.pakr_status.argtypes = [vp, C.POINTER(Stats)]
        L.pakr_status.restype = C.c_int
        L.pakr_solutions.argtypes = [vp, C.POINTER(Solution), C.c_int, C.POINTER(C.c_int)]
        L.pakr_solutions.restype = C.c_int
        L.pakr_extract_path.argtypes = [vp, C.POINTER(C.c_float), C.POINTER(C.c_float), C.c_int,
                                        C.POINTER(C.c_int), C.POINTER(C.c_double)]
        L.pakr_extract_path.restype = C.c_int
        L.pakr_copy_tree.argtypes = [vp, C.POINTER(C.c_float), C.POINTER(C.c_float),
                                     C.POINTER(C.c_int), C.POINTER(C.c_float), C.c_int,
                                     C.POINTER(C.c_int)]
        L.pakr_copy_tree.restype = C.c_int
        L.pakr_last_error.argtypes = [vp]
        L.pakr_last_error.restype = C.c_char_p
        L.pakr_error_string.argtypes = [C.c_int]
        L.pakr_error_string.restype = C.c_char_p
        L.pakr_batch_workspace_size.argtypes = [C.c_int, C.POINTER(System), C.POINTER(Scene),
                                                C.POINTER(Params)]
        L.pakr_batch_workspace_size.restype = sz
        L.pakr_batch_init.argtypes = [C.c_int, C.POINTER(System), C.POINTER(Scene),
                                      C.POINTER(C.POINTER(C.c_float)), C.POINTER(Goal),
                                      C.POINTER(Params), vp, sz, vp, C.POINTER(vp)]
        L.pakr_batch_init.restype = C.c_int
        L.pakr_batch_replan.argtypes = [vp, C.c_double, C.c_int, C.c_longlong]
        L.pakr_batch_replan.restype = C.c_int
        L.pakr_batch_graph_capture.argtypes = [vp, C.c_double, C.c_int, C.c_longlong]
        L.pakr_batch_graph_capture.restype = C.c_int
        L.pakr_batch_graph_launch.argtypes = [vp]
        L.pakr_batch_graph_launch.restype = C.c_int
        L.pakr_batch_status.argtypes = [vp, C.c_int, C.POINTER(Stats)]
        L.pakr_batch_status.restype = C.c_int
        L.pakr_batch_solutions.argtypes = [vp, C.c_int, C.POINTER(Solution), C.c_int,
                                           C.POINTER(C.c_int)]
        L.pakr_batch_solutions.restype = C.c_int
        L.pakr_batch_extract_path.argtypes = [vp, C.c_int, C.POINTER(C.c_float),
                                              C.POINTER(C.c_float), C.c_int, C.POINTER(C.c_int),
                                              C.POINTER(C.c_double)]
        L.pakr_batch_extract_path.restype = C.c_int
        L.pakr_batch_grid.argtypes = [vp]
        L.pakr_batch_grid.restype = C.c_int
        L.pakr_batch_team.argtypes = [vp, C.c_int]
        L.pakr_batch_team.restype = C.c_int
        L.pakr_batch_trace_bytes.argtypes = [vp, C.c_int, C.c_int]
        L.pakr_batch_trace_bytes.restype = sz
        L.pakr_batch_expand.argtypes = [vp, C.c_int, C.POINTER(vp), C.POINTER(sz)]
        L.pakr_batch_expand.restype = C.c_int
        L.pakr_batch_copy_tree.argtypes = [vp, C.c_int, C.POINTER(C.c_float),
                                           C.POINTER(C.c_float), C.POINTER(C.c_int),
                                           C.POINTER(C.c_float), C.c_int, C.POINTER(C.c_int)]
        L.pakr_batch_copy_tree.restype = C.c_int
        L.pakr_set_barrier_timeout.argtypes = [C.c_double]
        L.pakr_set_barrier_timeout.restype = C.c_int
        L.pakr_batch_last_error.argtypes = [vp]
        L.pakr_batch_last_error.restype = C.c_char_p
        L.pakr_batch_destroy.argtypes = [vp]
        L.pakr_batch_destroy.restype = None
        L.pakr_refiner_init.argtypes = [C.POINTER(System), C.POINTER(Scene), C.POINTER(Goal),
                                        C.POINTER(Params), C.POINTER(RefineParams), vp,
                                        C.POINTER(vp)]
        L.pakr_refiner_init.restype = C.c_int
        L.pakr_refiner_set_params.argtypes = [vp, C.POINTER(RefineParams)]
        L.pakr_refiner_set_params.restype = C.c_int
        L.pakr_rollout_ckpt_bytes.argtypes = [vp, C.c_int, C.c_int]
        L.pakr_rollout_ckpt_bytes.restype = sz
        L.pakr_rollout_fwd.argtypes = [vp, C.c_int, C.c_int, vp, vp, vp, sz, vp]
        L.pakr_rollout_fwd.restype = C.c_int
        L.pakr_rollout_bwd.argtypes = [vp, C.c_int, C.c_int, vp, vp, sz, vp, vp]
        L.pakr_rollout_bwd.restype = C.c_int
        L.pakr_refine_step.argtypes = [vp, C.c_int, C.c_int, vp, vp, vp, vp, C.c_int, C.c_float]
        L.pakr_refine_step.restype = C.c_int
        L.pakr_refine_workspace_size.argtypes = [vp, C.c_int, C.c_int]
        L.pakr_refine_workspace_size.restype = sz
        L.pakr_refine_paths.argtypes = [vp, C.c_int, C.c_int, vp, vp, C.c_int, C.c_float, vp, sz,
                                        vp, vp]
        L.pakr_refine_paths.restype = C.c_int
        L.pakr_refine_paths_static.argtypes = [vp, C.c_int, C.c_int, vp, vp, C.c_int, C.c_float,
                                               vp, vp]
        L.pakr_refine_paths_static.restype = C.c_int
        L.pakr_check_path.argtypes = [vp, C.c_int, C.c_int, vp, vp, vp, vp]
        L.pakr_check_path.restype = C.c_int
        L.pakr_refiner_last_error.argtypes = [vp]
        L.pakr_refiner_last_error.restype = C.c_char_p
        L.pakr_refiner_destroy.argtypes = [vp]
        L.pakr_refiner_destroy.restype = None
        _lib = L
    return _lib


def _fp(a):
    return a.ctypes.data_as(C.POINTER(C.c_float))


class CQuery:
    """The C structs of one Problem (holds the host arrays alive)."""

    def __init__(self, prob: W.Problem, grid: int = 0, max_path_edges: int = 0, lanes: int = 0,
                 wg_per_cu: int = 0, spec: int = 0, tier0: int = 0, tier1: int = 0,
                 tier1_grid: int = 0, tier_scan: int = 0):
        self.prob = prob
        s = System()
        s.id, s.d, s.m = prob.system, prob.d, prob.m
        for i in range(8):
            s.dyn[i] = float(prob.dyn[i])
        for i in range(prob.d):
            s.sample_lo[i], s.sample_hi[i] = float(prob.sample_lo[i]), float(prob.sample_hi[i])
            s.lim_lo[i], s.lim_hi[i] = float(prob.lim_lo[i]), float(prob.lim_hi[i])
        for i in range(prob.m):
            s.u_lo[i], s.u_hi[i] = float(prob.u_lo[i]), float(prob.u_hi[i])
        s.vnorm_max = float(prob.vnorm_max)
        self.system = s
        P = prob.npos
        self._bc = np.ascontiguousarray(prob.box_c, np.float32).reshape(-1)
        self._bh = np.ascontiguousarray(prob.box_h, np.float32).reshape(-1)
        self._sc = np.ascontiguousarray(prob.sph_c, np.float32).reshape(-1)
        self._sr = np.ascontiguousarray(prob.sph_r, np.float32).reshape(-1)
        sc = Scene()
        sc.npos = P
        for c in range(P):
            sc.ws_lo[c], sc.ws_hi[c] = float(prob.ws_lo[c]), float(prob.ws_hi[c])
        sc.n_box, sc.box_c, sc.box_h = int(prob.box_c.shape[0]), _fp(self._bc), _fp(self._bh)
        sc.n_sphere, sc.sph_c, sc.sph_r = int(prob.sph_r.shape[0]), _fp(self._sc), _fp(self._sr)
        self.scene = sc
        g = Goal()
        for c in range(P):
            g.center[c] = float(prob.goal_c[c])
        g.radius = float(prob.goal_r)
        self.goal = g
        self.x_init = np.ascontiguousarray(prob.x_init, np.float32)
        p = Params()
        p.B, p.A, p.T, p.dt, p.n_cap = prob.B, prob.A, prob.T, float(prob.dt), prob.n_cap
        p.cost_kind, p.heuristic_kind, p.h_speed = prob.cost_kind, prob.h_kind, float(prob.h_speed)
        p.cost_bound = float(prob.c0)
        p.seed, p.query_id = int(prob.seed), int(prob.qid)
        p.max_iters_per_round = int(prob.max_iters_per_round)
        p.grid, p.max_path_edges = int(grid), int(max_path_edges)
        p.lanes_per_candidate = int(lanes)
        p.workgroups_per_cu = int(wg_per_cu)
        p.spec_tiles = int(spec)
        p.tier0_nodes = int(tier0)
        p.tier1_nodes = int(tier1)
        p.tier1_grid = int(tier1_grid)
        p.tier_scan_cycles = int(tier_scan)
        self.params = p


def _stats_dict(s: "Stats") -> dict:
    out = {f[0]: getattr(s, f[0]) for f in Stats._fields_}
    for k in ("step_ms", "tier_nodes", "tier_grid"):
        out[k] = list(out[k])
    return out


def workspace_size(q: CQuery) -> int:
    return int(load().pakr_workspace_size(C.byref(q.system), C.byref(q.params), C.byref(q.scene)))


def _check(rc: int, handle=None):
    if rc != PAKR_OK:
        msg = load().pakr_last_error(handle)
        raise PakrError(rc, msg.decode() if msg else "")


def plan_init(q: CQuery, d_workspace: int, ws_bytes: int, stream: int) -> int:
    h = C.c_void_p()
    rc = load().pakr_plan_init(C.byref(q.system), C.byref(q.scene), _fp(q.x_init), C.byref(q.goal),
                               C.byref(q.params), C.c_void_p(d_workspace), ws_bytes,
                               C.c_void_p(stream), C.byref(h))
    _check(rc, None)
    return h.value


class Plan:
    """One planning query on the current GPU.

    The workspace (tree, work buffers) is a torch uint8 tensor on the device;
    calls are enqueued on torch's current stream.
    """

    def __init__(self, prob: W.Problem, grid: int = 0, max_path_edges: int = 0, device=None,
                 lanes: int = 0, wg_per_cu: int = 0, spec: int = 0, tier0: int = 0,
                 tier1: int = 0, tier1_grid: int = 0, tier_scan: int = 0):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("libpakr needs a ROCm GPU; none is visible")
        self.torch = torch
        self.prob = prob
        self.q = CQuery(prob, grid=grid, max_path_edges=max_path_edges, lanes=lanes,
                        wg_per_cu=wg_per_cu, spec=spec, tier0=tier0, tier1=tier1,
                        tier1_grid=tier1_grid, tier_scan=tier_scan)
        self.device = torch.device(device or "cuda")
        nbytes = workspace_size(self.q)
        if nbytes == 0:
            raise PakrError(-1, "workspace_size rejected the query")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        self._ws_ptr = (base + 255) & ~255
        self.stream = torch.cuda.current_stream(self.device)
        self.h = plan_init(self.q, self._ws_ptr, nbytes, self.stream.cuda_stream)
        self.K, self.B, self.d, self.m = prob.K, prob.B, prob.d, prob.m

    def close(self):
        h = getattr(self, "h", None)
        if h:
            load().pakr_plan_destroy(h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # --- C calls -----------------------------------------------------------
    def trace_bytes(self, n_iters: int) -> int:
        return int(load().pakr_trace_bytes(self.h, n_iters))

    def expand(self, n_iters: int, trace: bool = False):
        """Run n_iters iterations; with trace=True return the decoded records."""
        buf = None
        nbytes = 0
        if trace:
            nbytes = self.trace_bytes(n_iters)
            buf = self.torch.zeros(nbytes // 4, dtype=self.torch.int32, device=self.device)
        _check(load().pakr_expand(self.h, n_iters, C.c_void_p(buf.data_ptr() if trace else 0),
                                  nbytes), self.h)
        if not trace:
            return None
        self.torch.cuda.synchronize(self.device)
        return self.decode_trace(buf.cpu().numpy(), n_iters)

    def replan(self, budget_ms: float = 0.0, max_rounds: int = 0, max_iters: int = 0):
        _check(load().pakr_replan(self.h, float(budget_ms), int(max_rounds), int(max_iters)), self.h)

    def status(self) -> dict:
        s = Stats()
        _check(load().pakr_status(self.h, C.byref(s)), self.h)
        return _stats_dict(s)

    def solutions(self) -> list:
        n = C.c_int(0)
        _check(load().pakr_solutions(self.h, None, 0, C.byref(n)), self.h)
        arr = (Solution * max(n.value, 1))()
        _check(load().pakr_solutions(self.h, arr, n.value, C.byref(n)), self.h)
        cnt = min(n.value, 1024)
        return [{f[0]: getattr(arr[i], f[0]) for f in Solution._fields_} for i in range(cnt)]

    def extract_path(self):
        ne = C.c_int(0)
        cost = C.c_double(0)
        rc = load().pakr_extract_path(self.h, None, None, 0, C.byref(ne), C.byref(cost))
        if rc == -6:
            return None
        if rc not in (0, -7):
            _check(rc, self.h)
        n = ne.value
        states = np.zeros((n + 1, self.d), np.float32)
        actions = np.zeros((max(n, 1), self.m), np.float32)
        _check(load().pakr_extract_path(self.h, _fp(states), _fp(actions), n, C.byref(ne),
                                        C.byref(cost)), self.h)
        return states, actions[:n], cost.value

    def copy_tree(self):
        return _copy_tree(lambda *a: _check(load().pakr_copy_tree(self.h, *a), self.h),
                          self.d, self.m)

    # --- trace decoding ----------------------------------------------------
    def decode_trace(self, words: np.ndarray, n_iters: int) -> list:
        return decode_trace(words, n_iters, self.K, self.B, self.d, self.m)


def _copy_tree(call, d: int, m: int):
    """Node-major tree of a plan or batch query through a pakr_*copy_tree call."""
    n = C.c_int(0)
    call(None, None, None, None, 0, C.byref(n))
    nn = n.value
    states = np.zeros((nn, d), np.float32)
    actions = np.zeros((nn, m), np.float32)
    parents = np.zeros(nn, np.int32)
    costs = np.zeros(nn, np.float32)
    call(_fp(states), _fp(actions), parents.ctypes.data_as(C.POINTER(C.c_int)), _fp(costs), nn,
         C.byref(n))
    return states, actions, parents, costs


def decode_trace(words: np.ndarray, n_iters: int, K: int, B: int, d: int, m: int) -> list:
    """Decode n_iters trace records (int32 words, layout of pakr_expand in pakr.h)."""
    per = TRACE_HDR_WORDS + K * d + K + B * m + B * d + 3 * B
    out = []
    for i in range(n_iters):
        w = words[i * per:(i + 1) * per]
        h = w[:TRACE_HDR_WORDS]
        o = TRACE_HDR_WORDS
        f32 = lambda a: a.view(np.float32)
        targets = f32(w[o:o + K * d]).reshape(K, d); o += K * d
        parents = w[o:o + K].copy(); o += K
        controls = f32(w[o:o + B * m]).reshape(B, m); o += B * m
        xnew = f32(w[o:o + B * d]).reshape(B, d); o += B * d
        cnew = f32(w[o:o + B]).copy(); o += B
        flags = w[o:o + B].copy(); o += B
        slots = w[o:o + B].copy(); o += B
        out.append(dict(round=int(h[0]), iter=int(h[1]), n0=int(h[2]), n1=int(h[3]),
                        goal_j=int(h[4]), goal_slot=int(h[5]), end=int(h[6]),
                        c_best_before=float(h[7:8].view(np.float32)[0]),
                        c_best_after=float(h[8:9].view(np.float32)[0]),
                        survivors=int(h[9]), targets=targets.copy(), parents=parents,
                        controls=controls.copy(), xnew=xnew.copy(), cnew=cnew, flags=flags,
                        slots=slots))
    return out


def set_barrier_timeout(ms: float):
    """Grid-barrier wait limit of later launches (ms <= 0: the default 2000 ms)."""
    _check(load().pakr_set_barrier_timeout(float(ms)), None)


def _bcheck(rc: int, handle=None):
    if rc != PAKR_OK:
        msg = load().pakr_batch_last_error(handle)
        raise PakrError(rc, msg.decode() if msg else "")


class CBatch:
    """The C arrays of a list of Problems (holds the host arrays alive)."""

    def __init__(self, probs, lanes=0, teams=0, spec=0, tier0=0):
        self.probs = list(probs)
        n = self.n = len(self.probs)
        per = lambda v: [int(v)] * n if isinstance(v, int) else [int(x) for x in v]
        teams, lanes, spec, tier0 = per(teams), per(lanes), per(spec), per(tier0)
        self.qs = [CQuery(p, lanes=v, grid=t, spec=s, tier0=z)
                   for p, v, t, s, z in zip(self.probs, lanes, teams, spec, tier0)]
        self.sys = (System * n)(*[q.system for q in self.qs])
        self.sc = (Scene * n)(*[q.scene for q in self.qs])
        self.goal = (Goal * n)(*[q.goal for q in self.qs])
        self.prm = (Params * n)(*[q.params for q in self.qs])
        self.x = (C.POINTER(C.c_float) * n)(*[_fp(q.x_init) for q in self.qs])


def batch_workspace_size(cb: CBatch) -> int:
    return int(load().pakr_batch_workspace_size(cb.n, cb.sys, cb.sc, cb.prm))


def batch_init(cb: CBatch, d_workspace: int, ws_bytes: int, stream: int) -> int:
    h = C.c_void_p()
    rc = load().pakr_batch_init(cb.n, cb.sys, cb.sc, cb.x, cb.goal, cb.prm,
                                C.c_void_p(d_workspace), ws_bytes, C.c_void_p(stream), C.byref(h))
    _bcheck(rc, None)
    return h.value


class BatchPlan:
    """Many queries planned by one persistent launch (a team of workgroups per query).

    Query q's results equal those of Plan(probs[q], lanes=...) with the same
    parameters; the workspace is one torch uint8 tensor.  `lanes` and `teams`
    (an int for every query or a list) set the lanes per candidate and the
    team sizes; team 0 lets the library size each team by the query's share of
    the estimated work.
    """

    def __init__(self, probs, lanes=0, device=None, teams=0, spec=0, tier0=0):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("libpakr needs a ROCm GPU; none is visible")
        self.torch = torch
        self.cb = CBatch(probs, lanes=lanes, teams=teams, spec=spec, tier0=tier0)
        self.probs = self.cb.probs
        nbytes = batch_workspace_size(self.cb)
        if nbytes == 0:
            batch_init(self.cb, 0, 0, 0)  # reports which query is malformed
            raise PakrError(-1, "batch_workspace_size rejected the queries")
        self.device = torch.device(device or "cuda")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        ptr = (self.workspace.data_ptr() + 255) & ~255
        self.stream = torch.cuda.current_stream(self.device)
        self.h = batch_init(self.cb, ptr, nbytes, self.stream.cuda_stream)
        self.n = self.cb.n

    def close(self):
        h = getattr(self, "h", None)
        if h:
            load().pakr_batch_destroy(h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def grid(self) -> int:
        return int(load().pakr_batch_grid(self.h))

    def team(self, q: int) -> int:
        return int(load().pakr_batch_team(self.h, int(q)))

    def replan(self, budget_ms: float = 0.0, max_rounds: int = 0, max_iters: int = 0):
        _bcheck(load().pakr_batch_replan(self.h, float(budget_ms), int(max_rounds),
                                         int(max_iters)), self.h)

    def expand(self, n_iters: int, trace: bool = False):
        """Run n_iters iterations of every query in one launch; with trace=True
        return, per query, the decoded records (as Plan.expand)."""
        n = self.n
        bufs, nbytes = [], []
        if trace:
            for q in range(n):
                nb = int(load().pakr_batch_trace_bytes(self.h, q, n_iters))
                bufs.append(self.torch.zeros(nb // 4, dtype=self.torch.int32, device=self.device))
                nbytes.append(nb)
        ptrs = (C.c_void_p * n)(*[b.data_ptr() for b in bufs]) if trace else None
        sizes = (C.c_size_t * n)(*nbytes) if trace else None
        _bcheck(load().pakr_batch_expand(self.h, int(n_iters), ptrs, sizes), self.h)
        if not trace:
            return None
        self.torch.cuda.synchronize(self.device)
        return [decode_trace(b.cpu().numpy(), n_iters, p.K, p.B, p.d, p.m)
                for b, p in zip(bufs, self.probs)]

    def copy_tree(self, q: int):
        p = self.probs[q]
        return _copy_tree(lambda *a: _bcheck(load().pakr_batch_copy_tree(self.h, q, *a), self.h),
                          p.d, p.m)

    def graph_capture(self, budget_ms: float = 0.0, max_rounds: int = 0, max_iters: int = 0):
        _bcheck(load().pakr_batch_graph_capture(self.h, float(budget_ms), int(max_rounds),
                                                int(max_iters)), self.h)

    def graph_launch(self):
        _bcheck(load().pakr_batch_graph_launch(self.h), self.h)

    def status(self, q: int) -> dict:
        s = Stats()
        _bcheck(load().pakr_batch_status(self.h, q, C.byref(s)), self.h)
        return _stats_dict(s)

    def solutions(self, q: int) -> list:
        n = C.c_int(0)
        _bcheck(load().pakr_batch_solutions(self.h, q, None, 0, C.byref(n)), self.h)
        arr = (Solution * max(n.value, 1))()
        _bcheck(load().pakr_batch_solutions(self.h, q, arr, n.value, C.byref(n)), self.h)
        return [{f[0]: getattr(arr[i], f[0]) for f in Solution._fields_}
                for i in range(min(n.value, 1024))]

    def extract_path(self, q: int):
        ne = C.c_int(0)
        cost = C.c_double(0)
        rc = load().pakr_batch_extract_path(self.h, q, None, None, 0, C.byref(ne), C.byref(cost))
        if rc == -6:
            return None
        if rc not in (0, -7):
            _bcheck(rc, self.h)
        n = ne.value
        d, m = self.probs[q].d, self.probs[q].m
        states = np.zeros((n + 1, d), np.float32)
        actions = np.zeros((max(n, 1), m), np.float32)
        _bcheck(load().pakr_batch_extract_path(self.h, q, _fp(states), _fp(actions), n,
                                               C.byref(ne), C.byref(cost)), self.h)
        return states, actions[:n], cost.value


# C-ABI names at module level
def expand(plan: Plan, n_iters: int, trace: bool = False):
    return plan.expand(n_iters, trace)


def replan(plan: Plan, budget_ms: float = 0.0, max_rounds: int = 0, max_iters: int = 0):
    return plan.replan(budget_ms, max_rounds, max_iters)


def status(plan: Plan) -> dict:
    return plan.status()


def extract_path(plan: Plan):
    return plan.extract_path()
