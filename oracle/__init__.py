"""FP64 reference planner (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It wraps ``pakr_oracle.c`` (plain C,
double precision) with ctypes and shares no code with the HIP implementation.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pakr_oracle.c")
_HDR = os.path.join(_HERE, "pakr_oracle.h")
_LIB = os.path.join(_HERE, "liboracle.so")

F_VALID, F_PRUNE_OK, F_KEEP, F_GOAL, F_INSERTED = 1, 2, 4, 8, 16
A_VALID, A_PRUNE, A_GOAL = 1, 2, 4
END_NONE, END_GOAL, END_TREE_FULL, END_ITER_CAP = 0, 1, 2, 3

CFLAGS = ["-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
          "-Wall", "-Wno-unused-variable"]


def build(force: bool = True) -> str:
    """Compile the reference with gcc (double precision, no FP contraction)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= max(
            os.path.getmtime(_SRC), os.path.getmtime(_HDR)):
        return _LIB
    tmp = _LIB + f".tmp{os.getpid()}"
    subprocess.check_call(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


_fp = C.POINTER(C.c_float)
_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)
_u32p = C.POINTER(C.c_uint32)


class _Problem(C.Structure):
    _fields_ = [
        ("system", C.c_int), ("d", C.c_int), ("m", C.c_int), ("npos", C.c_int),
        ("dyn", _fp), ("sample_lo", _fp), ("sample_hi", _fp), ("u_lo", _fp), ("u_hi", _fp),
        ("lim_lo", _fp), ("lim_hi", _fp), ("vnorm_max", C.c_float),
        ("ws_lo", _fp), ("ws_hi", _fp),
        ("n_box", C.c_int), ("box_c", _fp), ("box_h", _fp),
        ("n_sph", C.c_int), ("sph_c", _fp), ("sph_r", _fp),
        ("goal_c", _fp), ("goal_r", C.c_float), ("x_init", _fp),
        ("B", C.c_int), ("A", C.c_int), ("T", C.c_int), ("dt", C.c_float), ("n_cap", C.c_int),
        ("cost_kind", C.c_int), ("h_kind", C.c_int), ("h_speed", C.c_float), ("c0", C.c_double),
        ("seed", C.c_uint64), ("qid", C.c_uint32), ("max_iters_per_round", C.c_int),
        ("eps", C.c_double),
    ]


class _Refine(C.Structure):
    _fields_ = [("w_u", C.c_double), ("w_g", C.c_double), ("w_c", C.c_double),
                ("beta", C.c_double), ("delta", C.c_double), ("u_ref", C.c_double * 4),
                ("u_scale", C.c_double * 4)]


class _Steer(C.Structure):
    _fields_ = [("parents", _ip), ("flags", _ip), ("goal_j", C.c_int)]


class _Report(C.Structure):
    _fields_ = [
        ("targets", _fp), ("parents", _ip), ("nn_d2", _dp), ("nn_tie", _ip), ("controls", _fp),
        ("xnew", _dp), ("cnew", _dp), ("hval", _dp), ("flags", _ip), ("amb", _ip),
        ("slots", _ip),
        ("n0", C.c_int), ("n1", C.c_int), ("round", C.c_int), ("iter", C.c_int),
        ("goal_j", C.c_int), ("goal_slot", C.c_int), ("end_reason", C.c_int),
        ("c_best_before", C.c_double), ("c_best_after", C.c_double),
        ("n_steered", C.c_int), ("n_mismatch", C.c_int), ("goal_tie", C.c_int),
    ]


class _Solution(C.Structure):
    _fields_ = [("round", C.c_int), ("iter", C.c_int), ("node", C.c_int), ("n_nodes", C.c_int),
                ("total_iter", C.c_long), ("cost", C.c_double)]


class _State(C.Structure):
    _fields_ = [("n", C.c_int), ("round", C.c_int), ("iter", C.c_int),
                ("n_solutions", C.c_int), ("last_end", C.c_int),
                ("total_iters", C.c_long), ("expansions", C.c_long),
                ("insertions", C.c_long), ("c_best", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = C.CDLL(_LIB)
        vp = C.c_void_p
        L.orc_philox4x32_10.argtypes = [_u32p, _u32p, _u32p]
        L.orc_u32_to_range.argtypes = [C.c_uint32, C.c_float, C.c_float]
        L.orc_u32_to_range.restype = C.c_float
        L.orc_sample_state.argtypes = [C.POINTER(_Problem), C.c_uint32, C.c_uint32, C.c_uint32, _fp]
        L.orc_sample_control.argtypes = [C.POINTER(_Problem), C.c_uint32, C.c_uint32, C.c_uint32,
                                         C.c_uint32, _fp]
        L.orc_u32_to_range_n.argtypes = [_u32p, C.c_int, C.c_float, C.c_float, _fp]
        L.orc_dynamics.argtypes = [C.POINTER(_Problem), _dp, _dp, _dp]
        L.orc_rk4_step.argtypes = [C.POINTER(_Problem), _dp, _dp, C.c_double, _dp]
        L.orc_rollout.argtypes = [C.POINTER(_Problem), _dp, _dp, C.c_int, C.c_double, _dp]
        L.orc_state_valid.argtypes = [C.POINTER(_Problem), _dp, C.c_double, _ip, _dp]
        L.orc_state_valid.restype = C.c_int
        L.orc_edge.argtypes = [C.POINTER(_Problem), _dp, C.c_double, _dp, _dp, _dp, _ip]
        L.orc_edge.restype = C.c_int
        L.orc_heuristic.argtypes = [C.POINTER(_Problem), _dp]
        L.orc_heuristic.restype = C.c_double
        L.orc_nearest.argtypes = [_dp, C.c_int, C.c_int, _dp, _dp, _dp]
        L.orc_nearest.restype = C.c_int
        L.orc_plan_create.argtypes = [C.POINTER(_Problem)]
        L.orc_plan_create.restype = vp
        L.orc_plan_destroy.argtypes = [vp]
        L.orc_plan_iterate.argtypes = [vp, C.POINTER(_Steer), C.POINTER(_Report)]
        L.orc_plan_iterate.restype = C.c_int
        L.orc_plan_run.argtypes = [vp, C.c_int, C.c_long]
        L.orc_plan_run.restype = C.c_int
        L.orc_plan_get.argtypes = [vp, C.POINTER(_State)]
        L.orc_plan_tree.argtypes = [vp, _dp, _dp, _ip, _dp, C.c_int]
        L.orc_plan_tree.restype = C.c_int
        L.orc_plan_load_tree.argtypes = [vp, _fp, _fp, _ip, _fp, C.c_int, C.c_int, C.c_int,
                                         C.c_double]
        L.orc_plan_load_tree.restype = C.c_int
        L.orc_plan_solutions.argtypes = [vp, C.POINTER(_Solution), C.c_int]
        L.orc_plan_solutions.restype = C.c_int
        L.orc_plan_best_path.argtypes = [vp, _dp, _dp, C.c_int, _ip, _dp]
        L.orc_plan_best_path.restype = C.c_int
        L.orc_traj_cost.argtypes = [C.POINTER(_Problem), C.POINTER(_Refine), _dp, _dp, C.c_int]
        L.orc_traj_cost.restype = C.c_double
        L.orc_traj_grad.argtypes = [C.POINTER(_Problem), C.POINTER(_Refine), _dp, _dp, C.c_int,
                                    _dp]
        _lib = L
    return _lib


def _ptr(a, ct):
    return a.ctypes.data_as(C.POINTER(ct)) if a is not None else None


class CProblem:
    """ctypes view of a workloads.Problem; keeps the numpy buffers alive."""

    def __init__(self, prob, eps: float = 1e-5):
        f = lambda x: np.ascontiguousarray(np.asarray(x, dtype=np.float32).reshape(-1))
        self.keep = {
            "dyn": f(prob.dyn), "slo": f(prob.sample_lo), "shi": f(prob.sample_hi),
            "ulo": f(prob.u_lo), "uhi": f(prob.u_hi), "llo": f(prob.lim_lo), "lhi": f(prob.lim_hi),
            "wlo": f(prob.ws_lo), "whi": f(prob.ws_hi), "bc": f(prob.box_c), "bh": f(prob.box_h),
            "sc": f(prob.sph_c), "sr": f(prob.sph_r), "gc": f(prob.goal_c), "xi": f(prob.x_init),
        }
        k = self.keep
        fp = lambda a: _ptr(a, C.c_float)
        self.s = _Problem(
            system=prob.system, d=prob.d, m=prob.m, npos=prob.npos, dyn=fp(k["dyn"]),
            sample_lo=fp(k["slo"]), sample_hi=fp(k["shi"]), u_lo=fp(k["ulo"]), u_hi=fp(k["uhi"]),
            lim_lo=fp(k["llo"]), lim_hi=fp(k["lhi"]), vnorm_max=float(prob.vnorm_max),
            ws_lo=fp(k["wlo"]), ws_hi=fp(k["whi"]),
            n_box=int(prob.box_c.shape[0]), box_c=fp(k["bc"]), box_h=fp(k["bh"]),
            n_sph=int(prob.sph_r.shape[0]), sph_c=fp(k["sc"]), sph_r=fp(k["sr"]),
            goal_c=fp(k["gc"]), goal_r=float(prob.goal_r), x_init=fp(k["xi"]),
            B=prob.B, A=prob.A, T=prob.T, dt=float(prob.dt), n_cap=prob.n_cap,
            cost_kind=prob.cost_kind, h_kind=prob.h_kind, h_speed=float(prob.h_speed),
            c0=float(prob.c0), seed=int(prob.seed), qid=int(prob.qid),
            max_iters_per_round=int(prob.max_iters_per_round), eps=eps)
        self.prob = prob

    @property
    def ref(self):
        return C.byref(self.s)


# ---------------------------------------------------------------------------
# primitive wrappers
# ---------------------------------------------------------------------------

def philox(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint32))
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint32))
    out = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(_ptr(c, C.c_uint32), _ptr(k, C.c_uint32), _ptr(out, C.c_uint32))
    return out


def u32_to_range(x: int, lo: float, hi: float) -> np.float32:
    return np.float32(lib().orc_u32_to_range(int(x), float(lo), float(hi)))


def sample_state(cp: CProblem, k: int, it: int, rnd: int) -> np.ndarray:
    out = np.zeros(cp.prob.d, np.float32)
    lib().orc_sample_state(cp.ref, k, it, rnd, _ptr(out, C.c_float))
    return out


def sample_control(cp: CProblem, k: int, a: int, it: int, rnd: int) -> np.ndarray:
    out = np.zeros(cp.prob.m, np.float32)
    lib().orc_sample_control(cp.ref, k, a, it, rnd, _ptr(out, C.c_float))
    return out


def u32_to_range_n(x, lo: float, hi: float) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.uint32)
    out = np.zeros(x.size, np.float32)
    lib().orc_u32_to_range_n(_ptr(x, C.c_uint32), x.size, lo, hi, _ptr(out, C.c_float))
    return out


def _d(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def dynamics(cp: CProblem, x, u) -> np.ndarray:
    x, u = _d(x), _d(u)
    out = np.zeros(cp.prob.d)
    lib().orc_dynamics(cp.ref, _ptr(x, C.c_double), _ptr(u, C.c_double), _ptr(out, C.c_double))
    return out


def rk4_step(cp: CProblem, x, u, h: float) -> np.ndarray:
    x, u = _d(x), _d(u)
    out = np.zeros(cp.prob.d)
    lib().orc_rk4_step(cp.ref, _ptr(x, C.c_double), _ptr(u, C.c_double), h, _ptr(out, C.c_double))
    return out


def rollout(cp: CProblem, x0, u, T: int, h: float) -> np.ndarray:
    x0, u = _d(x0), _d(u)
    out = np.zeros((T + 1, cp.prob.d))
    lib().orc_rollout(cp.ref, _ptr(x0, C.c_double), _ptr(u, C.c_double), T, h,
                      _ptr(out, C.c_double))
    return out


def state_valid(cp: CProblem, x, eps: float = 1e-5):
    x = _d(x)
    near = C.c_int(0)
    margin = C.c_double(0)
    v = lib().orc_state_valid(cp.ref, _ptr(x, C.c_double), eps, C.byref(near), C.byref(margin))
    return bool(v), bool(near.value), margin.value


def edge(cp: CProblem, x0, c0: float, u):
    x0, u = _d(x0), _d(u)
    xT = np.zeros(cp.prob.d)
    cost = C.c_double(0)
    amb = C.c_int(0)
    v = lib().orc_edge(cp.ref, _ptr(x0, C.c_double), float(c0), _ptr(u, C.c_double),
                       _ptr(xT, C.c_double), C.byref(cost), C.byref(amb))
    return bool(v), xT, cost.value, bool(amb.value)


def heuristic(cp: CProblem, x) -> float:
    x = _d(x)
    return lib().orc_heuristic(cp.ref, _ptr(x, C.c_double))


def nearest(states, q):
    s = _d(states)
    n, d = s.shape
    q = _d(q)
    b1, b2 = C.c_double(0), C.c_double(0)
    i = lib().orc_nearest(_ptr(s, C.c_double), n, d, _ptr(q, C.c_double), C.byref(b1),
                          C.byref(b2))
    return i, b1.value, b2.value


# ---------------------------------------------------------------------------
# planner
# ---------------------------------------------------------------------------

class Report:
    """Arrays of one iteration's decisions, filled by OraclePlan.iterate."""

    def __init__(self, prob):
        K, B, d, m = prob.K, prob.B, prob.d, prob.m
        self.targets = np.zeros((K, d), np.float32)
        self.parents = np.zeros(K, np.int32)
        self.nn_d2 = np.zeros(K)
        self.nn_tie = np.zeros(K, np.int32)
        self.controls = np.zeros((B, m), np.float32)
        self.xnew = np.zeros((B, d))
        self.cnew = np.zeros(B)
        self.hval = np.zeros(B)
        self.flags = np.zeros(B, np.int32)
        self.amb = np.zeros(B, np.int32)
        self.slots = np.zeros(B, np.int32)
        self.s = _Report(
            targets=_ptr(self.targets, C.c_float), parents=_ptr(self.parents, C.c_int),
            nn_d2=_ptr(self.nn_d2, C.c_double), nn_tie=_ptr(self.nn_tie, C.c_int),
            controls=_ptr(self.controls, C.c_float), xnew=_ptr(self.xnew, C.c_double),
            cnew=_ptr(self.cnew, C.c_double), hval=_ptr(self.hval, C.c_double),
            flags=_ptr(self.flags, C.c_int), amb=_ptr(self.amb, C.c_int),
            slots=_ptr(self.slots, C.c_int))

    def __getattr__(self, name):
        s = self.__dict__.get("s")
        if s is not None and name in {f[0] for f in _Report._fields_}:
            return getattr(s, name)
        raise AttributeError(name)


class OraclePlan:
    def __init__(self, prob, eps: float = 1e-5):
        self.cp = CProblem(prob, eps)
        self.prob = prob
        self.h = lib().orc_plan_create(self.cp.ref)

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            lib().orc_plan_destroy(h)
            self.h = None

    def iterate(self, steer: Optional[dict] = None, report: bool = True):
        rep = Report(self.prob) if report else None
        st = None
        keep = []
        if steer is not None:
            par = steer.get("parents")
            fl = steer.get("flags")
            par = None if par is None else np.ascontiguousarray(par, dtype=np.int32)
            fl = None if fl is None else np.ascontiguousarray(fl, dtype=np.int32)
            keep = [par, fl]
            st = _Steer(parents=_ptr(par, C.c_int), flags=_ptr(fl, C.c_int),
                        goal_j=int(steer.get("goal_j", -1)))
        end = lib().orc_plan_iterate(self.h, C.byref(st) if st is not None else None,
                                     C.byref(rep.s) if rep is not None else None)
        del keep
        if rep is not None:
            rep.end = end
        return rep if rep is not None else end

    def run(self, max_rounds: int = 0, max_iters: int = 0) -> int:
        return lib().orc_plan_run(self.h, max_rounds, max_iters)

    def state(self) -> dict:
        s = _State()
        lib().orc_plan_get(self.h, C.byref(s))
        return {f[0]: getattr(s, f[0]) for f in _State._fields_}

    def tree(self):
        st = self.state()
        n, d, m = st["n"], self.prob.d, self.prob.m
        states = np.zeros((n, d))
        actions = np.zeros((n, m))
        parents = np.zeros(n, np.int32)
        costs = np.zeros(n)
        lib().orc_plan_tree(self.h, _ptr(states, C.c_double), _ptr(actions, C.c_double),
                            _ptr(parents, C.c_int), _ptr(costs, C.c_double), n)
        return states, actions, parents, costs

    def load_tree(self, states, actions, parents, costs, rnd: int, it: int, c_best: float):
        states = np.ascontiguousarray(states, dtype=np.float32)
        n = states.shape[0]
        actions = None if actions is None else np.ascontiguousarray(actions, dtype=np.float32)
        parents = None if parents is None else np.ascontiguousarray(parents, dtype=np.int32)
        costs = np.ascontiguousarray(costs, dtype=np.float32)
        rc = lib().orc_plan_load_tree(self.h, _ptr(states, C.c_float), _ptr(actions, C.c_float),
                                      _ptr(parents, C.c_int), _ptr(costs, C.c_float), n, rnd, it,
                                      float(c_best))
        if rc != 0:
            raise ValueError("load_tree: bad size")

    def solutions(self):
        n = lib().orc_plan_solutions(self.h, None, 0)
        arr = (_Solution * max(n, 1))()
        lib().orc_plan_solutions(self.h, arr, n)
        return [{f[0]: getattr(arr[i], f[0]) for f in _Solution._fields_} for i in range(n)]

    def best_path(self):
        ne = C.c_int(0)
        cost = C.c_double(0)
        rc = lib().orc_plan_best_path(self.h, None, None, 0, C.byref(ne), C.byref(cost))
        if rc == -1:
            return None
        n = ne.value
        states = np.zeros((n + 1, self.prob.d))
        actions = np.zeros((max(n, 1), self.prob.m))
        lib().orc_plan_best_path(self.h, _ptr(states, C.c_double), _ptr(actions, C.c_double), n,
                                 C.byref(ne), C.byref(cost))
        return states, actions[:n], cost.value


# ---------------------------------------------------------------------------
# trajectory refinement objective (complex-step gradient)
# ---------------------------------------------------------------------------

def refine_params(w_u, w_g, w_c, beta, delta, u_ref, u_scale):
    r = _Refine(w_u=w_u, w_g=w_g, w_c=w_c, beta=beta, delta=delta)
    for i in range(len(u_ref)):
        r.u_ref[i] = float(u_ref[i])
        r.u_scale[i] = float(u_scale[i])
    for i in range(len(u_ref), 4):
        r.u_scale[i] = 1.0
    return r


def traj_cost(cp: CProblem, rp, x0, U) -> float:
    x0, U = _d(x0), _d(U)
    M = U.shape[0]
    return lib().orc_traj_cost(cp.ref, C.byref(rp), _ptr(x0, C.c_double), _ptr(U, C.c_double), M)


def traj_grad(cp: CProblem, rp, x0, U) -> np.ndarray:
    x0, U = _d(x0), _d(U)
    M = U.shape[0]
    g = np.zeros_like(U)
    lib().orc_traj_grad(cp.ref, C.byref(rp), _ptr(x0, C.c_double), _ptr(U, C.c_double), M,
                        _ptr(g, C.c_double))
    return g
