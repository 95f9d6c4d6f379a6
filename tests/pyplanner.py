"""A second, deliberately naive transcription of Alg. 1 for tiny double-integrator
problems, used only to cross-check the C reference.  It takes the random draws
from the reference's (separately pinned) sampling functions and writes every
other step out again in numpy: RK4, clamp-to-box collision, arg-min NN,
insertion in candidate order, goal selection and the AO-x round logic.
"""
import math

import numpy as np

import oracle


def _f(x, u, D):
    return np.concatenate([x[D:], u])


def _rk4(x, u, h, D):
    k1 = _f(x, u, D)
    k2 = _f(x + h / 2 * k1, u, D)
    k3 = _f(x + h / 2 * k2, u, D)
    k4 = _f(x + h * k3, u, D)
    return x + h / 6 * (k1 + 2 * k2 + 2 * k3 + k4)


def _valid(p, x, D):
    pos = x[:D]
    if np.any(pos < p.ws_lo) or np.any(pos > p.ws_hi):
        return False
    if p.vnorm_max > 0 and np.linalg.norm(x[D:]) > p.vnorm_max:
        return False
    for c, h in zip(p.box_c.astype(float), p.box_h.astype(float)):
        q = np.clip(pos, c - h, c + h)
        if np.linalg.norm(pos - q) == 0.0:
            return False
    for c, r in zip(p.sph_c.astype(float), p.sph_r.astype(float)):
        if np.linalg.norm(pos - c) <= r:
            return False
    return True


class PyPlanner:
    def __init__(self, prob):
        assert prob.system in (0, 1)
        self.p = prob
        self.cp = oracle.CProblem(prob)
        self.D = prob.npos
        self.c_best = prob.c0
        self.round = 0
        self.solutions = []
        self._new_round()

    def _new_round(self):
        p = self.p
        self.X = [p.x_init.astype(float)]
        self.U = [np.zeros(p.m)]
        self.P = [-1]
        self.C = [0.0]
        self.iter = 0

    def _h(self, x):
        p = self.p
        dist = float(np.linalg.norm(x[:self.D] - p.goal_c.astype(float)))
        gap = max(0.0, dist - float(p.goal_r))
        return gap / float(p.h_speed) if p.cost_kind == 0 else gap

    def step(self):
        p, D = self.p, self.D
        K = p.B // p.A
        h = float(p.dt)
        X = np.array(self.X)
        cands = []
        for k in range(K):
            q = oracle.sample_state(self.cp, k, self.iter, self.round).astype(float)
            par = int(np.argmin(((X - q) ** 2).sum(axis=1)))
            for a in range(p.A):
                u = oracle.sample_control(self.cp, k, a, self.iter, self.round).astype(float)
                x = X[par].copy()
                ok = True
                length = 0.0
                for _ in range(p.T):
                    xn = _rk4(x, u, h, D)
                    length += float(np.linalg.norm(xn[:D] - x[:D]))
                    ok = ok and _valid(p, xn, D)
                    x = xn
                edge = p.T * h if p.cost_kind == 0 else length
                c = self.C[par] + edge
                keep = ok and (c + self._h(x) < self.c_best)
                goal = float(np.linalg.norm(x[:D] - p.goal_c.astype(float))) <= float(p.goal_r)
                cands.append((keep, goal, x, u, par, c))
        best = None
        for j, (keep, goal, x, u, par, c) in enumerate(cands):
            if not keep or len(self.X) >= p.n_cap:
                continue
            self.X.append(x)
            self.U.append(u)
            self.P.append(par)
            self.C.append(c)
            if goal and (best is None or c < best[1]):
                best = (len(self.X) - 1, c)
        if best is not None:
            self.c_best = best[1]
            self.solutions.append((self.round, self.iter, best[0], best[1]))
            self.round += 1
            self._new_round()
            return "goal"
        if len(self.X) >= p.n_cap:
            self.round += 1
            self._new_round()
            return "full"
        if self.iter + 1 >= p.max_iters_per_round:
            self.round += 1
            self._new_round()
            return "cap"
        self.iter += 1
        return None
