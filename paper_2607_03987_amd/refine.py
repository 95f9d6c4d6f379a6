"""Trajectory refinement through libpakr's hand-written RK4 adjoint.

A path found by the planner (a start state and M piecewise-constant controls,
each held for one edge of T RK4 steps, as Sec. IV-A builds edges) is improved
by gradient steps on a smooth objective: control effort, a terminal goal
term and a softplus obstacle/bound penalty summed over every sub-step state.
The rollout, its adjoint, the optimizer step and the final hard check all run
in libpakr kernels (``pakr_rollout_fwd``, ``pakr_rollout_bwd``,
``pakr_refine_step``, ``pakr_check_path``); this module marshals arguments.

``RolloutFn`` exposes the rollout as a ``torch.autograd.Function`` (forward
stores the per-step checkpoints, backward runs the adjoint from them), so the
objective composes with torch code; ``refine_path`` calls the library's own
refinement loop (``pakr_refine_paths``): Adam steps in controls normalised
by the control box, each kept only if it lowers J, with a per-path step size
that halves after a rejected trial.
"""
from __future__ import annotations

import ctypes as C
import math

from . import pakr, workloads as W


def _rcheck(rc: int, handle=None):
    if rc != pakr.PAKR_OK:
        msg = pakr.load().pakr_refiner_last_error(handle)
        raise pakr.PakrError(rc, msg.decode() if msg else "")


def c_refine_params(rs: W.RefineSettings) -> pakr.RefineParams:
    rp = pakr.RefineParams()
    rp.w_effort, rp.w_goal, rp.w_collision = rs.w_u, rs.w_g, rs.w_c
    rp.beta, rp.delta = rs.beta, rs.delta
    for c in range(pakr.MAX_M):
        rp.u_ref[c] = rs.u_ref[c] if c < len(rs.u_ref) else 0.0
        rp.u_scale[c] = rs.u_scale[c] if c < len(rs.u_scale) else 1.0
    return rp


class Refiner:
    """One scene's refinement context on the current GPU and torch stream."""

    def __init__(self, prob: W.Problem, settings: W.RefineSettings | None = None, device=None):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("libpakr needs a ROCm GPU; none is visible")
        self.torch = torch
        self.prob = prob
        self.settings = settings or W.refine_settings(prob)
        self.q = pakr.CQuery(prob)
        self.rp = c_refine_params(self.settings)
        self.device = torch.device(device or "cuda")
        self.stream = torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        rc = pakr.load().pakr_refiner_init(C.byref(self.q.system), C.byref(self.q.scene),
                                           C.byref(self.q.goal), C.byref(self.q.params),
                                           C.byref(self.rp), C.c_void_p(self.stream.cuda_stream),
                                           C.byref(h))
        _rcheck(rc, None)
        self.h = h.value
        self.d, self.m = prob.d, prob.m

    def close(self):
        h = getattr(self, "h", None)
        if h:
            pakr.load().pakr_refiner_destroy(h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_settings(self, settings: W.RefineSettings):
        rp = c_refine_params(settings)
        _rcheck(pakr.load().pakr_refiner_set_params(self.h, C.byref(rp)), self.h)
        self.settings, self.rp = settings, rp

    def _f32(self, t, shape):
        t = t.to(device=self.device, dtype=self.torch.float32).contiguous()
        if tuple(t.shape) != tuple(shape):
            raise ValueError(f"expected shape {tuple(shape)}, got {tuple(t.shape)}")
        return t

    def ckpt_bytes(self, n: int, M: int) -> int:
        return int(pakr.load().pakr_rollout_ckpt_bytes(self.h, n, M))

    def forward(self, x0, U):
        """J [n] and the checkpoints x_0..x_N [n][M*T+1][d] of U [n][M][m]."""
        n, M = int(U.shape[0]), int(U.shape[1])
        U = self._f32(U, (n, M, self.m))
        x0 = self._f32(x0, (n, self.d))
        T = self.prob.T
        ckpt = self.torch.empty((n, M * T + 1, self.d), dtype=self.torch.float32,
                                device=self.device)
        J = self.torch.empty(n, dtype=self.torch.float32, device=self.device)
        rc = pakr.load().pakr_rollout_fwd(self.h, n, M, x0.data_ptr(), U.data_ptr(),
                                          ckpt.data_ptr(), ckpt.numel() * 4, J.data_ptr())
        _rcheck(rc, self.h)
        return J, ckpt

    def backward(self, U, ckpt, gJ):
        """gU [n][M][m] = gJ * dJ/dU from the checkpoints of forward(x0, U)."""
        n, M = int(U.shape[0]), int(U.shape[1])
        U = self._f32(U, (n, M, self.m))
        ckpt = self._f32(ckpt, (n, M * self.prob.T + 1, self.d))
        gJ = self._f32(gJ, (n,))
        gU = self.torch.empty_like(U)
        rc = pakr.load().pakr_rollout_bwd(self.h, n, M, U.data_ptr(), ckpt.data_ptr(),
                                          ckpt.numel() * 4, gJ.data_ptr(), gU.data_ptr())
        _rcheck(rc, self.h)
        return gU

    def step(self, U, gU, m1, m2, step: int, lr: float):
        """In-place projected Adam step on U (all float32, contiguous, on the device)."""
        n, M = int(U.shape[0]), int(U.shape[1])
        for t in (U, gU, m1, m2):
            if not (t.is_contiguous() and t.dtype == self.torch.float32 and t.numel() == n * M * self.m):
                raise ValueError("U, gU, m1, m2 must be contiguous float32 [n][M][m]")
        rc = pakr.load().pakr_refine_step(self.h, n, M, U.data_ptr(), gU.data_ptr(), m1.data_ptr(),
                                          m2.data_ptr(), int(step), float(lr))
        _rcheck(rc, self.h)

    def check(self, x0, U):
        """(ok [n] int32: bit 0 valid, bit 1 in goal; cost [n]) -- the planner's test."""
        n, M = int(U.shape[0]), int(U.shape[1])
        U = self._f32(U, (n, M, self.m))
        x0 = self._f32(x0, (n, self.d))
        ok = self.torch.empty(n, dtype=self.torch.int32, device=self.device)
        cost = self.torch.empty(n, dtype=self.torch.float32, device=self.device)
        rc = pakr.load().pakr_check_path(self.h, n, M, x0.data_ptr(), U.data_ptr(), ok.data_ptr(),
                                         cost.data_ptr())
        _rcheck(rc, self.h)
        return ok, cost


def _rollout_fn():
    import torch

    class RolloutFn(torch.autograd.Function):
        """J(U) of n trajectories; backward is libpakr's RK4 adjoint."""

        @staticmethod
        def forward(ctx, U, x0, refiner):
            J, ckpt = refiner.forward(x0, U)
            ctx.save_for_backward(U.detach().to(torch.float32).contiguous(), ckpt)
            ctx.refiner = refiner
            return J

        @staticmethod
        def backward(ctx, gJ):
            U, ckpt = ctx.saved_tensors
            gU = ctx.refiner.backward(U, ckpt, gJ)
            return gU, None, None

    return RolloutFn


_FN = None


def rollout_cost(refiner: Refiner, x0, U):
    """Differentiable J [n] of controls U [n][M][m] from starts x0 [n][d]."""
    global _FN
    if _FN is None:
        _FN = _rollout_fn()
    return _FN.apply(U, x0, refiner)


def refine_path(refiner: Refiner, x0, U, steps: int | None = None, lr: float | None = None,
                cost_bound: float = math.inf):
    """Refine n paths: `steps` safeguarded Adam iterations (pakr_refine_paths).

    x0 [n][d], U [n][M][m] (not modified).  Returns a dict with the refined
    controls, J before and after (J never increases), and the planner's hard
    check of the refined paths; a refined path is accepted when every
    sub-step is valid, its final state is in the goal ball and its cost does
    not exceed cost_bound.  Rejected paths keep their original controls in
    ``U_out``.
    """
    torch = refiner.torch
    s = refiner.settings
    steps = s.steps if steps is None else int(steps)
    lr = s.lr if lr is None else float(lr)
    n, M = int(U.shape[0]), int(U.shape[1])
    x0 = refiner._f32(x0, (n, refiner.d))
    U0 = refiner._f32(U, (n, M, refiner.m))
    Uw = U0.clone()
    nbytes = int(pakr.load().pakr_refine_workspace_size(refiner.h, n, M))
    if nbytes == 0:
        raise pakr.PakrError(-1, "pakr_refine_workspace_size rejected the sizes")
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=refiner.device)
    ws_ptr = (ws.data_ptr() + 255) & ~255
    J0 = torch.empty(n, dtype=torch.float32, device=refiner.device)
    J1 = torch.empty_like(J0)
    rc = pakr.load().pakr_refine_paths(refiner.h, n, M, x0.data_ptr(), Uw.data_ptr(), steps, lr,
                                       ws_ptr, nbytes, J0.data_ptr(), J1.data_ptr())
    _rcheck(rc, refiner.h)
    ok, cost = refiner.check(x0, Uw)
    accepted = (ok == 3) & (cost <= cost_bound)
    U_out = torch.where(accepted[:, None, None], Uw, U0)
    return dict(U_refined=Uw, U_out=U_out, J_before=J0, J_after=J1, ok=ok, cost=cost,
                accepted=accepted, workspace=ws)


REFINE_STATIC_BYTES = 16 << 20  # PAKR_REFINE_STATIC_BYTES


def refine_controls_static(refiner: Refiner, x0, U, steps: int | None = None,
                           lr: float | None = None):
    """pakr_refine_paths_static: the refinement loop of `refine_path` with its
    work buffers in the library's static per-GPU array (no workspace is
    allocated by the call).  U [n][M][m] is refined in place; returns
    (J_before, J_after).  Calls on one GPU share the array: do not overlap
    them."""
    torch = refiner.torch
    s = refiner.settings
    steps = s.steps if steps is None else int(steps)
    lr = s.lr if lr is None else float(lr)
    n, M = int(U.shape[0]), int(U.shape[1])
    dev = refiner.device.index if refiner.device.index is not None else torch.cuda.current_device()
    if not (U.is_cuda and U.get_device() == dev and U.is_contiguous() and
            U.dtype == torch.float32):
        raise ValueError("U must be a contiguous float32 tensor on the refiner's device")
    x0 = refiner._f32(x0, (n, refiner.d))
    J0 = torch.empty(n, dtype=torch.float32, device=refiner.device)
    J1 = torch.empty_like(J0)
    rc = pakr.load().pakr_refine_paths_static(refiner.h, n, M, x0.data_ptr(), U.data_ptr(),
                                              steps, lr, J0.data_ptr(), J1.data_ptr())
    _rcheck(rc, refiner.h)
    return J0, J1
