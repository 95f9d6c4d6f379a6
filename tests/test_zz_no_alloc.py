"""pakr_refine_paths_static (work buffers in the library's static per-GPU
array, nothing allocated by the call) against pakr_refine_paths (caller
workspace): the same refined controls and J, bit for bit, on two calls in a
row -- the second with fewer and shorter paths, so it runs on what the first
left in the array -- and a size beyond the array is refused before any launch.
"""
import numpy as np
import pytest

from paper_2607_03987_amd import pakr, refine, workloads as W

pytestmark = pytest.mark.gpu


def _inputs(prob, n, M, seed):
    rng = np.random.default_rng(seed)
    lo = np.asarray(prob.u_lo, np.float64)[:prob.m]
    hi = np.asarray(prob.u_hi, np.float64)[:prob.m]
    U = lo + (hi - lo) * rng.uniform(0.2, 0.8, (n, M, prob.m))
    x0 = np.repeat(np.asarray(prob.x_init, np.float32)[None], n, 0)
    return x0, U.astype(np.float32)


@pytest.mark.parametrize("cfg", ["c4", "c3"])
def test_static_refinement_equals_workspace_refinement(cfg):
    import torch

    prob = W.CONFIGS[cfg](seed=1)
    rs = W.refine_settings(prob)
    ref = refine.Refiner(prob, rs)
    for (n, M, seed) in [(24, 6, 0), (5, 3, 1)]:
        print(f"{prob.name}: {n} paths of {M} edges", flush=True)
        x0, U = _inputs(prob, n, M, seed)
        x0_t = torch.from_numpy(x0).cuda()
        U_t = torch.from_numpy(U).cuda()
        want = refine.refine_path(ref, x0_t, U_t, steps=12)
        U_s = U_t.clone()
        J0, J1 = refine.refine_controls_static(ref, x0_t, U_s, steps=12)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(U_s.cpu().numpy(), want["U_refined"].cpu().numpy())
        np.testing.assert_array_equal(J0.cpu().numpy(), want["J_before"].cpu().numpy())
        np.testing.assert_array_equal(J1.cpu().numpy(), want["J_after"].cpu().numpy())
        # the refinement did something and J never increased
        assert (J1 <= J0).all() and (J1 < J0).any()
    ref.close()


def test_static_refinement_refuses_sizes_beyond_the_array():
    import torch

    prob = W.config_c4(seed=1)
    ref = refine.Refiner(prob, W.refine_settings(prob))
    n, M = 4096, 40  # checkpoints alone: 4096 * (40 * 40 + 1) * 12 floats
    assert pakr.load().pakr_refine_workspace_size(ref.h, n, M) > refine.REFINE_STATIC_BYTES
    x0 = torch.zeros(n, prob.d, device="cuda")
    U = torch.zeros(n, M, prob.m, device="cuda")
    with pytest.raises(pakr.PakrError) as e:
        refine.refine_controls_static(ref, x0, U, steps=1)
    assert e.value.code == -4  # PAKR_E_WORKSPACE_TOO_SMALL
    ref.close()
