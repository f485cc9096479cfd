"""storm_rollout_grad_noalloc (the adjoint with its partials in the
library's static per-device scratch, for callers that cannot allocate)
against storm_rollout_grad on the same context and inputs, through the C ABI:
two calls in a row, the second on a smaller context (marked gpu)."""
import numpy as np
import pytest

from paper_2104_13542_amd import inputs

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _case(N, H, seed):
    prob = inputs.config4(seed)
    prob.params.n_particles = N
    prob.params.horizon = H
    prob.params.dt = np.full(H, 0.02)
    prob.params.n_null = 1
    return prob


def _grad(storm, fn, r, mean, goal, noise):
    g = torch.full((r.H, 7), float("nan"), dtype=torch.float32, device="cuda")
    J = torch.full((1,), float("nan"), dtype=torch.float32, device="cuda")
    rc = fn(r._h, storm._ptr(r.x0), storm._ptr(goal), storm._ptr(mean), storm._ptr(noise), storm._ptr(g),
            storm._ptr(J), storm._stream())
    assert rc == 0, storm.status_str(rc)
    torch.cuda.synchronize()
    return g.cpu().numpy(), J.cpu().numpy()


def test_grad_noalloc_matches_grad():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2104_13542_amd import storm

    L = storm.lib()
    # a full-size context first, then a smaller one: the second call must not
    # see the first call's partials
    for N, H, seed in ((1024, 30, 3), (37, 16, 4)):
        prob = _case(N, H, seed)
        r = storm.Rollout(prob)
        try:
            rng = np.random.default_rng(seed)
            mean = torch.tensor(rng.normal(size=(H, 7)) * 0.5, dtype=torch.float32, device="cuda")
            noise = torch.tensor(rng.standard_normal((7, N, H)), dtype=torch.float32, device="cuda")
            goal = torch.tensor([1, 0, 0, 0, -1, 0, 0, 0, -1, 0.45, 0.05, 0.4], dtype=torch.float32,
                                device="cuda")
            g_ref, J_ref = _grad(storm, L.storm_rollout_grad, r, mean, goal, noise)
            g_na, J_na = _grad(storm, L.storm_rollout_grad_noalloc, r, mean, goal, noise)
            assert np.all(np.isfinite(g_ref)) and np.isfinite(J_ref[0])
            np.testing.assert_array_equal(g_na, g_ref)
            np.testing.assert_array_equal(J_na, J_ref)
            # and again after the other entry point ran on the same context
            g_na2, J_na2 = _grad(storm, L.storm_rollout_grad_noalloc, r, mean, goal, noise)
            np.testing.assert_array_equal(g_na2, g_ref)
        finally:
            r.close()
