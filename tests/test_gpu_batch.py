"""GPU tests of the batched form: every problem of a batch computes what the
plain single-problem context computes (bit for bit with the same launch
shape), graph replays equal eager calls, the autotuner picks a valid shape,
and the closed-loop plant integrates Eq. 7 (marked gpu)."""
import numpy as np
import pytest

from paper_2104_13542_amd import inputs

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2104_13542_amd import storm

    storm.lib()


def _problems(n, seed0=0):
    out = []
    for p in range(n):
        pr = inputs.config3_problem(seed0 + p)
        # keep the test small: cut N, keep the uneven H and obstacle counts
        pr.params.n_particles = 40 + 37 * p
        pr.params.n_halton = pr.params.n_particles // 2
        pr.params.n_null = p % 3
        out.append(pr)
    return out


def _goals(problems):
    g = []
    for k, pr in enumerate(problems):
        g.append([1, 0, 0, 0, -1, 0, 0, 0, -1, 0.4 + 0.02 * k, 0.1 - 0.03 * k, 0.45])
    return torch.tensor(g, dtype=torch.float32, device="cuda")


@pytest.mark.parametrize("waves,cost_order,exact", [(16, 1, True), (16, 0, True), (8, 1, False)])
def test_batch_matches_plain(waves, cost_order, exact):
    from paper_2104_13542_amd import storm

    probs = _problems(6)
    goals = _goals(probs)
    b = storm.Batch(probs)
    b.set_config(waves, 97, cost_order)
    plains = [storm.Rollout(pr) for pr in probs]
    try:
        for step in range(3):
            b.step(goals)
            cmd_b = b.update(shift=True)
            cmds = []
            Cs = []
            for k, r in enumerate(plains):
                out = r.step(goals[k])
                c, _, _ = r.update(shift=True)
                cmds.append(c.clone())
                Cs.append(out["C"].cpu().numpy())
            torch.cuda.synchronize()
            for k in range(len(probs)):
                Cb = b.costs(k)
                mb, sb, stb = b.get_state(k)
                mp, sp, stp = plains[k].get_state()
                assert stb == stp == step + 1
                if exact:
                    assert np.array_equal(Cb, Cs[k]), (step, k)
                    assert np.array_equal(mb, mp) and np.array_equal(sb, sp)
                    assert torch.equal(cmd_b[k], cmds[k])
                else:
                    np.testing.assert_allclose(Cb, Cs[k], rtol=2e-6, atol=1e-5)
    finally:
        b.close()
        for r in plains:
            r.close()


def test_batch_graph_replays_match_eager():
    from paper_2104_13542_amd import storm

    probs = _problems(5, seed0=10)
    goals = _goals(probs)
    eager = storm.Batch(probs)
    graphed = storm.Batch(probs)
    try:
        x0 = graphed.x0.clone()
        cmd = torch.zeros((len(probs), 7), dtype=torch.float32, device="cuda")
        g = graphed.graph(x0, goals, cmd, iterations=1, shift=True)
        for rep in range(4):
            eager.step(goals, x0=x0)
            ce = eager.update(shift=True)
            g.launch()
            torch.cuda.synchronize()
            assert torch.equal(ce, cmd), rep
            for k in range(len(probs)):
                assert np.array_equal(eager.costs(k), graphed.costs(k))
            # the closed loop moves the shared state between replays
            storm.plant_step(x0, cmd, 0.01)
            torch.cuda.synchronize()
        g.close()
    finally:
        eager.close()
        graphed.close()


def test_batch_autotune_picks_valid_shape():
    from paper_2104_13542_amd import storm

    probs = _problems(4, seed0=20)
    goals = _goals(probs)
    b = storm.Batch(probs)
    try:
        best, times = b.autotune(goals, reps=2)
        assert best["waves"] in (8, 16) and best["grid"] >= 1
        assert len(times) == 16 and np.all(times > 0)
        assert b.config() == best
        # after tuning the batch still steps and updates
        b.step(goals)
        b.update()
        torch.cuda.synchronize()
        with pytest.raises(storm.StormError):
            b.update()
    finally:
        b.close()


def test_plant_step_closed_form():
    from paper_2104_13542_amd import storm

    rng = np.random.default_rng(3)
    x = rng.normal(size=(9, 3, 7)).astype(np.float32)
    u = rng.normal(size=(9, 7)).astype(np.float32)
    xt = torch.tensor(x, device="cuda")
    storm.plant_step(xt, torch.tensor(u, device="cuda"), 0.01)
    got = xt.cpu().numpy()
    v = x[:, 1] + 0.01 * u
    np.testing.assert_allclose(got[:, 1], v, rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(got[:, 0], x[:, 0] + 0.01 * v, rtol=1e-6, atol=1e-7)
    np.testing.assert_array_equal(got[:, 2], u)


def _refine_problems(n):
    probs = _problems(n, seed0=20)
    for pr in probs:
        pr.params.grad_mask = inputs.COST_POSE | inputs.COST_JOINT
    return probs


def test_batch_refine_matches_plain():
    """One batched adjoint launch per Adam step gives every problem the
    refinement its plain context computes (bit for bit at 16 waves)."""
    from paper_2104_13542_amd import storm

    probs = _refine_problems(5)
    goals = _goals(probs)
    b = storm.Batch(probs)
    b.set_config(16, 64, 1)
    plains = [storm.Rollout(pr) for pr in probs]
    try:
        for step in range(2):
            b.step(goals)
            b.update(shift=False)
            cmd_b = b.refine(goals, iterations=3, lr=0.05, shift=True).clone()
            cmds = []
            for k, r in enumerate(plains):
                r.step(goals[k])
                r.update(shift=False)
                cmds.append(r.refine(goals[k], iterations=3, lr=0.05, shift=True).clone())
            torch.cuda.synchronize()
            for k in range(len(probs)):
                mb, sb, _ = b.get_state(k)
                mp, sp, _ = plains[k].get_state()
                assert np.array_equal(mb, mp) and np.array_equal(sb, sp), (step, k)
                assert torch.equal(cmd_b[k], cmds[k]), (step, k)
    finally:
        b.close()
        for r in plains:
            r.close()


def test_batch_refine_graph_replays_match_eager():
    from paper_2104_13542_amd import storm

    probs = _refine_problems(4)
    goals = _goals(probs)
    eager = storm.Batch(probs)
    graphed = storm.Batch(probs)
    try:
        eager.set_config(16, 64, 1)
        graphed.set_config(16, 64, 1)
        cmd_g = torch.zeros((len(probs), 7), device="cuda")
        x0 = graphed.x0.clone()
        g = graphed.graph(x0, goals, cmd_g, iterations=1, shift=True, refine_iters=3, lr=0.05)
        for rep in range(3):
            eager.step(goals)
            eager.update(shift=False)
            cmd_e = eager.refine(goals, iterations=3, lr=0.05, shift=True).clone()
            g.launch()
            torch.cuda.synchronize()
            assert torch.equal(cmd_e, cmd_g), rep
            for k in range(len(probs)):
                assert np.array_equal(eager.get_state(k)[0], graphed.get_state(k)[0]), (rep, k)
        g.close()
    finally:
        eager.close()
        graphed.close()


def test_batch_refine_rejects_collision_gradients():
    from paper_2104_13542_amd import storm

    probs = _problems(2)  # every cost term, grad_mask 0
    b = storm.Batch(probs)
    try:
        with pytest.raises(storm.StormError) as e:
            b.refine(_goals(probs))
        assert e.value.code == storm.STORM_E_UNSUPPORTED
    finally:
        b.close()
