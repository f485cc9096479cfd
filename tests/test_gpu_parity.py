"""GPU parity of the HIP path against the FP64 oracle (marked gpu).

Every test calls the C ABI through the ctypes binding and compares element by
element with the oracle on the same seeded inputs: states to 1e-5, running and
horizon costs to 1e-4 relative, the updated mean to 1e-4."""
import numpy as np
import pytest

from paper_2104_13542_amd import inputs
from tests.gpu_common import (COST_FLOOR, TOL_COST_REL, TOL_MEAN, TOL_STATE, assert_states, cost_error, f32,
                              manip_values, run_pair, to_nhj)

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2104_13542_amd import storm

    storm.lib()


def _update_bound(ro, up, gC, beta):
    """First-order bound of the updated-mean error caused by the horizon-cost
    error dC: |d mu'_hj| <= (1/beta) sum_i w_i |u_ihj - mu'_hj| |dC_i - dC_w|
    with dC_w the weighted mean of dC (a common shift of all C changes
    nothing)."""
    w = up["w"]
    dC = gC - ro["C"]
    dCc = dC - np.sum(w * dC)
    dev = np.abs(ro["u"] - up["mean"][None])
    return np.sum(w[:, None, None] * dev * np.abs(dCc)[:, None, None], axis=0) / beta


def test_fk_parity(oracle_lib):
    from paper_2104_13542_amd import storm

    rng = np.random.default_rng(0)
    n = 777
    q = f32(np.stack([inputs.random_q(rng) for _ in range(n)]))
    pose, manip = storm.fk(torch.tensor(q, dtype=torch.float32, device="cuda"))
    pose = pose.cpu().double().numpy()
    manip = manip.cpu().double().numpy()
    dh = f32(inputs.PANDA_DH)
    # m = sqrt(det A), A = J J^T (6 x 6, symmetric positive definite), from
    # FP32 frames, products and L D L^T.  A relative perturbation g of A
    # moves log det A by at most 6 g kappa (Weyl: |d lambda_i| <= g
    # lambda_max, divided by lambda_i >= lambda_min), so |dm| / m <=
    # 3 g kappa to first order, kappa = lambda_max / lambda_min: the error
    # scales with m kappa, not with 1 / m.  The FP32 path's worst case over
    # these configurations is 0.06 x 2^-24 kappa m beyond a 2e-6 floor (the
    # rounding of m itself); the limit is 0.5 x 2^-24 kappa m + 2e-6.
    worst = 0.0
    for k in range(n):
        T = oracle_lib.fk(dh, q[k])
        ref = np.concatenate([T[7][:3, :3].reshape(-1), T[7][:3, 3]])
        assert np.max(np.abs(pose[k] - ref)) < 2e-6
        J = oracle_lib.jacobian(T)
        m = oracle_lib.manipulability(J)
        ev = np.linalg.eigvalsh(J @ J.T)
        kappa = ev[-1] / ev[0]
        dm = abs(manip[k] - m)
        worst = max(worst, max(dm - 2e-6, 0.0) / (2.0 ** -24 * kappa * m))
        assert dm <= 0.5 * 2.0 ** -24 * kappa * m + 2e-6, (k, m, kappa, dm)
    print("largest |dm| / (2^-24 kappa m) beyond 2e-6: %.3g (limit 0.5)" % worst)
    # empty batch is a no-op
    storm.fk(torch.zeros((0, 7), device="cuda"))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_config1_noise_override(oracle_lib, seed):
    prob = inputs.config1(seed)
    p = prob.params
    eps = inputs.standard_normal(100 + seed, (p.n_particles, p.horizon, 7))
    g, ro, up, o, _ = run_pair(prob, oracle_lib, noise_nhj=eps)
    assert_states(g, ro)
    assert np.max(cost_error(g["c"], ro["c"])) <= TOL_COST_REL
    assert np.max(cost_error(g["C"], ro["C"])) <= TOL_COST_REL
    np.testing.assert_allclose(g["terms"][..., :3], ro["terms"][..., :3], rtol=1e-4, atol=2e-6)
    # decoupled update: the oracle's update on the GPU's horizon costs and controls
    upd = o.update(g["C"], g["u"], np.zeros((p.horizon, 7)), f32(np.asarray(p.sigma_init) ** 2))
    assert np.max(np.abs(g["mean"] - upd["mean"])) <= TOL_MEAN
    assert np.max(np.abs(g["sigma2"] - upd["sigma2"])) <= 1e-4 * np.max(upd["sigma2"])
    np.testing.assert_allclose(g["cmd"], upd["cmd"], atol=TOL_MEAN)
    # end to end, within 1e-4 plus the propagated cost rounding
    bound = _update_bound(ro, up, g["C"], p.beta)
    assert np.all(np.abs(g["mean"] - up["mean"]) <= TOL_MEAN + 2.0 * bound)
    # stored state: shifted mean, new variance, step counter advanced
    mean_s, sig_s, step = g["state_after"]
    np.testing.assert_allclose(mean_s[:-1], g["mean"][1:], atol=0)
    assert np.all(mean_s[-1] == 0)
    np.testing.assert_allclose(sig_s, g["sigma2"], atol=0)
    assert step == 1


@pytest.mark.parametrize("seed", [0, 3])
def test_config1_philox_noise(oracle_lib, seed):
    prob = inputs.config1(seed, v0_random=True)
    g, ro, up, o, eps = run_pair(prob, oracle_lib)
    assert_states(g, ro)
    assert np.max(cost_error(g["c"], ro["c"])) <= TOL_COST_REL
    assert np.max(cost_error(g["C"], ro["C"])) <= TOL_COST_REL
    bound = _update_bound(ro, up, g["C"], prob.params.beta)
    assert np.all(np.abs(g["mean"] - up["mean"]) <= TOL_MEAN + 2.0 * bound)


@pytest.mark.parametrize("c,H", [((0.4, 0.4, 0.2), 16), ((1.0, -0.5, 0.25), 16), ((0.5, 0.3, 0.2), 64)])
def test_config1_comb_filter(oracle_lib, c, H):
    """Comb-filtered Gaussian noise (Sec. 3.3): the kernel's convolution with
    the filter's response against the oracle's recursion in step order; null
    particles stay unfiltered (and zero)."""
    prob = inputs.config1(2, v0_random=True)
    prob.params.horizon = H
    prob.params.dt = np.full(H, 0.02)
    prob.params.n_null = 3
    prob.params.comb_filter = 1
    prob.params.comb = c
    g, ro, up, o, eps = run_pair(prob, oracle_lib)
    assert_states(g, ro)
    assert np.max(cost_error(g["c"], ro["c"])) <= TOL_COST_REL
    assert np.max(cost_error(g["C"], ro["C"])) <= TOL_COST_REL
    bound = _update_bound(ro, up, g["C"], prob.params.beta)
    assert np.all(np.abs(g["mean"] - up["mean"]) <= TOL_MEAN + 2.0 * bound)


def test_config2_mixed_sampling(oracle_lib):
    """The paper's "mixed" sampling (Sec. 5 ablation): 0.6 N Halton + B-spline
    particles and 0.4 N comb-filtered Gaussian particles, every cost term;
    n_halton is odd, so one tile holds a particle of each kind."""
    prob = inputs.config2(7, n_particles=201, horizon=30)
    prob.params.n_halton = 121
    prob.params.comb_filter = 1
    prob.params.comb = (0.4, 0.4, 0.2)
    g, ro, up, o, _ = run_pair(prob, oracle_lib)
    _config2_checks(g, ro, o, prob)


def _config2_checks(g, ro, o, prob):
    p = prob.params
    assert_states(g, ro)
    # the manipulability cost jumps by (1 - k_m) at m = k_m: states within
    # 1e-4 of the threshold may fall on either side in FP32 and are masked
    m = manip_values(o, ro["q"])
    near = np.abs(m - p.k_m) < 1e-4
    err = cost_error(g["c"], ro["c"])
    assert np.max(np.where(near, 0.0, err)) <= TOL_COST_REL, "max running-cost error %.3g" % np.max(err[~near])
    clean = ~near.any(axis=1)
    assert clean.sum() >= 0.9 * p.n_particles
    assert np.max(cost_error(g["C"], ro["C"])[clean]) <= TOL_COST_REL
    # individual terms (unweighted), scaled by their weights
    wts = np.array([p.w_pos, p.w_rot, p.a_joint, p.a_vel, p.a_stop, p.a_manip, p.a_coll, p.a_coll])
    for k in range(8):
        d = np.abs(g["terms"][..., k] - ro["terms"][..., k]) * wts[k]
        d = np.where(near, 0.0, d)
        assert np.max(d / np.maximum(np.abs(ro["c"]), COST_FLOOR)) <= TOL_COST_REL, "term %d" % k
    return clean


@pytest.mark.parametrize("seed", [0, 1])
def test_config2_full(oracle_lib, seed):
    prob = inputs.config2(seed)
    g, ro, up, o, _ = run_pair(prob, oracle_lib)
    clean = _config2_checks(g, ro, o, prob)
    # collision terms are exercised by this scene
    assert np.any(ro["terms"][..., 6] > 0) or np.any(ro["terms"][..., 7] > 0)
    p = prob.params
    sig2_0 = f32(np.asarray(p.sigma_init) ** 2)
    upd = o.update(g["C"], g["u"], np.zeros((p.horizon, 7)), sig2_0)
    assert np.max(np.abs(g["mean"] - upd["mean"])) <= TOL_MEAN
    assert np.max(np.abs(g["sigma2"] - upd["sigma2"])) <= 1e-4 * np.max(upd["sigma2"])
    # end to end: the oracle's own update, except that a particle with a
    # state within 1e-4 of the manipulability threshold (whose cost may
    # legitimately differ by the jump of the term) takes the kernel's C
    n_masked = int((~clean).sum())
    print("config 2 seed %d: %d particle(s) masked at the manipulability threshold" % (seed, n_masked))
    C_ref = np.where(clean, ro["C"], g["C"])
    up_h = o.update(C_ref, ro["u"], np.zeros((p.horizon, 7)), sig2_0)
    ro_h = dict(ro, C=C_ref)
    bound = _update_bound(ro_h, up_h, g["C"], p.beta)
    assert np.all(np.abs(g["mean"] - up_h["mean"]) <= TOL_MEAN + 2.0 * bound)
    if n_masked == 0:
        assert np.array_equal(C_ref, ro["C"])


def test_config2_override_and_halton_table(oracle_lib):
    """Noise override on a STORM-shaped problem with null particles, and the
    Halton + B-spline table against the oracle's."""
    prob = inputs.config2(5, n_particles=123, horizon=30)
    prob.params.n_null = 7
    p = prob.params
    g, ro, up, o, eps = run_pair(prob, oracle_lib)
    _config2_checks(g, ro, o, prob)
    sig = np.sqrt(f32(np.asarray(p.sigma_init) ** 2))
    # recover the GPU's standard noise of the Halton particles from u = sigma eps (mu = 0)
    eps_gpu = g["u"][: p.n_halton] / sig
    ref = oracle_lib.halton_noise(p.n_halton, p.horizon, p.n_knots)
    assert np.max(np.abs(eps_gpu - ref)) < 2e-5
    assert np.all(g["u"][p.n_particles - p.n_null:] == 0.0)


@pytest.mark.parametrize("N,H", [(1, 1), (1, 64), (3, 64), (5, 33), (70, 7), (130, 21), (257, 16), (64, 30)])
def test_shapes_and_ragged(oracle_lib, N, H):
    prob = inputs.config2(11, n_particles=N, horizon=H, n_obs_spheres=5, n_obs_cuboids=5)
    prob.params.n_halton = N // 3
    prob.params.n_null = 1 if N > 2 else 0
    prob.params.gamma = 0.97
    prob.params.w_term = 3.0
    g, ro, up, o, _ = run_pair(prob, oracle_lib)
    _config2_checks(g, ro, o, prob)


def test_zero_variance(oracle_lib):
    """The degenerate distribution: sigma^2 = 0 (set through set_state), so
    every sampled particle follows the mean exactly and only the null
    particles differ.  Against the oracle: states, costs and the update on
    the kernel's costs, with the new variance held at its floor (Eq. 5 gives
    zero)."""
    prob = inputs.config2(17, n_particles=96, horizon=30, n_obs_spheres=10, n_obs_cuboids=10)
    p = prob.params
    p.n_null = 2
    p.sigma2_min = 1e-3
    H = p.horizon
    mean = (0.2 * np.sin(np.linspace(0.0, 3.0, H))[:, None] * np.linspace(-1.0, 1.0, 7)[None, :]).astype(np.float32)
    sig2 = np.zeros(7, dtype=np.float32)
    g, ro, up, o, _ = run_pair(prob, oracle_lib, step_index=5, mean=mean, sigma2=sig2)
    _config2_checks(g, ro, o, prob)
    live = p.n_particles - p.n_null
    assert np.all(g["u"][:live] == mean[None]), "sampled controls equal the mean"
    assert np.all(g["u"][live:] == 0.0)
    # the same trajectory in every sampled particle: equal costs up to the
    # order of the sums, which depends on where the particle sits in its tile
    # (no state of it lies near the manipulability threshold, where the term
    # jumps)
    assert not (np.abs(manip_values(o, ro["q"][:1]) - p.k_m) < 1e-4).any()
    assert np.max(np.abs(g["C"][:live] - g["C"][0])) <= 1e-6 * abs(g["C"][0])
    upd = o.update(g["C"], g["u"], f32(mean), f32(sig2))
    assert np.max(np.abs(g["mean"] - upd["mean"])) <= TOL_MEAN
    np.testing.assert_allclose(upd["sigma2"], p.sigma2_min, rtol=1e-12)
    np.testing.assert_allclose(g["sigma2"], p.sigma2_min, rtol=1e-6)
    assert np.max(np.abs(g["cmd"] - upd["cmd"])) <= TOL_MEAN


@pytest.mark.parametrize("kind", ["halton", "gaussian", "null"])
def test_one_kind_of_particle(oracle_lib, kind):
    """Every particle of one kind: all Halton + B-spline, all Gaussian, or
    all null (u = 0 everywhere, so every particle holds the start state and
    the weights are uniform: the update moves the mean to (1 - alpha_mu) mu).
    Against the oracle: states, costs, terms and the update."""
    prob = inputs.config2(19, n_particles=70, horizon=20, n_obs_spheres=8, n_obs_cuboids=8)
    p = prob.params
    N, H = p.n_particles, p.horizon
    p.n_halton = N if kind == "halton" else 0
    p.n_null = N if kind == "null" else 0
    mean = (0.1 * np.cos(np.linspace(0.0, 2.0, H))[:, None] * np.linspace(1.0, -0.5, 7)[None, :]).astype(np.float32)
    sig2 = f32(np.asarray(p.sigma_init) ** 2)
    g, ro, up, o, _ = run_pair(prob, oracle_lib, step_index=2, mean=mean, sigma2=sig2)
    _config2_checks(g, ro, o, prob)
    upd = o.update(g["C"], g["u"], f32(mean), sig2)
    assert np.max(np.abs(g["mean"] - upd["mean"])) <= TOL_MEAN
    assert np.max(np.abs(g["sigma2"] - upd["sigma2"])) <= 1e-4 * np.max(upd["sigma2"])
    if kind == "null":
        assert np.all(g["u"] == 0.0)
        # uniform on the oracle's own costs (the kernel's differ by the order
        # of their sums, which beta = 0.1 turns into weights a few percent apart)
        np.testing.assert_allclose(up["w"], 1.0 / N, rtol=1e-12)
        np.testing.assert_allclose(g["mean"], (1.0 - p.alpha_mu) * f32(mean), atol=TOL_MEAN)


def test_determinism():
    from paper_2104_13542_amd import storm

    prob = inputs.config2(2)
    outs = []
    for _ in range(2):
        r = storm.Rollout(prob)
        from tests.gpu_common import device_goal  # noqa: F401
        goal = torch.zeros(12, device="cuda")
        goal[0] = goal[4] = goal[8] = 1.0
        goal[9:] = torch.tensor([0.5, 0.0, 0.5])
        o = r.step(goal, debug=True)
        cmd, mean, sig = r.update()
        o2 = r.step(goal, debug=True)
        torch.cuda.synchronize()
        outs.append([o["C"].cpu(), o["c"].cpu(), o["q"].cpu(), mean.cpu(), sig.cpu(), o2["C"].cpu()])
        r.close()
    for a, b in zip(*outs):
        assert torch.equal(a, b)


def test_multi_step_shift_chain(oracle_lib):
    """Three control steps (step, update with shift) compared with the oracle
    chain fed the same noise; the oracle update runs on the GPU's costs so the
    chain does not drift through the softmin."""
    from paper_2104_13542_amd import storm
    from tests.gpu_common import device_goal

    prob = inputs.config1(4)
    p = prob.params
    N, H = p.n_particles, p.horizon
    prob.q0, prob.v0, prob.a0 = f32(prob.q0), f32(prob.v0), f32(prob.a0)
    o = oracle_lib.Oracle(prob, dh=f32(inputs.PANDA_DH), q_min=f32(inputs.PANDA_Q_MIN),
                          q_max=f32(inputs.PANDA_Q_MAX), qd_max=f32(inputs.PANDA_QD_MAX))
    o.goal = f32(o.goal)
    r = storm.Rollout(prob)
    goal = device_goal(o)
    mean = np.zeros((H, 7))
    sig2 = f32(np.asarray(p.sigma_init) ** 2)
    try:
        for step in range(3):
            eps = f32(inputs.standard_normal(500 + step, (N, H, 7)))
            nt = torch.tensor(eps.transpose(2, 0, 1).copy(), dtype=torch.float32, device="cuda")
            out = r.step(goal, noise=nt, debug=True)
            cmd, mean_new, sig_new = r.update(shift=True)
            torch.cuda.synchronize()
            ro = o.rollout(mean, np.sqrt(sig2), eps)
            assert np.max(np.abs(to_nhj(out["q"]) - ro["q"])) <= TOL_STATE
            gC = out["C"].cpu().double().numpy()
            assert np.max(cost_error(gC, ro["C"])) <= TOL_COST_REL
            upd = o.update(gC, to_nhj(out["u"]), mean, sig2)
            assert np.max(np.abs(mean_new.cpu().numpy() - upd["mean"])) <= TOL_MEAN
            mean = f32(upd["mean_shift"])
            sig2 = f32(sig_new.cpu().numpy())
            gm, gs, gstep = r.get_state()
            assert np.max(np.abs(gm - mean)) <= TOL_MEAN
            assert gstep == step + 1
    finally:
        r.close()


def test_state_roundtrip_reproduces(oracle_lib):
    """get_state / set_state restore a run bit for bit (counter-based RNG)."""
    from paper_2104_13542_amd import storm

    prob = inputs.config2(6, n_particles=200, horizon=30)
    goal = torch.tensor([1, 0, 0, 0, -1, 0, 0, 0, -1, 0.5, 0.1, 0.4], dtype=torch.float32, device="cuda")
    r = storm.Rollout(prob)
    try:
        for _ in range(3):
            r.step(goal)
            r.update()
        snap = r.get_state()
        ref = []
        for _ in range(2):
            o = r.step(goal)
            c, m, s = r.update()
            ref.append((o["C"].clone(), m.clone()))
        r.set_state(*snap)
        for k in range(2):
            o = r.step(goal)
            c, m, s = r.update()
            assert torch.equal(o["C"], ref[k][0]) and torch.equal(m, ref[k][1])
    finally:
        r.close()


def test_nonfinite_cost_keeps_policy():
    """A non-finite start state makes every cost non-finite: the update keeps
    mu and sigma2 and raises the status flag (forced from the host)."""
    from paper_2104_13542_amd import storm

    prob = inputs.config1(0)
    r = storm.Rollout(prob)
    try:
        goal = torch.tensor([1, 0, 0, 0, 1, 0, 0, 0, 1, 0.5, 0, 0.5], dtype=torch.float32, device="cuda")
        mean0, sig0, _ = r.get_state()
        x0 = r.x0.clone()
        x0[0] = float("nan")
        r.step(goal, x0=x0)
        cmd, mean, sig = r.update(shift=False)
        torch.cuda.synchronize()
        assert np.array_equal(mean.cpu().numpy(), mean0)
        assert np.array_equal(sig.cpu().numpy(), sig0)
        assert r.status() & storm.FLAG_NONFINITE_COST
        assert r.status() == 0  # cleared by the read
    finally:
        r.close()


def test_abi_errors_on_gpu():
    from paper_2104_13542_amd import storm

    prob = inputs.config1(0)
    r = storm.Rollout(prob)
    try:
        with pytest.raises(storm.StormError) as e:
            r.update()
        assert e.value.code == storm.STORM_E_STATE
        cmd = torch.zeros(7, dtype=torch.float32, device="cuda")
        goal = torch.zeros(12, dtype=torch.float32, device="cuda")
        with pytest.raises(storm.StormError) as e:
            r.control(r.x0, goal, cmd, iterations=0)
        assert e.value.code == storm.STORM_E_RANGE
    finally:
        r.close()


@pytest.mark.parametrize("iterations", [1, 2])
def test_graph_replays_match_eager(iterations):
    """A captured control step (K iterations of step + update, shift on the
    last) replayed several times, with eager work and host synchronisation
    between the replays, equals the eager calls bit for bit at every replay;
    so does the one-call eager control step (storm_rollout_control)."""
    from paper_2104_13542_amd import storm

    prob = inputs.config2(7, n_particles=300, horizon=30)
    eager = storm.Rollout(prob)
    graphed = storm.Rollout(prob)
    control = storm.Rollout(prob)
    try:
        x0 = eager.x0.clone()
        goal = torch.tensor([1, 0, 0, 0, -1, 0, 0, 0, -1, 0.45, 0.1, 0.5], dtype=torch.float32, device="cuda")
        cmd_g = torch.zeros(7, dtype=torch.float32, device="cuda")
        cmd_c = torch.zeros(7, dtype=torch.float32, device="cuda")
        g = graphed.graph(x0, goal, cmd_g, iterations=iterations, shift=True)
        for rep in range(4):
            for k in range(iterations):
                eager.step(goal, x0=x0)
                cmd_e, _, _ = eager.update(shift=(k == iterations - 1))
            g.launch()
            control.control(x0, goal, cmd_c, iterations=iterations, shift=True)
            torch.cuda.synchronize()
            assert torch.equal(cmd_e, cmd_g), rep
            assert torch.equal(cmd_e, cmd_c), rep
            me, se, ste = eager.get_state()
            mg, sg, stg = graphed.get_state()
            mc, sc, stc = control.get_state()
            assert np.array_equal(me, mg) and np.array_equal(se, sg) and ste == stg == iterations * (rep + 1)
            assert np.array_equal(me, mc) and np.array_equal(se, sc) and stc == ste
            # eager work on the graphed context's inputs between replays
            x0.add_(0.001)
            torch.cuda.synchronize()
        g.close()
        # the control step leaves no step pending
        with pytest.raises(storm.StormError) as e:
            control.update()
        assert e.value.code == storm.STORM_E_STATE
    finally:
        eager.close()
        graphed.close()
        control.close()


def test_command_to_pinned_host_memory():
    """The update kernel writes the command straight into pinned host memory
    (readable after the stream synchronises, no copy): eager control steps
    and graph replays give the same commands, bit for bit, as the same calls
    writing device memory."""
    from paper_2104_13542_amd import storm

    prob = inputs.config2(11, n_particles=200, horizon=30)
    prob.params.grad_mask = inputs.COST_POSE | inputs.COST_JOINT
    modes = ("device", "pinned", "graph_device", "graph_pinned", "refine_device", "refine_pinned")
    ctx = {m: storm.Rollout(prob) for m in modes}
    try:
        x0 = ctx["device"].x0.clone()
        goal = torch.tensor([1, 0, 0, 0, -1, 0, 0, 0, -1, 0.45, 0.1, 0.5], dtype=torch.float32, device="cuda")
        cmd = {m: (torch.zeros(7, dtype=torch.float32, pin_memory=True) if "pinned" in m
                   else torch.zeros(7, dtype=torch.float32, device="cuda")) for m in ctx}
        graphs = {m: ctx[m].graph(x0, goal, cmd[m], iterations=1, shift=True) for m in ("graph_device", "graph_pinned")}
        # the refinement graph writes the command from the Adam kernel
        graphs.update({m: ctx[m].graph(x0, goal, cmd[m], iterations=1, shift=True, refine_iters=2, lr=0.05)
                       for m in ("refine_device", "refine_pinned")})
        for step in range(5):
            ctx["device"].control(x0, goal, cmd["device"])
            ctx["pinned"].control(x0, goal, cmd["pinned"])
            for m in graphs:
                graphs[m].launch()
            torch.cuda.synchronize()
            ref = cmd["device"].cpu()
            assert torch.equal(ref, cmd["pinned"]), step
            assert torch.equal(ref, cmd["graph_device"].cpu()), step
            assert torch.equal(ref, cmd["graph_pinned"]), step
            assert torch.equal(cmd["refine_device"].cpu(), cmd["refine_pinned"]), step
            x0.add_(0.002)
        for g in graphs.values():
            g.close()
    finally:
        for r in ctx.values():
            r.close()


@pytest.mark.parametrize("N,H,beta", [(5000, 16, 1e6), (700, 30, 1e6), (3000, 8, 50.0), (2500, 30, 0.1),
                                      (1088, 30, 1e6), (512, 64, 0.1), (2048, 16, 1e6)])
def test_update_dense_and_sparse_paths(oracle_lib, N, H, beta):
    """The update holds the controls in registers when every thread needs at
    most 32 of them (N <= 32 floor(1024 / H), N <= 2048: the last three cases
    sit on that edge), else gathers only particles with nonzero weight when
    they fit the compaction list (4096), else streams every particle; each
    must equal the oracle's update on the same costs and controls."""
    prob = inputs.config1(8)
    prob.params.n_particles = N
    prob.params.horizon = H
    prob.params.dt = np.full(H, 0.02)
    prob.params.beta = beta
    prob.params.n_null = 3
    eps = inputs.standard_normal(900 + N, (N, H, 7))
    g, ro, up, o, _ = run_pair(prob, oracle_lib, noise_nhj=eps)
    upd = o.update(g["C"], g["u"], np.zeros((H, 7)), f32(np.asarray(prob.params.sigma_init) ** 2))
    assert np.max(np.abs(g["mean"] - upd["mean"])) <= TOL_MEAN
    assert np.max(np.abs(g["sigma2"] - upd["sigma2"])) <= 1e-4 * np.max(upd["sigma2"])


def _sig2_init32(p):
    s = np.asarray(p.sigma_init, dtype=np.float32).astype(np.float64)
    return (s * s).astype(np.float32)


@pytest.mark.parametrize("cfg", ["config1", "config2"])
def test_per_step_covariance(oracle_lib, cfg):
    """Eq. 5 kept per (step, joint): each step's noise is scaled by its own
    sigma, the update gives every (step, joint) its own weighted variance, and
    the stored state moves forward with sigma_init^2 appended (Alg. 1)."""
    if cfg == "config1":
        prob = inputs.config1(4, v0_random=True)
        prob.params.n_null = 2
    else:
        prob = inputs.config2(5, n_particles=160, horizon=30)
    p = prob.params
    p.cov_per_step = 1
    H = p.horizon
    rng = np.random.default_rng(11)
    sig2 = f32(np.asarray(p.sigma_init) ** 2 * rng.uniform(0.3, 2.0, (H, 7)))
    mean = f32(rng.normal(scale=0.2, size=(H, 7)))
    g, ro, up, o, eps = run_pair(prob, oracle_lib, mean=mean, sigma2=sig2)
    if cfg == "config1":
        assert_states(g, ro)
        assert np.max(cost_error(g["c"], ro["c"])) <= TOL_COST_REL
        assert np.max(cost_error(g["C"], ro["C"])) <= TOL_COST_REL
    else:
        _config2_checks(g, ro, o, prob)
    # the controls carry the per-step sigma
    live = p.n_particles - p.n_null
    np.testing.assert_allclose(g["u"][:live], mean + np.sqrt(sig2) * eps[:live], atol=2e-6)
    assert g["sigma2"].shape == (H, 7)
    upd = o.update(g["C"], g["u"], mean, sig2)
    assert np.max(np.abs(g["mean"] - upd["mean"])) <= TOL_MEAN
    assert np.max(np.abs(g["sigma2"] - upd["sigma2"])) <= 1e-4 * np.max(upd["sigma2"])
    # the variances differ from step to step
    assert np.ptp(upd["sigma2"], axis=0).min() > 0
    mean_s, sig_s, step = g["state_after"]
    assert sig_s.shape == (H, 7) and step == 1
    np.testing.assert_array_equal(sig_s[:-1], g["sigma2"][1:].astype(np.float32))
    np.testing.assert_array_equal(sig_s[-1], _sig2_init32(p))
    np.testing.assert_array_equal(mean_s[:-1], g["mean"][1:].astype(np.float32))


def test_per_step_covariance_initial_state_and_round_trip():
    """A fresh per-step context holds sigma_init^2 at every step; set_state
    and get_state move the [H][7] array unchanged; the non-shifting update
    keeps the steps in place."""
    from paper_2104_13542_amd import storm

    prob = inputs.config1(6)
    p = prob.params
    p.cov_per_step = 1
    H = p.horizon
    r = storm.Rollout(prob)
    try:
        _, s0, _ = r.get_state()
        assert s0.shape == (H, 7)
        np.testing.assert_array_equal(s0, np.broadcast_to(_sig2_init32(p), (H, 7)))
        s = np.random.default_rng(2).uniform(1e-3, 1e-1, (H, 7)).astype(np.float32)
        r.set_state(sigma2=s)
        _, s1, _ = r.get_state()
        np.testing.assert_array_equal(s1, s)
        goal = torch.tensor([1, 0, 0, 0, -1, 0, 0, 0, -1, 0.4, 0.1, 0.45], dtype=torch.float32, device="cuda")
        r.step(goal)
        _, _, s_new = r.update(shift=False)
        torch.cuda.synchronize()
        _, s2, _ = r.get_state()
        np.testing.assert_array_equal(s2, s_new.cpu().numpy())
    finally:
        r.close()


@pytest.mark.parametrize("cfg", ["config1", "config2"])
def test_task_space_velocity_and_acceleration(oracle_lib, cfg):
    """Flange velocity and acceleration (Eq. 8) at every (particle, step):
    the kernel's outward pass against the oracle's J qd and Jdot qd + J qdd
    (Jdot from its definition) at the kernel's own float32 states; the
    task-space form leaves the costs as the plain form computes them."""
    prob = inputs.config1(3, v0_random=True) if cfg == "config1" else inputs.config2(4, n_particles=100)
    prob.params.n_null = 3  # null particles: qdd = 0, so xdd = Jdot qd
    p = prob.params
    g, ro, up, o, eps = run_pair(prob, oracle_lib, task_space=True)
    assert_states(g, ro)
    assert g["xd"].shape == (p.n_particles, p.horizon, 6)
    err_v = err_a = 0.0
    for i in range(p.n_particles):
        for h in range(p.horizon):
            xd, xdd = oracle_lib.task_space(o.dh, g["q"][i, h], g["v"][i, h], g["a"][i, h])
            err_v = max(err_v, np.max(np.abs(g["xd"][i, h] - xd)) / max(1.0, np.max(np.abs(xd))))
            err_a = max(err_a, np.max(np.abs(g["xdd"][i, h] - xdd)) / max(1.0, np.max(np.abs(xdd))))
    assert err_v <= 2e-6 and err_a <= 1e-5, (err_v, err_a)
    # the same step through the plain form (same noise draw: step counter 0)
    g2, _, _, _, _ = run_pair(prob, oracle_lib)
    np.testing.assert_allclose(g2["C"], g["C"], rtol=1e-6)
    np.testing.assert_allclose(g2["q"], g["q"], rtol=0, atol=1e-6)


@pytest.mark.parametrize("seed,N,n_null", [(0, 64, 0), (1, 203, 0), (2, 97, 5)])
def test_ball_on_tray(oracle_lib, seed, N, n_null):
    """The ball term (appendix on dynamic object balancing) against the
    oracle: the ball's in-plane trajectory under the rolled-out flange
    orientations, its distance from the tray centre, the running and
    horizon costs, and the update that follows."""
    prob = inputs.config_ball(seed, n_particles=N)
    prob.params.ball_center = (0.01, -0.015)
    prob.params.n_null = n_null
    p = prob.params
    g, ro, up, o, eps = run_pair(prob, oracle_lib)
    assert_states(g, ro)
    assert np.max(np.abs(ro["terms"][..., 8])) > 0.05
    live = p.n_particles - p.n_null
    np.testing.assert_allclose(g["terms"][:live, :, 8], ro["terms"][:live, :, 8], atol=2e-5)
    # manipulability threshold crossings aside, every running cost agrees
    m = manip_values(o, ro["q"])
    near = np.abs(m - p.k_m) < 1e-4
    err = cost_error(g["c"], ro["c"])
    assert np.max(np.where(near, 0.0, err)) <= TOL_COST_REL
    clean = ~near.any(axis=1)
    assert np.max(cost_error(g["C"], ro["C"])[clean]) <= TOL_COST_REL
    upd = o.update(g["C"], g["u"], np.zeros((p.horizon, 7)), f32(np.asarray(p.sigma_init) ** 2))
    assert np.max(np.abs(g["mean"] - upd["mean"])) <= TOL_MEAN


def test_ball_state_is_read_at_every_step():
    """A new ball state changes the next step's ball term, and a graph
    replay reads the state set before it: graph and eager steps of two
    contexts in the same state give the same command for each ball state."""
    from paper_2104_13542_amd import storm

    prob = inputs.config_ball(2, n_particles=64)
    H = prob.params.horizon
    r = storm.Rollout(prob)
    rg = storm.Rollout(prob)
    try:
        goal = torch.tensor([1, 0, 0, 0, -1, 0, 0, 0, -1, 0.4, 0.1, 0.45], dtype=torch.float32, device="cuda")
        noise = torch.tensor(inputs.standard_normal(9, (7, 64, H)), dtype=torch.float32, device="cuda")
        x0 = r.x0.clone()
        E = storm.fk(x0[:7].reshape(1, 7).contiguous())[0][0]  # [R (9), p (3)] of the flange at q0
        at_centre = torch.cat([E[9:12], torch.zeros(3, device="cuda")]).contiguous()
        off_centre = torch.cat([E[9:12] + 0.05 * E[0:9:3], torch.zeros(3, device="cuda")]).contiguous()
        r.set_ball(off_centre)
        a = r.step(goal, noise=noise, debug=True)["terms"][8].clone()
        r.update(shift=False, want_mean=False)
        r.set_ball(at_centre)
        b = r.step(goal, noise=noise, debug=True)["terms"][8].clone()
        r.update(shift=False, want_mean=False)
        torch.cuda.synchronize()
        # 5 cm along the tray's x axis: the first step's distance is 5 cm more
        assert abs(float(a[0, 0] - b[0, 0]) - 0.05) < 2e-3
        # graph (rg) against eager (r) from the same state and counter
        r.close()
        r = storm.Rollout(prob)
        cmd_g = torch.empty(7, device="cuda")
        cmd_e = torch.empty(7, device="cuda")
        graph = rg.graph(x0, goal, cmd_g, iterations=1, shift=True)
        cmds = []
        for ball in (off_centre, at_centre):
            rg.set_ball(ball)
            graph.launch()
            r.set_ball(ball)
            r.step(goal, x0=x0)
            r.update(shift=True, want_mean=False, cmd=cmd_e)
            torch.cuda.synchronize()
            assert torch.equal(cmd_g, cmd_e)
            cmds.append(cmd_g.clone())
        assert not torch.equal(cmds[0], cmds[1])
        graph.close()
    finally:
        r.close()
        rg.close()


def _net_parts(prm):
    parts, k = {}, 0
    for name, shape in inputs.SELF_MLP_LAYOUT:
        n = int(np.prod(shape))
        parts[name] = prm[k:k + n].reshape(shape)
        k += n
    return parts


def _net_forward(prm, q):
    """The network's output d in FP64 for rows q [R][7] (numpy, from the
    layout of the flat parameter array)."""
    P = _net_parts(prm)
    x = np.concatenate([np.sin(q), np.cos(q)], axis=1)
    a1 = np.maximum(x @ P["W1"].T + P["b1"], 0.0)
    a2 = np.maximum(a1 @ P["W2"].T + P["b2"], 0.0)
    a3 = np.maximum(a2 @ P["W3"].T + P["b3"], 0.0)
    return a3 @ P["w4"] + P["b4"][0]


# The kernel carries every activation as an FP16 (hi, lo) pair with FP16
# weights and FP32 accumulation: its d agrees with the FP64 network to FP32
# rounding (at most 8e-8 m measured over these shapes).  An FP16-only
# evaluation errs by up to 2e-4 m on these states and fails this bound.
TOL_NET = 1e-6


@pytest.mark.parametrize("seed,N,H,extra", [(0, 64, 30, 0), (1, 500, 30, 0), (2, 1, 64, 0), (3, 37, 7, 0),
                                             (4, 150, 30, 12)])
def test_self_collision_network(oracle_lib, seed, N, H, extra):
    """The learned self-collision model (Eq. 13, jointNERF form) on the
    matrix cores against the FP64 oracle: max(0, d) at the kernel's own
    states to TOL_NET (m), and the running and horizon costs of the
    oracle's rollout with the network term to 1e-4 relative.  extra = 12
    adds small flange spheres (a 64-sphere model: the sphere count does not
    change the network pass)."""
    prob = inputs.config_self_mlp(seed, n_particles=N, horizon=H)
    if extra:
        add = np.array([[8.0, 0.0, 0.0, 0.01 * k, 0.02] for k in range(extra)])
        prob.spheres = np.concatenate([prob.spheres, add])
    o0 = oracle_lib.Oracle(prob)
    q0s = o0.rollout(np.zeros((H, 7)), np.asarray(prob.params.sigma_init), o0.noise(0))["q"].reshape(-1, 7)
    d0 = _net_forward(prob.self_mlp, q0s)
    prob.self_mlp[-1] = float(np.float32(prob.self_mlp[-1] - np.median(d0)))  # both signs occur
    p = prob.params
    g, ro, up, o, eps = run_pair(prob, oracle_lib)
    assert_states(g, ro)
    q = g["q"].reshape(-1, 7)
    d_ref = _net_forward(prob.self_mlp, q)
    # the FP64 network of the oracle agrees with the numpy forward pass
    for r in range(0, q.shape[0], 97):
        assert oracle_lib.self_mlp(prob.self_mlp, q[r]) == pytest.approx(d_ref[r], rel=1e-12, abs=1e-12)
    term = g["terms"][..., 6].reshape(-1)
    ref = np.maximum(d_ref, 0.0)
    if N * H >= 1000:
        assert (d_ref > 0).mean() > 0.1 and (d_ref < 0).mean() > 0.1
    err = np.abs(term - ref)
    print("network term: max |error| %.3g m over %d rows" % (np.max(err), err.size))
    assert np.max(err) <= TOL_NET, "max |d error| %.3g m" % np.max(err)
    # the oracle's rollout with the network term: running and horizon costs
    m = manip_values(o, ro["q"])
    near = np.abs(m - p.k_m) < 1e-4
    errc = cost_error(g["c"], ro["c"])
    assert np.max(np.where(near, 0.0, errc)) <= TOL_COST_REL, "running cost %.3g" % np.max(errc[~near])
    clean = ~near.any(axis=1)
    assert clean.sum() >= 0.9 * p.n_particles
    assert np.max(cost_error(g["C"], ro["C"])[clean]) <= TOL_COST_REL
    # the network term at the oracle's states, weighted, within the cost bar
    dt6 = np.abs(g["terms"][..., 6] - ro["terms"][..., 6]) * p.a_coll
    assert np.max(np.where(near, 0.0, dt6) / np.maximum(np.abs(ro["c"]), COST_FLOOR)) <= TOL_COST_REL
    upd = o.update(g["C"], g["u"], np.zeros((p.horizon, 7)), f32(np.asarray(p.sigma_init) ** 2))
    assert np.max(np.abs(g["mean"] - upd["mean"])) <= TOL_MEAN


def test_self_collision_network_in_a_graph():
    """A captured control step with the network pass equals the eager step
    (same commands over three steps)."""
    from paper_2104_13542_amd import storm

    prob = inputs.config_self_mlp(2, n_particles=200)
    r = storm.Rollout(prob)
    rg = storm.Rollout(prob)
    try:
        goal = torch.tensor([1, 0, 0, 0, -1, 0, 0, 0, -1, 0.4, 0.1, 0.45], dtype=torch.float32, device="cuda")
        x0 = r.x0.clone()
        cmd_g = torch.empty(7, device="cuda")
        cmd_e = torch.empty(7, device="cuda")
        graph = rg.graph(x0, goal, cmd_g, iterations=1, shift=True)
        for _ in range(3):
            graph.launch()
            r.step(goal, x0=x0)
            r.update(shift=True, want_mean=False, cmd=cmd_e)
            torch.cuda.synchronize()
            assert torch.equal(cmd_g, cmd_e)
        graph.close()
    finally:
        r.close()
        rg.close()


def test_per_step_covariance_graph_with_two_iterations():
    """K = 2 iterations per control step with a per-step covariance: the
    captured graph (two rollouts and updates, the shift after the second)
    gives the eager sequence's commands and state, bit for bit."""
    from paper_2104_13542_amd import storm

    prob = inputs.config2(6, n_particles=150)
    prob.params.cov_per_step = 1
    r = storm.Rollout(prob)
    rg = storm.Rollout(prob)
    try:
        goal = torch.tensor([1, 0, 0, 0, -1, 0, 0, 0, -1, 0.4, 0.1, 0.45], dtype=torch.float32, device="cuda")
        x0 = r.x0.clone()
        cmd_g = torch.empty(7, device="cuda")
        cmd_e = torch.empty(7, device="cuda")
        graph = rg.graph(x0, goal, cmd_g, iterations=2, shift=True)
        for _ in range(3):
            graph.launch()
            for k in range(2):
                r.step(goal, x0=x0)
                r.update(shift=k == 1, want_mean=False, cmd=cmd_e)
            torch.cuda.synchronize()
            assert torch.equal(cmd_g, cmd_e)
        me, se, ste = r.get_state()
        mg, sg, stg = rg.get_state()
        assert se.shape == (prob.params.horizon, 7)
        assert np.array_equal(me, mg) and np.array_equal(se, sg) and ste == stg == 6
        graph.close()
    finally:
        r.close()
        rg.close()


@pytest.mark.parametrize("cfg", ["config1", "config2"])
def test_two_iterations_against_oracle_chain(oracle_lib, cfg):
    """K = 2 iterations in one control step (Alg. 1, inner loop): rollout,
    update without a shift, a second rollout from the unshifted mean with
    the noise counter one further, update, then the shift.  Each iteration
    is compared with the oracle fed the same mean and variance: states to
    1e-5, running and horizon costs to 1e-4 relative, the updated mean and
    variance (the oracle's update on the kernel's costs) to 1e-4; the first
    iteration also end to end."""
    from paper_2104_13542_amd import storm
    from tests.gpu_common import device_goal

    if cfg == "config1":
        prob = inputs.config1(5, v0_random=True)
        prob.params.n_null = 2
    else:
        prob = inputs.config2(8, n_particles=200)
    p = prob.params
    N, H = p.n_particles, p.horizon
    prob.spheres, prob.obstacles = f32(prob.spheres), f32(prob.obstacles)
    prob.q0, prob.v0, prob.a0 = f32(prob.q0), f32(prob.v0), f32(prob.a0)
    o = oracle_lib.Oracle(prob, dh=f32(inputs.PANDA_DH), q_min=f32(inputs.PANDA_Q_MIN),
                          q_max=f32(inputs.PANDA_Q_MAX), qd_max=f32(inputs.PANDA_QD_MAX))
    o.dt = f32(p.dt)
    o.goal = f32(o.goal)
    r = storm.Rollout(prob)
    goal = device_goal(o)
    mean = np.zeros((H, 7))
    sig2 = f32(np.asarray(p.sigma_init) ** 2)
    try:
        for k in range(2):
            out = r.step(goal, debug=True)
            cmd, mean_new, sig_new = r.update(shift=(k == 1))
            torch.cuda.synchronize()
            g = {key: v.detach().cpu().double().numpy() for key, v in out.items()}
            for key in ("u", "q", "v", "a"):
                g[key] = g[key].transpose(1, 2, 0)
            g["terms"] = g["terms"].transpose(1, 2, 0)
            eps = o.noise(k)  # the counter advances with every update
            eps[N - p.n_null:] = 0.0
            ro = o.rollout(mean, np.sqrt(sig2), eps)
            if cfg == "config1":
                assert_states(g, ro)
                assert np.max(cost_error(g["c"], ro["c"])) <= TOL_COST_REL
                assert np.max(cost_error(g["C"], ro["C"])) <= TOL_COST_REL
            else:
                _config2_checks(g, ro, o, prob)
            upd = o.update(g["C"], g["u"], mean, sig2)
            gm = mean_new.cpu().double().numpy()
            gs = sig_new.cpu().double().numpy()
            assert np.max(np.abs(gm - upd["mean"])) <= TOL_MEAN, k
            assert np.max(np.abs(gs - upd["sigma2"])) <= 1e-4 * np.max(upd["sigma2"]), k
            if k == 0 and cfg == "config1":
                up = o.update(ro["C"], ro["u"], mean, sig2)
                bound = _update_bound(ro, up, g["C"], p.beta)
                assert np.all(np.abs(gm - up["mean"]) <= TOL_MEAN + 2.0 * bound)
            mean_s, sig_s, step = r.get_state()
            assert step == k + 1
            if k == 0:
                # no shift between the iterations: the stored mean is mu'
                np.testing.assert_array_equal(mean_s, mean_new.cpu().numpy())
            else:
                np.testing.assert_array_equal(mean_s[:-1], mean_new.cpu().numpy()[1:])
                assert np.all(mean_s[-1] == 0)
                np.testing.assert_allclose(cmd.cpu().double().numpy(), upd["cmd"], atol=TOL_MEAN)
                np.testing.assert_allclose(mean_s, f32(upd["mean_shift"]), atol=TOL_MEAN)
            # the next iteration samples around the kernel's (unshifted) mean
            mean, sig2 = f32(gm), f32(gs)
    finally:
        r.close()
