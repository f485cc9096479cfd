"""GPU parity of the collision terms (Eq. 13-14) in scenes built to exercise
the rollout kernel's broad phase: dense scenes with more than two 64-obstacle
chunks and obstacles planted on the body spheres, a sphere-obstacle grazing
contact, and a tile whose other particle is non-finite (marked gpu).

Culling may only skip pairs that touch at no point, so every comparison is
the usual one against the oracle, which tests every pair."""
import numpy as np
import pytest

from paper_2104_13542_amd import inputs
from tests.gpu_common import COST_FLOOR, TOL_COST_REL, TOL_STATE, cost_error, f32, o_fk, run_pair
from tests.test_gpu_parity import _config2_checks

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2104_13542_amd import storm

    storm.lib()


def _body_centres(o, spheres, q):
    """World centres of the body spheres at configuration q (oracle FK)."""
    T = np.asarray(o_fk(o, q)).reshape(8, 4, 4)
    return np.array([T[int(r[0]) - 1, :3, :3] @ r[1:4] + T[int(r[0]) - 1, :3, 3] for r in spheres])


def _planted_scene(oracle_lib, prob, rng, n_sph, n_box):
    """Obstacles centred near randomly chosen body spheres of the start
    configuration (offsets ~ N(0, 0.05) m), so that the narrow phase of both
    obstacle kinds runs and many states collide."""
    o = oracle_lib.Oracle(prob)
    cen = _body_centres(o, prob.spheres, prob.q0)
    rows = []
    for k in range(n_sph + n_box):
        row = np.zeros(inputs.OBSTACLE_STRIDE)
        row[1:4] = cen[rng.integers(len(cen))] + rng.normal(0.0, 0.05, 3)
        if k < n_sph:
            row[0] = inputs.OBS_SPHERE
            row[4] = rng.uniform(0.02, 0.08)
            row[7:16] = np.eye(3).reshape(-1)
        else:
            row[0] = inputs.OBS_CUBOID
            row[4:7] = rng.uniform(0.02, 0.08, 3)
            row[7:16] = inputs.random_rotation(rng).reshape(-1)
        rows.append(row)
    return np.array(rows)


@pytest.mark.parametrize("n_sph,n_box", [(70, 60), (0, 65), (65, 0)])
def test_dense_planted_scene(oracle_lib, n_sph, n_box):
    """Up to three obstacle chunks; planted obstacles plus far random ones."""
    rng = np.random.default_rng(31 + n_sph)
    prob = inputs.config2(21, n_particles=96, horizon=30, n_obs_spheres=n_sph // 2, n_obs_cuboids=n_box // 2)
    prob.params.n_null = 4  # null particles sit at the start configuration
    planted = _planted_scene(oracle_lib, prob, rng, n_sph - n_sph // 2, n_box - n_box // 2)
    prob.obstacles = np.concatenate([prob.obstacles.reshape(-1, inputs.OBSTACLE_STRIDE), planted])
    g, ro, up, o, _ = run_pair(prob, oracle_lib)
    _config2_checks(g, ro, o, prob)
    env = ro["terms"][..., 7]
    assert np.mean(env > 0) > 0.2, "the planted scene should collide often"


def test_grazing_sphere_obstacles(oracle_lib):
    """Sphere obstacles whose surface lies within 1e-6 m of a body sphere at
    the start configuration, on both sides of contact; null particles hold
    that configuration at every step."""
    rng = np.random.default_rng(44)
    prob = inputs.config2(23, n_particles=64, horizon=30, n_obs_spheres=4, n_obs_cuboids=4)
    prob.params.n_null = 8
    o = oracle_lib.Oracle(prob)
    cen = _body_centres(o, f32(prob.spheres), f32(prob.q0))
    rows = []
    for k, gap in enumerate([-1e-6, -1e-7, 0.0, 1e-7, 1e-6, -3e-6]):
        s = rng.integers(len(cen))
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        r_o = 0.05
        row = np.zeros(inputs.OBSTACLE_STRIDE)
        row[0] = inputs.OBS_SPHERE
        row[1:4] = cen[s] + d * (prob.spheres[s, 4] + r_o + gap)
        row[4] = r_o
        row[7:16] = np.eye(3).reshape(-1)
        rows.append(row)
    prob.obstacles = np.concatenate([prob.obstacles.reshape(-1, inputs.OBSTACLE_STRIDE), np.array(rows)])
    g, ro, up, o, _ = run_pair(prob, oracle_lib)
    _config2_checks(g, ro, o, prob)


def test_nonfinite_particle_leaves_tile_neighbours_exact(oracle_lib):
    """An infinite noise value makes one particle's states non-finite; the
    other particle of its 64-lane tile must still get every collision term
    (a non-finite centre turns the culling off for that tile)."""
    prob = inputs.config2(24, n_particles=64, horizon=30)
    prob.obstacles = np.concatenate([prob.obstacles.reshape(-1, inputs.OBSTACLE_STRIDE),
                                     _planted_scene(oracle_lib, prob, np.random.default_rng(5), 10, 10)])
    eps = inputs.standard_normal(77, (64, 30, 7))
    eps[0, 5, 2] = np.inf
    g, ro, up, o, _ = run_pair(prob, oracle_lib, noise_nhj=eps)
    fin = np.arange(1, 64)
    for k in ("u", "q", "v"):
        assert np.max(np.abs(g[k][fin] - ro[k][fin])) <= TOL_STATE, k
    assert not np.all(np.isfinite(g["c"][0]))
    # particle 1 shares tile 0 with the non-finite particle 0
    assert np.any(ro["terms"][1, :, 7] > 0) or np.any(ro["terms"][1, :, 6] > 0)
    p = prob.params
    wts = np.array([p.w_pos, p.w_rot, p.a_joint, p.a_vel, p.a_stop, p.a_manip, p.a_coll, p.a_coll])
    for k in (6, 7):
        d = np.abs(g["terms"][fin, :, k] - ro["terms"][fin, :, k]) * wts[k]
        assert np.max(d / np.maximum(np.abs(ro["c"][fin]), COST_FLOOR)) <= TOL_COST_REL, "term %d" % k


@pytest.mark.parametrize("q0", [[0.794, -0.812, -2.66, -3.022, 1.815, 3.424, 0.618],
                                [1.635, -1.566, 2.819, -2.644, 0.923, 0.507, -0.996],
                                [1.638, 1.227, 0.041, -3.039, 0.047, 1.228, 0.314]])
def test_self_colliding_start(oracle_lib, q0):
    """Folded start configurations whose body spheres overlap (found by
    sampling the joint box with the oracle's self-collision term), so that
    the self-collision narrow phase reports penetrations."""
    prob = inputs.config2(25, n_particles=128, horizon=30)
    prob.q0 = np.array(q0)
    prob.params.n_null = 2
    g, ro, up, o, _ = run_pair(prob, oracle_lib)
    _config2_checks(g, ro, o, prob)
    assert np.mean(ro["terms"][..., 6] > 0) > 0.2, "the start should self-collide often"


def _odd_sphere_model():
    """32 spheres with 3, 5, 1, 7, 2, 6, 5, 3 per body, taken (cycling, with a
    1 cm shift on repeats) from the rows of the 52-sphere model: pair groups
    of one to four spheres and odd partner ranges (3 and 9 partners)."""
    base = inputs.panda_spheres()
    counts = [3, 5, 1, 7, 2, 6, 5, 3]
    rows = []
    for b, n in enumerate(counts, start=1):
        own = base[base[:, 0] == b]
        for k in range(n):
            r = own[k % len(own)].copy()
            r[3] += 0.01 * (k // len(own))
            rows.append(r)
    return np.array(rows)


@pytest.mark.parametrize("q0", [[0.794, -0.812, -2.66, -3.022, 1.815, 3.424, 0.618],
                                [1.638, 1.227, 0.041, -3.039, 0.047, 1.228, 0.314]])
def test_self_collision_odd_groups(oracle_lib, q0):
    """A sphere model whose self-collision groups hold one to four spheres and
    whose partner ranges have odd lengths, so that the kernel's last round of
    a group tests a single partner; folded starts so that pairs penetrate."""
    prob = inputs.config2(27, n_particles=96, horizon=30, n_obs_spheres=6, n_obs_cuboids=4)
    prob.spheres = _odd_sphere_model()
    prob.q0 = np.array(q0)
    g, ro, up, o, _ = run_pair(prob, oracle_lib)
    _config2_checks(g, ro, o, prob)
    assert np.mean(ro["terms"][..., 6] > 0) > 0.05, "the start should self-collide"


@pytest.mark.parametrize("q_near", [[0.794, -0.812, -2.66, -3.022, 1.815, 3.424, 0.618],
                                    [1.635, -1.566, 2.819, -2.644, 0.923, 0.507, -0.996],
                                    [1.638, 1.227, 0.041, -3.039, 0.047, 1.228, 0.314]])
def test_self_collision_grazing(oracle_lib, q_near):
    """Start states at the edge of self-contact: on the segment from the
    ready configuration (apart) to a folded one (penetrating), bisection with
    the oracle's signed self distance finds the point of 0.2 mm penetration,
    and small noise (sigma 0.01 rad) keeps the rollouts within millimetres of
    contact on both sides.  The self-collision term, whose pair work the
    kernel culls per (group, body) item, must equal the oracle's (which tests
    every pair) at every point, penetrations of micrometres included."""
    prob = inputs.config2(29, n_particles=128, horizon=30, n_obs_spheres=0, n_obs_cuboids=0)
    o = oracle_lib.Oracle(prob)
    qa, qb = inputs.PANDA_READY.copy(), np.array(q_near)
    assert o.self_distance(qa) < 0.0 < o.self_distance(qb)
    lo, hi = 0.0, 1.0
    for _ in range(50):
        mid = 0.5 * (lo + hi)
        if o.self_distance(qa + mid * (qb - qa)) < 2e-4:
            lo = mid
        else:
            hi = mid
    prob.q0 = qa + hi * (qb - qa)
    prob.params.sigma_init = np.full(7, 0.01)
    g, ro, up, o, _ = run_pair(prob, oracle_lib)
    s_g, s_o = g["terms"][..., 6], ro["terms"][..., 6]
    touching = s_o > 0.0
    assert 0.5 < touching.mean() < 0.95, "the rollouts should stay near contact on both sides"
    assert np.mean(touching & (s_o < 1e-3)) > 0.3, "many penetrations below a millimetre"
    # FP32 kinematics and distances err by a fraction of a micrometre; a pair the
    # broad phase wrongly skipped would lose its whole penetration (up to
    # millimetres here)
    err = np.abs(s_g - s_o)
    print("grazing self contact: %.0f%% of states touching, max |error| %.2g m" % (100 * touching.mean(), err.max()))
    assert np.max(err) <= 2e-6, "max self-term error %.3g m" % np.max(err)  # measured 1.5e-7


def test_sweeping_trajectories_dense_scene(oracle_lib):
    """Rollouts that sweep far over a long horizon (start velocity 2 rad/s,
    H = 64, 100 obstacles in a metre cube): the wave's bounding ball of a
    body sphere then meets most obstacles, so the broad phase refines it into
    eight balls of eight lanes.  Every term must still equal the oracle's."""
    prob = inputs.config5_problem(0)
    prob.params.n_particles, prob.params.n_halton = 96, 48
    prob.params.sigma_init = np.full(7, 0.03)
    v = np.random.default_rng(77).normal(size=7)
    prob.v0 = 2.0 * v / np.linalg.norm(v)
    g, ro, up, o, _ = run_pair(prob, oracle_lib)
    _config2_checks(g, ro, o, prob)
    e_g, e_o = g["terms"][..., 7], ro["terms"][..., 7]
    print("sweeping: %.0f%% of states touch an obstacle, max |env error| %.2g m" %
          (100 * np.mean(e_o > 0), np.max(np.abs(e_g - e_o))))
    assert np.mean(e_o > 0) > 0.2, "the sweeping rollouts should meet obstacles"
    assert np.max(np.abs(e_g - e_o)) <= 2e-5 * max(1.0, float(np.max(e_o)))
