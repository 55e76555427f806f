"""Block selection on the device (ri_sched_step): Algorithm 1 step 3 with the fixed or
Eq. 14 probabilities of Sec. IV, against the library's host Eq. 14 (itself pinned to the
oracle in test_abi.py) and against direct host draws; and the solver's host loop around
it (masks, graph replay, plain steps interleaved)."""
import numpy as np
import pytest
import torch

import synth
from helpers import rel_l2
from oracle.probs import adaptive_probabilities, residual_energy

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    import paper_1610_08895_amd as R

    assert torch.cuda.is_available()
    return R


def _sched(R, d, T, stats, **kw):
    from paper_1610_08895_amd.ops import DeviceSchedule

    eps = kw.pop("eps", np.ones(d))
    return DeviceSchedule(d, T, eps, stats, **kw)


@pytest.mark.parametrize("d,n,pmin,pmax", [(16, 4.0, 0.05, 0.5), (64, 16.0, 0.05, 0.5), (128, 32.0, 0.05, 0.5),
                                           (7, 2.0, 0.1, 0.9), (300, 30.0, 0.01, 0.2)])
def test_device_eq14_matches_host(R, d, n, pmin, pmax):
    from paper_1610_08895_amd._lib import SCHED_ADAPTIVE, SCHED_DRAW

    rng = np.random.default_rng(d)
    T = 5
    stats = torch.zeros(d, 2, dtype=torch.float64, device="cuda")
    u = rng.uniform(size=(T, d))
    for trial in range(3):
        c = rng.lognormal(0, 2, d) * (rng.uniform(size=d) < 0.7)
        if trial == 2:
            c[:] = 0.0  # sum c = 0: every p_i = n/d
        sc = _sched(R, d, T, stats, u=u, c0=c, n_nodes=n, p_min=pmin, p_max=pmax)
        for t in range(T):
            sc.step(SCHED_ADAPTIVE | SCHED_DRAW)
        p_dev = sc.p_log.cpu().numpy()
        p_host, _ = R.probabilities(c, n, pmin, pmax)
        p_orc, _ = adaptive_probabilities(c, n, pmin, pmax)
        assert np.allclose(p_dev, p_host[None, :], rtol=0, atol=1e-12)
        assert np.allclose(p_dev, p_orc[None, :], rtol=0, atol=1e-12)
        assert np.array_equal(sc.mask_log.cpu().numpy(), (u < p_dev).astype(np.uint8))
        assert int(sc.counter.item()) == T
        assert np.array_equal(sc.mask.cpu().numpy(), (u[T - 1] < p_dev[T - 1]).astype(np.uint8))


def test_device_update_and_refresh(R):
    """UPDATE refreshes c_i (Eq. 13) from the last step's statistics for the blocks of the
    last mask only, and not before the first draw; REFRESH sets every c_i."""
    from paper_1610_08895_amd._lib import SCHED_ADAPTIVE, SCHED_DRAW, SCHED_REFRESH, SCHED_UPDATE

    d, T = 10, 4
    rng = np.random.default_rng(3)
    eps = rng.uniform(0.5, 2.0, d)
    c0 = rng.uniform(0.0, 1.0, d)
    stats = torch.tensor(rng.uniform(0.1, 9.0, (d, 2)), dtype=torch.float64, device="cuda")
    res = torch.tensor(rng.uniform(0.1, 9.0, (d, 2)), dtype=torch.float64, device="cuda")
    masks = (rng.uniform(size=(T, d)) < 0.5).astype(np.uint8)
    sc = _sched(R, d, T, stats, stats_x=res, masks=masks, c0=c0, eps=eps, n_nodes=3.0, p_min=0.05, p_max=0.9)
    sc.step(SCHED_UPDATE)  # counter 0: nothing to update yet
    assert np.array_equal(sc.c.cpu().numpy(), c0)
    sc.step(SCHED_ADAPTIVE | SCHED_DRAW)  # iteration 0 draws masks[0]
    sc.step(SCHED_UPDATE)
    want = c0.copy()
    act = np.flatnonzero(masks[0])
    want[act] = residual_energy(np.sqrt(stats.cpu().numpy()[act, 1]), eps[act])
    assert np.allclose(sc.c.cpu().numpy(), want, rtol=1e-14, atol=0)
    sc.step(SCHED_REFRESH)
    assert np.allclose(sc.c.cpu().numpy(), residual_energy(np.sqrt(res.cpu().numpy()[:, 1]), eps), rtol=1e-14, atol=0)
    # replayed masks wrap modulo T
    for _ in range(T + 1):
        sc.step(SCHED_DRAW)
    assert int(sc.counter.item()) == T + 2
    assert np.array_equal(sc.mask.cpu().numpy(), masks[(T + 1) % T])


def test_device_schedule_rejects_bad_arguments(R):
    from paper_1610_08895_amd import _lib as L
    from paper_1610_08895_amd._lib import SCHED_ADAPTIVE, SCHED_DRAW

    d, T = 8, 2
    stats = torch.zeros(d, 2, dtype=torch.float64, device="cuda")
    sc = _sched(R, d, T, stats, u=np.zeros((T, d)), n_nodes=1.0, p_min=0.2, p_max=0.5)
    with pytest.raises(L.RIError):
        sc.step(SCHED_ADAPTIVE | SCHED_DRAW)  # p_min > n/d
    with pytest.raises(L.RIError):
        sc.step(64)
    assert L.load().ri_sched_step(None, SCHED_DRAW, None) == L.RI_EINVAL


def _solver_problem(R, d=16, seed=21):
    from helpers import problem
    from oracle.measurement import Measurement

    n, M = 64, 12000
    x, uv, off = problem(n, M, d, "equal", seed)
    meas = Measurement(uv, off, (n, n))
    y0 = meas.phi(x)
    sig = synth.noise_sigma(y0, 20.0)
    y = y0 + synth.complex_noise(M, sig, np.random.default_rng(seed))
    eps = synth.l2_ball_radii(off, sig)
    return n, uv, off, y, eps


def _solver(R, n, uv, off, y, eps):
    from paper_1610_08895_amd.solver import Solver

    plan = R.Plan(n, uv, off)
    y_plan = torch.tensor(y[plan.order()], dtype=torch.complex64, device="cuda")
    return Solver(plan, R.Sara(n), y_plan, eps, 3.0, 2000.0)


def test_run_without_uniforms_draws_blocks(R):
    """A schedule with p < 1 and no uniforms or masks draws seeded uniforms itself: the mean
    number of active blocks is about p d, and the batched and plain forms, with the same seed,
    draw the same masks."""
    from paper_1610_08895_amd.solver import Schedule

    n, uv, off, y, eps = _solver_problem(R)
    d, T = 16, 200
    a = _solver(R, n, uv, off, y, eps)
    h = a.run(T, Schedule("uniform", p=0.25), refresh=0, seed=5)
    m = np.array(h["masks"])
    assert m.shape == (T, d)
    mean = m.sum(1).mean()
    sd = np.sqrt(d * 0.25 * 0.75 / T)
    assert abs(mean - 0.25 * d) < 4 * sd, mean
    assert np.array_equal(m, (np.random.default_rng(5).random((T, d)) < 0.25).astype(np.uint8))
    b = _solver(R, n, uv, off, y, eps)
    hb = b.run(20, Schedule("uniform", p=0.25), refresh=0, seed=5, plain=True)
    assert np.array_equal(np.array(hb["masks"]), (np.random.default_rng(5).random((20, d)) < 0.25))
    c = _solver(R, n, uv, off, y, eps)
    hc = c.run(20, Schedule("uniform", p=0.25), refresh=0, seed=5, graph=True)
    b2 = _solver(R, n, uv, off, y, eps)
    h2 = b2.run(20, Schedule("uniform", p=0.25), refresh=0, seed=5)
    assert np.array_equal(np.array(hc["masks"]), np.array(h2["masks"]))
    assert rel_l2(c.x(), b2.x()) < 1e-6
    assert rel_l2(b.x(), b2.x()) < 1e-5  # plain and batched, same masks


def test_adaptive_graph_run_equals_eager(R):
    """The adaptive schedule with the exact Eq. 13 refresh every K iterations, replayed from
    two captured graphs, follows the eager run: same masks, same probabilities."""
    from paper_1610_08895_amd.solver import Schedule

    n, uv, off, y, eps = _solver_problem(R, seed=22)
    sch = Schedule("adaptive", n_nodes=4.0, p_min=0.05, p_max=0.5, refresh_every=5)
    u = synth.activity_uniforms(30, 16, 7)
    a = _solver(R, n, uv, off, y, eps)
    ha = a.run(30, sch, uniforms=u, refresh=16)
    b = _solver(R, n, uv, off, y, eps)
    hb = b.run(30, sch, uniforms=u, refresh=16, graph=True)
    assert np.array_equal(np.array(ha["masks"]), np.array(hb["masks"]))
    assert np.allclose(np.array(ha["p"]), np.array(hb["p"]), rtol=1e-9, atol=1e-12)
    assert rel_l2(a.x(), b.x()) < 1e-6
    # the host-driven plain form draws the same masks from the same probabilities
    c = _solver(R, n, uv, off, y, eps)
    hc = c.run(30, sch, uniforms=u, refresh=16, plain=True)
    assert np.allclose(np.array(hc["p"]), np.array(ha["p"]), rtol=1e-6, atol=1e-9)
    assert rel_l2(c.x(), a.x()) < 1e-5


def test_graph_plain_and_eager_steps_interleave(R):
    """Graph replays, plain per-block steps and eager steps, alternated on one solver, follow
    a solver that only takes eager steps (the per-block halo rings start from zero whatever
    the batched launches left in them)."""
    n, uv, off, y, eps = _solver_problem(R, d=6, seed=23)
    ref = _solver(R, n, uv, off, y, eps)
    mix = _solver(R, n, uv, off, y, eps)
    rng = np.random.default_rng(4)
    kinds = ["graph", "plain", "plain", "graph", "eager", "plain", "graph", "graph", "plain", "eager"]
    for t, kind in enumerate(kinds):
        mask = (rng.uniform(size=6) < 0.7).astype(np.uint8)
        ref.step(mask)
        mix.step(mask, graph=kind == "graph", plain=kind == "plain")
        torch.cuda.synchronize()
        assert rel_l2(mix.x(), ref.x()) < 1e-5, (t, kind)
        assert rel_l2(mix.pd.get(3).cpu().numpy(), ref.pd.get(3).cpu().numpy()) < 1e-5, (t, kind)
