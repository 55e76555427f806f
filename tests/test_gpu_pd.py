"""GPU parity of Algorithm 1 (ri_pd_step, ri_pd_step_plain) against the FP64 oracle.

Per-iteration states agree to FP32 rounding (relative l2 <= 1e-4 over a few tens of
iterations); the reconstruction SNR after a full run agrees within 0.05 dB."""
import numpy as np
import pytest
import torch

import synth
from helpers import problem, rel_l2, to_plan, to_user
from oracle import pd as opd
from oracle.measurement import Measurement
from oracle.metrics import snr
from oracle.power import phi_norm as oracle_phi_norm
from oracle.wavelets import Sara as OSara

# Relative error of the iterates (x, x~, s, v) against the oracle after t + 1 steps: the
# FP32 operators add about 1e-6 per step (observed at most 1.4e-6 (1 + t) on the random-mask
# runs below), which the next steps carry forward, so the bound grows linearly in t.
STATE_TOL = 1e-5

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    import paper_1610_08895_amd as R

    assert torch.cuda.is_available()
    return R


def _setup(R, n=64, M=8192, d=4, scheme="equal", seed=2, isnr=30.0, blobs=5, points=10, **tune):
    x, uv, off = problem(n, M, d, scheme, seed, blobs, points)
    meas = Measurement(uv, off, (n, n))
    osara = OSara(n)
    y0 = meas.phi(x)
    sig = synth.noise_sigma(y0, isnr)
    y = y0 + synth.complex_noise(M, sig, np.random.default_rng(seed + 100))
    eps = synth.l2_ball_radii(off, sig)
    phin, _ = oracle_phi_norm(meas, synth.power_start(n, seed), tol=0.0, max_it=100)
    prm = opd.default_params(3.0, phin)
    plan = R.Plan(n, uv, off, **tune)
    order = plan.order()
    sara = R.Sara(n)
    y_plan = torch.tensor(to_plan(y, order), dtype=torch.complex64, device="cuda")
    return dict(x=x, uv=uv, off=off, meas=meas, osara=osara, y=y, eps=eps, phin=phin, prm=prm, plan=plan,
                order=order, sara=sara, y_plan=y_plan)


def _pd(R, S):
    p = S["prm"]
    return R.PD(S["plan"], S["sara"], S["y_plan"], S["eps"], p.tau, p.sigma, p.varsigma, p.kappa, 3.0, S["phin"])


def _v_user(pdg, S):
    return to_user(pdg.get(3).cpu().numpy(), S["order"])


@pytest.mark.parametrize("plain,tune", [(False, {}), (True, {}), (False, {"slice_vis": 150, "bin": 64})])
def test_iterations_match_oracle_with_random_masks(R, plain, tune):
    """Batched, plain per-block, and batched with every tile split into slices of
    at most 150 visibilities (items of at most 64)."""
    S = _setup(R, n=64, M=6000, d=5, scheme="lognormal", seed=3, **tune)
    pdg = _pd(R, S)
    meas, osara = S["meas"], S["osara"]
    yb = opd.split_blocks(meas, S["y"])
    st = opd.init_state(meas, osara)
    rng = np.random.default_rng(4)
    stats = torch.zeros(5, 2, dtype=torch.float64, device="cuda")
    worst = 0.0
    for t in range(15):
        mask = (rng.uniform(size=5) < 0.6).astype(np.uint8)
        if t == 0:
            mask[:] = 1
        if t == 7:
            mask[:] = 0          # empty active set
        ost = opd.iteration(meas, osara, yb, S["eps"], S["prm"], st, mask.astype(bool))
        if plain:
            pdg.step_plain(mask, stats)
        else:
            pdg.step(torch.tensor(mask, device="cuda"), stats)
        gst = np.sqrt(stats.cpu().numpy())
        for i in range(5):
            if mask[i]:
                assert gst[i] == pytest.approx(ost[i], rel=1e-4), (t, i)
            else:
                assert np.isnan(gst[i]).all()
        errs = [rel_l2(pdg.get(0).cpu().numpy(), st.x), rel_l2(pdg.get(1).cpu().numpy(), st.xt),
                rel_l2(pdg.get(2).cpu().numpy(), st.s)]
        vo = np.concatenate(st.v)
        if np.linalg.norm(vo) > 0:
            errs.append(rel_l2(_v_user(pdg, S), vo))
        worst = max(worst, max(errs) / (1 + t))
        for k, e in enumerate(errs):
            assert e < STATE_TOL * (1 + t), (t, k, e)
    print(f"worst relative error of x, x~, s, v per iteration: {worst:.2e} x (1 + t)")


def test_light_units_in_the_step_match_oracle(R):
    """Sparse coverage (most tiles light, several blocks per tile) through masked and
    all-blocks steps of Algorithm 1 against the oracle."""
    n, M, d = 128, 4000, 6
    rng = np.random.default_rng(21)
    x = synth.sky(n, 5, 10, rng)
    uvs, off, _ = synth.partition(rng.uniform(-np.pi, np.pi, (M, 2)).astype(np.float32), d, "equal")
    meas = Measurement(uvs, off, (n, n))
    osara = OSara(n)
    y0 = meas.phi(x)
    sig = synth.noise_sigma(y0, 20.0)
    y = y0 + synth.complex_noise(M, sig, rng)
    eps = synth.l2_ball_radii(off, sig)
    prm = opd.default_params(3.0, 60.0)
    plan = R.Plan(n, uvs, off)
    order = plan.order()
    pdg = R.PD(plan, R.Sara(n), torch.tensor(to_plan(y, order), dtype=torch.complex64, device="cuda"), eps,
               prm.tau, prm.sigma, prm.varsigma, prm.kappa, 3.0, 60.0)
    yb = opd.split_blocks(meas, y)
    st = opd.init_state(meas, osara)
    worst = 0.0
    for t in range(8):
        mask = (rng.uniform(size=d) < 0.6).astype(np.uint8) if t % 2 else np.ones(d, np.uint8)
        opd.iteration(meas, osara, yb, eps, prm, st, mask.astype(bool))
        pdg.step(None if t % 2 == 0 else torch.tensor(mask, device="cuda"))
        errs = [rel_l2(pdg.get(0).cpu().numpy(), st.x)]
        vo = np.concatenate(st.v)
        if np.linalg.norm(vo) > 0:
            errs.append(rel_l2(to_user(pdg.get(3).cpu().numpy(), order), vo))
        worst = max(worst, max(errs) / (1 + t))
        assert max(errs) < 1e-4 * (1 + t), (t, errs)
    print(f"worst relative error of x, v per iteration: {worst:.2e} x (1 + t)")


def test_inactive_blocks_keep_their_duals_bitwise(R):
    S = _setup(R, n=64, M=6000, d=4, seed=5)
    pdg = _pd(R, S)
    for _ in range(3):
        pdg.step()
    v0 = pdg.get(3).cpu().numpy()
    mask = np.array([0, 1, 0, 1], np.uint8)
    pdg.step(torch.tensor(mask, device="cuda"))
    v1 = pdg.get(3).cpu().numpy()
    off = S["off"]
    for i in (0, 2):
        assert np.array_equal(v0[off[i]:off[i + 1]], v1[off[i]:off[i + 1]])


def test_batched_equals_plain(R):
    S = _setup(R, n=64, M=8192, d=6, scheme="lognormal", seed=6)
    a, b = _pd(R, S), _pd(R, S)
    rng = np.random.default_rng(0)
    for _ in range(12):
        mask = (rng.uniform(size=6) < 0.7).astype(np.uint8)
        a.step(torch.tensor(mask, device="cuda"))
        b.step_plain(mask)
    assert rel_l2(a.get(0).cpu().numpy(), b.get(0).cpu().numpy()) < 1e-5
    assert rel_l2(a.get(3).cpu().numpy(), b.get(3).cpu().numpy()) < 1e-5


@pytest.mark.parametrize("tune", [{}, {"slice_vis": 150, "bin": 64}])
def test_all_blocks_rebuild_equals_masked_update(R, tune):
    """A step without a mask (every block active: the grid sum rebuilt from the new duals,
    reading r only) and a step with an all-ones mask (the changes added to the kept sum)
    give the same iterates, also with tiles split into slices; both match the oracle."""
    S = _setup(R, n=64, M=8000, d=5, scheme="lognormal", seed=12, **tune)
    a, b = _pd(R, S), _pd(R, S)
    ones = torch.ones(5, dtype=torch.uint8, device="cuda")
    sa = torch.zeros(5, 2, dtype=torch.float64, device="cuda")
    sb = torch.zeros_like(sa)
    meas, osara = S["meas"], S["osara"]
    yb = opd.split_blocks(meas, S["y"])
    st = opd.init_state(meas, osara)
    worst = 0.0
    for t in range(10):
        a.step(None, sa)
        b.step(ones, sb)
        opd.iteration(meas, osara, yb, S["eps"], S["prm"], st, np.ones(5, bool))
        # the two differ by the FP32 rounding of the kept sum's updates only
        assert rel_l2(a.get(0).cpu().numpy(), b.get(0).cpu().numpy()) < 1e-5, t
        assert rel_l2(a.get(3).cpu().numpy(), b.get(3).cpu().numpy()) < 1e-5, t
        assert torch.allclose(sa, sb, rtol=1e-5)
        ea, eb = rel_l2(a.get(0).cpu().numpy(), st.x), rel_l2(b.get(0).cpu().numpy(), st.x)
        worst = max(worst, max(ea, eb) / (1 + t))
        assert ea < 1e-4 * (1 + t), t
        assert eb < 1e-4 * (1 + t), t
    assert rel_l2(a.get(5).cpu().numpy(), b.get(5).cpu().numpy()) < 1e-5
    print(f"worst relative error of x per iteration: {worst:.2e} x (1 + t)")


def test_snr_parity_small_workload(R):
    """The smallest workload (64x64, M = 8192, 4 blocks, p = 1, 200 iterations)."""
    w = synth.WORKLOADS["n64_m8k_d4"]
    inp = synth.make_inputs(w)
    meas = Measurement(inp.uv, inp.block_off, (w.n, w.n))
    y, sig, eps = synth.add_noise(w, meas.phi(inp.x_true), inp.block_off)
    phin, _ = oracle_phi_norm(meas, synth.power_start(w.n, w.seed(synth.SEED_POWER)), tol=0.0, max_it=100)
    prm = opd.default_params(3.0, phin)
    T = w.iterations
    st, hist = opd.run(meas, OSara(w.n), y, eps, prm, np.ones((T, w.d), bool), x_true=inp.x_true)
    plan = R.Plan(w.n, inp.uv, inp.block_off)
    order = plan.order()
    from paper_1610_08895_amd.solver import Solver

    sol = Solver(plan, R.Sara(w.n), torch.tensor(to_plan(y, order), dtype=torch.complex64, device="cuda"),
                 eps, 3.0, phin)
    sol.run(T, refresh=64)
    s_gpu, s_ref = snr(inp.x_true, sol.x()), hist[-1]["snr"]
    print(f"SNR oracle {s_ref:.4f} dB, GPU {s_gpu:.4f} dB")
    assert s_ref > 15.0
    assert abs(s_gpu - s_ref) <= 0.05


def test_adaptive_run_replays_oracle_masks(R):
    """Eq. 14 schedule (annuli blocks): GPU driven with the oracle's mask log."""
    S = _setup(R, n=64, M=12000, d=8, scheme="annuli", seed=8, isnr=20.0)
    T = 120
    u = synth.activity_uniforms(T, S["plan"].d, 99)
    st, hist, masks, probs = opd.run_adaptive(S["meas"], S["osara"], S["y"], S["eps"], S["prm"], u,
                                              n_nodes=3.0, p_min=0.05, p_max=0.8, x_true=S["x"])
    assert 0 < masks.sum() < masks.size
    from paper_1610_08895_amd.solver import Solver

    sol = Solver(S["plan"], S["sara"], S["y_plan"], S["eps"], 3.0, S["phin"])
    sol.run(T, masks=masks, refresh=32)
    assert abs(snr(S["x"], sol.x()) - hist[-1]["snr"]) <= 0.05
    # the first iteration's probabilities from Eq. 13 at x = 0 match the oracle's
    from paper_1610_08895_amd.solver import Schedule

    sol2 = Solver(S["plan"], S["sara"], S["y_plan"], S["eps"], 3.0, S["phin"])
    h2 = sol2.run(1, Schedule("adaptive", n_nodes=3.0, p_min=0.05, p_max=0.8), uniforms=u)
    assert np.allclose(h2["p"][0], probs[0], rtol=1e-6, atol=1e-9)


def test_refresh_and_checkpoint_resume(R):
    S = _setup(R, n=64, M=8192, d=4, seed=9)
    a = _pd(R, S)
    for _ in range(20):
        a.step()
    x_before = a.get(0).clone()
    a.refresh()
    saved = [a.get(w).clone() for w in (0, 1, 2, 3)]
    for _ in range(5):
        a.step()
    b = _pd(R, S)
    for w, v in zip((0, 1, 2, 3), saved):
        b.set(w, v)
    b.iteration = 20
    for _ in range(5):
        b.step()
    assert b.iteration == 25 == a.iteration
    assert rel_l2(a.get(0).cpu().numpy(), b.get(0).cpu().numpy()) < 1e-5
    assert torch.equal(saved[0], x_before)


def test_graph_replay_matches_eager(R):
    from paper_1610_08895_amd.solver import Solver

    S = _setup(R, n=64, M=8192, d=5, scheme="lognormal", seed=10)
    eager = Solver(S["plan"], S["sara"], S["y_plan"], S["eps"], 3.0, S["phin"])
    plan2 = R.Plan(64, S["uv"], S["off"])          # the graph baked in plan buffers of its own
    graph = Solver(plan2, R.Sara(64), S["y_plan"], S["eps"], 3.0, S["phin"])
    rng = np.random.default_rng(1)
    for t in range(8):
        mask = (rng.uniform(size=5) < 0.6).astype(np.uint8)
        eager.step(mask)
        graph.step(mask, graph=True)
        torch.cuda.synchronize()
        assert rel_l2(graph.x(), eager.x()) < 1e-5, t
        assert torch.allclose(graph.stats_dev.nan_to_num(-1), eager.stats_dev.nan_to_num(-1), rtol=1e-5)


def test_pd_residual_matches_oracle(R):
    """ri_pd_residual: ||Phi_i x - y_i||^2 and ||v_i + Phi_i x - y_i||^2 for every block at a
    seeded x and v; at x = 0 the first is the data's own per-block energy."""
    S = _setup(R, n=64, M=12000, d=8, scheme="annuli", seed=13, isnr=20.0)
    pdg = _pd(R, S)
    meas = S["meas"]
    yb = opd.split_blocks(meas, S["y"])
    rng = np.random.default_rng(14)
    x = np.abs(synth.sky(64, 5, 10, rng))
    v_user = 0.01 * (rng.standard_normal(meas.M) + 1j * rng.standard_normal(meas.M))
    pdg.set(0, torch.tensor(x, dtype=torch.float32, device="cuda"))
    pdg.set(3, torch.tensor(to_plan(v_user, S["order"]), dtype=torch.complex64, device="cuda"))
    out = pdg.residual().cpu().numpy()
    xf = x.astype(np.float32).astype(np.float64)
    ref1 = opd.residual_norms(meas, xf, yb) ** 2
    b_full = meas.F(meas.Z(xf))
    vb = opd.split_blocks(meas, v_user.astype(np.complex64))
    ref0 = np.array([np.linalg.norm(vb[i] + meas.Gi(i, meas.Mi(i, b_full)) - yb[i]) ** 2 for i in range(meas.d)])
    assert np.allclose(out[:, 1], ref1, rtol=1e-4)
    assert np.allclose(out[:, 0], ref0, rtol=1e-4)
    pdg.set(0, torch.zeros(64, 64, dtype=torch.float32, device="cuda"))
    out0 = pdg.residual().cpu().numpy()
    assert np.allclose(out0[:, 1], S["plan"].block_sumsq(S["y_plan"]).cpu().numpy(), rtol=1e-12)


def test_pd_residual_leaves_the_state(R):
    """A residual evaluation between two steps changes nothing the next step computes."""
    S = _setup(R, n=64, M=8192, d=4, seed=15)
    a, b = _pd(R, S), _pd(R, S)
    mask = torch.tensor([1, 0, 1, 1], dtype=torch.uint8, device="cuda")
    for pdg in (a, b):
        pdg.step()
        pdg.step(mask)
    e_before = a.get(5).clone()
    a.residual()
    assert torch.equal(a.get(5), e_before)
    for pdg in (a, b):
        pdg.step(mask)
    for which in (0, 1, 2, 3, 5):
        assert torch.equal(a.get(which), b.get(which)), which


def test_adaptive_refresh_matches_oracle(R):
    """Eq. 14 with c_i refreshed from Eq. 13 at x every K iterations: the GPU solver, driven
    with the oracle's mask log, computes the oracle's probabilities at every iteration."""
    from paper_1610_08895_amd.solver import Schedule, Solver

    S = _setup(R, n=64, M=12000, d=8, scheme="annuli", seed=8, isnr=20.0)
    T, K = 40, 8
    u = synth.activity_uniforms(T, S["plan"].d, 98)
    st, hist, masks, probs = opd.run_adaptive(S["meas"], S["osara"], S["y"], S["eps"], S["prm"], u, n_nodes=3.0,
                                              p_min=0.05, p_max=0.8, x_true=S["x"], refresh_every=K)
    sol = Solver(S["plan"], S["sara"], S["y_plan"], S["eps"], 3.0, S["phin"])
    h = sol.run(T, Schedule("adaptive", n_nodes=3.0, p_min=0.05, p_max=0.8, refresh_every=K), masks=masks,
                refresh=16)
    gp = np.array(h["p"])
    assert np.allclose(gp, probs, rtol=0, atol=2e-3)
    assert abs(snr(S["x"], sol.x()) - hist[-1]["snr"]) <= 0.05


def test_adaptive_run_survives_an_empty_active_set(R):
    """An iteration with no active block leaves every c_i unchanged (Eq. 13 has nothing new)."""
    from paper_1610_08895_amd.solver import Schedule, Solver

    S = _setup(R, n=64, M=8192, d=4, seed=16)
    sol = Solver(S["plan"], S["sara"], S["y_plan"], S["eps"], 3.0, S["phin"])
    masks = np.zeros((3, 4), np.uint8)
    masks[0] = 1
    h = sol.run(3, Schedule("adaptive", n_nodes=2.0, p_min=0.1, p_max=0.9), masks=masks)
    assert np.array_equal(h["p"][1], h["p"][2])


def test_pd_residual_with_split_tiles_and_bad_arguments(R):
    """The residual pass over all items also covers tiles split into slices; NULL arguments
    are rejected with an error code, and a wrongly shaped output by the binding."""
    from paper_1610_08895_amd import _lib as L

    S = _setup(R, n=64, M=6000, d=5, scheme="lognormal", seed=17, slice_vis=150, bin=64)
    pdg = _pd(R, S)
    rng = np.random.default_rng(18)
    x = np.abs(synth.sky(64, 5, 10, rng))
    pdg.set(0, torch.tensor(x, dtype=torch.float32, device="cuda"))
    out = pdg.residual().cpu().numpy()
    ref = opd.residual_norms(S["meas"], x.astype(np.float32).astype(np.float64), opd.split_blocks(S["meas"], S["y"]))
    assert np.allclose(out[:, 1], ref ** 2, rtol=1e-4)
    assert L.load().ri_pd_residual(None, None, None) == -1
    with pytest.raises(ValueError):
        pdg.residual(torch.empty(5, 3, dtype=torch.float64, device="cuda"))
