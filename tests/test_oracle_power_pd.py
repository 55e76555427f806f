"""Pins of the oracle's power method and Algorithm 1."""
import numpy as np
import pytest
from scipy.optimize import minimize

import synth
from oracle import metrics, pd, power
from oracle.measurement import Measurement
from oracle.wavelets import Sara


def test_power_method_matches_svd():
    rng = np.random.default_rng(1)
    A = rng.standard_normal((30, 20))
    nrm, _ = power.power_method(lambda x: A.T @ (A @ x), rng.standard_normal(20), tol=1e-13, max_it=5000)
    assert nrm == pytest.approx(np.linalg.norm(A, 2), rel=1e-9)


def test_phi_norm_matches_svd_of_assembled_real_operator():
    rng = np.random.default_rng(2)
    n, M = 8, 60
    uv = (rng.standard_normal((M, 2)) * np.pi / 4).clip(-3.1, 3.1).astype(np.float32)
    m = Measurement(uv, [0, 30, M], (n, n))
    P = np.stack([m.phi(e.reshape(n, n)) for e in np.eye(n * n)], axis=1)
    ref = np.linalg.norm(np.vstack([P.real, P.imag]), 2)      # Phi on real images
    nrm, _ = power.phi_norm(m, rng.standard_normal((n, n)), tol=1e-13, max_it=5000)
    assert nrm == pytest.approx(ref, rel=1e-8)


def _tiny_problem(seed=3, n=8, M=40):
    rng = np.random.default_rng(seed)
    uv = (rng.standard_normal((M, 2)) * np.pi / 4).clip(-3.1, 3.1).astype(np.float32)
    meas = Measurement(uv, [0, M // 2, M], (n, n))
    sara = Sara(n, levels=1, wavelets=(1, 2))
    x_true = np.zeros((n, n))
    x_true[2, 3] = 1.0
    x_true[5, 5] = 0.5
    x_true[4:6, 1:3] += 0.3
    y0 = meas.phi(x_true)
    sig = 0.05 * np.linalg.norm(y0) / np.sqrt(M)
    y = y0 + sig / np.sqrt(2) * (rng.standard_normal(M) + 1j * rng.standard_normal(M))
    eps = np.array([np.linalg.norm((y - y0)[: M // 2]), np.linalg.norm((y - y0)[M // 2:])])
    pn, _ = power.psi_norm(sara, rng.standard_normal((n, n)))
    fn, _ = power.phi_norm(meas, rng.standard_normal((n, n)))
    return meas, sara, x_true, y, eps, pd.default_params(pn, fn)


def _slsqp_solution(meas, sara, y, eps):
    """min ||Psi^dagger x||_1 s.t. ||Phi_i x - y_i|| <= eps_i, x >= 0, by SLSQP on (x, t)."""
    n = meas.ny
    N = n * n
    Phi = np.stack([meas.phi(e.reshape(n, n)) for e in np.eye(N)], axis=1)
    W = np.stack([sara.adj(e.reshape(n, n)).ravel() for e in np.eye(N)], axis=1)
    B = W.shape[0]
    cons = [{"type": "ineq", "fun": lambda z: z[N:] - W @ z[:N], "jac": lambda z: np.hstack([-W, np.eye(B)])},
            {"type": "ineq", "fun": lambda z: z[N:] + W @ z[:N], "jac": lambda z: np.hstack([W, np.eye(B)])}]
    for i in range(meas.d):
        lo, hi = meas.block_range(i)
        Ar = np.vstack([Phi[lo:hi].real, Phi[lo:hi].imag])
        yr = np.concatenate([y[lo:hi].real, y[lo:hi].imag])
        cons.append({"type": "ineq",
                     "fun": lambda z, Ar=Ar, yr=yr, e=eps[i]: e * e - np.sum((Ar @ z[:N] - yr) ** 2),
                     "jac": lambda z, Ar=Ar, yr=yr: np.concatenate([-2 * Ar.T @ (Ar @ z[:N] - yr), np.zeros(B)])})
    z0 = np.concatenate([np.full(N, 0.1), np.full(B, 1.0)])
    res = minimize(lambda z: z[N:].sum(), z0, jac=lambda z: np.concatenate([np.zeros(N), np.ones(B)]),
                   constraints=cons, bounds=[(0, None)] * N + [(None, None)] * B, method="SLSQP",
                   options={"maxiter": 3000, "ftol": 1e-14})
    return res.x[:N].reshape(n, n), res.fun


def test_pd_converges_to_the_constrained_minimiser():
    meas, sara, x_true, y, eps, prm = _tiny_problem()
    assert prm.condition(1.0 / np.sqrt(prm.varsigma)) < 1.0
    x_ref, f_ref = _slsqp_solution(meas, sara, y, eps)
    st, _ = pd.run(meas, sara, y, eps, prm, np.ones((1500, meas.d), bool))
    assert metrics.l1_analysis(sara, st.x) == pytest.approx(f_ref, rel=1e-6)
    assert np.all(metrics.ball_ratio(meas, st.x, y, eps) <= 1 + 1e-6)
    assert np.linalg.norm(st.x - x_ref) <= 1e-4 * np.linalg.norm(x_ref)


def test_pd_invariants_every_iteration():
    meas, sara, x_true, y, eps, prm = _tiny_problem(seed=5)
    yb = pd.split_blocks(meas, y)
    st = pd.init_state(meas, sara)
    rng = np.random.default_rng(0)
    for t in range(60):
        mask = rng.uniform(size=meas.d) < 0.6
        before = st.copy()
        stats = pd.iteration(meas, sara, yb, eps, prm, st, mask)
        assert np.all(st.x >= 0)
        assert np.abs(st.s).max() <= prm.alpha * (1 + 1e-9)   # z - S(z) in FP64 rounding
        for i in range(meas.d):
            if not mask[i]:                       # step 11
                assert np.array_equal(st.v[i], before.v[i]) and np.array_equal(st.vt[i], before.vt[i])
                assert np.isnan(stats[i]).all()
            elif stats[i, 0] <= eps[i]:           # inside the ball: the dual vanishes
                assert np.abs(st.v[i]).max() == 0.0
        assert np.array_equal(st.xt, 2 * st.x - before.x)


def test_zero_is_the_solution_when_the_balls_hold_the_origin():
    meas, sara, _, y, _, prm = _tiny_problem(seed=6)
    eps = np.array([np.linalg.norm(b) for b in pd.split_blocks(meas, y)]) * 1.01
    st, _ = pd.run(meas, sara, y, eps, prm, np.ones((20, meas.d), bool))
    assert np.abs(st.x).max() == 0.0


def test_mask_of_ones_equals_deterministic_run_and_adaptive_path():
    meas, sara, x_true, y, eps, prm = _tiny_problem(seed=7)
    st1, _ = pd.run(meas, sara, y, eps, prm, np.ones((30, meas.d), bool))
    # the adaptive driver with p = 1 everywhere (n = d = p_max) activates every block
    st2, _, masks, probs = pd.run_adaptive(meas, sara, y, eps, prm, np.random.default_rng(0).random((30, meas.d)),
                                           n_nodes=float(meas.d), p_min=0.5, p_max=1.0)
    assert masks.all() and np.allclose(probs, 1.0)
    assert np.array_equal(st1.x, st2.x)


def test_small_workload_trends():
    # the smallest synthetic workload, shortened: SNR rises, data fidelity approaches the balls
    w = synth.WORKLOADS["n64_m8k_d4"]
    inp = synth.make_inputs(w)
    meas = Measurement(inp.uv, inp.block_off, (w.n, w.n))
    sara = Sara(w.n)
    y, _, eps = synth.add_noise(w, meas.phi(inp.x_true), inp.block_off)
    fn, _ = power.phi_norm(meas, synth.power_start(w.n, w.seed(synth.SEED_POWER)), tol=1e-6)
    prm = pd.default_params(3.0, fn)
    st, hist = pd.run(meas, sara, y, eps, prm, np.ones((60, meas.d), bool), x_true=inp.x_true)
    s = [h["snr"] for h in hist]
    assert s[-1] > s[5] > 0.0
    assert s[-1] > 10.0
    assert np.max(metrics.ball_ratio(meas, st.x, y, eps)) < 3.0


def test_residual_norms_against_the_direct_dft():
    """Eq. 13's residual ||Phi_i x - y_i||: zero image gives ||y_i|| exactly; data made by
    the direct non-uniform DFT plus a known per-block offset gives that offset's norm, to
    the kernel's interpolation accuracy (Phi matches the direct DFT to < 1e-6)."""
    from oracle.measurement import nudft

    rng = np.random.default_rng(11)
    n, M = 16, 300
    uv = (rng.standard_normal((M, 2)) * np.pi / 4).clip(-3.1, 3.1).astype(np.float32)
    meas = Measurement(uv, [0, 100, 220, M], (n, n))
    x = np.abs(rng.standard_normal((n, n)))
    delta = 0.1 * (rng.standard_normal(M) + 1j * rng.standard_normal(M))
    y = nudft(x, uv) + delta
    yb = pd.split_blocks(meas, y)
    r0 = pd.residual_norms(meas, np.zeros((n, n)), yb)
    assert np.array_equal(r0, np.array([np.linalg.norm(b) for b in yb]))
    r = pd.residual_norms(meas, x, yb)
    ref = np.array([np.linalg.norm(b) for b in pd.split_blocks(meas, delta)])
    scale = np.array([np.linalg.norm(b) for b in pd.split_blocks(meas, nudft(x, uv))])
    assert np.all(np.abs(r - ref) <= 2e-6 * scale)


def test_adaptive_refresh_takes_eq13_at_the_primal_iterate():
    """With refresh_every = K, the probabilities of iteration K come from Eq. 13 evaluated
    at x^(K) for every block: recomputed here from the direct DFT residual of the x reached
    by replaying the same masks, then Eq. 14."""
    from oracle.measurement import nudft
    from oracle.probs import adaptive_probabilities, residual_energy

    meas, sara, x_true, y, eps, prm = _tiny_problem(seed=12, n=8, M=60)
    K, T = 3, 5
    u = np.random.default_rng(5).random((T, meas.d))
    st, _, masks, probs = pd.run_adaptive(meas, sara, y, eps, prm, u, n_nodes=1.2, p_min=0.3, p_max=1.0,
                                          refresh_every=K)
    st_k, _ = pd.run(meas, sara, y, eps, prm, masks[:K])
    resid = y - nudft(st_k.x, meas.uv.astype(np.float32))
    rn = np.array([np.linalg.norm(b) for b in pd.split_blocks(meas, resid)])
    p_ref, _ = adaptive_probabilities(residual_energy(rn, eps), 1.2, 0.3, 1.0)
    assert np.allclose(probs[K], p_ref, rtol=1e-4, atol=1e-6)
    # without the refresh the probabilities of iteration K differ (inactive blocks' c_i stale
    # or taken at x~ rather than x)
    _, _, _, probs0 = pd.run_adaptive(meas, sara, y, eps, prm, u, n_nodes=1.2, p_min=0.3, p_max=1.0)
    assert not np.allclose(probs0[K], p_ref, rtol=1e-4, atol=1e-6)
