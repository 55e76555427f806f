"""Reweighted SARA on the GPU (ri_pd_reweight, RI_PD_W) against the oracle's weighted l1
prior (oracle/reweight.py): the weights, a reweighted run of Algorithm 1, and the state
handling of the weights."""
import numpy as np
import pytest
import torch

import synth
from helpers import problem, rel_l2, to_plan
from oracle import pd as opd
from oracle.measurement import Measurement
from oracle.metrics import snr
from oracle.power import phi_norm as oracle_phi_norm
from oracle.reweight import run_reweighted, weights
from oracle.wavelets import Sara as OSara

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    import paper_1610_08895_amd as R

    assert torch.cuda.is_available()
    return R


def _setup(R, n=64, M=8192, d=4, seed=31):
    x, uv, off = problem(n, M, d, "equal", seed)
    meas = Measurement(uv, off, (n, n))
    y0 = meas.phi(x)
    sig = synth.noise_sigma(y0, 30.0)
    y = y0 + synth.complex_noise(M, sig, np.random.default_rng(seed + 1))
    eps = synth.l2_ball_radii(off, sig)
    phin, _ = oracle_phi_norm(meas, synth.power_start(n, seed), tol=0.0, max_it=100)
    plan = R.Plan(n, uv, off)
    y_plan = torch.tensor(to_plan(y, plan.order()), dtype=torch.complex64, device="cuda")
    return dict(x=x, meas=meas, y=y, eps=eps, phin=phin, plan=plan, y_plan=y_plan, n=n, d=d)


def _solver(R, S):
    from paper_1610_08895_amd.solver import Solver

    return Solver(S["plan"], R.Sara(S["n"]), S["y_plan"], S["eps"], 3.0, S["phin"])


@pytest.mark.parametrize("delta", [1e-3, 0.05, 2.0])
def test_weights_match_oracle(R, delta):
    S = _setup(R)
    sol = _solver(R, S)
    rng = np.random.default_rng(7)
    x = np.abs(synth.sky(S["n"], 5, 10, rng)).astype(np.float32)
    sol.pd.set(0, torch.tensor(x, device="cuda"))
    assert not sol.pd.weighted
    sol.pd.reweight(delta)
    assert sol.pd.weighted
    w = sol.pd.get(6).cpu().numpy().astype(np.float64)
    c_ref = np.abs(OSara(S["n"]).adj(x.astype(np.float64)))
    ref = weights(OSara(S["n"]), x.astype(np.float64), delta)
    assert np.all((w > 0) & (w <= 1))
    # w is delta / (delta + |c|) of the FP32 coefficients c = Psi^dagger x: compare the
    # coefficient magnitudes the weights imply (FP32 Psi^dagger is good to ~1e-6 of max |c|),
    # and the weights themselves where they are insensitive to that rounding
    c_gpu = delta / w - delta
    assert np.max(np.abs(c_gpu - c_ref)) < 2e-6 * c_ref.max() + 1e-6 * delta
    flat = delta / (delta + c_ref) ** 2 * c_ref.max() < 10.0
    assert np.max(np.abs(w - ref)[flat]) < 1e-5


def test_reweighted_run_matches_oracle(R):
    """64x64, M = 8192, 4 blocks, p = 1: 90 iterations with the weights refreshed every 30
    (delta 0.02, then 0.01); the batched graph form and the plain form follow the oracle's
    reweighted run within 0.05 dB, with the final x within 1e-4."""
    from paper_1610_08895_amd.solver import Reweight

    S = _setup(R)
    T, every, d0, beta = 90, 30, 0.02, 0.5
    prm = opd.default_params(3.0, S["phin"])
    osara = OSara(S["n"])
    st, hist, deltas = run_reweighted(S["meas"], osara, S["y"], S["eps"], prm, np.ones((T, S["d"]), bool), every,
                                      d0, beta, x_true=S["x"])
    assert deltas == [0.02, 0.01]
    plain_ref, plain_hist = opd.run(S["meas"], osara, S["y"], S["eps"], prm, np.ones((T, S["d"]), bool),
                                    x_true=S["x"])
    print(f"oracle SNR plain {plain_hist[-1]['snr']:.3f} dB, reweighted {hist[-1]['snr']:.3f} dB")
    for form in ("graph", "plain"):
        sol = _solver(R, S)
        sol.run(T, refresh=0, graph=form == "graph", plain=form == "plain", reweight=Reweight(every, d0, beta))
        xg = sol.x()
        print(f"{form}: SNR {snr(S['x'], xg):.4f} dB, rel x {rel_l2(xg, st.x):.2e}")
        assert abs(snr(S["x"], xg) - hist[-1]["snr"]) <= 0.05
        assert rel_l2(xg, st.x) < 1e-4
        assert rel_l2(sol.pd.get(2).cpu().numpy(), st.s) < 1e-3
        wg = sol.pd.get(6).cpu().numpy()
        assert np.max(np.abs(wg - st.w)) < 1e-4
        assert np.all(np.abs(sol.pd.get(2).cpu().numpy()) <= 3e-3 * wg * (1 + 1e-6))


def test_weight_state_handling(R):
    from paper_1610_08895_amd import _lib as L

    S = _setup(R)
    sol = _solver(R, S)
    with pytest.raises(L.RIError):
        sol.pd.get(6)  # no weights yet
    b, n = 9, S["n"]
    ones = torch.ones(b, n, n, dtype=torch.float32, device="cuda")
    ref = _solver(R, S)
    sol.pd.set(6, ones)  # w = 1 is the plain prior: the same steps bitwise
    for _ in range(5):
        sol.pd.step()
        ref.pd.step()
    assert torch.equal(sol.pd.get(0), ref.pd.get(0)) and torch.equal(sol.pd.get(2), ref.pd.get(2))
    half = 0.5 * ones
    sol.pd.set(6, half)
    assert torch.equal(sol.pd.get(6), half)
    sol.pd.unweight()
    assert not sol.pd.weighted
    with pytest.raises(L.RIError):
        sol.pd.reweight(0.0)
    assert L.load().ri_pd_reweight(None, 1.0, None) == L.RI_EINVAL
