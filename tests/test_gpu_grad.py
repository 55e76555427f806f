"""GPU differentiation against the FP64 oracle: autograd through Phi and Psi, and the
reverse sweep of unrolled Algorithm 1 (d SNR / d(tau, sigma), masks fixed).

Tolerances: relative 1e-5 for the operator gradients (FP32 against FP64, as for the
operators themselves); relative 2e-3 for the unrolled gradients, which are sums of
products over every iteration and step (the oracle's own gradients agree with central
differences to better than 1e-6)."""
import json
import os

import numpy as np
import pytest
import torch

import synth
from helpers import problem, rel_l2, to_plan
from oracle import grad as og
from oracle import pd as opd
from oracle.measurement import Measurement
from oracle.power import phi_norm as oracle_phi_norm
from oracle.wavelets import Sara as OSara

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def R():
    import paper_1610_08895_amd as R

    assert torch.cuda.is_available()
    return R


def test_phi_autograd_gives_the_data_fit_gradient(R):
    from paper_1610_08895_amd import autograd as AG

    n, M = 64, 8192
    x, uv, off = problem(n, M, 4, "equal", 11)
    plan = R.Plan(n, uv, off)
    order = plan.order()
    rng = np.random.default_rng(12)
    y = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    xt = torch.tensor(x, dtype=torch.float32, device="cuda", requires_grad=True)
    yt = torch.tensor(to_plan(y, order), dtype=torch.complex64, device="cuda")
    loss = 0.5 * (AG.phi(plan, xt) - yt).abs().pow(2).sum()
    loss.backward()
    ref = og.data_fit_grad(Measurement(uv, off, (n, n)), x, y)
    assert rel_l2(xt.grad.cpu().numpy(), ref) < 1e-5
    # phi_adj's backward is Phi: d/dy of <w, Re Phi^dagger y> = Phi w
    w = torch.tensor(rng.standard_normal((n, n)), dtype=torch.float32, device="cuda")
    ya = yt.clone().requires_grad_(True)
    (AG.phi_adj(plan, ya) * w).sum().backward()
    assert rel_l2(ya.grad.cpu().numpy(), plan.phi(w).cpu().numpy()) < 1e-6


def test_psi_autograd_gives_the_synthesis_fit_gradient(R):
    from paper_1610_08895_amd import autograd as AG

    n = 64
    sara = R.Sara(n)
    osara = OSara(n)
    rng = np.random.default_rng(13)
    s = rng.standard_normal((9, n, n))
    t = rng.standard_normal((n, n))
    st = torch.tensor(s, dtype=torch.float32, device="cuda", requires_grad=True)
    tt = torch.tensor(t, dtype=torch.float32, device="cuda")
    (0.5 * (AG.psi(sara, st) - tt).pow(2).sum()).backward()
    ref = osara.adj(osara.fwd(s) - t)
    assert rel_l2(st.grad.cpu().numpy(), ref) < 1e-5
    xt = tt.clone().requires_grad_(True)
    (AG.psi_adj(sara, xt) * st.detach()).sum().backward()
    assert rel_l2(xt.grad.cpu().numpy(), osara.fwd(s)) < 1e-5


def _unrolled(R, T=10, seed=21, n=64, M=6000, d=4, p=0.7):
    x, uv, off = problem(n, M, d, "lognormal", seed)
    meas = Measurement(uv, off, (n, n))
    y0 = meas.phi(x)
    sig = synth.noise_sigma(y0, 25.0)
    y = y0 + synth.complex_noise(M, sig, np.random.default_rng(seed + 1))
    eps = synth.l2_ball_radii(off, sig)
    phin, _ = oracle_phi_norm(meas, synth.power_start(n, seed), tol=0.0, max_it=80)
    prm = opd.default_params(3.0, phin)
    masks = np.random.default_rng(seed + 2).uniform(size=(T, d)) < p
    masks[0] = True
    plan = R.Plan(n, uv, off)
    yp = torch.tensor(to_plan(y, plan.order()), dtype=torch.complex64, device="cuda")
    return x, meas, y, eps, prm, masks, plan, yp


def _gpu_grad(R, plan, yp, eps, prm, masks, x, checkpoint):
    from paper_1610_08895_amd import autograd as AG

    params = torch.tensor([prm.tau, prm.sigma], dtype=torch.float64, requires_grad=True)
    xT = AG.unrolled_pd(params, plan, R.Sara(plan.n), yp, eps, prm.varsigma, prm.kappa, 3.0, 1.0 / np.sqrt(prm.varsigma),
                        masks, checkpoint=checkpoint)
    xtrue = torch.tensor(x, dtype=torch.float64, device="cuda")
    err = xtrue - xT.double()
    snr = 20.0 * torch.log10(xtrue.norm() / err.norm())
    snr.backward()
    return float(snr.detach()), params.grad.numpy().copy()


# The FP32 noise of the unrolled forward and reverse sweeps reaches both components of
# (dSNR/dtau, dSNR/dsigma) with about the same absolute size, so the error is bounded
# relative to the gradient's norm: observed at most 6e-6 of it (2.4e-5 absolute in a
# dSNR/dsigma of 0.09, next to a dSNR/dtau of 4.1).
GRAD_TOL = 3e-5


def _check_grad(g, ref):
    ref = np.asarray(ref, dtype=np.float64)
    err = np.abs(np.asarray(g, dtype=np.float64) - ref)
    assert np.all(err <= GRAD_TOL * np.linalg.norm(ref)), (g, ref, err / np.linalg.norm(ref))


@pytest.mark.parametrize("checkpoint", [5, 1, 10])
def test_unrolled_gradient_matches_oracle(R, checkpoint):
    """10 iterations with fixed random masks (p = 0.7), segments of 5, 1 and 10."""
    x, meas, y, eps, prm, masks, plan, yp = _unrolled(R)
    s_ref, dtau, dsig = og.unrolled_gradient(meas, OSara(64), y, eps, prm, masks, x)
    s_gpu, g = _gpu_grad(R, plan, yp, eps, prm, masks, x, checkpoint)
    print(f"SNR {s_gpu:.6f} / {s_ref:.6f}; dtau {g[0]:.7g} / {dtau:.7g}; dsigma {g[1]:.7g} / {dsig:.7g}")
    assert s_gpu == pytest.approx(s_ref, abs=1e-3)
    _check_grad(g, [dtau, dsig])


def test_unrolled_gradient_reference_512(R):
    """512 x 512, M = 2^20 in 32 blocks, p = 1, 20 iterations, checkpoints every 5: against
    the oracle's stored reverse-sweep gradient."""
    path = os.path.join(GOLDEN, "grad_reference_n512_m1m_d32.json")
    if not os.path.exists(path):
        pytest.skip("no stored reference gradient")
    ref = json.load(open(path))
    w = synth.WORKLOADS[ref["workload"]]
    inp = synth.make_inputs(w)
    meas = Measurement(inp.uv, inp.block_off, (w.n, w.n))
    y, sig, eps = synth.add_noise(w, meas.phi(inp.x_true), inp.block_off)
    assert np.allclose(eps, ref["eps"], rtol=1e-12)
    plan = R.Plan(w.n, inp.uv, inp.block_off)
    yp = torch.tensor(to_plan(y, plan.order()), dtype=torch.complex64, device="cuda")
    prm = opd.Params(tau=ref["tau"], sigma=ref["sigma"], varsigma=ref["varsigma"], kappa=ref["kappa"],
                     psi_norm=ref["psi_norm"])
    masks = np.ones((ref["iterations"], plan.d), bool)
    s_gpu, g = _gpu_grad(R, plan, yp, eps, prm, masks, inp.x_true, 5)
    print(f"SNR {s_gpu:.6f} / {ref['snr']:.6f}; dtau {g[0]:.7g} / {ref['dsnr_dtau']:.7g}; "
          f"dsigma {g[1]:.7g} / {ref['dsnr_dsigma']:.7g}")
    assert s_gpu == pytest.approx(ref["snr"], abs=1e-3)
    _check_grad(g, [ref["dsnr_dtau"], ref["dsnr_dsigma"]])
