"""The DDE-aware G on the GPU (ri_plan_dde) against the oracle's DDE-aware operator
(oracle/dde.py): Phi, Phi^dagger and Algorithm 1 steps, over several tiles, DDE widths,
ragged blocks and random masks.  Tolerance: relative l2 <= 1e-5 per operator output."""
import numpy as np
import pytest
import torch

import synth
from helpers import problem, rel_l2, to_plan, to_user
from oracle import pd as opd
from oracle.dde import DDEMeasurement
from oracle.measurement import Measurement
from oracle.wavelets import Sara as OSara

pytestmark = pytest.mark.gpu
TOL = 1e-5


@pytest.fixture(scope="module")
def R():
    import paper_1610_08895_amd as R

    assert torch.cuda.is_available()
    return R


@pytest.mark.parametrize("n,M,d,jd,tile", [(64, 8192, 4, 5, 32), (64, 6000, 3, 3, 16), (128, 20000, 5, 7, 64),
                                           (32, 1500, 2, 1, 32), (128, 30000, 7, 5, 32)])
def test_dde_phi_and_adjoint_match_oracle(R, n, M, d, jd, tile):
    x, uv, off = problem(n, M, d, "lognormal" if d > 2 else "equal", seed=jd + tile)
    rng = np.random.default_rng(n + jd)
    taps = synth.dde_taps(M, jd, rng, strength=0.3)
    dm = DDEMeasurement(Measurement(uv, off, (n, n)), taps)
    plan = R.Plan(n, uv, off, tile=tile)
    plan.set_dde(taps)
    order = plan.order()
    y = to_user(plan.phi(torch.tensor(x, dtype=torch.float32, device="cuda")).cpu().numpy(), order)
    assert rel_l2(y, dm.phi(x)) < TOL
    w = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    xa = plan.phi_adj(torch.tensor(to_plan(w, order), dtype=torch.complex64, device="cuda")).cpu().numpy()
    assert rel_l2(xa, dm.phi_adj_real(w)) < TOL
    # a block mask: only the masked blocks' rows and adjoints
    mask = np.zeros(d, np.uint8)
    mask[::2] = 1
    mk = torch.tensor(mask, device="cuda")
    xm = plan.phi_adj(torch.tensor(to_plan(w, order), dtype=torch.complex64, device="cuda"), mask=mk).cpu().numpy()
    assert rel_l2(xm, dm.phi_adj_real(w, blocks=np.flatnonzero(mask))) < TOL


def test_delta_dde_equals_the_plain_operator_and_removal(R):
    n, M = 64, 8000
    x, uv, off = problem(n, M, 4, "equal", seed=3)
    plan = R.Plan(n, uv, off)
    xt = torch.tensor(x, dtype=torch.float32, device="cuda")
    y0 = plan.phi(xt).cpu().numpy()
    taps = np.zeros((M, 3, 3), np.complex64)
    taps[:, 1, 1] = 1.0
    plan.set_dde(taps)
    y1 = plan.phi(xt).cpu().numpy()
    assert rel_l2(y1, y0) < 1e-6
    plan.set_dde(None)
    assert np.array_equal(plan.phi(xt).cpu().numpy(), y0)


def test_dde_adjoint_identity_512(R):
    """512^2, M = 2^20 in 32 blocks, jd = 5: <Phi x, y> = <x, Re Phi^dagger y> at full size."""
    w = synth.WORKLOADS["n512_m1m_d32"]
    inp = synth.make_inputs(w)
    plan = R.Plan(w.n, inp.uv, inp.block_off)
    plan.set_dde(synth.dde_taps(w.M, 5, np.random.default_rng(5)))
    g = torch.Generator(device="cuda").manual_seed(6)
    x = torch.rand(w.n, w.n, device="cuda", generator=g)
    yv = torch.randn(w.M, dtype=torch.complex64, device="cuda", generator=g)
    lhs = (plan.phi(x).to(torch.complex128).conj() * yv.to(torch.complex128)).sum().real
    rhs = (x.double() * plan.phi_adj(yv).double()).sum()
    assert float(abs(lhs - rhs) / abs(rhs)) < 1e-5


@pytest.mark.parametrize("plain", [False, True])
def test_dde_pd_iterations_match_oracle(R, plain):
    """Algorithm 1 on the DDE-aware operator, random masks with an empty active set, batched
    and plain per-block forms, against the oracle's Algorithm 1 on its DDE operator."""
    n, M, d = 64, 6000, 5
    x, uv, off = problem(n, M, d, "lognormal", seed=9)
    rng = np.random.default_rng(10)
    taps = synth.dde_taps(M, 5, rng, strength=0.3)
    dm = DDEMeasurement(Measurement(uv, off, (n, n)), taps)
    y0 = dm.phi(x)
    sig = synth.noise_sigma(y0, 30.0)
    y = y0 + synth.complex_noise(M, sig, rng)
    eps = synth.l2_ball_radii(off, sig)
    prm = opd.default_params(3.0, 80.0)
    plan = R.Plan(n, uv, off)
    plan.set_dde(taps)
    order = plan.order()
    pdg = R.PD(plan, R.Sara(n), torch.tensor(to_plan(y, order), dtype=torch.complex64, device="cuda"), eps,
               prm.tau, prm.sigma, prm.varsigma, prm.kappa, 3.0, 80.0)
    osara = OSara(n)
    yb = opd.split_blocks(dm, y)
    st = opd.init_state(dm, osara)
    stats = torch.zeros(d, 2, dtype=torch.float64, device="cuda")
    for t in range(12):
        mask = (rng.uniform(size=d) < 0.6).astype(np.uint8)
        if t == 0:
            mask[:] = 1
        if t == 6:
            mask[:] = 0
        ost = opd.iteration(dm, osara, yb, eps, prm, st, mask.astype(bool))
        if plain:
            pdg.step_plain(mask, stats)
        else:
            pdg.step(torch.tensor(mask, device="cuda"), stats)
        gst = np.sqrt(stats.cpu().numpy())
        for i in np.flatnonzero(mask):
            assert gst[i] == pytest.approx(ost[i], rel=1e-4), (t, i)
        assert rel_l2(pdg.get(0).cpu().numpy(), st.x) < 2e-5 * (1 + t), t
        vo = np.concatenate(st.v)
        if np.linalg.norm(vo) > 0:
            assert rel_l2(to_user(pdg.get(3).cpu().numpy(), order), vo) < 2e-5 * (1 + t), t
