"""CPU checks of the C ABI: the library loads, exports every declared symbol, and its
host-side entry points (Eqs. 13-14) agree with the oracle.  No GPU work is launched."""
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "ri.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ri_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    from paper_1610_08895_amd import _lib

    lib = _lib.load()
    names = _declared()
    assert len(names) >= 25
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(_lib.SIGNATURES), set(names) ^ set(_lib.SIGNATURES)
    assert lib.ri_version() >= 10000


@pytest.mark.parametrize("seed", range(5))
def test_probabilities_match_oracle(seed):
    import paper_1610_08895_amd as R
    from oracle.probs import adaptive_probabilities, residual_energy

    rng = np.random.default_rng(seed)
    d = 32
    c = rng.lognormal(0, 2, d) * (rng.uniform(size=d) < 0.7)
    for n, pmin, pmax in [(8.0, 0.05, 0.5), (4.0, 0.05, 1.0), (16.0, 0.1, 0.5), (2.0, 0.0625, 0.0625)]:
        p, a = R.probabilities(c, n, pmin, pmax)
        pr, ar = adaptive_probabilities(c, n, pmin, pmax)
        assert np.allclose(p, pr, rtol=0, atol=1e-12)
        assert p.sum() == pytest.approx(n, abs=1e-10)
    r = rng.uniform(0.5, 2.0, d)
    e = rng.uniform(0.5, 2.0, d)
    assert np.allclose(R.residual_energy(r, e), residual_energy(r, e), rtol=1e-14, atol=0)


def test_probabilities_reject_bad_input():
    import paper_1610_08895_amd as R
    from paper_1610_08895_amd._lib import RIError

    with pytest.raises(RIError):
        R.probabilities(np.ones(4), 3.0, 0.1, 0.5)
    with pytest.raises(RIError):
        R.probabilities(np.array([1.0, -1.0]), 1.0, 0.1, 0.9)
    p, a = R.probabilities(np.zeros(4), 2.0, 0.1, 0.9)
    assert np.allclose(p, 0.5) and a == 0.0
