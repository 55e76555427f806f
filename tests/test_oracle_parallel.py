"""The oracle's optional thread pool changes nothing: an iteration of Algorithm 1 and the
SARA pair give bitwise the same results with one worker and with four."""
import numpy as np

import synth
from oracle import parallel
from oracle import pd as opd
from oracle.measurement import Measurement
from oracle.wavelets import Sara


def _run(workers):
    parallel.set_workers(workers)
    try:
        rng = np.random.default_rng(3)
        n, M, d = 32, 3000, 5
        x = synth.sky(n, 3, 5, rng)
        uv, off, _ = synth.partition(synth.uv_coverage(M, rng), d, "equal")
        meas = Measurement(uv, off, (n, n))
        sara = Sara(n, 3)
        y = meas.phi(x) + 0.01 * (rng.standard_normal(M) + 1j * rng.standard_normal(M))
        eps = np.full(d, 0.2)
        prm = opd.default_params(3.0, 60.0)
        masks = rng.uniform(size=(4, d)) < 0.6
        st, _ = opd.run(meas, sara, y, eps, prm, masks)
        return st, sara.adj(x), sara.fwd(sara.adj(x))
    finally:
        parallel.set_workers(1)


def test_thread_pool_is_bitwise_neutral():
    a, b = _run(1), _run(4)
    assert np.array_equal(a[0].x, b[0].x) and np.array_equal(a[0].s, b[0].s)
    assert all(np.array_equal(u, v) for u, v in zip(a[0].v, b[0].v))
    assert np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])
