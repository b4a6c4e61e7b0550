"""The seeded input generators: determinism, shapes and value ranges."""
import numpy as np

from paper_2403_16341_amd import inputs


def test_config_determinism_and_layout():
    for k in (1, 2, 3, 4):
        a = inputs.config(k, M=257)
        b = inputs.config(k, M=257)
        assert np.array_equal(a.params, b.params) and np.array_equal(a.u0, b.u0)
        assert a.p_off[-1] == a.params.size and a.u_off[-1] == a.u0.size
        for s in (0, 100, 256):
            f, n, alg, p, u0 = a.system(s)
            assert p.size == inputs.nparams(f, n) and u0.size == n


def test_config_distributions():
    b = inputs.config(1, M=512)
    assert b.uniform() == (inputs.CUBIC, 4, inputs.NEWTON) and b.maxiters == 50
    assert np.all(b.u0 == 0)
    A = b.params.reshape(512, 20)[:, :16].reshape(512, 4, 4)
    d = A[:, np.arange(4), np.arange(4)]
    assert abs(d.mean() - 4.0) < 0.1
    b2 = inputs.config(2, M=512)
    assert b2.uniform() == (inputs.CUBIC, 8, inputs.ARMIJO) and b2.maxiters == 100
    assert b2.u0.min() >= -3 and b2.u0.max() <= 3
    b3 = inputs.config(3, M=512)
    assert b3.uniform() == (inputs.TANH, 16, inputs.DOGLEG)
    beta = b3.params.reshape(512, -1)[:, -1]
    assert beta.min() >= 0.05 and beta.max() <= 0.5
    b4 = inputs.config(4, M=20000)
    assert b4.uniform() is None
    freq = np.array([(b4.n == n).mean() for n in inputs.CFG4_NS])
    assert np.abs(freq - inputs.CFG4_WEIGHTS).max() < 0.02
    assert set(np.unique(b4.alg)) == {inputs.ARMIJO, inputs.DOGLEG}


def test_subset_and_concat_roundtrip():
    b = inputs.config(4, M=300)
    idx = np.array([5, 0, 299, 17])
    s = b.subset(idx)
    for j, i in enumerate(idx):
        x, y = s.system(j), b.system(i)
        assert x[:3] == y[:3] and np.array_equal(x[3], y[3]) and np.array_equal(x[4], y[4])
    c = inputs.concat([s, b])
    assert c.M == s.M + b.M and np.array_equal(c.system(4)[3], b.system(0)[3])


def test_serving_requests():
    reqs = inputs.serving_requests(20, rate_hz=100.0)
    assert len(reqs) == 20
    t = [r.arrival for r in reqs]
    assert all(t[i] <= t[i + 1] for i in range(19))
    for r in reqs:
        u = r.batch.uniform()
        assert 1 <= r.batch.M <= 65536 and 2 <= u[1] <= 64
