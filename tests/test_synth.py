"""The seeded input generator: shapes, distributions and determinism (no method arithmetic)."""
import numpy as np

import bsh_synth as S


def test_velocity_magnitude_bounded():
    t = np.linspace(0, 2 * S.YEAR, 5000)
    for d in (0, 1):
        v = S.velocity_over_c(t, d)
        n = np.linalg.norm(v, axis=1)
        assert n.max() <= S.V_ORBIT + S.V_SPIN + 1e-18
        assert n.min() >= S.V_ORBIT - S.V_SPIN - 1e-18


def test_config2_shapes_and_gaps():
    w = S.config2()
    seg = w.segments[0]
    assert seg.n_seg == 4000 and seg.power.shape == (4000, 134) and seg.k_lo == 180000 - 22
    assert abs(float(seg.weight.mean()) - 1.0) < 1e-6
    starts = seg.t_mid - 0.5 * S.T_COH
    for d in (0, 1):
        s = starts[seg.detector == d]
        assert np.all(np.diff(s) >= S.T_COH)              # distinct Tc slots
        assert s.max() < 2858 * S.T_COH
    # Exp(1) powers: mean 1, P(rho > 1.6) = e^-1.6
    assert abs(float(seg.power.mean()) - 1.0) < 0.01
    assert abs(float((seg.power > 1.6).mean()) - np.exp(-1.6)) < 0.005


def test_generator_is_deterministic():
    a, b = S.config1(), S.config1()
    assert np.array_equal(a.segments[0].power, b.segments[0].power)
    assert np.array_equal(a.segments[0].t_mid, b.segments[0].t_mid)
    c3a = S.config3(build_items=[5])
    c3b = S.config3(build_items=[5, 6])
    assert np.array_equal(c3a.segments[5].power, c3b.segments[5].power)
    n = c3a.segments[5].n_seg
    assert 3000 <= n <= 6000


def test_fibonacci_sphere_unit_and_spread():
    s = S.fibonacci_sphere(256)
    assert np.allclose(np.linalg.norm(s, axis=1), 1.0)
    assert abs(s.mean(axis=0)).max() < 0.01


def test_injection_raises_mean_power():
    rng = np.random.default_rng(0)
    pw = np.ones((20000, 3), np.float32)
    pw[:] = rng.exponential(1.0, pw.shape)
    cols = np.full(20000, 1)
    cols[::2] = -1
    S.inject(pw, np.random.default_rng(1), [cols, np.full(20000, 1)], [2.0, 1.5])
    assert abs(float(pw[1::2, 1].mean()) - 4.5) < 0.1    # two signals on one bin add SNRs
    assert abs(float(pw[0::2, 1].mean()) - 2.5) < 0.1
    assert abs(float(pw[:, 0].mean()) - 1.0) < 0.05      # untouched bins keep Exp(1)
