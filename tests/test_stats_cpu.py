"""Checks of the chain statistics against closed forms (no GPU)."""
import numpy as np

from paper_1808_00128_amd import stats


def ar1(rho, n, reps, rng):
    x = np.zeros((reps, n))
    e = rng.standard_normal((reps, n))
    x[:, 0] = e[:, 0] / np.sqrt(1 - rho**2)
    for t in range(1, n):
        x[:, t] = rho * x[:, t - 1] + e[:, t]
    return x


def test_tau_int_ar1_closed_form():
    """AR(1) with coefficient rho has tau_int = (1 + rho) / (2 (1 - rho))."""
    rng = np.random.default_rng(0)
    for rho in (0.0, 0.5, 0.9):
        x = ar1(rho, 20000, 4, rng)
        tau, W, err = stats.tau_int(x)
        exact = (1 + rho) / (2 * (1 - rho))
        assert abs(tau - exact) < max(4 * err, 0.05 * exact), (rho, tau, exact, err)


def test_ess_iid():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((8, 5000))
    e = stats.ess(x)
    assert 0.8 * x.size < e < 1.25 * x.size


def test_total_variation_and_cost():
    p = np.array([0.5, 0.25, 0.25, 0.0])
    assert stats.total_variation(np.array([0, 0, 1, 2]), p) == 0.0
    assert abs(stats.total_variation(np.array([3, 3]), p) - 1.0) < 1e-15
    # C(z) for one triple d = 1: z_a z_b z_c / 2
    tri = np.array([[0, 1, 2]])
    x = np.array([0b000, 0b001, 0b011, 0b111], np.uint64)
    np.testing.assert_allclose(stats.qaoa_cost(x, tri, np.array([1])), [0.5, -0.5, 0.5, -0.5])
