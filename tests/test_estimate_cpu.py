"""Host logic of the parameter-estimation driver: the limited-memory BFGS
with Armijo backtracking (no GPU)."""
import numpy as np

from paper_2207_00426_amd.estimate import lbfgs


def _rosen(x):
    f = 100.0 * (x[1] - x[0] ** 2) ** 2 + (1.0 - x[0]) ** 2
    g = np.array([-400.0 * x[0] * (x[1] - x[0] ** 2) - 2.0 * (1.0 - x[0]),
                  200.0 * (x[1] - x[0] ** 2)])
    return f, g


def test_lbfgs_solves_rosenbrock():
    x, f, trace = lbfgs(_rosen, [-1.2, 1.0], n_steps=200)
    assert np.allclose(x, [1.0, 1.0], atol=1e-5) and f < 1e-10
    fs = [t[0] for t in trace]
    assert all(b <= a for a, b in zip(fs, fs[1:]))  # monotone under Armijo


def test_lbfgs_badly_scaled_quadratic_with_approximate_gradient():
    # curvatures 1 and 1e4 (like log q vs log sigma); the gradient carries a
    # 5% relative error but stays a descent direction
    H = np.diag([1.0, 1e4])
    xs = np.array([0.3, -0.2])

    def fg(x):
        r = x - xs
        g = H @ r
        return 0.5 * r @ H @ r, g * np.array([1.05, 0.95])

    x, f, trace = lbfgs(fg, [2.0, 1.0], n_steps=60, max_step=1.0)
    assert np.linalg.norm(x - xs) < 1e-3
    assert len(trace) <= 61
