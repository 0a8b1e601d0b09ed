"""Pins of the environment-light prefiltering oracle (Sec. 5.4): the
compact-eps support angle against the lobe's own definition, its limits, the
box side N theta / pi, and the averaged query against explicit averages of a
reconstructed tensor."""
import math

import numpy as np

from oracle import cp_als, ndf, query, sg


def test_support_angle_is_where_the_lobe_equals_eps():
    rng = np.random.default_rng(1)
    lam = np.exp(rng.uniform(np.log(2.0), np.log(2000.0), 1000))
    amp = rng.uniform(0.31, 20.0, 1000)
    theta = sg.support_angle(lam, amp, 0.3)
    inside = (0.0 < theta) & (theta < math.pi)
    assert inside.sum() > 900
    assert np.allclose(sg.sg_value(lam[inside], amp[inside], theta[inside]), 0.3, rtol=1e-10)
    # monotone: above eps inside the support, below outside
    assert np.all(sg.sg_value(lam[inside], amp[inside], 0.999 * theta[inside]) > 0.3)
    assert np.all(sg.sg_value(lam[inside], amp[inside], 1.001 * theta[inside]) < 0.3)


def test_support_angle_limits():
    # amplitude equal to eps: support shrinks to the axis; weaker lobes clamp to 0
    assert sg.support_angle(10.0, 0.3, 0.3) == 0.0
    assert sg.support_angle(10.0, 0.1, 0.3) == 0.0
    # (ln eps - ln A) / lambda = -2 reaches the antipode; stronger lobes clamp to pi
    lam = 2.0
    amp = 0.3 * math.exp(4.0)
    assert abs(sg.support_angle(lam, amp, 0.3) - math.pi) < 1e-7
    assert sg.support_angle(lam, 10 * amp, 0.3) == math.pi
    # sharper lobes have narrower support
    th = sg.support_angle(np.array([10.0, 100.0, 1000.0]), 5.0)
    assert th[0] > th[1] > th[2] > 0


def test_box_side_is_n_theta_over_pi():
    N = 64
    theta = np.array([0.0, math.pi / 8, math.pi / 4, math.pi / 2, math.pi])
    # centre on a bin boundary's midpoint so the width in bins is exact
    h = np.zeros(theta.shape) + 1.0 / N       # the centre of bin N/2
    lo, hi = sg.box_bins(h, theta, N)
    width = hi - lo
    assert list(width) == [1, 9, 17, 33, 64]            # N theta / pi bins around the centre bin
    # zero width: the point query of the bin holding h
    lo, hi = sg.box_bins(np.array([-1.0, -0.99, 0.0, 0.999]), np.zeros(4), N)
    assert list(lo) == [0, 0, 32, 63] and list(hi) == [1, 1, 33, 64]


def test_query_sg_is_the_average_of_the_reconstructed_tensor_over_the_box():
    rng = np.random.default_rng(3)
    nu, nv, nl, N, R = 4, 3, 2, 16, 5
    F = [rng.random((n, R)) for n in (nu, nv, nl, N, N)]
    T = cp_als.reconstruct(*F)
    n = 300
    uvl = np.stack([rng.integers(0, nu, n), rng.integers(0, nv, n), rng.integers(0, nl, n)], axis=1)
    h = rng.uniform(-1.0, 1.0, (n, 2))
    lam = np.exp(rng.uniform(np.log(1.0), np.log(500.0), n))
    amp = rng.uniform(0.2, 10.0, n)
    got, q = sg.query_sg(F[0], F[1], F[2], query.cumulative(F[3]), query.cumulative(F[4]), uvl, h, lam, amp)
    for i in range(n):
        u, v, l, slo, shi, tlo, thi = q[i]
        assert 0 <= slo < shi <= N and 0 <= tlo < thi <= N
        assert abs(got[i] - T[u, v, l, slo:shi, tlo:thi].mean()) <= 1e-12 * T.max()
    # a whole-image box of a normalised NDF averages to 1 / N^2
    nxy = np.zeros((2, 2, 2))
    Tn = ndf.ndf_bruteforce(nxy, N, 0.05, 1)
    Fn = cp_als.cp_als(Tn, [np.ones((d, 1)) for d in (2, 2, 1, N, N)], iters=30)["factors"]
    avg, _ = sg.query_sg(Fn[0], Fn[1], Fn[2], query.cumulative(Fn[3]), query.cumulative(Fn[4]),
                         np.zeros((1, 3), dtype=np.int64), np.zeros((1, 2)), np.array([0.01]), np.array([1e6]))
    assert abs(avg[0] - 1.0 / N ** 2) < 1e-10
