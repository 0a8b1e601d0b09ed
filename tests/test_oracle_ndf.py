"""Pins of the FP64 oracle's NDF tensor and range integral (CPU only)."""
import json
import math
import os

import mpmath
import numpy as np
import pytest

import gen
from oracle import ndf


# --------------------------------------------------------------------------
# bin masses: Eq. geom integrated over a bin, against high-precision quadrature
# --------------------------------------------------------------------------

def _mp_interval(a, b):
    mpmath.mp.dps = 40
    f = lambda x: mpmath.exp(-x * x / 2) / mpmath.sqrt(2 * mpmath.pi)
    return float(mpmath.quad(f, [a, b]))


@pytest.mark.parametrize("a,b", [(-0.3, 0.7), (1.0, 1.5), (5.0, 9.0), (-12.0, -9.5),
                                 (-40.0, 40.0), (0.0, 0.25), (7.9, 8.1)])
def test_gauss_interval_against_quadrature(a, b):
    got = float(ndf.gauss_interval(a, b))
    ref = _mp_interval(a, b)
    # libm-class erfc keeps ~1e-14 relative accuracy deep in the tails
    assert abs(got - ref) <= 5e-14 * max(ref, 1e-300) + 1e-300


def test_axis_masses_against_quadrature_of_the_gaussian():
    """Each bin mass is the integral of the sigma-Gaussian over the bin,
    divided by its integral over [-1, 1] (renormalised leak)."""
    mpmath.mp.dps = 40
    N, sigma = 8, 0.13
    for n in (-0.97, -0.31, 0.0, 0.52, 0.999):
        m = ndf.axis_masses(n, N, sigma)
        g = lambda x: mpmath.exp(-((x - n) / sigma) ** 2 / 2)
        Z = mpmath.quad(g, [-1, 1])
        for i in range(N):
            e0, e1 = -1 + i * 2 / N, -1 + (i + 1) * 2 / N
            ref = float(mpmath.quad(g, [e0, e1]) / Z)
            assert abs(m[i] - ref) <= 1e-14 + 1e-12 * ref
        assert abs(m.sum() - 1.0) < 1e-14


def test_bin_index_edges_go_up():
    N = 4
    # exact edges -1, -0.5, 0, 0.5, 1
    assert list(ndf.bin_index([-1.0, -0.5, 0.0, 0.5, 1.0], N)) == [0, 1, 2, 3, 3]
    assert list(ndf.bin_index([-0.5000001, 0.4999999, -2.0, 2.0], N)) == [0, 2, 0, 3]


# --------------------------------------------------------------------------
# hand-counted worked example (sigma -> 0)
# --------------------------------------------------------------------------

def _delta_map(golden_dir):
    with open(os.path.join(golden_dir, "delta_map_4x4.json")) as f:
        g = json.load(f)
    ix = np.array(g["ix"])
    iy = np.array(g["iy"])
    nxy = np.stack([-0.75 + 0.5 * ix, -0.75 + 0.5 * iy], axis=-1).astype(np.float32)
    return g, nxy


def test_delta_map_golden_tensor(golden_dir):
    g, nxy = _delta_map(golden_dir)
    T = ndf.ndf_bruteforce(nxy, g["nbins"], g["sigma"], g["nlevels"])
    ix, iy = np.array(g["ix"]), np.array(g["iy"])
    # level 0: one unit entry per texel
    for u in range(4):
        for v in range(4):
            want = np.zeros((4, 4))
            want[ix[u, v], iy[u, v]] = 1.0
            assert np.array_equal(T[u, v, 0], want)
    for cell in g["level1_cells"]:
        want = np.zeros((4, 4))
        for s, t, val in cell["entries"]:
            want[s, t] += val
        assert np.array_equal(T[cell["u"], cell["v"], 1], want), cell


def test_delta_map_golden_range_queries(golden_dir):
    g, nxy = _delta_map(golden_dir)
    q = np.array([r["q"] for r in g["range_queries"]])
    want = np.array([r["value"] for r in g["range_queries"]])
    got = ndf.range_bruteforce(nxy, g["nbins"], g["sigma"], g["nlevels"], q)
    assert np.array_equal(got, want)
    T = ndf.ndf_bruteforce(nxy, g["nbins"], g["sigma"], g["nlevels"])
    assert np.array_equal(ndf.box_sum(T, q), want)


# --------------------------------------------------------------------------
# invariants on the C1 flake map (64x64, N = 32, 5 levels)
# --------------------------------------------------------------------------

@pytest.fixture(scope="module")
def c1_tensor():
    cfg = gen.config("c1")
    nxy = gen.normal_map(cfg)
    T = ndf.ndf_bruteforce(nxy, cfg.nbins, cfg.sigma, cfg.nlevels)
    return cfg, nxy, T


def test_c1_nonnegative_and_unit_mass(c1_tensor):
    _, _, T = c1_tensor
    assert T.min() >= 0.0
    mass = T.sum(axis=(3, 4))
    assert np.max(np.abs(mass - 1.0)) < 1e-13


def test_c1_level_doubling_identity(c1_tensor):
    """A 2k box at u splits into two k boxes anchored at u - ceil(k/2) and
    u + floor(k/2), so T_{l+1} is the mean of four shifted T_l."""
    _, _, T = c1_tensor
    for l in range(T.shape[2] - 1):
        k = 1 << l
        a = [-((k + 1) // 2), k // 2]
        acc = np.zeros_like(T[:, :, l])
        for da in a:
            for db in a:
                acc += np.roll(np.roll(T[:, :, l], -da, axis=0), -db, axis=1)
        assert np.max(np.abs(acc / 4.0 - T[:, :, l + 1])) < 1e-14


def test_c1_spatial_mean_independent_of_level(c1_tensor):
    _, _, T = c1_tensor
    means = T.mean(axis=(0, 1))
    for l in range(1, T.shape[2]):
        assert np.max(np.abs(means[l] - means[0])) < 1e-15


def test_c1_level0_slices_are_rank_one(c1_tensor):
    _, _, T = c1_tensor
    for (u, v) in [(0, 0), (5, 17), (63, 40)]:
        sv = np.linalg.svd(T[u, v, 0], compute_uv=False)
        assert sv[1] <= 1e-14 * sv[0]


def test_constant_normal_map_is_outer_product_everywhere():
    nxy = np.zeros((8, 8, 2), dtype=np.float32)
    nxy[..., 0] = 0.1875
    nxy[..., 1] = -0.4
    T = ndf.ndf_bruteforce(nxy, 16, 0.05, 4)
    ms = ndf.axis_masses(0.1875, 16, 0.05)
    mt = ndf.axis_masses(np.float32(-0.4), 16, 0.05)
    want = np.outer(ms, mt)
    assert np.max(np.abs(T - want)) < 1e-15


def test_c1_range_bruteforce_equals_box_sum(c1_tensor):
    cfg, nxy, T = c1_tensor
    q = gen.make_queries(cfg, nxy, nq=400)
    qb = ndf.range_bruteforce(nxy, cfg.nbins, cfg.sigma, cfg.nlevels, q)
    bs = ndf.box_sum(T, q)
    assert np.max(np.abs(qb - bs)) < 1e-13
    assert np.count_nonzero(qb > 1e-3) > 40          # the batch is not all empty


def test_tiny_dropped_term_is_caught():
    """A plausible slip (forgetting the 1/k^2 weight) breaks unit mass."""
    nxy = gen.flake_map(8, 8, 5, 0.2, 3)
    T = ndf.ndf_bruteforce(nxy, 8, 0.05, 3)
    mass = T.sum(axis=(3, 4))
    assert np.allclose(mass, 1.0, atol=1e-14)
    assert not np.allclose(mass[:, :, 2] * 16.0, 1.0)
