"""Pins of the hierarchical importance-sampling oracle (Sec. 5.2): a
hand-worked descent, pdf = normalised NDF mass, the sample histogram against
the NDF image, empty quads and the failure rule."""
import json
import os

import numpy as np

from oracle import query, sampling


def _tables(rng, nu, nv, nl, N, R, positive=True):
    f = (lambda s: rng.random(s) + 0.05) if positive else (lambda s: rng.standard_normal(s))
    U, V, L, S, Tf = (f((d, R)) for d in (nu, nv, nl, N, N))
    return U, V, L, query.cumulative(S), query.cumulative(Tf)


def _image(U, V, L, CS, CT, u, v, l):
    N = CS.shape[0] - 1
    recs = np.array([[u, v, l, s, s + 1, t, t + 1] for s in range(N) for t in range(N)])
    return query.range_query(U, V, L, CS, CT, recs).reshape(N, N)


def test_hand_worked_descent(golden_dir):
    with open(os.path.join(golden_dir, "sampling_4x4.json")) as fh:
        g = json.load(fh)
    one = np.ones((1, 1))
    CS = query.cumulative(np.array(g["S"])[:, None])
    CT = query.cumulative(np.array(g["T"])[:, None])
    assert np.allclose(sampling.quad_masses(one, one, one, CS, CT, 0, 0, 0, 0, 4, 0, 4), g["level1_masses"])
    assert np.allclose(sampling.quad_masses(one, one, one, CS, CT, 0, 0, 0, 2, 4, 0, 2), g["level2_masses"])
    h, pdf, b = sampling.sample_one(one, one, one, CS, CT, 0, 0, 0, np.array(g["rnd"]))
    assert tuple(b) == tuple(g["bin"])
    assert np.allclose(h, g["h"], rtol=0, atol=1e-15)
    assert abs(pdf - g["pdf"]) < 1e-15


def test_pdf_is_the_normalised_ndf_mass():
    rng = np.random.default_rng(1)
    U, V, L, CS, CT = _tables(rng, 3, 4, 2, 16, 3)
    uvl = np.stack([rng.integers(0, 3, 400), rng.integers(0, 4, 400), rng.integers(0, 2, 400)], axis=1)
    rnd = rng.random((400, 6))
    h, pdf, b = sampling.sample(U, V, L, CS, CT, uvl, rnd)
    w = 2.0 / 16
    for i in range(400):
        img = _image(U, V, L, CS, CT, *uvl[i])
        assert abs(pdf[i] * w * w - img[b[i, 0], b[i, 1]] / img.sum()) <= 1e-12
        assert b[i, 0] <= (h[i, 0] + 1) / w < b[i, 0] + 1
        assert b[i, 1] <= (h[i, 1] + 1) / w < b[i, 1] + 1


def test_histogram_matches_the_ndf_image():
    """The check the paper makes (Sec. 5.2): the histogram of many samples
    converges to the NDF image (chi-square at 4x4 bins, 20000 samples)."""
    rng = np.random.default_rng(2)
    U, V, L, CS, CT = _tables(rng, 2, 2, 1, 4, 2)
    n = 20000
    uvl = np.zeros((n, 3), dtype=np.int64)
    _, _, b = sampling.sample(U, V, L, CS, CT, uvl, rng.random((n, 4)))
    counts = np.zeros((4, 4))
    np.add.at(counts, (b[:, 0], b[:, 1]), 1)
    img = _image(U, V, L, CS, CT, 0, 0, 0)
    expect = n * img / img.sum()
    chi2 = float(np.sum((counts - expect) ** 2 / expect))
    assert chi2 < 45.0          # 15 degrees of freedom: P(chi2 > 45) < 1e-4


def test_empty_quads_are_never_chosen():
    """Bins of zero mass (S zero on bins 1 and 2) receive no samples."""
    rng = np.random.default_rng(3)
    S = np.array([[1.0], [0.0], [0.0], [2.0], [1.0], [0.0], [3.0], [1.0]])
    Tf = np.array([[1.0], [2.0], [0.0], [1.0], [1.0], [1.0], [1.0], [0.0]])
    one = np.ones((1, 1))
    CS, CT = query.cumulative(S), query.cumulative(Tf)
    rnd = rng.random((3000, 5))
    rnd[:10, :3] = 0.0
    rnd[10:20, :3] = np.nextafter(1.0, 0.0)
    _, pdf, b = sampling.sample(one, one, one, CS, CT, np.zeros((3000, 3), dtype=np.int64), rnd)
    assert np.all(S[b[:, 0], 0] > 0) and np.all(Tf[b[:, 1], 0] > 0)
    assert np.all(pdf > 0)


def test_no_positive_mass_fails():
    one = np.ones((1, 1))
    CS = query.cumulative(-np.ones((8, 1)))
    CT = query.cumulative(np.ones((8, 1)))
    h, pdf, b = sampling.sample(one, one, one, CS, CT, np.zeros((2, 3), dtype=np.int64), np.full((2, 5), 0.3))
    assert np.all(pdf == 0) and np.all(b == -1) and np.all(h == 0)
