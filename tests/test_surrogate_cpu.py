"""The surrogate's baselines on the CPU (no GPU): what the method offers for
new motion parameters without the network.  The affine fit reproduces an
affine function of the scaled parameters (with the phase through its sine and
cosine) to round-off; the nearest case is a training row, found across the
phase's wrap-around; the mean is the training mean."""

import numpy as np

from paper_2002_04353_amd import surrogate as S


def _feats(X):
    ph = np.pi * (X[:, 4] + 1.0)
    return np.column_stack([np.ones(len(X)), X[:, :4], np.sin(ph), np.cos(ph)])


def test_affine_fit_reproduces_an_affine_target():
    rng = np.random.default_rng(1)
    Xtr, Xte = rng.uniform(-1, 1, (60, 5)), rng.uniform(-1, 1, (9, 5))
    C = rng.normal(size=(7, 12))
    b = S.baselines(Xtr, _feats(Xtr) @ C, Xte)
    np.testing.assert_allclose(b["linear"], _feats(Xte) @ C, rtol=0, atol=1e-10)
    np.testing.assert_allclose(b["mean"], np.broadcast_to((_feats(Xtr) @ C).mean(0), (9, 12)))


def test_nearest_case_wraps_the_phase():
    Xtr = np.array([[0, 0, 0, 0, -0.98], [0, 0, 0, 0, 0.5], [0.3, 0, 0, 0, 0.9]])
    Ytr = np.arange(3, dtype=float)[:, None] * np.ones((1, 4))
    # phase 0.99 is 0.03 from -0.98 across the wrap, 0.49 from 0.5 and 0.09 (+0.3 in Ma) from the third
    b = S.baselines(Xtr, Ytr, np.array([[0, 0, 0, 0, 0.99]]))
    assert b["nearest"][0, 0] == 0.0
    b = S.baselines(Xtr, Ytr, np.array([[0.01, 0, 0, 0, 0.45]]))
    assert b["nearest"][0, 0] == 1.0


def test_rms_splits_lift_and_moment():
    Y = np.zeros((3, 8))
    P = np.zeros((3, 8))
    P[:, :4] = 2.0
    P[:, 4:] = -1.0
    assert S.rms_cl_cm(P, Y) == (2.0, 1.0)
