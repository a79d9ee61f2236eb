"""Host logic of the learned predictor: feature layout and standardisation."""
import numpy as np
import pytest

from paper_2005_02088_amd import camelot as cm

BATCHES = [1, 2, 4, 8, 16, 32, 64, 128]


def _tables():
    k, s, b = np.meshgrid(np.arange(3), np.arange(32), np.arange(8), indexing="ij")
    hbm = (k + s / 100.0 + b / 1000.0).astype(np.float32)
    mfma = (10 + k + s / 100.0 + b / 1000.0).astype(np.float32)
    return cm.SoloTablesArrays(8, BATCHES, hbm, mfma)


def test_feature_layout_three_stages():
    t = _tables()
    f = cm.camelot_predictor_features(t, [2, 0, 1], [16, 64, 8], [1, 3, 7])
    # row 0: kind 2, 16 CUs (share index 1), batch 2 (index 1)
    np.testing.assert_allclose(f[0, :4], [16 / 256, 1 / 7, 2 + 0.01 + 0.001, 12 + 0.01 + 0.001], rtol=1e-6)
    assert list(f[0, 4:7]) == [0, 0, 1]
    # co-runners in order: kind 0 (64 CUs, batch 8), kind 1 (8 CUs, batch 128)
    np.testing.assert_allclose(f[0, 7:11], [64 / 256, 3 / 7, 0 + 0.07 + 0.003, 10 + 0.07 + 0.003], rtol=1e-6)
    np.testing.assert_allclose(f[0, 11:15], [8 / 256, 7 / 7, 1 + 0.0 + 0.007, 11 + 0.0 + 0.007], rtol=1e-6)
    np.testing.assert_allclose(f[:, 15], (16 + 64 + 8) / 256)
    # row 1 (kind 0) sees kinds 2 and 1 as co-runners
    assert list(f[1, 4:7]) == [1, 0, 0]
    np.testing.assert_allclose(f[1, 7], 16 / 256)
    np.testing.assert_allclose(f[1, 11], 8 / 256)


def test_feature_layout_solo_has_empty_corunner_slots():
    t = _tables()
    f = cm.camelot_predictor_features(t, [1], [256], [0])
    assert np.all(f[0, 7:15] == 0)
    np.testing.assert_allclose(f[0, 15], 1.0)
    np.testing.assert_allclose(f[0, 0], 1.0)


def test_feature_validation():
    t = _tables()
    for kinds, cu, bi in (([3], [8], [0]), ([0], [12], [0]), ([0], [264], [0]), ([0], [8], [8])):
        with pytest.raises(cm.CamelotError):
            cm.camelot_predictor_features(t, kinds, cu, bi)


def test_standardisation_matches_numpy():
    x = np.random.default_rng(3).normal(5, 2, (500, 16)).astype(np.float32)
    x[:, 4] = 1.0                               # a constant column: std floored, not zero
    mean, std = cm.camelot_predictor_fit_norm(x)
    np.testing.assert_allclose(mean, x.mean(axis=0), rtol=1e-5, atol=1e-6)
    np.testing.assert_allclose(std[np.arange(16) != 4], x.std(axis=0)[np.arange(16) != 4], rtol=1e-4)
    assert std[4] >= 1e-6
    z = cm.camelot_predictor_standardize(x, mean, std)
    np.testing.assert_allclose(z, (x - mean) / std, rtol=1e-5, atol=1e-5)
