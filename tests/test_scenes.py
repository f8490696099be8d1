"""Seeded input generators: reproducible, with the stated shapes and ranges."""
import math

import numpy as np

from paper_1512_02110_amd import scenes


def test_configs_reproducible_and_shaped():
    for make, shape, bmax, ncam, npx in [(scenes.config1, (16, 16, 16), 10.0, 4, 32),
                                          (scenes.config2, (64, 64, 64), 50.0, 9, 128)]:
        a, b = make(n_photons=10), make(n_photons=10)
        assert np.array_equal(a.beta, b.beta)
        assert (a.nz, a.ny, a.nx) == shape and a.beta.size == np.prod(shape)
        assert a.beta.min() >= 0 and abs(a.beta.max() - bmax) < 0.05 * bmax
        assert a.n_cams == ncam and all(c.width == npx == c.height for c in a.cameras)


def test_config1_blob_values():
    s = scenes.config1()
    b3 = s.beta3d()
    # voxel centre (0.425, 0.425, 0.425) km is 0.025*sqrt(3) km from the blob centre
    r2 = 3 * 0.025 ** 2
    assert abs(b3[8, 8, 8] - 10 * math.exp(-r2 / (2 * 0.04))) < 1e-12
    assert abs(s.cameras[0].fx - 16 / math.tan(math.radians(30))) < 1e-12


def test_config2_column_optical_depth():
    s = scenes.config2(n_photons=1)
    col = s.beta3d().sum(axis=0) * s.dz
    assert 10 < col.max() < 80          # cloud-like: thick columns exist
    assert (col == 0).mean() > 0.01     # and clear columns too


def test_config3_initial_is_smoothed_truth():
    t, i = scenes.config3_truth(n_photons=1), scenes.config3_initial(n_photons=1)
    # smoothing moves a little mass across the boundary ('nearest' padding)
    assert abs(i.beta.sum() - 0.7 * t.beta.sum()) < 0.01 * t.beta.sum()
    assert i.beta.max() < 0.7 * t.beta.max()
