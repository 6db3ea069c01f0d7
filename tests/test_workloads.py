"""CPU checks of the seeded input generators (they draw random numbers only)."""

import numpy as np

from workloads import cells_two_contrast


def test_two_contrast_values_and_layers():
    lam, betas = 0.4, (0.3, 0.6)
    for dims in (2, 3):
        c = cells_two_contrast(12, lam, betas, 0.5, seed=5, dims=dims)
        assert c.shape == (12,) * dims
        vals = set(np.round(np.unique(c), 12))
        assert vals <= {lam, lam + betas[0], lam + betas[1]} and len(vals) == 3
        assert 0.3 < np.mean(c > lam) < 0.7                      # occupancy near p
        lay = cells_two_contrast(12, lam, betas, 1.0, seed=5, layered=True, layer=3, dims=dims)
        for i in range(12):
            want = lam + (betas[0] if (i // 3) % 2 == 0 else betas[1])
            assert np.all(lay[i] == want)                        # p = 1: every cell of layer i
    a = cells_two_contrast(8, lam, betas, 0.5, seed=11)
    b = cells_two_contrast(8, lam, betas, 0.5, seed=11)
    assert np.array_equal(a, b)
