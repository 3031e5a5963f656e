"""The seeded input generators follow their stated recipes (shapes, rings, distributions,
determinism).  They hold none of the method's arithmetic; both the oracle and the GPU path
take their inputs from them."""
import math

import numpy as np

from paper_1511_04292_amd import workloads as W


def test_batch_sides_log_uniform_and_never_powers_of_two():
    N, P = W.batch_sizes(count=1024)
    assert N.shape == P.shape == (1024,)
    assert N.min() >= 32 and N.max() <= 1024
    assert not np.any((N & (N - 1)) == 0)
    assert P.min() >= 3 and P.max() <= 8 and set(P.tolist()) == set(range(3, 9))
    # log-uniform on [32, 1024]: the median side is near sqrt(32 * 1024) = 181 and the total
    # is about 1.6e8 points (mean N^2 = (1024^2 - 32^2) / (2 ln 32) = 1.5e5)
    assert 150 <= np.median(N) <= 215
    assert 1.3e8 <= float(np.sum(N.astype(np.float64) ** 2)) <= 1.9e8
    N2, P2 = W.batch_sizes(count=1024)
    assert np.array_equal(N, N2) and np.array_equal(P, P2)
    N3, _ = W.batch_sizes(count=1024, seed=4)
    assert not np.array_equal(N, N3)


def test_small_2d_manufactured_source_plus_noise():
    wl = W.small_2d(64, seed=0)
    n = 64
    f = wl["f"]
    assert f.shape == (n + 2, n + 2) and wl["h"] == 1.0 / 65
    assert not f[0].any() and not f[-1].any() and not f[:, 0].any() and not f[:, -1].any()
    x = np.arange(1, n + 1) / 65.0
    noise = f[1:-1, 1:-1] - 2.0 * math.pi ** 2 * np.outer(np.sin(math.pi * x), np.sin(math.pi * x))
    assert abs(noise.std() - 1e-3) < 0.05e-3 and abs(noise.mean()) < 1e-4
    assert not wl["u0"].any()


def test_blobs_ring_and_source():
    wl = W.blobs_2d(256, seed=0)
    u0, f = wl["u0"], wl["f"]
    ring = np.concatenate([u0[0], u0[-1], u0[1:-1, 0], u0[1:-1, -1]])
    assert ring.min() >= -1.0 and ring.max() <= 1.0 and abs(ring.mean()) < 0.1
    assert not u0[1:-1, 1:-1].any()
    assert not f[0].any() and not f[-1].any() and not f[:, 0].any() and not f[:, -1].any()
    assert np.abs(f[1:-1, 1:-1]).max() > 0.1
    again = W.blobs_2d(256, seed=0)
    assert np.array_equal(again["f"], f) and np.array_equal(again["u0"], u0)


def test_blobs_device_form_has_the_same_structure():
    wl = W.blobs_2d_device(96, seed=0, device="cpu")
    u0, f = wl["u0"].numpy(), wl["f"].numpy()
    assert u0.shape == f.shape == (98, 98)
    assert not u0[1:-1, 1:-1].any() and np.abs(u0[0]).max() <= 1.0 and np.abs(u0[0]).max() > 0.5
    assert not f[0].any() and not f[:, -1].any()
    assert np.abs(f[1:-1, 1:-1]).max() > 0.1


def test_smooth_3d_is_one_neighbour_mean_of_uniform_noise():
    n = 24
    wl = W.smooth_3d(n, seed=0)
    f = wl["f"]
    assert f.shape == (n + 2,) * 3 and wl["h"] == 1.0 / (n + 1)
    assert not f[0].any() and not f[-1].any() and not f[:, 0].any() and not f[:, :, -1].any()
    # the mean of six i.i.d. U(-1, 1) values has variance (1/3) / 6 = 1/18 away from the ring
    core = f[3:-3, 3:-3, 3:-3]
    assert abs(core.var() - 1.0 / 18.0) < 0.1 / 18.0
    rng = np.random.default_rng(0)
    v = np.zeros_like(f)
    v[1:-1, 1:-1, 1:-1] = rng.uniform(-1.0, 1.0, size=(n, n, n))
    i, j, k = 5, 7, 9
    want = (v[i, j, k - 1] + v[i, j, k + 1] + v[i, j - 1, k] + v[i, j + 1, k] + v[i - 1, j, k] + v[i + 1, j, k]) / 6.0
    assert abs(f[i, j, k] - want) <= 1e-15
