"""Statistics and reproducibility of the seeded synthetic workloads (CPU)."""
import numpy as np

from paper_1910_02480_amd import synth


def test_param_init_statistics():
    p = synth.init_params(0)
    assert p.dtype == np.float32 and p.size == 206819
    off = 0
    for _, ci, co in synth._INIT_LAYERS:
        w = p[off:off + co * 9 * ci]
        b = p[off + co * 9 * ci: off + co * 9 * ci + co]
        std = np.sqrt(2.0 / (9 * ci))
        if w.size > 1000:
            assert abs(w.std() / std - 1) < 0.05
        assert np.all(np.abs(b) <= 1 / np.sqrt(9 * ci))
        off += co * 9 * ci + co
    np.testing.assert_array_equal(p, synth.init_params(0))
    assert not np.array_equal(p, synth.init_params(1))


def test_radiance_map_statistics():
    x = synth.radiance_maps(64, 32, 32)
    assert x.shape == (64, 32, 32, 7) and x.dtype == np.float32
    rad = np.expm1(x[..., :3].astype(np.float64))
    assert np.all(rad > 0)
    # log-radiance above mu + 2.5 sigma (+ firefly lift) stays a small tail
    frac_bright = np.mean(np.min(np.log(rad), axis=-1) > -1 + 1.5 * 2.5)
    assert frac_bright < 0.05
    nrm = x[..., 3:6]
    np.testing.assert_allclose(np.linalg.norm(nrm, axis=-1), 1.0, atol=1e-6)
    d = x[..., 6]
    assert d.min() >= 0.1 and d.max() <= 10.0
    assert abs(d.mean() - 5.05) < 0.1


def test_lognormal_moments_and_firefly_rate():
    """Redraw the first two streams of a map and check mu, sigma and p."""
    n = 0
    logs, fires = [], []
    for m in range(40):
        rng = np.random.default_rng([synth.SEED_MAPS, m])
        rgb = rng.lognormal(-1.0, 1.5, size=(32, 32, 3))
        fire = rng.random((32, 32)) < 0.02
        x = synth.radiance_map(m, 32, 32)
        exp = np.log1p(np.where(fire[..., None], rgb * 100, rgb)).astype(np.float32)
        np.testing.assert_array_equal(x[..., :3], exp)
        logs.append(np.log(rgb).ravel())
        fires.append(fire.ravel())
        n += fire.size
    logs = np.concatenate(logs)
    rate = np.concatenate(fires).mean()
    assert abs(logs.mean() + 1.0) < 0.02 and abs(logs.std() - 1.5) < 0.02
    sigma = np.sqrt(0.02 * 0.98 / n)
    assert abs(rate - 0.02) < 3 * sigma


def test_subset_reproducibility():
    full = synth.radiance_maps(8, 16, 16)
    part = synth.radiance_maps(3, 16, 16, start=4)
    np.testing.assert_array_equal(full[4:7], part)


def test_training_pairs():
    x, t = synth.training_batch(4, 32)
    assert x.shape == (4, 32, 32, 7) and t.shape == (4, 32, 32, 3)
    assert np.all(t >= 0) and np.all(np.isfinite(x))
    # target is smooth: neighbouring pixels differ far less than the noisy input
    dt = np.abs(np.diff(t, axis=2)).mean()
    dx = np.abs(np.diff(x[..., :3], axis=2)).mean()
    assert dt < 0.5 * dx
    x2, t2 = synth.training_batch(2, 32, start=2)
    np.testing.assert_array_equal(x[2:], x2)
    np.testing.assert_array_equal(t[2:], t2)


def test_mixed_resolutions():
    r = synth.mixed_resolutions(6000)
    assert (r == 32).sum() == 3000 and (r == 64).sum() == 2100 and (r == 128).sum() == 900
    np.testing.assert_array_equal(r, synth.mixed_resolutions(6000))
    assert not np.array_equal(r[:100], np.sort(r)[:100])
    x, xo, yo = synth.mixed_frame(r[:10])
    assert xo[0] == 0 and x.size == int((r[:10].astype(np.int64) ** 2).sum()) * 7
    m = 3
    np.testing.assert_array_equal(
        x[xo[m]:xo[m] + r[m] * r[m] * 7].reshape(r[m], r[m], 7),
        synth.radiance_map(m, int(r[m]), int(r[m])))
    assert yo[1] == r[0] * r[0] * 3
