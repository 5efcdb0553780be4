"""Pins of the FP64 environment-map sampling oracle against closed forms,
special cases and brute force (Sec. 3 MIS of R; Sec. 4.3 map projection)."""
import numpy as np
import pytest

from oracle import envmap as E


def _const(n, H, W, c=0.7):
    return np.full((n, H, W, 3), c)


@pytest.mark.parametrize("H,W", [(1, 1), (4, 8), (32, 32), (64, 64), (7, 5)])
def test_constant_map_is_the_solid_angle_cdf(H, W):
    # Equal radiance everywhere: row masses follow the pixels' solid angles,
    # and a sum of sines at row centres telescopes to the polar-cap area, so
    # the marginal CDF at the lower edge of row v is 1 - cos((v + 1) pi / (2H)).
    cdf_u, cdf_v, total = E.build(_const(2, H, W))
    np.testing.assert_allclose(cdf_v[0], 1.0 - np.cos((np.arange(H) + 1) * np.pi / (2 * H)), atol=1e-13)
    np.testing.assert_allclose(cdf_u[1], np.broadcast_to((np.arange(W) + 1.0) / W, (H, W)), atol=1e-15)
    assert np.all(total > 0)


@pytest.mark.parametrize("H,W", [(4, 8), (16, 16)])
def test_constant_map_density_at_row_centres(H, W):
    # Solid-angle density of a constant map at a row centre theta_c:
    # p(v) H / (pi^2 sin theta_c) with p(v) = cos(a) - cos(b) = 2 sin(theta_c) sin(pi / 4H).
    cdf_u, cdf_v, _ = E.build(_const(1, H, W))
    th = (np.arange(H) + 0.5) * np.pi / (2 * H)
    ph = (np.arange(W) + 0.5) * 2 * np.pi / W
    T, P = np.meshgrid(th, ph, indexing="ij")
    d = np.stack([np.sin(T) * np.cos(P), np.sin(T) * np.sin(P), np.cos(T)], -1).reshape(1, -1, 3)
    p = E.pdf(cdf_u, cdf_v, d)
    np.testing.assert_allclose(p, 2 * H * np.sin(np.pi / (4 * H)) / np.pi ** 2, rtol=1e-12)
    assert abs(2 * 256 * np.sin(np.pi / 1024) / np.pi ** 2 - 1 / (2 * np.pi)) < 1e-5  # uniform limit


def test_luminance_weights_and_channel_order():
    # One row holding pure red, pure green and pure blue pixels of equal value:
    # the conditional probabilities are the BT.709 luminance weights, in order.
    rgb = np.zeros((1, 1, 3, 3))
    rgb[0, 0, 0, 0] = rgb[0, 0, 1, 1] = rgb[0, 0, 2, 2] = 2.0
    cdf_u, cdf_v, _ = E.build(rgb)
    np.testing.assert_allclose(np.diff(cdf_u[0, 0], prepend=0.0), [0.2126, 0.7152, 0.0722], atol=1e-15)
    # grey keeps its value: the weights sum to one
    g = np.full((1, 2, 2, 3), 3.0)
    np.testing.assert_allclose(E.pixel_weights(g)[0, :, 0], 3.0 * np.sin((np.arange(2) + 0.5) * np.pi / 4),
                               rtol=1e-15)


def test_delta_map():
    H, W, v0, u0 = 8, 16, 5, 11
    rgb = np.zeros((1, H, W, 3))
    rgb[0, v0, u0] = (1.0, 2.0, 3.0)
    cdf_u, cdf_v, total = E.build(rgb)
    assert total[0] > 0
    np.testing.assert_array_equal(cdf_v[0], (np.arange(H) >= v0).astype(float))
    np.testing.assert_array_equal(cdf_u[0, v0], (np.arange(W) >= u0).astype(float))
    others = np.delete(cdf_u[0], v0, axis=0)
    np.testing.assert_allclose(others, np.broadcast_to((np.arange(W) + 1.0) / W, others.shape), atol=1e-15)
    xi = np.random.default_rng(0).random((1, 200, 2))
    d, p, pix = E.sample(cdf_u, cdf_v, xi)
    assert np.all(pix == v0 * W + u0)
    th = np.arctan2(np.hypot(d[..., 0], d[..., 1]), d[..., 2])
    np.testing.assert_allclose(p, H * W / (np.pi ** 2 * np.sin(th)), rtol=1e-12)
    assert np.all((th >= v0 * np.pi / (2 * H) - 1e-12) & (th <= (v0 + 1) * np.pi / (2 * H) + 1e-12))


@pytest.mark.parametrize("fill", [0.0, -1.0])
def test_dark_or_negative_maps_fall_back_to_uniform(fill):
    H, W = 4, 6
    cdf_u, cdf_v, total = E.build(np.full((1, H, W, 3), fill))
    assert total[0] == 0
    np.testing.assert_allclose(cdf_v[0], (np.arange(H) + 1.0) / H, atol=1e-15)
    np.testing.assert_allclose(cdf_u[0], np.broadcast_to((np.arange(W) + 1.0) / W, (H, W)), atol=1e-15)


def test_joint_probabilities_brute_force():
    # p(v) p(u | v) must equal f[v, u] / sum f for every pixel (the
    # marginal / conditional factorisation of a 2-D table), on a tiny map.
    rgb = np.random.default_rng(3).random((1, 3, 4, 3)) - 0.2
    f = np.zeros((3, 4))
    for v in range(3):
        for u in range(4):
            y = 0.2126 * rgb[0, v, u, 0] + 0.7152 * rgb[0, v, u, 1] + 0.0722 * rgb[0, v, u, 2]
            f[v, u] = max(y, 0.0) * np.sin((v + 0.5) * np.pi / 6)
    cdf_u, cdf_v, total = E.build(rgb)
    joint = np.diff(cdf_v[0], prepend=0.0)[:, None] * np.diff(cdf_u[0], axis=1, prepend=0.0)
    np.testing.assert_allclose(joint, f / f.sum(), atol=1e-15)
    assert abs(total[0] - f.sum()) < 1e-14


def test_density_integrates_to_one_over_the_hemisphere():
    # pdf * sin(theta) is piecewise constant on the pixel grid, so the
    # midpoint rule on a refined grid integrates it exactly.
    H, W, k = 8, 12, 3
    rgb = np.random.default_rng(4).lognormal(size=(1, H, W, 3))
    cdf_u, cdf_v, _ = E.build(rgb)
    th = (np.arange(H * k) + 0.5) * np.pi / (2 * H * k)
    ph = (np.arange(W * k) + 0.5) * 2 * np.pi / (W * k)
    T, P = np.meshgrid(th, ph, indexing="ij")
    d = np.stack([np.sin(T) * np.cos(P), np.sin(T) * np.sin(P), np.cos(T)], -1).reshape(1, -1, 3)
    p = E.pdf(cdf_u, cdf_v, d).reshape(H * k, W * k)
    integral = (p * np.sin(T)).sum() * (np.pi / (2 * H * k)) * (2 * np.pi / (W * k))
    assert abs(integral - 1.0) < 1e-12
    # nothing below the horizon
    assert E.pdf(cdf_u, cdf_v, np.array([[[0.3, 0.1, -0.2]]]))[0, 0] == 0.0


def test_sampling_matches_density_and_distribution():
    H, W = 6, 10
    rgb = np.random.default_rng(5).lognormal(size=(1, H, W, 3))
    cdf_u, cdf_v, _ = E.build(rgb)
    # the density a sample reports is the density of its direction
    xi = np.random.default_rng(6).random((1, 500, 2))
    d, p, pix = E.sample(cdf_u, cdf_v, xi)
    np.testing.assert_allclose(p, E.pdf(cdf_u, cdf_v, d), rtol=1e-9)
    np.testing.assert_allclose(np.linalg.norm(d, axis=-1), 1.0, atol=1e-14)
    # a stratified grid of xi lands in each pixel in proportion to its mass
    g = (np.arange(200) + 0.5) / 200
    X1, X2 = np.meshgrid(g, g, indexing="ij")
    xi = np.stack([X1.ravel(), X2.ravel()], -1)[None]
    _, _, pix = E.sample(cdf_u, cdf_v, xi)
    freq = np.bincount(pix[0], minlength=H * W) / xi.shape[1]
    joint = (np.diff(cdf_v[0], prepend=0.0)[:, None] * np.diff(cdf_u[0], axis=1, prepend=0.0)).ravel()
    assert np.abs(freq - joint).max() < 2.5 / 200


def test_sampling_inverts_the_cdf_at_row_edges():
    # For a constant map the marginal CDF is 1 - cos(theta_edge); feeding
    # that value back returns exactly the edge angle.
    H, W = 16, 8
    cdf_u, cdf_v, _ = E.build(_const(1, H, W))
    edges = np.arange(1, H) * np.pi / (2 * H)
    xi = np.stack([1 - np.cos(edges), np.full(H - 1, 0.5)], -1)[None]
    d, _, pix = E.sample(cdf_u, cdf_v, xi)
    th = np.arctan2(np.hypot(d[0, :, 0], d[0, :, 1]), d[0, :, 2])
    np.testing.assert_allclose(th, edges, atol=1e-12)
    # which of the two rows meeting at an edge is picked depends on rounding
    assert np.all(np.abs(pix[0] // W - np.arange(0.5, H - 1)) == 0.5)
