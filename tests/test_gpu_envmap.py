"""Environment-map sampling of predicted maps on the GPU against the FP64
oracle (Sec. 3 MIS of R; Sec. 4.3 hemispherical lat-long maps).

Tolerances, from the FP32 arithmetic of the kernels (u = 2^-24): a pixel
weight carries a few rounding errors (luminance, sine, product), a row
prefix at most log2(64) + (64-column chunks) more, a row total the same,
the marginal prefix log2(64) + (64-row chunks) more, and each normalisation
one; with numerator and denominator both in error, every CDF entry (at most
1) is within delta = 2 (24 + ceil(W / 64) + ceil(H / 64)) u of the exact
value (3.1e-6 at 64 x 64). A probability is a difference of two CDF entries
(error 2 delta); a density p_v p_u H W / (pi^2 sin t) is therefore within
(2 delta (p_u + p_v) + 4 delta^2) H W / (pi^2 sin t), plus a relative 1e-5
for the sine. The row and column a sample picks are decided by comparing
xi with CDF entries, so they are compared exactly only where xi is farther
than MARGIN = 1e-5 (> 2 delta at the sampled sizes) from every oracle entry
it is compared with; elsewhere the GPU's choice must bracket xi within
that margin.
"""
import numpy as np
import pytest
import torch

from oracle import envmap as E
from paper_1910_02480_amd import binding as B
from paper_1910_02480_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
MARGIN = 1e-5


def _delta(H, W):
    return 2 * (24 + -(-W // 64) + -(-H // 64)) * 2.0 ** -24


def _gpu_build(y):
    n, H, W, _ = y.shape
    yd = torch.from_numpy(np.ascontiguousarray(y, dtype=np.float32)).to(DEV)
    cu = torch.full((n, H, W), float("nan"), device=DEV)
    cv = torch.full((n, H), float("nan"), device=DEV)
    tot = torch.full((n,), float("nan"), device=DEV)
    print(f"[envmap] build n={n} H={H} W={W}", flush=True)
    B.drc_envmap_build(yd, cu, cv, tot)
    torch.cuda.synchronize()
    return cu, cv, tot


def _check_tables(cu, cv, tot, y):
    cu_o, cv_o, tot_o = E.build(y)
    g_u, g_v, g_t = cu.cpu().double().numpy(), cv.cpu().double().numpy(), tot.cpu().double().numpy()
    delta = _delta(*cu_o.shape[1:])
    np.testing.assert_allclose(g_u, cu_o, atol=delta, rtol=0)
    np.testing.assert_allclose(g_v, cv_o, atol=delta, rtol=0)
    np.testing.assert_allclose(g_t, tot_o, rtol=1e-5, atol=0)
    _check_valid(g_u, g_v)
    return cu_o, cv_o


def _check_valid(g_u, g_v):
    """Properties that hold at any size: non-decreasing, in [0, 1], last entry exactly 1."""
    for c in (g_u, g_v):
        assert np.all(np.diff(c, axis=-1) >= 0)
        assert np.all(c[..., -1] == 1.0)
        assert np.all((c >= 0) & (c <= 1))


def _mass_tol(pv, pu, H, W, st):
    d = _delta(H, W)
    return (2 * d * (pu + pv) + 4 * d ** 2) * H * W / (np.pi ** 2 * np.maximum(st, 1e-30))


def _margin(cdf_row, xi):
    return np.min(np.abs(np.concatenate([[0.0], cdf_row]) - xi))


@pytest.mark.parametrize("n,H,W", [(3, 64, 64), (5, 32, 32), (2, 128, 128), (3, 7, 5), (2, 3, 100),
                                   (1, 1, 1), (2, 16, 1024), (1, 4096, 2), (4, 24, 40)])
def test_build_matches_oracle(n, H, W):
    y = synth.predicted_maps(n, H, W)
    cu, cv, tot = _gpu_build(y)
    _check_tables(cu, cv, tot, y)


def test_build_degenerate_maps():
    H, W = 16, 16
    y = np.zeros((6, H, W, 3), np.float32)               # 0: dark -> uniform
    y[1] = -0.5                                          # 1: negative -> uniform
    y[2, 5, 11] = (1.0, 2.0, 3.0)                        # 2: delta
    y[3] = 0.7                                           # 3: constant
    y[4] = synth.predicted_map(0, H, W)                  # 4: rows 3..7 dark
    y[4, 3:8] = 0.0
    y[5] = np.where(np.arange(W)[None, :, None] % 2 == 0, 0.4, -0.4)  # 5: every other column dark
    cu, cv, tot = _gpu_build(y)
    _check_tables(cu, cv, tot, y)
    t = tot.cpu().numpy()
    assert t[0] == 0 and t[1] == 0 and np.all(t[2:] > 0)
    g_v = cv.cpu().double().numpy()
    # constant map: the polar-cap CDF 1 - cos(theta_edge)
    np.testing.assert_allclose(g_v[3], 1 - np.cos((np.arange(H) + 1) * np.pi / (2 * H)), atol=_delta(H, W))
    np.testing.assert_array_equal(g_v[2], (np.arange(H) >= 5).astype(float))


def test_empty_batches_are_no_ops():
    y = torch.zeros((0, 8, 8, 3), device=DEV)
    cu = torch.zeros((0, 8, 8), device=DEV)
    cv = torch.zeros((0, 8), device=DEV)
    tot = torch.zeros((0,), device=DEV)
    B.drc_envmap_build(y, cu, cv, tot)
    cu1 = torch.rand((1, 8, 8), device=DEV)
    cv1 = torch.rand((1, 8), device=DEV)
    B.drc_envmap_sample(cu1, cv1, torch.zeros((1, 0, 2), device=DEV), torch.zeros((1, 0, 3), device=DEV),
                        torch.zeros((1, 0), device=DEV), torch.zeros((1, 0), dtype=torch.int32, device=DEV))
    torch.cuda.synchronize()


def _sample(cu, cv, xi):
    n, S = xi.shape[:2]
    xd = torch.from_numpy(np.ascontiguousarray(xi, dtype=np.float32)).to(DEV)
    d = torch.full((n, S, 3), float("nan"), device=DEV)
    p = torch.full((n, S), float("nan"), device=DEV)
    pix = torch.full((n, S), -1, dtype=torch.int32, device=DEV)
    print(f"[envmap] sample n={n} S={S}", flush=True)
    B.drc_envmap_sample(cu, cv, xd, d, p, pix)
    torch.cuda.synchronize()
    return d.cpu().double().numpy(), p.cpu().double().numpy(), pix.cpu().numpy()


def _pdf(cu, cv, dirs):
    n, S = dirs.shape[:2]
    dd = torch.from_numpy(np.ascontiguousarray(dirs, dtype=np.float32)).to(DEV)
    p = torch.full((n, S), float("nan"), device=DEV)
    print(f"[envmap] pdf n={n} S={S}", flush=True)
    B.drc_envmap_pdf(cu, cv, dd, p)
    torch.cuda.synchronize()
    return p.cpu().double().numpy()


def _angles(d):
    th = np.arctan2(np.hypot(d[..., 0], d[..., 1]), d[..., 2])
    ph = np.mod(np.arctan2(d[..., 1], d[..., 0]), 2 * np.pi)
    return th, ph


def _compare_samples(cu_o, cv_o, xi, d_g, p_g, pix_g):
    n, H, W = cu_o.shape
    xi = xi.astype(np.float32).astype(np.float64)   # the values the GPU saw
    d_o, p_o, pix_o = E.sample(cu_o, cv_o, xi)
    pv_all = np.diff(cv_o, axis=-1, prepend=0.0)
    pu_all = np.diff(cu_o, axis=-1, prepend=0.0)
    th_g, ph_g = _angles(d_g)
    th_o, ph_o = _angles(d_o)
    exact = 0
    for m in range(n):
        for s in range(xi.shape[1]):
            v_o, u_o = divmod(int(pix_o[m, s]), W)
            v_g, u_g = divmod(int(pix_g[m, s]), W)
            mv = _margin(cv_o[m], xi[m, s, 0])
            mu = _margin(cu_o[m, v_o], xi[m, s, 1])
            if mv > MARGIN and mu > MARGIN:
                exact += 1
                assert (v_g, u_g) == (v_o, u_o), (m, s)
                pv, pu = pv_all[m, v_o], pu_all[m, v_o, u_o]
                tol_t = (np.pi / 2) / H * 2 * _delta(H, W) / pv + 1e-6
                tol_p = 2 * np.pi / W * 2 * _delta(H, W) / pu + 1e-6
                assert abs(th_g[m, s] - th_o[m, s]) <= tol_t, (m, s)
                dp = abs(ph_g[m, s] - ph_o[m, s])
                assert min(dp, 2 * np.pi - dp) <= tol_p, (m, s)
                st = np.sin(th_o[m, s])
                assert abs(p_g[m, s] - p_o[m, s]) <= _mass_tol(pv, pu, H, W, st) + 1e-5 * p_o[m, s] \
                    + p_o[m, s] * tol_t / max(np.tan(th_o[m, s]), 1e-30), (m, s)
            else:
                # near a CDF boundary: the GPU's row and column must bracket xi
                lo = cv_o[m, v_g - 1] if v_g > 0 else 0.0
                assert lo - MARGIN <= xi[m, s, 0] <= cv_o[m, v_g] + MARGIN
                lo = cu_o[m, v_g, u_g - 1] if u_g > 0 else 0.0
                assert lo - MARGIN <= xi[m, s, 1] <= cu_o[m, v_g, u_g] + MARGIN
    assert exact >= 0.9 * xi.shape[0] * xi.shape[1]
    np.testing.assert_allclose(np.linalg.norm(d_g, axis=-1), 1.0, atol=1e-6)


@pytest.mark.parametrize("n,H,W,S", [(3, 64, 64, 300), (4, 32, 32, 200), (2, 7, 5, 200), (2, 3, 100, 200)])
def test_sample_and_pdf_match_oracle(n, H, W, S):
    y = synth.predicted_maps(n, H, W)
    cu, cv, tot = _gpu_build(y)
    cu_o, cv_o = _check_tables(cu, cv, tot, y)
    xi = np.random.default_rng(11).random((n, S, 2))
    d_g, p_g, pix_g = _sample(cu, cv, xi)
    _compare_samples(cu_o, cv_o, xi, d_g, p_g, pix_g)
    # the density of the GPU's own samples, evaluated by the GPU, is the density they report
    p_eval = _pdf(cu, cv, d_g)
    th_g, ph_g = _angles(d_g)
    pv = np.diff(cv_o, axis=-1, prepend=0.0)
    for m in range(n):
        v = pix_g[m] // W
        u = pix_g[m] % W
        tol = _mass_tol(pv[m, v], np.diff(cu_o[m], axis=-1, prepend=0.0)[v, u], H, W, np.sin(th_g[m]))
        # away from pixel edges, where the two kernels may pick neighbouring pixels
        inside = (np.abs(np.modf(th_g[m] / (np.pi / 2) * H)[0] - 0.5) < 0.49) & \
                 (np.abs(np.modf(ph_g[m] / (2 * np.pi) * W)[0] - 0.5) < 0.49)
        np.testing.assert_array_less(np.abs(p_eval[m] - p_g[m])[inside], (2 * tol + 1e-5 * p_g[m])[inside])


@pytest.mark.parametrize("n,H,W", [(3, 64, 64), (2, 9, 13)])
def test_pdf_matches_oracle(n, H, W):
    y = synth.predicted_maps(n, H, W)
    cu, cv, tot = _gpu_build(y)
    cu_o, cv_o = _check_tables(cu, cv, tot, y)
    rng = np.random.default_rng(12)
    dirs = rng.standard_normal((n, 400, 3)) * rng.uniform(0.5, 2.0, (n, 400, 1))  # any length, both hemispheres
    dirs[:, 0] = (0.0, 0.0, 1.0)       # along the normal
    dirs[:, 1] = (1.0, 0.0, 0.0)       # on the horizon
    dirs = dirs.astype(np.float32).astype(np.float64)
    p_g = _pdf(cu, cv, dirs)
    p_o = E.pdf(cu_o, cv_o, dirs)
    th, ph = _angles(dirs)
    fv, fu = th / (np.pi / 2) * H, ph / (2 * np.pi) * W
    near = (np.abs(fv - np.round(fv)) < 1e-4) | (np.abs(fu - np.round(fu)) < 1e-4)
    assert np.all(p_g[dirs[..., 2] < 0] == 0.0) and np.all(p_g[:, 0] == 0.0)
    v = np.minimum(fv.astype(int), H - 1)
    u = np.minimum(fu.astype(int), W - 1)
    mi = np.arange(n)[:, None]
    pv = np.diff(cv_o, axis=-1, prepend=0.0)[mi, v]
    pu = np.diff(cu_o, axis=-1, prepend=0.0)[mi, v, u]
    tol = _mass_tol(pv, pu, H, W, np.sin(th)) + 1e-5 * p_o
    ok = near | (np.abs(p_g - p_o) <= tol)
    assert ok.all(), np.argwhere(~ok)[:5]
    assert (~near).sum() >= 0.95 * near.size


def test_full_batch_4096x64x64():
    """The bench's build launch (4096 maps of 64 x 64): sampled maps against
    the oracle, CDF properties on every map."""
    n, H = 4096, 64
    y = synth.predicted_maps(n, H, H)
    cu, cv, tot = _gpu_build(y)
    _check_valid(cu.cpu().double().numpy(), cv.cpu().double().numpy())
    idx = np.random.default_rng(13).choice(n, 12, replace=False)
    idx.sort()
    t = torch.from_numpy(idx).to(DEV)
    _check_tables(cu[t], cv[t], tot[t], y[idx])
