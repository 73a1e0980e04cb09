"""Pins of the evaluation oracle (section 2.3: RMS-ID, CC, DSC, contour propagation by
opening and boundary extraction, surface-to-surface distance statistics) against library
routines and closed forms.  CPU only."""
import numpy as np
import pytest
from scipy import ndimage, stats

import oracle
from oracle import evaluate as ev

CROSS = ndimage.generate_binary_structure(3, 1)


def _blobs(shape, seed, p=0.55):
    """Random blobby mask that touches the volume border."""
    rng = np.random.default_rng(seed)
    f = ndimage.gaussian_filter(rng.normal(size=shape), 1.5)
    return f > np.quantile(f, p)


@pytest.mark.parametrize("radius", [1, 2])
def test_opening_equals_scipy(radius):
    m = _blobs((14, 17, 19), 1)
    ref = ndimage.binary_opening(m, structure=CROSS, iterations=radius, border_value=0)
    np.testing.assert_array_equal(ev.opening(m, radius), ref)
    np.testing.assert_array_equal(ev.erode(m), ndimage.binary_erosion(m, CROSS, border_value=0))
    np.testing.assert_array_equal(ev.dilate(m), ndimage.binary_dilation(m, CROSS, border_value=0))


def test_boundary_equals_set_minus_erosion():
    m = _blobs((12, 15, 13), 2)
    np.testing.assert_array_equal(ev.boundary(m), m & ~ndimage.binary_erosion(m, CROSS, border_value=0))
    # a solid box: its boundary is the box minus its interior
    b = np.zeros((8, 9, 10), bool)
    b[2:6, 2:7, 3:8] = True
    assert ev.boundary(b).sum() == 4 * 5 * 5 - 2 * 3 * 3


def test_surface_distances_equal_exact_distance_transform():
    """Brute force over point pairs equals scipy's exact Euclidean distance transform with
    anisotropic sampling (an independent algorithm), axis order included."""
    sp = (1.97, 1.6, 2.5)
    t = _blobs((16, 18, 20), 3, 0.7)
    d = _blobs((16, 18, 20), 4, 0.7)
    bt, bd = ev.boundary(t), ev.boundary(d)
    got = ev.surface_distances(bd, bt, sp)
    edt = ndimage.distance_transform_edt(~bt, sampling=[np.float32(sp[2]), np.float32(sp[1]), np.float32(sp[0])])
    np.testing.assert_allclose(got, edt[bd], rtol=1e-12, atol=0)


def test_concentric_cubes_are_one_voxel_apart():
    t = np.zeros((12, 12, 12), bool)
    t[1:11, 1:11, 1:11] = True
    d = np.zeros_like(t)
    d[2:10, 2:10, 2:10] = True
    dist = ev.surface_distances(ev.boundary(d), ev.boundary(t), (2.0, 2.0, 2.0))
    assert len(dist) == 8 ** 3 - 6 ** 3
    np.testing.assert_array_equal(dist, 2.0)
    s = ev.distance_stats(dist)
    assert s["mean"] == 2.0 and s["sd"] == 0.0 and s["p95"] == 2.0
    assert np.all(ev.surface_distances(ev.boundary(t), ev.boundary(t)) == 0.0)


def test_distance_stats_closed_form():
    s = ev.distance_stats(np.array([4.0, 1.0, 3.0, 2.0]))
    assert s["mean"] == 2.5
    assert s["sd"] == pytest.approx(np.sqrt(1.25), rel=1e-15)          # population SD
    assert s["p95"] == pytest.approx(3.85, rel=1e-15)                  # 3 + 0.85 (4 - 3)
    assert np.isnan(ev.distance_stats(np.zeros(0))["mean"])


def test_dsc_of_shifted_cube():
    a, t = 10, 3
    T = np.zeros((16, 16, 20), bool)
    T[3:13, 3:13, 2:12] = True
    D = np.zeros_like(T)
    D[3:13, 3:13, 2 + t:12 + t] = True
    r = ev.dsc(D, T)
    assert r["dsc"] == pytest.approx((a - t) / a, rel=1e-15)
    assert ev.dsc(T, T)["dsc"] == 1.0
    assert np.isnan(ev.dsc(np.zeros_like(T), np.zeros_like(T))["dsc"])


def test_rms_and_cc():
    rng = np.random.default_rng(7)
    T = rng.normal(0, 200, (6, 7, 8))
    r = ev.rms_cc(T + 7.0, T)
    assert r["rms_id"] == pytest.approx(7.0, rel=1e-12) and r["cc"] == pytest.approx(1.0, rel=1e-12)
    assert ev.rms_cc(-T, T)["cc"] == pytest.approx(-1.0, rel=1e-12)
    A = T + rng.normal(0, 50, T.shape)
    assert ev.rms_cc(A, T)["cc"] == pytest.approx(stats.pearsonr(A.ravel(), T.ravel())[0], rel=1e-12)
    region = rng.uniform(size=T.shape) > 0.5
    r = ev.rms_cc(A, T, region)
    assert r["voxels"] == region.sum()
    assert r["rms_id"] == pytest.approx(np.sqrt(np.mean((A - T)[region] ** 2)), rel=1e-12)


def test_deformed_mask_shifts_and_knife_edges():
    """The mask warp moves a mask by whole voxels exactly (no knife-edge voxel); under a
    half-voxel shift every voxel on the moving face has the value 0.5 exactly, counts as
    inside, and is listed as knife-edge; elsewhere the decision is scipy's interpolation
    thresholded at 0.5."""
    from scipy import ndimage
    rng = np.random.default_rng(8)
    m = (rng.uniform(size=(11, 13, 17)) > 0.6).astype(np.uint8)
    u = np.zeros((3, 11, 13, 17), np.float32)
    u[0] = 1.0
    u[2] = -2.0
    got, knife = ev.deformed_mask(m, u)
    # pull-back by whole voxels with a clamped border: out(x, y, z) = m(x + 1, y, z - 2)
    zi = np.clip(np.arange(11) - 2, 0, 10)
    xi = np.clip(np.arange(17) + 1, 0, 16)
    np.testing.assert_array_equal(got, m[zi][:, :, xi].astype(bool))
    assert len(knife) == 0
    cube = np.zeros((8, 9, 10), np.uint8)
    cube[2:6, 3:7, 3:8] = 1
    half = np.zeros((3,) + cube.shape, np.float32)
    half[0] = 0.5
    got, knife = ev.deformed_mask(cube, half)
    face = np.zeros(cube.shape, bool)
    face[2:6, 3:7, 2] = True          # value (0 + 1) / 2 at x = 2
    face[2:6, 3:7, 7] = True          # value (1 + 0) / 2 at x = 7
    np.testing.assert_array_equal(np.sort(knife), np.flatnonzero(face))
    expect = np.zeros(cube.shape, bool)
    expect[2:6, 3:7, 2:8] = True
    np.testing.assert_array_equal(got, expect)
    from paper_1301_0970_amd import phantom as P
    u = P.random_smooth_field((17, 13, 11), 3.0, 9).astype(np.float32)
    got, knife = ev.deformed_mask(m, u)
    nz, ny, nx = m.shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    coords = [np.clip(z + u[2].astype(np.float64), 0, nz - 1), np.clip(y + u[1].astype(np.float64), 0, ny - 1),
              np.clip(x + u[0].astype(np.float64), 0, nx - 1)]
    val = ndimage.map_coordinates(m.astype(np.float64), coords, order=1, mode="nearest")
    decided = np.abs(val - 0.5) > 1e-9
    np.testing.assert_array_equal(got[decided], (val >= 0.5)[decided])
    np.testing.assert_array_equal(np.sort(knife), np.flatnonzero(np.abs(val - 0.5) <= ev.KNIFE_EDGE))


def test_evaluate_flips_only_knife_edge_voxels():
    """A knife-edge voxel decided the other way changes the overlap counts by one; any other
    voxel is refused."""
    T = np.zeros((8, 9, 10), np.uint8)
    T[2:6, 3:7, 3:8] = 1
    u = np.zeros((3,) + T.shape, np.float32)
    u[0] = 0.5
    img = T.astype(np.float32)
    r0 = ev.evaluate(img, img, T[None], T[None], u, spacing=(1, 1, 1), radius=0)
    knife = r0["structures"][0]["knife_edge"]
    assert len(knife) == 32
    r1 = ev.evaluate(img, img, T[None], T[None], u, spacing=(1, 1, 1), radius=0, flips=[knife[:1]])
    assert r1["structures"][0]["deformed"] == r0["structures"][0]["deformed"] - 1
    with pytest.raises(ValueError):
        ev.evaluate(img, img, T[None], T[None], u, spacing=(1, 1, 1), radius=0, flips=[[0]])


def test_evaluate_identity_and_known_shift():
    """Identical images and masks under u = 0: RMS-ID 0, CC 1, DSC 1, and the contour of each
    opened structure within one voxel of its own surface; a whole-voxel shift field moves a
    cube by exactly that shift."""
    from paper_1301_0970_amd import phantom as P
    pair = P.plain_pair(dims=(40, 36, 24), amp=2.0, iters=1)
    z = np.zeros((3,) + pair.target.shape, np.float32)
    r = ev.evaluate(pair.target, pair.target, pair.target_masks, pair.target_masks, z)
    assert r["whole"]["rms_id"] == 0.0 and r["whole"]["cc"] == pytest.approx(1.0, rel=1e-12)
    s = r["structures"][0]
    assert s["dsc"] == 1.0
    assert 0.0 <= s["ssd"]["mean"] <= 2.5 and s["ssd"]["points"] > 0
    T = np.zeros((16, 16, 20), np.uint8)
    T[3:13, 3:13, 4:14] = 1
    M = np.zeros_like(T)
    M[3:13, 3:13, 6:16] = 1          # the moving cube sits 2 voxels further along x
    u = np.zeros((3,) + T.shape, np.float32)
    u[0] = 2.0                       # pull-back: I0 o u (x) = I0(x + 2) brings it back
    r = ev.evaluate(T.astype(np.float32), M.astype(np.float32), T[None], M[None], u, spacing=(1, 1, 1), radius=0)
    s = r["structures"][0]
    assert s["dsc"] == 1.0 and s["ssd"]["mean"] == 0.0 and s["ssd"]["p95"] == 0.0
