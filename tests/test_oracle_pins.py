"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: hand-worked values
of Eq.7 (tests/golden), numerical minimisation of Eq.6, library routines that compute
the same textbook operation (scipy's Gaussian filter, linear map_coordinates, binary
dilation), closed forms on ramps / affine / quadratic fields, and invariants (identity,
scale invariance, constants).  Together they are meant to catch a dropped term, a wrong
sign or index, or a transposed operand anywhere in the oracle.
"""
import os

import numpy as np
import pytest
from scipy import ndimage, optimize

from paper_1301_0970_amd import phantom as P

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rows(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append([float(v) for v in line.split()])
    return rows


def _grid(shape):
    nz, ny, nx = shape
    return np.meshgrid(np.arange(nz, dtype=float), np.arange(ny, dtype=float),
                       np.arange(nx, dtype=float), indexing="ij")


# ------------------------------------------------------------------ Eq.7 (section 2.1)

def test_eq7_hand_worked(orc):
    """Eq.7 on hand-worked cases (tests/golden/eq7_worked.txt)."""
    for r in _rows("eq7_worked.txt"):
        a0, d, k = r[0], r[1], int(r[2])
        lam = [r[3 + 3 * i] for i in range(k)]
        a = [r[4 + 3 * i] for i in range(k)]
        di = [r[5 + 3 * i] for i in range(k)]
        num, den = r[3 + 3 * k], r[4 + 3 * k]
        assert orc.eq7(a0, d, lam, a, di) == pytest.approx(num / den, rel=1e-15)


def _E1(v, a0, d, lam, a, di):
    """Eq.6 with beta = d^2: the linearised energy along n."""
    e = 0.5 * (a0 * v - d) ** 2 + 0.5 * d * d * v * v
    for li, ai, dd in zip(lam, a, di):
        e += 0.5 * li * (ai * v - dd) ** 2
    return e


def test_eq7_is_argmin_of_eq6(orc):
    """P1: the closed form of Eq.7 minimises Eq.6 (numerical minimisation)."""
    rng = np.random.default_rng(1)
    for _ in range(2000):
        k = int(rng.integers(0, 9))
        a0 = float(rng.uniform(0.1, 300))
        d = float(rng.normal(0, 100))
        lam = rng.uniform(0, 2e-3, k)
        a = rng.normal(0, 500, k)
        di = rng.normal(0, 500, k)
        v = orc.eq7(a0, d, lam, a, di)
        # E1 is quadratic in v: recover its vertex from three evaluations
        e0, ep, em = (_E1(t, a0, d, lam, a, di) for t in (0.0, 1.0, -1.0))
        A = 0.5 * (ep + em) - e0
        B = 0.5 * (ep - em)
        assert v == pytest.approx(-B / (2 * A), rel=1e-9, abs=1e-12)
    for _ in range(100):
        k = int(rng.integers(1, 5))
        a0 = float(rng.uniform(1, 50))
        d = float(rng.normal(0, 30))
        lam = rng.uniform(0, 1e-2, k)
        a = rng.normal(0, 50, k)
        di = rng.normal(0, 50, k)
        res = optimize.minimize_scalar(lambda t: _E1(t, a0, d, lam, a, di), bracket=(-5, 5),
                                       tol=1e-12)
        assert orc.eq7(a0, d, lam, a, di) == pytest.approx(res.x, abs=1e-6)


def test_demons_special_case_and_bound(orc):
    """P2: with k = 0 the step is Thirion's demons force d g / (|g|^2 + d^2), |du| <= 1/2."""
    rng = np.random.default_rng(2)
    shape = (6, 7, 9)
    wI0 = rng.normal(0, 100, shape)
    T0 = rng.normal(0, 100, shape)
    du = orc.force(wI0, T0, [], [], [])
    g = orc.gradient(wI0)
    d = T0 - wI0
    expect = d * g / ((g * g).sum(0) + d * d)
    np.testing.assert_allclose(du, expect, rtol=1e-12, atol=1e-15)
    assert np.sqrt((du * du).sum(0)).max() <= 0.5 + 1e-12


def test_force_minimises_linearised_energy_along_n(orc):
    """P1 at the voxel level: du = v n minimises Eq.5 restricted to du in span(n), with
    n along the gradient of the warped moving image and the modified images' gradients."""
    rng = np.random.default_rng(3)
    shape = (5, 6, 7)
    k = 3
    wI0 = rng.normal(0, 50, shape)
    T0 = rng.normal(0, 50, shape)
    wIp = [rng.normal(1000, 80, shape) for _ in range(k)]
    Tp = [rng.normal(1000, 80, shape) for _ in range(k)]
    lam = [1e-3, 5e-3, 2e-2]
    du = orc.force(wI0, T0, wIp, Tp, lam)
    g0 = orc.gradient(wI0)
    gi = [orc.gradient(w) for w in wIp]
    for (l, j, i) in [(2, 3, 3), (0, 0, 0), (4, 5, 6), (1, 2, 5)]:
        n = g0[:, l, j, i] / np.linalg.norm(g0[:, l, j, i])

        def energy(t):
            dv = t * n
            e = 0.5 * (g0[:, l, j, i] @ dv - (T0 - wI0)[l, j, i]) ** 2
            e += 0.5 * ((T0 - wI0)[l, j, i] ** 2) * (dv @ dv)
            for s in range(k):
                e += 0.5 * lam[s] * (gi[s][:, l, j, i] @ dv - (Tp[s] - wIp[s])[l, j, i]) ** 2
            return e
        res = optimize.minimize_scalar(energy, bracket=(-3, 3), tol=1e-12)
        np.testing.assert_allclose(du[:, l, j, i], res.x * n, atol=1e-6)
        # the step is along n
        assert abs(np.cross(du[:, l, j, i], n)).max() < 1e-12


def test_zero_gradient_gives_zero_step(orc):
    """Reading: where grad I0~ = 0 the direction n is undefined and du = 0."""
    shape = (4, 5, 6)
    wI0 = np.full(shape, 7.0)
    T0 = np.full(shape, 9.0)
    du = orc.force(wI0, T0, [wI0 + 1000], [T0 + 1000], [1e-3])
    assert np.all(du == 0.0)


# ------------------------------------------------------------------ the ramp (worked)

def test_ramp_step_hand_worked(orc):
    """P3: on a ramp one full iteration moves the interior by -(s+c)/(1+(s+c)^2)
    (tests/golden/ramp_step.txt); the sign drives u towards -s."""
    shape = (24, 20, 40)
    z, y, x = _grid(shape)
    for a, s, c, expect in _rows("ramp_step.txt"):
        I0 = a * x
        T0 = a * (x - s)
        u = np.zeros((3,) + shape)
        u[0] = c
        un, _ = orc.step(I0, T0, [], [], [], 1.0, 1.0, u)
        # interior: away from the x borders by the gather range + both smoothing radii
        core = un[:, 8:-8, 8:-8, 12:-12]
        np.testing.assert_allclose(core[0], expect, atol=1e-12)
        np.testing.assert_allclose(core[1:], 0.0, atol=1e-12)


def test_ramp_iterates_to_the_shift(orc):
    shape = (20, 16, 48)
    z, y, x = _grid(shape)
    I0 = 10.0 * x
    T0 = 10.0 * (x - 2.0)
    u = np.zeros((3,) + shape)
    for _ in range(40):
        u, _ = orc.step(I0, T0, [], [], [], 1.0, 1.0, u)
    np.testing.assert_allclose(u[0, 8:-8, 6:-6, 20:-20], -2.0, atol=1e-6)


# ------------------------------------------------------------------ Gaussian (section 2.2)

@pytest.mark.parametrize("sigma", [1.0, 1.5, 0.7])
def test_gaussian_matches_scipy(orc, sigma):
    """P7: separable sampled Gaussian with clamped borders == scipy's gaussian_filter
    (mode 'nearest' replicates the edge; truncate 3 gives radius ceil(3 sigma) here)."""
    rng = np.random.default_rng(4)
    f = rng.normal(0, 1, (11, 13, 17))
    R = int(np.ceil(3 * sigma))
    truncate = (R + 0.25) / sigma   # scipy radius = int(truncate * sigma + 0.5) = R
    ref = ndimage.gaussian_filter(f, sigma, mode="nearest", truncate=truncate)
    np.testing.assert_allclose(orc.smooth(f, sigma), ref, rtol=0, atol=1e-13)
    w = orc.gauss_weights(sigma)
    assert len(w) == 2 * R + 1 and abs(w.sum() - 1) < 1e-15


def test_gaussian_invariants(orc):
    rng = np.random.default_rng(5)
    c = np.full((9, 9, 9), 3.25)
    np.testing.assert_allclose(orc.smooth(c, 1.0), 3.25, rtol=1e-15)
    imp = np.zeros((9, 9, 9))
    imp[4, 4, 4] = 1.0
    w = orc.gauss_weights(1.0)
    outer = w[:, None, None] * w[None, :, None] * w[None, None, :]
    np.testing.assert_allclose(orc.smooth(imp, 1.0)[1:8, 1:8, 1:8], outer, atol=1e-17)
    # direct 3D convolution with per-axis clamped indices, brute force
    f = rng.normal(0, 1, (5, 6, 7))
    out = np.zeros_like(f)
    R = 3
    for l in range(5):
        for j in range(6):
            for i in range(7):
                s = 0.0
                for cc in range(-R, R + 1):
                    for b in range(-R, R + 1):
                        for a in range(-R, R + 1):
                            s += (w[a + R] * w[b + R] * w[cc + R]
                                  * f[min(max(l + cc, 0), 4), min(max(j + b, 0), 5), min(max(i + a, 0), 6)])
                out[l, j, i] = s
    np.testing.assert_allclose(orc.smooth(f, 1.0), out, atol=1e-13)


# ------------------------------------------------------------------ interpolation

def test_trilinear_matches_map_coordinates(orc):
    """P8: trilinear with clamped positions == scipy map_coordinates(order=1, 'nearest')."""
    rng = np.random.default_rng(6)
    f = rng.normal(0, 1, (6, 7, 8))
    u = rng.uniform(-3, 3, (3, 6, 7, 8))
    z, y, x = _grid(f.shape)
    coords = np.stack([z + u[2], y + u[1], x + u[0]])
    ref = ndimage.map_coordinates(f, coords, order=1, mode="nearest")
    np.testing.assert_allclose(orc.warp(f, u), ref, atol=1e-13)
    assert orc.sample(f, 2.5, 3.25, 1.75) == pytest.approx(
        ndimage.map_coordinates(f, [[1.75], [3.25], [2.5]], order=1, mode="nearest")[0], abs=1e-14)


def test_trilinear_exact_on_affine_and_shifts(orc):
    shape = (8, 9, 10)
    z, y, x = _grid(shape)
    f = 3.0 + 0.5 * x - 2.0 * y + 0.25 * z
    u = np.zeros((3,) + shape)
    u[0], u[1], u[2] = 0.3, -0.6, 0.45
    w = orc.warp(f, u)
    inner = (slice(1, -1), slice(1, -1), slice(1, -1))
    expect = 3.0 + 0.5 * (x + 0.3) - 2.0 * (y - 0.6) + 0.25 * (z + 0.45)
    np.testing.assert_allclose(w[inner], expect[inner], atol=1e-12)
    u[:] = 0
    u[0] = 2.0
    np.testing.assert_array_equal(orc.warp(f, u)[:, :, :-2], f[:, :, 2:])


def test_mask_warp_threshold(orc):
    m = np.zeros((3, 3, 8), np.uint8)
    m[:, :, 4:] = 1
    u = np.zeros((3, 3, 3, 8))
    u[0] = 0.5   # samples half way: value 0.5 at x = 3 counts as inside
    out = orc.warp_mask(m, u)
    np.testing.assert_array_equal(out[1, 1], [0, 0, 0, 1, 1, 1, 1, 1])
    u[0] = 0.49
    np.testing.assert_array_equal(orc.warp_mask(m, u)[1, 1], [0, 0, 0, 0, 1, 1, 1, 1])


# ------------------------------------------------------------------ gradient

def test_central_differences(orc):
    """P9: exact on quadratics in the interior; == numpy's central differences there."""
    shape = (7, 8, 9)
    z, y, x = _grid(shape)
    f = x * x - 3 * y * y + 0.5 * z * z + x * y
    g = orc.gradient(f)
    inner = (slice(1, -1), slice(1, -1), slice(1, -1))
    np.testing.assert_allclose(g[0][inner], (2 * x + y)[inner], atol=1e-12)
    np.testing.assert_allclose(g[1][inner], (-6 * y + x)[inner], atol=1e-12)
    np.testing.assert_allclose(g[2][inner], z[inner], atol=1e-12)
    rng = np.random.default_rng(7)
    r = rng.normal(0, 1, shape)
    gz, gy, gx = np.gradient(r)
    gr = orc.gradient(r)
    np.testing.assert_allclose(gr[0][:, :, 1:-1], gx[:, :, 1:-1], atol=1e-14)
    np.testing.assert_allclose(gr[1][:, 1:-1], gy[:, 1:-1], atol=1e-14)
    np.testing.assert_allclose(gr[2][1:-1], gz[1:-1], atol=1e-14)
    # clamped border: half the one-sided difference
    np.testing.assert_allclose(gr[0][:, :, 0], 0.5 * (r[:, :, 1] - r[:, :, 0]), atol=1e-14)


# ------------------------------------------------------------------ composite update

def test_compose_identities(orc):
    """P10: du = 0 keeps u; constant u = c gives du + c; affine u is exact inside."""
    rng = np.random.default_rng(8)
    shape = (6, 7, 8)
    u = rng.normal(0, 1, (3,) + shape)
    np.testing.assert_array_equal(orc.compose(u, np.zeros_like(u)), u)
    du = rng.uniform(-0.5, 0.5, (3,) + shape)
    c = np.zeros_like(u)
    c[0], c[1], c[2] = 1.5, -0.25, 2.0
    np.testing.assert_allclose(orc.compose(c, du), du + c, atol=1e-14)
    z, y, x = _grid(shape)
    A = np.array([[0.1, -0.2, 0.05], [0.0, 0.3, -0.1], [0.2, 0.1, 0.0]])
    b = np.array([0.5, -1.0, 0.25])
    pos = np.stack([x, y, z])
    ua = np.einsum("ij,j...->i...", A, pos) + b[:, None, None, None]
    dv = rng.uniform(-0.4, 0.4, (3,) + shape)
    expect = dv + np.einsum("ij,j...->i...", A, pos + dv) + b[:, None, None, None]
    inner = (slice(None), slice(1, -1), slice(1, -1), slice(1, -1))
    np.testing.assert_allclose(orc.compose(ua, dv)[inner], expect[inner], atol=1e-12)


# ------------------------------------------------------------------ pyramid

def test_restrict_matches_filter_then_decimate(orc):
    """P11: restriction == scipy Gaussian (sigma 1, clamped) then every other voxel."""
    rng = np.random.default_rng(9)
    for shape in [(9, 10, 11), (8, 8, 8), (1, 3, 5)]:
        f = rng.normal(0, 1, shape)
        ref = ndimage.gaussian_filter(f, 1.0, mode="nearest", truncate=3.25)[::2, ::2, ::2]
        out = orc.restrict(f, 1.0)
        assert out.shape == tuple((n + 1) // 2 for n in shape)
        np.testing.assert_allclose(out, ref, atol=1e-13)
    np.testing.assert_allclose(orc.restrict(np.full((7, 6, 5), 2.5)), 2.5, rtol=1e-15)


def test_prolong_constants_and_affine(orc):
    cshape = (4, 5, 6)
    fine = (11, 10, 8)    # (nx, ny, nz) with ceil(n/2) == coarse
    uc = np.zeros((3,) + cshape)
    uc[0], uc[1], uc[2] = 1.0, -2.0, 0.5
    uf = orc.prolong(uc, fine)
    assert uf.shape == (3, 8, 10, 11)
    np.testing.assert_allclose(uf[0], 2.0)
    np.testing.assert_allclose(uf[1], -4.0)
    z, y, x = _grid(cshape)
    uc[0] = 0.25 * x - 0.5 * y + z
    uf = orc.prolong(uc, fine)
    zf, yf, xf = _grid((8, 10, 11))
    expect = 2 * (0.25 * xf / 2 - 0.5 * yf / 2 + zf / 2)
    inner = (xf / 2 <= 5) & (yf / 2 <= 4) & (zf / 2 <= 3)
    np.testing.assert_allclose(uf[0][inner], expect[inner], atol=1e-12)


def test_decimate_masks_closed_form(orc):
    """Masks at a coarser level (contour terms below the finest level): a fine box
    [a, b] (inclusive, per axis) becomes the coarse box [ceil(a/2), floor(b/2)], and after two
    levels [ceil(a/4), floor(b/4)]; any nonzero fine value counts as inside; dims ceil(n/2)."""
    shape = (13, 19, 23)                       # (nz, ny, nx)
    lo, hi = (3, 5, 2), (10, 12, 19)           # z, y, x bounds of the box
    m = np.zeros((2,) + shape, np.uint8)
    m[0][lo[0]:hi[0] + 1, lo[1]:hi[1] + 1, lo[2]:hi[2] + 1] = 7
    m[1][12, 18, 22] = 255                     # the last voxel, all indices even
    m[1][8, 16, 20] = 1                        # indices divisible by 4
    m[1][11, 0, 0] = 1                         # odd z index: dropped
    c1 = orc.decimate_masks(m)
    c2 = orc.decimate_masks(c1)
    assert c1.shape == (2, 7, 10, 12) and c2.shape == (2, 4, 5, 6)
    for c, f in ((c1, 2), (c2, 4)):
        box = np.zeros(c.shape[1:], np.uint8)
        box[-(-lo[0] // f):hi[0] // f + 1, -(-lo[1] // f):hi[1] // f + 1, -(-lo[2] // f):hi[2] // f + 1] = 1
        np.testing.assert_array_equal(c[0], box)
    assert sorted(map(tuple, np.argwhere(c1[1]))) == [(4, 8, 10), (6, 9, 11)]
    assert sorted(map(tuple, np.argwhere(c2[1]))) == [(2, 4, 5)]
    assert c1.max() == 1


# ------------------------------------------------------------------ UROI and signs

def test_uroi_matches_binary_dilation(orc):
    """P12: UROI == scipy binary dilation of the union with the ellipsoid element."""
    rng = np.random.default_rng(10)
    shape = (14, 20, 22)
    masks = (rng.uniform(size=(2,) + shape) > 0.995).astype(np.uint8)
    r = (5, 5, 4)
    c, b, a = np.meshgrid(np.arange(-r[2], r[2] + 1), np.arange(-r[1], r[1] + 1),
                          np.arange(-r[0], r[0] + 1), indexing="ij")
    elem = (a / r[0]) ** 2 + (b / r[1]) ** 2 + (c / r[2]) ** 2 <= 1.0
    ref = ndimage.binary_dilation(masks.any(0), structure=elem)
    np.testing.assert_array_equal(orc.uroi(masks, r), ref.astype(np.uint8))


def test_auto_sign(orc):
    shape = (20, 24, 24)
    T0 = np.full(shape, 40.0)
    m = np.zeros(shape, np.uint8)
    m[8:12, 9:15, 9:15] = 1
    T0[m == 1] = 60.0
    assert orc.auto_sign(T0, m) == 1
    T0[m == 1] = 20.0
    assert orc.auto_sign(T0, m) == -1


def test_modified_image_definition(orc):
    """Section 2.1: I_i = (1 + M_i/2) I with M_i = +-1 inside the structure, 0 outside,
    on CT numbers (HU + c0)."""
    F = np.array([-1000.0, 40.0, 55.0, 1200.0]).reshape(1, 1, 4)
    m = np.array([0, 1, 1, 0], np.uint8).reshape(1, 1, 4)
    np.testing.assert_allclose(orc.modified_image(F, m, 1).ravel(), [0.0, 1560.0, 1582.5, 2200.0])
    np.testing.assert_allclose(orc.modified_image(F, m, -1).ravel(), [0.0, 520.0, 527.5, 2200.0])


# ------------------------------------------------------------------ whole-algorithm invariants

def _small_pair(**kw):
    return P.plain_pair(dims=(24, 20, 16), amp=2.0, **kw)


def test_identity_gives_zero_field(orc):
    """P4: identical images and masks -> du == 0 everywhere, u stays exactly 0."""
    p = _small_pair()
    for mask in (1, 3):   # contour terms at the finest level only, and at both levels
        prm = orc.params_for(p, levels=2, iters=(5, 5), contour_level_mask=mask)
        u, _, _ = orc.register(p.target, p.target, p.target_masks, p.target_masks, prm)
        assert np.all(u == 0.0)


def test_contour_term_vanishes_when_masks_agree(orc):
    """P5: identical images and masks -> the contour numerator sum lam a_i d_i is 0, so du
    is unchanged by lambda; with the moving mask shifted the contour term moves u toward
    the shift, only near the structure."""
    shape = (20, 24, 32)
    z, y, x = _grid(shape)
    rng = np.random.default_rng(11)
    img = 40.0 + 20.0 * np.sin(x / 3.0) * np.cos(y / 4.0) + rng.normal(0, 5, shape)
    tm = ((x - 15) ** 2 / 36 + (y - 12) ** 2 / 25 + (z - 10) ** 2 / 16 <= 1).astype(np.uint8)
    lamb = [1e-2]
    Ip = [orc.modified_image(img, tm, 1)]
    Tp = [orc.modified_image(img, tm, 1)]
    du = orc.force(img, img, Ip, Tp, lamb)
    assert np.all(du == 0.0)
    # moving mask displaced by +2 in x: I(x + 2) carries the target structure, u* = +2
    mm = np.roll(tm, 2, axis=2)
    Ip = [orc.modified_image(img, mm, 1)]
    du = orc.force(img, img, Ip, Tp, lamb)
    near = ndimage.binary_dilation(tm | mm, iterations=2)
    assert du[0][near].mean() > 0.05
    assert np.abs(du[:, ~ndimage.binary_dilation(near, iterations=2)]).max() == 0.0


def test_scale_invariance(orc):
    """P6: (I0, T0, c0) -> (a I0, a T0, a c0) leaves the result unchanged (Eq.7 is
    homogeneous of degree 0 in the intensities)."""
    p = _small_pair()
    prm = orc.params_for(p, levels=1, iters=(4,))
    u1, _, _ = orc.register(p.target, p.moving, p.target_masks, p.moving_masks, prm)
    prm.c0 = 1000.0 * 3.5
    u2, _, _ = orc.register(3.5 * p.target.astype(float), 3.5 * p.moving.astype(float),
                            p.target_masks, p.moving_masks, prm)
    np.testing.assert_allclose(u1, u2, atol=1e-12)


def test_recovery_of_known_deformation(orc):
    """P13: a known smooth deformation is recovered within 0.5 voxel RMS over the body
    of a textured phantom (3 levels x 100 iterations)."""
    p = P.plain_pair(texture_hu=100.0, levels=3, iters=100)
    gt = P.ground_truth_u(p)
    u, _, _ = orc.register(p.target, p.moving, p.target_masks, p.moving_masks, orc.params_for(p))
    z, y, x = _grid(p.target.shape)
    body = p.phantom[0].inside(x, y, z)
    err = np.sqrt(((u - gt) ** 2).sum(0))[body]
    init = np.sqrt((gt ** 2).sum(0))[body]
    rms = np.sqrt((err ** 2).mean())
    assert rms <= 0.5, rms
    assert rms < 0.5 * np.sqrt((init ** 2).mean())


def test_contour_term_improves_dice(orc):
    """P14 (directional, Table 2): on low-contrast structures the contour term raises the
    Dice overlap of the propagated moving masks with the target masks."""
    p = P.head_neck_pair(dims=(64, 64, 40), amp=4.0, k=3, levels=2, iters=60, sigma=1.5)

    def dice(prm):
        u, _, _ = orc.register(p.target, p.moving, p.target_masks, p.moving_masks, prm)
        out = []
        for i in range(p.k):
            w = orc.warp_mask(p.moving_masks[i], u).astype(bool)
            t = p.target_masks[i].astype(bool)
            out.append(2 * (w & t).sum() / (w.sum() + t.sum()))
        return np.array(out)
    with_c = dice(orc.params_for(p))
    without = dice(orc.params_for(p, lambdas=[0.0] * p.k))
    assert with_c.mean() > without.mean(), (with_c, without)


def test_stopping_rule(orc):
    """Stopping rule (section 2.2, read as: after every 10 finest-level iterations stop when
    delta_{n-10} - delta_n <= eps)."""
    p = _small_pair()
    base = dict(levels=1, iters=(60,), stop_mode=1)
    _, h, n = orc.register(p.target, p.moving, p.target_masks, p.moving_masks,
                           orc.params_for(p, stop_eps=1e9, **base), want_delta=True)
    assert n == 20 and len(h) == 20
    _, h, n = orc.register(p.target, p.moving, p.target_masks, p.moving_masks,
                           orc.params_for(p, stop_eps=-1e9, **base), want_delta=True)
    assert n == 60
    eps = float(np.median(h[9:50] - h[19:60]))
    _, h2, n2 = orc.register(p.target, p.moving, p.target_masks, p.moving_masks,
                             orc.params_for(p, stop_eps=eps, **base), want_delta=True)
    np.testing.assert_array_equal(h2, h[:n2])
    first = next(m for m in range(19, 60, 10) if h[m - 10] - h[m] <= eps)
    assert n2 == first + 1
    # delta is the UROI RMS of (T0 - I0~) / 2500 at the current field: check iteration 0
    ur = orc.uroi(p.target_masks)
    d0 = (p.target.astype(float) - p.moving.astype(float))[ur == 1] / 2500.0
    assert h[0] == pytest.approx(np.sqrt((d0 ** 2).mean()), rel=1e-12)


def test_step_matches_register_single_iteration(orc):
    """The step entry point and Algorithm A agree for one finest-level iteration from a
    given field (warm start)."""
    p = _small_pair()
    u0 = P.random_smooth_field(p.dims, 1.5, 5)
    prm = orc.params_for(p, levels=1, iters=(1,))
    u_reg, _, _ = orc.register(p.target, p.moving, p.target_masks, p.moving_masks, prm, initial_u=u0)
    Ip = [orc.modified_image(p.moving, p.moving_masks[i], 1) for i in range(p.k)]
    Tp = [orc.modified_image(p.target, p.target_masks[i], 1) for i in range(p.k)]
    u_step, _ = orc.step(p.moving, p.target, Ip, Tp, [1e-3] * p.k, p.sigma, p.sigma, u0)
    np.testing.assert_array_equal(u_reg, u_step)


def _scipy_step(I0, T0, Ip, Tp, lam, sf, sd, u, h=(1.0, 1.0, 1.0)):
    """One iteration of Algorithm A's loop rebuilt from library routines: linear
    map_coordinates (warp and composition), edge-padded central differences, Eq.7 in
    numpy, scipy's Gaussian filter for both smoothings."""
    z, y, x = _grid(I0.shape)

    def warp(f, v):
        return ndimage.map_coordinates(f, [z + v[2], y + v[1], x + v[0]], order=1, mode="nearest")

    def grad(f):   # per unit of h
        p = np.pad(f, 1, mode="edge")
        return np.stack([(p[1:-1, 1:-1, 2:] - p[1:-1, 1:-1, :-2]) / (2 * h[0]),
                         (p[1:-1, 2:, 1:-1] - p[1:-1, :-2, 1:-1]) / (2 * h[1]),
                         (p[2:, 1:-1, 1:-1] - p[:-2, 1:-1, 1:-1]) / (2 * h[2])])

    def gauss(f, s):   # sigma s in the unit of h: s / h voxels along each axis, radius ceil(3 sigma)
        sv = [s / h[2], s / h[1], s / h[0]]
        return ndimage.gaussian_filter(f, sv, mode="nearest", radius=[int(np.ceil(3 * v)) for v in sv])

    wI0 = warp(I0, u)
    g0 = grad(wI0)
    a0 = np.sqrt((g0 * g0).sum(0))
    n = g0 / a0
    d = T0 - wI0
    num = a0 * d
    den = a0 * a0 + d * d
    for li, I, T in zip(lam, Ip, Tp):
        wI = warp(I, u)
        ai = (grad(wI) * n).sum(0)
        num = num + li * ai * (T - wI)
        den = den + li * ai * ai
    du = (num / den) * n / np.asarray(h, float)[:, None, None, None]    # to voxels
    dus = np.stack([gauss(c, sf) for c in du])
    uc = dus + np.stack([warp(c, dus) for c in u])
    return np.stack([gauss(c, sd) for c in uc])


def test_step_follows_algorithm_a(orc):
    """The oracle's iteration == the same iteration rebuilt from library routines, in
    Algorithm A's order: Eq.7 -> smooth du -> composite update -> smooth u."""
    p = P.head_neck_pair(dims=(40, 36, 24), amp=3.0, k=2, levels=1, iters=1)
    u0 = P.random_smooth_field(p.dims, 2.0, 9).astype(float)
    Ip = [orc.modified_image(p.moving, p.moving_masks[i], 1) for i in range(p.k)]
    Tp = [orc.modified_image(p.target, p.target_masks[i], 1) for i in range(p.k)]
    lam = [1e-3, 4e-3]
    un, _ = orc.step(p.moving, p.target, Ip, Tp, lam, 1.5, 1.0, u0)
    ref = _scipy_step(p.moving.astype(float), p.target.astype(float), Ip, Tp, lam, 1.5, 1.0, u0)
    np.testing.assert_allclose(un, ref, atol=1e-9)


def test_contour_terms_at_a_coarse_level_follow_algorithm_a(orc):
    """Contour terms at the coarse level of a two-level pyramid (the finest level runs no
    iteration): the result equals Algorithm A's loop rebuilt from library routines at that
    level, on images restricted by scipy's Gaussian then every other voxel and on masks
    taken at the even voxels, then prolongated as 2 u(x / 2) by scipy's linear interpolation."""
    p = P.head_neck_pair(dims=(38, 34, 22), amp=3.0, k=2, levels=2, iters=1)
    lam = [2e-3, 5e-3]
    prm = orc.params_for(p, levels=2, iters=(0, 3), lambdas=lam, contour_level_mask=2)
    u, _, _ = orc.register(p.target, p.moving, p.target_masks, p.moving_masks, prm)

    def down(f):
        return ndimage.gaussian_filter(f.astype(float), 1.0, mode="nearest", truncate=3.25)[::2, ::2, ::2]
    I0, T0 = down(p.moving), down(p.target)
    mm, tm = p.moving_masks[:, ::2, ::2, ::2], p.target_masks[:, ::2, ::2, ::2]
    Ip = [orc.modified_image(I0, mm[i], p.signs[i]) for i in range(p.k)]
    Tp = [orc.modified_image(T0, tm[i], p.signs[i]) for i in range(p.k)]
    uc = np.zeros((3,) + I0.shape)
    for _ in range(3):
        uc = _scipy_step(I0, T0, Ip, Tp, lam, p.sigma, p.sigma, uc)
    z, y, x = _grid(p.target.shape)
    ref = np.stack([2.0 * ndimage.map_coordinates(c, [z / 2, y / 2, x / 2], order=1, mode="nearest")
                    for c in uc])
    np.testing.assert_allclose(u, ref, atol=1e-9)
    # the same run without contour terms differs, and contour bits beyond the levels are refused
    u0, _, _ = orc.register(p.target, p.moving, p.target_masks, p.moving_masks,
                            orc.params_for(p, levels=2, iters=(0, 3), lambdas=lam, contour_level_mask=0))
    assert np.abs(u - u0).max() > 1e-3
    with pytest.raises(ValueError):
        orc.register(p.target, p.moving, p.target_masks, p.moving_masks,
                     orc.params_for(p, levels=2, iters=(0, 3), contour_level_mask=4))


def test_step_in_physical_units_follows_algorithm_a(orc):
    """With a voxel size h the gradients are per unit of h, Eq.7's step v n is in that unit and
    becomes h-scaled voxels, and both Gaussians take sigma in that unit (sigma / h voxels per
    axis): the oracle's iteration == the same iteration rebuilt from library routines."""
    p = P.head_neck_pair(dims=(40, 36, 24), amp=3.0, k=2, levels=1, iters=1)
    u0 = P.random_smooth_field(p.dims, 2.0, 9).astype(float)
    Ip = [orc.modified_image(p.moving, p.moving_masks[i], 1) for i in range(p.k)]
    Tp = [orc.modified_image(p.target, p.target_masks[i], 1) for i in range(p.k)]
    lam = [1e-3, 4e-3]
    h = (1.97, 1.6, 2.5)
    un, _ = orc.step(p.moving, p.target, Ip, Tp, lam, 3.0, 2.2, u0, spacing=h)
    ref = _scipy_step(p.moving.astype(float), p.target.astype(float), Ip, Tp, lam, 3.0, 2.2, u0, h=h)
    np.testing.assert_allclose(un, ref, atol=1e-9)
    # a unit voxel size is the voxel-unit iteration itself
    a, _ = orc.step(p.moving, p.target, Ip, Tp, lam, 1.5, 1.0, u0, spacing=(1.0, 1.0, 1.0))
    b, _ = orc.step(p.moving, p.target, Ip, Tp, lam, 1.5, 1.0, u0)
    np.testing.assert_array_equal(a, b)


def test_anisotropic_gaussian_and_gradient(orc):
    rng = np.random.default_rng(12)
    f = rng.normal(0, 1, (11, 13, 17))
    sig = (1.3, 0.7, 2.0)                      # x, y, z voxels
    rad = [int(np.ceil(3 * v)) for v in sig[::-1]]
    ref = ndimage.gaussian_filter(f, sig[::-1], mode="nearest", radius=rad)
    np.testing.assert_allclose(orc.smooth_axes(f, sig), ref, rtol=0, atol=1e-13)
    # central differences per unit length: exact on quadratics of the physical coordinates
    h = (1.97, 1.5, 2.5)
    z, y, x = _grid((7, 8, 9))
    X, Y, Z = x * h[0], y * h[1], z * h[2]
    g = orc.gradient(X * X - 3 * Y * Y + 0.5 * Z * Z + X * Y, spacing=h)
    inner = (slice(1, -1), slice(1, -1), slice(1, -1))
    np.testing.assert_allclose(g[0][inner], (2 * X + Y)[inner], atol=1e-11)
    np.testing.assert_allclose(g[1][inner], (-6 * Y + X)[inner], atol=1e-11)
    np.testing.assert_allclose(g[2][inner], Z[inner], atol=1e-11)


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("h", [(1.97, 1.97, 2.5), (0.9, 1.3, 2.5)], ids=["square in-plane", "x != y"])
def test_force_on_a_physical_ramp(orc, axis, h):
    """A ramp of slope a HU per unit length along one axis, target offset by c: the gradient
    is a, the demons step is c a / (a^2 + c^2) in length units, i.e. that over h voxels."""
    a, c = 40.0, 25.0
    z, y, x = _grid((9, 10, 11))
    coord = (x, y, z)[axis] * h[axis]
    I = a * coord
    du = orc.force(I, I + c, [], [], [], spacing=h)
    inner = (slice(1, -1), slice(1, -1), slice(1, -1))
    np.testing.assert_allclose(du[axis][inner], c * a / (a * a + c * c) / h[axis], rtol=1e-13)
    for other in {0, 1, 2} - {axis}:
        assert np.all(du[other][inner] == 0.0)
