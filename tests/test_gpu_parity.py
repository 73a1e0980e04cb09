"""Parity of the HIP path (through the C-ABI) with the FP64 oracle.

Tolerances are those of the method's acceptance bar: one teacher-forced iteration
agrees to 1e-4 voxel (max-abs over the field); a full registration to 1e-2 voxel, with
the warped moving images within 1e-3 of the 2500 HU intensity range (2.5 HU RMS).
"""
import numpy as np
import pytest

from paper_1301_0970_amd import phantom as P

pytestmark = pytest.mark.gpu

STEP_TOL = 1e-4
FINAL_TOL = 1e-2
WARP_RMS_TOL = 2.5


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1301_0970_amd import cgdir
    assert torch.cuda.is_available()
    c = cgdir.Context(6 << 30, max_slots=4)
    yield c
    c.close()


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def gpu_register(ctx, pair, prm, initial=None, delta=False, masks=True):
    from paper_1301_0970_amd import cgdir  # noqa: F401
    tm = dev(pair.target_masks) if masks and pair.k else None
    mm = dev(pair.moving_masks) if masks and pair.k else None
    res = ctx.register(dev(pair.target), dev(pair.moving), tm, mm, prm,
                       initial=dev(initial) if initial is not None else None, delta=delta)
    if delta:
        u, h, n = res
        return u.cpu().numpy(), np.array(h), n
    return res.cpu().numpy()


def oracle_step(orc, pair, u0, sigma_f, sigma_d, lambdas, signs, c0=1000.0):
    Ip = [orc.modified_image(pair.moving, pair.moving_masks[i], signs[i], c0) for i in range(len(lambdas))]
    Tp = [orc.modified_image(pair.target, pair.target_masks[i], signs[i], c0) for i in range(len(lambdas))]
    u, _ = orc.step(pair.moving, pair.target, Ip, Tp, lambdas, sigma_f, sigma_d, u0.astype(np.float64))
    return u


STEP_CASES = [
    # name, generator kwargs, k, sigma, field amplitude
    ("plain k1 ragged", dict(kind="plain", dims=(97, 45, 23), amp=3.0), 1, 1.0, 2.5),
    ("demons k0", dict(kind="plain", dims=(80, 72, 33), amp=3.0), 0, 1.0, 2.0),
    ("head_neck k3 sigma1.5", dict(kind="head_neck", dims=(130, 70, 40), amp=4.0, k=3), 3, 1.5, 3.0),
    ("head_neck k5 sigma1.5", dict(kind="head_neck", dims=(128, 96, 48), amp=5.0, k=5), 5, 1.5, 4.0),
    ("pelvis k8", dict(kind="pelvis", dims=(160, 136, 48), amp=6.0, k=8, bulge=3.0), 8, 1.0, 6.0),
    ("pelvis k2 thin", dict(kind="pelvis", dims=(200, 66, 9), amp=2.0, k=2, bulge=0.0), 2, 1.0, 1.5),
]


def _make(kind, **kw):
    if kind == "plain":
        return P.plain_pair(**kw)
    if kind == "head_neck":
        return P.head_neck_pair(**kw)
    return P.pelvis_pair(**kw)


@pytest.mark.parametrize("name,kw,k,sigma,famp", STEP_CASES, ids=[c[0] for c in STEP_CASES])
def test_teacher_forced_step(ctx, orc, name, kw, k, sigma, famp):
    """One iteration from the same fp32 field u^n: GPU vs FP64 oracle, <= 1e-4 voxel."""
    from paper_1301_0970_amd import cgdir
    pair = _make(**kw)
    if k == 0:
        pair.target_masks = pair.target_masks[:0]
        pair.moving_masks = pair.moving_masks[:0]
        pair.signs = ()
    u0 = P.random_smooth_field(pair.dims, famp, 101)
    lam = [1e-3 * (1 + i) for i in range(pair.k)]
    sg = [1 if i % 3 else -1 for i in range(pair.k)]
    prm = cgdir.make_params(levels=1, iters=(1,), sigma_fluid=sigma, sigma_diff=sigma, lambdas=lam, signs=sg)
    say("step case %s dims %s k %d" % (name, pair.dims, pair.k))
    ug = gpu_register(ctx, pair, prm, initial=u0)
    uo = oracle_step(orc, pair, u0, sigma, sigma, lam, sg)
    err = np.abs(ug - uo).max()
    say("  max |du| %.3g  max err %.3g" % (np.abs(uo - u0).max(), err))
    assert err <= STEP_TOL


@pytest.mark.parametrize("sigma", [1.0, 0.6], ids=["radius 3", "radius 2"])
def test_structures_at_every_border_under_every_tile_shape(ctx, orc, sigma):
    """Structures cut by the volume's faces (one around the corner (0, 0, 0), one around the
    opposite corner, one slab through every plane), so that the step kernel stages structure
    bits and K~ at clamped planes, rows and columns: one teacher-forced iteration under every
    tile shape the autotuner tries is bitwise the same field, and within 1e-4 voxel of the
    FP64 oracle (Gaussian radius 3 and 2, whose 16-row tiles stage K~ in LDS)."""
    from paper_1301_0970_amd import cgdir
    pair = P.plain_pair(dims=(140, 52, 20), amp=3.0)
    nx, ny, nz = pair.dims
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")

    def masks(d):  # d: shift of the moving masks against the target's
        a = ((x - d) ** 2 + (y - d) ** 2 + (z - d) ** 2 <= 11 ** 2)
        b = ((x - (nx - 1) + d) ** 2 + (y - (ny - 1)) ** 2 + (z - (nz - 1) + d) ** 2 <= 9 ** 2)
        c = (np.abs(x - 70 - d) <= 6) & (np.abs(y - 26) <= 8)
        return np.stack([a, b, c]).astype(np.uint8)
    pair.target_masks, pair.moving_masks, pair.signs = masks(0), masks(1), (1, -1, 1)
    u0 = P.random_smooth_field(pair.dims, 2.5, 303)
    lam, sg = [1e-3, 2e-3, 3e-3], [1, -1, 1]
    prm = cgdir.make_params(levels=1, iters=(1,), sigma_fluid=sigma, sigma_diff=sigma, lambdas=lam, signs=sg)
    say("structures at the borders: every tile shape (sigma %g)" % sigma)
    first = gpu_register(ctx, pair, prm, initial=u0)
    for i in range(18):               # the autotuner's candidate shapes, then the tuned one
        again = gpu_register(ctx, pair, prm, initial=u0)
        assert np.array_equal(first, again), i
    uo = oracle_step(orc, pair, u0, sigma, sigma, lam, sg)
    err = np.abs(first - uo).max()
    say("  max |du| %.3g  max err %.3g" % (np.abs(uo - u0).max(), err))
    assert err <= STEP_TOL


@pytest.mark.parametrize("n", [0, 1, 10, 50, 99])
def test_teacher_forced_step_along_the_oracle_trajectory(ctx, orc, n):
    """Config 1 (64x64x32, k = 1, 100 iterations): the oracle's own field after n iterations,
    rounded to FP32, is the start of one GPU iteration and of one FP64 oracle iteration; they
    agree to 1e-4 voxel at every n, from the first iteration to the last."""
    from paper_1301_0970_amd import cgdir
    pair = P.plain_pair()
    un, _, _ = orc.register(pair.target, pair.moving, pair.target_masks, pair.moving_masks,
                            orc.params_for(pair, iters=(n,)))
    u0 = un.astype(np.float32)
    prm = cgdir.params_for_pair(pair, iters=(1,))
    say("trajectory step from oracle iteration %d" % n)
    ug = gpu_register(ctx, pair, prm, initial=u0)
    uo, _, _ = orc.register(pair.target, pair.moving, pair.target_masks, pair.moving_masks,
                            orc.params_for(pair, iters=(1,)), initial_u=u0.astype(np.float64))
    err = np.abs(ug - uo).max()
    say("  max |u| %.3g, step up to %.3g, max err %.3g" % (np.abs(uo).max(), np.abs(uo - u0).max(), err))
    assert err <= STEP_TOL


def test_step_with_different_sigmas(ctx, orc):
    from paper_1301_0970_amd import cgdir
    pair = P.head_neck_pair(dims=(100, 90, 30), amp=4.0, k=2)
    u0 = P.random_smooth_field(pair.dims, 3.0, 7)
    prm = cgdir.make_params(levels=1, iters=(1,), sigma_fluid=2.0, sigma_diff=0.6, lambdas=[2e-3, 1e-3])
    say("step sigma_f 2.0 sigma_d 0.6")
    ug = gpu_register(ctx, pair, prm, initial=u0)
    uo = oracle_step(orc, pair, u0, 2.0, 0.6, [2e-3, 1e-3], [1, 1])
    assert np.abs(ug - uo).max() <= STEP_TOL


@pytest.mark.parametrize("spacing,sigma", [((1.97, 1.97, 2.5), 1.97), ((1.2, 1.2, 3.0), 2.0),
                                           ((0.9, 1.3, 2.5), 1.5), ((1.4, 0.8, 1.1), 1.2)],
                         ids=["1.97x1.97x2.5 mm sigma 1.97", "1.2x1.2x3 mm sigma 2",
                              "0.9x1.3x2.5 mm sigma 1.5", "1.4x0.8x1.1 mm sigma 1.2"])
def test_step_in_physical_units(ctx, orc, spacing, sigma):
    """Anisotropic voxels: gradients per mm, the step in mm converted to voxels, Gaussians of
    sigma mm (in the second case radius 5 in-plane and 2 or 3 along z: the z taps are
    zero-padded to the launch radius; in the last two x and y differ, with radii 5, 4, 2 and
    3, 5, 4 along x, y, z)."""
    from paper_1301_0970_amd import cgdir
    pair = P.head_neck_pair(dims=(110, 84, 40), amp=4.0, k=3)
    u0 = P.random_smooth_field(pair.dims, 3.0, 17)
    lam, sg = [1e-3, 2e-3, 3e-3], [1, -1, 1]
    prm = cgdir.make_params(levels=1, iters=(1,), sigma_fluid=sigma, sigma_diff=0.8 * sigma, lambdas=lam,
                            signs=sg, spacing=spacing)
    say("step in mm %s sigma %.2f" % (spacing, sigma))
    ug = gpu_register(ctx, pair, prm, initial=u0)
    Ip = [orc.modified_image(pair.moving, pair.moving_masks[i], sg[i]) for i in range(3)]
    Tp = [orc.modified_image(pair.target, pair.target_masks[i], sg[i]) for i in range(3)]
    h = [float(np.float32(v)) for v in spacing]
    uo, _ = orc.step(pair.moving, pair.target, Ip, Tp, lam, float(np.float32(sigma)),
                     float(np.float32(0.8 * sigma)), u0.astype(np.float64), spacing=h)
    err = np.abs(ug - uo).max()
    say("  max |du| %.3g  max err %.3g" % (np.abs(uo - u0).max(), err))
    assert err <= STEP_TOL


def test_pyramid_in_physical_units(ctx, orc):
    """Two levels with voxel size 1.97 x 1.97 x 2.5 mm (3.94 x 3.94 x 5 at the coarse level)."""
    from paper_1301_0970_amd import cgdir
    pair = P.head_neck_pair(dims=(90, 76, 40), amp=4.0, k=3, levels=2, iters=25)
    h = (1.97, 1.97, 2.5)
    say("pyramid in mm")
    ug = gpu_register(ctx, pair, cgdir.params_for_pair(pair, sigma_fluid=2.5, sigma_diff=2.5, spacing=h))
    uo, _, _ = orc.register(pair.target, pair.moving, pair.target_masks, pair.moving_masks,
                            orc.params_for(pair, sigma_fluid=float(np.float32(2.5)),
                                           sigma_diff=float(np.float32(2.5)),
                                           spacing=[float(np.float32(v)) for v in h]))
    err = np.abs(ug - uo).max()
    rms = np.sqrt(((orc.warp(pair.moving, ug) - orc.warp(pair.moving, uo)) ** 2).mean())
    say("  final max err %.3g voxel, warped rms %.3g HU" % (err, rms))
    assert err <= FINAL_TOL and rms <= WARP_RMS_TOL
    # x and y voxel sizes that differ
    h2 = (1.2, 1.6, 2.0)
    ug = gpu_register(ctx, pair, cgdir.params_for_pair(pair, sigma_fluid=2.0, sigma_diff=2.0, spacing=h2))
    uo, _, _ = orc.register(pair.target, pair.moving, pair.target_masks, pair.moving_masks,
                            orc.params_for(pair, sigma_fluid=2.0, sigma_diff=2.0,
                                           spacing=[float(np.float32(v)) for v in h2]))
    err = np.abs(ug - uo).max()
    rms = np.sqrt(((orc.warp(pair.moving, ug) - orc.warp(pair.moving, uo)) ** 2).mean())
    say("  %s mm: final max err %.3g voxel, warped rms %.3g HU" % (h2, err, rms))
    assert err <= FINAL_TOL and rms <= WARP_RMS_TOL
    for bad in ((1.0, 1.0, -2.0), (0.2, 0.2, 0.2)):   # negative; sigma 1 mm = 5 voxels -> radius 15
        with pytest.raises(cgdir.CgdirError) as e:
            gpu_register(ctx, pair, cgdir.params_for_pair(pair, spacing=bad))
        assert e.value.code == cgdir.E_INVAL, bad


def test_full_run_plain(ctx, orc):
    """Config 1 in full: 64x64x32, 1 level x 100 iterations, k = 1."""
    from paper_1301_0970_amd import cgdir
    pair = P.plain_pair()
    say("full run plain 64x64x32 x100")
    ug = gpu_register(ctx, pair, cgdir.params_for_pair(pair))
    uo, _, _ = orc.register(pair.target, pair.moving, pair.target_masks, pair.moving_masks, orc.params_for(pair))
    err = np.abs(ug - uo).max()
    wg = orc.warp(pair.moving, ug)
    wo = orc.warp(pair.moving, uo)
    rms = np.sqrt(((wg - wo) ** 2).mean())
    say("  final max err %.3g voxel, warped rms %.3g HU" % (err, rms))
    assert err <= FINAL_TOL and rms <= WARP_RMS_TOL


def test_full_run_pyramid(ctx, orc):
    """Three levels (demons on the coarse two, CG-DIR at the finest) on a ragged
    head-and-neck-like pair."""
    from paper_1301_0970_amd import cgdir
    pair = P.head_neck_pair(dims=(99, 83, 45), amp=5.0, k=4, levels=3, iters=30)
    say("full run pyramid 99x83x45 3x30")
    ug = gpu_register(ctx, pair, cgdir.params_for_pair(pair))
    uo, _, _ = orc.register(pair.target, pair.moving, pair.target_masks, pair.moving_masks, orc.params_for(pair))
    err = np.abs(ug - uo).max()
    rms = np.sqrt(((orc.warp(pair.moving, ug) - orc.warp(pair.moving, uo)) ** 2).mean())
    say("  final max err %.3g voxel, warped rms %.3g HU" % (err, rms))
    assert err <= FINAL_TOL and rms <= WARP_RMS_TOL


def test_restrict_and_prolong_through_schedule(ctx, orc):
    """levels=2 with iterations (0 finest, 1 coarse): the output is the prolonged first
    coarse step on the restricted images -- checks restriction, the coarse demons step
    and prolongation at 1e-4."""
    from paper_1301_0970_amd import cgdir
    pair = P.pelvis_pair(dims=(77, 64, 31), amp=3.0, k=3, levels=2, iters=1, bulge=0.0)
    prm = cgdir.params_for_pair(pair, iters=(0, 1))
    say("pyramid schedule (0, 1)")
    ug = gpu_register(ctx, pair, prm)
    uo, _, _ = orc.register(pair.target, pair.moving, pair.target_masks, pair.moving_masks,
                            orc.params_for(pair, iters=(0, 1)))
    assert np.abs(uo).max() > 0.05
    assert np.abs(ug - uo).max() <= STEP_TOL * 2  # prolongation doubles the coarse field


@pytest.mark.parametrize("levels,mask,it,spacing", [(2, 2, (0, 1), None), (3, 4, (0, 0, 1), None),
                                                    (3, 6, (0, 1, 1), None), (2, 3, (0, 1), (1.2, 1.2, 3.0))],
                         ids=["L2 coarse", "L3 coarsest", "L3 both coarse", "L2 coarse mm"])
def test_contour_terms_at_coarse_levels_schedule(ctx, orc, levels, mask, it, spacing):
    """Contour terms below the finest level (masks taken at the voxels the restriction
    keeps): with single iterations at coarse levels and none at the finest, the output is
    those iterations prolongated, at 1e-4 per doubling.  Ragged dims exercise the ceil(n/2)
    levels; the overlapping structures exercise the multi-structure path at a coarse level."""
    from paper_1301_0970_amd import cgdir
    pair = P.pelvis_pair(dims=(77, 66, 31), amp=3.0, k=3, levels=levels, iters=1, bulge=0.0)
    rng = np.random.default_rng(levels * 10 + mask)
    grow = lambda b: np.maximum(b, np.roll(b, 3, axis=2))             # noqa: E731
    pair.target_masks = np.stack([pair.target_masks[0], grow(pair.target_masks[0]), pair.target_masks[2]])
    pair.moving_masks = np.stack([pair.moving_masks[0], grow(pair.moving_masks[0]), pair.moving_masks[2]])
    lam = [float(v) for v in rng.uniform(1e-3, 5e-3, 3)]
    extra = {} if spacing is None else dict(spacing=spacing, sigma_fluid=1.5, sigma_diff=1.5)
    prm = cgdir.params_for_pair(pair, iters=it, contour_level_mask=mask, lambdas=lam, **extra)
    say("coarse contour schedule levels=%d mask=%d spacing=%s" % (levels, mask, spacing))
    ug = gpu_register(ctx, pair, prm)
    uo, _, _ = orc.register(pair.target, pair.moving, pair.target_masks, pair.moving_masks,
                            orc.params_for(pair, iters=it, contour_level_mask=mask, lambdas=lam, **extra))
    u0, _, _ = orc.register(pair.target, pair.moving, pair.target_masks, pair.moving_masks,
                            orc.params_for(pair, iters=it, contour_level_mask=0, lambdas=lam, **extra))
    assert np.abs(uo - u0).max() > 1e-3         # the contour terms act at that level
    err = np.abs(ug - uo).max()
    say("  max err %.3g" % err)
    assert err <= STEP_TOL * 2 ** (levels - 1)


def test_full_run_pyramid_contour_terms_at_every_level(ctx, orc):
    """Three levels with contour terms at each (the finest as in Algorithm A, the coarse two
    on masks at the kept voxels), 30 iterations per level."""
    from paper_1301_0970_amd import cgdir
    pair = P.head_neck_pair(dims=(99, 83, 45), amp=5.0, k=4, levels=3, iters=30)
    say("full run pyramid 99x83x45 3x30, contour terms at every level")
    ug = gpu_register(ctx, pair, cgdir.params_for_pair(pair, contour_level_mask=7))
    uo, _, _ = orc.register(pair.target, pair.moving, pair.target_masks, pair.moving_masks,
                            orc.params_for(pair, contour_level_mask=7))
    err = np.abs(ug - uo).max()
    rms = np.sqrt(((orc.warp(pair.moving, ug) - orc.warp(pair.moving, uo)) ** 2).mean())
    say("  final max err %.3g voxel, warped rms %.3g HU" % (err, rms))
    assert err <= FINAL_TOL and rms <= WARP_RMS_TOL


def test_full_run_pyramid_anisotropic_in_plane_with_contour_terms_at_every_level(ctx, orc):
    """Three levels in physical units with x, y and z voxel sizes that all differ (1.1 x 1.6 x
    2.2 mm, sigma 2 mm: radii 6, 4, 3 at the finest level) and contour terms at each level,
    20 iterations per level: every launch takes the kernels' general instantiation."""
    from paper_1301_0970_amd import cgdir
    pair = P.pelvis_pair(dims=(90, 70, 36), amp=4.0, k=3, levels=3, iters=20, bulge=2.0, seed=91)
    h = (1.1, 1.6, 2.2)
    say("full run pyramid 90x70x36 3x20 in %s mm, contour terms at every level" % (h,))
    ug = gpu_register(ctx, pair, cgdir.params_for_pair(pair, sigma_fluid=2.0, sigma_diff=2.0, spacing=h,
                                                       contour_level_mask=7))
    uo, _, _ = orc.register(pair.target, pair.moving, pair.target_masks, pair.moving_masks,
                            orc.params_for(pair, sigma_fluid=2.0, sigma_diff=2.0, contour_level_mask=7,
                                           spacing=[float(np.float32(v)) for v in h]))
    err = np.abs(ug - uo).max()
    rms = np.sqrt(((orc.warp(pair.moving, ug) - orc.warp(pair.moving, uo)) ** 2).mean())
    say("  final max err %.3g voxel, warped rms %.3g HU" % (err, rms))
    assert err <= FINAL_TOL and rms <= WARP_RMS_TOL


def test_identity_stays_zero(ctx):
    """P4 on the GPU: identical images and masks give exactly u = 0."""
    from paper_1301_0970_amd import cgdir
    pair = P.plain_pair(dims=(70, 50, 20), amp=2.0)
    pair.moving = pair.target.copy()
    pair.moving_masks = pair.target_masks.copy()
    say("identity")
    ug = gpu_register(ctx, pair, cgdir.params_for_pair(pair, levels=2, iters=(5, 5)))
    assert np.all(ug == 0.0)


def test_delta_history_and_stop_rule(ctx, orc):
    from paper_1301_0970_amd import cgdir
    pair = P.plain_pair(dims=(64, 48, 24), amp=2.0, iters=40)
    prm = cgdir.params_for_pair(pair)
    say("delta history")
    ug, hg, n = gpu_register(ctx, pair, prm, delta=True)
    uo, ho, no = orc.register(pair.target, pair.moving, pair.target_masks, pair.moving_masks,
                              orc.params_for(pair), want_delta=True)
    assert n == no == 40
    np.testing.assert_allclose(hg, ho, rtol=1e-4)
    # stopping: pick eps between the two largest progress values at the check points so
    # that no check sits near a tie; the GPU decision must be valid on its own history
    # and equal the oracle's
    d = sorted(ho[m - 10] - ho[m] for m in (19, 29, 39))
    eps = 0.5 * (d[1] + d[2])
    say("stop rule eps %.3g" % eps)
    prm = cgdir.params_for_pair(pair, stop_mode=1, stop_eps=eps)
    _, hs, ns = gpu_register(ctx, pair, prm, delta=True)
    first = next((m for m in range(19, 40, 10) if hs[m - 10] - hs[m] <= float(np.float32(eps))), 39)
    assert ns == first + 1 and ns < 40
    _, _, no2 = orc.register(pair.target, pair.moving, pair.target_masks, pair.moving_masks,
                             orc.params_for(pair, stop_mode=1, stop_eps=eps), want_delta=True)
    assert ns == no2


def test_auto_sign(ctx, orc):
    from paper_1301_0970_amd import cgdir
    pair = P.head_neck_pair(dims=(96, 80, 32), amp=3.0, k=3)
    # make structure 1 darker than its surroundings in the target
    t = pair.target.copy()
    t[pair.target_masks[1] == 1] -= 60.0
    pair.target = t
    u0 = P.random_smooth_field(pair.dims, 2.0, 3)
    prm = cgdir.make_params(levels=1, iters=(1,), sigma_fluid=1.5, sigma_diff=1.5, lambdas=[5e-3] * 3,
                            signs=[0, 0, 0])
    say("auto sign")
    ug = gpu_register(ctx, pair, prm, initial=u0)
    signs = [orc.auto_sign(pair.target, pair.target_masks[i]) for i in range(3)]
    assert signs[1] == -1
    uo = oracle_step(orc, pair, u0, 1.5, 1.5, [5e-3] * 3, signs)
    assert np.abs(ug - uo).max() <= STEP_TOL


def test_warp_linear_and_mask(ctx, orc):
    import torch
    from paper_1301_0970_amd import cgdir
    rng = np.random.default_rng(5)
    dims = (67, 41, 19)
    src = rng.normal(0, 300, dims[::-1]).astype(np.float32)
    u = P.random_smooth_field(dims, 4.0, 11)
    say("warp linear")
    out = ctx.warp(dev(src), dev(u)).cpu().numpy()
    ref = orc.warp(src, u)
    assert np.abs(out - ref).max() <= 1e-3
    # host buffers take the same path through a device copy
    out_h = ctx.warp(torch.from_numpy(src), torch.from_numpy(u)).numpy()
    np.testing.assert_array_equal(out_h, out)
    m = (rng.uniform(size=dims[::-1]) > 0.7).astype(np.uint8)
    say("warp mask")
    mo = ctx.warp(dev(m), dev(u), mode=cgdir.WARP_MASK).cpu().numpy()
    ref_val = orc.warp(m.astype(np.float64), u)
    decided = np.abs(ref_val - 0.5) > 1e-5
    np.testing.assert_array_equal(mo[decided], (ref_val >= 0.5)[decided].astype(np.uint8))


def test_host_inputs_match_device_inputs(ctx):
    import torch
    from paper_1301_0970_amd import cgdir
    pair = P.head_neck_pair(dims=(64, 64, 24), amp=3.0, k=2, levels=2, iters=5)
    prm = cgdir.params_for_pair(pair)
    say("host inputs")
    ud = gpu_register(ctx, pair, prm)
    uh = ctx.register(torch.from_numpy(pair.target), torch.from_numpy(pair.moving),
                      torch.from_numpy(pair.target_masks), torch.from_numpy(pair.moving_masks), prm).numpy()
    np.testing.assert_array_equal(ud, uh)


def test_invalid_arguments(ctx):
    import torch
    from paper_1301_0970_amd import cgdir
    pair = P.plain_pair(dims=(32, 32, 16), amp=1.0, iters=2)
    t, m = dev(pair.target), dev(pair.moving)
    tm, mm = dev(pair.target_masks), dev(pair.moving_masks)
    say("invalid arguments")
    with pytest.raises(cgdir.CgdirError) as e:
        ctx.register(t, m[:8], tm, mm, cgdir.params_for_pair(pair))
    assert e.value.code == cgdir.E_INVAL
    with pytest.raises(cgdir.CgdirError) as e:
        ctx.register(t, m, tm, mm[:0], cgdir.params_for_pair(pair))
    assert e.value.code == cgdir.E_INVAL
    for bad in (dict(levels=0), dict(sigma_fluid=5.0), dict(norm_range=0.0), dict(uroi_margin=(9, 1, 1))):
        with pytest.raises(cgdir.CgdirError) as e:
            ctx.register(t, m, tm, mm, cgdir.params_for_pair(pair, **bad))
        assert e.value.code == cgdir.E_INVAL, bad
    with pytest.raises(cgdir.CgdirError) as e:   # contour terms at a level that does not exist
        ctx.register(t, m, tm, mm, cgdir.params_for_pair(pair, contour_level_mask=2))
    assert e.value.code == cgdir.E_INVAL
    big = torch.zeros((256, 1024, 1024), dtype=torch.float32, device="cuda")
    one = cgdir.make_params(levels=1, iters=(1,))
    assert cgdir.footprint(1024, 1024, 256, 0, one) > (6 << 30)   # more than the context's pool
    with pytest.raises(cgdir.CgdirError) as e:
        ctx.register(big, big, None, None, one)
    assert e.value.code == cgdir.E_NOMEM


def test_inputs_still_being_computed_on_the_torch_stream(ctx):
    """The binding orders the library's stream after the caller's current stream: an input that
    torch is still writing (behind a 20 ms spin on its stream) when register is called is read
    only once written, and tensors of the wrong dtype or layout are refused."""
    import torch
    from paper_1301_0970_amd import cgdir
    pair = P.plain_pair(dims=(96, 80, 40), amp=3.0, iters=4)
    prm = cgdir.params_for_pair(pair)
    t, m, tm, mm = dev(pair.target), dev(pair.moving), dev(pair.target_masks), dev(pair.moving_masks)
    ref = ctx.register(t, m, tm, mm, prm).cpu().numpy()
    say("inputs written behind a spin on the torch stream")
    late = torch.zeros_like(m)
    torch.cuda._sleep(50_000_000)   # bounded spin, about 20 ms
    late.copy_(m)
    got = ctx.register(t, late, tm, mm, prm).cpu().numpy()
    np.testing.assert_array_equal(got, ref)
    with pytest.raises(ValueError):
        ctx.register(t, m.double(), tm, mm, prm)
    with pytest.raises(ValueError):
        ctx.register(t.transpose(1, 2), m.transpose(1, 2), None, None, prm)
    with pytest.raises(ValueError):
        ctx.register(t, m, tm, mm, prm, out=torch.empty((3, 2, 2, 2), device="cuda"))


def test_nonfinite_input_reported(ctx):
    from paper_1301_0970_amd import cgdir
    pair = P.plain_pair(dims=(40, 36, 20), amp=1.0, iters=3)
    pair.moving = pair.moving.copy()
    pair.moving[10, 18, 20] = np.nan
    say("nonfinite")
    with pytest.raises(cgdir.CgdirError) as e:
        gpu_register(ctx, pair, cgdir.params_for_pair(pair))
    assert e.value.code == cgdir.E_NONFINITE
