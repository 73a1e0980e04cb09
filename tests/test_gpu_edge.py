"""Edge cases of the method and of the volume shapes, against the FP64 oracle.

* Overlapping structures: where two or more structures meet in one stencil the step kernel
  re-warps each structure's masked image from the field (the multi-structure path).
* Degenerate volumes: single voxels, rows, columns and planes, and a 2x2x2 cube; every
  border clamp is active.
* Flat images: the gradient is zero everywhere, so no step is taken (R5).
* Empty inputs are rejected.
"""
import numpy as np
import pytest

from paper_1301_0970_amd import phantom as P

pytestmark = pytest.mark.gpu

STEP_TOL = 1e-4


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1301_0970_amd import cgdir
    assert torch.cuda.is_available()
    c = cgdir.Context(1 << 30)
    yield c
    c.close()


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def one_step(ctx, orc, T, I, tm, mm, u0, lam, sg, sigma=1.0):
    from paper_1301_0970_amd import cgdir
    prm = cgdir.make_params(levels=1, iters=(1,), sigma_fluid=sigma, sigma_diff=sigma, lambdas=lam, signs=sg)
    k = len(lam)
    ug = ctx.register(dev(T), dev(I), dev(tm) if k else None, dev(mm) if k else None, prm,
                      initial=dev(u0)).cpu().numpy()
    Ip = [orc.modified_image(I, mm[i], sg[i]) for i in range(k)]
    Tp = [orc.modified_image(T, tm[i], sg[i]) for i in range(k)]
    uo, _ = orc.step(I, T, Ip, Tp, lam, sigma, sigma, u0.astype(np.float64))
    return ug, uo


def _ball(shape, c, r):
    z, y, x = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    return (((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2) <= r * r).astype(np.uint8)


def test_overlapping_structures(ctx, orc):
    """Three structures that overlap pairwise and all together, on both images."""
    shape = (40, 48, 56)                     # z, y, x
    rng = np.random.default_rng(31)
    base = 40.0 + 30.0 * _ball(shape, (28, 24, 20), 14) + rng.normal(0, 20, shape)
    d = 1.5
    tm = np.stack([_ball(shape, (24, 24, 20), 9), _ball(shape, (32, 24, 20), 9), _ball(shape, (28, 30, 22), 8)])
    mm = np.stack([_ball(shape, (24 + d, 24, 20), 9), _ball(shape, (32 + d, 24, 21), 9),
                   _ball(shape, (28, 30 - d, 22), 8)])
    T = (base + 15.0 * tm.sum(0)).astype(np.float32)
    I = (np.roll(base, 1, axis=2) + 15.0 * mm.sum(0) + rng.normal(0, 5, shape)).astype(np.float32)
    assert (tm.sum(0) >= 2).sum() > 500 and (tm.sum(0) == 3).sum() > 50
    u0 = P.random_smooth_field((shape[2], shape[1], shape[0]), 1.5, 5)
    lam, sg = [2e-3, 1e-3, 3e-3], [1, -1, 1]
    say("overlapping structures")
    ug, uo = one_step(ctx, orc, T, I, tm, mm, u0, lam, sg)
    err = np.abs(ug - uo).max()
    say("  max |du| %.3g  max err %.3g" % (np.abs(uo - u0).max(), err))
    assert err <= STEP_TOL


@pytest.mark.parametrize("shape", [(1, 1, 1), (1, 1, 9), (1, 7, 1), (6, 1, 1), (2, 2, 2), (3, 1, 70), (5, 9, 1)],
                         ids=lambda s: "x".join(map(str, s[::-1])))
def test_degenerate_volumes(ctx, orc, shape):
    """shape is (nz, ny, nx)."""
    rng = np.random.default_rng(sum(shape))
    T = rng.normal(0, 100, shape).astype(np.float32)
    I = (T + rng.normal(0, 30, shape)).astype(np.float32)
    tm = (rng.uniform(size=(1,) + shape) > 0.5).astype(np.uint8)
    mm = (rng.uniform(size=(1,) + shape) > 0.5).astype(np.uint8)
    u0 = rng.normal(0, 0.7, (3,) + shape).astype(np.float32)
    say("degenerate volume %s" % (shape[::-1],))
    ug, uo = one_step(ctx, orc, T, I, tm, mm, u0, [2e-3], [1])
    assert np.abs(ug - uo).max() <= STEP_TOL


def test_flat_images_take_no_step(ctx):
    from paper_1301_0970_amd import cgdir
    shape = (12, 20, 33)
    T = np.full(shape, 40.0, np.float32)
    I = np.full(shape, -25.0, np.float32)
    say("flat images")
    u = ctx.register(dev(T), dev(I), None, None, cgdir.make_params(levels=2, iters=(5, 5))).cpu().numpy()
    assert np.all(u == 0.0)


def test_empty_inputs_are_rejected(ctx):
    import torch
    from paper_1301_0970_amd import cgdir
    e0 = torch.zeros((0, 8, 8), device="cuda")
    with pytest.raises(cgdir.CgdirError) as e:
        ctx.register(e0, e0, None, None, cgdir.make_params(iters=(1,)), out=torch.zeros((3, 1, 8, 8), device="cuda"))
    assert e.value.code == cgdir.E_INVAL
