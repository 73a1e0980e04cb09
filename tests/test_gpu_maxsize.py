"""The largest volume the library accepts: 2^30 voxels (4096 x 1024 x 256, x at its 4096-voxel
limit), where the 32-bit byte offsets of the kernels reach 2^32 - 4.  Seeded inputs are drawn on
the device (smooth random CT-like images, two structures, one at the far x border, a smooth
random field); one teacher-forced iteration runs in the launch configuration of any other
registration, and the FP64 oracle recomputes it on 81^3 crops around sampled centres, including
the corners of the volume (the crop-edge argument of the full-size pelvis test applies: the
compared voxels lie 34 voxels inside the crop).  About 75 GB of device memory."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

STEP_TOL = 1e-4
CROP, INNER = 40, 6
NX, NY, NZ = 4096, 1024, 256


def say(msg):
    print(msg, flush=True)


def _inputs():
    import torch
    import torch.nn.functional as F
    g = torch.Generator(device="cuda")
    g.manual_seed(13010970)

    def smooth(coarse, scale):
        c = torch.randn(coarse, device="cuda", generator=g)
        return F.interpolate(c[None, None], size=(NZ, NY, NX), mode="trilinear", align_corners=True)[0, 0] * scale

    T = smooth((6, 10, 24), 300.0)
    T += 40.0
    T.add_(torch.randn((NZ, NY, NX), device="cuda", generator=g), alpha=20.0)
    I = T.clone()
    I.add_(torch.randn((NZ, NY, NX), device="cuda", generator=g), alpha=10.0)
    z = torch.arange(NZ, device="cuda", dtype=torch.float32)[:, None, None]
    y = torch.arange(NY, device="cuda", dtype=torch.float32)[None, :, None]
    x = torch.arange(NX, device="cuda", dtype=torch.float32)[None, None, :]

    def ball(cx, cy, cz, ax, ay, az):
        return (((x - cx) / ax) ** 2 + ((y - cy) / ay) ** 2 + ((z - cz) / az) ** 2 <= 1.0).to(torch.uint8)
    tm = torch.stack([ball(2048, 512, 128, 60, 40, 20), ball(4090, 700, 200, 30, 25, 15)])
    mm = torch.stack([ball(2050.5, 511, 128, 60, 40, 20), ball(4088, 701.5, 199, 30, 25, 15)])
    T.add_(tm.sum(0, dtype=torch.float32), alpha=25.0)
    I.add_(mm.sum(0, dtype=torch.float32), alpha=25.0)
    u0 = torch.stack([smooth((4, 8, 16), 2.0) for _ in range(3)])
    return T, I, tm, mm, u0


def test_one_iteration_at_the_maximum_volume(orc):
    import torch
    from paper_1301_0970_amd import cgdir
    assert NX * NY * NZ == 1 << 30
    lam, sg = [2e-3, 3e-3], [1, 1]
    prm = cgdir.make_params(levels=1, iters=(1,), sigma_fluid=1.0, sigma_diff=1.0, lambdas=lam, signs=sg)
    need = cgdir.footprint(NX, NY, NZ, 2, prm)
    free, _ = torch.cuda.mem_get_info()
    if free < need + (40 << 30):
        pytest.skip("needs %.0f GB of free device memory" % ((need + (40 << 30)) / 1e9))
    say("max size: drawing 2^30-voxel inputs on the device")
    T, I, tm, mm, u0 = _inputs()
    say("max size: one iteration, pool %.1f GB" % (need / 1e9))
    # (the inputs are still being drawn on torch's stream: the binding orders the library's
    # work after it)
    with cgdir.Context(need + (256 << 20)) as ctx:
        u = ctx.register(T, I, tm, mm, prm, initial=u0)
        torch.cuda.synchronize()
    centres = [(NX // 2, NY // 2, NZ // 2), (2048 + 60, 512, 128), (4090, 700, 200), (0, 0, 0),
               (NX - 1, NY - 1, NZ - 1), (NX - 1, 0, NZ // 3)]
    for c in centres:
        lo = [max(0, c[a] - CROP) for a in range(3)]
        hi = [min(n, c[a] + CROP + 1) for a, n in enumerate((NX, NY, NZ))]
        sl = (slice(lo[2], hi[2]), slice(lo[1], hi[1]), slice(lo[0], hi[0]))
        say("  oracle block at %s" % (c,))
        Tc, Ic = T[sl].cpu().numpy(), I[sl].cpu().numpy()
        tmc, mmc = tm[(slice(None),) + sl].cpu().numpy(), mm[(slice(None),) + sl].cpu().numpy()
        uc = u0[(slice(None),) + sl].cpu().numpy().astype(np.float64)
        Ip = [orc.modified_image(Ic, mmc[i], sg[i]) for i in range(2)]
        Tp = [orc.modified_image(Tc, tmc[i], sg[i]) for i in range(2)]
        uo, _ = orc.step(Ic, Tc, Ip, Tp, lam, 1.0, 1.0, uc)
        inner = tuple(slice(max(0, c[a] - INNER) - lo[a], min(n, c[a] + INNER + 1) - lo[a])
                      for a, n in reversed(list(enumerate((NX, NY, NZ)))))
        gsl = tuple(slice(s.start + lo[a], s.stop + lo[a]) for s, a in zip(inner, (2, 1, 0)))
        ug = u[(slice(None),) + gsl].cpu().numpy()
        err = np.abs(ug - uo[(slice(None),) + inner]).max()
        moved = np.abs(uo[(slice(None),) + inner] - uc[(slice(None),) + inner]).max()
        say("    max err %.3g (step up to %.3g)" % (err, moved))
        assert err <= STEP_TOL, c
    del T, I, tm, mm, u0, u
    torch.cuda.empty_cache()   # the later tests need none of this memory
