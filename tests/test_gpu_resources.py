"""Every entry point returns what it takes from the context's pool: with a pool of one
registration's footprint plus the same again, thirty rounds of every call that uses the pool
(blocking registration from device and host buffers, warp of host buffers, evaluation,
batched registration, served registration from device and from host buffers) all succeed and give the same field each round."""
import numpy as np
import pytest

from paper_1301_0970_amd import phantom as P

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


def test_pool_is_returned_by_every_call():
    import torch
    from paper_1301_0970_amd import cgdir
    pair = P.pelvis_pair(dims=(48, 40, 24), amp=2.0, k=3, levels=2, iters=3, bulge=0.0)
    prm = cgdir.params_for_pair(pair, stop_mode=1)
    need = cgdir.footprint(*pair.dims, pair.k, prm)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()   # noqa: E731
    host = lambda a: torch.from_numpy(np.ascontiguousarray(a))          # noqa: E731
    t, m, tm, mm = dev(pair.target), dev(pair.moving), dev(pair.target_masks), dev(pair.moving_masks)
    with cgdir.Context(2 * need, max_slots=2) as ctx:
        ref = ctx.register(t, m, tm, mm, prm).cpu().numpy()
        say("30 rounds in a pool of %d bytes" % (2 * need))
        for rnd in range(30):
            u = ctx.register(t, m, tm, mm, prm)
            np.testing.assert_array_equal(u.cpu().numpy(), ref)
            uh = ctx.register(host(pair.target), host(pair.moving), host(pair.target_masks),
                              host(pair.moving_masks), prm, out=torch.empty((3,) + pair.target.shape))
            np.testing.assert_array_equal(uh.numpy(), ref)
            w = ctx.warp(host(pair.moving), host(ref))
            assert torch.isfinite(w).all()
            wm = ctx.warp(host(pair.moving_masks[0]), host(ref), mode=cgdir.WARP_MASK)
            assert int(wm.sum()) > 0
            ev = ctx.evaluate(t, m, tm, mm, u)
            assert len(ev["structures"]) == pair.k
            outs = [torch.empty_like(u)]
            rc, st = ctx.register_batch([(t, m, tm, mm)], [prm], outs)
            assert rc == cgdir.OK and st == [cgdir.OK]
            np.testing.assert_array_equal(outs[0].cpu().numpy(), ref)
            o = torch.empty_like(u)
            tk = ctx.submit(t, m, tm, mm, prm, o)
            assert ctx.wait(tk, int(60e9)) == cgdir.OK, rnd
            np.testing.assert_array_equal(o.cpu().numpy(), ref)
            oh = torch.empty((3,) + pair.target.shape)   # served from and to host memory
            tk = ctx.submit(host(pair.target), host(pair.moving), host(pair.target_masks),
                            host(pair.moving_masks), prm, oh)
            assert ctx.wait(tk, int(60e9)) == cgdir.OK, rnd
            np.testing.assert_array_equal(oh.numpy(), ref)
