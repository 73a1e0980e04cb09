"""cgdir_register_static (the registration that allocates nothing: its buffers live in the
library's static device scratch) against cgdir_register: two calls in a row, the second on a
smaller pair, each bitwise equal to the ordinary entry point's field; a registration larger than
the scratch is refused."""
import numpy as np
import pytest

from paper_1301_0970_amd import phantom as P

pytestmark = pytest.mark.gpu


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def test_static_entry_point_equals_register_twice_then_refuses_oversize():
    import torch
    from paper_1301_0970_amd import cgdir
    big = P.head_neck_pair(dims=(112, 96, 48), amp=4.0, k=3, levels=2, iters=12, seed=91)
    small = P.pelvis_pair(dims=(64, 56, 24), amp=3.0, k=2, levels=2, iters=9, bulge=0.0, seed=92)
    with cgdir.Context(1 << 30) as ctx:
        for pair in (big, small):
            prm = cgdir.params_for_pair(pair)
            need = cgdir.footprint(*pair.dims, pair.k, prm)
            assert need <= cgdir.STATIC_SCRATCH_BYTES
            it = (dev(pair.target), dev(pair.moving), dev(pair.target_masks), dev(pair.moving_masks))
            ref = ctx.register(*it, prm=prm).cpu().numpy()
            out = torch.full((3,) + tuple(pair.target.shape), float("nan"), device="cuda")
            got = ctx.register_static(*it, prm=prm, out=out).cpu().numpy()
            np.testing.assert_array_equal(got, ref)
        # larger than the scratch: refused before any device work
        huge = torch.zeros((128, 256, 256), device="cuda")
        hm = torch.zeros((8, 128, 256, 256), dtype=torch.uint8, device="cuda")
        prm = cgdir.make_params(levels=3, iters=(5, 5, 5), lambdas=[1e-3] * 8, signs=[1] * 8)
        assert cgdir.footprint(256, 256, 128, 8, prm) > cgdir.STATIC_SCRATCH_BYTES
        with pytest.raises(cgdir.CgdirError) as e:
            ctx.register_static(huge, huge, hm, hm, prm)
        assert e.value.code == cgdir.E_SCRATCH
        # host buffers and the stopping rule are not for this entry point
        with pytest.raises(cgdir.CgdirError) as e:
            ctx.register_static(torch.from_numpy(small.target), torch.from_numpy(small.moving), None, None,
                                cgdir.make_params(levels=1, iters=(2,)),
                                out=torch.empty((3,) + tuple(small.target.shape), device="cuda"))
        assert e.value.code == cgdir.E_INVAL
        with pytest.raises(cgdir.CgdirError) as e:
            it = (dev(small.target), dev(small.moving), None, None)
            ctx.register_static(*it, prm=cgdir.make_params(levels=1, iters=(20,), stop_mode=1))
        assert e.value.code == cgdir.E_UNIMPL
