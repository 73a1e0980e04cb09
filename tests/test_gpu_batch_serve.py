"""Batched and served registration: every pair's result equals its result alone."""
import time

import numpy as np
import pytest

from paper_1301_0970_amd import phantom as P

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _pairs():
    return [
        P.head_neck_pair(dims=(96, 64, 40), amp=4.0, k=3, levels=2, iters=6, seed=11),
        P.pelvis_pair(dims=(128, 80, 24), amp=3.0, k=8, levels=3, iters=4, bulge=0.0, seed=12),
        P.plain_pair(dims=(64, 64, 32), amp=3.0, iters=9, seed=13),
        P.head_neck_pair(dims=(72, 100, 36), amp=4.0, k=1, levels=2, iters=(7), seed=14),
    ]


def _items(pairs):
    return [(dev(p.target), dev(p.moving), dev(p.target_masks), dev(p.moving_masks)) for p in pairs]


def test_batch_equals_alone():
    import torch
    from paper_1301_0970_amd import cgdir
    pairs = _pairs()
    items = _items(pairs)
    prms = [cgdir.params_for_pair(p) for p in pairs]
    with cgdir.Context(4 << 30) as ctx:
        say("alone")
        alone = [ctx.register(*it, prm=pr).cpu().numpy() for it, pr in zip(items, prms)]
        outs = [torch.empty((3,) + tuple(p.target.shape), device="cuda") for p in pairs]
        say("batch")
        rc, st = ctx.register_batch(items, prms, outs)
        assert rc == cgdir.OK and st == [0] * len(pairs)
        for a, o in zip(alone, outs):
            np.testing.assert_array_equal(a, o.cpu().numpy())


def test_batch_rejects_when_pool_too_small():
    import torch
    from paper_1301_0970_amd import cgdir
    pairs = _pairs()
    items = _items(pairs)
    prms = [cgdir.params_for_pair(p) for p in pairs]
    need = sum(cgdir.footprint(*p.dims, p.k, pr) for p, pr in zip(pairs, prms))
    with cgdir.Context(need // 2) as ctx:
        outs = [torch.empty((3,) + tuple(p.target.shape), device="cuda") for p in pairs]
        say("batch nomem")
        rc, st = ctx.register_batch(items, prms, outs)
        assert rc == cgdir.E_NOMEM


def test_served_equals_alone_and_reports_latency():
    import torch
    from paper_1301_0970_amd import cgdir
    pairs = _pairs() * 2
    items = _items(pairs)
    prms = [cgdir.params_for_pair(p) for p in pairs]
    with cgdir.Context(4 << 30, max_slots=3) as ctx:
        say("serve alone")
        alone = [ctx.register(*it, prm=pr).cpu().numpy() for it, pr in zip(items, prms)]
        outs = [torch.empty((3,) + tuple(p.target.shape), device="cuda") for p in pairs]
        say("serve submit")
        tickets = []
        for it, pr, o in zip(items, prms, outs):
            tickets.append(ctx.submit(*it, pr, o))
            time.sleep(0.002)
        for t in tickets:
            assert ctx.wait(t, int(60e9)) == cgdir.OK
        for t, a, o in zip(tickets, alone, outs):
            st = ctx.poll(t)
            assert st.state == cgdir.DONE
            assert st.t_submit_ns <= st.t_admit_ns <= st.t_done_ns
            np.testing.assert_array_equal(a, o.cpu().numpy())
        with pytest.raises(cgdir.CgdirError):
            ctx.poll(987654)


def test_serving_isolates_a_failing_request():
    import torch
    from paper_1301_0970_amd import cgdir
    good = P.plain_pair(dims=(48, 48, 24), amp=2.0, iters=6, seed=21)
    bad = P.plain_pair(dims=(48, 48, 24), amp=2.0, iters=6, seed=22)
    bad.moving = bad.moving.copy()
    bad.moving[5, 5, 5] = np.inf
    with cgdir.Context(1 << 30, max_slots=2) as ctx:
        say("serve failure isolation")
        ref = ctx.register(*_items([good])[0], prm=cgdir.params_for_pair(good)).cpu().numpy()
        og = torch.empty((3, 24, 48, 48), device="cuda")
        ob = torch.empty((3, 24, 48, 48), device="cuda")
        tb = ctx.submit(*_items([bad])[0], cgdir.params_for_pair(bad), ob)
        tg = ctx.submit(*_items([good])[0], cgdir.params_for_pair(good), og)
        assert ctx.wait(tb, int(30e9)) == cgdir.E_NONFINITE
        assert ctx.wait(tg, int(30e9)) == cgdir.OK
        assert ctx.poll(tb).state == cgdir.FAILED
        np.testing.assert_array_equal(og.cpu().numpy(), ref)


def test_cancel_and_oversize():
    import torch
    from paper_1301_0970_amd import cgdir
    p = P.plain_pair(dims=(64, 64, 32), amp=2.0, iters=50, seed=31)
    with cgdir.Context(256 << 20, max_slots=1) as ctx:
        it = _items([p])[0]
        outs = [torch.empty((3, 32, 64, 64), device="cuda") for _ in range(3)]
        say("cancel")
        t1 = ctx.submit(*it, cgdir.params_for_pair(p), outs[0])
        t2 = ctx.submit(*it, cgdir.params_for_pair(p), outs[1])
        t3 = ctx.submit(*it, cgdir.params_for_pair(p), outs[2])
        assert ctx.cancel(t3) == cgdir.OK
        assert ctx.wait(t3) == cgdir.E_CANCELLED
        assert ctx.poll(t3).state == cgdir.CANCELLED
        assert ctx.wait(t1, int(30e9)) == cgdir.OK
        assert ctx.wait(t2, int(30e9)) == cgdir.OK
        assert ctx.cancel(t1) == cgdir.E_BUSY
        big = torch.zeros((128, 512, 512), device="cuda")
        with pytest.raises(cgdir.CgdirError) as e:
            ctx.submit(big, big, None, None, cgdir.make_params(), torch.empty((3, 128, 512, 512), device="cuda"))
        assert e.value.code == cgdir.E_NOMEM


def test_batch_of_many_small_pairs_spans_several_launches():
    """More pairs than one launch's descriptor table holds (16 for the step, 20 for the
    smoothing): chunked launches, results still equal to each pair alone."""
    import torch
    from paper_1301_0970_amd import cgdir
    pairs = []
    for i in range(26):
        dims = (40 + 8 * (i % 5), 36 + 4 * (i % 3), 16 + 2 * (i % 4))
        if i % 3 == 0:
            pairs.append(P.plain_pair(dims=dims, amp=1.5, iters=3, seed=100 + i))
        else:
            pairs.append(P.head_neck_pair(dims=dims, amp=1.5, k=1 + i % 4, levels=2, iters=2,
                                          sigma=1.5 if i % 2 else 1.0, seed=100 + i))
    items = _items(pairs)
    prms = [cgdir.params_for_pair(p) for p in pairs]
    with cgdir.Context(2 << 30) as ctx:
        say("alone x26")
        alone = [ctx.register(*it, prm=pr).cpu().numpy() for it, pr in zip(items, prms)]
        outs = [torch.empty((3,) + tuple(p.target.shape), device="cuda") for p in pairs]
        say("batch x26")
        rc, st = ctx.register_batch(items, prms, outs)
        assert rc == cgdir.OK and st == [0] * len(pairs)
        for a, o in zip(alone, outs):
            np.testing.assert_array_equal(a, o.cpu().numpy())
