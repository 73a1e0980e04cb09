"""Batched and served registration: every pair's result equals its result alone, and a mixed
batch of uneven pairs, batched and served, agrees with the FP64 oracle's Algorithm A."""
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


def _pairs(scale=1):
    return [
        P.head_neck_pair(dims=(96, 64, 40), amp=4.0, k=3, levels=2, iters=6 * scale, seed=11),
        P.pelvis_pair(dims=(128, 80, 24), amp=3.0, k=8, levels=3, iters=4 * scale, bulge=0.0, seed=12),
        P.plain_pair(dims=(64, 64, 32), amp=3.0, iters=9 * scale, seed=13),
        P.head_neck_pair(dims=(72, 100, 36), amp=4.0, k=1, levels=2, iters=7 * scale, seed=14),
    ]


def _items(pairs):
    return [(dev(p.target), dev(p.moving), dev(p.target_masks), dev(p.moving_masks)) for p in pairs]


@pytest.mark.parametrize("lanes", ["1", "2"])
def test_batch_equals_alone(lanes, monkeypatch):
    """Batched fields equal each pair alone, in one lockstep group and with the radius groups
    on two streams (CGDIR_BATCH_LANES, read when the context is created)."""
    import torch
    from paper_1301_0970_amd import cgdir
    monkeypatch.setenv("CGDIR_BATCH_LANES", lanes)
    pairs = _pairs()
    items = _items(pairs)
    prms = [cgdir.params_for_pair(p) for p in pairs]
    with cgdir.Context(4 << 30) as ctx:
        say("alone")
        alone = [ctx.register(*it, prm=pr).cpu().numpy() for it, pr in zip(items, prms)]
        outs = [torch.empty((3,) + tuple(p.target.shape), device="cuda") for p in pairs]
        say("batch, %s lane(s)" % lanes)
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


@pytest.mark.parametrize("policy,large", [("2", None), ("2", "200000"), ("1", "200000"), ("0", "200000")],
                         ids=["default", "lanes one at a time", "lanes", "lockstep"])
def test_served_equals_alone_and_reports_latency(policy, large, monkeypatch):
    """Served fields equal each pair alone under every serving policy; with the large-request
    threshold below three of the four pair sizes (CGDIR_SERVE_LARGE, read when the context is
    created) requests change lanes as others join and leave."""
    import torch
    from paper_1301_0970_amd import cgdir
    monkeypatch.setenv("CGDIR_SERVE_POLICY", policy)
    if large is not None:
        monkeypatch.setenv("CGDIR_SERVE_LARGE", large)
    pairs = _pairs(scale=10) * 2
    items = _items(pairs)
    prms = [cgdir.params_for_pair(p) for p in pairs]
    with cgdir.Context(4 << 30, max_slots=3) as ctx:
        say("serve alone")
        alone = [ctx.register(*it, prm=pr).cpu().numpy() for it, pr in zip(items, prms)]
        outs = [torch.empty((3,) + tuple(p.target.shape), device="cuda") for p in pairs]
        say("serve submit")
        tickets = [ctx.submit(*it, pr, o) for it, pr, o in zip(items, prms, outs)]
        for t in tickets:
            assert ctx.wait(t, int(60e9)) == cgdir.OK
        sts = []
        for t, a, o in zip(tickets, alone, outs):
            st = ctx.poll(t)
            assert st.state == cgdir.DONE
            assert st.t_submit_ns <= st.t_admit_ns <= st.t_done_ns
            np.testing.assert_array_equal(a, o.cpu().numpy())
            sts.append(st)
        # the requests shared the device: one was admitted before an earlier one finished
        assert any(b.t_admit_ns < a.t_done_ns for i, a in enumerate(sts) for b in sts[i + 1:])
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
    """More pairs than one launch's descriptor table holds (12 for the step, 16 for the
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


def test_served_records_are_bounded():
    """A context keeps the final status of its KEEP_FINISHED latest finished requests: after
    more tiny served registrations than that, the oldest tickets are unknown, the latest are
    done, and their fields equal the same registration alone."""
    import torch
    from paper_1301_0970_amd import cgdir
    pair = P.plain_pair(dims=(8, 8, 4), amp=0.5, iters=1, seed=5)
    items = _items([pair])[0]
    prm = cgdir.params_for_pair(pair)
    n = cgdir.KEEP_FINISHED + 40
    with cgdir.Context(1 << 30, max_slots=16) as ctx:
        ref = ctx.register(*items, prm=prm).cpu().numpy()
        outs = [torch.empty((3,) + tuple(pair.target.shape), device="cuda") for _ in range(n)]
        say("served x%d tiny" % n)
        tickets = [ctx.submit(*items, prm, o) for o in outs]
        for t in tickets[-64:]:
            assert ctx.wait(t) == cgdir.OK
        for t in tickets:            # every request has finished by now
            rc, st = cgdir.poll(ctx.handle, t)
            assert rc in (cgdir.OK, cgdir.E_NOTFOUND)
            if rc == cgdir.OK:
                assert st.state == cgdir.DONE
        known = [cgdir.poll(ctx.handle, t)[0] == cgdir.OK for t in tickets]
        assert sum(known) == cgdir.KEEP_FINISHED and not any(known[:40]) and all(known[-64:])
        assert cgdir.wait(ctx.handle, tickets[0]) == cgdir.E_NOTFOUND
        assert cgdir.cancel(ctx.handle, tickets[0]) == cgdir.E_NOTFOUND
        for o in outs[:3] + outs[-3:]:
            np.testing.assert_array_equal(o.cpu().numpy(), ref)


def test_early_stop_on_the_device_alone_batched_and_served():
    """The stopping rule runs on the device: each pair stops at its own iteration whether it
    runs alone, batched or served, and the launches after its stop leave its field as it was
    at the stop."""
    import ctypes

    import torch
    from paper_1301_0970_amd import cgdir
    pairs = [P.plain_pair(dims=(64, 48, 24), amp=a, iters=60, seed=s) for a, s in ((2.0, 21), (3.0, 22), (1.5, 23))]
    items = _items(pairs)
    with cgdir.Context(2 << 30) as ctx:
        say("stop: histories")
        hist = [ctx.register(*it, prm=cgdir.params_for_pair(p), delta=True)[1] for it, p in zip(items, pairs)]
        prog = sorted(h[m - 10] - h[m] for h in hist for m in range(19, 60, 10))
        mid = len(prog) // 2
        eps = 0.5 * (prog[mid - 1] + prog[mid])   # between two progress values, away from all
        prms = [cgdir.params_for_pair(p, stop_mode=1, stop_eps=eps) for p in pairs]
        say("stop: alone (eps %.3g)" % eps)
        alone = [ctx.register(*it, prm=pr, delta=True) for it, pr in zip(items, prms)]
        ns = [a[2] for a in alone]
        assert any(n < 60 for n in ns), ns
        for (u, h, n), hfull in zip(alone, hist):
            np.testing.assert_array_equal(h, hfull[:n])
            first = next((m for m in range(19, 60, 10) if h[m - 10] - h[m] <= float(np.float32(eps))), 59) \
                if n >= 20 else n - 1
            assert n == first + 1
        say("stop: fixed-count reruns")
        for it, p, (u, _, n) in zip(items, pairs, alone):
            u_n = ctx.register(*it, prm=cgdir.params_for_pair(p, iters=(n,)))
            np.testing.assert_array_equal(u.cpu().numpy(), u_n.cpu().numpy())
        say("stop: batched")
        done = [ctypes.c_int(0) for _ in pairs]
        for pr, d in zip(prms, done):
            pr.iters_done = ctypes.pointer(d)
        outs = [torch.empty((3,) + tuple(p.target.shape), device="cuda") for p in pairs]
        rc, st = ctx.register_batch(items, prms, outs)
        assert rc == cgdir.OK and st == [0] * len(pairs)
        assert [d.value for d in done] == ns
        for (u, _, _), o in zip(alone, outs):
            np.testing.assert_array_equal(u.cpu().numpy(), o.cpu().numpy())
        say("stop: served")
        for d in done:
            d.value = 0
        outs = [torch.empty_like(o) for o in outs]
        tickets = [ctx.submit(*it, pr, o) for it, pr, o in zip(items, prms, outs)]
        for t in tickets:
            assert ctx.wait(t, int(60e9)) == cgdir.OK
        assert [d.value for d in done] == ns
        for (u, _, _), o in zip(alone, outs):
            np.testing.assert_array_equal(u.cpu().numpy(), o.cpu().numpy())


def test_concurrent_submitters_and_a_blocking_registration():
    """Four threads submit and poll at once while the main thread runs blocking registrations
    on the same context: every result equals the pair's result alone, and poll answers while a
    blocking registration holds the launch lock."""
    import threading

    import torch
    from paper_1301_0970_amd import cgdir
    pairs = _pairs()
    items = _items(pairs)
    prms = [cgdir.params_for_pair(p) for p in pairs]
    with cgdir.Context(4 << 30, max_slots=3) as ctx:
        say("concurrent: alone")
        alone = [ctx.register(*it, prm=pr).cpu().numpy() for it, pr in zip(items, prms)]
        results, errors = {}, []

        def worker(w):
            try:
                outs, tickets = [], []
                for j in range(len(pairs)):
                    q = (j + w) % len(pairs)
                    o = torch.empty((3,) + tuple(pairs[q].target.shape), device="cuda")
                    tickets.append((q, ctx.submit(*items[q], prms[q], o), o))
                for q, t, o in tickets:
                    while ctx.poll(t).state not in (cgdir.DONE, cgdir.FAILED, cgdir.CANCELLED):
                        time.sleep(0.001)
                    assert ctx.wait(t) == cgdir.OK
                    results[(w, q)] = o.cpu().numpy()
            except Exception as e:  # noqa: BLE001 - reported below
                errors.append(repr(e))

        say("concurrent: 4 submitters + blocking registrations")
        threads = [threading.Thread(target=worker, args=(w,)) for w in range(4)]
        for th in threads:
            th.start()
        blocking = [ctx.register(*items[q], prm=prms[q]).cpu().numpy() for q in (2, 0)]
        for th in threads:
            th.join(120)
        assert not errors, errors
        assert len(results) == 4 * len(pairs)
        for (w, q), o in results.items():
            np.testing.assert_array_equal(o, alone[q])
        np.testing.assert_array_equal(blocking[0], alone[2])
        np.testing.assert_array_equal(blocking[1], alone[0])


def test_mixed_parameters_batched_and_served_equal_alone():
    """Pairs whose parameters differ in every way a launch groups by or carries per pair
    (physical spacing with sigma in mm, contour terms at coarse levels, automatic signs, the
    device-side stopping rule, no structures, ragged sizes) give bitwise the same field alone,
    in one batch and served together.  (Alone, the launches of a level without contour terms
    take the step kernel's instantiation without them; batched with pairs that have them, the
    general one: both give the same field.)"""
    import torch
    from paper_1301_0970_amd import cgdir
    pairs = [P.head_neck_pair(dims=(70, 58, 30), amp=3.0, k=3, levels=2, iters=8, seed=61),
             P.pelvis_pair(dims=(90, 66, 26), amp=3.0, k=4, levels=3, iters=5, bulge=0.0, seed=62),
             P.plain_pair(dims=(61, 47, 23), amp=2.0, iters=25, seed=63),
             P.head_neck_pair(dims=(50, 70, 34), amp=3.0, k=2, levels=2, iters=6, seed=64),
             P.plain_pair(dims=(40, 36, 20), amp=2.0, iters=7, seed=65)]
    prms = [cgdir.params_for_pair(pairs[0], spacing=(1.97, 1.97, 2.5), sigma_fluid=2.0, sigma_diff=2.0),
            cgdir.params_for_pair(pairs[1], contour_level_mask=7, signs=[0, 1, 0, -1]),
            cgdir.params_for_pair(pairs[2], stop_mode=1, stop_eps=1e-3),
            cgdir.params_for_pair(pairs[3], spacing=(1.2, 1.2, 3.0), contour_level_mask=3),
            cgdir.params_for_pair(pairs[4], lambdas=[0.0] * pairs[4].k)]
    items = _items(pairs)
    items[4] = items[4][:2] + (None, None)   # plain demons: no structures
    with cgdir.Context(2 << 30, max_slots=8) as ctx:
        say("mixed: alone")
        alone = [ctx.register(*it, prm=pr).cpu().numpy() for it, pr in zip(items, prms)]
        say("mixed: batch")
        outs = [torch.empty((3,) + tuple(p.target.shape), device="cuda") for p in pairs]
        rc, st = ctx.register_batch(items, prms, outs)
        assert rc == cgdir.OK and st == [cgdir.OK] * len(pairs)
        for i, (a, o) in enumerate(zip(alone, outs)):
            np.testing.assert_array_equal(a, o.cpu().numpy(), err_msg="batched pair %d" % i)
        say("mixed: served")
        outs = [torch.empty((3,) + tuple(p.target.shape), device="cuda") for p in pairs]
        tickets = [ctx.submit(*it, pr, o) for it, pr, o in zip(items, prms, outs)]
        for t in tickets:
            assert ctx.wait(t, int(60e9)) == cgdir.OK
        for i, (a, o) in enumerate(zip(alone, outs)):
            np.testing.assert_array_equal(a, o.cpu().numpy(), err_msg="served pair %d" % i)


def test_square_and_anisotropic_in_plane_voxels_share_a_launch():
    """A pair with square in-plane voxels batched with one whose x and y voxel sizes differ (the
    same Gaussian radii, so their tiles share every launch, which then takes the kernels'
    general instantiation): each field equals the pair's alone bitwise, also served."""
    import torch
    from paper_1301_0970_amd import cgdir
    pairs = [P.head_neck_pair(dims=(70, 58, 30), amp=3.0, k=3, levels=2, iters=6, seed=71),
             P.pelvis_pair(dims=(76, 64, 28), amp=3.0, k=4, levels=2, iters=6, bulge=0.0, seed=72)]
    # sigma 2 mm: radii 5, 5, 3 (x, y, z) for the first, 5, 4, 3 for the second
    prms = [cgdir.params_for_pair(pairs[0], spacing=(1.2, 1.2, 2.0), sigma_fluid=2.0, sigma_diff=2.0),
            cgdir.params_for_pair(pairs[1], spacing=(1.25, 1.5, 2.0), sigma_fluid=2.0, sigma_diff=2.0)]
    items = _items(pairs)
    with cgdir.Context(2 << 30, max_slots=4) as ctx:
        say("square and anisotropic: alone")
        alone = [ctx.register(*it, prm=pr).cpu().numpy() for it, pr in zip(items, prms)]
        outs = [torch.empty((3,) + tuple(p.target.shape), device="cuda") for p in pairs]
        say("square and anisotropic: batch")
        rc, st = ctx.register_batch(items, prms, outs)
        assert rc == cgdir.OK and st == [cgdir.OK] * len(pairs)
        for i, (a, o) in enumerate(zip(alone, outs)):
            np.testing.assert_array_equal(a, o.cpu().numpy(), err_msg="batched pair %d" % i)
        say("square and anisotropic: served")
        outs = [torch.empty((3,) + tuple(p.target.shape), device="cuda") for p in pairs]
        tickets = [ctx.submit(*it, pr, o) for it, pr, o in zip(items, prms, outs)]
        for t in tickets:
            assert ctx.wait(t, int(60e9)) == cgdir.OK
        for i, (a, o) in enumerate(zip(alone, outs)):
            np.testing.assert_array_equal(a, o.cpu().numpy(), err_msg="served pair %d" % i)


def test_tuning_export_and_import():
    """A context's settled tile-shape groups export as text; a fresh context that imports them
    launches with those shapes without timing candidates (every group forced to one shape is
    reported back unchanged after a registration) and gives bitwise the same field."""
    from paper_1301_0970_amd import cgdir
    pair = P.head_neck_pair(dims=(80, 64, 36), amp=3.0, k=2, levels=2, iters=24, seed=71)
    it = _items([pair])[0]
    prm = cgdir.params_for_pair(pair)
    with cgdir.Context(1 << 30) as c1:
        u1 = c1.register(*it, prm=prm).cpu().numpy()
        text = c1.tuning_export()
    lines = [l for l in text.splitlines() if l]
    say("exported %d groups" % len(lines))
    assert any(l.startswith("U") for l in lines) and any(l.startswith("S") for l in lines)
    forced = "\n".join("%s 4 8" % l.split()[0] for l in lines) + "\n"
    with cgdir.Context(1 << 30) as c2:
        c2.tuning_import(forced)
        u2 = c2.register(*it, prm=prm).cpu().numpy()
        back = set(l for l in c2.tuning_export().splitlines() if l)
    assert set(forced.splitlines()) <= back
    np.testing.assert_array_equal(u1, u2)
    with cgdir.Context(1 << 30) as c3:
        c3.tuning_import("\n" + text + "\n\n")
        u3 = c3.register(*it, prm=prm).cpu().numpy()
        assert set(lines) <= set(l for l in c3.tuning_export().splitlines() if l)
        np.testing.assert_array_equal(u1, u3)
        for bad in ("U3:8x8x8/9 5 5\n", "X3:8x8x8/9 8 32\n", "U3:8x8x8/9 8\n", "U3:8x8x8/9 8 32 1\n"):
            with pytest.raises(cgdir.CgdirError) as e:
                c3.tuning_import(bad)
            assert e.value.code == cgdir.E_INVAL, bad


def _mixed():
    """Uneven pairs: structure counts 0 to 8, sigma 1 and 1.5, one in physical units
    (1.97 x 1.97 x 2.5 mm voxels, sigmas in mm), one with contour terms at every level; each
    with the oracle's parameters beside the library's."""
    from paper_1301_0970_amd import cgdir
    import oracle
    out = []
    a = P.plain_pair(dims=(64, 48, 30), amp=3.0, iters=30, seed=51)
    out.append((a, {}))
    b = P.head_neck_pair(dims=(72, 60, 36), amp=4.0, k=3, levels=2, iters=20, sigma=1.5, seed=52)
    out.append((b, {}))
    c = P.pelvis_pair(dims=(96, 80, 24), amp=3.0, k=8, levels=3, iters=15, bulge=0.0, seed=53)
    out.append((c, {}))
    d = P.head_neck_pair(dims=(60, 56, 40), amp=3.0, k=1, levels=2, iters=20, sigma=1.0, seed=54)
    d.target_masks, d.moving_masks, d.signs = d.target_masks[:0], d.moving_masks[:0], ()
    out.append((d, {}))
    e = P.plain_pair(dims=(56, 52, 28), amp=3.0, iters=20, levels=2, seed=55)
    out.append((e, dict(spacing=(1.97, 1.97, 2.5), sigma_fluid=2.0, sigma_diff=2.0)))
    f = P.pelvis_pair(dims=(80, 64, 32), amp=3.0, k=2, levels=2, iters=20, bulge=0.0, seed=56)
    out.append((f, dict(contour_level_mask=3)))
    res = []
    for pair, over in out:
        res.append((pair, cgdir.params_for_pair(pair, **over), oracle.params_for(pair, **over)))
    return res


@pytest.mark.timeout(300)
def test_mixed_batch_and_served_against_oracle(orc, progress):
    """Each pair of an uneven mix, registered in one batch and served with overlapping requests,
    against the oracle's Algorithm A: final field within 1e-2 voxel (max-abs), warped moving
    image within 2.5 HU RMS."""
    import torch
    from paper_1301_0970_amd import cgdir
    mix = _mixed()
    pairs = [m[0] for m in mix]
    items = _items(pairs)
    prms = [m[1] for m in mix]
    refs = []
    for pair, _, op in mix:
        progress("oracle: %s %s k %d" % (pair.name, pair.dims, pair.k))
        u, _, _ = orc.register(pair.target, pair.moving, pair.target_masks, pair.moving_masks, op)
        refs.append((u, orc.warp(pair.moving, u)))
    with cgdir.Context(2 << 30, max_slots=4) as ctx:
        outs_b = [torch.empty((3,) + tuple(p.target.shape), device="cuda") for p in pairs]
        progress("mixed batch")
        rc, st = ctx.register_batch(items, prms, outs_b)
        assert rc == cgdir.OK and st == [0] * len(pairs)
        outs_s = [torch.empty((3,) + tuple(p.target.shape), device="cuda") for p in pairs]
        progress("mixed served")
        tickets = [ctx.submit(*it, pr, o) for it, pr, o in zip(items, prms, outs_s)]
        for t in tickets:
            assert ctx.wait(t, int(60e9)) == cgdir.OK
        sts = [ctx.poll(t) for t in tickets]
        assert any(b.t_admit_ns < a.t_done_ns for i, a in enumerate(sts) for b in sts[i + 1:])
        for mode, outs in (("batched", outs_b), ("served", outs_s)):
            for j, ((pair, _, _), (uo, wo), o) in enumerate(zip(mix, refs, outs)):
                warped = ctx.warp(items[j][1], o).cpu().numpy().astype(np.float64)
                ug = o.cpu().numpy()
                err = float(np.abs(ug - uo).max())
                rms = float(np.sqrt(np.mean((warped - wo) ** 2)))
                progress("  %s %s %s k %d: max err %.3g voxel, warped RMS %.3g HU"
                         % (mode, pair.name, pair.dims, pair.k, err, rms))
                assert err <= 1e-2, (mode, pair.name)
                assert rms <= 2.5, (mode, pair.name)
