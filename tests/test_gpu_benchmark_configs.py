"""Parity at the benchmark configurations, over every voxel, against the FP64 oracle.

The head-and-neck workload (256 x 256 x 128, 3 levels x 100 iterations, sigma 1.5, k = 5) and
the pelvis workload (512 x 512 x 128, 3 levels x 150 iterations, sigma 1, k = 8), the seeded
phantoms the benchmark registers:

* the oracle's own trajectory: Algorithm A through the coarse levels and the prolongation to
  the finest level (the oracle's register with no finest-level iteration returns that field),
  then the finest-level loop one iteration at a time with the oracle's step, which is the
  iteration its register runs (pinned on the CPU);
* teacher-forced iterations (Eq.7 and Algorithm A steps 1-4): at n = 0, 1, 10, 50 and the last
  iteration, one GPU iteration from fp32(u_n) against the oracle's iteration from the same
  field, max-abs over every voxel <= 1e-4 voxel;
* the full registration in the benchmark's launch configuration (a context whose tile autotuner
  picks the shapes, the pair's own parameters) against the oracle's field after the last
  iteration: max-abs over every voxel <= 1e-2 voxel, and the moving image warped by each field
  within 2.5 HU RMS (1e-3 of the 2500 HU range).

The pelvis trajectory does not keep the final-field bar.  Its finest level amplifies
perturbations of the size of one iteration's single-precision rounding: the FP64 oracle run
twice, once with a random perturbation of +-2e-6 voxel added after every iteration, differs
from itself by 0.038 voxel after 75 iterations, 0.14 after 100 and 0.018 after 150 (the GPU
against the oracle from the same start: 0.0042, 0.175 and 0.030, at the same voxels), while a
single rounding of the start field alone stays below 1e-6.  The final field differs from the
oracle's by 0.037 voxel at most (271 of 100.7 M components above 1e-2, at the volume's top
plane in air); that test is an expected failure with this reason, and its figures are printed.
The teacher-forced bar and the warped-image bar hold.

The oracle needs about a minute (head-and-neck) and four (pelvis) on 16 host threads; each
run reports its progress as it goes.
"""
import time

import numpy as np
import pytest

from paper_1301_0970_amd import phantom as P

pytestmark = pytest.mark.gpu

STEP_TOL = 1e-4
FINAL_TOL = 1e-2
WARP_RMS_TOL = 2.5


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _worst(err, u):
    """Where the largest error is: (component, z, y, x), the error and |u| there."""
    idx = np.unravel_index(int(np.argmax(err)), err.shape)
    return "at (c, z, y, x) = %s: err %.3g, |u| %.3g" % (tuple(int(i) for i in idx), float(err[idx]),
                                                          float(abs(u[idx])))


def _run(pair, orc, say):
    """GPU registration and teacher-forced iterations against the oracle's trajectory: the
    per-iteration errors, the final-field error and the warped-image RMS difference."""
    from paper_1301_0970_amd import cgdir
    name = pair.name
    lam, sg = [1e-3] * pair.k, list(pair.signs)
    n_fin = pair.iters[0]
    snaps = sorted({0, 1, 10, 50, n_fin - 1})
    t, m, tm, mm = dev(pair.target), dev(pair.moving), dev(pair.target_masks), dev(pair.moving_masks)
    pool = 3 * cgdir.footprint(*pair.dims, pair.k, cgdir.params_for_pair(pair)) + (256 << 20)
    step_err = {}
    with cgdir.Context(pool) as ctx:
        say("%s %s: GPU registration %d levels x %s" % (name, pair.dims, pair.levels, pair.iters))
        ug = ctx.register(t, m, tm, mm, cgdir.params_for_pair(pair)).cpu().numpy()
        wg = ctx.warp(m, dev(ug)).cpu().numpy()
        t0 = time.time()
        say("%s: oracle coarse levels and prolongation" % name)
        prm0 = orc.params_for(pair, iters=(0,) + tuple(pair.iters[1:]))
        u, _, _ = orc.register(pair.target, pair.moving, pair.target_masks, pair.moving_masks, prm0)
        Ip = [orc.modified_image(pair.moving, pair.moving_masks[i], sg[i]) for i in range(pair.k)]
        Tp = [orc.modified_image(pair.target, pair.target_masks[i], sg[i]) for i in range(pair.k)]
        one = cgdir.params_for_pair(pair, levels=1, iters=(1,))
        say("%s: oracle at the finest level (%.0f s so far)" % (name, time.time() - t0))
        for n in range(n_fin):
            if n in snaps:
                u32 = u.astype(np.float32)
                ref, _ = orc.step(pair.moving, pair.target, Ip, Tp, lam, pair.sigma, pair.sigma,
                                  u32.astype(np.float64))
                got = ctx.register(t, m, tm, mm, one, initial=dev(u32)).cpu().numpy()
                err = np.abs(got - ref)
                step_err[n] = float(err.max())
                say("%s: teacher-forced iteration %d: max |du| %.3g, max err %.3g %s"
                    % (name, n, float(np.abs(ref - u32).max()), step_err[n], _worst(err, ref)))
                del ref, got, err
            u, _ = orc.step(pair.moving, pair.target, Ip, Tp, lam, pair.sigma, pair.sigma, u)
            if (n + 1) % 10 == 0:
                say("%s: oracle finest iteration %d/%d (%.0f s)" % (name, n + 1, n_fin, time.time() - t0))
    err = np.abs(ug - u)
    final = float(err.max())
    say("%s: final field max err %.3g %s; %d components above %g"
        % (name, final, _worst(err, u), int((err > FINAL_TOL).sum()), FINAL_TOL))
    wo = orc.warp(pair.moving, u)
    rms = float(np.sqrt(np.mean((wg.astype(np.float64) - wo) ** 2)))
    say("%s: warped moving image RMS difference %.3g HU" % (name, rms))
    return {"step_err": step_err, "final": final, "warp_rms": rms}


@pytest.fixture(scope="module")
def head_neck_run(orc, progress):
    return _run(P.head_neck_pair(), orc, progress)


@pytest.fixture(scope="module")
def pelvis_run(orc, progress):
    return _run(P.pelvis_pair(), orc, progress)


def _check_steps(res):
    bad = {n: e for n, e in res["step_err"].items() if not e <= STEP_TOL}
    assert not bad, "teacher-forced iterations above %g voxel: %s" % (STEP_TOL, bad)


@pytest.mark.timeout(900)
def test_head_neck_teacher_forced(head_neck_run):
    _check_steps(head_neck_run)


def test_head_neck_final_field_and_warped_image(head_neck_run):
    assert head_neck_run["final"] <= FINAL_TOL
    assert head_neck_run["warp_rms"] <= WARP_RMS_TOL


@pytest.mark.timeout(1200)
def test_pelvis_teacher_forced(pelvis_run):
    _check_steps(pelvis_run)


def test_pelvis_warped_image(pelvis_run):
    assert pelvis_run["warp_rms"] <= WARP_RMS_TOL


@pytest.mark.xfail(strict=False, reason="the pelvis finest level amplifies per-iteration rounding-size "
                   "perturbations to 1e-2..1e-1 voxel in the FP64 oracle itself (module docstring)")
def test_pelvis_final_field(pelvis_run):
    assert pelvis_run["final"] <= FINAL_TOL
