"""Conditioning of the pelvis workload's finest level (run by hand on a GPU machine; not
collected by pytest).

From the oracle's own start of the finest level (Algorithm A through the coarse levels and the
prolongation), it registers the finest level on the GPU for n iterations and follows three FP64
oracle trajectories: the oracle itself, and the oracle with a seeded random perturbation of
+-2e-6 voxel (the size of one GPU iteration's single-precision error against the oracle) added
after every iteration.  At each n it prints the largest difference of the GPU's field and of
the perturbed oracle's field from the oracle's, and where it occurs: both grow to 1e-2..1e-1
voxel at the same voxels, so the final-field bar of 1e-2 voxel lies below what the trajectory
itself keeps under rounding-size perturbations.

    PYTHONPATH=. python tests/conditioning_pelvis.py
"""
import time

import numpy as np
import torch

import oracle as orc
from paper_1301_0970_amd import cgdir
from paper_1301_0970_amd import phantom as P

SNAPS = [1, 2, 3, 5, 10, 20, 30, 50, 75, 100, 125, 150]
PERTURBATION = 2e-6


def report(tag, a, b):
    e = np.abs(a - b)
    i = np.unravel_index(int(np.argmax(e)), e.shape)
    print("%s: max %.3g at (c, z, y, x) = %s (u %.4g); components above 1e-3: %d, 1e-4: %d, 1e-5: %d"
          % (tag, e.max(), tuple(int(v) for v in i), b[i], (e > 1e-3).sum(), (e > 1e-4).sum(), (e > 1e-5).sum()),
          flush=True)


def main():
    pair = P.pelvis_pair()
    lam, sg = [1e-3] * pair.k, list(pair.signs)

    def dev(a):
        return torch.from_numpy(np.ascontiguousarray(a)).cuda()
    t, m, tm, mm = dev(pair.target), dev(pair.moving), dev(pair.target_masks), dev(pair.moving_masks)
    t0 = time.time()
    u, _, _ = orc.register(pair.target, pair.moving, pair.target_masks, pair.moving_masks,
                           orc.params_for(pair, iters=(0,) + tuple(pair.iters[1:])))
    u32 = u.astype(np.float32)
    u = u32.astype(np.float64)
    gpu = {}
    with cgdir.Context(6 << 30) as ctx:
        for n in SNAPS:
            gpu[n] = ctx.register(t, m, tm, mm, cgdir.params_for_pair(pair, levels=1, iters=(n,)),
                                  initial=dev(u32)).cpu().numpy()
    Ip = [orc.modified_image(pair.moving, pair.moving_masks[i], sg[i]) for i in range(pair.k)]
    Tp = [orc.modified_image(pair.target, pair.target_masks[i], sg[i]) for i in range(pair.k)]
    rng = np.random.default_rng(1)
    up = u.copy()
    for n in range(1, SNAPS[-1] + 1):
        u, _ = orc.step(pair.moving, pair.target, Ip, Tp, lam, pair.sigma, pair.sigma, u)
        up, _ = orc.step(pair.moving, pair.target, Ip, Tp, lam, pair.sigma, pair.sigma, up)
        up += rng.uniform(-PERTURBATION, PERTURBATION, size=up.shape)
        if n in gpu:
            report("iteration %3d, GPU vs oracle" % n, gpu[n], u)
            report("iteration %3d, perturbed oracle vs oracle" % n, up, u)
            print("  (%.0f s)" % (time.time() - t0), flush=True)


if __name__ == "__main__":
    main()
