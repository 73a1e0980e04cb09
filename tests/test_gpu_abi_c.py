"""A registration driven from plain C through include/cgdir.h: tests/c_register.c, built
with the system C compiler and linked against libcgdir.so, registers a pair held in host
memory with a library-owned pool and writes the field.  It must equal, bit for bit, the same
registration through the Python binding with device tensors (results do not depend on where
the inputs live or on the tile shapes).

The C program runs as a child process before this process touches the GPU (this file sorts
first among the GPU tests)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_1301_0970_amd import phantom as P

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def say(msg):
    print(msg, flush=True)


def test_registration_from_c_equals_the_binding(tmp_path):
    from paper_1301_0970_amd import cgdir
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    libdir = os.path.dirname(cgdir.LIB_PATH)
    exe = tmp_path / "c_register"
    subprocess.run([cc, "-std=c99", "-O2", "-Wall", "-Wextra", "-Werror", "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "c_register.c"), "-L", libdir, "-lcgdir",
                    "-Wl,-rpath," + libdir, "-o", str(exe)], check=True)
    pair = P.head_neck_pair(dims=(61, 47, 29), amp=3.0, k=3, levels=2, iters=12, seed=77)
    prm = cgdir.params_for_pair(pair, contour_level_mask=3, signs=[0, 1, -1])
    nx, ny, nz = pair.dims
    files = {}
    for name, arr in (("target", pair.target.astype(np.float32)), ("moving", pair.moving.astype(np.float32)),
                      ("tmasks", pair.target_masks.astype(np.uint8)), ("mmasks", pair.moving_masks.astype(np.uint8))):
        files[name] = tmp_path / name
        np.ascontiguousarray(arr).tofile(files[name])
    (tmp_path / "params.bin").write_bytes(bytes(prm))
    out = tmp_path / "out.f32"
    say("registration from C, %dx%dx%d k=%d" % (nx, ny, nz, pair.k))
    r = subprocess.run([str(exe), str(nx), str(ny), str(nz), str(pair.k), str(tmp_path / "params.bin"),
                        str(files["target"]), str(files["moving"]), str(files["tmasks"]), str(files["mmasks"]),
                        str(out)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    u_c = np.fromfile(out, dtype=np.float32).reshape((3, nz, ny, nx))
    assert np.isfinite(u_c).all() and np.abs(u_c).max() > 0.1

    import torch
    say("the same registration through the binding")
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()   # noqa: E731
    with cgdir.Context(1 << 30) as ctx:
        u_py = ctx.register(dev(pair.target), dev(pair.moving), dev(pair.target_masks), dev(pair.moving_masks),
                            prm).cpu().numpy()
    np.testing.assert_array_equal(u_c, u_py)
