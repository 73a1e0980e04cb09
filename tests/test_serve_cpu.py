"""The serving loop's scheduling rules on the CPU, over a simulated device.

`paper_1301_0970_amd/csrc/cgdir_serve.h` holds the queue, the admission and the serving loop
that libcgdir runs over its device executor; `tests/serve_cpu/sim_serve.cpp` instantiates the
same template over a simulated device and checks, scenario by scenario: first-in first-out
admission by free slots and memory, with nothing overtaking a head that waits for memory; slot
and memory reuse; the lanes of each policy (large and small requests apart, the large ones one
at a time while nothing waits, every admitted request in the ticks while requests wait);
regrouping when a request joins or leaves; cancel, poll and wait on queued, running, finished
and unknown tickets; failures that stay with their request; stop; the bound on kept records;
and submit, poll, wait and cancel from several threads at once.

Every scenario runs in a plain build and in a ThreadSanitizer build (clang's runtime: the GCC
runtime in this image does not intercept the clock-based condition-variable wait that
libstdc++ uses for timed waits, and reports false double locks).  On the CPU a race planted in
a copy of the header, the request's published error written outside the queue lock, fails the
stress scenario under ThreadSanitizer in most runs.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "serve_cpu", "sim_serve.cpp")
INC = ["-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(ROOT, "paper_1301_0970_amd", "csrc")]
CLANG = "/opt/rocm/lib/llvm/bin/clang++"

SCENARIOS = ["fifo", "memory", "lanes_serial", "lanes_backlog", "lanes_all", "lockstep", "regroup",
             "cancel", "failures", "stop", "keep", "stress"]


def _build(out, compiler, flags):
    cmd = [compiler, "-std=c++17", "-pthread", *flags, *INC, SRC, "-o", out]
    subprocess.run(cmd, check=True, capture_output=True, text=True, timeout=300)
    return out


@pytest.fixture(scope="module")
def plain(tmp_path_factory):
    gxx = shutil.which("g++")
    if not gxx:
        pytest.skip("no g++")
    return _build(str(tmp_path_factory.mktemp("serve") / "sim_serve"), gxx, ["-O2", "-Wall", "-Wextra", "-Werror"])


@pytest.fixture(scope="module")
def tsan(tmp_path_factory):
    if not os.path.exists(CLANG):
        pytest.skip("no clang++ with a ThreadSanitizer runtime")
    return _build(str(tmp_path_factory.mktemp("serve_tsan") / "sim_serve_tsan"), CLANG,
                  ["-O1", "-g", "-fsanitize=thread"])


def _run(exe, scenario, env=None):
    p = subprocess.run([exe, scenario], capture_output=True, text=True, timeout=240, env=env)
    assert p.returncode == 0 and ("ok %s" % scenario) in p.stdout, \
        "rc %d\n%s\n%s" % (p.returncode, p.stdout[-3000:], p.stderr[-6000:])


@pytest.mark.parametrize("scenario", SCENARIOS)
def test_scheduler_rules(plain, scenario):
    _run(plain, scenario)


@pytest.mark.parametrize("scenario", SCENARIOS)
def test_scheduler_rules_under_thread_sanitizer(tsan, scenario):
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 exitcode=66")
    _run(tsan, scenario, env)
