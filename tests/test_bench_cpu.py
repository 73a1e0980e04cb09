"""The bench line's roofline block follows from its inputs (CPU, no GPU).

`bench.roofline` takes the per-launch HIP-event timings of the finest-level step and smoothing
launches and the committed counter summaries under profiles/; these checks recompute each field
from the same inputs: the fraction is the algorithmic bytes of one whole iteration (34 B per
voxel with contour terms: u read and written, I0, T0, the two bit-planes) over the sum of the
two launches' times against 8 TB/s, the traffic is the summaries' per-launch bytes, the VALU
ceiling is their instruction count at 256 CUs x 2.4 GHz, and `bound` names the resource
closer to its ceiling.
"""
import os
import re

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


class _Pelvis:
    k = 8
    dims = (512, 512, 128)


def _stats(t_step, t_smooth, n=33554432, launches=10):
    return [{"name": "step@L0", "voxels": float(n) * launches, "launches": launches, "total_ms": t_step * launches},
            {"name": "smooth@L0", "voxels": float(n) * launches, "launches": launches, "total_ms": t_smooth * launches},
            {"name": "step@L1", "voxels": float(n // 8) * launches, "launches": launches, "total_ms": 0.06 * launches}]


def test_bytes_per_voxel_split():
    assert bench.iteration_bytes_per_voxel(8, False) == 34
    assert bench.iteration_bytes_per_voxel(0, False) == 32
    assert bench.iteration_bytes_per_voxel(3, True) == 35
    for k, metric in ((8, False), (0, False), (5, True)):
        assert (bench.kernel_bytes_per_voxel("step", k, metric) + bench.kernel_bytes_per_voxel("smooth", k, metric)
                == bench.iteration_bytes_per_voxel(k, metric))


def test_fraction_is_the_whole_iteration_against_8_tbs():
    t_step, t_smooth, n = 0.47, 0.38, 33554432
    r = bench.roofline(_stats(t_step, t_smooth, n), _Pelvis, False, "no_such_workload", 5100.0)
    achieved = 34 * n / ((t_step + t_smooth) * 1e-3) / 1e9
    assert r["achieved"] == pytest.approx(achieved, rel=1e-3)
    assert r["frac"] == pytest.approx(achieved / 8000.0, abs=1e-4)
    assert r["peak"] == 8000.0 and r["unit"] == "GB/s"
    assert r["iteration_ms"] == pytest.approx(t_step + t_smooth, abs=1e-5)
    # without counter summaries for the workload: no traffic and no VALU evidence
    assert r["traffic"] is None and "valu" not in r
    per = r["kernels"]
    assert per["step"]["frac"] == pytest.approx(18 * n / (t_step * 1e-3) / 1e9 / 8000.0, abs=1e-4)
    assert per["smooth"]["frac"] == pytest.approx(16 * n / (t_smooth * 1e-3) / 1e9 / 8000.0, abs=1e-4)


def _summary_value(name, key):
    txt = open(os.path.join(ROOT, "profiles", "iteration_pelvis_%s.md" % name)).read()
    return float(re.search(r"^%s:\s*([-0-9.eE+]+)\s*$" % key, txt, re.M).group(1))


def test_counter_summaries_feed_traffic_valu_and_bound():
    if bench.read_profile("pelvis", "hbm") is None or bench.read_profile("pelvis", "valu") is None:
        pytest.skip("the counter summaries were taken on another kernel source")
    t_step, t_smooth, n = 0.47, 0.38, 33554432
    copy = 5100.0
    r = bench.roofline(_stats(t_step, t_smooth, n), _Pelvis, False, "pelvis", copy)
    traffic = _summary_value("hbm", "step_hbm_bytes_per_launch") + _summary_value("hbm", "smooth_hbm_bytes_per_launch")
    assert r["traffic"] == pytest.approx(traffic)
    assert r["traffic_over_algorithmic"] == pytest.approx(traffic / (34 * n), abs=1e-3)
    measured = traffic / ((t_step + t_smooth) * 1e-3) / 1e9
    assert r["measured_gbs"] == pytest.approx(measured, abs=0.1)
    insts = _summary_value("valu", "step_valu_insts_per_launch") + _summary_value("valu", "smooth_valu_insts_per_launch")
    ceiling_ms = insts / (256 * 2.4e9) * 1e3
    assert r["valu"]["ceiling_ms"] == pytest.approx(ceiling_ms, abs=1e-5)
    assert r["valu"]["frac"] == pytest.approx(ceiling_ms / (t_step + t_smooth), abs=1e-4)
    assert r["valu"]["insts_per_voxel"] == pytest.approx(64 * insts / n, abs=0.1)
    hbm_busy = measured / copy
    assert r["bound"] == ("hbm" if hbm_busy >= r["valu"]["frac"] else "alu")
    assert "waves waiting" in r["bound_evidence"]


def test_kernel_source_hash_follows_code_not_comments(tmp_path, monkeypatch):
    """The counter summaries are matched to the kernel sources by a hash that ignores comments
    and blank space: editing a comment keeps it, editing code changes it."""
    src = os.path.join(ROOT, "paper_1301_0970_amd", "csrc")
    dst = tmp_path / "paper_1301_0970_amd" / "csrc"
    dst.mkdir(parents=True)
    for name in ("cgdir_kernels.hip", "cgdir_internal.h"):
        (dst / name).write_text(open(os.path.join(src, name)).read())
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    base = bench.kernel_source_hash()
    k = dst / "cgdir_kernels.hip"
    text = k.read_text()
    k.write_text(text.replace("// ", "//  a reworded comment ", 1) + "\n/* a new\n block comment */\n\n")
    assert bench.kernel_source_hash() == base
    k.write_text(text.replace("kTileX", "kTileX ", 1).replace("+ 1", "+ 2", 1))
    assert bench.kernel_source_hash() != base
