"""Host logic of bench.py, without a GPU: the nearest-rank percentile, the
algorithmic byte counts the roofline divides by (pinned to the figures worked
out by hand from the per-unit formulas at the full workload sizes), the
recorded-traffic lookup and its hash guard, and the one-GPU limit.
"""

import os
import subprocess
import sys
from types import SimpleNamespace

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_percentile_is_nearest_rank():
    xs = list(range(1, 101))
    assert bench.percentile(xs, 50) == 50
    assert bench.percentile(xs, 99) == 99
    assert bench.percentile(xs, 100) == 100
    assert bench.percentile(xs[::-1], 1) == 1
    assert bench.percentile([7.0], 50) == 7.0
    # 10 samples: rank ceil(0.99 * 10) = 10, the largest
    assert bench.percentile([3, 1, 2, 9, 4, 5, 6, 8, 7, 10], 99) == 10


def _level(dim, degree, n_dofs, n_cells, ncomp=1):
    return SimpleNamespace(dim=dim, degree=degree, n_dofs=n_dofs, n_cells=n_cells, ncomp=ncomp)


@pytest.mark.parametrize("word,expected", [(8, 402_397_200), (4, 215_354_376)])
def test_operator_bytes_of_the_64_cube(word, expected):
    # 2 s N + 4 C q + s C q d(d+1)/2 with N = 129^3, C = 64^3, q = 27
    fine = _level(3, 2, 129 ** 3, 64 ** 3)
    assert bench.vmult_bytes(fine, word) == expected


def test_operator_bytes_of_the_q3_ball_and_the_beam():
    # 96^3 Q3 ball: N = 289^3, C = 96^3, q = 64
    assert bench.vmult_bytes(_level(3, 3, 289 ** 3, 96 ** 3), 8) == 3_330_602_512
    # elasticity stores J^-1 and w det J: d^2 + 1 = 10 words per point; the
    # vectors count the three components (N = 3 x 161 x 33 x 33 nodes)
    beam = _level(3, 2, 3 * 161 * 33 * 33, 80 * 16 * 16, ncomp=3)
    assert bench.vmult_bytes(beam, 8) == 2 * 8 * beam.n_dofs + 4 * beam.n_cells * 27 + 8 * beam.n_cells * 27 * 10
    # several right-hand sides: the vectors count nr times, the map and geometry once
    fine = _level(3, 2, 129 ** 3, 64 ** 3)
    assert bench.vmult_bytes(fine, 8, nr=4) - bench.vmult_bytes(fine, 8) == 3 * 2 * 8 * fine.n_dofs


def test_transfer_bytes_of_the_64_cube():
    # 2,048,383 unconstrained fine points (127^3) owned by 29^3 coarse cells
    coarse = _level(3, 2, 59 ** 3, 29 ** 3)
    npts = 127 ** 3
    # prolongation: per point 4 + 3 s + 2 s, per coarse cell 8 + 4 q + s q
    assert bench.transfer_bytes(coarse, npts, 8, True) == 98_226_000
    assert bench.transfer_bytes(coarse, npts, 4, True) == 54_624_328
    # restriction: per point 4 + 3 s + s, per coarse cell 8 + 4 q + 2 s q
    assert bench.transfer_bytes(coarse, npts, 8, False) == 87_106_960
    assert bench.transfer_bytes(coarse, npts, 4, False) == 49_064_808


def test_flop_counts_at_the_full_sizes():
    # 75^3 Q4 ball: C = 421,875 cells, n = 5: 12 sweeps of 2 n^4 and 15 flops per Gauss point
    fine = _level(3, 4, 301 ** 3, 75 ** 3)
    assert bench.vmult_flops(fine) == 421_875 * (24 * 625 + 15 * 125) == 7_119_140_625
    assert bench.vmult_flops(fine, nr=4) == 4 * 7_119_140_625
    # 2D Q1: 8 sweeps of 2 n^3 and 6 flops per point
    assert bench.vmult_flops(_level(2, 1, 65 ** 2, 64 ** 2)) == 64 ** 2 * (8 * 2 * 8 + 6 * 4)
    assert bench.vmult_flops(_level(3, 2, 100, 10, ncomp=3)) is None
    # transfer at Q4: 3 bases of 24 flops and 2 (125 + 25 + 5) per value
    coarse = _level(3, 4, 137 ** 3, 34 ** 3)
    assert bench.transfer_flops(coarse, 1000) == 1000 * (72 + 310)
    assert bench.transfer_flops(coarse, 1000, nr=2) == 1000 * (72 + 620)


def test_recorded_traffic_is_dropped_when_the_kernels_changed(tmp_path, monkeypatch):
    good = tmp_path / "good.txt"
    good.write_text("# comment\n"
                    f"kernel_sources_sha256_16 = {bench.kernel_source_hash()}\n"
                    "traffic_bytes.operator_fp64 = 259350727\n"
                    "# traffic_bytes.operator_fp32 = 1\n")
    stale = tmp_path / "stale.txt"
    stale.write_text("kernel_sources_sha256_16 = 0000000000000000\n"
                     "traffic_bytes.operator_fp64 = 259350727\n")
    paths = {"good": str(good), "stale": str(stale), "missing": str(tmp_path / "none.txt")}
    monkeypatch.setattr(bench, "traffic_file", lambda tag: paths[tag])
    assert bench.recorded_traffic("good") == {"operator_fp64": 259350727.0}
    assert bench.recorded_traffic("stale") == {}
    assert bench.recorded_traffic("missing") == {}


def test_operator_traffic_follows_the_variant_that_ran():
    traffic = {"operator_fp64": 1.0, "kernel:vmult_kernel<3, 5, double, 1, 0, 1, 0, 1, 1>": 100.0,
               "kernel:gather_kernel<1, 1, double>@fine": 20.0, "kernel:copy_idx_kernel<double>@fine": 1.5,
               "prolongate_fp64": 7.0}
    ran = {"launches": ["vmult_kernel<3, 5, double, 1, 0, 1, 0, 1, 1>", "gather_kernel<1, 1, double>",
                        "copy_idx_kernel<double>"]}
    other = {"launches": ["vmult_kernel<3, 5, double, 1, 0, 1, 1, 0, 1>", "gather_kernel<1, 1, double>",
                          "copy_idx_kernel<double>"]}
    assert bench.entry_traffic(traffic, "operator_fp64", ran) == 121.5
    assert bench.entry_traffic(traffic, "operator_fp64", other) is None  # not profiled: no claim
    assert bench.entry_traffic(traffic, "prolongate_fp64", {}) == 7.0


def test_committed_traffic_summaries_parse():
    keys = {"operator_fp64", "operator_fp32", "prolongate_fp64", "prolongate_fp32", "restrict_fp64",
            "restrict_fp32"}
    for tag in ("cube_q2_64", "beam_q2", "ball_q3_96", "ball_q4_75"):
        kv = {}
        for line in open(bench.traffic_file(tag)).read().splitlines():
            if "=" in line and not line.lstrip().startswith("#"):
                k, v = line.split("=", 1)
                kv[k.strip()] = v.strip()
        assert len(kv["kernel_sources_sha256_16"]) == 16, tag
        got = {k[len("traffic_bytes."):] for k in kv if k.startswith("traffic_bytes.")}
        assert keys <= got, tag
        assert all(float(kv["traffic_bytes." + k]) > 0 for k in keys), tag


def test_operator_kernel_names_follow_degree_and_variant():
    lv = SimpleNamespace(dim=3, degree=4, operator="laplace", VARIANTS=("trilinear+slots", "trilinear+atomic",
                                                                        "metric+slots", "metric+atomic",
                                                                        "trilinear+entity", "metric+entity",
                                                                        "trilinear+slots+transposed", None,
                                                                        "metric+slots+transposed", None,
                                                                        "trilinear+entity+transposed",
                                                                        "metric+entity+transposed"),
                         variant=0, group=1)
    lv.variant_of = lambda dtype: lv.variant
    lv.cells_per_block = lambda dtype: (5 * lv.group, 5, 101)
    assert bench.operator_kernel_names(lv, 8) == ["vmult_kernel<3, 5, double, 1, 0, 1, 0, 0, 1>",
                                                  "gather_kernel<1, 1, double>", "copy_idx_kernel<double>"]
    lv.variant = 2
    assert bench.operator_kernel_names(lv, 4, nr=4) == ["vmult_kernel<3, 5, float, 0, 0, 0, 0, 0, 1>",
                                                        "gather_kernel<1, 4, float>", "copy_idx_kernel<float>"]
    lv.variant = 3
    assert bench.operator_kernel_names(lv, 8) == ["vmult_kernel<3, 5, double, 0, 1, 1, 0, 0, 1>", "fill_kernel<double>",
                                                  "copy_idx_kernel<double>"]
    lv.variant = 4
    assert bench.operator_kernel_names(lv, 8) == ["vmult_kernel<3, 5, double, 1, 0, 1, 1, 0, 1>",
                                                  "gather_kernel<1, 1, double>", "copy_idx_kernel<double>"]
    lv.variant = 5
    assert bench.operator_kernel_names(lv, 4) == ["vmult_kernel<3, 5, float, 0, 0, 1, 1, 0, 1>",
                                                  "gather_kernel<1, 1, float>", "copy_idx_kernel<float>"]
    lv.variant = 10
    assert bench.operator_kernel_names(lv, 4) == ["vmult_kernel<3, 5, float, 1, 0, 1, 1, 1, 1>",
                                                  "gather_kernel<1, 1, float>", "copy_idx_kernel<float>"]
    lv.group = 2
    assert bench.operator_kernel_names(lv, 4) == ["vmult_kernel<3, 5, float, 1, 0, 1, 1, 1, 2>",
                                                  "gather_kernel<1, 1, float>", "copy_idx_kernel<float>"]
    lv.variant = 3  # the atomic variants run one layout block per workgroup
    assert bench.operator_kernel_names(lv, 8)[0] == "vmult_kernel<3, 5, double, 0, 1, 1, 0, 0, 1>"
    el = SimpleNamespace(dim=3, degree=2, operator="elasticity")
    assert bench.operator_kernel_names(el, 8, nr=4) == ["elasticity_kernel<3, double, 0>",
                                                        "gather_kernel<3, 4, double>", "copy_idx_kernel<double>"]


def test_default_workload_is_the_largest_single_gpu_ball():
    wl = bench.WORKLOADS[bench.DEFAULT_WORKLOAD]
    # Q4 on 75^3: (4 * 75 + 1)^3 = 27,270,901 DoFs, five non-nested levels
    assert wl["degree"] == 4 and wl["cells"][-1] == 75 and len(wl["cells"]) == 5
    assert (wl["degree"] * wl["cells"][-1] + 1) ** 3 == 27_270_901
    assert bench.EXTRA_WORKLOADS[bench.DEFAULT_WORKLOAD] == ["ball_q3"]
    assert (3 * bench.WORKLOADS["ball_q3"]["cells"][-1] + 1) ** 3 == 24_137_569


def test_goldens_quoted_by_the_bench_parse():
    for name in {w["golden"] for w in bench.WORKLOADS.values() if w.get("golden")}:
        g = bench.load_golden(name)
        levels = [int(v) for v in g["level_dofs"].split()]
        assert len(g["samples"]) == int(g["samples"].shape[0]) > 0 and g["samples"].shape[1] == 4
        assert int(g["iterations_fp64"]) == len(g["history_fp64"].split()) - 1
        assert all(f"bounds.{l}" in g for l in range(1, len(levels)))


def test_more_than_one_gpu_is_refused_before_any_gpu_work():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""
