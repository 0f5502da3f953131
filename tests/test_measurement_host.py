"""Host-side measurement code (no GPU): the bench's per-kernel roofline
accounting and the rocprofv3 summariser."""
import csv
import os

import bench
from paper_1801_08361_amd import rocprof_summary as rs


def test_refinement_rounds_follow_the_library_plan():
    """A plain call at N = 1024 culls and refines separately while more than
    64 hypotheses are planned live (rounds 0-3) and in one kernel after; a
    batch fuses from the latest such round of its attempts and only while it
    plans at most 1024 survivors."""
    res = [dict(mode_evals=0, pair_evals=0, n_valid=1000, n_rounds=10)]
    kernels = {"k_b_refine": (1.0, 4), "k_b_cull_refine": (1.0, 6), "k_b_score": (1.0, 10)}
    r = bench.rooflines(kernels, res, [(100, 5, False, 1024)], batch_pixels=500)
    per = 4 * 500 + bench.REFINE_BYTES_PER_SURVIVOR
    surv = [500, 250, 125, 63, 32, 16, 8, 4, 2, 1]
    assert r["k_b_refine"]["work_per_launch"] * 4 == sum(surv[:4]) * per
    live = [1000] + surv[:-1]
    cull = sum(na * (8 + 4 * 63 + 8) + k * 12 for na, k in zip(live[4:], surv[4:]))
    assert r["k_b_cull_refine"]["work_per_launch"] * 6 == cull + sum(surv[4:]) * per
    # a batch of 40 attempts at N = 256 plans 40 * 32 = 1280 survivors at
    # round 2 (split sums and solve), 640 at round 3: rounds 3-7 fused
    res_b = [dict(mode_evals=0, pair_evals=0, n_valid=256, n_rounds=8)] * 40
    r = bench.rooflines({"k_b_refine": (1.0, 1), "k_b_cull_refine": (1.0, 1)}, res_b,
                        [(100, 5, False, 256)] * 40, batch_pixels=64, batched=True)
    per = 4 * 64 + bench.REFINE_BYTES_PER_SURVIVOR
    surv = [128, 64, 32, 16, 8, 4, 2, 1]
    live = [256] + surv[:-1]
    cull = sum(na * (8 + 4 * 8 + 8) + k * 12 for na, k in zip(live[3:], surv[3:]))
    assert r["k_b_cull_refine"]["work_per_launch"] == 40 * (cull + sum(surv[3:]) * per)
    assert r["k_b_refine"]["work_per_launch"] == 0


def _write(path, header, rows):
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(header)
        w.writerows(rows)


def test_rocprof_summary_scales_by_the_calibration_kernel(tmp_path):
    hdr = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    os.makedirs(tmp_path / "f")
    os.makedirs(tmp_path / "w")
    _write(tmp_path / "f" / "x_counter_collection.csv", hdr, [
        (1, "at::fill_kernel", "FETCH_SIZE", 0.0),
        (2, "at::vectorized_elementwise_kernel<MulFunctor>", "FETCH_SIZE", 131072.0),
        (3, "void rl::k_b_score<4>(rl::Attempt const*)", "FETCH_SIZE", 100.0),
        (4, "void rl::k_b_score<4>(rl::Attempt const*)", "FETCH_SIZE", 300.0),
        (5, "at::huge_render_kernel", "FETCH_SIZE", 9e9)])
    _write(tmp_path / "w" / "x_counter_collection.csv", hdr, [
        (2, "at::vectorized_elementwise_kernel<MulFunctor>", "WRITE_SIZE", 262144.0),
        (3, "void rl::k_b_score<4>(rl::Attempt const*)", "WRITE_SIZE", 10.0),
        (4, "void rl::k_b_score<4>(rl::Attempt const*)", "WRITE_SIZE", 30.0)])
    text = rs.counters(str(tmp_path / "f"), str(tmp_path / "w"))
    assert "| FETCH_SIZE | 131072.0 | 262144 | 2.00000 |" in text
    assert "| k_b_score<4> | 2 | 400 | 20 |" in text


def test_rocprof_summary_stats(tmp_path):
    hdr = ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs", "StdDev"]
    _write(tmp_path / "s_kernel_stats.csv", hdr, [
        ("void rl::k_b_leaves<4>(rl::Attempt const*, rl::Stage)", 2, 80000, 40000, 50, 35000, 45000, 1),
        ("at::other", 1, 1000, 1000, 1, 1000, 1000, 0)])
    text = rs.stats(str(tmp_path))
    assert "| k_b_leaves<4> | 2 | 0.080 | 40.00 | 35.00 | 45.00 |" in text
    assert "other" not in text
