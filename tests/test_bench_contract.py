"""CPU checks of the benchmark's measurement constants."""
import json
import os

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_flop_count_per_item():
    # integrand 289 x 72 + 17 columns x 8, separable projection for 9 form factors 13,176
    assert bench.item_flops(9, 1, True) == 289 * 72 + 17 * 8 + 13176 == 34120
    # dense Gram: 4 children x 2 M^2 (81 + 25)
    assert bench.item_flops(25, 2, False) == 289 * 72 + 17 * 8 + 4 * 2 * 625 * 106


def test_traffic_belongs_to_the_profiled_kernel():
    """The HBM bytes per item come from counters taken with one version of
    the kernel; if its sources change, the counters must be taken again and
    the hash and figure in bench.py updated (the benchmark otherwise reports
    null traffic)."""
    assert bench.kernel_sources_sha256() == bench.TRAFFIC_SOURCES_SHA256
    with open(os.path.join(ROOT, "profiles", "k_children_c2_counters.md")) as f:
        txt = f.read()
    assert f"per work item {bench.TRAFFIC_BYTES_PER_ITEM} B" in txt


def test_shipped_launch_profile_is_complete():
    with open(os.path.join(ROOT, "paid_1610_09991_amd", "tuned_c2.json")) as f:
        cfg = json.load(f)["config"]
    assert set(cfg) == {"batch", "batch_max", "max_active", "eval_wg_per_cu"}
    assert 1 <= cfg["batch"] <= cfg["batch_max"]


def test_half_zone_variant_counts_only_computed_pairs():
    """the survey's integral count: pairs zero by the inversion symmetry are not
    computed in the half-zone mode and are not counted (20 of 45 for the 9-box
    set, 6 of 15 for the 5-function set, 156 of 325 for the 25-box set)"""
    import workloads as W
    assert bench.computed_pairs(W.config("C2")["ff"], 1) == 25
    assert bench.computed_pairs(W.config("C1")["ff"], 1) == 9
    assert bench.computed_pairs(W.config("C4")["ff"], 2) == 169


def test_cpu_baseline_reports_both_oracle_rates():
    """The oracle's rate on the host: OpenMP over containers and one core
    (the serial algorithm), with the sample and the host processor named."""
    import workloads as W
    cfg = W.config("C1")
    r = bench.cpu_baseline(cfg, 5.0, 2, nq=1, max_rows=1)
    assert r["kind"] == "oracle" and r["cores"] == 2 and r["value"] > 0
    assert r["single_thread"]["cores"] == 1 and r["single_thread"]["value"] > 0
    assert "threads visible" in r["host_cpu"]
