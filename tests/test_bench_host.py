"""Host logic of bench.py: kernel classes of rocprofv3 names, the roofline
bound of a class, the whole-solve figures, and the traffic summaries written
from counter output (no GPU)."""
import csv
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


@pytest.mark.parametrize("name,cls", [
    ("void gk::panel_kernel<4, 2, true, false, false, true, true, false>(gk::PanelArgs)", "panel_update_self"),
    ("void gk::panel_kernel<4, 1, false, false, true, false, false, false>(gk::PanelArgs)", "panel_gramv"),
    ("void gk::panel_kernel<4, 0, false, true, false, true, false, false>(gk::PanelArgs)", "panel_apply_self"),
    ("void gk::panel_kernel<4, 0, false, true, false, false, true, true>(gk::PanelArgs)", "panel_apply_write"),
    ("void gk::tsgemm_mfma_kernel<false, true>(long, int, void const*)", "assemble"),
    ("void gk::tsgemm_mfma_kernel<false, false>(long, int, void const*)", "tsgemm"),
    ("gk::gram_f32mma_kernel(long, int, float const*, long, int)", "arch_gram"),
    ("gk::tsgemm_f32mma_kernel(long, int, float const*)", "arch_update"),
    ("gk::update_bf3_kernel(long, int, float const*, long, int, double const*, double*, int const*)", "arch_update"),
    ("gk::assemble_f32mma_kernel(long, int, float const*)", "assemble"),
    ("gk::gram_mfma_kernel(long, int, double const*)", "gram"),
    ("void gk::arch_gram_kernel<4>(long, float const*)", "arch_gram"),
    ("void gk::spmm_gram64_kernel<2>(long, int const*)", "spmm_diff"),
    ("void gk::spmm_diff_kernel<4, 2, true>(gk::SpmmShape, gk::SpmmGraph)", "spmm_diff"),
    ("gk::cholqr_blk_batch_kernel(gk::CholqrBatch)", "cholqr"),
    ("gk::btd_cheb_tile_kernel(int, int)", "cheb_step"),
    ("__amd_rocclr_copyBuffer", None),
    ("gk::zero_kernel(unsigned long*, unsigned long)", None),
])
def test_kernel_class_of(name, cls):
    assert bench.kernel_class_of(name) == cls


def test_classify_bound_follows_intensity():
    # 1 GB in 1 ms: 1000 GB/s below the FP64 ridge (78.6 / 8 = 9.8 flop/B)
    low = bench.classify(dict(name="panel_update_self", total_ms=1.0, alg_bytes=1e9, alg_flops=5e9))
    assert low["bound"] == "hbm" and low["achieved"] == pytest.approx(1000.0)
    assert low["frac"] == pytest.approx(1000.0 / bench.HBM_PEAK_GBS)
    # 100 flop/B on the FP32 matrix cores: compute-bound against 157.3 TF/s
    high = bench.classify(dict(name="arch_gram", total_ms=1.0, alg_bytes=1e9, alg_flops=1e11))
    assert high["bound"] == "mfma" and high["peak"] == 157.3
    assert high["achieved"] == pytest.approx(100.0)
    # the archive update runs on the BF16 cores (six part products per float32
    # product): at 32 flop/B it sits below that ridge (52 flop/B) on HBM
    upd = bench.classify(dict(name="arch_update", total_ms=1.0, alg_bytes=1e9, alg_flops=3.2e10))
    assert upd["bound"] == "hbm" and upd["ridge"] == pytest.approx(2500.0 / 6 / 8)
    # single-workgroup chains carry no chip-wide fraction
    lat = bench.classify(dict(name="cholqr", total_ms=1.0, alg_bytes=1e6, alg_flops=1e6))
    assert lat["bound"] == "latency" and lat["frac"] is None


def test_kernel_table_whole_solve():
    agg = {"spmm_diff": dict(name="spmm_diff", launches=20, total_ms=2.0, alg_bytes=8e9, alg_flops=8e9),
           "cholqr": dict(name="cholqr", launches=40, total_ms=1.0, alg_bytes=1e6, alg_flops=1e6)}
    table, whole = bench.kernel_table(agg, 2)
    assert table["spmm_diff"]["ms_per_step"] == pytest.approx(1.0)
    assert table["spmm_diff"]["avg_launch_us"] == pytest.approx(100.0)
    assert whole["latency_chain_ms"] == pytest.approx(0.5)
    # 4 GB per solve at 8 TB/s
    assert whole["t_bound_ms"] == pytest.approx(0.5)
    assert whole["alg_bytes_per_solve"] == pytest.approx(4e9)


def _pmc_csv(d, counter, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "pmc_counter_collection.csv"), "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for i, (name, v) in enumerate(rows):
            w.writerow(dict(Dispatch_Id=i, Kernel_Name=name, Counter_Name=counter, Counter_Value=v))


def test_traffic_summary_calibration(tmp_path):
    # the calibration copy moves 1 GiB; FETCH_SIZE counts it as half that
    kib = (1 << 30) / 1024.0
    spmm = "void gk::spmm_diff_kernel<4, 2, true>(gk::SpmmShape)"
    _pmc_csv(tmp_path / "f", "FETCH_SIZE", [("__amd_rocclr_copyBuffer", kib / 2), (spmm, 1000.0), (spmm, 3000.0)])
    _pmc_csv(tmp_path / "w", "WRITE_SIZE", [("__amd_rocclr_copyBuffer", kib), (spmm, 500.0), (spmm, 500.0)])
    out = tmp_path / "profiles"
    out.mkdir()
    bench.summarize_profiles(None, str(tmp_path / "f"), str(tmp_path / "w"), "unit", "unit", "stats-cmd",
                             "pmc {ctr}", out_dir=str(out))
    text = (out / "spmm_diff_unit_traffic.txt").read_text()
    vals = dict(line.split(":", 1) for line in text.splitlines() if ":" in line and not line.startswith("#"))
    # per dispatch: fetch 2000 KiB x 2 + write 500 KiB x 1
    assert float(vals["hbm_bytes_per_launch"]) == pytest.approx(1024.0 * (2000.0 * 2 + 500.0))
    h = bench._kernel_hash(bench._sources("spmm_diff"))
    assert vals["source_hash"].strip() == h
    assert bench._traffic_from_profile("spmm_diff", "unit", h, str(out)) == pytest.approx(1024.0 * 4500.0)
    # a summary taken on other sources is not used
    assert bench._traffic_from_profile("spmm_diff", "unit", "0" * 16, str(out)) is None
