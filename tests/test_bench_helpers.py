"""Host-side helpers of bench.py that turn rocprofv3 output into the committed profile summaries:
kernel names with nested template arguments, and the counter summary's scaling by a plain copy."""
import csv
import json
import os

import bench


def test_kernel_short_keeps_nested_template_arguments():
    full = ("void vem::(anonymous namespace)::k_scg_prod<float, 256, vem::(anonymous namespace)::"
            "BlockViewT<float, 6> >(int, vem::(anonymous namespace)::BlockViewT<float, 6>, float const*)")
    assert bench.kernel_short(full) == "k_scg_prod<float, 256, BlockViewT<float, 6> >"
    assert bench.kernel_short("vem::(anonymous namespace)::k_spmv(vem::(anonymous namespace)::SellViewT<double>, "
                              "double const*, double*)") == "k_spmv"
    assert bench.kernel_short("void vem::(anonymous namespace)::k_dots<6>(long, double const*)") == "k_dots<6>"
    assert bench.kernel_short("void at::native::vectorized_elementwise_kernel<4, at::native::neg_kernel>()") is None


def _write_counters(d, counter, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "pmc_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for name, grid, kib in rows:
            w.writerow({"Kernel_Name": name, "Grid_Size": grid, "Counter_Name": counter, "Counter_Value": kib})
    probe = {"copy_read_bytes": 512 * 2**20, "copy_write_bytes": 512 * 2**20,
             "kernels": {"cheb_schur": {"avg_us": 6.0, "algorithmic_bytes": 30.0e6}}}
    with open(os.path.join(d, "probe.json"), "w") as f:
        f.write(json.dumps(probe) + "\n")


def test_counter_summary_scales_by_the_copy(tmp_path, capsys):
    """FETCH_SIZE reading half of the copy's bytes gives factor 2; a kernel's counters are scaled by
    the factors and compared with its algorithmic bytes."""
    copy = "void at::native::vectorized_elementwise_kernel<4, at::native::neg_kernel_cuda>()"
    cheb = "void vem::(anonymous namespace)::k_cheb_iter<double, true, false, false>(vem::SellViewT<double>)"
    fetch, write = str(tmp_path / "fetch"), str(tmp_path / "write")
    _write_counters(fetch, "FETCH_SIZE", [(copy, 1024, 256 * 1024), (cheb, 262144, 15.0e6 / 1024)])
    _write_counters(write, "WRITE_SIZE", [(copy, 1024, 512 * 1024), (cheb, 262144, 2.0e6 / 1024)])
    bench.summarize_pmc(fetch, write)
    out = capsys.readouterr().out
    rec = json.loads(out.strip().splitlines()[-1])
    tv = rec["traffic_value"]
    assert abs(tv["fetch_bytes"] - 30.0e6) < 1.0 and abs(tv["write_bytes"] - 2.0e6) < 1.0
    assert abs(tv["ratio_to_algorithmic"] - 32.0 / 30.0) < 1e-9
    assert "factor 2.0000" in out and "factor 1.0000" in out
