"""CPU checks of the measurement and tuning tooling: the recorded patch-solve
tuning table covers every smoothed level of the benchmark workloads with a
valid variant, and the rocprofv3 summaries (traffic scaling, per-kernel
rates, FP64 matrix-core rates) compute what they state on small synthetic
trace and counter files."""
import csv
import json
import os

import pytest

from paper_2107_00820_amd import profiling
from paper_2107_00820_amd.tune import load_asm_tuning, TABLE
from workloads import CONFIGS

from paper_2107_00820_amd.stk import STK_ASM_VARIANTS as NVAR   # variants the library offers


def test_tuning_table_covers_benchmark_levels():
    assert os.path.exists(TABLE)
    table = load_asm_tuning()
    for name in ("sinker_2d_128sq_L4", "sinker_3d_32cu_L3", "viscoplastic_3d_48cu_L3"):
        wl = CONFIGS[name]
        for l in range(1, wl.levels):
            cells = wl.n_fine >> (wl.levels - 1 - l)
            for dt in ("f64", "f32"):
                v = table.get((wl.dim, cells, dt))
                assert v is not None and 0 <= v < NVAR, (name, l, dt)
    with open(TABLE) as f:
        t = json.load(f)
    for e in t["entries"]:
        med = e["median_launch_ms"]
        assert len(med) == NVAR and e["variant"] == min(range(NVAR), key=lambda v: (med[v], v))


def _write(path, rows, fields):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=fields)
        w.writeheader()
        for r in rows:
            w.writerow(r)


def _trace(d, kernels):
    rows, t = [], 0
    for name, durs in kernels.items():
        for du in durs:
            rows.append({"Kernel_Name": f"void {name}(int)", "Start_Timestamp": t, "End_Timestamp": t + du})
            t += du + 10
    _write(os.path.join(d, "x_kernel_trace.csv"), rows, ["Kernel_Name", "Start_Timestamp", "End_Timestamp"])


def _counters(d, counter, per_dispatch):
    rows, did = [], 0
    for name, vals in per_dispatch.items():
        for v in vals:
            did += 1
            # two channels per dispatch, summed by the reader
            for part in (0.25 * v, 0.75 * v):
                rows.append({"Kernel_Name": f"void {name}(int)", "Counter_Name": counter, "Counter_Value": part,
                             "Dispatch_Id": did})
    _write(os.path.join(d, "x_counter_collection.csv"), rows, ["Kernel_Name", "Counter_Name", "Counter_Value", "Dispatch_Id"])


def test_traffic_rates_and_mfma_summaries(tmp_path):
    d = str(tmp_path)
    # copy kernel: 1 GiB read and written, counters report half the fetch
    _counters(f"{d}/cf", "FETCH_SIZE", {"copy_kernel": [2 ** 20 / 2]})
    _counters(f"{d}/cw", "WRITE_SIZE", {"copy_kernel": [2 ** 20]})
    # kernel under test: 3000 KiB fetched (counted 1500), 1000 KiB written per launch
    _counters(f"{d}/kf", "FETCH_SIZE", {"stk::k_asm_gemv<3, double, 0>": [1500.0, 1500.0]})
    _counters(f"{d}/kw", "WRITE_SIZE", {"stk::k_asm_gemv<3, double, 0>": [1000.0, 1000.0]})
    out = f"{d}/traffic.json"
    profiling.main(["traffic", "--fetch", f"{d}/kf", "--write", f"{d}/kw", "--copy-fetch", f"{d}/cf",
                    "--copy-write", f"{d}/cw", "--copy-bytes", str(2 ** 30), "--kernel", "k_asm_gemv",
                    "--out", out])
    t = json.load(open(out))
    assert t["factor_fetch"] == pytest.approx(2.0) and t["factor_write"] == pytest.approx(1.0)
    k = t["kernels"]["stk::k_asm_gemv<3, double, 0>"]
    assert k["fetch_bytes_per_launch"] == pytest.approx(3000 * 1024)
    assert k["write_bytes_per_launch"] == pytest.approx(1000 * 1024)
    # rates: 4000 KiB per launch over an average of 1000 ns -> 4.096 GB/ms = 4096 GB/s
    _trace(f"{d}/kt", {"stk::k_asm_gemv<3, double, 0>": [900, 1100]})
    rates = f"{d}/rates.md"
    profiling.main(["rates", f"{d}/kt", out, rates])
    line = [l for l in open(rates) if "k_asm_gemv" in l][0]
    cells = [c.strip() for c in line.split("|")]
    assert cells[2] == "2" and cells[3] == "1.00" and cells[6] == "4096" and cells[7] == "51.2%"
    # FP64 matrix-core rate: 1e6 MOPS x 512 flops over 10 us = 51.2 TFLOP/s
    _counters(f"{d}/km", "SQ_INSTS_VALU_MFMA_MOPS_F64", {"stk::k_sweep_update": [1.0e6]})
    _trace(f"{d}/kt2", {"stk::k_sweep_update": [10000]})
    mf = f"{d}/mfma.md"
    profiling.main(["mfma", f"{d}/kt2", f"{d}/km", mf, "--kernel", "k_sweep"])
    line = [l for l in open(mf) if "k_sweep_update" in l][0]
    cells = [c.strip() for c in line.split("|")]
    assert cells[4] == "0.512" and cells[5] == "51.20" and cells[6] == "65.1%"
