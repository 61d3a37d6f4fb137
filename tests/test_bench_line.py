"""The benchmark's last stdout line: short enough to be read whole, and
carrying the keys of the contract (metric, value, roofline, cpu_baseline ...).
Built from synthetic section results on the CPU; no GPU involved."""

import json

import bench


def fake_sections():
    args = bench.parse([])
    roof = {"bound": "alu", "achieved": 10.45, "peak": 39.32, "unit": "TOP/s", "frac": 0.2658,
            "traffic": 8.27e9, "kernel": "k_gemm_simple<L=8> grouped leaf products",
            "op": "32x32->64-bit limb multiply-accumulate, L^2=64 per MP multiply-add", "launch_ms": 26.99,
            "units_per_launch": 4406636544.0, "leaf_share_of_step": 0.8512}
    h = {"ms": 31.14123456, "rate": 5.5167891234e11, "roofline": roof,
         "parity": "whole 2048x2048 result bit-identical to the C oracle (sha256)",
         "others_ms": {"simple": 51.12, "block": 67.13, "strassen": 31.55}}
    cpu = {"value": 2.28e8, "unit": "2mln/s", "cores": 16, "kind": "oracle",
           "sample": "C oracle winograd (cutoff 64, peel) on the leading 1024x1024 blocks of the same 256-bit "
                     "log-uniform A and B, 19.9 s on 16 threads"}
    slice_res = {"value": 2.21e12, "ms_per_step": 7.812, "speedup_vs_limb": 4.012, "windows": [296, 296],
                 "roofline": {"bound": "mfma", "achieved": 2090.0, "peak": 5000.0, "unit": "TOP/s int8",
                              "frac": 0.418, "kernel": "k_slice_gemm v_mfma_i32_32x32x32_i8", "launch_ms": 7.31},
                 "other_ms": 0.512, "early_stop": {"u0": 35, "diagonals": 75, "tiles_recomputed": 0, "tiles": 64,
                                                  "second_pass_ms": 0.01, "one_pass_ms_per_step": 13.3}}
    acc = {"limb_winograd": 7.9e6, "slice": 0.0, "entries": 8191}
    lu = {k: {"info": 0, "lu_ms": 13.21, "solve_ms": 5.812, "rate": 6.8e9, "residual_log2": -1001.25,
              "max_abs_x_minus_1_log10": -149.35} for k in ("random", "hilbert")}
    c2 = {nn: {a: 6.571 for a in ("simple", "block", "strassen", "winograd")} for nn in (1023, 1024)}
    serve = {"requests": 10000, "p50_ms": 1.472, "p99_ms": 24.91, "req_per_s": 1279.0, "gemm_2mln_per_s": 3.1e11,
             "saturated_req_per_s": 1601.0, "arrival_rate": 1280.8, "peak_admitted_gb": 3.712, "failed": 0,
             "identical_alone_vs_mix": "256/256"}
    return args, h, cpu, slice_res, acc, lu, c2, serve


def test_final_line_is_short_and_complete():
    args, h, cpu, slice_res, acc, lu, c2, serve = fake_sections()
    out = bench.final_line(args, h, cpu, slice_res, acc, lu, c2, serve)
    line = json.dumps(out, separators=(",", ":"))
    assert len(line) < bench.FINAL_LINE_MAX, len(line)
    back = json.loads(line)
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline", "parity"):
        assert k in back, k
    assert "workload" in back["config"]
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in back["roofline"], k
    for k in ("value", "unit", "cores", "kind", "sample"):
        assert k in back["cpu_baseline"], k
    assert back["n_gpus"] == 1 and back["higher_is_better"] is True


def test_sig_rounds_to_significant_digits():
    assert bench.sig(5.5167891234e11) == 5.517e11
    assert bench.sig(0.26583) == 0.2658
    assert bench.sig(None) is None and bench.sig(0) == 0


def test_more_than_one_gpu_is_refused():
    import pytest
    with pytest.raises(SystemExit) as e:
        bench.main(["--gpus", "2"])
    assert e.value.code == 2
