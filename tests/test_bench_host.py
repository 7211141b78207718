"""bench.py host logic that runs without a GPU: the one-GPU contract and the
rocprofv3 trace summary."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_summarize_trace(tmp_path):
    """Per (kernel, grid) rows: the grid in workgroups tells the levels of
    the same kernel apart; averages in microseconds."""
    rows = [("ddi::k_sweep2<false>(args)", 6912 * 128, 128, 1000, 61000),
            ("ddi::k_sweep2<false>(args)", 6912 * 128, 128, 2000, 61000),
            ("ddi::k_sweep2<false>(args)", 120 * 128, 128, 500, 12500),
            ("ddi::k_decide<3>(args)", 64, 64, 0, 4000)]
    p = tmp_path / "trace.csv"
    with open(p, "w") as fh:
        fh.write("Kernel_Name,Grid_Size_X,Grid_Size_Y,Grid_Size_Z,Workgroup_Size_X,"
                 "Workgroup_Size_Y,Workgroup_Size_Z,Start_Timestamp,End_Timestamp\n")
        for name, gx, wx, t0, t1 in rows:
            fh.write(f'"{name}",{gx},1,1,{wx},1,1,{t0},{t1}\n')
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--summarize-trace",
                        str(p)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    lines = [ln for ln in r.stdout.splitlines() if ln.startswith("| ddi::")]
    cells = {(ln.split("|")[1].strip(), int(ln.split("|")[2])): ln.split("|") for ln in lines}
    big = cells[("ddi::k_sweep2<false>", 6912)]
    assert int(big[3]) == 2 and float(big[4]) == 59.5  # calls, average us
    assert float(big[5]) == 59.0 and float(big[6]) == 60.0  # min, max
    assert int(cells[("ddi::k_sweep2<false>", 120)][3]) == 1
    assert ("ddi::k_decide<3>", 1) in cells


def test_psnr_against_worked_values():
    """PSNR = 10 log10(255^2 / MSE) over all pixels and channels: a uniform
    error of 1 grey level is 48.13 dB, of 255 is 0 dB; identical images give
    infinity; the MSE averages over every element."""
    import math
    import torch
    sys.path.insert(0, ROOT)
    import bench
    a = torch.zeros((3, 4, 5))
    assert bench.psnr(a, a) == float("inf")
    assert abs(bench.psnr(a, a + 1.0) - 20 * math.log10(255.0)) < 1e-9
    assert abs(bench.psnr(a, a + 255.0)) < 1e-9
    b = a.clone()
    b[0, 0, 0] = 60.0  # MSE = 3600 / 60 = 60
    assert abs(bench.psnr(a, b) - 10 * math.log10(255.0 ** 2 / 60.0)) < 1e-9


def test_precision_roofline_bound_by_intensity():
    """The mixed-precision leg's roofline: flops from the residual of every
    block plus the CG steps run, bytes from the correction-sweep model,
    bound chosen against the 9.8 flops/byte ridge; None without timings."""
    import bench
    prm = bench.precision_params()
    assert bench.precision_roofline(prm, {"t": [], "steps": 0.0, "refs": 0}) is None
    # 2 solves x 2 steps x 2 sweeps, 100 us each
    m = prm["inner_sweeps"]
    iso = {"t": [[0.1] * (2 * m)] * 2, "refs": 4}
    nblk = 64 * 36 * 3
    few = bench.precision_roofline(prm, dict(iso, steps=0.0))
    many = bench.precision_roofline(prm, dict(iso, steps=8.0 * nblk * len(iso["t"]) * 2 * m))
    assert few["bound"] == "hbm" and many["bound"] == "alu"
    assert few["avg_launch_us"] == 100.0
    bytes_ = bench.correction_bytes(m, 1) * 4
    assert abs(few["hbm_gbs"] - bytes_ / (0.1 * 8 * 1e-3) / 1e9) < 0.1
    flops = 64 * 64 * (8 * nblk * (bench.FLOPS_RESIDUAL + 1))
    assert abs(few["valu_tflops"] - flops / (0.8e-3) / 1e12) < 1e-3
