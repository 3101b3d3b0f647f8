"""Host logic of bench.py that needs no GPU: which roofline a process is measured against, the
sweep's markdown table, and the refusal of more than one GPU."""
import bench


def test_roofline_bound_follows_the_machine_balance():
    # 78.6 TFLOP/s over 8 TB/s: about 9.8 flops per byte
    assert bench.roofline_bound(136, 4 * 300) == "hbm"          # e+e- -> mu+mu-: 4 helicities, ~300 flops each
    assert bench.roofline_bound(224, 64 * (26795 + 2401)) == "alu"   # gg -> tt~gg
    balance = bench.FP64_VALU_PEAK_TFLOPS * 1e12 / (bench.HBM_PEAK_GBS * 1e9)
    assert bench.roofline_bound(100, 0.99 * balance * 100) == "hbm"
    assert bench.roofline_bound(100, 1.01 * balance * 100) == "alu"


def test_sweep_markdown_table():
    res = {"gg_tt": [{"precision": "fp64", "n_evt": 256, "MEs_per_s": 1.0e8},
                     {"precision": "fp64", "n_evt": 1024, "MEs_per_s": 2.0e8},
                     {"precision": "mixed_fp16", "n_evt": 256, "MEs_per_s": 1.5e8}]}
    lines = bench.sweep_markdown(res).splitlines()
    assert lines[0] == "| process | form | 2^8 | 2^10 |"
    assert lines[2] == "| gg_tt | fp64 | 1e+08 | 2e+08 |"
    assert lines[3] == "| gg_tt | mixed_fp16 | 1.5e+08 | - |"


def test_more_than_one_gpu_is_refused():
    """the measurement covers one GPU; asked for more, bench.py says so and exits with status 2
    before touching a device"""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=root)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
