"""bench.py pieces that need no GPU: the one-GPU refusal, the counter-summary lookup
behind `roofline.traffic`, and the U-Net FLOP count behind its TFLOP/s."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""


def test_traffic_comes_only_from_counters_of_the_current_kernel(tmp_path, monkeypatch):
    f = tmp_path / "counters.json"
    rec = {"kernel_hash": bench.kernel_hash(), "nodes": 64, "tile_width": 128, "bytes_per_launch": 123.0}
    f.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "COUNTERS_FILE", str(f))
    assert bench.measured_traffic(64, 128) == 123.0
    assert bench.measured_traffic(64, 64) is None            # another tile width
    assert bench.measured_traffic(65, 128) is None           # another lattice
    f.write_text(json.dumps(dict(rec, kernel_hash="0" * 16)))
    assert bench.measured_traffic(64, 128) is None           # the kernel changed since
    monkeypatch.setattr(bench, "COUNTERS_FILE", str(tmp_path / "missing.json"))
    assert bench.measured_traffic(64, 128) is None


def test_kernel_hash_covers_every_kernel_source(tmp_path, monkeypatch):
    srcs = []
    for i in range(3):
        p = tmp_path / f"s{i}.hip"
        p.write_text(f"// {i}\n")
        srcs.append(str(p))
    monkeypatch.setattr(bench, "KERNEL_SOURCES", srcs)
    h0 = bench.kernel_hash()
    assert len(h0) == 16 and int(h0, 16) >= 0
    (tmp_path / "s2.hip").write_text("// changed\n")
    assert bench.kernel_hash() != h0


def test_unet_flop_count():
    # 2 x 9 x Cin x Cout per output pixel over the 15 layers (channels padded to 32, the
    # 5 input channels to 32), at 256^2: 23.56 GFLOP forward, and three times that minus
    # the first layer's data gradient for a training step
    fwd, train = bench.unet_flops_per_sample()
    first = 2.0 * 9 * 32 * 32 * 256 * 256
    assert abs(fwd - 23.56e9) < 0.01e9
    assert train == 3 * fwd - first
    assert abs(train - 69.46e9) < 0.01e9


def test_unet_bound_is_at_least_the_matrix_core_time_and_the_traffic_time():
    # the bound sums, per kernel, the larger of matrix-core time and HBM time: it can be
    # no less than either summed alone, and the forward pass is part of the iteration
    b = bench.unet_bound_us(batch=8)
    fwd, train = bench.unet_flops_per_sample()
    mfma_train_us = 8 * train / (bench.BF16_PEAK_TFLOPS * 1e12) * 1e6
    mfma_fwd_us = 8 * fwd / (bench.BF16_PEAK_TFLOPS * 1e12) * 1e6
    assert b["train_us"] >= mfma_train_us and b["forward_us"] >= mfma_fwd_us
    assert b["forward_us"] < b["train_us"]
    # the level-0 activations alone: 8 x 256^2 pixels x 32 channels in BF16, read and
    # written by the two encoder convolutions at 8 TB/s
    assert b["forward_us"] > 2 * (8 * 256 * 256 * 64 * 2) / (bench.HBM_PEAK_GBS * 1e9) * 1e6
    # doubling the batch doubles every per-pixel term; Adam and the weight casts stay
    b2 = bench.unet_bound_us(batch=16)
    assert abs(b2["forward_us"] - 2 * b["forward_us"]) < 0.2
    assert 1.9 * b["train_us"] < b2["train_us"] < 2 * b["train_us"]
