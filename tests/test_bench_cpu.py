"""bench.py's host logic: the one-GPU contract and the roofline object."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def _quiet(monkeypatch):
    monkeypatch.setattr(bench, "log", lambda *a: None)


def test_roofline_ranks_each_transform_pass_as_its_own_kernel(monkeypatch):
    _quiet(monkeypatch)
    # both passes of the accumulators' INTT together take longer than the key
    # products, but neither pass alone does
    prof = {"passB_kip": (4.1, 20), "intt_acc.passA": (2.0, 20), "intt_acc.passB": (2.5, 20),
            "tensor": (1.7, 20)}
    rl = bench.roofline(prof, 20, 1 << 16, 3, 24, 24, 24, 8)
    assert rl["kernel"] == "passB_kip"
    assert rl["avg_launch_us"] == 205.0


def test_whole_path_bytes_per_multiply():
    """The per-multiply algorithmic bytes of the whole multiply: k inputs, the
    keys once per batch, the output (C3: 734.5 MB alone, 220.7 MB in a batch
    of 8; C2 batch 16: 24.1 MB)."""
    assert abs(bench.mult_bytes(1 << 16, 8, 32, 8, 8, 1) / 1e6 - 734.5) < 0.1
    assert abs(bench.mult_bytes(1 << 16, 8, 32, 8, 8, 8) / 1e6 - 220.7) < 0.1
    assert abs(bench.mult_bytes(1 << 15, 4, 16, 4, 4, 16) / 1e6 - 24.1) < 0.1


def test_roofline_fraction_is_whole_path_bytes_over_the_dominant_launch(monkeypatch):
    _quiet(monkeypatch)
    N, k, level, K, alpha, jobs = 1 << 16, 8, 32, 8, 8, 8
    rl = bench.roofline({"modup_bconv_passA": (25.4, 20), "passB_kip": (20.0, 20)}, 20, N, k, level, K, alpha, jobs)
    assert rl["kernel"] == "modup_bconv_passA" and rl["bound"] == "hbm" and rl["unit"] == "GB/s"
    path = jobs * bench.mult_bytes(N, k, level, K, alpha, jobs)
    assert rl["algorithmic_bytes_per_launch"] == int(path) and rl["multiplies_per_launch"] == jobs
    assert abs(rl["achieved"] - path / 1.27e-3 / 1e9) < 0.1
    assert abs(rl["frac"] - path / 1.27e-3 / 1e9 / bench.HBM_PEAK_GBS) < 1e-4
    # the kernel's own 32-bit multiplies: per converted limb alpha 64-bit
    # multiply-adds (2 each) and one Montgomery reduction (4) per element, and
    # 8 stages of N/2 Shoup products (3 each) of pass A
    new_limbs = (k - 1) * (4 * (level + K) - level)
    mults = jobs * new_limbs * (N * (2 * alpha + 4) + N / 2 * 8 * 3)
    assert rl["int32_mult"]["per_launch"] == int(mults)
    assert abs(rl["int32_mult"]["frac"] - mults / 1.27e-3 / 1e12 / bench.ALU_PEAK_TOPS) < 1e-4
    # the instruction model stays as a diagnostic
    b, ops = bench.site_work("modup_bconv_passA", N, k, level, K, alpha, jobs)
    assert rl["valu_model"]["kernel_bytes_per_launch"] == b and rl["valu_model"]["valu_ops_per_launch"] == ops


def test_transform_pass_work_is_half_the_transform(monkeypatch):
    _quiet(monkeypatch)
    N, k, level, K, alpha, jobs = 1 << 16, 8, 32, 8, 8, 8
    b, ops = bench.site_work("intt_d", N, k, level, K, alpha, jobs)
    n = jobs * (k - 1) * level
    assert b == 2 * 4.0 * N * n
    assert ops == n * (N / 2) * 16 * 9.0  # 16 stages of N/2 butterflies
    rl = bench.roofline({"intt_d.passA": (5.0, 20)}, 20, N, k, level, K, alpha, jobs)
    assert abs(rl["valu_model"]["frac"] - (ops / 2) / 250e-6 / 1e12 / bench.ALU_PEAK_TOPS) < 1e-3
    assert rl["int32_mult"]["per_launch"] == int(n * (N / 2) * 3 * 16 / 2)


def test_source_hash_ignores_comments_and_whitespace():
    a = 'int f(int x) {  // doubles\n  return 2 * x; /* no overflow\n here */ }\nconst char* s = "a // b";\n'
    b = 'int f(int x) { return 2 * x; }\nconst char* s = "a // b";'
    c = 'int f(int x) { return 3 * x; }\nconst char* s = "a // b";'
    d = 'int f(int x) { return 2 * x; }\nconst char* s = "a  b";'
    assert bench._code_tokens(a) == bench._code_tokens(b)
    assert bench._code_tokens(b) != bench._code_tokens(c)
    assert bench._code_tokens(b) != bench._code_tokens(d)  # literals are code


def test_fused_tensor_site_is_the_tensor_plus_pass_b(monkeypatch):
    _quiet(monkeypatch)
    N, k, level, K, alpha, jobs = 1 << 16, 8, 32, 8, 8, 8
    tb, tops = bench.site_work("tensor", N, k, level, K, alpha, jobs)
    fb, fops = bench.site_work("tensor_inttB", N, k, level, K, alpha, jobs)
    n = jobs * (k - 1) * level
    assert fb == tb + 4.0 * N * n  # pass B's output written, nothing read back
    assert fops == tops + n * (N / 2) * 8 * 9.0  # 8 of the 16 stages
