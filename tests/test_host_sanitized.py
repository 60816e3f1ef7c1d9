"""The library's host C++ (samplers, primes, codec, CRT in host_math.cpp, the
work queue's workspace arena in arena.h) built on its own with the address
and undefined-behaviour sanitizers and run on the CPU.

* arena: random take / give sequences and deliberate fragmentation; the
  driver checks overlap, bounds, the used count and full coalescing.
* samplers: the host samplers' outputs against the oracle's and against the
  known answers of the generator spec (published SplitMix64 outputs).
"""
import json
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import ckks, params, prng

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "host", "host_check.cpp")
HOST_MATH = os.path.join(ROOT, "paper_2601_15401_amd", "csrc", "host_math.cpp")


@pytest.fixture(scope="module")
def host_check(tmp_path_factory):
    if not shutil.which("g++"):
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("host") / "host_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", SRC, HOST_MATH, "-o", exe]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    assert r.returncode == 0, r.stdout
    return exe


def _run(exe, mode):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([exe, mode], stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr, r.stderr[-4000:]
    return json.loads(r.stdout)


def test_arena_under_sanitizers(host_check):
    assert _run(host_check, "arena") == {"arena": "ok"}


def test_host_samplers_under_sanitizers_match_oracle(host_check):
    out = _run(host_check, "samplers")
    q = params.primes_below(30, 1 << 14, 4)
    assert [int(x) for x in out["primes30_n8192"]] == q
    assert [int(x) for x in out["psi_n8192"]] == [params.min_psi(x, 1 << 13) for x in q]
    assert [int(x) for x in out["keys"]] == [prng.stream_key(1, "SK"), prng.stream_key(7, "EVK_A", 3, 1, 5),
                                             prng.stream_key((1 << 64) - 1, "ENC_V", 2)]
    # the published SplitMix64 outputs of state 0 and the hand-worked ternary vectors
    assert [int(x) for x in out["draws0"]] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F,
                                               0xF88BB8A8724C81EC, 0x1B39896A51A8749B, 0x53CB9F0C747EA2EA,
                                               0x2C829ABE1F4532E1, 0xC584133AC916AB3C]
    assert out["ternary_key0_n4_h2"] == [0, 0, 1, 1]
    assert out["ternary_keyG_n4_h2"] == [-1, 0, -1, 0]
    assert out["ternary_sk_n64_h16"] == prng.ternary_hw(prng.stream_key(3, "SK"), 64, 16).tolist()
    B, T = prng.cdt_table(3.2)
    assert [int(x) for x in out["gauss_table"]] == T
    assert out["gauss_64"] == prng.gaussian(prng.stream_key(11, "PK_E"), 64, 3.2).tolist()
    assert [int(x) for x in out["uniform_32"]] == prng.uniform_mod(prng.stream_key(1, "PK_A", 0), q[0], 32).tolist()
    n = 32
    re = np.array([0.25 * j / n - 0.1 for j in range(n // 2)])
    im = np.array([0.5 - 0.03 * j for j in range(n // 2)])
    want = ckks.encode(re, im, n, 2.0 ** 40)
    assert np.abs(np.array(out["encode_n32"]) - want).max() <= 1
    assert out["codec_roundtrip_err"] < 1e-9
    assert out["crt_mismatches"] == 0
    assert int(out["inv_pow"][0]) == pow(12345, -1, q[0]) and int(out["inv_pow"][1]) == 1
