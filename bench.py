"""Throughput of the k-input RNS-CKKS multiply on one MI355X.

Workload (default): the eight-input multiply at N = 2^16 with 32 ciphertext
primes of 30 bits, 8 special primes of 31 bits, dnum = 4, scale 2^30, keys
for s^2..s^8, as a batch of 8 independent multiplies (tensor product,
relinearisation, combined 7-level rescale) per step.  Inputs are encryptions
of seeded synthetic messages (slots uniform in [-1, 1)^2), resident in HBM
before timing starts.

One JSON line on stdout: the metric (batched ct-mults/s), the plain
per-multiply launch rate beside it, per-step latency percentiles, the
roofline of the dominant kernel from HIP events recorded on its stream
during the timed steps, and the CPU oracle timed on one multiply.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz: one 32-bit integer VALU op per lane
# per clock.  Measured on the device (mick_rates): v_mul_lo_u32 52,
# v_mul_hi_u32 56, v_mad_u64_u32 50 lane-ops per CU per clock of the 64.
ALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
MUL_LO_MEASURED_TOPS = 31.97

WORKLOADS = {
    # name: (log_n, L, K, dnum, k, level, batch)
    "n16_k8_b8": (16, 32, 8, 4, 8, 32, 8),
    "n15_k4_b16": (15, 16, 4, 4, 4, 16, 16),
    "n13_k3": (13, 3, 1, 3, 3, 3, 1),
    # the paper's own setting (Sec. VI): one key-switching digit, K = L = 24
    "paper3": (16, 24, 24, 1, 3, 24, 8),
    "mixed512": None,  # heterogeneous batch, see run_mixed
    "serve5000": None,  # open-loop serving, see run_serve
    "trees": None,  # flat / planned tree / binary tree of two-input multiplies, see run_trees
    "tensor_methods": None,  # the three forms of the tensor product at the three workload shapes
    "bconv": None,  # the standalone basis conversion on the vector ALUs and on the int8 matrix cores
}
# parameter sets of the mixed workload: log_n -> (L, K, dnum)
MIXED_PARAMS = {13: (3, 1, 3), 14: (8, 2, 4), 15: (16, 4, 4), 16: (32, 8, 4)}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def site_work(site, N, k, level, K, alpha, jobs):
    """Algorithmic bytes and 32-bit integer ops of one launch at `site`.

    Bytes: every input element read once and every output element written once
    (4 bytes each); key material counted once per launch.  Ops: a radix-2
    butterfly mod q is counted as 9 VALU operations (Shoup product 4, lazy
    reduction 2, add 1, subtract-and-offset 2); a key product accumulated into
    an exact 96-bit sum as 2 (multiply-add, carry) and each such sum's final
    reduction mod q as 30."""
    E = level + K
    B = -(-level // alpha)
    mu = k - 1
    limb = 4.0 * N
    new_limbs = (k - 1) * (B * E - level)  # ModUp outputs that are transformed
    bfly = 9.0
    log_n = int(N).bit_length() - 1
    stages_a = 8 if log_n >= 15 else 7  # the default split of log N into passes A and B
    stages_b = log_n - stages_a
    if site == "modup_bconv_passA":
        # reads the d_t limbs once, writes pass-A outputs of the new limbs
        n_in, n_out = jobs * (k - 1) * level, jobs * new_limbs
        return limb * (n_in + n_out), jobs * new_limbs * (N * (2 * alpha + 12.0) + (N / 2) * stages_a * bfly)
    if site == "passB_kip":
        # reads pass-A outputs, the digits' own d_t, d_0 and d_1, the keys once per
        # batch; writes the two accumulators after the first pass of their INTT
        x = jobs * (new_limbs + (k - 1) * level)
        keys = (k - 1) * B * 2 * E
        return limb * (x + keys + jobs * 2 * level + jobs * 2 * E), \
            jobs * ((new_limbs + 2 * E) * (N / 2) * stages_b * bfly + (k - 1) * B * E * N * 2 * 2.0
                    + 2 * E * N * 30.0)
    if site.startswith("intt_d"):
        n = jobs * (k - 1) * level
        return 2 * limb * n, n * (N / 2) * log_n * bfly
    if site.startswith("intt_acc"):
        n = jobs * 2 * E
        return 2 * limb * n, n * (N / 2) * log_n * bfly
    if site.startswith("ntt_out"):
        n = jobs * 2 * (level - mu)
        return 2 * limb * n, n * (N / 2) * log_n * bfly
    if site == "tensor":
        n_in, n_out = jobs * k * 2 * level, jobs * (k + 1) * level
        return limb * (n_in + n_out), jobs * level * N * (k * (k + 1) - 2) * 7.0
    if site == "tensor_inttB":
        # the tensor product, then pass B of d_2..d_k's INTT on the tile in
        # LDS: the pass's output is written, nothing is read back
        tb, tops = site_work("tensor", N, k, level, K, alpha, jobs)
        n = jobs * (k - 1) * level
        return tb + limb * n, tops + n * (N / 2) * stages_b * bfly
    if site == "moddown_rescale":
        return limb * jobs * (2 * E + 2 * (level - mu)), jobs * 2 * (level - mu) * N * (2 * (K + mu) + 30.0)
    return 0.0, 0.0


def site_mults(site, N, k, level, K, alpha, jobs):
    """32-bit integer multiplies of one launch at `site`, counted as the
    whole-path work table does: a Shoup product by a constant is 3, a
    Montgomery product or reduction 4, a 64-bit multiply-accumulate 2."""
    E = level + K
    B = -(-level // alpha)
    mu = k - 1
    new_limbs = (k - 1) * (B * E - level)
    log_n = int(N).bit_length() - 1
    stages_a = 8 if log_n >= 15 else 7
    stages_b = log_n - stages_a
    bf = N / 2 * 3.0  # Shoup products of one stage of one limb
    if site == "modup_bconv_passA":
        return jobs * new_limbs * (N * (2.0 * alpha + 4.0) + bf * stages_a)
    if site == "passB_kip":
        return jobs * ((new_limbs + 2 * E) * bf * stages_b + (k - 1) * B * E * N * 2 * 2.0 + 2 * E * N * 10.0)
    if site.startswith("intt_d"):
        return jobs * (k - 1) * level * bf * log_n
    if site.startswith("intt_acc"):
        return jobs * 2 * E * bf * log_n
    if site.startswith("ntt_out"):
        return jobs * 2 * (level - mu) * bf * log_n
    if site == "tensor":
        return jobs * level * N * (k * (k + 1) - 2) * 4.0
    if site == "tensor_inttB":
        return site_mults("tensor", N, k, level, K, alpha, jobs) + jobs * (k - 1) * level * bf * stages_b
    if site == "moddown_rescale":
        return jobs * 2 * (level - mu) * N * (2.0 * (K + mu) + 8.0)
    return 0.0


def roofline(prof, steps, N, k, level, K, alpha, jobs):
    """Dominant kernel by total time (each pass of a two-pass transform is its
    own kernel).  The fraction is the HBM roofline of the whole multiply:
    the algorithmic bytes of the multiplies one launch serves (k inputs read,
    the keys read once per batch, the output written; intermediates count
    zero) over the dominant launch's duration, against 8 TB/s.  Beside it:
    the kernel's own 32-bit multiplies (Shoup 3, Montgomery 4, 64-bit
    multiply-add 2) against the int32 VALU peak, and, as a diagnostic, the
    instruction model of site_work (bytes the kernel itself moves, VALU ops)."""
    table = []
    for site, (ms, cnt) in prof.items():
        base = site.split(".")[0]
        b, ops = site_work(base, N, k, level, K, alpha, jobs)
        if "." in site:  # one pass of a transform
            ops = ops / 2
        avg_s = ms / cnt / 1e3
        table.append((ms, site, cnt, avg_s, b / avg_s / 1e9 if b else 0.0, ops / avg_s / 1e12 if ops else 0.0,
                      b, ops))
    table.sort(reverse=True)
    for ms, site, cnt, avg_s, gbs, tops, b, ops in table:
        log("  %-18s %8.3f ms/step %4d launches  avg %8.1f us  %7.0f GB/s (%4.1f%% HBM)  %6.2f Tops (%4.1f%% ALU)"
            % (site, ms / steps, cnt, avg_s * 1e6, gbs, 100 * gbs / HBM_PEAK_GBS, tops, 100 * tops / ALU_PEAK_TOPS))
    ms, site, cnt, avg_s, gbs, tops, b, ops = table[0]
    path_bytes = jobs * mult_bytes(N, k, level, K, alpha, jobs)
    path_gbs = path_bytes / avg_s / 1e9
    mults = site_mults(site.split(".")[0], N, k, level, K, alpha, jobs) / (2 if "." in site else 1)
    mul_t = mults / avg_s / 1e12
    return {"kernel": site, "bound": "hbm", "achieved": round(path_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(path_gbs / HBM_PEAK_GBS, 4), "traffic": None, "avg_launch_us": round(avg_s * 1e6, 2),
            "algorithmic_bytes_per_launch": int(path_bytes), "multiplies_per_launch": jobs,
            "int32_mult": {"per_launch": int(mults), "achieved": round(mul_t, 3), "peak": round(ALU_PEAK_TOPS, 2),
                           "unit": "Tmul/s", "frac": round(mul_t / ALU_PEAK_TOPS, 4),
                           "frac_of_measured_v_mul_lo_rate": round(mul_t / MUL_LO_MEASURED_TOPS, 4)},
            "valu_model": {"kernel_bytes_per_launch": b, "kernel_bytes_frac": round(gbs / HBM_PEAK_GBS, 4),
                           "valu_ops_per_launch": ops, "achieved_tops": round(tops, 3),
                           "frac": round(tops / ALU_PEAK_TOPS, 4)}}


def _code_tokens(text):
    """C/C++ source without comments and with whitespace collapsed (string
    and character literals are kept as they are)."""
    import re
    pat = re.compile(r'//[^\n]*|/\*.*?\*/|"(?:\\.|[^"\\])*"|\'(?:\\.|[^\'\\])*\'', re.S)
    code = pat.sub(lambda m: " " if m.group(0).startswith("/") else m.group(0), text)
    return " ".join(code.split())


def kernel_source_hash():
    """First 16 hex digits of a SHA-256 over the kernel sources (csrc/*.hip,
    csrc/*.h in name order, comments and whitespace ignored), recorded with
    the counter summaries."""
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2601_15401_amd", "csrc", "*.hip")) +
                    glob.glob(os.path.join(ROOT, "paper_2601_15401_amd", "csrc", "*.h"))):
        h.update(os.path.basename(f).encode())
        h.update(_code_tokens(open(f, encoding="utf-8").read()).encode())
    return h.hexdigest()[:16]


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None when the kernel sources have changed since the counters
    were taken (the summary records their hash)."""
    path = os.path.join(ROOT, "profiles", "hbm_counters_n16_k8_b8.txt")
    if not os.path.exists(path):
        return None
    sha = kernel_source_hash()
    for line in open(path):
        if line.startswith("TRAFFIC "):
            f = dict(kv.split("=", 1) for kv in line.split()[1:])
            if f.get("kernel") == kernel and f.get("src_sha256_16") == sha:
                return int(f["bytes"])
    return None


def mult_bytes(N, k, level, K, alpha, jobs):
    """Algorithmic HBM bytes of one multiply in a batch of `jobs` sharing keys:
    k inputs read, the evaluation keys read once per batch, output written."""
    B = -(-level // alpha)
    E = level + K
    inputs = k * 2 * level * N * 4
    keys = (k - 1) * B * 2 * E * N * 4 / jobs
    out = 2 * (level - k + 1) * N * 4
    return inputs + keys + out


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


_CPU_CASE = {}


def _oracle_one(seed):
    """One oracle multiply on seeded uniform inputs (pool worker; the
    parameters and keys come from the parent by fork)."""
    from oracle import mult
    prm, ks, k, level = _CPU_CASE["case"]
    rng = np.random.default_rng(seed)
    cts = [np.stack([np.stack([rng.integers(0, q, prm.N, dtype=np.int64).astype(np.uint64) for q in prm.q[:level]])
                     for _ in range(2)]) for _ in range(k)]
    t0 = time.perf_counter()
    mult.mul_relin_rescale(prm, ks, cts, level)
    return time.perf_counter() - t0


def cpu_baseline(log_n, L, K, dnum, k, level, pool=True):
    """The oracle (exact numpy / Python-int path) timed on the host: one
    multiply on one core, then one multiply per worker of a process pool
    over the host's cores (at most 16) running concurrently."""
    import multiprocessing as mp
    from oracle import keys as okeys, params as oparams
    prm = oparams.make_params(log_n, L, K, dnum)
    log("cpu baseline: oracle keygen ...")
    ks = okeys.keygen(prm, 99, k)
    _CPU_CASE["case"] = (prm, ks, k, level)
    log("cpu baseline: timing one multiply on one core ...")
    dt = _oracle_one(99)
    log("cpu baseline: %.1f s per multiply" % dt)
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    workers = max(1, min(avail, 16))
    model = cpu_model()
    single = {"value": round(1.0 / dt, 5), "cores": 1, "seconds_per_mult": round(dt, 2)}
    if not pool or workers < 2:
        return {"value": single["value"], "unit": "ct-mults/s", "cores": 1, "kind": "oracle",
                "sample": "one %d-input multiply at N=2^%d, level %d (tensor, relin, %d-level rescale), %.1f s on "
                          "one core of %s" % (k, log_n, level, k - 1, dt, model), "cpu_model": model}
    log("cpu baseline: %d multiplies on a pool of %d processes ..." % (workers, workers))
    ctx = mp.get_context("fork")
    with ctx.Pool(workers) as p:
        t0 = time.perf_counter()
        per = p.map(_oracle_one, [1000 + i for i in range(workers)], chunksize=1)
        wall = time.perf_counter() - t0
    log("cpu baseline: pool %.1f s wall for %d multiplies" % (wall, workers))
    return {"value": round(workers / wall, 5), "unit": "ct-mults/s", "cores": workers, "kind": "oracle",
            "sample": "%d concurrent %d-input multiplies at N=2^%d, level %d (tensor, relin, %d-level rescale), "
                      "one per process, %.1f s wall (%.1f s mean per multiply) on %s"
                      % (workers, k, log_n, level, k - 1, wall, float(np.mean(per)), model),
            "cpu_model": model, "single_core": single}


def mixed_jobs(n_jobs, seed):
    """(log_n, k, level) per job: N uniform over the four sets, k uniform in
    [2, min(12, L)], level uniform in [k, L]."""
    rng = np.random.default_rng(seed)
    jobs = []
    for _ in range(n_jobs):
        ln = int(rng.choice(sorted(MIXED_PARAMS)))
        L = MIXED_PARAMS[ln][0]
        k = int(rng.integers(2, min(12, L) + 1))
        level = int(rng.integers(k, L + 1))
        jobs.append((ln, k, level))
    return jobs


def job_bytes(N, k, level, K, alpha):
    """Algorithmic HBM bytes of one multiply with its own key reads."""
    return mult_bytes(N, k, level, K, alpha, 1)


def run_mixed(args, torch, mick):
    """The mixed workload on its own: one JSON line."""
    leg = mixed_leg(args, torch, mick, args.steps, args.warmup, args.plain_steps, with_queue=True,
                    with_plain=not args.no_plain)
    rec = {
        "metric": "k-input ct-mults/s at N=2^16 (batched vs plain), % HBM peak; p50/p99 latency",
        "value": leg["value"], "unit": "ct-mults/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": leg["ms_per_512"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": "512 multiplies, N uniform over 2^13..2^16, k uniform 2..min(12,L), level "
                               "uniform k..L, one graph of four job-table plans", "batch": 512,
                   "parallelism": "none"},
        **{k: v for k, v in leg.items() if k not in ("value", "ms_per_512")},
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(rec), flush=True)


def mixed_leg(args, torch, mick, steps, warmup, plain_steps, with_queue=False, with_plain=True):
    """512 multiplies of mixed ring degree, k and level: the batched form runs
    one plan per ring degree (one launch per stage over a device job table),
    captured into one graph; the plain form launches each multiply alone."""
    n_jobs = 512
    spec = mixed_jobs(n_jobs, 4)
    prms, keys, pools, specs, plans = {}, {}, {}, {}, {}
    gen = torch.Generator(device="cuda")
    gen.manual_seed(4)
    for ln, (L, K, dnum) in MIXED_PARAMS.items():
        log("params N=2^%d L=%d K=%d dnum=%d; keygen k_max=%d ..." % (ln, L, K, dnum, min(12, L)))
        prms[ln] = mick.Params(ln, L, K, dnum)
        mick.autotune(prms[ln])
        keys[ln] = mick.Keys(prms[ln], 40 + ln, min(12, L))
    schedules = {str(ln): mick.schedule(prms[ln]) for ln in prms}
    log("transform schedules (first-pass log size): %s" % schedules)
    log("inputs (uniform residues per limb) ...")
    for ln, k, level in spec:
        if (ln, level) not in pools:
            q = torch.tensor(prms[ln].q[:level], dtype=torch.int64, device="cuda").view(1, 1, level, 1)
            r = torch.randint(0, 1 << 62, (12, 2, level, 1 << ln), generator=gen, device="cuda", dtype=torch.int64)
            pools[(ln, level)] = (r % q).to(torch.int32)
        specs.setdefault(ln, []).append(([pools[(ln, level)][u] for u in range(k)], level, None))
    for ln in MIXED_PARAMS:
        if ln in specs:
            plans[ln] = mick.Plan(prms[ln], keys[ln], specs[ln])
    torch.cuda.synchronize()

    def step():
        for p in plans.values():
            p.run()

    log("warmup ...")
    mick.profile_enable(True)
    for _ in range(max(1, warmup)):
        step()
    torch.cuda.synchronize()
    mick.profile_collect()
    mick.profile_enable(False)
    log("capturing one graph of %d plans ..." % len(plans))
    g = torch.cuda.CUDAGraph()
    cs = torch.cuda.Stream()
    with torch.cuda.stream(cs):
        with torch.cuda.graph(g, stream=cs):
            step()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    for _ in range(3):  # untimed replays (the first runs slower)
        g.replay()
    torch.cuda.synchronize()
    # replays back to back between one pair of events; the per-replay
    # latencies from a second pass with an event after every replay
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for i in range(steps):
        g.replay()
    e1.record(stream)
    torch.cuda.synchronize()
    mean_ms = e0.elapsed_time(e1) / steps
    value = n_jobs / (mean_ms / 1e3)
    log("batched (graph): %.3f ms per 512 multiplies, %.1f ct-mults/s" % (mean_ms, value))
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    ev[0].record(stream)
    for i in range(steps):
        g.replay()
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    step_ms = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(steps)])
    # eager steps with the event profiler for the per-site breakdown
    mick.profile_enable(True)
    for _ in range(2):
        step()
    torch.cuda.synchronize()
    prof = mick.profile_collect()
    mick.profile_enable(False)
    for site, (ms, cnt) in sorted(prof.items(), key=lambda x: -x[1][0]):
        log("  %-20s %8.3f ms/step %5d launches" % (site, ms / 2, cnt // 2))

    plain = None
    if with_plain:
        wss = {ln: mick.workspace(prms[ln], mick.OP_MUL_RELIN_RESCALE, min(12, MIXED_PARAMS[ln][0]),
                                  MIXED_PARAMS[ln][0]) for ln in prms}
        outs = {ln: [torch.empty(2, lv - len(c) + 1, 1 << ln, dtype=torch.int32, device="cuda")
                     for c, lv, _ in specs[ln]] for ln in specs}

        def plain_step():
            for ln in specs:
                for (c, lv, _), o in zip(specs[ln], outs[ln]):
                    mick.mul_relin_rescale(prms[ln], keys[ln], c, lv, out=o, ws=wss[ln])

        plain_step()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(plain_steps):
            plain_step()
        e1.record(stream)
        torch.cuda.synchronize()
        pms = e0.elapsed_time(e1) / plain_steps
        plain = {"value": round(n_jobs / (pms / 1e3), 2), "unit": "ct-mults/s", "ms_per_512": round(pms, 3)}
        log("plain: %.3f ms per 512 multiplies, %.1f ct-mults/s" % (pms, n_jobs / (pms / 1e3)))
        for ln in specs:  # the two forms agree
            for o, b in zip(outs[ln], plans[ln].outs):
                assert torch.equal(o, b)
    queue = None
    if with_queue:
        # the same 512 jobs through the native work queue (host admission, one
        # plan per ring degree per run, event completion), wall clock incl. host
        order = sorted(prms)
        qsets = [(prms[ln], keys[ln]) for ln in order]
        qjobs, qi = [], 0
        for ln in order:
            for c, lv, _ in specs.get(ln, []):
                qjobs.append((qi, order.index(ln), c, lv,
                              torch.empty(2, lv - len(c) + 1, 1 << ln, dtype=torch.int32, device="cuda")))
                qi += 1
        qu = mick.Queue(qsets, capacity=1 << 36)
        qu.push(qjobs)
        qu.drain()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            qu.push(qjobs)
            qu.drain()
        torch.cuda.synchronize()
        q_ms = (time.perf_counter() - t0) * 1e3 / steps
        log("queue: %.3f ms per 512 multiplies (wall), %.1f ct-mults/s" % (q_ms, n_jobs / (q_ms / 1e3)))
        for ln in order:  # the queue's outputs equal the graph's
            outs_q = [j[4] for j in qjobs if j[1] == order.index(ln)]
            for o, b in zip(outs_q, plans[ln].outs):
                assert torch.equal(o, b)
        qu.close()
        queue = {"value": round(n_jobs / (q_ms / 1e3), 2), "unit": "ct-mults/s", "ms_per_512_wall": round(q_ms, 3)}
    total_bytes = sum(job_bytes(1 << ln, k, lv, MIXED_PARAMS[ln][1], prms[ln].alpha) for ln, k, lv in spec)
    leg = {
        "value": round(value, 2), "unit": "ct-mults/s", "ms_per_512": round(mean_ms, 4),
        "steps": steps, "plain": plain,
        "batched_over_plain": round(value / plain["value"], 3) if plain else None,
        "schedules": schedules,
        "latency_ms": {"p50": round(float(np.percentile(step_ms, 50)), 4),
                       "p99": round(float(np.percentile(step_ms, 99)), 4), "of": "one graph replay of 512 multiplies"},
        "hbm_frac_whole_path": round(total_bytes / (mean_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 5),
        "algorithmic_bytes_per_mult": int(total_bytes / n_jobs),
    }
    if queue:
        leg["queue"] = queue
    del plans, g
    import gc
    gc.collect()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return leg


def run_serve(args, torch, mick):
    """The serving workload on its own: one JSON line."""
    leg = serve_leg(args, torch, mick, 5000, (0.5, 0.8, 0.95))
    top = leg["rates"][-1]
    rec = {
        "metric": "k-input ct-mults/s at N=2^16 (batched vs plain), % HBM peak; p50/p99 latency",
        "value": top["ct_mults_per_s"], "unit": "ct-mults/s", "n_gpus": 1, "steps": 5000, "warmup": 64,
        "ms_per_step": round(1e3 / top["ct_mults_per_s"], 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": "serving: 5000 requests, open-loop Poisson at 0.95 x measured saturation, mixed N "
                               "2^13..2^16 with 10%% heavy (N=2^16, k=12), HBM budget %d GB" % leg["hbm"]["budget_gb"],
                   "batch": "continuous", "max_batch": args.serve_max_batch, "streams": args.serve_streams,
                   "parallelism": "none"},
        **{k: v for k, v in leg.items() if k != "hbm_budget"},
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(rec), flush=True)


def serve_leg(args, torch, mick, n_req, loads):
    """Open-loop serving of n_req requests (the mixed-workload mixture plus 10%
    heavy N = 2^16, k = 12 requests) through the continuous-batching server:
    first all requests at once (saturation throughput), then Poisson
    arrivals at the given fractions of that rate.  Latency is completion (a
    HIP event after the request's plan) minus scheduled arrival."""
    from paper_2601_15401_amd import serve
    budget = 200 * 10 ** 9
    mix = serve.request_mix(n_req, 5, MIXED_PARAMS)
    import gc
    gc.collect()  # earlier legs' objects release their device memory first
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    free0, total = torch.cuda.mem_get_info()
    prms, keys, pools = {}, {}, {}
    for ln, (L, K, dnum) in MIXED_PARAMS.items():
        log("params N=2^%d L=%d K=%d dnum=%d; keygen k_max=%d ..." % (ln, L, K, dnum, min(12, L)))
        prms[ln] = mick.Params(ln, L, K, dnum)
        mick.autotune(prms[ln])
        keys[ln] = mick.Keys(prms[ln], 50 + ln, min(12, L))
    log("input state: 12 ciphertexts per (N, level) in use ...")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(5)
    for ln, k, level in mix:
        if (ln, level) not in pools:
            q = torch.tensor(prms[ln].q[:level], dtype=torch.int64, device="cuda").view(1, 1, level, 1)
            r = torch.randint(0, 1 << 62, (12, 2, level, 1 << ln), generator=gen, device="cuda", dtype=torch.int64)
            pools[(ln, level)] = (r % q).to(torch.int32)
            del r
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    resident = free0 - torch.cuda.mem_get_info()[0]
    log("resident keys + input state: %.2f GB" % (resident / 1e9))

    def requests(arrivals):
        out = []
        for i, ((ln, k, level), t) in enumerate(zip(mix, arrivals)):
            out.append(serve.Request(i, ln, k, level, t, inputs=[pools[(ln, level)][u] for u in range(k)]))
        return out

    check = set(range(0, n_req, 97 if n_req > 2000 else 29))
    ex = serve.GpuExecutor(mick, torch, prms, keys, n_streams=args.serve_streams, keep=lambda r: r.rid in check)
    srv = serve.Server(ex, budget, resident=resident, max_batch=args.serve_max_batch)
    log("warmup ...")
    ex.start()
    srv.run(requests([0.0] * n_req)[:64])
    torch.cuda.synchronize()
    torch.cuda.reset_peak_memory_stats()
    reserved0 = torch.cuda.memory_reserved()
    log("saturation: %d requests at t = 0 ..." % n_req)
    ex.start()
    sat = srv.run(requests([0.0] * n_req))
    sat_rate = sat.summary()["ct_mults_per_s"]
    log("  %s host launch %.3f s" % (sat.summary(), ex.host_launch_s))
    results = []
    for frac, seed in zip(loads, (50, 51, 52, 53, 54)):
        rate = frac * sat_rate
        log("open loop at %.2f x saturation = %.0f requests/s ..." % (frac, rate))
        ex.start()
        st = srv.run(requests(serve.poisson_arrivals(n_req, rate, seed)))
        summ = st.summary()
        summ["host_launch_s"] = round(ex.host_launch_s, 3)
        heavy = [r.done - r.arrival for r in st.completed if r.k == 12 and r.log_n == 16]
        light = [r.done - r.arrival for r in st.completed if r.log_n < 16]
        summ.update({"offered_per_s": round(rate, 1), "load": frac,
                     "p99_heavy_ms": round(float(np.percentile(heavy, 99)) * 1e3, 3) if heavy else None,
                     "p99_light_ms": round(float(np.percentile(light, 99)) * 1e3, 3) if light else None})
        log("  %s" % summ)
        results.append(summ)
    torch.cuda.synchronize()
    peak_hbm = resident + torch.cuda.max_memory_reserved() - reserved0
    # each sampled request's served output equals the same multiply launched alone
    kept = [r for r in st.completed if r.rid in check]
    for r in kept:
        o = mick.mul_relin_rescale(prms[r.log_n], keys[r.log_n], r.inputs, r.level)
        assert torch.equal(o, r.output), "request %d differs from its plain multiply" % r.rid
    log("alone == in the mix for %d sampled requests" % len(kept))
    # plain: every request of a 500-request sample launched alone, back to back
    sample = requests([0.0] * n_req)[:min(500, n_req)]
    wss = {ln: mick.workspace(prms[ln], mick.OP_MUL_RELIN_RESCALE, min(12, MIXED_PARAMS[ln][0]),
                              MIXED_PARAMS[ln][0]) for ln in prms}
    outs = [torch.empty(2, r.level - r.k + 1, 1 << r.log_n, dtype=torch.int32, device="cuda") for r in sample]
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for rep in range(2):
        e0.record(stream)
        for r, o in zip(sample, outs):
            mick.mul_relin_rescale(prms[r.log_n], keys[r.log_n], r.inputs, r.level, out=o, ws=wss[r.log_n])
        e1.record(stream)
        torch.cuda.synchronize()
    plain_rate = len(sample) / (e0.elapsed_time(e1) / 1e3)
    log("plain: %.1f ct-mults/s over the first %d requests" % (plain_rate, len(sample)))
    top = results[-1]
    leg = {
        "requests": n_req,
        "saturation_per_s": sat_rate,
        "rates": results,
        "latency_ms": {"p50": top["p50_ms"], "p99": top["p99_ms"],
                       "of": "one request, arrival to completion, at %.2f x saturation" % loads[-1]},
        "plain": {"value": round(plain_rate, 2), "unit": "ct-mults/s",
                  "sample": "first %d requests, each alone" % len(sample)},
        "served_over_plain": round(top["ct_mults_per_s"] / plain_rate, 3),
        "saturation_over_plain": round(sat_rate / plain_rate, 3),
        "alone_equals_mix_checked": len(kept),
        "hbm": {"budget_gb": budget / 1e9, "resident_gb": round(resident / 1e9, 3),
                "peak_gb": round(peak_hbm / 1e9, 3), "device_gb": round(total / 1e9, 1)},
    }
    del pools, ex, srv
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return leg


def run_tensor_methods(args, torch, mick):
    """The fused multiply with each tensor-product method (chain of linear
    factors, balanced product tree, tree with fast-filtering nodes) at the
    three workload shapes: the fused tensor kernel's average duration (HIP
    events around it) and the whole batched step, medians over three
    interleaved rounds; every method's outputs are checked equal."""
    names = {0: "chain", 1: "tree", 2: "tree+fast filtering"}
    table = []
    for wl in ("n13_k3", "n15_k4_b16", "n16_k8_b8"):
        log_n, L, K, dnum, k, level, jobs = WORKLOADS[wl]
        prm = mick.Params(log_n, L, K, dnum)
        keys = mick.Keys(prm, 7, k)
        gen = torch.Generator(device="cuda")
        gen.manual_seed(7)
        q = torch.tensor(prm.q[:level], dtype=torch.int64, device="cuda").view(1, 1, 1, level, 1)
        cts = (torch.randint(0, 1 << 62, (jobs, k, 2, level, prm.N), generator=gen, device="cuda",
                             dtype=torch.int64) % q).to(torch.int32)
        ws = mick.batch_workspace(prm, jobs, k, level)
        out = torch.empty(jobs, 2, level - k + 1, prm.N, dtype=torch.int32, device="cuda")
        ref = None
        stream = torch.cuda.current_stream()
        step, kern = {m: [] for m in names}, {m: [] for m in names}
        for rnd in range(3):
            for m in names:
                mick.set_tensor_method(prm, m)
                for _ in range(max(1, args.warmup)):
                    mick.mul_relin_rescale_batch(prm, keys, cts, level, out=out, ws=ws)
                torch.cuda.synchronize()
                if ref is None:
                    ref = out.clone()
                assert torch.equal(out, ref), "tensor method %d differs" % m
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                for _ in range(args.steps):
                    mick.mul_relin_rescale_batch(prm, keys, cts, level, out=out, ws=ws)
                e1.record(stream)
                torch.cuda.synchronize()
                step[m].append(e0.elapsed_time(e1) / args.steps)
                mick.profile_select(["tensor_inttB"])
                mick.profile_enable(True)
                for _ in range(args.steps):
                    mick.mul_relin_rescale_batch(prm, keys, cts, level, out=out, ws=ws)
                torch.cuda.synchronize()
                t_ms, cnt = mick.profile_collect()["tensor_inttB"]
                mick.profile_enable(False)
                mick.profile_select(None)
                kern[m].append(t_ms / cnt * 1e3)
        for m in names:
            st_ms, k_us = float(np.median(step[m])), float(np.median(kern[m]))
            row = {"workload": wl, "method": names[m], "tensor_kernel_us": round(k_us, 2),
                   "step_ms": round(st_ms, 4), "ct_mults_per_s": round(jobs / (st_ms / 1e3), 1)}
            log("  %-11s %-20s tensor kernel %8.2f us   step %8.4f ms   %9.1f ct-mults/s"
                % (wl, names[m], k_us, st_ms, row["ct_mults_per_s"]))
            table.append(row)
        mick.set_tensor_method(prm, 0)
        del cts, ws, out, ref
        torch.cuda.empty_cache()
    print(json.dumps({"tensor_methods": table}), flush=True)


def run_bconv(args, torch, mick):
    """The standalone fast basis conversion, 64-bit multiply-adds on the vector
    ALUs against the int8 matrix cores, on the ModUp volume of one digit of a
    batched step: (k - 1) x batch polynomials of the eight-input and
    four-input workloads.  Medians over three interleaved rounds of HIP
    events; both forms' outputs are checked equal."""
    rows = []
    for wl, digit in (("n16_k8_b8", 0), ("n16_k8_b8", 3), ("n15_k4_b16", 1)):
        log_n, L, K, dnum, k, level, jobs = WORKLOADS[wl]
        prm = mick.Params(log_n, L, K, dnum)
        na = min(prm.alpha, level - digit * prm.alpha)
        polys = (k - 1) * jobs
        gen = torch.Generator(device="cuda")
        gen.manual_seed(11)
        qs = torch.tensor(prm.q[digit * prm.alpha:digit * prm.alpha + na], dtype=torch.int64,
                          device="cuda").view(1, na, 1)
        src = (torch.randint(0, 1 << 62, (polys, na, prm.N), generator=gen, device="cuda", dtype=torch.int64)
               % qs).to(torch.int32)
        outs = [mick.bconv(prm, src, level, digit, m) for m in (0, 1)]
        torch.cuda.synchronize()
        assert torch.equal(outs[0], outs[1]), "the two forms differ"
        T = outs[0].shape[1]
        stream = torch.cuda.current_stream()
        times = {0: [], 1: []}
        for _ in range(3):
            for m in (0, 1):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                for _ in range(args.steps):
                    mick.bconv(prm, src, level, digit, m, out=outs[m])
                e1.record(stream)
                torch.cuda.synchronize()
                times[m].append(e0.elapsed_time(e1) / args.steps * 1e3)
        for m, name in ((0, "valu"), (1, "mfma_i8")):
            us = float(np.median(times[m]))
            elems = polys * T * prm.N
            rows.append({"workload": wl, "digit": digit, "digit_primes": na, "targets": T, "polys": polys,
                         "method": name, "us_per_launch": round(us, 2),
                         "ns_per_1k_outputs": round(us * 1e3 / (elems / 1e3), 3),
                         "hbm_gbs": round((polys * (na + T) * prm.N * 4) / (us * 1e-6) / 1e9, 1)})
            log("  %-11s digit %d (%d primes -> %d targets, %d polys)  %-8s %9.2f us   %7.1f GB/s"
                % (wl, digit, na, T, polys, name, us, rows[-1]["hbm_gbs"]))
        del src, outs
        torch.cuda.empty_cache()
    print(json.dumps({"bconv": rows}), flush=True)


def relin_transforms(k, level, mu, K, alpha):
    """(I)NTT limb transforms of one relinearise-and-rescale of a degree-k
    product at `level` with mu rescales: INTT of d_2..d_k, NTT of the ModUp
    outputs, INTT of the accumulators, NTT of the output."""
    B = -(-level // alpha)
    return (k - 1) * B * (level + K) + 2 * K + 4 * level - 2 * mu


def run_trees(args, torch, mick):
    """n = 3..12 inputs at N = 2^16 (32 + 8 primes, dnum 4): the flat multiply
    (depth n - 1), the planned tree of Sec. V-C (depth ceil(log2 n)) and a
    binary tree of two-input multiplies each with its own relinearisation and
    rescale (the paper's baseline, same depth).  Per method: time per
    multiply (single launches, HIP events), output level, limb transforms,
    key bytes read, and the largest slot error of the decoded product."""
    log_n, L, K, dnum = 16, 32, 8, 4
    prm = mick.Params(log_n, L, K, dnum)
    keys = mick.Keys(prm, 21, 12)
    N, alpha = prm.N, prm.alpha
    scale = 2.0 ** 30
    rng = np.random.default_rng(21)
    cts, zs = [], []
    for u in range(12):
        re, im = rng.uniform(-1, 1, N // 2), rng.uniform(-1, 1, N // 2)
        zs.append(re + 1j * im)
        cts.append(mick.encrypt(prm, keys, mick.encode(prm, re, im, scale), L, 21, u))
    stream = torch.cuda.current_stream()

    def timed(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            out = fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return out, e0.elapsed_time(e1) / reps

    def error(out, level, dropped_levels, n):
        sc = scale ** n
        for j in dropped_levels:
            sc /= prm.q[j]
        re, im = mick.decode(prm, mick.decrypt(prm, keys, out, level), sc)
        want = np.prod(np.stack(zs[:n]), axis=0)
        return float(np.abs(re + 1j * im - want).max())

    def key_bytes(k, level):
        return (k - 1) * (-(-level // alpha)) * 2 * (level + K) * N * 4

    def binary(tree, inputs, end):
        """Evaluates the binary tree with two-input multiplies; returns
        (ciphertext at level `end`, transforms, key bytes, dropped levels)."""
        if isinstance(tree, int):
            if tree == 1:
                c = inputs.pop(0)
                return c[:, :end].contiguous() if c.shape[1] != end else c, 0, 0, []
            a, b = inputs.pop(0), inputs.pop(0)
            lv = end + 1
            a, b = a[:, :lv].contiguous(), b[:, :lv].contiguous()
            return (mick.mul_relin_rescale(prm, keys, [a, b], lv), relin_transforms(2, lv, 1, K, alpha),
                    key_bytes(2, lv), [lv - 1])
        lv = end + 1
        parts = [binary(c, inputs, lv) for c in tree]
        out = mick.mul_relin_rescale(prm, keys, [p[0] for p in parts], lv)
        return (out, sum(p[1] for p in parts) + relin_transforms(2, lv, 1, K, alpha),
                sum(p[2] for p in parts) + key_bytes(2, lv), sum((p[3] for p in parts), []) + [lv - 1])

    def binary_plan(n):
        if n <= 2:
            return n
        p = 1 << (math.ceil(math.log2(n)) - 1)
        return (binary_plan(p), binary_plan(n - p))

    rows = []
    for n in range(3, 13):
        row = {"n": n}
        # flat
        out, ms = timed(lambda: mick.mul_relin_rescale(prm, keys, cts[:n], L))
        lv = L - n + 1
        row["flat"] = {"ms": round(ms, 3), "out_level": lv, "transforms": relin_transforms(n, L, n - 1, K, alpha),
                       "key_MB": round(key_bytes(n, L) / 1e6, 1),
                       "max_err": error(out, lv, list(range(lv, L)), n)}
        # planned tree
        tree = mick.tree_plan(n)
        ws = mick.tree_workspace(prm, tree, L)
        _, depth, units = mick.tree_shape(tree)
        lv = L - depth
        out_t = torch.empty(2, lv, N, dtype=torch.int32, device="cuda")
        out, ms = timed(lambda: mick.mul_tree(prm, keys, cts[:n], L, tree, out=out_t, ws=ws))
        resc = mick.tree_rescales(tree, L)
        root_prod, root_mu = resc[-1]
        pre = 0
        nodes = []

        def deg_walk(t):  # polynomials rescaled per node, post-order like tree_rescales
            if isinstance(t, int):
                if t > 1:
                    nodes.append(t + 1)
                return t
            d = sum(deg_walk(c) for c in t)
            nodes.append(d + 1)
            return d
        deg_walk(tree)
        for (prod, mu), npoly in zip(resc[:-1], nodes[:-1]):
            pre += npoly * prod  # Algorithm 1: mu INTT + (prod - mu) NTT per polynomial
        drops = [j for prod, mu in resc for j in range(prod - mu, prod)]
        row["tree"] = {"partition": str(tree), "ms": round(ms, 3), "out_level": lv, "rs_units": units,
                       "transforms": pre + relin_transforms(n, root_prod, root_mu, K, alpha),
                       "key_MB": round(key_bytes(n, root_prod) / 1e6, 1), "max_err": error(out, lv, drops, n)}
        del ws
        # binary tree of two-input multiplies
        bt = binary_plan(n)
        res, ms = timed(lambda: binary(bt, list(cts[:n]), L - _depth(bt)))
        out, tr, kb, dropped = res
        row["binary"] = {"partition": str(bt), "ms": round(ms, 3), "out_level": L - _depth(bt), "transforms": tr,
                         "key_MB": round(kb / 1e6, 1), "max_err": error(out, L - _depth(bt), dropped, n)}
        log("n=%2d flat %7.3f ms (level %2d, err %.1e) | tree %-22s %7.3f ms (level %2d, err %.1e) | "
            "binary %7.3f ms (err %.1e)" % (n, row["flat"]["ms"], row["flat"]["out_level"], row["flat"]["max_err"],
                                            str(tree), row["tree"]["ms"], row["tree"]["out_level"],
                                            row["tree"]["max_err"], row["binary"]["ms"], row["binary"]["max_err"]))
        rows.append(row)
    r12 = rows[-1]
    rec = {
        "metric": "k-input ct-mults/s at N=2^16 (batched vs plain), % HBM peak; p50/p99 latency",
        "value": round(1e3 / r12["tree"]["ms"], 2), "unit": "ct-mults/s", "n_gpus": 1, "steps": 5, "warmup": 1,
        "ms_per_step": r12["tree"]["ms"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32", "data": "synthetic",
        "config": {"workload": "n-input multiplies n=3..12 at N=2^16, 32+8 primes, dnum=4: flat, planned tree, "
                               "binary tree of two-input multiplies (value: planned 12-input tree, one at a time)",
                   "parallelism": "none"},
        "rows": rows, "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(rec), flush=True)


def _depth(t):
    return t - 1 if isinstance(t, int) else max(_depth(c) for c in t) + len(t) - 1


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    # after the set-up the first tens of milliseconds of steps run slower
    # (about 10% at the four-input N = 2^15 batch over its first 20 ms, 1-2%
    # at the eight-input batch); the default warmup covers them
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--workload", default="n16_k8_b8", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--plain-steps", type=int, default=3)
    ap.add_argument("--serve-streams", type=int, default=4, help="serve5000: concurrent micro-batches")
    ap.add_argument("--serve-max-batch", type=int, default=32, help="serve5000: most requests per micro-batch")
    ap.add_argument("--no-systems", action="store_true",
                    help="default workload: skip the mixed-batch and serving legs")
    ap.add_argument("--mixed-steps", type=int, default=5, help="default workload: graph replays of the mixed batch")
    ap.add_argument("--serve-requests", type=int, default=2000, help="default workload: requests of the serving leg")
    ap.add_argument("--settings", default="", metavar="A/T/M",
                    help="skip the autotuner: first-pass log A, tensor method T, ModUp targets M (e.g. 8/0/2)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="copy a MIB-sized buffer once before timing (reference kernel for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only; this build has no multi-GPU path (use --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2601_15401_amd import mick

    torch.cuda.set_device(0)
    if args.workload == "mixed512":
        run_mixed(args, torch, mick)
        return
    if args.workload == "serve5000":
        run_serve(args, torch, mick)
        return
    if args.workload == "trees":
        run_trees(args, torch, mick)
        return
    if args.workload == "tensor_methods":
        run_tensor_methods(args, torch, mick)
        return
    if args.workload == "bconv":
        run_bconv(args, torch, mick)
        return
    log_n, L, K, dnum, k, level, jobs = WORKLOADS[args.workload]
    prm = mick.Params(log_n, L, K, dnum)
    if args.settings:
        # fixed settings instead of the autotuner: profiler runs that must
        # see the same kernels from one run to the next
        a, tm, mt = (int(v) for v in args.settings.split("/"))
        log("params N=2^%d L=%d K=%d dnum=%d; settings %s; keygen k_max=%d ..." % (log_n, L, K, dnum, args.settings, k))
        mick.set_schedule(prm, a)
        mick.set_tensor_method(prm, tm)
        mick.set_modup_targets(prm, mt)
        table = {}
    else:
        log("params N=2^%d L=%d K=%d dnum=%d; autotune; keygen k_max=%d ..." % (log_n, L, K, dnum, k))
        mick.autotune(prm)
        table = {"%d/%d/%d" % c: round(us, 1) for c, us in mick.autotune_report(prm)}
    tuning = {"first_pass_log": mick.schedule(prm), "tensor_method": mick.tensor_method(prm),
              "modup_targets": mick.modup_targets(prm), "autotuned": not args.settings,
              "table_us_per_mult": table}
    log("settings (first-pass log, tensor method, ModUp targets): %s" % str(tuning))
    keys = mick.Keys(prm, 3, k)
    N = prm.N
    scale = 2.0 ** 30
    rng = np.random.default_rng(2024)
    cts = torch.empty(jobs, k, 2, level, N, dtype=torch.int32, device="cuda")
    log("encrypting %d inputs ..." % (jobs * k))
    for j in range(jobs):
        for u in range(k):
            re = rng.uniform(-1, 1, N // 2)
            im = rng.uniform(-1, 1, N // 2)
            m = mick.encode(prm, re, im, scale)
            mick.encrypt(prm, keys, m, level, 3, j * k + u, out=cts[j, u])
    out = torch.empty(jobs, 2, level - k + 1, N, dtype=torch.int32, device="cuda")
    ws = mick.batch_workspace(prm, jobs, k, level)
    stream = torch.cuda.current_stream()

    if args.copy_calibration:
        a = torch.ones(args.copy_calibration << 18, dtype=torch.int32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log("calibration copy of %d MiB done" % args.copy_calibration)
        del a, b
    log("warmup %d steps (every launch timed after the first step) ..." % args.warmup)
    mick.profile_select(None)
    # the first step's launches include loading each kernel's code: that
    # step is not profiled (unless it is the only warmup step)
    cold = 1 if args.warmup > 1 else 0
    for w in range(args.warmup):
        if w == cold:
            torch.cuda.synchronize()
            mick.profile_enable(True)
        mick.mul_relin_rescale_batch(prm, keys, cts, level, out=out, ws=ws)
    torch.cuda.synchronize()
    # the dominant kernel from the warmup; the timed steps record events
    # around that kernel only, so the other launches run back to back
    dominant = roofline(mick.profile_collect(), args.warmup - cold, N, k, level, K, prm.alpha, jobs)["kernel"]
    mick.profile_select([dominant])

    # The K timed steps run back to back between one pair of events (and the
    # pair around the dominant kernel in each step); the per-step latencies
    # come from a second pass with an event at every step boundary.
    log("timing %d batched steps ..." % args.steps)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for i in range(args.steps):
        mick.mul_relin_rescale_batch(prm, keys, cts, level, out=out, ws=ws)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = mick.profile_collect()
    mick.profile_enable(False)
    mick.profile_select(None)
    total_ms = e0.elapsed_time(e1)
    value = jobs * args.steps / (total_ms / 1e3)
    log("batched: %.3f ms/step, %.1f ct-mults/s (host wall %.3f s)" % (total_ms / args.steps, value, wall))
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    ev[0].record(stream)
    for i in range(args.steps):
        mick.mul_relin_rescale_batch(prm, keys, cts, level, out=out, ws=ws)
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    step_ms = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(args.steps)])
    log("per-step latency pass: %.3f ms/step mean" % step_ms.mean())
    rl = roofline(prof, args.steps, N, k, level, K, prm.alpha, jobs)
    if args.workload == "n16_k8_b8":
        rl["traffic"] = measured_traffic(rl["kernel"])

    plain = None
    lists = [[cts[j, u] for u in range(k)] for j in range(jobs)]
    if not args.no_plain:
        ws1 = mick.workspace(prm, mick.OP_MUL_RELIN_RESCALE, k, level)
        for j in range(jobs):
            mick.mul_relin_rescale(prm, keys, lists[j], level, out=out[j], ws=ws1)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            for j in range(jobs):
                mick.mul_relin_rescale(prm, keys, lists[j], level, out=out[j], ws=ws1)
        e1.record(stream)
        torch.cuda.synchronize()
        pms = e0.elapsed_time(e1) / (args.steps * jobs)
        plain = {"value": round(1e3 / pms, 2), "unit": "ct-mults/s", "ms_per_mult": round(pms, 4)}
        log("plain: %.3f ms per multiply, %.1f ct-mults/s" % (pms, 1e3 / pms))

    unfused = None
    if args.workload == "paper3" and not args.no_plain:
        # the same multiply without relocation: tensor product, relinearisation
        # with its own ModDown back to the NTT domain, then the (k-1)-level
        # rescale of Algorithm 1 as a separate call
        d = torch.empty(k + 1, level, N, dtype=torch.int32, device="cuda")
        y = torch.empty(2, level, N, dtype=torch.int32, device="cuda")
        wsr = mick.workspace(prm, mick.OP_RELIN, k, level)
        wss = mick.workspace(prm, mick.OP_RESCALE, k - 1, level)

        def unfused_one(j):
            mick.mul_k(prm, lists[j], level, out=d)
            mick.relin_k(prm, keys, d, k, level, out=y, ws=wsr)
            mick.rescale_multi(prm, y, level, k - 1, out=out[j], ws=wss)

        for j in range(jobs):
            unfused_one(j)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            for j in range(jobs):
                unfused_one(j)
        e1.record(stream)
        torch.cuda.synchronize()
        ums = e0.elapsed_time(e1) / (args.steps * jobs)
        unfused = {"value": round(1e3 / ums, 2), "unit": "ct-mults/s", "ms_per_mult": round(ums, 4),
                   "path": "mul_k + relin_k + rescale_multi"}
        log("unfused: %.3f ms per multiply, %.1f ct-mults/s" % (ums, 1e3 / ums))

    bytes_per_mult = mult_bytes(N, k, level, K, prm.alpha, jobs)
    systems = {}
    if args.workload == "n16_k8_b8" and not args.no_systems:
        # the systems forms beside the headline batch: the mixed 512-multiply
        # batch (graph of job-table plans against each multiply alone) and a
        # shorter serving run with per-request latency
        del cts, out, ws, lists
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        log("mixed leg: 512 multiplies, %d graph replays ..." % args.mixed_steps)
        systems["mixed512"] = mixed_leg(args, torch, mick, args.mixed_steps, 1, 1)
        log("serving leg: %d requests ..." % args.serve_requests)
        systems["serving"] = serve_leg(args, torch, mick, args.serve_requests, (0.5, 0.8, 0.95))
    cpu = None if args.no_cpu_baseline else cpu_baseline(log_n, L, K, dnum, k, level)
    rec = {
        "metric": "k-input ct-mults/s at N=2^16 (batched vs plain), % HBM peak; p50/p99 latency",
        "value": round(value, 2),
        "unit": "ct-mults/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(total_ms / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "%d-input multiply, N=2^%d, %d+%d primes, dnum=%d, level %d, batch %d"
                               % (k, log_n, L, K, dnum, level, jobs),
                   "k": k, "log_n": log_n, "level": level, "batch": jobs, "parallelism": "none"},
        "tuning": tuning,
        "plain": plain,
        "batched_over_plain": round(value / plain["value"], 3) if plain else None,
        **({"unfused": unfused} if unfused else {}),
        "latency_ms": {"p50": round(float(np.percentile(step_ms, 50)), 4),
                       "p99": round(float(np.percentile(step_ms, 99)), 4),
                       "of": "one batched step, an event at every step boundary"},
        "hbm_frac_whole_path": round(value * bytes_per_mult / 1e9 / HBM_PEAK_GBS, 5),
        "algorithmic_bytes_per_mult": int(bytes_per_mult),
        "roofline": rl,
        "cpu_baseline": cpu,
        **systems,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
