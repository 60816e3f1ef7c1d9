"""Work queue, transform schedules, autotuner cache and allocator on the GPU.

Every multiply result is compared bit for bit with the same multiply
launched alone (itself checked against the oracle by the parity tests), and
every alternative transform schedule with the oracle's transform."""

import numpy as np
import pytest
import torch

from oracle import ntt as ontt, params as oparams
from paper_2601_15401_amd import mick

pytestmark = pytest.mark.gpu

SETS = [(13, 3, 1, 3), (14, 8, 2, 4)]


def _rand_ct(rng, moduli, n):
    return mick.from_numpy_u32(np.stack([np.stack([rng.integers(0, m, n, dtype=np.int64).astype(np.uint32)
                                                   for m in moduli]) for _ in range(2)]))


@pytest.fixture(scope="module")
def sets():
    out = []
    for i, (ln, L, K, d) in enumerate(SETS):
        prm = mick.Params(ln, L, K, d)
        out.append((prm, mick.Keys(prm, 90 + i, min(12, L))))
    return out


def _jobs(sets, n, seed):
    rng = np.random.default_rng(seed)
    jobs = []
    for i in range(n):
        st = int(rng.integers(0, len(sets)))
        prm = sets[st][0]
        k = int(rng.integers(2, min(12, prm.L) + 1))
        level = int(rng.integers(k, prm.L + 1))
        cts = [_rand_ct(rng, prm.q[:level], prm.N) for _ in range(k)]
        out = torch.empty(2, level - k + 1, prm.N, dtype=torch.int32, device="cuda")
        jobs.append((1000 + i, st, cts, level, out))
    return jobs


def _check_alone(sets, jobs):
    for jid, st, cts, level, out in jobs:
        prm, keys = sets[st]
        alone = mick.mul_relin_rescale(prm, keys, cts, level)
        assert torch.equal(out, alone), "job %d (set %d, k=%d, level=%d)" % (jid, st, len(cts), level)


def test_queue_run_poll_under_a_small_arena(sets):
    jobs = _jobs(sets, 40, 1)
    q = mick.Queue(sets, capacity=256)  # smaller than any job: rejected at push
    with pytest.raises(mick.MickError):
        q.push(jobs[:1])
    biggest = max(q.job_bytes(st, len(c), lv) for _, st, c, lv, _ in jobs)
    q.close()
    q = mick.Queue(sets, capacity=3 * biggest)
    q.push(jobs)
    assert q.info()[0] == 40
    done, rounds = [], 0
    while len(done) < 40:
        q.run()
        pending, running, used = q.info()
        assert used <= 3 * biggest
        done += q.poll()
        rounds += 1
        assert rounds < 100000
    torch.cuda.synchronize()
    assert sorted(done) == [j[0] for j in jobs]
    assert q.info() == (0, 0, 0)
    _check_alone(sets, jobs)
    q.close()


def test_queue_drain_and_mixed_streams(sets):
    jobs = _jobs(sets, 30, 2)
    q = mick.Queue(sets, capacity=1 << 31)
    q.push(jobs[:15])
    s2 = torch.cuda.Stream()
    q.run()  # current stream
    with torch.cuda.stream(s2):
        q.push(jobs[15:])
        q.run()
    torch.cuda.synchronize()
    got = []
    while len(got) < 30:
        got += q.poll()
    assert sorted(got) == [j[0] for j in jobs]
    _check_alone(sets, jobs)
    jobs2 = _jobs(sets, 12, 3)
    q.push(jobs2)
    q.drain()
    assert q.info() == (0, 0, 0)
    _check_alone(sets, jobs2)
    q.close()


@pytest.mark.parametrize("ln,L,K,dnum", [(14, 8, 2, 4), (15, 16, 4, 4)])
def test_alternative_schedules_are_exact(ln, L, K, dnum):
    prm = mick.Params(ln, L, K, dnum)
    default = mick.schedule(prm)
    keys = mick.Keys(prm, 5, 6)
    rng = np.random.default_rng(ln)
    level = L
    cts = [_rand_ct(rng, prm.q[:level], prm.N) for _ in range(4)]
    want = mick.mul_relin_rescale(prm, keys, cts, level)
    # six inputs: the fused tensor kernel's 1024-residue tiles, whose row
    # blocks follow the schedule (2^6, 2^7 or 2^8 rows)
    cts6 = [_rand_ct(rng, prm.q[:level], prm.N) for _ in range(6)]
    want6 = mick.mul_relin_rescale(prm, keys, cts6, level)
    op = oparams.make_params(ln, L, K, dnum)
    # two q limbs and the first special prime (prime index L)
    mods, psis = [op.q[0], op.q[1], op.p[0]], [op.psi_q[0], op.psi_q[1], op.psi_p[0]]
    limbs = np.stack([rng.integers(0, m, prm.N, dtype=np.int64).astype(np.uint64) for m in mods])
    ref = ontt.ntt(limbs, mods, psis)
    for a in (7, 8):
        mick.set_schedule(prm, a)
        assert mick.schedule(prm) == a
        xq = mick.from_numpy_u32(limbs[:2].astype(np.uint32))
        xp = mick.from_numpy_u32(limbs[2:].astype(np.uint32))
        mick.ntt(prm, xq, 0)
        mick.ntt(prm, xp, L)
        got_f = np.concatenate([mick.to_numpy_u32(xq), mick.to_numpy_u32(xp)]).astype(np.uint64)
        assert np.array_equal(got_f, ref), "schedule %d forward" % a
        mick.ntt(prm, xq, 0, inverse=True)
        mick.ntt(prm, xp, L, inverse=True)
        got_i = np.concatenate([mick.to_numpy_u32(xq), mick.to_numpy_u32(xp)]).astype(np.uint64)
        assert np.array_equal(got_i, limbs), "schedule %d inverse" % a
        got = mick.mul_relin_rescale(prm, keys, cts, level)
        assert torch.equal(got, want), "schedule %d multiply" % a
        got6 = mick.mul_relin_rescale(prm, keys, cts6, level)
        assert torch.equal(got6, want6), "schedule %d six-input multiply" % a
    mick.set_schedule(prm, default)
    with pytest.raises(mick.MickError):
        mick.set_schedule(prm, 6)


def test_autotune_cache(tmp_path):
    """Every (split, tensor method, ModUp targets) combination is timed on the
    whole multiply; the choice is recorded in the cache and reused."""
    path = str(tmp_path / "schedules.txt")
    prm = mick.Params(15, 16, 4, 4)
    a = mick.autotune(prm, path)
    assert a in (7, 8)
    table = mick.autotune_report(prm)
    # two splits x three tensor methods x one target (digits of 4 primes)
    assert sorted(c for c, _ in table) == [(s, t, 1) for s in (7, 8) for t in (0, 1, 2)]
    best = min(table, key=lambda x: x[1])[0]
    assert (mick.schedule(prm), mick.tensor_method(prm), mick.modup_targets(prm)) == best
    lines = open(path).read().splitlines()
    assert len(lines) == 1 and lines[0].startswith("mick-tune ")
    assert tuple(int(v) for v in lines[0].split()[-4:-1]) == best
    prm2 = mick.Params(15, 16, 4, 4)
    assert mick.autotune(prm2, path) == a  # from the cache: nothing appended, nothing timed
    assert (mick.schedule(prm2), mick.tensor_method(prm2), mick.modup_targets(prm2)) == best
    assert mick.autotune_report(prm2) == []
    assert len(open(path).read().splitlines()) == 1
    prm3 = mick.Params(16, 32, 8, 4)  # one split; three tensor methods x one or two ModUp targets
    assert mick.autotune(prm3, path) == 8
    assert sorted(c for c, _ in mick.autotune_report(prm3)) == [(8, t, m) for t in (0, 1, 2) for m in (1, 2)]
    assert len(open(path).read().splitlines()) == 2
    # the chosen settings change nothing in the result
    keys = mick.Keys(prm3, 5, 3)
    rng = np.random.default_rng(3)
    cts = [_rand_ct(rng, prm3.q[:6], prm3.N) for _ in range(3)]
    got = mick.mul_relin_rescale(prm3, keys, cts, 6)
    for t in (0, 1, 2):
        for m in (1, 2):
            mick.set_tensor_method(prm3, t)
            mick.set_modup_targets(prm3, m)
            assert torch.equal(mick.mul_relin_rescale(prm3, keys, cts, 6), got), (t, m)
    with pytest.raises(mick.MickError):
        mick.set_modup_targets(prm, 2)  # digits of four primes take one target


def test_torch_allocator_holds_keys():
    prm0 = mick.Params(14, 8, 2, 4)
    keys0 = mick.Keys(prm0, 11, 3)
    rng = np.random.default_rng(12)
    cts = [_rand_ct(rng, prm0.q[:8], prm0.N) for _ in range(3)]
    want = mick.mul_relin_rescale(prm0, keys0, cts, 8)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    mick.use_torch_allocator(True)
    try:
        prm = mick.Params(14, 8, 2, 4)
        keys = mick.Keys(prm, 11, 3)
        torch.cuda.synchronize()
        evk_bytes = 2 * 4 * 2 * (8 + 2) * prm.N * 4  # (k_max - 1) dnum 2 (L + K) N words
        assert torch.cuda.memory_allocated() - before >= evk_bytes
        got = mick.mul_relin_rescale(prm, keys, [c.clone() for c in cts], 8)
        assert torch.equal(got, want)
        del keys, prm, got
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() <= before + 4096
    finally:
        mick.use_torch_allocator(False)
