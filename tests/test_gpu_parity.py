"""GPU parity: the HIP library against the CPU oracle, residue by residue.

Every case feeds the same seeded inputs to both sides (random NTT-domain
residues from a test-local numpy generator, or encryptions both sides derive
from the same seed) and requires bit-exact equality: the path is exact
integer arithmetic, so the tolerance is zero.
"""
import numpy as np
import pytest
import torch

from oracle import ckks, keys as okeys, mult, ntt as ontt, params as oparams
from paper_2601_15401_amd import mick

pytestmark = pytest.mark.gpu

SCALE = 2.0 ** 30


def _eq(got_t, want, what):
    got = mick.to_numpy_u32(got_t).astype(np.uint64) if isinstance(got_t, torch.Tensor) else got_t.astype(np.uint64)
    want = np.asarray(want, dtype=np.uint64)
    assert got.shape == want.shape, (what, got.shape, want.shape)
    bad = np.argwhere(got != want)
    assert bad.size == 0, "%s: %d residues differ, first at %s" % (what, len(bad), bad[0].tolist())


def _rand_poly(rng, moduli, n):
    return np.stack([rng.integers(0, m, n, dtype=np.int64).astype(np.uint64) for m in moduli])


class Ctx:
    """Oracle and library parameters and keys for one parameter set."""

    def __init__(self, log_n, L, K, dnum, seed, k_max):
        self.op = oparams.make_params(log_n, L, K, dnum)
        self.ok = okeys.keygen(self.op, seed, k_max)
        self.prm = mick.Params(log_n, L, K, dnum)
        self.gk = mick.Keys(self.prm, seed, k_max)
        self.seed = seed


@pytest.fixture(scope="module")
def c1():
    return Ctx(13, 3, 1, 3, 1, 3)


@pytest.fixture(scope="module")
def hyb():
    # ragged digits at most levels: alpha = 2 over 8 primes
    return Ctx(13, 8, 2, 4, 7, 6)


# ------------------------------------------------------------------ params and transforms

@pytest.mark.parametrize("log_n", [13, 14, 15, 16])
def test_moduli_match_oracle(log_n):
    op = oparams.preset(log_n)
    prm = mick.Params(log_n, op.L, op.K, op.dnum)
    assert prm.q == op.q and prm.p == op.p and prm.alpha == op.alpha


@pytest.mark.parametrize("log_n", [13, 14, 15, 16])
def test_ntt_parity(log_n):
    op = oparams.preset(log_n)
    prm = mick.Params(log_n, op.L, op.K, op.dnum)
    moduli, psis = op.q + op.p, op.psi_q + op.psi_p
    rng = np.random.default_rng(log_n)
    a = _rand_poly(rng, moduli, op.N)
    d = mick.from_numpy_u32(a)
    mick.ntt(prm, d, 0, inverse=False)
    _eq(d, ontt.ntt(a, moduli, psis), "forward NTT N=2^%d" % log_n)
    mick.ntt(prm, d, 0, inverse=True)
    _eq(d, a, "inverse NTT N=2^%d" % log_n)
    # inverse on fresh data, and a limb range that starts inside the q primes
    b = _rand_poly(rng, moduli[3:], op.N)
    d = mick.from_numpy_u32(b)
    mick.ntt(prm, d, 3, inverse=True)
    _eq(d, ontt.intt(b, moduli[3:], psis[3:]), "INTT from prime 3")


# ------------------------------------------------------------------ keys and encryption

@pytest.mark.parametrize("ctx", ["c1", "hyb"])
def test_keygen_parity(ctx, request):
    c = request.getfixturevalue(ctx)
    assert np.array_equal(c.gk.export_secret(), c.ok.s)
    pk = c.gk.export_pk()
    _eq(pk[0], c.ok.pk_b, "pk b")
    _eq(pk[1], c.ok.pk_a, "pk a")
    for t in range(2, c.gk.k_max + 1):
        for b in range(c.op.dnum):
            ev = c.gk.export_evk(t, b)
            k0, k1 = c.ok.evk[(t, b)]
            _eq(ev[0], k0, "evk0 t=%d b=%d" % (t, b))
            _eq(ev[1], k1, "evk1 t=%d b=%d" % (t, b))


@pytest.mark.parametrize("level", [8, 5, 1])
def test_encrypt_decrypt_parity(hyb, level):
    c = hyb
    _, _, m = ckks.message(c.op, c.seed, 3, SCALE)
    ct = mick.encrypt(c.prm, c.gk, m, level, c.seed, 3)
    want = ckks.encrypt(c.op, c.ok, m, level, c.seed, 3)
    _eq(ct, want, "ciphertext")
    _eq(mick.decrypt_residues(c.prm, c.gk, ct, level), ckks.decrypt_residues(c.op, c.ok, want, level), "dec res")
    dec = mick.decrypt(c.prm, c.gk, ct, level)
    assert dec.tolist() == ckks.decrypt(c.op, c.ok, want, level)


def test_encode_within_one(c1):
    re, im, m = ckks.message(c1.op, 5, 0, SCALE)
    got = mick.encode(c1.prm, re, im, SCALE)
    assert np.abs(got - m).max() <= 1
    r2, i2 = mick.decode(c1.prm, got, SCALE)
    assert np.abs(r2 - re).max() < 1e-6 and np.abs(i2 - im).max() < 1e-6


# ------------------------------------------------------------------ hot-path steps

@pytest.mark.parametrize("k", [2, 3, 4, 6])
@pytest.mark.parametrize("level", [8, 3])
def test_tensor_parity(hyb, k, level):
    c = hyb
    rng = np.random.default_rng(100 + k * 10 + level)
    cts = [np.stack([_rand_poly(rng, c.op.q[:level], c.op.N) for _ in range(2)]) for _ in range(k)]
    d = mick.mul_k(c.prm, [mick.from_numpy_u32(x) for x in cts], level)
    _eq(d, mult.tensor(cts, c.op.q[:level]), "tensor k=%d level=%d" % (k, level))


@pytest.mark.parametrize("k,level", [(2, 8), (3, 7), (4, 5), (6, 6), (2, 2)])
def test_relin_parity(hyb, k, level):
    c = hyb
    rng = np.random.default_rng(200 + k * 10 + level)
    D = np.stack([_rand_poly(rng, c.op.q[:level], c.op.N) for _ in range(k + 1)])
    out = mick.relin_k(c.prm, c.gk, mick.from_numpy_u32(D), k, level)
    c0, c1_ = mult.relin_textbook(c.op, c.ok, D, level)
    _eq(out, np.stack([c0, c1_]), "relin k=%d level=%d" % (k, level))


@pytest.mark.parametrize("level,mu", [(8, 1), (8, 3), (7, 6), (5, 2), (2, 1)])
def test_rescale_multi_parity(hyb, level, mu):
    c = hyb
    rng = np.random.default_rng(300 + level * 10 + mu)
    A = np.stack([_rand_poly(rng, c.op.q[:level], c.op.N) for _ in range(2)])
    out = mick.rescale_multi(c.prm, mick.from_numpy_u32(A), level, mu)
    want = np.stack([mult.multi_rs_alg1(c.op, A[l], level, mu) for l in range(2)])
    _eq(out, want, "rescale level=%d mu=%d" % (level, mu))


# ------------------------------------------------------------------ whole multiply

def test_three_input_multiply_c1(c1):
    cts_o, cts_g = [], []
    for u in range(3):
        _, _, m = ckks.message(c1.op, c1.seed, u, SCALE)
        cts_o.append(ckks.encrypt(c1.op, c1.ok, m, 3, c1.seed, u))
        cts_g.append(mick.encrypt(c1.prm, c1.gk, m, 3, c1.seed, u))
    out = mick.mul_relin_rescale(c1.prm, c1.gk, cts_g, 3)
    _eq(out, mult.mul_relin_rescale(c1.op, c1.ok, cts_o, 3), "C1 product")


@pytest.mark.parametrize("k,level", [(2, 8), (3, 8), (4, 7), (5, 5), (6, 8), (6, 6)])
def test_multiply_parity_random_inputs(hyb, k, level):
    c = hyb
    rng = np.random.default_rng(400 + k * 10 + level)
    cts = [np.stack([_rand_poly(rng, c.op.q[:level], c.op.N) for _ in range(2)]) for _ in range(k)]
    out = mick.mul_relin_rescale(c.prm, c.gk, [mick.from_numpy_u32(x) for x in cts], level)
    _eq(out, mult.mul_relin_rescale(c.op, c.ok, cts, level), "k=%d level=%d" % (k, level))


def test_batch_equals_plain_and_oracle(hyb):
    c = hyb
    k, level, jobs = 4, 8, 3
    rng = np.random.default_rng(500)
    cts = np.stack([np.stack([np.stack([_rand_poly(rng, c.op.q[:level], c.op.N) for _ in range(2)])
                              for _ in range(k)]) for _ in range(jobs)])
    dev = mick.from_numpy_u32(cts)
    out = mick.mul_relin_rescale_batch(c.prm, c.gk, dev, level)
    for j in range(jobs):
        plain = mick.mul_relin_rescale(c.prm, c.gk, [dev[j, u] for u in range(k)], level)
        assert torch.equal(out[j], plain)
        _eq(out[j], mult.mul_relin_rescale(c.op, c.ok, list(cts[j]), level), "batch job %d" % j)


def test_heterogeneous_jobs_equal_plain(hyb):
    """A mixed batch (different k and level per job, one launch per stage) gives
    each job the bits of its own plain call, and the oracle's."""
    c = hyb
    rng = np.random.default_rng(700)
    shapes = [(2, 8), (3, 5), (2, 2), (6, 8), (4, 7), (3, 3), (5, 6), (2, 8), (6, 6)]
    specs, host = [], []
    for k, level in shapes:
        cts = [np.stack([_rand_poly(rng, c.op.q[:level], c.op.N) for _ in range(2)]) for _ in range(k)]
        host.append((cts, level))
        specs.append(([mick.from_numpy_u32(x) for x in cts], level, None))
    outs = mick.mul_relin_rescale_jobs(c.prm, c.gk, specs)
    for (cts_d, level, _), out, (cts, _) in zip(specs, outs, host):
        assert torch.equal(out, mick.mul_relin_rescale(c.prm, c.gk, cts_d, level))
    for i in (0, 3, 5):
        cts, level = host[i]
        _eq(outs[i], mult.mul_relin_rescale(c.op, c.ok, cts, level), "mixed job %d" % i)


def test_plan_replayed_from_a_graph(hyb):
    """The execute step of a planned batch is captured into a graph; every
    replay (with eager work in between) matches the eager run."""
    c = hyb
    rng = np.random.default_rng(800)
    shapes = [(3, 8), (2, 4), (5, 7)]
    specs = []
    for k, level in shapes:
        cts = [mick.from_numpy_u32(np.stack([_rand_poly(rng, c.op.q[:level], c.op.N) for _ in range(2)]))
               for _ in range(k)]
        specs.append((cts, level, None))
    plan = mick.Plan(c.prm, c.gk, specs)
    eager = [o.clone() for o in plan.run()]
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            plan.run()
    for rep in range(3):
        for o in plan.outs:
            o.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for o, e in zip(plan.outs, eager):
            assert torch.equal(o, e), rep
        # eager work between replays
        mick.mul_relin_rescale(c.prm, c.gk, specs[0][0], 8)
        torch.cuda.synchronize()


def test_repeated_calls_are_deterministic(hyb):
    c = hyb
    rng = np.random.default_rng(600)
    cts = [mick.from_numpy_u32(np.stack([_rand_poly(rng, c.op.q[:6], c.op.N) for _ in range(2)])) for _ in range(5)]
    ws = mick.workspace(c.prm, mick.OP_MUL_RELIN_RESCALE, 5, 6)
    ref = mick.mul_relin_rescale(c.prm, c.gk, cts, 6, ws=ws)
    for _ in range(5):
        ws.fill_(-1)
        assert torch.equal(mick.mul_relin_rescale(c.prm, c.gk, cts, 6, ws=ws), ref)


def test_binding_refuses_buffers_of_the_wrong_size(hyb):
    """The C ABI takes bare device pointers; the binding checks each buffer's
    size against the shape the call implies before any launch."""
    c = hyb
    N = c.prm.N
    z = lambda *shape: torch.zeros(*shape, dtype=torch.int32, device="cuda")
    ct8 = z(2, 8, N)
    with pytest.raises(ValueError, match="ct"):
        mick.mul_relin_rescale(c.prm, c.gk, [ct8, ct8, z(2, 7, N)], 8)
    with pytest.raises(ValueError, match="out"):
        mick.mul_relin_rescale(c.prm, c.gk, [ct8] * 3, 8, out=z(2, 5, N))
    with pytest.raises(ValueError, match="out"):
        mick.mul_k(c.prm, [ct8] * 3, 8, out=z(3, 8, N))
    with pytest.raises(ValueError, match="d"):
        mick.relin_k(c.prm, c.gk, z(3, 8, N), 3, 8)
    with pytest.raises(ValueError, match="ct"):
        mick.rescale_multi(c.prm, z(2, 7, N), 8, 2)
    with pytest.raises(ValueError):
        mick.ntt(c.prm, z(N), 0)
    torch.cuda.synchronize()


def test_error_codes(hyb):
    c = hyb
    ct = torch.zeros(2, 4, c.prm.N, dtype=torch.int32, device="cuda")
    ws = mick.workspace(c.prm, mick.OP_MUL_RELIN_RESCALE, 7, 8)
    out = torch.zeros(2, 4, c.prm.N, dtype=torch.int32, device="cuda")
    with pytest.raises(mick.MickError) as e:
        mick.mul_relin_rescale(c.prm, c.gk, [ct, ct, ct, ct, ct], 4, out=out, ws=ws)  # level < k
    assert e.value.status == -2
    ct8 = torch.zeros(2, 8, c.prm.N, dtype=torch.int32, device="cuda")
    with pytest.raises(mick.MickError) as e:
        mick.mul_relin_rescale(c.prm, c.gk, [ct8] * 7, 8, ws=ws)  # k > k_max
    assert e.value.status == -3
    small = torch.zeros(16, dtype=torch.int32, device="cuda")
    with pytest.raises(mick.MickError) as e:
        mick.mul_relin_rescale(c.prm, c.gk, [ct8] * 3, 8, ws=small)
    assert e.value.status == -7
    with pytest.raises(mick.MickError) as e:
        mick.Params(12, 3, 1, 3)
    assert e.value.status == -1


# ------------------------------------------------------------------ workload shapes

def _full_case(log_n, k, seed):
    op = oparams.preset(log_n)
    ok = okeys.keygen(op, seed, k)
    prm = mick.Params(log_n, op.L, op.K, op.dnum)
    gk = mick.Keys(prm, seed, k)
    ev = gk.export_evk(k, op.dnum - 1)
    _eq(ev[0], ok.evk[(k, op.dnum - 1)][0], "evk0 t=k, last digit")
    level = op.L
    cts_o, cts_g = [], []
    for u in range(k):
        _, _, m = ckks.message(op, seed, u, SCALE)
        cts_o.append(ckks.encrypt(op, ok, m, level, seed, u))
        cts_g.append(mick.encrypt(prm, gk, m, level, seed, u))
        _eq(cts_g[-1], cts_o[-1], "input ciphertext %d" % u)
    out = mick.mul_relin_rescale(prm, gk, cts_g, level)
    _eq(out, mult.mul_relin_rescale(op, ok, cts_o, level), "N=2^%d k=%d product" % (log_n, k))
    return op, ok, prm, gk, out


def test_four_input_n15_full():
    _full_case(15, 4, 2)


def test_eight_input_n16_full():
    op, ok, prm, gk, out = _full_case(16, 8, 3)
    # the product decrypts and decodes to the slot-wise product of the messages
    lvl = op.L - 7
    dec = mick.decrypt(prm, gk, out, lvl)
    scale_out = SCALE ** 8
    for t in range(op.L - 7, op.L):
        scale_out /= op.q[t]
    re, im = mick.decode(prm, dec, scale_out)
    want = np.ones(op.N // 2, dtype=np.complex128)
    for u in range(8):
        r, i, _ = ckks.message(op, 3, u, SCALE)
        want = want * (r + 1j * i)
    err = np.abs((re + 1j * im) - want)
    assert err.max() < 1e-2, err.max()
