"""Serving loop on the GPU: every request served in the mix gets the bits of
the same multiply launched alone (and, for the small ring, the oracle's)."""
import numpy as np
import pytest
import torch

from oracle import keys as okeys, mult, params as oparams
from paper_2601_15401_amd import mick, serve

pytestmark = pytest.mark.gpu

SETS = {13: (3, 1, 3), 14: (8, 2, 4)}


def _rand_ct(rng, moduli, n):
    return np.stack([np.stack([rng.integers(0, m, n, dtype=np.int64).astype(np.uint64) for m in moduli])
                     for _ in range(2)])


@pytest.fixture(scope="module")
def ctx():
    prms = {ln: mick.Params(ln, *v) for ln, v in SETS.items()}
    keys = {ln: mick.Keys(prms[ln], 60 + ln, min(12, SETS[ln][0])) for ln in SETS}
    return prms, keys


@pytest.mark.parametrize("rate,n_streams,max_batch", [(4000.0, 2, 16), (1e9, 3, 64)])
def test_served_equals_alone(ctx, rate, n_streams, max_batch):
    prms, keys = ctx
    n = 96
    mix = serve.request_mix(n, 21, SETS, heavy_frac=0.2)
    rng = np.random.default_rng(22)
    host, reqs = [], []
    for i, ((ln, k, level), t) in enumerate(zip(mix, serve.poisson_arrivals(n, rate, 23))):
        cts = [_rand_ct(rng, prms[ln].q[:level], 1 << ln) for _ in range(k)]
        host.append(cts)
        reqs.append(serve.Request(i, ln, k, level, t, inputs=[mick.from_numpy_u32(c) for c in cts]))
    ex = serve.GpuExecutor(mick, torch, prms, keys, n_streams=n_streams, keep=lambda r: True)
    srv = serve.Server(ex, budget=8 * 10 ** 9, max_batch=max_batch)
    ex.start()
    st = srv.run(reqs)
    torch.cuda.synchronize()
    assert sorted(r.rid for r in st.completed) == list(range(n))
    assert all(r.done >= r.arrival for r in reqs)
    for r in reqs:
        alone = mick.mul_relin_rescale(prms[r.log_n], keys[r.log_n], r.inputs, r.level)
        assert torch.equal(r.output, alone), "request %d (N=2^%d k=%d level=%d)" % (r.rid, r.log_n, r.k, r.level)
    # three small-ring requests against the oracle
    op = oparams.make_params(13, *SETS[13])
    ok = okeys.keygen(op, 73, 3)
    small = [r for r in reqs if r.log_n == 13][:3]
    assert small
    for r in small:
        want = mult.mul_relin_rescale(op, ok, host[r.rid], r.level)
        got = mick.to_numpy_u32(r.output).astype(np.uint64)
        assert np.array_equal(got, np.asarray(want, dtype=np.uint64)), r.rid
