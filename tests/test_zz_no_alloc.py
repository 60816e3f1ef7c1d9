"""The allocation-free multiply (static device workspace inside the library)
against the multiply with a caller workspace, bit for bit, on two calls in a
row (the second with a smaller input, so the workspace holds the first call's
larger contents), and its refusal of a multiply whose workspace exceeds the
static array."""
import numpy as np
import pytest
import torch

from paper_2601_15401_amd import mick

pytestmark = pytest.mark.gpu


def _cts(prm, k, level, seed):
    rng = np.random.default_rng(seed)
    return [mick.from_numpy_u32(np.stack([np.stack([rng.integers(0, q, prm.N, dtype=np.int64).astype(np.uint32)
                                                    for q in prm.q[:level]]) for _ in range(2)]))
            for _ in range(k)]


def test_noalloc_matches_the_workspace_multiply_twice():
    prm = mick.Params(15, 16, 4, 4)  # the four-input N = 2^15 set: 51 MB of workspace at k = 4, level 16
    keys = mick.Keys(prm, 17, 4)
    big = _cts(prm, 4, 16, 1)
    small = _cts(prm, 2, 5, 2)
    assert prm.workspace_bytes(mick.OP_MUL_RELIN_RESCALE, 4, 16) <= 64 << 20
    got1 = mick.mul_relin_rescale_noalloc(prm, keys, big, 16)
    got2 = mick.mul_relin_rescale_noalloc(prm, keys, small, 5)
    want1 = mick.mul_relin_rescale(prm, keys, big, 16)
    want2 = mick.mul_relin_rescale(prm, keys, small, 5)
    torch.cuda.synchronize()
    assert torch.equal(got1, want1)
    assert torch.equal(got2, want2)


def test_noalloc_on_a_second_parameter_set_and_refusal():
    prm = mick.Params(13, 3, 1, 3)
    keys = mick.Keys(prm, 18, 3)
    cts = _cts(prm, 3, 3, 3)
    got = mick.mul_relin_rescale_noalloc(prm, keys, cts, 3)
    assert torch.equal(got, mick.mul_relin_rescale(prm, keys, cts, 3))
    big = mick.Params(16, 32, 8, 4)
    bkeys = mick.Keys(big, 19, 8)
    assert big.workspace_bytes(mick.OP_MUL_RELIN_RESCALE, 8, 32) > 64 << 20
    z = torch.zeros(2, 32, big.N, dtype=torch.int32, device="cuda")
    with pytest.raises(mick.MickError) as e:
        mick.mul_relin_rescale_noalloc(big, bkeys, [z] * 8, 32)
    assert e.value.status == mick.E_WS and "static workspace" in str(e.value)
    torch.cuda.synchronize()
