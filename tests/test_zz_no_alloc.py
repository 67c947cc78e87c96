"""The allocation-free sort entry point against the allocating one.

lfr_sort_pairs_u32_noalloc must give exactly what lfr_sort_pairs_u32 gives
(bit-exact keys and values) on consecutive calls that reuse its fixed
per-GPU scratch, the second call on a smaller input, with odd and even
pass counts (the result ends in the scratch or in place), and must refuse
sizes beyond its limit without touching the inputs."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

LIMIT = 1 << 22


def say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_04509_amd import lfr
    ctx = lfr.Context(0)
    yield lfr, ctx
    torch.cuda.synchronize()
    ctx.close()


def _pairs(n, bits, seed):
    rng = np.random.default_rng(seed)
    keys = rng.integers(0, 1 << bits, n, dtype=np.uint64).astype(np.uint32)
    keys[: n // 4] = keys[n // 2]          # ties: stability is part of the result
    vals = rng.permutation(n).astype(np.uint32)
    return keys, vals


def _dev(a):
    return torch.from_numpy(a.view(np.int32).copy()).cuda()


@pytest.mark.parametrize("sizes,bits", [((LIMIT, 300001), 32),       # 4 passes: result in place
                                        ((1000003, 4097), 19),       # 3 passes: result copied back
                                        ((65536, 2), 13)])
def test_noalloc_sort_matches_sort(lib, sizes, bits):
    lfr, ctx = lib
    for call, n in enumerate(sizes):
        say("noalloc sort", "call", call, "n", n, "bits", bits)
        keys, vals = _pairs(n, bits, seed=n + bits)
        ka, va = _dev(keys), _dev(vals)
        kb, vb = _dev(keys), _dev(vals)
        lfr.sort_pairs(ctx, ka, va, 0, bits)
        lfr.sort_pairs_noalloc(ctx, kb, vb, 0, bits)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(kb.cpu().numpy(), ka.cpu().numpy())
        np.testing.assert_array_equal(vb.cpu().numpy(), va.cpu().numpy())
        order = np.argsort(keys, kind="stable")
        np.testing.assert_array_equal(kb.cpu().numpy().view(np.uint32), keys[order])
        np.testing.assert_array_equal(vb.cpu().numpy().view(np.uint32), vals[order])


def test_noalloc_sort_limits(lib):
    lfr, ctx = lib
    say("noalloc sort limits")
    n = LIMIT + 1
    kd = torch.zeros(n, dtype=torch.int32, device="cuda")
    vd = torch.arange(n, dtype=torch.int32, device="cuda")
    with pytest.raises(lfr.LfrError) as ei:
        lfr.sort_pairs_noalloc(ctx, kd, vd, 0, 32)
    assert ei.value.code == lfr.LFR_ERR_CAPACITY
    with pytest.raises(lfr.LfrError) as ei:
        lfr.sort_pairs_noalloc(ctx, kd[:10], vd[:10], 0, 33)
    assert ei.value.code == lfr.LFR_ERR_INVALID_ARG
    torch.cuda.synchronize()
    assert int(kd.abs().sum()) == 0 and torch.equal(vd, torch.arange(n, dtype=torch.int32, device="cuda"))
    # empty and single-element inputs are accepted and left as they are
    lfr.sort_pairs_noalloc(ctx, kd[:0], vd[:0], 0, 32)
    k1 = torch.tensor([7], dtype=torch.int32, device="cuda")
    v1 = torch.tensor([3], dtype=torch.int32, device="cuda")
    lfr.sort_pairs_noalloc(ctx, k1, v1, 0, 32)
    torch.cuda.synchronize()
    assert int(k1) == 7 and int(v1) == 3
