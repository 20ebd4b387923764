"""tqp_filter_noalloc, the filter entry point that allocates nothing (its scratch is a fixed device
array), against tqp_filter on the same inputs: two calls in a row, the second with a smaller input
(the second call must clear what the first one left in the shared array), a carried column, an
empty input, and the size limit refused before any launch."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(hip):
    return hip.Context(0)


def _cols(hip, n, seed):
    import torch
    rng = np.random.default_rng(seed)
    date = rng.integers(0, 2557, n).astype(np.int32)
    seg = rng.integers(0, 5, n).astype(np.int8)
    price = rng.integers(90_000, 10_500_000, n).astype(np.int64)
    carry = rng.integers(0, 1 << 30, n).astype(np.int32)
    host = [date, seg, price]
    dev = [torch.from_numpy(c).cuda() for c in host]
    return host, dev, carry, torch.from_numpy(carry).cuda()


@pytest.mark.parametrize("sizes", [(3_000_017, 1_000_003), (70_001, 5)])
def test_noalloc_matches_filter(hip, ctx, sizes):
    import torch
    preds = [(0, hip.TQP_LT, 2000), (1, hip.TQP_NE, 3), (2, hip.TQP_GE, 200_000)]
    for call, n in enumerate(sizes):
        host, dev, carry_h, carry_d = _cols(hip, n, 500 + call)
        want_rows, want_carry, want_cnt = hip.filter(ctx, dev, preds, carry=carry_d)
        torch.cuda.synchronize()
        cap = n
        out = torch.full((cap,), -7, dtype=torch.int32, device="cuda")
        outc = torch.full((cap,), -7, dtype=torch.int32, device="cuda")
        cnt = torch.full((1,), -7, dtype=torch.int64, device="cuda")
        hip.filter_noalloc(ctx, dev, preds, out, cnt, carry=carry_d, out_carry=outc)
        k = int(cnt.item())
        assert k == int(want_cnt.item())
        assert np.array_equal(out[:k].cpu().numpy(), want_rows[:k].cpu().numpy())
        assert np.array_equal(outc[:k].cpu().numpy(), want_carry[:k].cpu().numpy())
        assert (out[k:].cpu().numpy() == -7).all()            # nothing written past the count
        # and both equal the oracle's filter
        cols = [host[0], host[1], host[2]]
        want = oracle.filter_rows(cols, preds)
        assert np.array_equal(out[:k].cpu().numpy(), want)
        assert np.array_equal(outc[:k].cpu().numpy(), carry_h[want])
    assert ctx.errors() == 0


def test_noalloc_empty_and_limit(hip, ctx):
    import torch
    out = torch.empty(4, dtype=torch.int32, device="cuda")
    cnt = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    empty = [torch.empty(0, dtype=torch.int32, device="cuda")]
    hip.filter_noalloc(ctx, empty, [(0, hip.TQP_LT, 5)], out, cnt)
    assert int(cnt.item()) == 0
    # above the scratch limit: refused on the host, nothing launched (the column is never read)
    big = [torch.empty(8, dtype=torch.int32, device="cuda")]
    with pytest.raises(hip.TQPError):
        hip.filter_noalloc(ctx, big, [(0, hip.TQP_LT, 5)], out, cnt, n=hip._lib.FILTER_NOALLOC_MAX_ROWS + 1)
    assert ctx.errors() == 0
