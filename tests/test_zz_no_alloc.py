"""The no-allocation attention entry point (ci_attention_decode_noalloc)
against ci_attention_decode on the same inputs: bit-identical outputs on two
calls in a row, the second smaller than the first (the static scratch keeps
the first call's contents), both within the FP64 oracle's bound; oversized
requests are rejected on the host before any launch."""
import numpy as np
import pytest

import oracle
import synth
from oracle import decode as od

pytestmark = pytest.mark.gpu
U = 2.0 ** -24


@pytest.fixture(scope="module")
def ctx(dev):
    from paper_2501_16909_amd import coloc
    c = coloc.Context(0)
    yield c
    c.close()


def _t(x, dev):
    import torch
    return torch.from_numpy(np.require(x, requirements=["C", "W"])).to(dev)


def _bf16(x32):
    c = oracle.f32_to_bf16(np.asarray(x32, np.float32))
    return c.view(np.int16), oracle.bf16_to_f64(c).reshape(np.shape(x32))


def _case(dev, seed, batch, nq, nkv, d, max_ctx, qscale):
    q = synth.uniform_affine_f32(synth.seed_for(seed, 930), batch * nq * d, qscale).reshape(batch, nq, d)
    kc, kv = _bf16(synth.uniform_f32(synth.seed_for(seed, 931), batch * nkv * max_ctx * d))
    vc, vv = _bf16(synth.uniform_f32(synth.seed_for(seed, 932), batch * nkv * max_ctx * d))
    return (q, kv.reshape(batch, nkv, max_ctx, d), vv.reshape(batch, nkv, max_ctx, d),
            _t(q, dev), _t(kc, dev), _t(vc, dev))


def test_noalloc_matches_attention_decode_twice(ctx, dev):
    import torch
    from paper_2501_16909_amd import coloc
    cases = [  # (batch, n_q, n_kv, head_dim, max_ctx, positions, q scale); the second is smaller
        (8, 32, 8, 128, 8064, [0, 63, 64, 1000, 8063, 2047, 6333, 17], 4.0),   # the largest that fits
        (2, 4, 1, 256, 300, [299, 5], 1.0),
    ]
    for i, (batch, nq, nkv, d, max_ctx, pos, qs) in enumerate(cases):
        need = batch * nq * -(-max_ctx // 64) * (d + 2) * 4
        assert need <= coloc.NOALLOC_PART_BYTES
        print(f"noalloc case {i}: batch {batch} n_q {nq} n_kv {nkv} d {d} max_ctx {max_ctx}", flush=True)
        q, kv, vv, tq, tk, tv = _case(dev, 6 + i, batch, nq, nkv, d, max_ctx, qs)
        want = ctx.attention_decode(tq, tk, tv, pos, nq, nkv, d, max_ctx)
        out = torch.full((batch, nq * d), -1, dtype=torch.int16, device=dev)
        ctx.attention_decode_noalloc(tq, tk, tv, pos, nq, nkv, d, max_ctx, out)
        got = out.cpu().numpy()
        assert np.array_equal(got, want.cpu().numpy()), i
        vals = oracle.bf16_to_f64(got.view(np.uint16)).reshape(batch, nq, d)
        for b, p in enumerate(pos):
            ex = od.attention_decode(q[b].astype(np.float64), kv[b, :, :p + 1], vv[b, :, :p + 1])
            eps = (64 + (p // 64 + 1) + 8) * 2 * U * np.max(np.abs(vv[b, :, :p + 1]))
            lo, hi = od.q_bf16(ex - eps), od.q_bf16(ex + eps)
            assert np.all((vals[b] >= lo) & (vals[b] <= hi)), (i, b, p)


def test_noalloc_rejects_beyond_the_static_limit(ctx, dev):
    import torch
    from paper_2501_16909_amd import coloc
    batch, nq, nkv, d, max_ctx = 8, 32, 8, 128, 8065     # one chunk more than fits
    assert batch * nq * -(-max_ctx // 64) * (d + 2) * 4 > coloc.NOALLOC_PART_BYTES
    q = torch.zeros(batch * nq * d, dtype=torch.float32, device=dev)
    kc = torch.zeros(16, dtype=torch.int16, device=dev)       # never read: rejected on the host
    out = torch.zeros(batch * nq * d, dtype=torch.int16, device=dev)
    with pytest.raises(coloc.CiError) as ei:
        ctx.attention_decode_noalloc(q, kc, kc, [0] * batch, nq, nkv, d, max_ctx, out)
    assert ei.value.status == 1 and "static scratch limit" in str(ei.value)
    with pytest.raises(coloc.CiError) as ei:
        ctx.attention_decode_noalloc(q, kc, kc, [5000] + [0] * 7, nq, nkv, d, 4096, out)   # position >= max_ctx
    assert ei.value.status == 1
