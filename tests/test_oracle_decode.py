"""Pins of the decode-step oracle against closed forms, invariants and
special cases that reduce to hand-checkable values (no GPU)."""
import math

import numpy as np

from oracle import decode as od


# ------------------------------------------------------------- RMSNorm
def test_rmsnorm_constant_vector_gives_gain():
    g = np.array([0.5, 1.0, 2.0, -3.0])
    for c in (0.25, 7.0, -2.0):
        y = od.rmsnorm(np.full((1, 4), c), g, eps=0.0)
        assert np.allclose(y[0], g * np.sign(c), rtol=0, atol=1e-15)


def test_rmsnorm_unit_mean_square_and_scale_invariance():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((3, 64))
    y = od.rmsnorm(x, np.ones(64), eps=0.0)
    assert np.allclose(np.mean(y * y, axis=1), 1.0, rtol=1e-14)
    assert np.allclose(od.rmsnorm(5.5 * x, np.ones(64), 0.0), y, rtol=1e-14)
    # eps enters under the square root: x = 0 stays 0, and for mean square m
    # the factor is 1/sqrt(m + eps)
    z = od.rmsnorm(np.zeros((1, 8)), np.ones(8), eps=1e-5)
    assert np.all(z == 0)
    y = od.rmsnorm(np.full((1, 4), 3.0), np.ones(4), eps=7.0)   # 3 / sqrt(9 + 7)
    assert np.allclose(y, 0.75, rtol=1e-15)


# ---------------------------------------------------------------- RoPE
def test_rope_position_zero_is_identity_and_norms_are_kept():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((4, 128))
    assert np.array_equal(od.rope(x, 0, 500000.0), x)
    y = od.rope(x, 1234, 500000.0)
    n0 = x[:, :64] ** 2 + x[:, 64:] ** 2
    n1 = y[:, :64] ** 2 + y[:, 64:] ** 2
    assert np.allclose(n0, n1, rtol=1e-13)


def test_rope_rotations_compose():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2, 64))
    a = od.rope(od.rope(x, 17, 10000.0), 40, 10000.0)
    assert np.allclose(a, od.rope(x, 57, 10000.0), atol=1e-12)


def test_rope_pairing_sign_and_frequencies():
    # pair 0 turns by pos radians whatever the base; (1, 0) goes to (cos, sin)
    y = od.rope(np.array([1.0, 0.0]), 1, 12345.0)
    assert np.allclose(y, [math.cos(1.0), math.sin(1.0)], atol=1e-15)
    # head_dim 4, base 100: pair 1 (elements 1 and 3) turns by pos / 10
    e1 = np.array([0.0, 1.0, 0.0, 0.0])
    y = od.rope(e1, 10, 100.0)
    assert np.allclose(y, [0.0, math.cos(1.0), 0.0, math.sin(1.0)], atol=1e-14)
    e3 = np.array([0.0, 0.0, 0.0, 1.0])
    y = od.rope(e3, 10, 100.0)
    assert np.allclose(y, [0.0, -math.sin(1.0), 0.0, math.cos(1.0)], atol=1e-14)


# ----------------------------------------------------------- attention
def test_attention_single_position_returns_its_value():
    rng = np.random.default_rng(4)
    q = rng.standard_normal((4, 16))
    k = rng.standard_normal((2, 1, 16))
    v = rng.standard_normal((2, 1, 16))
    o = od.attention_decode(q, k, v)
    assert np.allclose(o, np.repeat(v[:, 0, :], 2, axis=0), atol=1e-15)


def test_attention_equal_keys_average_the_values():
    rng = np.random.default_rng(5)
    q = rng.standard_normal((1, 8))
    k = np.tile(rng.standard_normal((1, 1, 8)), (1, 5, 1))
    v = rng.standard_normal((1, 5, 8))
    assert np.allclose(od.attention_decode(q, k, v)[0], v[0].mean(axis=0), atol=1e-14)


def test_attention_scale_is_inverse_sqrt_head_dim():
    # scores differ by sqrt(d) ln 3: weights 3/4 and 1/4
    d = 16
    q = np.zeros((1, d))
    q[0, 0] = 1.0
    k = np.zeros((1, 2, d))
    k[0, 0, 0] = math.sqrt(d) * math.log(3.0)
    v = np.zeros((1, 2, d))
    v[0, 0, :] = 1.0
    v[0, 1, :] = 5.0
    assert np.allclose(od.attention_decode(q, k, v)[0], 0.75 * 1.0 + 0.25 * 5.0, atol=1e-14)


def test_attention_group_mapping():
    # four query heads over two key/value heads: heads 0, 1 read head 0
    rng = np.random.default_rng(6)
    q = rng.standard_normal((4, 8))
    k = rng.standard_normal((2, 3, 8))
    v = np.zeros((2, 3, 8))
    v[1] = 1.0
    o = od.attention_decode(q, k, v)
    assert np.all(o[:2] == 0) and np.allclose(o[2:], 1.0, atol=1e-15)


# --------------------------------------------------------------- SiLU
def test_silu_mul_values():
    assert od.silu_mul(0.0, 3.0) == 0.0
    assert abs(od.silu_mul(math.log(3.0), 2.0) - 2.0 * 0.75 * math.log(3.0)) < 1e-15
    assert abs(od.silu_mul(40.0, 1.0) - 40.0) < 1e-14
    assert abs(od.silu_mul(-40.0, 1.0)) < 1e-15


# ---------------------------------------------------------- whole step
def _cfg(**kw):
    c = dict(hidden=8, n_q=2, n_kv=1, head_dim=4, ffn=6, vocab=5, eps=1e-5, rope_base=10000.0)
    c.update(kw)
    return c


def _zero_layer(c):
    qkv_rows = (c["n_q"] + 2 * c["n_kv"]) * c["head_dim"]
    return dict(g_attn=np.ones(c["hidden"]), w_qkv=np.zeros((qkv_rows, c["hidden"])),
                w_o=np.zeros((c["hidden"], c["n_q"] * c["head_dim"])), g_mlp=np.ones(c["hidden"]),
                w_gu=np.zeros((2 * c["ffn"], c["hidden"])), w_down=np.zeros((c["hidden"], c["ffn"])))


def test_step_zero_weights_is_identity_on_the_residual_stream():
    c = _cfg()
    rng = np.random.default_rng(7)
    x = rng.standard_normal((3, 8))
    kc = rng.standard_normal((2, 3, 1, 16, 4))
    vc = rng.standard_normal((2, 3, 1, 16, 4))
    k0, v0 = kc.copy(), vc.copy()
    pos = np.array([0, 5, 15])
    out = od.decode_step(c, [_zero_layer(c), _zero_layer(c)],
                         dict(g=np.ones(8), w_lm=np.zeros((5, 8))), kc, vc, x, pos)
    assert np.array_equal(out["x_out"], x)
    assert np.all(out["logits"] == 0)
    for b, p in enumerate(pos):
        assert np.all(kc[:, b, :, p, :] == 0) and np.all(vc[:, b, :, p, :] == 0)
        keep = np.ones(16, bool)
        keep[p] = False
        assert np.array_equal(kc[:, b, :, keep, :], k0[:, b, :, keep, :])
        assert np.array_equal(vc[:, b, :, keep, :], v0[:, b, :, keep, :])


def test_step_by_hand_at_position_zero():
    """Position 0: attention returns the new value row, so the step is a
    small composition of products checked with scalar arithmetic.  Rows of
    the QKV weight: query heads, then the key head, then the value head;
    rows of the gate/up weight: gate, then up."""
    c = _cfg(hidden=2, n_q=1, n_kv=1, head_dim=2, ffn=1, vocab=1, eps=0.0)
    x = np.array([[3.0, 4.0]])                  # mean square 12.5
    s = 1.0 / math.sqrt(12.5)
    w = _zero_layer(c)
    w["w_qkv"][0] = [1.0, 0.0]                  # query row (any: one position)
    w["w_qkv"][2] = [0.0, 1.0]                  # key row 0 -> xn[1]
    w["w_qkv"][4] = [1.0, 0.0]                  # value row 0 -> xn[0]
    w["w_qkv"][5] = [0.0, 2.0]                  # value row 1 -> 2 xn[1]
    w["w_o"][:] = [[1.0, 0.0], [0.0, 1.0]]
    w["w_gu"][0] = [1.0, 0.0]                   # gate
    w["w_gu"][1] = [0.0, 1.0]                   # up
    w["w_down"][:] = [[1.0], [-1.0]]
    kc = np.zeros((1, 1, 1, 4, 2))
    vc = np.zeros((1, 1, 1, 4, 2))
    out = od.decode_step(c, [w], dict(g=np.ones(2), w_lm=np.array([[1.0, 1.0]])), kc, vc, x, np.array([0]))
    q = od.q_bf16
    xn = q(np.array([3.0 * s, 4.0 * s]))
    attn = q(np.array([xn[0], 2.0 * xn[1]]))
    x1 = np.array([3.0 + attn[0], 4.0 + attn[1]])
    r = 1.0 / math.sqrt((x1[0] ** 2 + x1[1] ** 2) / 2.0)
    xn2 = q(x1 * r)
    gate, up = xn2[0], xn2[1]
    h = q(np.array([gate / (1.0 + math.exp(-gate)) * up]))[0]
    x2 = np.array([x1[0] + h, x1[1] - h])
    assert np.allclose(out["x_out"][0], x2, rtol=1e-15, atol=0)
    rf = 1.0 / math.sqrt((x2[0] ** 2 + x2[1] ** 2) / 2.0)
    xf = q(x2 * rf)
    assert np.allclose(out["logits"][0], [xf[0] + xf[1]], rtol=1e-15)
    assert np.array_equal(vc[0, 0, 0, 0], q(np.array([xn[0], 2.0 * xn[1]])))
    assert np.array_equal(kc[0, 0, 0, 0], q(np.array([xn[1], 0.0])))   # position 0: no rotation


def test_q_bf16_rounds_through_fp32():
    # 1 + 2^-8 + 2^-30 rounds to FP32 1 + 2^-8 (the 2^-30 is lost), a BF16
    # tie that goes to the even code 1.0; direct FP64 rounding would give
    # 1 + 2^-7
    v = 1.0 + 2.0 ** -8 + 2.0 ** -30
    assert od.q_bf16(np.array([v]))[0] == 1.0
    assert od.q_bf16(np.array([1.0 + 3 * 2.0 ** -8]))[0] == 1.0 + 2.0 ** -6
