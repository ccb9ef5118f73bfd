"""CPU oracle of the synthetic decode-step victim.

TEST INFRASTRUCTURE ONLY: plain, slow and obviously correct; used by the
tests, the smoke check and the benchmark's CPU leg, never by the device
library, and it never imports it.

The paper's end-to-end victims are LLM decode steps (Llama 3.1 8B and
Gemma 3 1B served by vLLM; Sections 4.2-4.4, with the per-kernel latency
breakdown of one decode step in Fig. 5).  Their weights and the serving
fork are not available, so the victim stands in for them with one decode
step of a Llama-style decoder with random weights.  The paper does not
define the model, so this module writes out the standard definitions the
stand-in follows (each function states its own):

  * RMS normalisation with a learned gain,
  * rotary position embedding, rotate-half form,
  * grouped-query attention over a key/value cache, softmax scaled by
    1/sqrt(head_dim), query head h reading key/value head h // group,
  * gated MLP with the SiLU activation (x * sigmoid(x)),
  * residual connections around attention and MLP, a final
    normalisation and an output projection to the vocabulary.

Arithmetic is FP64.  The device rounds to BF16 at four points of the step
(normalised activations, the key/value entries it appends to the cache,
the attention output, the MLP activation); the oracle rounds at the same
points, from FP64 through FP32 to BF16, so that both sides feed the same
BF16 values to the next product except where the last FP32 bit decides a
rounding.

Parity status (pins in tests/test_oracle_decode.py):
  rmsnorm, rope, attention_decode, silu_mul, decode_step ...... pinned
"""
from __future__ import annotations

import math

import numpy as np

from . import bf16_to_f64, f32_to_bf16


def q_bf16(v) -> np.ndarray:
    """Round FP64 values to FP32, then to BF16 (nearest, ties to even), and
    return the BF16 values as FP64."""
    v = np.asarray(v, dtype=np.float64)
    return bf16_to_f64(f32_to_bf16(v.astype(np.float32))).reshape(v.shape)


def rmsnorm(x, g, eps: float) -> np.ndarray:
    """y = x / sqrt(mean(x^2) + eps) * g over the last axis."""
    x = np.asarray(x, dtype=np.float64)
    ms = np.mean(x * x, axis=-1, keepdims=True)
    return x / np.sqrt(ms + eps) * np.asarray(g, dtype=np.float64)


def rope_angles(pos: int, head_dim: int, base: float) -> np.ndarray:
    """Angle of pair i (0 <= i < head_dim/2) at position pos:
    pos * base^(-2i/head_dim)."""
    i = np.arange(head_dim // 2, dtype=np.float64)
    return float(pos) * np.power(float(base), -2.0 * i / head_dim)


def rope(x, pos: int, base: float) -> np.ndarray:
    """Rotary embedding, rotate-half form: element i and element
    i + head_dim/2 of each head form a pair rotated by angle i."""
    x = np.asarray(x, dtype=np.float64)
    d = x.shape[-1]
    h = d // 2
    a = rope_angles(pos, d, base)
    c, s = np.cos(a), np.sin(a)
    x1, x2 = x[..., :h], x[..., h:]
    return np.concatenate([x1 * c - x2 * s, x2 * c + x1 * s], axis=-1)


def attention_decode(q, k, v) -> np.ndarray:
    """One query per head against t cached positions.
    q: [n_q, d]; k, v: [n_kv, t, d]; query head h uses key/value head
    h // (n_q / n_kv).  Returns [n_q, d]."""
    q = np.asarray(q, dtype=np.float64)
    k = np.asarray(k, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    nq, d = q.shape
    group = nq // k.shape[0]
    out = np.empty((nq, d))
    for h in range(nq):
        kv = h // group
        s = k[kv] @ q[h] / math.sqrt(d)
        p = np.exp(s - s.max())
        p /= p.sum()
        out[h] = p @ v[kv]
    return out


def silu_mul(gate, up) -> np.ndarray:
    """SiLU(gate) * up with SiLU(x) = x / (1 + exp(-x))."""
    gate = np.asarray(gate, dtype=np.float64)
    return gate / (1.0 + np.exp(-gate)) * np.asarray(up, dtype=np.float64)


def decode_step(cfg: dict, layers: list, final: dict, kcache, vcache, x_in, pos) -> dict:
    """One decode step for a batch of sequences.

    cfg: hidden, n_q, n_kv, head_dim, ffn, vocab, eps, rope_base.
    layers[l]: FP64 values of the BF16 weights
        g_attn [hidden], w_qkv [(n_q + 2 n_kv) head_dim, hidden],
        w_o [hidden, n_q head_dim], g_mlp [hidden], w_gu [2 ffn, hidden]
        (gate rows, then up rows), w_down [hidden, ffn].
    final: g [hidden], w_lm [vocab, hidden] (vocab may be 0).
    kcache, vcache: [layers, batch, n_kv, max_ctx, head_dim] FP64 values of
        the BF16 cache; entry pos[b] of sequence b is written by this step
        (the arrays are updated in place, as the device's cache is).
    x_in: [batch, hidden] residual-stream input.
    pos: [batch] position of the new token; it attends to 0 .. pos[b].

    Returns the final residual stream, the logits and, per layer, the
    intermediates the per-kernel tests compare."""
    hid, nq, nkv, d, ffn = cfg["hidden"], cfg["n_q"], cfg["n_kv"], cfg["head_dim"], cfg["ffn"]
    eps, base = cfg["eps"], cfg["rope_base"]
    x = np.asarray(x_in, dtype=np.float64).copy()
    batch = x.shape[0]
    trace = []
    for li, w in enumerate(layers):
        st = {}
        xn = q_bf16(rmsnorm(x, w["g_attn"], eps))
        qkv = xn @ w["w_qkv"].T
        q = qkv[:, :nq * d].reshape(batch, nq, d)
        k = qkv[:, nq * d:(nq + nkv) * d].reshape(batch, nkv, d)
        v = qkv[:, (nq + nkv) * d:].reshape(batch, nkv, d)
        o = np.empty((batch, nq, d))
        qr = np.empty_like(q)
        for b in range(batch):
            p = int(pos[b])
            qr[b] = rope(q[b], p, base)
            kcache[li, b, :, p, :] = q_bf16(rope(k[b], p, base))
            vcache[li, b, :, p, :] = q_bf16(v[b])
            o[b] = attention_decode(qr[b], kcache[li, b, :, :p + 1, :], vcache[li, b, :, :p + 1, :])
        o = q_bf16(o.reshape(batch, nq * d))
        x = x + o @ w["w_o"].T
        xn2 = q_bf16(rmsnorm(x, w["g_mlp"], eps))
        gu = xn2 @ w["w_gu"].T
        h = q_bf16(silu_mul(gu[:, :ffn], gu[:, ffn:]))
        x_mid = x
        x = x + h @ w["w_down"].T
        st.update(xn=xn, qkv=qkv, q_rot=qr, attn=o, x_attn=x_mid, xn_mlp=xn2, gu=gu, h=h, x_out=x.copy())
        trace.append(st)
    xf = q_bf16(rmsnorm(x, final["g"], eps))
    logits = xf @ final["w_lm"].T if final["w_lm"].shape[0] else np.zeros((batch, 0))
    return {"x_out": x, "logits": logits, "xn_final": xf, "layers": trace}
