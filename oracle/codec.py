"""Decoder of the segment code of quantization indices (the producer is
``paper_2602_20097_amd.synth.encode_indices``) -- TEST INFRASTRUCTURE ONLY.
Shares nothing with the GPU library.

Each x-row is cut into segments of 32 voxels; a segment holds its first index
(base), the width b of its differences and 31 zigzag-coded differences to the
prior value, b bits each, LSB-first from the first bit of its payload words
(meta = first word << 8 | b).  Decoding is the prediction from one prior
value (Section III-A) undone: q_0 = base, q_i = q_{i-1} + unzigzag(code_i).
"""
from __future__ import annotations

import numpy as np


def _bits(payload, word, bit, width):
    """width bits of the payload starting at bit ``bit`` of word ``word``."""
    v = 0
    for k in range(width):
        w = word + (bit + k) // 32
        v |= ((int(payload[w]) >> ((bit + k) % 32)) & 1) << k
    return v


def decode_indices(code, shape):
    """Plain segment-by-segment decoder: returns int64 indices of ``shape``."""
    nz, ny, nx = shape
    seg_len = int(code["seg_len"])
    s_row = -(-nx // seg_len)
    base, meta, payload = code["base"], code["meta"], code["payload"]
    out = np.empty((nz * ny, nx), np.int64)
    for row in range(nz * ny):
        for s in range(s_row):
            k = row * s_row + s
            b = int(meta[k]) & 0xFF
            off = int(meta[k]) >> 8
            q = int(base[k])
            vals = [q]
            for i in range(1, seg_len):
                z = _bits(payload, off, (i - 1) * b, b)
                q += (z >> 1) ^ -(z & 1)
                vals.append(q)
            x0 = s * seg_len
            n = min(seg_len, nx - x0)
            out[row, x0:x0 + n] = vals[:n]
    return out.reshape(shape)


def decode_indices_fast(code, shape):
    """The same, vectorised over segments (for medium fields)."""
    nz, ny, nx = shape
    seg_len = int(code["seg_len"])
    s_row = -(-nx // seg_len)
    base = code["base"].astype(np.int64)
    meta = code["meta"].astype(np.uint64)
    payload = code["payload"].astype(np.uint64)
    b = (meta & np.uint64(0xFF)).astype(np.int64)
    off = (meta >> np.uint64(8)).astype(np.int64)
    i = np.arange(1, seg_len)
    pos = off[:, None] * 32 + (i[None, :] - 1) * b[:, None]
    w = np.minimum(pos // 32, len(payload) - 2)   # a width-0 segment reads nothing (its mask is 0)
    sh = (pos % 32).astype(np.uint64)
    two = payload[w] | (payload[w + 1] << np.uint64(32))
    mask = (np.uint64(1) << b.astype(np.uint64)) - np.uint64(1)
    z = ((two >> sh) & mask[:, None]).astype(np.int64)
    r = (z >> 1) ^ -(z & 1)
    q = np.concatenate([base[:, None], base[:, None] + np.cumsum(r, axis=1)], axis=1)
    q = q.reshape(nz * ny, s_row * seg_len)[:, :nx]
    return q.reshape(shape)
