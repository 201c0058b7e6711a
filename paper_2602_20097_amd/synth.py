"""Seeded synthetic inputs for the QAI post-pass.

This module only *produces* inputs: smooth random fields and their
pre-quantized (decompressed) form.  It holds none of the post-pass
arithmetic, imports neither the GPU binding nor the CPU oracle, and is the
one module both of them are fed from.

Pre-quantization follows the paper's Eq. 1 (Section III-A): an index
``q = round(x / 2eb)`` per value and the decompressed value ``x' = 2 eb q``,
so that ``|x - x'| <= eb``.  The error bound is value-range relative
(Section VII-B): ``eb = rel * (max x - min x)``.

Field recipes (the paper's datasets are not available, so these stand in
for them at the datasets' shapes, Table I):

* ``grf(shape, beta, seed)`` -- Gaussian random field whose Fourier
  *amplitude* falls as ``|k|^-beta`` (``|k|`` in cycles per voxel, the
  zero mode removed), normalised to zero mean and unit standard deviation.
* ``fourier_modes(shape, n_modes, seed)`` -- a sum of random plane waves
  with integer wave-vector components uniform in [-16, 16] (cycles per
  domain length, ``k != 0``), amplitude ``|k|^-2`` and uniform random phase,
  normalised, plus white noise of 1% of the field's standard deviation.
"""
from __future__ import annotations

import numpy as np

try:  # multi-threaded FFTs when scipy is present; numpy otherwise
    import scipy.fft as _fft

    def _rfftn(a):
        return _fft.rfftn(a, workers=-1)

    def _irfftn(a, s):
        return _fft.irfftn(a, s=s, workers=-1)
except Exception:  # pragma: no cover
    def _rfftn(a):
        return np.fft.rfftn(a)

    def _irfftn(a, s):
        return np.fft.irfftn(a, s=s)

SEED_BASE = 2602020097


def _as3(shape):
    shape = tuple(int(s) for s in shape)
    if len(shape) == 1:
        shape = (1, 1) + shape
    elif len(shape) == 2:
        shape = (1,) + shape
    if len(shape) != 3 or min(shape) < 1:
        raise ValueError(f"bad shape {shape}")
    return shape


def _normalise(x):
    x = x - x.mean()
    s = x.std()
    return x / s if s > 0 else x


def grf(shape, beta, seed):
    """Gaussian random field, amplitude spectrum ``|k|^-beta``; float64."""
    shape = _as3(shape)
    rng = np.random.default_rng(seed)
    white = rng.standard_normal(shape)
    spec = _rfftn(white)
    del white
    kz = np.fft.fftfreq(shape[0])[:, None, None]
    ky = np.fft.fftfreq(shape[1])[None, :, None]
    kx = np.fft.rfftfreq(shape[2])[None, None, :]
    k2 = kz * kz + ky * ky + kx * kx
    with np.errstate(divide="ignore"):
        amp = np.where(k2 > 0, k2 ** (-0.5 * beta), 0.0)
    del k2
    spec *= amp
    del amp
    x = _irfftn(spec, shape)
    return _normalise(x)


def fourier_modes(shape, n_modes=64, seed=0, kmax=16, noise=0.01):
    """Sum of ``n_modes`` random plane waves plus white noise; float64."""
    shape = _as3(shape)
    rng = np.random.default_rng(seed)
    spec = np.zeros(shape[:2] + (shape[2] // 2 + 1,), dtype=np.complex128)
    placed = 0
    while placed < n_modes:
        k = rng.integers(-kmax, kmax + 1, size=3)
        # axes of extent 1 carry no oscillation
        for a in range(3):
            if shape[a] == 1:
                k[a] = 0
        if not k.any():
            continue
        phase = rng.uniform(0.0, 2.0 * np.pi)
        amp = float(np.dot(k, k)) ** -1.0          # |k|^-2
        # keep the half-spectrum index with kx >= 0 (the mirror mode is implied)
        if k[2] < 0 or (k[2] == 0 and (k[1] < 0 or (k[1] == 0 and k[0] < 0))):
            k = -k
            phase = -phase
        iz, iy, ix = int(k[0]) % shape[0], int(k[1]) % shape[1], int(k[2])
        spec[iz, iy, ix] += amp * np.exp(1j * phase)
        placed += 1
    x = _irfftn(spec, shape)
    x = _normalise(x)
    x += noise * rng.standard_normal(shape)
    return _normalise(x)


def quantize(x, rel_eb):
    """Pre-quantize an original field (Eq. 1).

    Returns ``(x32, xq, q, eb)``: the original as float32, the decompressed
    float32 field ``2 eb q``, the int32 indices, and the absolute bound as a
    Python float holding an exact float32 value.
    """
    x32 = np.ascontiguousarray(x, dtype=np.float32)
    lo, hi = float(x32.min()), float(x32.max())
    eb = float(np.float32(rel_eb * (hi - lo)))
    if not eb > 0:
        raise ValueError("field has zero range; relative error bound undefined")
    q64 = np.rint(x32.astype(np.float64) / (2.0 * eb))
    if np.abs(q64).max() > 2 ** 21:
        raise ValueError("quantization index exceeds 2^21")
    q = q64.astype(np.int32)
    # decompression from the integer index (a zero index gives +0, as any
    # decoder of the indices does; the FP64 product is exact, rounded once)
    xq = (2.0 * eb * q.astype(np.float64)).astype(np.float32)
    return x32, xq, q, eb


# Named workloads: the shapes of the paper's datasets (Table I) and of its
# per-rank 512^3 blocks (Section VII-E2), filled with synthetic fields.
WORKLOADS = {
    "grf64_k3_eb1e-2": dict(shape=(64, 64, 64), kind="grf", beta=3.0, rel=1e-2, wid=1),
    "modes256x384x384_eb1e-4": dict(shape=(256, 384, 384), kind="modes", rel=1e-4, wid=2),
    "modes256x384x384_eb1e-3": dict(shape=(256, 384, 384), kind="modes", rel=1e-3, wid=2),
    "modes256x384x384_eb1e-2": dict(shape=(256, 384, 384), kind="modes", rel=1e-2, wid=2),
    "grf512_k11/3_eb1e-3": dict(shape=(512, 512, 512), kind="grf", beta=11.0 / 3.0, rel=1e-3, wid=3),
    "grf2d_1800x3600_k11/3_eb1e-3": dict(shape=(1, 1800, 3600), kind="grf", beta=11.0 / 3.0, rel=1e-3, wid=4),
    "grf256_k3_eb5e-3": dict(shape=(256, 256, 256), kind="grf", beta=3.0, rel=5e-3, wid=6),
}


def make_workload(name, seed_offset=0):
    """Build a named workload: returns ``(x32, xq, q, eb)``."""
    w = WORKLOADS[name]
    seed = SEED_BASE + w["wid"] + seed_offset
    if w["kind"] == "grf":
        x = grf(w["shape"], w["beta"], seed)
    else:
        x = fourier_modes(w["shape"], 64, seed)
    return quantize(x, w["rel"])


def batch_specs(seed=SEED_BASE + 5):
    """The 48-field uneven batch: 16 each of 100x500x500, 256x384x384 and
    128x128x1024, spectral exponent uniform in [2, 4] and relative bound
    log-uniform in [1e-4, 1e-2] per field.  Returns a list of dicts."""
    rng = np.random.default_rng(seed)
    shapes = [(100, 500, 500)] * 16 + [(256, 384, 384)] * 16 + [(128, 128, 1024)] * 16
    out = []
    for i, s in enumerate(shapes):
        out.append(dict(shape=s, beta=float(rng.uniform(2.0, 4.0)),
                        rel=float(10.0 ** rng.uniform(-4.0, -2.0)), seed=int(seed * 100 + i)))
    return out


def make_batch_field(spec):
    x = grf(spec["shape"], spec["beta"], spec["seed"])
    return quantize(x, spec["rel"])


# ------------------------------------------------------------- coded indices
# A simple pre-quantization code of the index array (the paper's Section
# III-A: the indices are predicted and encoded losslessly; its cuSZp
# comparison predicts from one prior value and uses fixed-length codes).
# Each x-row is cut into segments of SEG = 32 voxels (the last one padded by
# repeating the row's last value).  A segment stores its first index (base),
# the width b (0..32 bits) of its 31 zigzag-coded differences to the prior
# value, and those differences packed LSB-first from bit 0 of its own run of
# 32-bit payload words; meta = (first payload word << 8) | b.  The payload
# ends with one spare zero word, so a decoder may read two words from any
# difference's first word.  This module only produces code from indices; it
# decodes nothing.
SEG = 32


def encode_indices(q):
    """Encode an int32 index array ``(nz, ny, nx)``: returns a dict with
    ``base`` (int32[n_seg]), ``meta`` (uint64[n_seg]), ``payload``
    (uint32[words + 1]), ``seg_len`` and the compressed size in bytes."""
    q = np.asarray(q, dtype=np.int64)
    if q.ndim != 3:
        q = q.reshape((1,) * (3 - q.ndim) + q.shape)
    nz, ny, nx = q.shape
    s_row = -(-nx // SEG)
    rows = q.reshape(-1, nx)
    pad = s_row * SEG - nx
    if pad:
        rows = np.concatenate([rows, np.repeat(rows[:, -1:], pad, axis=1)], axis=1)
    seg = rows.reshape(-1, SEG)
    base = seg[:, 0].astype(np.int32)
    r = np.diff(seg, axis=1)                                  # 31 differences to the prior value
    z = ((r << 1) ^ (r >> 63)).astype(np.uint64)              # zigzag: small magnitudes, small codes
    zmax = z.max(axis=1)
    b = np.zeros(len(seg), np.int64)
    nzm = zmax > 0
    b[nzm] = np.floor(np.log2(zmax[nzm].astype(np.float64))).astype(np.int64) + 1
    # guard the float log at powers of two
    b[nzm] += (zmax[nzm] >> b[nzm].astype(np.uint64)) > 0
    b[nzm] -= (zmax[nzm] >> (b[nzm] - 1).astype(np.uint64)) == 0
    words = (31 * b + 31) // 32
    off = np.zeros(len(seg), np.int64)
    off[1:] = np.cumsum(words)[:-1]
    total = int(words.sum())
    payload = np.zeros(total + 1, np.uint32)
    for width in np.unique(b[b > 0]):
        idx = np.nonzero(b == width)[0]
        bits = ((z[idx][:, :, None] >> np.arange(width, dtype=np.uint64)) & 1).astype(np.uint8)
        bits = bits.reshape(len(idx), 31 * width)
        nw = (31 * width + 31) // 32
        bits = np.concatenate([bits, np.zeros((len(idx), nw * 32 - 31 * width), np.uint8)], axis=1)
        packed = np.packbits(bits.reshape(len(idx), nw, 32), axis=2, bitorder="little")
        wv = packed.view("<u4").reshape(len(idx), nw)
        payload[(off[idx][:, None] + np.arange(nw)).ravel()] = wv.ravel()
    meta = ((off.astype(np.uint64) << np.uint64(8)) | b.astype(np.uint64)).astype(np.uint64)
    nbytes = base.nbytes + meta.nbytes + payload.nbytes
    return dict(base=base, meta=meta, payload=payload, seg_len=SEG, shape=(nz, ny, nx), nbytes=nbytes)
