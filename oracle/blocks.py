"""Block-decomposed variants of the post-pass (the paper's distributed-memory
strategies, Section VI-B), written out on the CPU -- TEST INFRASTRUCTURE
ONLY.  Shares nothing with the GPU library.

The field is cut into a grid of blocks (extents split as evenly as possible,
the first blocks taking one voxel more).  Three strategies:

* embarrassingly parallel (``ep``): every block runs the whole algorithm on
  its own voxels (its faces are domain edges);
* approximate (``approximate``): a block sees one ghost layer of its
  neighbours' voxels in two rounds of stencil exchange -- the quantization
  indices for the boundary stencil of step A, then the propagated signs S of
  step B (computed by the neighbour on its own data) for the sign-flip
  stencil of step C -- while both EDTs stay local to the block;
* exact: the whole-field result (``oracle.qai``).

Each block is processed on its ghosted region (the block plus one layer on
every face that has a neighbour).  Ghost voxels lie on the edge of that region,
so Algorithm 2's edge rule keeps them out of B1 and B2 and only real voxels
are sites; real voxels on an inner face are interior and see their neighbours.
Steps A, B and D use the oracle's C routines (Algorithm 2, Algorithm 1 with
features); steps C and E are the paper's definitions in numpy.
"""
from __future__ import annotations

import numpy as np

from . import boundary_sign, edt, qai, recover_q


def block_bounds(n, k):
    """Origins and extents of k blocks over an axis of n voxels."""
    base, extra = divmod(n, k)
    ext = [base + (1 if i < extra else 0) for i in range(k)]
    org = np.concatenate([[0], np.cumsum(ext)[:-1]]).astype(int).tolist()
    return list(zip(org, ext))


def _grid(shape, blocks):
    axes = [block_bounds(n, k) for n, k in zip(shape, blocks)]
    out = []
    for iz, (oz, ez) in enumerate(axes[0]):
        for iy, (oy, ey) in enumerate(axes[1]):
            for ix, (ox, ex) in enumerate(axes[2]):
                out.append(((iz, iy, ix), (oz, oy, ox), (ez, ey, ex)))
    return out


def _ghosted(shape, org, ext, ghost):
    """Slices of the ghosted region in the field and of the real voxels in it."""
    lo = [max(0, o - ghost) if o > 0 else o for o in org]
    hi = [min(n, o + e + ghost) if o + e < n else o + e for n, o, e in zip(shape, org, ext)]
    region = tuple(slice(a, b) for a, b in zip(lo, hi))
    inner = tuple(slice(o - a, o - a + e) for o, a, e in zip(org, lo, ext))
    return region, inner


def _interior(shape):
    """Voxels interior on every axis of extent > 1 (Algorithm 2's edge rule)."""
    m = np.ones(shape, bool)
    for ax, n in enumerate(shape):
        if n > 1:
            idx = [slice(None)] * 3
            idx[ax] = 0
            m[tuple(idx)] = False
            idx[ax] = n - 1
            m[tuple(idx)] = False
    return m


def _flip_boundary(s, b1):
    """Step C (Algorithm 3): interior voxels off B1 with some 6-neighbour of
    another sign."""
    diff = np.zeros(s.shape, bool)
    for ax, n in enumerate(s.shape):
        if n < 2:
            continue
        a = [slice(None)] * 3
        b = [slice(None)] * 3
        a[ax], b[ax] = slice(1, None), slice(None, -1)
        ne = s[tuple(a)] != s[tuple(b)]
        diff[tuple(a)] |= ne
        diff[tuple(b)] |= ne
    return diff & _interior(s.shape) & (b1 == 0)


def _step_e(xq, s, d1sq, d2sq, eb, eta):
    """Step E (Section V): w = k2 / (k1 + k2) with w = 1 on B1 or without
    B2, w = 0 on B2; out = x' + w S eta eb (FP64)."""
    d1 = d1sq.astype(np.float64)
    d2 = d2sq.astype(np.float64)
    w = np.zeros(xq.shape)
    gen = (d1 > 0) & (d2 > 0)
    k1, k2 = np.sqrt(d1[gen]), np.sqrt(d2[gen])
    w[gen] = k2 / (k1 + k2)
    w[d2 < 0] = 1.0
    w[d1 == 0] = 1.0
    w[d2 == 0] = np.where(d1[d2 == 0] == 0, 1.0, 0.0)
    eta = float(np.float32(eta))
    return xq.astype(np.float64) + w * s.astype(np.float64) * eta * float(np.float32(eb))


def ep(xq, eb, blocks, eta=0.9):
    """Embarrassingly parallel: the oracle on every block alone."""
    xq = np.asarray(xq, np.float32)
    out = np.empty(xq.shape, np.float64)
    for _, org, ext in _grid(xq.shape, blocks):
        sl = tuple(slice(o, o + e) for o, e in zip(org, ext))
        out[sl] = qai(np.ascontiguousarray(xq[sl]), eb, eta)["out"]
    return out


def approximate(xq, eb, blocks, eta=0.9, taps=False):
    """Approximate: one-layer exchanges of q (step A) and S (step C), local
    EDTs.  Returns out (float64), and with ``taps`` a dict of the per-voxel
    b1, sb, s, b2, d1sq, d2sq of every block's real voxels."""
    xq = np.asarray(xq, np.float32)
    shape = xq.shape
    q = recover_q(xq, eb)
    grid = _grid(shape, blocks)
    parts = []
    s_global = np.zeros(shape, np.int8)
    for _, org, ext in grid:
        region, inner = _ghosted(shape, org, ext, 1)
        qb = np.ascontiguousarray(q[region])
        b1, sb = boundary_sign(qb)                       # step A on the ghosted region
        d1sq, i1 = edt(b1)                               # step B, local to the block
        s = np.zeros(qb.shape, np.int8)
        has = i1 >= 0
        s[has] = sb.reshape(-1)[i1[has]]                 # S = S_B[I1] (Algorithm 3)
        real = tuple(slice(o, o + e) for o, e in zip(org, ext))
        s_global[real] = s[inner]
        parts.append((region, inner, real, b1, sb, s, d1sq))
    out = np.empty(shape, np.float64)
    tp = {k: np.zeros(shape, np.int64) for k in ("b1", "sb", "s", "b2", "d1sq", "d2sq")} if taps else None
    for region, inner, real, b1, sb, s, d1sq in parts:
        sx = s_global[region].copy()                     # ghost layer: the neighbours' S
        sx[inner] = s[inner]
        b2 = _flip_boundary(sx, b1).astype(np.uint8)     # step C with the exchanged signs
        d2sq, _ = edt(b2)                                # step D, local
        ob = _step_e(xq[region], sx, d1sq, d2sq, eb, eta)
        out[real] = ob[inner]
        if taps:
            for k, v in (("b1", b1), ("sb", sb), ("s", sx), ("b2", b2), ("d1sq", d1sq), ("d2sq", d2sq)):
                tp[k][real] = v[inner]
    return (out, tp) if taps else out
