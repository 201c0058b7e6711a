"""Pins of the CPU oracle against facts fixed outside it.

Each test checks the oracle (``oracle/``) against something other than its own
code: brute-force minimisation of Eq. 2 on tiny grids, scipy's independent
EDT, closed forms derived by hand from Algorithms 2-4 on 1-D and 2-D
examples, invariants of the construction, and the bound printed in Table II.
"""
import itertools
import json
import os

import numpy as np
import pytest
import scipy.ndimage

import oracle
from paper_2602_20097_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
ETA = float(np.float32(0.9))


# ---------------------------------------------------------------- brute force
def brute_edt(mask):
    """Eq. 2 by exhaustive search: squared distance to the nearest seed and the
    smallest linear index among all seeds at that distance (-1: no seed)."""
    m = np.asarray(mask, bool)
    shape = m.shape
    coords = np.stack(np.meshgrid(*[np.arange(s) for s in shape], indexing="ij"), -1).reshape(-1, 3)
    seeds = np.flatnonzero(m.ravel())
    if seeds.size == 0:
        return -np.ones(shape, np.int64), -np.ones(shape, np.int64)
    diff = coords[:, None, :] - coords[seeds][None, :, :]
    d2 = (diff * diff).sum(-1)
    best = d2.min(1)
    # seeds are enumerated in increasing linear index, so argmin picks the smallest
    feat = seeds[np.argmin(d2, axis=1)]
    return best.reshape(shape), feat.reshape(shape)


def random_shapes(rng, count):
    out = []
    for _ in range(count):
        out.append(tuple(int(v) for v in rng.integers(1, 8, size=3)))
    return out


# --------------------------------------------------------------------- EDT
@pytest.mark.parametrize("seed", range(6))
def test_edt_matches_brute_force_tiny(seed):
    rng = np.random.default_rng(seed)
    for shape in random_shapes(rng, 25):
        for density in (0.02, 0.15, 0.5):
            mask = rng.random(shape) < density
            d, f = oracle.edt(mask)
            bd, bf = brute_edt(mask)
            assert np.array_equal(d, bd), (shape, density)
            assert np.array_equal(f, bf), (shape, density)


def test_edt_ties_follow_linear_index_order():
    # (1,1) is at squared distance 2 from both (0,2) and (2,0); the smaller linear
    # index is (0,2) (row 0).  A pass order that resolved ties on x first would
    # pick (2,0) instead.
    m = np.zeros((1, 3, 3), np.uint8)
    m[0, 0, 2] = 1
    m[0, 2, 0] = 1
    d, f = oracle.edt(m)
    assert d[0, 1, 1] == 2
    assert f[0, 1, 1] == 2


def test_edt_matches_scipy_medium():
    rng = np.random.default_rng(7)
    for shape, dens in (((24, 31, 40), 0.003), ((1, 130, 97), 0.01), ((40, 1, 64), 0.02), ((17, 23, 1), 0.05)):
        mask = rng.random(shape) < dens
        mask.flat[rng.integers(mask.size)] = True
        d, _ = oracle.edt(mask)
        ref = scipy.ndimage.distance_transform_edt(~mask)
        assert np.array_equal(d, np.rint(ref * ref).astype(np.int64)), shape


def test_edt_one_dimensional_closed_form():
    # 1-D: the squared distance to the nearest seed, min((x - L)^2, (R - x)^2).
    rng = np.random.default_rng(3)
    n = 200
    mask = rng.random(n) < 0.05
    mask[[17, 150]] = True
    d, f = oracle.edt(mask[None, None, :])
    s = np.flatnonzero(mask)
    for x in range(n):
        dist = np.abs(s - x)
        assert d[0, 0, x] == dist.min() ** 2
        assert f[0, 0, x] == s[np.argmin(dist)]


def test_edt_no_seed_and_all_seeds():
    d, f = oracle.edt(np.zeros((3, 4, 5), np.uint8))
    assert (d == -1).all() and (f == -1).all()
    d, f = oracle.edt(np.ones((3, 4, 5), np.uint8))
    assert (d == 0).all() and np.array_equal(f.ravel(), np.arange(60))


# ----------------------------------------------------- hand-derived examples
def run1d(q, eb=0.5):
    xq = (2.0 * eb * np.asarray(q, np.float64)).astype(np.float32)
    return oracle.qai(xq[None, None, :], eb), xq


def test_w8_bands_closed_form():
    """1-D staircase q = floor(k/8), eb = 0.5 so x' = q (derivation: Algorithm 2
    marks the two voxels beside each step, the lower one +, the upper one -;
    Algorithm 1 gives distances to them; Algorithm 3 flips the sign halfway
    through a band; the IDW weight of Section V-E is d2 / (d1 + d2))."""
    n = 32
    k = np.arange(n)
    x = ((k - 3.5) / 8.0).astype(np.float32)
    q_gen = np.rint(x.astype(np.float64))
    assert np.array_equal(q_gen, k // 8)
    r, xq = run1d(q_gen)
    r = {kk: v[0, 0] for kk, v in r.items()}
    assert np.array_equal(np.flatnonzero(r["b1"]), [7, 8, 15, 16, 23, 24])
    sb = np.zeros(n, int)
    sb[[7, 15, 23]] = 1
    sb[[8, 16, 24]] = -1
    assert np.array_equal(r["sb"], sb)
    seeds = np.array([7, 8, 15, 16, 23, 24])
    d1 = np.array([np.abs(seeds - i).min() for i in k])
    near = np.array([seeds[np.argmin(np.abs(seeds - i))] for i in k])
    s = sb[near]
    assert np.array_equal(r["d1sq"], d1 ** 2)
    assert np.array_equal(r["s"], s)
    b2 = np.array([11, 12, 19, 20])
    assert np.array_equal(np.flatnonzero(r["b2"]), b2)
    d2 = np.array([np.abs(b2 - i).min() for i in k])
    assert np.array_equal(r["d2sq"], d2 ** 2)
    w = np.where(d1 == 0, 1.0, np.where(d2 == 0, 0.0, d2 / np.maximum(d1 + d2, 1)))
    C = w * s * ETA * 0.5
    np.testing.assert_allclose(r["out"], xq + C, rtol=0, atol=1e-15)
    # inside an interior band the compensation is the straight line through
    # -eta*eb at its lower boundary and +eta*eb at its upper one (Section V)
    band = np.arange(8, 16)
    np.testing.assert_allclose((r["out"] - xq)[band] / (ETA * 0.5),
                               [-1, -2 / 3, -1 / 3, 0, 0, 1 / 3, 2 / 3, 1], atol=1e-12)


def test_w5_tie_goes_to_lower_index():
    """1-D q = floor(k/5): voxel 7 is equidistant from boundary voxels 5 (S=-)
    and 9 (S=+).  Algorithm 1's strict query comparison keeps 5, so S[7] = -,
    B2 = {7, 8}; the other tie-break would give B2 = {6, 7}."""
    k = np.arange(15)
    x = ((k - 2) / 5.0).astype(np.float32)
    q_gen = np.rint(x.astype(np.float64))
    assert np.array_equal(q_gen, k // 5)
    r, xq = run1d(q_gen)
    r = {kk: v[0, 0] for kk, v in r.items()}
    assert np.array_equal(np.flatnonzero(r["b1"]), [4, 5, 9, 10])
    assert r["s"][7] == -1
    assert np.array_equal(np.flatnonzero(r["b2"]), [7, 8])
    C = (r["out"] - xq) / (ETA * 0.5)
    np.testing.assert_allclose(C[5:10], [-1, -0.5, 0, 0, 1], atol=1e-12)


def test_gradient_threshold_is_inclusive_and_absolute():
    """A one-voxel band: |q[+1] - q[-1]| = 2 gives a central difference of
    exactly 1.0, which Algorithm 2 (>= 1.0) treats as fast-varying: S = 0.
    The decreasing ramp checks the absolute value is used."""
    r, xq = run1d([0, 0, 0, 1, 2, 2, 2])
    sb = r["sb"][0, 0]
    assert np.array_equal(np.flatnonzero(r["b1"][0, 0]), [2, 3, 4])
    assert list(sb[2:5]) == [1, 0, -1]
    # no sign-flip boundary: w = 1 off B1 (1/k2 = 0), so C = S * eta * eb everywhere
    assert not r["b2"].any() and (r["d2sq"] == -1).all()
    np.testing.assert_allclose((r["out"] - xq)[0, 0] / (ETA * 0.5), [1, 1, 1, 0, -1, -1, -1], atol=1e-12)
    r, _ = run1d([2, 2, 2, 1, 0, 0, 0])
    assert list(r["sb"][0, 0][2:5]) == [-1, 0, 1]


def test_first_differing_neighbour_sets_the_sign_2d():
    """3x3 slice, centre q = 0 with its +x neighbour 1 and +y neighbour -1:
    both central differences are 0.5, so the sign stays; the first differing
    neighbour in the order +x, -x, +y, -y gives S = +."""
    q = np.zeros((1, 3, 3))
    q[0, 1, 2] = 1
    q[0, 2, 1] = -1
    xq = q.astype(np.float32)
    r = oracle.qai(xq, 0.5)
    assert r["b1"].sum() == 1 and r["b1"][0, 1, 1] == 1
    assert r["sb"][0, 1, 1] == 1
    # every voxel's nearest boundary is the centre; no B2; C = +eta*eb everywhere
    assert (r["s"] == 1).all()
    np.testing.assert_allclose(r["out"] - xq, ETA * 0.5, atol=1e-15)


def test_3d_extrusion_matches_1d():
    """A 3 x 3 x 32 block constant in y and z: only the centre line is interior,
    so its seeds and signs are the 1-D ones; off-line voxels add their squared
    offset to both distances."""
    k = np.arange(32)
    q1 = k // 8
    r1, xq1 = run1d(q1)
    q = np.broadcast_to(q1, (3, 3, 32)).astype(np.float64)
    xq = q.astype(np.float32)
    r = oracle.qai(xq, 0.5)
    for key in ("b1", "sb", "s", "b2", "d1sq", "d2sq", "out"):
        assert np.array_equal(r[key][1, 1], r1[key][0, 0]), key
    for z, y in itertools.product(range(3), range(3)):
        off = (z - 1) ** 2 + (y - 1) ** 2
        assert np.array_equal(r["d1sq"][z, y], r1["d1sq"][0, 0] + off)
        assert np.array_equal(r["d2sq"][z, y], r1["d2sq"][0, 0] + off)
        assert np.array_equal(r["s"][z, y], r1["s"][0, 0])
        assert not r["b1"][z, y].any() or (z, y) == (1, 1)


# ------------------------------------------------------------ invariants
def small_field(seed, shape=(24, 30, 36), beta=3.0, rel=1e-2):
    x = synth.grf(shape, beta, seed)
    return synth.quantize(x, rel)


@pytest.mark.parametrize("seed", [0, 1])
def test_invariants_on_smooth_fields(seed):
    x32, xq, q, eb = small_field(seed)
    r = oracle.qai(xq, eb)
    assert np.array_equal(r["q"], q)                       # Eq. 1 inverted exactly
    C = r["out"] - xq.astype(np.float64)
    e = ETA * eb
    assert np.abs(C).max() <= e * (1 + 1e-12)               # |C| <= eta eb
    assert np.abs(r["out"] - x32).max() <= (1 + ETA) * eb * (1 + 1e-6)  # relaxed bound
    assert np.array_equal(np.rint(r["out"] / (2 * eb)), q)  # re-quantizes to q
    on1 = r["b1"] == 1
    np.testing.assert_allclose(C[on1], r["sb"][on1] * e, rtol=1e-12, atol=0)
    assert (C[r["b2"] == 1] == 0).all()
    assert (C[r["s"] == 0] == 0).all()
    assert not (r["b1"].astype(bool) & r["b2"].astype(bool)).any()
    # the sign carried to each voxel is the boundary sign at I1
    valid = r["i1"] >= 0
    assert np.array_equal(r["s"][valid], r["sb"].ravel()[r["i1"][valid]])
    # I1 is a nearest boundary voxel
    idx = np.argwhere(valid)
    pos = np.stack(np.unravel_index(r["i1"][valid], xq.shape), -1)
    assert np.array_equal(((idx - pos) ** 2).sum(-1), r["d1sq"][valid])


def test_constant_field_is_unchanged():
    xq = np.full((9, 10, 11), 3.0, np.float32)
    r = oracle.qai(xq, 0.5)
    assert np.array_equal(r["out"], xq.astype(np.float64))
    assert not r["b1"].any() and (r["d1sq"] == -1).all() and (r["s"] == 0).all()


def test_negation_index_shift_and_scaling():
    _, xq, q, eb = small_field(5, shape=(20, 21, 22))
    base = oracle.qai(xq, eb)["out"]
    neg = oracle.qai(-xq, eb)["out"]
    assert np.array_equal(neg, -base)
    # integer-valued decompressed data with eb = 0.5: a shift of the indices by c
    # shifts the output by c and leaves the compensation unchanged
    xi = q.astype(np.float32)
    a = oracle.qai(xi, 0.5)
    b = oracle.qai(xi + 7, 0.5)
    for key in ("b1", "sb", "s", "b2", "d1sq", "d2sq", "w"):
        assert np.array_equal(a[key], b[key]), key
    np.testing.assert_allclose(a["out"] + 7, b["out"], rtol=0, atol=1e-12)
    # power-of-two scaling of data and bound scales the output
    s4 = oracle.qai(xq * 4, eb * 4)["out"]
    assert np.array_equal(s4, base * 4)


def test_edge_voxels_are_never_boundaries():
    _, xq, _, eb = small_field(9, shape=(12, 13, 14), rel=5e-3)
    r = oracle.qai(xq, eb)
    for arr in (r["b1"], r["b2"]):
        assert not arr[0].any() and not arr[-1].any()
        assert not arr[:, 0].any() and not arr[:, -1].any()
        assert not arr[:, :, 0].any() and not arr[:, :, -1].any()


def test_table2_relaxed_bound():
    """Table II prints the maximum relative error of the compensated data at
    eps = 1e-3: 0.0019 for every field, i.e. (1 + eta) eps.  The oracle must
    stay within it on smooth synthetic fields and, like the paper's fields,
    come close to it."""
    with open(os.path.join(GOLDEN, "table2_max_rel_error.json")) as fh:
        g = json.load(fh)
    eps = g["eps"]
    bound = max(g["ours"].values())
    assert abs(bound - (1 + g["eta"]) * eps) < 1e-9
    worst = 0.0
    for seed in range(3):
        x = synth.grf((48, 48, 48), 3.0, 100 + seed)
        x32, xq, q, eb = synth.quantize(x, eps)
        rng_ = float(x32.max()) - float(x32.min())
        r = oracle.qai(xq, eb)
        rel = np.abs(r["out"] - x32).max() / rng_
        assert rel <= bound * (1 + 1e-5)
        worst = max(worst, rel)
    assert worst >= 0.9 * bound


# ------------------------------------------------- generalised IDW power p
def test_idw_power_closed_forms_on_the_w8_bands():
    """Step E's weight generalised to w = k1^-p / (k1^-p + k2^-p) (the
    differentiable form; p = 1 is Section V-E).  Inside an interior band of the
    W = 8 staircase the distances are d1 = (0,1,2,3,3,2,1,0) and
    d2 = (3,2,1,0,0,1,2,3) (test_w8_bands_closed_form), so for p = 2 the weight
    is d2^2 / (d1^2 + d2^2) = (1, 4/5, 1/5, 0, 0, 1/5, 4/5, 1) and for p = 1/2
    it is sqrt(d2) / (sqrt(d1) + sqrt(d2)); p = 1 gives the default call."""
    n = 32
    k = np.arange(n)
    q = k // 8
    xq = q.astype(np.float32)[None, None, :]
    band = np.arange(8, 16)
    s_band = np.array([-1, -1, -1, -1, 1, 1, 1, 1])
    d1 = np.array([0, 1, 2, 3, 3, 2, 1, 0], float)
    d2 = np.array([3, 2, 1, 0, 0, 1, 2, 3], float)
    with np.errstate(divide="ignore", invalid="ignore"):
        expect = {
            2.0: np.array([1, 4 / 5, 1 / 5, 0, 0, 1 / 5, 4 / 5, 1]),
            0.5: np.where(d1 == 0, 1.0, np.where(d2 == 0, 0.0, np.sqrt(d2) / (np.sqrt(d1) + np.sqrt(d2)))),
            1.0: np.where(d1 == 0, 1.0, np.where(d2 == 0, 0.0, d2 / (d1 + d2))),
        }
    default = oracle.qai(xq, 0.5)
    for p, w in expect.items():
        for eta in (0.9, 0.5):
            r = oracle.qai(xq, 0.5, eta, p)
            np.testing.assert_allclose(r["w"][0, 0, band], w, rtol=0, atol=1e-15)
            e = float(np.float32(eta)) * 0.5
            np.testing.assert_allclose(r["out"][0, 0, band] - xq[0, 0, band], w * s_band * e, rtol=0, atol=1e-15)
    assert np.array_equal(oracle.qai(xq, 0.5, 0.9, 1.0)["out"], default["out"])


def test_idw_power_symmetry_and_limits():
    """For every p, swapping the two distances turns w into 1 - w, equal
    distances give w = 1/2, and w grows with p where k1 < k2 (it tends to the
    nearest-boundary indicator as p grows).  Checked on a smooth field, where
    the pairs (k1, k2) come from the oracle's own transforms."""
    x32, xq, q, eb = small_field(3)
    base = oracle.qai(xq, eb)
    d1, d2 = base["d1sq"].astype(float), base["d2sq"].astype(float)
    gen = (d1 > 0) & (d2 > 0)
    assert gen.sum() > 100
    k1, k2 = np.sqrt(d1[gen]), np.sqrt(d2[gen])
    prev = None
    for p in (0.25, 0.5, 1.0, 2.0, 4.0):
        w = oracle.qai(xq, eb, 0.9, p)["w"][gen]
        # the weight depends on k1/k2 only: w = 1 / (1 + (k1/k2)^p)
        np.testing.assert_allclose(w, 1.0 / (1.0 + (k1 / k2) ** p), rtol=1e-12, atol=0)
        np.testing.assert_allclose(w[k1 == k2], 0.5, rtol=0, atol=1e-15)
        if prev is not None:
            closer = k1 < k2
            assert (w[closer] >= prev[closer] - 1e-15).all()
            assert (w[~closer & (k1 != k2)] <= prev[~closer & (k1 != k2)] + 1e-15).all()
        prev = w
    # the p = 1 weight of Section V-E, (1/k1) / (1/k1 + 1/k2) = k2 / (k1 + k2)
    np.testing.assert_allclose(base["w"][gen], k2 / (k1 + k2), rtol=1e-12, atol=0)
