"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Bit-exact for the indices, masks, signs and squared distances; the
compensated output within 1e-6 * max(|out_oracle|, eb), the FP32-vs-FP64
tolerance derived in the design notes (FP32 relative error of C is a few
ulp of |C| <= 0.9 eb, plus half an ulp of |out| from the final add)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2602_20097_amd import synth

from _parity import KEYS, assert_parity, gpu_run

pytestmark = pytest.mark.gpu


def test_w1_grf64():
    x32, xq, q, eb = synth.make_workload("grf64_k3_eb1e-2")
    g, _ = assert_parity(xq, eb, label="grf64")
    assert np.array_equal(g["q"], q)


@pytest.mark.parametrize("seed", range(4))
def test_random_tiny_grids(seed):
    rng = np.random.default_rng(1000 + seed)
    for it in range(30):
        shape = tuple(int(v) for v in rng.integers(1, 9, size=3))
        levels = int(rng.integers(1, 5))
        q = rng.integers(-levels, levels + 1, size=shape)
        xq = (q * 1.0).astype(np.float32)
        assert_parity(xq, 0.5, label=f"tiny{seed}.{it}")


def test_hand_examples():
    k = np.arange(32)
    for q in (k // 8, (np.arange(15) // 5), np.array([0, 0, 0, 1, 2, 2, 2]), np.array([2, 2, 2, 1, 0, 0, 0])):
        assert_parity(q.astype(np.float32)[None, None, :], 0.5, label="1d")
        assert_parity(q.astype(np.float32)[None, :, None], 0.5, label="1d-y")
        assert_parity(q.astype(np.float32)[:, None, None], 0.5, label="1d-z")
    q = np.zeros((1, 3, 3))
    q[0, 1, 2] = 1
    q[0, 2, 1] = -1
    assert_parity(q.astype(np.float32), 0.5, label="corner")
    assert_parity(np.broadcast_to(k // 8, (3, 3, 32)).astype(np.float32).copy(), 0.5, label="extrusion")


# (75, 48, 64): planes of whole waves of the streaming kernel (12 per plane) with a
# partial group of 8 and a partial chunk of planes in the needed-voxel search
SHAPES = [(5, 70, 130), (3, 65, 200), (1, 1, 1000), (1, 300, 1), (17, 1, 129), (9, 33, 1), (2, 2, 2),
          (1, 1, 1), (4, 129, 63), (70, 5, 66), (1, 257, 300), (33, 33, 33), (75, 48, 64)]


@pytest.mark.parametrize("shape", SHAPES)
def test_ragged_shapes_smooth_fields(shape):
    for rel in (2e-2, 2e-3):
        x = synth.grf(shape, 3.0, 77 + sum(shape))
        if np.ptp(x) == 0:  # a single voxel has no range: any bound will do
            x = np.zeros(shape)
            xq, eb = x.astype(np.float32), 0.5
        else:
            x32, xq, q, eb = synth.quantize(x, rel)
        assert_parity(xq, eb, label=f"ragged{shape}")


def test_adversarial_fields():
    n = (20, 24, 28)
    assert_parity(np.full(n, 3.0, np.float32), 0.5, label="constant")
    q = np.zeros(n)
    q[10, 12, 14] = 1
    assert_parity(q.astype(np.float32), 0.5, label="single-bump")
    cz, cy, cx = np.meshgrid(*[np.arange(s) for s in n], indexing="ij")
    assert_parity(((cz + cy + cx) % 2).astype(np.float32), 0.5, label="checkerboard")
    assert_parity(((cx // 3) % 2).astype(np.float32), 0.5, label="stripes")
    assert_parity((cx // 5 + cy // 7).astype(np.float32), 0.5, label="terraces")
    assert_parity(np.where(cx < 14, 0, 1).astype(np.float32), 0.5, label="one-step")
    big = np.zeros((3, 4, 700))
    big[1, 1, 350] = 2
    assert_parity(big.astype(np.float32), 0.5, label="far-single")
    # long lines and few sites: exercises long searches and absent sites
    q = np.zeros((3, 1500, 3))
    q[1, 100, 1] = 1
    assert_parity(q.astype(np.float32), 0.5, label="long-y")


def test_indices_of_values_off_the_quantization_grid():
    """x' that are not decompressed values: for about a fifth of the voxels the
    product with the rounded reciprocal of 2 eb lies farther than 0.4 from an
    integer, and some indices lie above 2^18, so the seed pass takes the exact
    quotient there (a wave at a time, voxel by voxel).  q and every other tap
    match the oracle."""
    rng = np.random.default_rng(5)
    xq = (rng.standard_normal((9, 40, 70)) * 3.7).astype(np.float32)
    xq[4, 20, 10:30] = np.linspace(0.2 * 2.7e5, 0.2 * 4.1e5, 20).astype(np.float32)
    frac = np.abs(xq / np.float32(0.2) - np.rint(xq / np.float32(0.2)))
    assert (frac > 0.4).mean() > 0.1
    assert_parity(xq, 0.1, label="off-grid values")


def test_parameters_eta_power():
    x32, xq, q, eb = synth.make_workload("grf64_k3_eb1e-2")
    for eta, p in ((0.5, 1.0), (1.0, 2.0), (0.9, 0.5)):
        assert_parity(xq, eb, eta, p, label=f"eta{eta}p{p}")


def test_determinism_and_in_place():
    import paper_2602_20097_amd as qai
    x32, xq, q, eb = synth.make_workload("grf64_k3_eb1e-2")
    t = torch.from_numpy(xq).cuda()
    a = qai.mitigate(t, eb)
    b = qai.mitigate(t, eb)
    c = qai.mitigate_simple(t, eb)
    u = t.clone()
    qai.mitigate(u, eb, out=u)
    torch.cuda.synchronize()
    assert torch.equal(a, b) and torch.equal(a, c) and torch.equal(a, u)


def test_unaligned_field_and_out_take_the_whole_pass():
    """A field or output not 16-byte aligned (a view at an odd storage offset)
    runs the second EDT's whole z pass and step E instead of the needed-voxel
    search; the output is the same bit for bit, also in place, and so are the
    gradients the adjoint derives from the saved distance words."""
    import paper_2602_20097_amd as qai
    x32, xq, q, eb = synth.quantize(synth.grf((20, 36, 50), 3.0, 4242), 2e-2)
    n = xq.size
    t = torch.from_numpy(xq).cuda()
    ws_a = qai.new_workspace(t.shape)
    ref = qai.mitigate(t, eb, workspace=ws_a)
    big = torch.empty(n + 8, dtype=torch.float32, device="cuda")
    f = big[1:1 + n].view(t.shape)            # 4 bytes past a 16-byte boundary
    f.copy_(t)
    o = torch.empty(n + 8, dtype=torch.float32, device="cuda")[3:3 + n].view(t.shape)
    ws_b = qai.new_workspace(t.shape)
    got = qai.mitigate(f, eb, out=o, workspace=ws_b)
    g = torch.randn_like(ref)
    ga = qai.backward(g, ws_a, t.shape, eb)
    gb = qai.backward(g, ws_b, t.shape, eb)
    inplace = big[1:1 + n].view(t.shape)
    qai.mitigate(inplace, eb, out=inplace)
    torch.cuda.synchronize()
    assert torch.equal(got, ref)
    assert torch.equal(inplace, ref)
    assert torch.equal(ga, gb)


def test_status_flag_for_out_of_range_indices():
    import paper_2602_20097_amd as qai
    xq = np.zeros((4, 5, 6), np.float32)
    xq[2, 2, 2] = 1e9
    t = torch.from_numpy(xq).cuda()
    ws = qai.new_workspace(t.shape)
    qai.mitigate(t, 0.5, workspace=ws)
    assert qai.device_status(ws) & qai.QAI_STATUS_QRANGE
    qai.mitigate(torch.zeros_like(t), 0.5, workspace=ws)
    assert qai.device_status(ws) == 0


@pytest.mark.parametrize("name", ["modes256x384x384_eb1e-2", "modes256x384x384_eb1e-3",
                                  "modes256x384x384_eb1e-4", "grf2d_1800x3600_k11/3_eb1e-3"])
def test_full_size_workloads(name):
    x32, xq, q, eb = synth.make_workload(name)
    g, r = assert_parity(xq, eb, label=name)
    assert np.array_equal(g["q"], q)


def test_headline_512_full_parity():
    x32, xq, q, eb = synth.make_workload("grf512_k11/3_eb1e-3")
    g, r = assert_parity(xq, eb, label="grf512")
    # the relaxed bound of Section VII-C on the whole field
    assert np.abs(g["out"].astype(np.float64) - x32).max() <= (1 + 0.9) * eb * (1 + 1e-6)


@pytest.mark.parametrize("shape", [(1, 40, 2000), (5, 7, 1100), (3, 9, 600), (4, 10, 1024), (3, 5, 2048),
                                   (2, 6, 3600), (1, 9, 4096), (1, 3, 4099)])
def test_long_lines(shape):
    """x-lines longer than 512 voxels: the register seed pass shares a line
    between two (up to 1024 voxels), four (2048) or eight waves (4096), longer
    lines go to the one-line-per-workgroup pass; explicit rows per block keep
    a line in one wave of the LDS-slab pass; all agree with the oracle."""
    import paper_2602_20097_amd as qai
    x32, xq, q, eb = synth.quantize(synth.grf(shape, 3.0, 900 + sum(shape)), 2e-2)
    assert_parity(xq, eb, label=f"long lines {shape}")
    base = qai.get_tuning()
    try:
        qai.set_tuning(seed_rows=2)
        assert_parity(xq, eb, label=f"long lines {shape}, slab")
    finally:
        qai.set_tuning(None)
    assert qai.get_tuning() == base


def test_blocked_handoff_to_the_needed_voxel_search():
    """With the second EDT's y pass on the per-lane envelope and its z pass
    automatic, a call without taps hands the y result to the needed-voxel
    search in the blocked layout [z][y/4][x][y%4] (rows per plane that are not
    a multiple of 4 exercise its padding); the output matches the tapped call
    bit for bit and the oracle."""
    import paper_2602_20097_amd as qai
    base = qai.get_tuning()
    try:
        qai.set_tuning(edt2_algo=[3, -1])
        for shape in ((6, 70, 130), (9, 33, 65), (5, 31, 100), (3, 64, 64), (2, 2, 300)):
            x32, xq, q, eb = synth.quantize(synth.grf(shape, 2.5, 77 + sum(shape)), 2e-2)
            assert_parity(xq, eb, label=f"blocked {shape}")
    finally:
        qai.set_tuning(None)
    assert qai.get_tuning() == base


@pytest.mark.parametrize("rel,dense", [(1e-3, True), (2e-2, False)])
def test_handoff_layout_follows_the_b1_density(rel, dense):
    """On automatic passes the y pass of the second EDT picks the handoff
    layout on the device from the first seed pass's B1 estimate: blocked where
    B1 covers at least 90% of the field, natural elsewhere.  Fields on both
    sides of that line (B1 checked with the oracle) match the tapped call and
    the oracle."""
    x32, xq, q, eb = synth.quantize(synth.grf((64, 128, 192), 3.0, 91), rel)
    g, r = assert_parity(xq, eb, label=f"handoff rel {rel}")
    needed = (r["s"] != 0) & (r["b1"] == 0)
    assert needed.sum() > 500
    assert (r["b1"].mean() >= 0.93) == dense and (r["b1"].mean() <= 0.87) == (not dense)


def test_first_edt_beyond_the_search_disc():
    """The first EDT's y and z passes run as one search over a disc of radius
    12 around each voxel when B1 covers at least 80% of the field; a voxel
    farther from B1 raises a flag and the separable passes behind the search
    recompute the field, and with sparser B1 the search stands down for
    them.  Dense B1 (random indices) around a 28-voxel plateau puts the
    plateau's centre 13 voxels from B1; a 30-voxel plateau in a smooth field
    makes B1 sparse; a constant field has no B1 at all."""
    rng = np.random.default_rng(31)
    xq = rng.integers(-3, 4, size=(96, 96, 96)).astype(np.float32)
    xq[34:62, 34:62, 34:62] = 7.0
    r = oracle.qai(xq, 0.5)
    assert r["b1"].mean() >= 0.9 and r["d1sq"].max() > 144
    assert_parity(xq, 0.5, label="dense with a hole")
    x32, xq, q, eb = synth.quantize(synth.grf((40, 40, 40), 3.0, 77), 1e-2)
    xq = xq.copy()
    xq[5:35, 5:35, 5:35] = xq[20, 20, 20]
    r = oracle.qai(xq, eb)
    assert r["b1"].mean() < 0.9 and r["d1sq"].max() > 144
    assert_parity(xq, eb, label="plateau")
    assert_parity(np.full((6, 8, 12), 3.0, np.float32), 0.5, label="constant")
    # 2-D fields take the separable passes (here a plateau farther than 12 from B1
    # and dense random indices)
    x2 = rng.integers(-3, 4, size=(1, 64, 72)).astype(np.float32)
    x2[:, 17:47, 20:50] = 7.0
    r = oracle.qai(x2, 0.5)
    assert r["d1sq"].max() > 144
    assert_parity(x2, 0.5, label="2-D plateau")
    assert_parity(rng.integers(-3, 4, size=(1, 50, 96)).astype(np.float32), 0.5, label="2-D dense")


def test_every_pass_algorithm_gives_the_same_transform():
    """Each per-pass algorithm choice (qai_tuning) computes the same exact EDTs."""
    import paper_2602_20097_amd as qai
    cases = [synth.make_workload("grf64_k3_eb1e-2")[1:4:2]]
    # (2, 1500, 64) and (2, 4096, 40): lines too long for the (c, h) form of the
    # per-lane envelope, so algorithm 3 takes its 24-bit and 64-bit fallbacks
    for shape in ((5, 70, 130), (33, 33, 33), (3, 65, 200), (2, 300, 77), (2, 1500, 64), (2, 4096, 40)):
        x32, xq, q, eb = synth.quantize(synth.grf(shape, 3.0, 5 + sum(shape)), 2e-2)
        cases.append((xq, eb))
    base = qai.get_tuning()
    try:
        for xq, eb in cases:
            r = oracle.qai(xq, eb)
            # seed_rows: 0 register variant, 1..8 the LDS-slab variant (8: 512-thread
            # workgroups), -1 one line per wave
            combos = [(a1, a2, 0) for a1 in (0, 1, 2, 4, 5) for a2 in (0, 1, 2, 3, 4, 5)] + \
                [(4, 3, r) for r in (8, 4, 2, 1, -1)]
            for a1, a2, rows in combos:
                qai.set_tuning(edt1_algo=[a1, a1], edt2_algo=[a2, a2], seed_rows=rows)
                print(f"tuning edt1 {a1} edt2 {a2} seed_rows {rows} shape {xq.shape}", flush=True)
                g = gpu_run(xq, eb)
                for k in KEYS:
                    assert np.array_equal(g[k].astype(np.int64), r[k].astype(np.int64)), (k, a1, a2, rows, xq.shape)
    finally:
        qai.set_tuning(None)
    assert qai.get_tuning() == base


def test_every_accepted_launch_setting_launches():
    """Every setting qai_tuning_set accepts must launch: workgroup sizes of the
    windowed search up to 1024 threads and LDS-slab seed passes of 1 to 8 waves
    per workgroup (the launcher refuses a block beyond a kernel's compiled
    bound on the host instead of launching it)."""
    import paper_2602_20097_amd as qai
    x32, xq, q, eb = synth.quantize(synth.grf((9, 70, 130), 3.0, 4321), 2e-2)
    r = oracle.qai(xq, eb)
    base = qai.get_tuning()
    try:
        for wt in (64, 128, 192, 256, 512, 1024):
            qai.set_tuning(edt1_algo=[1, 1], edt2_algo=[1, 1], window_threads=wt)
            assert_parity(xq, eb, label=f"window_threads {wt}", r=r)
        qai.set_tuning(None)
        for rows in range(-1, 9):
            for planes in (1, 3, 16):
                qai.set_tuning(seed_rows=rows, seed_planes=planes)
                assert_parity(xq, eb, label=f"seed_rows {rows} seed_planes {planes}", r=r)
    finally:
        qai.set_tuning(None)
    assert qai.get_tuning() == base


@pytest.mark.parametrize("shape,rel", [((20, 36, 48), 2e-2), ((33, 40, 64), 5e-3), ((5, 70, 130), 2e-2),
                                       ((96, 96, 96), None)])
def test_wide_index_variants(shape, rel):
    """force_wide = 1 takes the 64-bit variants that only fields beyond 2^29
    words (the needed-voxel search by 64-bit index) or 2^32 voxels (the fused
    first-EDT search) would take on their own, and the 64-bit arithmetic of the
    streaming envelopes; they must compute the same transforms.  The last case
    is dense B1 around a plateau, so the fused search hands over to the gated
    separable passes."""
    import paper_2602_20097_amd as qai
    if rel is None:
        rng = np.random.default_rng(31)
        xq = rng.integers(-3, 4, size=shape).astype(np.float32)
        xq[34:62, 34:62, 34:62] = 7.0
        eb = 0.5
    else:
        x32, xq, q, eb = synth.quantize(synth.grf(shape, 3.0, 11 + sum(shape)), rel)
    r = oracle.qai(xq, eb)
    base = qai.get_tuning()
    try:
        for cfg in (dict(force_wide=1), dict(force_wide=1, edt1_algo=[0, 0], edt2_algo=[0, 0]),
                    dict(force_wide=1, edt2_algo=[3, -1])):
            qai.set_tuning(None)
            qai.set_tuning(**cfg)
            assert_parity(xq, eb, label=f"wide {cfg} {shape}", r=r)
    finally:
        qai.set_tuning(None)
    assert qai.get_tuning() == base


@pytest.mark.parametrize("shape,rel", [((6, 200, 64), 2e-2), ((4, 300, 130), 3e-3), ((3, 513, 70), 2e-2),
                                       ((5, 257, 96), 5e-3), ((64, 256, 192), 1e-3), ((2, 640, 64), 1e-2)])
def test_tall_columns_with_few_tiles(shape, rel):
    """y passes over tall columns with few column tiles (rows per plane not a
    multiple of 4, sparse fields with long distances along y, and a dense one
    that hands the blocked layout to the needed-voxel search): the untapped
    call matches the tapped one bit for bit and both match the oracle."""
    x32, xq, q, eb = synth.quantize(synth.grf(shape, 3.0, 31 + sum(shape)), rel)
    assert_parity(xq, eb, label=f"tall columns {shape} rel {rel}")


def test_envelope_ring_overflow_hands_the_y_pass_to_the_banded_pass():
    """Sparse B2 over long x-lines in a field of more than 2048 column tiles
    (32 ring entries per lane): some column's live window outgrows the
    per-lane envelope's ring in the second EDT's y pass, the pass raises the
    header word and the banded pass (gated on it) redoes the whole y pass in
    the natural layout, which the needed-voxel search then reads.  The tapped
    call (whole z pass) takes the same hand-off ahead of its z pass.  The
    output matches the tapped call and the oracle."""
    import paper_2602_20097_amd as qai
    x32, xq, q, eb = synth.quantize(synth.grf((130, 128, 1024), 3.7, 77), 1.6e-4)
    t = torch.from_numpy(xq).cuda()
    ws = qai.new_workspace(t.shape)
    qai.mitigate(t, eb, workspace=ws)
    torch.cuda.synchronize()
    assert int(ws[68:72].view(torch.int32).item()) != 0  # header word 17: the ring overflowed
    ws2 = qai.new_workspace(t.shape)
    qai.mitigate(t, eb, taps=True, workspace=ws2)
    torch.cuda.synchronize()
    assert int(ws2[68:72].view(torch.int32).item()) != 0
    assert_parity(xq, eb, label="ring overflow (130, 128, 1024)")


@pytest.mark.parametrize("shape", [(64, 128, 192), (8, 300, 512)])
def test_sparse_b1_takes_the_whole_z_pass_beside_the_search(shape):
    """Where B1 covers under 60% of the field most voxels need d2, and on z
    passes of at most 2048 column tiles (64 x 128 x 192: 384) the whole z pass
    with step E runs on the side stream instead of the needed-voxel search
    (both are launched, each gated on the first seed pass's B1 estimate); on
    larger ones (8 x 300 x 512: 2400) the search runs alone.  Either way the
    output matches the tapped call and the oracle."""
    x32, xq, q, eb = synth.quantize(synth.grf(shape, 3.0, 17), 2e-2)
    g, r = assert_parity(xq, eb, label=f"sparse B1 {shape}")
    assert r["b1"].mean() < 0.55
