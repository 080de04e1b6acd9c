"""Pins of the CPU oracle against values fixed by the paper's definitions and by mathematics.

Each test pins one part of the oracle to something other than its own code:
hand-worked census words, the bit-loop definition of the Hamming distance,
brute-force minimisation over all labelings of short chains (the energy the
SGM path recurrence minimises), closed forms of special penalty settings,
exact parabola vertices, hand-built left-right cases, a library median, and
the noise model's rounding and clipping rules.
"""
import itertools

import numpy as np
import pytest

from synth import PairSpec, make_shift_pair


# ----------------------------------------------------------------- census
IMG5 = np.array([[12, 50, 33, 71, 8],
                 [90, 41, 66, 2, 57],
                 [23, 77, 45, 19, 88],
                 [64, 5, 98, 36, 70],
                 [15, 83, 29, 60, 47]], np.uint8)
IMG3 = np.array([[90, 20, 70],
                 [40, 50, 10],
                 [30, 80, 60]], np.uint8)


def test_census_hand_3x3(orc):
    # centre pixel: a>i, b>h, c>g, d>f -> 1,0,1,1 -> 0b1101
    assert orc.census(IMG3, 3, 3, 0)[1, 1] == 13
    # full: e>a..i (raster, centre skipped): 0,1,0,1,1,1,0,0
    assert orc.census(IMG3, 3, 3, 1)[1, 1] == 58
    # corner (0,0) with clamp-to-edge: a>e, a>d, b>d, a>b -> 1,1,0,1
    assert orc.census(IMG3, 3, 3, 0)[0, 0] == 11


def test_census_hand_5x5_orientation(orc):
    # 3 wide x 5 tall window at the centre of IMG5
    assert orc.census(IMG5, 3, 5, 0)[2, 2] == 74
    assert orc.census(IMG5, 3, 5, 1)[2, 2] == 5546
    # 5 wide x 3 tall window
    assert orc.census(IMG5, 5, 3, 0)[2, 2] == 67


def test_census_bits(orc):
    assert orc.census_bits(7, 9, 0) == 31
    assert orc.census_bits(7, 9, 1) == 62
    assert orc.census_bits(3, 3, 0) == 4


def test_census_invariants(orc):
    rng = np.random.default_rng(1)
    img = rng.permutation(np.arange(256))[: 16 * 16].reshape(16, 16).astype(np.uint8)  # tie-free
    for mode in (0, 1):
        bits = orc.census_bits(7, 9, mode)
        c = orc.census(img, 7, 9, mode)
        assert int(c.max()) < (1 << bits)
        # constant image -> 0
        assert not orc.census(np.full((12, 13), 77, np.uint8), 7, 9, mode).any()
        # invariant under a strictly increasing intensity map (no clipping)
        small = rng.integers(0, 128, (15, 17)).astype(np.uint8)
        mono = (2 * small.astype(np.int32) + 1).astype(np.uint8)
        assert np.array_equal(orc.census(mono, 7, 9, mode), orc.census(small, 7, 9, mode))
    # CS: rotating the image by 180 degrees flips every bit of a tie-free window
    c = orc.census(img, 7, 9, 0)
    cr = orc.census(np.ascontiguousarray(img[::-1, ::-1]), 7, 9, 0)
    inner = c[4:-4, 3:-3]
    inner_rot = cr[::-1, ::-1][4:-4, 3:-3]
    assert np.array_equal(inner ^ inner_rot, np.full_like(inner, (1 << 31) - 1))


def test_hamming_bit_loop(orc):
    rng = np.random.default_rng(2)
    for _ in range(200):
        a, b = (int(v) for v in rng.integers(0, 2**63, 2, dtype=np.uint64))
        ref = sum(((a ^ b) >> k) & 1 for k in range(64))
        assert orc.popcount(a ^ b) == ref
        assert orc.popcount(a ^ a) == 0
        assert orc.popcount(a ^ b) == orc.popcount(b ^ a)
        c = int(rng.integers(0, 2**63, dtype=np.uint64))
        assert orc.popcount(a ^ c) <= orc.popcount(a ^ b) + orc.popcount(b ^ c)


def test_cost_out_of_range(orc):
    rng = np.random.default_rng(3)
    cl = rng.integers(0, 2**31, (3, 10), dtype=np.uint64)
    cr = rng.integers(0, 2**31, (3, 10), dtype=np.uint64)
    C = orc.cost(cl, cr, 6, 31)
    for y in range(3):
        for x in range(10):
            for d in range(6):
                want = 31 if x - d < 0 else bin(int(cl[y, x]) ^ int(cr[y, x - d])).count("1")
                assert C[y, x, d] == want


# ----------------------------------------------------------------- aggregation
def _brute_chain(costs, p1, p2):
    """Normalised path values on a chain by exhaustive search over all labelings."""
    n, D = costs.shape

    def V(a, b):
        return 0 if a == b else (p1 if abs(a - b) == 1 else p2)

    raw = np.zeros((n, D), np.int64)
    for i in range(n):
        for d in range(D):
            best = None
            for lab in itertools.product(range(D), repeat=i):
                labs = lab + (d,)
                e = sum(int(costs[j, labs[j]]) for j in range(i + 1))
                e += sum(V(labs[j], labs[j - 1]) for j in range(1, i + 1))
                best = e if best is None else min(best, e)
            raw[i, d] = best
    out = raw.copy()
    for i in range(1, n):
        out[i] = raw[i] - raw[i - 1].min()
    return out


@pytest.mark.parametrize("n,D,p1,p2,seed", [(6, 4, 3, 9, 0), (5, 5, 2, 20, 1), (6, 3, 5, 5, 2),
                                             (4, 5, 0, 7, 3), (6, 5, 7, 86, 4)])
def test_path_brute_force_chain(orc, n, D, p1, p2, seed):
    rng = np.random.default_rng(seed)
    chain = rng.integers(0, 32, (n, D)).astype(np.uint8)
    want = _brute_chain(chain, p1, p2)
    # horizontal, forward: a 1 x n image
    L = orc.path(chain[None, :, :], 1, 0, p1, p2)[0]
    assert np.array_equal(L.astype(np.int64), want)
    # horizontal, backward: the chain laid out reversed
    L = orc.path(chain[None, ::-1, :], -1, 0, p1, p2)[0][::-1]
    assert np.array_equal(L.astype(np.int64), want)
    # vertical down / up
    L = orc.path(chain[:, None, :], 0, 1, p1, p2)[:, 0]
    assert np.array_equal(L.astype(np.int64), want)
    L = orc.path(chain[::-1, None, :], 0, -1, p1, p2)[::-1, 0]
    assert np.array_equal(L.astype(np.int64), want)
    # the four diagonals: put the chain on a diagonal of an n x n image
    for dx, dy in ((1, 1), (-1, 1), (1, -1), (-1, -1)):
        C = rng.integers(0, 32, (n, n, D)).astype(np.uint8)
        pts = []
        for i in range(n):
            x = i if dx > 0 else n - 1 - i
            y = i if dy > 0 else n - 1 - i
            C[y, x] = chain[i]
            pts.append((y, x))
        L = orc.path(C, dx, dy, p1, p2)
        got = np.array([L[y, x] for y, x in pts], np.int64)
        assert np.array_equal(got, want), (dx, dy)


def test_path_zero_penalties_and_large_penalties(orc):
    rng = np.random.default_rng(5)
    C = rng.integers(0, 32, (7, 9, 6)).astype(np.uint8)
    # P1 = P2 = 0: every path reproduces the cost, so S = P * C
    for P in (2, 4, 8):
        S = orc.aggregate(C, P, 0, 0)
        assert np.array_equal(S, P * C.astype(np.uint32))
    # huge penalties: a path never changes label, so the raw value is a running sum
    big = 10000
    L = orc.path(C, 1, 0, big, big).astype(np.int64)
    cum = np.cumsum(C.astype(np.int64), axis=1)
    want = cum.copy()
    want[:, 1:] = cum[:, 1:] - cum[:, :-1].min(axis=2, keepdims=True)
    assert np.array_equal(L, want)


def test_path_bounds(orc):
    rng = np.random.default_rng(6)
    bits, p1, p2 = 31, 7, 86
    C = rng.integers(0, bits + 1, (11, 13, 16)).astype(np.uint8)
    for dx, dy in orc.path_dirs(8):
        L = orc.path(C, dx, dy, p1, p2).astype(np.int64)
        assert L.min() >= 0 and L.max() <= bits + p2
        assert L.min(axis=2).max() <= bits


def test_path_dirs(orc):
    assert orc.path_dirs(2) == [(1, 0), (-1, 0)]
    assert orc.path_dirs(4)[2:] == [(0, 1), (0, -1)]
    assert sorted(orc.path_dirs(8)[4:]) == [(-1, -1), (-1, 1), (1, -1), (1, 1)]


# ----------------------------------------------------------------- winner, uniqueness, sub-pixel
def test_wta_parabola_vertex(orc):
    # S(d) = 16 (d - delta)^2 + beta with delta = d0 + 1/4 or d0 - 1/4 is integer-valued;
    # the three-point parabola fit through it returns delta exactly.
    D = 12
    rows = []
    deltas = []
    winners = []
    for d0 in range(2, 10):
        for q in (1, -1, 2):   # offsets +1/4, -1/4, +1/2
            delta = d0 + q / 4.0
            d = np.arange(D, dtype=np.float64)
            s = 16 * (d - delta) ** 2 + 100
            assert np.allclose(s, np.round(s))
            rows.append(np.round(s).astype(np.uint32))
            deltas.append(delta)
            winners.append(d0)  # nearest integer; at +1/2 the tie goes to the lower d
    S = np.stack(rows)[None]
    dint, s1, s2, vu, dsub = orc.wta(S, 0, 1)
    for i, delta in enumerate(deltas):
        assert dint[0, i] == winners[i]
        assert dsub[0, i] == pytest.approx(delta, abs=1e-12)
        assert -0.5 < dsub[0, i] - dint[0, i] <= 0.5


def test_wta_ties_second_best_uniqueness(orc):
    D = 8
    S = np.full((1, 6, D), 50, np.uint32)
    S[0, 0, 3] = S[0, 0, 5] = 10             # tie -> lowest d
    S[0, 1, 4] = 10; S[0, 1, 5] = 11; S[0, 1, 0] = 40   # d*+1 excluded from the second best
    S[0, 2, :] = 200; S[0, 2, 4] = 90; S[0, 2, 1] = 100  # 100*90 <= 90*100: passes at u = 10
    S[0, 3, :] = 200; S[0, 3, 4] = 91; S[0, 3, 1] = 100  # 100*91 > 90*100: fails
    S[0, 4, :] = 7; S[0, 4, 0] = 3           # d* = 0
    S[0, 5, :] = 7; S[0, 5, 7] = 3           # d* = D-1
    dint, s1, s2, vu, dsub = orc.wta(S, 10, 1)
    assert dint[0, 0] == 3 and s1[0, 0] == 10 and s2[0, 0] == 10 and vu[0, 0] == 0
    assert dint[0, 1] == 4 and s2[0, 1] == 40
    assert dint[0, 2] == 4 and s2[0, 2] == 100 and vu[0, 2] == 1
    assert dint[0, 3] == 4 and s2[0, 3] == 100 and vu[0, 3] == 0
    assert dint[0, 4] == 0 and dsub[0, 4] == 0.0
    assert dint[0, 5] == 7 and dsub[0, 5] == 7.0
    # D = 2: no candidate for the second best -> passes
    d2 = orc.wta(np.array([[[5, 9]]], np.uint32), 50, 1)
    assert d2[2][0, 0] == -1 and d2[3][0, 0] == 1


# ----------------------------------------------------------------- left-right check
def test_right_disp_and_lr_hand_case(orc):
    W, D = 10, 4
    # pixel x has a single zero-cost disparity dmap[x]
    dmap = [0, 1, 1, 2, 3, 1, 3, 2, 0, 1]
    S = np.full((1, W, D), 10, np.uint32)
    for x, d in enumerate(dmap):
        S[0, x, d] = 0
    dR = orc.right_disp(S)
    # by hand: dR(xr) is the lowest d with dmap[xr + d] == d, or 0 when every value ties
    assert list(dR[0]) == [0, 1, 0, 3, 1, 2, 0, 0, 0, 0]
    dint = np.array([dmap], np.int32)
    # by hand: x -> xr = x - dmap[x] -> compare dmap[x] with dR(xr) at lr = 0
    assert list(orc.lr_check(dint, dR, 0)[0]) == [1, 0, 1, 0, 0, 1, 1, 1, 1, 0]
    v = orc.lr_check(dint, dR, 1)
    assert list(v[0]) == [1, 1, 1, 1, 0, 1, 1, 1, 1, 1]  # only x=4 (|3-1| = 2) fails
    # x - d* < 0 is invalid
    assert orc.lr_check(np.array([[3, 0]], np.int32), np.zeros((1, 2), np.int32), 1)[0, 0] == 0
    # lr < 0 disables the check
    assert orc.lr_check(dint, dR, -1).all()


def test_lr_constant_shift(orc):
    d0 = 5
    rng = np.random.default_rng(7)
    W, D = 40, 12
    C = rng.integers(5, 31, (3, W, D)).astype(np.uint8)
    C[:, :, d0] = 0
    S = orc.aggregate(C, 2, 7, 86)
    dR = orc.right_disp(S)
    assert (dR[:, : W - D] == d0).all()


# ----------------------------------------------------------------- median, depth, noise
def test_median_matches_library(orc):
    rng = np.random.default_rng(8)
    a = rng.random((9, 11)) * 50
    a[rng.random(a.shape) < 0.3] = 0.0
    m = orc.median3(a)
    win = np.stack([a[1 + dy:a.shape[0] - 1 + dy, 1 + dx:a.shape[1] - 1 + dx]
                    for dy in (-1, 0, 1) for dx in (-1, 0, 1)])
    assert np.array_equal(m[1:-1, 1:-1], np.median(win, axis=0))
    assert np.array_equal(m[0], a[0]) and np.array_equal(m[:, -1], a[:, -1])


def test_depth_closed_form(orc):
    disp = np.array([0.0, 1.0, 2.5, 64.0, -1.0])
    dep = orc.depth(disp, 920.0, 0.055)
    assert dep[0] == 0 and dep[4] == 0
    assert dep[1] == pytest.approx(50.6) and dep[2] == pytest.approx(20.24) and dep[3] == pytest.approx(0.790625)


def test_noise_rounding_and_clipping(orc):
    img = np.array([10, 11, 250, 3, 100, 0], np.uint8)
    g = np.array([1, 1, 1, 1, 1.5, 2], np.float32)
    n = np.array([0.5, 0.5, 10, -7, 0.25, -0.5], np.float32)
    # 10.5 -> 10 (ties to even), 11.5 -> 12, 260 -> 255, -4 -> 0, 150.25 -> 150, -0.5 -> 0
    assert list(orc.ir_noise(img, g, n)) == [10, 12, 255, 0, 150, 0]
    ident = np.arange(256, dtype=np.uint8)
    assert np.array_equal(orc.ir_noise(ident, np.ones(256, np.float32), np.zeros(256, np.float32)), ident)


def test_noise_moments_paper_mode(orc):
    from scipy import stats
    from synth import noise_draws
    spec = PairSpec(200, 200, noise="paper")
    g, n = noise_draws(spec, (200, 200), 11, 4)
    k, th = 3.98, 0.254
    assert g.mean() == pytest.approx(k * th, rel=0.01)
    assert g.var() == pytest.approx(k * th * th, rel=0.03)
    assert n.mean() == pytest.approx(-0.231, abs=0.01)
    assert n.std() == pytest.approx(0.83, rel=0.01)
    assert stats.kstest(g.ravel()[:20000], "gamma", args=(k, 0, th)).pvalue > 1e-3
    img = np.full(g.shape, 100, np.uint8)
    out = orc.ir_noise(img, g, n).astype(np.float64)
    assert out.mean() == pytest.approx(100 * k * th - 0.231, rel=0.01)


# ----------------------------------------------------------------- end to end
def test_end_to_end_constant_shift(orc):
    W, H, D, d0 = 96, 40, 32, 9
    left, right = make_shift_pair(W, H, d0, seed=21)
    params = dict(width=W, height=H, max_disp=D, census_w=7, census_h=9, census_mode=0, p1=7, p2=86,
                  uniqueness_pct=10, lr_max_diff=1, num_paths=8, median=3, subpixel=1,
                  focal_px=400.0, baseline_m=0.055)
    r = orc.sgm(params, left, right)
    rw = 3
    inner = (slice(None), slice(d0 + rw, W - rw))
    assert (r.dint[inner] == d0).all()
    assert (r.flags[inner] & 3 == 3).all()
    m = r.disp > 0
    assert np.allclose(r.depth[m], 400.0 * np.float64(np.float32(0.055)) / r.disp[m], rtol=1e-6)


# ----------------------------------------------------------------- full right-referenced run
def test_right_reference_mirror_identity(orc):
    """Matching the right image against the left is left-referenced matching of
    the x-flipped census maps with the roles swapped: the path set is closed
    under the flip, so the right-referenced cost, aggregate and winner equal the
    flipped left-referenced ones computed by the independent left-side functions."""
    rng = np.random.default_rng(11)
    H, W, D, bits = 9, 23, 7, 31
    cl = rng.integers(0, 2 ** 31, (H, W)).astype(np.uint64)
    cr = rng.integers(0, 2 ** 31, (H, W)).astype(np.uint64)
    CR = orc.cost_right(cl, cr, D, bits)
    CM = orc.cost(cr[:, ::-1], cl[:, ::-1], D, bits)
    assert np.array_equal(CR, CM[:, ::-1])
    for paths in (2, 4, 8):
        SM = orc.aggregate(CM, paths, 7, 40)
        dm = SM.argmin(axis=2)[:, ::-1]  # numpy argmin takes the lowest index on ties
        assert np.array_equal(orc.right_disp_full(cl, cr, D, bits, paths, 7, 40), dm)


def test_right_reference_constant_shift(orc):
    """right(x) = left(x + d0): the right-referenced run recovers d0 wherever
    x + d0 and the census window stay inside the image, and the full-run LR
    check then keeps every interior pixel of the left result."""
    W, H, D, d0 = 96, 40, 32, 9
    left, right = make_shift_pair(W, H, d0, seed=21)
    cl, cr = orc.census(left), orc.census(right)
    dR = orc.right_disp_full(cl, cr, D, 31, 8, 7, 86)
    rw = 3
    assert (dR[:, rw: W - d0 - rw] == d0).all()
    params = dict(width=W, height=H, max_disp=D, census_w=7, census_h=9, census_mode=0, p1=7, p2=86,
                  uniqueness_pct=10, lr_max_diff=1, num_paths=8, median=3, subpixel=1,
                  focal_px=400.0, baseline_m=0.055, lr_mode=1)
    r = orc.sgm(params, left, right)
    assert np.array_equal(r.dright, dR)
    inner = (slice(None), slice(d0 + rw, W - rw))
    assert (r.dint[inner] == d0).all() and (r.flags[inner] & 3 == 3).all()
    # the lr_mode only changes the right disparity and what depends on it
    r0 = orc.sgm(dict(params, lr_mode=0), left, right)
    assert np.array_equal(r0.dint, r.dint) and np.array_equal(r0.dsub, r.dsub)
    assert np.array_equal(r0.flags & 5, r.flags & 5)


# ----------------------------------------------------------------- semi-global block matching (SGBM)
def test_block_cost_is_a_clamped_box_filter(orc):
    """The block cost equals the box filter of each disparity slice with
    edge-replicating borders (scipy's uniform_filter, mode='nearest') times the
    block area; a 1x1 block is the pixel cost; a constant slice scales by the area."""
    from scipy.ndimage import uniform_filter
    rng = np.random.default_rng(5)
    H, W, D = 11, 17, 6
    C = rng.integers(0, 32, (H, W, D)).astype(np.uint16)
    assert np.array_equal(orc.block_cost(C, 1, 1), C)
    for bw, bh in ((3, 3), (5, 3), (3, 7), (1, 5)):
        want = np.stack([np.rint(uniform_filter(C[:, :, d].astype(np.float64), size=(bh, bw), mode="nearest")
                                 * (bw * bh)) for d in range(D)], axis=2)
        assert np.array_equal(orc.block_cost(C, bw, bh), want.astype(np.uint16)), (bw, bh)
    K = np.full((H, W, D), 7, np.uint16)
    assert (orc.block_cost(K, 5, 3) == 7 * 15).all()


def test_sgbm_constant_shift_and_right_reference(orc):
    """A noise-free constant shift is recovered exactly by block matching away
    from the borders; the right-referenced block run obeys the flip identity."""
    W, H, D, d0 = 96, 40, 32, 9
    left, right = make_shift_pair(W, H, d0, seed=23)
    params = dict(width=W, height=H, max_disp=D, census_w=5, census_h=5, census_mode=0, p1=20, p2=120,
                  uniqueness_pct=10, lr_max_diff=1, num_paths=8, median=3, subpixel=1,
                  focal_px=400.0, baseline_m=0.055, block_w=3, block_h=3)
    r = orc.sgm(params, left, right)
    m = 2 + 1  # census radius + block radius
    inner = (slice(None), slice(d0 + m, W - m))
    assert (r.dint[inner] == d0).all()
    cl, cr = orc.census(left, 5, 5, 0), orc.census(right, 5, 5, 0)
    bits = orc.census_bits(5, 5, 0)
    CB = orc.block_cost(orc.cost_right(cl, cr, D, bits), 3, 3)
    CM = orc.block_cost(orc.cost(cr[:, ::-1], cl[:, ::-1], D, bits), 3, 3)
    assert np.array_equal(CB, CM[:, ::-1])
    dm = orc.aggregate(CM, 8, 20, 120).argmin(axis=2)[:, ::-1]
    assert np.array_equal(orc.right_disp_full(cl, cr, D, bits, 8, 20, 120, 3, 3), dm)
