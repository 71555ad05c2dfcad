"""Parity of the multi-scalar multiplication (Alg. 2, LS-PPG, and its
Presort-PPG baseline) and the batch scalar multiplication with the oracle,
bit-exact: the result is an affine
point in canonical form, which is unique, so the HIP output must equal the
oracle's word for word.

Cases: small inputs against the plain sum of products for window widths
1..20 (one window, many windows, a ragged top window) and the edge scalars
(0, 1, r - 1, 2^256 - 1, the subgroup order, equal points, a point and its
negative, the points of order 1, 2 and 4); medium and ragged sizes with walk-generated points, whose sum has
a closed form by linearity; and the full 2^22-point configuration with points
k_i G produced by the batch scalar multiplication, where the result must be
((sum_i S_i k_i) mod l) G. The oracle (oracle/msm.py) is pinned in
test_msm_oracle.py."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import seeded_inputs as si
from oracle import msm as M

torch = pytest.importorskip("torch")
import paper_2604_17808_amd as fr  # noqa: E402
from paper_2604_17808_amd import frntt as B  # noqa: E402

pytestmark = pytest.mark.gpu

L_ORDER = 2736030358979909402780800718157159386076813972158567259200215660948447373041
BASE8 = (5299619240641551281634865583518297030282874472190772894086521144482721001553,
         16950150798460657717958625567821834550301663161624707787222815936182638968203)
ORDER = 8 * L_ORDER  # kills every point of the curve


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = fr.Context(0, max_log_n=12)
    yield c
    torch.cuda.synchronize()
    c.close()


def _dev_words(ints):
    """Python integers below 2^256 -> (n, 8) uint32 device tensor."""
    a = si.from_ints(ints) if len(ints) else np.zeros((0, 4), dtype=np.uint64)
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int32).reshape(-1, 8)).cuda()


def _dev_points(points):
    xs = _dev_words([p[0] for p in points])
    ys = _dev_words([p[1] for p in points])
    return torch.cat([xs, ys], dim=1).contiguous()


def _host_point(t):
    w = t.cpu().view(torch.int32).numpy().view(np.uint32).astype(np.uint64)
    x = sum(int(w[i]) << (32 * i) for i in range(8))
    y = sum(int(w[8 + i]) << (32 * i) for i in range(8))
    return (x, y)


def _host_points(t):
    w = t.cpu().view(torch.int32).numpy().view(np.uint32).astype(np.uint64).reshape(-1, 16)
    out = []
    for row in w:
        out.append((sum(int(row[i]) << (32 * i) for i in range(8)),
                    sum(int(row[8 + i]) << (32 * i) for i in range(8))))
    return out


def _msm(ctx, scalars, points, window=0):
    """LS-PPG result, after checking that the Presort-PPG baseline agrees."""
    n = len(scalars)
    sc = _dev_words(scalars) if n else torch.zeros((1, 8), dtype=torch.int32, device="cuda")
    pt = _dev_points(points) if n else torch.zeros((1, 16), dtype=torch.int32, device="cuda")
    out = torch.empty(16, dtype=torch.int32, device="cuda")
    base = torch.empty(16, dtype=torch.int32, device="cuda")
    ctx.msm(sc.data_ptr(), pt.data_ptr(), n, out.data_ptr(), window)
    ctx.msm_presort(sc.data_ptr(), pt.data_ptr(), n, base.data_ptr(), window)
    torch.cuda.synchronize()
    got = _host_point(out)
    assert _host_point(base) == got, "Presort-PPG and LS-PPG differ"
    return got


def _rand_points(n, seed):
    rnd = np.random.default_rng(seed)
    out = []
    while len(out) < n:
        x = int.from_bytes(rnd.bytes(32), "little") % M.R
        p = M.point_from_x(x)
        if p is not None:
            out.append(p)
    return out


def _walk_points(n, seed, m=16):
    """P_i = base_(i mod m) + (i div m) H, with random base points and H."""
    pts = _rand_points(m + 1, seed)
    bases, h = pts[:m], pts[m]
    cur = list(bases)
    out = []
    while len(out) < n:
        for b in range(m):
            if len(out) == n:
                break
            out.append(cur[b])
            cur[b] = M.add(cur[b], h)
    return out, bases, h


def _walk_expected(scalars, bases, h):
    m = len(bases)
    acc = M.ZERO
    for b in range(m):
        acc = M.add(acc, M.mul(sum(scalars[b::m]) % ORDER, bases[b]))
    hs = sum(s * (i // m) for i, s in enumerate(scalars)) % ORDER
    return M.add(acc, M.mul(hs, h))


def _scalars(n, seed):
    return si.to_ints(si.field_elements(seed, n, stream=7))


EDGE = [0, 1, (1 << 256) - 1, M.R - 1, L_ORDER, 1 << 255, ORDER]


@pytest.mark.parametrize("window", [1, 2, 4, 7, 13, 16, 20])
def test_msm_small_matches_sum_of_products(ctx, window):
    pts = _rand_points(len(EDGE) + 6, 100 + window)
    sc = EDGE + _scalars(6, 200 + window)
    _say(f"msm small window={window} n={len(sc)}")
    assert _msm(ctx, sc, pts, window) == M.msm_naive(sc, pts)


@pytest.mark.parametrize("n", [1, 2, 3, 17])
def test_msm_tiny_auto_window(ctx, n):
    pts = _rand_points(n, 300 + n)
    sc = _scalars(n, 400 + n)
    _say(f"msm tiny n={n} window={fr.msm_window(n)}")
    assert _msm(ctx, sc, pts) == M.msm_naive(sc, pts)


def test_msm_empty_is_zero_point(ctx):
    assert _msm(ctx, [], []) == M.ZERO


def test_msm_cancelling_and_equal_terms(ctx):
    p, q = _rand_points(2, 500)
    # equal points and scalars share buckets; P and -P with one scalar cancel
    sc = [5, 5, 5, 9, 12345, 12345, 0, 77]
    pts = [p, p, q, q, p, M.neg(p), q, M.neg(q)]
    for window in (0, 3, 8):
        assert _msm(ctx, sc, pts, window) == M.msm_naive(sc, pts)
    assert _msm(ctx, [ORDER, L_ORDER * 8], [p, q]) == M.ZERO
    assert _msm(ctx, [0] * 5, [p, q, p, q, p]) == M.ZERO


def test_msm_non_canonical_coordinates_read_mod_r(ctx):
    p = _rand_points(1, 600)[0]
    q = (p[0] + M.R, p[1] + M.R)  # still below 2^256
    assert q[0] < (1 << 256) and q[1] < (1 << 256)
    assert _msm(ctx, [123456789], [q]) == M.mul(123456789, p)


@pytest.mark.parametrize("n,window", [(4096, 0), (4096 + 37, 5), (65536 + 11, 0)])
def test_msm_walk_points_closed_form(ctx, n, window):
    pts, bases, h = _walk_points(n, 700 + n)
    sc = _scalars(n, 800 + n)
    _say(f"msm walk n={n} window={window or fr.msm_window(n)}")
    assert _msm(ctx, sc, pts, window) == _walk_expected(sc, bases, h)


@pytest.mark.parametrize("kind", ["equal", "top_bits", "small"])
def test_msm_skewed_digits(ctx, kind):
    # buckets far above the mean size: every point in one bucket per window,
    # a third of the points in each of three top-window buckets, or only the
    # low windows in use
    n = 40000
    pts, bases, h = _walk_points(n, 1000)
    rnd = np.random.default_rng(5)
    if kind == "equal":
        sc = [0x1234567890ABCDEF1234567890ABCDEF] * n
    elif kind == "top_bits":
        sc = [int(v) << 252 for v in rnd.integers(1, 4, n)]
    else:
        sc = [int(v) for v in rnd.integers(0, 1 << 20, n)]
    for window in (0, 14):
        _say(f"msm skewed {kind} n={n} window={window or fr.msm_window(n)}")
        assert _msm(ctx, sc, pts, window) == _walk_expected(sc, bases, h)


def test_ec_mul_matches_oracle(ctx):
    n = 40
    pts = _rand_points(n, 900)
    sc = EDGE + _scalars(n - len(EDGE), 901)
    out = torch.empty((n, 16), dtype=torch.int32, device="cuda")
    s_t, p_t = _dev_words(sc), _dev_points(pts)
    ctx.ec_mul(s_t.data_ptr(), p_t.data_ptr(), n, out.data_ptr())
    torch.cuda.synchronize()
    got = _host_points(out)
    for i in range(n):
        assert got[i] == M.mul(sc[i], pts[i]), i


def _full_size_inputs(ctx, n):
    k = si.field_elements(11, n, stream=1)
    s = si.field_elements(11, n, stream=2)
    k_t = torch.from_numpy(k.view(np.int32).reshape(n, 8)).cuda()
    s_t = torch.from_numpy(s.view(np.int32).reshape(n, 8)).cuda()
    g = _dev_points([BASE8]).expand(n, 16).contiguous()
    pts = torch.empty((n, 16), dtype=torch.int32, device="cuda")
    ctx.ec_mul(k_t.data_ptr(), g.data_ptr(), n, pts.data_ptr())
    torch.cuda.synchronize()
    del g
    return k, s, s_t, pts


def test_msm_full_size_generator_multiples(ctx):
    n = 1 << 22
    _say(f"msm full size n={n} window={fr.msm_window(n)}")
    k, s, s_t, pts = _full_size_inputs(ctx, n)
    # a sample of the generated points against the oracle
    got = _host_points(pts[[0, 1, n // 3, n - 1]])
    kk = si.to_ints(k[[0, 1, n // 3, n - 1]])
    for j in range(4):
        assert got[j] == M.mul(kk[j], BASE8)
    out = torch.empty(16, dtype=torch.int32, device="cuda")
    base = torch.empty(16, dtype=torch.int32, device="cuda")
    ctx.msm(s_t.data_ptr(), pts.data_ptr(), n, out.data_ptr())
    ctx.msm_presort(s_t.data_ptr(), pts.data_ptr(), n, base.data_ptr())
    torch.cuda.synchronize()
    total = sum(a * b for a, b in zip(si.to_ints(s), si.to_ints(k))) % L_ORDER
    assert _host_point(out) == M.mul(total, BASE8)
    assert _host_point(base) == _host_point(out)


def test_msm_argument_errors(ctx):
    L = fr.lib()
    t = torch.zeros((8, 16), dtype=torch.int32, device="cuda")
    o = torch.zeros(16, dtype=torch.int32, device="cuda")
    p = t.data_ptr()
    assert L.frntt_msm(None, p, p, 1, 0, o.data_ptr(), None) == B.EINVAL
    assert L.frntt_msm(ctx._h, None, p, 1, 0, o.data_ptr(), None) == B.EINVAL
    assert L.frntt_msm(ctx._h, p, p, 1, 0, None, None) == B.EINVAL
    assert L.frntt_msm(ctx._h, p, p, -1, 0, o.data_ptr(), None) == B.EINVAL
    assert L.frntt_msm(ctx._h, p, p, 1, 21, o.data_ptr(), None) == B.ERANGE
    assert L.frntt_msm(ctx._h, p, p, 1, -1, o.data_ptr(), None) == B.ERANGE
    assert L.frntt_msm(ctx._h, p, p, (1 << 28) + 1, 0, o.data_ptr(), None) == B.ERANGE
    assert L.frntt_msm(ctx._h, p + 4, p, 1, 0, o.data_ptr(), None) == B.EALIGN
    assert L.frntt_msm_presort(ctx._h, p, p + 4, 1, 0, o.data_ptr(), None) == B.EALIGN
    assert L.frntt_msm_presort(ctx._h, p, p, 1, 21, o.data_ptr(), None) == B.ERANGE
    assert L.frntt_ec_mul(ctx._h, p, p + 4, 1, o.data_ptr(), None) == B.EALIGN
    assert L.frntt_ec_mul(ctx._h, p, p, -1, o.data_ptr(), None) == B.EINVAL
    assert L.frntt_ec_mul(ctx._h, p, p, 0, o.data_ptr(), None) == B.OK
    assert fr.msm_workspace_bytes(-1) == 0 and fr.msm_workspace_bytes(10, 21) == 0


def test_msm_refuses_stream_capture(ctx):
    # an MSM is never captured into a graph (its sort clears counters with
    # memset nodes): under a capture the call returns ESTATE, enqueues
    # nothing, and the stream works as before afterwards
    pts = _rand_points(3, 1100)
    sc = _scalars(3, 1101)
    s_t, p_t = _dev_words(sc), _dev_points(pts)
    out = torch.full((16,), 7, dtype=torch.int32, device="cuda")
    st = torch.cuda.Stream()
    L = fr.lib()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(st):
        with torch.cuda.graph(g, stream=st):
            rc = L.frntt_msm(ctx._h, s_t.data_ptr(), p_t.data_ptr(), 3, 0, out.data_ptr(), st.cuda_stream)
            rcb = L.frntt_msm_presort(ctx._h, s_t.data_ptr(), p_t.data_ptr(), 3, 0, out.data_ptr(),
                                      st.cuda_stream)
    assert rc == B.ESTATE and rcb == B.ESTATE
    torch.cuda.synchronize()
    assert bool((out == 7).all())
    with torch.cuda.stream(st):
        ctx.msm(s_t.data_ptr(), p_t.data_ptr(), 3, out.data_ptr(), 0, st.cuda_stream)
    torch.cuda.synchronize()
    assert _host_point(out) == M.msm_naive(sc, pts)


def _small_order_points():
    """The zero point (0, 1), the point of order 2 (0, -1) and the two
    points of order 4 (+-1/sqrt(a), 0)."""
    u = pow(M.sqrt_mod(M.A), -1, M.R)
    pts = [(0, 1), (0, M.R - 1), (u, 0), (M.R - u, 0)]
    assert all(M.on_curve(p) for p in pts)
    return pts


def test_msm_small_order_points(ctx):
    tors = _small_order_points()
    rnd = _rand_points(4, 1200)
    pts = tors + rnd + tors
    sc = [5, 7, 9, 11] + _scalars(4, 1201) + [(1 << 256) - 1, 2, 3, 1]
    for window in (0, 2, 5, 16):
        assert _msm(ctx, sc, pts, window) == M.msm_naive(sc, pts)
    # only small-order points: the sum is a small-order point too
    assert _msm(ctx, [3, 1, 1, 2], tors) == M.msm_naive([3, 1, 1, 2], tors)


def test_ec_mul_small_order_points(ctx):
    tors = _small_order_points()
    pts = tors * 3
    sc = [0, 1, 2, 3, 4, 5, 6, 7, (1 << 256) - 1, M.R - 1, 8, 9]
    out = torch.empty((len(pts), 16), dtype=torch.int32, device="cuda")
    s_t, p_t = _dev_words(sc), _dev_points(pts)
    ctx.ec_mul(s_t.data_ptr(), p_t.data_ptr(), len(pts), out.data_ptr())
    torch.cuda.synchronize()
    got = _host_points(out)
    for i in range(len(pts)):
        assert got[i] == M.mul(sc[i], pts[i]), i


def test_msm_batch_matches_single_calls(ctx):
    # independent MSMs of different sizes (one empty) on the side streams,
    # each against the oracle
    sizes = [4096 + 3, 0, 17, 40000]
    cases = []
    for j, n in enumerate(sizes):
        pts, bases, h = _walk_points(n, 1300 + j) if n else ([], [], None)
        sc = _scalars(n, 1400 + j)
        want = _walk_expected(sc, bases, h) if n else M.ZERO
        s_t = _dev_words(sc) if n else torch.zeros((1, 8), dtype=torch.int32, device="cuda")
        p_t = _dev_points(pts) if n else torch.zeros((1, 16), dtype=torch.int32, device="cuda")
        cases.append((n, s_t, p_t, torch.full((16,), 5, dtype=torch.int32, device="cuda"), want))
    for window in (0, 9):
        ctx.msm_batch([c[1].data_ptr() for c in cases], [c[2].data_ptr() for c in cases],
                      [c[0] for c in cases], [c[3].data_ptr() for c in cases], window)
        torch.cuda.synchronize()
        for n, _, _, o, want in cases:
            assert _host_point(o) == want, (n, window)


def test_msm_batch_argument_errors(ctx):
    t = torch.zeros((8, 16), dtype=torch.int32, device="cuda")
    o = torch.full((16,), 3, dtype=torch.int32, device="cuda")
    p = t.data_ptr()
    with pytest.raises(B.FrnttError) as e:
        ctx.msm_batch([p, p], [p, p + 4], [1, 1], [o.data_ptr(), o.data_ptr()])
    assert e.value.status == B.EALIGN
    with pytest.raises(B.FrnttError) as e:
        ctx.msm_batch([p], [p], [-1], [o.data_ptr()])
    assert e.value.status == B.EINVAL
    with pytest.raises(B.FrnttError) as e:
        ctx.msm_batch([p], [p], [1], [o.data_ptr()], window=21)
    assert e.value.status == B.ERANGE
    torch.cuda.synchronize()
    assert bool((o == 3).all())  # nothing ran
    assert ctx.msm_batch([], [], [], []) == B.OK
