"""GPU parity of the learned cross-rank path: the network's forward /
backward / Adam / initialisation against the FP64 oracle (tolerance), the
bounded search against the oracle's search (bit-exact ranks, probes and
fallbacks), the learned partition against the oracle's cross ranks
(bit-exact), and the gain of the trained network over the plain search."""
import numpy as np
import pytest
import torch

import datagen
import oracle
from helpers import dev, flush, host, rand_sorted
from oracle import mlp

pytestmark = pytest.mark.gpu

import paper_1202_6575_amd as sm  # noqa: E402
from paper_1202_6575_amd import learned  # noqa: E402

DTYPES = [np.int32, np.uint32, np.uint64, np.int64, np.float32, np.float64]


def f32(a):
    return np.asarray(a, dtype=np.float32)


def grad_tol(g_ref):
    return 1e-4 * np.max(np.abs(g_ref)) + 1e-6


@pytest.mark.parametrize("dtype", DTYPES)
def test_mlp_grad_matches_oracle(dtype):
    g = np.random.default_rng(1)
    for S in (1, 1000, 70_001):
        keys = rand_sorted(g, S, 1 << 20, dtype)
        target = f32(g.random(S))
        params = f32(g.normal(size=mlp.NPARAM) * np.r_[np.full(32, 2.0), np.full(32, 0.5),
                                                       np.full(33, 0.3)])
        flush(f"mlp grad dtype={np.dtype(dtype).name} S={S}")
        grad, loss = learned.mlp_grad(dev(params), dev(keys), dev(target))
        torch.cuda.synchronize()
        L_ref, g_ref = mlp.loss_and_grad(params.astype(np.float64), mlp.features(keys),
                                         target.astype(np.float64))
        gg = host(grad).astype(np.float64)
        assert np.all(np.abs(gg - g_ref) <= grad_tol(g_ref)), np.max(np.abs(gg - g_ref))
        assert abs(float(host(loss)[0]) - L_ref) <= 1e-5 * abs(L_ref) + 1e-9


def test_mlp_grad_reproducible():
    g = np.random.default_rng(2)
    keys = dev(rand_sorted(g, 300_000, 1 << 30, np.uint32))
    target = dev(f32(g.random(300_000)))
    params = dev(f32(g.normal(size=mlp.NPARAM)))
    a = learned.mlp_grad(params, keys, target)
    b = learned.mlp_grad(params, keys, target)
    torch.cuda.synchronize()
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])


def test_mlp_adam_matches_oracle():
    g = np.random.default_rng(3)
    p = f32(g.normal(size=mlp.NPARAM))
    m = f32(g.normal(size=mlp.NPARAM) * 0.1)
    v = f32(g.random(mlp.NPARAM) * 0.01)
    grad = f32(g.normal(size=mlp.NPARAM))
    for step in (1, 2, 17, 1000):
        dp, dm, dv = dev(p), dev(m), dev(v)
        learned.mlp_adam(dp, dm, dv, dev(grad), step, 3e-3)
        torch.cuda.synchronize()
        # the oracle takes the same (FP32) hyper-parameters the kernel receives
        b1, b2, eps, lr = (float(np.float32(x)) for x in (0.9, 0.999, 1e-8, 3e-3))
        rp, rm, rv = mlp.adam_step(p.astype(np.float64), grad.astype(np.float64),
                                   m.astype(np.float64), v.astype(np.float64), step, lr,
                                   b1, b2, eps)
        # FP32 updates: a few ulps of the largest operand of each update
        ulp = lambda a: 4 * np.spacing(np.float32(np.max(np.abs(a))))
        assert np.all(np.abs(host(dm) - rm) <= ulp(m) + ulp(grad) * 0.1)
        assert np.all(np.abs(host(dv) - rv) <= ulp(v) + ulp(grad * grad) * 1e-3)
        assert np.all(np.abs(host(dp) - rp) <= ulp(p) + 1e-5 * 3e-3)


@pytest.mark.parametrize("dtype", DTYPES)
def test_mlp_init_and_predict_match_oracle(dtype):
    g = np.random.default_rng(4)
    keys = rand_sorted(g, 40_000, 1 << 16, dtype)
    target = f32(np.sort(g.random(40_000)))
    p = learned.mlp_init(dev(keys), dev(target))
    torch.cuda.synchronize()
    ref = mlp.init_params(mlp.features(keys), target.astype(np.float64))
    got = host(p).astype(np.float64)
    assert np.allclose(got[0:64], ref[0:64], rtol=1e-6, atol=1e-7)
    assert np.allclose(got[96], ref[96], rtol=1e-6)
    # output weights are differences of slopes t-gap / knot-gap.  The GPU's
    # knots are FP32 features, within delta = 4 ulp(1) = 2^-21 of the FP64
    # ones, so a slope s over a gap g is off by up to |s| * 2 delta / g (the
    # bound grows where keys crowd into a narrow feature range)
    c = -ref[32:64]
    gaps = np.diff(c)
    delta = 2.0 ** -21
    slope = np.cumsum(ref[64:96])[:31]
    slope_err = np.where(gaps > 1e-6, np.abs(slope) * 2 * delta / np.maximum(gaps, 1e-30), 0.0)
    bound = np.concatenate([slope_err, [0.0]]) + np.concatenate([[0.0], slope_err])
    assert np.all(np.abs(got[64:96] - ref[64:96]) <= 2 * bound + 1e-4 * np.max(np.abs(ref[64:96])) + 1e-6)
    # predictions of the GPU network against the oracle's own network: the
    # interpolant moves by at most the steepest slope times the knot and
    # query feature shifts (4 delta)
    q = rand_sorted(g, 5000, 1 << 16, dtype)
    L = 1 << 24
    rh = host(learned.mlp_predict(p, dev(q), L))
    rr = mlp.predict_rank(ref, q, L)
    steep = float(np.max(np.abs(slope))) if len(slope) else 0.0
    assert np.max(np.abs(rh - rr)) <= (1e-4 + 4 * delta * steep) * L + 1


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("is_high", [False, True])
def test_rank_search_matches_oracle(dtype, is_high):
    """Guesses = exact rank + seeded errors; every rank, probe count and
    fallback flag equals the oracle's search."""
    g = np.random.default_rng(5)
    X = rand_sorted(g, 100_000, 5000, dtype)
    Q = rand_sorted(g, 600, 5200, dtype)
    exact = np.array([oracle.rank_high(x, X) if is_high else oracle.rank_low(x, X) for x in Q])
    dX, dQ = dev(X), dev(Q)
    for spread in (0, 3, 100, 5000, 200_000):
        err = (g.normal(size=len(Q)) * spread).astype(np.int64) if spread else np.zeros(len(Q), np.int64)
        guess = exact + err
        for step0 in (1, 4, 64):
            for window in (0, 16, 1024, 1 << 20):
                flush(f"search dtype={np.dtype(dtype).name} high={is_high} spread={spread} "
                      f"step0={step0} W={window}")
                r, pr, fb = learned.rank_search(dX, dQ, dev(guess), is_high, step0, window)
                torch.cuda.synchronize()
                r, pr, fb = host(r), host(pr), host(fb)
                assert np.array_equal(r, exact)
                for i in range(0, len(Q), 7):
                    rr, pp, ff = oracle.gallop(Q[i], X, is_high, int(guess[i]), window, step0)
                    assert (rr, pp, ff) == (r[i], pr[i], bool(fb[i])), i


@pytest.mark.slow
@pytest.mark.parametrize("is_high", [False, True])
def test_rank_search_beyond_2e31(is_high):
    """An array of 2^31 + 2^20 uint32 keys (the 64-bit bisection of the
    corrective search): X[i] = floor(i / 2), so rank_low(q) = 2q and
    rank_high(q) = 2q + 2 for q below the largest key; guesses far off and
    a window that forces the fallback half the time."""
    N = (1 << 31) + (1 << 20)
    X = (torch.arange(N, device="cuda:0", dtype=torch.int64) // 2).to(torch.uint32)
    g = np.random.default_rng(31)
    q = np.sort(g.integers(0, N // 2 - 1, size=4096)).astype(np.int64)
    exact = 2 * q + (2 if is_high else 0)
    guess = np.clip(exact + g.integers(-(1 << 31), 1 << 31, size=len(q)), 0, N)
    flush(f"rank search beyond 2^31 high={is_high}")
    r, _, fb = learned.rank_search(X, dev(q.astype(np.uint32)), dev(guess), is_high, 1, 1 << 30)
    torch.cuda.synchronize()
    assert np.array_equal(host(r), exact)
    assert 0 < int(host(fb).sum()) < len(q)
    del X


@pytest.mark.slow
def test_merge_learned_lognormal_2e28_full():
    """The learned-partition workload at full size: n = m = 2^28 uint32 keys
    from the log-normal mixture, blocks of 16, trained models; the whole
    output equals the oracle's merge."""
    import datagen.torch_gen as tg
    n = m = 1 << 28
    flush("learned 2^28 generate")
    A = tg.lognormal_mixture(n, seed=datagen.BASE_SEED + 6)
    B = tg.lognormal_mixture(m, seed=datagen.BASE_SEED + 7)
    pb, lb = learned.train_rank_model(B, A, False, 1 << 18, 400, seed=11)
    pa, la = learned.train_rank_model(A, B, True, 1 << 18, 400, seed=12)
    torch.cuda.synchronize()
    s0a = learned.step0_from_loss(float(host(lb)[0]), m)
    s0b = learned.step0_from_loss(float(host(la)[0]), n)
    keys = torch.cat([A, B])
    flush("learned 2^28 merge")
    ok, _, hist, cnt = learned.merge_learned(keys, n, m, pb, pa, s0a, s0b, 16, 1 << 24)
    torch.cuda.synchronize()
    got = host(ok)
    c = host(cnt).astype(np.int64)
    assert c[0] == 2 * (n // 16)
    flush("learned 2^28 oracle")
    ref, _ = oracle.merge(host(A), host(B))
    assert np.array_equal(got, ref)


def train_pair(A, B, samples=1 << 15, steps=400):
    dA, dB = dev(A), dev(B)
    pb, lb = learned.train_rank_model(dB, dA, False, samples, steps, seed=11)   # B's CDF, A's queries
    pa, la = learned.train_rank_model(dA, dB, True, samples, steps, seed=12)    # A's CDF, B's queries
    torch.cuda.synchronize()
    return pb, float(host(lb)[0]), pa, float(host(la)[0])


def test_learned_partition_exact():
    """Any window and initial step: the same cross ranks as the oracle."""
    n, m = 1 << 20, 600_000
    A = datagen.lognormal_mixture(n, 21)
    B = datagen.lognormal_mixture(m, 22)
    pb, lb, pa, la = train_pair(A, B)
    keys = dev(np.concatenate([A, B]))
    p_a, p_b = n // 16, (m + 15) // 16
    xr, yr = oracle.cross_ranks(A, B, p_a, p_b)
    s0a, s0b = learned.step0_from_loss(lb, m), learned.step0_from_loss(la, n)
    for (sa, sb, W) in [(1, 1, 0), (1, 1, 64), (s0a, s0b, 1 << 40), (s0a, s0b, 4 * s0a),
                        (64, 64, 1024)]:
        flush(f"learned partition step0=({sa},{sb}) W={W}")
        xb, yb, hist, cnt = learned.partition_learned(keys, n, m, p_a, p_b, pb, pa, sa, sb, W)
        torch.cuda.synchronize()
        assert np.array_equal(host(xb), xr) and np.array_equal(host(yb), yr)
        h, c = host(hist).astype(np.int64), host(cnt).astype(np.int64)
        assert c[0] == p_a + p_b and h.sum() == c[0]
        if W == 0:
            assert c[1] == c[0]                       # every walk is refused: all fall back
        if W >= 1 << 40:
            assert c[1] == 0
    # a network that predicts nothing useful (all parameters zero: every
    # guess is 0) changes only the work, never the ranks
    zero = torch.zeros(learned.NPARAM, dtype=torch.float32, device="cuda:0")
    for W in (0, 64, 1 << 40):
        xz, yz, hz, cz = learned.partition_learned(keys, n, m, p_a, p_b, zero, zero, 1, 1, W)
        torch.cuda.synchronize()
        assert np.array_equal(host(xz), xr) and np.array_equal(host(yz), yr)
    # the ranks drive the merge: output equals the oracle's merge
    ck, _ = sm.merge_pieces(keys, n, m, p_a, p_b, xb, yb)
    torch.cuda.synchronize()
    assert np.array_equal(host(ck), oracle.merge(A, B)[0])


def test_merge_learned_end_to_end():
    """The composite entry point: learned partition + Steps 3-4 give the
    oracle's stable merge (keys and payloads) for several block lengths,
    windows and a model that predicts nothing useful."""
    n, m = 300_001, 200_003
    A = datagen.lognormal_mixture(n, 41)
    B = datagen.lognormal_mixture(m, 42)
    pb, lb, pa, la = train_pair(A, B, samples=1 << 14, steps=200)
    keys = dev(np.concatenate([A, B]))
    pay = np.arange(n + m, dtype=np.uint32)
    rk, rp = oracle.merge(A, B, pay[:n], pay[n:])
    zero = torch.zeros(learned.NPARAM, dtype=torch.float32, device="cuda:0")
    s0a, s0b = learned.step0_from_loss(lb, m), learned.step0_from_loss(la, n)
    for (mb, ma, sa, sb, block, W) in [(pb, pa, s0a, s0b, 16, 1 << 40), (pb, pa, 1, 1, 16, 64),
                                       (pb, pa, s0a, s0b, 1, 1 << 20), (pb, pa, 1, 1, 64, 256),
                                       (zero, zero, 1, 1, 16, 0), (pb, pa, 1, 1, 5000, 256)]:
        flush(f"merge_learned block={block} W={W} step0=({sa},{sb})")
        ok, op, hist, cnt = learned.merge_learned(keys, n, m, mb, ma, sa, sb, block, W, dev(pay))
        torch.cuda.synchronize()
        assert np.array_equal(host(ok), rk) and np.array_equal(host(op), rp)
        c = host(cnt).astype(np.int64)
        pa_, pb_ = -(-n // block), -(-m // block)
        assert c[0] == pa_ + pb_ and host(hist).astype(np.int64).sum() == c[0]
        okk, _, _, _ = learned.merge_learned(keys, n, m, mb, ma, sa, sb, block, W)
        torch.cuda.synchronize()
        assert np.array_equal(host(okk), rk)
    # empty sides
    for (nn, mm) in [(0, 1000), (1000, 0), (0, 0), (1, 1)]:
        A2, B2 = A[:nn], B[:mm]
        k2 = dev(np.concatenate([A2, B2])) if nn + mm else dev(np.zeros(1, np.uint32))
        ok, _, _, _ = learned.merge_learned(k2, nn, mm, pb, pa, 1, 1, 16, 256)
        torch.cuda.synchronize()
        assert np.array_equal(host(ok)[:nn + mm], oracle.merge(A2, B2)[0])


def test_merge_learned_errors():
    keys = dev(np.arange(100, dtype=np.uint32))
    zero = torch.zeros(learned.NPARAM, dtype=torch.float32, device="cuda:0")
    with pytest.raises(sm.SMError):
        learned.merge_learned(keys, 50, 50, zero, zero, 1, 1, 0, 256)
    with pytest.raises(sm.SMError):
        learned.merge_learned(keys, 50, 50, zero, zero, 1, 1, 16, 256, out_keys=keys)
    small = torch.empty(8, dtype=torch.uint8, device="cuda:0")
    with pytest.raises(sm.SMError) as e:
        learned.merge_learned(keys, 50, 50, zero, zero, 1, 1, 16, 256, workspace=small)
    assert e.value.code == -4


def test_trained_network_gain():
    """On the log-normal mixture, the trained network brings the search to
    fewer probes per rank than the plain binary search (floor(log2 len) + 1
    reads), and training lowers the rank error of the initial network."""
    n = m = 1 << 22
    A = datagen.lognormal_mixture(n, 31)
    B = datagen.lognormal_mixture(m, 32)
    dA, dB = dev(A), dev(B)
    keys = dev(np.concatenate([A, B]))
    p_a = p_b = n // 16
    pb0, lb0 = learned.train_rank_model(dB, dA, False, 1 << 16, 0, seed=1)     # init only
    pb, lb = learned.train_rank_model(dB, dA, False, 1 << 16, 1000, seed=1)
    pa, la = learned.train_rank_model(dA, dB, True, 1 << 16, 1000, seed=2)
    torch.cuda.synchronize()
    lb0, lb, la = float(host(lb0)[0]), float(host(lb)[0]), float(host(la)[0])
    flush(f"rms before {np.sqrt(lb0) * m:.0f} after {np.sqrt(lb) * m:.0f}")
    assert lb < lb0
    s0a, s0b = learned.step0_from_loss(lb, m), learned.step0_from_loss(la, n)
    xb, yb, hist, cnt = learned.partition_learned(keys, n, m, p_a, p_b, pb, pa, s0a, s0b, 1 << 40)
    torch.cuda.synchronize()
    c = host(cnt).astype(np.int64)
    learned_probes = c[2] / c[0]
    plain_probes = int(np.floor(np.log2(m))) + 1
    flush(f"probes per rank: learned {learned_probes:.2f} plain {plain_probes}")
    assert learned_probes < plain_probes - 3
    xr, yr = oracle.cross_ranks(A, B, p_a, p_b)
    assert np.array_equal(host(xb), xr) and np.array_equal(host(yb), yr)


def test_predictor_save_load_round_trip():
    """A trained handle saved to host bytes and loaded again holds the same
    parameters and metadata, and the whole learned merge through either
    handle writes the same bytes (and the same histogram and counters) --
    the oracle's merge."""
    g = np.random.default_rng(91)
    n, m = 300_001, 200_003
    A, B = rand_sorted(g, n, 1 << 24, np.uint32), rand_sorted(g, m, 1 << 24, np.uint32)
    keys = dev(np.concatenate([A, B]))
    flush("predictor create / train / save / load")
    pb = learned.Predictor.create(torch.uint32, False).train(keys[n:], keys[:n], samples=1 << 14,
                                                             steps=200, seed=3)
    pa = learned.Predictor.create(torch.uint32, True).train(keys[:n], keys[n:], samples=1 << 14,
                                                            steps=200, seed=4)
    blob_b, blob_a = pb.save(), pa.save()
    assert len(blob_b) == learned.BLOB_BYTES == 432
    lb, la = learned.Predictor.load(blob_b), learned.Predictor.load(blob_a)
    assert lb.save() == blob_b and la.save() == blob_a
    assert torch.equal(lb.params(), pb.params()) and torch.equal(la.params(), pa.params())
    ib, il = pb.info(), lb.info()
    assert ib == il and ib[0] == 1 and ib[1] is False and ib[2] == m and ib[3] < 1.0
    assert la.info()[1] is True and la.info()[2] == n
    s0a = learned.step0_from_loss(ib[3], m)
    s0b = learned.step0_from_loss(la.info()[3], n)
    outs = []
    for mb, ma in ((pb, pa), (lb, la)):
        ok, _, h, c = learned.merge_learned(keys, n, m, mb, ma, s0a, s0b, block=16, window=1 << 12)
        torch.cuda.synchronize()
        outs.append((host(ok), host(h), host(c)))
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1]) and np.array_equal(outs[0][2], outs[1][2])
    ref, _ = oracle.merge(A, B)
    assert np.array_equal(outs[0][0], ref)
    # the loaded handle outlives the one it came from
    pb.close()
    ok, _, _, _ = learned.merge_learned(keys, n, m, lb, la, s0a, s0b, block=16, window=1 << 12)
    torch.cuda.synchronize()
    assert np.array_equal(host(ok), ref)
    for h in (pa, lb, la):
        h.close()
