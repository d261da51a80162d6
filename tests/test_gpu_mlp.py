"""The learned variant dispatcher on the GPU: its forward pass, gradient and
Adam step against the fp64 reference (oracle/mlp.py), training on costs the
count kernels measure, and dispatch through the trained network leaving every
result unchanged."""
import sys

import numpy as np
import pytest

import oracle
import synth
from oracle import mlp

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def rg():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1709_07821_amd as rg

    return rg


@pytest.fixture(scope="module")
def ctx(rg):
    c = rg.Context(0)
    yield c
    c.close()


def _problem(seed, n):
    rng = np.random.default_rng(seed)
    p = rng.normal(0.0, 0.3, mlp.N_PARAMS).astype(np.float32)
    x = rng.normal(0.0, 1.0, (n, 12)).astype(np.float32)
    t = rng.normal(0.0, 1.0, (n, 6)).astype(np.float32)
    m = (rng.random((n, 6)) < 0.7).astype(np.uint8)
    return p, x, t, m


@pytest.mark.parametrize("n", [1, 255, 700])
def test_forward_and_gradient_match_fp64_reference(rg, ctx, n):
    import torch

    p, x, t, m = _problem(n, n)
    dev = "cuda"
    tp, tx, tt, tm = (torch.from_numpy(a).to(dev) for a in (p, x, t, m))
    y = rg.mlp_forward(ctx, tp, tx).cpu().numpy().astype(np.float64)
    y0, _ = mlp.forward(p.astype(np.float64), x.astype(np.float64))
    assert np.abs(y - y0).max() <= 1e-5 * max(1.0, np.abs(y0).max())
    g, loss = rg.mlp_grad(ctx, tp, tx, tt, tm)
    g0 = mlp.grad(p.astype(np.float64), x.astype(np.float64), t.astype(np.float64), m.astype(np.float64))
    l0 = mlp.loss(p.astype(np.float64), x.astype(np.float64), t.astype(np.float64), m.astype(np.float64))
    got, ref = mlp.unpack(g.cpu().numpy().astype(np.float64)), mlp.unpack(g0)
    for k in ref:
        d = np.abs(got[k] - ref[k]).max()
        assert d <= 1e-4 * np.abs(ref[k]).max() + 1e-7, (n, k, d)
    assert abs(float(loss.item()) - l0) <= 1e-5 * max(1.0, l0)


def test_adam_steps_match_reference(rg, ctx):
    import torch

    p, x, t, m = _problem(3, 300)
    tp = torch.from_numpy(p).cuda()
    am = torch.zeros_like(tp)
    av = torch.zeros_like(tp)
    rp, rm, rv = p.astype(np.float64), np.zeros(mlp.N_PARAMS), np.zeros(mlp.N_PARAMS)
    for step in range(1, 4):
        g = mlp.grad(rp, x, t, m).astype(np.float32)
        rg.mlp_adam(ctx, tp, torch.from_numpy(g).cuda(), am, av, step, 1e-3)
        rp, rm, rv = mlp.adam(rp, g.astype(np.float64), rm, rv, step, lr=1e-3)
        torch.cuda.synchronize()
    assert np.abs(tp.cpu().numpy() - rp).max() <= 1e-6


def test_trained_dispatch_keeps_every_result(rg, ctx):
    """Samples measured by the kernels, training lowers the loss, the table only
    names variants that apply, and learned dispatch gives the oracle's counts."""
    import torch

    bs, ia, ib = synth.array_stress(n_pairs=3000)
    mixed = synth.mixed_small(n_bitmaps=40)
    A = rg.Pool.from_sets(bs.values, bs.offsets)
    Mx = rg.Pool.from_sets(mixed.values, mixed.offsets)
    tia = torch.from_numpy(ia.view(np.int32)).cuda()
    tib = torch.from_numpy(ib.view(np.int32)).cuda()
    X, T, M = rg.dispatch_samples(ctx, A, A, tia, tib)
    ma, mb = synth.consecutive_pairs(len(mixed))
    tma = torch.from_numpy(ma.view(np.int32)).cuda()
    tmb = torch.from_numpy(mb.view(np.int32)).cuda()
    X2, T2, M2 = rg.dispatch_samples(ctx, Mx, Mx, tma, tmb)
    X, T, M = torch.cat([X, X2]), torch.cat([T, T2]), torch.cat([M, M2])
    per_variant = M.sum(0).tolist()
    _say(f"[dispatch] samples {X.shape[0]}, per variant {per_variant}")
    assert all(v > 0 for v in per_variant)
    params, losses = rg.dispatch_train(ctx, X, T, M, epochs=30, batch=4096, lr=2e-3, seed=11)
    losses = losses.cpu().numpy()
    _say(f"[dispatch] epoch losses {losses[0]:.3f} -> {losses[-1]:.3f}")
    assert np.isfinite(losses).all() and losses[-1] < 0.5 * losses[0]
    rg.dispatch_set_mlp(ctx, params)
    try:
        tab = rg.dispatch_table(ctx)
        # every cell names a variant that applies to its types (cell layout as in the header)
        cells = np.arange(rg.RG_MLP_TABLE)
        tb = (cells // (17 * 17 * 144)) % 3 + 1
        ta = cells // (3 * 17 * 17 * 144) + 1
        arr_a, arr_b = ta == 1, tb == 1
        bad = ((tab == 3) | (tab == 4)) & ~(arr_a & arr_b)
        bad |= (tab == 5) & ~((arr_a & (tb == 2)) | ((ta == 2) & arr_b))
        bad |= (tab == 6) & ~((ta == 3) | (tb == 3))
        qa = (cells // (17 * 144)) % 17
        qb = (cells // 144) % 17
        bad |= (tab == 7) & ~((arr_a & (qa <= 5)) | (arr_b & (qb <= 5)))
        bad |= (tab < 2) | (tab > 7)
        assert not bad.any()
        _say(f"[dispatch] table bins {np.bincount(tab, minlength=9).tolist()}")
        for P, pa, pb, sets in ((A, ia, ib, bs), (Mx, ma, mb, mixed)):
            ta_, tb_ = torch.from_numpy(pa.view(np.int32)).cuda(), torch.from_numpy(pb.view(np.int32)).cuda()
            for op in ("and", "or", "xor", "andnot"):
                _, cards, jacc = rg.batch(ctx, op, P, P, ta_, tb_, materialize=False, card=True, jaccard=True)
                cards = cards.cpu().numpy().view(np.uint64)
                jacc = jacc.cpu().numpy()
                for q in range(0, len(pa), max(1, len(pa) // 64)):
                    a, b = sets[int(pa[q])], sets[int(pb[q])]
                    assert int(cards[q]) == oracle.count(op, a, b) and jacc[q] == oracle.jaccard(a, b), (op, q)
    finally:
        ctx.set_dispatch(rg.RG_DISPATCH_HEURISTIC)


def _median_ms(fn, reps=7):
    import time

    import torch

    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - t) * 1e3)
    return float(np.median(ts))


def test_learned_dispatch_gain_on_held_out_pairs(rg, ctx):
    """What the trained network gains over the size-ratio heuristic it replaces:
    trained on kernel-measured costs of array-stress, mixed and array-bitset
    pools, it is timed against the heuristic on held-out pairs (other seeds)
    with identical counts. On mid-size array pairs (9..62 against 9..300 values)
    the heuristic sends every pair to the workgroup merge while the network
    learns that one thread per pair is cheaper: measured 4.4x; the test asks
    for at least 1.5x there and records every ratio."""
    import torch

    import bench

    X, T, M = bench.dispatch_training_set(ctx)
    params, losses = rg.dispatch_train(ctx, X, T, M, epochs=30, batch=4096, lr=2e-3, seed=11)
    losses = losses.cpu().numpy()
    assert losses[-1] < 0.5 * losses[0]
    ratios = {}
    for name, (bs, ia, ib) in bench.dispatch_eval_sets().items():
        P = rg.Pool.from_sets(bs.values, bs.offsets)
        a = torch.from_numpy(ia.view(np.int32)).cuda()
        b = torch.from_numpy(ib.view(np.int32)).cuda()
        cards = torch.zeros(len(ia), dtype=torch.int64, device="cuda")
        jacc = torch.zeros(len(ia), dtype=torch.float64, device="cuda")
        flags = rg.RG_FLAG_CARD | rg.RG_FLAG_JACCARD

        def run():
            ctx.check(rg.roaring_batch(ctx, "and", P, P, a, b, flags, None, cards, jacc))

        ctx.set_dispatch(rg.RG_DISPATCH_HEURISTIC)
        heur = _median_ms(run)
        ref_c, ref_j = cards.clone(), jacc.clone()
        rg.dispatch_set_mlp(ctx, params)
        try:
            learned = _median_ms(run)
            assert torch.equal(cards, ref_c) and torch.equal(jacc, ref_j), name
        finally:
            ctx.set_dispatch(rg.RG_DISPATCH_HEURISTIC)
        c = cards.cpu().numpy()
        j = jacc.cpu().numpy()
        for q in range(0, len(ia), max(1, len(ia) // 50)):
            A, B = bs[int(ia[q])], bs[int(ib[q])]
            assert int(c[q]) == oracle.count("and", A, B) and j[q] == oracle.jaccard(A, B), (name, q)
        ratios[name] = heur / learned
        _say(f"[dispatch gain] {name}: heuristic {heur:.3f} ms, learned {learned:.3f} ms, x{heur / learned:.2f}")
    mid = [v for k, v in ratios.items() if k.startswith("mid-size")][0]
    assert mid >= 1.5, ratios
