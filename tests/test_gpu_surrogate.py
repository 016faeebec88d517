"""GPU checks of the learned pre-screen against the oracle (oracle/surrogate.py
and the oracle GA's candidate streams).

- Every layer of the forward pass and of the backward pass is compared with
  FP64 computed from the GPU's own BF16 operands of that layer.  A product of
  two BF16 values is exact in FP32, so an FP32 sum of K of them differs from
  the FP64 sum by at most K * 2^-24 * sum |a_i b_i|; a BF16 output adds one
  rounding (half an ulp, 2^-9 relative).
- One Adam step equals the FP64 update from the same gradients.
- Features and exact targets of every candidate are bit-exact.
- With the GPU's chosen candidate streams replayed, the oracle GA follows the
  same trajectory bit for bit.
- A measured (not pinned) gain: after online training, the chosen candidates
  decode better than the plain GA's candidate 0.
"""
import numpy as np
import pytest

import oracle
from gpu_util import assert_same_state, ensure_built, say
from oracle import surrogate as sg
from paper_1903_10722_amd import inputs

pytestmark = pytest.mark.gpu

U = 2.0 ** -24


def _ctx(w, k=8, warmup=3, seed=11):
    from paper_1903_10722_amd import Context
    ctx = Context(device=0)
    ctx.add_instance(w["m"], w["p"], w["islands"], interval=w["interval"], theta=w.get("theta", 1.0),
                     topology=w.get("topology", 0), seed=seed, surrogate_k=k, surrogate_warmup=warmup)
    ctx.bind()
    return ctx


def _small(seed=1, n=40, S=5, side=8):
    m, p = inputs.make_instance(n, S, 2, 6, seed=seed)
    isl = [inputs.cellular(side, side, 0.9, 0.1), inputs.pseudo(side * side, 0.75, 0.0)]
    return dict(m=m, p=p, islands=isl, interval=10)


def _params(ctx):
    from paper_1903_10722_amd.binding import PARAM_SLICES
    v = ctx.surrogate_params()
    out = {}
    for k, (o, shp) in PARAM_SLICES.items():
        out[k] = v[o:o + int(np.prod(shp))].reshape(shp)
    return v, out


def _bf(x):
    return sg.bf16_to_f32(sg.bf16(np.asarray(x, dtype=np.float32))).astype(np.float64)


def _to_dev(a_u16):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a_u16).view(np.int16)).cuda()


def _from_dev(t):
    return t.cpu().numpy().view(np.uint16)


def _rand_features(rows, seed):
    rng = np.random.default_rng(seed)
    x = rng.random((rows, 256)).astype(np.float32) * 2.0
    x[:, 200:240] = 0.0
    return sg.bf16(x)


def _check_bf16_layer(got_u16, z_ref, absprod, K):
    """got = bf16(relu(z)) computed in FP32; z_ref FP64 from the same operands."""
    got = sg.bf16_to_f32(got_u16).astype(np.float64)
    want = np.maximum(z_ref, 0.0)
    tol = K * U * absprod + np.abs(want) * 2.0 ** -8 + 1e-30
    bad = np.abs(got - want) > tol
    assert not bad.any(), f"{bad.sum()} entries beyond the bound, worst {np.max(np.abs(got - want) - tol)}"


def test_forward_layers_match_fp64():
    ensure_built()
    import torch
    w = _small()
    say("[surrogate] forward layer-wise")
    ctx = _ctx(w)
    _, P = _params(ctx)
    W1, W2, w3 = _bf(P["W1"]), _bf(P["W2"]), _bf(P["w3"])
    X = _rand_features(256, 3)
    Xf = sg.bf16_to_f32(X).astype(np.float64)
    y, H1, H2 = ctx.mlp_forward(_to_dev(X))
    H1h, H2h, yh = _from_dev(H1), _from_dev(H2), y.cpu().numpy().astype(np.float64)
    z1 = Xf @ W1.T + P["b1"]
    _check_bf16_layer(H1h, z1, np.abs(Xf) @ np.abs(W1.T) + np.abs(P["b1"]), 257)
    h1 = sg.bf16_to_f32(H1h).astype(np.float64)
    z2 = h1 @ W2.T + P["b2"]
    _check_bf16_layer(H2h, z2, np.abs(h1) @ np.abs(W2.T) + np.abs(P["b2"]), 513)
    h2 = sg.bf16_to_f32(H2h).astype(np.float64)
    yr = h2 @ w3 + P["b3"][0]
    bound = 513 * U * (np.abs(h2) @ np.abs(w3) + abs(P["b3"][0])) + 1e-30
    assert (np.abs(yh - yr) <= bound).all()
    ctx.close()
    torch.cuda.synchronize()


@pytest.mark.parametrize("M", [512, 4096])
def test_gradients_layers_match_fp64_and_adam_step(M):
    """Layer-wise backward and one Adam step; M = 4096 is the minibatch of
    the online training step (the split-K weight-gradient GEMMs then sum 32
    partial products)."""
    ensure_built()
    import torch
    w = _small(seed=2)
    say(f"[surrogate] backward layer-wise + Adam, {M} rows")
    ctx = _ctx(w)
    v0, P = _params(ctx)
    W2, w3 = _bf(P["W2"]), _bf(P["w3"])
    X = _rand_features(M, 5)
    Xf = sg.bf16_to_f32(X).astype(np.float64)
    t = np.random.default_rng(6).random(M).astype(np.float32)
    Xd, td = _to_dev(X), torch.from_numpy(t).cuda()
    y, H1, H2 = ctx.mlp_forward(Xd)
    g, dZ2, dZ1 = ctx.mlp_gradients(Xd, td)
    g = g.cpu().numpy().astype(np.float64)
    h1 = sg.bf16_to_f32(_from_dev(H1)).astype(np.float64)
    h2 = sg.bf16_to_f32(_from_dev(H2)).astype(np.float64)
    yv = y.cpu().numpy().astype(np.float64)
    dz2 = sg.bf16_to_f32(_from_dev(dZ2)).astype(np.float64)
    dz1 = sg.bf16_to_f32(_from_dev(dZ1)).astype(np.float64)
    from paper_1903_10722_amd.binding import PARAM_SLICES

    def grad(name):
        o, shp = PARAM_SLICES[name]
        return g[o:o + int(np.prod(shp))].reshape(shp)

    dy = 2.0 * (yv - t) / M
    # output layer
    assert np.all(np.abs(grad("w3") - h2.T @ dy) <= (M + 8) * U * (np.abs(h2.T) @ np.abs(dy)) * 2 + 1e-30)
    assert abs(grad("b3")[0] - dy.sum()) <= (M + 8) * U * np.abs(dy).sum() * 2
    # dZ2 = bf16(dy * w3) on positive H2
    ref = np.outer(dy, w3) * (h2 > 0)
    assert np.all(np.abs(dz2 - ref) <= np.abs(ref) * 2.0 ** -8 + 1e-30)
    # weight gradient of layer 2 from the GPU's dZ2 and H1
    dW2 = dz2.T @ h1
    assert np.all(np.abs(grad("W2") - dW2) <= (M + 8) * U * (np.abs(dz2.T) @ np.abs(h1)) + 1e-30)
    assert np.all(np.abs(grad("b2") - dz2.sum(axis=0)) <= (M + 8) * U * np.abs(dz2).sum(axis=0) + 1e-30)
    # dZ1 = bf16(dZ2 W2) on positive H1
    ref1 = (dz2 @ W2) * (h1 > 0)
    bound1 = 513 * U * (np.abs(dz2) @ np.abs(W2)) + np.abs(ref1) * 2.0 ** -8 + 1e-30
    assert np.all(np.abs(dz1 - ref1) <= bound1)
    dW1 = dz1.T @ Xf
    assert np.all(np.abs(grad("W1") - dW1) <= (M + 8) * U * (np.abs(dz1.T) @ np.abs(Xf)) + 1e-30)
    assert np.all(np.abs(grad("b1") - dz1.sum(axis=0)) <= (M + 8) * U * np.abs(dz1).sum(axis=0) + 1e-30)
    # the whole chain against the unrounded FP64 backward: same direction
    full = sg.mlp_backward(Xf, t.astype(np.float64), _bf(P["W1"]).T, P["b1"], W2.T, P["b2"], w3, P["b3"][0])
    for name, key in [("W1", "W1"), ("W2", "W2"), ("w3", "w3")]:
        a = grad(name).reshape(-1)
        b = (full[key].T if name != "w3" else full[key]).reshape(-1)
        cos = a @ b / (np.linalg.norm(a) * np.linalg.norm(b))
        assert cos > 0.999, (name, cos)
    # one Adam step from zero moments (first step of this context)
    ctx.mlp_train_step(Xd, td)
    v1 = ctx.surrogate_params().astype(np.float64)
    want, _, _ = sg.adam(v0.astype(np.float64), g, np.zeros_like(g), np.zeros_like(g), step=1)
    assert np.allclose(v1, want, rtol=1e-6, atol=1e-8)
    ctx.close()


def test_candidate_features_and_exact_targets_bit_exact():
    ensure_built()
    w = _small(seed=3, n=60, S=10)
    say("[surrogate] candidate features")
    ctx = _ctx(w)
    ga = oracle.GA(w["m"], w["p"], w["islands"], interval=w["interval"], seed=11)
    res = ctx.surrogate_candidates(exact=True, features=True)
    genes0, mk0 = ga.population(0)
    LB = sg.lower_bound(w["m"], w["p"])
    for cell in range(0, 64, 5):
        for c in range(8):
            child, meta = ga.cell_candidate(0, cell, c)
            f = sg.features(w["m"], w["p"], child, int(mk0[meta[0]]), int(mk0[meta[1]]), meta)
            assert np.array_equal(res["features"][cell, c], f), (cell, c)
            tgt = sg.target(oracle.decode(w["m"], w["p"], child), LB)
            assert res["exact"][cell, c] == tgt, (cell, c)
    assert (res["choice"] == np.argmin(res["pred"], axis=1)).all()
    ctx.close()


def test_replayed_trajectory_and_ring_bit_exact():
    """The GA with the pre-screen, replayed by the oracle from the GPU's
    choices, generation by generation; the replay ring holds the features
    and exact targets of the decoded children."""
    ensure_built()
    w = _small(seed=4)
    say("[surrogate] replay trajectory")
    warmup = 3
    ctx = _ctx(w, warmup=warmup)
    ga = oracle.GA(w["m"], w["p"], w["islands"], interval=w["interval"], seed=11)
    LB = sg.lower_bound(w["m"], w["p"])
    cells = 64
    for g in range(1, 16):
        prev_genes, prev_mk = ga.population(0)
        ctx.evolve(1)
        ch = ctx.surrogate_choices() if g > warmup else np.zeros(cells, dtype=np.int32)
        if g > warmup:
            ga.set_cell_choices(0, ch)
        ga.evolve(1)
        assert_same_state(ctx, ga, 0, 2, f"generation {g}")
        X, t = ctx.surrogate_ring((g - 1) * cells, cells)
        # rebuild the decoded candidates from generation g-1's population
        tmp = oracle.GA(w["m"], w["p"], w["islands"], interval=w["interval"], seed=11)
        tmp.set_population(0, prev_genes, prev_mk)
        tmp.set_generation(g - 1)
        for cell in range(0, cells, 9):
            child, meta = tmp.cell_candidate(0, cell, int(ch[cell]))
            f = sg.features(w["m"], w["p"], child, int(prev_mk[meta[0]]), int(prev_mk[meta[1]]), meta)
            assert np.array_equal(X[cell], f), (g, cell)
            assert t[cell] == sg.target(oracle.decode(w["m"], w["p"], child), LB)
    ctx.close()


def test_same_seed_same_choices():
    ensure_built()
    w = _small(seed=5)
    say("[surrogate] determinism")
    runs = []
    for _ in range(2):
        ctx = _ctx(w, warmup=2)
        ctx.evolve(8)
        runs.append((ctx.surrogate_choices(), ctx.population(0, 0)[1], ctx.surrogate_params()))
        ctx.close()
    assert np.array_equal(runs[0][0], runs[1][0])
    assert np.array_equal(runs[0][1], runs[1][1])
    assert np.array_equal(runs[0][2], runs[1][2])


def test_trained_prescreen_picks_better_children():
    """Measured gain: after online training on the GA's own decodes, the
    candidate the network picks decodes better, on average over all cells,
    than candidate 0 (the child the GA without the pre-screen would take),
    and predictions rank the candidates better than chance."""
    ensure_built()
    m, p = inputs.make_instance(200, 10, 2, 6, seed=9)
    isl = [inputs.cellular(32, 32, 0.9, 0.1), inputs.pseudo(1024, 0.75, 0.0)]
    w = dict(m=m, p=p, islands=isl, interval=20)
    say("[surrogate] gain after training, n=200 S=10 32x32")
    ctx = _ctx(w, warmup=5)
    ctx.evolve(60)
    res = ctx.surrogate_candidates(exact=True)
    ex, pred = res["exact"].astype(np.float64), res["pred"].astype(np.float64)
    chosen = ex[np.arange(ex.shape[0]), res["choice"]]
    gain = ex[:, 0].mean() - chosen.mean()
    rho = sg.spearman(pred.reshape(-1), ex.reshape(-1))
    rho_within = np.mean([sg.spearman(pred[i], ex[i]) for i in range(ex.shape[0]) if np.ptp(ex[i]) > 0])
    mae = np.abs(pred - ex).mean()
    say(f"[surrogate] gain {gain:.5f} (candidate 0 {ex[:, 0].mean():.5f} -> chosen {chosen.mean():.5f}), "
        f"spearman {rho:.3f}, within-cell {rho_within:.3f}, MAE {mae:.5f}")
    # selection only needs the ranking inside each cell's candidates
    assert rho_within > 0.1
    assert gain > 0.0
    assert chosen.mean() < ex.mean()
    ctx.close()


@pytest.mark.timeout(600)
def test_surrogate_workload_size_features_and_replay():
    """The pre-screen at its own workload size (n=1000, S=20, m in [2,6],
    64x64 + 4096, k=8): features and exact targets of sampled cells'
    candidates are bit-exact at generation 0, and two screened generations
    (after one warm-up generation) replay exactly on the oracle, with the
    replay ring's rows of sampled cells."""
    ensure_built()
    w = inputs.workload("surrogate", seed=1)
    say("[surrogate] workload size n=1000 S=20 64x64 k=8")
    ctx = _ctx(w, k=8, warmup=1)
    ga = oracle.GA(w["m"], w["p"], w["islands"], interval=w["interval"], seed=11)
    LB = sg.lower_bound(w["m"], w["p"])
    res = ctx.surrogate_candidates(exact=True, features=True)
    genes0, mk0 = ga.population(0)
    cells = list(range(0, 4096, 171)) + [4095]
    for cell in cells:
        for c in range(8):
            child, meta = ga.cell_candidate(0, cell, c)
            f = sg.features(w["m"], w["p"], child, int(mk0[meta[0]]), int(mk0[meta[1]]), meta)
            assert np.array_equal(res["features"][cell, c], f), (cell, c)
            assert res["exact"][cell, c] == sg.target(oracle.decode(w["m"], w["p"], child), LB), (cell, c)
    assert (res["choice"] == np.argmin(res["pred"], axis=1)).all()
    say("[surrogate] workload size: generation-0 candidates match")
    for g in (1, 2, 3):
        prev_genes, prev_mk = ga.population(0)
        ctx.evolve(1)
        ch = ctx.surrogate_choices() if g > 1 else np.zeros(4096, dtype=np.int32)
        if g > 1:
            ga.set_cell_choices(0, ch)
        ga.evolve(1)
        assert_same_state(ctx, ga, 0, 2, f"generation {g}")
        X, t = ctx.surrogate_ring((g - 1) * 4096, 4096)
        tmp = oracle.GA(w["m"], w["p"], w["islands"], interval=w["interval"], seed=11)
        tmp.set_population(0, prev_genes, prev_mk)
        tmp.set_generation(g - 1)
        for cell in cells[:8]:
            child, meta = tmp.cell_candidate(0, cell, int(ch[cell]))
            f = sg.features(w["m"], w["p"], child, int(prev_mk[meta[0]]), int(prev_mk[meta[1]]), meta)
            assert np.array_equal(X[cell], f), (g, cell)
            assert t[cell] == sg.target(oracle.decode(w["m"], w["p"], child), LB)
        say(f"[surrogate] workload size: generation {g} replayed")
    ctx.close()


@pytest.mark.parametrize("shape", [(60, 10, 99, 0), (1000, 20, 99, 0), (37, 3, 99, 0), (90, 7, 3000, 0),
                                   (200, 30, 99, 2)],
                         ids=["n60_S10", "n1000_S20", "n37_S3", "wide_p", "S30_tournaments"])
def test_one_wave_per_cell_candidate_features(shape):
    """Scoring builds the candidates one wave per cell and sums the features
    from a job-major table; every candidate's features equal the oracle's
    (and those of the per-stage candidate kernel that also decodes them)."""
    ensure_built()
    n, S, p_hi, sel = shape
    m, p = inputs.make_instance(n, S, 2, 6, p_hi=p_hi, seed=n + S)
    isl = [dict(inputs.cellular(8, 8, 0.9, 0.1), sel=sel), inputs.pseudo(64, 0.75, 0.0)]
    w = dict(m=m, p=p, islands=isl, interval=10)
    say(f"[surrogate] one wave per cell: n={n} S={S} p<={p_hi} selection={sel}")
    ctx = _ctx(w)
    ga = oracle.GA(w["m"], w["p"], w["islands"], interval=w["interval"], seed=11)
    fast = ctx.surrogate_candidates(exact=False, features=True)
    slow = ctx.surrogate_candidates(exact=True, features=True)
    assert np.array_equal(fast["features"], slow["features"])
    genes0, mk0 = ga.population(0)
    for cell in range(0, 64, 7):
        for c in range(8):
            child, meta = ga.cell_candidate(0, cell, c)
            f = sg.features(w["m"], w["p"], child, int(mk0[meta[0]]), int(mk0[meta[1]]), meta)
            assert np.array_equal(fast["features"][cell, c], f), (cell, c)
    ctx.close()


def test_captured_epochs_match_eager_generations():
    """Past the warm-up, whole migration epochs with the pre-screen replay one
    captured graph (batch rows and Adam bias corrections read on the device).
    Each replay, with eager reads and synchronisations in between, leaves the
    same state as generation-by-generation eager launches: populations,
    network parameters, Adam moments and step count, replay ring, choices."""
    ensure_built()
    w = _small(seed=6)
    say("[surrogate] captured epochs against eager generations")
    eager = _ctx(w, warmup=3, seed=21)
    eager.set_graphs(False)
    graph = _ctx(w, warmup=3, seed=21)
    graph.evolve(10)             # warm-up and the first epoch run eagerly
    for _ in range(10):
        eager.evolve(1)
    for epoch in range(4):
        graph.evolve(10)
        for _ in range(10):
            eager.evolve(1)
        gen = 20 + 10 * epoch
        for isl in range(2):
            ge, me = eager.population(0, isl)
            gg, mg = graph.population(0, isl)
            assert np.array_equal(ge, gg) and np.array_equal(me, mg), (gen, isl)
        assert np.array_equal(eager.surrogate_choices(), graph.surrogate_choices()), gen
        assert np.array_equal(eager.surrogate_params(), graph.surrogate_params()), gen
        assert eager.checkpoint() == graph.checkpoint(), gen
    eager.close()
    graph.close()
