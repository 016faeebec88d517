"""Pins of the pre-screen's oracle (oracle/surrogate.py) and of the GA's
candidate streams: BF16 rounding against torch, features against a hand
computation, the FP64 backward against central finite differences, Adam's
first step against its closed form, rank correlation against scipy, and
replayed candidate choices against the plain GA."""
import json
import os

import numpy as np
import pytest

import oracle
from oracle import surrogate as sg
from paper_1903_10722_amd import inputs

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_bf16_rounding_matches_torch():
    import torch
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(20000).astype(np.float32) * 10.0 ** rng.integers(-8, 8, 20000),
                        np.array([0.0, -0.0, 1.0, 1.00390625, 1.005859375, 1.001953125, 3.0e38, 1e-38],
                                 dtype=np.float32)]).astype(np.float32)
    # exact ties: low half 0x8000 with even and odd upper halves
    ties = (np.arange(1000, dtype=np.uint32) << 16 | 0x8000).astype(np.uint32) + (0x3F80 << 16)
    x = np.concatenate([x, ties.view(np.float32)])
    want = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(sg.bf16(x), want)
    assert np.array_equal(sg.bf16_to_f32(want), torch.from_numpy(want.view(np.int16)).view(torch.bfloat16).float().numpy())


def test_features_worked_example():
    g = json.load(open(os.path.join(GOLD, "features_worked_example.json")))
    want = np.zeros(256, dtype=np.float32)
    for k, v in g["nonzero"].items():
        want[int(k)] = np.float32(v)
    got = sg.features(g["machines"], g["p"], g["child"], g["mk1"], g["mk2"], g["meta"])
    assert np.array_equal(got, sg.bf16(want))


def test_features_invariants():
    """Bucket loads of a stage sum to the stage total, so every stage's
    features sum to B (before rounding) for any permutation."""
    rng = np.random.default_rng(1)
    for n, S in [(100, 5), (1000, 20), (37, 7)]:
        m, p = inputs.make_instance(n, S, 1, 5, seed=n)
        child = rng.permutation(n)
        f = sg.bf16_to_f32(sg.features(m, p, child, 100, 120, [0, 0, 1, 3, 9, 1, 2, 5])).astype(np.float64)
        B = 240 // S
        per_stage = f[:B * S].reshape(B, S).sum(axis=0)
        assert np.allclose(per_stage, B, rtol=B * 2 ** -7)
        assert (f[B * S:240] == 0).all() and (f[252:] == 0).all()


def _rand_net(rng, din=6, h=5):
    return (rng.standard_normal((din, h)), rng.standard_normal(h) * 0.1, rng.standard_normal((h, h)),
            rng.standard_normal(h) * 0.1, rng.standard_normal(h), 0.3)


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(2)
    W1, b1, W2, b2, w3, b3 = _rand_net(rng)
    x = rng.standard_normal((9, 6))
    t = rng.standard_normal(9)
    g = sg.mlp_backward(x, t, W1, b1, W2, b2, w3, b3)
    params = dict(W1=W1, b1=b1, W2=W2, b2=b2, w3=w3)
    h = 1e-6
    for name, P in params.items():
        flat = P.reshape(-1)
        for idx in range(flat.size):
            old = flat[idx]
            flat[idx] = old + h
            lp = sg.mlp_loss(x, t, W1, b1, W2, b2, w3, b3)
            flat[idx] = old - h
            lm = sg.mlp_loss(x, t, W1, b1, W2, b2, w3, b3)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[name].reshape(-1)[idx]) <= 1e-6 * max(1.0, abs(fd)), (name, idx)
    lp = sg.mlp_loss(x, t, W1, b1, W2, b2, w3, b3 + h)
    lm = sg.mlp_loss(x, t, W1, b1, W2, b2, w3, b3 - h)
    assert abs((lp - lm) / (2 * h) - g["b3"]) < 1e-6


def test_forward_matches_layers_and_relu_semantics():
    rng = np.random.default_rng(3)
    W1, b1, W2, b2, w3, b3 = _rand_net(rng)
    x = rng.standard_normal((7, 6))
    fw = sg.mlp_forward(x, W1, b1, W2, b2, w3, b3, bf16_activations=False)
    z1, z2, y = sg.mlp_layers(x, W1, b1, W2, b2, w3, b3)
    assert np.allclose(fw["y"], y) and np.allclose(fw["z1"], z1) and np.allclose(fw["z2"], z2)
    # all-negative first layer: the output is relu(b2) . w3 + b3
    y0 = sg.mlp_forward(np.abs(x), -np.abs(W1), -np.ones(5), W2, b2, w3, b3, bf16_activations=False)["y"]
    assert np.allclose(y0, np.maximum(b2, 0) @ w3 + b3)


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(4)
    p = rng.standard_normal(100)
    g = rng.standard_normal(100)
    p1, m, v = sg.adam(p, g, np.zeros(100), np.zeros(100), step=1, lr=1e-3)
    # bias-corrected first moments equal g and g^2, so the step is lr * g / (|g| + eps)
    assert np.allclose(p1, p - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_spearman_matches_scipy():
    from scipy.stats import spearmanr
    rng = np.random.default_rng(5)
    a = rng.standard_normal(500)
    b = a + rng.standard_normal(500)
    assert abs(sg.spearman(a, b) - spearmanr(a, b).correlation) < 1e-12


def test_candidate_stream_zero_is_the_plain_ga():
    w = inputs.workload("tiny", seed=5)
    a = oracle.GA(w["m"], w["p"], w["islands"], interval=10, seed=3)
    b = oracle.GA(w["m"], w["p"], w["islands"], interval=10, seed=3)
    N = w["islands"][0]["size"]
    for _ in range(12):
        # candidate 0 of every cell is exactly the plain GA's offspring
        genes0, mk0 = a.population(0)
        child, meta = a.cell_candidate(0, 5, 0)
        a.evolve(1)
        b.set_cell_choices(0, np.zeros(N, dtype=np.int32))
        b.evolve(1)
        for i in range(2):
            assert np.array_equal(a.population(i)[0], b.population(i)[0])
        c = oracle.decode(w["m"], w["p"], child)
        new = a.population(0)[0][5]
        assert new.tolist() == (child.tolist() if c < mk0[5] else genes0[5].tolist())


def test_replayed_choices_change_only_the_chosen_streams():
    w = inputs.workload("tiny", seed=6)
    N = w["islands"][0]["size"]
    g = oracle.GA(w["m"], w["p"], w["islands"], interval=0, seed=4)
    genes0, mk0 = g.population(0)
    choices = np.arange(N, dtype=np.int32) % 8
    cands = [g.cell_candidate(0, s, int(choices[s]))[0] for s in range(N)]
    g.set_cell_choices(0, choices)
    g.evolve(1)
    genes1, mk1 = g.population(0)
    for s in range(N):
        c = oracle.decode(w["m"], w["p"], cands[s])
        if c < mk0[s]:
            assert genes1[s].tolist() == cands[s].tolist() and mk1[s] == c
        else:
            assert genes1[s].tolist() == genes0[s].tolist() and mk1[s] == mk0[s]


def test_spearman_on_tied_data_matches_scipy():
    """Tied values share their mean rank, as in scipy's spearmanr; a
    position-ordered (ordinal) ranking of ties would differ here."""
    from scipy.stats import spearmanr
    rng = np.random.default_rng(7)
    for _ in range(20):
        a = rng.integers(0, 4, size=60).astype(np.float64)      # many ties
        b = a + rng.integers(0, 3, size=60)
        assert abs(sg.spearman(a, b) - spearmanr(a, b).correlation) < 1e-12
    # by hand: a = [1, 1, 2], b = [1, 2, 3]: ranks (1.5, 1.5, 3) and (1, 2, 3)
    # give rho = 1.5 / sqrt(1.5 * 2) = sqrt(3) / 2
    assert abs(sg.spearman([1, 1, 2], [1, 2, 3]) - np.sqrt(3) / 2) < 1e-15
    assert np.isnan(sg.spearman([2, 2, 2], [1, 2, 3]))
