"""GPU parity of the learned proposal: the BF16 MFMA network against the
oracle network (same BF16 rounding points, FP32 sums in a different order),
and the learned Metropolis chain against the oracle chain."""
import sys

import numpy as np
import pytest

import oracle as O
from oracle import mlp as OM
from paper_1808_00128_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1808_00128_amd import binding

    binding.lib()
    return binding


def host_ctx(B, n=8):
    circ = W.from_list(n, [(W.OP_H, q, 0) for q in range(n)])
    return B.Context([dict(circuit=circ, chi=1, mode="exact", seed=0)])


def varied_params(n, H, seed):
    p = W.mlp_init(n, H, seed=seed, flip_bias=-1.0)
    rng = np.random.default_rng(seed + 100)
    p["b1"] = rng.uniform(-0.3, 0.3, H).astype(np.float32)
    p["b2"] = rng.uniform(-0.3, 0.3, H).astype(np.float32)
    p["b3"] = rng.uniform(-2, 0, n).astype(np.float32)
    p["W3"] = (p["W3"] * 5).astype(np.float32)
    return p


@pytest.mark.parametrize("n,H,batch", [(50, 256, 64), (12, 64, 37), (64, 256, 130), (1, 16, 5)])
def test_mlp_forward_matches_oracle(B, n, H, batch):
    say(f"mlp forward n={n} H={H} batch={batch}")
    ctx = host_ctx(B)
    p = varied_params(n, H, seed=n)
    net = B.MLP(ctx, n, H, max(batch, 64), p)
    ref = OM.MLPRef(p, n, H)
    x = W.random_bitstrings(n, batch, np.random.default_rng(n))
    got = net.forward(x)
    exp, _ = ref.forward(x)
    exp = np.asarray(exp, np.float32)
    scale = np.max(np.abs(exp)) + 1e-6
    assert np.max(np.abs(got - exp)) <= 1e-4 * scale, np.max(np.abs(got - exp)) / scale
    net.close()
    ctx.close()


@pytest.mark.parametrize("n,H", [(50, 256), (13, 48)])
def test_mlp_fused_forward_equals_product_path(B, n, H):
    """Batches up to 256 rows run the fused one-kernel network, larger ones
    the three BF16 products; the shared rows agree bit for bit (same MFMAs
    over the same k blocks, same epilogues)."""
    say(f"mlp fused vs products n={n} H={H}")
    ctx = host_ctx(B)
    p = varied_params(n, H, seed=3 + n)
    net = B.MLP(ctx, n, H, 300, p)
    x = W.random_bitstrings(n, 300, np.random.default_rng(7 + n))
    big = net.forward(x)          # 300 rows: products
    small = net.forward(x[:201])  # 201 rows: fused
    assert np.array_equal(big[:201], small)
    net.close()
    ctx.close()


@pytest.mark.parametrize("n,H,batch", [(50, 256, 128), (12, 64, 100)])
def test_mlp_gradients_match_oracle(B, n, H, batch):
    say(f"mlp gradients n={n} H={H} batch={batch}")
    ctx = host_ctx(B)
    p = varied_params(n, H, seed=10 + n)
    net = B.MLP(ctx, n, H, batch, p)
    ref = OM.MLPRef(p, n, H)
    rng = np.random.default_rng(3)
    x = W.random_bitstrings(n, batch, rng)
    t = W.random_bitstrings(n, batch, rng) & W.random_bitstrings(n, batch, rng)
    loss, g = net.loss_grad(x, t)
    eloss, eg = ref.loss_and_grad(x, t)
    assert abs(loss - eloss) <= 1e-5 * abs(eloss)
    for k in OM.PARAM_ORDER:
        a, e = np.asarray(g[k], np.float64), np.asarray(eg[k], np.float64)
        assert np.linalg.norm(a - e) <= 3e-3 * np.linalg.norm(e) + 1e-9, (k, np.linalg.norm(a - e) / np.linalg.norm(e))
        big = np.abs(e) > 1e-2 * np.max(np.abs(e))
        assert np.all(np.abs(a[big] - e[big]) <= 1e-2 * np.abs(e[big])), k
    net.close()
    ctx.close()


def test_mlp_training_step_matches_oracle_and_reduces_loss(B):
    n, H = 20, 64
    say("mlp training")
    ctx = host_ctx(B)
    p = W.mlp_init(n, H, seed=4)
    net = B.MLP(ctx, n, H, 256, p)
    ref = OM.MLPRef(p, n, H)
    rng = np.random.default_rng(5)
    x = W.random_bitstrings(n, 256, rng)
    # a learnable target: flip the bits where x has a 1 in a fixed pattern
    pattern = np.uint64(0b10110011100101001101)
    t = x & pattern
    l0 = net.train(x, t, batch=256, epochs=1, lr=1e-3)
    loss, grads = ref.loss_and_grad(x, t)
    ref.adam_step(grads, 1e-3)
    got = net.params()
    for k in OM.PARAM_ORDER:
        # one Adam step moves every weight by ~lr; compare the moves
        d_gpu = got[k] - p[k]
        d_ref = ref.p[k] - p[k]
        agree = np.mean(np.sign(d_gpu) == np.sign(d_ref))
        assert agree > 0.97, (k, agree)
    losses = net.train(x, t, batch=64, epochs=60, lr=3e-3)
    assert losses[-1] < 0.5 * l0[0], (l0, losses[-5:])
    net.close()
    ctx.close()


def chain_setup(B, n, chi, mode, seed):
    rng = np.random.default_rng(seed)
    circ = W.random_circuit(n, 10 * n, rng.uniform(0, 2 * np.pi, size=5), rng)
    spec = dict(circuit=circ, chi=chi, mode=mode, seed=seed)
    ctx = B.Context([spec])
    ctx.apply_circuit(circ)
    T = O.Terms(circ, chi, O.EXACT if mode == "exact" else O.SPARSIFY, seed=seed)
    return ctx, T, rng


def start_states(T, n, count, rng, chi):
    xs = []
    while len(xs) < count:
        a = int(rng.integers(chi))
        x = T.term(a).sample(int(W.random_bitstrings(n, 1, rng)[0]))
        if abs(T.amplitudes(np.array([x], np.uint64))[0]) > 0:
            xs.append(x)
    return np.array(xs, np.uint64)


def test_learned_chain_eps_one_equals_plain_chain(B):
    n, chi = 8, 32
    say("learned chain eps=1")
    ctx, T, rng = chain_setup(B, n, chi, "exact", 11)
    x0 = start_states(T, n, 4, rng, chi)
    net = B.MLP(ctx, n, 32, 64, W.mlp_init(n, 32))
    u_mix, j, u_bits, u = W.learned_streams(n, 4, 150, rng)
    ctx.metropolis_init(x0)
    tr, acc, fl, amp = ctx.metropolis_step_learned(net, u_mix, j, u_bits, u, 1.0, 0.01, 0.5)
    otr, oacc, oamp = T.metropolis(x0, j, u)
    assert np.array_equal(tr, otr) and np.array_equal(acc, oacc)
    assert np.all(fl == 1)


def test_learned_chain_matches_oracle_until_near_tie(B):
    n, chi = 8, 32
    say("learned chain eps=0.2 vs oracle")
    ctx, T, rng = chain_setup(B, n, chi, "exact", 12)
    p = varied_params(n, 32, seed=2)
    net = B.MLP(ctx, n, 32, 64, p)
    ref = OM.MLPRef(p, n, 32)
    C_, steps = 4, 120
    x0 = start_states(T, n, C_, rng, chi)
    u_mix, j, u_bits, u = W.learned_streams(n, C_, steps, rng)
    ctx.metropolis_init(x0)
    tr, acc, fl, amp = ctx.metropolis_step_learned(net, u_mix, j, u_bits, u, 0.2, 0.01, 0.5)
    otr, oacc, ofl, tie = OM.learned_chain(T, ref, x0, u_mix, j, u_bits, u, 0.2, 0.01, 0.5)
    compared = 0
    for c in range(C_):
        k = int(tie[c])
        assert np.array_equal(tr[c, :k], otr[c, :k]), c
        assert np.array_equal(acc[c, :k], oacc[c, :k]), c
        assert np.array_equal(fl[c, :k], ofl[c, :k]), c
        compared += k
    assert compared >= 0.9 * C_ * steps
    assert fl.mean() > 1.0  # multi-bit moves happen


def test_learned_chain_full_grid_matches_oracle(B):
    """chi = 2^19 (2048 tiles of 256 terms, as many as the QAOA workload's
    grid holds per 2^20 / 2): the flip-mask proposal kernel and the
    corrected accept step against the oracle chain until the first near tie."""
    n, chi, C_, steps = 10, 1 << 19, 4, 30
    rng = np.random.default_rng(6200)
    circ = W.random_circuit(n, 60, rng.uniform(0, 2 * np.pi, size=20), rng)
    spec = dict(circuit=circ, chi=chi, mode="sparsify", seed=612)
    say(f"learned chain full grid n={n} chi={chi} chains={C_} steps={steps}")
    ctx = B.Context([spec])
    ctx.apply_circuit(circ)
    T = O.Terms(circ, chi, O.SPARSIFY, seed=612)
    x0 = start_states(T, n, C_, rng, chi)
    p = varied_params(n, 32, seed=5)
    net = B.MLP(ctx, n, 32, 64, p)
    ref = OM.MLPRef(p, n, 32)
    u_mix, j, u_bits, u = W.learned_streams(n, C_, steps, rng)
    ctx.metropolis_init(x0)
    tr, acc, fl, amp = ctx.metropolis_step_learned(net, u_mix, j, u_bits, u, 0.2, 0.01, 0.5)
    otr, oacc, ofl, tie = OM.learned_chain(T, ref, x0, u_mix, j, u_bits, u, 0.2, 0.01, 0.5)
    compared = 0
    for c in range(C_):
        k = int(tie[c])
        assert np.array_equal(tr[c, :k], otr[c, :k]), c
        assert np.array_equal(acc[c, :k], oacc[c, :k]), c
        assert np.array_equal(fl[c, :k], ofl[c, :k]), c
        compared += k
    assert compared >= 0.9 * C_ * steps
    assert fl.mean() > 1.0
    net.close()
    ctx.close()


def test_learned_chain_stationary_law(B):
    """The corrected chain samples P: TV to the exact law at n = 8."""
    n, chi = 8, 64
    say("learned chain stationarity")
    rng = np.random.default_rng(13)
    circ = W.qaoa_circuit(n, 6, rng)[0]
    spec = dict(circuit=circ, chi=chi, mode="sparsify", seed=13)
    ctx = B.Context([spec])
    ctx.apply_circuit(circ)
    T = O.Terms(circ, chi, O.SPARSIFY, seed=13)
    P = np.abs(T.amplitudes(np.arange(2**n, dtype=np.uint64))) ** 2
    P /= P.sum()
    p = W.mlp_init(n, 32, flip_bias=-1.5)
    net = B.MLP(ctx, n, 32, 64, p)
    C_, steps = 32, 6000
    x0 = np.array(rng.choice(2**n, size=C_, p=P), np.uint64)
    u_mix, j, u_bits, u = W.learned_streams(n, C_, steps, rng)
    ctx.metropolis_init(x0)
    tr, acc, fl, amp = ctx.metropolis_step_learned(net, u_mix, j, u_bits, u, 0.2, 0.02, 0.5)
    from paper_1808_00128_amd import stats
    tv = stats.total_variation(tr[:, 500:].ravel(), P)
    assert tv < 0.05, tv


def test_learned_chain_with_underflowing_proposal_density(B):
    """pi_min = pi_max = 1e-6 and u_bits = 0: every step proposes the mask of
    all n = 62 bits, whose proposal density (1 - eps) 1e-6^62 ~ 1e-372 is
    below the smallest double.  The density ratio is evaluated in the log
    domain on both sides, so the chain still accepts iff U < P(y)/P(x), step
    for step as the oracle chain (a 0/0 ratio would reject every move).

    The circuit is H on every qubit followed by diagonal gates and phase
    slots.  Each sparsified term then contributes b_alpha i^{q(x)} with the
    branch phases of the phase-gate decomposition, and complementing every bit
    conjugates the branch-dependent part, so P(y) = P(x) for y = x ^ 1...1 and
    every proposal is accepted."""
    n, chi, C_, steps = 62, 128, 4, 40
    say("learned chain, underflowing proposal density n=62")
    # H on every qubit, then diagonal gates: every term has |v| = n, so every
    # string (the all-flip proposals included) has a nonzero amplitude.
    rng = np.random.default_rng(14)
    gates = [(W.OP_H, q, 0) for q in range(n)]
    gates += W.random_clifford_gates(n, 4 * n, rng, ops=(W.OP_S, W.OP_CZ))
    for q in rng.choice(n, size=6, replace=False).tolist():
        gates.append((W.OP_SLOT, q, 0, float(rng.uniform(0, 2 * np.pi))))
    circ = W.from_list(n, gates)
    ctx = B.Context([dict(circuit=circ, chi=chi, mode="sparsify", seed=14)])
    ctx.apply_circuit(circ)
    T = O.Terms(circ, chi, O.SPARSIFY, seed=14)
    x0 = start_states(T, n, C_, rng, chi)
    p = varied_params(n, 32, seed=6)
    net = B.MLP(ctx, n, 32, 64, p)
    ref = OM.MLPRef(p, n, 32)
    u_mix = np.full((C_, steps), 0.99)
    j = rng.integers(0, n, size=(C_, steps), dtype=np.uint32)
    u_bits = np.zeros((C_, steps, n))
    u = rng.random(size=(C_, steps))
    ctx.metropolis_init(x0)
    tr, acc, fl, amp = ctx.metropolis_step_learned(net, u_mix, j, u_bits, u, 0.1, 1e-6, 1e-6)
    otr, oacc, ofl, tie = OM.learned_chain(T, ref, x0, u_mix, j, u_bits, u, 0.1, 1e-6, 1e-6, tie=1e-9)
    assert np.all(fl == n) and np.all(ofl == n)
    for c in range(C_):
        k = int(tie[c])
        assert k >= steps - 2, (c, k)
        assert np.array_equal(tr[c, :k], otr[c, :k]), c
        assert np.array_equal(acc[c, :k], oacc[c, :k]), c
    assert acc.mean() == 1.0 and oacc.mean() == 1.0
    net.close()
    ctx.close()


def test_trained_network_beats_untrained_on_qaoa_twin(B):
    """What training buys, on the n = 12 twin of the QAOA chain workload
    (p = 1, 16 triples, beta = pi/4, gamma = 0.35; Sec. "Quantum approximate
    optimization algorithm"): the proposal network trained on plain chains
    (pairs x_t, x_t ^ x_{t + Delta}, Delta = tau_int of the plain chain) mixes
    faster than the same network untrained.  64 chains start from the exact
    law P (the oracle's amplitudes over all 4096 strings) and run 1600 steps
    with the same random streams; the trained chain's pooled samples are
    closer to P in total variation, and the Hamming weight decorrelates in
    fewer steps."""
    from paper_1808_00128_amd import stats

    n, triples, chi, C_, steps = 12, 16, 4096, 64, 1600
    say(f"trained vs untrained proposal, QAOA n={n} chi={chi}")
    rng = np.random.default_rng(2012)
    circ = W.qaoa_circuit(n, triples, rng, gamma=0.35, beta=np.pi / 4)[0]
    ctx = B.Context([dict(circuit=circ, chi=chi, mode="sparsify", seed=2012)])
    ctx.apply_circuit(circ)
    T = O.Terms(circ, chi, O.SPARSIFY, seed=2012)
    P = np.abs(T.amplitudes(np.arange(2**n, dtype=np.uint64))) ** 2
    P /= P.sum()
    x0 = np.array(rng.choice(2**n, size=C_, p=P), np.uint64)

    def weight(tr):
        t = tr.astype(np.uint64)
        return np.array([bin(int(v)).count("1") for v in t.ravel()], np.float64).reshape(t.shape)

    j, u = W.metropolis_streams(n, C_, steps, rng, shared_j=True)
    ctx.metropolis_init(x0)
    tr, _, _ = ctx.metropolis_step(j, u)
    tau_plain, _, _ = stats.tau_int(weight(tr))
    delta = max(1, int(round(tau_plain)))
    xt = tr[:, :-delta].ravel()
    tgt = xt ^ tr[:, delta:].ravel()
    net = B.MLP(ctx, n, 128, 1024, W.mlp_init(n, 128))
    losses = net.train(xt, tgt, batch=1024, epochs=30, lr=1e-3)
    assert losses[-1] < losses[0]
    untrained = B.MLP(ctx, n, 128, 1024, W.mlp_init(n, 128))
    streams = W.learned_streams(n, C_, steps, rng)
    result = {}
    for name, m in (("trained", net), ("untrained", untrained)):
        ctx.metropolis_init(x0)
        ltr, _, _, _ = ctx.metropolis_step_learned(m, *streams, 0.1, 0.002, 0.5)
        tau, _, _ = stats.tau_int(weight(ltr))
        result[name] = (stats.total_variation(ltr.ravel(), P), tau)
        m.close()
    ctx.close()
    (tv_t, tau_t), (tv_u, tau_u) = result["trained"], result["untrained"]
    say(f"TV trained {tv_t:.4f} untrained {tv_u:.4f}; tau_int {tau_t:.2f} vs {tau_u:.2f} (plain {tau_plain:.2f})")
    assert tv_t < 0.85 * tv_u, result
    assert tau_t < tau_u, result
