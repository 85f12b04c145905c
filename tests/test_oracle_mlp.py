"""Pins of the oracle's proposal network and learned chain (no GPU)."""
import numpy as np
import pytest

import oracle as O
from oracle import mlp as OM
from paper_1808_00128_amd import workloads as W


def test_bf16_rounding_known_values():
    x = np.array([1.0, -2.0, 0.0, 1.0 + 2**-8, 1.0 + 3 * 2**-9, 3.140625, 1e-40], np.float32)
    r = OM.bf16(x)
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: ties to even -> 1.0
    assert list(r[:4]) == [1.0, -2.0, 0.0, 1.0]
    assert r[4] == np.float32(1.0 + 2**-7)   # 1 + 3*2^-9 rounds up
    assert r[5] == np.float32(3.140625)      # exactly representable
    assert r[6] == OM.bf16(np.array([1e-40], np.float32))[0]
    # idempotent and within half an ulp: 8 significant bits, so 2^-8 relative
    y = np.random.default_rng(0).standard_normal(10000).astype(np.float32)
    b = OM.bf16(y)
    assert np.array_equal(OM.bf16(b), b)
    assert np.max(np.abs(b - y) / np.abs(y)) <= 2**-8 + 1e-12


def small_mlp(n=5, H=8, seed=3):
    p = W.mlp_init(n, H, seed=seed, flip_bias=0.2)
    rng = np.random.default_rng(seed)
    for k in ("b1", "b2"):
        p[k] = rng.uniform(-0.5, 0.5, size=p[k].shape).astype(np.float32)
    p["W3"] = (p["W3"] * 10).astype(np.float32)
    return OM.MLPRef(p, n, H)


def test_backward_matches_finite_differences():
    n, H = 5, 8
    m = small_mlp(n, H)
    rng = np.random.default_rng(1)
    x = W.random_bitstrings(n, 16, rng)
    t = W.random_bitstrings(n, 16, rng)
    loss, grads = m.loss_and_grad(x, t, exact=True)
    base = {k: v.astype(np.float64) for k, v in m.p.items()}
    h = 1e-6
    for k in OM.PARAM_ORDER:
        flat = base[k].ravel()
        for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            for sgn, store in ((1, "p"), (-1, "m")):
                pass
            pp = flat.copy(); pp[idx] += h
            pm = flat.copy(); pm[idx] -= h
            m.p[k] = pp.reshape(base[k].shape)
            lp = m.loss(x, t, exact=True)
            m.p[k] = pm.reshape(base[k].shape)
            lm = m.loss(x, t, exact=True)
            m.p[k] = base[k].copy()
            fd = (lp - lm) / (2 * h)
            an = grads[k].ravel()[idx]
            assert abs(fd - an) <= 1e-6 + 1e-5 * abs(fd), (k, idx, fd, an)


def test_bf16_path_close_to_exact():
    n, H = 12, 32
    p = W.mlp_init(n, H, seed=5)
    m = OM.MLPRef(p, n, H)
    rng = np.random.default_rng(2)
    x = W.random_bitstrings(n, 64, rng)
    t = W.random_bitstrings(n, 64, rng)
    l_b, g_b = m.loss_and_grad(x, t)
    l_e, g_e = m.loss_and_grad(x, t, exact=True)
    assert abs(l_b - l_e) < 1e-2 * abs(l_e)
    for k in OM.PARAM_ORDER:
        # bf16 rounding of back-propagated gradients compounds layer by layer
        assert np.linalg.norm(g_b[k] - g_e[k]) <= 5e-2 * np.linalg.norm(g_e[k]) + 1e-7


def test_loss_closed_form_and_adam_first_step():
    n, H = 4, 8
    p = {k: np.zeros_like(v) for k, v in W.mlp_init(n, H).items()}
    m = OM.MLPRef(p, n, H)
    x = np.arange(8, dtype=np.uint64)
    assert abs(m.loss(x, x) - np.log(2.0)) < 1e-7  # all logits 0
    g = {k: np.full_like(v, 0.5) for k, v in m.p.items()}
    g["b3"] = np.array([0.5, -0.25, 1e-3, 0.0], np.float32)
    m.adam_step(g, lr=0.01)
    # first Adam step: -lr * g / (|g| + eps)
    exp = -0.01 * g["b3"] / (np.abs(g["b3"]) + 1e-8)
    np.testing.assert_allclose(m.p["b3"], exp, rtol=1e-5, atol=1e-9)


def test_learned_chain_with_eps_one_is_the_plain_chain():
    """eps = 1: every proposal is the single-bit flip, q(x|y) = q(y|x), and the
    chain equals the paper's chain step for step."""
    rng = np.random.default_rng(8)
    n = 6
    circ = W.random_circuit(n, 40, rng.uniform(0, 2 * np.pi, size=3), rng)
    T = O.Terms(circ, 8, O.EXACT)
    P = np.abs(T.amplitudes(np.arange(2**n, dtype=np.uint64))) ** 2
    x0 = np.array([int(np.argmax(P))], np.uint64)
    u_mix, j, u_bits, U = W.learned_streams(n, 1, 200, rng)
    m = OM.MLPRef(W.mlp_init(n, 16), n, 16)
    tr, acc, flips, tie = OM.learned_chain(T, m, x0, u_mix, j, u_bits, U, 1.0, 0.01, 0.5)
    ptr, pacc, _ = T.metropolis(x0, j, U)
    assert np.array_equal(tr, ptr) and np.array_equal(acc, pacc)
    assert np.all(flips == 1)


def test_learned_chain_stationary_law():
    """With eps = 0.2 and an untrained network the corrected chain still samples
    P (restricted to the start's flip-connected component)."""
    rng = np.random.default_rng(9)
    n = 5
    circ = W.random_circuit(n, 30, rng.uniform(0, 2 * np.pi, size=3), rng)
    T = O.Terms(circ, 8, O.EXACT)
    P = np.abs(T.amplitudes(np.arange(2**n, dtype=np.uint64))) ** 2
    P /= P.sum()
    x0 = np.array([int(np.argmax(P))], np.uint64)
    steps = 6000
    u_mix, j, u_bits, U = W.learned_streams(n, 1, steps, rng)
    m = OM.MLPRef(W.mlp_init(n, 8, flip_bias=-1.0), n, 8)
    tr, acc, flips, _ = OM.learned_chain(T, m, x0, u_mix, j, u_bits, U, 0.2, 0.02, 0.5)
    from test_oracle_pins import component  # reuse the reachability helper

    # multi-bit moves can join components: use the component under all moves
    # the proposal can make (every mask has positive probability here)
    sup = P > 1e-14
    hist = np.bincount(tr[0, 500:].astype(np.int64), minlength=2**n) / (steps - 500)
    Pc = np.where(sup, P, 0.0)
    Pc /= Pc.sum()
    tv = 0.5 * np.abs(hist - Pc).sum()
    assert tv < 0.06, tv
    assert flips.mean() > 1.0


def test_mixture_density_at_extreme_flip_probabilities():
    """log q of the mixture proposal stays exact where the product of flip
    probabilities underflows a double: |m| = 62 bits at pi = 1e-6 gives a
    product of 1e-372.  Closed forms: for |m| != 1, log q = log(1 - eps) + lp;
    for |m| = 1, log q = log(eps / n + (1 - eps) e^{lp}); eps = 1 leaves only
    the single-flip term."""
    n, eps = 62, 0.1
    pi = np.full(n, 1e-6)
    m = np.ones(n, np.float32)
    lp = n * np.log(1e-6)
    assert lp < -745  # exp(lp) is 0 in double precision
    got = OM.log_q(pi, m, eps, n)
    assert np.isfinite(got)
    assert abs(got - (np.log1p(-eps) + lp)) <= 1e-12 * abs(lp)
    # the Metropolis-Hastings factor between two such masks is finite and exact
    pi2 = np.full(n, 2e-6)
    r = np.exp(OM.log_q(pi2, m, eps, n) - got)
    assert abs(r - 2.0**n) <= 1e-9 * 2.0**n
    one = np.zeros(n, np.float32)
    one[5] = 1
    lp1 = np.log(1e-6) + (n - 1) * np.log1p(-1e-6)
    assert abs(OM.log_q(pi, one, eps, n) - np.log(eps / n + (1 - eps) * np.exp(lp1))) < 1e-12
    assert abs(OM.log_q(pi, one, 1.0, n) - np.log(1.0 / n)) < 1e-15
    assert OM.log_q(pi, m, 1.0, n) == -np.inf  # eps = 1 never proposes a multi-bit mask
    # moderate values agree with the direct formula
    rng = np.random.default_rng(0)
    for _ in range(100):
        p = rng.uniform(0.01, 0.5, size=10)
        mm = (rng.random(10) < 0.3).astype(np.float32)
        lpp = float(np.where(mm > 0, np.log(p), np.log1p(-p)).sum())
        single = 0.2 / 10 if mm.sum() == 1 else 0.0
        assert abs(OM.log_q(p, mm, 0.2, 10) - np.log(single + 0.8 * np.exp(lpp))) < 1e-12
