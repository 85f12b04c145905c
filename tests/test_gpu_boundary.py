"""GPU tests of the C ABI's state rules: the CH-form invariant check
(chsim_validate), the range checks of chsim_set_terms, and chains dropped by
every call that changes the terms.

The invariant test needs no oracle: it evolves terms, corrupts one entry of
a downloaded term in a way that breaks a named invariant of Eq. (tableaux),
uploads it, and expects the check to name that term and that invariant.
"""
import sys

import numpy as np
import pytest

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


def evolved(B, n, chi, seed, slots=6, gates=None):
    rng = np.random.default_rng(seed)
    circ = W.random_circuit(n, gates or 20 * n, rng.uniform(0, 2 * np.pi, size=slots), rng)
    spec = dict(circuit=circ, chi=chi, mode="sparsify", seed=seed)
    ctx = B.Context([spec])
    ctx.apply_circuit(circ)
    return ctx, circ, rng


@pytest.mark.parametrize("n,chi", [(1, 5), (7, 300), (33, 1000), (50, 4099), (64, 257)])
def test_validate_accepts_evolved_terms(B, n, chi):
    say(f"validate evolved n={n} chi={chi}")
    ctx, _, _ = evolved(B, n, chi, 3000 + n)
    assert ctx.validate() == (0, None, 0)
    assert ctx.validate(first=chi // 3, count=chi - chi // 3) == (0, None, 0)
    assert ctx.validate(first=chi, count=0) == (0, None, 0)
    with pytest.raises(B.ChsimError, match="EINVAL"):
        ctx.validate(first=1, count=chi)
    ctx.close()


def _upload(ctx, a, t):
    ctx.set_terms(a, t["F"], t["G"], t["M"], t["gamma"], t["v"], t["s"], t["omega"], t["b"])


@pytest.mark.parametrize("n", [5, 40, 64])
def test_validate_names_each_broken_invariant(B, n):
    """Flip one bit of F (breaks F G^T = I), one bit of gamma's low plane
    (breaks gamma_p = F_p . M_p), and one bit of M (breaks M F^T symmetric or,
    when column j of F is e_p, gamma's parity): each corrupted term is found,
    the smallest index is reported, and the flag names the invariant."""
    chi = 600
    ctx, _, rng = evolved(B, n, chi, 3100 + n)
    assert ctx.validate() == (0, None, 0)
    base = {a: ctx.get_terms(a, 1) for a in (17, 301, 599)}
    # F row 0, bit n-1
    t = {k: v.copy() for k, v in base[301].items()}
    t["F"][0, 0] ^= np.uint64(1 << (n - 1))
    _upload(ctx, 301, t)
    nb, fb, what = ctx.validate()
    assert (nb, fb) == (1, 301) and what & B.CHSIM_BAD_TABLEAU, what
    # gamma low bit of the last row
    t = {k: v.copy() for k, v in base[599].items()}
    t["gamma"][0, n - 1] ^= 1
    _upload(ctx, 599, t)
    nb, fb, what = ctx.validate()
    assert (nb, fb) == (2, 301) and what & B.CHSIM_BAD_GAMMA, what
    # M row p, bit j
    t = {k: v.copy() for k, v in base[17].items()}
    p, j = n // 2, (n // 3) % n
    t["M"][0, p] ^= np.uint64(1 << j)
    _upload(ctx, 17, t)
    nb, fb, what = ctx.validate()
    assert (nb, fb) == (3, 17), (nb, fb)
    only17 = ctx.validate(first=0, count=100)
    assert only17[0] == 1 and only17[1] == 17
    assert only17[2] & (B.CHSIM_BAD_SYMMETRY | B.CHSIM_BAD_GAMMA)
    # restoring the terms clears every flag
    for a, t in base.items():
        _upload(ctx, a, t)
    assert ctx.validate() == (0, None, 0)
    ctx.close()


def test_set_terms_rejects_out_of_range_words(B):
    n, chi = 12, 40
    say("set_terms range checks")
    ctx, _, _ = evolved(B, n, chi, 3200)
    good = ctx.get_terms(3, 1)
    before = ctx.get_terms(0, chi)
    for field, value in (("v", 1 << n), ("s", 1 << 63), ("omega", 8), ("gamma", 4)):
        t = {k: v.copy() for k, v in good.items()}
        if field == "gamma":
            t["gamma"][0, 2] = value
        else:
            t[field][0] = value
        with pytest.raises(B.ChsimError, match="EINVAL"):
            _upload(ctx, 3, t)
    for field in ("F", "G", "M"):
        t = {k: v.copy() for k, v in good.items()}
        t[field][0, 5] |= np.uint64(1 << n)
        with pytest.raises(B.ChsimError, match="EINVAL"):
            _upload(ctx, 3, t)
    after = ctx.get_terms(0, chi)
    for k in before:
        assert np.array_equal(before[k], after[k]), k
    ctx.close()


def _chains(B, ctx, n, rng, count=4):
    chi = ctx.info()[1]
    xs = []
    while len(xs) < count:
        cand = ctx.sample_terms(rng.integers(0, chi, size=8), W.random_bitstrings(n, 8, rng))
        amp = ctx.amplitudes(cand)
        xs += [int(x) for x, a in zip(cand, amp) if abs(a) > 0]
    return np.array(xs[:count], np.uint64)


def test_term_mutations_drop_chains(B):
    """After chsim_metropolis_init, each call that changes the terms (one more
    gate, set_terms, a projection, a copy into the instance, a reset) makes the
    next step fail with EINVAL, plain and graph, until the chains start again;
    the restarted chains step normally."""
    import torch

    n, chi = 10, 200
    say("chains dropped by term mutations")
    rng = np.random.default_rng(3300)
    circ = W.random_circuit(n, 100, rng.uniform(0, 2 * np.pi, size=5), rng)
    spec = dict(circuit=circ, chi=chi, mode="sparsify", seed=9)
    ctx = B.Context([spec, spec])
    ctx.apply_circuit(circ, inst=0)
    ctx.apply_circuit(circ, inst=1)
    j, u = W.metropolis_streams(n, 4, 5, rng)
    t0 = ctx.get_terms(0, chi)

    def mutations():
        yield "apply_clifford", lambda: ctx.apply_gates(B.gate_array(W.from_list(n, [(W.OP_S, 2, 0)])))
        yield "set_terms", lambda: ctx.set_terms(0, t0["F"], t0["G"], t0["M"], t0["gamma"], t0["v"],
                                                 t0["s"], t0["omega"], t0["b"])
        yield "project_z", lambda: ctx.project_z([1], [0])
        yield "terms_copy", lambda: ctx.copy_terms(1, 0)
        yield "terms_reset", lambda: (ctx.reset(9), ctx.apply_circuit(circ))

    for name, mutate in mutations():
        ctx.copy_terms(1, 0)
        x0 = _chains(B, ctx, n, rng)
        ctx.metropolis_init(x0)
        ctx.metropolis_step(j, u, graph=True)
        mutate()
        with pytest.raises(B.ChsimError, match="EINVAL"):
            ctx.metropolis_step(j, u)
        with pytest.raises(B.ChsimError, match="EINVAL"):
            ctx.metropolis_step(j, u, graph=True)
        if name != "project_z":
            x0 = _chains(B, ctx, n, rng)
            ctx.metropolis_init(x0)
            tr, acc, _ = ctx.metropolis_step(j, u, graph=True)
            assert tr.shape == (4, 5)
    # a mutation of another instance leaves these chains alone
    ctx.copy_terms(1, 0)
    x0 = _chains(B, ctx, n, rng)
    ctx.metropolis_init(x0)
    ctx.project_z([0], [1], inst=1)
    ctx.metropolis_step(j, u)
    torch.cuda.synchronize()
    ctx.close()
