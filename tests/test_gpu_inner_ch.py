"""GPU parity of inner products with general stabilizer states (CH forms):
chsim_inner_products_ch against the oracle's CH x CH inner product.

The bra states are the terms of a second instance (random Clifford circuits
with phase slots, so the terms are distinct stabilizer states).  Overlaps and
totals within 1e-12 normwise of the oracle; the equatorial special case also
against the GPU's own equatorial path, which the oracle checks elsewhere.
"""
import sys

import numpy as np
import pytest

import oracle as O
from paper_1808_00128_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


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


def normwise(a, ref):
    rms = np.sqrt(np.mean(np.abs(ref) ** 2))
    if rms == 0:
        return float(np.max(np.abs(a)))
    return float(np.max(np.abs(a - ref)) / rms)


def _shallow(n, rng, slots):
    """H on a few qubits, then S/CX/CZ and phase slots: terms near basis
    states, so many pairs of supports do not meet."""
    gates = [(W.OP_H, q, 0) for q in rng.choice(n, size=min(n, 3), replace=False).tolist()]
    body = W.random_clifford_gates(n, 8 * n, rng, ops=(W.OP_S, W.OP_CX, W.OP_CZ))
    pos = set(rng.choice(len(body), size=slots, replace=False).tolist())
    for i, g in enumerate(body):
        gates.append(g)
        if i in pos:
            q = int(rng.integers(n))
            gates += [(W.OP_SLOT, q, 0, float(rng.uniform(0, 2 * np.pi))), (W.OP_H, q, 0)]
    return W.from_list(n, gates)


CASES = [
    # (n, ket gates, ket slots, chi_ket, bra gates, bra slots, chi_bra, shallow)
    (1, 10, 2, 4, 10, 3, 5, False),
    (5, 80, 4, 40, 60, 6, 33, False),
    (12, 200, 6, 300, 150, 8, 70, False),
    (12, 0, 5, 200, 0, 6, 64, True),
    (33, 500, 8, 257, 400, 10, 65, False),
    (50, 900, 10, 200, 600, 12, 64, False),
    (64, 700, 8, 129, 500, 10, 40, False),
]


@pytest.mark.parametrize("case", CASES, ids=[f"n{c[0]}-k{c[3]}-b{c[6]}{'-shallow' if c[7] else ''}" for c in CASES])
def test_inner_ch_matches_oracle(B, case):
    n, gk, mk, chik, gb, mb, chib, shallow = case
    rng = np.random.default_rng(1300 + n + chib)
    if shallow:
        ck, cb = _shallow(n, rng, mk), _shallow(n, rng, mb)
    else:
        ck = W.random_circuit(n, gk, rng.uniform(0, 2 * np.pi, size=mk), rng)
        cb = W.random_circuit(n, gb, rng.uniform(0, 2 * np.pi, size=mb), rng)
    sk = dict(circuit=ck, chi=chik, mode="sparsify", seed=11 + n)
    sb = dict(circuit=cb, chi=chib, mode="sparsify", seed=12 + n)
    say(f"inner CH x CH n={n} chi_ket={chik} chi_bra={chib} shallow={shallow}")
    ctx = B.Context([sk, sb])
    ctx.apply_circuit(ck, inst=0)
    ctx.apply_circuit(cb, inst=1)
    ov, tot = ctx.inner_products_ch(1, inst=0)
    Tk = O.Terms(ck, chik, O.SPARSIFY, seed=sk["seed"])
    Tb = O.Terms(cb, chib, O.SPARSIFY, seed=sb["seed"])
    ref, rtot = Tk.inner_ch(Tb)
    assert normwise(ov, ref) < TOL64
    assert abs(tot - rtot) <= TOL64 * max(1.0, np.sqrt(np.sum(np.abs(ref) ** 2)))
    if shallow:
        # pairs whose supports miss each other (zero inner product) occur
        zero = sum(O.inner_ch(Tb.term(l), Tk.term(a)) == 0 for l in range(8) for a in range(40))
        assert zero > 0
    if n <= 33:
        # <Omega|Omega> of the ket set by all chi^2 pairs
        _, self_tot = ctx.inner_products_ch(0, inst=0)
        _, rself = Tk.inner_ch(Tk)
        assert abs(self_tot - rself) <= TOL64 * max(1.0, abs(rself))
        assert abs(self_tot.imag) <= TOL64 * max(1.0, abs(rself))
    ctx.close()


@pytest.mark.parametrize("n", [8, 40])
def test_inner_ch_equatorial_case_matches_equatorial_path(B, n):
    """A bra instance holding phi_A (H on every qubit, S^{A_aa}, CZ for
    A_ab = 1) gives the overlap of the equatorial-state path."""
    rng = np.random.default_rng(1400 + n)
    ck = W.random_circuit(n, 25 * n, rng.uniform(0, 2 * np.pi, size=6), rng)
    Aoff, Adiag = W.random_equatorial(n, 1, rng)
    gates = [(W.OP_H, q, 0) for q in range(n)]
    for q in range(n):
        gates += [(W.OP_S, q, 0)] * int(Adiag[0, q])
        gates += [(W.OP_CZ, q, r) for r in range(q + 1, n) if (int(Aoff[0, q]) >> r) & 1]
    ca = W.from_list(n, gates)
    say(f"inner CH x CH equatorial n={n}")
    ctx = B.Context([dict(circuit=ck, chi=500, mode="sparsify", seed=3),
                     dict(circuit=ca, chi=1, mode="exact", seed=0)])
    ctx.apply_circuit(ck, inst=0)
    ctx.apply_circuit(ca, inst=1)
    ov, _ = ctx.inner_products_ch(1, inst=0)
    eq, _, _ = ctx.inner_products(Aoff, Adiag, inst=0)
    assert abs(ov[0] - eq[0]) <= TOL64 * max(abs(eq[0]), 1e-300)
    ctx.close()


def _with_slots(n, gates, rng, slots):
    """The gates with phase slots (S-power branches, left rules) inserted at
    random positions after the first gate."""
    out = list(gates)
    for _ in range(slots):
        pos = int(rng.integers(1, len(out) + 1))
        out.insert(pos, (W.OP_SLOT, int(rng.integers(n)), 0, float(rng.uniform(0, 2 * np.pi))))
    return out


@pytest.mark.parametrize("k", [30, 31, 32, 33])
def test_inner_ch_free_variable_count_boundary(B, k):
    """Kets with v = {0, ..., k-1} (Hadamards on k fresh qubits of |0^n>, then
    only S, CX, CZ and phase slots, which are left rules and keep v) against
    bras with v = every qubit (no equations): every pair has exactly k free
    variables, on both sides of the 31 at which the pair kernel changes from
    32-bit to 64-bit rows."""
    n = 40
    rng = np.random.default_rng(1600 + k)
    left = (W.OP_S, W.OP_CX, W.OP_CZ)
    kg = [(W.OP_H, q, 0) for q in range(k)]
    kg += _with_slots(n, W.random_clifford_gates(n, 300, rng, ops=left), rng, 6)
    bg = [(W.OP_H, q, 0) for q in range(n)]
    bg += _with_slots(n, W.random_clifford_gates(n, 200, rng, ops=left), rng, 4)
    ck, cb = W.from_list(n, kg), W.from_list(n, bg)
    sk = dict(circuit=ck, chi=64, mode="sparsify", seed=1610 + k)
    sb = dict(circuit=cb, chi=8, mode="sparsify", seed=1620 + k)
    say(f"inner CH x CH free-variable boundary k={k}")
    ctx = B.Context([sk, sb])
    ctx.apply_circuit(ck, inst=0)
    ctx.apply_circuit(cb, inst=1)
    Tk = O.Terms(ck, 64, O.SPARSIFY, seed=sk["seed"])
    Tb = O.Terms(cb, 8, O.SPARSIFY, seed=sb["seed"])
    assert all(int(Tk.term(a).export()["v"]) == (1 << k) - 1 for a in range(64))
    assert all(int(Tb.term(l).export()["v"]) == (1 << n) - 1 for l in range(8))
    ov, tot = ctx.inner_products_ch(1, inst=0)
    ref, rtot = Tk.inner_ch(Tb)
    assert normwise(ov, ref) < TOL64
    assert abs(tot - rtot) <= TOL64 * max(1.0, np.sqrt(np.sum(np.abs(ref) ** 2)))
    ctx.close()


def test_inner_ch_norm_config_subset(B):
    """The norm-estimation workload's circuit (n = 40, 30 slots), its first 256
    terms against 8 random stabilizer states (terms of a random Clifford +
    phase-slot circuit) on the oracle."""
    cfg = W.config_norm(L=8)
    rng = np.random.default_rng(1500)
    cb = W.random_circuit(40, 400, rng.uniform(0, 2 * np.pi, size=30), rng)
    sk = dict(cfg, chi=256)
    sb = dict(circuit=cb, chi=8, mode="sparsify", seed=1501)
    say("inner CH x CH norm config subset n=40 chi=256 L=8")
    ctx = B.Context([sk, sb])
    ctx.apply_circuit(cfg["circuit"], inst=0)
    ctx.apply_circuit(cb, inst=1)
    ov, tot = ctx.inner_products_ch(1, inst=0)
    Tk = O.Terms(cfg["circuit"], 256, O.SPARSIFY, seed=cfg["seed"])
    Tb = O.Terms(cb, 8, O.SPARSIFY, seed=1501)
    ref, rtot = Tk.inner_ch(Tb)
    assert normwise(ov, ref) < TOL64
    ctx.close()


def test_inner_ch_rejects_mismatched_instances(B):
    c4 = W.from_list(4, [(W.OP_H, 0, 0)])
    c5 = W.from_list(5, [(W.OP_H, 0, 0)])
    ctx = B.Context([dict(circuit=c4, chi=2, mode="sparsify", seed=0),
                     dict(circuit=c5, chi=2, mode="sparsify", seed=0)])
    with pytest.raises(B.ChsimError, match="EINVAL"):
        ctx.inner_products_ch(1, inst=0)
    with pytest.raises(B.ChsimError, match="EINVAL"):
        ctx.inner_products_ch(2, inst=0)
    ctx.close()
