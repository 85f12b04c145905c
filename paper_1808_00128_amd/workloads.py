"""Seeded synthetic inputs for the sum-over-Cliffords hot path.

This module only draws inputs: circuits over {H, S, CX, CZ} with diagonal
phase-gate slots, bitstrings, equatorial-state matrices A and the random
streams a Metropolis chain consumes.  It holds none of the method's arithmetic
(no decompositions, no CH-form algebra) and is the one module that both the
HIP path and the CPU oracle take their inputs from.

Shapes follow the paper's workloads:
  * random Clifford+phase circuits (circuit form U = D_m V_m ... V_1 D_0 of
    Sec. "Simulation algorithms"), with the phase gate diag(1, e^{i theta});
  * QAOA for Max-E3LIN2 (Sec. "Quantum approximate optimization algorithm"):
    H on every qubit, exp(-i gamma d Z_a Z_b Z_c) per triple, then exp(-i beta X_j);
  * uniformly random equatorial states, A uniform on M_n (Lemma (Norm Estimation)).

Conventions: qubit p is bit p of a uint64 bitstring.  Gate codes:
H=0, S=1, CX=2 (q = control, r = target), CZ=3, SLOT=4 (phase gate on q,
angle theta[slot]), CCZ=5 (doubly controlled Z on q, r, t).  SLOT and CCZ
entries are the circuit's non-Clifford slots, numbered together in circuit
order; a CCZ slot's theta entry is unused (0).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

OP_H, OP_S, OP_CX, OP_CZ, OP_SLOT, OP_CCZ = 0, 1, 2, 3, 4, 5
OP_NAMES = {OP_H: "H", OP_S: "S", OP_CX: "CX", OP_CZ: "CZ", OP_SLOT: "SLOT", OP_CCZ: "CCZ"}


@dataclass
class Circuit:
    n: int
    op: np.ndarray  # uint8
    q: np.ndarray   # uint8
    r: np.ndarray   # uint8
    theta: np.ndarray = field(default_factory=lambda: np.zeros(0))  # float64, one per slot
    t: np.ndarray = field(default_factory=lambda: np.zeros(0, np.uint8))  # third qubit of CCZ (else 0)

    @property
    def n_slot(self) -> int:
        return int(self.theta.size)

    @property
    def n_gates(self) -> int:
        return int(self.op.size)

    def third(self) -> np.ndarray:
        """Third qubit of every gate (0 where the gate has none)."""
        return self.t if self.t.size == self.op.size else np.zeros(self.op.size, np.uint8)

    def slot_ops(self) -> np.ndarray:
        """Op code (SLOT or CCZ) of each slot, in slot order."""
        return self.op[(self.op == OP_SLOT) | (self.op == OP_CCZ)]

    def gates(self):
        """Iterate (op, q, r, extra): extra is theta for SLOT, the third qubit
        for CCZ, None otherwise."""
        k = 0
        for o, a, b, c in zip(self.op.tolist(), self.q.tolist(), self.r.tolist(), self.third().tolist()):
            if o == OP_SLOT:
                yield o, a, b, float(self.theta[k])
                k += 1
            elif o == OP_CCZ:
                yield o, a, b, int(c)
                k += 1
            else:
                yield o, a, b, None


def _arr(lst, dt=np.uint8):
    return np.asarray(lst, dtype=dt)


def from_list(n: int, gates) -> Circuit:
    """Build a Circuit from (op, q, r[, theta]) tuples; a CCZ is (CCZ, q, r, t)."""
    op, q, r, t, th = [], [], [], [], []
    for g in gates:
        o = g[0]
        op.append(o)
        q.append(g[1])
        r.append(g[2] if len(g) > 2 and g[2] is not None else 0)
        t.append(g[3] if o == OP_CCZ else 0)
        if o == OP_SLOT:
            th.append(g[3])
        elif o == OP_CCZ:
            th.append(0.0)
    return Circuit(n, _arr(op), _arr(q), _arr(r), np.asarray(th, np.float64), _arr(t))


def random_clifford_gates(n: int, count: int, rng: np.random.Generator, ops=(OP_H, OP_S, OP_CX, OP_CZ)):
    """count gates drawn uniformly from ops; 1-qubit gates on a uniform qubit,
    2-qubit gates on a uniform ordered pair q != r."""
    out = []
    ops = list(ops)
    if n < 2:
        ops = [o for o in ops if o in (OP_H, OP_S)]
    for _ in range(count):
        o = ops[int(rng.integers(len(ops)))]
        if o in (OP_CX, OP_CZ):
            q = int(rng.integers(n))
            r = int(rng.integers(n - 1))
            if r >= q:
                r += 1
            out.append((o, q, r))
        else:
            out.append((o, int(rng.integers(n)), 0))
    return out


def random_circuit(n: int, n_clifford: int, thetas, rng: np.random.Generator,
                   qubits=None) -> Circuit:
    """Random Clifford circuit with one phase-gate slot per entry of thetas,
    each at a uniformly random gate boundary on a uniformly random qubit."""
    gates = random_clifford_gates(n, n_clifford, rng)
    thetas = list(thetas)
    pos = np.sort(rng.integers(0, n_clifford + 1, size=len(thetas))) if thetas else []
    out = []
    k = 0
    for i in range(n_clifford + 1):
        while k < len(thetas) and pos[k] == i:
            out.append((OP_SLOT, int(rng.integers(n)), 0, float(thetas[k])))
            k += 1
        if i < n_clifford:
            out.append(gates[i])
    if qubits is not None:
        qubits = list(qubits)
        out = [(g[0], qubits[g[1]], qubits[g[2]] if g[0] in (OP_CX, OP_CZ) else 0) + tuple(g[3:])
               for g in out]
        n = max(qubits) + 1
    return from_list(n, out)


def random_bitstrings(n: int, count: int, rng: np.random.Generator) -> np.ndarray:
    """count uniform strings in {0,1}^n as uint64 (bit p = qubit p)."""
    lo = rng.integers(0, 2**32, size=count, dtype=np.uint64)
    hi = rng.integers(0, 2**32, size=count, dtype=np.uint64)
    x = (hi << np.uint64(32)) | lo
    if n < 64:
        x &= np.uint64((1 << n) - 1)
    return x


def random_equatorial(n: int, L: int, rng: np.random.Generator):
    """L matrices A uniform on M_n: symmetric, off-diagonal bits, diagonal in Z_4.

    Returns (Aoff, Adiag): Aoff[l, a] is row a as uint64 (bit b = A_ab, bit a = 0),
    Adiag[l, a] = A_aa in {0,1,2,3}."""
    Aoff = np.zeros((L, n), np.uint64)
    for l in range(L):
        upper = np.triu(rng.integers(0, 2, size=(n, n), dtype=np.uint64), 1)
        full = upper | upper.T
        weights = np.uint64(1) << np.arange(n, dtype=np.uint64)
        Aoff[l] = (full * weights[None, :]).sum(axis=1, dtype=np.uint64)
    Adiag = rng.integers(0, 4, size=(L, n), dtype=np.uint8)
    return Aoff, Adiag


def metropolis_streams(n: int, n_chain: int, steps: int, rng: np.random.Generator, shared_j: bool = False):
    """Random inputs a single-bit-flip chain consumes: the bit to flip and the
    uniform for the accept test, per chain and step.  shared_j: one bit per
    step for every chain (each chain is still the paper's chain: its proposal
    is a uniform bit independent of its state), so a step reads one row of
    every term's tableau for all chains."""
    if shared_j:
        j = np.repeat(rng.integers(0, n, size=(1, steps), dtype=np.uint32), n_chain, axis=0)
    else:
        j = rng.integers(0, n, size=(n_chain, steps), dtype=np.uint32)
    u = rng.random(size=(n_chain, steps))
    return j, u


# ---------------------------------------------------------------------------
# The workload configurations (seed = 1000 + configuration number).
# ---------------------------------------------------------------------------
def config_tiny(seed: int = 1001) -> dict:
    """n = 12; 200 uniform {H,S,CX,CZ} gates; 8 T gates (theta = pi/4) at random
    positions; exact expansion chi = 2^8; all 4096 bitstrings."""
    rng = np.random.default_rng(seed)
    circ = random_circuit(12, 200, [np.pi / 4] * 8, rng)
    x = np.arange(4096, dtype=np.uint64)
    return dict(name="tiny-n12-exact", circuit=circ, chi=256, mode="exact", x=x, seed=seed)


def config_amplitudes(seed: int = 1002, chi: int = 1 << 16, n_x: int = 4096) -> dict:
    """n = 50; 2000 Clifford gates + 40 phase slots, theta ~ U(0, 2 pi); sparsified
    chi = 2^16; 4096 uniform bitstrings."""
    rng = np.random.default_rng(seed)
    thetas = rng.uniform(0.0, 2 * np.pi, size=40)
    circ = random_circuit(50, 2000, thetas, rng)
    x = random_bitstrings(50, n_x, rng)
    return dict(name="amplitudes-n50-chi65536-x4096", circuit=circ, chi=chi, mode="sparsify", x=x,
                seed=seed)


def config_norm(seed: int = 1003, chi: int = 1 << 18, L: int = 1024) -> dict:
    """n = 40; 200 Clifford gates + 30 phase slots, theta ~ U(0, 2 pi); sparsified
    chi = 2^18; L = 1024 equatorial states with A uniform on M_40."""
    rng = np.random.default_rng(seed)
    thetas = rng.uniform(0.0, 2 * np.pi, size=30)
    circ = random_circuit(40, 200, thetas, rng)
    Aoff, Adiag = random_equatorial(40, L, rng)
    return dict(name="norm-n40-chi262144-L1024", circuit=circ, chi=chi, mode="sparsify", Aoff=Aoff,
                Adiag=Adiag, seed=seed)


def qaoa_circuit(n: int, n_triples: int, rng: np.random.Generator, gamma=None, beta=None) -> tuple:
    """p = 1 QAOA for Max-E3LIN2 (Sec. "Quantum approximate optimization
    algorithm"): U = exp(-i beta B) exp(-i gamma C^) H^n with
    C^ = (1/2) sum_t d_t Z_a Z_b Z_c over random distinct triples, d = +-1, and
    B = sum_j X_j.

    exp(-i (gamma d / 2) Z_a Z_b Z_c) = CX_{a,c} CX_{b,c} exp(-i g Z_c) CX_{b,c} CX_{a,c}
    with g = gamma d / 2, and exp(-i g Z) = e^{-i g} diag(1, e^{2 i g}): a phase
    slot with theta = gamma d.  exp(-i beta X) = H exp(-i beta Z) H: a slot with
    theta = 2 beta between two H.  The global phases e^{-i g} and e^{-i beta}
    are dropped, so the circuit prepares e^{i (gamma sum_t d_t / 2 + n beta)}
    times U|0^n>.  Returns (circuit, triples, d, gamma, beta)."""
    if gamma is None:
        gamma = rng.uniform(0.0, np.pi)
    if beta is None:
        beta = rng.uniform(0.0, np.pi)
    gates = [(OP_H, j, 0) for j in range(n)]
    triples = []
    seen = set()
    while len(triples) < n_triples:
        t = tuple(sorted(rng.choice(n, size=3, replace=False).tolist()))
        if t in seen:
            continue
        seen.add(t)
        triples.append(t)
    d = rng.choice([-1, 1], size=n_triples)
    for (a, b, c), dd in zip(triples, d.tolist()):
        gates += [(OP_CX, a, c), (OP_CX, b, c), (OP_SLOT, c, 0, gamma * dd), (OP_CX, b, c),
                  (OP_CX, a, c)]
    for j in range(n):
        gates += [(OP_H, j, 0), (OP_SLOT, j, 0, 2 * beta), (OP_H, j, 0)]
    return from_list(n, gates), np.asarray(triples), d, gamma, beta


def config_qaoa(seed: int = 1004, n: int = 50, n_triples: int = 60, chi: int = 1 << 20,
                n_chain: int = 64, steps: int = 1000, gamma=None, beta=None, shared_j: bool = False) -> dict:
    """QAOA workload: the p = 1 circuit of qaoa_circuit (gamma, beta drawn
    uniformly in (0, pi) unless given), chi sparsified terms, and the random
    inputs of n_chain single-flip chains of `steps` steps."""
    rng = np.random.default_rng(seed)
    circ, triples, d, gamma, beta = qaoa_circuit(n, n_triples, rng, gamma=gamma, beta=beta)
    j, u = metropolis_streams(n, n_chain, steps, rng, shared_j=shared_j)
    return dict(name=f"qaoa-n{n}-chi{chi}-chains{n_chain}x{steps}", circuit=circ, chi=chi,
                mode="sparsify", triples=triples, d=d, gamma=gamma, beta=beta, jstream=j,
                ustream=u, seed=seed, n_chain=n_chain, steps=steps)


def hidden_shift_circuit(n: int, n_ccz: int, rng: np.random.Generator, n_cz: int | None = None,
                         n_z: int | None = None) -> tuple:
    """Hidden shift for a Maiorana-McFarland bent function (Sec. "The hidden
    shift algorithm"; Roetteler's construction), with CCZ as the non-Clifford gate.

    n = 2m qubits: x = qubits 0..m-1, y = qubits m..2m-1.  f(x, y) = x.y + g(y)
    with g a random cubic form: n_ccz / 2 products y_a y_b y_c (CCZ), n_cz
    products y_a y_b (CZ) and n_z linear terms (Z = S S).  Its dual is
    f~(x, y) = x.y + g(x).  Circuit: H^n, X^s O_f X^s, H^n, O_f~, H^n (X = H S S H),
    whose output is exactly |s>.  Returns (circuit, s) with s a uint64."""
    if n % 2 or n < 6 or n_ccz % 2:
        raise ValueError("hidden shift needs even n >= 6 and an even CCZ count")
    m = n // 2
    n_cz = m if n_cz is None else n_cz
    n_z = m // 2 if n_z is None else n_z
    triples = [tuple(sorted(rng.choice(m, size=3, replace=False).tolist())) for _ in range(n_ccz // 2)]
    pairs = [tuple(sorted(rng.choice(m, size=2, replace=False).tolist())) for _ in range(n_cz)]
    lin = rng.integers(0, m, size=n_z).tolist()
    s_bits = rng.integers(0, 2, size=n).tolist()
    s = sum(int(b) << i for i, b in enumerate(s_bits))

    def g_on(base):
        out = [(OP_CCZ, base + a, base + b, base + c) for a, b, c in triples]
        out += [(OP_CZ, base + a, base + b) for a, b in pairs]
        for a in lin:
            out += [(OP_S, base + a, 0), (OP_S, base + a, 0)]
        return out

    def x_shift():
        out = []
        for i, b in enumerate(s_bits):
            if b:
                out += [(OP_H, i, 0), (OP_S, i, 0), (OP_S, i, 0), (OP_H, i, 0)]
        return out

    inner = [(OP_CZ, i, m + i) for i in range(m)]
    hs = [(OP_H, i, 0) for i in range(n)]
    gates = hs + x_shift() + g_on(m) + inner + x_shift() + hs + g_on(0) + inner + hs
    return from_list(n, gates), s


def config_hidden_shift(seed: int = 1006, n: int = 40, n_ccz: int = 16, delta: float = 0.3,
                        n_x: int = 4096) -> dict:
    """n = 40 hidden-shift circuit with n_ccz CCZ gates, sparsified with the
    paper's term count for target error delta, chi = floor(((3/4)^-u / delta)^2);
    the bitstrings are s followed by n_x - 1 uniform strings."""
    rng = np.random.default_rng(seed)
    circ, s = hidden_shift_circuit(n, n_ccz, rng)
    chi = int(np.floor(((4.0 / 3.0) ** n_ccz / delta) ** 2))
    x = np.concatenate([np.asarray([s], np.uint64), random_bitstrings(n, n_x - 1, rng)])
    return dict(name=f"hidden-shift-n{n}-ccz{n_ccz}-chi{chi}-x{n_x}", circuit=circ, chi=chi,
                mode="sparsify", x=x, s=s, seed=seed, n_ccz=n_ccz, delta=delta)


def config_uneven(seed: int = 1005, n_inst: int = 64, n_x: int = 1024, chi_lo: int = 10,
                  chi_hi: int = 20) -> dict:
    """64 independent circuits: n ~ U{20..60}, 10..60 phase slots, 40 n Clifford
    gates, chi log-uniform in [2^chi_lo, 2^chi_hi], n_x bitstrings each."""
    rng = np.random.default_rng(seed)
    inst = []
    for i in range(n_inst):
        n = int(rng.integers(20, 61))
        m = int(rng.integers(10, 61))
        thetas = rng.uniform(0.0, 2 * np.pi, size=m)
        circ = random_circuit(n, 40 * n, thetas, rng)
        chi = int(round(2 ** rng.uniform(chi_lo, chi_hi)))
        x = random_bitstrings(n, n_x, rng)
        inst.append(dict(circuit=circ, chi=chi, mode="sparsify", x=x, seed=seed * 1000 + i))
    return dict(name=f"uneven-{n_inst}x", instances=inst, seed=seed)


# ---------------------------------------------------------------------------
# Learned proposal: initial network weights and the random inputs it consumes.
# ---------------------------------------------------------------------------
def mlp_init(n: int, hidden: int = 256, seed: int = 7, flip_bias: float = -3.0) -> dict:
    """Initial parameters of the proposal network n -> hidden -> hidden -> n:
    weights uniform in +-sqrt(6 / fan_in), hidden biases 0, output bias
    flip_bias (sigmoid(-3) ~ 0.047 flips per bit before training)."""
    rng = np.random.default_rng(seed)

    def u(shape, fan_in):
        b = np.sqrt(6.0 / fan_in)
        return rng.uniform(-b, b, size=shape).astype(np.float32)

    return {"W1": u((hidden, n), n), "b1": np.zeros(hidden, np.float32),
            "W2": u((hidden, hidden), hidden), "b2": np.zeros(hidden, np.float32),
            "W3": (0.1 * u((n, hidden), hidden)).astype(np.float32),
            "b3": np.full(n, flip_bias, np.float32)}


def learned_streams(n: int, n_chain: int, steps: int, rng: np.random.Generator):
    """Random inputs of the learned proposal per chain and step: the mixture
    draw, the single-flip bit, one uniform per bit for the flip mask, and the
    accept uniform."""
    u_mix = rng.random(size=(n_chain, steps))
    j = rng.integers(0, n, size=(n_chain, steps), dtype=np.uint32)
    u_bits = rng.random(size=(n_chain, steps, n))
    u = rng.random(size=(n_chain, steps))
    return u_mix, j, u_bits, u
