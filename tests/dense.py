"""Textbook dense statevector simulator (numpy), used only to pin the oracle.

Written independently of the oracle: a 2^n complex vector, qubit p = bit p of
the basis index, gates applied by index arithmetic.
"""
import numpy as np

from paper_1808_00128_amd.workloads import OP_CCZ, OP_CX, OP_CZ, OP_H, OP_S, OP_SLOT


def zero_state(n):
    psi = np.zeros(2**n, np.complex128)
    psi[0] = 1.0
    return psi


def apply(psi, n, op, q, r=0, theta=None):
    idx = np.arange(2**n)
    bq = (idx >> q) & 1
    if op == OP_H:
        i0 = idx & ~(1 << q)
        i1 = idx | (1 << q)
        return (psi[i0] + np.where(bq == 1, -1.0, 1.0) * psi[i1]) / np.sqrt(2.0)
    if op == OP_S:
        return psi * np.where(bq == 1, 1j, 1.0)
    if op == OP_CZ:
        br = (idx >> r) & 1
        return psi * np.where((bq & br) == 1, -1.0, 1.0)
    if op == OP_CX:
        return psi[idx ^ (bq << r)]
    if op == OP_SLOT:
        return psi * np.where(bq == 1, np.exp(1j * theta), 1.0)
    if op == OP_CCZ:  # theta carries the third qubit
        br = (idx >> r) & 1
        bt = (idx >> theta) & 1
        return psi * np.where((bq & br & bt) == 1, -1.0, 1.0)
    raise ValueError(op)


def run(circuit):
    n = circuit.n
    psi = zero_state(n)
    for op, q, r, th in circuit.gates():
        psi = apply(psi, n, op, q, r, th)
    return psi


def run_gates(n, gates):
    psi = zero_state(n)
    for g in gates:
        psi = apply(psi, n, g[0], g[1], g[2] if len(g) > 2 else 0, g[3] if len(g) > 3 else None)
    return psi


def equatorial(n, Aoff_row, Adiag_row):
    """phi_A = 2^{-n/2} sum_x i^{x A x^T} |x> (Eq. (eqa1))."""
    idx = np.arange(2**n)
    bits = (idx[:, None] >> np.arange(n)[None, :]) & 1
    A = np.zeros((n, n), np.int64)
    for a in range(n):
        for b in range(n):
            A[a, b] = (int(Aoff_row[a]) >> b) & 1
        A[a, a] = int(Adiag_row[a])
    quad = np.einsum("xa,ab,xb->x", bits, A, bits) % 4
    return (1j ** quad) / 2 ** (n / 2)


def expsum_brute(B):
    """sum over x in {0,1}^N of i^{x B x^T}, B symmetric integer matrix."""
    N = B.shape[0]
    if N == 0:
        return 1.0 + 0j
    idx = np.arange(2**N)
    bits = (idx[:, None] >> np.arange(N)[None, :]) & 1
    quad = np.einsum("xa,ab,xb->x", bits, B.astype(np.int64), bits) % 4
    return complex(np.sum(1j ** quad))
