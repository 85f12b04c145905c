"""Host-side checks of libchsim.so that need no GPU.

The library must load and export every entry point include/chsim.h declares;
argument checks must reject bad input before touching a device; the host
decomposition helper must reproduce diag(1, e^{i theta}) exactly.
"""
import ctypes as C
import os
import re

import numpy as np

import dense
import pytest

import oracle as O
from paper_1808_00128_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "chsim.h")).read()
    return sorted(set(re.findall(r"^(?:chsim_status|const char\*)\s+(chsim_\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_symbol():
    L = B.lib()
    names = header_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(L, name), name
    assert sorted(B.EXPORTED) == names


def test_decompose_phase_is_exact_and_matches_oracle():
    S = np.diag([1, 1j])
    for theta in np.concatenate([np.linspace(-7, 7, 301), [0.0, np.pi / 4, np.pi / 2, 3 * np.pi / 2]]):
        d = B.PhaseDecomposition(theta, 5)
        c0, c1 = d.c
        off = list(d.off)
        k0 = off[1] - off[0]
        k1 = off[2] - off[1]
        assert (k0 + 1) % 4 == k1 % 4
        for gi in range(off[2]):
            assert d.gates[gi].op == B.W.OP_S and d.gates[gi].q == 5
        lhs = c0 * np.linalg.matrix_power(S, k0) + c1 * np.linalg.matrix_power(S, k1)
        np.testing.assert_allclose(lhs, np.diag([1, np.exp(1j * theta)]), atol=1e-14)
        o0, o1, ok = O.phase_decomp(theta)
        assert ok == k0
        assert abs(o0 - c0) < 1e-15 and abs(o1 - c1) < 1e-15


def test_decompose_phase_rejects_bad_input():
    with pytest.raises(B.ChsimError):
        B.PhaseDecomposition(float("nan"), 0)
    with pytest.raises(B.ChsimError):
        B.PhaseDecomposition(0.3, 64)


@pytest.mark.parametrize("qubits", [(0, 1, 2), (7, 2, 5), (63, 0, 31)])
def test_decompose_ccz_is_exact_and_matches_oracle(qubits):
    a, b, c = qubits
    d = B.CCZDecomposition(a, b, c)
    assert d.decomp.n_branch == 8 and d.off[8] == 24
    got = d.branches()
    oc, ob = O.ccz_decomp(a, b, c)
    np.testing.assert_array_equal(np.array(d.c), oc)  # same order, same doubles
    for j in range(8):
        assert sorted(got[j]) == sorted(ob[j])  # diagonal gates: order within a branch is free
    # sum_j c_j K_j = CCZ on the three qubits (relabelled 0, 1, 2; dense)
    lab = {a: 0, b: 1, c: 2}
    total = np.zeros(8, np.complex128)
    for cj, K in zip(d.c, got):
        diag = np.ones(8, np.complex128)
        for op, q, r in K:
            diag = dense.apply(diag, 3, op, lab[q], lab.get(r, 0))
        total += cj * diag
    np.testing.assert_allclose(total, [1, 1, 1, 1, 1, 1, 1, -1], atol=1e-15)


def test_decompose_ccz_rejects_bad_input():
    for args in [(0, 0, 1), (1, 2, 2), (3, 4, 3), (64, 0, 1), (0, 1, 99)]:
        with pytest.raises(B.ChsimError):
            B.CCZDecomposition(*args)


def test_gate_array_numbers_phase_and_ccz_slots_together():
    circ = B.W.from_list(6, [(B.W.OP_H, 0, 0), (B.W.OP_CCZ, 0, 1, 2), (B.W.OP_SLOT, 3, 0, 0.4),
                             (B.W.OP_CX, 1, 4), (B.W.OP_CCZ, 5, 3, 1)])
    g = B.gate_array(circ)
    assert g["op"].tolist() == [B.W.OP_H, B.W.OP_SLOT, B.W.OP_SLOT, B.W.OP_CX, B.W.OP_SLOT]
    assert g["slot"].tolist() == [0, 0, 1, 0, 2]
    decs = B.slot_decompositions(circ)
    assert [type(x).__name__ for x in decs] == ["CCZDecomposition", "PhaseDecomposition", "CCZDecomposition"]


def make_instance(n, chi, mode=B.CHSIM_SPARSIFY, n_slot=0):
    return B.Instance(n, n_slot, None, chi, mode, 0)


@pytest.mark.parametrize("n,chi,mode", [(0, 4, B.CHSIM_SPARSIFY), (65, 4, B.CHSIM_SPARSIFY),
                                        (5, 0, B.CHSIM_SPARSIFY), (5, 2, B.CHSIM_EXACT)])
def test_terms_init_rejects_bad_instances(n, chi, mode):
    """Invalid instances fail with EINVAL before any device is touched."""
    insts = (B.Instance * 1)()
    insts[0] = make_instance(n, chi, mode)
    h = C.c_void_p()
    st = B.lib().chsim_terms_init(C.byref(h), 0, 1, insts)
    assert st == B.CHSIM_EINVAL
    assert not h.value
    assert len(B.lib().chsim_last_error()) > 0


def test_null_context_rejected():
    L = B.lib()
    assert L.chsim_amplitudes(None, 0, None, 0, None, 0, None) == B.CHSIM_EINVAL
    assert L.chsim_amplitudes_batch(None, None, 0, 0, None) == B.CHSIM_EINVAL
    assert L.chsim_destroy(None) == B.CHSIM_OK


def test_gate_array_numbers_slots_in_order():
    from paper_1808_00128_amd import workloads as W
    circ = W.from_list(3, [(W.OP_H, 0, 0), (W.OP_SLOT, 1, 0, 0.3), (W.OP_CX, 0, 2),
                           (W.OP_SLOT, 2, 0, 0.5)])
    g = B.gate_array(circ)
    assert list(g["op"]) == [0, 4, 2, 4]
    assert list(g["slot"]) == [0, 0, 0, 1]
    assert list(g["r"]) == [0, 0, 2, 0]
