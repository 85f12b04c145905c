"""ctypes front end of the CPU oracle (test infrastructure only).

Wraps ``liboracle.so`` built from ``chsim_oracle.cpp``.  Only the tests, the
smoke check and the benchmark's CPU-baseline leg use it.  Each function names
the passage of Bravyi et al., arXiv:1808.00128, that the C++ code follows.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# A sanitizer build of the same source can be substituted for checking runs.
LIB_PATH = os.environ.get("CHSIM_ORACLE_LIB") or os.path.join(HERE, "liboracle.so")

_lib = None

u8p = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")
u32p = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
u64p = np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")
f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")


def lib():
    """Load (building first if needed) the oracle library."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        from .build_oracle import build

        build()
    L = C.CDLL(LIB_PATH)
    L.orc_philox.argtypes = [u32p, u32p, u32p]
    L.orc_uniform.argtypes = [C.c_uint64, C.c_uint64, C.c_uint32, C.c_uint32]
    L.orc_uniform.restype = C.c_double
    L.orc_stream_sparsify.restype = C.c_uint32
    L.orc_coverage.argtypes = [np.ctypeslib.ndpointer(dtype=np.int64), C.c_int]
    L.orc_ch_new.argtypes = [C.c_int]
    L.orc_ch_new.restype = C.c_void_p
    L.orc_ch_free.argtypes = [C.c_void_p]
    L.orc_ch_apply.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int]
    L.orc_ch_apply_right.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int]
    L.orc_ch_export.argtypes = [C.c_void_p, u64p, u64p, u64p, u8p, u64p, u64p, i32p]
    L.orc_ch_amplitude.argtypes = [C.c_void_p, C.c_uint64, C.POINTER(C.c_int), C.POINTER(C.c_int)]
    L.orc_ch_sample.argtypes = [C.c_void_p, C.c_uint64]
    L.orc_ch_sample.restype = C.c_uint64
    L.orc_ch_check.argtypes = [C.c_void_p]
    L.orc_ch_inner.argtypes = [C.c_void_p, u64p, u8p, C.POINTER(C.c_int), C.POINTER(C.c_int)]
    L.orc_phase_decomp.argtypes = [C.c_double, f64p, C.POINTER(C.c_int)]
    L.orc_expsum.argtypes = [C.c_int, u8p, i32p]
    L.orc_terms_build.argtypes = [C.c_int, C.c_int, u8p, u8p, u8p, u8p, C.c_int, f64p, C.c_uint64,
                                  C.c_int, C.c_uint64, C.c_void_p, C.c_uint64, C.c_int]
    L.orc_ccz_decomp.argtypes = [C.c_int, C.c_int, C.c_int, f64p, u32p, i32p]
    L.orc_terms_project.argtypes = [C.c_void_p, C.c_int, i32p, u8p, C.c_int]
    L.orc_ch_project.argtypes = [C.c_void_p, C.c_int, C.c_int]
    L.orc_terms_project_pauli.argtypes = [C.c_void_p, C.c_int, u8p, u64p, u64p, C.c_int]
    L.orc_ch_project_pauli.argtypes = [C.c_void_p, C.c_int, C.c_uint64, C.c_uint64]
    L.orc_ch_inner_ch.argtypes = [C.c_void_p, C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_int)]
    L.orc_ch_inner_brute.argtypes = [C.c_void_p, C.c_void_p, f64p]
    L.orc_terms_inner_ch.argtypes = [C.c_void_p, C.c_void_p, f64p, f64p, C.c_int]
    L.orc_terms_clone.argtypes = [C.c_void_p]
    L.orc_terms_clone.restype = C.c_void_p
    L.orc_ccz_decomp.restype = C.c_int
    L.orc_terms_build.restype = C.c_void_p
    L.orc_terms_free.argtypes = [C.c_void_p]
    L.orc_terms_error.argtypes = [C.c_void_p]
    L.orc_terms_l1.argtypes = [C.c_void_p]
    L.orc_terms_l1.restype = C.c_double
    L.orc_terms_count.argtypes = [C.c_void_p]
    L.orc_terms_count.restype = C.c_uint64
    L.orc_terms_ch.argtypes = [C.c_void_p, C.c_uint64]
    L.orc_terms_ch.restype = C.c_void_p
    L.orc_terms_b.argtypes = [C.c_void_p, C.c_uint64, f64p]
    L.orc_terms_branch.argtypes = [C.c_void_p, C.c_uint64, u8p]
    L.orc_terms_amplitudes.argtypes = [C.c_void_p, u64p, C.c_uint64, f64p, C.c_int]
    L.orc_terms_inner.argtypes = [C.c_void_p, u64p, u8p, C.c_uint64, f64p, f64p, C.c_int]
    L.orc_metropolis.argtypes = [C.c_void_p, C.c_uint32, C.c_uint32, u64p, u32p, f64p, u64p, u8p,
                                 f64p, C.c_int]
    _lib = L
    return L


def default_threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


# ---------------------------------------------------------------------------
# Counter-based generator (Philox4x32-10) and the uniform it feeds.
# ---------------------------------------------------------------------------
def philox(ctr, key):
    out = np.zeros(4, np.uint32)
    lib().orc_philox(np.asarray(ctr, np.uint32), np.asarray(key, np.uint32), out)
    return out


def uniform(seed: int, index: int, sub: int, stream: int) -> float:
    return lib().orc_uniform(seed, index, sub, stream)


def stream_sparsify() -> int:
    return lib().orc_stream_sparsify()


def coverage(reset: bool = False) -> np.ndarray:
    out = np.zeros(19, np.int64)
    lib().orc_coverage(out, 1 if reset else 0)
    return out


# ---------------------------------------------------------------------------
# One CH-form (Sec. "Phase-sensitive Clifford simulator").
# ---------------------------------------------------------------------------
class CHForm:
    """|phi> = omega U_C U_H |s>, evolved gate by gate from |0^n>."""

    def __init__(self, n: int, _handle=None, _owner=None):
        self.n = n
        if _handle is None:
            self._h = lib().orc_ch_new(n)
            if not self._h:
                raise ValueError("n must be in [1, 64]")
            self._own = True
        else:
            self._h = _handle
            self._own = False
            self._owner = _owner

    def __del__(self):
        if getattr(self, "_own", False) and self._h:
            lib().orc_ch_free(self._h)
            self._h = None

    def apply(self, op: int, q: int, r: int = 0) -> None:
        rc = lib().orc_ch_apply(self._h, op, q, r)
        if rc:
            raise ValueError(f"gate ({op},{q},{r}) rejected or failed: rc={rc}")

    def apply_right(self, op: int, q: int, r: int = 0) -> None:
        if lib().orc_ch_apply_right(self._h, op, q, r):
            raise ValueError("bad right-multiplication gate")

    def export(self) -> dict:
        n = self.n
        F = np.zeros(n, np.uint64)
        G = np.zeros(n, np.uint64)
        M = np.zeros(n, np.uint64)
        g = np.zeros(n, np.uint8)
        v = np.zeros(1, np.uint64)
        s = np.zeros(1, np.uint64)
        w = np.zeros(1, np.int32)
        lib().orc_ch_export(self._h, F, G, M, g, v, s, w)
        return dict(F=F, G=G, M=M, gamma=g, v=int(v[0]), s=int(s[0]), omega=int(w[0]))

    def amplitude_record(self, x: int):
        """(nonzero, k8, |v|) with <x|phi> = e^{i pi k8/4} 2^{-|v|/2}; Eq. (amplitude1)."""
        k = C.c_int(0)
        vc = C.c_int(0)
        nz = lib().orc_ch_amplitude(self._h, int(x), C.byref(k), C.byref(vc))
        return nz, k.value, vc.value

    def amplitude(self, x: int) -> complex:
        nz, k, vc = self.amplitude_record(x)
        if not nz:
            return 0j
        return complex(np.exp(1j * np.pi * k / 4) * 2.0 ** (-vc / 2))

    def project(self, q: int, bit: int) -> int:
        """(I + (-1)^bit Z_q) / 2 in place (end of Sec. "Phase-sensitive Clifford
        simulator"): returns 1 (state unchanged), 0 (projected to zero) or 2 (the
        state is now 2^{-1/2} times this CH form)."""
        code = lib().orc_ch_project(self._h, int(q), int(bit))
        if code < 0:
            raise RuntimeError("projection produced an invalid CH form")
        return code

    def project_pauli(self, a: int, x: int, z: int) -> int:
        """(I + P) / 2 in place for the Hermitian Pauli P = i^a X(x) Z(z) (end of
        Sec. "Phase-sensitive Clifford simulator"): returns 1 (unchanged), 0
        (projected to zero) or 2 (the state is now 2^{-1/2} times this CH form)."""
        code = lib().orc_ch_project_pauli(self._h, int(a), int(x), int(z))
        if code < 0:
            raise RuntimeError("projection produced an invalid CH form (or P is not Hermitian)")
        return code

    def sample(self, flips: int) -> int:
        return int(lib().orc_ch_sample(self._h, int(flips)))

    def check(self) -> int:
        return lib().orc_ch_check(self._h)

    def inner_record(self, Aoff, Adiag):
        """<phi_A|phi> as (rc, k8, e2): 0, or e^{i pi k8/4} 2^{e2/2}; Lemma (Inner Product)."""
        k = C.c_int(0)
        e2 = C.c_int(0)
        rc = lib().orc_ch_inner(self._h, np.ascontiguousarray(Aoff, np.uint64),
                                np.ascontiguousarray(Adiag, np.uint8), C.byref(k), C.byref(e2))
        return rc, k.value, e2.value


def inner_ch_record(bra: CHForm, ket: CHForm):
    """<bra|ket> of two CH forms as (rc, k8, e2): 0, or e^{i pi k8/4} 2^{e2/2}
    (the sum over the intersection of the two supports by Lemma (Exponential
    Sum)); rc < 0 flags an inconsistency."""
    k = C.c_int(0)
    e2 = C.c_int(0)
    rc = lib().orc_ch_inner_ch(bra._h, ket._h, C.byref(k), C.byref(e2))
    return rc, k.value, e2.value


def inner_ch(bra: CHForm, ket: CHForm) -> complex:
    rc, k, e2 = inner_ch_record(bra, ket)
    if rc < 0:
        raise RuntimeError(f"inner product record failed ({rc})")
    return 0j if rc == 0 else complex(np.exp(1j * np.pi * k / 4) * 2.0 ** (e2 / 2))


def inner_ch_brute(bra: CHForm, ket: CHForm) -> complex:
    """<bra|ket> = sum_x conj(<x|bra>) <x|ket> over all 2^n strings."""
    out = np.zeros(2)
    lib().orc_ch_inner_brute(bra._h, ket._h, out)
    return complex(out[0], out[1])


def phase_decomp(theta: float):
    """diag(1, e^{i theta}) = c0 S^k + c1 S^{k+1}; Eq. (Rtheta) after the theta reduction."""
    c = np.zeros(4)
    k = C.c_int(0)
    lib().orc_phase_decomp(float(theta), c, C.byref(k))
    return complex(c[0], c[1]), complex(c[2], c[3]), k.value


def ccz_decomp(a: int, b: int, c: int):
    """CCZ_{abc} = sum_j c_j K_j by the lifting lemma, Eq. (CCZ decomposition).

    Returns (coeffs, branches): coeffs[j] complex, branches[j] the list of
    (op, q, r) gates of K_j in order."""
    coeff = np.zeros(16)
    off = np.zeros(9, np.uint32)
    gates = np.zeros(96, np.int32)
    lib().orc_ccz_decomp(int(a), int(b), int(c), coeff, off, gates)
    g = gates.reshape(-1, 3)
    branches = [[tuple(int(v) for v in g[i]) for i in range(off[j], off[j + 1])] for j in range(8)]
    return coeff[0::2] + 1j * coeff[1::2], branches


def expsum(B: np.ndarray):
    """Z(B) = sum_x i^{x B x^T} as (re_sign, re_exp, im_sign, im_exp); Lemma (Exponential Sum)."""
    B = np.ascontiguousarray(B, np.uint8)
    N = B.shape[0]
    out = np.zeros(4, np.int32)
    lib().orc_expsum(N, B, out)
    return tuple(int(t) for t in out)


def expsum_value(B: np.ndarray) -> complex:
    rs, re, is_, ie = expsum(B)
    return complex(rs * 2.0 ** re if rs else 0.0, is_ * 2.0 ** ie if is_ else 0.0)


# ---------------------------------------------------------------------------
# Sum-over-Cliffords terms (Eqs. (Udecomp), (Vphi), Lemma (Sparsification)).
# ---------------------------------------------------------------------------
EXACT = 0
SPARSIFY = 1


class Terms:
    """The chi CH-form terms of a circuit (or a chosen subset of them)."""

    def __init__(self, circuit, chi: int, mode: int, seed: int = 0, alphas=None,
                 threads: int | None = None):
        self.n = circuit.n
        self.circuit = circuit
        op = np.ascontiguousarray(circuit.op, np.uint8)
        q = np.ascontiguousarray(circuit.q, np.uint8)
        r = np.ascontiguousarray(circuit.r, np.uint8)
        t = np.ascontiguousarray(circuit.third(), np.uint8)
        th = np.ascontiguousarray(circuit.theta, np.float64)
        if th.size == 0:
            th = np.zeros(1)
        threads = default_threads() if threads is None else threads
        if alphas is None:
            ap, na = None, 0
        else:
            self._alphas = np.ascontiguousarray(alphas, np.uint64)
            ap, na = self._alphas.ctypes.data_as(C.c_void_p), self._alphas.size
        self._h = lib().orc_terms_build(circuit.n, op.size, op, q, r, t, int(circuit.theta.size), th,
                                        int(chi), int(mode), int(seed), ap, na, threads)
        err = lib().orc_terms_error(self._h)
        if err:
            lib().orc_terms_free(self._h)
            self._h = None
            raise ValueError(f"oracle term build failed (code {err})")
        self.count = int(lib().orc_terms_count(self._h))
        self.chi = int(chi)
        self.l1 = float(lib().orc_terms_l1(self._h))
        self.threads = threads

    def __del__(self):
        if getattr(self, "_h", None):
            lib().orc_terms_free(self._h)
            self._h = None

    def term(self, i: int) -> CHForm:
        return CHForm(self.n, _handle=lib().orc_terms_ch(self._h, i), _owner=self)

    def b(self, i: int) -> complex:
        out = np.zeros(2)
        lib().orc_terms_b(self._h, i, out)
        return complex(out[0], out[1])

    def branch(self, i: int) -> np.ndarray:
        out = np.zeros(max(1, self.circuit.theta.size), np.uint8)
        lib().orc_terms_branch(self._h, i, out)
        return out[: self.circuit.theta.size]

    def amplitudes(self, x) -> np.ndarray:
        """<x|psi> = sum_alpha b_alpha <x|phi_alpha> over the built terms."""
        x = np.ascontiguousarray(x, np.uint64)
        out = np.zeros(2 * x.size)
        lib().orc_terms_amplitudes(self._h, x, x.size, out, self.threads)
        return out[0::2] + 1j * out[1::2]

    def inner(self, Aoff, Adiag):
        """overlap_l = <phi_{A_l}|psi>, eta_l = 2^n |overlap_l|^2 (Lemma (Norm Estimation))."""
        Aoff = np.ascontiguousarray(Aoff, np.uint64)
        Adiag = np.ascontiguousarray(Adiag, np.uint8)
        L = Aoff.shape[0]
        ov = np.zeros(2 * L)
        eta = np.zeros(L)
        bad = lib().orc_terms_inner(self._h, Aoff, Adiag, L, ov, eta, self.threads)
        if bad:
            raise RuntimeError("oracle inner product produced an invalid record")
        return ov[0::2] + 1j * ov[1::2], eta

    def inner_ch(self, bra: "Terms"):
        """overlap_l = <theta_l|psi> = sum_alpha b_alpha <theta_l|phi_alpha> with
        theta_l the CH form of bra's term l (its coefficient not included), and
        total = sum_l conj(b_l) overlap_l = <psi_bra|psi>."""
        ov = np.zeros(2 * bra.count)
        tot = np.zeros(2)
        if lib().orc_terms_inner_ch(self._h, bra._h, ov, tot, self.threads):
            raise RuntimeError("oracle CH x CH inner product produced an invalid record")
        return ov[0::2] + 1j * ov[1::2], complex(tot[0], tot[1])

    def clone(self) -> "Terms":
        """An independent copy of the built terms (CH forms, b, branches)."""
        c = Terms.__new__(Terms)
        c.__dict__.update({k: v for k, v in self.__dict__.items() if k != "_h"})
        c._h = lib().orc_terms_clone(self._h)
        return c

    def project(self, qubits, bits) -> None:
        """Apply prod_j (I + (-1)^{bits_j} Z_{qubits_j}) / 2 to every term: CH forms
        updated, b_alpha scaled by 2^{-1/2} or set to zero (Sec. "Phase-sensitive
        Clifford simulator", projective gates)."""
        qs = np.ascontiguousarray(qubits, np.int32)
        bs = np.ascontiguousarray(bits, np.uint8)
        if lib().orc_terms_project(self._h, qs.size, qs, bs, self.threads):
            raise RuntimeError("projection produced an invalid CH form")

    def project_pauli(self, a, x, z) -> None:
        """Apply prod_j (I + P_j) / 2, P_j = i^{a_j} X(x_j) Z(z_j) Hermitian, to
        every term in order (CH forms updated, b_alpha scaled by 2^{-1/2} or set
        to zero)."""
        a = np.ascontiguousarray(a, np.uint8)
        x = np.ascontiguousarray(x, np.uint64)
        z = np.ascontiguousarray(z, np.uint64)
        if lib().orc_terms_project_pauli(self._h, a.size, a, x, z, self.threads):
            raise RuntimeError("projection produced an invalid CH form")

    def sample_marginal(self, qubits, Aoff, Adiag, u):
        """Chain-rule sampling of the listed qubits' bits (Sec. "Fast norm
        estimation", sampling paragraph): P_w(x_1..x_w) = ||Pi psi||^2 / ||psi||^2
        with Pi = prod_j (I + (-1)^{x_j} Z_j) / 2, and the bits drawn one by one
        from P_j(x_j | x_1..x_{j-1}).  Each conditional is
        e(x_1..x_{j-1}, 0) / (e(.., 0) + e(.., 1)), e the norm estimate (mean of
        eta over the given equatorial states) of the projected terms; 1/2 when
        both are zero.  Bit j is 0 iff u[j] < that probability.  Returns
        (bits, probability of each chosen bit, the estimates e(.., 0), e(.., 1))."""
        bits, probs, e0s, e1s = [], [], [], []
        for j in range(len(qubits)):
            est = []
            for b in (0, 1):
                c = self.clone()
                c.project(qubits[: j + 1], bits + [b])
                _, eta = c.inner(Aoff, Adiag)
                est.append(float(np.mean(eta)))
                del c
            tot = est[0] + est[1]
            p0 = est[0] / tot if tot > 0 else 0.5
            x = 0 if u[j] < p0 else 1
            bits.append(x)
            probs.append(p0 if x == 0 else 1.0 - p0)
            e0s.append(est[0])
            e1s.append(est[1])
        return bits, probs, e0s, e1s

    def sparsification_bound(self, Aoff, Adiag):
        """Lemma (Sparsification tail bound), Eq. (event): ||psi - Omega||^2 <=
        <Omega|Omega> - 1 + delta^2 for chi = ||c||_1^2 / delta^2, with
        <Omega|Omega> estimated by norm estimation (Lemma (Norm Estimation))
        over the given equatorial states.  Returns (estimate, standard error,
        delta^2, bound)."""
        _, eta = self.inner(Aoff, Adiag)
        est = float(np.mean(eta))
        sem = float(np.std(eta, ddof=1) / np.sqrt(eta.size))
        delta2 = self.l1**2 / self.chi
        return est, sem, delta2, est - 1.0 + delta2

    def metropolis(self, x_init, jstream, ustream):
        """Plain single-bit-flip chains (Sec. "Heuristic Metropolis simulator")."""
        x_init = np.ascontiguousarray(x_init, np.uint64)
        jstream = np.ascontiguousarray(jstream, np.uint32)
        ustream = np.ascontiguousarray(ustream, np.float64)
        n_chain = x_init.size
        steps = jstream.size // max(1, n_chain)
        trace = np.zeros(n_chain * steps, np.uint64)
        acc = np.zeros(n_chain * steps, np.uint8)
        amp = np.zeros(2 * n_chain)
        bad = lib().orc_metropolis(self._h, n_chain, steps, x_init, jstream.reshape(-1),
                                   ustream.reshape(-1), trace, acc, amp, self.threads)
        if bad:
            raise ValueError("a chain started at a string with P(x) = 0")
        return (trace.reshape(n_chain, steps), acc.reshape(n_chain, steps),
                amp[0::2] + 1j * amp[1::2])
