"""Thin ctypes front end of libchsim.so (the C ABI in include/chsim.h).

Argument marshalling only: every step of the hot path runs in the HIP
kernels behind the C ABI.  Inputs may be numpy arrays (host pointers) or torch
tensors on the GPU (device pointers, enqueued on torch's current stream).
If the library is missing, every entry point raises: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import workloads as W

PKG = os.path.dirname(os.path.abspath(__file__))
# CHSIM_LIB names another build of the same sources (the host-only sanitizer
# build used for checking runs); by default the in-tree library.
LIB_PATH = os.environ.get("CHSIM_LIB") or os.path.join(PKG, "libchsim.so")

CHSIM_OK, CHSIM_EINVAL, CHSIM_ENOMEM, CHSIM_EDEVICE, CHSIM_EUNSUPPORTED, CHSIM_ESTATE = range(6)
STATUS_NAMES = {0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "EDEVICE", 4: "EUNSUPPORTED", 5: "ESTATE"}
CHSIM_EXACT, CHSIM_SPARSIFY = 0, 1
CHSIM_FP64, CHSIM_FP32C, CHSIM_DEVICE_PTRS, CHSIM_GRAPH = 0, 1, 0x100, 0x200
CHSIM_TUNE_EVOLVE_LANES = 1
CHSIM_TUNE_PREFIX_SHARE = 2
CHSIM_TUNE_AMP_STRINGS = 3
CHSIM_EVOLVE_LDS = 0x100
CHSIM_BAD_TABLEAU, CHSIM_BAD_SYMMETRY, CHSIM_BAD_GAMMA, CHSIM_BAD_RANGE = 1, 2, 4, 8
# evolution shapes the autotuner times, in the order of its timings
TUNE_SHAPES = (4, 8, 16, 32, 64, 4 | CHSIM_EVOLVE_LDS, 8 | CHSIM_EVOLVE_LDS, 16 | CHSIM_EVOLVE_LDS)
MAX_BRANCH = 8

EXPORTED = [
    "chsim_terms_init", "chsim_terms_reset", "chsim_apply_clifford", "chsim_amplitudes",
    "chsim_amplitudes_batch", "chsim_amplitudes_noalloc", "chsim_inner_products", "chsim_inner_products_ch", "chsim_sparsification_bound",
    "chsim_project_z", "chsim_project_pauli", "chsim_terms_copy", "chsim_sample_marginal",
    "chsim_metropolis_init", "chsim_metropolis_step", "chsim_sample_terms", "chsim_get_terms",
    "chsim_set_terms", "chsim_validate", "chsim_decompose_phase", "chsim_decompose_ccz", "chsim_set_tuning", "chsim_get_tuning",
    "chsim_instance_info", "chsim_evolution_stats", "chsim_measure_peaks", "chsim_destroy", "chsim_mlp_create", "chsim_mlp_destroy",
    "chsim_mlp_get_params", "chsim_mlp_set_params", "chsim_mlp_forward", "chsim_mlp_loss_grad",
    "chsim_mlp_train", "chsim_metropolis_step_learned",
    "chsim_last_error",
]


class ChsimError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"chsim {STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class Gate(C.Structure):
    _fields_ = [("op", C.c_uint8), ("q", C.c_uint8), ("r", C.c_uint8), ("pad", C.c_uint8),
                ("slot", C.c_uint32)]


class Decomp(C.Structure):
    _fields_ = [("n_branch", C.c_uint32), ("coeff", C.POINTER(C.c_double)),
                ("off", C.POINTER(C.c_uint32)), ("gates", C.POINTER(Gate))]


class Instance(C.Structure):
    _fields_ = [("n", C.c_uint32), ("n_slot", C.c_uint32), ("slot_decomp", C.POINTER(Decomp)),
                ("chi", C.c_uint64), ("mode", C.c_uint32), ("seed", C.c_uint64)]


class AmpRequest(C.Structure):
    _fields_ = [("inst", C.c_uint32), ("reserved", C.c_uint32), ("x", C.c_void_p),
                ("n_x", C.c_size_t), ("out", C.c_void_p)]


class LearnedArgs(C.Structure):
    _fields_ = [("eps", C.c_float), ("pi_min", C.c_float), ("pi_max", C.c_float),
                ("u_mix", C.c_void_p), ("j", C.c_void_p), ("u_bits", C.c_void_p),
                ("u", C.c_void_p)]


PARAM_ORDER = ("W1", "b1", "W2", "b2", "W3", "b3")


def pack_params(params):
    return np.ascontiguousarray(np.concatenate([np.asarray(params[k], np.float32).ravel()
                                                for k in PARAM_ORDER]))


def unpack_params(flat, n, H):
    shapes = {"W1": (H, n), "b1": (H,), "W2": (H, H), "b2": (H,), "W3": (n, H), "b3": (n,)}
    out, off = {}, 0
    for k in PARAM_ORDER:
        size = int(np.prod(shapes[k]))
        out[k] = flat[off:off + size].reshape(shapes[k]).copy()
        off += size
    return out


GATE_DTYPE = np.dtype([("op", "u1"), ("q", "u1"), ("r", "u1"), ("pad", "u1"), ("slot", "<u4")])

_lib = None


def lib():
    """Load libchsim.so; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                           "(or python paper_1808_00128_amd/build.py)")
    L = C.CDLL(LIB_PATH)
    vp, u32, u64, dbl = C.c_void_p, C.c_uint32, C.c_uint64, C.c_double
    L.chsim_terms_init.argtypes = [C.POINTER(C.c_void_p), C.c_int, u32, C.POINTER(Instance)]
    L.chsim_terms_reset.argtypes = [vp, u32, u64, vp]
    L.chsim_apply_clifford.argtypes = [vp, u32, vp, C.c_size_t, vp]
    L.chsim_amplitudes.argtypes = [vp, u32, vp, C.c_size_t, vp, u32, vp]
    L.chsim_amplitudes_noalloc.argtypes = [vp, u32, vp, C.c_size_t, vp, u32, vp]
    L.chsim_inner_products.argtypes = [vp, u32, vp, vp, C.c_size_t, vp, vp, vp, u32, vp]
    L.chsim_inner_products_ch.argtypes = [vp, u32, u32, vp, vp, u32, vp]
    L.chsim_sparsification_bound.argtypes = [vp, u32, vp, vp, C.c_size_t, C.POINTER(C.c_double), vp]
    L.chsim_project_z.argtypes = [vp, u32, vp, vp, u32, vp]
    L.chsim_project_pauli.argtypes = [vp, u32, vp, vp, vp, u32, vp]
    L.chsim_terms_copy.argtypes = [vp, u32, u32, vp]
    L.chsim_sample_marginal.argtypes = [vp, u32, u32, vp, u32, vp, vp, C.c_size_t, vp, vp, vp, vp, vp]
    L.chsim_metropolis_init.argtypes = [vp, u32, u32, vp, vp, u32, vp]
    L.chsim_metropolis_step.argtypes = [vp, u32, u32, vp, vp, vp, vp, vp, u32, vp]
    L.chsim_sample_terms.argtypes = [vp, u32, C.c_size_t, vp, vp, vp]
    L.chsim_get_terms.argtypes = [vp, u32, u64, u64, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.chsim_set_terms.argtypes = [vp, u32, u64, u64, vp, vp, vp, vp, vp, vp, vp, vp]
    L.chsim_validate.argtypes = [vp, u32, u64, u64, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64),
                                 C.POINTER(C.c_uint32)]
    L.chsim_decompose_phase.argtypes = [dbl, u32, C.POINTER(C.c_double), C.POINTER(C.c_uint32),
                                        C.POINTER(Gate), C.POINTER(Decomp)]
    L.chsim_decompose_ccz.argtypes = [u32, u32, u32, C.POINTER(C.c_double), C.POINTER(C.c_uint32),
                                      C.POINTER(Gate), C.POINTER(Decomp)]
    L.chsim_set_tuning.argtypes = [vp, u32, u32, C.c_int32]
    L.chsim_get_tuning.argtypes = [vp, u32, u32, C.POINTER(C.c_int32), C.POINTER(C.c_float)]
    L.chsim_instance_info.argtypes = [vp, u32, C.POINTER(C.c_uint32), C.POINTER(C.c_uint64),
                                      C.POINTER(C.c_double)]
    L.chsim_destroy.argtypes = [vp]
    L.chsim_measure_peaks.argtypes = [C.c_int, C.POINTER(C.c_double)]
    L.chsim_mlp_create.argtypes = [vp, u32, u32, u32, vp, C.POINTER(C.c_void_p)]
    L.chsim_mlp_destroy.argtypes = [vp]
    L.chsim_mlp_get_params.argtypes = [vp, vp]
    L.chsim_mlp_set_params.argtypes = [vp, vp]
    L.chsim_mlp_forward.argtypes = [vp, vp, u32, vp, u32, vp]
    L.chsim_mlp_loss_grad.argtypes = [vp, vp, vp, u32, C.POINTER(C.c_double), vp, u32, vp]
    L.chsim_mlp_train.argtypes = [vp, vp, vp, u64, u32, u32, C.c_float, vp, u32, vp]
    L.chsim_metropolis_step_learned.argtypes = [vp, u32, vp, u32, C.POINTER(LearnedArgs), vp, vp,
                                                vp, vp, u32, vp]
    L.chsim_last_error.restype = C.c_char_p
    for name in EXPORTED:
        if name != "chsim_last_error":
            getattr(L, name).restype = C.c_int32
    _lib = L
    return L


def _check(status):
    if status != CHSIM_OK:
        raise ChsimError(status, lib().chsim_last_error().decode())


def _ptr(a):
    """Pointer and device flag of a numpy array or torch tensor."""
    if a is None:
        return None, 0
    if isinstance(a, np.ndarray):
        if not a.flags["C_CONTIGUOUS"]:
            raise ValueError("array must be C-contiguous")
        return a.ctypes.data_as(C.c_void_p), 0
    if hasattr(a, "data_ptr"):
        if not a.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return C.c_void_p(a.data_ptr()), (CHSIM_DEVICE_PTRS if a.is_cuda else 0)
    raise TypeError(type(a))


def _stream(stream):
    if stream is not None:
        return C.c_void_p(int(stream))
    try:
        import torch

        if torch.cuda.is_available() and torch.cuda.is_initialized():
            return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    except Exception:  # noqa: BLE001
        pass
    return None


def measure_peaks(device: int = 0) -> dict:
    """Microbenchmarked peaks of the device: int32 VALU ops/s, HBM copy
    bytes/s (read + write), LDS 8-byte-read bytes/s (chsim_measure_peaks)."""
    out = (C.c_double * 3)()
    st = lib().chsim_measure_peaks(int(device), out)
    if st != CHSIM_OK:
        raise ChsimError(st, "chsim_measure_peaks failed")
    return {"int32_valu_ops_per_s": out[0], "hbm_copy_bytes_per_s": out[1], "lds_read_bytes_per_s": out[2]}


def gate_array(circuit: W.Circuit) -> np.ndarray:
    """Circuit -> chsim_gate[]: SLOT and CCZ entries become CHSIM_SLOT gates,
    numbered together in circuit order."""
    g = np.zeros(circuit.n_gates, GATE_DTYPE)
    is_slot = (circuit.op == W.OP_SLOT) | (circuit.op == W.OP_CCZ)
    g["op"] = np.where(is_slot, W.OP_SLOT, circuit.op)
    g["q"] = circuit.q
    g["r"] = circuit.r
    slot = np.cumsum(is_slot) - 1
    g["slot"] = np.where(is_slot, slot, 0).astype(np.uint32)
    return g


class PhaseDecomposition:
    """chsim_decompose_phase output kept alive for the init call."""

    def __init__(self, theta: float, qubit: int):
        self.coeff = (C.c_double * 4)()
        self.off = (C.c_uint32 * 3)()
        self.gates = (Gate * 8)()
        self.decomp = Decomp()
        _check(lib().chsim_decompose_phase(float(theta), int(qubit), self.coeff, self.off, self.gates,
                                           C.byref(self.decomp)))

    @property
    def c(self):
        return complex(self.coeff[0], self.coeff[1]), complex(self.coeff[2], self.coeff[3])


class CCZDecomposition:
    """chsim_decompose_ccz output kept alive for the init call."""

    def __init__(self, a: int, b: int, c: int):
        self.coeff = (C.c_double * 16)()
        self.off = (C.c_uint32 * 9)()
        self.gates = (Gate * 24)()
        self.decomp = Decomp()
        _check(lib().chsim_decompose_ccz(int(a), int(b), int(c), self.coeff, self.off, self.gates,
                                         C.byref(self.decomp)))

    @property
    def c(self):
        return [complex(self.coeff[2 * j], self.coeff[2 * j + 1]) for j in range(8)]

    def branches(self):
        return [[(self.gates[k].op, self.gates[k].q, self.gates[k].r) for k in range(self.off[j], self.off[j + 1])]
                for j in range(8)]


def slot_decompositions(circ: W.Circuit) -> list:
    """One decomposition per slot of the circuit, in slot order."""
    decs = []
    third = circ.third()
    for o, q, r, t, in zip(circ.op.tolist(), circ.q.tolist(), circ.r.tolist(), third.tolist()):
        if o == W.OP_SLOT:
            decs.append(PhaseDecomposition(circ.theta[len(decs)], q))
        elif o == W.OP_CCZ:
            decs.append(CCZDecomposition(q, r, t))
    return decs


class Context:
    """A set of circuit instances and their chi CH-form terms on one GPU."""

    def __init__(self, specs, device: int = 0):
        """specs: list of dicts with keys circuit, chi, mode ('exact'|'sparsify'), seed."""
        L = lib()
        self._keep = []
        insts = (Instance * len(specs))()
        self.specs = specs
        for i, sp in enumerate(specs):
            circ = sp["circuit"]
            decs = slot_decompositions(circ)
            arr = (Decomp * max(1, len(decs)))()
            for k, d in enumerate(decs):
                arr[k] = d.decomp
            self._keep += [decs, arr]
            mode = CHSIM_EXACT if sp.get("mode", "sparsify") == "exact" else CHSIM_SPARSIFY
            insts[i] = Instance(circ.n, len(decs), arr, int(sp["chi"]), mode, int(sp.get("seed", 0)))
        h = C.c_void_p()
        _check(L.chsim_terms_init(C.byref(h), device, len(specs), insts))
        self._h = h
        self.device = device

    def close(self):
        if getattr(self, "_h", None):
            lib().chsim_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass

    def set_evolve_lanes(self, lanes, inst=0):
        """Lanes per term of the evolution kernel (4, 8, 16, 32, 64 with rows in
        registers; 4, 8, 16 | CHSIM_EVOLVE_LDS with rows in LDS; 0 = default;
        -1 = autotune at the next evolution from |0^n>)."""
        _check(lib().chsim_set_tuning(self._h, inst, CHSIM_TUNE_EVOLVE_LANES, int(lanes)))

    def set_prefix_share(self, mode, inst=0):
        """Shared-prefix evolution: 0 off, 1 auto (default), 2 whenever it saves work."""
        _check(lib().chsim_set_tuning(self._h, inst, CHSIM_TUNE_PREFIX_SHARE, int(mode)))

    def set_amp_strings(self, value):
        """Bitstrings per work item of the amplitude kernel (256 or 512; 0 =
        default; -1 = autotune at the next amplitude call), for the context."""
        _check(lib().chsim_set_tuning(self._h, 0, CHSIM_TUNE_AMP_STRINGS, int(value)))

    def amp_strings(self):
        """(bitstrings per work item in use, autotuner timings in ms for 256 and 512)."""
        v = C.c_int32()
        t = (C.c_float * 2)()
        _check(lib().chsim_get_tuning(self._h, 0, CHSIM_TUNE_AMP_STRINGS, C.byref(v), t))
        return v.value, list(t)

    def prefix_share(self, inst=0):
        """(mode, checkpoint levels of the last plan, estimated work fraction)."""
        v = C.c_int32()
        t = (C.c_float * 5)()
        _check(lib().chsim_get_tuning(self._h, inst, CHSIM_TUNE_PREFIX_SHARE, C.byref(v), t))
        return v.value, int(t[0]), float(t[1])

    def evolution_stats(self, inst=0, max_levels=64):
        """Gate applications of the last evolution by kind (H, CX, CZ, S-type,
        general-branch) and the distinct prefix counts per checkpoint level."""
        apps = (C.c_uint64 * 5)()
        lv = C.c_uint32()
        dist = (C.c_uint64 * max_levels)()
        _check(lib().chsim_evolution_stats(self._h, inst, apps, C.byref(lv), dist, max_levels))
        return dict(H=apps[0], CX=apps[1], CZ=apps[2], S=apps[3], cond=apps[4],
                    levels=lv.value, distinct=list(dist)[:min(lv.value, max_levels)])

    def evolve_lanes(self, inst=0):
        """(lanes value in use, autotuner timings in ms for each of TUNE_SHAPES)."""
        v = C.c_int32()
        t = (C.c_float * len(TUNE_SHAPES))()
        _check(lib().chsim_get_tuning(self._h, inst, CHSIM_TUNE_EVOLVE_LANES, C.byref(v), t))
        return v.value, list(t)

    def info(self, inst=0):
        n = C.c_uint32()
        chi = C.c_uint64()
        l1 = C.c_double()
        _check(lib().chsim_instance_info(self._h, inst, C.byref(n), C.byref(chi), C.byref(l1)))
        return n.value, chi.value, l1.value

    # ---- step (a) ----
    def reset(self, seed, inst=0, stream=None):
        """Re-draw the terms with a new seed and return them to |0^n> (no allocation)."""
        _check(lib().chsim_terms_reset(self._h, inst, int(seed), _stream(stream)))
        self.specs[inst] = dict(self.specs[inst], seed=int(seed))

    def apply_gates(self, gates: np.ndarray, inst=0, stream=None):
        gates = np.ascontiguousarray(gates, GATE_DTYPE)
        p, _ = _ptr(gates)
        _check(lib().chsim_apply_clifford(self._h, inst, p, gates.size, _stream(stream)))

    def apply_circuit(self, circuit: W.Circuit, inst=0, stream=None):
        self.apply_gates(gate_array(circuit), inst, stream)

    # ---- step (b) ----
    def amplitudes(self, x, inst=0, fp32c=False, out=None, stream=None):
        """<x_i|psi>.  numpy uint64 in -> numpy complex128 out; a CUDA int64
        tensor in -> a CUDA float64 tensor [n_x, 2] out (asynchronous)."""
        flags = CHSIM_FP32C if fp32c else CHSIM_FP64
        if isinstance(x, np.ndarray):
            x = np.ascontiguousarray(x, np.uint64)
            res = np.zeros(2 * x.size)
            px, _ = _ptr(x)
            po, _ = _ptr(res)
            _check(lib().chsim_amplitudes(self._h, inst, px, x.size, po, flags, _stream(stream)))
            return res[0::2] + 1j * res[1::2]
        import torch

        if out is None:
            out = torch.empty((x.numel(), 2), dtype=torch.float64, device=x.device)
        px, f1 = _ptr(x)
        po, f2 = _ptr(out)
        if not (f1 and f2):
            raise ValueError("torch inputs must be on the GPU")
        _check(lib().chsim_amplitudes(self._h, inst, px, x.numel(), po, flags | CHSIM_DEVICE_PTRS,
                                      _stream(stream)))
        return out

    def amplitudes_noalloc(self, x, out, inst=0, fp32c=False, stream=None):
        """chsim_amplitudes_noalloc: x a CUDA int64 tensor, out a CUDA float64
        tensor [n_x, 2] the caller allocated; the library allocates nothing."""
        flags = (CHSIM_FP32C if fp32c else CHSIM_FP64) | CHSIM_DEVICE_PTRS
        px, f1 = _ptr(x)
        po, f2 = _ptr(out)
        if not (f1 and f2):
            raise ValueError("chsim_amplitudes_noalloc takes device tensors")
        _check(lib().chsim_amplitudes_noalloc(self._h, inst, px, x.numel(), po, flags, _stream(stream)))
        return out

    def amplitudes_batch(self, requests, fp32c=False, stream=None):
        """Several (inst, x) requests in one launch.  All numpy uint64 -> list
        of numpy complex128; all CUDA int64 tensors -> list of CUDA float64
        tensors [n_x, 2] (asynchronous)."""
        flags = CHSIM_FP32C if fp32c else CHSIM_FP64
        reqs = (AmpRequest * len(requests))()
        keep, outs = [], []
        host = all(isinstance(x, np.ndarray) for _, x in requests)
        if not host:
            import torch
        for k, (inst, x) in enumerate(requests):
            if host:
                x = np.ascontiguousarray(x, np.uint64)
                o = np.zeros(2 * x.size)
                n_x = x.size
            else:
                o = torch.empty((x.numel(), 2), dtype=torch.float64, device=x.device)
                n_x = x.numel()
            px, f1 = _ptr(x)
            po, f2 = _ptr(o)
            if not host and not (f1 and f2):
                raise ValueError("torch inputs must be on the GPU")
            keep.append(x)
            outs.append(o)
            reqs[k] = AmpRequest(inst, 0, px.value, n_x, po.value)
        if not host:
            flags |= CHSIM_DEVICE_PTRS
        _check(lib().chsim_amplitudes_batch(self._h, reqs, len(requests), flags, _stream(stream)))
        if host:
            return [o[0::2] + 1j * o[1::2] for o in outs]
        return outs

    # ---- step (c) ----
    def inner_products(self, Aoff, Adiag, inst=0, stream=None):
        """(overlap complex[L], eta[L], eta_mean) for equatorial states A_l."""
        Aoff = np.ascontiguousarray(Aoff, np.uint64)
        Adiag = np.ascontiguousarray(Adiag, np.uint8)
        L = Aoff.shape[0]
        ov = np.zeros(2 * L)
        eta = np.zeros(L)
        mean = C.c_double()
        _check(lib().chsim_inner_products(self._h, inst, _ptr(Aoff)[0], _ptr(Adiag)[0], L,
                                          _ptr(ov)[0], _ptr(eta)[0], C.byref(mean), 0,
                                          _stream(stream)))
        return ov[0::2] + 1j * ov[1::2], eta, mean.value

    def inner_products_ch(self, bra_inst, inst=0, stream=None):
        """(overlap complex[chi_bra], total): overlap_l = <theta_l|psi_inst> with
        theta_l the CH form of term l of bra_inst; total = <psi_bra|psi_inst>."""
        chi_b = self.info(bra_inst)[1]
        ov = np.zeros(2 * chi_b)
        tot = np.zeros(2)
        _check(lib().chsim_inner_products_ch(self._h, inst, bra_inst, _ptr(ov)[0], _ptr(tot)[0], 0,
                                             _stream(stream)))
        return ov[0::2] + 1j * ov[1::2], complex(tot[0], tot[1])

    def project_z(self, qubits, bits, inst=0, stream=None):
        """Apply prod_j (I + (-1)^{bits_j} Z_{qubits_j}) / 2 to every term in place."""
        qs = np.ascontiguousarray(qubits, np.uint32)
        bs = np.ascontiguousarray(bits, np.uint8)
        _check(lib().chsim_project_z(self._h, inst, _ptr(qs)[0], _ptr(bs)[0], qs.size, _stream(stream)))

    def project_pauli(self, a, x, z, inst=0, stream=None):
        """Apply prod_j (I + i^{a_j} X(x_j) Z(z_j)) / 2 (Hermitian Paulis) to every term in place."""
        a = np.ascontiguousarray(a, np.uint8)
        x = np.ascontiguousarray(x, np.uint64)
        z = np.ascontiguousarray(z, np.uint64)
        _check(lib().chsim_project_pauli(self._h, inst, _ptr(a)[0], _ptr(x)[0], _ptr(z)[0], a.size,
                                         _stream(stream)))

    def copy_terms(self, src_inst, dst_inst, stream=None):
        _check(lib().chsim_terms_copy(self._h, src_inst, dst_inst, _stream(stream)))

    def sample_marginal(self, qubits, Aoff, Adiag, u, inst=0, scratch_inst=1, stream=None):
        """(bits, probability of each chosen bit, estimates [w, 2]) by the chain rule."""
        qs = np.ascontiguousarray(qubits, np.uint32)
        Aoff = np.ascontiguousarray(Aoff, np.uint64)
        Adiag = np.ascontiguousarray(Adiag, np.uint8)
        u = np.ascontiguousarray(u, np.float64)
        bits = np.zeros(qs.size, np.uint8)
        prob = np.zeros(qs.size)
        est = np.zeros(2 * qs.size)
        _check(lib().chsim_sample_marginal(self._h, inst, scratch_inst, _ptr(qs)[0], qs.size, _ptr(Aoff)[0],
                                           _ptr(Adiag)[0], Aoff.shape[0], _ptr(u)[0], _ptr(bits)[0],
                                           _ptr(prob)[0], _ptr(est)[0], _stream(stream)))
        return bits, prob, est.reshape(-1, 2)

    def sparsification_bound(self, Aoff, Adiag, inst=0, stream=None):
        """(<Omega|Omega> estimate, its standard error, delta^2, bound on
        ||psi - Omega||^2) from chsim_sparsification_bound."""
        Aoff = np.ascontiguousarray(Aoff, np.uint64)
        Adiag = np.ascontiguousarray(Adiag, np.uint8)
        out = (C.c_double * 4)()
        _check(lib().chsim_sparsification_bound(self._h, inst, _ptr(Aoff)[0], _ptr(Adiag)[0], Aoff.shape[0],
                                                out, _stream(stream)))
        return tuple(out)

    # ---- Metropolis ----
    def metropolis_init(self, x0, inst=0, stream=None):
        x0 = np.ascontiguousarray(x0, np.uint64)
        amp = np.zeros(2 * x0.size)
        _check(lib().chsim_metropolis_init(self._h, inst, x0.size, _ptr(x0)[0], _ptr(amp)[0], 0,
                                           _stream(stream)))
        self._n_chain = x0.size
        return amp[0::2] + 1j * amp[1::2]

    def metropolis_step(self, jstream, ustream, inst=0, trace=True, stream=None, graph=False):
        """Advance all chains; jstream/ustream are [n_chain, n_steps]; graph=True
        replays the steps from a cached HIP graph."""
        j = np.ascontiguousarray(jstream, np.uint32)
        u = np.ascontiguousarray(ustream, np.float64)
        n_chain, n_steps = j.shape
        tr = np.zeros((n_chain, n_steps), np.uint64) if trace else None
        acc = np.zeros((n_chain, n_steps), np.uint8) if trace else None
        amp = np.zeros(2 * n_chain)
        _check(lib().chsim_metropolis_step(self._h, inst, n_steps, _ptr(j)[0], _ptr(u)[0],
                                           _ptr(tr)[0], _ptr(acc)[0], _ptr(amp)[0],
                                           CHSIM_GRAPH if graph else 0, _stream(stream)))
        return tr, acc, amp[0::2] + 1j * amp[1::2]

    def metropolis_step_device(self, jstream, ustream, trace=None, accepted=None, amp=None,
                               inst=0, stream=None, graph=False):
        """Device-pointer variant: torch tensors on the GPU; enqueues only."""
        n_chain, n_steps = jstream.shape
        if jstream.element_size() != 4 or ustream.element_size() != 8:
            raise ValueError("jstream must be 32-bit integers and ustream float64")
        args = [_ptr(t)[0] for t in (jstream, ustream, trace, accepted, amp)]
        flags = CHSIM_DEVICE_PTRS | (CHSIM_GRAPH if graph else 0)
        _check(lib().chsim_metropolis_step(self._h, inst, n_steps, *args, flags, _stream(stream)))

    def sample_terms(self, alpha, flips, inst=0):
        alpha = np.ascontiguousarray(alpha, np.uint64)
        flips = np.ascontiguousarray(flips, np.uint64)
        out = np.zeros(alpha.size, np.uint64)
        _check(lib().chsim_sample_terms(self._h, inst, alpha.size, _ptr(alpha)[0], _ptr(flips)[0],
                                        _ptr(out)[0]))
        return out

    # ---- term store access ----
    def get_terms(self, first, count, inst=0):
        n, chi, _ = self.info(inst)
        m = self.specs[inst]["circuit"].n_slot
        F = np.zeros((count, n), np.uint64)
        G = np.zeros((count, n), np.uint64)
        M = np.zeros((count, n), np.uint64)
        g = np.zeros((count, n), np.uint8)
        v = np.zeros(count, np.uint64)
        s = np.zeros(count, np.uint64)
        w = np.zeros(count, np.uint8)
        b = np.zeros(2 * count)
        br = np.zeros((count, max(1, m)), np.uint8)
        _check(lib().chsim_get_terms(self._h, inst, first, count, *[_ptr(a)[0] for a in
                                                                  (F, G, M, g, v, s, w, b, br)]))
        return dict(F=F, G=G, M=M, gamma=g, v=v, s=s, omega=w, b=b[0::2] + 1j * b[1::2],
                    branch=br[:, :m])

    def set_terms(self, first, F, G, M, gamma, v, s, omega, b, inst=0):
        count = len(v)
        arrs = [np.ascontiguousarray(F, np.uint64), np.ascontiguousarray(G, np.uint64),
                np.ascontiguousarray(M, np.uint64), np.ascontiguousarray(gamma, np.uint8),
                np.ascontiguousarray(v, np.uint64), np.ascontiguousarray(s, np.uint64),
                np.ascontiguousarray(omega, np.uint8)]
        bb = np.zeros(2 * count)
        bb[0::2] = np.real(b)
        bb[1::2] = np.imag(b)
        _check(lib().chsim_set_terms(self._h, inst, first, count, *[_ptr(a)[0] for a in arrs],
                                     _ptr(bb)[0]))

    def validate(self, first=0, count=None, inst=0):
        """CH-form invariants of terms [first, first + count): (bad terms, first
        bad index or None, OR of the CHSIM_BAD_* flags).  Raises nothing for
        bad terms (the call's ESTATE is reported through the counts)."""
        if count is None:
            count = self.info(inst)[1] - first
        nb, fb, what = C.c_uint64(), C.c_uint64(), C.c_uint32()
        st = lib().chsim_validate(self._h, inst, first, count, C.byref(nb), C.byref(fb), C.byref(what))
        if st not in (CHSIM_OK, CHSIM_ESTATE):
            _check(st)
        return nb.value, (fb.value if nb.value else None), what.value

    def metropolis_step_learned(self, mlp, u_mix, j, u_bits, u, eps, pi_min, pi_max, inst=0,
                                stream=None):
        """Advance all chains with the learned proposal (host arrays)."""
        u_mix = np.ascontiguousarray(u_mix, np.float64)
        j = np.ascontiguousarray(j, np.uint32)
        u_bits = np.ascontiguousarray(u_bits, np.float64)
        u = np.ascontiguousarray(u, np.float64)
        n_chain, n_steps = j.shape
        keep = (u_mix, j, u_bits, u)
        a = LearnedArgs(eps, pi_min, pi_max, *[_ptr(t)[0] for t in keep])
        tr = np.zeros((n_chain, n_steps), np.uint64)
        acc = np.zeros((n_chain, n_steps), np.uint8)
        fl = np.zeros((n_chain, n_steps), np.uint32)
        amp = np.zeros(2 * n_chain)
        _check(lib().chsim_metropolis_step_learned(self._h, inst, mlp._h, n_steps, C.byref(a),
                                                   _ptr(tr)[0], _ptr(acc)[0], _ptr(fl)[0],
                                                   _ptr(amp)[0], 0, _stream(stream)))
        return tr, acc, fl, amp[0::2] + 1j * amp[1::2]

    def metropolis_step_learned_device(self, mlp, u_mix, j, u_bits, u, eps, pi_min, pi_max,
                                       trace=None, accepted=None, n_flips=None, inst=0,
                                       stream=None):
        """Device-pointer variant (torch tensors on the GPU); enqueues only."""
        n_chain, n_steps = j.shape
        keep = (u_mix, j, u_bits, u)
        a = LearnedArgs(eps, pi_min, pi_max, *[_ptr(t)[0] for t in keep])
        _check(lib().chsim_metropolis_step_learned(self._h, inst, mlp._h, n_steps, C.byref(a),
                                                   _ptr(trace)[0], _ptr(accepted)[0],
                                                   _ptr(n_flips)[0], None, CHSIM_DEVICE_PTRS,
                                                   _stream(stream)))


class MLP:
    """Proposal network n -> H -> H -> n on the context's GPU (BF16 MFMA)."""

    def __init__(self, ctx: Context, n: int, hidden: int, max_batch: int, params: dict):
        self.n, self.H, self.cap = n, hidden, max_batch
        self.ctx = ctx
        flat = pack_params(params)
        h = C.c_void_p()
        _check(lib().chsim_mlp_create(ctx._h, n, hidden, max_batch, _ptr(flat)[0], C.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().chsim_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass

    def params(self):
        flat = np.zeros(self._count(), np.float32)
        _check(lib().chsim_mlp_get_params(self._h, _ptr(flat)[0]))
        return unpack_params(flat, self.n, self.H)

    def set_params(self, params):
        flat = pack_params(params)
        _check(lib().chsim_mlp_set_params(self._h, _ptr(flat)[0]))

    def _count(self):
        n, H = self.n, self.H
        return H * n + H + H * H + H + n * H + n

    def forward(self, x):
        x = np.ascontiguousarray(x, np.uint64)
        out = np.zeros((x.size, self.n), np.float32)
        _check(lib().chsim_mlp_forward(self._h, _ptr(x)[0], x.size, _ptr(out)[0], 0, None))
        return out

    def loss_grad(self, x, target):
        x = np.ascontiguousarray(x, np.uint64)
        t = np.ascontiguousarray(target, np.uint64)
        g = np.zeros(self._count(), np.float32)
        loss = C.c_double()
        _check(lib().chsim_mlp_loss_grad(self._h, _ptr(x)[0], _ptr(t)[0], x.size, C.byref(loss),
                                         _ptr(g)[0], 0, None))
        return loss.value, unpack_params(g, self.n, self.H)

    def train(self, x, target, batch, epochs, lr):
        x = np.ascontiguousarray(x, np.uint64)
        t = np.ascontiguousarray(target, np.uint64)
        losses = np.zeros(epochs)
        _check(lib().chsim_mlp_train(self._h, _ptr(x)[0], _ptr(t)[0], x.size, batch, epochs,
                                     float(lr), _ptr(losses)[0], 0, None))
        return losses
