"""Python binding of libgpqmc.so (the C ABI in include/gpqmc.h).

Argument marshalling only: every step of the sweep runs in the HIP library.
PyTorch supplies the device workspace and the stream.  The binding refuses to
run without the built library (there is no fallback path).
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libgpqmc.so")

OK, EINVAL, ENOMEM, EHIP, EDEGENERATE, EUNSTABLE, ESTATE = 0, -1, -2, -3, -4, -5, -6
FP64, MIXED, MIXED_FP32_BASIS, FP64_WRAP = 0, 1, 2, 3
MODEL_HUBBARD, MODEL_TV = 0, 1
_STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "EDEGENERATE",
           -5: "EUNSTABLE", -6: "ESTATE"}


class ChainDesc(ctypes.Structure):
    _fields_ = [
        ("n_sites", ctypes.c_int32), ("n_up", ctypes.c_int32), ("n_dn", ctypes.c_int32),
        ("hopping", ctypes.POINTER(ctypes.c_double)),
        ("sublattice", ctypes.POINTER(ctypes.c_int8)),
        ("trial_potential", ctypes.POINTER(ctypes.c_double)),
        ("U", ctypes.c_double), ("dtau", ctypes.c_double), ("g", ctypes.c_double),
        ("m_neel", ctypes.c_double),
        ("l_half", ctypes.c_int32), ("stab_interval", ctypes.c_int32),
        ("delay_rank", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("seed", ctypes.c_uint64), ("chain_id", ctypes.c_uint64), ("trace", ctypes.c_int32),
        ("model", ctypes.c_int32), ("V", ctypes.c_double), ("n_bonds", ctypes.c_int32),
        ("bonds", ctypes.POINTER(ctypes.c_int32)),
    ]


class Options(ctypes.Structure):
    _fields_ = [("meas_capacity", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("drift_tol", ctypes.c_double), ("particle_hole", ctypes.c_int32)]


class ChainInfo(ctypes.Structure):
    _fields_ = [("sign", ctypes.c_int32), ("flags", ctypes.c_int32), ("n_meas", ctypes.c_int32),
                ("sign_mismatch", ctypes.c_int32), ("sweep", ctypes.c_int32),
                ("max_drift", ctypes.c_float), ("last_drift", ctypes.c_float),
                ("accepted", ctypes.c_int64), ("proposed", ctypes.c_int64),
                ("max_rel_drift", ctypes.c_float), ("last_rel_drift", ctypes.c_float),
                ("particle_hole", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class GpqmcError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None
EXPORTS = [
    "gpqmc_create", "gpqmc_workspace_bytes", "gpqmc_bind_workspace", "gpqmc_init_trial",
    "gpqmc_sweep", "gpqmc_measure_energy", "gpqmc_measure_double_occupancy",
    "gpqmc_measure_sign", "gpqmc_measure_structure_factor", "gpqmc_get_measurements",
    "gpqmc_reset_measurements",
    "gpqmc_set_field", "gpqmc_get_field", "gpqmc_get_green", "gpqmc_get_chain_info",
    "gpqmc_set_debug", "gpqmc_get_trace", "gpqmc_get_trace_logdet", "gpqmc_logdet",
    "gpqmc_debug_gemm", "gpqmc_gemm_noalloc", "gpqmc_chain_status",
    "gpqmc_time_kernel", "gpqmc_set_kernel_timing", "gpqmc_get_kernel_timing",
    "gpqmc_debug_step", "gpqmc_debug_read", "gpqmc_last_error", "gpqmc_destroy",
]


def load():
    """Load libgpqmc.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2303_13403_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64, D, VP = ctypes.POINTER, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
    sig = {
        "gpqmc_create": [I32, P(ChainDesc), P(Options), VP, P(VP)],
        "gpqmc_workspace_bytes": [VP, P(ctypes.c_size_t)],
        "gpqmc_bind_workspace": [VP, VP, ctypes.c_size_t],
        "gpqmc_init_trial": [VP],
        "gpqmc_sweep": [VP, I32, I32],
        "gpqmc_measure_energy": [VP, I32, P(D), P(D)],
        "gpqmc_measure_double_occupancy": [VP, I32, P(D), P(D)],
        "gpqmc_measure_sign": [VP, I32, P(D), P(D)],
        "gpqmc_measure_structure_factor": [VP, I32, P(D), P(D)],
        "gpqmc_get_measurements": [VP, I32, P(D), I32, P(I32)],
        "gpqmc_reset_measurements": [VP],
        "gpqmc_set_field": [VP, I32, P(ctypes.c_int8)],
        "gpqmc_get_field": [VP, I32, P(ctypes.c_int8)],
        "gpqmc_get_green": [VP, I32, I32, P(D)],
        "gpqmc_get_chain_info": [VP, I32, P(ChainInfo)],
        "gpqmc_set_debug": [VP, I32],
        "gpqmc_get_trace": [VP, I32, P(D), P(D), P(D), P(I32)],
        "gpqmc_get_trace_logdet": [VP, I32, P(D)],
        "gpqmc_logdet": [VP, I32, P(D), P(I32)],
        "gpqmc_debug_gemm": [I32, I32, I32, I32, I32, VP, I32, VP, I32, VP, I32, VP],
        "gpqmc_gemm_noalloc": [I32, I32, I32, I32, I32, VP, I32, VP, I32, VP, I32, VP],
        "gpqmc_chain_status": [VP, I32],
        "gpqmc_time_kernel": [VP, I32, I32, P(ctypes.c_float)],
        "gpqmc_set_kernel_timing": [VP, I32],
        "gpqmc_get_kernel_timing": [VP, I32, P(ctypes.c_float), P(ctypes.c_int32)],
        "gpqmc_debug_step": [VP, I32, I32, I32, I32],
        "gpqmc_debug_read": [VP, I32, I32, I32, P(D), I64],
        "gpqmc_last_error": [VP],
        "gpqmc_destroy": [VP],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int32
    lib.gpqmc_last_error.restype = ctypes.c_char_p
    lib.gpqmc_destroy.restype = None
    _lib = lib
    return lib


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def chain_desc_arrays(w, chain_id: int, precision: int, trace: bool = False, seed=None):
    """Host arrays of one chain described by a workloads.Workload (Hubbard) or
    workloads.TVWorkload (spinless t-V)."""
    if hasattr(w, "V"):
        K, eps, bonds = w.lattice()
        return dict(K=np.ascontiguousarray(K, np.float64), eps=np.ascontiguousarray(eps, np.int8),
                    pot=None, n_up=w.n_particles, n_dn=0, U=0.0, dtau=w.dtau, g=w.g,
                    m_neel=w.delta_c, l_half=w.l_half, n_s=w.stab_interval, k=w.delay_rank,
                    precision=precision, seed=w.seed if seed is None else seed,
                    chain_id=chain_id, trace=trace, model=MODEL_TV, V=w.V,
                    bonds=np.ascontiguousarray(bonds, np.int32))
    K, eps, _ = w.lattice()
    pot = w.trial_potential()
    return dict(K=np.ascontiguousarray(K, np.float64), eps=np.ascontiguousarray(eps, np.int8),
                pot=None if pot is None else np.ascontiguousarray(pot, np.float64),
                n_up=w.n_up, n_dn=w.n_dn, U=w.U, dtau=w.dtau, g=w.g, m_neel=w.m_neel,
                l_half=w.l_half, n_s=w.stab_interval, k=w.delay_rank, precision=precision,
                seed=w.seed if seed is None else seed, chain_id=chain_id, trace=trace)


class Context:
    """A batch of Markov chains on one GPU.

    ``chains``: list of dicts from :func:`chain_desc_arrays`.  Device memory is
    a torch uint8 tensor owned by this object; work runs on ``self.stream``.
    """

    def __init__(self, chains: Sequence[dict], device: str = "cuda:0", meas_capacity: int = 4096,
                 use_graph: bool = True, drift_tol: float = 0.0, stream=None,
                 workspace_fill: Optional[float] = None, particle_hole: bool = False):
        import torch

        self.lib = load()
        self.torch = torch
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        self._keep = []
        descs = (ChainDesc * len(chains))()
        for i, c in enumerate(chains):
            d = descs[i]
            K = np.ascontiguousarray(c["K"], np.float64)
            eps = np.ascontiguousarray(c["eps"], np.int8)
            self._keep += [K, eps]
            d.n_sites = K.shape[0]
            d.n_up, d.n_dn = c["n_up"], c["n_dn"]
            d.hopping = _dptr(K)
            d.sublattice = eps.ctypes.data_as(ctypes.POINTER(ctypes.c_int8))
            if c.get("pot") is not None:
                pot = np.ascontiguousarray(c["pot"], np.float64)
                self._keep.append(pot)
                d.trial_potential = _dptr(pot)
            d.U, d.dtau, d.g, d.m_neel = c["U"], c["dtau"], c["g"], c["m_neel"]
            d.l_half, d.stab_interval, d.delay_rank = c["l_half"], c["n_s"], c["k"]
            d.precision = c["precision"]
            d.seed, d.chain_id = int(c["seed"]), int(c["chain_id"])
            d.trace = 1 if c.get("trace") else 0
            d.model = c.get("model", MODEL_HUBBARD)
            if d.model == MODEL_TV:
                bonds = np.ascontiguousarray(c["bonds"], np.int32)
                self._keep.append(bonds)
                d.V = c["V"]
                d.n_bonds = len(bonds)
                d.bonds = bonds.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        self.n_chains = len(chains)
        # HS fields per slice: sites, or bonds (t-V)
        self.nprop = [len(c["bonds"]) if c.get("model", MODEL_HUBBARD) == MODEL_TV
                      else np.asarray(c["K"]).shape[0] for c in chains]
        self.sizes = [(descs[i].n_sites, descs[i].n_up, descs[i].n_dn) for i in range(len(chains))]
        self.l_half = descs[0].l_half
        self.n_slices = 2 * self.l_half + 2
        opts = Options(meas_capacity, 1 if use_graph else 0, drift_tol, 1 if particle_hole else 0)
        ctx = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            st = self.lib.gpqmc_create(len(chains), descs, ctypes.byref(opts),
                                       ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(ctx))
        if st != OK:
            msg = self.lib.gpqmc_last_error(ctx).decode() if ctx.value else ""
            if ctx.value:
                self.lib.gpqmc_destroy(ctx)
            raise GpqmcError(st, msg)
        self.ctx = ctx
        nbytes = ctypes.c_size_t()
        self._check(self.lib.gpqmc_workspace_bytes(self.ctx, ctypes.byref(nbytes)))
        self.workspace_bytes = nbytes.value
        self.workspace = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
        if workspace_fill is not None:
            # testing: start from a known memory content (e.g. NaN) so that a
            # read of memory the library never wrote shows up in the results
            n8 = nbytes.value // 8
            self.workspace[: n8 * 8].view(torch.float64).fill_(workspace_fill)
            self.workspace[n8 * 8:].fill_(0)
        with torch.cuda.device(self.device):
            self._check(self.lib.gpqmc_bind_workspace(self.ctx,
                                                      ctypes.c_void_p(self.workspace.data_ptr()),
                                                      nbytes.value))

    def _check(self, st):
        if st != OK:
            raise GpqmcError(st, self.lib.gpqmc_last_error(self.ctx).decode())

    def _call(self, name, *args):
        with self.torch.cuda.device(self.device):
            self._check(getattr(self.lib, name)(self.ctx, *args))

    # -- hot path ---------------------------------------------------------------
    def init_trial(self):
        self._call("gpqmc_init_trial")
        return self

    def sweep(self, n: int = 1, measure: bool = True):
        self._call("gpqmc_sweep", n, 1 if measure else 0)
        return self

    def synchronize(self):
        self.stream.synchronize()

    # -- measurements -------------------------------------------------------------
    def _measure(self, name, chain):
        m, e = ctypes.c_double(), ctypes.c_double()
        self._call(name, chain, ctypes.byref(m), ctypes.byref(e))
        return m.value, e.value

    def measure_energy(self, chain: int = -1):
        return self._measure("gpqmc_measure_energy", chain)

    def measure_double_occupancy(self, chain: int = -1):
        return self._measure("gpqmc_measure_double_occupancy", chain)

    def measure_sign(self, chain: int = -1):
        return self._measure("gpqmc_measure_sign", chain)

    def measure_structure_factor(self, chain: int = -1):
        """S_AFM = (1/N^2) sum_ij eps_i eps_j <S_i . S_j> (sign-weighted)."""
        return self._measure("gpqmc_measure_structure_factor", chain)

    def measurements(self, chain: int, capacity: int = 1 << 16) -> np.ndarray:
        buf = np.zeros((capacity, 4), np.float64)       # sign, E/N, D, S_AFM
        n = ctypes.c_int32()
        self._call("gpqmc_get_measurements", chain, _dptr(buf), capacity, ctypes.byref(n))
        return buf[: n.value].copy()

    def reset_measurements(self):
        self._call("gpqmc_reset_measurements")

    # -- state and testing hooks ----------------------------------------------------
    def set_field(self, chain: int, field):
        f = np.ascontiguousarray(np.asarray(field, np.int8).reshape(self.n_slices,
                                                                     self.nprop[chain]))
        self._call("gpqmc_set_field", chain, f.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)))

    def get_field(self, chain: int) -> np.ndarray:
        f = np.zeros((self.n_slices, self.nprop[chain]), np.int8)
        self._call("gpqmc_get_field", chain, f.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)))
        return f

    def get_green(self, chain: int, spin: int) -> np.ndarray:
        N = self.sizes[chain][0]
        G = np.zeros((N, N), np.float64)
        self._call("gpqmc_get_green", chain, spin, _dptr(G))
        return G

    def chain_info(self, chain: int) -> dict:
        info = ChainInfo()
        self._call("gpqmc_get_chain_info", chain, ctypes.byref(info))
        return {k: getattr(info, k) for k, _ in ChainInfo._fields_}

    def logdet(self, chain: int):
        """((log|W_up|, log|W_dn|), (sgn W_up, sgn W_dn)) at the last checkpoint."""
        la = np.zeros(2, np.float64)
        sg = np.zeros(2, np.int32)
        self._call("gpqmc_logdet", chain, _dptr(la), sg.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
        return la, sg

    def trace_logdet(self, chain: int) -> np.ndarray:
        """(n_ck, 2, 2): (log|W_sigma|, sgn W_sigma) of both spins at every
        checkpoint of the last pass (chains created with trace)."""
        nck = ctypes.c_int32()
        self._call("gpqmc_get_trace", chain, None, None, None, ctypes.byref(nck))
        out = np.zeros((nck.value, 2, 2), np.float64)
        self._call("gpqmc_get_trace_logdet", chain, _dptr(out))
        return out

    def status(self, chain: int) -> int:
        with self.torch.cuda.device(self.device):
            return self.lib.gpqmc_chain_status(self.ctx, chain)

    def set_debug(self, force_reject: bool):
        self._call("gpqmc_set_debug", 1 if force_reject else 0)

    def trace(self, chain: int):
        """(ratios (M+2, P, 2), greens (n_ck, 2, N, N), drifts (n_ck,)) of the last
        pass; P = N sites (Hubbard: r_up, r_dn) or the bonds (t-V: r, 0)."""
        N = self.sizes[chain][0]
        nck = ctypes.c_int32()
        self._call("gpqmc_get_trace", chain, None, None, None, ctypes.byref(nck))
        r = np.zeros((self.n_slices, self.nprop[chain], 2), np.float64)
        g = np.zeros((nck.value, 2, N, N), np.float64)
        d = np.zeros(nck.value, np.float64)
        self._call("gpqmc_get_trace", chain, _dptr(r), _dptr(g), _dptr(d), ctypes.byref(nck))
        return r, g, d

    def time_kernel(self, kernel: int = 0, reps: int = 20) -> float:
        """Average ms per launch of the wrap GEMM (0) or propagation GEMM (1)."""
        ms = ctypes.c_float()
        self._call("gpqmc_time_kernel", kernel, reps, ctypes.byref(ms))
        return ms.value

    def set_kernel_timing(self, mask: int):
        """Record HIP events around every launch, in later sweeps, of the timed
        kernels in ``mask``: bit 0 the wrap GEMM, bit 1 the B-scaled
        propagation GEMM, bit 2 the slice's delayed update (passes then launch
        directly); clears what was recorded."""
        self._call("gpqmc_set_kernel_timing", mask)

    def kernel_timing(self, kernel: int):
        """(total ms, launches) of timed kernel ``kernel`` since the last
        :meth:`set_kernel_timing`."""
        ms, n = ctypes.c_float(), ctypes.c_int32()
        self._call("gpqmc_get_kernel_timing", kernel, ctypes.byref(ms), ctypes.byref(n))
        return ms.value, n.value

    def debug_step(self, stage: int, l: int, s0: int = 0, s1: int = 0):
        self._call("gpqmc_debug_step", stage, l, s0, s1)

    def debug_read(self, chain: int, what: int, spin: int, count: int) -> np.ndarray:
        out = np.zeros(count, np.float64)
        self._call("gpqmc_debug_read", chain, what, spin, _dptr(out), count)
        return out

    def close(self):
        if getattr(self, "ctx", None) is not None and self.ctx.value:
            self.stream.synchronize()
            self.lib.gpqmc_destroy(self.ctx)
            self.ctx = None
            self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def gemm_noalloc(A, B, C, trans_a: bool = False, precision: int = FP64, stream=None,
                 large_tile: bool = False):
    """C = op(A) B through gpqmc_gemm_noalloc into the caller's C (torch device
    tensors, contiguous, in the precision's dtype); enqueued on ``stream``."""
    import torch

    lib = load()
    M = A.shape[1] if trans_a else A.shape[0]
    K = A.shape[0] if trans_a else A.shape[1]
    N = B.shape[1]
    assert C.shape == (M, N) and C.is_contiguous() and A.is_contiguous() and B.is_contiguous()
    s = stream if stream is not None else torch.cuda.current_stream(A.device)
    st = lib.gpqmc_gemm_noalloc(precision, M, N, K, (1 if trans_a else 0) | (2 if large_tile else 0),
                                ctypes.c_void_p(A.data_ptr()), A.shape[1],
                                ctypes.c_void_p(B.data_ptr()), B.shape[1],
                                ctypes.c_void_p(C.data_ptr()), N, ctypes.c_void_p(s.cuda_stream))
    if st != OK:
        raise GpqmcError(st, "gemm_noalloc")
    return C


def debug_gemm(A, B, trans_a: bool = False, precision: int = FP64, stream=None,
               large_tile: bool = False):
    """C = op(A) B with one of the library's MFMA tile kernels (torch device
    tensors); large_tile selects the 128 x 128 kernel of the wrap, the slice
    update and the FP64 basis propagation (FP32 or FP64 by ``precision``)."""
    import torch

    lib = load()
    dt = torch.float64 if precision == FP64 else torch.float32
    A = A.to(dt).contiguous()
    B = B.to(dt).contiguous()
    M = A.shape[1] if trans_a else A.shape[0]
    K = A.shape[0] if trans_a else A.shape[1]
    N = B.shape[1]
    C = torch.empty((M, N), dtype=dt, device=A.device)
    s = stream if stream is not None else torch.cuda.current_stream(A.device)
    st = lib.gpqmc_debug_gemm(precision, M, N, K, (1 if trans_a else 0) | (2 if large_tile else 0),
                              ctypes.c_void_p(A.data_ptr()), A.shape[1],
                              ctypes.c_void_p(B.data_ptr()), B.shape[1],
                              ctypes.c_void_p(C.data_ptr()), N, ctypes.c_void_p(s.cuda_stream))
    if st != OK:
        raise GpqmcError(st, "debug_gemm")
    return C
