"""ctypes binding of libmpdo (include/mpdo.h).

Argument marshalling only: every step of the update runs in the HIP library.  PyTorch
supplies the device workspace (torch's caching allocator owns it) and the HIP stream.
The binding refuses to run when libmpdo.so is missing or no GPU is visible.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Iterable, Optional, Sequence

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libmpdo.so")

MPDO_FP64 = 0
MPDO_FP32 = 1
MPDO_BF16X3 = 2

STATUS = {0: "OK", 1: "E_ARG", 2: "E_STATE", 3: "E_NOMEM", 4: "E_DEVICE", 5: "E_NUMERIC",
          6: "E_UNSUPPORTED"}

EXPORTS = (
    "mpdo_create", "mpdo_destroy", "mpdo_workspace_bytes", "mpdo_bind_workspace",
    "mpdo_init_product_state", "mpdo_apply_gate", "mpdo_apply_gate_kraus", "mpdo_apply_gate_crosstalk",
    "mpdo_apply_channel", "mpdo_truncate", "mpdo_expect", "mpdo_expect2", "mpdo_trace", "mpdo_bond_dims",
    "mpdo_get_site", "mpdo_set_state", "mpdo_canonical_centre", "mpdo_move_centre", "mpdo_synchronize", "mpdo_last_error", "mpdo_version",
    "mpdo_profile_enable", "mpdo_profile_enable_mask", "mpdo_profile_stride", "mpdo_profile_read", "mpdo_batch_workspace_bytes", "mpdo_run_batch",
    "mpdo_cgemm", "mpdo_eigh",
)

PROF_FAMILIES = ("gemm", "eig_pair", "eig_rotate", "eig_small", "phys", "transfer", "other",
                 "tri_reduce", "tri_solve", "tri_back", "theta", "pchol", "split_sum")


class Config(C.Structure):
    _fields_ = [("n_sites", C.c_int), ("d", C.c_int), ("chi_max", C.c_int),
                ("precision", C.c_int), ("cutoff_rel", C.c_double), ("ppt", C.c_int),
                ("renorm_trace", C.c_int), ("hip_stream", C.c_void_p)]


class TruncInfo(C.Structure):
    _fields_ = [("bond", C.c_int), ("chi_l", C.c_int), ("chi_mid", C.c_int), ("chi_r", C.c_int),
                ("kept", C.c_int), ("path", C.c_int), ("eig_calls", C.c_int),
                ("ppt_feasible", C.c_int), ("trace_before", C.c_double),
                ("trace_after", C.c_double), ("xi_before", C.c_double),
                ("xi_after", C.c_double), ("ppt_theta", C.c_double),
                ("discarded_weight", C.c_double), ("max_abs_imag_t", C.c_double),
                ("sigma_max", C.c_double), ("sigma_min_kept", C.c_double),
                ("sigma_next", C.c_double), ("sigma_gap_at_cut", C.c_double),
                ("sigma_next_exact", C.c_int), ("retried", C.c_int)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class Circuit(C.Structure):
    _fields_ = [("n_sites", C.c_int), ("d", C.c_int), ("chi_max", C.c_int), ("precision", C.c_int),
                ("ppt", C.c_int), ("n_ops", C.c_int), ("op_kind", C.POINTER(C.c_int)),
                ("op_site", C.POINTER(C.c_int)), ("op_set", C.POINTER(C.c_int)),
                ("set_count", C.POINTER(C.c_int)), ("set_offset", C.POINTER(C.c_long)),
                ("kraus", C.POINTER(C.c_double)), ("rho0", C.POINTER(C.c_double)),
                ("n_terms", C.c_int), ("term_first", C.POINTER(C.c_int)),
                ("term_len", C.POINTER(C.c_int)), ("term_ops", C.POINTER(C.c_double)),
                ("out", C.POINTER(C.c_double)), ("out_trace", C.POINTER(C.c_double)),
                ("out_bonds", C.POINTER(C.c_int)), ("status", C.c_int), ("seconds", C.c_double)]


class MpdoError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"libmpdo {STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None


def library_path() -> str:
    return _LIB_PATH


def load_library() -> C.CDLL:
    """Load libmpdo.so (no GPU needed for loading).  Raises if it was not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(f"{_LIB_PATH} is missing: run paper_2309_08572_amd.build first")
    lib = C.CDLL(_LIB_PATH)
    dp = C.POINTER(C.c_double)
    ip = C.POINTER(C.c_int)
    ctx = C.c_void_p
    lib.mpdo_create.argtypes = [C.POINTER(Config), C.POINTER(ctx)]
    lib.mpdo_destroy.argtypes = [ctx]
    lib.mpdo_workspace_bytes.argtypes = [C.POINTER(Config)]
    lib.mpdo_workspace_bytes.restype = C.c_size_t
    lib.mpdo_bind_workspace.argtypes = [ctx, C.c_void_p, C.c_size_t]
    lib.mpdo_init_product_state.argtypes = [ctx, dp]
    lib.mpdo_apply_gate.argtypes = [ctx, C.c_int, dp, C.POINTER(TruncInfo)]
    lib.mpdo_apply_gate_kraus.argtypes = [ctx, C.c_int, C.c_int, dp, C.POINTER(TruncInfo)]
    lib.mpdo_apply_gate_crosstalk.argtypes = [ctx, C.c_int, C.c_int, dp, C.POINTER(TruncInfo)]
    lib.mpdo_apply_channel.argtypes = [ctx, C.c_int, C.c_int, dp]
    lib.mpdo_truncate.argtypes = [ctx, C.c_int, C.c_int, C.POINTER(TruncInfo)]
    lib.mpdo_expect.argtypes = [ctx, C.c_int, ip, ip, dp, C.c_int, dp]
    lib.mpdo_trace.argtypes = [ctx, dp]
    lib.mpdo_bond_dims.argtypes = [ctx, ip]
    lib.mpdo_get_site.argtypes = [ctx, C.c_int, dp, ip]
    lib.mpdo_set_state.argtypes = [ctx, ip, dp, C.c_int]
    lib.mpdo_canonical_centre.argtypes = [ctx, ip]
    lib.mpdo_move_centre.argtypes = [ctx, C.c_int]
    lib.mpdo_synchronize.argtypes = [ctx]
    lib.mpdo_last_error.argtypes = [ctx]
    lib.mpdo_last_error.restype = C.c_char_p
    lib.mpdo_version.restype = C.c_char_p
    lib.mpdo_profile_enable.argtypes = [ctx, C.c_int]
    lib.mpdo_profile_enable_mask.argtypes = [ctx, C.c_uint]
    lib.mpdo_profile_stride.argtypes = [ctx, C.c_int]
    lib.mpdo_batch_workspace_bytes.argtypes = [C.POINTER(Circuit), C.c_int]
    lib.mpdo_batch_workspace_bytes.restype = C.c_size_t
    lib.mpdo_run_batch.argtypes = [C.POINTER(Circuit), C.c_int, C.c_int, C.c_void_p, C.c_size_t]
    lib.mpdo_profile_read.argtypes = [ctx, dp, C.c_int]
    lib.mpdo_cgemm.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, dp, dp, C.c_int, dp, C.c_int, dp, dp, C.c_int]
    lib.mpdo_eigh.argtypes = [C.c_int, dp, C.c_double, C.c_int, ip, dp, dp]
    for name in EXPORTS:
        if name not in ("mpdo_workspace_bytes", "mpdo_last_error", "mpdo_version",
                        "mpdo_batch_workspace_bytes"):
            getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def _cplx(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.complex128))


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class MPDO:
    """One density-operator MPO on the GPU (a libmpdo context)."""

    def __init__(self, n_sites: int, d: int, chi_max: int, precision: int = MPDO_FP64,
                 cutoff_rel: float = 0.0, ppt: bool = True, renorm_trace: bool = False,
                 device: int = 0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("libmpdo needs a visible GPU; no CPU fallback exists")
        self._torch = torch
        self.lib = load_library()
        self.n, self.d, self.chi = n_sites, d, chi_max
        self.device = torch.device("cuda", device)
        stream = torch.cuda.current_stream(self.device)
        self.cfg = Config(n_sites, d, chi_max, precision, cutoff_rel, int(ppt), int(renorm_trace),
                          C.c_void_p(stream.cuda_stream))
        self.ctx = C.c_void_p()
        self._check(self.lib.mpdo_create(C.byref(self.cfg), C.byref(self.ctx)), None)
        nbytes = self.lib.mpdo_workspace_bytes(C.byref(self.cfg))
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self._check(self.lib.mpdo_bind_workspace(self.ctx, C.c_void_p(self.workspace.data_ptr()),
                                                 nbytes))

    # ------------------------------------------------------------ plumbing
    def _check(self, status: int, ctx="self"):
        if status != 0:
            c = self.ctx if ctx == "self" else None
            msg = self.lib.mpdo_last_error(c)
            raise MpdoError(status, msg.decode() if msg else "")

    def close(self):
        if getattr(self, "ctx", None) and self.ctx.value:
            self.lib.mpdo_destroy(self.ctx)
            self.ctx = C.c_void_p()
            self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ the C ABI
    def init_product_state(self, rhos: Sequence[np.ndarray]):
        arr = _cplx(np.stack([np.asarray(r) for r in rhos]))
        assert arr.shape == (self.n, self.d, self.d)
        self._check(self.lib.mpdo_init_product_state(self.ctx, _dptr(arr)))

    def apply_gate(self, site: int, superop: np.ndarray, info: bool = False):
        S = _cplx(superop)
        ti = TruncInfo()
        self._check(self.lib.mpdo_apply_gate(self.ctx, site, _dptr(S),
                                             C.byref(ti) if info else None))
        return ti.as_dict() if info else None

    def apply_gate_kraus(self, site: int, kraus: Iterable[np.ndarray], info: bool = False):
        K = _cplx(np.stack([np.asarray(k) for k in kraus]))
        ti = TruncInfo()
        self._check(self.lib.mpdo_apply_gate_kraus(self.ctx, site, K.shape[0], _dptr(K),
                                                   C.byref(ti) if info else None))
        return ti.as_dict() if info else None

    def apply_gate_crosstalk(self, site: int, rydberg: int, u4, info: bool = False):
        """Pair gate with nearest-neighbour Rydberg crosstalk: u4[a + 2b] is the pair unitary
        with the detunings shifted by the blockade when neighbour site-1 (a) / site+2 (b) is
        in the Rydberg level."""
        U = _cplx(np.stack([np.asarray(u) for u in u4]))
        if U.shape[0] != 4:
            raise ValueError("four pair unitaries expected")
        ti = TruncInfo()
        self._check(self.lib.mpdo_apply_gate_crosstalk(self.ctx, site, rydberg, _dptr(U),
                                                       C.byref(ti) if info else None))
        return ti.as_dict() if info else None

    def apply_channel(self, site: int, kraus: Iterable[np.ndarray]):
        K = _cplx(np.stack([np.asarray(k) for k in kraus]))
        self._check(self.lib.mpdo_apply_channel(self.ctx, site, K.shape[0], _dptr(K)))

    def truncate(self, bond: int, chi: int, info: bool = True):
        ti = TruncInfo()
        self._check(self.lib.mpdo_truncate(self.ctx, bond, chi, C.byref(ti) if info else None))
        return ti.as_dict() if info else None

    def expect(self, terms, normalize: bool = True) -> np.ndarray:
        """terms: list of (first_site, [O_first, O_first+1, ...])."""
        first = np.array([t[0] for t in terms], dtype=np.int32)
        lens = np.array([len(t[1]) for t in terms], dtype=np.int32)
        ops = _cplx(np.concatenate([np.stack([np.asarray(o) for o in t[1]]).reshape(-1)
                                    for t in terms])) if terms else np.zeros(2)
        out = np.zeros(2 * len(terms), dtype=np.float64)
        self._check(self.lib.mpdo_expect(self.ctx, len(terms),
                                         first.ctypes.data_as(C.POINTER(C.c_int)),
                                         lens.ctypes.data_as(C.POINTER(C.c_int)), _dptr(ops),
                                         int(normalize), _dptr(out)))
        return out[0::2] + 1j * out[1::2]

    def expect2(self, terms, normalize: bool = True) -> np.ndarray:
        """Second-order terms: list of (first_site, [M_first, M_first+1, ...]), each M a D2 x D2
        matrix on (eta, eta') of the two copies of vec(rho); other atoms are traced out."""
        first = np.array([t[0] for t in terms], dtype=np.int32)
        lens = np.array([len(t[1]) for t in terms], dtype=np.int32)
        ops = _cplx(np.concatenate([np.stack([np.asarray(o) for o in t[1]]).reshape(-1)
                                    for t in terms])) if terms else np.zeros(2)
        out = np.zeros(2 * len(terms), dtype=np.float64)
        self._check(self.lib.mpdo_expect2(self.ctx, len(terms),
                                          first.ctypes.data_as(C.POINTER(C.c_int)),
                                          lens.ctypes.data_as(C.POINTER(C.c_int)), _dptr(ops),
                                          int(normalize), _dptr(out)))
        return out[0::2] + 1j * out[1::2]

    def trace(self) -> complex:
        out = np.zeros(2)
        self._check(self.lib.mpdo_trace(self.ctx, _dptr(out)))
        return complex(out[0], out[1])

    def bond_dims(self):
        out = np.zeros(self.n - 1, dtype=np.int32)
        self._check(self.lib.mpdo_bond_dims(self.ctx, out.ctypes.data_as(C.POINTER(C.c_int))))
        return [int(x) for x in out]

    def get_site(self, j: int) -> np.ndarray:
        shape = np.zeros(3, dtype=np.int32)
        sp = shape.ctypes.data_as(C.POINTER(C.c_int))
        self._check(self.lib.mpdo_get_site(self.ctx, j, None, sp))
        out = np.zeros(int(np.prod(shape)), dtype=np.complex128)
        self._check(self.lib.mpdo_get_site(self.ctx, j, _dptr(out), sp))
        return out.reshape(tuple(int(x) for x in shape))

    def canonical_centre(self):
        """(atom holding the canonical centre, direction of the last sweep)."""
        out = np.zeros(2, dtype=np.int32)
        self._check(self.lib.mpdo_canonical_centre(self.ctx, out.ctypes.data_as(C.POINTER(C.c_int))))
        return int(out[0]), int(out[1])

    def move_centre(self, site: int):
        """Move the canonical centre to atom `site` (exact up to the rounding floor)."""
        self._check(self.lib.mpdo_move_centre(self.ctx, int(site)))

    def get_state(self):
        """(bond dimensions, list of site tensors, canonical centre) of the chain."""
        return self.bond_dims(), [self.get_site(j) for j in range(self.n)], self.canonical_centre()[0]

    def set_state(self, bonds, sites, centre: int = -1):
        """Load site tensors [chi_l][D2][chi_r]; centre >= 0 vouches for the mixed canonical
        form about that atom, -1 lets the library canonicalise."""
        b = np.ascontiguousarray(bonds, dtype=np.int32)
        data = _cplx(np.concatenate([np.asarray(a).reshape(-1) for a in sites]))
        self._check(self.lib.mpdo_set_state(self.ctx, b.ctypes.data_as(C.POINTER(C.c_int)), _dptr(data),
                                            int(centre)))

    def profile(self, enable: bool):
        self._check(self.lib.mpdo_profile_enable(self.ctx, int(enable)))

    def profile_families(self, names):
        """Record HIP events around the launches of the named families only (see
        PROF_FAMILIES); an empty list stops recording."""
        mask = 0
        for nm in names:
            mask |= 1 << PROF_FAMILIES.index(nm)
        self._check(self.lib.mpdo_profile_enable_mask(self.ctx, mask))

    def profile_stride(self, stride: int):
        """Stamp only every stride-th launch of the GEMM families while recording."""
        self._check(self.lib.mpdo_profile_stride(self.ctx, int(stride)))

    def profile_read(self) -> dict:
        nf = len(PROF_FAMILIES)
        out = np.zeros(4 * nf)
        self._check(self.lib.mpdo_profile_read(self.ctx, _dptr(out), nf))
        res = {}
        for f, name in enumerate(PROF_FAMILIES):
            res[name] = {"launches": int(out[4 * f]), "ms": float(out[4 * f + 1]),
                         "flops": float(out[4 * f + 2]), "bytes": float(out[4 * f + 3])}
        return res

    def synchronize(self):
        self._check(self.lib.mpdo_synchronize(self.ctx))


def cgemm(precision: int, A, B, op_a: int = 0, op_b: int = 0, alpha=1.0, beta=0.0, C0=None,
          split_k: bool = False, device: int = 0) -> np.ndarray:
    """alpha op(A) op(B) + beta C0 through the library's matrix-core product kernels
    (mpdo_cgemm); op 0: as stored, 1: transpose, 2: conjugate transpose."""
    import torch
    lib = load_library()
    torch.cuda.set_device(device)
    A, B = _cplx(A), _cplx(B)
    M = A.shape[0] if op_a == 0 else A.shape[1]
    K = A.shape[1] if op_a == 0 else A.shape[0]
    N = B.shape[1] if op_b == 0 else B.shape[0]
    if (B.shape[0] if op_b == 0 else B.shape[1]) != K:
        raise ValueError("inner dimensions differ")
    Cm = np.zeros((M, N), dtype=np.complex128) if C0 is None else _cplx(C0).copy()
    al = np.array([complex(alpha).real, complex(alpha).imag])
    be = np.array([complex(beta).real, complex(beta).imag])
    st = lib.mpdo_cgemm(int(precision), M, N, K, _dptr(al), _dptr(A), int(op_a), _dptr(B), int(op_b), _dptr(be),
                        _dptr(Cm), int(split_k))
    if st != 0:
        raise MpdoError(st, lib.mpdo_last_error(None).decode())
    return Cm


def eigh(H, tau: float = 0.0, cap: Optional[int] = None, device: int = 0):
    """The update's FP64 eigensolver on a host Hermitian matrix (mpdo_eigh): the eigenpairs
    above tau * lambda_max, at most cap, largest first -> (evals (m,), V (n, m))."""
    import torch
    lib = load_library()
    torch.cuda.set_device(device)
    H = _cplx(H)
    n = H.shape[0]
    if H.shape != (n, n):
        raise ValueError("H must be square")
    cap = n if cap is None else int(cap)
    m = np.zeros(1, dtype=np.int32)
    ev = np.zeros(max(cap, 1))
    V = np.zeros((n, max(cap, 1)), dtype=np.complex128)
    st = lib.mpdo_eigh(n, _dptr(H), float(tau), cap, m.ctypes.data_as(C.POINTER(C.c_int)), _dptr(ev), _dptr(V))
    if st != 0:
        raise MpdoError(st, lib.mpdo_last_error(None).decode())
    k = int(m[0])
    return ev[:k].copy(), V[:, :k].copy()


def run_batch(descs, n_workers: int = 8, device: int = 0):
    """Run circuit descriptions (dicts from circuits.describe) through mpdo_run_batch.

    Returns one dict per circuit: observables (complex array), trace, bonds, status,
    seconds.  The device workspace comes from torch."""
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("libmpdo needs a visible GPU; no CPU fallback exists")
    lib = load_library()
    n = len(descs)
    arr = (Circuit * n)()
    keep = []
    outs = []
    ip = C.POINTER(C.c_int)

    def iptr(a):
        a = np.ascontiguousarray(a, dtype=np.int32)
        keep.append(a)
        return a.ctypes.data_as(ip)

    for i, dsc in enumerate(descs):
        c = arr[i]
        c.n_sites, c.d, c.chi_max = dsc["n"], dsc["d"], dsc["chi"]
        c.precision, c.ppt = dsc.get("precision", MPDO_FP64), int(dsc.get("ppt", True))
        c.n_ops = len(dsc["op_kind"])
        c.op_kind, c.op_site, c.op_set = iptr(dsc["op_kind"]), iptr(dsc["op_site"]), iptr(dsc["op_set"])
        c.set_count = iptr(dsc["set_count"])
        off = np.ascontiguousarray(dsc["set_offset"], dtype=np.int64)
        keep.append(off)
        c.set_offset = off.ctypes.data_as(C.POINTER(C.c_long))
        kr = _cplx(dsc["kraus"])
        rho = _cplx(dsc["rho0"])
        tops = _cplx(dsc["term_ops"])
        keep.extend([kr, rho, tops])
        c.kraus, c.rho0, c.term_ops = _dptr(kr), _dptr(rho), _dptr(tops)
        c.n_terms = len(dsc["term_first"])
        c.term_first, c.term_len = iptr(dsc["term_first"]), iptr(dsc["term_len"])
        out = np.zeros(2 * c.n_terms)
        tr = np.zeros(2)
        bonds = np.zeros(dsc["n"] - 1, dtype=np.int32)
        keep.extend([out, tr, bonds])
        c.out, c.out_trace = _dptr(out), _dptr(tr)
        c.out_bonds = bonds.ctypes.data_as(ip)
        outs.append((out, tr, bonds))
    per = lib.mpdo_batch_workspace_bytes(arr, n)
    workers = max(1, min(n_workers, n))
    ws = torch.empty(per * workers, dtype=torch.uint8, device=torch.device("cuda", device))
    torch.cuda.synchronize()
    status = lib.mpdo_run_batch(arr, n, workers, C.c_void_p(ws.data_ptr()), per * workers)
    res = []
    for i in range(n):
        out, tr, bonds = outs[i]
        res.append({"values": out[0::2] + 1j * out[1::2], "trace": complex(tr[0], tr[1]),
                    "bonds": [int(b) for b in bonds], "status": int(arr[i].status),
                    "seconds": float(arr[i].seconds)})
    del ws
    if status != 0:
        bad = [i for i in range(n) if arr[i].status != 0]
        raise MpdoError(status, f"batch circuits failed: {bad[:8]}; first: {lib.mpdo_last_error(None).decode()}")
    return res
