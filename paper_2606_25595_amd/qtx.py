"""Python binding of libqtx_rgf.so (ctypes; argument marshalling only).

Every step of the solve runs in the library's HIP kernels; torch provides the
device memory (complex128 tensors) and the current HIP stream.  The names
mirror the C ABI in include/qtx_rgf.h:

  Context                  qtx_rgf_create / qtx_rgf_destroy
  Context.solve            qtx_rgf_solve
  Context.footprint        qtx_rgf_footprint
  Context.zgemm            qtx_zgemm (noalloc=True: qtx_zgemm_noalloc)
  Context.zinv             qtx_zinv
  Context.observables      qtx_rgf_observables

There is no fallback: if the shared library is missing this module raises.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqtx_rgf.so")

QTX_OK, QTX_ERR_ARG, QTX_ERR_NOMEM, QTX_ERR_HIP, QTX_ERR_UNSUPPORTED, QTX_ERR_SINGULAR, QTX_ERR_NONFINITE = range(7)
QTX_FP64, QTX_FP32, QTX_BF16_SPLIT, QTX_FP16_SPLIT, QTX_INT8_OZAKI2 = range(5)
QTX_S_IDENTITY = 1
QTX_SIGMA_DIAG = 2
QTX_WANT_GREATER = 8
QTX_SPLIT_CHAIN = 16
PREC_NAMES = {"fp64": QTX_FP64, "fp32": QTX_FP32, "bf16": QTX_BF16_SPLIT, "fp16": QTX_FP16_SPLIT,
              "int8": QTX_INT8_OZAKI2}

EXPORTED = ("qtx_rgf_create", "qtx_rgf_solve", "qtx_rgf_destroy", "qtx_rgf_footprint", "qtx_status_str",
            "qtx_zgemm", "qtx_zinv", "qtx_rgf_observables", "qtx_rgf_profile", "qtx_rgf_profile_read",
            "qtx_rgf_set_option", "qtx_rgf_get_stat", "qtx_ozaki2_bits", "qtx_rgf_tune", "qtx_w_assemble",
            "qtx_fpx_encode", "qtx_fpx_decode", "qtx_zgemm_noalloc", "qtx_rgf_bond_currents")
QTX_OPT_GRAPH, QTX_OPT_RESERVE_WORKSPACE, QTX_OPT_INT8_TILE_VARIANT, QTX_OPT_OVERLAP, QTX_OPT_LANE_SPLIT = 1, 2, 3, 4, 5
QTX_STAT_GRAPH_LAUNCHES, QTX_STAT_GRAPH_CAPTURES, QTX_STAT_WORKSPACE_BYTES, QTX_STAT_TUNE_RECORDS = 1, 2, 3, 4
QTX_KERNEL_GEMM, QTX_KERNEL_INV, QTX_KERNEL_CONVERT = 0, 1, 2


class QtxError(RuntimeError):
    def __init__(self, code, what=""):
        self.code = code
        super().__init__("%s failed: %s" % (what, status_str(code)))


class _Problem(ctypes.Structure):
    _fields_ = [
        ("n_b", ctypes.c_int32), ("b", ctypes.c_int32), ("n_e", ctypes.c_int32),
        ("prec", ctypes.c_int32), ("n_slices", ctypes.c_int32),
        ("prec_lesser", ctypes.c_int32), ("n_slices_lesser", ctypes.c_int32), ("flags", ctypes.c_uint32),
        ("energies", ctypes.POINTER(ctypes.c_double)),
        ("H_d", ctypes.c_void_p), ("H_u", ctypes.c_void_p), ("H_l", ctypes.c_void_p),
        ("S_d", ctypes.c_void_p), ("S_u", ctypes.c_void_p), ("S_l", ctypes.c_void_p),
        ("SR_d", ctypes.c_void_p), ("SR_u", ctypes.c_void_p), ("SR_l", ctypes.c_void_p),
        ("SL_d", ctypes.c_void_p), ("SL_u", ctypes.c_void_p), ("SL_l", ctypes.c_void_p),
        ("SG_d", ctypes.c_void_p), ("SG_u", ctypes.c_void_p), ("SG_l", ctypes.c_void_p),
        ("GR_d", ctypes.c_void_p), ("GR_u", ctypes.c_void_p), ("GR_l", ctypes.c_void_p),
        ("GL_d", ctypes.c_void_p), ("GL_u", ctypes.c_void_p),
        ("GG_d", ctypes.c_void_p), ("GG_u", ctypes.c_void_p),
        ("status", ctypes.c_void_p),
        ("out_bits", ctypes.c_int32),
        ("partitions", ctypes.c_int32),
    ]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("libqtx_rgf.so not found at %s: run __graft_entry__.build() "
                          "(or python -m paper_2606_25595_amd.build_lib) first" % path)
    lib = ctypes.CDLL(path)
    vp, i32, i64, dbl, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
    lib.qtx_rgf_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, sz, ctypes.c_char_p]
    lib.qtx_rgf_create.restype = ctypes.c_int
    lib.qtx_rgf_solve.argtypes = [vp, ctypes.POINTER(_Problem), i32, vp]
    lib.qtx_rgf_solve.restype = ctypes.c_int
    lib.qtx_rgf_destroy.argtypes = [vp]
    lib.qtx_rgf_destroy.restype = ctypes.c_int
    lib.qtx_rgf_footprint.argtypes = [ctypes.POINTER(_Problem)]
    lib.qtx_rgf_footprint.restype = sz
    lib.qtx_status_str.argtypes = [ctypes.c_int]
    lib.qtx_status_str.restype = ctypes.c_char_p
    lib.qtx_zgemm.argtypes = [vp, ctypes.c_char, ctypes.c_char, i32, i32, i32, dbl, dbl, vp, i64, i64, vp, i64, i64,
                              dbl, dbl, vp, i64, i64, i32, i32, i32, vp]
    lib.qtx_zgemm.restype = ctypes.c_int
    lib.qtx_zgemm_noalloc.argtypes = lib.qtx_zgemm.argtypes
    lib.qtx_zgemm_noalloc.restype = ctypes.c_int
    lib.qtx_zinv.argtypes = [vp, i32, vp, i64, vp, i64, i32, vp, vp]
    lib.qtx_zinv.restype = ctypes.c_int
    lib.qtx_rgf_observables.argtypes = [vp, i32, i32, vp, vp, i64, vp, vp, vp, vp, vp]
    lib.qtx_rgf_observables.restype = ctypes.c_int
    lib.qtx_rgf_bond_currents.argtypes = [vp, i32, i32, i32, vp, vp, vp, vp, i64, vp, vp]
    lib.qtx_rgf_bond_currents.restype = ctypes.c_int
    lib.qtx_rgf_profile.argtypes = [vp, ctypes.c_int]
    lib.qtx_rgf_profile.restype = ctypes.c_int
    lib.qtx_rgf_profile_read.argtypes = [vp, ctypes.c_int, ctypes.POINTER(dbl), ctypes.POINTER(i64),
                                         ctypes.POINTER(dbl)]
    lib.qtx_rgf_profile_read.restype = ctypes.c_int
    lib.qtx_rgf_set_option.argtypes = [vp, ctypes.c_int, i64]
    lib.qtx_rgf_set_option.restype = ctypes.c_int
    lib.qtx_rgf_get_stat.argtypes = [vp, ctypes.c_int, ctypes.POINTER(i64)]
    lib.qtx_rgf_get_stat.restype = ctypes.c_int
    lib.qtx_ozaki2_bits.argtypes = [i32, i32, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32)]
    lib.qtx_ozaki2_bits.restype = ctypes.c_int
    lib.qtx_rgf_tune.argtypes = [vp, i32, i32, i32, i32, vp, ctypes.POINTER(i32), ctypes.POINTER(dbl), i32,
                                 ctypes.POINTER(i32)]
    lib.qtx_rgf_tune.restype = ctypes.c_int
    lib.qtx_w_assemble.argtypes = [vp, i32, i32, i32, i32, i32] + [vp] * 16
    lib.qtx_w_assemble.restype = ctypes.c_int
    for name in ("qtx_fpx_encode", "qtx_fpx_decode"):
        getattr(lib, name).argtypes = [vp, i32, i64, vp, vp, vp]
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def status_str(code: int) -> str:
    return load_library().qtx_status_str(int(code)).decode()


def ozaki2_bits(p: int, K: int):
    """(moduli used, kbits) of the INT8 modular scheme asked for p moduli at
    contraction length K (host computation, no device)."""
    mods = (ctypes.c_int32 * max(p, 1))()
    pu, kb = ctypes.c_int32(0), ctypes.c_int32(0)
    rc = load_library().qtx_ozaki2_bits(int(p), int(K), mods, ctypes.byref(pu), ctypes.byref(kb))
    if rc != QTX_OK:
        raise QtxError(rc, "qtx_ozaki2_bits")
    return [int(m) for m in mods[:pu.value]], int(kb.value)


def _ptr(t):
    """Device pointer of a torch tensor (or None)."""
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


@dataclasses.dataclass
class DeviceProblem:
    """Device tensors of one problem (inputs and caller-allocated outputs)."""
    energies: np.ndarray
    H_d: object
    H_u: object
    H_l: object
    SR_d: object
    SL_d: object
    GR_d: object
    GR_u: object
    GR_l: object
    GL_d: object
    GL_u: object
    status: object
    S_d: object = None
    S_u: object = None
    S_l: object = None
    SR_u: object = None
    SR_l: object = None
    SL_u: object = None
    SG_d: object = None
    SG_u: object = None
    GG_d: object = None
    GG_u: object = None
    split: bool = False     # QTX_SPLIT_CHAIN: two half-chains per energy
    sigma_diag: bool = False   # QTX_SIGMA_DIAG: SR_d / SL_d / SG_d are [n_e, n_b, b] diagonals
    out_bits: int = 64      # 64: complex128 outputs; 16..56: GR_u/GR_l/GL_u/GG_u as FPX bytes
    partitions: int = 0     # P >= 2: P-way partitioned solve of every energy

    @property
    def n_b(self):
        return int(self.H_d.shape[0])

    @property
    def b(self):
        return int(self.H_d.shape[1])

    @property
    def n_e(self):
        return int(self.energies.shape[0])

    def outputs(self):
        """Host copies of the outputs, keyed like the oracle's results (FPX outputs as
        their bytes, [n_e, n_b - 1, b * b * out_bits / 4] uint8)."""
        out = {k: getattr(self, k).cpu().numpy() for k in ("GR_d", "GR_u", "GR_l", "GL_d", "GL_u")}
        if self.GG_d is not None:
            out["GG_d"] = self.GG_d.cpu().numpy()
            out["GG_u"] = self.GG_u.cpu().numpy()
        out["status"] = self.status.cpu().numpy()
        return out


def to_device(p, device="cuda", greater: Optional[bool] = None, sigma_diag: bool = False,
              out_bits: int = 64) -> DeviceProblem:
    """Copy a host problem (paper_2606_25595_amd.inputs.BTProblem) to the device
    and allocate its outputs (uninitialised).  A BT Sigma^< / Sigma^> travels as its
    upper blocks only (SL_u / SG_u): the library takes the lower blocks as
    -(upper)^H, so SL_l / SG_l are not copied.  sigma_diag: the diagonal self-energy
    blocks travel as their diagonals (they must be diagonal matrices).  out_bits < 64:
    the off-diagonal outputs are FPX byte buffers of that width."""
    import torch

    def dev(a):
        if a is None:
            return None
        return torch.from_numpy(np.require(a, dtype=np.complex128, requirements=["C", "W"])).to(device)

    def sdiag(a):
        if a is None or not sigma_diag:
            return dev(a)
        d = np.diagonal(a, axis1=-2, axis2=-1)
        off = ~np.eye(a.shape[-1], dtype=bool)
        if np.any(a[..., off] != 0):
            raise ValueError("sigma_diag: a diagonal self-energy block has off-diagonal entries")
        return dev(d)

    n_e, n_b, b = p.n_e, p.n_b, p.b
    if greater is None:
        greater = p.SG_d is not None
    out_bits = 64 if out_bits in (0, 64) else int(out_bits)
    kw = dict(dtype=torch.complex128, device=device)

    def offdiag():
        if out_bits == 64:
            return torch.empty((n_e, max(n_b - 1, 0), b, b), **kw)
        return torch.empty((n_e, max(n_b - 1, 0), b * b * out_bits // 4), dtype=torch.uint8, device=device)
    dp = DeviceProblem(
        energies=np.ascontiguousarray(p.energies, dtype=np.float64),
        H_d=dev(p.H_d), H_u=dev(p.H_u), H_l=dev(p.H_l), SR_d=sdiag(p.SR_d), SL_d=sdiag(p.SL_d),
        GR_d=torch.empty((n_e, n_b, b, b), **kw), GR_u=offdiag(), GR_l=offdiag(),
        GL_d=torch.empty((n_e, n_b, b, b), **kw), GL_u=offdiag(),
        status=torch.full((n_e,), -1, dtype=torch.int32, device=device),
        S_d=dev(p.S_d), S_u=dev(p.S_u), S_l=dev(p.S_l), SR_u=dev(p.SR_u), SR_l=dev(p.SR_l),
        SL_u=dev(p.SL_u), sigma_diag=bool(sigma_diag), out_bits=out_bits)
    if greater:
        dp.SG_d = sdiag(p.SG_d)
        dp.SG_u = dev(p.SG_u)
        dp.GG_d = torch.empty((n_e, n_b, b, b), **kw)
        dp.GG_u = offdiag()
    return dp


@dataclasses.dataclass
class DeviceW:
    """Device tensors of a screened Coulomb (W) system (paper_2606_25595_amd.inputs.WProblem)."""
    n_e: int
    V_d: object
    V_u: object
    PR_d: object
    PR_u: object
    PR_l: object
    PL_d: object
    PL_u: object
    PG_d: object = None
    PG_u: object = None

    @property
    def n_b(self):
        return int(self.V_d.shape[0])

    @property
    def b(self):
        return int(self.V_d.shape[1])


def w_to_device(w, device="cuda", greater: Optional[bool] = None) -> DeviceW:
    """Copy a WProblem to the device.  P^<> travel as diagonal and upper blocks
    (the library takes the lower blocks as -(upper)^H)."""
    import torch

    def dev(a):
        if a is None:
            return None
        return torch.from_numpy(np.require(a, dtype=np.complex128, requirements=["C", "W"])).to(device)
    if greater is None:
        greater = w.PG_d is not None
    return DeviceW(n_e=w.n_e, V_d=dev(w.V_d), V_u=dev(w.V_u), PR_d=dev(w.PR_d), PR_u=dev(w.PR_u),
                   PR_l=dev(w.PR_l), PL_d=dev(w.PL_d), PL_u=dev(w.PL_u),
                   PG_d=dev(w.PG_d) if greater else None, PG_u=dev(w.PG_u) if greater else None)


def _problem_struct(dp: DeviceProblem, prec: int, n_slices: int, prec_lesser: int = -1, n_slices_lesser: int = -1):
    st = _Problem()
    st.n_b, st.b, st.n_e = dp.n_b, dp.b, dp.n_e
    st.prec, st.n_slices = int(prec), int(n_slices)
    st.prec_lesser, st.n_slices_lesser = int(prec_lesser), int(n_slices_lesser)
    flags = 0
    if dp.S_d is None:
        flags |= QTX_S_IDENTITY
    if dp.GG_d is not None:
        flags |= QTX_WANT_GREATER
    if dp.split:
        flags |= QTX_SPLIT_CHAIN
    if dp.sigma_diag:
        flags |= QTX_SIGMA_DIAG
    st.flags = flags
    st.out_bits = int(dp.out_bits)
    st.partitions = int(dp.partitions)
    en = np.ascontiguousarray(dp.energies, dtype=np.float64)
    st.energies = en.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    for name in ("H_d", "H_u", "H_l", "S_d", "S_u", "S_l", "SR_d", "SR_u", "SR_l", "SL_d", "SL_u", "SG_d", "SG_u",
                 "GR_d", "GR_u", "GR_l", "GL_d", "GL_u", "GG_d", "GG_u", "status"):
        t = getattr(dp, name)
        if t is not None and t.numel() == 0:
            t = None
        setattr(st, name, _ptr(t))
    return st, en


class Context:
    """One library context on one device (qtx_rgf_create)."""

    def __init__(self, device: int = 0, workspace_bytes: int = 0, tune_cache: Optional[str] = None):
        self.lib = load_library()
        h = ctypes.c_void_p()
        rc = self.lib.qtx_rgf_create(ctypes.byref(h), int(device), int(workspace_bytes),
                                     tune_cache.encode() if tune_cache else None)
        if rc != QTX_OK:
            raise QtxError(rc, "qtx_rgf_create")
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            self.lib.qtx_rgf_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- FPX storage codec
    def fpx_encode(self, x, bits: int, out=None, stream=None):
        """qtx_fpx_encode of a float64 / complex128 device tensor; returns the uint8 codes."""
        import torch
        xd = torch.view_as_real(x) if x.is_complex() else x
        assert xd.dtype == torch.float64 and xd.is_contiguous()
        n = xd.numel()
        if out is None:
            out = torch.empty(n * bits // 8, dtype=torch.uint8, device=x.device)
        rc = self.lib.qtx_fpx_encode(self.handle, int(bits), n, _ptr(xd) if n else None, _ptr(out) if n else None,
                                     _stream_ptr(stream))
        if rc != QTX_OK:
            raise QtxError(rc, "qtx_fpx_encode")
        return out

    def fpx_decode(self, data, bits: int, n: int, out=None, stream=None):
        """qtx_fpx_decode of n values from a uint8 device tensor; returns float64."""
        import torch
        if out is None:
            out = torch.empty(n, dtype=torch.float64, device=data.device)
        rc = self.lib.qtx_fpx_decode(self.handle, int(bits), int(n), _ptr(data) if n else None,
                                     _ptr(out) if n else None, _stream_ptr(stream))
        if rc != QTX_OK:
            raise QtxError(rc, "qtx_fpx_decode")
        return out

    # -- screened Coulomb system
    def w_assemble(self, dw: DeviceW, prec="fp64", n_slices=0, stream=None, check: bool = True):
        """qtx_w_assemble: BT blocks of V P^R and V P^<> V^H (dict of device tensors
        VPR_d/u/l, BL_d/u, and BG_d/u when P^> is given)."""
        import torch
        n_e, n_b, b = dw.n_e, dw.n_b, dw.b
        kw = dict(dtype=torch.complex128, device=dw.V_d.device)
        nu = max(n_b - 1, 0)
        out = {"VPR_d": torch.empty((n_e, n_b, b, b), **kw), "VPR_u": torch.empty((n_e, nu, b, b), **kw),
               "VPR_l": torch.empty((n_e, nu, b, b), **kw), "BL_d": torch.empty((n_e, n_b, b, b), **kw),
               "BL_u": torch.empty((n_e, nu, b, b), **kw)}
        if dw.PG_d is not None:
            out["BG_d"] = torch.empty((n_e, n_b, b, b), **kw)
            out["BG_u"] = torch.empty((n_e, nu, b, b), **kw)
        p = lambda t: _ptr(t if (t is not None and t.numel()) else None)
        rc = self.lib.qtx_w_assemble(self.handle, n_b, b, n_e, PREC_NAMES.get(prec, prec), int(n_slices),
                                     p(dw.V_d), p(dw.V_u), p(dw.PR_d), p(dw.PR_u), p(dw.PR_l), p(dw.PL_d),
                                     p(dw.PL_u), p(dw.PG_d), p(dw.PG_u), p(out["VPR_d"]), p(out["VPR_u"]),
                                     p(out["VPR_l"]), p(out["BL_d"]), p(out["BL_u"]), p(out.get("BG_d")),
                                     p(out.get("BG_u")), _stream_ptr(stream))
        if check and rc != QTX_OK:
            raise QtxError(rc, "qtx_w_assemble")
        return out if check else rc

    def w_problem(self, dw: DeviceW, asm) -> DeviceProblem:
        """The W system as a DeviceProblem for qtx_rgf_solve: energies 1, S = I,
        H = 0, Sigma^R = BT(V P^R), Sigma^<> = BT(V P^<> V^H); outputs allocated."""
        import torch
        n_e, n_b, b = dw.n_e, dw.n_b, dw.b
        kw = dict(dtype=torch.complex128, device=dw.V_d.device)
        nu = max(n_b - 1, 0)
        z = torch.zeros((n_b, b, b), **kw)
        zu = torch.zeros((nu, b, b), **kw)
        dp = DeviceProblem(
            energies=np.ones(n_e), H_d=z, H_u=zu, H_l=zu, SR_d=asm["VPR_d"], SL_d=asm["BL_d"],
            GR_d=torch.empty((n_e, n_b, b, b), **kw), GR_u=torch.empty((n_e, nu, b, b), **kw),
            GR_l=torch.empty((n_e, nu, b, b), **kw), GL_d=torch.empty((n_e, n_b, b, b), **kw),
            GL_u=torch.empty((n_e, nu, b, b), **kw),
            status=torch.full((n_e,), -1, dtype=torch.int32, device=dw.V_d.device),
            SR_u=asm["VPR_u"], SR_l=asm["VPR_l"], SL_u=asm["BL_u"])
        if "BG_d" in asm:
            dp.SG_d, dp.SG_u = asm["BG_d"], asm["BG_u"]
            dp.GG_d = torch.empty((n_e, n_b, b, b), **kw)
            dp.GG_u = torch.empty((n_e, nu, b, b), **kw)
        return dp

    def w_solve(self, dw: DeviceW, prec="fp64", n_slices=0, stream=None, **kw) -> DeviceProblem:
        """Assemble the W system (qtx_w_assemble, FP64 products) and solve it
        (qtx_rgf_solve with the given schemes); returns the solved DeviceProblem."""
        asm = self.w_assemble(dw, stream=stream)
        dp = self.w_problem(dw, asm)
        self.solve(dp, prec=prec, n_slices=n_slices, stream=stream, **kw)
        return dp

    # -- qtx_rgf_solve
    def solve(self, problems, prec="fp64", n_slices=0, stream=None, check: bool = True,
              prec_lesser=None, n_slices_lesser=-1) -> int:
        """prec / n_slices: scheme of the retarded-chain products; prec_lesser /
        n_slices_lesser: scheme of the lesser-chain products (None = same).  Each
        may be one value for all problems or a list with one per problem."""
        if isinstance(problems, DeviceProblem):
            problems = [problems]
        n = len(problems)

        def per(x):
            return list(x) if isinstance(x, (list, tuple)) else [x] * n
        precs, nss, pls, nsls = per(prec), per(n_slices), per(prec_lesser), per(n_slices_lesser)
        arr = (_Problem * n)()
        keep = []
        for k, dp in enumerate(problems):
            pl = -1 if pls[k] is None else PREC_NAMES.get(pls[k], pls[k])
            st, en = _problem_struct(dp, PREC_NAMES.get(precs[k], precs[k]), nss[k], pl, nsls[k])
            arr[k] = st
            keep.append(en)
        rc = self.lib.qtx_rgf_solve(self.handle, arr, len(problems), _stream_ptr(stream))
        if check and rc != QTX_OK:
            raise QtxError(rc, "qtx_rgf_solve")
        return rc

    def footprint(self, dp: DeviceProblem, prec="fp64") -> int:
        st, _ = _problem_struct(dp, PREC_NAMES.get(prec, prec), 0)
        return int(self.lib.qtx_rgf_footprint(ctypes.byref(st)))

    # -- qtx_zgemm:  C = alpha op(A) op(B) + beta C  over a batch
    def zgemm(self, A, B, C, opA="N", opB="N", alpha=1.0, beta=0.0, prec="fp64", n_slices=0, stream=None,
              check=True, noalloc=False):
        """A, B, C: complex128 tensors [batch][rows][cols] (or 2-D, batch 1).
        noalloc: call qtx_zgemm_noalloc (fixed per-GPU scratch, no allocation)."""
        def as3(t):
            return t if t.dim() == 3 else t.unsqueeze(0)
        A3, B3, C3 = as3(A), as3(B), as3(C)
        batch = C3.shape[0]
        M, N = C3.shape[1], C3.shape[2]
        K = A3.shape[2] if opA == "N" else A3.shape[1]
        sA = A3.shape[1] * A3.shape[2] if A3.shape[0] > 1 else 0
        sB = B3.shape[1] * B3.shape[2] if B3.shape[0] > 1 else 0
        alpha, beta = complex(alpha), complex(beta)
        fn = self.lib.qtx_zgemm_noalloc if noalloc else self.lib.qtx_zgemm
        rc = fn(self.handle, opA.encode(), opB.encode(), M, N, K, alpha.real, alpha.imag,
                _ptr(A3), A3.shape[2], sA, _ptr(B3), B3.shape[2], sB, beta.real, beta.imag,
                _ptr(C3), C3.shape[2], M * N, batch, PREC_NAMES.get(prec, prec), n_slices,
                _stream_ptr(stream))
        if check and rc != QTX_OK:
            raise QtxError(rc, "qtx_zgemm_noalloc" if noalloc else "qtx_zgemm")
        return rc

    # -- qtx_zinv
    def zinv(self, A, Ainv, status=None, stream=None, check=True):
        A3 = A if A.dim() == 3 else A.unsqueeze(0)
        O3 = Ainv if Ainv.dim() == 3 else Ainv.unsqueeze(0)
        n = A3.shape[1]
        rc = self.lib.qtx_zinv(self.handle, n, _ptr(A3), n * n, _ptr(O3), n * n, A3.shape[0], _ptr(status),
                               _stream_ptr(stream))
        if check and rc != QTX_OK:
            raise QtxError(rc, "qtx_zinv")
        return rc

    # -- qtx_rgf_profile / qtx_rgf_profile_read
    def profile(self, enable: bool = True):
        rc = self.lib.qtx_rgf_profile(self.handle, 1 if enable else 0)
        if rc != QTX_OK:
            raise QtxError(rc, "qtx_rgf_profile")

    def profile_read(self, family: int = QTX_KERNEL_GEMM):
        """(total_ms, launches, flops) of the family's launches since the last read."""
        ms, n, fl = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double()
        rc = self.lib.qtx_rgf_profile_read(self.handle, int(family), ctypes.byref(ms), ctypes.byref(n),
                                           ctypes.byref(fl))
        if rc != QTX_OK:
            raise QtxError(rc, "qtx_rgf_profile_read")
        return ms.value, n.value, fl.value

    # -- qtx_rgf_set_option / qtx_rgf_get_stat
    def set_graph(self, enable: bool = True):
        rc = self.lib.qtx_rgf_set_option(self.handle, QTX_OPT_GRAPH, 1 if enable else 0)
        if rc != QTX_OK:
            raise QtxError(rc, "qtx_rgf_set_option")

    def reserve_workspace(self, nbytes: int):
        rc = self.lib.qtx_rgf_set_option(self.handle, QTX_OPT_RESERVE_WORKSPACE, int(nbytes))
        if rc != QTX_OK:
            raise QtxError(rc, "qtx_rgf_set_option(reserve)")

    def set_overlap(self, enable: bool = True):
        """Run the products independent of each forward inversion on a side stream."""
        rc = self.lib.qtx_rgf_set_option(self.handle, QTX_OPT_OVERLAP, 1 if enable else 0)
        if rc != QTX_OK:
            raise QtxError(rc, "qtx_rgf_set_option(overlap)")

    def set_lane_split(self, parts: int = 1):
        """QTX_OPT_LANE_SPLIT: run each batch group as `parts` batches on parallel streams."""
        rc = self.lib.qtx_rgf_set_option(self.handle, QTX_OPT_LANE_SPLIT, int(parts))
        if rc != QTX_OK:
            raise QtxError(rc, "qtx_rgf_set_option(LANE_SPLIT)")

    def set_int8_tile_variant(self, variant: int = -1):
        """-1: the autotuner's choice per shape; 0.. : force one tile variant."""
        rc = self.lib.qtx_rgf_set_option(self.handle, QTX_OPT_INT8_TILE_VARIANT, int(variant))
        if rc != QTX_OK:
            raise QtxError(rc, "qtx_rgf_set_option(int8 tile variant)")

    # -- qtx_rgf_tune
    def tune(self, b: int, prec="int8", n_slices: int = 0, batch: int = 1, stream=None):
        """Time the product kernel's tile variants for b x b x b products over
        `batch` entries; returns (chosen variant, [ms per product of each variant])."""
        v = ctypes.c_int32()
        cnt = ctypes.c_int32()
        ms = (ctypes.c_double * 16)()
        rc = self.lib.qtx_rgf_tune(self.handle, int(b), PREC_NAMES.get(prec, prec), int(n_slices), int(batch),
                                   _stream_ptr(stream), ctypes.byref(v), ms, 16, ctypes.byref(cnt))
        if rc != QTX_OK:
            raise QtxError(rc, "qtx_rgf_tune")
        return v.value, [ms[i] for i in range(cnt.value)]

    def stat(self, which: int) -> int:
        v = ctypes.c_int64()
        rc = self.lib.qtx_rgf_get_stat(self.handle, int(which), ctypes.byref(v))
        if rc != QTX_OK:
            raise QtxError(rc, "qtx_rgf_get_stat")
        return v.value

    # -- qtx_rgf_observables
    def observables(self, dp: DeviceProblem, gamma_L, f_L, stream=None):
        """(T_L, j_L) per energy as device float64 tensors."""
        return self.observables_blocks(dp.GR_d, dp.GL_d, gamma_L, f_L, stream=stream)

    def observables_right(self, dp: DeviceProblem, gamma_R, f_R, stream=None):
        """(T_R, j_R) per energy: the observables of the last block (the right contact,
        broadening gamma_R, occupation f_R), from the same kernel as the left ones."""
        import torch
        n_e, n_b, b = dp.n_e, dp.n_b, dp.b
        T = torch.empty(n_e, dtype=torch.float64, device=dp.GR_d.device)
        j = torch.empty_like(T)
        fR = torch.as_tensor(np.ascontiguousarray(f_R, dtype=np.float64)).to(dp.GR_d.device)
        g = torch.as_tensor(np.ascontiguousarray(gamma_R, dtype=np.complex128)).to(dp.GR_d.device)
        if not (dp.GR_d.is_contiguous() and dp.GL_d.is_contiguous()):
            raise ValueError("GR_d / GL_d must be contiguous")
        off = (n_b - 1) * b * b * 16                      # bytes to block n_b - 1 of energy 0
        gr = ctypes.c_void_p(dp.GR_d.data_ptr() + off)
        gl = ctypes.c_void_p(dp.GL_d.data_ptr() + off)
        rc = self.lib.qtx_rgf_observables(self.handle, b, n_e, gr, gl, n_b * b * b, _ptr(g), _ptr(fR), _ptr(T),
                                          _ptr(j), _stream_ptr(stream))
        if rc != QTX_OK:
            raise QtxError(rc, "qtx_rgf_observables")
        return T, j

    def bond_currents(self, dp: DeviceProblem, stream=None):
        """J[e][i] = 2 Re Tr[(H_{i,i+1} - E S_{i,i+1}) G^<_{i+1,i}] per energy and bond,
        a device float64 tensor [n_e][n_b - 1] (qtx_rgf_bond_currents)."""
        import torch
        n_e, n_b, b = dp.n_e, dp.n_b, dp.b
        J = torch.empty((n_e, max(n_b - 1, 0)), dtype=torch.float64, device=dp.GR_d.device)
        if n_b < 2:
            return J
        E = torch.as_tensor(np.ascontiguousarray(dp.energies, dtype=np.float64)).to(dp.GR_d.device)
        rc = self.lib.qtx_rgf_bond_currents(self.handle, b, n_b, n_e, _ptr(dp.H_u), _ptr(dp.S_u), _ptr(E),
                                            _ptr(dp.GL_u), (n_b - 1) * b * b, _ptr(J), _stream_ptr(stream))
        if rc != QTX_OK:
            raise QtxError(rc, "qtx_rgf_bond_currents")
        return J

    def observables_blocks(self, GR_d, GL_d, gamma_L, f_L, stream=None):
        """(T_L, j_L) per energy from [n_e][n_b][b][b] G^R / G^< diagonal-block tensors
        (contiguous; only block 0 of each energy is read)."""
        import torch
        if not (GR_d.is_contiguous() and GL_d.is_contiguous()) or GR_d.shape != GL_d.shape or GR_d.dim() != 4:
            raise ValueError("GR_d / GL_d: contiguous [n_e][n_b][b][b] tensors of one shape")
        n_e, n_b, b = int(GR_d.shape[0]), int(GR_d.shape[1]), int(GR_d.shape[2])
        T = torch.empty(n_e, dtype=torch.float64, device=GR_d.device)
        j = torch.empty_like(T)
        fL = torch.as_tensor(np.ascontiguousarray(f_L, dtype=np.float64)).to(GR_d.device)
        g = torch.as_tensor(np.ascontiguousarray(gamma_L, dtype=np.complex128)).to(GR_d.device)
        rc = self.lib.qtx_rgf_observables(self.handle, b, n_e, _ptr(GR_d), _ptr(GL_d), n_b * b * b, _ptr(g),
                                          _ptr(fL), _ptr(T), _ptr(j), _stream_ptr(stream))
        if rc != QTX_OK:
            raise QtxError(rc, "qtx_rgf_observables")
        return T, j
