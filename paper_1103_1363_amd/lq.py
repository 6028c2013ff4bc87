"""Python binding of liblq.so (include/lq.h): argument marshalling only.

Device fields are torch uint8 CUDA tensors of lq_field_bytes() bytes; every
step of the operator and the solvers runs in the HIP library.  Importing
this module fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as ct
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# LQ_LIBRARY selects another build of the same library (tuning experiments)
LIB_PATH = os.environ.get("LQ_LIBRARY") or os.path.join(_HERE, "liblq.so")

F64, F32, F16 = 0, 1, 2
F16X = 3  # multi-RHS interleaved FP16 fields (one parity, up to 16 right-hand sides)
EVEN, ODD, FULL = 0, 1, 2
CGNR, BICGSTAB, FGMRES_NET, FCG_NET = 0, 1, 2, 3
PREC = {"f64": F64, "f32": F32, "f16": F16}

STATUS = {0: "LQ_OK", -1: "LQ_EINVAL", -2: "LQ_ENOMEM", -3: "LQ_EHIP", -4: "LQ_ENOCONV",
          -5: "LQ_ESTATE", -6: "LQ_ENAN"}


class LQError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class SolverParams(ct.Structure):
    _fields_ = [("solver", ct.c_int), ("inner_prec", ct.c_int), ("maxiter", ct.c_int),
                ("delta", ct.c_double), ("restart", ct.c_int), ("check_every", ct.c_int),
                ("use_graph", ct.c_int), ("fault_inject", ct.c_int), ("profile", ct.c_int),
                ("batched", ct.c_int), ("deflate", ct.c_int), ("dev_xref", ct.c_void_p)]


class SolveReport(ct.Structure):
    _fields_ = [("iterations", ct.c_int), ("reliable_updates", ct.c_int),
                ("fallback", ct.c_int), ("dslash_calls", ct.c_int),
                ("true_residual", ct.c_double), ("schur_residual", ct.c_double),
                ("seconds", ct.c_double), ("bytes", ct.c_double),
                ("kernel_ms", ct.c_double * 5), ("kernel_bytes", ct.c_double * 5),
                ("kernel_calls", ct.c_int * 5), ("ref_error", ct.c_double)]

    def as_dict(self):
        d = {}
        for k, _ in self._fields_:
            v = getattr(self, k)
            d[k] = list(v) if hasattr(v, "__len__") else v
        return d


class SapParams(ct.Structure):
    _fields_ = [("block", ct.c_int * 4), ("ncycles", ct.c_int), ("nmr", ct.c_int),
                ("restart", ct.c_int), ("maxiter", ct.c_int), ("deflate", ct.c_int),
                ("block_fp16", ct.c_int), ("block_eo", ct.c_int)]


class EnsembleReport(ct.Structure):
    _fields_ = [("tile_sites", ct.c_int), ("tile_from_cache", ct.c_int),
                ("tune_ms", ct.c_double * 3), ("graph_captures", ct.c_int),
                ("replays", ct.c_int), ("iterations", ct.c_int), ("seconds", ct.c_double),
                ("bytes", ct.c_double)]

    def as_dict(self):
        d = {}
        for k, _ in self._fields_:
            v = getattr(self, k)
            d[k] = list(v) if hasattr(v, "__len__") else v
        return d


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_1103_1363_amd.build` (no CPU fallback exists)")
        # torch ships its own HIP runtime; load it first so that liblq.so binds
        # to the same runtime instance (two HIP runtimes in one process do not
        # share devices, streams or allocations)
        import torch  # noqa: F401
        L = ct.CDLL(LIB_PATH)
        vp, dp, ip = ct.c_void_p, ct.POINTER(ct.c_double), ct.c_int
        L.lq_create.argtypes = [ct.POINTER(ct.c_int), ip, vp, ct.POINTER(vp)]
        L.lq_create.restype = ip
        L.lq_destroy.argtypes = [vp]
        L.lq_destroy.restype = None
        L.lq_last_error.argtypes = [vp]
        L.lq_last_error.restype = ct.c_char_p
        L.lq_field_bytes.argtypes = [vp, ip, ip, ip]
        L.lq_field_bytes.restype = ct.c_size_t
        L.lq_volume.argtypes = [vp]
        L.lq_volume.restype = ct.c_int64
        L.lq_upload_gauge.argtypes = [vp, dp]
        L.lq_set_clover.argtypes = [vp, ct.c_double, ct.c_double]
        L.lq_spinor_to_device.argtypes = [vp, vp, dp, ip, ip, ip]
        L.lq_spinor_to_host.argtypes = [vp, dp, vp, ip, ip, ip]
        L.lq_dslash.argtypes = [vp, vp, vp, ip, ip, ip, ip]
        L.lq_clover_apply.argtypes = [vp, vp, vp, ip, ip, ip, ip]
        L.lq_schur.argtypes = [vp, vp, vp, vp, ip, ip, ip]
        L.lq_schur_noalloc.argtypes = [vp, vp, vp, ip, ip, ip]
        L.lq_stream_copy.argtypes = [vp, vp, ct.c_size_t, vp]
        L.lq_stream_copy.restype = ip
        L.lq_site_array_bytes.argtypes = [ct.c_int64, ip, ip]
        L.lq_site_array_bytes.restype = ct.c_size_t
        L.lq_site_array_to_device.argtypes = [vp, dp, ct.c_int64, ip, ip, vp]
        L.lq_site_array_to_host.argtypes = [dp, vp, ct.c_int64, ip, ip, vp]
        L.lq_su3_mul.argtypes = [vp, vp, vp, vp, ct.c_int64, ip, ip, vp]
        L.lq_su3_spinor_mul.argtypes = [vp, vp, vp, ct.c_int64, ip, ip, vp]
        for name in ("lq_site_array_to_device", "lq_site_array_to_host", "lq_su3_mul",
                     "lq_su3_spinor_mul"):
            getattr(L, name).restype = ip
        L.lq_norm2.argtypes = [vp, dp, vp, ip, ip]
        L.lq_dot.argtypes = [vp, dp, vp, vp, ip, ip]
        L.lq_solve.argtypes = [vp, dp, dp, ip, ct.c_double, ct.c_double, ct.c_double,
                               ct.POINTER(SolverParams), ct.POINTER(SolveReport)]
        L.lq_solve_device.argtypes = [vp, vp, vp, ip, ct.c_double, ct.c_double, ct.c_double,
                                      ct.POINTER(SolverParams), ct.POINTER(SolveReport)]
        L.lq_net_create.argtypes = [vp, ip, ct.POINTER(vp)]
        L.lq_net_destroy.argtypes = [vp]
        L.lq_net_destroy.restype = None
        L.lq_net_set_weights.argtypes = [vp, dp]
        L.lq_net_get_weights.argtypes = [vp, dp]
        L.lq_net_init_neumann.argtypes = [vp, ct.c_double]
        L.lq_net_apply.argtypes = [vp, vp, vp, ip]
        L.lq_net_loss_grad.argtypes = [vp, vp, vp, ip, dp, dp]
        L.lq_net_adam_step.argtypes = [vp, ct.c_double, ct.c_double, ct.c_double, ct.c_double]
        L.lq_net_train.argtypes = [vp, vp, vp, ip, ip, ip, ct.c_double, ct.c_uint, dp]
        L.lq_net_save.argtypes = [vp, ct.c_char_p]
        L.lq_net_load.argtypes = [vp, ct.c_char_p]
        L.lq_solve_net.argtypes = [vp, vp, dp, dp, ip, ct.c_double, ct.c_double, ct.c_double,
                                   ct.POINTER(SolverParams), ct.POINTER(SolveReport)]
        L.lq_sap_apply.argtypes = [vp, vp, vp, ct.POINTER(SapParams)]
        L.lq_solve_sap.argtypes = [vp, vp, vp, ct.c_double, ct.c_double, ct.c_double,
                                   ct.POINTER(SapParams), ct.POINTER(SolveReport)]
        L.lq_ensemble_create.argtypes = [ct.POINTER(vp), ip, ct.POINTER(vp)]
        L.lq_ensemble_destroy.argtypes = [vp]
        L.lq_ensemble_destroy.restype = None
        L.lq_ensemble_last_error.argtypes = [vp]
        L.lq_ensemble_last_error.restype = ct.c_char_p
        L.lq_ensemble_tune.argtypes = [vp, ip, ct.c_char_p, ct.POINTER(EnsembleReport)]
        L.lq_ensemble_solve.argtypes = [vp, ct.POINTER(vp), ct.POINTER(vp), dp, dp, ct.c_double,
                                        ct.POINTER(SolverParams), ct.POINTER(SolveReport),
                                        ct.POINTER(EnsembleReport)]
        for name in ("lq_ensemble_create", "lq_ensemble_tune", "lq_ensemble_solve"):
            getattr(L, name).restype = ip
        L.lq_set_tiling.argtypes = [vp, ct.c_int64, ct.c_int64]
        L.lq_set_tiling.restype = ip
        L.lq_get_tiling.argtypes = [vp, ct.POINTER(ct.c_int), ct.POINTER(ct.c_int)]
        L.lq_get_tiling.restype = ip
        L.lq_tune_tiles.argtypes = [ct.POINTER(ct.c_int), ip, ip, ip, ct.c_char_p,
                                    ct.POINTER(TuneReport)]
        L.lq_tune_tiles.restype = ip
        L.lq_tune_last_error.argtypes = []
        L.lq_tune_last_error.restype = ct.c_char_p
        for name in ("lq_upload_gauge", "lq_set_clover", "lq_spinor_to_device",
                     "lq_spinor_to_host", "lq_dslash", "lq_clover_apply", "lq_schur",
                     "lq_schur_noalloc",
                     "lq_norm2", "lq_dot", "lq_solve", "lq_solve_device", "lq_sap_apply",
                     "lq_solve_sap", "lq_net_create",
                     "lq_net_set_weights", "lq_net_get_weights", "lq_net_init_neumann", "lq_net_apply",
                     "lq_net_loss_grad", "lq_net_adam_step", "lq_net_train", "lq_solve_net",
                     "lq_net_save", "lq_net_load"):
            getattr(L, name).restype = ip
        _lib = L
    return _lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ct.POINTER(ct.c_double))


def _torch():
    import torch
    return torch


def current_stream_handle():
    torch = _torch()
    return ct.c_void_p(torch.cuda.current_stream().cuda_stream)


@dataclass
class Report:
    iterations: int
    reliable_updates: int
    fallback: int
    dslash_calls: int
    true_residual: float
    schur_residual: float
    seconds: float
    bytes: float
    kernel_ms: list
    kernel_bytes: list
    kernel_calls: list
    ref_error: float = -1.0


TUNE_MAX = 8


class TuneReport(ct.Structure):
    _fields_ = [("ncand", ct.c_int), ("target", ct.c_int64 * TUNE_MAX),
                ("tiles", (ct.c_int * 4) * TUNE_MAX), ("us", ct.c_double * TUNE_MAX),
                ("best", ct.c_int), ("from_cache", ct.c_int)]

    def as_dict(self):
        n = self.ncand
        return {"candidates": [{"max_tile_sites": int(self.target[i]),
                                "tile": list(self.tiles[i]), "us": round(self.us[i], 2)}
                               for i in range(n)],
                "chosen": int(self.target[self.best]), "from_cache": bool(self.from_cache)}


def tune_tiles(dims, prec, nrhs=1, cache_path=None, antiperiodic_t=True):
    """lq_tune_tiles: the fastest tile for `dims` at `prec` (LQ_F16X with nrhs
    for the multi-RHS numbering), and every candidate's time."""
    L = lib()
    arr = (ct.c_int * 4)(*[int(d) for d in dims])
    rep = TuneReport()
    rc = L.lq_tune_tiles(arr, int(bool(antiperiodic_t)), int(prec), int(nrhs),
                         str(cache_path).encode() if cache_path else None, ct.byref(rep))
    if rc != 0:
        raise LQError(rc, L.lq_tune_last_error().decode())
    return rep


class Lattice:
    """One lq context: lattice geometry, gauge field, clover term, solvers.
    tile_sites / mr_tile_sites (0: the library's default) set the tiling
    (lq_set_tiling) before anything is laid out."""

    def __init__(self, dims, antiperiodic_t=True, stream=None, tile_sites=0, mr_tile_sites=0):
        self._L = lib()
        self.dims = tuple(int(d) for d in dims)
        arr = (ct.c_int * 4)(*self.dims)
        h = ct.c_void_p()
        st = stream if stream is not None else current_stream_handle()
        rc = self._L.lq_create(arr, int(bool(antiperiodic_t)), st, ct.byref(h))
        if rc != 0:
            raise LQError(rc, self._L.lq_last_error(None).decode())
        self._h = h
        self.volume = int(self._L.lq_volume(h))
        if tile_sites or mr_tile_sites:
            self.set_tiling(tile_sites, mr_tile_sites)

    def set_tiling(self, tile_sites=0, mr_tile_sites=0):
        self._check(self._L.lq_set_tiling(self._h, int(tile_sites), int(mr_tile_sites)))

    def tiling(self):
        a, b = (ct.c_int * 4)(), (ct.c_int * 4)()
        self._check(self._L.lq_get_tiling(self._h, a, b))
        return list(a), list(b)

    def close(self):
        if getattr(self, "_h", None):
            self._L.lq_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != 0:
            raise LQError(rc, self._L.lq_last_error(self._h).decode())

    # -- fields ---------------------------------------------------------
    def field_bytes(self, parity, prec, nrhs=1):
        return int(self._L.lq_field_bytes(self._h, parity, prec, nrhs))

    def new_field(self, parity, prec, nrhs=1):
        torch = _torch()
        return torch.zeros(self.field_bytes(parity, prec, nrhs), dtype=torch.uint8,
                           device="cuda")

    def to_device(self, host, parity, prec, out=None):
        """Host (nrhs?, sites, 4, 3) complex128 -> new (or given) device field."""
        host = np.ascontiguousarray(host, dtype=np.complex128)
        nsite = self.volume if parity == FULL else self.volume // 2
        nrhs = host.size // (nsite * 12)
        assert nrhs * nsite * 12 == host.size, "host array size does not match the parity"
        if out is None:
            out = self.new_field(parity, prec, nrhs)
        self._check(self._L.lq_spinor_to_device(self._h, ct.c_void_p(out.data_ptr()),
                                                _dptr(host.view(np.float64)), parity, prec,
                                                nrhs))
        return out

    def to_host(self, dev, parity, prec, nrhs=1):
        nsite = self.volume if parity == FULL else self.volume // 2
        out = np.empty((nrhs, nsite, 4, 3), dtype=np.complex128)
        self._check(self._L.lq_spinor_to_host(self._h, _dptr(out.view(np.float64)),
                                              ct.c_void_p(dev.data_ptr()), parity, prec, nrhs))
        return out[0] if nrhs == 1 else out

    # -- operator -------------------------------------------------------
    def upload_gauge(self, u):
        u = np.ascontiguousarray(u, dtype=np.complex128)
        assert u.size == self.volume * 36
        self._check(self._L.lq_upload_gauge(self._h, _dptr(u.view(np.float64))))

    def set_clover(self, kappa, csw):
        self._check(self._L.lq_set_clover(self._h, float(kappa), float(csw)))

    def dslash(self, out, inp, out_parity, dagger=False, prec=F64, nrhs=1):
        self._check(self._L.lq_dslash(self._h, ct.c_void_p(out.data_ptr()),
                                      ct.c_void_p(inp.data_ptr()), out_parity, int(dagger),
                                      prec, nrhs))

    def clover(self, out, inp, parity, inverse=False, prec=F64, nrhs=1):
        self._check(self._L.lq_clover_apply(self._h, ct.c_void_p(out.data_ptr()),
                                            ct.c_void_p(inp.data_ptr()), parity,
                                            int(inverse), prec, nrhs))

    def schur(self, out, inp, tmp, dagger=False, prec=F64, nrhs=1):
        self._check(self._L.lq_schur(self._h, ct.c_void_p(out.data_ptr()),
                                     ct.c_void_p(inp.data_ptr()), ct.c_void_p(tmp.data_ptr()),
                                     int(dagger), prec, nrhs))

    def schur_noalloc(self, out, inp, dagger=False, prec=F64, nrhs=1):
        """lq_schur without a temporary buffer (static device scratch; allocates
        nothing)."""
        self._check(self._L.lq_schur_noalloc(self._h, ct.c_void_p(out.data_ptr()),
                                             ct.c_void_p(inp.data_ptr()), int(dagger), prec,
                                             nrhs))

    def norm2(self, a, parity=EVEN, prec=F64):
        v = np.zeros(1)
        self._check(self._L.lq_norm2(self._h, _dptr(v), ct.c_void_p(a.data_ptr()), parity,
                                     prec))
        return float(v[0])

    def dot(self, a, b, parity=EVEN, prec=F64):
        v = np.zeros(2)
        self._check(self._L.lq_dot(self._h, _dptr(v), ct.c_void_p(a.data_ptr()),
                                   ct.c_void_p(b.data_ptr()), parity, prec))
        return complex(v[0], v[1])

    # -- solver ---------------------------------------------------------
    def solve(self, b, kappa, csw, tol=1e-10, solver=CGNR, inner_prec=F64, maxiter=0,
              delta=0.0, restart=0, check_every=0, use_graph=0, fault_inject=0,
              profile=0, batched=0, raise_on_noconv=True):
        """Solve M x = b on the full lattice; b has shape (nrhs?, V-sites..., 4, 3).
        batched=1 runs all right-hand sides through the multi-RHS operator as
        independent CG recurrences, batched=2 as one block CG."""
        b = np.ascontiguousarray(b, dtype=np.complex128)
        nrhs = b.size // (self.volume * 12)
        assert nrhs * self.volume * 12 == b.size
        x = np.zeros_like(b)
        p = SolverParams(solver, inner_prec, maxiter, delta, restart, check_every, use_graph,
                         fault_inject, profile, batched)
        reps = (SolveReport * nrhs)()
        rc = self._L.lq_solve(self._h, _dptr(x.view(np.float64)), _dptr(b.view(np.float64)),
                              nrhs, float(kappa), float(csw), float(tol), ct.byref(p), reps)
        reports = [Report(**r.as_dict()) for r in reps]
        if rc != 0 and (rc != -4 or raise_on_noconv):
            self._check(rc)
        return x, reports

    def solve_device(self, dev_x, dev_b, kappa, csw, tol=1e-10, nrhs=1, solver=CGNR,
                     inner_prec=F64, maxiter=0, delta=0.0, restart=0, check_every=0,
                     use_graph=0, fault_inject=0, profile=0, batched=0,
                     raise_on_noconv=True, xref=None):
        """Solve with device-resident full-lattice FP64 fields (see lq_solve_device);
        xref: optional device reference solution(s), reported as ref_error."""
        p = SolverParams(solver, inner_prec, maxiter, delta, restart, check_every, use_graph,
                         fault_inject, profile, batched, 0,
                         xref.data_ptr() if xref is not None else None)
        reps = (SolveReport * nrhs)()
        rc = self._L.lq_solve_device(self._h, ct.c_void_p(dev_x.data_ptr()),
                                     ct.c_void_p(dev_b.data_ptr()), nrhs, float(kappa),
                                     float(csw), float(tol), ct.byref(p), reps)
        reports = [Report(**r.as_dict()) for r in reps]
        if rc != 0 and (rc != -4 or raise_on_noconv):
            self._check(rc)
        return reports


    # -- SAP preconditioner and FGCR ------------------------------------
    @staticmethod
    def _sap_params(block, ncycles, nmr, restart=0, maxiter=0, deflate=0, block_fp16=0,
                    block_eo=0):
        return SapParams((ct.c_int * 4)(*[int(b) for b in block]), int(ncycles), int(nmr),
                         int(restart), int(maxiter), int(deflate), int(bool(block_fp16)),
                         int(bool(block_eo)))

    def sap_apply(self, dev_out, dev_in, block, ncycles=0, nmr=0, block_fp16=False,
                  block_eo=False):
        """dev_out = K dev_in on full-lattice FP32 fields (see lq_sap_apply)."""
        p = self._sap_params(block, ncycles, nmr, block_fp16=block_fp16, block_eo=block_eo)
        self._check(self._L.lq_sap_apply(self._h, ct.c_void_p(dev_out.data_ptr()),
                                         ct.c_void_p(dev_in.data_ptr()), ct.byref(p)))

    def solve_sap_device(self, dev_x, dev_b, kappa, csw, tol=1e-10, block=(4, 4, 4, 4),
                         ncycles=0, nmr=0, restart=0, maxiter=0, raise_on_noconv=True,
                         deflate=0, block_fp16=False, block_eo=False):
        """SAP-preconditioned FGCR, or FGMRES-DR with `deflate` deflated vectors, on
        full-lattice FP64 device fields (see lq_solve_sap)."""
        p = self._sap_params(block, ncycles, nmr, restart, maxiter, deflate, block_fp16,
                             block_eo)
        rep = SolveReport()
        rc = self._L.lq_solve_sap(self._h, ct.c_void_p(dev_x.data_ptr()),
                                  ct.c_void_p(dev_b.data_ptr()), float(kappa), float(csw),
                                  float(tol), ct.byref(p), ct.byref(rep))
        if rc != 0 and (rc != -4 or raise_on_noconv):
            self._check(rc)
        return Report(**rep.as_dict())

    def solve_sap(self, b, kappa, csw, tol=1e-10, block=(4, 4, 4, 4), **kw):
        """The same from and to host arrays (one full-lattice right-hand side)."""
        db = self.to_device(b, FULL, F64)
        dx = self.new_field(FULL, F64)
        rep = self.solve_sap_device(dx, db, kappa, csw, tol, block, **kw)
        return self.to_host(dx, FULL, F64).reshape(np.shape(b)), rep


NET_K = 9  # weight matrices per layer: W0, then (Wp_mu, Wm_mu) for mu = 0..3


class Net:
    """Learned gauge-covariant preconditioner on a Lattice (see lq_net_* in
    include/lq.h).  Weights: complex array (nlayers, 9, 4, 4); device fields
    of its calls: FP32 even fields (Lattice.field_bytes(EVEN, F32, n))."""

    def __init__(self, lat, nlayers=4):
        self.lat = lat
        self._L = lat._L
        self.nlayers = int(nlayers)
        h = ct.c_void_p()
        lat._check(self._L.lq_net_create(lat._h, self.nlayers, ct.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self._L.lq_net_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_weights(self, w):
        w = np.ascontiguousarray(w, dtype=np.complex128)
        assert w.shape == (self.nlayers, NET_K, 4, 4)
        self.lat._check(self._L.lq_net_set_weights(self._h, _dptr(w.view(np.float64))))

    def init_neumann(self, kappa):
        self.lat._check(self._L.lq_net_init_neumann(self._h, float(kappa)))

    def get_weights(self):
        w = np.zeros((self.nlayers, NET_K, 4, 4), dtype=np.complex128)
        self.lat._check(self._L.lq_net_get_weights(self._h, _dptr(w.view(np.float64))))
        return w

    def apply(self, out, inp, adjoint=False, fp16=False):
        mode = (1 if adjoint else 0) | (2 if fp16 else 0)
        self.lat._check(self._L.lq_net_apply(self._h, ct.c_void_p(out.data_ptr()),
                                             ct.c_void_p(inp.data_ptr()), mode))

    def loss_grad(self, dev_b, dev_x, npairs):
        loss = np.zeros(1)
        g = np.zeros((self.nlayers, NET_K, 4, 4), dtype=np.complex128)
        self.lat._check(self._L.lq_net_loss_grad(self._h, ct.c_void_p(dev_b.data_ptr()),
                                                 ct.c_void_p(dev_x.data_ptr()), int(npairs),
                                                 _dptr(loss), _dptr(g.view(np.float64))))
        return float(loss[0]), g

    def adam_step(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.lat._check(self._L.lq_net_adam_step(self._h, lr, beta1, beta2, eps))

    def train(self, dev_b, dev_x, npairs, epochs, batch=8, lr=1e-3, seed=0):
        hist = np.zeros(int(epochs))
        self.lat._check(self._L.lq_net_train(self._h, ct.c_void_p(dev_b.data_ptr()),
                                             ct.c_void_p(dev_x.data_ptr()), int(npairs),
                                             int(epochs), int(batch), float(lr), int(seed),
                                             _dptr(hist)))
        return hist

    def save(self, path):
        """Checkpoint weights, Adam moments and step, shuffle state (lq_net_save)."""
        self.lat._check(self._L.lq_net_save(self._h, str(path).encode()))

    def load(self, path):
        self.lat._check(self._L.lq_net_load(self._h, str(path).encode()))

    def solve(self, b, kappa, csw, tol=1e-10, solver=FGMRES_NET, maxiter=0, restart=0,
              raise_on_noconv=True, deflate=0):
        """Solve M x = b (full lattice, host arrays) with a flexible solver
        preconditioned by this net (FGMRES-DR when deflate > 0)."""
        b = np.ascontiguousarray(b, dtype=np.complex128)
        nrhs = b.size // (self.lat.volume * 12)
        assert nrhs * self.lat.volume * 12 == b.size
        x = np.zeros_like(b)
        p = SolverParams(solver, F32, maxiter, 0.0, restart, 0, 0, 0, 0, 0, deflate)
        reps = (SolveReport * nrhs)()
        rc = self._L.lq_solve_net(self.lat._h, self._h, _dptr(x.view(np.float64)),
                                  _dptr(b.view(np.float64)), nrhs, float(kappa), float(csw),
                                  float(tol), ct.byref(p), reps)
        reports = [Report(**r.as_dict()) for r in reps]
        if rc != 0 and (rc != -4 or raise_on_noconv):
            self.lat._check(rc)
        return x, reports


class Ensemble:
    """Uneven batch of independent solves on several Lattice objects (see
    lq_ensemble_* in include/lq.h).  The lattices must outlive the batch."""

    def __init__(self, lattices):
        self.lats = list(lattices)
        self._L = lib()
        arr = (ct.c_void_p * len(self.lats))(*[l._h.value for l in self.lats])
        h = ct.c_void_p()
        rc = self._L.lq_ensemble_create(arr, len(self.lats), ct.byref(h))
        if rc != 0:
            raise LQError(rc, self._L.lq_ensemble_last_error(None).decode())
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self._L.lq_ensemble_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != 0:
            raise LQError(rc, self._L.lq_ensemble_last_error(self._h).decode())

    def tune(self, inner_prec=F16, cache_path=None):
        rep = EnsembleReport()
        path = cache_path.encode() if cache_path else None
        self._check(self._L.lq_ensemble_tune(self._h, inner_prec, path, ct.byref(rep)))
        return rep.as_dict()

    def solve_device(self, dev_x, dev_b, kappas, csws, tol=1e-10, inner_prec=F16, maxiter=0,
                     delta=0.0, check_every=0, use_graph=0, fault_inject=0,
                     raise_on_noconv=True):
        """dev_x[j], dev_b[j]: full-lattice FP64 device fields of lattice j.
        Returns (member reports, batch report dict)."""
        n = len(self.lats)
        assert len(dev_x) == n and len(dev_b) == n and len(kappas) == n and len(csws) == n
        xs = (ct.c_void_p * n)(*[t.data_ptr() for t in dev_x])
        bs = (ct.c_void_p * n)(*[t.data_ptr() for t in dev_b])
        ka = np.ascontiguousarray(kappas, dtype=np.float64)
        cs = np.ascontiguousarray(csws, dtype=np.float64)
        p = SolverParams(CGNR, inner_prec, maxiter, delta, 0, check_every, use_graph,
                         fault_inject, 0, 0)
        reps = (SolveReport * n)()
        er = EnsembleReport()
        rc = self._L.lq_ensemble_solve(self._h, xs, bs, _dptr(ka), _dptr(cs), float(tol),
                                       ct.byref(p), reps, ct.byref(er))
        reports = [Report(**r.as_dict()) for r in reps]
        if rc != 0 and (rc != -4 or raise_on_noconv):
            self._check(rc)
        return reports, er.as_dict()


# ---------------------------------------------------------------- fused site expressions
SITE_SU3, SITE_SPINOR = 0, 1
SU3_VW, SU3_VWDAG, SU3_VDAGW, SU3_VWX = 0, 1, 2, 3


def _stream():
    return ct.c_void_p(_torch().cuda.current_stream().cuda_stream)


def _expr_check(rc, what):
    if rc != 0:
        raise LQError(rc, what)


def site_array_bytes(n, kind, prec):
    return int(lib().lq_site_array_bytes(int(n), kind, prec))


def site_array_to_device(host, kind, prec):
    """Host (n, 3, 3) matrices or (n, 4, 3) spinors, complex128 -> device array."""
    host = np.ascontiguousarray(host, dtype=np.complex128)
    n = host.shape[0]
    torch = _torch()
    dev = torch.empty(site_array_bytes(n, kind, prec), dtype=torch.uint8, device="cuda")
    _expr_check(lib().lq_site_array_to_device(ct.c_void_p(dev.data_ptr()),
                                              _dptr(host.view(np.float64)), n, kind, prec,
                                              _stream()), "lq_site_array_to_device")
    return dev


def site_array_to_host(dev, n, kind, prec):
    shape = (n, 3, 3) if kind == SITE_SU3 else (n, 4, 3)
    out = np.empty(shape, dtype=np.complex128)
    _expr_check(lib().lq_site_array_to_host(_dptr(out.view(np.float64)),
                                            ct.c_void_p(dev.data_ptr()), n, kind, prec,
                                            _stream()), "lq_site_array_to_host")
    return out


def su3_mul(out, v, w, n, form=SU3_VW, prec=F64, x=None):
    """out = V W (or the form's product) on n matrices; one fused kernel."""
    _expr_check(lib().lq_su3_mul(ct.c_void_p(out.data_ptr()), ct.c_void_p(v.data_ptr()),
                                 ct.c_void_p(w.data_ptr()),
                                 ct.c_void_p(x.data_ptr() if x is not None else 0), int(n),
                                 form, prec, _stream()), "lq_su3_mul")


def su3_spinor_mul(out, u, psi, n, adjoint=False, prec=F64):
    _expr_check(lib().lq_su3_spinor_mul(ct.c_void_p(out.data_ptr()), ct.c_void_p(u.data_ptr()),
                                        ct.c_void_p(psi.data_ptr()), int(n), int(adjoint), prec,
                                        _stream()), "lq_su3_spinor_mul")
