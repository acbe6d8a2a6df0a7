"""Thin Python binding of the C ABI in include/fmmcph.h (argument marshalling only).

Every step of an evaluation runs in the HIP kernels of ``libfmmcph.so``; this
module only checks tensor dtypes/devices and passes raw pointers.  PyTorch
provides device memory and the stream.  There is no fallback: if the library
is missing, importing the loader raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfmmcph.so")

FMM_OK = 0
FMM_E_INVALID = 1
FMM_E_OOM = 2
FMM_E_HIP = 3
FMM_E_UNSUPPORTED = 4
FMM_E_NONFINITE = 5
FMM_E_SITE = 6
FMM_E_COINCIDENT = 7
STATUS_NAMES = {0: "FMM_OK", 1: "FMM_E_INVALID", 2: "FMM_E_OOM", 3: "FMM_E_HIP",
                4: "FMM_E_UNSUPPORTED", 5: "FMM_E_NONFINITE", 6: "FMM_E_SITE",
                7: "FMM_E_COINCIDENT"}

FMM_OPEN = 0
FMM_PERIODIC = 1
FMM_FP64 = 0
FMM_MIXED_F32 = 1
FMM_MIXED_BF16X3 = 2
PRECISIONS = {"fp64": FMM_FP64, "f32": FMM_MIXED_F32, "bf16x3": FMM_MIXED_BF16X3}


class fmm_params(ctypes.Structure):
    _fields_ = [
        ("depth", ctypes.c_int32),
        ("order_p", ctypes.c_int32),
        ("boundary", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("coulomb_k", ctypes.c_double),
        ("max_atoms", ctypes.c_int64),
        ("max_sites", ctypes.c_int64),
        ("max_replicas", ctypes.c_int32),
        ("check", ctypes.c_int32),
        ("m2l_kernel", ctypes.c_int32),
        ("m2l_chunk", ctypes.c_int32),
        ("p2p_waves", ctypes.c_int32),
        ("graph", ctypes.c_int32),
        ("p2p_split", ctypes.c_int32),
        ("hamiltonian", ctypes.c_int32),
    ]


EXPORTS = ["fmm_plan_create", "fmm_eval", "fmm_eval_adjoint", "fmm_eval_batched",
           "fmm_eval_tautomer", "fmm_eval_tautomer_batched",
           "fmm_sync_check", "fmm_last_error", "fmm_plan_destroy", "fmm_profile",
           "fmm_profile_select", "fmm_plan_info", "fmm_host_operator",
           "fmm_lambda_step", "fmm_lambda_dbo", "fmm_lambda_pfc", "fmm_set_exclusions",
           "fmm_eval_adjoint_phi", "fmm_eval_adjoint_full", "fmm_eval_noalloc"]
PHASES = ["bin", "p2m", "m2m", "root", "m2l", "l2l", "near_far", "reduce"]

_lib = None


class FmmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


def load_library(path: str = LIB_PATH):
    """Load libfmmcph.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libfmmcph.so is not built: run __graft_entry__.build() or "
                           "python paper_2410_01626_amd/build_lib.py")
    lib = ctypes.CDLL(path)
    vp, i64, i32, dp = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p
    lib.fmm_plan_create.restype = ctypes.c_int
    lib.fmm_plan_create.argtypes = [ctypes.POINTER(fmm_params), vp, ctypes.POINTER(vp)]
    lib.fmm_eval.restype = ctypes.c_int
    lib.fmm_eval.argtypes = [vp, i64, vp, vp, vp, vp, i64, vp, vp, vp, vp, vp, vp]
    lib.fmm_eval_noalloc.restype = ctypes.c_int
    lib.fmm_eval_noalloc.argtypes = [vp, i64, vp, vp, vp, vp, i64, vp, vp, vp, vp, vp, vp]
    lib.fmm_eval_adjoint.restype = ctypes.c_int
    lib.fmm_eval_adjoint.argtypes = [vp, i64, vp, vp, vp, vp, i64, vp, vp, vp,
                                     vp, vp, vp, vp, vp, vp, vp, vp]
    lib.fmm_eval_batched.restype = ctypes.c_int
    lib.fmm_eval_batched.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.fmm_eval_tautomer.restype = ctypes.c_int
    lib.fmm_eval_tautomer.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, i64, vp, vp, vp, vp, vp,
                                      vp, vp, vp]
    lib.fmm_eval_tautomer_batched.restype = ctypes.c_int
    lib.fmm_eval_tautomer_batched.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp,
                                              vp, vp, vp, vp, vp, vp]
    lib.fmm_sync_check.restype = ctypes.c_int
    lib.fmm_sync_check.argtypes = [vp]
    lib.fmm_last_error.restype = ctypes.c_char_p
    lib.fmm_last_error.argtypes = [vp]
    lib.fmm_plan_destroy.restype = None
    lib.fmm_plan_destroy.argtypes = [vp]
    lib.fmm_profile.restype = ctypes.c_int
    lib.fmm_profile.argtypes = [vp, i32, i32, vp]
    lib.fmm_profile_select.restype = ctypes.c_int
    lib.fmm_profile_select.argtypes = [vp, ctypes.c_uint32, i32]
    lib.fmm_plan_info.restype = ctypes.c_int
    lib.fmm_plan_info.argtypes = [vp, vp]
    lib.fmm_host_operator.restype = ctypes.c_int64
    lib.fmm_host_operator.argtypes = [i32, i32, dp]
    lib.fmm_eval_adjoint_phi.restype = ctypes.c_int
    lib.fmm_eval_adjoint_phi.argtypes = [vp, i64, vp, vp, vp, vp, i64, vp, vp, ctypes.c_double,
                                         vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.fmm_eval_adjoint_full.restype = ctypes.c_int
    lib.fmm_eval_adjoint_full.argtypes = [vp, i64, vp, vp, vp, vp, i64, vp, vp, vp, vp, vp,
                                          vp, vp, vp, vp, vp, vp, vp, vp]
    lib.fmm_set_exclusions.restype = ctypes.c_int
    lib.fmm_set_exclusions.argtypes = [vp, i64, vp, vp]
    lib.fmm_lambda_step.restype = ctypes.c_int
    lib.fmm_lambda_step.argtypes = [vp, i32, vp, i64, vp, i32] + [vp] * 16
    lib.fmm_lambda_dbo.restype = ctypes.c_int
    lib.fmm_lambda_dbo.argtypes = [vp, i32, vp, i64, i32, i32, vp, ctypes.c_double] + [vp] * 9
    lib.fmm_lambda_pfc.restype = ctypes.c_int
    lib.fmm_lambda_pfc.argtypes = [vp, i32, vp, i64, ctypes.c_double, vp, vp, vp, vp, vp]
    _lib = lib
    return lib


# ----------------------------------------------------------------- raw C names

def fmm_plan_create(params: fmm_params, hip_stream=None):
    lib = load_library()
    out = ctypes.c_void_p()
    st = lib.fmm_plan_create(ctypes.byref(params), ctypes.c_void_p(hip_stream or 0),
                             ctypes.byref(out))
    if st != FMM_OK:
        raise FmmError(st, "fmm_plan_create")
    return out


def fmm_plan_destroy(plan):
    load_library().fmm_plan_destroy(plan)


def fmm_last_error(plan) -> str:
    return load_library().fmm_last_error(plan).decode()


def fmm_sync_check(plan) -> int:
    return load_library().fmm_sync_check(plan)


def fmm_eval(plan, n, x, qA, qB, site, n_sites, lam, box, E, F, phi, dVdl) -> int:
    return load_library().fmm_eval(plan, n, x, qA, qB, site, n_sites, lam, box, E, F, phi, dVdl)


def fmm_eval_adjoint(plan, n, x, qA, qB, site, n_sites, lam, box, gE, gx, gqA, gqB, glam,
                     E, F, phi, dVdl) -> int:
    return load_library().fmm_eval_adjoint(plan, n, x, qA, qB, site, n_sites, lam, box, gE,
                                           gx, gqA, gqB, glam, E, F, phi, dVdl)


def fmm_eval_batched(plan, R, atom_off, site_off, x, qA, qB, site_local, lam, boxes, E, F,
                     phi, dVdl) -> int:
    return load_library().fmm_eval_batched(plan, R, atom_off, site_off, x, qA, qB, site_local,
                                           lam, boxes, E, F, phi, dVdl)


def fmm_eval_tautomer(plan, n, x, qA, qB, qC, qD, site, n_sites, lam_p, lam_t, box, E, F, phi,
                      dVdl_p, dVdl_t) -> int:
    return load_library().fmm_eval_tautomer(plan, n, x, qA, qB, qC, qD, site, n_sites, lam_p,
                                            lam_t, box, E, F, phi, dVdl_p, dVdl_t)


def fmm_eval_tautomer_batched(plan, R, atom_off, site_off, x, qA, qB, qC, qD, site_local, lam_p,
                              lam_t, boxes, E, F, phi, dVdl_p, dVdl_t) -> int:
    return load_library().fmm_eval_tautomer_batched(plan, R, atom_off, site_off, x, qA, qB, qC,
                                                    qD, site_local, lam_p, lam_t, boxes, E, F,
                                                    phi, dVdl_p, dVdl_t)


def fmm_profile(plan, mode: int, capacity: int = 0, out=None) -> int:
    return load_library().fmm_profile(plan, mode, capacity,
                                      ctypes.c_void_p(0) if out is None else out.ctypes.data)


def fmm_profile_select(plan, phase_mask: int, every: int = 1) -> int:
    return load_library().fmm_profile_select(plan, phase_mask, every)


def fmm_host_operator(order_p: int, which: int, point=None) -> np.ndarray:
    """FP64 operator tables a plan uploads (host only, no GPU needed)."""
    K = (order_p + 1) ** 2
    size = {0: 343 * K * K, 1: 8 * K * K, 2: 8 * K * K, 3: K * K, 4: K, 5: K}[which]
    out = np.zeros(max(size, 3))
    if which == 4:
        out[:3] = np.asarray(point, dtype=np.float64)
    n = load_library().fmm_host_operator(order_p, which, out.ctypes.data)
    if n != size:
        raise ValueError("fmm_host_operator(%d, %d) failed" % (order_p, which))
    out = out[:size]
    if which == 0:
        return out.reshape(7, 7, 7, K, K)
    if which in (1, 2):
        return out.reshape(8, K, K)
    if which == 3:
        return out.reshape(K, K)
    return out


# ----------------------------------------------------------------- torch layer

def _ptr(t):
    return ctypes.c_void_p(0) if t is None else ctypes.c_void_p(t.data_ptr())


class Plan:
    """A plan bound to one device and one stream (torch's current stream by default)."""

    def __init__(self, depth: int, order: int, periodic: bool = False,
                 precision: str = "fp64", coulomb_k: float = 1.0, max_atoms: int = 1,
                 max_sites: int = 1, max_replicas: int = 1, check: bool = False,
                 stream=None, device=None, m2l_kernel: int = 0, m2l_chunk: int = 0,
                 p2p_waves: int = 0, graph: bool = False, p2p_split: int = 0,
                 hamiltonian: bool = False):
        import torch
        dev = torch.device(device) if device is not None else torch.device("cuda")
        if dev.type == "cuda" and dev.index is None:
            dev = torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        if self.device.type != "cuda":
            raise ValueError("the FMM library runs on a GPU device only")
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.params = fmm_params(depth, order, FMM_PERIODIC if periodic else FMM_OPEN,
                                 PRECISIONS[precision], float(coulomb_k), int(max_atoms),
                                 int(max_sites), int(max_replicas), 1 if check else 0,
                                 int(m2l_kernel), int(m2l_chunk), int(p2p_waves),
                                 1 if graph else 0, int(p2p_split), 1 if hamiltonian else 0)
        self.periodic = periodic
        self.precision = precision
        self.dtype = torch.float64 if precision == "fp64" else torch.float32
        with torch.cuda.device(self.device):
            self.handle = fmm_plan_create(self.params, self.stream.cuda_stream)

    def close(self):
        if getattr(self, "handle", None) is not None:
            fmm_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _raise(self, st, what):
        if st != FMM_OK:
            raise FmmError(st, "%s: %s" % (what, fmm_last_error(self.handle)))

    def _check(self, t, dtype, shape=None, name="tensor"):
        if t.device != self.device:
            raise ValueError("%s must live on %s" % (name, self.device))
        if t.dtype != dtype:
            raise ValueError("%s must be %s, got %s" % (name, dtype, t.dtype))
        if not t.is_contiguous():
            raise ValueError("%s must be contiguous" % name)
        if shape is not None and tuple(t.shape) != tuple(shape):
            raise ValueError("%s must have shape %s, got %s" % (name, shape, tuple(t.shape)))

    def _inputs(self, x, qA, qB, site, lam):
        import torch
        n = x.shape[0]
        self._check(x, self.dtype, (n, 3), "x")
        self._check(qA, self.dtype, (n,), "qA")
        self._check(qB, self.dtype, (n,), "qB")
        self._check(site, torch.int32, (n,), "site")
        self._check(lam, torch.float64, None, "lambda")
        return n, lam.numel()

    def _box(self, box):
        if not self.periodic:
            if box is not None:
                raise ValueError("open plan takes no box")
            return None, ctypes.c_void_p(0)
        b = np.ascontiguousarray(np.broadcast_to(np.asarray(box, dtype=np.float64), (3,)))
        return b, ctypes.c_void_p(b.ctypes.data)

    def eval(self, x, qA, qB, site, lam, box=None, want=("E", "F", "phi", "dVdl"), out=None):
        """Enqueue fmm_eval; returns dict of output tensors (E is a 1-element FP64 tensor).

        `out` may hold preallocated outputs (reused pointers let a graph plan replay)."""
        import torch
        n, S = self._inputs(x, qA, qB, site, lam)
        if out is None:
            opt = dict(device=self.device)
            out = {"E": torch.empty(1, dtype=torch.float64, **opt)}
            out["F"] = torch.empty((n, 3), dtype=self.dtype, **opt) if "F" in want else None
            out["phi"] = torch.empty(n, dtype=self.dtype, **opt) if "phi" in want else None
            out["dVdl"] = torch.empty(S, dtype=torch.float64, **opt) if "dVdl" in want else None
        b, bp = self._box(box)
        st = fmm_eval(self.handle, n, _ptr(x), _ptr(qA), _ptr(qB), _ptr(site), S, _ptr(lam), bp,
                      _ptr(out["E"]), _ptr(out["F"]), _ptr(out["phi"]), _ptr(out["dVdl"]))
        self._raise(st, "fmm_eval")
        return out

    def eval_noalloc(self, x, qA, qB, site, lam, box=None, out=None):
        """Enqueue fmm_eval_noalloc (the evaluation of eval() with its scratch in
        the library's static array); `out` as in eval()."""
        import torch
        n, S = self._inputs(x, qA, qB, site, lam)
        if out is None:
            opt = dict(device=self.device)
            out = {"E": torch.empty(1, dtype=torch.float64, **opt),
                   "F": torch.empty((n, 3), dtype=self.dtype, **opt),
                   "phi": torch.empty(n, dtype=self.dtype, **opt),
                   "dVdl": torch.empty(S, dtype=torch.float64, **opt)}
        b, bp = self._box(box)
        st = load_library().fmm_eval_noalloc(
            self.handle, n, _ptr(x), _ptr(qA), _ptr(qB), _ptr(site), S, _ptr(lam), bp,
            _ptr(out["E"]), _ptr(out["F"]), _ptr(out["phi"]), _ptr(out["dVdl"]))
        self._raise(st, "fmm_eval_noalloc")
        return out

    def eval_adjoint(self, x, qA, qB, site, lam, gE, box=None):
        """Enqueue fmm_eval_adjoint; returns dict of gradients and forward outputs."""
        import torch
        n, S = self._inputs(x, qA, qB, site, lam)
        self._check(gE, torch.float64, None, "gE")
        opt = dict(device=self.device)
        out = {"E": torch.empty(1, dtype=torch.float64, **opt),
               "F": torch.empty((n, 3), dtype=self.dtype, **opt),
               "phi": torch.empty(n, dtype=self.dtype, **opt),
               "dVdl": torch.empty(S, dtype=torch.float64, **opt),
               "grad_x": torch.empty((n, 3), dtype=self.dtype, **opt),
               "grad_qA": torch.empty(n, dtype=self.dtype, **opt),
               "grad_qB": torch.empty(n, dtype=self.dtype, **opt),
               "grad_lambda": torch.empty(S, dtype=torch.float64, **opt)}
        b, bp = self._box(box)
        st = fmm_eval_adjoint(self.handle, n, _ptr(x), _ptr(qA), _ptr(qB), _ptr(site), S,
                              _ptr(lam), bp, _ptr(gE), _ptr(out["grad_x"]), _ptr(out["grad_qA"]),
                              _ptr(out["grad_qB"]), _ptr(out["grad_lambda"]), _ptr(out["E"]),
                              _ptr(out["F"]), _ptr(out["phi"]), _ptr(out["dVdl"]))
        self._raise(st, "fmm_eval_adjoint")
        return out

    def eval_adjoint_phi(self, x, qA, qB, site, lam, gE: float, gphi, box=None):
        """Enqueue fmm_eval_adjoint_phi (weights gE on E, gphi on phi); returns
        dict of gradients and forward outputs."""
        import torch
        n, S = self._inputs(x, qA, qB, site, lam)
        self._check(gphi, self.dtype, (n,), "gphi")
        opt = dict(device=self.device)
        out = {"E": torch.empty(1, dtype=torch.float64, **opt),
               "F": torch.empty((n, 3), dtype=self.dtype, **opt),
               "phi": torch.empty(n, dtype=self.dtype, **opt),
               "dVdl": torch.empty(S, dtype=torch.float64, **opt),
               "grad_x": torch.empty((n, 3), dtype=self.dtype, **opt),
               "grad_qA": torch.empty(n, dtype=self.dtype, **opt),
               "grad_qB": torch.empty(n, dtype=self.dtype, **opt),
               "grad_lambda": torch.empty(S, dtype=torch.float64, **opt)}
        b, bp = self._box(box)
        st = load_library().fmm_eval_adjoint_phi(
            self.handle, n, _ptr(x), _ptr(qA), _ptr(qB), _ptr(site), S, _ptr(lam), bp, float(gE),
            _ptr(gphi), _ptr(out["grad_x"]), _ptr(out["grad_qA"]), _ptr(out["grad_qB"]),
            _ptr(out["grad_lambda"]), _ptr(out["E"]), _ptr(out["F"]), _ptr(out["phi"]),
            _ptr(out["dVdl"]))
        self._raise(st, "fmm_eval_adjoint_phi")
        return out

    def eval_adjoint_full(self, x, qA, qB, site, lam, gE=None, gphi=None, gF=None, box=None):
        """Enqueue fmm_eval_adjoint_full: gradients of gE E + gphi . phi + gF . F
        (gE a 1-element FP64 device tensor or None; gphi (n,) and gF (n, 3) of
        the plan's type or None); returns dict of gradients and forward outputs."""
        import torch
        n, S = self._inputs(x, qA, qB, site, lam)
        if gE is not None:
            self._check(gE, torch.float64, (1,), "gE")
        if gphi is not None:
            self._check(gphi, self.dtype, (n,), "gphi")
        if gF is not None:
            self._check(gF, self.dtype, (n, 3), "gF")
        opt = dict(device=self.device)
        out = {"E": torch.empty(1, dtype=torch.float64, **opt),
               "F": torch.empty((n, 3), dtype=self.dtype, **opt),
               "phi": torch.empty(n, dtype=self.dtype, **opt),
               "dVdl": torch.empty(S, dtype=torch.float64, **opt),
               "grad_x": torch.empty((n, 3), dtype=self.dtype, **opt),
               "grad_qA": torch.empty(n, dtype=self.dtype, **opt),
               "grad_qB": torch.empty(n, dtype=self.dtype, **opt),
               "grad_lambda": torch.empty(S, dtype=torch.float64, **opt)}
        b, bp = self._box(box)
        st = load_library().fmm_eval_adjoint_full(
            self.handle, n, _ptr(x), _ptr(qA), _ptr(qB), _ptr(site), S, _ptr(lam), bp, _ptr(gE),
            _ptr(gphi), _ptr(gF), _ptr(out["grad_x"]), _ptr(out["grad_qA"]), _ptr(out["grad_qB"]),
            _ptr(out["grad_lambda"]), _ptr(out["E"]), _ptr(out["F"]), _ptr(out["phi"]),
            _ptr(out["dVdl"]))
        self._raise(st, "fmm_eval_adjoint_full")
        return out

    def eval_batched(self, atom_off, site_off, x, qA, qB, site_local, lam, boxes=None,
                     out=None):
        """Enqueue fmm_eval_batched over R replicas (offsets are host sequences);
        `out` may hold preallocated outputs (reused pointers let a graph plan
        replay)."""
        import torch
        ao = np.ascontiguousarray(atom_off, dtype=np.int64)
        so = np.ascontiguousarray(site_off, dtype=np.int64)
        R = ao.size - 1
        n, S = self._inputs(x, qA, qB, site_local, lam)
        if ao[-1] != n or so[-1] != S:
            raise ValueError("offsets do not match the concatenated arrays")
        if out is None:
            opt = dict(device=self.device)
            out = {"E": torch.empty(R, dtype=torch.float64, **opt),
                   "F": torch.empty((n, 3), dtype=self.dtype, **opt),
                   "phi": torch.empty(n, dtype=self.dtype, **opt),
                   "dVdl": torch.empty(S, dtype=torch.float64, **opt)}
        if self.periodic:
            bx = np.ascontiguousarray(np.asarray(boxes, dtype=np.float64).reshape(R, 3))
            bp = ctypes.c_void_p(bx.ctypes.data)
        else:
            bx, bp = None, ctypes.c_void_p(0)
        st = fmm_eval_batched(self.handle, R, ctypes.c_void_p(ao.ctypes.data),
                              ctypes.c_void_p(so.ctypes.data), _ptr(x), _ptr(qA), _ptr(qB),
                              _ptr(site_local), _ptr(lam), bp, _ptr(out["E"]), _ptr(out["F"]),
                              _ptr(out["phi"]), _ptr(out["dVdl"]))
        self._raise(st, "fmm_eval_batched")
        return out

    def _forms(self, n, S, qC, qD, lam_t):
        import torch
        self._check(qC, self.dtype, (n,), "qC")
        self._check(qD, self.dtype, (n,), "qD")
        self._check(lam_t, torch.float64, (S,), "lambda_t")

    def eval_tautomer(self, x, qA, qB, qC, qD, site, lam_p, lam_t, box=None,
                      want=("E", "F", "phi", "dVdl_p", "dVdl_t"), out=None):
        """Enqueue fmm_eval_tautomer (four charge forms per site, two lambda
        coordinates); returns dict of output tensors."""
        import torch
        n, S = self._inputs(x, qA, qB, site, lam_p)
        self._forms(n, S, qC, qD, lam_t)
        if out is None:
            opt = dict(device=self.device)
            out = {"E": torch.empty(1, dtype=torch.float64, **opt)}
            out["F"] = torch.empty((n, 3), dtype=self.dtype, **opt) if "F" in want else None
            out["phi"] = torch.empty(n, dtype=self.dtype, **opt) if "phi" in want else None
            for k in ("dVdl_p", "dVdl_t"):
                out[k] = torch.empty(S, dtype=torch.float64, **opt) if k in want else None
        b, bp = self._box(box)
        st = fmm_eval_tautomer(self.handle, n, _ptr(x), _ptr(qA), _ptr(qB), _ptr(qC), _ptr(qD),
                               _ptr(site), S, _ptr(lam_p), _ptr(lam_t), bp, _ptr(out["E"]),
                               _ptr(out["F"]), _ptr(out["phi"]), _ptr(out["dVdl_p"]),
                               _ptr(out["dVdl_t"]))
        self._raise(st, "fmm_eval_tautomer")
        return out

    def eval_tautomer_batched(self, atom_off, site_off, x, qA, qB, qC, qD, site_local, lam_p,
                              lam_t, boxes=None):
        """Enqueue fmm_eval_tautomer_batched over R replicas (host offsets)."""
        import torch
        ao = np.ascontiguousarray(atom_off, dtype=np.int64)
        so = np.ascontiguousarray(site_off, dtype=np.int64)
        R = ao.size - 1
        n, S = self._inputs(x, qA, qB, site_local, lam_p)
        self._forms(n, S, qC, qD, lam_t)
        if ao[-1] != n or so[-1] != S:
            raise ValueError("offsets do not match the concatenated arrays")
        opt = dict(device=self.device)
        out = {"E": torch.empty(R, dtype=torch.float64, **opt),
               "F": torch.empty((n, 3), dtype=self.dtype, **opt),
               "phi": torch.empty(n, dtype=self.dtype, **opt),
               "dVdl_p": torch.empty(S, dtype=torch.float64, **opt),
               "dVdl_t": torch.empty(S, dtype=torch.float64, **opt)}
        if self.periodic:
            bx = np.ascontiguousarray(np.asarray(boxes, dtype=np.float64).reshape(R, 3))
            bp = ctypes.c_void_p(bx.ctypes.data)
        else:
            bx, bp = None, ctypes.c_void_p(0)
        st = fmm_eval_tautomer_batched(self.handle, R, ctypes.c_void_p(ao.ctypes.data),
                                       ctypes.c_void_p(so.ctypes.data), _ptr(x), _ptr(qA),
                                       _ptr(qB), _ptr(qC), _ptr(qD), _ptr(site_local),
                                       _ptr(lam_p), _ptr(lam_t), bp, _ptr(out["E"]),
                                       _ptr(out["F"]), _ptr(out["phi"]), _ptr(out["dVdl_p"]),
                                       _ptr(out["dVdl_t"]))
        self._raise(st, "fmm_eval_tautomer_batched")
        return out

    def profile_select(self, phases=None, every: int = 1):
        """Record events only at the boundaries of `phases` (names from PHASES;
        None = all), on every `every`-th evaluation.  Call before profile_start."""
        mask = 0xFFFFFFFF if phases is None else sum(1 << PHASES.index(p) for p in phases)
        self._raise(fmm_profile_select(self.handle, mask, every), "fmm_profile_select")

    def profile_start(self, capacity: int):
        self._raise(fmm_profile(self.handle, 1, capacity), "fmm_profile")

    def profile_stop(self):
        self._raise(fmm_profile(self.handle, 0), "fmm_profile")

    def profile_read(self):
        """{phase: (total_ms, count)} over the evaluations recorded so far."""
        out = np.zeros(2 * len(PHASES))
        self._raise(fmm_profile(self.handle, 2, 0, out), "fmm_profile")
        return {ph: (out[i], int(out[len(PHASES) + i])) for i, ph in enumerate(PHASES)}

    def set_exclusions(self, start, idx):
        """fmm_set_exclusions from host arrays (start: n + 1 offsets, idx: the
        partners); start=None removes the lists."""
        if start is None:
            self._raise(load_library().fmm_set_exclusions(self.handle, 0, None, None),
                        "fmm_set_exclusions")
            return
        st = np.ascontiguousarray(start, dtype=np.int32)
        ix = np.ascontiguousarray(idx, dtype=np.int32)
        self._raise(load_library().fmm_set_exclusions(self.handle, st.size - 1, st.ctypes.data,
                                                      ix.ctypes.data if ix.size else None),
                    "fmm_set_exclusions")

    def info(self):
        """Resolved launch configuration of the plan (see fmm_plan_info)."""
        out = (ctypes.c_int64 * 10)()
        self._raise(load_library().fmm_plan_info(self.handle, ctypes.cast(out, ctypes.c_void_p)),
                    "fmm_plan_info")
        keys = ["m2l_kernel", "m2l_chunk", "m2l_chunks", "m2l_workgroups", "p2p_waves",
                "m2l_lds_bytes", "workspace_bytes", "graph", "p2p_split"]
        return dict(zip(keys, list(out)))

    def m2l_kernel_mode(self):
        return self.info()["m2l_kernel"]

    def sync_check(self):
        st = fmm_sync_check(self.handle)
        self._raise(st, "fmm_sync_check")
