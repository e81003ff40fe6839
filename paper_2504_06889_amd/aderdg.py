"""Python binding of libaderdg.so (argument marshalling only).

Every step of the ADER-DG path runs in the library's HIP kernels; PyTorch is
used for device memory and the HIP stream.  The library must be built
(``python -m paper_2504_06889_amd.build``); importing this module on a
machine without it raises instead of falling back to anything else.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libaderdg.so")

PDE = {"acoustic": 0, "elastic": 1, "euler": 2, "swe": 3}
KERNEL = {"predictor": 0, "volume": 1, "flux": 2, "storage": 3}
PREC = {"fp64": 0, "fp32": 1, "bf16": 2, "fp16": 3}
STATUS = {0: "OK", -1: "INVALID", -2: "UNSUPPORTED", -3: "OOM", -4: "DEVICE", -5: "NONFINITE"}


class AderdgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (STATUS.get(code, code), msg))
        self.code = code


class NonFiniteError(AderdgError):
    pass


class _Config(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("order", ctypes.c_int), ("cells", ctypes.c_int * 3),
                ("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3), ("pde", ctypes.c_int),
                ("params", ctypes.c_double * 8), ("picard_iters", ctypes.c_int)]


EXPORTS = [
    "aderdg_create", "aderdg_destroy", "aderdg_set_state", "aderdg_get_state", "aderdg_set_material",
    "aderdg_set_precision", "aderdg_max_dt", "aderdg_step", "aderdg_set_time", "aderdg_get_time",
    "aderdg_set_source", "aderdg_set_receivers", "aderdg_read_receivers", "aderdg_step_adjoint",
    "aderdg_receivers_adjoint", "aderdg_nodes", "aderdg_info", "aderdg_state_ptr", "aderdg_last_error",
    "aderdg_set_timing", "aderdg_get_timing", "aderdg_copy_faces", "aderdg_step_adjoint_faces",
    "aderdg_set_predictor", "aderdg_step_adjoint_faces_noalloc",
]
PREDICTORS = {"picard": 0, "ck": 1}

_lib = None


def lib():
    """Load libaderdg.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libaderdg.so is not built (run python -m paper_2504_06889_amd.build)")
    L = ctypes.CDLL(LIB_PATH)
    vp, dp, i, d = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int, ctypes.c_double
    sig = {
        "aderdg_create": [ctypes.POINTER(_Config), vp, ctypes.POINTER(vp)],
        "aderdg_destroy": [vp],
        "aderdg_set_state": [vp, vp, i],
        "aderdg_get_state": [vp, vp, i],
        "aderdg_set_material": [vp, vp, i],
        "aderdg_set_precision": [vp, i, i],
        "aderdg_max_dt": [vp, d, dp],
        "aderdg_step": [vp, d, i],
        "aderdg_set_time": [vp, d],
        "aderdg_get_time": [vp, dp],
        "aderdg_set_source": [vp, dp, d, d, d],
        "aderdg_set_receivers": [vp, i, dp],
        "aderdg_read_receivers": [vp, vp, i],
        "aderdg_step_adjoint": [vp, d, d, vp, vp, vp],
        "aderdg_receivers_adjoint": [vp, vp, vp],
        "aderdg_nodes": [i, dp, dp],
        "aderdg_info": [vp, ctypes.POINTER(ctypes.c_longlong)],
        "aderdg_state_ptr": [vp, ctypes.POINTER(vp)],
        "aderdg_last_error": [vp],
        "aderdg_set_timing": [vp, i],
        "aderdg_get_timing": [vp, dp],
        "aderdg_copy_faces": [vp, vp, i],
        "aderdg_step_adjoint_faces": [vp, d, d, vp, vp, vp, vp],
        "aderdg_set_predictor": [vp, i],
        "aderdg_step_adjoint_faces_noalloc": [vp, d, d, vp, vp, vp, vp],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_char_p if name == "aderdg_last_error" else ctypes.c_int
    _lib = L
    return L


def nodes(n):
    """Gauss-Legendre nodes and weights on [0, 1] as built by the library."""
    xi, w = np.zeros(n), np.zeros(n)
    rc = lib().aderdg_nodes(n, xi.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                            w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    if rc != 0:
        raise AderdgError(rc, "bad node count")
    return xi, w


def _torch():
    import torch
    return torch


def check_tensor(x, name, numel, dtype="float64", device=None):
    """Validate a tensor before its pointer goes to the library: dtype, contiguity
    and element count first (these checks need no GPU), then that it lives on the
    solver's device.  Raises ValueError; nothing is launched."""
    return check_tensors([(x, name, numel, dtype)], device)[0]


def check_tensors(items, device=None):
    """check_tensor over (tensor, name, numel[, dtype]) items: the host-side
    checks of every item before the device checks of any."""
    torch = _torch()
    for it in items:
        x, name, numel = it[:3]
        dtype = it[3] if len(it) > 3 else "float64"
        if not isinstance(x, torch.Tensor):
            raise ValueError("%s must be a torch tensor, got %s" % (name, type(x).__name__))
        if x.dtype != getattr(torch, dtype):
            raise ValueError("%s must be %s, got %s" % (name, dtype, x.dtype))
        if not x.is_contiguous():
            raise ValueError("%s must be contiguous" % name)
        if x.numel() != numel:
            raise ValueError("%s must hold %d elements, got %d" % (name, numel, x.numel()))
    for it in items:
        x, name = it[:2]
        if not x.is_cuda:
            raise ValueError("%s must be a device (CUDA/HIP) tensor" % name)
        if device is not None and x.device.index != device:
            raise ValueError("%s is on device %s, the solver on cuda:%d" % (name, x.device, device))
    return [it[0] for it in items]


class Solver:
    """One ADER-DG solver on the current HIP device and stream (see include/aderdg.h)."""

    def __init__(self, dim, order, cells, lo, hi, pde, params, picard_iters=0, stream=None):
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the ADER-DG library runs on the GPU only")
        c = _Config()
        c.dim, c.order = dim, order
        cells = list(cells) + [1] * (3 - len(cells))
        lo = list(lo) + [0.0] * (3 - len(lo))
        hi = list(hi) + [1.0] * (3 - len(hi))
        for k in range(3):
            c.cells[k], c.lo[k], c.hi[k] = int(cells[k]), float(lo[k]), float(hi[k])
        c.pde = PDE[pde] if isinstance(pde, str) else int(pde)
        params = list(params) + [0.0] * (8 - len(params))
        for k in range(8):
            c.params[k] = float(params[k])
        c.picard_iters = int(picard_iters)
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        self.device = torch.cuda.current_device()
        handle = ctypes.c_void_p()
        rc = lib().aderdg_create(ctypes.byref(c), ctypes.c_void_p(stream.cuda_stream), ctypes.byref(handle))
        if rc != 0:
            raise AderdgError(rc, lib().aderdg_last_error(None).decode())
        self._h = handle
        info = (ctypes.c_longlong * 8)()
        lib().aderdg_info(self._h, info)
        self.n, self.d, self.V, self.S, self.F, self.iters, self.ncell = [int(x) for x in info[:7]]
        self.dim, self.order, self.pde = dim, order, pde
        self.cells = cells[:dim]
        self.lo, self.hi = lo[:dim], hi[:dim]
        self.h = (hi[0] - lo[0]) / cells[0]

    @classmethod
    def from_scenario(cls, sc, cells=None, picard_iters=0, stream=None):
        return cls(sc.dim, sc.order, cells or sc.cells, sc.lo, sc.hi, sc.pde, sc.params,
                   picard_iters=picard_iters, stream=stream)

    def close(self):
        if getattr(self, "_h", None):
            lib().aderdg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != 0:
            msg = lib().aderdg_last_error(self._h).decode()
            if rc == -5:
                raise NonFiniteError(rc, msg)
            raise AderdgError(rc, msg)

    @property
    def shape(self):
        return (self.ncell, self.V, self.S)

    def _state_numel(self):
        return self.ncell * self.V * self.S

    # -- state ---------------------------------------------------------------
    def set_state(self, Q):
        torch = _torch()
        if isinstance(Q, torch.Tensor) and Q.is_cuda:
            check_tensor(Q, "Q", self._state_numel(), device=self.device)
            self._check(lib().aderdg_set_state(self._h, ctypes.c_void_p(Q.data_ptr()), 1))
        else:
            Qh = np.ascontiguousarray(Q, dtype=np.float64)
            assert Qh.shape == self.shape, (Qh.shape, self.shape)
            self._check(lib().aderdg_set_state(self._h, ctypes.c_void_p(Qh.ctypes.data), 0))

    def get_state(self, out=None):
        """Copy the state out: into `out` (a CUDA float64 tensor) or a new numpy array."""
        torch = _torch()
        if out is not None and isinstance(out, torch.Tensor):
            check_tensor(out, "out", self._state_numel(), device=self.device)
            self._check(lib().aderdg_get_state(self._h, ctypes.c_void_p(out.data_ptr()), 1))
            return out
        Qh = np.empty(self.shape)
        self._check(lib().aderdg_get_state(self._h, ctypes.c_void_p(Qh.ctypes.data), 0))
        return Qh

    def set_material(self, c):
        torch = _torch()
        if isinstance(c, torch.Tensor) and c.is_cuda:
            check_tensor(c, "c", self.ncell, device=self.device)
            self._check(lib().aderdg_set_material(self._h, ctypes.c_void_p(c.data_ptr()), 1))
        else:
            ch = np.ascontiguousarray(c, dtype=np.float64).reshape(-1)
            if ch.size != self.ncell:
                raise ValueError("c must hold %d values, got %d" % (self.ncell, ch.size))
            self._check(lib().aderdg_set_material(self._h, ctypes.c_void_p(ch.ctypes.data), 0))

    def set_precision(self, kernel, prec):
        k = KERNEL[kernel] if isinstance(kernel, str) else int(kernel)
        p = PREC[prec] if isinstance(prec, str) else int(prec)
        self._check(lib().aderdg_set_precision(self._h, k, p))

    def set_predictor(self, kind):
        """"picard" (eq. Picard) or "ck" (Cauchy-Kowalevskaya, linear PDEs)."""
        self._check(lib().aderdg_set_predictor(self._h, PREDICTORS[kind] if isinstance(kind, str) else int(kind)))
        self.predictor = kind

    def set_precisions(self, predictor="fp64", volume="fp64", flux="fp64"):
        self.set_precision("predictor", predictor)
        self.set_precision("volume", volume)
        self.set_precision("flux", flux)

    def max_dt(self, cfl):
        dt = ctypes.c_double()
        self._check(lib().aderdg_max_dt(self._h, float(cfl), ctypes.byref(dt)))
        return dt.value

    def step(self, dt, nsteps=1):
        self._check(lib().aderdg_step(self._h, float(dt), int(nsteps)))

    @property
    def time(self):
        t = ctypes.c_double()
        self._check(lib().aderdg_get_time(self._h, ctypes.byref(t)))
        return t.value

    @time.setter
    def time(self, t):
        self._check(lib().aderdg_set_time(self._h, float(t)))

    def set_timing(self, enable=True):
        self._check(lib().aderdg_set_timing(self._h, 1 if enable else 0))

    def get_timing(self):
        """Kernel times since timing was enabled: total ms of the separate predictor and
        corrector launches, of the fused (corrector + predictor) launches, their counts
        and the number of steps."""
        out = (ctypes.c_double * 5)()
        self._check(lib().aderdg_get_timing(self._h, out))
        return {"predictor_ms": out[0], "corrector_ms": out[1], "steps": int(out[2]), "fused_ms": out[3],
                "fused_launches": int(out[4])}

    # -- source and receivers ---------------------------------------------------
    def set_source(self, x, f0, t0, amp=1.0):
        xs = (ctypes.c_double * 3)(*(list(map(float, x)) + [0.0] * (3 - len(x))))
        self._check(lib().aderdg_set_source(self._h, xs, float(f0), float(t0), float(amp)))

    def set_receivers(self, xyz):
        xyz = np.asarray(xyz, dtype=np.float64).reshape(-1, self.d)
        pts = np.zeros((xyz.shape[0], 3))
        pts[:, :self.d] = xyz
        self.nrec = xyz.shape[0]
        self._check(lib().aderdg_set_receivers(self._h, self.nrec,
                                               pts.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))

    def read_receivers(self, out=None):
        if out is not None:
            check_tensor(out, "out", self.nrec, device=self.device)
            self._check(lib().aderdg_read_receivers(self._h, ctypes.c_void_p(out.data_ptr()), 1))
            return out
        r = np.zeros(self.nrec)
        self._check(lib().aderdg_read_receivers(self._h, ctypes.c_void_p(r.ctypes.data), 0))
        return r

    # -- adjoint ------------------------------------------------------------------
    def face_bytes(self):
        """Bytes of the face buffer (all cells) in the current FLUX format."""
        info = (ctypes.c_longlong * 8)()
        lib().aderdg_info(self._h, info)
        return int(info[7]) * self.ncell

    def copy_faces(self, out):
        """Copy the last step's face data into `out` (a CUDA uint8 tensor of face_bytes())."""
        nb = self.face_bytes()
        check_tensor(out, "out", out.numel(), dtype="uint8", device=self.device)
        if out.numel() < nb:
            raise ValueError("out must hold at least %d bytes, got %d" % (nb, out.numel()))
        self._check(lib().aderdg_copy_faces(self._h, ctypes.c_void_p(out.data_ptr()), 1))
        return out

    def step_adjoint(self, dt, t, Qn, lam, grad, fwd_faces=None):
        """lam <- (step Jacobian)^T lam, grad += d<lam, step(Qn)>/dc (device tensors).
        fwd_faces: the face data copied right after the forward step from Qn (else they
        are recomputed from Qn)."""
        check_tensors([(Qn, "Qn", self._state_numel()), (lam, "lam", self._state_numel()),
                       (grad, "grad", self.ncell)], self.device)
        if fwd_faces is None:
            self._check(lib().aderdg_step_adjoint(self._h, float(dt), float(t), ctypes.c_void_p(Qn.data_ptr()),
                                                  ctypes.c_void_p(lam.data_ptr()),
                                                  ctypes.c_void_p(grad.data_ptr())))
        else:
            check_tensor(fwd_faces, "fwd_faces", fwd_faces.numel(), dtype="uint8", device=self.device)
            if fwd_faces.numel() < self.face_bytes():
                raise ValueError("fwd_faces must hold at least %d bytes" % self.face_bytes())
            self._check(lib().aderdg_step_adjoint_faces(
                self._h, float(dt), float(t), ctypes.c_void_p(Qn.data_ptr()), ctypes.c_void_p(fwd_faces.data_ptr()),
                ctypes.c_void_p(lam.data_ptr()), ctypes.c_void_p(grad.data_ptr())))

    def step_adjoint_noalloc(self, dt, t, Qn, lam, grad, fwd_faces):
        """step_adjoint with the forward face data given, through the entry point that
        allocates no device memory (the library's static scratch array; small grids)."""
        check_tensors([(Qn, "Qn", self._state_numel()), (lam, "lam", self._state_numel()),
                       (grad, "grad", self.ncell), (fwd_faces, "fwd_faces", fwd_faces.numel(), "uint8")],
                      self.device)
        if fwd_faces.numel() < self.face_bytes():
            raise ValueError("fwd_faces must hold at least %d bytes" % self.face_bytes())
        self._check(lib().aderdg_step_adjoint_faces_noalloc(
            self._h, float(dt), float(t), ctypes.c_void_p(Qn.data_ptr()), ctypes.c_void_p(fwd_faces.data_ptr()),
            ctypes.c_void_p(lam.data_ptr()), ctypes.c_void_p(grad.data_ptr())))

    def receivers_adjoint(self, weight, lam):
        """lam[cell][0][node] += sum_r weight[r] phi_node(x_r) (device tensors)."""
        check_tensors([(weight, "weight", getattr(self, "nrec", 0)), (lam, "lam", self._state_numel())],
                      self.device)
        self._check(lib().aderdg_receivers_adjoint(self._h, ctypes.c_void_p(weight.data_ptr()),
                                                   ctypes.c_void_p(lam.data_ptr())))

    # -- geometry -------------------------------------------------------------------
    def node_coords(self):
        xi, _ = nodes(self.n)
        return [self.lo[j] + self.h * (np.arange(self.cells[j])[:, None] + xi[None, :])
                for j in range(self.d)]

    def weights(self):
        _, w = nodes(self.n)
        W = np.ones(1)
        for _ in range(self.d):
            W = np.multiply.outer(w, W).reshape(-1)
        return W
