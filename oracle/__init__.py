"""FP64 CPU oracle of the ADER-DG time step (arXiv 2504.06889, Sec. 3).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The product library
(``paper_2504_06889_amd``) never imports or links it, and it imports nothing
from the product.

``aderdg_oracle.c`` is the step itself (plain loops, FP64); ``brute.py`` holds
independent NumPy brute-force checks (a dense space-time solve, the N = 0
finite-volume scheme) used to pin it.  Functions without such a pin are
marked "parity unpinned" where they are defined.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "aderdg_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

ACOUSTIC, ELASTIC, EULER, SWE = 0, 1, 2, 3
FP64, FP32, BF16, FP16 = 0, 1, 2, 3
PDE_IDS = {"acoustic": ACOUSTIC, "elastic": ELASTIC, "euler": EULER, "swe": SWE}
PREC_IDS = {"fp64": FP64, "fp32": FP32, "bf16": BF16, "fp16": FP16}


def build(force=False):
    """Compile the oracle with gcc (-O3, OpenMP, no FMA contraction)."""
    if not force and os.path.exists(_LIB_PATH) and os.path.getmtime(_LIB_PATH) >= max(
            os.path.getmtime(_SRC), os.path.getmtime(os.path.join(_HERE, "aderdg_oracle.h"))):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O3", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
           _SRC, "-o", tmp, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Config(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("order", ctypes.c_int), ("cells", ctypes.c_int * 3),
                ("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3), ("pde", ctypes.c_int),
                ("params", ctypes.c_double * 8), ("picard_iters", ctypes.c_int),
                ("prec", ctypes.c_int * 3), ("predictor", ctypes.c_int), ("storage", ctypes.c_int),
                ("semantics", ctypes.c_int), ("prec_picard", ctypes.c_int)]

PREDICTORS = {"picard": 0, "ck": 1}


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        vp = ctypes.c_void_p
        L.or_round.restype = ctypes.c_double
        L.or_round.argtypes = [ctypes.c_int, ctypes.c_double]
        L.or_basis.argtypes = [ctypes.c_int] + [dp] * 10
        L.or_nvars.argtypes = [ctypes.c_int, ctypes.c_int]
        L.or_create.restype = vp
        L.or_create.argtypes = [ctypes.POINTER(_Config)]
        L.or_destroy.argtypes = [vp]
        L.or_set_state.argtypes = [vp, dp]
        L.or_get_state.argtypes = [vp, dp]
        L.or_set_material.argtypes = [vp, dp]
        L.or_set_source.argtypes = [vp, dp, ctypes.c_double, ctypes.c_double, ctypes.c_double]
        L.or_max_eig.restype = ctypes.c_double
        L.or_max_eig.argtypes = [vp]
        L.or_max_dt.restype = ctypes.c_double
        L.or_max_dt.argtypes = [vp, ctypes.c_double]
        L.or_predict_cell.argtypes = [vp, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                      dp, dp, dp, dp]
        L.or_step.argtypes = [vp, ctypes.c_double, ctypes.c_double]
        L.or_step_cells.argtypes = [vp, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                    ctypes.POINTER(ctypes.c_int64), dp]
        L.or_sample_points.argtypes = [vp, ctypes.c_int, dp, ctypes.c_int, dp]
        L.or_info.argtypes = [vp, ctypes.POINTER(ctypes.c_int)]
        L.or_cell_size.restype = ctypes.c_double
        L.or_cell_size.argtypes = [vp]
        L.or_num_threads.restype = ctypes.c_int
        L.or_set_num_threads.argtypes = [ctypes.c_int]
        L.or_adjoint_step.argtypes = [vp, dp, ctypes.c_double, ctypes.c_double, dp, dp, dp]
        L.or_point_weights.argtypes = [vp, dp, ctypes.POINTER(ctypes.c_int64), dp]
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def round_p(p, x):
    """Round x to format p (FP32 first, then p; RNE), as the emulated mode does."""
    p = PREC_IDS.get(p, p)
    return lib().or_round(int(p), float(x))


def basis(n):
    """Gauss-Legendre nodes/weights on [0,1] and the derived operators (Sec. 3).

    D[i, j] = psi_j'(xi_i); F0/F1 = psi(0)/psi(1); K1 = the time matrix of
    eq. Picard; Atau = K1^{-1} diag(w); Kxi[k, l] = w_l D[l, k] / w_k (weak-form
    volume); L0/L1 = F0/w, F1/w (face lifts)."""
    out = {k: np.zeros(n) for k in ("xi", "w", "F0", "F1", "L0", "L1")}
    out.update({k: np.zeros((n, n)) for k in ("D", "K1", "Atau", "Kxi")})
    rc = lib().or_basis(n, *[_ptr(out[k]) for k in
                             ("xi", "w", "D", "F0", "F1", "K1", "Atau", "Kxi", "L0", "L1")])
    if rc != 0:
        raise ValueError("unsupported number of nodes %d" % n)
    return out


def num_threads():
    """OpenMP threads the oracle's loops use."""
    return lib().or_num_threads()


def set_num_threads(n):
    """Threads the oracle's loops use from now on."""
    lib().or_set_num_threads(int(n))


def nvars(pde, dim):
    return lib().or_nvars(PDE_IDS.get(pde, pde), dim)


class Oracle:
    """FP64 CPU ADER-DG on a periodic Cartesian grid (state layout [cell][var][node])."""

    def __init__(self, dim, order, cells, lo, hi, pde, params, picard_iters=0,
                 prec=(FP64, FP64, FP64), predictor="picard", storage="fp64", semantics="build",
                 prec_picard=None):
        c = _Config()
        c.dim, c.order = dim, order
        cells = list(cells) + [1] * (3 - len(cells))
        lo = list(lo) + [0.0] * (3 - len(lo))
        hi = list(hi) + [1.0] * (3 - len(hi))
        for i in range(3):
            c.cells[i], c.lo[i], c.hi[i] = cells[i], lo[i], hi[i]
        c.pde = PDE_IDS.get(pde, pde)
        params = list(params) + [0.0] * (8 - len(params))
        for i in range(8):
            c.params[i] = params[i]
        c.picard_iters = picard_iters
        for i in range(3):
            c.prec[i] = PREC_IDS.get(prec[i], prec[i])
        c.predictor = PREDICTORS[predictor]
        self.predictor = predictor
        c.storage = PREC_IDS.get(storage, storage)
        self.storage = storage
        # "build": contraction inputs rounded, FP32 accumulation (the GPU path's
        # semantics); "paper": each kernel computes and stores in its type
        # (prec[0] predictor kernel, prec_picard its Picard loop, prec[2] corrector)
        c.semantics = {"build": 0, "paper": 1}[semantics]
        c.prec_picard = -1 if prec_picard is None else PREC_IDS.get(prec_picard, prec_picard)
        self.semantics = semantics
        self._cfg = c
        self._h = lib().or_create(ctypes.byref(c))
        if not self._h:
            raise ValueError("invalid oracle configuration")
        info = (ctypes.c_int * 7)()
        lib().or_info(self._h, info)
        self.n, self.d, self.V, self.S, self.F, self.I, self.ncell = list(info)
        self.h = lib().or_cell_size(self._h)
        self.dim, self.order = dim, order
        self.cells = cells[:dim]
        self.lo, self.hi = lo[:dim], hi[:dim]

    def __del__(self):
        if getattr(self, "_h", None):
            lib().or_destroy(self._h)
            self._h = None

    @property
    def shape(self):
        return (self.ncell, self.V, self.S)

    def set_state(self, Q):
        Q = np.ascontiguousarray(Q, dtype=np.float64)
        assert Q.shape == self.shape, (Q.shape, self.shape)
        lib().or_set_state(self._h, _ptr(Q))

    def get_state(self):
        Q = np.empty(self.shape)
        lib().or_get_state(self._h, _ptr(Q))
        return Q

    def set_material(self, c_per_cell):
        c = np.ascontiguousarray(c_per_cell, dtype=np.float64).reshape(-1)
        assert c.size == self.ncell
        if lib().or_set_material(self._h, _ptr(c)) != 0:
            raise ValueError("material only for acoustics")

    def set_source(self, x, f0, t0, amp=1.0):
        x = np.ascontiguousarray(list(x) + [0.0] * (3 - len(x)), dtype=np.float64)
        if lib().or_set_source(self._h, _ptr(x), f0, t0, amp) != 0:
            raise ValueError("bad source")

    def max_eig(self):
        return lib().or_max_eig(self._h)

    def max_dt(self, cfl):
        return lib().or_max_dt(self._h, cfl)

    def step(self, t, dt):
        if lib().or_step(self._h, t, dt) != 0:
            raise MemoryError("oracle step failed")

    def run(self, nsteps, dt, t0=0.0):
        for k in range(nsteps):
            self.step(t0 + k * dt, dt)
        return self.get_state()

    def predict_cell(self, cell, t, dt):
        """Predictor outputs of one cell: final iterate [n][V][S], qbar, fbar[d], nbar."""
        qst = np.zeros((self.n, self.V, self.S))
        qbar = np.zeros((self.V, self.S))
        fbar = np.zeros((self.d, self.V, self.S))
        nbar = np.zeros((self.V, self.S))
        lib().or_predict_cell(self._h, cell, t, dt, _ptr(qst), _ptr(qbar), _ptr(fbar), _ptr(nbar))
        return qst, qbar, fbar, nbar

    def step_cells(self, t, dt, ids):
        """One step evaluated at the listed cells only (state unchanged)."""
        ids = np.ascontiguousarray(ids, dtype=np.int64)
        out = np.zeros((ids.size, self.V, self.S))
        rc = lib().or_step_cells(self._h, t, dt, int(ids.size),
                                 ids.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _ptr(out))
        if rc != 0:
            raise ValueError("bad cell id")
        return out

    def sample_points(self, xyz, var=0):
        xyz = np.asarray(xyz, dtype=np.float64).reshape(-1, self.d)
        pts = np.zeros((xyz.shape[0], 3))
        pts[:, :self.d] = xyz
        out = np.zeros(xyz.shape[0])
        if lib().or_sample_points(self._h, xyz.shape[0], _ptr(pts), var, _ptr(out)) != 0:
            raise ValueError("point outside the domain")
        return out

    def adjoint_step(self, Qn, t, dt, lam, grad):
        """Reverse-mode adjoint of one step (acoustics with material): returns
        (J^T lam, grad + d<lam, step(Qn)>/dc).  Qn is the state at the step start.
        With the predictor and volume precisions both below FP64 (flux FP64) the
        transposed contractions run in those formats (emulated, FP32 accumulation)."""
        Qn = np.ascontiguousarray(Qn, dtype=np.float64)
        lam = np.ascontiguousarray(lam, dtype=np.float64)
        mu = np.zeros_like(lam)
        g = np.array(grad, dtype=np.float64, copy=True)
        if lib().or_adjoint_step(self._h, _ptr(Qn), t, dt, _ptr(lam), _ptr(mu), _ptr(g)) != 0:
            raise ValueError("adjoint needs acoustics with a material, the Picard predictor, "
                             "FP64 storage and flux, and predictor and volume both FP64 or both lower")
        return mu, g

    def point_weights(self, x):
        """(cell, phi[S]) of point x: the receiver read-out is sum_k phi_k Q[cell, 0, k]."""
        xx = np.zeros(3)
        xx[:self.d] = x
        cell = ctypes.c_int64()
        w = np.zeros(self.S)
        if lib().or_point_weights(self._h, _ptr(xx), ctypes.byref(cell), _ptr(w)) != 0:
            raise ValueError("point outside the domain")
        return cell.value, w

    def node_coords(self):
        """Physical coordinates of the nodes along each dimension, [C_j, n]."""
        xi = basis(self.n)["xi"]
        return [self.lo[j] + self.h * (np.arange(self.cells[j])[:, None] + xi[None, :])
                for j in range(self.d)]

    def weights(self):
        """Gauss weights of the nodes in a cell, [S] (x fastest)."""
        w = basis(self.n)["w"]
        W = np.ones(1)
        for _ in range(self.d):
            W = np.multiply.outer(w, W).reshape(-1)
        return W

    def l2(self, A, B=None):
        """L2 norm of eq. L2gauss, sqrt(sum h^d W_i (A - B)^2) over cells/nodes/vars."""
        diff = A if B is None else A - B
        W = self.weights()
        return float(np.sqrt(np.sum((diff ** 2) * W[None, None, :]) * self.h ** self.d))
