"""Pins of the oracle's emulation of the paper's precision semantics (each
kernel computes and stores in its own type, Sec. 4.1; the runs of Sec. 7):

* with every type FP64 it is the FP64 step (a separately written code path);
* at N = 0, with one type everywhere, a step is the first-order Rusanov
  finite-volume update computed operation by operation in that type by NumPy
  (float32, float16) or torch (bfloat16) -- bit for bit;
* its error levels against FP64 sit at the type's unit roundoff, and a
  mistyped kernel moves them (FP32 error below BF16 error, corrector-only
  errors below all-kernel errors)."""
import math

import numpy as np
import pytest

from _util import small
from oracle import brute

TWO_PI = 2 * math.pi


def _sc(pde, N, cells, params, ic, extra=None, cfl=0.5):
    h = 1.0 / cells[0]
    return small(pde, 2, N, cells, (0.0, 0.0), (cells[0] * h, cells[1] * h), params, ic, extra, cfl)


CASES = {
    "acoustic": _sc("acoustic", 3, (5, 4), (1.0, 1.0), "planar_acoustic", {"k": (TWO_PI, TWO_PI)}),
    "elastic": _sc("elastic", 3, (4, 5), (1.0, 2.0, 1.0), "planar_elastic", {"kP": TWO_PI, "kS": TWO_PI}),
    "euler": _sc("euler", 3, (5, 4), (1.4,), "euler_density_wave"),
    "swe": _sc("swe", 3, (5, 4), (9.81,), "swe_bump"),
}


def _oracle(oracle_mod, sc, prec=("fp64",) * 3, storage="fp64", semantics="build", prec_picard=None, cells=None):
    cells = cells or sc.cells
    return oracle_mod.Oracle(sc.dim, sc.order, cells, sc.lo, sc.hi, sc.pde, sc.params, prec=prec, storage=storage,
                             semantics=semantics, prec_picard=prec_picard)


@pytest.mark.parametrize("name", list(CASES))
def test_paper_semantics_in_fp64_is_the_fp64_step(oracle_mod, name):
    sc = CASES[name]
    a = _oracle(oracle_mod, sc)
    b = _oracle(oracle_mod, sc, semantics="paper")
    Q0 = sc.initial_state(a.node_coords())
    Q0 = Q0 + 1e-3 * np.abs(Q0).max() * np.random.default_rng(1).standard_normal(Q0.shape) * (name != "swe")
    a.set_state(Q0)
    b.set_state(Q0)
    dt = a.max_dt(sc.cfl)
    A = a.run(3, dt)
    B = b.run(3, dt)
    rel = np.abs(B - A).max() / np.abs(A).max()
    assert rel <= 1e-13, rel
    assert np.abs(B - Q0).max() > 1e-6 * np.abs(Q0).max()  # the state moved


def _acoustic_fv(xp, dtype, K, rho):
    Kp, rp = (np.asarray(K, dtype=dtype), np.asarray(rho, dtype=dtype)) if xp is np else \
        (xp.tensor(K, dtype=dtype), xp.tensor(rho, dtype=dtype))

    def flux(q, j):
        out = [Kp * q[1 + j]] + [q[0] / rp if i == j else q[0] * 0 for i in range(2)]
        return xp.stack(out)

    def speed(q, j):
        s = xp.sqrt(Kp / rp)
        return s + q[0] * 0

    return flux, speed


def _euler_fv(xp, dtype, gamma):
    g = np.asarray(gamma, dtype=dtype) if xp is np else xp.tensor(gamma, dtype=dtype)
    one = np.asarray(1.0, dtype=dtype) if xp is np else xp.tensor(1.0, dtype=dtype)
    half = np.asarray(0.5, dtype=dtype) if xp is np else xp.tensor(0.5, dtype=dtype)

    def pressure(q):
        ke = q[1] * q[1] + q[2] * q[2]
        return (g - one) * (q[3] - (half * ke) / q[0])

    def flux(q, j):
        p = pressure(q)
        uj = q[1 + j] / q[0]
        return xp.stack([q[1 + j], q[1] * uj + p if j == 0 else q[1] * uj,
                         q[2] * uj + p if j == 1 else q[2] * uj, uj * (q[3] + p)])

    def speed(q, j):
        return xp.abs(q[1 + j] / q[0]) + xp.sqrt((g * pressure(q)) / q[0])

    return flux, speed


@pytest.mark.parametrize("pde", ["acoustic", "euler"])
@pytest.mark.parametrize("p", ["fp32", "fp16", "bf16"])
def test_paper_semantics_at_order_zero_is_typed_finite_volumes(oracle_mod, pde, p):
    if pde == "acoustic":
        sc = _sc("acoustic", 0, (7, 5), (1.3, 2.1), "planar_acoustic", {"k": (TWO_PI, TWO_PI)})
    else:
        sc = _sc("euler", 0, (7, 5), (1.4,), "euler_density_wave")
    o = _oracle(oracle_mod, sc, prec=(p,) * 3, storage=p, semantics="paper")
    Q0 = sc.initial_state(o.node_coords())
    if pde == "acoustic":
        Q0 = Q0 + 0.3 * np.random.default_rng(5).standard_normal(Q0.shape)
    # start from values of the type (both sides read the same numbers)
    Q0 = np.vectorize(lambda x: oracle_mod.round_p(p, x))(Q0)
    o.set_state(Q0)
    dt = 0.4 * o.h / (2 * 3.0)
    A = o.run(2, dt)
    # the same two steps with NumPy / torch in the type: U[V, C0, C1]
    C0, C1 = sc.cells
    U = Q0[:, :, 0].reshape(C1, C0, -1).transpose(2, 1, 0)
    if p == "bf16":
        import torch
        xp, dt_ = torch, torch.bfloat16
        U = torch.from_numpy(np.ascontiguousarray(U)).to(dt_)
    else:
        xp, dt_ = np, {"fp32": np.float32, "fp16": np.float16}[p]
        U = U.astype(dt_)
    flux, speed = _acoustic_fv(xp, dt_, sc.params[1], sc.params[0]) if pde == "acoustic" else _euler_fv(xp, dt_, 1.4)
    for _ in range(2):
        U = brute.fv_rusanov_step_typed(U, dt, o.h, flux, speed, xp, dt_)
    Ub = U.float().numpy().astype(np.float64) if p == "bf16" else U.astype(np.float64)
    B = Ub.transpose(2, 1, 0).reshape(C0 * C1, -1)[:, :, None]
    np.testing.assert_array_equal(A, B)


def test_paper_semantics_error_levels(oracle_mod):
    """Acoustic planar wave, 6^2 cells, N = 3, 20 steps: the error of each typed run
    against FP64 sits at its type's unit roundoff and orders as the types do."""
    sc = _sc("acoustic", 3, (6, 6), (1.0, 1.0), "planar_acoustic", {"k": (TWO_PI, TWO_PI)})
    ref = _oracle(oracle_mod, sc)
    Q0 = sc.initial_state(ref.node_coords())
    ref.set_state(Q0)
    dt = ref.max_dt(sc.cfl)
    A = ref.run(20, dt)

    def err(**kw):
        o = _oracle(oracle_mod, sc, semantics="paper", **kw)
        o.set_state(Q0)
        B = o.run(20, dt)
        return ref.l2(B, A) / ref.l2(A)

    e32 = err(prec=("fp32",) * 3, storage="fp32")
    e16 = err(prec=("fp16",) * 3, storage="fp32")
    eb16 = err(prec=("bf16",) * 3, storage="fp32")
    ecorr = err(prec=("fp64", "fp64", "bf16"), storage="fp64")
    epic = err(prec=("fp64", "fp64", "fp64"), prec_picard="bf16", storage="fp64")
    print("paper-semantics levels: fp32 %.2e fp16 %.2e bf16 %.2e corrector-bf16 %.2e picard-bf16 %.2e"
          % (e32, e16, eb16, ecorr, epic))
    assert 1e-8 < e32 < 1e-5
    assert 1e-5 < e16 < 3e-2 and e16 > 10 * e32
    assert eb16 > 2 * e16
    assert 1e-5 < ecorr < eb16 and 1e-5 < epic
