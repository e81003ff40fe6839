"""Pins of the oracle's storage precision (the persistent state held in FP32, BF16 or
FP16 between traversals, Sec. 4.1): FP64 storage is the plain step; every stored
value is representable in the format; at N = 0 a step is the textbook Rusanov
finite-volume update rounded to the format (independent code and rounding); the
difference to FP64 storage stays at the level of the format's spacing."""
import math

import numpy as np
import pytest

from _util import small

EPS = {"fp32": 2.0 ** -24, "bf16": 2.0 ** -8, "fp16": 2.0 ** -11}


def _oracle(oracle_mod, sc, storage):
    return oracle_mod.Oracle(sc.dim, sc.order, sc.cells, sc.lo, sc.hi, sc.pde, sc.params, storage=storage)


def _wave():
    return small("acoustic", 2, 3, (6, 5), (0.0, 0.0), (1.0, 5 / 6), (1.0, 1.0), "planar_acoustic",
                 {"k": (2 * math.pi, 0.0)}, cfl=0.7)


def test_fp64_storage_is_the_plain_step(oracle_mod):
    sc = _wave()
    a = oracle_mod.Oracle(sc.dim, sc.order, sc.cells, sc.lo, sc.hi, sc.pde, sc.params)
    b = _oracle(oracle_mod, sc, "fp64")
    Q = sc.initial_state(a.node_coords())
    a.set_state(Q)
    b.set_state(Q)
    dt = a.max_dt(sc.cfl)
    np.testing.assert_array_equal(a.run(3, dt), b.run(3, dt))


@pytest.mark.parametrize("p", ["fp32", "bf16", "fp16"])
def test_stored_values_are_in_the_format(oracle_mod, p):
    sc = _wave()
    o = _oracle(oracle_mod, sc, p)
    o.set_state(sc.initial_state(o.node_coords()))
    A = o.run(3, o.max_dt(sc.cfl))
    R = np.vectorize(lambda x: oracle_mod.round_p(p, x))(A)
    np.testing.assert_array_equal(R, A)
    assert np.abs(A).max() > 0


@pytest.mark.parametrize("p", ["bf16", "fp16", "fp32"])
def test_order_zero_is_rounded_textbook_finite_volumes(oracle_mod, p):
    """At N = 0 the step is the Rusanov finite-volume update (brute.py); with a
    storage format the state is that update rounded to the format (numpy's own
    float16 / the bfloat16 bit rounding below), every step."""
    from oracle import brute
    import torch
    K, rho = 2.0, 0.5
    cells = (5, 4)
    o = oracle_mod.Oracle(2, 0, cells, (0.0, 0.0), (1.0, 0.8), "acoustic", (rho, K), storage=p)
    def rnd(x):
        x32 = np.asarray(x, dtype=np.float32)
        if p == "fp16":
            return x32.astype(np.float16).astype(np.float64)
        if p == "bf16":
            return torch.from_numpy(x32).to(torch.bfloat16).to(torch.float64).numpy()
        return x32.astype(np.float64)
    U = rnd(np.random.default_rng(7).standard_normal((3,) + cells[::-1]))
    fl = [(lambda j: (lambda q: np.stack([K * q[1 + j]] + [q[0] / rho if i == j else 0 * q[0]
                                                       for i in range(2)])))(j) for j in range(2)]
    sp = [(lambda q: math.sqrt(K / rho))] * 2
    o.set_state(np.moveaxis(U, 0, -1).reshape(-1, 3, 1))
    dt = 0.1 * o.h
    for k in range(3):
        o.step(k * dt, dt)
        U = rnd(brute.fv_rusanov_step(U, dt, o.h, fl, sp))
    A, B = o.get_state(), np.moveaxis(U, 0, -1).reshape(-1, 3, 1)
    # the two FP64 updates differ by rounding order (1e-16), which can move a
    # value across a rounding boundary of the format: one spacing at most, rarely
    ulp = {"fp32": 2.0 ** -23, "bf16": 2.0 ** -7, "fp16": 2.0 ** -10}[p] * np.abs(B)
    assert np.all(np.abs(A - B) <= ulp)
    assert np.mean(A == B) > 0.9


@pytest.mark.parametrize("p", ["fp32", "bf16", "fp16"])
def test_difference_to_fp64_storage_at_the_format_level(oracle_mod, p):
    sc = _wave()
    a = _oracle(oracle_mod, sc, "fp64")
    b = _oracle(oracle_mod, sc, p)
    Q = sc.initial_state(a.node_coords())
    a.set_state(Q)
    b.set_state(Q)
    dt = a.max_dt(sc.cfl)
    A, B = a.run(4, dt), b.run(4, dt)
    r = a.l2(B, A) / a.l2(A)
    assert 0.01 * EPS[p] < r < 20 * EPS[p], (p, r)
