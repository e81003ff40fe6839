"""GPU parity of the storage precision (the state held between traversals in FP32,
BF16 or FP16) against the oracle's emulation of the same rounding points, and its
plumbing: the FP64 ABI round trip, re-encoding on a change of format, receivers,
max_dt, fused and single steps bit for bit, the adjoint refused."""
import math

import numpy as np
import pytest

from _util import gpu_solver, rel_l2, small

pytestmark = pytest.mark.gpu

TWO_PI = 2 * math.pi
EPS = {"fp32": 2.0 ** -24, "bf16": 2.0 ** -8, "fp16": 2.0 ** -11}


def _grid(pde, dim, N, cells, params, ic, extra, cfl=0.5):
    h = 1.0 / max(cells)
    return small(pde, dim, N, cells, (0.0,) * dim, tuple(c * h for c in cells), params, ic, extra, cfl)


CASES = {
    "elastic3d_n5": (_grid("elastic", 3, 5, (3, 2, 4), (2.7, 32.4, 32.398), "planar_elastic",
                           {"kP": TWO_PI, "kS": TWO_PI}), ("fp16", "fp16", "fp64")),
    "acoustic2d_n3": (_grid("acoustic", 2, 3, (7, 5), (1.0, 1.0), "planar_acoustic", {"k": (TWO_PI, TWO_PI)}, 0.7),
                      ("fp64",) * 3),
    # bf16 contractions: their level sits well above the FP32 noise of the two
    # sides' different accumulation orders, which FP32 storage rounding would see
    "euler2d_n3": (_grid("euler", 2, 3, (5, 7), (1.4,), "euler_density_wave", None, 0.6),
                   ("bf16", "bf16", "fp64")),
    "swe2d_n3": (_grid("swe", 2, 3, (5, 7), (9.81,), "swe_bump", None, 0.45), ("fp64",) * 3),
}


def _oracle(oracle_mod, sc, prec, storage):
    return oracle_mod.Oracle(sc.dim, sc.order, sc.cells, sc.lo, sc.hi, sc.pde, sc.params, prec=prec,
                             storage=storage)


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("sp", ["fp32", "bf16", "fp16"])
def test_storage_matches_oracle_emulation(oracle_mod, name, sp):
    sc, prec = CASES[name]
    print("case", name, sp, flush=True)
    ref = _oracle(oracle_mod, sc, ("fp64",) * 3, "fp64")
    emu = _oracle(oracle_mod, sc, prec, sp)
    Q0 = sc.initial_state(ref.node_coords())
    ref.set_state(Q0)
    dt = ref.max_dt(sc.cfl)
    A = ref.run(3, dt)
    emu.set_state(Q0)
    E = emu.run(3, dt)
    g = gpu_solver(sc, sc.cells, prec=prec)
    g.set_precision("storage", sp)
    g.set_state(Q0)
    g.step(dt, 3)
    B = g.get_state()
    assert np.all(np.isfinite(B))
    r_emu, r_ge = rel_l2(ref, E, A), rel_l2(ref, B, E)
    print("levels", name, sp, "emu-vs-fp64 %.3e gpu-vs-emu %.3e" % (r_emu, r_ge))
    # both sides round the same values at the same points; FP64 rounding-order
    # differences can move a value across a rounding boundary (one spacing)
    assert r_ge < 0.5 * r_emu + 1e-15
    assert r_ge < 2 * EPS[sp]
    # every value the GPU holds is representable in the storage format
    R = np.vectorize(lambda x: oracle_mod.round_p(sp, x))(B)
    np.testing.assert_array_equal(R, B)


def test_storage_round_trip_and_reencoding(oracle_mod):
    sc, _ = CASES["acoustic2d_n3"]
    o = _oracle(oracle_mod, sc, ("fp64",) * 3, "fp64")
    Q0 = sc.initial_state(o.node_coords()) * (1 + 1e-3 * np.random.default_rng(2).standard_normal((1,)))
    g = gpu_solver(sc, sc.cells)
    g.set_state(Q0)
    np.testing.assert_array_equal(g.get_state(), Q0)
    g.set_precision("storage", "fp32")  # re-encodes the held state
    np.testing.assert_array_equal(g.get_state(), Q0.astype(np.float32).astype(np.float64))
    g.set_precision("storage", "fp16")
    np.testing.assert_array_equal(g.get_state(), Q0.astype(np.float32).astype(np.float16).astype(np.float64))
    g.set_precision("storage", "fp64")  # widening keeps the FP16 values
    np.testing.assert_array_equal(g.get_state(), Q0.astype(np.float32).astype(np.float16).astype(np.float64))
    # max_dt and receivers read the stored values
    g.set_precision("storage", "bf16")
    g.set_state(Q0)
    Qb = g.get_state()
    o.set_state(Qb)
    assert abs(g.max_dt(sc.cfl) - o.max_dt(sc.cfl)) <= 1e-14 * o.max_dt(sc.cfl)
    pts = np.random.default_rng(3).uniform(0, 1, size=(5, 2)) * np.array(sc.hi)
    g.set_receivers(pts)
    np.testing.assert_allclose(g.read_receivers(), o.sample_points(pts, 0), rtol=0,
                               atol=1e-12 * np.abs(Qb[:, 0]).max())


@pytest.mark.parametrize("sp", ["fp32", "fp16"])
def test_storage_fused_steps_match_single_steps(oracle_mod, sp):
    sc, prec = CASES["elastic3d_n5"]
    o = _oracle(oracle_mod, sc, ("fp64",) * 3, "fp64")
    Q0 = sc.initial_state(o.node_coords())
    o.set_state(Q0)
    dt = 0.5 * o.max_dt(sc.cfl)
    g = gpu_solver(sc, sc.cells, prec=prec)
    g.set_precision("storage", sp)
    g.set_state(Q0)
    g.time = 0.0
    g.step(dt, 3)
    A = g.get_state()
    g.set_state(Q0)
    g.time = 0.0
    for _ in range(3):
        g.step(dt, 1)
    np.testing.assert_array_equal(g.get_state(), A)


def test_adjoint_refused_with_lower_storage():
    from paper_2504_06889_amd.aderdg import AderdgError
    import torch
    sc = _grid("acoustic", 3, 2, (3, 3, 3), (1.0, 2.25), "zeros", None)
    g = gpu_solver(sc, sc.cells)
    g.set_material(np.full(27, 1.5))
    g.set_precision("storage", "fp32")
    Qn = torch.zeros(g.shape, dtype=torch.float64, device="cuda")
    lam = torch.zeros_like(Qn)
    grad = torch.zeros(27, dtype=torch.float64, device="cuda")
    with pytest.raises(AderdgError) as e:
        g.step_adjoint(1e-3, 0.0, Qn, lam, grad)
    assert e.value.code == -2


@pytest.mark.parametrize("sp,nbytes", [("fp32", 4), ("bf16", 2), ("fp16", 2)])
def test_storage_state_is_narrow_in_device_memory(sp, nbytes):
    """The state buffer is reallocated in the storage format: the device memory
    it frees is the difference of the element sizes (4-byte or 2-byte elements
    instead of 8), and the raw FP64 pointer is refused while it is narrow."""
    import torch
    import ctypes

    from paper_2504_06889_amd.aderdg import lib
    sc = _grid("elastic", 3, 5, (16, 16, 16), (2.7, 32.4, 32.398), "planar_elastic", {"kP": TWO_PI, "kS": TWO_PI})
    g = gpu_solver(sc, sc.cells, prec=CASES["elastic3d_n5"][1])
    state_bytes = g.ncell * g.V * g.S * 8
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    g.set_precision("storage", sp)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    saved = free1 - free0
    expect = state_bytes * (8 - nbytes) // 8
    print("storage", sp, "freed", saved, "expected", expect, flush=True)
    assert abs(saved - expect) <= 0.05 * state_bytes, (saved, expect)
    p = ctypes.c_void_p()
    assert lib().aderdg_state_ptr(g._h, ctypes.byref(p)) == -2
    g.set_precision("storage", "fp64")
    assert lib().aderdg_state_ptr(g._h, ctypes.byref(p)) == 0
