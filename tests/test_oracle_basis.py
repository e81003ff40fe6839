"""Pins of the oracle's basis and operators against closed forms, library routines
and identities (arXiv 2504.06889, Sec. 3: Gauss-Legendre support points,
eq. Picard time matrix, eq. weak_form_volume_surface volume and face terms)."""
import math

import numpy as np
import pytest

from oracle import brute


@pytest.mark.parametrize("n,xi,w", [
    (1, [0.5], [1.0]),
    (2, [0.5 - math.sqrt(3) / 6, 0.5 + math.sqrt(3) / 6], [0.5, 0.5]),
    (3, [0.5 - math.sqrt(15) / 10, 0.5, 0.5 + math.sqrt(15) / 10], [5 / 18, 4 / 9, 5 / 18]),
])
def test_gauss_legendre_closed_forms(oracle_mod, n, xi, w):
    b = oracle_mod.basis(n)
    np.testing.assert_allclose(b["xi"], xi, rtol=0, atol=2e-16)
    np.testing.assert_allclose(b["w"], w, rtol=0, atol=2e-16)


@pytest.mark.parametrize("n", range(1, 11))
def test_gauss_legendre_vs_numpy(oracle_mod, n):
    b = oracle_mod.basis(n)
    x, w = brute.gl_nodes01(n)
    np.testing.assert_allclose(b["xi"], x, rtol=0, atol=1e-15)
    np.testing.assert_allclose(b["w"], w, rtol=0, atol=2e-15)
    # exact for monomials up to degree 2N+1 = 2n-1
    for m in range(2 * n):
        assert abs(np.dot(b["w"], b["xi"] ** m) - 1.0 / (m + 1)) < 2e-15


@pytest.mark.parametrize("n", range(1, 10))
def test_derivative_and_extrapolation_exact_on_polynomials(oracle_mod, n):
    b = oracle_mod.basis(n)
    xi = b["xi"]
    rng = np.random.default_rng(n)
    for _ in range(3):
        c = rng.standard_normal(n)  # degree N = n-1
        vals = np.polyval(c, xi)
        dvals = np.polyval(np.polyder(c), xi)
        scale = max(1.0, np.abs(dvals).max())
        assert np.abs(b["D"] @ vals - dvals).max() < 1e-12 * scale * n
        assert abs(b["F0"] @ vals - np.polyval(c, 0.0)) < 1e-13 * max(1, abs(vals).max())
        assert abs(b["F1"] @ vals - np.polyval(c, 1.0)) < 1e-13 * max(1, abs(vals).max())
    # D annihilates constants exactly (negative-sum diagonal)
    assert np.all(b["D"].sum(axis=1) == 0.0) or np.abs(b["D"].sum(axis=1)).max() < 1e-13
    np.testing.assert_allclose(b["F0"].sum(), 1.0, atol=1e-14)
    np.testing.assert_allclose(b["F1"].sum(), 1.0, atol=1e-14)


@pytest.mark.parametrize("n", range(1, 10))
def test_time_matrix_against_exact_integrals(oracle_mod, n):
    b = oracle_mod.basis(n)
    _, _, T1, F0, _ = brute.one_d_integrals(n)
    np.testing.assert_allclose(b["K1"], T1, rtol=0, atol=1e-11 * max(1, np.abs(T1).max()))
    # K1 1 = psi(0): so K1^{-1} psi(0) = 1, the Picard initial-guess property
    np.testing.assert_allclose(b["K1"] @ np.ones(n), b["F0"], atol=1e-12 * n)
    # Atau = K1^{-1} W
    np.testing.assert_allclose(b["K1"] @ b["Atau"], np.diag(b["w"]), atol=1e-13 * n)


@pytest.mark.parametrize("n", range(2, 10))
def test_picard_operator_identities(oracle_mod, n):
    """Atau 1 = xi (exact integration of q_t = 1) and w^T Atau^k 1 = 1/(k+1)!."""
    b = oracle_mod.basis(n)
    A = b["Atau"]
    np.testing.assert_allclose(A @ np.ones(n), b["xi"], atol=5e-15 * n)
    v = np.ones(n)
    for k in range(n):
        assert abs(b["w"] @ v - 1.0 / math.factorial(k + 1)) < 1e-14
        v = A @ v


@pytest.mark.parametrize("n", range(1, 10))
def test_summation_by_parts_and_volume_conservation(oracle_mod, n):
    b = oracle_mod.basis(n)
    WD = np.diag(b["w"]) @ b["D"]
    np.testing.assert_allclose(WD + WD.T, np.outer(b["F1"], b["F1"]) - np.outer(b["F0"], b["F0"]),
                               atol=2e-13 * n * n)
    # weak-form volume operator has zero weighted column sums (conserves the mean)
    np.testing.assert_allclose(b["w"] @ b["Kxi"], 0.0, atol=1e-12 * n * n)
    np.testing.assert_allclose(b["Kxi"], (np.diag(b["w"]) @ b["D"]).T / b["w"][:, None], atol=1e-13)
    np.testing.assert_allclose(b["L0"] * b["w"], b["F0"], atol=1e-15)
    np.testing.assert_allclose(b["L1"] * b["w"], b["F1"], atol=1e-15)


def _bf16_reference(x):
    """float32 -> bfloat16 round-to-nearest-even via torch (library routine)."""
    import torch
    return torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()


def test_rounding_matches_library_conversions(oracle_mod):
    rng = np.random.default_rng(7)
    vals = np.concatenate([
        rng.standard_normal(200) * 10.0 ** rng.integers(-9, 6, 200),
        [0.0, -0.0, 1.0, 65504.0, 65519.0, 65520.0, 1e5, -1e5, 6.0e-8, 3.0e-8, 2.9e-8,
         1.0 / 3.0, 2.0 ** -24, 2.0 ** -25, 1.5 * 2.0 ** -25, 3.4e38, 1e-39, 1e-45],
    ])
    for x in vals:
        f32 = np.float32(x)
        assert oracle_mod.round_p("fp32", x) == float(f32)
        h = float(np.float16(f32))  # IEEE binary16, RNE
        got = oracle_mod.round_p("fp16", x)
        assert got == h or (math.isinf(got) and math.isinf(h) and got == h), (x, got, h)
        b = float(_bf16_reference(float(f32)))
        got = oracle_mod.round_p("bf16", x)
        assert got == b or (math.isinf(got) and math.isinf(b)), (x, got, b)


def test_cast_error_ratios_follow_mantissa_bits(oracle_mod):
    """Initial-error ratios of Sec. 6.1: fp16/fp32 ~ 2^13 and bf16/fp16 ~ 2^3."""
    rng = np.random.default_rng(3)
    x = rng.uniform(-1, 1, 4000)
    err = {}
    for p in ("fp32", "fp16", "bf16"):
        r = np.array([oracle_mod.round_p(p, v) for v in x])
        err[p] = np.sqrt(np.mean((r - x) ** 2))
    assert 2 ** 12 < err["fp16"] / err["fp32"] < 2 ** 14
    assert 2 ** 2 < err["bf16"] / err["fp16"] < 2 ** 4
