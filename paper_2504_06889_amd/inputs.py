"""Seeded, synthetic inputs: scenario definitions and analytic initial states.

This module holds none of the method's arithmetic.  It evaluates closed-form
initial conditions (and exact solutions) at node coordinates that the caller
supplies, draws the seeded per-cell material and receiver positions, and
names the five benchmark configurations.  Both the GPU path and the CPU
oracle take their inputs from here.

Scenarios (arXiv 2504.06889, Sec. 5):
  planar waves  Q = omega sin(omega t - k.x) q0 with (omega, q0) an eigenpair
                of sum_j k_j A_j (Sec. 5.2, planar waves), acoustic and elastic,
                and 3-D elastic P and S plane waves along an oblique k;
  Euler         advected density sine wave (exact: shifted initial state), the
                smooth Gaussian bell (Sec. 5.3.1, exp(-50 r^2) reading) and the
                static isentropic vortex (Sec. 5.3.2, with p = (1+dT)^(g/(g-1))
                and v_inf + dv, the reading that keeps p / rho^g = 1);
  shallow water lake at rest (Sec. 5.4.1) and a bump with a small sine
                perturbation of the surface.
"""
import math
from dataclasses import dataclass, field
from typing import Tuple

import numpy as np


# --------------------------------------------------------------------------
# Node-coordinate grids (broadcast over [cells..., nodes...], x fastest)
# --------------------------------------------------------------------------

def _grid(coords):
    """Broadcast per-dimension node coordinates [C_j, n] to the state layout.

    Returns d arrays that broadcast to shape (C_{d-1}, ..., C_0, n, ..., n)."""
    d = len(coords)
    out = []
    for j, c in enumerate(coords):
        shape = [1] * (2 * d)
        shape[d - 1 - j] = c.shape[0]
        shape[2 * d - 1 - j] = c.shape[1]
        out.append(c.reshape(shape))
    return out


def _pack(fields, coords):
    """Stack per-variable arrays into the [cell][var][node] layout."""
    d = len(coords)
    C = [c.shape[0] for c in coords]
    n = coords[0].shape[1]
    full = tuple(C[::-1]) + (n,) * d
    arr = np.stack([np.broadcast_to(f, full) for f in fields], axis=d)
    ncell = int(np.prod(C))
    return np.ascontiguousarray(arr.reshape(ncell, len(fields), n ** d))


# --------------------------------------------------------------------------
# Planar waves (Sec. 5.2.1)
# --------------------------------------------------------------------------

def acoustic_eigvec(k, K, rho):
    """(omega, q0) with (sum_j k_j A_j) q0 = omega q0 for acoustics; q0[0] = 1."""
    kn = math.sqrt(sum(x * x for x in k))
    c = math.sqrt(K / rho)
    omega = c * kn
    return omega, np.array([1.0] + [kj / (rho * omega) for kj in k])


def planar_acoustic(coords, t, k, K, rho):
    X = _grid(coords)
    omega, q0 = acoustic_eigvec(k, K, rho)
    phase = omega * t - sum(kj * Xj for kj, Xj in zip(k, X))
    s = omega * np.sin(phase)
    return _pack([q0[v] * s for v in range(len(q0))], coords)


def elastic_waves(d, rho, lam, mu):
    """P wave along x and S wave along y (polarised along x), unit velocity amplitude.

    Variables: 2-D (sxx, syy, sxy, vx, vy); 3-D (sxx, syy, szz, sxy, syz, sxz,
    vx, vy, vz).  Returns ((cp, rP), (cs, rS))."""
    cp = math.sqrt((lam + 2 * mu) / rho)
    cs = math.sqrt(mu / rho)
    if d == 2:
        rP = np.array([-rho * cp, -lam / cp, 0.0, 1.0, 0.0])
        rS = np.array([0.0, 0.0, -rho * cs, 1.0, 0.0])
    elif d == 3:
        rP = np.array([-rho * cp, -lam / cp, -lam / cp, 0, 0, 0, 1.0, 0, 0])
        rS = np.array([0, 0, 0, -rho * cs, 0, 0, 1.0, 0, 0])
    else:
        raise ValueError("elastic waves need d = 2 or 3")
    return (cp, rP), (cs, rS)


def planar_elastic(coords, t, rho, lam, mu, kP, kS):
    """omega_P sin(omega_P t - kP x) rP + omega_S sin(omega_S t - kS y) rS."""
    d = len(coords)
    X = _grid(coords)
    (cp, rP), (cs, rS) = elastic_waves(d, rho, lam, mu)
    wP, wS = cp * kP, cs * kS
    sP = wP * np.sin(wP * t - kP * X[0])
    sS = wS * np.sin(wS * t - kS * X[1])
    return _pack([rP[v] * sP + rS[v] * sS for v in range(len(rP))], coords)


def elastic_plane_waves(coords, t, rho, lam, mu, k, pols):
    """Superposed plane waves of the 3-D elastic system along one wave vector k.

    The system (the 3-D form of eq. equations_of_motion): d sigma_ij/dt =
    lambda delta_ij div v + mu (d_i v_j + d_j v_i), rho dv_i/dt = sum_j
    d_j sigma_ij.  For a velocity v = a d sin(omega t - k.x) with a unit
    polarisation d, the momentum and stress equations hold when
    rho omega^2 d = (lambda + mu) k (k.d) + mu |k|^2 d, i.e. d parallel to k
    with omega = cp |k| (P wave) or d orthogonal to k with omega = cs |k|
    (S wave), and the stress amplitude is
        S_ij = -(lambda delta_ij (k.d) + mu (k_i d_j + k_j d_i)) / omega.
    `pols` lists (amplitude, polarisation) pairs; each polarisation must be
    parallel or orthogonal to k.  Variables (sxx, syy, szz, sxy, syz, sxz, vx,
    vy, vz); k must be periodic on the domain."""
    X = _grid(coords)
    k = np.asarray(k, dtype=np.float64)
    kn = float(np.linalg.norm(k))
    cp = math.sqrt((lam + 2 * mu) / rho)
    cs = math.sqrt(mu / rho)
    phase_x = sum(k[j] * X[j] for j in range(3))
    fields = [0.0 * phase_x for _ in range(9)]
    pairs = ((0, 0, 0), (1, 1, 1), (2, 2, 2), (3, 0, 1), (4, 1, 2), (5, 0, 2))
    for amp, d in pols:
        d = np.asarray(d, dtype=np.float64)
        d = d / np.linalg.norm(d)
        kd = float(k @ d)
        if abs(abs(kd) - kn) < 1e-12 * kn:
            omega = cp * kn
        elif abs(kd) < 1e-12 * kn:
            omega = cs * kn
        else:
            raise ValueError("polarisation must be parallel or orthogonal to k")
        s = amp * np.sin(omega * t - phase_x)
        for v, i, j in pairs:
            S = -((lam * kd if i == j else 0.0) + mu * (k[i] * d[j] + k[j] * d[i])) / omega
            fields[v] = fields[v] + S * s
        for i in range(3):
            fields[6 + i] = fields[6 + i] + d[i] * s
    return _pack(fields, coords)


def planar_elastic_oblique(coords, t, rho, lam, mu, k=(2 * math.pi,) * 3, amp_p=1.0, amp_s=1.0):
    """P wave and S wave along k (default 2 pi (1, 1, 1)), the S wave polarised
    along (k_y, -k_x, 0): every stress and velocity component varies, and
    sigma_yz and sigma_xz differ."""
    k = np.asarray(k, dtype=np.float64)
    dP = k / np.linalg.norm(k)
    dS = np.array([k[1], -k[0], 0.0])
    return elastic_plane_waves(coords, t, rho, lam, mu, k, [(amp_p, dP), (amp_s, dS)])


# --------------------------------------------------------------------------
# Euler (Sec. 5.3)
# --------------------------------------------------------------------------

def euler_density_wave(coords, t, gamma, amp=0.2, u=1.0, p=1.0):
    """rho = 1 + amp sin(2 pi (sum x_j - d u t)), velocity u in every direction."""
    d = len(coords)
    X = _grid(coords)
    rho = 1.0 + amp * np.sin(2 * np.pi * (sum(X) - d * u * t))
    E = p / (gamma - 1.0) + 0.5 * rho * d * u * u
    return _pack([rho] + [rho * u] * d + [E], coords)


def _periodic_offset(x, c, L):
    r = x - c
    return r - L * np.round(r / L)


def euler_bell(coords, t, gamma, lo=-1.0, hi=1.0, rho0=0.02):
    """2-D smooth density bell advected with v = (1, 1), p = 1 (exp(-50 r^2))."""
    X = _grid(coords)
    L = hi - lo
    r2 = sum(_periodic_offset(Xj, t, L) ** 2 for Xj in X)
    rho = rho0 * (1.0 + np.exp(-50.0 * r2))
    return _pack([rho, rho, rho, 1.0 / (gamma - 1.0) + rho], coords)


def euler_vortex(coords, gamma, beta=5.0):
    """2-D static isentropic vortex (Hu-Shu), rho_inf = p_inf = 1, v_inf = 0."""
    X, Y = _grid(coords)
    r2 = X * X + Y * Y
    dT = (1.0 - gamma) * beta ** 2 / (8.0 * gamma * np.pi ** 2) * np.exp(1.0 - r2)
    rho = (1.0 + dT) ** (1.0 / (gamma - 1.0))
    p = (1.0 + dT) ** (gamma / (gamma - 1.0))
    u = -Y * beta / (2 * np.pi) * np.exp(0.5 * (1.0 - r2))
    v = X * beta / (2 * np.pi) * np.exp(0.5 * (1.0 - r2))
    E = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)
    return _pack([rho, rho * u, rho * v, E], coords)


# --------------------------------------------------------------------------
# Shallow water (Sec. 5.4)
# --------------------------------------------------------------------------

def swe_lake_at_rest(coords, eta0=2.0):
    X, Y = _grid(coords)
    b = np.sin(2 * np.pi * (X + Y))
    return _pack([eta0 - b, 0.0 * b, 0.0 * b, b], coords)


def swe_bump(coords, eta0=2.0, bump=0.1, width=200.0, pert=0.01):
    """b = bump exp(-width r^2) around (1/2, 1/2); h = eta0 - b + pert sin(2 pi (x+y))."""
    X, Y = _grid(coords)
    b = bump * np.exp(-width * ((X - 0.5) ** 2 + (Y - 0.5) ** 2))
    h = eta0 - b + pert * np.sin(2 * np.pi * (X + Y))
    return _pack([h, 0.0 * h, 0.0 * h, b + 0.0 * h], coords)


def swe_gravity_wave(coords, t, g, depth=2.0, bottom=0.25, flow=(0.4, -0.25),
                     k=(2 * math.pi, 4 * math.pi), eps=1e-7):
    """Small gravity wave on a uniform stream over a flat bottom.

    Linearising eq. swe about h = depth, v = flow, b = bottom (constant) gives
    h'_t + flow.grad h' + depth div v' = 0 and v'_t + flow.grad v' + g grad h' = 0,
    solved by h' = eps sin(k.x - omega t), v' = eps (c / depth) k/|k| sin(k.x - omega t)
    with c = sqrt(g depth) and omega = k.flow + c |k|.  The state is
    (depth + h', (depth + h') (flow + v'), bottom): the full nonlinear system
    differs from it by O(eps^2)."""
    X, Y = _grid(coords)
    kx, ky = k
    kn = math.hypot(kx, ky)
    c = math.sqrt(g * depth)
    omega = kx * flow[0] + ky * flow[1] + c * kn
    s = eps * np.sin(kx * X + ky * Y - omega * t)
    h = depth + s
    u = flow[0] + (c / depth) * (kx / kn) * s
    v = flow[1] + (c / depth) * (ky / kn) * s
    return _pack([h, h * u, h * v, bottom + 0.0 * h], coords)


def zeros(coords, nvars):
    X = _grid(coords)
    z = 0.0 * sum(X)
    return _pack([z] * nvars, coords)


# --------------------------------------------------------------------------
# Seeded random inputs (adjoint configuration)
# --------------------------------------------------------------------------

def lognormal_speed(ncell, mean=1.5, sigma=0.2, seed=0):
    """Per-cell sound speed c_i = mean * exp(sigma z_i), z ~ N(0, 1), C order."""
    z = np.random.default_rng(seed).standard_normal(ncell)
    return mean * np.exp(sigma * z)


def receivers_near(center, h, nrec=64, half_cells=2.5, seed=1, dim=3):
    """nrec points uniform in the (2*half_cells)^d cell block around `center`."""
    u = np.random.default_rng(seed).uniform(-half_cells, half_cells, size=(nrec, dim))
    return np.asarray(center)[None, :dim] + h * u


# --------------------------------------------------------------------------
# Benchmark configurations
# --------------------------------------------------------------------------

@dataclass
class Scenario:
    name: str
    pde: str
    dim: int
    order: int
    cells: Tuple[int, ...]
    lo: Tuple[float, ...]
    hi: Tuple[float, ...]
    params: Tuple[float, ...]      # acoustic: rho,K | elastic: rho,lambda,mu | euler: gamma | swe: g
    steps: int
    cfl: float                     # C_CFL in dt = C h / (d (2N+1) lambda_max)
    ic: str
    extra: dict = field(default_factory=dict)

    def initial_state(self, coords, t=0.0):
        return evaluate(self, coords, t)

    def with_cells(self, cells):
        return Scenario(self.name, self.pde, self.dim, self.order, tuple(cells), self.lo,
                        self.hi, self.params, self.steps, self.cfl, self.ic, dict(self.extra))


def _elastic_params(rho, cp, cs):
    mu = rho * cs * cs
    lam = rho * cp * cp - 2.0 * mu
    return (rho, lam, mu)


SCENARIOS = {
    # 2-D linear acoustics (p, u, v), N = 3, 16^2 cells on the periodic unit square,
    # rho = K = 1, planar sine wave along (1, 1), 10 steps.
    "acoustic2d_n3_16": Scenario("acoustic2d_n3_16", "acoustic", 2, 3, (16, 16), (0.0, 0.0),
                                 (1.0, 1.0), (1.0, 1.0), 10, 0.7, "planar_acoustic",
                                 {"k": (2 * math.pi, 2 * math.pi)}),
    # 3-D elastic wave (9 vars), N = 5, 64^3 periodic cells, rho = 2.7, cp = 6, cs = 3.464,
    # planar P + S wave along k = 2 pi (1, 1, 1) (S polarised along (1, -1, 0)), 100 steps.
    "elastic3d_n5_64": Scenario("elastic3d_n5_64", "elastic", 3, 5, (64, 64, 64), (0.0,) * 3,
                                (1.0,) * 3, _elastic_params(2.7, 6.0, 3.464), 100, 0.5,
                                "planar_elastic_oblique", {"k": (2 * math.pi,) * 3}),
    # 3-D compressible Euler, N = 4, 48^3 cells, density sine wave, 200 steps.
    "euler3d_n4_48": Scenario("euler3d_n4_48", "euler", 3, 4, (48, 48, 48), (0.0,) * 3,
                              (1.0,) * 3, (1.4,), 200, 0.6, "euler_density_wave"),
    # 2-D shallow water (h, hu, hv, b), N = 6, 512^2 cells, g = 9.81, Gaussian bump + sine
    # perturbation on h = 2, 500 steps.
    "swe2d_n6_512": Scenario("swe2d_n6_512", "swe", 2, 6, (512, 512), (0.0, 0.0), (1.0, 1.0),
                             (9.81,), 500, 0.45, "swe_bump"),
    # Adjoint: 3-D acoustics (p, u, v, w), N = 5, 64^3 cells on [0, 20]^3, rho = 1, per-cell
    # log-normal sound speed (mean 1.5, sigma 0.2, seed 0), Ricker source f0 = 5, 200 steps,
    # 64 receivers, checkpoint every 20 steps.
    "adjoint_acoustic3d_n5_64": Scenario(
        "adjoint_acoustic3d_n5_64", "acoustic", 3, 5, (64, 64, 64), (0.0,) * 3, (20.0,) * 3,
        (1.0, 1.5 ** 2), 200, 0.5, "zeros",
        {"f0": 5.0, "t0": 0.2, "amp": 1.0, "src_cell": (32, 32, 32), "nrec": 64,
         "checkpoint": 20, "c_mean": 1.5, "c_sigma": 0.2, "seed_c": 0, "seed_rec": 1}),
}

# The paper's 2-D scenarios of its mixed-precision study (Sec. 5, Sec. 7): 27^2 cells,
# order 5, periodic.  Each runs to extra["t_end"] (steps = 0: the step count follows from
# dt = C h / (d (2N+1) lambda_max) of the initial state); extra["exact"] says whether the
# scenario has a closed-form solution at t_end.
#  - acoustic planar wave (Sec. 5.2.1): [-1,1]^2, K = 4, rho = 1 (c = 2), wave along the
#    diagonal, k = (pi, pi): the state returns to the initial one at t = sqrt(2) (t_end);
#  - elastic planar waves (Sec. 5.2.1): [-1,1]^2, lambda = 2, mu = 1, rho = 1 (cp = 2,
#    cs = 1), P wave along x (k = pi) and S wave along y (k = 2 pi), both of period 1 (t_end);
#  - Euler Gaussian bell (Sec. 5.3.1): rho = 0.02 (1 + exp(-50 r^2)), v = (1, 1), p = 1 on
#    [-1,1]^2, t_end = 2 (one period of the advection);
#  - static isentropic vortex (Sec. 5.3.2): beta = 5 on [-5,5]^2, t_end = 10;
#  - lake at rest (Sec. 5.4.1): b = sin(2 pi (x + y)), h = eta0 - b, eta0 = 2, g = 9.81 on
#    [-1,1]^2, t_end = 1.
PAPER_SUITE = {
    "acoustic2d_n5_27_planar": Scenario(
        "acoustic2d_n5_27_planar", "acoustic", 2, 5, (27, 27), (-1.0, -1.0), (1.0, 1.0), (1.0, 4.0), 0, 0.5,
        "planar_acoustic", {"k": (math.pi, math.pi), "t_end": math.sqrt(2.0), "exact": True}),
    "elastic2d_n5_27_planar": Scenario(
        "elastic2d_n5_27_planar", "elastic", 2, 5, (27, 27), (-1.0, -1.0), (1.0, 1.0), (1.0, 2.0, 1.0), 0, 0.5,
        "planar_elastic", {"kP": math.pi, "kS": 2 * math.pi, "t_end": 1.0, "exact": True}),
    "euler2d_n5_27_bell": Scenario(
        "euler2d_n5_27_bell", "euler", 2, 5, (27, 27), (-1.0, -1.0), (1.0, 1.0), (1.4,), 0, 0.5,
        "euler_bell", {"t_end": 2.0, "exact": True}),
    "euler2d_n5_27_vortex": Scenario(
        "euler2d_n5_27_vortex", "euler", 2, 5, (27, 27), (-5.0, -5.0), (5.0, 5.0), (1.4,), 0, 0.5,
        "euler_vortex", {"t_end": 10.0, "exact": True}),
    "swe2d_n5_27_lake": Scenario(
        "swe2d_n5_27_lake", "swe", 2, 5, (27, 27), (-1.0, -1.0), (1.0, 1.0), (9.81,), 0, 0.5,
        "swe_lake", {"eta0": 2.0, "t_end": 1.0, "exact": True}),
}


def evaluate(sc, coords, t=0.0):
    """Initial (t = 0) or exact state of scenario `sc` at the given node coordinates."""
    if sc.ic == "planar_acoustic":
        rho, K = sc.params[0], sc.params[1]
        return planar_acoustic(coords, t, sc.extra["k"], K, rho)
    if sc.ic == "planar_elastic":
        rho, lam, mu = sc.params[:3]
        return planar_elastic(coords, t, rho, lam, mu, sc.extra["kP"], sc.extra["kS"])
    if sc.ic == "planar_elastic_oblique":
        rho, lam, mu = sc.params[:3]
        ex = sc.extra
        return planar_elastic_oblique(coords, t, rho, lam, mu, ex.get("k", (2 * math.pi,) * 3),
                                      ex.get("amp_p", 1.0), ex.get("amp_s", 1.0))
    if sc.ic == "elastic_plane_waves":
        rho, lam, mu = sc.params[:3]
        return elastic_plane_waves(coords, t, rho, lam, mu, sc.extra["k"], sc.extra["pols"])
    if sc.ic == "swe_gravity_wave":
        ex = {k_: v_ for k_, v_ in sc.extra.items() if k_ in ("depth", "bottom", "flow", "k", "eps")}
        return swe_gravity_wave(coords, t, sc.params[0], **ex)
    if sc.ic == "euler_density_wave":
        return euler_density_wave(coords, t, sc.params[0])
    if sc.ic == "euler_bell":
        return euler_bell(coords, t, sc.params[0], sc.lo[0], sc.hi[0])
    if sc.ic == "euler_vortex":
        return euler_vortex(coords, sc.params[0])
    if sc.ic == "swe_bump":
        return swe_bump(coords)
    if sc.ic == "swe_lake":
        return swe_lake_at_rest(coords, sc.extra.get("eta0", 2.0))
    if sc.ic == "zeros":
        nv = {"acoustic": 1 + sc.dim, "euler": 2 + sc.dim}[sc.pde]
        return zeros(coords, nv)
    raise KeyError(sc.ic)


def source_point(sc, h):
    """Physical position of the point source: centre of the named cell."""
    c = sc.extra["src_cell"]
    return np.array([sc.lo[j] + h * (c[j] + 0.5) for j in range(sc.dim)])
