"""Seeded synthetic inputs for the paper's workloads.

This module is shared by the oracle side and the GPU side of the tests and by
``bench.py``.  It holds problem *set-ups* only -- parameter sets in the
paper's notation and initial order-parameter fields built from the paper's
initial-condition formulas -- and none of the lattice Boltzmann method's
arithmetic (no equilibria, no relaxation rates, no stencils).  Each side
translates a :class:`Case` into its own parameter struct.

Geometry: node (i, j) sits at (i + 1/2, j + 1/2) in lattice units; walls lie
on the domain faces x = 0, x = nx, y = 0, y = ny.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np

SEED = 211100847


@dataclasses.dataclass
class Case:
    nx: int
    ny: int
    wall_x: bool = False
    wall_y: bool = False
    visc_law: str = "linear_mu"      # "linear_mu" | "inverse_nu"
    model: str = "present"           # "present" | "original" | "corrected"
    phase_eq: str = "allen_cahn"     # "allen_cahn" | "cahn_hilliard" (Sec. 2, Eqs. ACE / CHE)
    grad_scheme: str = "stencil"     # "stencil" (Eq. central1) | "local" (Eq. local, Allen-Cahn)
    phiA: float = 1.0
    phiB: float = 0.0
    rhoA: float = 1.0
    rhoB: float = 1.0
    nuA: float = 0.1
    nuB: float = 0.1
    sigma: float = 0.0
    W: float = 4.0
    M: float = 0.1
    eta: float = 1.0
    s_f: Tuple[float, ...] = (0.0,) * 9   # <= 0: the paper's default
    s_g: Tuple[float, ...] = (0.0,) * 9
    body_force: Tuple[float, float] = (0.0, 0.0)
    gravity: Tuple[float, float] = (0.0, 0.0)
    rho_ref: float = 0.0
    theta: Tuple[float, float, float, float] = (math.pi / 2,) * 4
    rho0: float = 0.0
    eps_n: float = 1e-4
    dtype: str = "f32"
    steps: int = 0
    name: str = ""

    def replace(self, **kw) -> "Case":
        return dataclasses.replace(self, **kw)

    @property
    def nodes(self) -> int:
        return self.nx * self.ny


def grid(case: Case):
    x = np.arange(case.nx) + 0.5
    y = np.arange(case.ny) + 0.5
    X, Y = np.meshgrid(x, y)          # [ny][nx]
    return X, Y


def tanh_profile(d, W, phiA=1.0, phiB=0.0):
    """(phiA+phiB)/2 + (phiA-phiB)/2 tanh(2 d / W), d the signed distance (positive in A)."""
    return 0.5 * (phiA + phiB) + 0.5 * (phiA - phiB) * np.tanh(2.0 * d / W)


# ---------------------------------------------------------------- square droplet
def to_cahn_hilliard(case: Case, phi0):
    """The same set-up with the Cahn-Hilliard phase field (Sec. 2, Eq. CHE) and phi
    in [-1, 1] (phi_A = 1, phi_B = -1, as the paper uses it in Secs. 4.1 and 4.4);
    phi0 given in [0, 1]."""
    return case.replace(phase_eq="cahn_hilliard", phiA=1.0, phiB=-1.0), 2.0 * np.asarray(phi0) - 1.0


def square_droplet_ch(n: int = 200, R: float = 50.0, W: float = 4.0, rho_ratio: float = 1000.0,
                      nu: float = 0.1, M: float = 0.1, sigma: float = 1e-5, dtype: str = "f64",
                      model: str = "present"):
    """Sec. 4.1 with the Cahn-Hilliard phase field: a square of side
    D = sqrt(pi R^2 + (4 - pi) W^2 / 4) (the area of the final circle of radius R)
    in a periodic n x n box, phi in [-1, 1], heavy phase A inside.  The paper's
    units (domain [-1, 1]^2, W = 4 dx = 0.04, c = 100, nu = 0.1, M = 0.1,
    sigma = 1e-3) map to lattice units dx = 0.01, dt = 1e-4: n = 200, R = 50,
    nu = M = 0.1, sigma = 1e-3 dt^2 / dx^3 = 1e-5."""
    D = math.sqrt(math.pi * R * R + (4.0 - math.pi) * W * W / 4.0)
    case = Case(nx=n, ny=n, rhoA=rho_ratio, rhoB=1.0, nuA=nu, nuB=nu, sigma=sigma, W=W, M=M, dtype=dtype,
                phase_eq="cahn_hilliard", phiA=1.0, phiB=-1.0, model=model, name=f"square_droplet_ch_{n}")
    X, Y = grid(case)
    a = D / 2.0
    r = W / 2.0
    b = a - r
    qx = np.abs(X - n / 2.0) - b
    qy = np.abs(Y - n / 2.0) - b
    outside = np.hypot(np.maximum(qx, 0), np.maximum(qy, 0)) + np.minimum(np.maximum(qx, qy), 0) - r
    return case, tanh_profile(-outside, W, 1.0, -1.0)


def square_droplet(n: int = 64, side: float = 32.0, dtype: str = "f64", steps: int = 2000):
    """Square droplet of side ``side`` centred in an n x n periodic box; density
    ratio 10, nu = 0.1 in both phases, sigma = 0.01, M = 0.02, W = 4.

    The paper's piecewise profile (Sec. 4.1) jumps by (1 - tanh 1)/2 at depth W/2;
    the continuous profile 0.5 + 0.5 tanh(2 d / W) is used instead, with d the
    signed distance to a square whose corners are rounded with radius W/2."""
    W = 4.0
    case = Case(nx=n, ny=n, rhoA=10.0, rhoB=1.0, nuA=0.1, nuB=0.1, sigma=0.01, W=W, M=0.02,
                dtype=dtype, steps=steps, name=f"square_droplet_{n}x{n}")
    X, Y = grid(case)
    a = side / 2.0
    r = W / 2.0
    b = a - r
    qx = np.abs(X - n / 2.0) - b
    qy = np.abs(Y - n / 2.0) - b
    outside = np.hypot(np.maximum(qx, 0), np.maximum(qy, 0)) + np.minimum(np.maximum(qx, qy), 0) - r
    phi0 = tanh_profile(-outside, W)
    return case, phi0


# ---------------------------------------------------------------- layered Poiseuille
def layered_mu(y, case: Case):
    """Linear dynamic viscosity across the tanh layer profile (Sec. 4.2)."""
    muA, muB = case.rhoA * case.nuA, case.rhoB * case.nuB
    return 0.5 * (muA + muB) + 0.5 * (muA - muB) * np.tanh(-2.0 * y / case.W)


def layered_poiseuille_profile(y, case: Case, G: float, nquad: int = 200001):
    """Steady solution of d/dy(mu du/dy) = -G with u(+-h) = 0 for the smooth mu(y);
    it is the paper's U_e(y) written with the forcing G instead of U_c."""
    h = case.ny / 2.0
    yy = np.linspace(-h, h, nquad)
    mu = layered_mu(yy, case)
    inv = 1.0 / mu
    from scipy.integrate import cumulative_trapezoid
    I1 = cumulative_trapezoid(inv, yy, initial=0.0)
    Iy = cumulative_trapezoid(yy * inv, yy, initial=0.0)
    A, B = Iy[-1], I1[-1]
    u = G * (-Iy + (A / B) * I1)
    return np.interp(y, yy, u)


def layered_poiseuille(nx: int = 4, ny: int = 256, density_ratio: float = 100.0,
                       visc_ratio: float = 10.0, umax: float = 1e-3, dtype: str = "f32",
                       steps: int = 50000, W: float = 4.0, sigma: float = 1e-3, M: float = 0.1,
                       muB: float = 0.1):
    """Two-layer channel flow: heavy fluid A (phi = 1) in the lower half, periodic x,
    bounce-back walls at y = 0 and y = ny, forcing G chosen so max u = umax."""
    rhoB = 1.0
    rhoA = density_ratio * rhoB
    muA = visc_ratio * muB
    case = Case(nx=nx, ny=ny, wall_y=True, rhoA=rhoA, rhoB=rhoB, nuA=muA / rhoA, nuB=muB / rhoB,
                sigma=sigma, W=W, M=M, dtype=dtype, steps=steps,
                name=f"layered_poiseuille_{nx}x{ny}")
    yy = np.linspace(-ny / 2.0, ny / 2.0, 20001)
    G = umax / np.max(layered_poiseuille_profile(yy, case, 1.0))
    case = case.replace(body_force=(float(G), 0.0))
    X, Y = grid(case)
    yc = Y - ny / 2.0
    phi0 = tanh_profile(-yc, W)
    return case, phi0


# ---------------------------------------------------------------- Rayleigh-Taylor
def rti(nx: int = 256, ny: int = 1024, dtype: str = "f32", steps: int = 20000,
        W: float = 5.0, Re: float = 3000.0, atwood: float = 0.5, sqrt_gd: float = 0.04,
        sigma: float = 5e-5):
    """Rayleigh-Taylor instability (Sec. 4.4): heavy fluid A on top, periodic x,
    no-slip/no-flux walls top and bottom, interface y = ny/2 + 0.1 nx cos(2 pi x / nx),
    body force -(rho - (rhoA+rhoB)/2) g in y, s_f^3 = s_f^5 = 0.9, s_g^4 = s_g^6 = 1.7."""
    d = float(nx)
    g = sqrt_gd ** 2 / d
    nu = d * sqrt_gd / Re
    rhoB = 1.0
    rhoA = rhoB * (1 + atwood) / (1 - atwood)
    sf = [0.0] * 9
    sf[3] = sf[5] = 0.9
    sg = [0.0] * 9
    sg[4] = sg[6] = 1.7
    M = (1.0 / 0.9 - 0.5) / 3.0   # the mobility that s_f = 0.9 encodes
    case = Case(nx=nx, ny=ny, wall_y=True, rhoA=rhoA, rhoB=rhoB, nuA=nu, nuB=nu, sigma=sigma,
                W=W, M=M, s_f=tuple(sf), s_g=tuple(sg), gravity=(0.0, -g),
                rho_ref=0.5 * (rhoA + rhoB), dtype=dtype, steps=steps, name=f"rti_{nx}x{ny}")
    X, Y = grid(case)
    h = ny / 2.0 + 0.1 * nx * np.cos(2 * np.pi * X / nx)
    phi0 = tanh_profile(Y - h, W)
    return case, phi0


# ---------------------------------------------------------------- droplet spreading
SPREAD_SIZES = [(128, 64), (256, 128), (512, 256)]


def spreading_case(nx: int, ny: int, theta_deg: float, dtype: str = "f32", steps: int = 10000,
                   R0: Optional[float] = None, rho_ratio: float = 1000.0, mu_ratio: float = 100.0,
                   sigma: float = 1e-3, W: float = 5.0, M: float = 0.1, nuB: float = 0.1):
    """Semicircular droplet of radius R0 (default nx/8) centred at (nx/2, 0) on a wetting
    bottom wall (contact angle theta), neutral top wall, periodic x (Sec. 4.3)."""
    R0 = nx / 8.0 if R0 is None else R0
    rhoB = 1.0
    rhoA = rho_ratio * rhoB
    muB = rhoB * nuB
    muA = mu_ratio * muB
    th = math.radians(theta_deg)
    case = Case(nx=nx, ny=ny, wall_y=True, rhoA=rhoA, rhoB=rhoB, nuA=muA / rhoA, nuB=nuB,
                sigma=sigma, W=W, M=M, theta=(math.pi / 2, math.pi / 2, th, math.pi / 2),
                dtype=dtype, steps=steps, name=f"spreading_{nx}x{ny}_{theta_deg:.1f}deg")
    X, Y = grid(case)
    phi0 = tanh_profile(R0 - np.hypot(X - nx / 2.0, Y), W)
    return case, phi0


def spreading_batch(ncases: int = 64, seed: int = SEED, dtype: str = "f32", steps: int = 10000):
    """The batched mix: sizes drawn uniformly from SPREAD_SIZES, then contact
    angles uniform in [30, 150] degrees, from numpy's default_rng(seed)."""
    rng = np.random.default_rng(seed)
    idx = rng.integers(0, len(SPREAD_SIZES), size=ncases)
    thetas = rng.uniform(30.0, 150.0, size=ncases)
    out = []
    for k in range(ncases):
        nx, ny = SPREAD_SIZES[int(idx[k])]
        out.append(spreading_case(nx, ny, float(thetas[k]), dtype=dtype, steps=steps))
    return out


# ---------------------------------------------------------------- dam break
def dam_break(nx: int = 1024, ny: int = 512, column: Optional[int] = None, dtype: str = "f32",
              steps: int = 4000, g: float = 1e-6, theta_deg: float = 90.0, Re: float = 1e4,
              a: float = 256.0, nu_ratio: float = 14.72, sigma: float = 0.02, M: float = 0.03,
              W: float = 4.0, rho_ratio: float = 1000.0):
    """Dam break (Sec. 4.5): heavy column of width ``column`` (default nx/4) over the
    full height at the left wall, walls on all four sides with one contact angle,
    inverse-linear kinematic viscosity, body force (0, -rho g).  nu_A follows from
    Re = a sqrt(g a) / nu_A with a = 256; nu_B / nu_A is the water/air ratio."""
    column = nx // 4 if column is None else column
    nuA = a * math.sqrt(g * a) / Re
    th = math.radians(theta_deg)
    case = Case(nx=nx, ny=ny, wall_x=True, wall_y=True, visc_law="inverse_nu", rhoA=rho_ratio,
                rhoB=1.0, nuA=nuA, nuB=nuA * nu_ratio, sigma=sigma, W=W, M=M,
                gravity=(0.0, -g), rho_ref=0.0, theta=(th, th, th, th), dtype=dtype,
                steps=steps, name=f"dam_break_{nx}x{ny}")
    X, Y = grid(case)
    phi0 = tanh_profile(column - X, W)
    return case, phi0


# ---------------------------------------------------------------- small pin cases
def static_droplet(n: int = 64, R: float = 16.0, rho_ratio: float = 10.0, sigma: float = 0.01,
                   W: float = 4.0, M: float = 0.02, nu: float = 0.1, dtype: str = "f64"):
    case = Case(nx=n, ny=n, rhoA=rho_ratio, rhoB=1.0, nuA=nu, nuB=nu, sigma=sigma, W=W, M=M,
                dtype=dtype, name=f"static_droplet_{n}_R{R}")
    X, Y = grid(case)
    phi0 = tanh_profile(R - np.hypot(X - n / 2.0, Y - n / 2.0), W)
    return case, phi0


def flat_interface(nx: int = 4, ny: int = 128, W: float = 4.0, rho_ratio: float = 10.0,
                   sigma: float = 0.01, M: float = 0.05, dtype: str = "f64", offset: float = 0.0):
    """Two flat interfaces in a periodic box (a slab of A between y = ny/4 and 3 ny/4)."""
    case = Case(nx=nx, ny=ny, rhoA=rho_ratio, rhoB=1.0, nuA=0.1, nuB=0.1, sigma=sigma, W=W, M=M,
                dtype=dtype, name=f"flat_interface_{ny}_W{W}")
    X, Y = grid(case)
    d = np.minimum(Y - (ny / 4.0 + offset), (3 * ny / 4.0 + offset) - Y)
    phi0 = tanh_profile(d, W)
    return case, phi0


def random_state_fields(case: Case, seed: int = 7, amp_u: float = 1e-3):
    """A smooth random phi0 in (0, 1) and small random u0, p0 for step-map tests."""
    rng = np.random.default_rng(seed)
    X, Y = grid(case)
    phi = np.full((case.ny, case.nx), 0.5)
    for _ in range(4):
        kx = rng.integers(1, 4) * 2 * np.pi / case.nx
        ky = rng.integers(1, 4) * 2 * np.pi / case.ny
        phi += 0.1 * np.sin(kx * X + rng.uniform(0, 6.3)) * np.cos(ky * Y + rng.uniform(0, 6.3))
    u0 = amp_u * rng.standard_normal((2, case.ny, case.nx))
    p0 = 1e-4 * rng.standard_normal((case.ny, case.nx))
    return np.clip(phi, 0.02, 0.98), u0, p0
