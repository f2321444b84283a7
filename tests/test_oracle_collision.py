"""Pin of the oracle's collision: the moment form it runs (Eq. evoPF, second
line; Remark 2 for g) equals the velocity-space matrix form the paper writes
first, f - Lambda (f - f^eq) + (I - Lambda/2) R with Lambda = M^-1 S M
(Eq. evoPF, first line; Eq. evoNS), on random inputs and random rates.

Everything on the matrix side is built here, independently of the oracle's
tables: M from the polynomial definitions of its rows over the velocity set,
Lambda with numpy's inverse, f^eq and R in velocity space from their
definitions (f^eq_i = w_i phi (1 + c_i.u / cs^2) with eta = 1, and
R_i = w_i c_i.V / cs^2 for the source whose moments the App. C list
gives: V = d_t(phi u) + cs^2 lambda n), g^eq and F_i from the direct Sec. 3
forms (Eq. geq and the force distribution with M_2F in the second way of
Remark 1).  A dropped (I - S/2), a rate on the wrong row, a transposed
Lambda or a wrong inverse fails these checks.
"""
import numpy as np
import pytest

import oracle
import workloads as W

CX, CY, WT, _, _ = oracle.lattice()
CS2 = 1.0 / 3.0


def _m_matrix():
    """Rows of M1 (App. C) as polynomials of the velocity: 1, energy -4 + 3|c|^2,
    energy square 4 - 21|c|^2/2 + 9|c|^4/2, c_x, heat flux (3|c|^2 - 5) c_x, c_y,
    (3|c|^2 - 5) c_y, c_x^2 - c_y^2, c_x c_y."""
    cx, cy = CX.astype(float), CY.astype(float)
    c2 = cx * cx + cy * cy
    return np.stack([np.ones(9), -4 + 3 * c2, 4 - 10.5 * c2 + 4.5 * c2 * c2, cx, (3 * c2 - 5) * cx, cy,
                     (3 * c2 - 5) * cy, cx * cx - cy * cy, cx * cy])


M = _m_matrix()
MINV = np.linalg.inv(M)


def _matrix_form(S, fv, feq, R):
    lam = MINV @ np.diag(S) @ M
    return fv - lam @ (fv - feq) + (np.eye(9) - 0.5 * lam) @ R


@pytest.mark.parametrize("rates", ["paper_default", "random"])
def test_phase_field_collision_moment_form_equals_matrix_form(rates):
    rng = np.random.default_rng(211 if rates == "random" else 212)
    case = W.Case(nx=4, ny=4, M=0.05)
    sM = 1.0 / (case.M / CS2 + 0.5)
    for _ in range(20):
        phi, u, v = rng.uniform(0, 1), rng.normal(0, 0.05), rng.normal(0, 0.05)
        lnx, lny = rng.normal(0, 0.2), rng.normal(0, 0.2)
        dpu, dpv = rng.normal(0, 1e-3), rng.normal(0, 1e-3)
        S = np.ones(9)
        S[3] = S[5] = sM
        if rates == "random":
            S = rng.uniform(0.3, 1.9, 9)
        fv = rng.uniform(0, 0.5, 9)
        meq, mR = oracle.moments_f(case, phi, u, v, lnx, lny, dpu, dpv)
        out = oracle.collide_node(S, fv, meq, mR)
        cu = CX * u + CY * v
        feq = WT * phi * (1 + cu / CS2)
        V = (dpu + CS2 * lnx, dpv + CS2 * lny)
        R = WT * (CX * V[0] + CY * V[1]) / CS2
        ref = _matrix_form(S, fv, feq, R)
        np.testing.assert_allclose(out, ref, rtol=0, atol=1e-14 * max(1.0, np.abs(ref).max()))


@pytest.mark.parametrize("rates", ["paper_default", "random"])
def test_hydrodynamic_collision_moment_form_equals_matrix_form(rates):
    rng = np.random.default_rng(311 if rates == "random" else 312)
    case = W.Case(nx=4, ny=4, rhoA=10.0, rhoB=1.0, rho0=0.3)
    for _ in range(20):
        a = dict(rho=rng.uniform(1, 10), pr=rng.normal(0, 1e-2), u=rng.normal(0, 0.05), v=rng.normal(0, 0.05),
                 mx=rng.normal(0, 0.01), my=rng.normal(0, 0.01), Fx=rng.normal(0, 1e-3), Fy=rng.normal(0, 1e-3),
                 drx=rng.normal(0, 0.5), dry=rng.normal(0, 0.5), d_umx=rng.normal(0, 1e-4),
                 d_vmy=rng.normal(0, 1e-4), d_cross=rng.normal(0, 1e-4))
        args = [a[k] for k in ("rho", "pr", "u", "v", "mx", "my", "Fx", "Fy", "drx", "dry", "d_umx", "d_vmy",
                               "d_cross")]
        S = np.ones(9)
        S[7] = S[8] = rng.uniform(0.5, 1.9)
        if rates == "random":
            S = rng.uniform(0.3, 1.9, 9)
        gv = rng.normal(0, 0.1, 9)
        meq, mF = oracle.moments_g(case, *args)
        out = oracle.collide_node(S, gv, meq, mF)
        geq, Fi = oracle.direct_g(case, *args)
        ref = _matrix_form(S, gv, geq, Fi)
        np.testing.assert_allclose(out, ref, rtol=0, atol=1e-14 * max(1.0, np.abs(ref).max()))


def test_matrix_built_here_equals_the_oracles_table():
    """The oracle's M1 table is the matrix of the row polynomials."""
    _, _, _, Mo, Mio = oracle.lattice()
    np.testing.assert_array_equal(Mo, M)
    np.testing.assert_allclose(Mio, MINV, atol=1e-15)
