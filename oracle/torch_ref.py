"""Differentiable FP64 re-implementation of the time step on the CPU.

TEST INFRASTRUCTURE ONLY (part of the oracle: only ``tests/`` may use it).
It is the reference gradient for the hand-written adjoint of the GPU library:
the same method as ``lbm_oracle.c``, restated with whole-field PyTorch
operations so that ``torch.autograd`` differentiates a trajectory with respect
to the initial order parameter, the gravity vector and the four contact
angles.  It shares no code with the GPU library and does not call the C
oracle; the tests pin its forward map to the C oracle and its gradient to
central finite differences of the C oracle.

State of level n, as in the oracle's ``set_state``: post-streaming
populations f^n, g^n ([9][ny][nx]), the order parameter and velocity of
level n-1 (``phi_prev`` [ny][nx], ``u_prev`` [2][ny][nx]; unused at n = 0)
and n.  Stages of one step, in the order in which Sec. 3 defines them:
phi; ghost layer (periodic or Eq. Dwetting); stencils (App. C, Eqs. central1,
central2); closure (Sec. 2); u (Eq. comU); explicit-Euler time derivatives of
phi u, phi v, u m_x, v m_y, u m_y + v m_x (App. C); p (Eq. computP, second way
of Remark 1); both MRT collisions in moment space (Eq. MfMRAC1, Eq. MgMF1);
streaming with half-way bounce-back.
"""
from __future__ import annotations

import torch

CX = (0, 1, 0, -1, 0, 1, -1, -1, 1)
CY = (0, 0, 1, 0, -1, 1, 1, -1, -1)
WT = (4.0 / 9,) + (1.0 / 9,) * 4 + (1.0 / 36,) * 4
CS2 = 1.0 / 3.0
OPP = (0, 3, 4, 1, 2, 7, 8, 5, 6)
F64 = torch.float64


def moment_matrix() -> torch.Tensor:
    """M1 of App. C from its row polynomials in c_i: 1, e = -4 + 3|c|^2,
    eps = 4 - 21/2 |c|^2 + 9/2 |c|^4, j_x = c_x, q_x = (-5 + 3|c|^2) c_x,
    j_y, q_y likewise, p_xx = c_x^2 - c_y^2, p_xy = c_x c_y."""
    M = torch.zeros(9, 9, dtype=F64)
    for i in range(9):
        cx, cy = CX[i], CY[i]
        c2 = cx * cx + cy * cy
        M[0, i] = 1.0
        M[1, i] = -4.0 + 3.0 * c2
        M[2, i] = 4.0 - 10.5 * c2 + 4.5 * c2 * c2
        M[3, i] = cx
        M[4, i] = (-5.0 + 3.0 * c2) * cx
        M[5, i] = cy
        M[6, i] = (-5.0 + 3.0 * c2) * cy
        M[7, i] = cx * cx - cy * cy
        M[8, i] = cx * cy
    return M


class TorchRef:
    """One lattice; parameters from a ``workloads.Case``.  Gravity and contact
    angles are call arguments (tensors) so that gradients flow to them."""

    def __init__(self, case):
        self.c = case
        self.nx, self.ny = case.nx, case.ny
        self.n = case.nx * case.ny
        dphi = case.phiA - case.phiB
        self.dphi = dphi
        self.beta = 12.0 * case.sigma / (case.W * dphi ** 4)
        self.kap = 1.5 * case.sigma * case.W / dphi ** 2
        self.lamc = 4.0 / (case.W * dphi)           # sqrt(2 beta / k)
        self.drho = (case.rhoA - case.rhoB) / dphi
        sM = 1.0 / (case.M / (case.eta * CS2) + 0.5)
        self.sf = [s if s > 0 else 1.0 for s in case.s_f]
        if not case.s_f[3] > 0:
            self.sf[3] = sM
        if not case.s_f[5] > 0:
            self.sf[5] = sM
        self.sg = [s if s > 0 else 1.0 for s in case.s_g]
        self.snu_local = not (case.s_g[7] > 0 and case.s_g[8] > 0)
        self.M = moment_matrix()
        self.Minv = torch.linalg.inv(self.M)
        self.src = self._pull_index()

    # ---------------------------------------------------------------- streaming
    def _pull_index(self) -> torch.Tensor:
        """Flat index into the post-collision field [9][n] of every post-streaming
        population: f_i(x) comes from x - c_i, or, when x - c_i lies beyond a
        wall face, from the opposite population of x (half-way bounce-back)."""
        nx, ny, n = self.nx, self.ny, self.n
        y, x = torch.meshgrid(torch.arange(ny), torch.arange(nx), indexing="ij")
        idx = torch.empty(9, ny, nx, dtype=torch.long)
        for i in range(9):
            sx, sy = x - CX[i], y - CY[i]
            out = torch.zeros(ny, nx, dtype=torch.bool)
            if self.c.wall_x:
                out |= (sx < 0) | (sx >= nx)
            if self.c.wall_y:
                out |= (sy < 0) | (sy >= ny)
            sx, sy = sx % nx, sy % ny
            direct = i * n + sy * nx + sx
            back = OPP[i] * n + y * nx + x
            idx[i] = torch.where(out, back, direct)
        return idx.reshape(-1)

    def stream(self, post: torch.Tensor) -> torch.Tensor:
        return post.reshape(-1)[self.src].reshape(9, self.ny, self.nx)

    # ---------------------------------------------------------------- stencils
    def wet_ghost(self, theta, phi1, phi2):
        """Ghost value behind a wall of contact angle theta (Eq. Dwetting): the
        root phi_w of a phi_w^2 + b phi_w + c = 0 chosen by the paper, written
        -2c / (b + sqrt(b^2 - 4ac)), and the quadratic through (0, phi_w),
        (1/2, phi1), (3/2, phi2) evaluated at -1/2."""
        c = self.c
        a = 4.0 * torch.cos(theta) / (c.W * self.dphi)
        b = 8.0 / 3.0 - a * (c.phiA + c.phiB)
        cc = a * c.phiA * c.phiB + phi2 / 3.0 - 3.0 * phi1
        D = torch.clamp(b * b - 4.0 * a * cc, min=0.0)
        pw = -2.0 * cc / (b + torch.sqrt(D))
        return (8.0 * pw - 6.0 * phi1 + phi2) / 3.0

    def extend(self, phi, theta):
        """[ny+2][nx+2] field with one ghost layer: x-walls first, then y-walls
        over the extended rows (corners)."""
        if self.c.wall_x:
            left = self.wet_ghost(theta[0], phi[:, 0], phi[:, 1])
            right = self.wet_ghost(theta[1], phi[:, -1], phi[:, -2])
        else:
            left, right = phi[:, -1], phi[:, 0]
        mid = torch.cat([left[:, None], phi, right[:, None]], dim=1)
        if self.c.wall_y:
            bot = self.wet_ghost(theta[2], mid[0], mid[1])
            top = self.wet_ghost(theta[3], mid[-1], mid[-2])
        else:
            bot, top = mid[-1], mid[0]
        return torch.cat([bot[None], mid, top[None]], dim=0)

    def stencils(self, ext):
        """Isotropic gradient and Laplacian (App. C): sums over the eight
        neighbours with weights w_i c_i / cs^2 and 2 w_i (phi_i - phi) / cs^2."""
        ny, nx = self.ny, self.nx
        ctr = ext[1:ny + 1, 1:nx + 1]
        gx = torch.zeros_like(ctr)
        gy = torch.zeros_like(ctr)
        lap = torch.zeros_like(ctr)
        for i in range(1, 9):
            nb = ext[1 + CY[i]:1 + CY[i] + ny, 1 + CX[i]:1 + CX[i] + nx]
            gx = gx + WT[i] * CX[i] * nb
            gy = gy + WT[i] * CY[i] * nb
            lap = lap + 2.0 * WT[i] * (nb - ctr)
        return gx / CS2, gy / CS2, lap / CS2

    # ---------------------------------------------------------------- closure
    def closure(self, phi, gx, gy, lap, gravity):
        c = self.c
        out = {}
        out["mu"] = 4.0 * self.beta * (phi - c.phiA) * (phi - c.phiB) * (phi - 0.5 * (c.phiA + c.phiB)) \
            - self.kap * lap
        out["rho"] = self.drho * (phi - c.phiB) + c.rhoB
        out["drx"] = self.drho * gx
        out["dry"] = self.drho * gy
        gn = torch.sqrt(gx * gx + gy * gy + c.eps_n ** 2)
        lam = self.lamc * (c.phiA - phi) * (phi - c.phiB)
        out["lnx"] = lam * gx / gn
        out["lny"] = lam * gy / gn
        if c.model == "original":
            out["mx"] = torch.zeros_like(phi)
            out["my"] = torch.zeros_like(phi)
        else:
            out["mx"] = -self.drho * c.M * (gx - out["lnx"])
            out["my"] = -self.drho * c.M * (gy - out["lny"])
        out["Fx"] = out["mu"] * gx + c.body_force[0] + (out["rho"] - c.rho_ref) * gravity[0]
        out["Fy"] = out["mu"] * gy + c.body_force[1] + (out["rho"] - c.rho_ref) * gravity[1]
        t = (phi - c.phiB) / self.dphi
        if c.visc_law == "linear_mu":
            nu = (t * (c.rhoA * c.nuA - c.rhoB * c.nuB) + c.rhoB * c.nuB) / out["rho"]
        else:
            nu = 1.0 / (t * (1.0 / c.nuA - 1.0 / c.nuB) + 1.0 / c.nuB)
        out["snu"] = 1.0 / (nu / CS2 + 0.5) if self.snu_local else torch.full_like(phi, self.sg[7])
        return out

    # ---------------------------------------------------------------- moments
    def _mv(self, A, f):
        return torch.tensordot(A, f, dims=([1], [0]))

    def init(self, phi0, p0=None):
        """Level 0: f = M1^-1 m^eq_f(phi0, 0), g = M1^-1 m^eq_g(rho, p0, 0)."""
        c = self.c
        phi0 = phi0.to(F64)
        z = torch.zeros_like(phi0)
        pr = z if p0 is None else p0.to(F64)
        meq_f = torch.stack([phi0, -4.0 * phi0 + 2.0 * c.eta * phi0, 4.0 * phi0 - 3.0 * c.eta * phi0,
                             z, z, z, z, z, z])
        meq_g = torch.stack([z + c.rho0, -4.0 * c.rho0 + 6.0 * pr, 4.0 * c.rho0 - 9.0 * pr,
                             z, z, z, z, z, z])
        return dict(f=self._mv(self.Minv, meq_f), g=self._mv(self.Minv, meq_g),
                    phi_prev=phi0, u_prev=torch.zeros(2, self.ny, self.nx, dtype=F64), n=0)

    def macroscopic(self, st, gravity, theta):
        c = self.c
        f, g = st["f"], st["g"]
        phi = f.sum(0)
        gx, gy, lap = self.stencils(self.extend(phi, theta))
        cl = self.closure(phi, gx, gy, lap, gravity)
        jx = sum(CX[i] * g[i] for i in range(9) if CX[i])
        jy = sum(CY[i] * g[i] for i in range(9) if CY[i])
        u = (jx + 0.5 * cl["Fx"]) / cl["rho"]
        v = (jy + 0.5 * cl["Fy"]) / cl["rho"]
        prods = [phi * u, phi * v, u * cl["mx"], v * cl["my"], u * cl["my"] + v * cl["mx"]]
        if st["n"] > 0:
            pp, up, vp = st["phi_prev"], st["u_prev"][0], st["u_prev"][1]
            gxp, gyp, lapp = self.stencils(self.extend(pp, theta))
            clp = self.closure(pp, gxp, gyp, lapp, gravity)
            prev = [pp * up, pp * vp, up * clp["mx"], vp * clp["my"], up * clp["my"] + vp * clp["mx"]]
            d = [a - b for a, b in zip(prods, prev)]
        else:
            d = [torch.zeros_like(phi)] * 5
        Hc = (self.sg[2] - self.sg[0]) / (9.0 * self.sg[0] * self.sg[2])
        ugr = u * cl["drx"] + v * cl["dry"]
        trQ = cl["rho"] * (u * u + v * v) + (u * cl["mx"] + v * cl["my"])
        s0 = WT[0] * (-CS2 * trQ) / (2.0 * CS2 * CS2)
        uF = u * cl["Fx"] + v * cl["Fy"]
        pr = CS2 / (1.0 - WT[0]) * (g[1:].sum(0) + (0.5 + Hc) * ugr + s0 + (1.0 / 3.0) * (2.0 * uF + d[2] + d[3]))
        return dict(phi=phi, u=u, v=v, p=pr, d=d, **cl)

    def step(self, st, gravity, theta):
        c = self.c
        m = self.macroscopic(st, gravity, theta)
        phi, u, v, d = m["phi"], m["u"], m["v"], m["d"]
        z = torch.zeros_like(phi)
        # phase field (Eq. MfMRAC1)
        meq = torch.stack([phi, -4.0 * phi + 2.0 * c.eta * phi, 4.0 * phi - 3.0 * c.eta * phi,
                           phi * u, -phi * u, phi * v, -phi * v, z, z])
        rx = m["lnx"] / 3.0 + d[0]
        ry = m["lny"] / 3.0 + d[1]
        mR = torch.stack([z, z, z, rx, -rx, ry, -ry, z, z])
        mf = self._mv(self.M, st["f"])
        sf = torch.tensor(self.sf, dtype=F64)[:, None, None]
        fs = self._mv(self.Minv, mf - sf * (mf - meq) + (1.0 - sf / 2.0) * mR)
        # flow (Eq. MgMF1)
        rho, mx, my, Fx, Fy = m["rho"], m["mx"], m["my"], m["Fx"], m["Fy"]
        uu = u * u + v * v
        um = u * mx + v * my
        dum = d[2] + d[3]
        ugr = u * m["drx"] + v * m["dry"]
        uF = u * Fx + v * Fy
        r0 = c.rho0
        meqg = torch.stack([z + r0, -4.0 * r0 + (6.0 * m["p"] + 3.0 * rho * uu + 3.0 * um),
                            4.0 * r0 - (9.0 * m["p"] + 3.0 * rho * uu + 3.0 * um),
                            rho * u, -rho * u, rho * v, -rho * v,
                            u * mx - v * my + rho * (u * u - v * v),
                            (u * my + v * mx + 2.0 * rho * u * v) / 2.0])
        e1 = 3.0 * dum + 6.0 * uF
        mF = torch.stack([ugr, e1, -ugr - e1, Fx, -Fx, Fy, -Fy,
                          2.0 / 3.0 * (u * m["drx"] - v * m["dry"]) + 2.0 * (u * Fx - v * Fy) + (d[2] - d[3]),
                          1.0 / 3.0 * (u * m["dry"] + v * m["drx"]) + (2.0 * (u * Fy + v * Fx) + d[4]) / 2.0])
        sg = [torch.full_like(phi, s) for s in self.sg]
        sg[7] = m["snu"]
        sg[8] = m["snu"]
        sg = torch.stack(sg)
        mg = self._mv(self.M, st["g"])
        gs = self._mv(self.Minv, mg - sg * (mg - meqg) + (1.0 - sg / 2.0) * mF)
        return dict(f=self.stream(fs), g=self.stream(gs), phi_prev=phi, u_prev=torch.stack([u, v]),
                    n=st["n"] + 1)

    def run(self, st, nsteps, gravity, theta):
        for _ in range(nsteps):
            st = self.step(st, gravity, theta)
        return st

    @staticmethod
    def phi(st):
        return st["f"].sum(0)


def as_params(case):
    """Gravity and contact angles of a case as FP64 tensors requiring grad."""
    g = torch.tensor(list(case.gravity), dtype=F64, requires_grad=True)
    th = torch.tensor(list(case.theta), dtype=F64, requires_grad=True)
    return g, th


def loss_and_grads(case, phi0, target, nsteps, p0=None):
    """L = sum (phi^N - target)^2 from level 0 = init(phi0, p0) and its gradient
    with respect to phi0, gravity (2) and theta (4), by autograd."""
    ref = TorchRef(case)
    phi0 = torch.as_tensor(phi0, dtype=F64).clone().requires_grad_(True)
    p0 = None if p0 is None else torch.as_tensor(p0, dtype=F64)
    grav, theta = as_params(case)
    st = ref.run(ref.init(phi0, p0), nsteps, grav, theta)
    L = ((ref.phi(st) - torch.as_tensor(target, dtype=F64)) ** 2).sum()
    L.backward()
    return float(L.detach()), phi0.grad.numpy(), grav.grad.numpy(), theta.grad.numpy()


__all__ = ["TorchRef", "moment_matrix", "loss_and_grads", "as_params", "CX", "CY", "WT", "OPP"]
