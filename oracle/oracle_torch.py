"""Second FP64 oracle in plain PyTorch CPU tensor ops.  TEST INFRASTRUCTURE ONLY.

Written separately from the C oracle (vectorised over whole fields instead of per-cell
loops) so that agreement between the two is a check on both.  Its main job is the
reference adjoint: autograd through this forward gives exact FP64 gradients of any
final-time stress/moment loss with respect to psi0, k_on, k_off and v0.

Kinks use one fixed branch rule, the same the hand-written adjoint has to follow:
`min` keeps its first argument on <=, `max` its first on >=, a superbee pair with a*b <= 0
takes the zero branch, and a donor-cell face with velocity exactly 0 takes the left cell.
`torch.where` routes the whole gradient to the chosen branch.

Model: Cook & Shinar, Sec. 2 Eqs. (1)-(6), Alg. 1 and Alg. 2 (see oracle.c for the readings
of the discretisation, which are the same here).
"""
from __future__ import annotations

import math

import torch
from torch.utils.checkpoint import checkpoint

TWO_PI = 2.0 * math.pi
f64 = torch.float64


def superbee(a, b):
    """sgn(b) max(min(2|a|,|b|), min(|a|,2|b|)) where a*b > 0, else 0."""
    aa, ab = a.abs(), b.abs()
    p = torch.where(2.0 * aa <= ab, 2.0 * aa, ab)
    q = torch.where(aa <= 2.0 * ab, aa, 2.0 * ab)
    r = torch.where(p >= q, p, q)
    signed = torch.where(b > 0, r, -r)
    return torch.where(a * b <= 0, torch.zeros_like(a), signed)


def motor_rhs(z, k_on, k_off, v0, ds, limiter=0):
    """Walk + attach/detach right-hand side along the last axis (s)."""
    zero = torch.zeros_like(z[..., :1])
    z_left = torch.cat([zero, z[..., :-1]], dim=-1)          # ghost z_{-1} = 0
    z_right = torch.cat([z[..., 1:], z[..., -1:]], dim=-1)   # ghost z_{ns} = z_{ns-1}
    if limiter == 0:
        sig = superbee(z - z_left, z_right - z)
    else:
        sig = torch.zeros_like(z)
    inner = v0 * (z[..., :-1] + 0.5 * sig[..., :-1])        # faces 1/2 .. ns-3/2
    outflow = v0 * z[..., -1:]                                # face ns-1/2, first order
    right = torch.cat([inner, outflow], dim=-1)               # Phi_{l+1/2}
    left = torch.cat([zero, right[..., :-1]], dim=-1)         # Phi_{l-1/2}, Phi_{-1/2} = 0
    return -(right - left) / ds + k_on - k_off * z


def motor_step(M, k_on, k_off, v0, dt, ds, limiter=0):
    Ms = M + (0.5 * dt) * motor_rhs(M, k_on, k_off, v0, ds, limiter)
    return M + dt * motor_rhs(Ms, k_on, k_off, v0, ds, limiter)


def s_moments(M, L):
    ns = M.shape[-1]
    ds = L / ns
    s = (torch.arange(ns, dtype=f64) + 0.5) * ds
    m0 = (M * ds).sum(-1)
    m1 = (M * ((s - 0.5 * L) * ds)).sum(-1)
    return m0, m1


def _tables(nth):
    dth = TWO_PI / nth
    k = torch.arange(nth, dtype=f64)
    return (torch.cos(k * dth), torch.sin(k * dth),
            torch.cos((k + 0.5) * dth), torch.sin((k + 0.5) * dth), dth)


def _donor(A, left, right):
    return torch.where(A >= 0, A * left, A * right)


def psi_step(psi, m0, u, G, F, dt, lx, ly):
    nx, ny, nth = psi.shape
    dx, dy = lx / nx, ly / ny
    cs, sn, ch, sh, dth = _tables(nth)
    ax = u[0][:, :, None] - F * m0 * cs
    ay = u[1][:, :, None] - F * m0 * sn
    Ax = 0.5 * (ax + torch.roll(ax, -1, 0))       # face i+1/2
    Ay = 0.5 * (ay + torch.roll(ay, -1, 1))       # face j+1/2
    Gxx, Gxy, Gyx, Gyy = (G[c][:, :, None] for c in range(4))
    At = -sh * (Gxx * ch + Gxy * sh) + ch * (Gyx * ch + Gyy * sh)   # face k+1/2
    fx = _donor(Ax, psi, torch.roll(psi, -1, 0))
    fy = _donor(Ay, psi, torch.roll(psi, -1, 1))
    ft = _donor(At, psi, torch.roll(psi, -1, 2))
    div = ((fx - torch.roll(fx, 1, 0)) / dx + (fy - torch.roll(fy, 1, 1)) / dy
           + (ft - torch.roll(ft, 1, 2)) / dth)
    return psi - dt * div


def theta_moments(psi, m0, m1, F, sigma_f):
    """Returns stress[3] (xx, xy, yy) and moments[7] (c, nx, ny, Dxx, Dxy, Dyy, B)."""
    nth = psi.shape[-1]
    dth = TWO_PI / nth
    th = torch.arange(nth, dtype=f64) * dth
    c, s = torch.cos(th), torch.sin(th)
    h1, h2 = 0.5 * torch.cos(2 * th), 0.5 * torch.sin(2 * th)
    w = lambda x: (psi * x).sum(-1) * dth
    mom = torch.stack([w(torch.ones_like(c)), w(c), w(s), w(c * c), w(c * s), w(s * s), w(m0)])
    stress = torch.stack([w(sigma_f * h1 + F * m1 * c * c),
                          w(sigma_f * h2 + F * m1 * c * s),
                          w(-sigma_f * h1 + F * m1 * s * s)])
    return stress, mom


def motor_force(psi, M, F, L, lx, ly):
    """Eq. (10): F p psi M ds dth of every motor cell spread from its head position
    (x, y) + (s - L/2) p onto the cell centres with the bilinear hat, periodic."""
    nx, ny, nth, ns = M.shape
    dx, dy, dth, ds = lx / nx, ly / ny, TWO_PI / nth, L / ns
    th = torch.arange(nth, dtype=f64) * dth
    co, si = torch.cos(th), torch.sin(th)
    lever = (torch.arange(ns, dtype=f64) + 0.5) * ds - 0.5 * L
    xc = (torch.arange(nx, dtype=f64) + 0.5) * dx
    yc = (torch.arange(ny, dtype=f64) + 0.5) * dy
    hx = xc[:, None, None, None] + lever[None, None, None, :] * co[None, None, :, None]
    hy = yc[None, :, None, None] + lever[None, None, None, :] * si[None, None, :, None]
    fx, fy = hx / dx - 0.5, hy / dy - 0.5
    ix, iy = torch.floor(fx), torch.floor(fy)
    ax, ay = fx - ix, fy - iy
    i0 = torch.remainder(ix.long(), nx)
    j0 = torch.remainder(iy.long(), ny)
    i0, j0 = torch.broadcast_to(i0, M.shape), torch.broadcast_to(j0, M.shape)
    v = F * psi[..., None] * M * (ds * dth)
    out = torch.zeros(2, nx * ny, dtype=f64)
    for di, dj, w in ((0, 0, (1 - ax) * (1 - ay)), (1, 0, ax * (1 - ay)), (0, 1, (1 - ax) * ay), (1, 1, ax * ay)):
        cell = ((i0 + di) % nx) * ny + (j0 + dj) % ny
        vw = torch.broadcast_to(v * w, M.shape)
        out[0].index_add_(0, cell.reshape(-1), (vw * co[None, None, :, None]).reshape(-1))
        out[1].index_add_(0, cell.reshape(-1), (vw * si[None, None, :, None]).reshape(-1))
    return out.reshape(2, nx, ny)


class Problem:
    """Grid constants of one run (plain attributes, float64 everywhere)."""

    def __init__(self, p):
        self.p = p
        self.ds = p.L / p.ns

    def depletion(self, psi, M, k_on):
        """Eqs. (5)-(6) with the over-binding clamp of Alg. 2 on the current state: the coarse
        bound density B = sum_th psi m0 dth per (x, y); where B > m_total every column there
        is scaled by m_total / B and the free pool is 0, elsewhere the pool is m_total - B.
        Returns the scaled M and the attachment source k_on * pool, shaped to broadcast."""
        p = self.p
        dth = TWO_PI / p.ntheta
        m0, _ = s_moments(M, p.L)
        B = (psi * m0).sum(-1) * dth
        over = B > p.m_total
        # the masked branch divides by 1, not by B: where B = 0 a division by B would carry
        # 0 * inf = NaN into the gradient even though its value is discarded
        scale = torch.where(over, p.m_total / torch.where(over, B, torch.ones_like(B)),
                            torch.ones_like(B))
        src = torch.where(over, torch.zeros_like(B), k_on * (p.m_total - B))
        return M * scale[:, :, None, None], src[:, :, None, None]

    def substeps(self, v0, k_off, dt):
        """Alg. 2's inner loop: n steps of dt/n, n = ceil(dt (v0/ds + k_off) / motor_cfl) (at
        least 1), the motor stability limit being the same at every point; 1 without
        sub-cycling."""
        cfl = getattr(self.p, "motor_cfl", 0.0)
        if not cfl > 0.0:
            return 1
        rate = float(v0) / (self.p.L / self.p.ns) + float(k_off)
        return max(1, int(math.ceil(dt * rate / cfl)))

    def step(self, psi, M, k_on, k_off, v0, u, G, dt):
        """Motors (n sub-steps, each starting with the clamp and the pool of the current
        sub-state when m_total > 0), then psi driven by the new m0."""
        p = self.p
        n = self.substeps(v0, k_off, dt)
        M1 = M
        for _ in range(n):
            src = k_on
            if getattr(p, "m_total", 0.0) > 0.0:
                M1, src = self.depletion(psi, M1, k_on)
            M1 = motor_step(M1, src, k_off, v0, dt / n, self.ds, p.limiter)
        m0, _ = s_moments(M1, p.L)
        psi1 = psi_step(psi, m0, u, G, p.F, dt, p.lx, p.ly)
        return psi1, M1

    def outputs(self, psi, M):
        m0, m1 = s_moments(M, self.p.L)
        return theta_moments(psi, m0, m1, self.p.F, self.p.sigma_f)

    def run(self, psi, M, k_on, k_off, v0, fluids, K, nsteps, dt, ckpt=0):
        """nsteps micro-steps; fluid field e = step // K.  ckpt > 0 recomputes segments of
        ckpt steps in the backward pass instead of storing every intermediate."""
        def seg(psi, M, k_on, k_off, v0, n0, n1):
            for n in range(n0, n1):
                u, G = fluids[min(n // K, len(fluids) - 1)]
                psi, M = self.step(psi, M, k_on, k_off, v0, u, G, dt)
            return psi, M

        if ckpt <= 0:
            return seg(psi, M, k_on, k_off, v0, 0, nsteps)
        for n0 in range(0, nsteps, ckpt):
            n1 = min(nsteps, n0 + ckpt)
            psi, M = checkpoint(seg, psi, M, k_on, k_off, v0, n0, n1, use_reentrant=False)
        return psi, M


def to_t(a):
    return torch.as_tensor(a, dtype=f64)


def forward(p, psi0, M0, fluids, K, nsteps, dt):
    """Final (psi, M, stress, moments) as float64 tensors."""
    pr = Problem(p)
    fl = [(to_t(u), to_t(g)) for u, g in fluids]
    with torch.no_grad():
        psi, M = pr.run(to_t(psi0), to_t(M0), to_t(p.k_on), to_t(p.k_off), to_t(p.v0),
                        fl, K, nsteps, dt)
        stress, mom = pr.outputs(psi, M)
    return psi, M, stress, mom


def gradients(p, psi0, M0, fluids, K, nsteps, dt, g_stress=None, g_mom=None,
              loss_fn=None, ckpt=0):
    """Gradients of L(stress(T), moments(T)) with respect to psi0, k_on, k_off, v0.

    L is <g_stress, stress> + <g_mom, moments> (a vector-Jacobian product), or loss_fn(stress,
    moments) when given.  dt is held fixed.  Returns (L, g_psi0, [g_kon, g_koff, g_v0]).
    """
    pr = Problem(p)
    fl = [(to_t(u), to_t(g)) for u, g in fluids]
    psi = to_t(psi0).clone().requires_grad_(True)
    kon = to_t(p.k_on).clone().requires_grad_(True)
    koff = to_t(p.k_off).clone().requires_grad_(True)
    v0 = to_t(p.v0).clone().requires_grad_(True)
    psiT, MT = pr.run(psi, to_t(M0), kon, koff, v0, fl, K, nsteps, dt, ckpt=ckpt)
    stress, mom = pr.outputs(psiT, MT)
    if loss_fn is not None:
        loss = loss_fn(stress, mom)
    else:
        loss = torch.zeros((), dtype=f64)
        if g_stress is not None:
            loss = loss + (stress * to_t(g_stress)).sum()
        if g_mom is not None:
            loss = loss + (mom * to_t(g_mom)).sum()
    gp, g1, g2, g3 = torch.autograd.grad(loss, [psi, kon, koff, v0], allow_unused=True)
    z = lambda g: 0.0 if g is None else float(g)
    return float(loss.detach()), gp.detach().numpy(), [z(g1), z(g2), z(g3)]
