"""Gradient-based search for the minimum of Omega_eps(Delta, q) per point and band.

Algorithm 1 of the paper scans a dense (Delta, q) grid.  With the gradient
of Omega available, the same minimum can be located by a quasi-Newton method
started from the best cells of a coarse grid.  Each (point, band) is an
independent problem in x = (Delta, qx) (Q on the kx axis, as in the grid
workloads).  The problems are solved together: one batched gradient launch per
function evaluation, and per-problem BFGS updates and step lengths, with x
kept inside the box [lo, hi] by projection.
"""
from __future__ import annotations

import math

import torch

from . import api


def bfgs_box(fun, x0, lo, hi, max_iter: int = 60, gtol: float = 1e-10,
             ftol: float = 1e-15, max_ls: int = 20):
    """Minimise many independent smooth functions at once.

    fun(x, sel) -> (f [k], g [k, n]) for the problems indexed by sel (a long
    tensor) at x [k, n].  x0 [P, n]; lo, hi broadcastable to x0.
    Projected BFGS with Armijo backtracking per problem.  A bound is active
    while x sits on it and the gradient pushes outward; the search direction
    has no component along active bounds.  Returns (x, f, iterations, converged)."""
    x = torch.minimum(torch.maximum(x0.clone(), lo), hi)
    P, n = x.shape
    dev, dt = x.device, x.dtype
    all_idx = torch.arange(P, device=dev)
    f, g = fun(x, all_idx)
    H = torch.eye(n, dtype=dt, device=dev).repeat(P, 1, 1)
    done = torch.zeros(P, dtype=torch.bool, device=dev)
    iters = torch.zeros(P, dtype=torch.long, device=dev)
    lo_b = lo.expand_as(x)
    hi_b = hi.expand_as(x)

    def free_mask(xx, gg, l, h):
        at_lo = (xx <= l) & (gg > 0)
        at_hi = (xx >= h) & (gg < 0)
        return ~(at_lo | at_hi)

    for it in range(max_iter):
        act = (~done).nonzero().flatten()
        if act.numel() == 0:
            break
        xa, fa, ga, Ha = x[act], f[act], g[act], H[act]
        la, ha = lo_b[act], hi_b[act]
        free = free_mask(xa, ga, la, ha)
        pg = torch.where(free, ga, torch.zeros_like(ga))
        conv = pg.abs().amax(dim=1) <= gtol
        d = -(Ha @ pg.unsqueeze(-1)).squeeze(-1)
        d = torch.where(free, d, torch.zeros_like(d))
        # fall back to steepest descent where BFGS does not descend
        bad = (d * pg).sum(dim=1) >= 0
        d = torch.where(bad.unsqueeze(1), -pg, d)
        alpha = torch.ones(act.numel(), dtype=dt, device=dev)
        accepted = conv.clone()
        x_new, f_new, g_new = xa.clone(), fa.clone(), ga.clone()
        for _ in range(max_ls):
            pend = (~accepted).nonzero().flatten()
            if pend.numel() == 0:
                break
            xt = torch.minimum(torch.maximum(xa[pend] + alpha[pend, None] * d[pend], la[pend]),
                               ha[pend])
            ft, gt = fun(xt, act[pend])
            ok = ft <= fa[pend] + 1e-4 * (ga[pend] * (xt - xa[pend])).sum(dim=1)
            okp = pend[ok]
            x_new[okp], f_new[okp], g_new[okp] = xt[ok], ft[ok], gt[ok]
            accepted[okp] = True
            alpha[pend[~ok]] *= 0.25
        # problems whose line search failed keep x and are considered converged
        stuck = ~accepted
        s = x_new - xa
        y = g_new - ga
        sy = (s * y).sum(dim=1)
        upd = (sy > 1e-12 * s.norm(dim=1) * y.norm(dim=1)) & accepted & ~conv
        if upd.any():
            rho = 1.0 / sy[upd]
            I = torch.eye(n, dtype=dt, device=dev).expand(int(upd.sum()), n, n)
            su, yu = s[upd], y[upd]
            V = I - rho[:, None, None] * su.unsqueeze(2) @ yu.unsqueeze(1)
            Ha[upd] = V @ Ha[upd] @ V.transpose(1, 2) + rho[:, None, None] * su.unsqueeze(2) @ su.unsqueeze(1)
        small = (fa - f_new).abs() <= ftol * fa.abs().clamp_min(1e-300)
        x[act], f[act], g[act], H[act] = x_new, f_new, g_new, Ha
        iters[act] += 1
        done[act] = conv | stuck | (small & accepted & (s.abs().amax(dim=1) == 0))
    return x, f, iters, done


def coarse_starts(model, pts, n_delta: int = 16, n_q: int = 8, dmax: float = 0.6,
                  qmax: float = math.pi / 8, k: int = 3, bands: int = api.OMEGA_BAND_BOTH,
                  device="cuda"):
    """The k lowest cells of a coarse (Delta, qx) grid per point and band.

    Delta: inclusive linspace(0, dmax, n_delta).  qx: n_q lattice momenta
    2 pi m / Lx spread over [0, qmax] (all points must share Lx).
    Returns starts [n_pts, nb, k, 2] (Delta, qx) and their Omega [n_pts, nb, k]."""
    Lx = pts[0][2]
    assert all(p[2] == Lx for p in pts), "coarse_starts needs one Lx per call"
    step = 2.0 * math.pi / Lx
    m_max = int(math.floor(qmax / step + 1e-9))
    ms = torch.unique(torch.round(torch.linspace(0, m_max, n_q, dtype=torch.float64)))
    delta = torch.linspace(0.0, dmax, n_delta, dtype=torch.float64, device=device)
    qx = (ms * step).to(device)
    q = torch.stack([qx, torch.zeros_like(qx)], dim=1)
    om = api.grid(model, pts, delta, q, bands, device=device)        # [P, nb, nq, nd]
    P, nb = om.shape[:2]
    vals, flat = torch.topk(om.reshape(P, nb, -1), k, dim=-1, largest=False)
    iq, idl = flat // n_delta, flat % n_delta
    starts = torch.stack([delta[idl], qx[iq]], dim=-1)
    return starts, vals


def _solve(model, owner_pts, x0, lo, hi, q_fixed, bands, max_iter, gtol, device, evals):
    """Minimise Omega_eps per owner point and band slot.

    x0 [O, nb, n]: n = 2 -> x = (Delta, qx); n = 1 -> x = (Delta,) with qx
    from q_fixed [O, nb].  Omega and its gradient are scaled per site."""
    O, nb, n = x0.shape
    n_site = torch.tensor([p[2] * p[3] for p in owner_pts], dtype=torch.float64,
                          device=device).repeat_interleave(nb)

    def fun(x, sel):
        own = sel // nb
        owners = torch.unique(own)
        r = torch.searchsorted(owners, own)
        bb = sel % nb
        xd = torch.zeros((owners.numel(), nb), dtype=torch.float64, device=device)
        xq = torch.zeros((owners.numel(), nb, 2), dtype=torch.float64, device=device)
        xd[r, bb] = x[:, 0]
        xq[r, bb, 0] = x[:, 1] if n == 2 else q_fixed.reshape(-1)[sel]
        pt_list = [owner_pts[o] for o in owners.tolist()]
        om, gd, gq, _ = api.grad(model, pt_list, xd, xq, bands, device=device)
        evals[0] += 1
        f = om[r, bb] / n_site[sel]
        if n == 2:
            g = torch.stack([gd[r, bb], gq[r, bb, 0]], dim=1) / n_site[sel, None]
        else:
            g = (gd[r, bb] / n_site[sel]).unsqueeze(1)
        return f, g

    x, f, iters, done = bfgs_box(fun, x0.reshape(O * nb, n), lo, hi, max_iter=max_iter,
                                 gtol=gtol)
    return x.reshape(O, nb, n), (f * n_site).reshape(O, nb), iters.reshape(O, nb), \
        done.reshape(O, nb)


def minimize_points(model, pts, starts, lo=(0.0, 0.0), hi=(0.6, math.pi / 8),
                    bands: int = api.OMEGA_BAND_BOTH, max_iter: int = 100, gtol: float = 1e-10,
                    device="cuda"):
    """Gradient-based search for the minimum of Omega_eps per point and band.

    1. From each start, quasi-Newton over continuous (Delta, qx) in the box.
    2. On a periodic Lx lattice the pair momentum is a multiple of 2 pi / Lx
       (Algorithm 1 scans such q); away from them Omega carries lattice-scale
       ripples at low T.  The continuous qx* is therefore snapped to its two
       neighbouring lattice momenta and Delta is minimised again at each.
    3. The lowest result over starts and neighbours wins.
    starts [n_pts, nb, k, 2] as (Delta, qx).  Returns (Delta, qx) [n_pts, nb, 2],
    Omega [n_pts, nb] and a statistics dict."""
    P, nb, k, _ = starts.shape
    evals = [0]
    lo_t = torch.tensor(lo, dtype=torch.float64, device=device)
    hi_t = torch.tensor(hi, dtype=torch.float64, device=device)
    own_pts = [pts[p] for p in range(P) for _ in range(k)]          # owner = p * k + s
    x0 = starts.permute(0, 2, 1, 3).reshape(P * k, nb, 2)
    x0 = torch.minimum(torch.maximum(x0, lo_t), hi_t)
    x1, f1, it1, done1 = _solve(model, own_pts, x0, lo_t, hi_t, None, bands, max_iter, gtol,
                                device, evals)
    # snap qx to the lattice: 2 neighbours per (owner, band)
    step = torch.tensor([2.0 * math.pi / p[2] for p in own_pts], dtype=torch.float64,
                        device=device)[:, None]
    m_lo = torch.floor(x1[..., 1] / step + 1e-12)
    m_hi_max = torch.floor(hi_t[1] / step + 1e-9)
    q_lo = m_lo * step
    q_hi = torch.minimum(m_lo + 1, m_hi_max) * step
    q_fix = torch.stack([q_lo, q_hi], dim=1)                          # [P*k, 2, nb]
    own2 = [p for p in own_pts for _ in range(2)]                      # owner = (p*k+s)*2 + c
    x2_0 = x1[..., :1].repeat_interleave(2, dim=0)                      # [P*k*2, nb, 1]
    x2, f2, it2, done2 = _solve(model, own2, x2_0, lo_t[:1], hi_t[:1],
                                q_fix.reshape(P * k * 2, nb), bands, max_iter, gtol,
                                device, evals)
    f2 = f2.reshape(P, k * 2, nb)
    best = f2.argmin(dim=1)                                             # [P, nb]
    d_all = x2[..., 0].reshape(P, k * 2, nb)
    q_all = q_fix.reshape(P, k * 2, nb)
    db = torch.gather(d_all, 1, best[:, None, :]).squeeze(1)
    qb = torch.gather(q_all, 1, best[:, None, :]).squeeze(1)
    fb = torch.gather(f2, 1, best[:, None, :]).squeeze(1)
    stats = {"gradient_launches": evals[0],
             "iterations_max": int(max(int(it1.max()), int(it2.max()))),
             "converged_fraction": float(torch.cat([done1.flatten(), done2.flatten()])
                                         .float().mean())}
    return torch.stack([db, qb], dim=-1), fb, stats
