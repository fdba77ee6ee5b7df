"""FP64 PyTorch-CPU forward used only for exact reverse-mode gradients.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper differentiates the ReLU-polynomial kernel to optimise scenes with
it (Sec. 4.3 ablation, Sec. 5.3). This module writes the whole forward pass
again, independently of ``oracle.c``, with plain float64 torch operations on
the CPU, so that autograd gives the exact derivative of the piecewise-smooth
image with respect to every scene parameter. Discrete decisions (near-plane
cull, tile rectangles, alpha < eps skips, early termination) are taken on
detached values, exactly as in the brute-force reference, and carry no
gradient; on an included pair alpha >= eps > 0, so the polynomial is strictly
positive there and the ReLU kink never enters a gradient.

Pins: the forward matches ``oracle.c`` to 1e-10 on the same inputs, and the
gradient matches FP64 central finite differences of ``oracle.c`` (tests).
Small problems only: it loops over splats in Python and keeps every pixel.
"""
import math

import numpy as np
import torch

KERNEL_EXP, KERNEL_POLY = 0, 1
RADIUS_SIGMA3, RADIUS_POLY_UNIVERSAL, RADIUS_POLY_OPACITY, RADIUS_EXP_OPACITY = 0, 1, 2, 3

_PI = math.pi


def _sh_basis(deg, d):
    """Real SH basis (3DGS ordering and signs) at unit directions d [n, 3]."""
    x, y, z = d[:, 0], d[:, 1], d[:, 2]
    Y = [torch.full_like(x, math.sqrt(1.0 / (4.0 * _PI)))]
    if deg >= 1:
        k1 = math.sqrt(3.0 / (4.0 * _PI))
        Y += [-k1 * y, k1 * z, -k1 * x]
    if deg >= 2:
        a, b, c = math.sqrt(15.0 / (4.0 * _PI)), math.sqrt(5.0 / (16.0 * _PI)), math.sqrt(15.0 / (16.0 * _PI))
        Y += [a * x * y, -a * y * z, b * (2 * z * z - x * x - y * y), -a * x * z, c * (x * x - y * y)]
    if deg >= 3:
        a = math.sqrt(35.0 / (32.0 * _PI))
        b = math.sqrt(105.0 / (4.0 * _PI))
        c = math.sqrt(21.0 / (32.0 * _PI))
        dd = math.sqrt(7.0 / (16.0 * _PI))
        e = math.sqrt(105.0 / (16.0 * _PI))
        Y += [-a * y * (3 * x * x - y * y), b * x * y * z, -c * y * (4 * z * z - x * x - y * y),
              dd * z * (2 * z * z - 3 * x * x - 3 * y * y), -c * x * (4 * z * z - x * x - y * y),
              e * z * (x * x - y * y), -a * x * (x * x - 3 * y * y)]
    return torch.stack(Y, dim=1)


def _first_root(c, order, target):
    """First x >= 0 with p(x) = target (bisection on a scanned bracket)."""
    p = lambda x: sum(c[i] * x ** i for i in range(order + 1)) - target
    if p(0.0) < 0:
        return -1.0
    if p(0.0) == 0:
        return 0.0
    a, h = 0.0, 1.0 / 1024.0
    while a < 4096.0:
        b = a + h
        if p(b) <= 0:
            lo, hi = a, b
            for _ in range(200):
                m = 0.5 * (lo + hi)
                if m <= lo or m >= hi:
                    break
                if p(m) > 0:
                    lo = m
                else:
                    hi = m
            return hi
        a = b
    return -1.0


def project(means3d, scales, quats, opacities, sh, sh_degree, cam, cfg):
    """Differentiable projection. Returns a dict of torch tensors (u, v, conic
    a, b, c, opacity, rgb) plus detached numpy rect, depth32 and visibility."""
    vm = torch.as_tensor(np.asarray(cam.viewmat, np.float64))
    R, tv = vm[:3, :3], vm[:3, 3]
    fx, fy, cx, cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    W, H = int(cam.width), int(cam.height)
    t = means3d @ R.T + tv
    tz = t[:, 2]
    visible = (tz.detach() >= cfg.near_z)

    q = quats / quats.norm(dim=1, keepdim=True)
    w, x, y, z = q.unbind(1)
    Rq = torch.stack([
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1)], 1)
    M = Rq * scales[:, None, :]
    Sig = M @ M.transpose(1, 2)

    limx, limy = 1.3 * W / (2.0 * fx), 1.3 * H / (2.0 * fy)
    txz = torch.clamp(t[:, 0] / tz, -limx, limx)
    tyz = torch.clamp(t[:, 1] / tz, -limy, limy)
    zero = torch.zeros_like(tz)
    J = torch.stack([torch.stack([fx / tz, zero, -fx * txz / tz], -1),
                     torch.stack([zero, fy / tz, -fy * tyz / tz], -1)], 1)
    TW = J @ R
    S2 = TW @ Sig @ TW.transpose(1, 2)
    a0, b0, c0 = S2[:, 0, 0], 0.5 * (S2[:, 0, 1] + S2[:, 1, 0]), S2[:, 1, 1]
    det0 = a0 * c0 - b0 * b0
    aa, ca = a0 + cfg.aa_v, c0 + cfg.aa_v
    deta = aa * ca - b0 * b0
    opac = opacities * torch.sqrt(torch.clamp(det0 / deta, min=0.0))
    con_a, con_b, con_c = ca / deta, -b0 / deta, aa / deta
    u = fx * t[:, 0] / tz + cx
    v = fy * t[:, 1] / tz + cy

    campos = -(R.T @ tv)
    d = means3d - campos
    d = d / d.norm(dim=1, keepdim=True)
    Y = _sh_basis(sh_degree, d)
    rgb = torch.clamp(torch.einsum("nk,nkc->nc", Y, sh) + 0.5, min=0.0)

    # discrete part: radius, rectangle, culls (no gradient)
    with torch.no_grad():
        on = opac.detach().numpy()
        mid = 0.5 * (aa + ca).detach().numpy()
        dn = deta.detach().numpy()
        lmax = mid + np.sqrt(np.maximum(mid * mid - dn, 0.0))
        n = on.shape[0]
        k = np.zeros(n)
        ok = visible.numpy() & (dn > 0)
        c = list(cfg.coeffs) + [0.0] * 4
        for i in range(n):
            if not ok[i]:
                continue
            if cfg.radius_mode == RADIUS_SIGMA3:
                k[i] = 3.0
            elif cfg.radius_mode == RADIUS_POLY_UNIVERSAL:
                k[i] = math.sqrt(_first_root(c, cfg.order, 0.0))
            elif cfg.radius_mode == RADIUS_POLY_OPACITY:
                xr = _first_root(c, cfg.order, cfg.eps / on[i]) if on[i] > 0 else -1.0
                if xr < 0:
                    ok[i] = False
                else:
                    k[i] = math.sqrt(xr)
            else:
                if on[i] >= cfg.eps:
                    k[i] = math.sqrt(2.0 * math.log(on[i] / cfg.eps))
                else:
                    ok[i] = False
        r = k * np.sqrt(lmax) * cfg.radius_pad
        T = cfg.tile
        gx, gy = (W + T - 1) // T, (H + T - 1) // T
        un, vn = u.detach().numpy(), v.detach().numpy()
        x0 = np.clip(np.floor((un - r) / T), 0, gx)
        x1 = np.clip(np.floor((un + r) / T), -1, gx - 1)
        y0 = np.clip(np.floor((vn - r) / T), 0, gy)
        y1 = np.clip(np.floor((vn + r) / T), -1, gy - 1)
        empty = ~ok | (x1 < x0) | (y1 < y0)
        rect = np.stack([x0, y0, x1, y1], 1).astype(np.int64)
        rect[empty] = (0, 0, -1, -1)
        depth32 = tz.detach().numpy().astype(np.float32)
    return dict(u=u, v=v, a=con_a, b=con_b, c=con_c, opac=opac, rgb=rgb, rect=rect, depth32=depth32)


def _kernel(cfg, x0, Q):
    if cfg.kind == KERNEL_EXP:
        return torch.exp(-0.5 * Q)
    c = list(cfg.coeffs) + [0.0] * 4
    p = sum(c[i] * Q ** i for i in range(cfg.order + 1))
    if cfg.order == 2:
        p = torch.where(Q.detach() >= x0, torch.zeros_like(p), p)
    return torch.clamp(p, min=0.0)


def render(means3d, scales, quats, opacities, sh, sh_degree, cam, cfg, proj=None):
    """Differentiable image [3, H, W] (plus final T) over every pixel."""
    if proj is None:
        proj = project(means3d, scales, quats, opacities, sh, sh_degree, cam, cfg)
    W, H, Tt = int(cam.width), int(cam.height), cfg.tile
    ys, xs = np.mgrid[0:H, 0:W]
    pxn, pyn = xs.ravel(), ys.ravel()
    px = torch.as_tensor(pxn + 0.5, dtype=torch.float64)
    py = torch.as_tensor(pyn + 0.5, dtype=torch.float64)
    tx, ty = pxn // Tt, pyn // Tt
    order = np.lexsort((np.arange(proj["depth32"].shape[0]), proj["depth32"]))
    x0 = _first_root(list(cfg.coeffs) + [0.0] * 4, cfg.order, 0.0) if cfg.kind == KERNEL_POLY else 0.0
    P = pxn.shape[0]
    T = torch.ones(P, dtype=torch.float64)
    C = torch.zeros(P, 3, dtype=torch.float64)
    done = np.zeros(P, bool)
    for i in order:
        r = proj["rect"][i]
        inrect = (tx >= r[0]) & (tx <= r[2]) & (ty >= r[1]) & (ty <= r[3]) & ~done
        if not inrect.any():
            continue
        dx, dy = px - proj["u"][i], py - proj["v"][i]
        Q = proj["a"][i] * dx * dx + 2.0 * proj["b"][i] * dx * dy + proj["c"][i] * dy * dy
        alpha = torch.clamp(proj["opac"][i] * _kernel(cfg, x0, Q), max=cfg.alpha_max)
        an = alpha.detach().numpy()
        inc = inrect & (an >= cfg.eps)
        Tn = T * (1.0 - alpha)
        stop = inc & (Tn.detach().numpy() < cfg.t_min)
        done |= stop
        inc &= ~stop
        m = torch.as_tensor(inc)
        C = C + torch.where(m[:, None], proj["rgb"][i][None, :] * (alpha * T)[:, None], torch.zeros_like(C))
        T = torch.where(m, Tn, T)
    bg = torch.as_tensor(np.asarray(cfg.bg, np.float64))
    img = C + T[:, None] * bg[None, :]
    return img.T.reshape(3, H, W), T.reshape(H, W)
