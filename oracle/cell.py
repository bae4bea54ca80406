"""Per-cell geometry and shading in float64 (oracle; test infrastructure).

Every function here takes torch float64 tensors and is differentiable, so the
adjoint can re-evaluate the same formulas under autograd.

Readings of the paper used here (each also recorded in the design notes):

* Power bisector.  From the power-cell definition (appendix B),
  ``pow(x,i) <= pow(x,j)`` expands to ``2 (x - p_i).m <= |m|^2 + w_i - w_j``
  with ``m = p_j - p_i``.  The paper prints the offset with the weight terms
  swapped; the expansion of its own definition gives the sign used here (a
  larger own weight gives a larger cell).
* Dipole (Sec. 3.3).  The plane through ``p_i`` with normal ``n_i`` splits the
  cell; the half ``(x - p_i).n < delta`` (the side the normal points away
  from) is dense, the other half is empty.
* Displacement (Sec. 3.4, Eq. svdisp).  ``delta`` is the soft-Voronoi blend of
  the detail sites' displacements, evaluated at the ray's hit ``xbar`` with
  the undisplaced face; the dense set is then bounded by the face moved by
  ``delta`` along the normal, and the texture point ``x`` is the ray's hit
  with that moved face.
* Detail sites live in the face's 2-D frame: origin ``p_i``, axes from the
  orthonormal basis of Duff et al. (JCGT 2017) built from ``n_i``.
* Radiance (Sec. 3.4, Eq. svrad; Sec. 3.6): the soft-Voronoi blend at ``x`` of
  each detail site's Spherical-Voronoi function, taken here as
  ``softmax_m(a_km . d)``-weighted colours ``c_km`` of M axes, added to the
  cell's base colour ``rgb_i``.
* Density ``sigma_i = sigma_scale * softplus(lambda_i)``, opacity
  ``alpha = 1 - exp(-sigma * len)`` of the dense part of the bounded interval
  (exact integral of a piecewise-constant density, Sec. 3.1).
"""
from __future__ import annotations

import torch

F64 = torch.float64


def scene_tensors(scene, requires_grad: bool = False):
    """float32 scene arrays -> dict of float64 torch tensors."""
    out = {}
    for name in ("p", "power", "radius", "normal", "occ_logit", "rgb", "tex"):
        t = torch.as_tensor(getattr(scene, name)).to(F64).clone()
        if requires_grad:
            t.requires_grad_(True)
        out[name] = t
    out["sigma_scale"] = float(scene.sigma_scale)
    out["tau"] = float(scene.tau)
    return out


def power_distance(x, p, w):
    """pow(x, i) = |x - p_i|^2 - w_i (appendix B, power distance)."""
    diff = x - p
    return (diff * diff).sum(-1) - w


def bisector(p_i, w_i, p_j, w_j):
    """Half-space of cell i against j:  (x - p_i) . m <= h."""
    m = p_j - p_i
    h = 0.5 * ((m * m).sum(-1) + w_i - w_j)
    return m, h


def plane_hit(o, d, p_i, m, h):
    """Ray parameter where x(t) = o + t d meets the plane (x - p_i).m = h;
    returns (a, b) with a = d.m, b = h - (o - p_i).m, so t = b / a and the
    half-space reads t a <= b."""
    a = (d * m).sum(-1)
    b = h - ((o - p_i) * m).sum(-1)
    return a, b


def sphere_interval(o, d, p, r):
    """Ray interval inside B(p, r): returns (t0, t1, D) with D the
    discriminant; the interval is empty when D <= 0."""
    oc = o - p
    beta = (oc * d).sum(-1)
    D = beta * beta - ((oc * oc).sum(-1) - r * r)
    sq = torch.sqrt(torch.clamp(D, min=0.0))
    return -beta - sq, -beta + sq, D


def onb(nh):
    """Orthonormal tangent frame (t1, t2) of unit normal ``nh`` following
    Duff et al., "Building an Orthonormal Basis, Revisited", JCGT 2017."""
    x, y, z = nh[..., 0], nh[..., 1], nh[..., 2]
    sign = torch.copysign(torch.ones_like(z), z)
    a = -1.0 / (sign + z)
    b = x * y * a
    t1 = torch.stack([1.0 + sign * x * x * a, sign * b, -sign * x], dim=-1)
    t2 = torch.stack([b, sign + y * y * a, -y], dim=-1)
    return t1, t2


def softplus(x):
    return torch.nn.functional.softplus(x)


def split_tex(tex, m_axes: int):
    """tex [..., K, 3+6M] -> s [...,K,2], disp [...,K], axes [...,K,M,3],
    colours [...,K,M,3]."""
    s = tex[..., 0:2]
    disp = tex[..., 2]
    axes = tex[..., 3:3 + 3 * m_axes].reshape(*tex.shape[:-1], m_axes, 3)
    cols = tex[..., 3 + 3 * m_axes:3 + 6 * m_axes].reshape(*tex.shape[:-1], m_axes, 3)
    return s, disp, axes, cols


def soft_voronoi_weights(u, s, tau: float):
    """w_k(u) = exp(-tau |u - s_k|) / sum_k' exp(-tau |u - s_k'|)
    (Sec. 3.4, Eq. svdisp / Eq. svrad).  u [...,2], s [...,K,2]."""
    dist = torch.linalg.norm(u.unsqueeze(-2) - s, dim=-1)
    return torch.softmax(-tau * dist, dim=-1)


def shade(o, d, lo, hi, p, nraw, lam, rgb, tex, sigma_scale: float, tau: float):
    """Opacity and radiance of one ray segment [lo, hi] of a bounded cell.

    Shapes: o [...,3] (or [3]), d [...,3], lo/hi [...], p/nraw/rgb [...,3],
    lam [...], tex [...,K,3+6M].  Returns (alpha, colour [...,3], length of
    the dense part)."""
    m_axes = (tex.shape[-1] - 3) // 6
    nh = nraw / torch.linalg.norm(nraw, dim=-1, keepdim=True)
    t1, t2 = onb(nh)
    s, disp, axes, cols = split_tex(tex, m_axes)

    den = (d * nh).sum(-1)
    e0 = ((p - o) * nh).sum(-1)
    nz = den != 0
    den_safe = torch.where(nz, den, torch.ones_like(den))

    # hit with the undisplaced face -> displacement (Eq. svdisp)
    tbar = e0 / den_safe
    rel = o + tbar.unsqueeze(-1) * d - p
    ubar = torch.stack([(rel * t1).sum(-1), (rel * t2).sum(-1)], dim=-1)
    w_disp = soft_voronoi_weights(ubar, s, tau)
    delta = torch.where(nz, (w_disp * disp).sum(-1), torch.zeros_like(den))

    # hit with the displaced face -> texture point x
    tx = (e0 + delta) / den_safe
    t_pt = torch.where(nz, tx, 0.5 * (lo + hi))
    rel = o + t_pt.unsqueeze(-1) * d - p
    u = torch.stack([(rel * t1).sum(-1), (rel * t2).sum(-1)], dim=-1)

    # dense part: (x - p).n < delta  <=>  t den < e0 + delta
    jlo = torch.where(nz & (den < 0), torch.maximum(lo, tx), lo)
    jhi = torch.where(nz & (den > 0), torch.minimum(hi, tx), hi)
    flat_dense = ((o - p) * nh).sum(-1) < 0
    ell = torch.clamp(jhi - jlo, min=0.0)
    ell = torch.where(nz | flat_dense, ell, torch.zeros_like(ell))

    sigma = sigma_scale * softplus(lam)
    alpha = -torch.expm1(-sigma * ell)

    # radiance at x (Eq. svrad) with per-site Spherical-Voronoi colours
    w_rad = soft_voronoi_weights(u, s, tau)                        # [...,K]
    logits = (axes * d.unsqueeze(-2).unsqueeze(-2)).sum(-1)        # [...,K,M]
    v = torch.softmax(logits, dim=-1)
    sv = (v.unsqueeze(-1) * cols).sum(-2)                          # [...,K,3]
    colour = rgb + (w_rad.unsqueeze(-1) * sv).sum(-2)
    return alpha, colour, ell
