"""Ray generation for central cameras, float64 (oracle; test infrastructure).

Pixel (x, y) is sampled at its centre (x + 1/2, y + 1/2).

* Pinhole: camera-space direction ``((u - cx)/fx, (v - cy)/fy, 1)``.
* Equidistant fisheye: the polar angle from the optical axis is proportional
  to the image radius, ``theta = rho / f``; pixels with ``theta > theta_max``
  see nothing (RGBA 0).  Non-pinhole rendering of the same representation is
  the case the paper describes in Sec. 3.2 (last paragraph) and appendix D.

Axes are OpenCV (x right, y down, z forward); ``c2w`` maps camera to world
and its last column is the camera centre, which every ray starts from
(t >= 0, no near clip).
"""
from __future__ import annotations

import math

import numpy as np
import torch

F64 = torch.float64


def pixel_rays(cam, xs, ys):
    """Rays through pixel centres (xs, ys) (float arrays, pixel units).

    Returns ``o`` [3], ``d`` [R,3] (unit), ``valid`` [R] (bool)."""
    c2w = torch.as_tensor(np.asarray(cam.c2w, dtype=np.float32), dtype=F64)
    u = torch.as_tensor(np.asarray(xs, dtype=np.float64), dtype=F64)
    v = torch.as_tensor(np.asarray(ys, dtype=np.float64), dtype=F64)
    if cam.model == 0:
        dc = torch.stack([(u - float(np.float32(cam.cx))) / float(np.float32(cam.fx)),
                          (v - float(np.float32(cam.cy))) / float(np.float32(cam.fy)),
                          torch.ones_like(u)], dim=-1)
        valid = torch.ones(u.shape, dtype=torch.bool)
    elif cam.model == 1:
        dx = u - float(np.float32(cam.cx))
        dy = v - float(np.float32(cam.cy))
        rho = torch.sqrt(dx * dx + dy * dy)
        theta = rho / float(np.float32(cam.f_fish))
        valid = theta <= float(np.float32(cam.theta_max))
        phi = torch.atan2(dy, dx)
        st = torch.sin(theta)
        dc = torch.stack([st * torch.cos(phi), st * torch.sin(phi), torch.cos(theta)], dim=-1)
    else:
        raise ValueError(f"unknown camera model {cam.model}")
    d = dc @ c2w[:, :3].T
    d = d / torch.linalg.norm(d, dim=-1, keepdim=True)
    o = c2w[:, 3].clone()
    return o, d, valid


def generate_rays(cam, pix=None):
    """Rays for row-major pixel indices ``pix`` (default: the whole image)."""
    if pix is None:
        pix = np.arange(cam.width * cam.height)
    pix = np.asarray(pix, dtype=np.int64)
    xs = (pix % cam.width).astype(np.float64) + 0.5
    ys = (pix // cam.width).astype(np.float64) + 0.5
    return pixel_rays(cam, xs, ys)


def fov_check_angle(cam, x: float, y: float) -> float:
    """Angle in radians between the ray through (x, y) and the optical axis;
    a helper for the tests' closed forms."""
    o, d, _ = pixel_rays(cam, np.array([x]), np.array([y]))
    axis = torch.as_tensor(np.asarray(cam.c2w, dtype=np.float32), dtype=F64)[:, 2]
    axis = axis / torch.linalg.norm(axis)
    return float(math.acos(max(-1.0, min(1.0, float(d[0] @ axis)))))
