"""Seeded synthetic inputs: scenes, cameras, targets and request streams.

This module only draws random numbers and packs them into plain arrays.  It
holds none of the renderer's arithmetic (no power distances, planes,
intervals, shading or compositing), so that the CPU oracle and the GPU
library can both take their inputs from it without sharing method code.

Scene parameters follow the cell parameterisation of the paper: a site
``p_i`` with a power weight ``w_i`` and a bounding-sphere radius ``r_i``
(Sec. 3.2, power cell definition), an oriented dipole normal ``n_i`` with a
density (Sec. 3.3), and ``K`` detail sites per dipole face, each carrying a
2-D position, a scalar displacement and a Spherical-Voronoi radiance with
``M`` axes (Sec. 3.4 and Sec. 3.6, "Model Configurations").

Texture layout per (cell, detail site), 3 + 6M floats:
``[s.x, s.y, d, a_0.xyz .. a_{M-1}.xyz, c_0.rgb .. c_{M-1}.rgb]``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

K_DETAIL = 8      # detail sites per dipole face (Sec. 3.6)
M_AXES = 8        # Spherical-Voronoi axes per detail site (Sec. 3.6)
SIGMA_SCALE = 10.0  # density scale per world unit (scene constant)
TAU = 20.0          # soft-Voronoi temperature per world unit (scene constant)

SEED_SCENE, SEED_CAMERAS, SEED_TARGETS, SEED_REQUESTS, SEED_FD, SEED_STEINER = 0, 1, 2, 3, 4, 5


def tex_width(m_axes: int) -> int:
    return 3 + 6 * m_axes


@dataclasses.dataclass
class Scene:
    """Structure-of-arrays cell parameters, all float32, C-contiguous."""
    p: np.ndarray          # [N,3] sites
    power: np.ndarray      # [N]   power weights w_i
    radius: np.ndarray     # [N]   bounding-sphere radii r_i
    normal: np.ndarray     # [N,3] dipole normals (raw, normalised on use)
    occ_logit: np.ndarray  # [N]   density logits
    rgb: np.ndarray        # [N,3] base colour
    tex: np.ndarray        # [N,K,3+6M] detail-site texture
    sigma_scale: float = SIGMA_SCALE
    tau: float = TAU

    @property
    def n(self) -> int:
        return int(self.p.shape[0])

    @property
    def k_detail(self) -> int:
        return int(self.tex.shape[1])

    @property
    def m_axes(self) -> int:
        return (int(self.tex.shape[2]) - 3) // 6

    def subset(self, idx) -> "Scene":
        idx = np.asarray(idx)
        return Scene(*(np.ascontiguousarray(getattr(self, f)[idx]) for f in
                       ("p", "power", "radius", "normal", "occ_logit", "rgb", "tex")),
                     sigma_scale=self.sigma_scale, tau=self.tau)

    def copy(self) -> "Scene":
        return self.subset(np.arange(self.n))


@dataclasses.dataclass
class Camera:
    """A central camera.  ``c2w`` is a row-major 3x4 camera-to-world matrix
    with OpenCV axes (x right, y down, z forward); its last column is the
    camera centre.  ``model`` 0 = pinhole, 1 = equidistant fisheye."""
    model: int
    width: int
    height: int
    c2w: np.ndarray        # [3,4] float32
    fx: float = 0.0
    fy: float = 0.0
    cx: float = 0.0
    cy: float = 0.0
    f_fish: float = 0.0
    theta_max: float = 0.0

    @property
    def n_rays(self) -> int:
        return self.width * self.height


def _attributes(rng: np.random.Generator, n: int, k: int, m: int):
    s = rng.uniform(0.02, 0.1, size=n)
    lam = rng.normal(0.0, 1.0, size=n)
    rgb = rng.uniform(0.0, 1.0, size=(n, 3))
    nrm = rng.normal(0.0, 1.0, size=(n, 3))
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    tex = rng.standard_normal(size=(n, k, tex_width(m)), dtype=np.float32) * np.float32(0.1)
    return s, lam, rgb, nrm, tex


def _pack(p, s, lam, rgb, nrm, tex) -> Scene:
    f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return Scene(p=f32(p), power=f32(s * s), radius=f32(1.5 * s), normal=f32(nrm),
                 occ_logit=f32(lam), rgb=f32(rgb), tex=f32(tex))


def scene_uniform(n: int = 1024, seed: int = SEED_SCENE, k: int = K_DETAIL,
                  m: int = M_AXES) -> Scene:
    """Sites uniform in [-1,1]^3; s~U(0.02,0.1), w=s^2, r=1.5 s."""
    rng = np.random.default_rng(seed)
    p = rng.uniform(-1.0, 1.0, size=(n, 3))
    return _pack(p, *_attributes(rng, n, k, m))


def _random_rotation(rng: np.random.Generator) -> np.ndarray:
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                     [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                     [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def scene_mixture(n: int, seed: int = SEED_SCENE, k: int = K_DETAIL, m: int = M_AXES,
                  n_gauss: int = 64, frac_surface: float = 0.8) -> Scene:
    """80% of sites from ``n_gauss`` flattened Gaussians (thin-axis sigma
    U(0.01,0.05), in-plane sigma U(0.1,0.3), centres U[-1,1]^3, random
    rotation, equal mixture weights) and 20% uniform in volume over the
    spherical shell of radii 3..6."""
    rng = np.random.default_rng(seed)
    n_surf = int(round(frac_surface * n))
    n_bg = n - n_surf
    comp = rng.integers(0, n_gauss, size=n_surf)
    centres = rng.uniform(-1.0, 1.0, size=(n_gauss, 3))
    sig = np.stack([rng.uniform(0.1, 0.3, size=n_gauss), rng.uniform(0.1, 0.3, size=n_gauss),
                    rng.uniform(0.01, 0.05, size=n_gauss)], axis=1)
    rots = np.stack([_random_rotation(rng) for _ in range(n_gauss)])
    z = rng.normal(size=(n_surf, 3)) * sig[comp]
    p_surf = centres[comp] + np.einsum("nij,nj->ni", rots[comp], z)
    u = rng.normal(size=(n_bg, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    rad = np.cbrt(rng.uniform(3.0 ** 3, 6.0 ** 3, size=n_bg))
    p_bg = u * rad[:, None]
    p = np.concatenate([p_surf, p_bg], axis=0)
    return _pack(p, *_attributes(rng, n, k, m))


def look_at(eye: np.ndarray, target=(0.0, 0.0, 0.0), up=(0.0, 0.0, 1.0)) -> np.ndarray:
    """Camera-to-world [3,4] for OpenCV axes (x right, y down, z forward)."""
    eye = np.asarray(eye, dtype=np.float64)
    f = np.asarray(target, dtype=np.float64) - eye
    f /= np.linalg.norm(f)
    up = np.asarray(up, dtype=np.float64)
    if abs(np.dot(f, up)) > 0.999:
        up = np.array([0.0, 1.0, 0.0])
    right = np.cross(f, up)
    right /= np.linalg.norm(right)
    down = np.cross(f, right)
    c2w = np.zeros((3, 4))
    c2w[:, 0], c2w[:, 1], c2w[:, 2], c2w[:, 3] = right, down, f, eye
    return c2w.astype(np.float32)


def pinhole(eye, width: int, height: int, fov_deg: float = 60.0, target=(0.0, 0.0, 0.0)) -> Camera:
    """Vertical field of view ``fov_deg``; square pixels; principal point at
    the image centre."""
    fy = (height / 2.0) / math.tan(math.radians(fov_deg) / 2.0)
    return Camera(model=0, width=width, height=height, c2w=look_at(eye, target),
                  fx=fy, fy=fy, cx=width / 2.0, cy=height / 2.0)


def fisheye(eye, width: int, height: int, fov_deg: float = 180.0, target=(0.0, 0.0, 0.0)) -> Camera:
    """Equidistant fisheye whose image circle of angle ``fov_deg`` fits the
    shorter image side."""
    theta_max = math.radians(fov_deg) / 2.0
    f = (min(width, height) / 2.0) / theta_max
    return Camera(model=1, width=width, height=height, c2w=look_at(eye, target),
                  cx=width / 2.0, cy=height / 2.0, f_fish=f, theta_max=theta_max)


def unit_vectors(rng: np.random.Generator, n: int) -> np.ndarray:
    v = rng.normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def random_eyes(n: int, distance: float, seed: int = SEED_CAMERAS) -> np.ndarray:
    return unit_vectors(np.random.default_rng(seed), n) * distance


# ---------------------------------------------------------------------------
# The named workloads (sites, cameras), as plain inputs.

def c1_scene(seed: int = SEED_SCENE) -> Scene:
    return scene_uniform(1024, seed)


def c1_camera(seed: int = SEED_CAMERAS) -> Camera:
    return pinhole(random_eyes(1, 3.0, seed)[0], 128, 128, 60.0)


def c2_scene(seed: int = SEED_SCENE, n: int = 262144) -> Scene:
    return scene_mixture(n, seed)


def c2_cameras(seed: int = SEED_CAMERAS, width: int = 1280, height: int = 720):
    eye = random_eyes(1, 4.0, seed)[0]
    return pinhole(eye, width, height, 60.0), fisheye(eye, 1024, 1024, 180.0)


def c3_scene(seed: int = SEED_SCENE, n: int = 1048576) -> Scene:
    return scene_mixture(n, seed)


def c3_cameras(seed: int = SEED_CAMERAS, n_views: int = 8, width: int = 1600,
               height: int = 1066) -> List[Camera]:
    return [pinhole(e, width, height, 60.0) for e in random_eyes(n_views, 4.0, seed)]


def targets(cams: List[Camera], seed: int = SEED_TARGETS) -> List[np.ndarray]:
    """Seeded U(0,1) RGB noise target images, one [H,W,3] float32 per view."""
    rng = np.random.default_rng(seed)
    return [rng.uniform(0.0, 1.0, size=(c.height, c.width, 3)).astype(np.float32) for c in cams]


SERVE_RESOLUTIONS = [(256, 256), (512, 512), (1280, 720), (1920, 1080)]


@dataclasses.dataclass
class Request:
    arrival_s: float
    camera: Camera
    scene_id: int = 0


def request_stream(rate_hz: float, duration_s: float, seed: int = SEED_REQUESTS,
                   frac_fisheye: float = 0.3, distance: float = 4.0,
                   n_scenes: int = 1, max_requests: Optional[int] = None) -> List[Request]:
    """Poisson arrivals; resolution uniform over ``SERVE_RESOLUTIONS``;
    ``frac_fisheye`` of the cameras are 180-degree equidistant fisheyes, the
    rest 60-degree pinholes; random poses on a sphere of radius ``distance``."""
    rng = np.random.default_rng(seed)
    out, t = [], 0.0
    while True:
        t += rng.exponential(1.0 / rate_hz)
        if t > duration_s or (max_requests is not None and len(out) >= max_requests):
            break
        w, h = SERVE_RESOLUTIONS[int(rng.integers(0, len(SERVE_RESOLUTIONS)))]
        eye = unit_vectors(rng, 1)[0] * distance
        fish = rng.uniform() < frac_fisheye
        cam = fisheye(eye, w, h) if fish else pinhole(eye, w, h)
        out.append(Request(arrival_s=t, camera=cam, scene_id=int(rng.integers(0, n_scenes))))
    return out


def pixel_sample(cam: Camera, n: int, seed: int) -> np.ndarray:
    """``n`` distinct seeded pixel indices (row-major) of a camera's image."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(cam.n_rays, size=min(n, cam.n_rays), replace=False))


def steiner_draws(rounds: int, n_cand: int, seed: int = SEED_STEINER) -> np.ndarray:
    """Standard normal draws ``[rounds, n_cand, 3]`` (float32) for the
    Steiner-cell candidates of each round."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal(size=(rounds, n_cand, 3), dtype=np.float32)
