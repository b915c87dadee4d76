"""Seeded synthetic scenes, cameras, rays, grids and weights.

Draw order is fixed and documented per function so that any consumer with
the same seed sees bit-identical float32 inputs.  Nothing here renders,
samples, interpolates or differentiates: those are the method under test.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

BOX_MIN = np.array([-1.0, -1.0, -1.0], dtype=np.float32)
BOX_MAX = np.array([1.0, 1.0, 1.0], dtype=np.float32)


# --------------------------------------------------------------------------
# cameras and rays
# --------------------------------------------------------------------------
def look_at_c2w(center, target=(0.0, 0.0, 0.0), up=(0.0, 0.0, 1.0)) -> np.ndarray:
    """3x3 camera-to-world rotation (columns right, up, back) for a pinhole
    camera at ``center`` looking at ``target``; the camera looks down its -z.
    When the view direction is (anti)parallel to ``up`` the y axis is used."""
    c = np.asarray(center, dtype=np.float64)
    fwd = np.asarray(target, dtype=np.float64) - c
    fwd /= np.linalg.norm(fwd)
    upv = np.asarray(up, dtype=np.float64)
    if abs(float(np.dot(fwd, upv))) > 0.999:
        upv = np.array([0.0, 1.0, 0.0])
    right = np.cross(fwd, upv)
    right /= np.linalg.norm(right)
    true_up = np.cross(right, fwd)
    return np.stack([right, true_up, -fwd], axis=1)


def pixel_rays(c2w: np.ndarray, center, H: int, W: int, focal: float, pi, pj):
    """Rays through pixel centres (row ``pi``, column ``pj``) of an H x W
    pinhole image with focal length ``focal`` pixels.  Returns float32
    origins [n,3] and unit directions [n,3] (normalised in float64)."""
    pi = np.asarray(pi, dtype=np.float64)
    pj = np.asarray(pj, dtype=np.float64)
    dc = np.stack([(pj + 0.5 - W * 0.5) / focal,
                   -(pi + 0.5 - H * 0.5) / focal,
                   -np.ones_like(pi)], axis=-1)
    d = dc @ np.asarray(c2w, dtype=np.float64).T
    d /= np.linalg.norm(d, axis=-1, keepdims=True)
    o = np.broadcast_to(np.asarray(center, dtype=np.float64), d.shape)
    return np.ascontiguousarray(o, dtype=np.float32), np.ascontiguousarray(d, dtype=np.float32)


def cube_vertex_cameras(radius: float = 4.0) -> np.ndarray:
    """Eight camera centres at the cube vertices (+-1,+-1,+-1) * radius/sqrt(3)."""
    s = radius / math.sqrt(3.0)
    out = []
    for sx in (-1.0, 1.0):
        for sy in (-1.0, 1.0):
            for sz in (-1.0, 1.0):
                out.append((sx * s, sy * s, sz * s))
    return np.array(out, dtype=np.float64)


def hemisphere_cameras(n: int, seed: int, radius: float = 4.0) -> np.ndarray:
    """``n`` camera centres uniform on the upper hemisphere (z >= 0) of the
    given radius.  Draws: z ~ U[0,1) then phi ~ U[0, 2pi), each as one
    vector of length n from ``default_rng(seed)``."""
    rng = np.random.default_rng(seed)
    z = rng.random(n)
    phi = rng.random(n) * 2.0 * math.pi
    rxy = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    return radius * np.stack([rxy * np.cos(phi), rxy * np.sin(phi), z], axis=-1)


def _rays_for_flat_pixels(centers, H, W, focal, flat):
    flat = np.asarray(flat, dtype=np.int64)
    cam = flat // (H * W)
    rem = flat % (H * W)
    pi, pj = rem // W, rem % W
    o = np.empty((flat.size, 3), np.float32)
    d = np.empty((flat.size, 3), np.float32)
    for c in np.unique(cam):
        sel = cam == c
        R = look_at_c2w(centers[c])
        o[sel], d[sel] = pixel_rays(R, centers[c], H, W, focal, pi[sel], pj[sel])
    return o, d, cam, pi, pj


def draw_pixels_without_replacement(rng, centers, H, W, focal, n):
    """``n`` distinct pixels over all cameras (one ``rng.choice`` draw)."""
    flat = rng.choice(len(centers) * H * W, size=n, replace=False)
    return _rays_for_flat_pixels(centers, H, W, focal, flat)


def draw_pixels_with_replacement(rng, centers, H, W, focal, n):
    """``n`` pixels drawn uniformly with replacement (one ``rng.integers``)."""
    flat = rng.integers(0, len(centers) * H * W, size=n)
    return _rays_for_flat_pixels(centers, H, W, focal, flat)


def image_rays(center, H, W, focal):
    """All H*W rays of one camera, row-major."""
    R = look_at_c2w(center)
    ii, jj = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    return pixel_rays(R, center, H, W, focal, ii.ravel(), jj.ravel())


# --------------------------------------------------------------------------
# the synthetic sphere scene
# --------------------------------------------------------------------------
@dataclass
class Spheres:
    center: np.ndarray   # [n,3] float64
    radius: np.ndarray   # [n]
    rho: np.ndarray      # [n] peak density
    rgb: np.ndarray      # [n,3]
    edge: float = 0.01   # soft-edge width

    def as_f32_table(self) -> np.ndarray:
        """[n, 8] float32 rows (cx, cy, cz, r, rho, R, G, B)."""
        return np.concatenate([self.center, self.radius[:, None], self.rho[:, None],
                               self.rgb], axis=1).astype(np.float32)


def random_spheres(seed: int, n: int = 64) -> Spheres:
    """Draws (one vector each, in this order): centres U[-0.7,0.7]^3,
    radii U[0.1,0.25], peak density in (0,50], RGB U[0,1]^3."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(-0.7, 0.7, size=(n, 3))
    r = rng.uniform(0.1, 0.25, size=n)
    rho = 50.0 * (1.0 - rng.random(n))
    rgb = rng.random((n, 3))
    return Spheres(c, r, rho, rgb)


def sphere_field(x: np.ndarray, sp: Spheres):
    """Scene definition: density sum_i rho_i * sigmoid((r_i - |x-c_i|)/edge)
    and density-weighted mean colour (0 where the density is 0).  float64."""
    x = np.asarray(x, dtype=np.float64)
    dist = np.linalg.norm(x[:, None, :] - sp.center[None, :, :], axis=-1)
    z = (sp.radius[None, :] - dist) / sp.edge
    sig_i = sp.rho[None, :] * (0.5 * (1.0 + np.tanh(0.5 * z)))
    sig = sig_i.sum(axis=1)
    col = sig_i @ sp.rgb
    with np.errstate(invalid="ignore", divide="ignore"):
        col = np.where(sig[:, None] > 0, col / np.maximum(sig[:, None], 1e-300), 0.0)
    return sig, col


def coarse_raw_from_spheres(sp: Spheres, n: int = 100, box_min=BOX_MIN, box_max=BOX_MAX,
                            floor: float = 1e-12, chunk: int = 1 << 16) -> np.ndarray:
    """Raw coarse density on an n^3 vertex grid spanning the box, chosen so
    that a unit softplus of it reproduces the scene density at each vertex:
    raw = log(expm1(max(sigma, floor))), evaluated stably.  float32 [n,n,n]."""
    ax = [np.linspace(float(box_min[i]), float(box_max[i]), n) for i in range(3)]
    X, Y, Z = np.meshgrid(*ax, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=-1)
    sig = np.empty(pts.shape[0])
    for s in range(0, pts.shape[0], chunk):
        sig[s:s + chunk] = sphere_field(pts[s:s + chunk], sp)[0]
    sig = np.maximum(sig, floor)
    raw = sig + np.log(-np.expm1(-sig))
    return raw.reshape(n, n, n).astype(np.float32)


# --------------------------------------------------------------------------
# network weights
# --------------------------------------------------------------------------
def xavier_uniform_mlp(rng, dims=(39, 128, 128, 3)):
    """Weights [out][in] ~ U(-a, a), a = sqrt(6/(fan_in+fan_out)), zero
    biases; one draw per layer in order.  float32."""
    Ws, bs = [], []
    for fi, fo in zip(dims[:-1], dims[1:]):
        a = math.sqrt(6.0 / (fi + fo))
        Ws.append(rng.uniform(-a, a, size=(fo, fi)).astype(np.float32))
        bs.append(np.zeros(fo, np.float32))
    return Ws, bs


# --------------------------------------------------------------------------
# workload configurations
# --------------------------------------------------------------------------
@dataclass
class RayBatch:
    o: np.ndarray
    d: np.ndarray
    target: np.ndarray
    jitter: np.ndarray | None


@dataclass
class Problem:
    """One training-step problem: grids, network, rays and hyperparameters."""
    box_min: np.ndarray
    box_max: np.ndarray
    density: np.ndarray            # [n,n,n] float32
    feat: np.ndarray               # [n,n,n,C] float32
    Ws: list
    bs: list
    step: float                    # sample spacing (world units, unit d)
    max_samples: int
    act_shift: float               # softplus shift b
    bg: np.ndarray                 # background colour
    rays: RayBatch
    coarse_raw: np.ndarray | None = None
    coarse_min: np.ndarray | None = None
    coarse_max: np.ndarray | None = None
    extra: dict = field(default_factory=dict)


def tiny_config(seed: int = 0, jitter: bool = False, n_rays: int = 4096, n: int = 32,
                channels: int = 12) -> Problem:
    """The small plain configuration: 32^3 density and 12-channel feature
    grids U(-1,1), 39-128-128-3 Xavier network, 4096 rays without replacement
    from 8 cameras (64x64, focal 80) at the cube vertices of radius 4,
    step half a voxel, cap 128, white background, targets U(0,1).

    Draw order from default_rng(seed): density, features, network weights,
    pixel choice, targets, jitter (only when requested)."""
    rng = np.random.default_rng(seed)
    dens = rng.uniform(-1, 1, size=(n, n, n)).astype(np.float32)
    feat = rng.uniform(-1, 1, size=(n, n, n, channels)).astype(np.float32)
    Ws, bs = xavier_uniform_mlp(rng, (channels + 27, 128, 128, 3))
    cams = cube_vertex_cameras(4.0)
    o, d, *_ = draw_pixels_without_replacement(rng, cams, 64, 64, 80.0, n_rays)
    tgt = rng.random((n_rays, 3)).astype(np.float32)
    jit = rng.random(n_rays).astype(np.float32) if jitter else None
    step = 0.5 * 2.0 / (n - 1)
    return Problem(BOX_MIN.copy(), BOX_MAX.copy(), dens, feat, Ws, bs, step, 128, 0.0,
                   np.ones(3, np.float32), RayBatch(o, d, tgt, jit))


FULL_N = 160
FULL_COARSE_N = 100
FULL_ALPHA_INIT = 1e-2
FULL_TAU = 1e-4


def full_scene(seed: int = 0, coarse_n: int = FULL_COARSE_N):
    """Sphere scene (seed), 100 training cameras (seed 1), 10 held-out
    cameras (seed 2) and the rasterised coarse raw density grid."""
    sp = random_spheres(seed)
    cams = hemisphere_cameras(100, 1)
    held = hemisphere_cameras(10, 2)
    raw = coarse_raw_from_spheres(sp, coarse_n)
    return sp, cams, held, raw


def full_config(seed: int = 0, n_rays: int = 8192, n: int = FULL_N, batch_seed: int = 1000,
                scene=None, channels: int = 12, max_samples: int | None = None) -> Problem:
    """The full plain configuration on the sphere scene: 160^3 grids
    initialised to zero (density and features), Xavier network drawn from
    default_rng(seed + 7), step half a fine voxel, one batch of ``n_rays``
    pixels drawn with replacement from default_rng(batch_seed) over the 100
    cameras (800x800, focal 1000), jitter drawn next from the same generator.
    Targets are left as zeros here: they come from rendering the scene."""
    sp, cams, held, raw = scene if scene is not None else full_scene(seed)
    rng_w = np.random.default_rng(seed + 7)
    Ws, bs = xavier_uniform_mlp(rng_w, (channels + 27, 128, 128, 3))
    dens = np.zeros((n, n, n), np.float32)
    feat = np.zeros((n, n, n, channels), np.float32)
    rng = np.random.default_rng(batch_seed)
    o, d, *_ = draw_pixels_with_replacement(rng, cams, 800, 800, 1000.0, n_rays)
    jit = rng.random(n_rays).astype(np.float32)
    step = 0.5 * 2.0 / (n - 1)
    if max_samples is None:
        # longest in-box chord is the diagonal 2*sqrt(3)
        max_samples = int(math.ceil(2.0 * math.sqrt(3.0) / step)) + 1
    prob = Problem(BOX_MIN.copy(), BOX_MAX.copy(), dens, feat, Ws, bs, step, max_samples,
                   0.0, np.ones(3, np.float32),
                   RayBatch(o, d, np.zeros((n_rays, 3), np.float32), jit),
                   coarse_raw=raw, coarse_min=BOX_MIN.copy(), coarse_max=BOX_MAX.copy())
    prob.extra.update(spheres=sp, cams=cams, held=held, alpha_init=FULL_ALPHA_INIT,
                      voxel=2.0 / (n - 1), tau=FULL_TAU)
    return prob


STRESS_N = 256
STRESS_MAX_SAMPLES = 800
STRESS_ALPHA_INIT = 1e-2


def stress_config(seed: int = 0, n_rays: int = 32768, n: int = STRESS_N, batch_seed: int = 2000,
                  max_samples: int = STRESS_MAX_SAMPLES) -> Problem:
    """Differentiation stress shapes: 256^3 density and 12-channel feature
    grids with values uniform in [-1, 1] from default_rng(seed) (density
    first), Xavier network with N(0, 0.1) biases from default_rng(seed + 7),
    step half a voxel, at most 800 samples per ray (the diagonal would need
    884), and ``n_rays`` pixels drawn with replacement over the 100 training
    cameras of the sphere scene from default_rng(batch_seed), jitter next.
    No coarse mask: every in-box sample is evaluated."""
    rng = np.random.default_rng(seed)
    dens = rng.uniform(-1.0, 1.0, (n, n, n)).astype(np.float32)
    feat = rng.uniform(-1.0, 1.0, (n, n, n, 12)).astype(np.float32)
    rng_w = np.random.default_rng(seed + 7)
    Ws, bs = xavier_uniform_mlp(rng_w, (39, 128, 128, 3))
    bs = [(rng_w.normal(size=b.shape) * 0.1).astype(np.float32) for b in bs]
    cams = hemisphere_cameras(100, 1)
    rng = np.random.default_rng(batch_seed)
    o, d, *_ = draw_pixels_with_replacement(rng, cams, 800, 800, 1000.0, n_rays)
    jit = rng.random(n_rays).astype(np.float32)
    step = 0.5 * 2.0 / (n - 1)
    prob = Problem(BOX_MIN.copy(), BOX_MAX.copy(), dens, feat, Ws, bs, step, max_samples, 0.0,
                   np.ones(3, np.float32), RayBatch(o, d, np.zeros((n_rays, 3), np.float32), jit))
    prob.extra.update(alpha_init=STRESS_ALPHA_INIT, voxel=2.0 / (n - 1))
    return prob


# --------------------------------------------------------------------------
# binary image of the image-fitting toy
# --------------------------------------------------------------------------
def binary_image(seed: int = 0, H: int = 256, W: int = 256, n_discs: int = 12, n_tris: int = 6) -> np.ndarray:
    """A seeded binary image [H, W] float32 (1 inside any shape, else 0):
    ``n_discs`` discs (centre U[0,1)^2 then radius U[0.03, 0.15), drawn disc
    by disc) and ``n_tris`` triangles (three vertices U[0,1)^2 each), in
    normalised image coordinates, tested at the pixel centres."""
    rng = np.random.default_rng(seed)
    y = (np.arange(H) + 0.5)[:, None] / H
    x = (np.arange(W) + 0.5)[None, :] / W
    img = np.zeros((H, W), bool)
    for _ in range(n_discs):
        cy, cx = rng.random(2)
        r = rng.uniform(0.03, 0.15)
        img |= (y - cy) ** 2 + (x - cx) ** 2 < r * r
    for _ in range(n_tris):
        p = rng.random((3, 2))
        side = []
        for k in range(3):
            (ay, ax), (by, bx) = p[k], p[(k + 1) % 3]
            side.append((bx - ax) * (y - ay) - (by - ay) * (x - ax) >= 0)
        img |= (side[0] & side[1] & side[2]) | (~side[0] & ~side[1] & ~side[2])
    return img.astype(np.float32)
