"""Seeded synthetic 3DGS-shaped scenes (input generator only).

This module draws the inputs that both the HIP path and the FP64 oracle
consume.  It holds none of the simplification method's arithmetic: it only
produces splats in the stored 3DGS parameterisation (centre, per-axis log
scale, raw quaternion, opacity logit, degree-3 SH), the same form a trained
3DGS PLY file carries.

Recipe (every draw comes from ``numpy.random.Generator(PCG64(seed))`` in the
order listed, computed in float64 and stored as float32):

1. surfaces: for each plane, centre ~ U[-8,8]^3, normal = normalise(N(0,I3)),
   half-extent h ~ U[2,8]; then for each sphere, centre ~ U[-8,8]^3,
   radius ~ U[1,4].
2. counts: n_clutter = round(clutter * n); the remaining points are split
   equally across the surfaces (the remainder goes to the first surface).
3. structured points: plane point = c + a*u + b*v with a, b ~ U[-h,h] and
   (u, v) an orthonormal basis of the plane; sphere point = c + r *
   normalise(N(0,I3)); every structured point gets N(0, jitter^2) per-axis
   jitter; the result is clipped to [-10,10]^3.
4. clutter points ~ U[-10,10]^3.
5. log-scales ~ N(-4, 0.5) per axis (stress mode: one uniformly chosen axis
   ~ N(-7, 0.5); a `needle` fraction of splats get two such axes).
6. raw quaternions ~ N(0, I4) (not normalised; uniform rotations once
   normalised), opacity logits ~ N(0, 1.5), SH DC ~ U(-1,1)^3, SH rest ~
   N(0, 0.05^2)^45.
7. a final random permutation, so the input order carries no locality.

The trained scenes the paper evaluates on (NeRF-Synthetic, Mip-NeRF 360,
Tanks&Temples, Deep Blending) are not available; these scenes stand in for
them with the same parameterisation: points concentrated on 2-D surfaces
with sparse clutter, small anisotropic Gaussians, broad opacities.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

SH_COEFFS = 48  # degree-3 spherical harmonics, 16 per colour channel


@dataclass
class Scene:
    """Stored-form splats, float32, row-major per splat."""

    pos: np.ndarray        # [n, 3] centres
    log_scale: np.ndarray  # [n, 3] per-axis log standard deviations
    rot: np.ndarray        # [n, 4] raw quaternion (w, x, y, z)
    opacity: np.ndarray    # [n]    opacity logit
    sh: np.ndarray         # [n, 48] f_dc_0..2 followed by f_rest_0..44

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])

    def subset(self, idx) -> "Scene":
        return Scene(self.pos[idx], self.log_scale[idx], self.rot[idx],
                     self.opacity[idx], self.sh[idx])

    def copy(self) -> "Scene":
        return Scene(self.pos.copy(), self.log_scale.copy(), self.rot.copy(),
                     self.opacity.copy(), self.sh.copy())


def _plane_basis(normal: np.ndarray):
    # helper axis: the coordinate axis least aligned with the normal
    e = np.zeros(3)
    e[int(np.argmin(np.abs(normal)))] = 1.0
    u = np.cross(normal, e)
    u /= np.linalg.norm(u)
    v = np.cross(normal, u)
    return u, v


def gen_scene(n: int, seed: int, n_planes: int = 8, n_spheres: int = 4,
              clutter: float = 0.10, jitter: float = 0.02,
              stress: bool = False, needle_frac: float = 0.05) -> Scene:
    """Draw one scene of ``n`` splats (see the module docstring)."""
    if n < 0:
        raise ValueError("n must be >= 0")
    rng = np.random.Generator(np.random.PCG64(seed))
    n_surf = n_planes + n_spheres
    planes = []
    for _ in range(n_planes):
        c = rng.uniform(-8.0, 8.0, 3)
        nrm = rng.normal(size=3)
        nrm /= np.linalg.norm(nrm)
        h = rng.uniform(2.0, 8.0)
        planes.append((c, nrm, h))
    spheres = []
    for _ in range(n_spheres):
        c = rng.uniform(-8.0, 8.0, 3)
        r = rng.uniform(1.0, 4.0)
        spheres.append((c, r))

    n_clutter = int(round(clutter * n)) if n_surf > 0 else n
    n_struct = n - n_clutter
    counts = [n_struct // n_surf] * n_surf if n_surf > 0 else []
    if n_surf > 0:
        counts[0] += n_struct - sum(counts)

    pts = []
    for s, cnt in enumerate(counts):
        if s < n_planes:
            c, nrm, h = planes[s]
            u, v = _plane_basis(nrm)
            ab = rng.uniform(-h, h, (cnt, 2))
            p = c + ab[:, :1] * u + ab[:, 1:] * v
        else:
            c, r = spheres[s - n_planes]
            d = rng.normal(size=(cnt, 3))
            d /= np.linalg.norm(d, axis=1, keepdims=True)
            p = c + r * d
        p = p + rng.normal(0.0, jitter, (cnt, 3))
        pts.append(np.clip(p, -10.0, 10.0))
    pts.append(rng.uniform(-10.0, 10.0, (n_clutter, 3)))
    pos = np.concatenate(pts, axis=0) if pts else np.zeros((0, 3))

    log_scale = rng.normal(-4.0, 0.5, (n, 3))
    if stress:
        flat_axis = rng.integers(0, 3, n)
        log_scale[np.arange(n), flat_axis] = rng.normal(-7.0, 0.5, n)
        needle = rng.random(n) < needle_frac
        second = (flat_axis + rng.integers(1, 3, n)) % 3
        idx = np.nonzero(needle)[0]
        log_scale[idx, second[idx]] = rng.normal(-7.0, 0.5, idx.size)
    rot = rng.normal(size=(n, 4))
    opacity = rng.normal(0.0, 1.5, n)
    sh = np.empty((n, SH_COEFFS))
    sh[:, :3] = rng.uniform(-1.0, 1.0, (n, 3))
    sh[:, 3:] = rng.normal(0.0, 0.05, (n, SH_COEFFS - 3))

    perm = rng.permutation(n)
    f32 = np.float32
    return Scene(pos[perm].astype(f32), log_scale[perm].astype(f32),
                 rot[perm].astype(f32), opacity[perm].astype(f32),
                 sh[perm].astype(f32))


def gen_scene_device(n: int, seed: int, out=None, stream=None):
    """One scene of ``n`` splats drawn on the GPU with the recipe above, for
    workloads with too many distinct scenes to draw on the host (a serving
    trace of thousands of requests).  The surfaces (2..8 planes, 0..4
    spheres, their centres, normals, extents and radii) come from
    ``numpy.random.Generator(PCG64(seed))``; the per-splat draws come from a
    CUDA ``torch.Generator`` seeded with ``seed`` and are made in float32, so
    the scene is not the one gen_scene would draw for that seed.  ``out``:
    optional stored-form tensors (pos, log_scale, rot, opacity, sh) of
    capacity n to fill; returns those tensors."""
    import torch
    rng = np.random.Generator(np.random.PCG64(seed))
    n_planes = int(rng.integers(2, 9))
    n_spheres = int(rng.integers(0, 5))
    surf = []
    for _ in range(n_planes):
        c = rng.uniform(-8.0, 8.0, 3)
        nrm = rng.normal(size=3)
        nrm /= np.linalg.norm(nrm)
        surf.append(("plane", c, _plane_basis(nrm), rng.uniform(2.0, 8.0)))
    for _ in range(n_spheres):
        surf.append(("sphere", rng.uniform(-8.0, 8.0, 3), None, rng.uniform(1.0, 4.0)))
    dev = torch.device("cuda")
    g = torch.Generator(device=dev)
    g.manual_seed(int(seed))
    if out is None:
        out = (torch.empty((n, 3), device=dev), torch.empty((n, 3), device=dev),
               torch.empty((n, 4), device=dev), torch.empty(n, device=dev),
               torch.empty((n, SH_COEFFS), device=dev))
    pos_o, ls_o, rot_o, op_o, sh_o = out
    ctx = torch.cuda.stream(stream) if stream is not None else torch.cuda.stream(
        torch.cuda.current_stream())
    with ctx:
        n_clutter = int(round(0.10 * n))
        n_struct = n - n_clutter
        counts = [n_struct // len(surf)] * len(surf)
        counts[0] += n_struct - sum(counts)
        pos = torch.empty((n, 3), device=dev)
        at = 0
        f32 = torch.float32
        for (kind, c, basis, ext), cnt in zip(surf, counts):
            ct = torch.tensor(c, dtype=f32, device=dev)
            if kind == "plane":
                u = torch.tensor(basis[0], dtype=f32, device=dev)
                v = torch.tensor(basis[1], dtype=f32, device=dev)
                ab = (torch.rand((cnt, 2), generator=g, device=dev) * 2.0 - 1.0) * float(ext)
                p = ct + ab[:, :1] * u + ab[:, 1:] * v
            else:
                d = torch.randn((cnt, 3), generator=g, device=dev)
                p = ct + float(ext) * (d / d.norm(dim=1, keepdim=True))
            p = p + 0.02 * torch.randn((cnt, 3), generator=g, device=dev)
            pos[at:at + cnt] = p.clamp_(-10.0, 10.0)
            at += cnt
        pos[at:] = torch.rand((n_clutter, 3), generator=g, device=dev) * 20.0 - 10.0
        perm = torch.randperm(n, generator=g, device=dev)
        pos_o.copy_(pos[perm])
        ls_o.copy_(torch.randn((n, 3), generator=g, device=dev) * 0.5 - 4.0)
        rot_o.copy_(torch.randn((n, 4), generator=g, device=dev))
        op_o.copy_(torch.randn(n, generator=g, device=dev) * 1.5)
        sh_o[:, :3] = torch.rand((n, 3), generator=g, device=dev) * 2.0 - 1.0
        sh_o[:, 3:] = torch.randn((n, SH_COEFFS - 3), generator=g, device=dev) * 0.05
    return out


# --- named workloads -------------------------------------------------------

def scene_cpu_scale():
    """20,000 splats, seed 1, 8 planes + 4 spheres, k=16, target 50%."""
    return gen_scene(20_000, 1), 16, 10_000


def scene_plain_gpu(n: int = 1_000_000):
    """1,000,000 splats, seed 2, same generator, k=16, target 10%."""
    return gen_scene(n, 2), 16, max(int(math.ceil(0.1 * n)), 1)


def scene_precision_stress(n: int = 6_000_000):
    """6,000,000 splats, seed 3, 64 planes, flat + 5% needle scales, k=24,
    target 1%."""
    return (gen_scene(n, 3, n_planes=64, n_spheres=0, stress=True), 24,
            max(int(math.ceil(0.01 * n)), 1))


def batch_specs(n_scenes: int = 64, seed: int = 4, lo: float = 5e4,
                hi: float = 2e6):
    """Per-scene (n, seed, planes, spheres, target_ratio) for the batched
    workload: n log-uniform in [lo, hi], surfaces U{4..64} (two thirds
    planes), target ratio from {0.5, 0.2, 0.1}."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(n_scenes):
        n = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        surf = int(rng.integers(4, 65))
        planes = int(math.ceil(2 * surf / 3))
        ratio = float(rng.choice([0.5, 0.2, 0.1]))
        out.append((n, 1000 + i, planes, surf - planes, ratio))
    return out


def serving_trace(rate: float = 20.0, duration: float = 120.0, seed: int = 5,
                  lo: float = 1e4, hi: float = 4e6):
    """Poisson arrivals: list of (t_arrival, n, scene_seed, ratio, k)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t, out, jid = 0.0, [], 0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        n = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        ratio = float(rng.choice([0.5, 0.1, 0.01]))
        k = int(rng.choice([16, 24]))
        out.append((t, n, 20000 + jid, ratio, k))
        jid += 1
    return out
