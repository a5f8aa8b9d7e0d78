"""Seeded synthetic polygon meshes (inputs of the mesh-to-DRK conversion).  Vertices are (nv, 3)
float64, faces (nf, m) int32 vertex indices listed counter-clockwise seen from outside, -1 padding.
No rasterizer arithmetic lives here."""
from __future__ import annotations

import math

import numpy as np


def mesh_icosphere(level: int):
    """Icosahedron subdivided `level` times (each triangle into four), vertices on the unit sphere:
    20 * 4^level triangles."""
    t = (1.0 + math.sqrt(5.0)) / 2.0
    V = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0), (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
         (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    V = [np.array(v, float) / np.linalg.norm(v) for v in V]
    F = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6),
         (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9), (4, 9, 5), (2, 4, 11), (6, 2, 10),
         (8, 6, 7), (9, 8, 1)]
    for _ in range(level):
        cache = {}
        nf = []

        def mid(a, b):
            key = (min(a, b), max(a, b))
            if key not in cache:
                m = V[a] + V[b]
                V.append(m / np.linalg.norm(m))
                cache[key] = len(V) - 1
            return cache[key]
        for a, b, c in F:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        F = nf
    return np.array(V), np.array(F, np.int32)


def mesh_torus(n_major: int, n_minor: int, R: float = 1.0, r: float = 0.35):
    """Torus around the z axis as an n_major x n_minor grid of quads (each nearly planar)."""
    u = 2 * math.pi * np.arange(n_major) / n_major
    v = 2 * math.pi * np.arange(n_minor) / n_minor
    uu, vv = np.meshgrid(u, v, indexing="ij")
    V = np.stack([(R + r * np.cos(vv)) * np.cos(uu), (R + r * np.cos(vv)) * np.sin(uu), r * np.sin(vv)], -1)
    V = V.reshape(-1, 3)
    i, j = np.meshgrid(np.arange(n_major), np.arange(n_minor), indexing="ij")
    a = i * n_minor + j
    b = ((i + 1) % n_major) * n_minor + j
    c = ((i + 1) % n_major) * n_minor + (j + 1) % n_minor
    d = i * n_minor + (j + 1) % n_minor
    F = np.stack([a, b, c, d], -1).reshape(-1, 4).astype(np.int32)
    return V, F


def mesh_scene(seed: int, n_instances: int = 24, ico_level: int = 3, torus=(48, 24), half: float = 3.0):
    """Randomly placed, rotated and scaled icospheres and tori in a box (faces padded to 4 vertices
    with -1).  Returns vertices (nv, 3), faces (nf, 4) int32, per-face RGB (nf, 3) float32."""
    rng = np.random.default_rng(seed)
    Vi, Fi = mesh_icosphere(ico_level)
    Fi = np.concatenate([Fi, -np.ones((Fi.shape[0], 1), np.int32)], 1)
    Vt, Ft = mesh_torus(*torus)
    Vs, Fs, Cs = [], [], []
    off = 0
    for k in range(n_instances):
        V, F = (Vi, Fi) if k % 2 == 0 else (Vt, Ft)
        g, r = np.linalg.qr(rng.standard_normal((3, 3)))
        Rm = g * np.sign(np.diag(r))[None, :]
        if np.linalg.det(Rm) < 0:
            Rm[:, 0] = -Rm[:, 0]          # a proper rotation keeps the faces' winding
        V = (V * rng.uniform(0.3, 0.9)) @ Rm.T + rng.uniform(-half, half, 3)
        Vs.append(V)
        Fs.append(np.where(F >= 0, F + off, -1).astype(np.int32))
        Cs.append(np.tile(rng.uniform(0.1, 1.0, 3), (F.shape[0], 1)) * rng.uniform(0.8, 1.0, (F.shape[0], 1)))
        off += V.shape[0]
    return np.concatenate(Vs), np.concatenate(Fs), np.concatenate(Cs).astype(np.float32)
