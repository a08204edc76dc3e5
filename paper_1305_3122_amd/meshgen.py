"""Seeded synthetic 2D triangle meshes (inputs only).

This module builds the vertex array ``q`` and the connectivity array ``me``
of the problem statement (Notations section): ``q`` is stored as an
``[nq][2]`` float64 array (the paper's 2 x nq column-major array, so memory
order x0,y0,x1,y1,...) and ``me`` as an ``[nme][3]`` int32 array of 0-based
vertex indices (the paper's 3 x nme array, 1-based).

It holds no finite element arithmetic: no areas, element matrices or
assembly.  Both the HIP path and the CPU oracle take their inputs from here,
and random numbers that the method would otherwise draw (weights, adjoint
seeds) are produced here and passed in.

Meshes
------
* ``unit_square(n, ...)``: [0,1]^2 split into n x n cells, each cut along the
  v00-v11 diagonal into two counter-clockwise triangles; interior vertices
  jittered by U(-j h, j h) per coordinate (boundary fixed, so the domain stays
  the unit square); then a uniform random relabelling of the vertices.
* ``unit_disk(K, ...)``: centre plus rings k = 1..K of radius k/K holding 6k
  vertices at angles 2 pi j / (6k); each annulus is triangulated by a
  counter-clockwise merge on angle (ties advance the inner ring); then a random
  relabelling.  nme = 6 K^2, nq = 1 + 3 K (K + 1).
* ``batch_of_squares(...)``: many independent unit-square meshes with uneven
  sizes, concatenated with vertex offsets (block-diagonal global matrix).
* ``unit_cube(n, ...)``: [0,1]^3 split into n^3 cells, each cut into the six
  tetrahedra around its v000-v111 diagonal (Kuhn; conforming across cells),
  all positively oriented before the jitter; interior vertices jittered by
  U(-j h, j h) per coordinate; then a random relabelling.  q is [nq][3] and
  me is [nme][4].

The paper measures on FreeFEM++ unit-disk meshes that are not available; these
seeded meshes stand in for them.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

#: base seed of every configuration (arXiv id 1305.3122)
BASE_SEED = 1305_3122


@dataclasses.dataclass
class Mesh:
    q: np.ndarray          # [nq][2] float64
    me: np.ndarray         # [nme][3] int32, 0-based
    name: str = ""

    @property
    def nq(self) -> int:
        return int(self.q.shape[0])

    @property
    def nme(self) -> int:
        return int(self.me.shape[0])


@dataclasses.dataclass
class Batch:
    q: np.ndarray          # [sum nq][2] float64 (concatenated)
    me: np.ndarray         # [sum nme][3] int32, GLOBAL vertex indices
    me_local: np.ndarray   # [sum nme][3] int32, indices local to each mesh
    vtx_off: np.ndarray    # [nb+1] int64
    elem_off: np.ndarray   # [nb+1] int64
    sizes: np.ndarray      # [nb] cells per side

    @property
    def nb(self) -> int:
        return int(self.sizes.shape[0])

    def mesh(self, b: int) -> Mesh:
        v0, v1 = int(self.vtx_off[b]), int(self.vtx_off[b + 1])
        e0, e1 = int(self.elem_off[b]), int(self.elem_off[b + 1])
        return Mesh(self.q[v0:v1].copy(), self.me_local[e0:e1].copy(), f"batch[{b}]")


def _relabel(rng: np.random.Generator, q: np.ndarray, me: np.ndarray):
    """Uniform random vertex relabelling pi: q'[pi(i)] = q[i], me' = pi(me)."""
    nq = q.shape[0]
    pi = rng.permutation(nq).astype(np.int64)
    q2 = np.empty_like(q)
    q2[pi] = q
    me2 = pi[me].astype(np.int32)
    return q2, me2


def unit_square(n: int, jitter: float = 0.2, seed: int | None = BASE_SEED,
                permute: bool = True) -> Mesh:
    """Unit square, n x n cells, 2 n^2 counter-clockwise triangles."""
    if n < 1:
        raise ValueError("n must be >= 1")
    rng = np.random.Generator(np.random.PCG64(seed))
    h = 1.0 / n
    ii, jj = np.meshgrid(np.arange(n + 1), np.arange(n + 1), indexing="xy")
    # vertex (i h, j h) has index j (n+1) + i  (row-major before relabelling)
    q = np.stack([ii.ravel() * h, jj.ravel() * h], axis=1).astype(np.float64)
    if jitter:
        d = rng.uniform(-jitter * h, jitter * h, size=q.shape)
        interior = ((ii.ravel() > 0) & (ii.ravel() < n) &
                    (jj.ravel() > 0) & (jj.ravel() < n))
        q[interior] += d[interior]
    ci, cj = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")
    ci = ci.ravel()
    cj = cj.ravel()
    v00 = cj * (n + 1) + ci
    v10 = v00 + 1
    v01 = v00 + (n + 1)
    v11 = v01 + 1
    me = np.empty((2 * n * n, 3), dtype=np.int64)
    me[0::2] = np.stack([v00, v10, v11], axis=1)
    me[1::2] = np.stack([v00, v11, v01], axis=1)
    if permute:
        q, me = _relabel(rng, q, me)
    return Mesh(np.ascontiguousarray(q), np.ascontiguousarray(me.astype(np.int32)),
                f"square{n}")


def unit_disk(K: int, seed: int | None = BASE_SEED, permute: bool = True) -> Mesh:
    """Unit disk from K concentric rings (polygon with 6K boundary vertices)."""
    if K < 1:
        raise ValueError("K must be >= 1")
    rng = np.random.Generator(np.random.PCG64(seed))
    nq = 1 + 3 * K * (K + 1)
    q = np.zeros((nq, 2), dtype=np.float64)
    tris = []
    for k in range(1, K + 1):
        n_out = 6 * k
        s_out = 1 + 3 * k * (k - 1)
        j = np.arange(n_out)
        ang = 2.0 * np.pi * j / n_out
        q[s_out:s_out + n_out, 0] = (k / K) * np.cos(ang)
        q[s_out:s_out + n_out, 1] = (k / K) * np.sin(ang)
        if k == 1:
            jn = (j + 1) % n_out
            tris.append(np.stack([np.zeros(n_out, np.int64), s_out + j, s_out + jn], 1))
            continue
        m_in = 6 * (k - 1)
        s_in = 1 + 3 * (k - 1) * (k - 2)
        # merge on angle: the inner ring advances at times (a+1)/m_in, the outer
        # ring at (b+1)/n_out (common denominator m_in n_out); ties: inner first
        t_in = (np.arange(m_in) + 1) * n_out * 2
        t_out = (np.arange(n_out) + 1) * m_in * 2 + 1
        is_inner = np.concatenate([np.ones(m_in, bool), np.zeros(n_out, bool)])
        order = np.argsort(np.concatenate([t_in, t_out]), kind="stable")
        ev_inner = is_inner[order]
        a = np.cumsum(ev_inner) - ev_inner          # inner events before this one
        b = np.cumsum(~ev_inner) - (~ev_inner)      # outer events before this one
        third = np.where(ev_inner, s_in + (a + 1) % m_in, s_out + (b + 1) % n_out)
        out = np.stack([s_in + a % m_in, s_out + b % n_out, third], axis=1)
        tris.append(out)
    me = np.concatenate(tris, axis=0)
    if permute:
        q, me = _relabel(rng, q, me)
    return Mesh(np.ascontiguousarray(q), np.ascontiguousarray(me.astype(np.int32)),
                f"disk{K}")


def batch_of_squares(nb: int = 512, n_min: int = 8, n_max: int = 512,
                     jitter: float = 0.2, seed: int | None = BASE_SEED) -> Batch:
    """nb unit-square meshes, cells per side log-uniform in [n_min, n_max]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = np.rint(np.exp(rng.uniform(math.log(n_min), math.log(n_max), size=nb))).astype(np.int64)
    sub_seeds = rng.integers(0, 2**62, size=nb)
    qs, mes = [], []
    vtx_off = np.zeros(nb + 1, np.int64)
    elem_off = np.zeros(nb + 1, np.int64)
    for b in range(nb):
        m = unit_square(int(sizes[b]), jitter=jitter, seed=int(sub_seeds[b]))
        qs.append(m.q)
        mes.append(m.me)
        vtx_off[b + 1] = vtx_off[b] + m.nq
        elem_off[b + 1] = elem_off[b] + m.nme
    me_local = np.concatenate(mes, axis=0).astype(np.int32)
    shift = np.repeat(vtx_off[:-1], np.diff(elem_off))
    me_glob = (me_local.astype(np.int64) + shift[:, None]).astype(np.int32)
    return Batch(np.ascontiguousarray(np.concatenate(qs, axis=0)), np.ascontiguousarray(me_glob),
                 np.ascontiguousarray(me_local), vtx_off, elem_off, sizes)


def unit_cube(n: int, jitter: float = 0.1, seed: int | None = BASE_SEED,
              permute: bool = True) -> Mesh:
    """Unit cube, n^3 cells, 6 n^3 tetrahedra (q [nq][3], me [nme][4])."""
    if n < 1:
        raise ValueError("n must be >= 1")
    rng = np.random.Generator(np.random.PCG64(seed))
    h = 1.0 / n
    m = n + 1
    kk, jj, ii = np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")
    # vertex (i h, j h, k h) has index (k m + j) m + i before relabelling
    q = np.stack([ii.ravel() * h, jj.ravel() * h, kk.ravel() * h], axis=1).astype(np.float64)
    if jitter:
        d = rng.uniform(-jitter * h, jitter * h, size=q.shape)
        interior = ((ii.ravel() > 0) & (ii.ravel() < n) & (jj.ravel() > 0) & (jj.ravel() < n) &
                    (kk.ravel() > 0) & (kk.ravel() < n))
        q[interior] += d[interior]
    ck, cj, ci = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    base = ((ck.ravel() * m + cj.ravel()) * m + ci.ravel()).astype(np.int64)
    step = np.array([1, m, m * m], dtype=np.int64)     # +x, +y, +z
    tets = []
    # the six monotone paths v000 -> v111; odd permutations swap the last two
    # vertices so that every tetrahedron is positively oriented
    for perm, odd in (((0, 1, 2), False), ((1, 2, 0), False), ((2, 0, 1), False),
                      ((0, 2, 1), True), ((2, 1, 0), True), ((1, 0, 2), True)):
        a = base
        b = a + step[perm[0]]
        c = b + step[perm[1]]
        d4 = c + step[perm[2]]
        tets.append(np.stack([a, b, d4, c] if odd else [a, b, c, d4], axis=1))
    me = np.stack(tets, axis=1).reshape(-1, 4)
    if permute:
        q, me = _relabel(rng, q, me)
    return Mesh(np.ascontiguousarray(q), np.ascontiguousarray(me.astype(np.int32)), f"cube{n}")


def random_tiny_tet_mesh(rng: np.random.Generator, max_q: int = 30):
    """A small random tetrahedron soup over <= max_q vertices in [-1, 1]^3
    (distinct vertices per element; elements may overlap, vertices may be
    unused); for brute-force cross-checks."""
    nq = int(rng.integers(4, max_q + 1))
    q = rng.uniform(-1.0, 1.0, size=(nq, 3))
    nme = int(rng.integers(1, 3 * nq))
    me = np.stack([rng.choice(nq, 4, replace=False) for _ in range(nme)]).astype(np.int32)
    return Mesh(q, me, "tiny_tets")


def weight_quadratic(q: np.ndarray) -> np.ndarray:
    """w(x, y) = 1 + x^2 + y^2 sampled at the vertices (Tw of the paper)."""
    return 1.0 + q[:, 0] ** 2 + q[:, 1] ** 2


def weight_uniform(nq: int, lo: float = 0.5, hi: float = 2.0, seed: int = BASE_SEED) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(lo, hi, size=nq)


def normal_seed(n: int, seed: int = BASE_SEED) -> np.ndarray:
    """N(0,1) values, e.g. the adjoint seed G on a CSR pattern of n entries."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal(n)


# ---- the workloads -------------------------------------------------------

def config_mesh(idx: int):
    """The seeded mesh of workload ``idx`` (1..5; see module docstring).

    1: square 32x32 (nq 1089, nme 2048)        2: square 2048x2048 (nme 8.4M)
    3: disk K=1024 (nme 6.3M)                  4: batch of 512 squares
    5: square 512x512 (nme 524288)
    """
    seed = BASE_SEED + idx
    if idx == 1:
        return unit_square(32, seed=seed)
    if idx == 2:
        return unit_square(2048, seed=seed)
    if idx == 3:
        return unit_disk(1024, seed=seed)
    if idx == 4:
        return batch_of_squares(512, 8, 512, seed=seed)
    if idx == 5:
        return unit_square(512, seed=seed)
    raise ValueError(idx)


def random_tiny_mesh(rng: np.random.Generator, max_q: int = 50):
    """A small random triangle soup over <= max_q vertices with distinct
    vertices per triangle (random coordinates, so no zero areas in practice);
    used for brute-force cross-checks.  Triangles may overlap and vertices may
    be unused (empty rows)."""
    nq = int(rng.integers(3, max_q + 1))
    q = rng.uniform(-1.0, 1.0, size=(nq, 2))
    nme = int(rng.integers(1, 3 * nq))
    me = np.empty((nme, 3), np.int32)
    for k in range(nme):
        me[k] = rng.choice(nq, size=3, replace=False)
    return Mesh(q, me, "tiny")
