"""Seeded synthetic inputs for the time-stepping workloads.

This module holds random draws and problem parameters only: no step of the
solver's arithmetic lives here. It feeds both the HIP path (through the
binding) and the CPU oracle (through the tests), so that the two sides see
bit-identical inputs.

Random numbers come from splitmix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014): the state advances by the
golden-ratio increment and each output is the state passed through the
64-bit finalizer.  Stream ``k`` of seed ``s`` starts from
``mix(s ^ mix(k + 1))``, so every quantity (direction, forcing, P, ...) has
its own reproducible stream.

Problems (the matrix itself is assembled on each side independently; this
module only fixes the parameters):

* convection-diffusion ``-div(kappa grad u) + beta . grad u`` on the unit
  square/cube, ``n`` interior nodes per axis, homogeneous Dirichlet,
  first-order upwind, implicit Euler with ``inv_dt = 1/dt``;
* 2-D direction ``beta = Pe (cos t, sin t)`` with ``t = 2 pi u``;
  3-D direction ``beta = Pe g/|g|`` with ``g`` a standard normal triple;
* forcing ``f`` i.i.d. U(0,1), drawn once and kept fixed over time;
* variable diffusion ``kappa = exp(z)``, ``z`` standard normal per node;
* the cut-space basis P: uniform entries on [-1, 1) from a counter-based
  hash (a random choice of P, which the method allows), see :func:`p_dense`;
* an unstructured matrix from a random geometric graph on the periodic unit
  3-torus (:func:`rgg`): identity plus graph Laplacian plus an antisymmetric
  convection term, rows relabelled by a random permutation.  Its CSR arrays
  are built here (the graph is the random input), identically for both sides.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

MASK64 = (1 << 64) - 1
GOLDEN = 0x9E3779B97F4A7C15

# stream ids
S_THETA, S_FORCING, S_P, S_KAPPA, S_DIR, S_BUMPS, S_XI, S_RGG = range(1, 9)


def mix64(z: int) -> int:
    """splitmix64 output finalizer on a Python int."""
    z &= MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def _mix64_np(z: np.ndarray) -> np.ndarray:
    z = z.astype(np.uint64, copy=True)
    with np.errstate(over="ignore"):
        z ^= z >> np.uint64(30)
        z *= np.uint64(0xBF58476D1CE4E5B9)
        z ^= z >> np.uint64(27)
        z *= np.uint64(0x94D049BB133111EB)
        z ^= z >> np.uint64(31)
    return z


def stream_start(seed: int, stream: int) -> int:
    return mix64((seed & MASK64) ^ mix64(stream + 1))


def u64(seed: int, stream: int, count: int, offset: int = 0) -> np.ndarray:
    """Outputs offset..offset+count-1 of the splitmix64 stream."""
    s0 = np.uint64(stream_start(seed, stream))
    i = np.arange(offset + 1, offset + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        state = s0 + i * np.uint64(GOLDEN)
    return _mix64_np(state)


def uniform(seed: int, stream: int, count: int, offset: int = 0) -> np.ndarray:
    """U[0,1) doubles from the top 53 bits."""
    return (u64(seed, stream, count, offset) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def normal(seed: int, stream: int, count: int, offset: int = 0) -> np.ndarray:
    """Standard normals by Box-Muller on consecutive uniform pairs.

    ``offset`` counts pairs (two uniforms each)."""
    m = (count + 1) // 2
    u = uniform(seed, stream, 2 * m, 2 * offset)
    u1, u2 = u[0::2], u[1::2]
    rad = np.sqrt(-2.0 * np.log1p(-u1))
    z = np.empty(2 * m)
    z[0::2] = rad * np.cos(2.0 * np.pi * u2)
    z[1::2] = rad * np.sin(2.0 * np.pi * u2)
    return z[:count]


def p_key(seed: int) -> int:
    """32-bit key of the cut-space basis P for ``seed`` (low word of stream S_P's start)."""
    return stream_start(seed, S_P) & 0xFFFFFFFF


def fmix32(h: np.ndarray) -> np.ndarray:
    """MurmurHash3 32-bit finalizer (Appleby), elementwise on uint32."""
    h = h.astype(np.uint32, copy=True)
    with np.errstate(over="ignore"):
        h ^= h >> np.uint32(16)
        h *= np.uint32(0x85EBCA6B)
        h ^= h >> np.uint32(13)
        h *= np.uint32(0xC2B2AE35)
        h ^= h >> np.uint32(16)
    return h


def p_dense(seed: int, n: int, s: int) -> np.ndarray:
    """Cut-space basis P (n x s, column-major), entries uniform on [-1, 1).

    Entry (i, q) = (t - 2^23) / 2^23 with t the top 24 bits of
    fmix32(key + (8 i + q) * 0x9E3779B9 mod 2^32): a counter-based draw, so any
    entry can be regenerated where it is needed, and exact in FP32 and FP64.
    Column q does not depend on s (s <= 8).
    """
    if not 1 <= s <= 8:
        raise ValueError("s must be in 1..8")
    if 8 * n >= 2 ** 32:
        raise ValueError("n too large for the 32-bit counter")
    key = np.uint32(p_key(seed))
    P = np.empty((n, s), dtype=np.float64, order="F")
    i = np.arange(n, dtype=np.uint64)
    for q in range(s):
        ctr = ((np.uint64(8) * i + np.uint64(q)) * np.uint64(0x9E3779B9) + np.uint64(key)) & np.uint64(0xFFFFFFFF)
        t = (fmix32(ctr.astype(np.uint32)) >> np.uint32(8)).astype(np.int64)
        P[:, q] = (t - (1 << 23)).astype(np.float64) * (2.0 ** -23)
    return P


@dataclass
class ConvDiff:
    """Parameters of one implicit-Euler convection-diffusion sequence."""
    dim: int
    n: int
    beta: tuple
    inv_dt: float
    f: np.ndarray
    kappa: np.ndarray | None = None
    name: str = ""
    seed: int = 0
    extra: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        return self.n ** self.dim

    def nnz(self) -> int:
        n, d = self.n, self.dim
        return n ** d + 2 * d * (n - 1) * n ** (d - 1)


def convdiff(dim: int, n: int, pe: float, seed: int, dt: float = 1e-3,
             variable_kappa: bool = False, forcing: str = "uniform",
             name: str = "") -> ConvDiff:
    if dim == 2:
        t = 2.0 * math.pi * float(uniform(seed, S_THETA, 1)[0])
        beta = (pe * math.cos(t), pe * math.sin(t), 0.0)
    elif dim == 3:
        g = normal(seed, S_DIR, 3)
        nrm = math.sqrt(float(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]))
        beta = tuple(float(pe * gi / nrm) for gi in g)
    else:
        raise ValueError("dim must be 2 or 3")
    N = n ** dim
    f = uniform(seed, S_FORCING, N) if forcing == "uniform" else np.zeros(N)
    kappa = np.exp(normal(seed, S_KAPPA, N)) if variable_kappa else None
    return ConvDiff(dim, n, beta, 1.0 / dt, f, kappa, name, seed)


def config(name: str, seed: int = 0, n: int | None = None) -> ConvDiff:
    """The convection-diffusion workloads by name.

    ``c1`` 2-D 64^2 Pe=50; ``c2`` 3-D 128^3 Pe=100; ``c3`` 3-D 256^3 Pe=200 with
    lognormal diffusion; ``c4`` 2-D 512^2 Pe=100 (moving Gaussian bumps).
    ``n`` overrides the grid size (for small test instances of the same kind).
    """
    if name == "c1":
        return convdiff(2, n or 64, 50.0, seed, name=name)
    if name == "c2":
        return convdiff(3, n or 128, 100.0, seed, name=name)
    if name == "c3":
        return convdiff(3, n or 256, 200.0, seed, variable_kappa=True, name=name)
    if name == "c4":
        cd = convdiff(2, n or 512, 100.0, seed, forcing="none", name=name)
        cd.extra["bumps"] = Bumps(seed)
        return cd
    raise KeyError(name)


class Bumps:
    """Forcing made of 8 Gaussian bumps that drift and reflect at the walls.

    Amplitude a ~ U(0.5,1.5), width sigma ~ U(0.02,0.06), centre ~ U(0.1,0.9)^2,
    velocity ~ U(-0.01,0.01)^2 per time step.
    """

    def __init__(self, seed: int, count: int = 8):
        u = uniform(seed, S_BUMPS, 7 * count).reshape(count, 7)
        self.a = 0.5 + u[:, 0]
        self.sigma = 0.02 + 0.04 * u[:, 1]
        self.c = 0.1 + 0.8 * u[:, 2:4]
        self.v = -0.01 + 0.02 * u[:, 4:6]

    def at(self, step: int, n: int) -> np.ndarray:
        """Forcing on the n x n interior grid (x fastest) at time step ``step``."""
        c = self.c + step * self.v
        # reflect into [0,1]
        c = np.abs(c) % 2.0
        c = np.where(c > 1.0, 2.0 - c, c)
        h = 1.0 / (n + 1)
        g = h * np.arange(1, n + 1)
        X, Y = np.meshgrid(g, g, indexing="xy")
        f = np.zeros((n, n))
        for k in range(len(self.a)):
            d2 = (X - c[k, 0]) ** 2 + (Y - c[k, 1]) ** 2
            f += self.a[k] * np.exp(-d2 / (2.0 * self.sigma[k] ** 2))
        return f.reshape(-1)


def tridiag_231(n: int = 40):
    """The finite-termination test matrix tridiag(2,3,1) (sub, diag, super) as CSR.

    Returns (row_ptr, col_idx, val) with int32 indices, columns sorted.
    """
    rp = [0]
    ci, va = [], []
    for i in range(n):
        if i > 0:
            ci.append(i - 1); va.append(2.0)
        ci.append(i); va.append(3.0)
        if i < n - 1:
            ci.append(i + 1); va.append(1.0)
        rp.append(len(ci))
    return (np.array(rp, dtype=np.int32), np.array(ci, dtype=np.int32),
            np.array(va, dtype=np.float64))


def sin_rhs(n: int = 40) -> np.ndarray:
    """b2 = sin(2 pi / n * (1..n))."""
    return np.sin(2.0 * np.pi / n * np.arange(1, n + 1, dtype=np.float64))


def white_noise(seed: int, step: int, N: int) -> np.ndarray:
    """xi ~ N(0,1) for step ``step`` (distinct block of the XI stream)."""
    return normal(seed, S_XI, N, offset=step * ((N + 1) // 2))


@dataclass
class Graph:
    """CSR of A = I + L + S on a random geometric graph (see :func:`rgg`)."""
    N: int
    radius: float
    beta: tuple
    row_ptr: np.ndarray
    col: np.ndarray
    val: np.ndarray
    seed: int = 0

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])


def rgg(N: int, seed: int, degree: float = 14.0) -> Graph:
    """Random geometric graph matrix on the periodic unit 3-torus.

    N points uniform on [0,1)^3 (stream RGG); an edge joins two points closer
    than r = (3 degree / (4 pi N))^(1/3) in the periodic metric (expected
    degree ``degree``).  With W the 0/1 adjacency, D its degrees and
    p_j - p_i the shortest periodic displacement,
        A = I + (D - W) + S,   S_ij = beta . (p_j - p_i) / (2 r)
    (S antisymmetric; beta a unit vector, a normalized standard normal triple
    of stream DIR).  Rows and columns are relabelled by one random
    permutation (the argsort of uniform keys that follow the points in the
    RGG stream); columns are sorted within each row.
    """
    from scipy.spatial import cKDTree
    pts = uniform(seed, S_RGG, 3 * N).reshape(N, 3)
    r = (3.0 * degree / (4.0 * math.pi * N)) ** (1.0 / 3.0)
    pairs = cKDTree(pts, boxsize=1.0).query_pairs(r, output_type="ndarray")
    i, j = pairs[:, 0].astype(np.int64), pairs[:, 1].astype(np.int64)
    del pairs
    g = normal(seed, S_DIR, 3)
    beta = g / math.sqrt(float(g @ g))
    disp = pts[j] - pts[i]
    disp -= np.round(disp)
    sij = (disp @ beta) / (2.0 * r)
    del disp
    deg = np.bincount(i, minlength=N) + np.bincount(j, minlength=N)
    perm = np.argsort(uniform(seed, S_RGG, N, offset=3 * N), kind="stable")
    new = np.empty(N, dtype=np.int64)
    new[perm] = np.arange(N, dtype=np.int64)          # old index -> new index
    rows = np.concatenate([new[i], new[j], new])
    cols = np.concatenate([new[j], new[i], new])
    vals = np.concatenate([-1.0 + sij, -1.0 - sij, 1.0 + deg.astype(np.float64)])
    del i, j, sij
    order = np.argsort(rows * N + cols, kind="stable")
    rows, cols, vals = rows[order], cols[order], vals[order]
    row_ptr = np.zeros(N + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=N), out=row_ptr[1:])
    return Graph(N, r, tuple(float(b) for b in beta), row_ptr.astype(np.int32),
                 cols.astype(np.int32), vals, seed)
