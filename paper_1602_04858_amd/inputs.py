"""Seeded synthetic inputs: permeability-coefficient fields and right-hand-side data.

This module holds no arithmetic of the solver: it only draws random numbers and
builds coefficient fields and source functions.  Both the GPU library and the CPU
oracle consume what it produces.

The paper's own fields (the foam / inclusion images of its first test set and the
SPE10 slices) are not available, so the generators below stand in for them with the
same kind of structure: a cellwise coefficient on a square grid, contrast of 1e4 to
1e8, thin connected high-permeability channels and horizontal layers (Section 4,
"Tests on some characteristic permeability fields" and "Tests with permeability of
SPE10 benchmark").  The coefficient returned is the equation coefficient kappa of
the Brinkman/Darcy system (Section 2.2); cells are ordered c = cy*N + cx.

Random numbers come from SplitMix64 (Steele, Lea, Flood 2014) turned into normals by
the Box-Muller transform; seed = 1000*config + problem index.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, n: int, offset: int = 0) -> np.ndarray:
    """n consecutive SplitMix64 outputs of the stream `seed`, starting at `offset`."""
    with np.errstate(over="ignore"):
        i = np.arange(offset + 1, offset + n + 1, dtype=np.uint64)
        z = np.uint64(seed) + _GOLDEN * i
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform(seed: int, n: int, offset: int = 0) -> np.ndarray:
    """Uniform numbers in the open interval (0, 1) (53 random bits)."""
    z = splitmix64(seed, n, offset)
    return ((z >> np.uint64(11)).astype(np.float64) + 0.5) * (1.0 / 9007199254740992.0)


def normal(seed: int, n: int, offset: int = 0) -> np.ndarray:
    """Standard normal numbers by Box-Muller on consecutive uniform pairs."""
    m = (n + 1) // 2
    u = uniform(seed, 2 * m, offset)
    u1, u2 = u[0::2], u[1::2]
    r = np.sqrt(-2.0 * np.log(u1))
    z = np.empty(2 * m)
    z[0::2] = r * np.cos(2.0 * math.pi * u2)
    z[1::2] = r * np.sin(2.0 * math.pi * u2)
    return z[:n]


class _Stream:
    """Sequential reader over one seeded uniform stream."""

    def __init__(self, seed: int):
        self.seed = int(seed)
        self.pos = 0

    def uniform(self, n: int) -> np.ndarray:
        out = uniform(self.seed, n, self.pos)
        self.pos += n
        return out

    def normal(self, n: int) -> np.ndarray:
        m = 2 * ((n + 1) // 2)
        out = normal(self.seed, n, self.pos)
        self.pos += m
        return out


def _channels(log10k: np.ndarray, st: _Stream, count: int, width: int, value: float) -> None:
    """Paint `count` meandering channels of `width` cells with log10 kappa = value.

    Each channel is horizontal or vertical (fair coin); its centre line starts at a
    uniform position and moves by -1, 0 or +1 cell per step (a random walk).
    """
    n = log10k.shape[0]
    for _ in range(count):
        horizontal = st.uniform(1)[0] < 0.5
        pos = int(st.uniform(1)[0] * (n - width + 1))
        steps = st.uniform(n)
        for t in range(n):
            if t > 0:
                pos += int(math.floor(steps[t] * 3.0)) - 1
                pos = min(max(pos, 0), n - width)
            if horizontal:
                log10k[pos:pos + width, t] = value     # rows cy, column cx = t
            else:
                log10k[t, pos:pos + width] = value


def kappa_lognormal_channels(n: int, seed: int, mean: float = -3.0, std: float = 1.5,
                             lo: float = -6.0, hi: float = 0.0, channels: int = 20,
                             width: int = 2) -> np.ndarray:
    """log10 kappa ~ N(mean, std) iid per cell, clipped to [lo, hi], plus channels at hi."""
    st = _Stream(seed)
    g = np.clip(mean + std * st.normal(n * n), lo, hi).reshape(n, n)
    _channels(g, st, channels, width, hi)
    return np.power(10.0, g).reshape(-1)


def kappa_layered(n: int, seed: int, layers: int = 85, channels: int = 20,
                  width: int = 4) -> np.ndarray:
    """Horizontal layers (each log-normal around its own mean) plus meandering channels.

    Layer l covers rows floor(l*n/layers) .. floor((l+1)*n/layers)-1; its mean of
    log10 kappa is U[-5, 0]; cells are N(mean, 1), clipped to [-6, 1]; channels of
    `width` cells carry kappa = 10.
    """
    st = _Stream(seed)
    means = -5.0 + 5.0 * st.uniform(layers)
    g = np.empty((n, n))
    for l in range(layers):
        r0, r1 = (l * n) // layers, ((l + 1) * n) // layers
        if r1 > r0:
            g[r0:r1, :] = means[l] + st.normal((r1 - r0) * n).reshape(r1 - r0, n)
    g = np.clip(g, -6.0, 1.0)
    _channels(g, st, channels, width, 1.0)
    return np.power(10.0, g).reshape(-1)


def kappa_layered3(n: int, seed: int, layers: int = 85) -> np.ndarray:
    """3-D stand-in for the layered SPE10 field (Section 4, 3-D Brinkman test): horizontal
    layers along z, layer l covering z-rows floor(l*n/layers) .. floor((l+1)*n/layers)-1,
    with log10 kappa of the layer ~ U[-5, 0] and cells N(mean, 1), clipped to [-6, 1].
    Cells are ordered c = (cz*N + cy)*N + cx."""
    st = _Stream(seed)
    means = -5.0 + 5.0 * st.uniform(layers)
    g = np.empty((n, n, n))
    for l in range(layers):
        z0, z1 = (l * n) // layers, ((l + 1) * n) // layers
        if z1 > z0:
            g[z0:z1] = means[l] + st.normal((z1 - z0) * n * n).reshape(z1 - z0, n, n)
    return np.power(10.0, np.clip(g, -6.0, 1.0)).reshape(-1)


# ---------------------------------------------------------------------------
# Two-phase fields (stand-ins for the open-foam / inclusion / connected-inclusion
# images of the robustness tests of Section 4: kappa = 1 in one phase, 10^-e in the
# other, given on a 128 x 128 pixel grid and resolved by finer meshes)
# ---------------------------------------------------------------------------
PHASE_KINDS = ("foam", "inclusions", "connected")


def _disks(st: _Stream, m: int, target: float, rmin: float, rmax: float, overlap: bool) -> list:
    """Random disks (cx, cy, r) in pixel units on an m x m grid until the covered
    fraction of the area reaches `target`; without `overlap` a disk is kept only if it
    keeps a gap of 2 pixels to every kept disk."""
    disks, covered, tries = [], 0.0, 0
    while covered < target and tries < 20000:
        u = st.uniform(3)
        tries += 1
        r = rmin + (rmax - rmin) * u[2]
        cx, cy = r + (m - 2 * r) * u[0], r + (m - 2 * r) * u[1]
        if not overlap and any((cx - a) ** 2 + (cy - b) ** 2 < (r + q + 2.0) ** 2 for a, b, q in disks):
            continue
        disks.append((cx, cy, r))
        covered += math.pi * r * r / (m * m)
    return disks


def _paint_disks(disks: list, m: int) -> np.ndarray:
    yy, xx = np.mgrid[0:m, 0:m] + 0.5
    out = np.zeros((m, m), dtype=bool)
    for cx, cy, r in disks:
        out |= (xx - cx) ** 2 + (yy - cy) ** 2 <= r * r
    return out


def _paint_segment(img: np.ndarray, a: tuple, b: tuple, width: int) -> None:
    """A straight band of `width` pixels from point a to point b."""
    m = img.shape[0]
    steps = int(2 * max(abs(b[0] - a[0]), abs(b[1] - a[1]))) + 1
    for t in np.linspace(0.0, 1.0, steps):
        x, y = a[0] + t * (b[0] - a[0]), a[1] + t * (b[1] - a[1])
        x0, y0 = int(x - width / 2 + 0.5), int(y - width / 2 + 0.5)
        img[max(y0, 0):min(y0 + width, m), max(x0, 0):min(x0 + width, m)] = True


def phase_image(kind: str, seed: int, m: int = 128) -> np.ndarray:
    """m x m boolean image of the structure phase (row = y pixel, column = x pixel).

    foam: the walls of a Voronoi tessellation of 40 random sites, 2 pixels thick -- a
          connected skeleton spanning the domain, open pores between;
    inclusions: disjoint disks of radius 3..8 pixels (2-pixel gaps), 20% of the area;
    connected: the inclusions joined into chains: every disk is linked to its nearest
          neighbour by a 2-pixel band, and the chain of disks nearest the left edge to
          the right edge, so that the structure phase spans the domain.
    """
    st = _Stream(seed)
    if kind == "foam":
        sites = st.uniform(80).reshape(40, 2) * m
        yy, xx = np.mgrid[0:m, 0:m] + 0.5
        d = np.sqrt((xx[..., None] - sites[:, 0]) ** 2 + (yy[..., None] - sites[:, 1]) ** 2)
        d.sort(axis=-1)
        return (d[..., 1] - d[..., 0]) < 2.0
    disks = _disks(st, m, 0.20, 3.0, 8.0, overlap=False)
    img = _paint_disks(disks, m)
    if kind == "inclusions":
        return img
    if kind != "connected":
        raise KeyError(kind)
    for i, (x, y, _) in enumerate(disks):
        j = min((k for k in range(len(disks)) if k != i),
                key=lambda k: (disks[k][0] - x) ** 2 + (disks[k][1] - y) ** 2)
        _paint_segment(img, (x, y), (disks[j][0], disks[j][1]), 2)
    # a spanning path: from the left edge through the disks ordered by x to the right edge
    order = sorted(range(len(disks)), key=lambda k: disks[k][0])
    band = sorted(order, key=lambda k: abs(disks[k][1] - m / 2))[: max(2, len(disks) // 4)]
    band.sort(key=lambda k: disks[k][0])
    pts = [(0.0, disks[band[0]][1])] + [(disks[k][0], disks[k][1]) for k in band] + [(float(m), disks[band[-1]][1])]
    for a, b in zip(pts[:-1], pts[1:]):
        _paint_segment(img, a, b, 2)
    return img


def kappa_two_phase(kind: str, seed: int, n: int, exponent: int, reverse: bool = False,
                    m: int = 128) -> np.ndarray:
    """Cellwise kappa on an n x n mesh (n a multiple of m) from the m x m phase image:
    the matrix phase kappa = 1 and the structure 10^-exponent (case (a)), or the reverse
    (case (b)); every pixel covers (n/m)^2 cells."""
    if n % m:
        raise ValueError("n must be a multiple of the image size")
    img = phase_image(kind, seed, m)
    low = img if not reverse else ~img
    k = np.where(low, 10.0 ** (-exponent), 1.0)
    r = n // m
    return np.repeat(np.repeat(k, r, axis=0), r, axis=1).reshape(-1)


def kappa_constant(n: int, value: float = 1.0) -> np.ndarray:
    return np.full(n * n, float(value))


def kappa_random_cells(n: int, seed: int, lo: float = 0.1, hi: float = 10.0) -> np.ndarray:
    """Cellwise kappa, log-uniform in [lo, hi] (small test problems)."""
    u = uniform(seed, n * n)
    return np.exp(math.log(lo) + (math.log(hi) - math.log(lo)) * u)


@dataclass
class SmoothSource:
    """f(x, y) = sum_m a_m * (cos th_m, sin th_m) * sin(2 pi (kx_m x + ky_m y) + ph_m)."""
    amp: np.ndarray
    theta: np.ndarray
    kx: np.ndarray
    ky: np.ndarray
    phase: np.ndarray

    def __call__(self, x: np.ndarray, y: np.ndarray) -> np.ndarray:
        out = np.zeros(x.shape + (2,))
        for a, th, kx, ky, ph in zip(self.amp, self.theta, self.kx, self.ky, self.phase):
            s = a * np.sin(2.0 * math.pi * (kx * x + ky * y) + ph)
            out[..., 0] += math.cos(th) * s
            out[..., 1] += math.sin(th) * s
        return out


def smooth_source(seed: int, modes: int = 4) -> SmoothSource:
    st = _Stream(seed)
    u = st.uniform(5 * modes).reshape(5, modes)
    return SmoothSource(amp=0.5 + u[0], theta=2.0 * math.pi * u[1],
                        kx=np.floor(1 + 3 * u[2]), ky=np.floor(1 + 3 * u[3]),
                        phase=2.0 * math.pi * u[4])


def constant_source(fx: float = 1.0, fy: float = 0.0):
    def f(x, y):
        out = np.zeros(np.shape(x) + (2,))
        out[..., 0] = fx
        out[..., 1] = fy
        return out
    return f


def random_vector(n: int, seed: int) -> np.ndarray:
    """Seeded N(0,1) vector (an algebraic right-hand side)."""
    return normal(seed, n)


# ---------------------------------------------------------------------------
# Workloads.  Boundary codes: 0 = Dirichlet (no-slip / prescribed), 1 = open.
# Side order: x = 0, x = 1, y = 0, y = 1.
# ---------------------------------------------------------------------------
DIRICHLET, OPEN = 0, 1


@dataclass
class Workload:
    name: str
    n0: int
    levels: int            # number of refinements J; the finest grid has n0 * 2**J cells per side
    k: int
    mu: float
    sigma: float
    bc: tuple
    kappa: np.ndarray
    source: object
    cycle: int             # 0 standard, 1 variable V-cycle
    m_fine: int
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.n0 << self.levels


def manufactured_c1():
    """u = curl(sin^2(pi x) sin^2(pi y)), p = 0 (u = 0 on the boundary)."""
    pi = math.pi

    def u(x, y):
        sx, cx, sy, cy = np.sin(pi * x), np.cos(pi * x), np.sin(pi * y), np.cos(pi * y)
        out = np.zeros(np.shape(x) + (2,))
        out[..., 0] = 2 * pi * sx * sx * sy * cy
        out[..., 1] = -2 * pi * sx * cx * sy * sy
        return out

    def f(x, y, mu, kap):
        # f = -mu lap u + kappa u (p = 0); lap of each component written out
        sx, cx, sy, cy = np.sin(pi * x), np.cos(pi * x), np.sin(pi * y), np.cos(pi * y)
        s2x, c2x, s2y, c2y = np.sin(2 * pi * x), np.cos(2 * pi * x), np.sin(2 * pi * y), np.cos(2 * pi * y)
        # u1 = pi * (1 - cos 2pi x)/2 * sin 2pi y ; lap u1 = pi*(2pi^2 cos2pi x sin2pi y) - pi*(1-cos2pi x)/2*4pi^2 sin 2pi y
        u1 = pi * 0.5 * (1 - c2x) * s2y
        lap1 = pi * (2 * pi * pi * c2x * s2y) - pi * 0.5 * (1 - c2x) * 4 * pi * pi * s2y
        # u2 = -pi * sin 2pi x * (1 - cos 2pi y)/2
        u2 = -pi * s2x * 0.5 * (1 - c2y)
        lap2 = pi * 4 * pi * pi * s2x * 0.5 * (1 - c2y) - pi * s2x * 2 * pi * pi * c2y
        out = np.zeros(np.shape(x) + (2,))
        out[..., 0] = -mu * lap1 + kap * u1
        out[..., 1] = -mu * lap2 + kap * u2
        return out
    return u, f


def workload(name: str, problem: int = 0) -> Workload:
    """The five benchmark shapes (C1..C5) plus the C4 batch members."""
    if name == "C1":
        return Workload("C1", 2, 2, 1, 1.0, 6.0, (DIRICHLET,) * 4, kappa_constant(8), None, 0, 1)
    if name == "C2":
        n = 256
        return Workload("C2", 2, 7, 1, 1e-2, 6.0, (DIRICHLET, DIRICHLET, OPEN, OPEN),
                        kappa_lognormal_channels(n, 2000 + problem), constant_source(1.0, 0.0), 1, 2)
    if name in ("C3", "C3darcy"):
        n = 1024
        mu = 0.0 if name == "C3darcy" else 1e-3
        return Workload(name, 2, 9, 1, mu, 6.0, (DIRICHLET, DIRICHLET, OPEN, OPEN),
                        kappa_lognormal_channels(n, 3000 + problem), constant_source(1.0, 0.0), 1, 2)
    if name == "C4":
        st = _Stream(4000 + 500 + problem)
        u = st.uniform(3)
        n = (128, 256, 384, 512)[min(int(u[0] * 4), 3)]
        n0 = 3 if n == 384 else 2
        c = 4.0 + 2.0 * u[1]
        mu = math.exp(math.log(1e-4) + (math.log(1.0) - math.log(1e-4)) * u[2])
        levels = int(round(math.log2(n // n0)))
        kap = kappa_lognormal_channels(n, 4000 + problem, mean=-c / 2, std=c / 4, lo=-c, hi=0.0)
        return Workload(f"C4.{problem}", n0, levels, 1, mu, 6.0, (DIRICHLET, DIRICHLET, OPEN, OPEN),
                        kap, smooth_source(4100 + problem), 1, 2)
    if name == "C5":
        n = 2048
        return Workload("C5", 2, 10, 2, 1e-2, 12.0, (DIRICHLET, DIRICHLET, OPEN, OPEN),
                        kappa_layered(n, 5000 + problem), smooth_source(5100 + problem), 1, 2)
    raise KeyError(name)


def scaled_workload(name: str, n: int, problem: int = 0) -> Workload:
    """The generator of workload `name` at a smaller grid of n cells per side."""
    w = workload(name, problem) if name != "C5" else None
    if name in ("C2", "C3", "C3darcy"):
        kap = kappa_lognormal_channels(n, (2000 if name == "C2" else 3000) + problem)
        mu = w.mu
        return Workload(f"{name}@{n}", 2, int(round(math.log2(n // 2))), 1, mu, 6.0, w.bc, kap,
                        constant_source(1.0, 0.0), 1, 2)
    if name == "C5":
        return Workload(f"C5@{n}", 2, int(round(math.log2(n // 2))), 2, 1e-2, 12.0,
                        (DIRICHLET, DIRICHLET, OPEN, OPEN), kappa_layered(n, 5000 + problem),
                        smooth_source(5100 + problem), 1, 2)
    raise KeyError(name)
