"""Seeded synthetic inputs: quadratures and problem definitions.

This module builds inputs only; it holds none of the method's arithmetic and
is shared by the HIP path's tests, the benchmark and the oracle's tests.
Random fields come from ``numpy.random.Generator(PCG64(seed))``; a draw
"log-uniform on [a, b]" is ``exp(U(ln a, ln b))``.

A problem is a dict with keys ``nx, ny, dx, dy`` (uniform Cartesian grid on
``[0, nx*dx] x [0, ny*dy]``, cell ``c = j*nx + i``), ``mu, eta, w`` (in-plane
direction cosines and weights of the ordinates, ``sum(w) = 4*pi``),
``sigma_a, sigma_s, q`` (per cell, ``q`` is the isotropic volumetric source
integrated over the sphere) and ``bnd_in`` (``None`` for vacuum, else
``[2*(nx+ny), K]`` incoming intensities on sides W, E, S, N in that order).
"""
import math

import numpy as np


# --------------------------------------------------------------------------
# Quadratures (Sec. 4.1: the sphere is split into K ordinates with weights).
# 2D problems are symmetric in z, so each pair of 3D ordinates (xi, -xi) is
# folded into one in-plane ordinate carrying both weights.
# --------------------------------------------------------------------------
def quad_s4():
    """Level-symmetric S4 folded to 2D: 3 ordinates per quadrant, K = 12.

    mu1 = 0.3500212 and mu2 from 2*mu1^2 + mu2^2 = 1; every ordinate carries
    4*pi/12.
    """
    m1 = 0.3500212
    m2 = math.sqrt(1.0 - 2.0 * m1 * m1)
    base = [(m1, m1), (m1, m2), (m2, m1)]
    mu, eta = [], []
    for sx, sy in [(1, 1), (-1, 1), (-1, -1), (1, -1)]:
        for a, b in base:
            mu.append(sx * a)
            eta.append(sy * b)
    K = len(mu)
    return np.array(mu), np.array(eta), np.full(K, 4.0 * math.pi / K)


def quad_product(n_polar, n_azimuth):
    """Gauss-Legendre polar x Chebyshev azimuthal product set folded to 2D.

    The polar cosines are the ``n_polar`` positive nodes of the
    ``2*n_polar``-point Gauss-Legendre rule (weights doubled by the fold);
    azimuths are ``(2j-1)*pi/n_azimuth``, ``j = 1..n_azimuth``, with equal
    weights ``2*pi/n_azimuth``. K = n_polar * n_azimuth.
    """
    x, wx = np.polynomial.legendre.leggauss(2 * n_polar)
    sel = x > 0
    xi, wxi = x[sel], 2.0 * wx[sel]
    phis = (2.0 * np.arange(1, n_azimuth + 1) - 1.0) * math.pi / n_azimuth
    wphi = 2.0 * math.pi / n_azimuth
    mu, eta, w = [], [], []
    for p in range(len(xi)):
        s = math.sqrt(1.0 - xi[p] * xi[p])
        for a in phis:
            mu.append(s * math.cos(a))
            eta.append(s * math.sin(a))
            w.append(wxi[p] * wphi)
    return np.array(mu), np.array(eta), np.array(w)


def quad_gl_product_full(n_theta, n_phi):
    """Gauss-Legendre in both angles, polar axis along x (as in the paper's 2D
    runs): mu = cos(theta), eta = sin(theta) cos(phi); not folded (K =
    n_theta * n_phi, opposite z-halves kept as separate ordinates)."""
    ct, wt = np.polynomial.legendre.leggauss(n_theta)
    up, wp = np.polynomial.legendre.leggauss(n_phi)
    ph = math.pi * (up + 1.0)
    wph = math.pi * wp
    mu, eta, w = [], [], []
    for a in range(n_theta):
        st = math.sqrt(1.0 - ct[a] * ct[a])
        for b in range(n_phi):
            mu.append(ct[a])
            eta.append(st * math.cos(ph[b]))
            w.append(wt[a] * wph[b])
    return np.array(mu), np.array(eta), np.array(w)


def _base(nx, ny, quad, lx=1.0, ly=1.0):
    mu, eta, w = quad
    return dict(nx=int(nx), ny=int(ny), dx=lx / nx, dy=ly / ny,
                mu=np.asarray(mu, np.float64), eta=np.asarray(eta, np.float64),
                w=np.asarray(w, np.float64), bnd_in=None)


def iso_inflow(nx, ny, K, west=0.0, east=0.0, south=0.0, north=0.0):
    """Isotropic incoming intensities per side (W, E, S, N face order)."""
    b = np.zeros((2 * (nx + ny), K))
    b[0:ny] = west
    b[ny:2 * ny] = east
    b[2 * ny:2 * ny + nx] = south
    b[2 * ny + nx:] = north
    return b


# --------------------------------------------------------------------------
# Workloads
# --------------------------------------------------------------------------
def homogeneous(nx=32, ny=32, quad=None, sigma_t=1.0, c=0.9, q=1.0):
    """Uniform medium with scattering ratio c = sigma_s/sigma_t, vacuum."""
    p = _base(nx, ny, quad if quad is not None else quad_s4())
    N = nx * ny
    p["sigma_s"] = np.full(N, c * sigma_t)
    p["sigma_a"] = np.full(N, (1.0 - c) * sigma_t)
    p["q"] = np.full(N, float(q))
    return p


def small_s4_32():
    """32 x 32 cells, S4, sigma_t = 1, c = 0.9, unit source, vacuum."""
    return homogeneous(32, 32, quad_s4(), 1.0, 0.9, 1.0)


def thick_square(n=256, quad=None, thick_sigma_t=1e3, thick_c=0.9999,
                 thin_sigma_t=1.0, thin_c=0.5):
    """Two-region multiscale medium on the unit square.

    Central square [1/4, 3/4]^2 (cells n/4 .. 3n/4-1 in both directions):
    sigma_t = 1e3, c = 0.9999, q = 1. Elsewhere sigma_t = 1, c = 0.5, q = 0.
    Vacuum boundaries. Default quadrature GL8+ x Chebyshev-32 (K = 128).
    """
    p = _base(n, n, quad if quad is not None else quad_product(4, 32))
    ii, jj = np.meshgrid(np.arange(n), np.arange(n))
    inside = ((ii >= n // 4) & (ii < 3 * n // 4) & (jj >= n // 4) & (jj < 3 * n // 4)).ravel()
    st = np.where(inside, thick_sigma_t, thin_sigma_t)
    cc = np.where(inside, thick_c, thin_c)
    p["sigma_s"] = cc * st
    p["sigma_a"] = st - p["sigma_s"]
    p["q"] = np.where(inside, 1.0, 0.0)
    return p


def checkerboard_blocks(n=1024, quad=None, blocks=7, seed=3):
    """7 x 7 blocks; per block (row-major) sigma_a ~ logU[1e-2, 1e2] then
    sigma_s ~ logU[1e-1, 1e4]; unit source everywhere; vacuum."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nb = blocks * blocks
    sa = np.exp(rng.uniform(math.log(1e-2), math.log(1e2), nb))
    ss = np.exp(rng.uniform(math.log(1e-1), math.log(1e4), nb))
    p = _base(n, n, quad if quad is not None else quad_product(4, 32))
    bi = (np.arange(n) * blocks) // n
    BI, BJ = np.meshgrid(bi, bi)           # BI: column block, BJ: row block
    idx = (BJ * blocks + BI).ravel()
    p["sigma_a"] = sa[idx]
    p["sigma_s"] = ss[idx]
    p["q"] = np.ones(n * n)
    return p


def batch_problems(count=64, seed=4, sizes=(64, 128, 256, 512)):
    """Uneven batch: per problem nx, ny ~ U{sizes}; quadrature one of
    (GL4+ 2 polar x 16 az), (GL4+ 2 x 32), (GL8+ 4 x 32); 8 x 8 blocks with
    sigma_t ~ logU[0.1, 1e4] and c ~ U[0.5, 0.9999]; q = 1; vacuum."""
    rng = np.random.Generator(np.random.PCG64(seed))
    quads = [(2, 16), (2, 32), (4, 32)]
    out = []
    for _ in range(count):
        nx = int(sizes[rng.integers(0, len(sizes))])
        ny = int(sizes[rng.integers(0, len(sizes))])
        qp, qa = quads[rng.integers(0, 3)]
        st = np.exp(rng.uniform(math.log(0.1), math.log(1e4), 64))
        cc = rng.uniform(0.5, 0.9999, 64)
        p = _base(nx, ny, quad_product(qp, qa))
        bi = (np.arange(nx) * 8) // nx
        bj = (np.arange(ny) * 8) // ny
        BI, BJ = np.meshgrid(bi, bj)
        idx = (BJ * 8 + BI).ravel()
        p["sigma_s"] = (cc * st)[idx]
        p["sigma_a"] = (st - cc * st)[idx]
        p["q"] = np.ones(nx * ny)
        out.append(p)
    return out


def noisy_thick_square(n=512, quad=None, seed=5, amp=0.2):
    """The two-region medium with +-20% per-cell noise on sigma_a and sigma_s
    (u, v ~ U[-1, 1] drawn in that order)."""
    p = thick_square(n, quad)
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.uniform(-1.0, 1.0, n * n)
    v = rng.uniform(-1.0, 1.0, n * n)
    p["sigma_a"] = p["sigma_a"] * (1.0 + amp * u)
    p["sigma_s"] = p["sigma_s"] * (1.0 + amp * v)
    return p


def detector_window(n=512):
    """Cell mask of the 32 x 32 detector: i in [27n/32, 29n/32), j in
    [15n/32, 17n/32) (i in [432, 464), j in [240, 272) at n = 512)."""
    i0, i1 = (27 * n) // 32, (29 * n) // 32
    j0, j1 = (15 * n) // 32, (17 * n) // 32
    m = np.zeros((n, n), bool)
    m[j0:j1, i0:i1] = True
    return m.ravel()


def adjoint_fd_cells(n=512, seed=55):
    """16 cells (caller's index j*n + i) for finite-difference checks of the
    detector gradient: 4 in the detector window, 4 on the thick square's
    east edge, 4 between the two, 4 anywhere; drawn with PCG64(seed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    i0, i1 = (27 * n) // 32, (29 * n) // 32
    j0, j1 = (15 * n) // 32, (17 * n) // 32
    e = (3 * n) // 4 - 1
    cells = []
    for _ in range(4):
        cells.append(int(rng.integers(j0, j1)) * n + int(rng.integers(i0, i1)))
    for _ in range(4):
        cells.append(int(rng.integers(n // 4, (3 * n) // 4)) * n + e)
    for _ in range(4):
        cells.append(int(rng.integers(j0, j1)) * n + int(rng.integers(e + 1, i0)))
    for _ in range(4):
        cells.append(int(rng.integers(0, n * n)))
    return np.array(cells)


def random_problem(nx, ny, quad=None, seed=0, sigma_range=(0.1, 10.0), c_range=(0.3, 0.95),
                   inflow=True):
    """Small random medium for parity tests: sigma_t log-uniform per cell,
    c uniform, q uniform in [0, 1], random isotropic inflow per face."""
    rng = np.random.Generator(np.random.PCG64(seed))
    p = _base(nx, ny, quad if quad is not None else quad_s4())
    N = nx * ny
    st = np.exp(rng.uniform(math.log(sigma_range[0]), math.log(sigma_range[1]), N))
    cc = rng.uniform(c_range[0], c_range[1], N)
    p["sigma_s"] = cc * st
    p["sigma_a"] = st - p["sigma_s"]
    p["q"] = rng.uniform(0.0, 1.0, N)
    if inflow:
        K = len(p["mu"])
        p["bnd_in"] = rng.uniform(0.0, 0.2, (2 * (nx + ny), K))
    return p


def diffusion_limit(n, eps):
    """Steady diffusion-limit problem (2D analogue of App. A): sigma_s =
    1/eps, sigma_a = 0, q = eps (source eps/(4 pi) per steradian), vacuum."""
    p = _base(n, n, quad_product(4, 16))
    N = n * n
    p["sigma_s"] = np.full(N, 1.0 / eps)
    p["sigma_a"] = np.zeros(N)
    p["q"] = np.full(N, eps)
    return p


def hot_wall_square(n=40, sigma_t=1.0, quad=None):
    """The paper's 2D steady test (Sec. 5.2): pure scatterer, bottom wall
    emits isotropically with energy density 1, other walls 1e-6."""
    p = _base(n, n, quad if quad is not None else quad_product(4, 32))
    N = n * n
    p["sigma_s"] = np.full(N, float(sigma_t))
    p["sigma_a"] = np.zeros(N)
    p["q"] = np.zeros(N)
    K = len(p["mu"])
    fourpi = 4.0 * math.pi
    p["bnd_in"] = iso_inflow(n, n, K, west=1e-6 / fourpi, east=1e-6 / fourpi,
                             south=1.0 / fourpi, north=1e-6 / fourpi)
    return p
