"""Seeded synthetic inputs shaped like the paper's workloads.

This module holds none of the method's arithmetic: it only places bodies
(random orientations, random sequential addition of bounding spheres, affine
rescaling of a periodic box) so that the GPU library and the CPU oracle can
be fed the same states.  Both sides import it; it imports neither.

Workload shapes (Sec. 5 of Palmer, Aktulga, Gao, arXiv 2506.14097):
  * two ellipsoids meeting head-on (inertial);
  * periodic packings of ellipsoids with semiaxes uniform in [0.5, 1.0] at a
    prescribed volume fraction (compacting suspension, Sec. 5.2);
  * monolayers of spherocylinders of diameter 1 (colony, Sec. 5.3);
  * a chainmail of interlaced rings (tori of major radius 1 and minor radius
    0.1) on a square lattice, pulled by the extensile field of Sec. 6.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

ELLIPSOID = 0
SPHEROCYLINDER = 1
TORUS = 2


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def shoemake_quaternions(rng: np.random.Generator, n: int) -> np.ndarray:
    """Uniform random unit quaternions, scalar first (Shoemake 1992)."""
    u1, u2, u3 = rng.random(n), rng.random(n), rng.random(n)
    a, b = np.sqrt(1.0 - u1), np.sqrt(u1)
    q = np.stack([b * np.cos(2 * np.pi * u3), a * np.sin(2 * np.pi * u2), a * np.cos(2 * np.pi * u2),
                  b * np.sin(2 * np.pi * u3)], axis=1)
    return q / np.linalg.norm(q, axis=1, keepdims=True)


def planar_quaternions(theta: np.ndarray) -> np.ndarray:
    """Rotations about z by theta (body x axis -> (cos, sin, 0))."""
    return np.stack([np.cos(theta / 2), np.zeros_like(theta), np.zeros_like(theta), np.sin(theta / 2)], axis=1)


def ellipsoid_volume(shape: np.ndarray) -> np.ndarray:
    return 4.0 / 3.0 * np.pi * shape[:, 0] * shape[:, 1] * shape[:, 2]


def bounding_radius(kind: np.ndarray, shape: np.ndarray) -> np.ndarray:
    return np.where(kind == ELLIPSOID, shape.max(axis=1),
                    np.where(kind == TORUS, shape[:, 0] + shape[:, 1], 0.5 * shape[:, 1] + shape[:, 0]))


# quaternions (scalar first) taking the body z axis to z, y and x
RING_FLAT = (1.0, 0.0, 0.0, 0.0)
RING_AXIS_Y = (math.cos(math.pi / 4), -math.sin(math.pi / 4), 0.0, 0.0)
RING_AXIS_X = (math.cos(math.pi / 4), 0.0, math.sin(math.pi / 4), 0.0)


def _qmul(a, b):
    s1, v1, s2, v2 = a[0], np.asarray(a[1:]), b[0], np.asarray(b[1:])
    return np.concatenate([[s1 * s2 - v1 @ v2], s1 * v2 + s2 * v1 + np.cross(v1, v2)])


def chainmail(nx: int = 5, ny: int = 5, R: float = 1.0, r: float = 0.1, slack: float = 0.45,
              xi: float = 1.0, jitter: float = 0.0, seed: int = 0) -> dict:
    """Interlaced rings on a square lattice (the paper's layout is not
    given; this one is ours): flat rings (axis z) at the nodes (i L, j L, 0)
    of an nx x ny lattice centred at the origin, and one connector ring per
    lattice edge at its midpoint, standing upright with its axis horizontal
    and normal to the edge (edges along x: axis y; along y: axis x).  A
    connector threads both rings of its edge: its centre circle crosses the
    plane z = 0 at L/2 - R from each node, inside the hole.  L is chosen so
    that pulling a connector and a node ring apart along the edge closes a
    surface gap of `slack` before the tubes touch: L/2 = 2 (R - r) - slack.
    jitter > 0 turns each ring by a seeded random angle of up to `jitter`
    (radians, random axis) and moves it by up to jitter / 2 along each
    coordinate, breaking the lattice's symmetry (keep it well below the
    smallest gap, about 0.3 at slack 0.45).  Overdamped drag xi; the
    extensile field is `extensile_field`."""
    half = 2.0 * (R - r) - slack
    if not (half > R + 2.0 * r and half < 2.0 * R - 2.0 * r):
        raise ValueError("slack outside the range that keeps the rings linked and apart")
    L = 2.0 * half
    x, q = [], []
    for j in range(ny):
        for i in range(nx):
            x.append((i * L, j * L, 0.0))
            q.append(RING_FLAT)
    for j in range(ny):
        for i in range(nx - 1):
            x.append(((i + 0.5) * L, j * L, 0.0))
            q.append(RING_AXIS_Y)
    for j in range(ny - 1):
        for i in range(nx):
            x.append((i * L, (j + 0.5) * L, 0.0))
            q.append(RING_AXIS_X)
    x = np.array(x, float)
    x -= np.array([(nx - 1) * L / 2, (ny - 1) * L / 2, 0.0])
    n = x.shape[0]
    if jitter > 0:
        rng = rng_for(seed)
        ax = rng.normal(size=(n, 3))
        ax /= np.linalg.norm(ax, axis=1, keepdims=True)
        ang = jitter * rng.random(n)
        q = [_qmul(np.concatenate([[math.cos(a / 2)], math.sin(a / 2) * e]), qi) for a, e, qi in zip(ang, ax, q)]
        x = x + 0.5 * jitter * rng.uniform(-1, 1, (n, 3))
    return dict(x=x, q=np.array(q, float), kind=np.full(n, TORUS, np.int32), shape=np.tile([R, r, 0.0], (n, 1)),
                rho_xi=np.full(n, xi), box=np.zeros(3), n_nodes=nx * ny, spacing=L)


def extensile_field(x: np.ndarray) -> np.ndarray:
    """External wrench of the chainmail (Sec. 6): the force
    F(x) = x (|x| - sin|x|) / |x|^2 at each ring's centre, no torque; the
    series |x|^3 / 6 - |x|^5 / 120 replaces |x| - sin|x| below |x| = 1e-3."""
    x = np.asarray(x, float).reshape(-1, 3)
    s = np.linalg.norm(x, axis=1)
    small = s < 1e-3
    num = np.where(small, s ** 3 / 6.0 - s ** 5 / 120.0, s - np.sin(s))
    with np.errstate(divide="ignore", invalid="ignore"):
        scale = np.where(s > 0, num / np.where(s > 0, s * s, 1.0), 0.0)
    f = np.zeros((x.shape[0], 6))
    f[:, :3] = x * scale[:, None]
    return f


def two_ellipsoids(seed: int = 0, separation: float = 3.0, closing_speed: float = 1.0, spin_sd: float = 0.05,
                   semiaxes=(1.0, 0.5, 0.5), density: float = 1.0):
    """Two ellipsoids approaching head-on along x with random orientations
    and small random spins (inertial two-body collision)."""
    rng = rng_for(seed)
    q = shoemake_quaternions(rng, 2)
    x = np.array([[-separation / 2, 0.0, 0.0], [separation / 2, 0.0, 0.0]])
    u = np.zeros((2, 6))
    u[0, 0], u[1, 0] = 0.5 * closing_speed, -0.5 * closing_speed
    u[:, 3:] = rng.normal(0.0, spin_sd, size=(2, 3))
    shape = np.array([semiaxes, semiaxes], dtype=np.float64)
    return dict(x=x, q=q, u=u, kind=np.zeros(2, np.int32), shape=shape, rho_xi=np.full(2, density),
                box=np.zeros(3))


_RSA_SRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "inputs_rsa.c")
_RSA_LIB = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_librsa.so")
_rsa = None


def glancing_ellipsoids(t0: float = 98.0, xi: float = 1.0) -> dict:
    """The two-ellipsoid sliding collision of Sec. 5.1: identical ellipsoids
    with semiaxes (1, 1, 2) lying in the x-y plane (long axis turned onto x,
    then 45 degrees about z), centres 1 apart along x, driven by unit forces
    along y towards each other (the upper body down, the lower up), linear
    drag xi with L = 4, open boundaries.  The paper leaves xi and the vertical
    offset out and puts first contact near t = 100.  The bodies touch at a
    centre separation of 3 along y (the boundary of the Minkowski sum of two
    parallel copies) and close at 2 / (4 xi), so the offset that puts first
    contact at t = 100 is 3 + 50 xi; free motion under a constant force is
    exact at any timestep, so the bodies start at time t0 as far apart as
    that offset leaves them then."""
    half = np.pi / 4
    qy = np.array([np.cos(half), 0.0, np.sin(half), 0.0])      # body z onto world x
    qz = np.array([np.cos(half / 2), 0.0, 0.0, np.sin(half / 2)])  # 45 degrees about z
    s1, v1, s2, v2 = qz[0], qz[1:], qy[0], qy[1:]
    q = np.concatenate([[s1 * s2 - v1 @ v2], s1 * v2 + s2 * v1 + np.cross(v1, v2)])
    q /= np.linalg.norm(q)
    sep = 3.0 + (100.0 - t0) * 2.0 / (4.0 * xi)
    x = np.array([[-0.5, -0.5 * sep, 0.0], [0.5, 0.5 * sep, 0.0]])
    fext = np.zeros((2, 6))
    fext[0, 1], fext[1, 1] = 1.0, -1.0
    return dict(x=x, q=np.stack([q, q]), kind=np.zeros(2, np.int32), shape=np.array([[1.0, 1.0, 2.0]] * 2),
                rho_xi=np.full(2, xi), box=np.zeros(3), fext=fext, t0=t0)


def build_rsa(force: bool = False) -> str:
    """Compile the placement helper (plain C, gcc)."""
    if force or not os.path.exists(_RSA_LIB) or os.path.getmtime(_RSA_LIB) < os.path.getmtime(_RSA_SRC):
        tmp = _RSA_LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-o", tmp, _RSA_SRC, "-lm"])
        os.replace(tmp, _RSA_LIB)
    return _RSA_LIB


def _rsa_lib():
    global _rsa
    if _rsa is None:
        build_rsa()
        _rsa = ctypes.CDLL(_RSA_LIB)
        _rsa.rsa_spheres.restype = ctypes.c_int
        _rsa.rsa_spheres.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                     ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p]
    return _rsa


def rsa_spheres(rng: np.random.Generator, radii: np.ndarray, box: np.ndarray, max_attempts: int = 20000,
                planar: bool = False) -> np.ndarray:
    """Random sequential addition of non-overlapping spheres (largest first)
    in a periodic box (z fixed at 0 when planar).  Raises if a sphere cannot
    be placed within max_attempts."""
    radii = np.ascontiguousarray(radii, dtype=np.float64)
    n = radii.size
    order = np.ascontiguousarray(np.argsort(-radii, kind="stable"), dtype=np.int32)
    box = np.ascontiguousarray(box, dtype=np.float64)
    pos = np.zeros((n, 3))
    seed = int(rng.integers(0, 1 << 62))
    got = _rsa_lib().rsa_spheres(n, radii.ctypes.data, order.ctypes.data, box.ctypes.data, 1 if planar else 0, seed,
                                 max_attempts, pos.ctypes.data)
    if got != n:
        raise RuntimeError("random sequential addition jammed; lower the density")
    return pos


def ellipsoid_packing(seed: int, n: int, phi: float | None = None, sphere_phi: float = 0.25,
                      semiaxis_lo: float = 0.5, semiaxis_hi: float = 1.0, xi: float = 1.0, compress: float = 1.0):
    """Periodic packing of n ellipsoids (semiaxes i.i.d. uniform) at volume
    fraction phi.  Bounding spheres are placed by random sequential addition
    at sphere volume fraction `sphere_phi`; the box and positions are then
    rescaled affinely to reach phi.  When phi is above the fraction of that
    sphere packing, the rescale creates overlaps (as an isotropic
    compression step does), which the time-step resolves.  With phi=None
    the rescale factor is `compress` instead."""
    rng = rng_for(seed)
    shape = rng.uniform(semiaxis_lo, semiaxis_hi, size=(n, 3))
    q = shoemake_quaternions(rng, n)
    R = shape.max(axis=1)
    vs = float(np.sum(4.0 / 3.0 * np.pi * R ** 3))
    L0 = (vs / sphere_phi) ** (1.0 / 3.0)
    box0 = np.full(3, L0)
    x = rsa_spheres(rng, R, box0)
    ve = float(np.sum(ellipsoid_volume(shape)))
    L = (ve / phi) ** (1.0 / 3.0) if phi is not None else L0 * compress
    s = L / L0
    return dict(x=x * s, q=q, kind=np.zeros(n, np.int32), shape=shape, rho_xi=np.full(n, xi), box=np.full(3, L),
                scale=s, phi=ve / L ** 3)


def spherocylinder_monolayer(seed: int, n: int, area_fraction: float | None = None, length_lo: float = 1.0,
                             length_hi: float = 2.0, radius: float = 0.5, disk_fraction: float = 0.3,
                             xi: float = 1.0, compress: float = 1.0):
    """Planar periodic layer of spherocylinders (radius 0.5, cylinder length
    uniform in [length_lo, length_hi], random in-plane orientations): bounding
    disks by random sequential addition at area fraction `disk_fraction`,
    then an affine rescale of the box to the requested capsule area
    fraction (overlaps appear when it exceeds the disk packing's), or by the
    factor `compress` when area_fraction is None."""
    rng = rng_for(seed)
    ell = rng.uniform(length_lo, length_hi, size=n)
    shape = np.stack([np.full(n, radius), ell, np.zeros(n)], axis=1)
    theta = rng.uniform(0.0, 2 * np.pi, size=n)
    q = planar_quaternions(theta)
    R = 0.5 * ell + radius
    a_disk = float(np.sum(np.pi * R ** 2))
    L0 = math.sqrt(a_disk / disk_fraction)
    box0 = np.array([L0, L0, 0.0])
    x = rsa_spheres(rng, R, box0, planar=True)
    a_caps = float(np.sum(np.pi * radius ** 2 + 2 * radius * ell))
    L = math.sqrt(a_caps / area_fraction) if area_fraction is not None else L0 * compress
    s = L / L0
    return dict(x=x * s, q=q, kind=np.full(n, SPHEROCYLINDER, np.int32), shape=shape, rho_xi=np.full(n, xi),
                box=np.array([L, L, 0.0]), scale=s, area_fraction=a_caps / L ** 2)


def batch_of_packings(seed: int, count: int, n_lo: int, n_hi: int, phi_lo: float, phi_hi: float,
                      sphere_phi: float = 0.25, rescale: bool = True):
    """`count` independent periodic ellipsoid packings with body counts
    log-uniform in [n_lo, n_hi] and volume fractions uniform in
    [phi_lo, phi_hi], concatenated with batch offsets.  With rescale=False
    every packing keeps the fraction of its sphere placement and the drawn
    fractions are only returned (as targets for a compression run)."""
    rng = rng_for(seed)
    ns = np.exp(rng.uniform(np.log(n_lo), np.log(n_hi), size=count)).astype(int)
    phis = rng.uniform(phi_lo, phi_hi, size=count)
    parts = [ellipsoid_packing(int(rng.integers(1 << 30)), int(k), float(p) if rescale else None,
                               sphere_phi=sphere_phi) for k, p in zip(ns, phis)]
    off = np.zeros(count + 1, np.int32)
    off[1:] = np.cumsum(ns)
    return dict(x=np.concatenate([p["x"] for p in parts]), q=np.concatenate([p["q"] for p in parts]),
                kind=np.concatenate([p["kind"] for p in parts]), shape=np.concatenate([p["shape"] for p in parts]),
                rho_xi=np.concatenate([p["rho_xi"] for p in parts]), box=np.stack([p["box"] for p in parts]),
                batch_off=off, phi=np.array([p["phi"] for p in parts]), phi_target=phis)


def lattice_lcp(seed: int, m_target: int, bonds_per_body: float = 1.3) -> dict:
    """A contact-shaped LCP of about m_target rows for timing the LCP loop
    alone at many sizes: bodies on a cubic lattice (index x-fastest, so
    lattice neighbours are 1, s and s^2 apart), each +x, +y, +z bond present
    with the probability that gives bonds_per_body rows per body (1.3 is the
    compaction at volume fraction 0.40), rows sorted by (a, b) as the step
    generates them; unit normals and lever arms of scale 0.5, K with
    k_t in [0.5, 1] and diagonal K_r in [0.5, 1], qv ~ N(0, 0.01).  Returns
    n, ia, ib, n (m x 3), ta, tb (m x 3), kt (n), Kr6 (6 x n: xx yy zz xy xz
    yz), qv (m) and E = sum over rows of the other rows at their two bodies
    (the stored off-diagonal entries of A over rows)."""
    rng = rng_for(seed)
    n = int(m_target / bonds_per_body)
    s = max(2, int(round(n ** (1.0 / 3.0))))
    n = s ** 3
    idx = np.arange(n)
    x, y, z = idx % s, (idx // s) % s, idx // (s * s)
    p = bonds_per_body / 3.0
    A, B = [], []
    for d, ok in ((1, x < s - 1), (s, y < s - 1), (s * s, z < s - 1)):
        pick = ok & (rng.random(n) < p)
        A.append(idx[pick])
        B.append(idx[pick] + d)
    ia = np.concatenate(A)
    ib = np.concatenate(B)
    o = np.lexsort((ib, ia))
    ia, ib = ia[o].astype(np.int32), ib[o].astype(np.int32)
    m = ia.size
    nrm = rng.normal(size=(m, 3))
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    ta = np.cross(rng.normal(size=(m, 3)) * 0.5, nrm)
    tb = np.cross(rng.normal(size=(m, 3)) * 0.5, nrm)
    kt = rng.uniform(0.5, 1.0, n)
    Kr6 = np.concatenate([rng.uniform(0.5, 1.0, (3, n)), np.zeros((3, n))], 0)
    qv = rng.normal(size=m) * 0.01
    deg = np.bincount(ia, minlength=n) + np.bincount(ib, minlength=n)
    E = int((deg[ia] + deg[ib] - 2).sum())
    return dict(n=n, ia=ia, ib=ib, nrm=nrm, ta=ta, tb=tb, kt=kt, Kr6=Kr6, qv=qv, E=E)
