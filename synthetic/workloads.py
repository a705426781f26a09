"""Seeded generators for the rigid-body immersed-boundary workloads.

Every workload is a periodic box of side L = n*h with rigid bodies described by
surface markers spaced about 2h apart (the marker-spacing rule of Sec. 6 and the
conclusions).  Spheres use a Fibonacci (golden-angle) placement, disks use equally
spaced points on a circle.  Centres are rejection-sampled so that body surfaces
stay at least ``gap`` apart under the periodic minimum image, over the whole
prescribed trajectory when bodies move.

Nothing here evaluates the method: marker velocities, kernels and solves are
computed independently by each consumer.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np


@dataclass
class Problem:
    """One constrained-Stokes workload.

    dim        2 or 3
    n          cells per direction (the box is n^dim cells, periodic)
    h          grid spacing; the box side is L = n*h
    rho, eta   density and viscosity; rho == 0 means steady Stokes
    dt         time step (ignored when steady)
    R          [N][dim] marker positions in [0, L)^dim, grouped by body
    offsets    [nb+1] start of each body's markers in R
    centres    [nb][dim] body reference points (sphere / disk centres)
    U          [nb][dim] prescribed linear velocities
    Omega      [nb][1 or 3] prescribed angular velocities (1 component in 2D)
    radius     [nb] geometric radii (for reporting only)
    nsteps     number of time steps the trajectory was checked for
    walls      0: periodic box; 1: no-slip walls at both ends of the last axis
               (z in 3D, y in 2D), periodic along the others; 2: no-slip
               walls on every side
    """

    dim: int
    n: int
    h: float
    rho: float
    eta: float
    dt: float
    R: np.ndarray
    offsets: np.ndarray
    centres: np.ndarray
    U: np.ndarray
    Omega: np.ndarray
    radius: np.ndarray
    nsteps: int = 0
    name: str = ""
    meta: dict = field(default_factory=dict)
    walls: int = 0     # 1: walls at both ends of the last axis (slit channel); 2: every side

    @property
    def L(self) -> float:
        return self.n * self.h

    @property
    def nbodies(self) -> int:
        return len(self.offsets) - 1

    @property
    def nmarkers(self) -> int:
        return int(self.offsets[-1])

    @property
    def steady(self) -> bool:
        return self.rho == 0.0


def fibonacci_sphere(nmark: int, radius: float, centre) -> np.ndarray:
    """Golden-angle points on a sphere: z_i = 1-(2i+1)/N, azimuth i*pi*(3-sqrt 5)."""
    i = np.arange(nmark, dtype=np.float64)
    z = 1.0 - (2.0 * i + 1.0) / nmark
    rxy = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = i * math.pi * (3.0 - math.sqrt(5.0))
    pts = np.stack([rxy * np.cos(phi), rxy * np.sin(phi), z], axis=1) * radius
    return pts + np.asarray(centre, dtype=np.float64)[None, :]


def icosphere_unit(level: int) -> np.ndarray:
    """Vertices of the icosahedron with every face split ``level`` times into
    four (edge midpoints pushed to the unit sphere): 10 * 4^level + 2 points
    (12, 42, 162, 642, 2562, ...)."""
    t = (1.0 + math.sqrt(5.0)) / 2.0
    verts = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0), (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
             (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    verts = [np.asarray(v, dtype=np.float64) / np.linalg.norm(v) for v in verts]
    faces = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4), (11, 10, 2),
             (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9), (4, 9, 5),
             (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    for _ in range(level):
        cache = {}

        def mid(a, b):
            key = (min(a, b), max(a, b))
            if key not in cache:
                m = verts[a] + verts[b]
                verts.append(m / np.linalg.norm(m))
                cache[key] = len(verts) - 1
            return cache[key]

        nf = []
        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = nf
    return np.asarray(verts)


def icosphere_spacing(level: int) -> float:
    """Mean nearest-neighbour distance of the unit icosphere of this level."""
    v = icosphere_unit(level)
    d = np.sqrt(((v[:, None, :] - v[None, :, :]) ** 2).sum(axis=2))
    np.fill_diagonal(d, np.inf)
    return float(d.min(axis=1).mean())


def disk_ring(nmark: int, radius: float, centre, phase: float = 0.0) -> np.ndarray:
    """nmark equally spaced points on a circle, starting at angle ``phase``."""
    t = phase + 2.0 * math.pi * np.arange(nmark, dtype=np.float64) / nmark
    pts = np.stack([np.cos(t), np.sin(t)], axis=1) * radius
    return pts + np.asarray(centre, dtype=np.float64)[None, :]


def _min_image(d: np.ndarray, L: float) -> np.ndarray:
    return d - L * np.round(d / L)


def sample_centres(rng: np.random.Generator, radii, L: float, dim: int, gap: float,
                   U: Optional[np.ndarray] = None, dt: float = 0.0, nsteps: int = 0,
                   max_tries: int = 200000) -> np.ndarray:
    """Rejection-sample body centres in [0, L)^dim.

    Surfaces of every pair stay at least ``gap`` apart (periodic minimum image),
    at every time level 0..nsteps of the straight trajectories c + t*dt*U.
    """
    radii = np.asarray(radii, dtype=np.float64)
    nb = len(radii)
    if U is None:
        U = np.zeros((nb, dim))
    steps = np.arange(nsteps + 1, dtype=np.float64) * dt
    centres = np.zeros((nb, dim))
    placed = 0
    tries = 0
    while placed < nb:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("could not place %d bodies with gap %g" % (nb, gap))
        c = rng.uniform(0.0, L, size=dim)
        ok = True
        for q in range(placed):
            # relative position over the whole trajectory
            rel = (c - centres[q])[None, :] + steps[:, None] * (U[placed] - U[q])[None, :]
            dist = np.sqrt((_min_image(rel, L) ** 2).sum(axis=1)).min()
            if dist < radii[placed] + radii[q] + gap:
                ok = False
                break
        if ok:
            centres[placed] = c
            placed += 1
    return centres


def _wrap(R: np.ndarray, L: float) -> np.ndarray:
    R = np.mod(R, L)
    R[R >= L] -= L  # guard against mod returning L for tiny negatives
    return R


def _assemble(dim, n, h, rho, eta, dt, bodies, centres, U, Omega, radii, nsteps, name, meta=None):
    offsets = np.zeros(len(bodies) + 1, dtype=np.int64)
    for p, b in enumerate(bodies):
        offsets[p + 1] = offsets[p] + len(b)
    R = _wrap(np.concatenate(bodies, axis=0), n * h)
    return Problem(dim=dim, n=n, h=h, rho=rho, eta=eta, dt=dt, R=R, offsets=offsets,
                   centres=np.asarray(centres, dtype=np.float64) % (n * h),
                   U=np.asarray(U, dtype=np.float64), Omega=np.asarray(Omega, dtype=np.float64),
                   radius=np.asarray(radii, dtype=np.float64), nsteps=nsteps, name=name,
                   meta=meta or {})


def sphere_markers_for(radius_h: float) -> int:
    """Marker count for a sphere of radius R (in units of h) at about 2h spacing: round(pi R^2)."""
    return int(round(math.pi * radius_h * radius_h))


def disk_markers_for(radius_h: float) -> int:
    """Marker count for a circle of radius R (in units of h) at about 2h spacing: round(pi R)."""
    return int(round(math.pi * radius_h))


def config0_disk2d(seed: int = 0, n: int = 64, radius_h: float = 8.0) -> Problem:
    """2D steady Stokes, periodic unit square, one disk of radius 8h, ~25 markers, U = (1, 0)."""
    rng = np.random.default_rng(seed)
    h = 1.0 / n
    c = rng.uniform(0.0, 1.0, size=2)
    phase = rng.uniform(0.0, 2.0 * math.pi)
    nm = disk_markers_for(radius_h)
    R = disk_ring(nm, radius_h * h, c, phase)
    return _assemble(2, n, h, 0.0, 1.0, 0.0, [R], [c], [[1.0, 0.0]], [[0.0]],
                     [radius_h * h], 0, "disk2d_%d" % n)


def config1_sphere3d(seed: int = 0, n: int = 64, radius_h: float = 8.0, nmark: int = 200) -> Problem:
    """3D steady Stokes, periodic unit cube, one sphere of radius 8h with 200 markers."""
    rng = np.random.default_rng(seed)
    h = 1.0 / n
    c = rng.uniform(0.0, 1.0, size=3)
    U = rng.uniform(-1.0, 1.0, size=3)
    W = rng.uniform(-1.0, 1.0, size=3)
    R = fibonacci_sphere(nmark, radius_h * h, c)
    return _assemble(3, n, h, 0.0, 1.0, 0.0, [R], [c], [U], [W], [radius_h * h], 0,
                     "sphere3d_%d" % n)


def config2_spheres_ns(seed: int = 0, re: float = 10.0, n: int = 128, nbodies: int = 16,
                       radius_h: float = 6.0, nmark: int = 110, nsteps: int = 20) -> Problem:
    """3D unsteady Navier-Stokes, periodic unit cube, moving spheres.

    Re = rho*V*R/eta with R = radius, V = 1, rho = 1, so eta = R/Re; dt = 0.5h/V.
    Velocities U_p ~ U[-1,1]^3, no rotation; centres keep a 4h surface gap over
    all ``nsteps`` steps.
    """
    rng = np.random.default_rng(seed)
    h = 1.0 / n
    rad = radius_h * h
    dt = 0.5 * h
    eta = rad / re
    U = rng.uniform(-1.0, 1.0, size=(nbodies, 3))
    centres = sample_centres(rng, [rad] * nbodies, 1.0, 3, 4.0 * h, U=U, dt=dt, nsteps=nsteps)
    bodies = [fibonacci_sphere(nmark, rad, c) for c in centres]
    return _assemble(3, n, h, 1.0, eta, dt, bodies, centres, U, np.zeros((nbodies, 3)),
                     [rad] * nbodies, nsteps, "spheres_ns_%d_re%g" % (n, re), {"re": re})


def config4_spheres256(seed: int = 0, n: int = 256, nbodies: int = 100, radius_h: float = 8.0,
                       nmark: int = 200) -> Problem:
    """3D steady Stokes, periodic unit cube 256^3, 100 spheres of radius 8h, 200 markers each."""
    rng = np.random.default_rng(seed)
    h = 1.0 / n
    rad = radius_h * h
    centres = sample_centres(rng, [rad] * nbodies, 1.0, 3, 4.0 * h)
    U = rng.uniform(-1.0, 1.0, size=(nbodies, 3))
    W = rng.uniform(-1.0, 1.0, size=(nbodies, 3))
    bodies = [fibonacci_sphere(nmark, rad, c) for c in centres]
    return _assemble(3, n, h, 0.0, 1.0, 0.0, bodies, centres, U, W, [rad] * nbodies, 0,
                     "spheres_%d" % n)


def sedimentation_problem(seed: int = 0, n: int = 128, nbodies: int = 16, radius_h: float = 6.0,
                          nmark: int = 110, weight: float = 1.0):
    """3D steady Stokes, periodic unit cube, spheres of radius 6h (110
    Fibonacci markers each) at seeded non-overlapping positions, all free and
    pulled by the same weight along -z with zero torque (a sedimenting
    suspension).  Returns (problem, F [nb, 3], T [nb, 3]); the problem's
    prescribed velocities are zero (unused for free bodies)."""
    rng = np.random.default_rng(seed)
    h = 1.0 / n
    rad = radius_h * h
    centres = sample_centres(rng, [rad] * nbodies, 1.0, 3, 4.0 * h)
    bodies = [fibonacci_sphere(nmark, rad, c) for c in centres]
    prob = _assemble(3, n, h, 0.0, 1.0, 0.0, bodies, centres, np.zeros((nbodies, 3)), np.zeros((nbodies, 3)),
                     [rad] * nbodies, 0, "sediment_%d" % n)
    F = np.zeros((nbodies, 3))
    F[:, 2] = -weight
    return prob, F, np.zeros((nbodies, 3))


def concentric_shells(n: int = 64, level: int = 1, V: float = 1.0, box_over_outer: float = 4.15,
                      walls: bool = False) -> Problem:
    """Two concentric icosahedral shells in a periodic unit cube, 3D steady
    Stokes, eta = 1 (the setting of the paper's concentric-shells study):
    outer radius R2 = 1 / box_over_outer, inner radius R1 = R2 / 4; inner shell
    of 10 * 4^level + 2 markers (body 0) translating with -V along x, outer
    shell two refinement levels finer (about 16 times the markers, similar
    spacing) at rest (body 1), both centred in the box.  This is the paper's
    configuration (cavity moving with V around a sphere at rest) seen from the
    cavity, so that the fluid outside the outer shell stays nearly at rest in
    the periodic box, as the paper's boundary conditions make it.  Levels 0, 1,
    2 give 12/162, 42/642 and 162/2562 markers, spaced about 2h at n = 32, 64,
    128.  walls: the closed box of the paper's study instead (no-slip walls on
    every side; its walls move with the cavity, so they rest in the cavity's
    frame)."""
    h = 1.0 / n
    R2 = 1.0 / box_over_outer
    R1 = R2 / 4.0
    c = np.array([0.5, 0.5, 0.5])
    bodies = [icosphere_unit(level) * R1 + c, icosphere_unit(level + 2) * R2 + c]
    U = np.array([[-V, 0.0, 0.0], [0.0, 0.0, 0.0]])
    prob = _assemble(3, n, h, 0.0, 1.0, 0.0, bodies, np.stack([c, c]), U, np.zeros((2, 3)), [R1, R2], 0,
                     "shells_%d_l%d%s" % (n, level, "_box" if walls else ""))
    prob.walls = 2 if walls else 0
    return prob


def single_shell(n: int = 64, level: int = 1, V: float = 1.0, box_over_outer: float = 4.15) -> Problem:
    """The inner shell of ``concentric_shells`` alone in the periodic unit cube,
    translating with V along x (its drag gives its hydrodynamic radius)."""
    R1 = 1.0 / box_over_outer / 4.0
    c = np.array([0.5, 0.5, 0.5])
    return _assemble(3, n, 1.0 / n, 0.0, 1.0, 0.0, [icosphere_unit(level) * R1 + c], c[None, :].copy(),
                     np.array([[V, 0.0, 0.0]]), np.zeros((1, 3)), [R1], 0, "shell_alone_%d_l%d" % (n, level))


def small_problem(seed: int, dim: int, n: int, nbodies: int = 1, radius_h: float = 3.0,
                  rho: float = 0.0, eta: float = 1.0, dt: float = 0.0, gap_h: float = 4.0,
                  rotate: bool = True, nsteps: int = 0, L: float = 1.0) -> Problem:
    """Small seeded problem for parity tests (oracle finishes in seconds)."""
    rng = np.random.default_rng(seed)
    h = L / n
    rad = radius_h * h
    U = rng.uniform(-1.0, 1.0, size=(nbodies, dim))
    centres = sample_centres(rng, [rad] * nbodies, L, dim, gap_h * h, U=U if nsteps else None,
                             dt=dt, nsteps=nsteps)
    if dim == 3:
        Om = rng.uniform(-1.0, 1.0, size=(nbodies, 3)) if rotate else np.zeros((nbodies, 3))
        nm = sphere_markers_for(radius_h)
        bodies = [fibonacci_sphere(nm, rad, c) for c in centres]
    else:
        Om = rng.uniform(-1.0, 1.0, size=(nbodies, 1)) if rotate else np.zeros((nbodies, 1))
        nm = disk_markers_for(radius_h)
        bodies = [disk_ring(nm, rad, c, rng.uniform(0, 2 * math.pi)) for c in centres]
    return _assemble(dim, n, h, rho, eta, dt, bodies, centres, U, Om, [rad] * nbodies, nsteps,
                     "small_%dd_%d" % (dim, n))


def shell_problem(seed: int = 0, n: int = 32, level: int = 2, filled: bool = False, re: float = 0.0,
                  spacing_h: float = 2.0, walls: bool = False) -> Problem:
    """One sphere in a periodic unit cube: an icosahedral shell of
    10 * 4^level + 2 markers (162 at level 2) with mean marker spacing
    ``spacing_h`` h, optionally filled with concentric shells of the same
    spacing (interior shells are golden-angle point sets of round(N (r/R)^2)
    markers at radii R - 2h, R - 4h, ... and a centre marker when the last
    radius is below 2h).  Centre ~ U[0,1)^3, U ~ U[-1,1]^3.  re = 0: steady
    Stokes, eta = 1, Omega ~ U[-1,1]^3; re > 0: one backward-Euler step of
    the unsteady system, rho = 1, eta = R/re, dt = 0.5h, Omega = 0.
    walls: the slit channel (no-slip walls at z = 0 and z = 1); the centre's
    z is then drawn so that the shell keeps 2h from both walls."""
    rng = np.random.default_rng(seed)
    h = 1.0 / n
    R = spacing_h * h / icosphere_spacing(level)
    centre = rng.uniform(0.0, 1.0, size=3)
    if walls:
        centre[2] = R + 2 * h + centre[2] * (1.0 - 2 * (R + 2 * h))
    shell = icosphere_unit(level)
    pts = [shell * R + centre]
    if filled:
        r = R - spacing_h * h
        while r > 0.5 * spacing_h * h:
            pts.append(fibonacci_sphere(max(1, int(round(len(shell) * (r / R) ** 2))), r, centre))
            r -= spacing_h * h
        pts.append(centre[None, :].copy())
    body = np.concatenate(pts, axis=0)
    U = rng.uniform(-1.0, 1.0, size=(1, 3))
    if re > 0:
        rho, eta, dt = 1.0, R / re, 0.5 * h
        Om = np.zeros((1, 3))
    else:
        rho, eta, dt = 0.0, 1.0, 0.0
        Om = rng.uniform(-1.0, 1.0, size=(1, 3))
    prob = _assemble(3, n, h, rho, eta, dt, [body], centre[None, :], U, Om, [R], 0,
                     "shell_l%d_%s_n%d_re%g%s" % (level, "filled" if filled else "empty", n, re,
                                                  "_walls" if walls else ""),
                     meta={"radius_h": R / h, "markers": len(body)})
    prob.walls = 1 if walls else 0
    return prob


SERVING_GRIDS = [(2, 32), (2, 128), (2, 256), (3, 32), (3, 64), (3, 128)]


def serving_trace(seed: int = 0, nreq: int = 2000, qps: float = 50.0) -> List[dict]:
    """Poisson arrivals of steady constrained solves with random sizes and bodies.

    Each request draws a grid from SERVING_GRIDS, 1-8 bodies of radius U[4h, 8h]
    (fewer if they do not fit with a 4h gap), markers at ~2h and U, Omega ~ U[-1,1].
    Returns a list of {"t": arrival time in s, "problem": Problem}.
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for r in range(nreq):
        t += rng.exponential(1.0 / qps)
        dim, n = SERVING_GRIDS[rng.integers(len(SERVING_GRIDS))]
        nb = int(rng.integers(1, 9))
        h = 1.0 / n
        radii_h = rng.uniform(4.0, 8.0, size=nb)
        while True:
            try:
                centres = sample_centres(rng, radii_h[:nb] * h, 1.0, dim, 4.0 * h, max_tries=200)
                break
            except RuntimeError:
                nb -= 1
        bodies = []
        for p in range(nb):
            if dim == 3:
                bodies.append(fibonacci_sphere(sphere_markers_for(radii_h[p]), radii_h[p] * h,
                                               centres[p]))
            else:
                bodies.append(disk_ring(disk_markers_for(radii_h[p]), radii_h[p] * h, centres[p],
                                        rng.uniform(0, 2 * math.pi)))
        U = rng.uniform(-1.0, 1.0, size=(nb, dim))
        Om = rng.uniform(-1.0, 1.0, size=(nb, 3 if dim == 3 else 1))
        prob = _assemble(dim, n, h, 0.0, 1.0, 0.0, bodies, centres, U, Om, radii_h[:nb] * h, 0,
                         "serve_%d_%dd_%d" % (r, dim, n))
        out.append({"t": t, "problem": prob})
    return out


def slit_problem(seed: int = 0, dim: int = 3, n: int = 32, nbodies: int = 2, radius_h: float = 3.0,
                 eta: float = 1.0, gap_h: float = 4.0, wall_gap_h: float = 2.0, rotate: bool = True,
                 L: float = 1.0, rho: float = 0.0, dt: float = 0.0) -> Problem:
    """Stokes (rho = 0) or unsteady (rho, dt > 0) flow in a slit channel:
    no-slip walls at z = 0 and z = L (y in 2D), periodic along the other
    axes; bodies as in ``small_problem``, with centres drawn so that every
    surface keeps ``wall_gap_h`` cells from the walls."""
    rng = np.random.default_rng(seed)
    h = L / n
    rad = radius_h * h
    U = rng.uniform(-1.0, 1.0, size=(nbodies, dim))
    lo = rad + wall_gap_h * h
    centres = np.zeros((nbodies, dim))
    placed = 0
    tries = 0
    while placed < nbodies:
        tries += 1
        if tries > 200000:
            raise RuntimeError("could not place %d bodies in the slit" % nbodies)
        c = rng.uniform(0.0, L, size=dim)
        c[-1] = rng.uniform(lo, L - lo)
        if all(np.sqrt((_min_image(c - centres[q], L) ** 2).sum()) >= 2 * rad + gap_h * h for q in range(placed)):
            centres[placed] = c
            placed += 1
    if dim == 3:
        Om = rng.uniform(-1.0, 1.0, size=(nbodies, 3)) if rotate else np.zeros((nbodies, 3))
        bodies = [fibonacci_sphere(sphere_markers_for(radius_h), rad, c) for c in centres]
    else:
        Om = rng.uniform(-1.0, 1.0, size=(nbodies, 1)) if rotate else np.zeros((nbodies, 1))
        bodies = [disk_ring(disk_markers_for(radius_h), rad, c, rng.uniform(0, 2 * math.pi)) for c in centres]
    prob = _assemble(dim, n, h, rho, eta, dt, bodies, centres, U, Om, [rad] * nbodies, 0,
                     "slit_%dd_%d" % (dim, n))
    prob.walls = 1
    return prob


def box_problem(seed: int = 0, dim: int = 3, n: int = 16, nbodies: int = 2, radius_h: float = 2.5,
                eta: float = 1.0, gap_h: float = 3.0, wall_gap_h: float = 1.0, rotate: bool = True,
                L: float = 1.0, rho: float = 0.0, dt: float = 0.0) -> Problem:
    """Stokes (rho = 0) or unsteady (rho, dt > 0) flow in a closed box: no-slip
    walls on every side; bodies as in ``small_problem``, every surface at
    least ``wall_gap_h`` cells from every wall and ``gap_h`` cells from the
    other bodies (plain distances: nothing wraps)."""
    rng = np.random.default_rng(seed)
    h = L / n
    rad = radius_h * h
    U = rng.uniform(-1.0, 1.0, size=(nbodies, dim))
    lo = rad + wall_gap_h * h
    centres = np.zeros((nbodies, dim))
    placed = 0
    tries = 0
    while placed < nbodies:
        tries += 1
        if tries > 200000:
            raise RuntimeError("could not place %d bodies in the box" % nbodies)
        c = rng.uniform(lo, L - lo, size=dim)
        if all(np.sqrt(((c - centres[q]) ** 2).sum()) >= 2 * rad + gap_h * h for q in range(placed)):
            centres[placed] = c
            placed += 1
    if dim == 3:
        Om = rng.uniform(-1.0, 1.0, size=(nbodies, 3)) if rotate else np.zeros((nbodies, 3))
        bodies = [fibonacci_sphere(sphere_markers_for(radius_h), rad, c) for c in centres]
    else:
        Om = rng.uniform(-1.0, 1.0, size=(nbodies, 1)) if rotate else np.zeros((nbodies, 1))
        bodies = [disk_ring(disk_markers_for(radius_h), rad, c, rng.uniform(0, 2 * math.pi)) for c in centres]
    prob = _assemble(dim, n, h, rho, eta, dt, bodies, centres, U, Om, [rad] * nbodies, 0,
                     "box_%dd_%d" % (dim, n))
    prob.walls = 2
    return prob


def box_shell(n: int = 32, level: int = 2, box_over_radius: float = 4.35, V: float = 1.0,
              filled: bool = False) -> Problem:
    """The non-periodic runs of Sec. 7.1: one sphere of markers (an
    icosahedral shell of 10 * 4^level + 2 markers, optionally filled with
    interior shells like ``shell_problem``) at the centre of a closed box of
    side about 4.35 sphere radii, no-slip walls on every side, translating
    with V along x through the stationary fluid; steady Stokes, eta = 1."""
    h = 1.0 / n
    radius = 1.0 / box_over_radius
    c = np.full(3, 0.5)
    shell = icosphere_unit(level)
    pts = [shell * radius + c]
    if filled:
        # interior shells as in shell_problem: the surface's mean spacing apart
        spacing = icosphere_spacing(level) * radius
        r = radius - spacing
        while r > 0.5 * spacing:
            pts.append(fibonacci_sphere(max(1, int(round(len(shell) * (r / radius) ** 2))), r, c))
            r -= spacing
        pts.append(c[None, :].copy())
    prob = _assemble(3, n, h, 0.0, 1.0, 0.0, [np.concatenate(pts)], c[None, :].copy(),
                     np.array([[V, 0.0, 0.0]]), np.zeros((1, 3)), [radius], 0,
                     "box_shell_%d_l%d%s" % (n, level, "_filled" if filled else ""))
    prob.walls = 2
    return prob


def slit_shell(n: int = 32, level: int = 0, height: float = 0.5, radius: float = 0.0625, V: float = 1.0) -> Problem:
    """One icosahedral shell (10 * 4^level + 2 markers) in the slit channel of
    the paper's slit study: unit cube, no-slip walls at z = 0 and z = 1,
    periodic along x and y, centre at height ``height`` (0.5: midplane, 0.25:
    quarter), translating with V along x, parallel to the walls; steady
    Stokes, eta = 1."""
    h = 1.0 / n
    c = np.array([0.5, 0.5, height])
    prob = _assemble(3, n, h, 0.0, 1.0, 0.0, [icosphere_unit(level) * radius + c], c[None, :].copy(),
                     np.array([[V, 0.0, 0.0]]), np.zeros((1, 3)), [radius], 0,
                     "slit_shell_%d_l%d_h%g" % (n, level, height))
    prob.walls = 1
    return prob


def array_shell(n: int = 16, level: int = 2, radius: float = 0.47, L: float = 1.0, V: float = 1.0) -> Problem:
    """One icosahedral shell (10 * 4^level + 2 markers) of the given radius at
    the centre of a periodic cube of side L, translating with V along x:
    with its periodic images, a simple-cubic array of spheres (the dense
    arrays of Sec. 7); steady Stokes, eta = 1."""
    h = L / n
    c = np.full(3, 0.5 * L)
    return _assemble(3, n, h, 0.0, 1.0, 0.0, [icosphere_unit(level) * radius + c], c[None, :].copy(),
                     np.array([[V, 0.0, 0.0]]), np.zeros((1, 3)), [radius], 0,
                     "array_shell_%d_l%d" % (n, level))
