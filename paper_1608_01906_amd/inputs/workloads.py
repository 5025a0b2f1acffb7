"""Seeded synthetic workloads: mesh, physical parameters and initial fields.

The paper's benchmarks (Section 3) use meshes and data that are not
published, so each workload here is a generated stand-in with the same
geometry class, parameter ranges and structure:

  droplet2d   periodic square, circular drop at rest (Section 3.1, in 2-D)
  channel2d   layered two-phase planar Poiseuille flow between walls
              (2-D analogue of the concurrent pipe flow of Section 3.3)
  rt2d        Rayleigh-Taylor: heavy over light between walls, cosine
              perturbation of the interface (2-D analogue of Section 3.4)
  droplet3d   periodic cube, spherical drop at rest (Section 3.1)
  ensemble2d  many independent periodic droplets of uneven size
  translate2d a drop carried through a periodic square by a uniform
              velocity (Section 3.2, droplet translation)
  pipe3d      concurrent two-phase flow in a circular pipe with a curved
              wall (Section 3.3); pipe_study3d the relative-permeability
              study over saturations and viscosity ratios

Initial fields are the caller's: density rho, velocity u and pressure p at
the nodes.  Phase labels follow the chemical-potential definition of
Section 2.1: rho_l is the heavy (liquid) phase and rho_v the light one.
The time step is 0.2 on unit-spaced meshes for every workload, with the
dimensionless relaxation time tau (lambda / dt) as stated: the
characteristic-Galerkin streaming is unstable at dt = 1 on these meshes, and
at 0.25 (the stability edge of the diagonal directions on +-0.2h jittered
meshes) the 1024 x 256 channel diverges within 250 steps even at density
ratio 2, while 0.2 runs it for its full length.

None of the method's arithmetic is here: the density profiles are the flat
tanh interface of width xi, and the channel velocity is the quadrature of
the steady Stokes equation for the given viscosity profile.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .mesh import box_mesh, grid_mesh_2d, grid_mesh_3d, pipe_mesh_3d, uniform01

DT_RUN = 0.2
CS2 = 1.0 / 3.0


@dataclass
class Phys:
    rho_l: float          # heavy / liquid bulk density
    rho_v: float          # light / vapour bulk density
    tau_l: float          # dimensionless relaxation time of the heavy phase
    tau_v: float          # ... of the light phase
    sigma: float          # surface tension
    xi: float             # interface width
    dt: float = DT_RUN
    grav: tuple = (0.0, 0.0, 0.0)

    def as_tuple(self):
        g = tuple(self.grav) + (0.0,) * (3 - len(self.grav))
        return (self.rho_l, self.rho_v, self.tau_l, self.tau_v, self.sigma, self.xi, self.dt) + g[:3]


@dataclass
class Instance:
    mesh: dict
    phys: Phys
    rho0: np.ndarray
    u0: np.ndarray
    p0: np.ndarray
    meta: dict = field(default_factory=dict)


@dataclass
class Workload:
    name: str
    lattice: int                  # 9 (D2Q9) or 19 (D3Q19)
    instances: list
    steps: int
    description: str = ""

    @property
    def n_nodes(self) -> int:
        return int(sum(i.mesh["xyz"].shape[0] for i in self.instances))


def _tanh_profile(signed_dist, rho_l, rho_v, xi):
    """Flat-interface density: heavy where signed_dist > 0."""
    return 0.5 * (rho_l + rho_v) + 0.5 * (rho_l - rho_v) * np.tanh(2.0 * signed_dist / xi)


def _min_image(d, L):
    if L > 0:
        d = d - L * np.round(d / L)
    return d


def droplet_instance(mesh, *, radius, rho_l, rho_v, sigma, xi, tau_l, tau_v, center=None,
                     dt=DT_RUN, u0=None) -> Instance:
    dim = mesh["dim"]
    box = mesh["box"]
    if center is None:
        center = box / 2.0
    d = np.stack([_min_image(mesh["xyz"][:, a] - center[a], box[a]) for a in range(dim)], axis=1)
    r = np.sqrt((d ** 2).sum(axis=1))
    rho = _tanh_profile(radius - r, rho_l, rho_v, xi)
    comp = (rho - rho_v) / (rho_l - rho_v)
    dp = (sigma / radius) * (dim - 1)          # Laplace jump: sigma/R in 2-D, 2 sigma/R in 3-D
    p = dp * comp
    u = np.zeros((mesh["xyz"].shape[0], dim))
    if u0 is not None:
        u[:] = np.asarray(u0, float)[:dim]
    phys = Phys(rho_l, rho_v, tau_l, tau_v, sigma, xi, dt)
    return Instance(mesh, phys, rho, u, p,
                    meta=dict(kind="droplet", radius=radius, center=np.asarray(center, float),
                              dp_laplace=dp))


def droplet2d(n=64, *, jitter=0.2, seed=1608, radius=None, rho_l=1.0, rho_v=0.1, sigma=0.01,
              xi=4.0, tau=0.05, steps=200) -> Workload:
    """Static drop in a periodic square (radius n/4 by default)."""
    mesh = grid_mesh_2d(n, n, jitter=jitter, seed=seed)
    inst = droplet_instance(mesh, radius=radius if radius is not None else n / 4.0,
                            rho_l=rho_l, rho_v=rho_v, sigma=sigma, xi=xi, tau_l=tau, tau_v=tau,
                            center=np.array([n / 2.0, n / 2.0]))
    return Workload(f"droplet2d_{n}x{n}", 9, [inst], steps,
                    "D2Q9 static droplet, periodic jittered P1 mesh")


def droplet3d(n=128, *, jitter=0.2, seed=1611, radius=None, rho_l=1.0, rho_v=0.01, sigma=0.005,
              xi=8.0, tau=0.05, steps=500) -> Workload:
    mesh = grid_mesh_3d(n, n, n, jitter=jitter, seed=seed)
    inst = droplet_instance(mesh, radius=radius if radius is not None else n / 4.0,
                            rho_l=rho_l, rho_v=rho_v, sigma=sigma, xi=xi, tau_l=tau, tau_v=tau,
                            center=np.full(3, n / 2.0))
    return Workload(f"droplet3d_{n}^3", 19, [inst], steps,
                    "D3Q19 static droplet, periodic jittered Kuhn-tet mesh")


def channel_profile(y, *, half_width, core, rho_heavy, rho_light, tau_heavy, tau_light, xi, g, dt,
                    sub=64):
    """Steady layered channel flow for a diffuse interface.

    y is measured from the channel centre; walls at |y| = half_width, light
    core |y| < core.  Solves d/dy(mu du/dy) = -rho g with u = 0 at the walls
    and du/dy = 0 at the centre: u(y) = int_|y|^L (int_0^s rho g) / mu(s) ds,
    with mu = rho cs^2 tau dt and 1/tau the composition-weighted harmonic
    mean of the bulk values.
    """
    L = half_width
    s = np.linspace(0.0, L, int(np.ceil(L * sub)) + 1)
    rho = _tanh_profile(np.abs(s) - core, rho_heavy, rho_light, xi)
    comp = np.clip((rho - rho_light) / (rho_heavy - rho_light), 0.0, 1.0)
    tau = 1.0 / (comp / tau_heavy + (1.0 - comp) / tau_light)
    mu = rho * CS2 * tau * dt
    ds = s[1] - s[0]
    inner = np.concatenate([[0.0], np.cumsum(0.5 * (rho[1:] + rho[:-1]) * g * ds)])
    integrand = inner / mu
    outer = np.concatenate([[0.0], np.cumsum(0.5 * (integrand[1:] + integrand[:-1]) * ds)])
    u_of_s = outer[-1] - outer                   # int_s^L
    return np.interp(np.abs(y), s, u_of_s)


def channel2d(nx=1024, ny=256, *, jitter=0.2, seed=1609, rho_heavy=1.0, rho_light=1e-3,
              tau_heavy=0.05, tau_light=1.0, sigma=0.01, xi=12.0, g=1e-7, steps=5000,
              dt=DT_RUN) -> Workload:
    """Layered Poiseuille flow: heavy fluid along both walls, light core.

    Walls are the node rows y = 0 and y = ny-1; flow along periodic x.
    """
    mesh = grid_mesh_2d(nx, ny, wall_y=True, jitter=jitter, seed=seed)
    yc = 0.5 * (ny - 1)
    L = 0.5 * (ny - 1)
    core = 0.25 * (ny - 1)
    y = mesh["xyz"][:, 1] - yc
    rho = _tanh_profile(np.abs(y) - core, rho_heavy, rho_light, xi)
    u = np.zeros((mesh["xyz"].shape[0], 2))
    u[:, 0] = channel_profile(y, half_width=L, core=core, rho_heavy=rho_heavy, rho_light=rho_light,
                              tau_heavy=tau_heavy, tau_light=tau_light, xi=xi, g=g, dt=dt)
    p = np.zeros(mesh["xyz"].shape[0])
    phys = Phys(rho_heavy, rho_light, tau_heavy, tau_light, sigma, xi, dt, (g, 0.0, 0.0))
    inst = Instance(mesh, phys, rho, u, p,
                    meta=dict(kind="channel", half_width=L, core=core, yc=yc, g=g))
    return Workload(f"channel2d_{nx}x{ny}", 9, [inst], steps,
                    "D2Q9 layered two-phase Poiseuille channel between bounce-back walls")


def rt2d(nx=1024, ny=4096, *, jitter=0.2, seed=1610, rho_heavy=1.0, rho_light=1.0 / 3.0,
         tau=0.05, xi=4.0, g=1e-5, amp=0.1, steps=2000) -> Workload:
    """Rayleigh-Taylor: heavy on top, light below, walls at y = 0 and y = ny-1."""
    mesh = grid_mesh_2d(nx, ny, wall_y=True, jitter=jitter, seed=seed)
    x, y = mesh["xyz"][:, 0], mesh["xyz"][:, 1]
    H = ny - 1.0
    yi = 0.5 * H + amp * nx * np.cos(2.0 * np.pi * x / nx)
    rho = _tanh_profile(y - yi, rho_heavy, rho_light, xi)
    # hydrostatic pressure of the unperturbed column, p(H) = 0: dp/dy = -rho g
    ys = np.linspace(0.0, H, int(H) * 8 + 1)
    rs = _tanh_profile(ys - 0.5 * H, rho_heavy, rho_light, xi)
    col = np.concatenate([[0.0], np.cumsum(0.5 * (rs[1:] + rs[:-1]) * (ys[1] - ys[0]))])
    p = g * np.interp(y, ys, col[-1] - col)
    u = np.zeros((x.size, 2))
    phys = Phys(rho_heavy, rho_light, tau, tau, 0.0, xi, DT_RUN, (0.0, -g, 0.0))
    inst = Instance(mesh, phys, rho, u, p, meta=dict(kind="rt", atwood=(rho_heavy - rho_light) /
                                                      (rho_heavy + rho_light)))
    return Workload(f"rt2d_{nx}x{ny}", 9, [inst], steps,
                    "D2Q9 Rayleigh-Taylor, heavy over light, walls top and bottom")


def ensemble2d(count=64, *, side_lo=32, side_hi=512, seed=16085, jitter=0.2, sigma=0.01, xi=None,
               tau=0.05, steps=1000, ratio_hi=1000.0, ratio_min=1.05) -> Workload:
    """Independent periodic droplets with sides ~ U{lo..hi}, density ratio log-uniform.

    Ratios below ratio_min are redrawn from the continuation of the stream
    (the free-energy coefficients scale with (rho_l - rho_v)^-4 and become
    stiff as the ratio tends to 1).
    """
    u = uniform01(seed, count)
    sides = side_lo + np.floor(u * (side_hi - side_lo + 1)).astype(int)
    ratios = []
    pos = count
    while len(ratios) < count:
        r = ratio_hi ** uniform01(seed, 1, pos)[0]
        pos += 1
        if r >= ratio_min:
            ratios.append(r)
    insts = []
    for i, (s, r) in enumerate(zip(sides, ratios)):
        mesh = grid_mesh_2d(int(s), int(s), jitter=jitter, seed=seed * 1000 + i)
        # sharper density ratios need wider interfaces to stay positive in the
        # light phase; never wider than half the radius
        w_i = xi if xi is not None else min(4.0 if r <= 10 else (8.0 if r <= 100 else 12.0), 0.125 * s)
        inst = droplet_instance(mesh, radius=0.25 * s, rho_l=1.0, rho_v=1.0 / r, sigma=sigma, xi=w_i,
                                tau_l=tau, tau_v=tau, center=np.array([s / 2.0, s / 2.0]))
        inst.meta.update(side=int(s), ratio=float(r), xi=w_i)
        insts.append(inst)
    return Workload(f"ensemble2d_{count}", 9, insts, steps,
                    "independent D2Q9 droplets of uneven size advanced together")


def translate2d(n=128, *, jitter=0.2, seed=1612, radius=None, rho_l=1.0, ratio=100.0, nu_ratio=1.0,
                sigma=0.01, xi=12.0, tau_l=0.05, u0=0.02, diagonal=False, trips=1, dt=DT_RUN) -> Workload:
    """Drop carried through a periodic square by a uniform velocity (the
    droplet translation test of Section 3.2, in 2-D): radius n/4, density
    contrast `ratio`, kinematic-viscosity contrast `nu_ratio` (light over
    heavy, so tau_v = nu_ratio * tau_l), speed u0 along x or along the
    diagonal.  The paper's contrasts (1000 and 60) drain the light-phase
    density next to the moving interface below zero within a few thousand
    steps on these meshes for every xi <= 12; the defaults (100, 1, xi = 12)
    are the largest that complete a round trip at u0 = 0.01 and 0.02.  One round trip takes n / u0 time units (n * sqrt(2) / u0 along
    the diagonal, where the drop crosses the box diagonally once per axis
    period); `steps` covers `trips` of them, after which the drop should be
    back where it started and still circular."""
    mesh = grid_mesh_2d(n, n, jitter=jitter, seed=seed)
    direction = np.array([1.0, 1.0]) / np.sqrt(2.0) if diagonal else np.array([1.0, 0.0])
    inst = droplet_instance(mesh, radius=radius if radius is not None else n / 4.0, rho_l=rho_l,
                            rho_v=rho_l / ratio, sigma=sigma, xi=xi, tau_l=tau_l, tau_v=tau_l * nu_ratio,
                            center=np.array([n / 2.0, n / 2.0]), dt=dt, u0=u0 * direction)
    period = n / u0 * (np.sqrt(2.0) if diagonal else 1.0)
    steps = int(round(trips * period / dt))
    inst.meta.update(kind="translation", u0=u0 * direction, period=period, trips=trips)
    return Workload(f"translate2d_{n}x{n}", 9, [inst], steps,
                    "D2Q9 drop translated by a uniform velocity through a periodic jittered P1 mesh")


def pipe_profile(r, *, radius, a, rho_w, rho_nw, tau_w, tau_nw, xi, g, dt, sub=64):
    """Steady axial velocity of concurrent pipe flow for a diffuse interface.

    The wetting phase (density rho_w) fills a < r <= radius, the
    non-wetting one (rho_nw) the core r < a, with the flat tanh profile of
    width xi across r = a.  The body force is the acceleration g along the
    axis, so the force per volume is rho g.  The axial Stokes equation
    (1/r) d/dr (r mu du/dr) = -rho g with u(radius) = 0 and u regular on the
    axis gives
        u(r) = int_r^radius (1 / (mu(s) s)) int_0^s rho(t) g t dt ds,
    with mu = rho cs^2 tau dt and 1/tau the composition-weighted harmonic
    mean of the bulk values.  For a sharp interface and equal densities it
    reduces to the two-parabola profile of Section 3.3.
    """
    s = np.linspace(0.0, radius, int(np.ceil(radius * sub)) + 1)
    rho = _tanh_profile(s - a, rho_w, rho_nw, xi)
    comp = np.clip((rho - rho_nw) / (rho_w - rho_nw), 0.0, 1.0)
    tau = 1.0 / (comp / tau_w + (1.0 - comp) / tau_nw)
    mu = rho * CS2 * tau * dt
    ds = s[1] - s[0]
    f = rho * g * s
    inner = np.concatenate([[0.0], np.cumsum(0.5 * (f[1:] + f[:-1]) * ds)])
    integrand = np.zeros_like(s)
    integrand[1:] = inner[1:] / (mu[1:] * s[1:])
    outer = np.concatenate([[0.0], np.cumsum(0.5 * (integrand[1:] + integrand[:-1]) * ds)])
    u_of_s = outer[-1] - outer                   # int_s^radius
    return np.interp(r, s, u_of_s)


def box_droplet(dims=(48, 48), *, mesh=None, radius=None, rho_l=1.0, rho_v=0.1, sigma=0.01, xi=4.0, tau=0.05,
                steps=200) -> Workload:
    """Static drop in the middle of a closed box with no-slip walls on every
    side: a generated box mesh of node shape `dims`, or any non-periodic
    mesh dictionary (for instance one read by inputs.mesh_files.read_gmsh).
    Radius a quarter of the smallest extent by default."""
    if mesh is None:
        mesh = box_mesh(dims)
    lo, hi = mesh["xyz"].min(axis=0), mesh["xyz"].max(axis=0)
    if radius is None:
        radius = 0.25 * float((hi - lo).min())
    inst = droplet_instance(mesh, radius=radius, rho_l=rho_l, rho_v=rho_v, sigma=sigma, xi=xi, tau_l=tau, tau_v=tau,
                            center=0.5 * (lo + hi))
    lattice = 9 if mesh["dim"] == 2 else 19
    return Workload(f"box_droplet_{mesh['xyz'].shape[0]}", lattice, [inst], steps,
                    "static drop in a closed box with bounce-back walls on every side")


PIPE_DT = 0.05


def pipe_instance(mesh, *, radius, s_w, visc_ratio, rho_w=1.0, rho_nw=0.95, tau_w=None, sigma=1e-4, xi=4.0,
                  g=4e-6, dt=PIPE_DT, phase=None) -> Instance:
    """Concurrent flow in a circular pipe (Section 3.3): wetting phase along
    the wall, non-wetting core of radius a = radius sqrt(1 - s_w), dynamic
    viscosity ratio visc_ratio = mu_nw / mu_w, driven along the axis by the
    acceleration g, started from the steady diffuse-interface profile.  The
    wetting phase is the heavy one (rho_l = rho_w); the paper's densities are
    equal, which the density-labelled phases of this model cannot represent,
    so rho_nw is close to rho_w, and the surface tension is small (the
    free-energy coefficients grow as (rho_w - rho_nw)^-4, and at sigma = 1e-3
    the interface currents reach a tenth of the axial speed; the axial flow
    does not depend on sigma).  The extruded-prism tetrahedra are not aligned
    with the lattice directions, and the streaming is stable on them at
    dt = 0.05, not at 0.1 or 0.2 (as on the periodic Delaunay meshes).  tau_w
    defaults to 1 / sqrt(visc_ratio), so that both relaxation times stay in
    [0.45, 2.4] over the viscosity ratios 0.2..5.  phase = "w" or "nw" fills
    the whole pipe with that phase (the single-phase reference flow of
    either fluid)."""
    if tau_w is None:
        tau_w = 1.0 / np.sqrt(visc_ratio)
    tau_nw = tau_w * visc_ratio * rho_w / rho_nw
    xyz = mesh["xyz"]
    r = np.hypot(xyz[:, 0] - radius, xyz[:, 1] - radius)
    a = radius * np.sqrt(max(1.0 - s_w, 0.0))
    n = xyz.shape[0]
    u = np.zeros((n, 3))
    if phase is None:
        rho = _tanh_profile(r - a, rho_w, rho_nw, xi)
        comp = (rho - rho_nw) / (rho_w - rho_nw)
        dp = sigma / max(a, 1e-12)               # Laplace jump of a cylinder: sigma / a, core above
        p = dp * (1.0 - comp)
        u[:, 2] = pipe_profile(r, radius=radius, a=a, rho_w=rho_w, rho_nw=rho_nw, tau_w=tau_w, tau_nw=tau_nw,
                               xi=xi, g=g, dt=dt)
    else:
        rb, tb = (rho_w, tau_w) if phase == "w" else (rho_nw, tau_nw)
        rho = np.full(n, rb)
        p = np.zeros(n)
        dp = 0.0
        u[:, 2] = rb * g * (radius ** 2 - r ** 2) / (4.0 * rb * CS2 * tb * dt)
    phys = Phys(rho_w, rho_nw, tau_w, tau_nw, sigma, xi, dt, (0.0, 0.0, g))
    return Instance(mesh, phys, rho, u, p,
                    meta=dict(kind="pipe", radius=radius, a=a, s_w=s_w, visc_ratio=visc_ratio, g=g, phase=phase,
                              dp_laplace=dp, axis=np.array([radius, radius])))


def pipe3d(radius=20.0, nz=4, *, s_w=0.5, visc_ratio=1.0, jitter=0.2, seed=1614, steps=2000, **kw) -> Workload:
    """One concurrent pipe flow on a D3Q19 tetrahedral pipe mesh."""
    mesh = pipe_mesh_3d(radius, nz, jitter=jitter, seed=seed)
    inst = pipe_instance(mesh, radius=radius, s_w=s_w, visc_ratio=visc_ratio, **kw)
    return Workload(f"pipe3d_r{radius:g}", 19, [inst], steps,
                    "D3Q19 concurrent two-phase flow in a circular pipe with a curved bounce-back wall")


def pipe_study3d(radius=20.0, nz=4, *, saturations=(0.25, 0.5, 0.75), visc_ratios=(0.2, 1.0, 5.0), jitter=0.2,
                 seed=1614, steps=2000, **kw) -> Workload:
    """The relative-permeability study of Section 3.3 as one batch: for each
    viscosity ratio, every wetting saturation and the single-phase flows of
    the wetting and of the non-wetting fluid (same relaxation times), all on
    the same mesh."""
    mesh = pipe_mesh_3d(radius, nz, jitter=jitter, seed=seed)
    insts = []
    for m in visc_ratios:
        insts += [pipe_instance(mesh, radius=radius, s_w=sw, visc_ratio=m, **kw) for sw in saturations]
        insts.append(pipe_instance(mesh, radius=radius, s_w=1.0, visc_ratio=m, phase="w", **kw))
        insts.append(pipe_instance(mesh, radius=radius, s_w=0.0, visc_ratio=m, phase="nw", **kw))
    return Workload(f"pipe_study3d_r{radius:g}", 19, insts, steps,
                    "D3Q19 concurrent pipe flows over saturations and viscosity ratios, with single-phase references")


WORKLOADS = {
    "droplet2d": droplet2d,
    "channel2d": channel2d,
    "rt2d": rt2d,
    "droplet3d": droplet3d,
    "ensemble2d": ensemble2d,
    "translate2d": translate2d,
    "pipe3d": pipe3d,
}
