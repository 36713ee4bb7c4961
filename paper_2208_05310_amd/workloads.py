"""Seeded synthetic workloads: mesh sizes, parameters, droplet layouts, noise.

This module holds inputs only -- no arithmetic of the method.  Both the HIP
path and the CPU oracle are driven from the same descriptions, and each side
builds its own mesh, metrics, Maxwell states and initial state from them.

Workload shapes follow the paper's droplet set-ups (tanh droplet profile of
Sec. 4.1.1/4.2, the head-on collision of Sec. 4.3, the sessile and sliding
configurations of Sec. 4.4) at the sizes of the benchmark configurations.  Fluid properties default to Table 1
(gamma_K = 1e-4, mu = 0.01, k = 1/150, c_v = 5) with the reduced van der
Waals constants of Sec. 2.1; Korteweg and relaxation parameters default to
alpha = 100, beta = 1000 (the values the paper uses most for bulk cases).
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace

import numpy as np

# Reduced van der Waals constants (Sec. 2.1) and Table 1 fluid properties.
TABLE1 = dict(R=8.0 / 3.0, a=3.0, b=1.0 / 3.0, cv=5.0, mu=0.01, kappa=1.0 / 150.0,
              gam=1e-4, alpha=100.0, beta=1000.0, cfl=0.9)

# Box side kinds: 0 periodic / none, 1 no-slip isothermal wall with a static
# contact angle (optionally moving), 2 slip adiabatic neutral wall, 3
# generalized Navier-slip wall (gamma_1..gamma_4; gamma_3 = inf: isothermal).
PERIODIC, NOSLIP_CA, SLIP, NAVIER = 0, 1, 2, 3
NO_GAMMA = (0.0, 0.0, float("inf"), 0.0)


@dataclass(frozen=True)
class Workload:
    name: str
    N: int
    n: tuple
    length: tuple = (1.0, 1.0, 1.0)
    periodic: tuple = (1, 1, 1)
    side_kind: tuple = (0, 0, 0, 0, 0, 0)
    side_twall: tuple = (0.0,) * 6
    side_theta: tuple = (90.0,) * 6
    T0: float = 0.85
    centres: tuple = ((0.5, 0.5, 0.5),)
    radii: tuple = (0.25,)
    width: float = 0.05
    steps: int = 20
    noise_seed: int | None = 1
    noise_amp: float = 1e-6
    params: dict = field(default_factory=lambda: dict(TABLE1))
    curve_amp: float = 0.0
    velocities: tuple | None = None   # one velocity per droplet, or None (at rest)
    rho_v: float = 0.0                # bulk densities; 0 selects the Maxwell states at T0
    rho_l: float = 0.0
    side_uwall: tuple | None = None   # per side wall velocity (kinds 1, 3), or None (fixed walls)
    side_gamma: tuple | None = None   # per side (gamma_1, gamma_2, gamma_3, gamma_4) of Navier-slip walls
    side_tgrad: tuple | None = None   # per side wall temperature gradient: T_wall(x) = twall + tgrad . x
    side_trate: tuple | None = None   # per side wall temperature rate: + trate * t
    cylinder_axis: int = -1           # droplets are cylinders along this axis (-1: spheres)
    ngeo: int = 0                     # geometry degree of curved elements (0: N when curve_amp != 0)

    @property
    def nelems(self) -> int:
        return self.n[0] * self.n[1] * self.n[2]

    @property
    def nnodes(self) -> int:
        return self.nelems * (self.N + 1) ** 3

    def noise(self) -> np.ndarray | None:
        """Uniform noise U(-amp, amp) on rho, one value per node in the
        state order [element][k][j][i] (numpy PCG64 with the workload seed)."""
        if self.noise_seed is None:
            return None
        rng = np.random.default_rng(self.noise_seed)
        return rng.uniform(-self.noise_amp, self.noise_amp, self.nnodes)

    def with_(self, **kw) -> "Workload":
        return replace(self, **kw)


def lobatto_points(n: int) -> np.ndarray:
    """Gauss-Lobatto points of degree n on [-1, 1]: the ends and the roots of
    the derivative of the Legendre polynomial P_n."""
    from numpy.polynomial import legendre as npleg
    inner = npleg.legroots(npleg.legder(np.eye(n + 1)[n])) if n > 1 else np.array([])
    return np.concatenate([[-1.0], np.sort(inner), [1.0]])


def box_map(X, length, lo=(0.0, 0.0, 0.0), curve_amp=0.0):
    """The mesh map of a box: the identity, perturbed by curve_amp * prod_d
    sin(2 pi (X_d - lo_d) / L_d) added to every component (a smooth curved
    mesh with the box's periodicity, flat on the box's sides)."""
    X = np.asarray(X, dtype=np.float64)
    if curve_amp == 0.0:
        return X.copy()
    s = np.prod([np.sin(2 * np.pi * (X[d] - lo[d]) / length[d]) for d in range(3)], axis=0)
    return X + curve_amp * s[None]


def box_geometry(n, length=(1.0, 1.0, 1.0), ngeo=1, curve_amp=0.0, lo=(0.0, 0.0, 0.0)) -> np.ndarray:
    """Geometry nodes of the n[0] x n[1] x n[2] elements of a box (element
    ex + nx (ey + ny ez)) on the Gauss-Lobatto points of degree ngeo:
    [nelems][(ngeo+1)^3][3], node a + (ngeo+1)(b + (ngeo+1) c), the box map
    (see box_map) at the points lo + h (e + (xi + 1)/2)."""
    nx, ny, nz = (int(v) for v in n)
    h = [length[d] / n[d] for d in range(3)]
    xl = lobatto_points(ngeo)
    g = ngeo + 1
    ez, ey, ex = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ee = [ex.reshape(-1), ey.reshape(-1), ez.reshape(-1)]
    c, b, a = np.meshgrid(np.arange(g), np.arange(g), np.arange(g), indexing="ij")
    ii = [a.reshape(-1), b.reshape(-1), c.reshape(-1)]
    X = np.stack([lo[d] + h[d] * (ee[d][:, None] + 0.5 * (xl[ii[d]][None, :] + 1.0)) for d in range(3)])
    x = box_map(X.reshape(3, -1), length, lo, curve_amp).reshape(3, nx * ny * nz, g ** 3)
    return np.ascontiguousarray(np.transpose(x, (1, 2, 0)))


def _periodic_dist(a, b, length, periodic):
    d = np.asarray(a, dtype=np.float64) - np.asarray(b, dtype=np.float64)
    L = np.asarray(length, dtype=np.float64)
    per = np.asarray(periodic, dtype=bool)
    d = np.where(per, d - L * np.round(d / L), d)
    return float(np.sqrt(np.sum(d * d)))


def random_droplets(seed, count, rmin, rmax, gap, length=(1.0, 1.0, 1.0), periodic=(1, 1, 1),
                    max_tries=100000):
    """Droplet centres uniform in the box and radii uniform in [rmin, rmax],
    sequential rejection until every pair is at least r_i + r_j + gap apart
    (distances as minimum images along periodic axes)."""
    rng = np.random.default_rng(seed)
    centres, radii = [], []
    tries = 0
    while len(centres) < count:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("droplet placement did not converge")
        c = rng.uniform(0.0, 1.0, 3) * np.asarray(length)
        r = rng.uniform(rmin, rmax) if rmax > rmin else rmin
        if all(_periodic_dist(c, c2, length, periodic) >= r + r2 + gap
               for c2, r2 in zip(centres, radii)):
            centres.append(tuple(float(v) for v in c))
            radii.append(float(r))
    return tuple(centres), tuple(radii)


def c1() -> Workload:
    """Periodic unit cube, 4^3 elements, N=3, one droplet r=0.25 at T=0.85."""
    return Workload(name="droplet_periodic_4x4x4_N3", N=3, n=(4, 4, 4), steps=20, noise_seed=1)


def c2() -> Workload:
    """Periodic unit cube, 16^3 elements, N=4, two droplets r=0.15 at seeded
    centres, T=0.85, beta=1e3; the FP64 throughput workload."""
    cen, rad = random_droplets(2, 2, 0.15, 0.15, 0.20)
    return Workload(name="two_droplets_periodic_16x16x16_N4", N=4, n=(16, 16, 16),
                    centres=cen, radii=rad, T0=0.85, steps=200, noise_seed=12)


def c3(n=32) -> Workload:
    """Periodic unit cube, n^3 elements (32 for the full case), N=5, eight
    droplets with radii in [0.05, 0.12] at T=0.9, at least 0.2 apart (surface to
    surface)."""
    cen, rad = random_droplets(3, 8, 0.05, 0.12, 0.20)
    return Workload(name=f"eight_droplets_periodic_{n}x{n}x{n}_N5", N=5, n=(n, n, n),
                    centres=cen, radii=rad, T0=0.9, steps=500, noise_seed=13)


def c4(scale=1) -> Workload:
    """Box (0,1)x(0,1)x(0,0.5), 48x48x24 elements at N=3 (divided by
    ``scale``), periodic in x and y, no-slip isothermal wall at T=0.9 with a
    60 degree contact angle at z=0, slip adiabatic wall at z=0.5; a
    hemispherical droplet r=0.2 on the wall, fluid at T=0.85."""
    n = (48 // scale, 48 // scale, 24 // scale)
    return Workload(name=f"sessile_wall_{n[0]}x{n[1]}x{n[2]}_N3", N=3, n=n,
                    length=(1.0, 1.0, 0.5), periodic=(1, 1, 0),
                    side_kind=(0, 0, 0, 0, NOSLIP_CA, SLIP),
                    side_twall=(0.0, 0.0, 0.0, 0.0, 0.9, 0.0),
                    side_theta=(90.0, 90.0, 90.0, 90.0, 60.0, 90.0),
                    T0=0.85, centres=((0.5, 0.5, 0.0),), radii=(0.2,), steps=1000,
                    noise_seed=14)


# Head-on collision regimes of Sec. 4.3 (Table 6): relative velocity and
# viscosity; the other properties are common (Table 5).
COLLISION = {"reflexive": (2.2, 6.944e-4), "toroidal": (4.0, 1.010e-3)}


def c5(scale=1, regime="reflexive") -> Workload:
    """Binary head-on droplet collision (Sec. 4.3): periodic unit cube, 50^3
    elements at N=3 (divided by ``scale``); droplets r=0.1 at (0.3,0.5,0.5)
    and (0.7,0.5,0.5) moving towards each other with u_rel/2 each; the
    Young-Laplace adjusted densities 0.3537 / 1.8493 at T=0.85 and interface
    width 0.0772 of Table 5 (tanh width 0.0772/4); gamma_K = 1/6000,
    alpha = 200, beta = 1000, k = 1/150, c_v = 5, mu of Table 6."""
    u_rel, mu = COLLISION[regime]
    n = 50 // scale
    params = dict(TABLE1, gam=1.0 / 6000.0, alpha=200.0, beta=1000.0, mu=mu)
    return Workload(name=f"collision_{regime}_{n}x{n}x{n}_N3", N=3, n=(n, n, n), T0=0.85,
                    centres=((0.3, 0.5, 0.5), (0.7, 0.5, 0.5)), radii=(0.1, 0.1), width=0.0772 / 4,
                    velocities=((u_rel / 2, 0.0, 0.0), (-u_rel / 2, 0.0, 0.0)), rho_v=0.3537, rho_l=1.8493,
                    steps=200, noise_seed=15, params=params)


def c6(scale=1, gamma1=0.0) -> Workload:
    """Droplet sliding under a moving lid (Sec. 4.4.2): box
    (0,1)x(0,0.5)x(0,0.25) of cube elements, 100x50x25 at N=3 (divided by
    ``scale``), periodic in x and y; a generalized Navier-slip isothermal floor
    at T=0.85 (gamma_2 = 8e-4, gamma_4 = 0, 90 degree static angle) and a
    no-slip isothermal lid at T=0.85 moving with (0.5, 0, 0); a half-sphere
    r=0.1 centred at (0.5, 0.25, 0) at the Maxwell densities of T=0.85,
    interface width L_i = 0.0598 of Table 1 (tanh width L_i/4; 0.05 on the
    coarse meshes of ``scale`` > 1, which cannot resolve it); alpha = 100,
    beta = 100, fluid at rest.  The paper's gamma_1 = 20 makes the wall terms
    far stiffer than the explicit step of the bulk operator allows, so the
    default is gamma_1 = 0 (the dynamic-angle terms are exercised at small
    gamma_1 and step size by the tests)."""
    n = (100 // scale, 50 // scale, max(1, 25 // scale))
    params = dict(TABLE1, alpha=100.0, beta=100.0)
    g1 = f"_g1_{gamma1:g}" if gamma1 else ""
    return Workload(name=f"sliding_droplet_{n[0]}x{n[1]}x{n[2]}_N3{g1}", N=3, n=n, length=(1.0, 0.5, 0.25),
                    periodic=(1, 1, 0), side_kind=(0, 0, 0, 0, NAVIER, NOSLIP_CA),
                    side_twall=(0.0, 0.0, 0.0, 0.0, 0.85, 0.85), side_theta=(90.0,) * 6,
                    side_uwall=((0.0, 0.0, 0.0),) * 5 + ((0.5, 0.0, 0.0),),
                    side_gamma=(NO_GAMMA,) * 4 + ((float(gamma1), 8e-4, float("inf"), 0.0), NO_GAMMA),
                    T0=0.85, centres=((0.5, 0.25, 0.0),), radii=(0.1,),
                    width=0.0598 / 4 if scale == 1 else 0.05, steps=200, noise_seed=16, params=params)


def c7(scale=1) -> Workload:
    """The sessile-droplet wall box of c4 with a floor temperature rising
    linearly along x, T_w = 0.85 + 0.1 x (0.85 .. 0.95), so the contact-angle
    constants (sigma_vl and the Maxwell states) vary along the wall and come
    from the wall-temperature table of Sec. 3.2 at every floor face point."""
    w = c4(scale)
    return w.with_(name=w.name.replace("sessile_wall", "graded_wall"),
                   side_twall=(0.0, 0.0, 0.0, 0.0, 0.85, 0.0),
                   side_tgrad=((0.0, 0.0, 0.0),) * 4 + ((0.1, 0.0, 0.0), (0.0, 0.0, 0.0)), noise_seed=17)


def c8(theta=60.0, n=(50, 50, 10)) -> Workload:
    """Liquid pillar between two walls (Sec. 4.4.1, static contact angles):
    box (0,1)x(0,1)x(0,0.2), periodic in x and y, isothermal no-slip walls at
    T=0.85 with the static angle ``theta`` at z=0 and z=0.2; a cylinder r=0.2
    about (0.5, 0.5) spanning the gap at the Maxwell densities of T=0.85,
    interface width L_i = 0.0598 of Table 1 (tanh width L_i/4); alpha = 100,
    beta = 100, fluid at rest.  The paper refines the centre to h = 0.01 with
    mortars (64000 elements); here a conforming mesh of n elements (h = 0.02
    at the default)."""
    params = dict(TABLE1, alpha=100.0, beta=100.0)
    return Workload(name=f"pillar_theta{theta:g}_{n[0]}x{n[1]}x{n[2]}_N3", N=3, n=tuple(n), length=(1.0, 1.0, 0.2),
                    periodic=(1, 1, 0), side_kind=(0, 0, 0, 0, NOSLIP_CA, NOSLIP_CA),
                    side_twall=(0.0, 0.0, 0.0, 0.0, 0.85, 0.85),
                    side_theta=(90.0, 90.0, 90.0, 90.0, float(theta), float(theta)),
                    T0=0.85, centres=((0.5, 0.5, 0.1),), radii=(0.2,), width=0.0598 / 4, cylinder_axis=2,
                    steps=1000, noise_seed=18, params=params)


def serving_stream(seed=5, count=256, rate=50.0):
    """Poisson request stream: arrival times (exponential gaps at ``rate``/s)
    and per-request workload descriptions.  Each request draws its grid from
    {4^3, 8^3, 12^3, 16^3}, N from {2,3,4,5}, T from U[0.80, 0.95] and either a
    periodic droplet (r=0.25) or a wall box with a hemispherical droplet
    (r=0.2) and a contact angle from U[45, 135] degrees; 200 RK steps each."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, count))
    reqs = []
    for k in range(count):
        g = int(rng.choice([4, 8, 12, 16]))
        N = int(rng.choice([2, 3, 4, 5]))
        T = float(rng.uniform(0.80, 0.95))
        wall = bool(rng.integers(0, 2))
        theta = float(rng.uniform(45.0, 135.0))
        nseed = int(rng.integers(0, 2**31 - 1))
        if wall:
            w = Workload(name=f"req{k}_wall_{g}_N{N}", N=N, n=(g, g, g), periodic=(1, 1, 0),
                         side_kind=(0, 0, 0, 0, NOSLIP_CA, SLIP),
                         side_twall=(0.0, 0.0, 0.0, 0.0, T, 0.0),
                         side_theta=(90.0, 90.0, 90.0, 90.0, theta, 90.0),
                         T0=T, centres=((0.5, 0.5, 0.0),), radii=(0.2,), steps=200,
                         noise_seed=nseed)
        else:
            w = Workload(name=f"req{k}_periodic_{g}_N{N}", N=N, n=(g, g, g), T0=T,
                         centres=((0.5, 0.5, 0.5),), radii=(0.25,), steps=200, noise_seed=nseed)
        reqs.append((float(t[k]), w))
    return reqs
