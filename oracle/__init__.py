"""FP64 CPU oracle for the DGSEM relaxation-model-1 NSK solver (test infrastructure).

This package is the reference the HIP library is checked against.  It is
used only by ``tests/``, by ``__graft_entry__.smoke()`` and by the CPU
baseline leg of ``bench.py``; the product path never imports it.  It shares
no code with the HIP library: the C source ``nskr_oracle.c`` has its own
basis, metrics, thermodynamics, fluxes, walls, time integration and
reductions, each written from the paper (arXiv 2208.05310, Sec. 2-3).

Pinned by ``tests/test_oracle_*.py`` against values the paper prints
(Tables 1, 2, 5), closed forms, DGSEM invariants (exactness, free-stream
preservation, conservation), the relaxation ODE, a convergence study on an
isentropic vortex (ideal-gas reduction) and a manufactured solution of the
full system, and a dense brute-force re-implementation on a tiny mesh.
The wall fluxes are pinned term by term by closed forms: a fluid at rest
between walls (pressure), Couette flow under a moving lid (no-slip and
Navier-slip tractions, the wall's work), steady conduction between
isothermal and between heat-transfer walls, the normal traction of a slip
wall under compression, closed-form rates of the gamma_1 and gamma_4 terms,
the contact-angle c-flux integral, and a lid moving over fluid at rest (its
ghost flux); the wall-temperature table by its grid values, the linear
interpolation bound and its time and stage evaluation.  A mutation test
(``tests/test_oracle_mutations.py``) plants 66 plausible mistakes in copies of
the C source and checks that the pins reject every one of them.  The Rusanov
dissipation speed (the larger of |u . n| + c on the two sides, as the flux is
stated in Sec. 3.1) is pinned by the discrete energy balance of a passive
order parameter that is constant per element (``tests/test_oracle_rusanov.py``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nskr_oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")
# a prebuilt variant of the oracle (the mutation tests build deliberately
# broken copies of the C source and check that the pins reject them)
_SO_OVERRIDE = os.environ.get("NSKR_ORACLE_SO")


def build() -> str:
    """Compile the oracle with gcc (FP64, no fast-math, OpenMP over elements)."""
    cmd = ["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-D_GNU_SOURCE",
           "-Wall", "-Wextra", "-o", _SO + ".tmp", _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_SO + ".tmp", _SO)
    return _SO


class Params(ctypes.Structure):
    _fields_ = [("R", ctypes.c_double), ("a", ctypes.c_double), ("b", ctypes.c_double),
                ("cv", ctypes.c_double), ("mu", ctypes.c_double), ("kappa", ctypes.c_double),
                ("gam", ctypes.c_double), ("alpha", ctypes.c_double), ("beta", ctypes.c_double),
                ("cfl", ctypes.c_double), ("model", ctypes.c_int)]


class Box(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int), ("n", ctypes.c_int * 3), ("lo", ctypes.c_double * 3),
                ("len", ctypes.c_double * 3), ("periodic", ctypes.c_int * 3),
                ("side_kind", ctypes.c_int * 6), ("side_twall", ctypes.c_double * 6),
                ("side_theta", ctypes.c_double * 6), ("curve_amp", ctypes.c_double),
                ("side_uwall", (ctypes.c_double * 3) * 6), ("side_g1", ctypes.c_double * 6),
                ("side_g2", ctypes.c_double * 6), ("side_g4", ctypes.c_double * 6),
                ("side_g3", ctypes.c_double * 6), ("side_tgrad", (ctypes.c_double * 3) * 6),
                ("side_trate", ctypes.c_double * 6), ("ngeo", ctypes.c_int)]


_lib = None
_D = ctypes.POINTER(ctypes.c_double)


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if _SO_OVERRIDE:
        L = ctypes.CDLL(_SO_OVERRIDE)
    else:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_SO)
    d, i, vp = ctypes.c_double, ctypes.c_int, ctypes.c_void_p
    sig = {
        "orc_create": (vp, [ctypes.POINTER(Params), ctypes.POINTER(Box), ctypes.c_char_p, i]),
        "orc_destroy": (None, [vp]),
        "orc_nnodes": (ctypes.c_long, [vp]),
        "orc_nelems": (i, [vp]),
        "orc_node_coords": (None, [vp, _D]),
        "orc_metrics": (None, [vp, _D, _D, _D]),
        "orc_rhs": (None, [vp, _D, _D]),
        "orc_lift1": (None, [vp, _D, _D]),
        "orc_lift2": (None, [vp, _D, _D]),
        "orc_dt": (d, [vp, _D]),
        "orc_rk_step": (None, [vp, _D, _D, d, d]),
        "orc_run": (None, [vp, _D, _D, d, d, i]),
        "orc_init_droplets": (i, [vp, d, i, _D, _D, d, _D, _D, _D, d, d, i]),
        "orc_numflux": (None, [ctypes.POINTER(Params), _D, d, _D, d, _D, _D]),
        "orc_reduce": (None, [vp, _D, _D]),
        "orc_maxwell": (i, [d, d, d, d, _D, _D, _D]),
        "orc_spinodal": (i, [d, d, d, d, _D, _D]),
        "orc_rho_of_p": (d, [d, d, d, d, d, i]),
        "orc_sigma": (d, [d, d, d, d, d]),
        "orc_sigma_panels": (d, [d, d, d, d, d, i]),
        "orc_sigma_gauss15": (d, [d, d, d, d, d]),
        "orc_table_build": (None, [d, d, d, _D]),
        "orc_set_time": (None, [vp, d]),
        "orc_table_lookup": (None, [_D, d, _D]),
        "orc_dpsiwall_dc": (d, [d, d, d, d, d]),
        "orc_psiwall": (d, [d, d, d, d, d]),
        "orc_basis": (None, [i, _D, _D, _D, _D, _D, _D]),
        "orc_lobatto": (None, [i, _D]),
        "orc_rk_coeffs": (None, [_D, _D, _D]),
        "orc_pressure": (d, [d, d, d, d, d]),
        "orc_cs2": (d, [d, d, d, d, d, d]),
        "orc_chempot": (d, [d, d, d, d, d]),
        "orc_set_threads": (None, [i]),
        "orc_get_threads": (i, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_D)


def make_params(R=8.0 / 3.0, a=3.0, b=1.0 / 3.0, cv=5.0, mu=0.01, kappa=1.0 / 150.0,
                gam=1e-4, alpha=100.0, beta=1000.0, cfl=0.9, model=1) -> Params:
    """model: relaxation model 1 (Rusanov flux) or 2 (modified pressure,
    HLLC flux)."""
    return Params(R, a, b, cv, mu, kappa, gam, alpha, beta, cfl, int(model))


def make_box(N, n, lo=(0.0, 0.0, 0.0), length=(1.0, 1.0, 1.0), periodic=(1, 1, 1),
             side_kind=(0,) * 6, side_twall=(0.0,) * 6, side_theta=(90.0,) * 6,
             curve_amp=0.0, side_uwall=((0.0, 0.0, 0.0),) * 6, side_g1=(0.0,) * 6,
             side_g2=(0.0,) * 6, side_g3=(float("inf"),) * 6, side_g4=(0.0,) * 6,
             side_tgrad=((0.0, 0.0, 0.0),) * 6, side_trate=(0.0,) * 6, ngeo=0) -> Box:
    """Wall kinds per side (x-, x+, y-, y+, z-, z+): 1 no-slip isothermal with a
    static contact angle, moving with side_uwall; 2 slip adiabatic neutral;
    3 generalized Navier slip with gamma_1..gamma_4 (side_g3 infinite =
    isothermal).  side_tgrad, side_trate: wall temperature twall + tgrad . x
    + trate t (kinds 1, 3), through the sigma/Maxwell table.  curve_amp: the
    smooth sine perturbation of the box map; ngeo: each element's geometry is
    the degree-ngeo Gauss-Lobatto interpolant of the map (0: degree N)."""
    uw = ((ctypes.c_double * 3) * 6)(*[(ctypes.c_double * 3)(*v) for v in side_uwall])
    tg = ((ctypes.c_double * 3) * 6)(*[(ctypes.c_double * 3)(*v) for v in side_tgrad])
    d6 = lambda v: (ctypes.c_double * 6)(*[float(x) for x in v])
    return Box(int(N), (ctypes.c_int * 3)(*n), (ctypes.c_double * 3)(*lo),
               (ctypes.c_double * 3)(*length), (ctypes.c_int * 3)(*periodic),
               (ctypes.c_int * 6)(*side_kind), d6(side_twall), d6(side_theta), float(curve_amp),
               uw, d6(side_g1), d6(side_g2), d6(side_g4), d6(side_g3), tg, d6(side_trate), int(ngeo))


class Oracle:
    """One discretised problem (mesh + parameters) on the CPU in FP64."""

    def __init__(self, params: Params, box: Box, threads: int | None = None):
        L = lib()
        if threads is not None:
            L.orc_set_threads(int(threads))
        err = ctypes.create_string_buffer(256)
        self.params, self.box = params, box
        self._c = L.orc_create(ctypes.byref(params), ctypes.byref(box), err, 256)
        if not self._c:
            raise ValueError(err.value.decode())
        self.N = box.N
        self.nnodes = int(L.orc_nnodes(self._c))
        self.nelems = int(L.orc_nelems(self._c))

    def __del__(self):
        if getattr(self, "_c", None):
            lib().orc_destroy(self._c)
            self._c = None

    def state(self) -> np.ndarray:
        return np.zeros((6, self.nnodes))

    def coords(self) -> np.ndarray:
        x = np.zeros((3, self.nnodes))
        lib().orc_node_coords(self._c, _ptr(x))
        return x

    def metrics(self):
        P = self.N + 1
        Ja = np.zeros((9, self.nnodes))
        J = np.zeros(self.nnodes)
        nv = np.zeros((3, self.nelems * 6 * P * P))
        lib().orc_metrics(self._c, _ptr(Ja), _ptr(J), _ptr(nv))
        return Ja, J, nv.reshape(3, self.nelems, 6, P * P)

    def set_time(self, t: float):
        """Time at which rhs() evaluates (walls whose temperature changes in
        time); run() and rk_step() set each stage's time themselves."""
        lib().orc_set_time(self._c, float(t))

    def rhs(self, U: np.ndarray) -> np.ndarray:
        U = np.ascontiguousarray(U, dtype=np.float64)
        Ut = np.zeros_like(U)
        lib().orc_rhs(self._c, _ptr(U), _ptr(Ut))
        return Ut

    def lift1(self, U):
        U = np.ascontiguousarray(U, dtype=np.float64)
        q = np.zeros((15, self.nnodes))
        lib().orc_lift1(self._c, _ptr(U), _ptr(q))
        return q

    def lift2(self, U):
        U = np.ascontiguousarray(U, dtype=np.float64)
        o = np.zeros((5, self.nnodes))
        lib().orc_lift2(self._c, _ptr(U), _ptr(o))
        return o

    def dt(self, U) -> float:
        U = np.ascontiguousarray(U, dtype=np.float64)
        return float(lib().orc_dt(self._c, _ptr(U)))

    def rk_step(self, U, R, t, dt):
        lib().orc_rk_step(self._c, _ptr(U), _ptr(R), float(t), float(dt))

    def run(self, U, R, t, dt, nsteps):
        lib().orc_run(self._c, _ptr(U), _ptr(R), float(t), float(dt), int(nsteps))

    def init_droplets(self, T0, centres, radii, width, noise=None, velocities=None, rho_v=0.0,
                      rho_l=0.0, cylinder_axis=-1) -> np.ndarray:
        U = self.state()
        cen = np.ascontiguousarray(np.asarray(centres, dtype=np.float64).reshape(-1, 3))
        rad = np.ascontiguousarray(np.asarray(radii, dtype=np.float64).reshape(-1))
        nz = None
        if noise is not None:
            nz = np.ascontiguousarray(noise, dtype=np.float64)
            assert nz.size == self.nnodes
        vel = None
        if velocities is not None:
            vel = np.ascontiguousarray(np.asarray(velocities, dtype=np.float64).reshape(-1, 3))
            assert vel.shape[0] == rad.size
        rc = lib().orc_init_droplets(self._c, float(T0), int(rad.size), _ptr(cen), _ptr(rad),
                                     float(width), _ptr(nz) if nz is not None else None, _ptr(U),
                                     _ptr(vel) if vel is not None else None, float(rho_v), float(rho_l),
                                     int(cylinder_axis))
        if rc != 0:
            raise ValueError("init failed (supercritical temperature?)")
        return U

    def reduce(self, U) -> np.ndarray:
        U = np.ascontiguousarray(U, dtype=np.float64)
        out = np.zeros(20)
        lib().orc_reduce(self._c, _ptr(U), _ptr(out))
        return out


# ---- thermodynamics and 1D operators ------------------------------------
def maxwell(T, R=8.0 / 3.0, a=3.0, b=1.0 / 3.0):
    rv, rl, ps = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    if not lib().orc_maxwell(R, a, b, T, ctypes.byref(rv), ctypes.byref(rl), ctypes.byref(ps)):
        raise ValueError("supercritical")
    return rv.value, rl.value, ps.value


def spinodal(T, R=8.0 / 3.0, a=3.0, b=1.0 / 3.0):
    v, l = ctypes.c_double(), ctypes.c_double()
    if not lib().orc_spinodal(R, a, b, T, ctypes.byref(v), ctypes.byref(l)):
        raise ValueError("supercritical")
    return v.value, l.value


def rho_of_p(T, p, branch, R=8.0 / 3.0, a=3.0, b=1.0 / 3.0):
    return lib().orc_rho_of_p(R, a, b, T, p, int(branch))


def sigma(T, gam=1e-4, R=8.0 / 3.0, a=3.0, b=1.0 / 3.0, panels=None):
    if panels is None:
        return lib().orc_sigma(R, a, b, T, gam)
    return lib().orc_sigma_panels(R, a, b, T, gam, int(panels))


def sigma_gauss15(T, gam=1e-4, R=8.0 / 3.0, a=3.0, b=1.0 / 3.0):
    return lib().orc_sigma_gauss15(R, a, b, T, gam)


NTAB = 10000  # wall-temperature table: equidistant on [0.3, 1]


def wall_table(R=8.0 / 3.0, a=3.0, b=1.0 / 3.0) -> np.ndarray:
    """[NTAB][3]: sigma/sqrt(2 gamma) (15-point Gauss), rho_v, rho_l."""
    tab = np.zeros((NTAB, 3))
    lib().orc_table_build(R, a, b, _ptr(tab))
    return tab


def wall_table_lookup(tab: np.ndarray, T: float) -> np.ndarray:
    out = np.zeros(3)
    lib().orc_table_lookup(_ptr(np.ascontiguousarray(tab)), float(T), _ptr(out))
    return out


def dpsiwall_dc(c, rv, rl, sig, costh):
    return lib().orc_dpsiwall_dc(c, rv, rl, sig, costh)


def psiwall(c, rv, rl, ssv, ssl):
    return lib().orc_psiwall(c, rv, rl, ssv, ssl)


def pressure(rho, T, R=8.0 / 3.0, a=3.0, b=1.0 / 3.0):
    return lib().orc_pressure(R, a, b, rho, T)


def cs2(rho, T, cv=5.0, R=8.0 / 3.0, a=3.0, b=1.0 / 3.0):
    return lib().orc_cs2(R, a, b, cv, rho, T)


def chempot(rho, T, R=8.0 / 3.0, a=3.0, b=1.0 / 3.0):
    return lib().orc_chempot(R, a, b, rho, T)


def basis(N):
    P = N + 1
    x, w, lm, lp = (np.zeros(P) for _ in range(4))
    D, Dh = np.zeros((P, P)), np.zeros((P, P))
    lib().orc_basis(int(N), _ptr(x), _ptr(w), _ptr(D), _ptr(Dh), _ptr(lm), _ptr(lp))
    return x, w, D, Dh, lm, lp


def lobatto(N):
    x = np.zeros(N + 1)
    lib().orc_lobatto(int(N), _ptr(x))
    return x


def rk_coeffs():
    A, B, C = np.zeros(5), np.zeros(5), np.zeros(5)
    lib().orc_rk_coeffs(_ptr(A), _ptr(B), _ptr(C))
    return A, B, C


def set_threads(n):
    lib().orc_set_threads(int(n))


def get_threads():
    return int(lib().orc_get_threads())


def numflux(params, UL, TL, UR, TR, n):
    """Interior numerical flux of the convective part (Rusanov for model 1,
    HLLC for model 2) between two face states, along the unit normal n."""
    out = np.zeros(6)
    UL = np.ascontiguousarray(UL, dtype=np.float64)
    UR = np.ascontiguousarray(UR, dtype=np.float64)
    nn = np.ascontiguousarray(n, dtype=np.float64)
    lib().orc_numflux(ctypes.byref(params), _ptr(UL), float(TL), _ptr(UR), float(TR), _ptr(nn), _ptr(out))
    return out
