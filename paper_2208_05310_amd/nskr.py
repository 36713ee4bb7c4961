"""ctypes binding of libnskr.so (include/nskr.h): argument marshalling only.

Every step of the solver runs in the gfx950 library; PyTorch provides the
device buffers and the stream.  There is no CPU fallback: if the library or
a device is missing, the calls raise.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SO = os.path.join(HERE, "libnskr.so")

NSKR_OK, NSKR_E_ARG, NSKR_E_STATE, NSKR_E_NOMEM, NSKR_E_HIP, NSKR_E_NONFINITE, NSKR_E_UNSUPPORTED = range(7)
NSKR_NSUMS = 20
SUM_NAMES = ["mass", "mom_x", "mom_y", "mom_z", "energy", "c", "kinetic", "gradient_energy",
             "relax_energy", "rho_minus_c_sq", "min_rho", "max_rho", "min_T", "max_T", "n_nonfinite",
             "n_rho_range", "n_T_nonpos", "n_cs2_neg", "entropy", "volume"]

EXPORTS = ["nskr_version", "nskr_create", "nskr_destroy", "nskr_mesh_upload", "nskr_state_size",
           "nskr_device_bytes", "nskr_init_droplets", "nskr_rhs", "nskr_lift1", "nskr_lift2", "nskr_dt",
           "nskr_rk_steps", "nskr_reduce", "nskr_set_profiling", "nskr_profile", "nskr_set_block",
           "nskr_get_block", "nskr_last_error", "nskr_batch_create", "nskr_batch_destroy",
           "nskr_batch_set_graph", "nskr_batch_admit", "nskr_batch_step", "nskr_batch_poll",
           "nskr_batch_retire", "nskr_batch_info", "nskr_batch_last_error", "nskr_set_time", "nskr_get_time",
           "nskr_dt_noalloc"]
KERNEL_KINDS = ["prolong", "lift1", "lift2", "update", "other"]


class NskrError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"nskr error {code}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [("R", ctypes.c_double), ("a", ctypes.c_double), ("b", ctypes.c_double),
                ("cv", ctypes.c_double), ("mu", ctypes.c_double), ("kappa", ctypes.c_double),
                ("gam", ctypes.c_double), ("alpha", ctypes.c_double), ("beta", ctypes.c_double),
                ("cfl", ctypes.c_double), ("precision", ctypes.c_int), ("kahan", ctypes.c_int),
                ("model", ctypes.c_int)]


class Bc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("twall", ctypes.c_double), ("theta_deg", ctypes.c_double),
                ("uwall", ctypes.c_double * 3), ("gamma1", ctypes.c_double), ("gamma2", ctypes.c_double),
                ("gamma3", ctypes.c_double), ("gamma4", ctypes.c_double), ("twall_grad", ctypes.c_double * 3),
                ("twall_rate", ctypes.c_double)]


class Mesh(ctypes.Structure):
    _fields_ = [("nelems", ctypes.c_int), ("ngeo", ctypes.c_int), ("xgeo", ctypes.POINTER(ctypes.c_double)),
                ("nbr", ctypes.POINTER(ctypes.c_int)), ("nbr_face", ctypes.POINTER(ctypes.c_int)),
                ("nbr_orient", ctypes.POINTER(ctypes.c_int)), ("bc", ctypes.POINTER(ctypes.c_int)),
                ("nbcs", ctypes.c_int), ("bcs", ctypes.POINTER(Bc))]


class Init(ctypes.Structure):
    _fields_ = [("T0", ctypes.c_double), ("ndrop", ctypes.c_int), ("centres", ctypes.POINTER(ctypes.c_double)),
                ("radii", ctypes.POINTER(ctypes.c_double)), ("width", ctypes.c_double),
                ("length", ctypes.c_double * 3), ("periodic", ctypes.c_int * 3),
                ("velocities", ctypes.POINTER(ctypes.c_double)), ("rho_v", ctypes.c_double),
                ("rho_l", ctypes.c_double), ("cylinder_axis", ctypes.c_int)]


_lib = None
ABI_VERSION = 9  # the struct layouts and semantics below


def lib():
    """Load libnskr.so (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(SO):
        raise ImportError(f"{SO} is missing; run paper_2208_05310_amd/build.py (or __graft_entry__.build())")
    L = ctypes.CDLL(SO)
    vp, i, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    sig = {
        "nskr_version": (i, []),
        "nskr_create": (i, [ctypes.POINTER(Params), i, i, ctypes.POINTER(vp)]),
        "nskr_destroy": (i, [vp]),
        "nskr_mesh_upload": (i, [vp, ctypes.POINTER(Mesh), vp]),
        "nskr_state_size": (i, [vp, ctypes.POINTER(ctypes.c_size_t)]),
        "nskr_device_bytes": (i, [vp, ctypes.POINTER(ctypes.c_size_t)]),
        "nskr_init_droplets": (i, [vp, ctypes.POINTER(Init), ctypes.POINTER(ctypes.c_double), vp, vp]),
        "nskr_rhs": (i, [vp, vp, vp, vp]),
        "nskr_lift1": (i, [vp, vp, vp, vp]),
        "nskr_lift2": (i, [vp, vp, vp, vp]),
        "nskr_dt": (i, [vp, vp, ctypes.POINTER(ctypes.c_double), vp]),
        "nskr_dt_noalloc": (i, [vp, vp, ctypes.POINTER(ctypes.c_double), vp]),
        "nskr_rk_steps": (i, [vp, vp, vp, d, i, vp]),
        "nskr_reduce": (i, [vp, vp, ctypes.POINTER(ctypes.c_double), vp]),
        "nskr_set_profiling": (i, [vp, i]),
        "nskr_profile": (i, [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_long), vp]),
        "nskr_set_block": (i, [vp, i]),
        "nskr_get_block": (i, [vp, ctypes.POINTER(i)]),
        "nskr_last_error": (ctypes.c_char_p, [vp]),
        "nskr_set_time": (i, [vp, d]),
        "nskr_get_time": (i, [vp, ctypes.POINTER(d)]),
        "nskr_batch_create": (i, [i, ctypes.c_size_t, ctypes.POINTER(vp)]),
        "nskr_batch_destroy": (i, [vp]),
        "nskr_batch_set_graph": (i, [vp, i]),
        "nskr_batch_admit": (i, [vp, vp, vp, vp, d, i, ctypes.POINTER(i)]),
        "nskr_batch_step": (i, [vp, vp]),
        "nskr_batch_poll": (i, [vp, ctypes.POINTER(i), i, ctypes.POINTER(i)]),
        "nskr_batch_retire": (i, [vp, i]),
        "nskr_batch_info": (i, [vp, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(i), ctypes.POINTER(ctypes.c_long)]),
        "nskr_batch_last_error": (ctypes.c_char_p, [vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    if L.nskr_version() != ABI_VERSION:
        raise ImportError(f"{SO} has ABI version {L.nskr_version()}, this binding expects {ABI_VERSION}; rebuild it")
    _lib = L
    return L


def box_mesh(n, length=(1.0, 1.0, 1.0), periodic=(1, 1, 1), side_kind=(0,) * 6, side_twall=(0.0,) * 6,
             side_theta=(90.0,) * 6, lo=(0.0, 0.0, 0.0), side_uwall=None, side_gamma=None, side_tgrad=None,
             side_trate=None):
    """Structured box of n[0] x n[1] x n[2] parallelepiped elements as host
    arrays for nskr_mesh_upload: corners, neighbours (periodic wrap or -1 at
    walls), opposite-face neighbour faces, wall indices and the wall table (one
    entry per non-periodic box side, a dict of the nskr_bc fields).
    side_uwall: per side wall velocity (kinds 1, 3); side_gamma: per side
    (gamma1, gamma2, gamma3, gamma4) of Navier-slip walls (gamma3 = inf:
    isothermal); side_tgrad, side_trate: per side wall temperature gradient
    and rate (kinds 1, 3: T_wall(x, t) = twall + tgrad . x + trate t)."""
    nx, ny, nz = (int(v) for v in n)
    E = nx * ny * nz
    h = [length[d] / n[d] for d in range(3)]
    ez, ey, ex = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ex, ey, ez = ex.reshape(-1), ey.reshape(-1), ez.reshape(-1)
    corners = np.zeros((E, 8, 3))
    for v in range(8):
        i, j, k = v & 1, (v >> 1) & 1, (v >> 2) & 1
        corners[:, v, 0] = lo[0] + h[0] * (ex + i)
        corners[:, v, 1] = lo[1] + h[1] * (ey + j)
        corners[:, v, 2] = lo[2] + h[2] * (ez + k)
    nbr = np.full((E, 6), -1, dtype=np.int32)
    nbf = np.zeros((E, 6), dtype=np.int32)
    bc = np.zeros((E, 6), dtype=np.int32)
    bcs = []
    side_index = {}
    for f in range(6):
        d, s = f // 2, f % 2
        if not periodic[d]:
            if side_kind[f] not in (1, 2, 3):
                raise ValueError(f"box side {f} is not periodic and has no wall kind")
            g = side_gamma[f] if side_gamma is not None else (0.0, 0.0, float("inf"), 0.0)
            bcs.append(dict(kind=int(side_kind[f]), twall=float(side_twall[f]), theta=float(side_theta[f]),
                            uwall=tuple(float(v) for v in (side_uwall[f] if side_uwall is not None else (0, 0, 0))),
                            gamma=tuple(float(v) for v in g),
                            tgrad=tuple(float(v) for v in (side_tgrad[f] if side_tgrad is not None else (0, 0, 0))),
                            trate=float(side_trate[f]) if side_trate is not None else 0.0))
            side_index[f] = len(bcs)
    idx = np.stack([ex, ey, ez])
    for f in range(6):
        d, s = f // 2, f % 2
        nn = idx.copy()
        nn[d] += 1 if s else -1
        inside = (nn[d] >= 0) & (nn[d] < n[d])
        if periodic[d]:
            nn[d] %= n[d]
            inside[:] = True
        ne = nn[0] + nx * (nn[1] + ny * nn[2])
        nbr[:, f] = np.where(inside, ne, -1)
        nbf[:, f] = f ^ 1
        if not periodic[d]:
            bc[:, f] = np.where(inside, 0, side_index[f])
    return corners, nbr, nbf, bc, bcs


def _stream_ptr(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


class Solver:
    """One problem instance on one GPU: parameters, polynomial degree, mesh."""

    def __init__(self, params: dict, N: int, precision: str = "fp64", device: int = 0, kahan: bool = True):
        """precision: "fp64" or "fp32_mixed"; kahan (FP32-mixed only): compensated
        state update.  params["model"] (default 1) picks relaxation model 1 or 2."""
        self.L = lib()
        self.N = int(N)
        self.precision = precision
        self.device = int(device)
        prec = {"fp64": 0, "fp32_mixed": 1}[precision]
        self.kahan = bool(kahan) and prec == 1
        p = Params(params["R"], params["a"], params["b"], params["cv"], params["mu"], params["kappa"],
                   params["gam"], params["alpha"], params["beta"], params.get("cfl", 0.9), prec,
                   1 if self.kahan else 0, int(params.get("model", 1)))
        self.params = dict(params)
        h = ctypes.c_void_p()
        rc = self.L.nskr_create(ctypes.byref(p), self.N, self.device, ctypes.byref(h))
        if rc != NSKR_OK:
            raise NskrError(rc, "nskr_create failed (no HIP device or no gfx950 code?)")
        self._h = h
        self.nnodes = 0

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self.L.nskr_destroy(h)
            self._h = None

    def _check(self, rc):
        if rc != NSKR_OK:
            raise NskrError(rc, self.L.nskr_last_error(self._h).decode())

    @property
    def dtype(self):
        import torch
        return torch.float64 if self.precision == "fp64" else torch.float32

    def upload_box(self, n, length=(1.0, 1.0, 1.0), periodic=(1, 1, 1), side_kind=(0,) * 6,
                   side_twall=(0.0,) * 6, side_theta=(90.0,) * 6, stream=None, side_uwall=None, side_gamma=None,
                   side_tgrad=None, side_trate=None, curve_amp=0.0, ngeo=1):
        """Structured box of parallelepipeds; with curve_amp != 0 (or ngeo >
        1) each element's geometry is given on the Gauss-Lobatto points of
        degree ngeo under the curved box map of workloads.box_map."""
        corners, nbr, nbf, bc, bcs = box_mesh(n, length, periodic, side_kind, side_twall, side_theta,
                                              side_uwall=side_uwall, side_gamma=side_gamma, side_tgrad=side_tgrad,
                                              side_trate=side_trate)
        if curve_amp != 0.0 or ngeo > 1:
            from . import workloads as wl
            xgeo = wl.box_geometry(n, length, ngeo, curve_amp)
            self.upload_mesh(xgeo, nbr, nbf, bc, bcs, stream, ngeo=ngeo)
        else:
            self.upload_mesh(corners, nbr, nbf, bc, bcs, stream)
        self.box = dict(n=tuple(n), length=tuple(length), periodic=tuple(periodic))

    def upload_mesh(self, xgeo, nbr, nbf, bc, bcs, stream=None, ngeo=1, nbo=None):
        """xgeo: [nelems][(ngeo+1)^3][3] geometry nodes on the Gauss-Lobatto
        points of degree ngeo (ngeo = 1: the 8 corners); nbr, nbf, nbo:
        [nelems][6] neighbour element (-1 on walls), its face, the face
        orientation (None: all 0); bc: [nelems][6] wall index (1-based) or 0."""
        xgeo = np.ascontiguousarray(xgeo, dtype=np.float64)
        nbr = np.ascontiguousarray(nbr, dtype=np.int32)
        nbf = np.ascontiguousarray(nbf, dtype=np.int32)
        nbo = None if nbo is None else np.ascontiguousarray(nbo, dtype=np.int32)
        bc = np.ascontiguousarray(bc, dtype=np.int32)
        if xgeo.size != nbr.shape[0] * (ngeo + 1) ** 3 * 3:
            raise ValueError("xgeo must hold (ngeo+1)^3 nodes of 3 coordinates per element")
        bc_arr = (Bc * max(1, len(bcs)))(*[Bc(b["kind"], b["twall"], b["theta"], (ctypes.c_double * 3)(*b["uwall"]),
                                                 *b["gamma"], (ctypes.c_double * 3)(*b.get("tgrad", (0, 0, 0))),
                                                 b.get("trate", 0.0))
                                              for b in bcs])
        ip = ctypes.POINTER(ctypes.c_int)
        m = Mesh(int(nbr.shape[0]), int(ngeo), xgeo.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                 nbr.ctypes.data_as(ip), nbf.ctypes.data_as(ip), None if nbo is None else nbo.ctypes.data_as(ip),
                 bc.ctypes.data_as(ip), len(bcs), bc_arr)
        self._check(self.L.nskr_mesh_upload(self._h, ctypes.byref(m), _stream_ptr(stream)))
        n = ctypes.c_size_t()
        self._check(self.L.nskr_state_size(self._h, ctypes.byref(n)))
        self.nnodes = n.value // 6
        self.nelems = int(nbr.shape[0])

    def set_time(self, t):
        """Simulation time for walls whose temperature changes in time
        (rk_steps advances it by nsteps dt)."""
        self._check(self.L.nskr_set_time(self._h, float(t)))

    def get_time(self):
        t = ctypes.c_double()
        self._check(self.L.nskr_get_time(self._h, ctypes.byref(t)))
        return t.value

    def device_bytes(self):
        b = ctypes.c_size_t()
        self._check(self.L.nskr_device_bytes(self._h, ctypes.byref(b)))
        return b.value

    def new_state(self):
        import torch
        return torch.empty((6, self.nnodes), dtype=self.dtype, device=f"cuda:{self.device}")

    def _state_ok(self, U, rows=6):
        import torch
        if not (isinstance(U, torch.Tensor) and U.is_cuda and U.dtype == self.dtype and U.is_contiguous()
                and U.numel() == rows * self.nnodes):
            raise ValueError(f"expected a contiguous {self.dtype} CUDA tensor with {rows} x {self.nnodes} values")
        return ctypes.c_void_p(U.data_ptr())

    def init_droplets(self, U, T0, centres, radii, width, noise=None, stream=None, velocities=None, rho_v=0.0,
                      rho_l=0.0, cylinder_axis=-1):
        cen = np.ascontiguousarray(np.asarray(centres, dtype=np.float64).reshape(-1, 3))
        rad = np.ascontiguousarray(np.asarray(radii, dtype=np.float64).reshape(-1))
        vel = None
        if velocities is not None:
            vel = np.ascontiguousarray(np.asarray(velocities, dtype=np.float64).reshape(-1, 3))
            if vel.shape[0] != rad.size:
                raise ValueError("one velocity per droplet")
        dp = ctypes.POINTER(ctypes.c_double)
        ic = Init(float(T0), int(rad.size), cen.ctypes.data_as(dp), rad.ctypes.data_as(dp), float(width),
                  (ctypes.c_double * 3)(*self.box["length"]), (ctypes.c_int * 3)(*self.box["periodic"]),
                  vel.ctypes.data_as(dp) if vel is not None else None, float(rho_v), float(rho_l),
                  int(cylinder_axis))
        nz = None
        if noise is not None:
            nz = np.ascontiguousarray(noise, dtype=np.float64)
            if nz.size != self.nnodes:
                raise ValueError("noise must have one value per node")
        self._check(self.L.nskr_init_droplets(self._h, ctypes.byref(ic),
                                              nz.ctypes.data_as(dp) if nz is not None else None,
                                              self._state_ok(U), _stream_ptr(stream)))
        return U

    def rhs(self, U, Ut, stream=None):
        self._check(self.L.nskr_rhs(self._h, self._state_ok(U), self._state_ok(Ut), _stream_ptr(stream)))
        return Ut

    def lift1(self, U, q, stream=None):
        self._check(self.L.nskr_lift1(self._h, self._state_ok(U), self._state_ok(q, 15), _stream_ptr(stream)))
        return q

    def lift2(self, U, out, stream=None):
        self._check(self.L.nskr_lift2(self._h, self._state_ok(U), self._state_ok(out, 5), _stream_ptr(stream)))
        return out

    def dt(self, U, stream=None) -> float:
        v = ctypes.c_double()
        self._check(self.L.nskr_dt(self._h, self._state_ok(U), ctypes.byref(v), _stream_ptr(stream)))
        return v.value

    def dt_noalloc(self, U, stream=None) -> float:
        """dt() through the entry point that allocates nothing (static device
        reduction scratch shared by every call on the device)."""
        v = ctypes.c_double()
        self._check(self.L.nskr_dt_noalloc(self._h, self._state_ok(U), ctypes.byref(v), _stream_ptr(stream)))
        return v.value

    def rk_steps(self, U, R, dt, nsteps=1, stream=None):
        self._check(self.L.nskr_rk_steps(self._h, self._state_ok(U), self._state_ok(R), float(dt), int(nsteps),
                                         _stream_ptr(stream)))

    def reduce(self, U, stream=None, check=True):
        out = (ctypes.c_double * NSKR_NSUMS)()
        rc = self.L.nskr_reduce(self._h, self._state_ok(U), out, _stream_ptr(stream))
        vals = np.array(out[:])
        if rc != NSKR_OK and (check or rc != NSKR_E_NONFINITE):
            raise NskrError(rc, self.L.nskr_last_error(self._h).decode())
        return vals


class Batch:
    """Many independent instances advanced together (one RK step per call),
    grouped by degree/precision/block size, captured into a HIP graph."""

    def __init__(self, budget_bytes: int, device: int = 0, graph: bool = True):
        self.L = lib()
        h = ctypes.c_void_p()
        rc = self.L.nskr_batch_create(int(device), int(budget_bytes), ctypes.byref(h))
        if rc != NSKR_OK:
            raise NskrError(rc, "nskr_batch_create failed")
        self._h = h
        self.device = device
        self.L.nskr_batch_set_graph(h, 1 if graph else 0)
        self._held = {}

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self.L.nskr_batch_destroy(h)
            self._h = None

    def _err(self, rc):
        raise NskrError(rc, self.L.nskr_batch_last_error(self._h).decode())

    def admit(self, solver: "Solver", U, R, dt: float, nsteps: int):
        """Slot index, or None when the memory budget has no room now."""
        slot = ctypes.c_int()
        rc = self.L.nskr_batch_admit(self._h, solver._h, solver._state_ok(U), solver._state_ok(R), float(dt),
                                     int(nsteps), ctypes.byref(slot))
        if rc == NSKR_E_NOMEM:
            return None
        if rc != NSKR_OK:
            self._err(rc)
        self._held[slot.value] = (solver, U, R)
        return slot.value

    def step(self, stream):
        rc = self.L.nskr_batch_step(self._h, _stream_ptr(stream))
        if rc != NSKR_OK:
            self._err(rc)

    def poll(self):
        n = ctypes.c_int()
        cap = 4096
        arr = (ctypes.c_int * cap)()
        rc = self.L.nskr_batch_poll(self._h, arr, cap, ctypes.byref(n))
        if rc != NSKR_OK:
            self._err(rc)
        return [arr[k] for k in range(min(n.value, cap))]

    def retire(self, slot):
        rc = self.L.nskr_batch_retire(self._h, int(slot))
        if rc != NSKR_OK:
            self._err(rc)
        return self._held.pop(slot, None)

    def info(self):
        used, act, steps = ctypes.c_size_t(), ctypes.c_int(), ctypes.c_long()
        self.L.nskr_batch_info(self._h, ctypes.byref(used), ctypes.byref(act), ctypes.byref(steps))
        return {"used_bytes": used.value, "active": act.value, "steps": steps.value}


def _profile_methods():
    def set_profiling(self, on=True):
        self._check(self.L.nskr_set_profiling(self._h, 1 if on else 0))

    def profile(self, stream=None):
        ms = (ctypes.c_double * 5)()
        cnt = (ctypes.c_long * 5)()
        self._check(self.L.nskr_profile(self._h, ms, cnt, _stream_ptr(stream)))
        return {k: (ms[i], cnt[i]) for i, k in enumerate(KERNEL_KINDS)}

    def set_block(self, threads):
        self._check(self.L.nskr_set_block(self._h, int(threads)))

    def get_block(self):
        v = ctypes.c_int()
        self._check(self.L.nskr_get_block(self._h, ctypes.byref(v)))
        return v.value

    Solver.set_profiling = set_profiling
    Solver.profile = profile
    Solver.set_block = set_block
    Solver.get_block = get_block


_profile_methods()


def solver_for(w, precision="fp64", device=0, kahan=True):
    """Solver with the mesh of a workload description (paper_2208_05310_amd.workloads)."""
    s = Solver(w.params, w.N, precision, device, kahan)
    ngeo = (w.ngeo or w.N) if w.curve_amp != 0.0 else max(w.ngeo, 1)
    s.upload_box(w.n, w.length, w.periodic, w.side_kind, w.side_twall, w.side_theta,
                 side_uwall=w.side_uwall, side_gamma=w.side_gamma, side_tgrad=w.side_tgrad, side_trate=w.side_trate,
                 curve_amp=w.curve_amp, ngeo=ngeo)
    return s


def init_workload(s: Solver, w, U=None):
    if U is None:
        U = s.new_state()
    return s.init_droplets(U, w.T0, w.centres, w.radii, w.width, w.noise(), velocities=w.velocities,
                           rho_v=w.rho_v, rho_l=w.rho_l, cylinder_axis=w.cylinder_axis)
