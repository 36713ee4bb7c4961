"""Test-side helpers: build oracle objects from a workload description."""
import numpy as np

import oracle
from paper_2208_05310_amd import workloads as wl


def oracle_for(w: wl.Workload, threads=None) -> oracle.Oracle:
    p = oracle.make_params(**w.params)
    return oracle.Oracle(p, box_for(w), threads=threads)


def box_for(w: wl.Workload) -> oracle.Box:
    g = w.side_gamma or (wl.NO_GAMMA,) * 6
    return oracle.make_box(w.N, w.n, (0.0, 0.0, 0.0), w.length, w.periodic, w.side_kind,
                           w.side_twall, w.side_theta, w.curve_amp,
                           side_uwall=w.side_uwall or ((0.0, 0.0, 0.0),) * 6,
                           side_g1=[v[0] for v in g], side_g2=[v[1] for v in g],
                           side_g3=[v[2] for v in g], side_g4=[v[3] for v in g],
                           side_tgrad=w.side_tgrad or ((0.0, 0.0, 0.0),) * 6, side_trate=w.side_trate or (0.0,) * 6)


def oracle_init(o: oracle.Oracle, w: wl.Workload) -> np.ndarray:
    return o.init_droplets(w.T0, w.centres, w.radii, w.width, w.noise(), w.velocities, w.rho_v, w.rho_l,
                           w.cylinder_axis)


def timed_wall_case():
    # a graded no-slip floor whose temperature also rises in time, and a
    # heat-transfer Navier-slip lid cooling in time
    return wl.c4(scale=12).with_(
        name="timed_walls_4x4x2_N3", side_kind=(0, 0, 0, 0, wl.NOSLIP_CA, wl.NAVIER),
        side_twall=(0.0, 0.0, 0.0, 0.0, 0.85, 0.9), side_theta=(90.0, 90.0, 90.0, 90.0, 60.0, 120.0),
        side_gamma=(wl.NO_GAMMA,) * 5 + ((0.0, 0.05, 0.02, 0.0),),
        side_tgrad=((0.0, 0.0, 0.0),) * 4 + ((0.05, 0.0, 0.0), (0.0, 0.0, 0.0)),
        side_trate=(0.0,) * 4 + (0.3, -0.2))
