"""Test-side helpers: build oracle objects from a workload description."""
import numpy as np

import oracle
from paper_2208_05310_amd import workloads as wl


def oracle_for(w: wl.Workload, threads=None) -> oracle.Oracle:
    p = oracle.make_params(**w.params)
    b = oracle.make_box(w.N, w.n, (0.0, 0.0, 0.0), w.length, w.periodic, w.side_kind,
                        w.side_twall, w.side_theta, w.curve_amp)
    return oracle.Oracle(p, b, threads=threads)


def oracle_init(o: oracle.Oracle, w: wl.Workload) -> np.ndarray:
    return o.init_droplets(w.T0, w.centres, w.radii, w.width, w.noise(), w.velocities, w.rho_v, w.rho_l)
