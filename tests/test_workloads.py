"""The seeded synthetic inputs (CPU): sizes of the benchmark workloads,
droplet placement rules, noise, and the request stream's distributions.
Both the HIP path and the oracle are driven from these descriptions, so a
change here changes every parity case and benchmark."""
import itertools

import numpy as np
import pytest

from paper_2208_05310_amd import workloads as wl


@pytest.mark.parametrize("make,nodes,N,T0", [
    (wl.c1, 4 ** 3 * 4 ** 3, 3, 0.85),
    (wl.c2, 16 ** 3 * 5 ** 3, 4, 0.85),
    (wl.c3, 32 ** 3 * 6 ** 3, 5, 0.9),
    (wl.c4, 48 * 48 * 24 * 4 ** 3, 3, 0.85),
    (wl.c5, 50 ** 3 * 4 ** 3, 3, 0.85),
])
def test_benchmark_workload_sizes(make, nodes, N, T0):
    w = make()
    assert w.nnodes == nodes and w.N == N and w.T0 == T0
    if make is not wl.c5:
        assert w.params == wl.TABLE1


def test_sizes_of_the_named_configurations():
    assert wl.c2().nnodes == 512000
    assert wl.c3().nnodes == 7077888
    assert wl.c4().nnodes == 3538944


@pytest.mark.parametrize("make,count,rmin,rmax,gap", [(wl.c2, 2, 0.15, 0.15, 0.20), (wl.c3, 8, 0.05, 0.12, 0.20)])
def test_droplets_respect_the_separation_rule(make, count, rmin, rmax, gap):
    w = make()
    assert len(w.centres) == count and len(w.radii) == count
    for c in w.centres:
        assert all(0.0 <= x < 1.0 for x in c)
    for r in w.radii:
        assert rmin <= r <= rmax
    for (c1, r1), (c2, r2) in itertools.combinations(zip(w.centres, w.radii), 2):
        d = np.array(c1) - np.array(c2)
        d -= np.round(d)                       # minimum image in the periodic unit cube
        assert np.linalg.norm(d) >= r1 + r2 + gap - 1e-15


def test_droplet_placement_is_seeded():
    assert wl.c3().centres == wl.c3().centres
    assert wl.random_droplets(7, 3, 0.1, 0.1, 0.1) != wl.random_droplets(8, 3, 0.1, 0.1, 0.1)


def test_noise_is_seeded_uniform_and_bounded():
    w = wl.c1()
    a, b = w.noise(), w.noise()
    assert np.array_equal(a, b) and a.shape == (w.nnodes,)
    assert np.all(np.abs(a) < w.noise_amp)
    assert abs(a.mean()) < 0.1 * w.noise_amp  # 4096 uniform draws
    assert w.with_(noise_seed=None).noise() is None
    assert not np.array_equal(a, w.with_(noise_seed=2).noise())


def test_sessile_wall_box():
    w = wl.c4()
    assert w.length == (1.0, 1.0, 0.5) and w.periodic == (1, 1, 0)
    assert w.side_kind[4] == wl.NOSLIP_CA and w.side_kind[5] == wl.SLIP
    assert w.side_twall[4] == 0.9 and w.side_theta[4] == 60.0
    # cube elements: the box is 1 x 1 x 0.5 with 48 x 48 x 24 elements
    assert {w.length[d] / w.n[d] for d in range(3)} == {1.0 / 48}
    assert wl.c4(scale=8).n == (6, 6, 3)


def test_request_stream_distributions():
    reqs = wl.serving_stream(seed=5, count=256, rate=50.0)
    assert reqs == wl.serving_stream(seed=5, count=256, rate=50.0)
    t = np.array([r[0] for r in reqs])
    assert np.all(np.diff(t) > 0)
    # mean inter-arrival 1/rate within a few standard errors (0.02 s / sqrt(256))
    assert abs(np.diff(np.concatenate([[0.0], t])).mean() - 0.02) < 4 * 0.02 / 16
    ws = [r[1] for r in reqs]
    assert {w.n[0] for w in ws} == {4, 8, 12, 16}
    assert {w.N for w in ws} == {2, 3, 4, 5}
    assert all(0.80 <= w.T0 <= 0.95 and w.steps == 200 for w in ws)
    walls = [w for w in ws if w.periodic == (1, 1, 0)]
    assert 0.35 < len(walls) / len(ws) < 0.65
    for w in walls:
        assert 45.0 <= w.side_theta[4] <= 135.0 and w.side_twall[4] == w.T0
    assert len({w.noise_seed for w in ws}) == len(ws)


def test_collision_workload_matches_tables_4_and_5():
    for regime, (u_rel, mu) in (("reflexive", (2.2, 6.944e-4)), ("toroidal", (4.0, 1.010e-3))):
        w = wl.c5(regime=regime)
        assert w.params["mu"] == mu and w.params["alpha"] == 200.0 and w.params["beta"] == 1000.0
        assert w.params["gam"] == 1.0 / 6000.0 and w.params["kappa"] == 1.0 / 150.0 and w.params["cv"] == 5.0
        assert (w.rho_v, w.rho_l, w.T0, w.radii) == (0.3537, 1.8493, 0.85, (0.1, 0.1))
        assert w.width == 0.0772 / 4
        # relative velocity u_rel along x, droplets approaching each other
        (v1, v2) = w.velocities
        assert v1[0] - v2[0] == u_rel and v1[0] > 0 > v2[0] and w.centres[0][0] < w.centres[1][0]
