"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The C oracle is built a second time with -fsanitize=address,undefined (no
recovery: the first finding aborts) and driven through every entry point the
pins use, in a fresh interpreter with the sanitizer runtime preloaded: a
periodic droplet box, a box with walls of all three kinds and a moving lid, a
curved box with quadratic geometry, relaxation model 2, a wall temperature
changing along the wall and in time, and the thermodynamics.  Any
out-of-bounds access, use after free or undefined operation fails the test.
"""
import os
import subprocess
import sys
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(ROOT, "oracle", "nskr_oracle.c")

DRIVER = r'''
import numpy as np
import oracle
from paper_2208_05310_amd import workloads as wl
from helpers import oracle_for, oracle_init

NAV = wl.NAVIER
cases = [
    wl.c1().with_(name="droplet", n=(2, 2, 2)),
    wl.c4(scale=12).with_(
        name="walls", periodic=(0, 0, 0),
        side_kind=(wl.NOSLIP_CA, wl.SLIP, NAV, wl.NOSLIP_CA, wl.NOSLIP_CA, NAV),
        side_twall=(0.9, 0.0, 0.88, 0.87, 0.9, 0.86), side_theta=(60.0, 90.0, 110.0, 90.0, 60.0, 120.0),
        side_uwall=((0.0, 0.0, 0.0),) * 5 + ((0.2, -0.1, 0.0),),
        side_gamma=(wl.NO_GAMMA,) * 2 + ((0.5, 0.05, 0.02, 0.3),) + (wl.NO_GAMMA,) * 2 +
                   ((0.0, 0.1, 0.01, 0.0),)),
    wl.c1().with_(name="curved", N=4, n=(2, 2, 2), curve_amp=0.05, ngeo=2),
    wl.c5(scale=25).with_(name="model2", params=dict(wl.c5().params, model=2)),
    wl.c4(scale=12).with_(
        name="graded", side_kind=(0, 0, 0, 0, wl.NOSLIP_CA, NAV),
        side_twall=(0.0, 0.0, 0.0, 0.0, 0.85, 0.9), side_theta=(90.0, 90.0, 90.0, 90.0, 60.0, 120.0),
        side_gamma=(wl.NO_GAMMA,) * 5 + ((0.0, 0.05, 0.02, 0.0),),
        side_tgrad=((0.0, 0.0, 0.0),) * 4 + ((0.08, 0.04, 0.0), (-0.05, 0.0, 0.0)),
        side_trate=(0.0,) * 4 + (0.3, -0.2)),
]
for w in cases:
    o = oracle_for(w, threads=2)
    U = oracle_init(o, w)
    q = o.lift1(U)
    l2 = o.lift2(U)
    Ut = o.rhs(U)
    dt = o.dt(U)
    R = np.zeros_like(U)
    o.run(U, R, 0.0, dt, 2)
    s = o.reduce(U)
    assert np.all(np.isfinite(U)) and np.all(np.isfinite(Ut)) and np.isfinite(dt), w.name
    print(w.name, "ok", float(s[0]), flush=True)
rv, rl, p = oracle.maxwell(0.85)
print("maxwell", rv, rl, oracle.sigma(0.85, 1e-4), flush=True)
'''


@pytest.mark.slow
def test_oracle_clean_under_address_and_undefined_sanitizers():
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("no AddressSanitizer runtime for gcc")
    with tempfile.TemporaryDirectory() as d:
        so = os.path.join(d, "liboracle_san.so")
        subprocess.run(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                        "-fno-sanitize-recover=all", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-D_GNU_SOURCE",
                        "-o", so, SRC, "-lm"], check=True, capture_output=True)
        env = dict(os.environ, NSKR_ORACLE_SO=so, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
                   UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", PYTHONPATH=os.pathsep.join([ROOT, HERE]))
        r = subprocess.run([sys.executable, "-c", DRIVER], cwd=ROOT, env=env, capture_output=True, text=True,
                           timeout=900)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-4000:]
    for name in ("droplet", "walls", "curved", "model2", "graded", "maxwell"):
        assert name in r.stdout, out[-4000:]
