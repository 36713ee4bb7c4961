"""CPU checks of the C ABI library: it loads, exports every entry point that
include/nskr.h declares, validates arguments before touching a device, and
the host-side mesh builder produces consistent connectivity."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2208_05310_amd import nskr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "nskr.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(nskr_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_binding_exports():
    assert declared_functions() == sorted(nskr.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = nskr.lib()
    for name in declared_functions():
        assert hasattr(L, name), name
    from paper_2208_05310_amd.nskr import ABI_VERSION
    assert L.nskr_version() == ABI_VERSION == 9


def test_create_validates_arguments_before_device():
    L = nskr.lib()
    good = dict(R=8 / 3, a=3.0, b=1 / 3, cv=5.0, mu=0.01, kappa=1 / 150, gam=1e-4, alpha=100.0, beta=1000.0,
                cfl=0.9)
    h = ctypes.c_void_p()

    def create(N=3, prec=0, model=1, **kw):
        d = dict(good, **kw)
        p = nskr.Params(d["R"], d["a"], d["b"], d["cv"], d["mu"], d["kappa"], d["gam"], d["alpha"], d["beta"],
                        d["cfl"], prec, 0, model)
        return L.nskr_create(ctypes.byref(p), N, 0, ctypes.byref(h))

    assert create(N=1) == nskr.NSKR_E_ARG
    assert create(N=6) == nskr.NSKR_E_ARG
    assert create(mu=-1.0) == nskr.NSKR_E_ARG
    assert create(cv=0.0) == nskr.NSKR_E_ARG
    assert create(cfl=float("nan")) == nskr.NSKR_E_ARG
    assert create(prec=2) == nskr.NSKR_E_ARG
    assert create(model=3) == nskr.NSKR_E_UNSUPPORTED
    assert create(model=-1) == nskr.NSKR_E_UNSUPPORTED
    import torch
    if not torch.cuda.is_available():
        # no device here: a valid request fails with the HIP error, never a CPU fallback
        assert create() == nskr.NSKR_E_HIP


def test_null_context_calls():
    L = nskr.lib()
    assert L.nskr_destroy(None) == nskr.NSKR_OK
    assert L.nskr_last_error(None) == b"nskr: null context"
    assert L.nskr_rhs(None, None, None, None) == nskr.NSKR_E_ARG
    assert L.nskr_rk_steps(None, None, None, 1e-5, 1, None) == nskr.NSKR_E_ARG


@pytest.mark.parametrize("periodic", [(1, 1, 1), (1, 1, 0), (0, 1, 0)])
def test_box_mesh_connectivity(periodic):
    n = (3, 4, 2)
    kinds = tuple(0 if periodic[f // 2] else (1 if f % 2 == 0 else 2) for f in range(6))
    corners, nbr, nbf, bc, bcs = nskr.box_mesh(n, (1.5, 1.0, 0.5), periodic, kinds, (0.9,) * 6, (60.0,) * 6)
    E = n[0] * n[1] * n[2]
    assert corners.shape == (E, 8, 3)
    for e in range(E):
        for f in range(6):
            nb = nbr[e, f]
            if nb >= 0:
                assert nbf[e, f] == f ^ 1 and nbr[nb, f ^ 1] == e and bc[e, f] == 0
            else:
                assert not periodic[f // 2] and 1 <= bc[e, f] <= len(bcs)
                assert bcs[bc[e, f] - 1]["kind"] == kinds[f]
    # elements are axis-aligned boxes of the right size
    h = np.array([0.5, 0.25, 0.25])
    assert np.allclose(corners[:, 7] - corners[:, 0], h)
    assert len(bcs) == sum(1 for f in range(6) if not periodic[f // 2])
