import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session")
def oracle_mod():
    from oracle import oracle as O
    O.build(force=not os.path.exists(O.LIB))
    return O


def _families(n):
    """Fields that share a scale: the f_i and the g_i of the 18 population
    rows, the two velocity components of the 4 moment rows, the two
    components of W or X."""
    if n == 18:
        return [list(range(9)), list(range(9, 18))]
    if n == 4:
        return [[0], [1, 2], [3]]
    if n == 2:
        return [[0, 1]]
    return [list(range(n))]


def rel_fields(a, b, axis=0):
    """Largest per-field relative difference between a GPU result `a` and the
    oracle's `b`.

    Each field (one index along `axis`: rho, u_x, u_y, T of the moments; f_i and
    g_i of each direction of the populations; the components of W or X, or of
    a node-major geometry array with axis=-1) is divided by its own largest
    oracle magnitude, so that a small field (a velocity next to a density, a
    diagonal population next to the rest one) is judged on its own scale.  A
    field below 1e-3 of the largest field of its family (the f_i together, the
    g_i together, the velocity components together) is zero in exact
    arithmetic or nearly so (u_y of a flow along x, f_0 at T = 1); its values
    are round-off of the family's magnitude, and it is judged on that."""
    import numpy as np
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if a.ndim == 1:
        a, b, axis = a[None], b[None], 0  # one field
    a = np.moveaxis(a, axis, 0)
    b = np.moveaxis(b, axis, 0)
    assert a.shape == b.shape, (a.shape, b.shape)
    a = a.reshape(a.shape[0], -1)
    b = b.reshape(b.shape[0], -1)
    if b.size == 0:
        return 0.0
    own = np.abs(b).max(axis=1)
    scale = own.copy()
    for fam in _families(a.shape[0]):
        top = own[fam].max()
        for r in fam:
            if own[r] < 1e-3 * top:
                scale[r] = top
    scale = np.maximum(scale, 1e-300)
    return float((np.abs(a - b).max(axis=1) / scale).max())


def assert_forces_match(fg, fo, chord, rtol=1e-10):
    """Wall force parity: pressure and viscous forces, their moments about the
    reference point, and c_L, c_D, c_m.  Each force component is judged on the
    scale of the largest force component, each moment on that scale times the
    chord (the sums cancel between the surfaces), each coefficient on its own
    magnitude with a floor of 1e-3."""
    import numpy as np
    Fs = max(float(np.abs(fo["F_p"]).max()), float(np.abs(fo["F_v"]).max()), 1e-300)
    for k in ("F_p", "F_v"):
        d = float(np.abs(np.asarray(fg[k]) - np.asarray(fo[k])).max())
        assert d <= rtol * Fs, (k, fg[k], fo[k])
    for k in ("M_p", "M_v"):
        assert abs(fg[k] - fo[k]) <= rtol * Fs * chord, (k, fg[k], fo[k])
    for k in ("cl", "cd", "cm"):
        assert abs(fg[k] - fo[k]) <= rtol * max(1e-3, abs(fo[k])), (k, fg[k], fo[k])
