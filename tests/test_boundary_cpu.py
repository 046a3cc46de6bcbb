"""Host-side checks of the C-ABI library that need no GPU: the library loads,
exports every entry point the header declares, and rejects bad meshes and
options before touching the device."""

import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2002_04353_amd import alelb, cases, meshgen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "alelb.h")
HEADER_MLP = os.path.join(ROOT, "include", "alelb_mlp.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(alelb.LIB_PATH):
        from paper_2002_04353_amd import build
        build.build()
    return alelb.load()


def test_exports_every_declared_symbol(lib):
    from paper_2002_04353_amd import mlp
    decl = set(re.findall(r"\b(ale_lb_\w+)\s*\(", open(HEADER).read()))
    decl_mlp = set(re.findall(r"\b(ale_mlp_\w+)\s*\(", open(HEADER_MLP).read()))
    out = subprocess.run(["nm", "-D", "--defined-only", alelb.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (ale_(?:lb|mlp)_\w+)", out))
    assert decl and decl_mlp, "no declarations parsed"
    assert decl | decl_mlp <= exported, (decl | decl_mlp) - exported
    assert set(alelb.SYMBOLS) <= decl
    assert set(mlp.SYMBOLS) <= decl_mlp
    for name in decl | decl_mlp:
        assert hasattr(lib, name)


def _create(mesh_arrays, params, **kw):
    return alelb.Solver(mesh_arrays, params, **kw)


def test_rejects_invalid_meshes_on_the_host(lib):
    c = cases.small("plunge", n_nodes=4000)
    m = c["mesh"].arrays()
    bad = dict(m)
    bad["nbr"] = m["nbr"].copy()
    bad["nbr"][0, 0] = m["nbr"][0, 0] + 1 if m["nbr"][0, 0] >= 0 else 5
    with pytest.raises(alelb.AleLbError) as e:
        _create(bad, c["params"])
    assert e.value.code == alelb.EMESH
    bad = dict(m)
    el = m["elem"].copy()
    el[3, [1, 2]] = el[3, [2, 1]]  # clockwise triangle
    bad["elem"] = el
    with pytest.raises(alelb.AleLbError) as e:
        _create(bad, c["params"])
    assert e.value.code == alelb.EMESH
    bad = dict(m)
    el = m["elem"].copy()
    el[7, 4] = 10 ** 8
    bad["elem"] = el
    with pytest.raises(alelb.AleLbError) as e:
        _create(bad, c["params"])
    assert e.value.code == alelb.EMESH
    bad = dict(m)
    bad["wall_edges"] = np.array([[0, 0]], dtype=np.int32) if m["nbr"][0, 0] != -1 else m["wall_edges"][:0]
    if bad["wall_edges"].size:
        with pytest.raises(alelb.AleLbError) as e:
            _create(bad, c["params"])
        assert e.value.code == alelb.EMESH


def test_rejects_bad_options(lib):
    c = cases.small("vortex", n=12)
    p = dict(c["params"])
    p["dt"] = -1.0
    with pytest.raises(alelb.AleLbError) as e:
        _create(c["mesh"].arrays(), p)
    assert e.value.code == alelb.EINVAL
    p = dict(c["params"])
    p["motion"] = 9
    with pytest.raises(alelb.AleLbError) as e:
        _create(c["mesh"].arrays(), p)
    assert e.value.code == alelb.EINVAL


def test_oracle_and_library_share_no_code():
    """The oracle and the HIP library are independent: neither includes the
    other's headers nor imports the other's modules."""
    csrc = os.path.join(ROOT, "paper_2002_04353_amd", "csrc")
    for f in os.listdir(csrc):
        txt = open(os.path.join(csrc, f)).read()
        assert "oracle" not in txt.lower()
    for f in ("alelb_oracle.c", "alelb_oracle.h", "oracle.py", "mlp_oracle.py"):
        txt = open(os.path.join(ROOT, "oracle", f)).read()
        assert '#include "alelb.h"' not in txt and "alelb_impl" not in txt and "alelb_mlp" not in txt
        assert "import paper_2002_04353_amd" not in txt and "from paper_2002_04353_amd" not in txt
    for f in ("alelb.py", "build.py", "meshgen.py", "cases.py", "mlp.py", "surrogate.py"):
        txt = open(os.path.join(ROOT, "paper_2002_04353_amd", f)).read()
        assert "import oracle" not in txt and "from oracle" not in txt


def test_batch_rejects_mixed_options_on_the_host(lib):
    e = cases.ensemble(n_cases=2, n_min=2000, n_max=2500)
    ms = [m.arrays() for m in e["meshes"]]
    p = [dict(q) for q in e["params"]]
    p[1]["motion"] = "plunge"
    with pytest.raises(alelb.AleLbError) as err:
        alelb.Solver(ms, p)
    assert err.value.code == alelb.EINVAL and "case 1" in str(err.value)
    p = [dict(q) for q in e["params"]]
    p[0]["mu"] = -1.0
    with pytest.raises(alelb.AleLbError) as err:
        alelb.Solver(ms, p)
    assert err.value.code == alelb.EINVAL and "case 0" in str(err.value)
    # a bad mesh in a later case names that case
    bad = dict(ms[1])
    el = ms[1]["elem"].copy()
    el[3, [1, 2]] = el[3, [2, 1]]
    bad["elem"] = el
    with pytest.raises(alelb.AleLbError) as err:
        alelb.Solver([ms[0], bad], e["params"])
    assert err.value.code == alelb.EMESH and "case 1" in str(err.value)
    with pytest.raises(alelb.AleLbError) as err:
        alelb.Solver(ms[:1], e["params"])
    assert err.value.code == alelb.EINVAL


def test_rejects_invalid_quadrilateral_meshes_on_the_host(lib):
    c = cases.small("vortex", n=8, elem="q2")
    m = c["mesh"].arrays()
    # a batch mixes no element kinds
    t = cases.small("vortex", n=8)
    with pytest.raises(alelb.AleLbError) as err:
        alelb.Solver([m, t["mesh"].arrays()], [c["params"], t["params"]])
    assert err.value.code == alelb.EINVAL and "case 1" in str(err.value)
    # clockwise quadrilateral
    bad = dict(m)
    el = m["elem"].copy()
    el[2, :4] = el[2, [0, 3, 2, 1]]
    bad["elem"] = el
    with pytest.raises(alelb.AleLbError) as err:
        _create(bad, c["params"])
    assert err.value.code == alelb.EMESH
    # an edge node away from the middle of its edge (the geometry is bilinear)
    bad = dict(m)
    X = m["X"].copy()
    X[m["elem"][5, 6]] += 0.05
    bad["X"] = X
    with pytest.raises(alelb.AleLbError) as err:
        _create(bad, c["params"])
    assert err.value.code == alelb.EMESH and "bilinear" in str(err.value)
    # a reflex corner
    q = meshgen.structured_square_quads(3, 3, 1.0, 1.0)
    X = q.X.copy()
    X[5] = [0.9, 0.9]
    with pytest.raises(alelb.AleLbError) as err:
        _create(dict(q.arrays(), X=X), c["params"])
    assert err.value.code == alelb.EMESH


def test_ensemble_draws_respect_their_ranges():
    e = cases.ensemble(n_cases=24, n_min=10_000, n_max=40_000, seed=5)
    d = e["motion"]
    for j, k in enumerate(("Ma", "k", "A_deg", "h_c", "phase_h")):
        lo, hi = cases.ENSEMBLE_RANGES[k]
        assert (d[:, j] >= lo).all() and (d[:, j] <= hi).all(), k
    assert len({m.n_nodes for m in e["meshes"]}) > 12
    init = cases.concat_init(e["inits"])
    assert init["rho"].shape == (sum(m.n_nodes for m in e["meshes"]),)


def test_mlp_rejects_bad_shapes_on_the_host(lib):
    """ale_mlp_create checks the network's shape and batch limit before it
    touches the device (the batch's 64-row tiles run along a grid dimension
    of at most 65535)."""
    from paper_2002_04353_amd import mlp
    mlp.load()
    for widths, max_batch in (([5], 16), ([5, 0, 3], 16), ([5, 4097], 16), ([5] * 18, 16), ([5, 8], 0),
                              ([5, 8], 65535 * 64 + 1)):
        with pytest.raises(alelb.AleLbError) as e:
            mlp.MLP(widths, max_batch, stream=0)
        assert e.value.code == alelb.EINVAL, (widths, max_batch)
