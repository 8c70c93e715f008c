"""Pins of the oracle's setup step (section 2.1): mesh adjacency, volumes,
face couplings g = A/(V h) and the window tau = min 1/d_{S,tet}, against
closed forms of the 6-tet cube split and invariants of any mesh."""
import math

import numpy as np
import pytest

from paper_1610_02258_amd import inputs as I
from tests.meshes import mirror_pair


def _inst(O, mesh, D=1e-12, tau=0.0):
    model = dict(D=np.array([D]), lhs=np.zeros((0, 1), np.int32), rhs=np.zeros((0, 1), np.int32),
                 kcst=np.zeros((1, 0)))
    return O.Instance(mesh, model, seed=1, tau_override=tau)


def test_unjittered_cube_closed_forms(oracle_lib):
    h = 1e-6
    mesh = I.box_mesh(3, 3, 3, h)
    inst = _inst(oracle_lib, mesh.as_dict())
    geo = inst.geometry()
    T = inst.T
    assert T == 162
    np.testing.assert_allclose(geo["vol"], h**3 / 6, rtol=1e-14)
    # faces opposite the diagonal ends (local 0 and 3) lie in cube faces; the
    # other two are interior to the cube
    np.testing.assert_allclose(geo["area"][:, [0, 3]], h * h / 2, rtol=1e-14)
    np.testing.assert_allclose(geo["area"][:, [1, 2]], math.sqrt(2) * h * h / 2, rtol=1e-14)
    inner = geo["nbr"] >= 0
    assert inner[:, 1].all() and inner[:, 2].all()
    dist = geo["dist"]
    np.testing.assert_allclose(dist[:, [1, 2]], math.sqrt(2) * h / 4, rtol=1e-13)
    np.testing.assert_allclose(dist[:, [0, 3]][inner[:, [0, 3]]], math.sqrt(6) * h / 4, rtol=1e-13)
    g = geo["g"]
    np.testing.assert_allclose(g[:, [1, 2]], 12 / h**2, rtol=1e-13)
    np.testing.assert_allclose(g[:, [0, 3]][inner[:, [0, 3]]], 2 * math.sqrt(6) / h**2, rtol=1e-13)
    assert np.all(g[~inner] == 0)
    # tau = 1/(D * max G), max G for a fully interior tet = 24 + 4 sqrt 6 (in 1/h^2)
    assert inst.tau == pytest.approx(h * h / (1e-12 * (24 + 4 * math.sqrt(6))), rel=1e-13)


def test_box_counts_and_neighbours(oracle_lib):
    mesh = I.box_mesh(6, 6, 6, 1e-6)
    geo = _inst(oracle_lib, mesh.as_dict()).geometry()
    nb = (geo["nbr"] >= 0).sum(1)
    # 6x6x6 box: 432 boundary triangles, 2376 interior faces
    assert (geo["nbr"] < 0).sum() == 6 * 36 * 2
    assert (geo["nbr"] >= 0).sum() == 2 * 2376
    assert np.bincount(nb, minlength=5).tolist() == [0, 0, 36, 360, 900]


@pytest.mark.parametrize("jitter", [0.0, 0.1])
def test_invariants(oracle_lib, jitter):
    h = 0.5e-6
    mesh = I.box_mesh(4, 3, 5, h, jitter=jitter, seed=11)
    inst = _inst(oracle_lib, mesh.as_dict())
    geo = inst.geometry()
    T = inst.T
    # volumes tile the box exactly (boundary vertices are not moved)
    assert geo["vol"].sum() == pytest.approx(4 * 3 * 5 * h**3, rel=1e-12)
    nbr = geo["nbr"]
    for i in range(T):
        for k in range(4):
            j = nbr[i, k]
            if j < 0:
                continue
            back = np.nonzero(nbr[j] == i)[0]
            assert back.size == 1
            kb = back[0]
            # shared face: same area, same barycentre distance, V_i g_ij = V_j g_ji
            assert geo["area"][i, k] == pytest.approx(geo["area"][j, kb], rel=1e-12)
            assert geo["dist"][i, k] == geo["dist"][j, kb]
            assert geo["vol"][i] * geo["g"][i, k] == pytest.approx(geo["vol"][j] * geo["g"][j, kb], rel=1e-12)
    # G is the sum of the couplings; the cumulative split fractions step by g_k/G
    np.testing.assert_allclose(geo["G"], geo["g"].sum(1), rtol=1e-14)
    cum = geo["cum"]
    assert np.all(cum[:, 3] == 1.0)
    step = np.diff(np.concatenate([np.zeros((T, 1)), cum[:, :3]], 1), axis=1)
    np.testing.assert_allclose(step, geo["g"][:, :3] / geo["G"][:, None], rtol=1e-12, atol=1e-15)
    last = np.array([max([k for k in range(4) if geo["g"][i, k] > 0]) for i in range(T)])
    np.testing.assert_allclose(cum[np.arange(T), np.minimum(last, 2)] * (last < 3) + (last == 3),
                               np.where(last < 3, 1.0, 1.0), rtol=1e-12)
    # N_A V[L]
    np.testing.assert_allclose(geo["nav"], 6.02214076e23 * geo["vol"] * 1e3, rtol=1e-15)
    assert inst.tau == pytest.approx(1.0 / (1e-12 * geo["G"].max()), rel=1e-15)


def test_mesh_errors(oracle_lib):
    m = mirror_pair()
    bad = dict(m)
    bad["tets"] = np.array([[0, 1, 2, 3], [0, 1, 2, 4], [0, 1, 2, 3]], np.int32)
    with pytest.raises(oracle_lib.OracleError) as e:
        _inst(oracle_lib, bad)
    assert e.value.code == -2
    flat = dict(m)
    flat["verts"] = m["verts"].copy()
    flat["verts"][3, 2] = 0.0  # tet 0 degenerates
    with pytest.raises(oracle_lib.OracleError):
        _inst(oracle_lib, flat)
    # no diffusive species and no override
    with pytest.raises(oracle_lib.OracleError) as e:
        _inst(oracle_lib, m, D=0.0)
    assert e.value.code == -3
    assert _inst(oracle_lib, m, D=0.0, tau=0.5).tau == 0.5
