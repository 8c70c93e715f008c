"""The synthetic workloads against the recipe they stand for: sizes, species
and reaction tables, rate ranges, totals, placement in proportion to volume,
mesh conformity and connectivity, the influx region, the ensemble's size
range and the request stream's arrival law.  CPU only (the oracle provides
the neighbour tables and tau)."""
import math

import numpy as np
import pytest
from scipy import sparse, stats
from scipy.sparse import csgraph

from paper_1610_02258_amd import inputs as I


def _faces(tets):
    f = np.concatenate([np.delete(tets, k, axis=1) for k in range(4)])
    return np.sort(f, axis=1)


def test_box_mesh_is_conforming_and_fills_the_box():
    nx, ny, nz, h = 3, 4, 5, 1e-6
    m = I.box_mesh(nx, ny, nz, h, jitter=0.1, seed=7)
    assert m.n_tets == 6 * nx * ny * nz
    vol = I.tet_volumes_for_sampling(m)
    assert vol.min() > 0.05 * h ** 3 / 6  # no flat or inverted tet after the jitter
    assert vol.sum() == pytest.approx(nx * ny * nz * h ** 3, rel=1e-12)
    # every face is shared by two tets except the box surface, two triangles
    # per cube face
    _, cnt = np.unique(_faces(m.tets), axis=0, return_counts=True)
    assert set(cnt.tolist()) <= {1, 2}
    assert (cnt == 1).sum() == 2 * 2 * (nx * ny + ny * nz + nx * nz)


def test_small_box_workload(oracle_lib):
    w = I.config_small()
    assert w.mesh.n_tets == 1296 and w.model.S == 3 and w.model.R == 2
    np.testing.assert_array_equal(w.counts.sum(axis=1), [2000, 2000, 0])
    assert w.t_end == 10e-3
    np.testing.assert_array_equal(I.config_small().counts, w.counts)  # seeded
    assert w.model.kcst[0].tolist() == [1e6, 10.0]
    assert np.all(w.model.D == 1e-12)
    tau = oracle_lib.Instance(w.mesh.as_dict(), w.model.as_dict(), w.seed).tau
    assert tau > w.t_end  # one truncated window


def test_placement_is_proportional_to_volume():
    m = I.box_mesh(6, 6, 6, 1e-6, jitter=0.3, seed=3)
    vol = I.tet_volumes_for_sampling(m)
    n = 400_000
    for place in (I.place_uniform, I.place_by_choice):
        c = place(m, [n], 11)[0]
        assert c.sum() == n
        exp = n * vol / vol.sum()
        assert stats.chisquare(c, exp).pvalue > 1e-3, place.__name__
    # and not in proportion to count: a volume-blind placement fails
    flat = np.random.default_rng(1).multinomial(n, np.full(m.n_tets, 1.0 / m.n_tets))
    assert stats.chisquare(flat, n * vol / vol.sum()).pvalue < 1e-6


def test_simple_model_workload(oracle_lib):
    w = I.config_simple()
    md = w.model
    assert w.mesh.n_tets == 480_000 and w.mesh.info["h"] == pytest.approx(0.5e-6)
    assert md.S == 10 and md.R == 12
    assert w.counts.sum() == 1_000_000 and w.t_end == 100e-3
    assert np.all((md.D >= 1e-13) & (md.D <= 1e-11)) and np.isclose(md.D.max(), 1e-11)
    order = md.lhs.sum(axis=1)
    np.testing.assert_array_equal(order, [1, 2] * 6)  # alternating uni- and bimolecular
    k = md.kcst[0]
    assert np.all((k[order == 1] >= 0.1) & (k[order == 1] <= 100.0))
    assert np.all((k[order == 2] >= 1e5) & (k[order == 2] <= 1e8))
    tau = oracle_lib.Instance(w.mesh.as_dict(), md.as_dict(), w.seed).tau
    assert tau == pytest.approx(0.456e-3, rel=0.01)
    assert math.ceil(w.t_end / tau) == 220


def test_dendrite_workload(oracle_lib):
    w = I.config_dendrite()
    md, m = w.model, w.mesh
    assert m.n_tets == 996_564
    assert md.S == 15 and md.R == 20 and md.kcst.shape[0] == 2
    # the zero-order influx acts in region 1 only, the 5% of tets nearest a
    # distal point
    src = np.flatnonzero(md.lhs.sum(axis=1) == 0)
    assert src.size == 1 and md.kcst[0, src[0]] == 0.0 and md.kcst[1, src[0]] > 0.0
    assert abs((m.region == 1).mean() - 0.05) < 0.005
    inst = oracle_lib.Instance(m.as_dict(), md.as_dict(), w.seed)
    assert inst.tau == pytest.approx(7.2e-6, rel=0.01)
    # one face-connected component
    nbr = inst.geometry()["nbr"]
    i, k = np.nonzero(nbr >= 0)
    g = sparse.coo_matrix((np.ones(i.size), (i, nbr[i, k])), shape=(m.n_tets, m.n_tets))
    n_comp, _ = csgraph.connected_components(g, directed=False)
    assert n_comp == 1
    # counts follow the concentrations over the mesh volume
    vol_l = I.tet_volumes_for_sampling(m).sum() * 1e3
    for s, name in enumerate(md.species):
        assert w.counts[s].sum() == int(round(I.CALCIUM_CONC[name] * 6.02214076e23 * vol_l))


def test_ensemble_sizes_and_parameters():
    runs = I.ensemble_runs(n_runs=256)
    T = np.array([r.mesh.n_tets for r in runs])
    assert T.min() >= 216 * 4 and T.max() <= 5e4 * 1.01  # 6 x 6 x n slabs around logU(1e3, 5e4)
    logT = np.log(T)
    assert stats.kstest((logT - math.log(1e3)) / (math.log(5e4) - math.log(1e3)), "uniform").pvalue > 1e-3
    base = I.model_abc_chain().kcst[0]
    scale = np.array([r.model.kcst[0] / base for r in runs])
    assert scale.min() >= 0.5 and scale.max() <= 1.5


def test_request_stream_is_poisson():
    reqs = I.request_stream(n_requests=2000)
    t = np.array([a for a, _ in reqs])
    gaps = np.diff(np.concatenate([[0.0], t]))
    assert gaps.mean() == pytest.approx(1 / 200.0, rel=0.06)
    assert stats.kstest(gaps * 200.0, "expon").pvalue > 1e-3
    assert all(w.model.S == 10 for _, w in reqs[:20])
