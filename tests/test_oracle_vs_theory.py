"""Mesh-level pins of the oracle: ensemble statistics of the operator-splitting
scheme against (a) the well-mixed chemical master equation, which the RDME's
stationary law of the totals reduces to for A + B <-> C, (b) the Bateman law
of a first-order decay chain, whose totals do not depend on diffusion, and (c)
an independent exact spatial SSA (Gillespie direct method) on a tiny mesh.
Moments are compared within 3 standard errors at 1000 runs or more."""
import math

import numpy as np

from paper_1610_02258_amd import inputs as I
from tests.meshes import model


def _cme_abc_moments(cf_tot, kb, A0, B0):
    n = min(A0, B0)
    logp = np.zeros(n + 1)
    for c in range(n):
        logp[c + 1] = logp[c] + math.log(cf_tot * (A0 - c) * (B0 - c) / (kb * (c + 1)))
    p = np.exp(logp - logp.max())
    p /= p.sum()
    k = np.arange(n + 1)
    mean = (k * p).sum()
    return mean, ((k - mean) ** 2 * p).sum()


def _abc_equilibrium(O, kf, kb, A0, B0, t_end, runs, tau_factor=1.0):
    mesh = I.box_mesh(2, 2, 2, 1e-6)
    md = model([1e-12] * 3, [(["A", "B"], ["C"], kf), (["C"], ["A", "B"], kb)], ["A", "B", "C"])
    base = O.Instance(mesh.as_dict(), md, 0)
    inst = O.Instance(mesh.as_dict(), md, 0, tau_override=base.tau * tau_factor)
    nav_tot = base.geometry()["nav"].sum()
    mean, var = _cme_abc_moments(kf / nav_tot, kb, A0, B0)
    c_tot = np.zeros(runs)
    for r in range(runs):
        counts = I.place_uniform(mesh, [A0, B0, 0], seed=10_000 + r)
        inst.reset(counts, seed=r)
        inst.run(t_end)
        c_tot[r] = inst.counts[2].sum()
    return c_tot, mean, var


def test_abc_equilibrium_on_mesh_matches_well_mixed_cme(oracle_lib):
    """Reaction-limited regime (per-tet c_f = 1.2/s against d = 34/s) at the
    method's own tau: mean and variance of total C within 3 SE at 1000 runs."""
    runs = 1000
    c_tot, mean, var = _abc_equilibrium(oracle_lib, 1.2e8, 1.0, 30, 30, 8.0, runs)
    se_mean = math.sqrt(var / runs)
    se_var = var * math.sqrt(2.0 / (runs - 1))
    assert abs(c_tot.mean() - mean) < 3 * se_mean, (c_tot.mean(), mean, se_mean)
    assert abs(c_tot.var(ddof=1) - var) < 3 * se_var, (c_tot.var(ddof=1), var, se_var)


def test_abc_equilibrium_diffusion_limited_converges_with_tau(oracle_lib):
    """Diffusion-limited regime (per-tet c_f = 12/s against d = 34/s): at the
    method's tau the operator-splitting mean of C sits about 3% above the CME
    (a splitting error of the scheme, documented); at tau/32 it agrees within
    3 SE at 1000 runs, as a consistent splitting scheme must."""
    runs = 1000
    c_tot, mean, var = _abc_equilibrium(oracle_lib, 1.2e9, 10.0, 30, 30, 2.0, runs, 1.0 / 32)
    se_mean = math.sqrt(var / runs)
    assert abs(c_tot.mean() - mean) < 3 * se_mean, (c_tot.mean(), mean, se_mean)


def test_decay_chain_totals_follow_bateman_law(oracle_lib):
    """X -> Y -> Z with diffusion: each molecule's fate is independent of where
    it is, so the totals are Multinomial with the Bateman probabilities."""
    mesh = I.box_mesh(2, 2, 1, 1e-6, jitter=0.1, seed=5)
    k1, k2 = 6.0, 2.5
    md = model([1e-12, 3e-13, 1e-12], [(["X"], ["Y"], k1), (["Y"], ["Z"], k2)], ["X", "Y", "Z"])
    inst = oracle_lib.Instance(mesh.as_dict(), md, 0)
    X0, runs, t = 60, 1000, 0.25
    px = math.exp(-k1 * t)
    py = k1 / (k2 - k1) * (math.exp(-k1 * t) - math.exp(-k2 * t))
    tot = np.zeros((runs, 3))
    for r in range(runs):
        counts = I.place_uniform(mesh, [X0, 0, 0], seed=r)
        inst.reset(counts, seed=5000 + r)
        inst.run(t)
        tot[r] = inst.counts.sum(1)
        assert tot[r].sum() == X0
    for j, p in enumerate([px, py, 1 - px - py]):
        se = math.sqrt(X0 * p * (1 - p) / runs)
        assert abs(tot[:, j].mean() - X0 * p) < 3 * se
        assert abs(tot[:, j].var(ddof=1) - X0 * p * (1 - p)) < 3 * X0 * p * (1 - p) * math.sqrt(2 / runs) + 0.2


def test_against_exact_spatial_ssa(oracle_lib):
    """A + B <-> C with diffusion on a 12-tet mesh, uniform start: ensemble
    means and variances of the totals, and the per-tet mean of A, at fixed
    times agree with Gillespie's direct method on the same mesh and model."""
    mesh = I.box_mesh(1, 1, 2, 1e-6, jitter=0.1, seed=6)
    kf, kb = 4e7, 5.0
    md = model([1e-12, 0.5e-12, 0.8e-12], [(["A", "B"], ["C"], kf), (["C"], ["A", "B"], kb)],
               ["A", "B", "C"])
    inst = oracle_lib.Instance(mesh.as_dict(), md, 0)
    tau = inst.tau
    t_rec = np.array([6 * tau, 20 * tau])
    runs = 1000
    os_rec = np.zeros((runs, 2, 3, inst.T))
    ex_rec = np.zeros((runs, 2, 3, inst.T))
    for r in range(runs):
        counts = I.place_uniform(mesh, [40, 30, 0], seed=20_000 + r)
        inst.reset(counts, seed=r)
        inst.step(6)
        os_rec[r, 0] = inst.counts
        inst.step(14)
        os_rec[r, 1] = inst.counts
        ex_rec[r] = oracle_lib.rdme_direct(inst, counts, t_rec, seed=777 + r)
    for ti in range(2):
        a = os_rec[:, ti].sum(2)   # totals per species
        b = ex_rec[:, ti].sum(2)
        se = np.sqrt(a.var(0, ddof=1) / runs + b.var(0, ddof=1) / runs)
        assert np.all(np.abs(a.mean(0) - b.mean(0)) < 3 * se + 1e-12), (ti, a.mean(0), b.mean(0), se)
        va, vb = a[:, 2].var(ddof=1), b[:, 2].var(ddof=1)
        assert abs(va - vb) < 3 * math.sqrt(2 / (runs - 1)) * max(va, vb)
    # spatial profile of A at the later time
    a = os_rec[:, 1, 0]
    b = ex_rec[:, 1, 0]
    se = np.sqrt(a.var(0, ddof=1) / runs + b.var(0, ddof=1) / runs)
    z = np.abs(a.mean(0) - b.mean(0)) / se
    assert z.max() < 3.5, z


def test_tree_selection_ssa_matches_direct(oracle_lib):
    """The exact SSA with sum-tree selection (the benchmark's serial-SSA
    context baseline) has the law of the plain direct method: A + B <-> C
    with diffusion on a 12-tet mesh, means and variances of the totals and
    the per-tet mean of A at a fixed time within 3 SE at 1000 runs each."""
    mesh = I.box_mesh(1, 1, 2, 1e-6, jitter=0.1, seed=6)
    md = model([1e-12, 0.5e-12, 0.8e-12], [(["A", "B"], ["C"], 4e7), (["C"], ["A", "B"], 5.0)],
               ["A", "B", "C"])
    inst = oracle_lib.Instance(mesh.as_dict(), md, 0)
    t_rec = [20 * inst.tau]
    runs = 1000
    a = np.zeros((runs, 3, inst.T))
    b = np.zeros((runs, 3, inst.T))
    for r in range(runs):
        counts = I.place_uniform(mesh, [40, 30, 0], seed=30_000 + r)
        a[r] = oracle_lib.rdme_direct(inst, counts, t_rec, seed=100 + r)[0]
        b[r] = oracle_lib.rdme_direct(inst, counts, t_rec, seed=5000 + r, method="tree")[0]
    ta, tb = a.sum(2), b.sum(2)
    se = np.sqrt(ta.var(0, ddof=1) / runs + tb.var(0, ddof=1) / runs)
    assert np.all(np.abs(ta.mean(0) - tb.mean(0)) < 3 * se + 1e-12), (ta.mean(0), tb.mean(0), se)
    va, vb = ta[:, 2].var(ddof=1), tb[:, 2].var(ddof=1)
    assert abs(va - vb) < 3 * math.sqrt(2 / (runs - 1)) * max(va, vb)
    pa, pb = a[:, 0], b[:, 0]
    z = np.abs(pa.mean(0) - pb.mean(0)) / np.sqrt(pa.var(0, ddof=1) / runs + pb.var(0, ddof=1) / runs)
    assert z.max() < 3.5, z
