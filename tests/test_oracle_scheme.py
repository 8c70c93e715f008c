"""Pins of the oracle's window scheme (Algorithm 1) against what the paper and
the mathematics fix: the window loop and its truncation, exact conservation,
the deterministic p = 1 swap, the exact per-molecule law of the diffusion
operator, the stationary law pi ~ V, and closed forms of the single-tet
reaction operator (first-order decay, mean occupancy, composition-rejection
branching ratios, bimolecular / homodimer / zero-order stationary laws)."""
import math

import numpy as np
import pytest
from scipy import stats

from paper_1610_02258_amd import inputs as I
from tests.meshes import mirror_pair, model, single_tet


def _chi2_sf(obs, exp, min_exp=5.0):
    obs = np.asarray(obs, float)
    exp = np.asarray(exp, float)
    keep = exp >= min_exp
    o = np.append(obs[keep], obs[~keep].sum())
    e = np.append(exp[keep], exp[~keep].sum())
    if e[-1] < min_exp:
        o[-2] += o[-1]; e[-2] += e[-1]; o = o[:-1]; e = e[:-1]
    return stats.chi2.sf(((o - e) ** 2 / e).sum(), len(o) - 1)


# ------------------------------------------------------------ window loop ----

def test_window_loop_truncation(oracle_lib):
    w = I.config_small()
    inst = oracle_lib.Instance(w.mesh.as_dict(), w.model.as_dict(), 0)
    tau = inst.tau
    inst.reset(w.counts)
    inst.run(10e-3)                  # 10 ms < tau: a single truncated window
    assert inst.window == 1 and inst.t == 10e-3
    inst.run(10e-3)                  # nothing left to do
    assert inst.window == 1
    inst.reset(w.counts)
    inst.run(3.5 * tau)              # three full windows and a half one
    assert inst.window == 4 and inst.t == 3.5 * tau
    inst.reset(w.counts)
    inst.step(5)
    assert inst.window == 5 and inst.tallies.voxel_steps == 5 * inst.T


def test_run_equals_windows(oracle_lib):
    """run(t_end) is the same as explicit windows of tau and a truncated tail."""
    w = I.config_small()
    a = oracle_lib.Instance(w.mesh.as_dict(), w.model.as_dict(), 5)
    b = oracle_lib.Instance(w.mesh.as_dict(), w.model.as_dict(), 5)
    a.reset(w.counts)
    b.reset(w.counts)
    t_end = 2.25 * a.tau
    a.run(t_end)
    b.window_explicit(b.tau, 0)
    b.window_explicit(b.tau, 1)
    b.window_explicit(t_end - 2 * b.tau, 2)
    np.testing.assert_array_equal(a.counts, b.counts)


# ----------------------------------------------------------- conservation ----

def test_conservation(oracle_lib):
    w = I.config_small()
    m = I.model_abc(kf=1e8, kb=10.0)
    inst = oracle_lib.Instance(w.mesh.as_dict(), m.as_dict(), 3)
    inst.reset(w.counts)
    for _ in range(40):
        inst.step(5)
        c = inst.counts
        assert c.min() >= 0
        assert c[0].sum() + c[2].sum() == 2000     # A + C
        assert c[1].sum() + c[2].sum() == 2000     # B + C
    assert inst.tallies.ssa_events > 100


def test_conservation_pure_diffusion_and_determinism(oracle_lib):
    w = I.config_small()
    m = I.model_abc(kf=0.0, kb=0.0)
    a = oracle_lib.Instance(w.mesh.as_dict(), m.as_dict(), 9)
    a.reset(w.counts)
    a.step(30)
    assert a.counts.sum(1).tolist() == [2000, 2000, 0]
    b = oracle_lib.Instance(w.mesh.as_dict(), m.as_dict(), 9)
    b.reset(w.counts)
    b.step(30)
    np.testing.assert_array_equal(a.counts, b.counts)
    c = oracle_lib.Instance(w.mesh.as_dict(), m.as_dict(), 10)
    c.reset(w.counts)
    c.step(30)
    assert not np.array_equal(a.counts, c.counts)


# ------------------------------------------------------------- p = 1 swap ----

def test_mirror_pair_swaps_every_window(oracle_lib):
    mesh = mirror_pair()
    md = model([1e-12], [], ["A"])
    inst = oracle_lib.Instance(mesh, md, 17)
    geo = inst.geometry()
    assert geo["G"][0] == pytest.approx(geo["G"][1], rel=1e-14)
    c0 = np.array([[37, 5]], np.int32)
    inst.reset(c0)
    for k in range(1, 7):
        inst.step(1)
        expect = c0 if k % 2 == 0 else c0[:, ::-1]
        np.testing.assert_array_equal(inst.counts, expect)


# -------------------------------------------------- diffusion operator law ----

def _transition_matrix(inst, D):
    geo = inst.geometry()
    T = inst.T
    P = np.zeros((T, T))
    for i in range(T):
        for k in range(4):
            j = geo["nbr"][i, k]
            if j >= 0:
                P[i, j] += inst.tau * D * geo["g"][i, k]
        P[i, i] = 1.0 - inst.tau * D * geo["G"][i]
    return P, geo


@pytest.mark.parametrize("n0,m", [(10, 1), (200, 1), (30, 4)])
def test_pure_diffusion_matches_markov_law(oracle_lib, n0, m):
    """Without reactions each molecule independently follows P = I - tau L per
    window, so after m windows the counts are Multinomial(n0, e_i0^T P^m).
    n0 = 10 exercises the per-molecule sampler, n0 = 200 the binomial one."""
    mesh = I.box_mesh(1, 1, 2, 1e-6, jitter=0.1, seed=4).as_dict()
    D = 1e-12
    inst = oracle_lib.Instance(mesh, model([D], [], ["A"]), 0)
    P, _ = _transition_matrix(inst, D)
    T = inst.T
    i0, runs = 3, 2000
    q = np.linalg.matrix_power(P, m)[i0]
    c0 = np.zeros((1, T), np.int32)
    c0[0, i0] = n0
    acc = np.zeros(T)
    acc2 = np.zeros(T)
    for r in range(runs):
        inst.reset(c0, seed=1000 + r)
        inst.step(m)
        acc += inst.counts[0]
        acc2 += inst.counts[0].astype(float) ** 2
    # pooled counts ~ Multinomial(n0 * runs, q)
    assert _chi2_sf(acc, n0 * runs * q) > 1e-3
    mean = acc / runs
    var = acc2 / runs - mean**2
    se = np.sqrt(n0 * q * (1 - q) / runs)
    assert np.all(np.abs(mean - n0 * q) <= 3.5 * se + 1e-12)
    np.testing.assert_allclose(var, n0 * q * (1 - q), rtol=0.25, atol=0.05)


def test_stationary_law_is_volume_weighted(oracle_lib):
    mesh = I.box_mesh(1, 2, 1, 1e-6, jitter=0.1, seed=8).as_dict()
    D = 1e-12
    inst = oracle_lib.Instance(mesh, model([D], [], ["A"]), 0)
    P, geo = _transition_matrix(inst, D)
    pi = geo["vol"] / geo["vol"].sum()
    # detailed balance V_j P_jk = V_k P_kj  =>  pi P = pi
    np.testing.assert_allclose(pi @ P, pi, rtol=1e-10)
    T = inst.T
    n0, runs = 24, 800
    c0 = np.zeros((1, T), np.int32)
    c0[0, 0] = n0
    acc = np.zeros(T)
    for r in range(runs):
        inst.reset(c0, seed=77 + r)
        inst.step(300)
        acc += inst.counts[0]
    assert _chi2_sf(acc, n0 * runs * pi) > 1e-3


# -------------------------------------------------- reaction operator pins ----

def test_first_order_decay_is_binomial(oracle_lib):
    """A -> B in one tet: N_A(t) ~ Bin(N0, exp(-k t)); windows chain exactly."""
    k, tau, m, N0, runs = 5.0, 0.05, 6, 40, 3000
    inst = oracle_lib.Instance(single_tet(), model([0, 0], [(["A"], ["B"], k)], ["A", "B"]), 0,
                               tau_override=tau)
    out = np.zeros(runs, int)
    for r in range(runs):
        inst.reset(np.array([[N0], [0]], np.int32), seed=r)
        inst.step(m)
        out[r] = inst.counts[0, 0]
        assert inst.counts[:, 0].sum() == N0
    p = math.exp(-k * tau * m)
    assert _chi2_sf(np.bincount(out, minlength=N0 + 1), runs * stats.binom.pmf(np.arange(N0 + 1), N0, p)) > 1e-3


def test_mean_occupancy_closed_form(oracle_lib):
    """A -> B over one window: E[Nbar_A] = N0 (1 - e^{-k tau}) / (k tau), and a
    species untouched by any event keeps Nbar = N exactly."""
    k, tau, N0, runs = 3.0, 0.2, 50, 4000
    inst = oracle_lib.Instance(single_tet(),
                               model([0, 0, 0], [(["A"], ["B"], k)], ["A", "B", "C"]), 0,
                               tau_override=tau)
    nbarA = np.zeros(runs)
    nbarB = np.zeros(runs)
    for r in range(runs):
        inst.seed = 500 + r
        n, nbar, ev = inst.ssa_only(0, tau, 0, np.array([N0, 0, 7], np.int32))
        assert ev == N0 - n[0]
        assert nbar[2] == 7.0
        nbarA[r], nbarB[r] = nbar[0], nbar[1]
        assert nbar[0] + nbar[1] == pytest.approx(N0, rel=1e-12)
    expect = N0 * (1 - math.exp(-k * tau)) / (k * tau)
    # per molecule: occupancy fraction of A is min(T_life, tau)/tau with T_life ~ Exp(k)
    x = k * tau
    e2 = (2 / x**2) * (1 - math.exp(-x) * (1 + x))  # E[(min(E,tau)/tau)^2]
    e1 = (1 - math.exp(-x)) / x
    var = N0 * (e2 - e1**2)
    se = math.sqrt(var / runs)
    assert abs(nbarA.mean() - expect) < 3 * se


def test_cr_branching_ratios(oracle_lib):
    """Competing first-order channels spread over several propensity groups
    (and two in one group): the product split is Multinomial(N0, k_j / sum k)."""
    ks = [1.0, 10.0, 1000.0, 5.0, 7.0, 0.3]
    prods = ["B", "C", "D", "E", "F", "G"]
    reactions = [(["A"], [p], k) for p, k in zip(prods, ks)]
    sp = ["A"] + prods
    inst = oracle_lib.Instance(single_tet(), model([0] * 7, reactions, sp), 0, tau_override=1.0)
    N0, runs = 500, 300
    tot = np.zeros(6)
    for r in range(runs):
        c0 = np.zeros((7, 1), np.int32)
        c0[0, 0] = N0
        inst.reset(c0, seed=r)
        inst.step(1)
        assert inst.counts[0, 0] == 0
        tot += inst.counts[1:, 0]
    p = np.array(ks) / sum(ks)
    assert _chi2_sf(tot, N0 * runs * p) > 1e-3


def _stationary_pmf(ratio, nmax):
    logp = np.zeros(nmax + 1)
    for c in range(nmax):
        r = ratio(c)
        logp[c + 1] = logp[c] + (math.log(r) if r > 0 else -np.inf)
    p = np.exp(logp - logp.max())
    return p / p.sum()


def test_bimolecular_stationary_law(oracle_lib):
    """A + B <-> C in one tet: P(c+1)/P(c) = c_f (A0-c)(B0-c) / (k_b (c+1)),
    c_f = k_f / (N_A V[L])."""
    kf, kb, A0, B0 = 2e6, 4.0, 12, 9
    inst = oracle_lib.Instance(single_tet(),
                               model([0, 0, 0], [(["A", "B"], ["C"], kf), (["C"], ["A", "B"], kb)],
                                     ["A", "B", "C"]), 0, tau_override=0.5)
    nav = inst.geometry()["nav"][0]
    cf = kf / nav
    pmf = _stationary_pmf(lambda c: cf * (A0 - c) * (B0 - c) / (kb * (c + 1)), min(A0, B0))
    runs = 3000
    hist = np.zeros(len(pmf))
    for r in range(runs):
        inst.reset(np.array([[A0], [B0], [0]], np.int32), seed=r)
        inst.step(8)  # 4 s >> 1/k_b
        c = inst.counts[2, 0]
        assert inst.counts[0, 0] + c == A0 and inst.counts[1, 0] + c == B0
        hist[c] += 1
    assert _chi2_sf(hist, runs * pmf) > 1e-3


def test_homodimer_stationary_law(oracle_lib):
    """2A <-> B: propensity c_f N(N-1)/2 with c_f = k_f/(N_A V[L])."""
    kf, kb, A0 = 3e6, 2.0, 14
    inst = oracle_lib.Instance(single_tet(),
                               model([0, 0], [(["A", "A"], ["B"], kf), (["B"], ["A", "A"], kb)],
                                     ["A", "B"]), 0, tau_override=1.0)
    cf = kf / inst.geometry()["nav"][0]
    pmf = _stationary_pmf(lambda b: cf * (A0 - 2 * b) * (A0 - 2 * b - 1) / 2 / (kb * (b + 1)), A0 // 2)
    runs = 3000
    hist = np.zeros(len(pmf))
    for r in range(runs):
        inst.reset(np.array([[A0], [0]], np.int32), seed=10 + r)
        inst.step(6)
        b = inst.counts[1, 0]
        assert inst.counts[0, 0] + 2 * b == A0
        hist[b] += 1
    assert _chi2_sf(hist, runs * pmf) > 1e-3


def test_zero_order_source_stationary_poisson(oracle_lib):
    """0 -> A at k0 (M/s) and A -> 0 at kd: stationary Poisson(k0 N_A V[L] / kd)."""
    kd = 3.0
    inst = oracle_lib.Instance(single_tet(), model([0], [([], ["A"], 1.0), (["A"], [], kd)], ["A"]),
                               0, tau_override=0.5)
    nav = inst.geometry()["nav"][0]
    k0 = 12.0 * kd / nav  # mean 12
    inst = oracle_lib.Instance(single_tet(), model([0], [([], ["A"], k0), (["A"], [], kd)], ["A"]),
                               0, tau_override=0.5)
    lam = k0 * nav / kd
    runs = 3000
    out = np.zeros(runs, int)
    for r in range(runs):
        inst.reset(np.array([[0]], np.int32), seed=r)
        inst.step(8)
        out[r] = inst.counts[0, 0]
    nmax = out.max() + 10
    assert _chi2_sf(np.bincount(out, minlength=nmax + 1)[: nmax + 1],
                    runs * stats.poisson.pmf(np.arange(nmax + 1), lam)) > 1e-3
