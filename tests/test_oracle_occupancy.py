"""Pins of the step that feeds the reaction occupancy into the diffusion
operator (Algorithm 1, diffusion operator): the mean occupancy N̄ = O/tau is
turned into a whole number of trials m by stochastic rounding, and the
leavers are capped at the count left after the reactions.

Every case runs on disjoint mirror pairs (two tets sharing one face, no other
face shared), so each pair is an independent sample of the same two-tet
system; one window of many pairs gives a large ensemble.  The expected values
come from the first-order decay law and the definitions, written out here:

* rounding: A -> B in tet 0, A immobile, B diffusive with p = 1.  B only
  rises within the window, so N̄_B <= N_post(B) and the cap cannot bind: all
  m trials leave, and B in tet 1 after the window equals m.  Unbiased
  rounding gives E[m] = E[N̄_B] = N0 (1 - (1 - e^{-k tau}) / (k tau)).
  Floor, round-to-nearest, or rounding up when u > frac all miss it.
* cap: A -> 0 with A diffusive.  With two molecules and one conversion at
  time t inside the window, N̄ = 1 + t/tau, N_post = 1: m = 2 with
  probability t/tau, and then two draws share a single leaver.  With p = 1,
  every survivor leaves and none is created: tet 0 ends at 0 and tet 1 holds
  Bin(N0, e^{-k tau}).
* one window, enumerated: A -> B with both species diffusive (p < 1), two
  tets, four molecules; the exact law of the end state, summed over the
  decay pattern, the occupancy of the conversions (sums of truncated
  exponentials), both roundings and the capped binomial leavers, against the
  oracle's histogram by chi-square.
"""
import math

import numpy as np
from scipy import stats

from tests.meshes import mirror_pairs, model


def _chi2_sf(obs, exp, min_exp=5.0):
    obs = np.asarray(obs, float)
    exp = np.asarray(exp, float)
    order = np.argsort(exp)[::-1]
    obs, exp = obs[order], exp[order]
    keep = exp >= min_exp
    o = np.append(obs[keep], obs[~keep].sum())
    e = np.append(exp[keep], exp[~keep].sum())
    if e[-1] < min_exp:
        o[-2] += o[-1]
        e[-2] += e[-1]
        o, e = o[:-1], e[:-1]
    return stats.chi2.sf(((o - e) ** 2 / e).sum(), len(o) - 1)


def _pairs_instance(O, n_pairs, D, reactions, species, seed, tau_override=0.0):
    return O.Instance(mirror_pairs(n_pairs), model(D, reactions, species), seed, tau_override)


# ------------------------------------------------------------ rounding ----

def _rounding_case(O, N0, n_pairs, seed):
    """A -> B at k = 3 / tau; returns (B in tet 1 of every pair, expected
    mean of m)."""
    probe = _pairs_instance(O, 1, [0.0, 1e-12], [(["A"], ["B"], 1.0)], ["A", "B"], 0)
    tau = probe.tau
    k = 3.0 / tau
    inst = _pairs_instance(O, n_pairs, [0.0, 1e-12], [(["A"], ["B"], k)], ["A", "B"], seed)
    # the translated copies differ from the probe by roundings only
    assert abs(inst.tau / tau - 1) < 1e-12
    c = np.zeros((2, 2 * n_pairs), np.int32)
    c[0, 0::2] = N0
    inst.reset(c)
    inst.step(1)
    kt = k * inst.tau
    expect = N0 * (1.0 - (1.0 - math.exp(-kt)) / kt)
    out = inst.counts
    # B never leaves tet 1 in this window (it arrives with the moves), A is
    # immobile, and the totals are conserved
    assert np.all(out[0, 1::2] == 0)
    assert np.all(out[0, 0::2] + out[1, 0::2] + out[1, 1::2] == N0)
    return out[1, 1::2].astype(float), expect


def test_stochastic_rounding_single_molecule(oracle_lib):
    """N0 = 1: m is 0 or 1, and P(m = 1) must equal E[N̄_B] = 0.6833 (floor
    gives 0, round-to-nearest 0.777, rounding up when u > frac 0.267)."""
    x, expect = _rounding_case(oracle_lib, 1, 40_000, 11)
    assert set(np.unique(x)) <= {0.0, 1.0}
    se = math.sqrt(expect * (1 - expect) / x.size)
    assert abs(x.mean() - expect) < 3 * se, (x.mean(), expect, se)


def test_stochastic_rounding_binomial_regime(oracle_lib):
    """N0 = 40: N̄_B is mostly above 16 (the binomial branch of the sampler);
    the mean of m is still E[N̄_B] (floor would be about 0.5 lower)."""
    x, expect = _rounding_case(oracle_lib, 40, 20_000, 12)
    assert (x > 16).mean() > 0.9
    se = x.std(ddof=1) / math.sqrt(x.size)
    assert abs(x.mean() - expect) < 3 * se, (x.mean(), expect, se)
    assert 3 * se < 0.1  # floor (a bias of about -0.5) would fail


# ----------------------------------------------------------------- cap ----

def _two_molecule_cap_expectation(p, kt):
    """E[leavers] of two molecules of A (A -> 0 at rate k, leave probability
    p): no conversion -> 2p; one conversion at t -> (1 - t/tau) p + (t/tau)
    (1 - (1 - p)^2); both converted -> 0."""
    none = math.exp(-2 * kt) * 2 * p
    # density of x = t / tau for the one molecule converting inside the
    # window while the other survives: 2 kt e^{-kt x} e^{-kt}
    int_e = (1 - math.exp(-kt)) / kt                     # int_0^1 e^{-kt x} dx
    int_xe = (1 - math.exp(-kt) * (1 + kt)) / kt ** 2    # int_0^1 x e^{-kt x} dx
    w = 2 * kt * math.exp(-kt)
    one = w * (p * int_e + ((1 - (1 - p) ** 2) - p) * int_xe)
    return none + one


def test_cap_at_post_reaction_count_two_molecules(oracle_lib):
    """p = 1/2, k tau = 1: the outflow of two molecules matches the capped
    law.  Capping at the pre-reaction count instead would add p^2 in every
    case with m = 2 and one molecule left (about 0.049 per pair, over six
    standard errors at 10^5 pairs); flooring N̄ would drop the second draw."""
    D = 1e-12
    probe = _pairs_instance(oracle_lib, 1, [D], [(["A"], [], 1.0)], ["A"], 0)
    tau = 0.5 * probe.tau
    k = 1.0 / tau
    n_pairs = 100_000
    inst = _pairs_instance(oracle_lib, n_pairs, [D], [(["A"], [], k)], ["A"], 21, tau_override=tau)
    G = inst.geometry()["G"][0]
    p = min(1.0, (tau * D) * G)
    assert abs(p - 0.5) < 1e-12
    c = np.zeros((1, 2 * n_pairs), np.int32)
    c[0, 0::2] = 2
    inst.reset(c)
    inst.step(1)
    out = inst.counts[0, 1::2].astype(float)
    assert inst.counts.min() >= 0
    expect = _two_molecule_cap_expectation(p, k * tau)
    se = out.std(ddof=1) / math.sqrt(n_pairs)
    assert abs(out.mean() - expect) < 3 * se, (out.mean(), expect, se)
    # the uncapped variant and the floor variant lie well outside
    x = 1 - 2 * math.exp(-1)  # int_0^1 x e^{-x} dx
    uncapped_extra = 2 * math.exp(-1) * x * p * p
    assert uncapped_extra > 6 * se


def test_cap_with_p1_every_survivor_leaves(oracle_lib):
    """p = 1, A -> 0 at k tau = 1: every molecule left after the reactions
    leaves and no more (tet 0 ends at exactly 0, nothing negative), so tet 1
    holds Bin(N0, e^{-1}); both sampler branches (N0 = 10 per-molecule, N0 =
    40 binomial)."""
    for N0, seed in ((10, 31), (40, 32)):
        probe = _pairs_instance(oracle_lib, 1, [1e-12], [(["A"], [], 1.0)], ["A"], 0)
        k = 1.0 / probe.tau
        n_pairs = 20_000
        inst = _pairs_instance(oracle_lib, n_pairs, [1e-12], [(["A"], [], k)], ["A"], seed)
        c = np.zeros((1, 2 * n_pairs), np.int32)
        c[0, 0::2] = N0
        inst.reset(c)
        inst.step(1)
        out = inst.counts
        assert out.min() >= 0
        assert np.all(out[0, 0::2] == 0)
        q = math.exp(-1.0)
        x = out[0, 1::2]
        # one nonzero (tet, species, face) move per pair with a survivor
        assert inst.tallies.face_moves == int((x > 0).sum())
        assert inst.tallies.moves == int(x.sum())
        obs = np.bincount(x, minlength=N0 + 1)[: N0 + 1]
        assert obs.sum() == n_pairs
        exp = n_pairs * stats.binom.pmf(np.arange(N0 + 1), N0, q)
        assert _chi2_sf(obs, exp) > 1e-3


# ------------------------------------------------- one window, enumerated ----

def _trunc_exp_sum_density(d, lam, x):
    """Density on x of the sum of d iid exponential(lam) variables
    conditioned to lie in [0, 1] (d = 1, 2)."""
    z = 1 - math.exp(-lam)
    if d == 1:
        return np.where((x >= 0) & (x <= 1), lam * np.exp(-lam * x) / z, 0.0)
    if d == 2:
        length = np.where(x <= 1, x, 2 - x)
        return np.where((x >= 0) & (x <= 2), lam ** 2 * np.exp(-lam * x) / z ** 2 * length, 0.0)
    raise ValueError(d)


def _round_weight(r, x):
    """P(stochastic rounding of x gives the integer r)."""
    return np.maximum(0.0, 1.0 - np.abs(x - r))


def _capped_binom(m, p, cap):
    """Law of min(Bin(m, p), cap) as {value: probability}."""
    out = {}
    for j in range(m + 1):
        v = min(j, cap)
        out[v] = out.get(v, 0.0) + math.comb(m, j) * p ** j * (1 - p) ** (m - j)
    return out


def _tet_law(a, b, lam, pA, pB):
    """Law of (A_post, A leavers, B_post, B leavers) of one tet in one
    window: a molecules of A converting to B at rate lam / tau, b of B."""
    grid = np.linspace(0.0, 2.0, 400_001)
    law = {}
    q = math.exp(-lam)
    for dec in range(a + 1):            # molecules of A converted in the window
        j = a - dec                      # A left after the reactions
        pdec = math.comb(a, dec) * (1 - q) ** dec * q ** j
        nB = b + dec                     # B left after the reactions
        if dec == 0:
            pairs = {(a, b): 1.0}        # nothing changed: N̄ = N exactly
        else:
            f = _trunc_exp_sum_density(dec, lam, grid)
            pairs = {}
            # N̄_A = j + X and N̄_B = nB - X, X the summed conversion times
            # over tau; the two roundings use independent draws
            for ra in range(dec + 1):
                for rb in range(dec + 1):
                    w = np.trapezoid(f * _round_weight(ra, grid) * _round_weight(rb, grid), grid)
                    if w > 0:
                        key = (j + ra, nB - rb)
                        pairs[key] = pairs.get(key, 0.0) + w
        for (mA, mB), pw in pairs.items():
            for lA, pa in _capped_binom(mA, pA, j).items():
                for lB, pb in _capped_binom(mB, pB, nB).items():
                    key = (j, lA, nB, lB)
                    law[key] = law.get(key, 0.0) + pdec * pw * pa * pb
    return law


def test_one_window_exact_law(oracle_lib):
    """Two tets, A -> B (k tau = 1.2), A and B diffusive with p_A = 0.8 and
    p_B = 0.48; start A = (2, 1), B = (1, 0).  The oracle's histogram of
    the end state (A0, A1, B0, B1) over 10^5 independent pairs against the
    exact one-window law."""
    D_A, D_B = 1e-12, 0.6e-12
    probe = _pairs_instance(oracle_lib, 1, [D_A, D_B], [(["A"], ["B"], 1.0)], ["A", "B"], 0)
    tau = 0.8 * probe.tau
    lam = 1.2
    k = lam / tau
    n_pairs = 100_000
    inst = _pairs_instance(oracle_lib, n_pairs, [D_A, D_B], [(["A"], ["B"], k)], ["A", "B"], 41,
                           tau_override=tau)
    G = inst.geometry()["G"][0]
    pA = min(1.0, (tau * D_A) * G)
    pB = min(1.0, (tau * D_B) * G)
    c = np.zeros((2, 2 * n_pairs), np.int32)
    c[0, 0::2], c[0, 1::2], c[1, 0::2] = 2, 1, 1
    inst.reset(c)
    inst.step(1)
    out = inst.counts
    law0 = _tet_law(2, 1, lam, pA, pB)
    law1 = _tet_law(1, 0, lam, pA, pB)
    assert abs(sum(law0.values()) - 1) < 1e-6 and abs(sum(law1.values()) - 1) < 1e-6
    exact = {}
    for (j0, lA0, n0, lB0), p0 in law0.items():
        for (j1, lA1, n1, lB1), p1 in law1.items():
            key = (j0 - lA0 + lA1, j1 - lA1 + lA0, n0 - lB0 + lB1, n1 - lB1 + lB0)
            exact[key] = exact.get(key, 0.0) + p0 * p1
    states = sorted(exact)
    index = {s: i for i, s in enumerate(states)}
    obs = np.zeros(len(states))
    got = np.stack([out[0, 0::2], out[0, 1::2], out[1, 0::2], out[1, 1::2]], 1)
    for row in map(tuple, got):
        assert row in index, row
        obs[index[row]] += 1
    exp = n_pairs * np.array([exact[s] for s in states])
    assert _chi2_sf(obs, exp) > 1e-3
