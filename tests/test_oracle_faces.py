"""Pins of the oracle's split of a binomial leaver count among the faces
(the diffusion step: leavers go to the face neighbours in proportion to the
face couplings, section 2.1).  A centre tet with 60 molecules and four
empty neighbours, one window: whatever the sampler, the molecules leaving
through face k are Bin(m, p c_k) by thinning, and two faces' counts have
covariance -m p^2 c_j c_k, where c_k are the couplings' shares.  A wrong
conditional share (say c_k instead of c_k / (1 - c_0 - ... - c_{k-1})) or
a leaver count dropped into the wrong face fails them."""
import numpy as np
from scipy import stats

from tests.meshes import model, stars


def _chi2_sf(x, n, q):
    ks = np.arange(n + 1)
    exp = stats.binom.pmf(ks, n, q) * x.size
    obs = np.bincount(x, minlength=n + 1)[: n + 1].astype(float)
    keep = exp >= 5
    o = np.append(obs[keep], obs[~keep].sum())
    e = np.append(exp[keep], exp[~keep].sum())
    if e[-1] < 5:
        o[-2] += o[-1]
        e[-2] += e[-1]
        o, e = o[:-1], e[:-1]
    return stats.chi2.sf(((o - e) ** 2 / e).sum(), len(o) - 1)


def test_face_split_of_binomial_leavers(oracle_lib):
    n_st, m = 40_000, 60
    D = 1e-12
    md = model([D], [], ["A"])
    probe = oracle_lib.Instance(stars(1), md, 1)
    geo = probe.geometry()
    G, cum = geo["G"][0], geo["cum"][0]
    assert geo["nbr"][0].min() >= 0  # every face of the centre is interior
    share = np.diff(np.concatenate([[0.0], cum]))
    assert share.min() > 0.1 and share.max() - share.min() > 0.02  # unequal faces
    tau = 0.45 / (D * G)  # p = 0.45: a binomial count per centre
    inst = oracle_lib.Instance(stars(n_st), md, 17, tau)
    c = np.zeros((1, 5 * n_st), np.int32)
    c[0, 0::5] = m
    inst.reset(c)
    inst.step(1)
    out = inst.counts[0].reshape(n_st, 5)
    stay, faces = out[:, 0], out[:, 1:]
    p = min(1.0, (inst.tau * D) * inst.geometry()["G"][0])
    assert abs(p - 0.45) < 1e-9
    assert np.array_equal(stay + faces.sum(axis=1), np.full(n_st, m))
    for k in range(4):
        assert _chi2_sf(faces[:, k], m, p * share[k]) > 1e-3, k
    cov = np.cov(faces.T)
    for j in range(4):
        for k in range(j + 1, 4):
            exp = -m * p * p * share[j] * share[k]
            se = np.sqrt((m * p * share[j]) * (m * p * share[k]) / n_st) * 1.2
            assert abs(cov[j, k] - exp) < 4 * se, (j, k, cov[j, k], exp)


def test_face_split_when_the_cap_binds(oracle_lib):
    """A -> 0 in the centre (k tau = 0.2) with p = 0.9 and 60 molecules: m
    (the rounded occupancy, about 54) times p often exceeds the 49 or so
    molecules left after the decays, so the leavers are capped in about half
    the stars.  Given the number n that left, the faces' counts are
    multinomial(n, shares) in both cases: capped (n = the post-reaction
    count, the centre ends empty) and not.  A capped split drawn with the
    p-scaled probabilities of the uncapped draw, or a cap taken out of the
    last face, moves a face's total many standard errors."""
    n_st, N0 = 40_000, 60
    D = 1e-12
    probe = oracle_lib.Instance(stars(1), model([D], [(["A"], [], 1.0)], ["A"]), 1)
    geo = probe.geometry()
    G, cum = geo["G"][0], geo["cum"][0]
    share = np.diff(np.concatenate([[0.0], cum]))
    tau = 0.9 / (D * G)
    k = 0.2 / tau
    inst = oracle_lib.Instance(stars(n_st), model([D], [(["A"], [], k)], ["A"]), 23, tau)
    p = min(1.0, (inst.tau * D) * inst.geometry()["G"][0])
    assert abs(p - 0.9) < 1e-9
    c = np.zeros((1, 5 * n_st), np.int32)
    c[0, 0::5] = N0
    inst.reset(c)
    inst.step(1)
    out = inst.counts[0].reshape(n_st, 5).astype(np.int64)
    centre, faces = out[:, 0], out[:, 1:]
    n = faces.sum(axis=1)
    capped = centre == 0
    assert 0.25 < capped.mean() < 0.75, capped.mean()
    for sel in (capped, ~capped):
        tot = n[sel].sum()
        for f in range(4):
            z = (faces[sel, f].sum() - share[f] * tot) / np.sqrt(tot * share[f] * (1 - share[f]))
            assert abs(z) < 4.0, (bool(sel[0]), f, z)
