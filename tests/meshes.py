"""Tiny hand-built meshes for the oracle pins (inputs only, no method arithmetic)."""
import numpy as np


def single_tet(scale=1e-6):
    verts = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], float) * scale
    return dict(verts=verts, tets=np.array([[0, 1, 2, 3]], np.int32), region=None)


def mirror_pair(scale=1e-6):
    """Two tets mirror-imaged through their shared face z = 0."""
    verts = np.array([[0, 0, 0], [1, 0, 0], [0.3, 0.9, 0], [0.4, 0.3, 0.8], [0.4, 0.3, -0.8]],
                     float) * scale
    tets = np.array([[0, 1, 2, 3], [0, 1, 2, 4]], np.int32)
    return dict(verts=verts, tets=tets, region=None)


def model(D, reactions, species, n_regions=1):
    S, R = len(species), len(reactions)
    idx = {s: i for i, s in enumerate(species)}
    lhs = np.zeros((R, S), np.int32)
    rhs = np.zeros((R, S), np.int32)
    k = np.zeros((n_regions, max(R, 1)))[:, :R]
    for r, (l, rr, kv) in enumerate(reactions):
        for s in l:
            lhs[r, idx[s]] += 1
        for s in rr:
            rhs[r, idx[s]] += 1
        k[:, r] = kv
    return dict(D=np.asarray(D, float), lhs=lhs, rhs=rhs, kcst=k)


def mirror_pairs(n, scale=1e-6):
    """n disjoint copies of the mirror pair, spaced 3 scale apart along x:
    tets 2j and 2j + 1 share one face, and no other face is shared, so each
    pair is an independent sample of the same two-tet system."""
    one = mirror_pair(scale)
    off = np.zeros((n, 1, 3))
    off[:, 0, 0] = 3.0 * scale * np.arange(n)
    verts = (one["verts"][None, :, :] + off).reshape(-1, 3)
    tets = (one["tets"][None, :, :] + 5 * np.arange(n, dtype=np.int32)[:, None, None]).reshape(-1, 4)
    return dict(verts=verts, tets=tets.astype(np.int32), region=None)


def stars(n, scale=1e-6):
    """n disjoint copies of a star: an irregular centre tet (tet 5j) and, across
    each of its four faces, one neighbour tet (5j + 1 + k, apex pushed out of
    face k), so that every face of the centre is interior and the centre's
    four face couplings differ."""
    c = np.array([[0, 0, 0], [1.1, 0, 0], [0.2, 0.9, 0], [0.3, 0.25, 0.7]], float)
    centroid = c.mean(axis=0)
    verts = [c]
    tets = [[0, 1, 2, 3]]
    for k in range(4):
        face = [v for v in range(4) if v != k]
        fc = c[face].mean(axis=0)
        out = fc - c[k]
        out /= np.linalg.norm(out)
        verts.append((fc + 0.6 * out)[None, :])
        tets.append(face + [4 + k])
    one_v = np.concatenate(verts)
    one_t = np.array(tets, np.int64)
    off = np.zeros((n, 1, 3))
    off[:, 0, 0] = 4.0 * np.arange(n)
    V = ((one_v[None] + off) * scale).reshape(-1, 3)
    Tt = (one_t[None] + 8 * np.arange(n)[:, None, None]).reshape(-1, 4)
    return dict(verts=V, tets=Tt.astype(np.int32), region=None)
