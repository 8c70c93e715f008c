"""Seeded synthetic inputs: tetrahedral meshes, reaction models, initial counts.

These generators feed both the HIP library and the CPU oracle.  They hold
none of the method's arithmetic (no couplings, no window length, no
propensities, no random draws of the scheme): they only produce the mesh
(vertex coordinates + tet connectivity + region labels), the model tables
(diffusion coefficients, stoichiometry, rate constants) and integer initial
counts.  Initial molecules are placed uniformly in space, i.e. each molecule
lands in a tet with probability proportional to its volume (the workloads of
section 3 place molecules uniformly); the volume used for that sampling is
computed here with numpy and is not the method's volume.

Workloads (stand-ins for the paper's, whose model parameters and meshes are
not available):
  * ``box_mesh``: a cuboid of cubes, each cut into 6 tets around its main
    diagonal, with optional interior vertex jitter (the "simple model"
    geometry of section 3.1 is a 10 x 10 x 100 um cuboid);
  * ``dendrite_mesh``: a seeded random branching tree of tapered cylinders,
    voxelised and cut into 6 tets per voxel (the Purkinje sub-branch / full
    dendrite meshes of section 3.2);
  * models: A + B <-> C, a 10-species / 12-reaction mass-action network, a
    15-species / 20-reaction calcium-buffer network with a zero-order calcium
    influx confined to a 5% region, and A + B <-> C plus a decay chain.
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass, field

import numpy as np

UM = 1e-6  # metres per micrometre

# Kuhn (Freudenthal) split of a unit cube into 6 tets around the (0,0,0)-(1,1,1)
# diagonal: one tet per permutation of the axes.  Every cube uses the same
# split, so neighbouring cubes share their triangulated faces.
_PERMS = list(itertools.permutations(range(3)))


def _kuhn_offsets() -> np.ndarray:
    out = np.zeros((6, 4, 3), np.int64)
    for t, perm in enumerate(_PERMS):
        p = np.zeros(3, np.int64)
        out[t, 0] = p
        for step, ax in enumerate(perm):
            p = p.copy()
            p[ax] += 1
            out[t, step + 1] = p
    return out


KUHN = _kuhn_offsets()


@dataclass
class Mesh:
    verts: np.ndarray                 # [V, 3] float64, metres
    tets: np.ndarray                  # [T, 4] int32
    region: np.ndarray | None = None  # [T] uint8
    name: str = ""
    info: dict = field(default_factory=dict)

    @property
    def n_tets(self) -> int:
        return int(self.tets.shape[0])

    def as_dict(self) -> dict:
        return dict(verts=self.verts, tets=self.tets, region=self.region)


@dataclass
class Model:
    species: list
    D: np.ndarray          # [S] m^2/s
    lhs: np.ndarray        # [R, S] int32
    rhs: np.ndarray        # [R, S] int32
    kcst: np.ndarray       # [n_regions, R] SI (order 0: M/s, 1: 1/s, 2: 1/(M s))
    reactions: list = field(default_factory=list)
    name: str = ""

    @property
    def S(self) -> int:
        return int(self.D.shape[0])

    @property
    def R(self) -> int:
        return int(self.lhs.shape[0])

    def as_dict(self) -> dict:
        return dict(D=self.D, lhs=self.lhs, rhs=self.rhs, kcst=self.kcst)


# ---------------------------------------------------------------- meshes ----

def box_mesh(nx: int, ny: int, nz: int, h: float, jitter: float = 0.0, seed: int = 0) -> Mesh:
    """nx*ny*nz cubes of edge h (metres), 6 tets each; tets ordered cube by
    cube (x fastest), 6 consecutive tets per cube.  Interior vertices are moved
    by U(-jitter*h, +jitter*h) per coordinate."""
    ix, iy, iz = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), np.arange(nz + 1), indexing="ij")
    # vertex id = (k*(ny+1) + j)*(nx+1) + i
    vid = lambda i, j, k: (k * (ny + 1) + j) * (nx + 1) + i  # noqa: E731
    V = (nx + 1) * (ny + 1) * (nz + 1)
    verts = np.zeros((V, 3))
    flat = vid(ix.ravel(), iy.ravel(), iz.ravel())
    verts[flat, 0] = ix.ravel() * h
    verts[flat, 1] = iy.ravel() * h
    verts[flat, 2] = iz.ravel() * h
    if jitter > 0.0:
        rng = np.random.default_rng(seed)
        d = rng.uniform(-jitter * h, jitter * h, size=(V, 3))
        interior = ((ix > 0) & (ix < nx) & (iy > 0) & (iy < ny) & (iz > 0) & (iz < nz)).ravel()
        verts[flat[interior]] += d[flat[interior]]
    cz, cy, cx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    cx, cy, cz = cx.ravel(), cy.ravel(), cz.ravel()  # cube order: x fastest, then y, then z
    tets = np.zeros((cx.size, 6, 4), np.int64)
    for t in range(6):
        for v in range(4):
            o = KUHN[t, v]
            tets[:, t, v] = vid(cx + o[0], cy + o[1], cz + o[2])
    return Mesh(verts=verts, tets=tets.reshape(-1, 4).astype(np.int32), region=None,
                name=f"box{nx}x{ny}x{nz}", info=dict(nx=nx, ny=ny, nz=nz, h=h, jitter=jitter))


def _tree_segments(rng: np.random.Generator, total_length: float, r_root: float,
                   r_min: float, seg_len: float):
    """Random branching tree of tapered cylinders: list of (p0, p1, r0, r1)."""
    segs = []
    length = 0.0
    # active tips: (position, direction, radius, remaining length of this branch)
    tips = [(np.zeros(3), np.array([0.0, 0.0, 1.0]), r_root, rng.uniform(40, 80) * UM)]
    while tips and length < total_length:
        pos, d, r, rem = tips.pop(0)
        step = min(seg_len, rem, total_length - length)
        nd = d + rng.normal(0.0, 0.15, 3)
        nd /= np.linalg.norm(nd)
        taper = r_min + (r - r_min) * 0.985
        p1 = pos + nd * step
        segs.append((pos, p1, r, max(taper, r_min)))
        length += step
        rem -= step
        if rem > 1e-12:
            tips.append((p1, nd, max(taper, r_min), rem))
        else:
            # bifurcate: two children, directions rotated away from the parent
            for sign in (-1.0, 1.0):
                perp = np.cross(nd, rng.normal(0.0, 1.0, 3))
                perp /= np.linalg.norm(perp)
                cd = nd + sign * 0.8 * perp
                cd /= np.linalg.norm(cd)
                cr = max(r_min, 0.8 * max(taper, r_min))
                tips.append((p1, cd, cr, rng.uniform(25, 60) * UM))
    return segs


def dendrite_mesh(target_tets: int = 1_000_000, total_length: float = 500 * UM,
                  r_root: float = 2.0 * UM, r_min: float = 0.5 * UM, seed: int = 2,
                  influx_fraction: float = 0.05) -> Mesh:
    """Voxelised random dendrite: voxel edge chosen so the tet count is close
    to ``target_tets``; 6 tets per voxel; largest face-connected component;
    region 1 = the ``influx_fraction`` of tets closest to a seeded distal point."""
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components

    rng = np.random.default_rng(seed)
    segs = _tree_segments(rng, total_length, r_root, r_min, seg_len=4 * UM)
    vol = sum(math.pi * (0.5 * (a + b)) ** 2 * np.linalg.norm(p1 - p0) for p0, p1, a, b in segs)
    h = (vol / (target_tets / 6.0)) ** (1.0 / 3.0)

    def voxelise(h):
        keys = []
        for p0, p1, r0, r1 in segs:
            rmax = max(r0, r1)
            lo = np.floor((np.minimum(p0, p1) - rmax) / h).astype(np.int64)
            hi = np.floor((np.maximum(p0, p1) + rmax) / h).astype(np.int64)
            gx, gy, gz = np.meshgrid(*[np.arange(lo[c], hi[c] + 1) for c in range(3)], indexing="ij")
            g = np.stack([gx.ravel(), gy.ravel(), gz.ravel()], 1)
            c = (g + 0.5) * h
            ax = p1 - p0
            L2 = float(ax @ ax)
            s = np.clip(((c - p0) @ ax) / L2, 0.0, 1.0)
            dist = np.linalg.norm(c - (p0 + s[:, None] * ax), axis=1)
            inside = dist <= r0 + (r1 - r0) * s
            keys.append(g[inside])
        g = np.unique(np.concatenate(keys), axis=0)
        return g

    for _ in range(3):  # refine the voxel edge towards the target count
        g = voxelise(h)
        n = 6 * g.shape[0]
        if abs(n - target_tets) < 0.03 * target_tets:
            break
        h *= (n / target_tets) ** (1.0 / 3.0)
    # largest face-connected component of voxels
    g0 = g.min(0)
    g = g - g0
    dims = g.max(0) + 2
    code = lambda a: (a[:, 2] * dims[1] + a[:, 1]) * dims[0] + a[:, 0]  # noqa: E731
    vcode = code(g)
    order = np.argsort(vcode)
    vcode_sorted = vcode[order]
    rows, cols = [], []
    for ax in range(3):
        nb = g.copy()
        nb[:, ax] += 1
        nc = code(nb)
        pos = np.searchsorted(vcode_sorted, nc)
        pos = np.minimum(pos, len(vcode_sorted) - 1)
        hit = vcode_sorted[pos] == nc
        rows.append(np.nonzero(hit)[0])
        cols.append(order[pos[hit]])
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    A = coo_matrix((np.ones(rows.size), (rows, cols)), shape=(g.shape[0], g.shape[0]))
    ncomp, lab = connected_components(A, directed=False)
    big = np.argmax(np.bincount(lab))
    g = g[lab == big]
    # order voxels along a space-filling-ish key for locality (z, y, x)
    g = g[np.lexsort((g[:, 0], g[:, 1], g[:, 2]))]
    # vertices: unique voxel corners
    corners = (g[:, None, :] + np.array(list(itertools.product((0, 1), repeat=3)))[None]).reshape(-1, 3)
    cdims = dims + 1
    ccode = (corners[:, 2] * cdims[1] + corners[:, 1]) * cdims[0] + corners[:, 0]
    uniq, inv = np.unique(ccode, return_inverse=True)
    vx = uniq % cdims[0]
    vy = (uniq // cdims[0]) % cdims[1]
    vz = uniq // (cdims[0] * cdims[1])
    verts = (np.stack([vx, vy, vz], 1) + g0).astype(np.float64) * h
    corner_id = inv.reshape(-1, 8)  # corner order: itertools.product((0,1),repeat=3) -> (x,y,z) bits
    def cid(o):
        return corner_id[:, o[0] * 4 + o[1] * 2 + o[2]]
    tets = np.zeros((g.shape[0], 6, 4), np.int64)
    for t in range(6):
        for v in range(4):
            tets[:, t, v] = cid(KUHN[t, v])
    tets = tets.reshape(-1, 4).astype(np.int32)
    # influx region: tets closest to a distal point of the tree
    bary = verts[tets].mean(1)
    far = np.argmax(np.linalg.norm(bary - bary.mean(0), axis=1))
    centre = bary[rng.integers(0, bary.shape[0])] * 0.5 + bary[far] * 0.5
    d = np.linalg.norm(bary - centre, axis=1)
    k = max(1, int(round(influx_fraction * tets.shape[0])))
    region = np.zeros(tets.shape[0], np.uint8)
    region[np.argpartition(d, k - 1)[:k]] = 1
    return Mesh(verts=verts, tets=tets, region=region, name="dendrite",
                info=dict(h=h, n_segments=len(segs), voxels=int(g.shape[0])))


def tet_volumes_for_sampling(mesh: Mesh) -> np.ndarray:
    """|det|/6 per tet, vectorised; used only to place molecules uniformly."""
    P, t = mesh.verts, mesh.tets
    p0 = P[t[:, 0]]
    a, b, c = P[t[:, 1]] - p0, P[t[:, 2]] - p0, P[t[:, 3]] - p0
    cx = b[:, 1] * c[:, 2] - b[:, 2] * c[:, 1]
    cy = b[:, 2] * c[:, 0] - b[:, 0] * c[:, 2]
    cz = b[:, 0] * c[:, 1] - b[:, 1] * c[:, 0]
    return np.abs(a[:, 0] * cx + a[:, 1] * cy + a[:, 2] * cz) / 6.0


def place_uniform(mesh: Mesh, totals, seed: int) -> np.ndarray:
    """counts[S, T] int32: totals[s] molecules of species s, each in a tet
    chosen with probability proportional to its volume."""
    rng = np.random.default_rng(seed)
    vol = tet_volumes_for_sampling(mesh)
    p = vol / vol.sum()
    out = np.zeros((len(totals), mesh.n_tets), np.int32)
    for s, n in enumerate(totals):
        if n > 0:
            out[s] = rng.multinomial(int(n), p)
    return out


def place_by_choice(mesh: Mesh, totals, seed: int) -> np.ndarray:
    """Same law as :func:`place_uniform` (each molecule independently in a tet
    chosen with probability proportional to its volume), drawn molecule by
    molecule: cheaper when there are fewer molecules than tets."""
    rng = np.random.default_rng(seed)
    cdf = getattr(mesh, "_volume_cdf", None)
    if cdf is None:
        cdf = np.cumsum(tet_volumes_for_sampling(mesh))
        cdf /= cdf[-1]
        mesh._volume_cdf = cdf
    out = np.zeros((len(totals), mesh.n_tets), np.int32)
    for s, n in enumerate(totals):
        if n > 0:
            # the molecules' order does not matter for the counts; sorted
            # uniforms make the table lookups sequential
            idx = np.searchsorted(cdf, np.sort(rng.random(int(n))), side="right")
            np.minimum(idx, mesh.n_tets - 1, out=idx)
            out[s] = np.bincount(idx, minlength=mesh.n_tets)
    return out


def place_concentration(mesh: Mesh, conc_molar, seed: int) -> np.ndarray:
    """Totals from molar concentrations over the mesh volume, then uniform placement."""
    vol_l = tet_volumes_for_sampling(mesh).sum() * 1e3
    totals = [int(round(c * 6.02214076e23 * vol_l)) for c in conc_molar]
    return place_uniform(mesh, totals, seed)


# ---------------------------------------------------------------- models ----

def _tables(species, reactions, D, n_regions=1, kcst_regions=None):
    S, R = len(species), len(reactions)
    idx = {s: i for i, s in enumerate(species)}
    lhs = np.zeros((R, S), np.int32)
    rhs = np.zeros((R, S), np.int32)
    k = np.zeros((n_regions, R))
    for r, (left, right, kval) in enumerate(reactions):
        for s in left:
            lhs[r, idx[s]] += 1
        for s in right:
            rhs[r, idx[s]] += 1
        k[:, r] = kval
    if kcst_regions is not None:
        for (reg, r), v in kcst_regions.items():
            k[reg, r] = v
    names = [" + ".join(l) + " -> " + " + ".join(rr) for l, rr, _ in reactions]
    return np.asarray(D, np.float64), lhs, rhs, k, names


def model_abc(kf: float = 1e6, kb: float = 10.0, D: float = 1e-12) -> Model:
    """A + B <-> C (the plain single-run workload)."""
    species = ["A", "B", "C"]
    reactions = [(["A", "B"], ["C"], kf), (["C"], ["A", "B"], kb)]
    D_, lhs, rhs, k, names = _tables(species, reactions, [D, D, D])
    return Model(species, D_, lhs, rhs, k, names, name="A+B<->C")


def model_simple10(seed: int = 1) -> Model:
    """10 diffusive species, 12 uni/bimolecular mass-action reactions.
    D ~ logU(1e-13, 1e-11) m^2/s, k1 ~ logU(0.1, 100) /s, k2 ~ logU(1e5, 1e8) /M/s."""
    rng = np.random.default_rng(seed)
    species = [f"S{i}" for i in range(10)]
    D = 10.0 ** rng.uniform(-13, -11, 10)
    D[int(rng.integers(0, 10))] = 1e-11  # one species at the top of the range
    reactions = []
    for r in range(12):
        if r % 2 == 0:
            a, b = rng.choice(10, 2, replace=False)
            k1 = 10.0 ** rng.uniform(-1, 2)
            if r % 4 == 0:
                c = int(rng.choice([x for x in range(10) if x not in (a, b)]))
                reactions.append(([species[a]], [species[b], species[c]], k1))
            else:
                reactions.append(([species[a]], [species[b]], k1))
        else:
            a, b, c = rng.choice(10, 3, replace=False)
            k2 = 10.0 ** rng.uniform(5, 8)
            reactions.append(([species[a], species[b]], [species[c]], k2))
    D_, lhs, rhs, k, names = _tables(species, reactions, D)
    return Model(species, D_, lhs, rhs, k, names, name="simple10")


CALCIUM_SPECIES = ["Ca", "Mg", "CBsf", "CBsCa", "CBfCa", "CBCaCa", "PV", "PVCa", "PVMg",
                   "PMCA", "PMCACa", "NCX", "NCXCa", "Fluo", "FluoCa"]


def model_calcium(influx_molar_per_s: float = 2e-3) -> Model:
    """15-species / 20-reaction calcium-buffer network in the style of a
    Purkinje dendrite calcium model: calbindin with two sites, parvalbumin
    (Ca/Mg), PMCA and NCX pumps, a dye, and a zero-order calcium influx that is
    active only in region 1."""
    sp = CALCIUM_SPECIES
    D = {"Ca": 2.0e-10, "Mg": 1.0e-10, "CBsf": 2.8e-11, "CBsCa": 2.8e-11, "CBfCa": 2.8e-11,
         "CBCaCa": 2.8e-11, "PV": 4.3e-11, "PVCa": 4.3e-11, "PVMg": 4.3e-11, "PMCA": 1e-13,
         "PMCACa": 1e-13, "NCX": 1e-13, "NCXCa": 1e-13, "Fluo": 1.0e-11, "FluoCa": 1.0e-11}
    R = [
        (["Ca", "CBsf"], ["CBsCa"], 5.5e6), (["CBsCa"], ["Ca", "CBsf"], 2.6),
        (["Ca", "CBsf"], ["CBfCa"], 4.35e7), (["CBfCa"], ["Ca", "CBsf"], 35.8),
        (["Ca", "CBsCa"], ["CBCaCa"], 4.35e7), (["CBCaCa"], ["Ca", "CBsCa"], 35.8),
        (["Ca", "CBfCa"], ["CBCaCa"], 5.5e6), (["CBCaCa"], ["Ca", "CBfCa"], 2.6),
        (["Ca", "PV"], ["PVCa"], 1.07e8), (["PVCa"], ["Ca", "PV"], 0.95),
        (["Mg", "PV"], ["PVMg"], 8.0e2), (["PVMg"], ["Mg", "PV"], 25.0),
        (["Ca", "PMCA"], ["PMCACa"], 1.5e8), (["PMCACa"], ["PMCA"], 12.0),
        (["Ca", "NCX"], ["NCXCa"], 1.8e8), (["NCXCa"], ["NCX"], 200.0),
        (["Ca", "Fluo"], ["FluoCa"], 2.0e8), (["FluoCa"], ["Ca", "Fluo"], 40.0),
        ([], ["Ca"], 0.0), (["PMCACa"], ["Ca", "PMCA"], 15.0),
    ]
    D_, lhs, rhs, k, names = _tables(sp, R, [D[s] for s in sp], n_regions=2,
                                     kcst_regions={(1, 18): influx_molar_per_s})
    return Model(sp, D_, lhs, rhs, k, names, name="calcium15")


CALCIUM_CONC = dict(Ca=45e-9, Mg=100e-6, CBsf=20e-6, CBsCa=1e-6, CBfCa=1e-6, CBCaCa=0.2e-6,
                    PV=10e-6, PVCa=2e-6, PVMg=10e-6, PMCA=2e-6, PMCACa=0.1e-6, NCX=0.5e-6,
                    NCXCa=0.02e-6, Fluo=5e-6, FluoCa=0.1e-6)


def model_abc_chain(scale=None) -> Model:
    """A + B <-> C plus the decay chain X -> Y -> Z; ``scale`` multiplies the
    four rate constants (per-run parameter sets)."""
    s = np.ones(4) if scale is None else np.asarray(scale, np.float64)
    species = ["A", "B", "C", "X", "Y", "Z"]
    reactions = [(["A", "B"], ["C"], 1e6 * s[0]), (["C"], ["A", "B"], 10.0 * s[1]),
                 (["X"], ["Y"], 2.0 * s[2]), (["Y"], ["Z"], 1.0 * s[3])]
    D_, lhs, rhs, k, names = _tables(species, reactions, [1e-12] * 6)
    return Model(species, D_, lhs, rhs, k, names, name="abc+chain")


# -------------------------------------------------------------- workloads ----

@dataclass
class Workload:
    name: str
    mesh: Mesh
    model: Model
    counts: np.ndarray     # [S, T] int32
    seed: int
    t_end: float
    description: str = ""


def config_small(seed: int = 0) -> Workload:
    """6x6x6 cubes of 1 um (1296 tets), A + B <-> C (kf 1e6 /M/s, kb 10 /s),
    D = 1e-12 m^2/s, 2000 A and 2000 B placed uniformly, 10 ms."""
    mesh = box_mesh(6, 6, 6, 1.0 * UM)
    model = model_abc()
    counts = place_uniform(mesh, [2000, 2000, 0], seed)
    return Workload("box6x6x6_abc", mesh, model, counts, seed, 10e-3,
                    "1296 tets, A+B<->C, 2000 A + 2000 B, 10 ms")


def config_simple(seed: int = 1) -> Workload:
    """10 x 10 x 100 um box of 0.5 um cubes (480,000 tets), 10% vertex jitter,
    10 species / 12 reactions, 1e6 molecules uniform, 100 ms."""
    mesh = box_mesh(20, 20, 200, 0.5 * UM, jitter=0.10, seed=seed)
    model = model_simple10(seed)
    rng = np.random.default_rng(seed + 100)
    w = rng.uniform(0.5, 1.5, model.S)
    totals = np.floor(1e6 * w / w.sum()).astype(np.int64)
    totals[0] += 1_000_000 - int(totals.sum())
    counts = place_uniform(mesh, totals, seed)
    return Workload("box20x20x200_simple10", mesh, model, counts, seed, 100e-3,
                    "480k tets, 10 species / 12 reactions, 1e6 molecules, 100 ms")


def config_simple_variant(density: float = 1.0, h_um: float = 0.5, extent_um=(10.0, 10.0, 100.0),
                          seed: int = 1, t_end: float = 100e-3) -> Workload:
    """The simple-model workload with its molecule density and its mesh
    resolution varied one at a time (the density and refinement series of
    section 3.1, figures 3 and 4): a cuboid of ``extent_um`` cut into cubes
    of edge ``h_um`` (6 tets each, 10% jitter), the same 10-species network,
    and ``density`` x 100 molecules per cubic micrometre (1e6 in the full
    10 x 10 x 100 um box), split among the species as in ``config_simple``."""
    dims = tuple(max(1, int(round(e / h_um))) for e in extent_um)
    mesh = box_mesh(*dims, h_um * UM, jitter=0.10, seed=seed)
    model = model_simple10(seed)
    rng = np.random.default_rng(seed + 100)
    w = rng.uniform(0.5, 1.5, model.S)
    total = int(round(density * 100.0 * float(np.prod([d * h_um for d in dims]))))
    totals = np.floor(total * w / w.sum()).astype(np.int64)
    totals[0] += total - int(totals.sum())
    counts = place_uniform(mesh, totals, seed)
    name = f"box{dims[0]}x{dims[1]}x{dims[2]}_h{h_um:g}um_simple10_density{density:g}x"
    return Workload(name, mesh, model, counts, seed, t_end,
                    f"{mesh.n_tets} tets of {h_um:g} um cubes, 10 species / 12 reactions, "
                    f"{total} molecules ({density:g}x density)")


def config_dendrite(seed: int = 2, target_tets: int = 1_000_000) -> Workload:
    """Random dendrite (~1e6 tets), calcium model, influx in 5% of tets, 50 ms."""
    mesh = dendrite_mesh(target_tets=target_tets, seed=seed)
    model = model_calcium()
    counts = place_concentration(mesh, [CALCIUM_CONC[s] for s in model.species], seed)
    return Workload("dendrite_calcium15", mesh, model, counts, seed, 50e-3,
                    f"{mesh.n_tets} tets dendrite, 15 species / 20 reactions, 5% influx, 50 ms")


def ensemble_runs(n_runs: int = 1024, seed: int = 3, t_lo: float = 1e3, t_hi: float = 5e4,
                  t_end: float = 1.0):
    """Many realisations of uneven size: 6 x 6 x n slabs of 1 um cubes with
    T ~ logU(t_lo, t_hi), A + B <-> C plus X -> Y -> Z with per-run rate
    constants scaled by U(0.5, 1.5); molecule totals proportional to T."""
    rng = np.random.default_rng(seed)
    runs = []
    meshes = {}
    for i in range(n_runs):
        T_target = math.exp(rng.uniform(math.log(t_lo), math.log(t_hi)))
        nz = max(1, int(round(T_target / 216.0)))
        mesh = meshes.get(nz) or meshes.setdefault(nz, box_mesh(6, 6, nz, 1.0 * UM))
        model = model_abc_chain(rng.uniform(0.5, 1.5, 4))
        per = mesh.n_tets / 1296.0
        totals = [int(2000 * per), int(2000 * per), 0, int(1000 * per), 0, 0]
        counts = place_by_choice(mesh, totals, seed * 100003 + i)
        runs.append(Workload(f"run{i}", mesh, model, counts, seed * 1000003 + i, t_end))
    return runs


def request_stream(n_requests: int = 2000, rate_per_s: float = 200.0, seed: int = 4,
                   t_lo: float = 1296, t_hi: float = 2e5, t_end: float = 100e-3):
    """Poisson arrivals of box-mesh simulations with the 10-species model;
    returns a list of (arrival_time_s, Workload)."""
    rng = np.random.default_rng(seed)
    model = model_simple10(1)
    t = 0.0
    out = []
    meshes = {}
    for i in range(n_requests):
        t += rng.exponential(1.0 / rate_per_s)
        T_target = math.exp(rng.uniform(math.log(t_lo), math.log(t_hi)))
        n = max(1, int(round((T_target / 6.0 / 25.0) ** 1.0)))
        mesh = meshes.get(n) or meshes.setdefault(n, box_mesh(5, 5, n, 0.5 * UM))
        totals = [int(2.0 * mesh.n_tets / 10)] * 10
        counts = place_by_choice(mesh, totals, seed * 7919 + i)
        out.append((t, Workload(f"req{i}", mesh, model, counts, seed * 104729 + i, t_end)))
    return out
