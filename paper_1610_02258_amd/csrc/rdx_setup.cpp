// rdx_setup.cpp -- the set-up step of "Parallel STEPS" section 2.1 on the host:
// face adjacency of the tetrahedral mesh, tet volumes, face couplings
// g_k = A_k / (V h_k) (finite-volume coupling: shared-face area over tet
// volume times barycentre distance), the per-tet total G = sum_k g_k, the
// cumulative face-split fractions, N_A V[L] per tet, and the window
// tau = min over (S, tet) of 1/d_{S,tet} with d_{S,tet} = D_S G_tet.
//
// Every floating-point expression is written as a fixed sequence of single
// IEEE-754 binary64 operations (the library is built with fp contraction off),
// so the derived values are a deterministic function of the mesh.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <numeric>

#include "rdx_internal.hpp"

namespace rdx {

namespace {

constexpr double kAvogadro = 6.02214076e23;  // 1/mol, exact since the 2019 SI

// Local vertex indices of the face opposite local vertex k, ascending.
constexpr int kFace[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};

struct Vec3 {
  double x, y, z;
};

inline Vec3 vert(const double* verts, int32_t v) {
  return Vec3{verts[3 * (size_t)v], verts[3 * (size_t)v + 1], verts[3 * (size_t)v + 2]};
}

inline Vec3 sub(Vec3 a, Vec3 b) { return Vec3{a.x - b.x, a.y - b.y, a.z - b.z}; }

inline Vec3 cross(Vec3 u, Vec3 w) {
  return Vec3{u.y * w.z - u.z * w.y, u.z * w.x - u.x * w.z, u.x * w.y - u.y * w.x};
}

// x*x + y*y, then + z*z
inline double norm2(Vec3 v) {
  double s = v.x * v.x + v.y * v.y;
  return s + v.z * v.z;
}

inline Vec3 barycentre(const double* verts, const int32_t* tv) {
  Vec3 p0 = vert(verts, tv[0]), p1 = vert(verts, tv[1]), p2 = vert(verts, tv[2]),
       p3 = vert(verts, tv[3]);
  Vec3 s{p0.x + p1.x, p0.y + p1.y, p0.z + p1.z};
  s = Vec3{s.x + p2.x, s.y + p2.y, s.z + p2.z};
  s = Vec3{s.x + p3.x, s.y + p3.y, s.z + p3.z};
  return Vec3{s.x * 0.25, s.y * 0.25, s.z * 0.25};
}

struct FaceRecord {
  std::array<int32_t, 3> key;  // sorted global vertex ids
  int32_t tet;
  int32_t face;
};

}  // namespace

rdx_status build_instance(const rdx_mesh* mesh, const rdx_model* model, double tau_override,
                          HostInstance* out, std::string* err) {
  if (!mesh || !model || !out) {
    *err = "null mesh, model or output";
    return RDX_EINVAL;
  }
  const int32_t T = mesh->n_tets, S = model->n_species, R = model->n_reactions;
  const int32_t NR = model->n_regions;
  if (T <= 0 || mesh->n_verts <= 0 || !mesh->verts || !mesh->tets) {
    *err = "mesh needs n_tets > 0, n_verts > 0, verts and tets";
    return RDX_EINVAL;
  }
  if (S < 1 || S > kMaxSpecies || R < 0 || R > kMaxReactions || NR < 1 || NR > kMaxRegions) {
    *err = "model sizes out of range (1<=S<=16, 0<=R<=32, 1<=n_regions<=8)";
    return RDX_EINVAL;
  }
  if (!model->diff_coef || (R > 0 && (!model->lhs || !model->rhs || !model->kcst))) {
    *err = "model arrays missing";
    return RDX_EINVAL;
  }
  if (!(std::isfinite(tau_override)) || tau_override < 0.0) {
    *err = "tau_override must be finite and >= 0";
    return RDX_EINVAL;
  }
  HostInstance& I = *out;
  I = HostInstance{};
  I.T = T;
  I.S = S;
  I.R = R;
  I.n_regions = NR;
  I.D.assign(model->diff_coef, model->diff_coef + S);
  for (double d : I.D)
    if (!(d >= 0.0) || !std::isfinite(d)) {
      *err = "diffusion coefficients must be finite and >= 0";
      return RDX_EINVAL;
    }
  if (R > 0) {
    I.lhs.assign(model->lhs, model->lhs + (size_t)R * S);
    I.rhs.assign(model->rhs, model->rhs + (size_t)R * S);
    I.kcst.assign(model->kcst, model->kcst + (size_t)R * NR);
  }
  for (int r = 0; r < R; ++r) {
    int order = 0, changes = 0;
    for (int s = 0; s < S; ++s) {
      int l = I.lhs[(size_t)r * S + s], q = I.rhs[(size_t)r * S + s];
      if (l < 0 || q < 0 || q > 100) {
        *err = "stoichiometry must lie in [0, 100]";
        return RDX_EINVAL;
      }
      order += l;
      if (q != l) ++changes;
    }
    if (order > 2) {
      *err = "reaction order above 2";
      return RDX_EINVAL;
    }
    if (changes > kMaxChanges) {
      *err = "a reaction changes more than 8 species";
      return RDX_EINVAL;
    }
  }
  for (double k : I.kcst)
    if (!(k >= 0.0) || !std::isfinite(k)) {
      *err = "rate constants must be finite and >= 0";
      return RDX_EINVAL;
    }
  I.region.assign((size_t)T, 0);
  if (mesh->region) {
    for (int32_t i = 0; i < T; ++i) {
      if (mesh->region[i] >= NR) {
        *err = "region label >= n_regions";
        return RDX_EINVAL;
      }
      I.region[i] = mesh->region[i];
    }
  }
  const double* verts = mesh->verts;
  const int32_t* tets = mesh->tets;
  for (size_t x = 0; x < 4 * (size_t)T; ++x)
    if (tets[x] < 0 || tets[x] >= mesh->n_verts) {
      *err = "tet vertex index out of range";
      return RDX_EMESH;
    }

  // volumes, N_A V[L], face areas
  std::vector<double> vol((size_t)T), area(4 * (size_t)T);
  I.nav.resize((size_t)T);
  for (int32_t i = 0; i < T; ++i) {
    const int32_t* tv = tets + 4 * (size_t)i;
    Vec3 p0 = vert(verts, tv[0]);
    Vec3 a = sub(vert(verts, tv[1]), p0), b = sub(vert(verts, tv[2]), p0),
         c = sub(vert(verts, tv[3]), p0);
    Vec3 bc = cross(b, c);
    double det = a.x * bc.x + a.y * bc.y;
    det = det + a.z * bc.z;
    double V = std::fabs(det) / 6.0;
    if (!(V > 0.0)) {
      *err = "tet " + std::to_string(i) + " has zero volume";
      return RDX_EMESH;
    }
    vol[i] = V;
    I.nav[i] = kAvogadro * (V * 1.0e3);
    for (int k = 0; k < 4; ++k) {
      Vec3 p = vert(verts, tv[kFace[k][0]]);
      Vec3 u = sub(vert(verts, tv[kFace[k][1]]), p);
      Vec3 w = sub(vert(verts, tv[kFace[k][2]]), p);
      area[4 * (size_t)i + k] = std::sqrt(norm2(cross(u, w))) * 0.5;
    }
  }

  // adjacency: sort all faces by their vertex triple; equal neighbours pair
  // up.  With fewer than 2^21 vertices the sorted triple packs into one
  // 63-bit key and the records are 16 bytes; otherwise 20-byte records with
  // a three-word key.  Both give the same pairs.
  I.nbr.assign(4 * (size_t)T, -1);
  auto pair_up = [&](size_t n, auto same_key, auto tf_of) -> bool {
    for (size_t a = 0; a < n;) {
      size_t b = a + 1;
      while (b < n && same_key(a, b)) ++b;
      if (b - a > 2 || (b - a == 2 && tf_of(a) / 4 == tf_of(a + 1) / 4)) return false;
      if (b - a == 2) {
        const int64_t x = tf_of(a), y = tf_of(a + 1);
        I.nbr[(size_t)x] = (int32_t)(y / 4);
        I.nbr[(size_t)y] = (int32_t)(x / 4);
      }
      a = b;
    }
    return true;
  };
  bool faces_ok;
  if (mesh->n_verts <= (1 << 21)) {
    struct Packed {
      uint64_t key;
      int64_t tf;  // 4 tet + face
    };
    std::vector<Packed> faces(4 * (size_t)T);
    for (int32_t i = 0; i < T; ++i)
      for (int k = 0; k < 4; ++k) {
        int32_t v[3];
        for (int j = 0; j < 3; ++j) v[j] = tets[4 * (size_t)i + kFace[k][j]];
        std::sort(v, v + 3);
        faces[4 * (size_t)i + k] = Packed{((uint64_t)v[0] << 42) | ((uint64_t)v[1] << 21) | (uint64_t)v[2],
                                          4 * (int64_t)i + k};
      }
    std::sort(faces.begin(), faces.end(), [](const Packed& x, const Packed& y) {
      return x.key != y.key ? x.key < y.key : x.tf < y.tf;
    });
    faces_ok = pair_up(faces.size(), [&](size_t a, size_t b) { return faces[a].key == faces[b].key; },
                       [&](size_t a) { return faces[a].tf; });
  } else {
    std::vector<FaceRecord> faces(4 * (size_t)T);
    for (int32_t i = 0; i < T; ++i)
      for (int k = 0; k < 4; ++k) {
        FaceRecord& f = faces[4 * (size_t)i + k];
        for (int j = 0; j < 3; ++j) f.key[j] = tets[4 * (size_t)i + kFace[k][j]];
        std::sort(f.key.begin(), f.key.end());
        f.tet = i;
        f.face = k;
      }
    std::sort(faces.begin(), faces.end(), [](const FaceRecord& x, const FaceRecord& y) {
      if (x.key != y.key) return x.key < y.key;
      if (x.tet != y.tet) return x.tet < y.tet;
      return x.face < y.face;
    });
    faces_ok = pair_up(faces.size(), [&](size_t a, size_t b) { return faces[a].key == faces[b].key; },
                       [&](size_t a) { return 4 * (int64_t)faces[a].tet + faces[a].face; });
  }
  if (!faces_ok) {
    *err = "a face is shared by more than two tets";
    return RDX_EMESH;
  }

  // couplings, their total, cumulative split fractions
  I.g.assign(4 * (size_t)T, 0.0);
  I.cum.assign(4 * (size_t)T, 0.0);
  I.G.assign((size_t)T, 0.0);
  for (int32_t i = 0; i < T; ++i) {
    Vec3 bi = barycentre(verts, tets + 4 * (size_t)i);
    double g[4];
    for (int k = 0; k < 4; ++k) {
      int32_t j = I.nbr[4 * (size_t)i + k];
      g[k] = 0.0;
      if (j < 0) continue;
      Vec3 bj = barycentre(verts, tets + 4 * (size_t)j);
      double h = std::sqrt(norm2(sub(bj, bi)));
      if (!(h > 0.0)) {
        *err = "coincident barycentres";
        return RDX_EMESH;
      }
      g[k] = area[4 * (size_t)i + k] / (vol[i] * h);
    }
    // G = g0 + (g1 + (g2 + g3)); cum_k = (g0 + ... + gk) / G summed left to right
    double G = g[3];
    G = g[2] + G;
    G = g[1] + G;
    G = g[0] + G;
    I.G[i] = G;
    double prefix = 0.0;
    for (int k = 0; k < 4; ++k) {
      I.g[4 * (size_t)i + k] = g[k];
      prefix = prefix + g[k];
      I.cum[4 * (size_t)i + k] = k == 3 ? 1.0 : (G > 0.0 ? prefix / G : 0.0);
    }
  }

  if (tau_override > 0.0) {
    I.tau = tau_override;
  } else {
    double dmax = 0.0;
    for (int32_t i = 0; i < T; ++i)
      for (int s = 0; s < S; ++s) dmax = std::max(dmax, I.D[s] * I.G[i]);
    if (!(dmax > 0.0)) {
      *err = "no diffusive species in a connected tet and no tau override";
      return RDX_ENODIFF;
    }
    I.tau = 1.0 / dmax;
  }
  return RDX_OK;
}

}  // namespace rdx
