/*
 * os_oracle.c -- serial CPU oracle of the operator-splitting (OS) stochastic
 * reaction-diffusion scheme of "Parallel STEPS" (Chen & De Schutter,
 * arXiv:1610.02258).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and
 * the CPU-baseline leg of the benchmark load this file's shared object.  The
 * product library never links, loads or calls it, and this file includes no
 * header of the product library.
 *
 * What it computes, in the paper's order (Algorithm 1, section 2.2):
 *   for each window of length tau (the last one truncated at t_end):
 *     for each tet: an exact SSA over the tet's reactions for the window,
 *                   tracking occupancy O_S of every species whose count changes;
 *     for each tet and diffusive species S: mean occupancy Nbar = O_S / tau,
 *                   a binomial number of leavers, split among face neighbours
 *                   in proportion to the face diffusion rates;
 *     apply all moves.
 * The window length is tau = min over (S, tet) of 1/d_{S,tet} (section 2.1).
 * Between windows the rate constants may be replaced (os_set_rates), the
 * piecewise-constant forcing of section 3.2.
 *
 * Readings of points the paper leaves open (each is listed in the design doc):
 *   - occupancy is finalised at the window end, O_S += N_S (tau - t_S), and a
 *     species whose count did not change keeps Nbar = N_S exactly;
 *   - only species whose count changes (net stoichiometry != 0) are tracked;
 *   - "binomial(Nbar, tau, d)" is Bin(m, p) with m = Nbar stochastically
 *     rounded and p = min(1, tau * D_S * G_tet); leavers are clamped to the
 *     post-reaction count;
 *   - all outflows are computed from post-reaction counts before any inflow
 *     is applied (snapshot reading of the local/remote application);
 *   - d_{S,tet,k} = D_S * A_k / (V_tet * h_k) (finite-volume coupling with
 *     A the shared face area and h the barycentre distance), boundary faces
 *     reflective;
 *   - the leavers and their faces are sampled per molecule for small counts:
 *     with m <= 16, each of the m molecules draws one 32-bit uniform u and
 *     goes to the first face k (before the last face present) with
 *     u < p cum_k, else to the last face if u < p, else stays; with m > 16,
 *     the faces in order take successive binomials (face k: Bin(rest,
 *     p s_k / (1 - p cum_{k-1})), s_k the face's share) and the rest stay;
 *     should more leave than the post-reaction count, that many leave, split
 *     afresh by the shares (successive binomials, the last face present
 *     taking the rest).  cum_k is the left-to-right prefix sum of the face
 *     couplings over G.  Both are exact samplers of binomial leavers split
 *     among neighbours by rate; binomials are drawn by sequential-search
 *     inversion;
 *   - composition-rejection selection groups reactions by the binary
 *     exponent of their propensity (Slepoy, Thompson & Plimpton 2008);
 *   - random numbers are Philox4x32-10 (Salmon et al., SC'11), keyed by the
 *     seed, with the counter (draw call, stream, tet, window);
 *   - ln is computed from basic IEEE operations (exponent extraction and an
 *     atanh series, with the Cody-Waite split of ln 2), so that any other
 *     implementation of the same sequence of operations rounds identically.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -fPIC -shared.
 * fp contraction must stay off: every floating-point operation below is one
 * IEEE-754 binary64 operation with round-to-nearest-even.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define OS_NA 6.02214076e23 /* Avogadro constant, 1/mol (SI 2019 exact value) */
#define OS_MAX_S 64
#define OS_MAX_R 64
#define OS_EVENT_CAP (1 << 22)   /* events per tet per window before an error */
#define OS_COUNT_CAP (1 << 30)   /* molecule count per tet/species before an error */
#define OS_TINY_PROP 0x1p-1000   /* propensities below this are taken as zero */

enum {
  OS_OK = 0, OS_EINVAL = -1, OS_EMESH = -2, OS_ENODIFF = -3, OS_ENOMEM = -4,
  OS_EOVERFLOW = -5, OS_EEVENTS = -9
};

/* ------------------------------------------------------------------------ */
/* Philox4x32-10, from its published definition (Salmon, Moraes, Dror, Shaw, */
/* "Parallel random numbers: as easy as 1, 2, 3", SC'11).                    */
/* ------------------------------------------------------------------------ */
void os_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += 0x9E3779B9u;   /* golden ratio Weyl increment */
      k1 += 0xBB67AE85u;   /* sqrt(3)-1 Weyl increment */
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t y0 = hi1 ^ x1 ^ k0;
    uint32_t y1 = lo1;
    uint32_t y2 = hi0 ^ x3 ^ k1;
    uint32_t y3 = lo0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* A draw stream: the counter is (call, stream id, tet, window); each Philox  */
/* call yields four 32-bit words, consumed in order.                          */
typedef struct {
  uint32_t key[2];
  uint32_t stream, tet, window;
  uint32_t call;      /* index of the next Philox call */
  uint32_t words[4];
  int pos;            /* next unread word; 4 = buffer empty */
} os_stream;

static void os_stream_init(os_stream* st, uint64_t seed, uint32_t stream_id,
                           uint32_t tet, uint32_t window)
{
  st->key[0] = (uint32_t)(seed & 0xffffffffu);
  st->key[1] = (uint32_t)(seed >> 32);
  st->stream = stream_id;
  st->tet = tet;
  st->window = window;
  st->call = 0;
  st->pos = 4;
}

static uint32_t os_next_word(os_stream* st)
{
  if (st->pos == 4) {
    uint32_t ctr[4] = { st->call, st->stream, st->tet, st->window };
    os_philox4x32_10(ctr, st->key, st->words);
    st->call += 1;
    st->pos = 0;
  }
  uint32_t w = st->words[st->pos];
  st->pos += 1;
  return w;
}

/* 53-bit integer from two consecutive words (high 32 bits, then 21 bits). */
static uint64_t os_next53(os_stream* st)
{
  uint32_t hi = os_next_word(st);
  uint32_t lo = os_next_word(st);
  return ((uint64_t)hi << 21) | (uint64_t)(lo >> 11);
}

/* uniform in [0, 1) with 53 random bits */
static double os_u53_co(os_stream* st) { return (double)os_next53(st) * 0x1p-53; }
/* uniform in (0, 1] with 53 random bits */
static double os_u53_oc(os_stream* st) { return (double)(os_next53(st) + 1u) * 0x1p-53; }
/* uniform in [0, 1) with 32 random bits */
static double os_u32_co(os_stream* st) { return (double)os_next_word(st) * 0x1p-32; }

/* ------------------------------------------------------------------------ */
/* Natural logarithm from basic operations.                                  */
/* x = m * 2^e with m in [sqrt(1/2), sqrt(2)); ln m = 2 atanh(s),             */
/* s = (m-1)/(m+1), atanh(s) = s * sum_k s^{2k}/(2k+1) (k = 0..10);          */
/* e*ln2 is added with the Cody-Waite two-part split of ln 2.                */
/* Valid for positive normal x.                                              */
/* ------------------------------------------------------------------------ */
double os_ln(double x)
{
  uint64_t bits;
  memcpy(&bits, &x, sizeof bits);
  int e = (int)((bits >> 52) & 0x7ffu) - 1022;
  uint64_t mbits = (bits & 0x000fffffffffffffull) | 0x3fe0000000000000ull;
  double m;
  memcpy(&m, &mbits, sizeof m);              /* m in [0.5, 1) */
  if (m < 0.70710678118654752440) {          /* bring m into [sqrt(1/2), sqrt(2)) */
    m = m + m;
    e = e - 1;
  }
  double s = (m - 1.0) / (m + 1.0);
  double z = s * s;
  double p = 1.0 / 21.0;
  p = p * z + 1.0 / 19.0;
  p = p * z + 1.0 / 17.0;
  p = p * z + 1.0 / 15.0;
  p = p * z + 1.0 / 13.0;
  p = p * z + 1.0 / 11.0;
  p = p * z + 1.0 / 9.0;
  p = p * z + 1.0 / 7.0;
  p = p * z + 1.0 / 5.0;
  p = p * z + 1.0 / 3.0;
  p = p * z + 1.0;
  double lnm = (s + s) * p;
  double de = (double)e;
  const double ln2_hi = 6.93147180369123816490e-01; /* 0x3fe62e42fee00000 */
  const double ln2_lo = 1.90821492927058770002e-10; /* 0x3dea39ef35793c76 */
  return de * ln2_hi + (de * ln2_lo + lnm);
}

/* ------------------------------------------------------------------------ */
/* Binomial variate by sequential-search inversion (one 32-bit uniform per   */
/* chunk of at most 1000 trials; chunking keeps q^c >= 2^-1000, and a sum    */
/* of independent Bin(c_i, p) is Bin(sum c_i, p)).                           */
/* ------------------------------------------------------------------------ */
static double os_powi(double q, int64_t c)
{
  double result = 1.0, base = q;
  while (c > 0) {
    if (c & 1) result = result * base;
    base = base * base;
    c >>= 1;
  }
  return result;
}

static int64_t os_binom_core(int64_t m, double p, os_stream* st)
{
  /* 0 < p <= 0.5, m > 0 */
  double q = 1.0 - p;
  double r = p / q;
  int64_t total = 0;
  while (m > 0) {
    int64_t c = m < 1000 ? m : 1000;
    double u = os_u32_co(st);
    double f = os_powi(q, c);
    double F = f;
    int64_t k = 0;
    while (u >= F && k < c) {
      /* the pmf ratio r (c - k) / (k + 1), its division taken as a product
         with the rounded reciprocal of k + 1 (which the GPU reads from a
         table instead of dividing at every step) */
      f = ((f * r) * (double)(c - k)) * (1.0 / (double)(k + 1));
      k = k + 1;
      F = F + f;
    }
    total += k;
    m -= c;
  }
  return total;
}

int64_t os_binom(int64_t m, double p, os_stream* st)
{
  if (m <= 0 || !(p > 0.0)) return 0;
  if (p >= 1.0) return m;
  if (p > 0.5) return m - os_binom_core(m, 1.0 - p, st);
  return os_binom_core(m, p, st);
}

/* ------------------------------------------------------------------------ */
/* Instance: mesh geometry, model tables, tau (section 2.1).                  */
/* ------------------------------------------------------------------------ */
typedef struct {
  int32_t T, S, R, n_regions;
  int32_t* nbr;      /* [T*4]  neighbour across the face opposite local vertex k, -1 = boundary */
  double* vol;       /* [T]    volume, m^3 */
  double* area;      /* [T*4]  face areas, m^2 */
  double* dist;      /* [T*4]  barycentre distances, m (0 on boundary faces) */
  double* g;         /* [T*4]  face coupling A_k/(V h_k), 1/m^2 (0 on boundary faces) */
  double* G;         /* [T]    sum of g over faces (right-to-left suffix sum) */
  double* cum;       /* [T*4]  cumulative split fraction (g_0 + ... + g_k) / G, k < 3; cum_3 = 1 */
  int32_t* last;     /* [T]    last face with g > 0, -1 if none */
  double* nav;       /* [T]    N_A * V[litre] */
  uint8_t* region;   /* [T] */
  double* D;         /* [S]    diffusion coefficients, m^2/s */
  int32_t* lhs;      /* [R*S] */
  int32_t* rhs;      /* [R*S] */
  double* kcst;      /* [n_regions*R] */
  int32_t* order;    /* [R] */
  uint64_t* deps;    /* [R] bit j set: reaction j's propensity depends on a species r changes */
  double tau;
} os_instance;

/* Tallies: windows, tets x windows, applied SSA events, molecules moved, and
 * the nonzero (tet, species, face) moves -- the count M that prices the
 * diffusion update's writes to neighbour counts. */
typedef struct {
  int64_t windows, voxel_steps, ssa_events, moves, face_moves;
} os_tallies;

static void os_free_instance(os_instance* I)
{
  if (!I) return;
  free(I->nbr); free(I->vol); free(I->area); free(I->dist); free(I->g);
  free(I->G); free(I->cum); free(I->last); free(I->nav); free(I->region);
  free(I->D); free(I->lhs); free(I->rhs); free(I->kcst); free(I->order);
  free(I->deps);
  free(I);
}

void os_destroy(os_instance* I) { os_free_instance(I); }

typedef struct { int32_t v[3]; int32_t tet; int32_t face; } os_facekey;

static int os_facekey_cmp(const void* a, const void* b)
{
  const os_facekey* x = (const os_facekey*)a;
  const os_facekey* y = (const os_facekey*)b;
  for (int i = 0; i < 3; ++i) {
    if (x->v[i] < y->v[i]) return -1;
    if (x->v[i] > y->v[i]) return 1;
  }
  if (x->tet != y->tet) return x->tet < y->tet ? -1 : 1;
  return x->face < y->face ? -1 : (x->face > y->face);
}

static void os_sort3(int32_t* a)
{
  int32_t t;
  if (a[0] > a[1]) { t = a[0]; a[0] = a[1]; a[1] = t; }
  if (a[1] > a[2]) { t = a[1]; a[1] = a[2]; a[2] = t; }
  if (a[0] > a[1]) { t = a[0]; a[0] = a[1]; a[1] = t; }
}

/* Vertices of the face opposite local vertex k, in ascending local order. */
static const int os_face_verts[4][3] = { {1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2} };

static void os_barycentre(const double* verts, const int32_t* tv, double b[3])
{
  for (int c = 0; c < 3; ++c) {
    double s = verts[3 * tv[0] + c] + verts[3 * tv[1] + c];
    s = s + verts[3 * tv[2] + c];
    s = s + verts[3 * tv[3] + c];
    b[c] = s * 0.25;
  }
}

int os_build(int32_t n_verts, const double* verts, int32_t T, const int32_t* tets,
             const uint8_t* region, int32_t S, int32_t R, int32_t n_regions,
             const double* D, const int32_t* lhs, const int32_t* rhs,
             const double* kcst, double tau_override, os_instance** out)
{
  *out = NULL;
  if (T <= 0 || S <= 0 || S > OS_MAX_S || R < 0 || R > OS_MAX_R || n_regions <= 0)
    return OS_EINVAL;
  for (int64_t i = 0; i < 4 * (int64_t)T; ++i)
    if (tets[i] < 0 || tets[i] >= n_verts) return OS_EMESH;
  os_instance* I = (os_instance*)calloc(1, sizeof *I);
  if (!I) return OS_ENOMEM;
  I->T = T; I->S = S; I->R = R; I->n_regions = n_regions;
  I->nbr = (int32_t*)malloc(sizeof(int32_t) * 4 * (size_t)T);
  I->vol = (double*)malloc(sizeof(double) * (size_t)T);
  I->area = (double*)malloc(sizeof(double) * 4 * (size_t)T);
  I->dist = (double*)malloc(sizeof(double) * 4 * (size_t)T);
  I->g = (double*)malloc(sizeof(double) * 4 * (size_t)T);
  I->G = (double*)malloc(sizeof(double) * (size_t)T);
  I->cum = (double*)malloc(sizeof(double) * 4 * (size_t)T);
  I->last = (int32_t*)malloc(sizeof(int32_t) * (size_t)T);
  I->nav = (double*)malloc(sizeof(double) * (size_t)T);
  I->region = (uint8_t*)malloc((size_t)T);
  I->D = (double*)malloc(sizeof(double) * (size_t)S);
  I->lhs = (int32_t*)malloc(sizeof(int32_t) * (size_t)(R * S + 1));
  I->rhs = (int32_t*)malloc(sizeof(int32_t) * (size_t)(R * S + 1));
  I->kcst = (double*)malloc(sizeof(double) * (size_t)(n_regions * R + 1));
  I->order = (int32_t*)malloc(sizeof(int32_t) * (size_t)(R + 1));
  I->deps = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(R + 1));
  if (!I->nbr || !I->vol || !I->area || !I->dist || !I->g || !I->G || !I->cum ||
      !I->last || !I->nav || !I->region || !I->D || !I->lhs || !I->rhs || !I->kcst ||
      !I->order || !I->deps) {
    os_free_instance(I);
    return OS_ENOMEM;
  }
  for (int32_t i = 0; i < T; ++i) {
    I->region[i] = region ? region[i] : 0;
    if (I->region[i] >= n_regions) { os_free_instance(I); return OS_EINVAL; }
  }
  for (int s = 0; s < S; ++s) {
    if (!(D[s] >= 0.0)) { os_free_instance(I); return OS_EINVAL; }
    I->D[s] = D[s];
  }
  memcpy(I->lhs, lhs, sizeof(int32_t) * (size_t)(R * S));
  memcpy(I->rhs, rhs, sizeof(int32_t) * (size_t)(R * S));
  memcpy(I->kcst, kcst, sizeof(double) * (size_t)(n_regions * R));
  for (int r = 0; r < R; ++r) {
    int ord = 0;
    for (int s = 0; s < S; ++s) {
      if (lhs[r * S + s] < 0 || rhs[r * S + s] < 0) { os_free_instance(I); return OS_EINVAL; }
      ord += lhs[r * S + s];
    }
    if (ord > 2) { os_free_instance(I); return OS_EINVAL; }
    I->order[r] = ord;
  }
  for (int64_t i = 0; i < (int64_t)n_regions * R; ++i)
    if (!(kcst[i] >= 0.0)) { os_free_instance(I); return OS_EINVAL; }
  /* deps(R): reactions whose propensity reads a species that r changes (section 2.1) */
  for (int r = 0; r < R; ++r) {
    uint64_t mask = 0;
    for (int j = 0; j < R; ++j)
      for (int s = 0; s < S; ++s)
        if (rhs[r * S + s] - lhs[r * S + s] != 0 && lhs[j * S + s] > 0) mask |= (uint64_t)1 << j;
    I->deps[r] = mask;
  }

  /* volumes */
  for (int32_t i = 0; i < T; ++i) {
    const int32_t* tv = tets + 4 * (size_t)i;
    const double* v0 = verts + 3 * (size_t)tv[0];
    const double* v1 = verts + 3 * (size_t)tv[1];
    const double* v2 = verts + 3 * (size_t)tv[2];
    const double* v3 = verts + 3 * (size_t)tv[3];
    double ax = v1[0] - v0[0], ay = v1[1] - v0[1], az = v1[2] - v0[2];
    double bx = v2[0] - v0[0], by = v2[1] - v0[1], bz = v2[2] - v0[2];
    double cx = v3[0] - v0[0], cy = v3[1] - v0[1], cz = v3[2] - v0[2];
    double crx = by * cz - bz * cy;
    double cry = bz * cx - bx * cz;
    double crz = bx * cy - by * cx;
    double det = ax * crx + ay * cry;
    det = det + az * crz;
    double V = fabs(det) / 6.0;
    if (!(V > 0.0)) { os_free_instance(I); return OS_EMESH; }
    I->vol[i] = V;
    I->nav[i] = OS_NA * (V * 1.0e3);
    for (int k = 0; k < 4; ++k) {
      const double* p = verts + 3 * (size_t)tv[os_face_verts[k][0]];
      const double* q = verts + 3 * (size_t)tv[os_face_verts[k][1]];
      const double* w = verts + 3 * (size_t)tv[os_face_verts[k][2]];
      double ux = q[0] - p[0], uy = q[1] - p[1], uz = q[2] - p[2];
      double wx = w[0] - p[0], wy = w[1] - p[1], wz = w[2] - p[2];
      double nx = uy * wz - uz * wy;
      double ny = uz * wx - ux * wz;
      double nz = ux * wy - uy * wx;
      double nn = nx * nx + ny * ny;
      nn = nn + nz * nz;
      I->area[4 * (size_t)i + k] = sqrt(nn) * 0.5;
    }
  }

  /* face adjacency: match sorted vertex triples */
  os_facekey* keys = (os_facekey*)malloc(sizeof(os_facekey) * 4 * (size_t)T);
  if (!keys) { os_free_instance(I); return OS_ENOMEM; }
  for (int32_t i = 0; i < T; ++i)
    for (int k = 0; k < 4; ++k) {
      os_facekey* fk = &keys[4 * (size_t)i + k];
      for (int j = 0; j < 3; ++j) fk->v[j] = tets[4 * (size_t)i + os_face_verts[k][j]];
      os_sort3(fk->v);
      fk->tet = i;
      fk->face = k;
      I->nbr[4 * (size_t)i + k] = -1;
    }
  qsort(keys, 4 * (size_t)T, sizeof(os_facekey), os_facekey_cmp);
  for (size_t a = 0; a < 4 * (size_t)T;) {
    size_t b = a + 1;
    while (b < 4 * (size_t)T && keys[b].v[0] == keys[a].v[0] && keys[b].v[1] == keys[a].v[1] &&
           keys[b].v[2] == keys[a].v[2])
      ++b;
    if (b - a > 2) { free(keys); os_free_instance(I); return OS_EMESH; }
    if (b - a == 2) {
      if (keys[a].tet == keys[a + 1].tet) { free(keys); os_free_instance(I); return OS_EMESH; }
      I->nbr[4 * (size_t)keys[a].tet + keys[a].face] = keys[a + 1].tet;
      I->nbr[4 * (size_t)keys[a + 1].tet + keys[a + 1].face] = keys[a].tet;
    }
    a = b;
  }
  free(keys);

  /* couplings g = A / (V h), their total G (right-to-left), cumulative split fractions */
  for (int32_t i = 0; i < T; ++i) {
    double bi[3];
    os_barycentre(verts, tets + 4 * (size_t)i, bi);
    double g[4];
    for (int k = 0; k < 4; ++k) {
      int32_t j = I->nbr[4 * (size_t)i + k];
      if (j < 0) {
        g[k] = 0.0;
        I->dist[4 * (size_t)i + k] = 0.0;
        continue;
      }
      double bj[3];
      os_barycentre(verts, tets + 4 * (size_t)j, bj);
      double dx = bj[0] - bi[0], dy = bj[1] - bi[1], dz = bj[2] - bi[2];
      double hh = dx * dx + dy * dy;
      hh = hh + dz * dz;
      double h = sqrt(hh);
      if (!(h > 0.0)) { os_free_instance(I); return OS_EMESH; }
      I->dist[4 * (size_t)i + k] = h;
      g[k] = I->area[4 * (size_t)i + k] / (I->vol[i] * h);
    }
    double G = g[3];
    G = g[2] + G;
    G = g[1] + G;
    G = g[0] + G;
    I->G[i] = G;
    double pre = 0.0;
    I->last[i] = -1;
    for (int k = 0; k < 4; ++k) {
      I->g[4 * (size_t)i + k] = g[k];
      pre = pre + g[k];
      I->cum[4 * (size_t)i + k] = k == 3 ? 1.0 : (G > 0.0 ? pre / G : 0.0);
      if (g[k] > 0.0) I->last[i] = k;
    }
  }

  /* tau = min over (S, tet) of 1/d_{S,tet}, d_{S,tet} = D_S * G_tet (section 2.1) */
  if (tau_override > 0.0) {
    I->tau = tau_override;
  } else {
    double dmax = 0.0;
    for (int32_t i = 0; i < T; ++i)
      for (int s = 0; s < S; ++s) {
        double d = I->D[s] * I->G[i];
        if (d > dmax) dmax = d;
      }
    if (!(dmax > 0.0)) { os_free_instance(I); return OS_ENODIFF; }
    I->tau = 1.0 / dmax;
  }
  *out = I;
  return OS_OK;
}

double os_get_tau(const os_instance* I) { return I->tau; }

/* Time-varying forcing: replace the [n_regions*R] rate constants between
 * windows (a piecewise-constant influx such as the calcium influx of section
 * 3.2 is a zero-order reaction whose constant changes over time).  The next
 * window uses the new constants; the window length tau depends only on the
 * diffusion coefficients and stays as it is. */
int os_set_rates(os_instance* I, const double* kcst)
{
  size_t n = (size_t)I->n_regions * (size_t)I->R;
  for (size_t i = 0; i < n; ++i)
    if (!(kcst[i] >= 0.0) || !isfinite(kcst[i])) return OS_EINVAL;
  memcpy(I->kcst, kcst, sizeof(double) * n);
  return OS_OK;
}

/* Export the derived geometry for tests (arrays sized as in os_instance). */
void os_get_geometry(const os_instance* I, int32_t* nbr, double* vol, double* area,
                     double* dist, double* g, double* G, double* cum, double* nav)
{
  size_t T = (size_t)I->T;
  if (nbr) memcpy(nbr, I->nbr, sizeof(int32_t) * 4 * T);
  if (vol) memcpy(vol, I->vol, sizeof(double) * T);
  if (area) memcpy(area, I->area, sizeof(double) * 4 * T);
  if (dist) memcpy(dist, I->dist, sizeof(double) * 4 * T);
  if (g) memcpy(g, I->g, sizeof(double) * 4 * T);
  if (G) memcpy(G, I->G, sizeof(double) * T);
  if (cum) memcpy(cum, I->cum, sizeof(double) * 4 * T);
  if (nav) memcpy(nav, I->nav, sizeof(double) * T);
}

/* ------------------------------------------------------------------------ */
/* Reaction SSA operator for one tet over one window (Algorithm 1, reaction   */
/* part), with composition-rejection selection.                              */
/* ------------------------------------------------------------------------ */
static double os_propensity(const os_instance* I, int32_t i, int r, const int32_t* N,
                            double inv_nav)
{
  int S = I->S;
  double k = I->kcst[(size_t)I->region[i] * I->R + r];
  double c;
  if (I->order[r] == 0) c = k * I->nav[i];
  else if (I->order[r] == 1) c = k;
  else c = k * inv_nav;
  double h = 1.0;
  for (int s = 0; s < S; ++s) {
    int nu = I->lhs[r * S + s];
    if (nu == 1) {
      h = h * (double)N[s];
    } else if (nu == 2) {
      double pairs = N[s] >= 2 ? ((double)N[s] * (double)(N[s] - 1)) * 0.5 : 0.0;
      h = h * pairs;
    }
  }
  double a = c * h;
  return a >= OS_TINY_PROP ? a : 0.0;
}

static int os_expfield(double a)
{
  uint64_t bits;
  memcpy(&bits, &a, sizeof bits);
  return (int)((bits >> 52) & 0x7ffu);
}

/* Composition (pick a group with probability proportional to its total,   */
/* groups visited from the largest binary exponent down), then rejection    */
/* within the group against the group's power-of-two upper bound.           */
static int os_cr_select(const double* a, int R, double a0, os_stream* st)
{
  double x = os_u53_co(st) * a0;
  int gprev = 4096, chosen = -1;
  for (;;) {
    int gcur = -1;
    for (int r = 0; r < R; ++r)
      if (a[r] > 0.0) {
        int E = os_expfield(a[r]);
        if (E < gprev && E > gcur) gcur = E;
      }
    if (gcur < 0) break;
    double sum = 0.0;
    for (int r = 0; r < R; ++r)
      if (a[r] > 0.0 && os_expfield(a[r]) == gcur) sum = sum + a[r];
    chosen = gcur;
    if (x < sum) break;
    x = x - sum;
    gprev = gcur;
  }
  int n = 0;
  for (int r = 0; r < R; ++r)
    if (a[r] > 0.0 && os_expfield(a[r]) == chosen) n++;
  uint64_t bbits = (uint64_t)(chosen + 1) << 52;  /* 2^(chosen-1022): group upper bound */
  double bound;
  memcpy(&bound, &bbits, sizeof bound);
  for (;;) {
    double u2 = os_u53_co(st);
    int j = (int)(u2 * (double)n);
    if (j >= n) j = n - 1;
    double u3 = os_u53_co(st);
    int r = 0, seen = 0;
    for (r = 0; r < R; ++r)
      if (a[r] > 0.0 && os_expfield(a[r]) == chosen) {
        if (seen == j) break;
        seen++;
      }
    if (u3 * bound < a[r]) return r;
  }
}

/* Runs the reaction SSA of tet i for a window of length tau_k.             */
/* N: counts, in/out.  O, tS, touched: occupancy bookkeeping, out.          */
static int os_ssa_window(const os_instance* I, int32_t i, double tau_k, uint64_t seed,
                         uint32_t window, int32_t* N, double* O, double* tS,
                         int* touched, int64_t* events)
{
  int S = I->S, R = I->R;
  double a[OS_MAX_R];
  double inv_nav = 1.0 / I->nav[i];
  for (int s = 0; s < S; ++s) { O[s] = 0.0; tS[s] = 0.0; touched[s] = 0; }
  for (int r = 0; r < R; ++r) a[r] = os_propensity(I, i, r, N, inv_nav);
  os_stream st;
  os_stream_init(&st, seed, 0u, (uint32_t)i, window);
  double dt = 0.0;
  int64_t n_ev = 0;
  int status = OS_OK;
  for (;;) {
    double a0 = 0.0;
    for (int r = 0; r < R; ++r) a0 = a0 + a[r];
    if (!(a0 > 0.0)) break;                       /* no reaction can fire */
    double u = os_u53_oc(&st);
    double t_reac = -os_ln(u) / a0;
    if (dt + t_reac > tau_k) break;               /* next event falls outside the window */
    int rn = os_cr_select(a, R, a0, &st);
    dt = dt + t_reac;
    for (int s = 0; s < S; ++s) {
      int delta = I->rhs[rn * S + s] - I->lhs[rn * S + s];
      if (delta != 0) {
        O[s] = O[s] + (double)N[s] * (dt - tS[s]);
        tS[s] = dt;
        touched[s] = 1;
        N[s] = N[s] + delta;
        if (N[s] > OS_COUNT_CAP) status = OS_EOVERFLOW;
      }
    }
    for (int r = 0; r < R; ++r)
      if ((I->deps[rn] >> r) & 1u) a[r] = os_propensity(I, i, r, N, inv_nav);
    n_ev++;
    if (status != OS_OK) break;
    if (n_ev >= OS_EVENT_CAP) { status = OS_EEVENTS; break; }
  }
  for (int s = 0; s < S; ++s)
    if (touched[s]) O[s] = O[s] + (double)N[s] * (tau_k - tS[s]);
  *events += n_ev;
  return status;
}

/* ------------------------------------------------------------------------ */
/* Diffusion operator of one (tet, species): m trials of leaving with        */
/* probability p, each leaver to a face in proportion to the face coupling,  */
/* at most npost leavers.  Returns the number of leavers; out[k] receives    */
/* the molecules sent across face k.                                         */
/* ------------------------------------------------------------------------ */
#define OS_SMALL_M 16

static int os_pick_face(const os_instance* I, int32_t i, double u, double scale)
{
  int last = I->last[i];
  for (int k = 0; k < last; ++k)
    if (u < scale * I->cum[4 * (size_t)i + k]) return k;
  return last;
}

static int64_t os_diffuse_leavers(const os_instance* I, int32_t i, int64_t m, double p,
                                  int64_t npost, os_stream* st, int64_t out[4])
{
  int64_t n = 0;
  if (m <= 0 || !(p > 0.0)) return 0;
  if (m <= OS_SMALL_M) {
    /* one uniform per molecule: leave to face k if it falls in that face's
       share of [0, p); later leavers stay once npost have left */
    for (int64_t j = 0; j < m; ++j) {
      double u = os_u32_co(st);
      if (u < p && n < npost) {
        out[os_pick_face(I, i, u, p)] += 1;
        n = n + 1;
      }
    }
    return n;
  }
  /* each of the m molecules stays (1 - p) or leaves through face k
     (p s_k, s_k = cum_k - cum_{k-1} the face's share of the couplings): a
     multinomial over the faces and staying, drawn as successive binomials
     over the faces: face k takes Bin(rest, p s_k / (1 - p cum_{k-1})) of
     the molecules not yet placed, and those left over stay.  The number
     that leave is then Bin(m, p) and, given it, their split among the faces
     is multinomial with the shares. */
  int last = I->last[i];
  int64_t f[4] = { 0, 0, 0, 0 };
  int64_t rest = m;
  double prev = 0.0;
  for (int k = 0; k <= last; ++k) {
    double cum = k == last ? 1.0 : I->cum[4 * (size_t)i + k];
    double den = 1.0 - p * prev;
    /* den is 0 only for p = 1 with the shares before face k summing to 1 */
    double q = den > 0.0 ? (p * (cum - prev)) / den : (k == last ? 1.0 : 0.0);
    f[k] = os_binom(rest, q, st);
    rest -= f[k];
    n += f[k];
    prev = cum;
  }
  if (n > npost) {
    /* more leavers than molecules left after the reactions: npost leave,
       split afresh among the faces by the shares (face k takes Bin(rest,
       its share of what faces k.. hold), the last face present takes what is
       left), from the next draws of the stream */
    n = npost;
    rest = npost;
    prev = 0.0;
    for (int k = 0; k < last; ++k) {
      double cum = I->cum[4 * (size_t)i + k];
      double q = (cum - prev) / (1.0 - prev);
      f[k] = os_binom(rest, q, st);
      rest -= f[k];
      prev = cum;
    }
    f[last] = rest;
    for (int k = last + 1; k < 4; ++k) f[k] = 0;
  }
  for (int k = 0; k < 4; ++k) out[k] += f[k];
  return n;
}

/* ------------------------------------------------------------------------ */
/* One window (Algorithm 1): reaction SSA then diffusion, all tets, with      */
/* outflows taken from post-reaction counts and applied afterwards.          */
/* counts: [S*T] species-major, in/out.  work: [S*T] scratch.               */
/* ------------------------------------------------------------------------ */
static int os_window(const os_instance* I, uint64_t seed, double tau_k, uint32_t window,
                     int32_t* counts, int32_t* next, os_tallies* tal)
{
  int S = I->S;
  int32_t T = I->T;
  int status = OS_OK;
  memset(next, 0, sizeof(int32_t) * (size_t)S * (size_t)T);
  for (int32_t i = 0; i < T; ++i) {
    int32_t N[OS_MAX_S];
    double O[OS_MAX_S], tS[OS_MAX_S];
    int touched[OS_MAX_S];
    for (int s = 0; s < S; ++s) N[s] = counts[(size_t)s * T + i];
    int st_ssa = os_ssa_window(I, i, tau_k, seed, window, N, O, tS, touched, &tal->ssa_events);
    if (st_ssa != OS_OK) status = st_ssa;
    double G = I->G[i];
    for (int s = 0; s < S; ++s) {
      int64_t n = 0;
      int64_t out[4] = { 0, 0, 0, 0 };
      if (I->D[s] > 0.0 && G > 0.0) {
        os_stream st;
        os_stream_init(&st, seed, 1u + (uint32_t)s, (uint32_t)i, window);
        double Nbar = touched[s] ? O[s] / tau_k : (double)N[s];
        double fl = floor(Nbar);
        double frac = Nbar - fl;
        int64_t m = (int64_t)fl;
        if (frac > 0.0) {
          double u = os_u32_co(&st);
          if (u < frac) m = m + 1;
        }
        double p = (tau_k * I->D[s]) * G;
        if (p > 1.0) p = 1.0;
        n = os_diffuse_leavers(I, i, m, p, N[s], &st, out);
      }
      next[(size_t)s * T + i] += (int32_t)(N[s] - n);
      for (int k = 0; k < 4; ++k)
        if (out[k] > 0) {
          next[(size_t)s * T + I->nbr[4 * (size_t)i + k]] += (int32_t)out[k];
          tal->moves += out[k];
          tal->face_moves += 1;
        }
    }
  }
  for (size_t x = 0; x < (size_t)S * (size_t)T; ++x) {
    if (next[x] > OS_COUNT_CAP) status = OS_EOVERFLOW;
    counts[x] = next[x];
  }
  tal->windows += 1;
  tal->voxel_steps += T;
  return status;
}

/* ------------------------------------------------------------------------ */
/* Runtime main loop (Algorithm 1): windows of tau from t to t_end, the last */
/* one truncated to t_end - t; after a truncated window t is set to t_end.   */
/* *t and *window are advanced.                                              */
/* ------------------------------------------------------------------------ */
int os_run(const os_instance* I, uint64_t seed, int32_t* counts, double* t, double t_end,
           int64_t* window, os_tallies* tal)
{
  int32_t* next = (int32_t*)malloc(sizeof(int32_t) * (size_t)I->S * (size_t)I->T);
  if (!next) return OS_ENOMEM;
  int status = OS_OK;
  double tt = *t;
  while (tt < t_end) {
    double tau_k = I->tau;
    int truncated = 0;
    if (tt + tau_k > t_end) { tau_k = t_end - tt; truncated = 1; }
    int st = os_window(I, seed, tau_k, (uint32_t)*window, counts, next, tal);
    *window += 1;
    tt = truncated ? t_end : tt + tau_k;
    if (st != OS_OK) { status = st; break; }
  }
  *t = tt;
  free(next);
  return status;
}

/* n full windows of length tau, regardless of any end time. */
int os_step(const os_instance* I, uint64_t seed, int32_t* counts, double* t, int64_t n,
            int64_t* window, os_tallies* tal)
{
  int32_t* next = (int32_t*)malloc(sizeof(int32_t) * (size_t)I->S * (size_t)I->T);
  if (!next) return OS_ENOMEM;
  int status = OS_OK;
  for (int64_t k = 0; k < n; ++k) {
    int st = os_window(I, seed, I->tau, (uint32_t)*window, counts, next, tal);
    *window += 1;
    *t = *t + I->tau;
    if (st != OS_OK) { status = st; break; }
  }
  free(next);
  return status;
}

/* One window of explicit length tau_k (window index given). */
int os_window_explicit(const os_instance* I, uint64_t seed, int32_t* counts, double tau_k,
                       int64_t window, os_tallies* tal)
{
  int32_t* next = (int32_t*)malloc(sizeof(int32_t) * (size_t)I->S * (size_t)I->T);
  if (!next) return OS_ENOMEM;
  int st = os_window(I, seed, tau_k, (uint32_t)window, counts, next, tal);
  free(next);
  return st;
}

/* ------------------------------------------------------------------------ */
/* Test hooks for the individual variates.                                   */
/* ------------------------------------------------------------------------ */
/* n samples of Bin(m, p); sample j uses stream (seed, stream_id, tet = j, window). */
void os_sample_binom(uint64_t seed, uint32_t stream_id, uint32_t window, int64_t m, double p,
                     int64_t n, int64_t* out)
{
  for (int64_t j = 0; j < n; ++j) {
    os_stream st;
    os_stream_init(&st, seed, stream_id, (uint32_t)j, window);
    out[j] = os_binom(m, p, &st);
  }
}

/* The first n 53-bit uniforms of one stream, both conventions. */
void os_sample_uniforms(uint64_t seed, uint32_t stream_id, uint32_t tet, uint32_t window,
                        int64_t n, double* co, double* oc, double* u32)
{
  os_stream a, b, c;
  os_stream_init(&a, seed, stream_id, tet, window);
  os_stream_init(&b, seed, stream_id, tet, window);
  os_stream_init(&c, seed, stream_id, tet, window);
  for (int64_t j = 0; j < n; ++j) {
    if (co) co[j] = os_u53_co(&a);
    if (oc) oc[j] = os_u53_oc(&b);
    if (u32) u32[j] = os_u32_co(&c);
  }
}

/* SSA-only window of one tet (no diffusion), for reaction-operator pins.   */
/* Returns the number of events; N is updated; Nbar receives mean occupancy.*/
int64_t os_ssa_only(const os_instance* I, int32_t tet, double tau_k, uint64_t seed,
                    uint32_t window, int32_t* N, double* Nbar)
{
  double O[OS_MAX_S], tS[OS_MAX_S];
  int touched[OS_MAX_S];
  int32_t N0[OS_MAX_S];
  int64_t ev = 0;
  for (int s = 0; s < I->S; ++s) N0[s] = N[s];
  os_ssa_window(I, tet, tau_k, seed, window, N, O, tS, touched, &ev);
  for (int s = 0; s < I->S; ++s) Nbar[s] = touched[s] ? O[s] / tau_k : (double)N0[s];
  return ev;
}
