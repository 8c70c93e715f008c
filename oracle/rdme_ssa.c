/*
 * rdme_ssa.c -- exact spatial SSA (Gillespie's direct method, 1976) of the
 * reaction-diffusion master equation on a tetrahedral mesh.
 *
 * TEST INFRASTRUCTURE ONLY: an independent algorithm against which the
 * operator-splitting oracle is checked statistically on tiny meshes.  It
 * plays the role of the paper's "serial SSA counterpart" (section 3): every
 * reaction in every tet and every diffusive jump across every face is one
 * channel, and no time window is involved.
 *
 * Channels:
 *   reaction r in tet i:       c_r(i) * h_r(N_i)      (same mass-action
 *                              convention as the operator-splitting model)
 *   jump of S from i across k: D_S * g_{i,k} * N_{S,i}
 * The random source is SplitMix64 (Steele, Lea & Flood 2014), unrelated to
 * the Philox streams of the operator-splitting scheme.
 */
#include <stdint.h>
#include <stdlib.h>
#include <math.h>

#define RS_NA 6.02214076e23

static uint64_t rs_splitmix(uint64_t* s)
{
  uint64_t z = (*s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

static double rs_uniform_oc(uint64_t* s) /* (0, 1] */
{
  return (double)((rs_splitmix(s) >> 11) + 1) * 0x1p-53;
}

static double rs_prop(int S, const int32_t* lhs_r, double k, int order, double nav,
                      const int32_t* N)
{
  double c = order == 0 ? k * nav : (order == 1 ? k : k / nav);
  double h = 1.0;
  for (int s = 0; s < S; ++s) {
    if (lhs_r[s] == 1) h *= (double)N[s];
    else if (lhs_r[s] == 2) h *= N[s] >= 2 ? 0.5 * (double)N[s] * (double)(N[s] - 1) : 0.0;
  }
  return c * h;
}

/*
 * counts: [S*T] species-major, advanced in place.
 * Records the counts at each of n_rec ascending times into rec [n_rec*S*T].
 * Returns the number of events, or -1 on bad input.
 */
int64_t rdme_direct(int32_t T, int32_t S, int32_t R, const int32_t* nbr, const double* g,
                    const double* D, const int32_t* lhs, const int32_t* rhs,
                    const double* kcst, const uint8_t* region, const double* nav,
                    int32_t* counts, int32_t n_rec, const double* t_rec, int32_t* rec,
                    uint64_t seed, int64_t max_events)
{
  if (T <= 0 || S <= 0 || R < 0) return -1;
  int* order = (int*)calloc((size_t)(R + 1), sizeof(int));
  int32_t* N = (int32_t*)malloc(sizeof(int32_t) * (size_t)S);
  if (!order || !N) { free(order); free(N); return -1; }
  for (int r = 0; r < R; ++r)
    for (int s = 0; s < S; ++s) order[r] += lhs[r * S + s];
  uint64_t rng = seed;
  double t = 0.0;
  int64_t events = 0;
  int32_t next_rec = 0;
  int64_t n_ch = (int64_t)T * (R + 4 * S);
  double* a = (double*)malloc(sizeof(double) * (size_t)(n_ch + 1));
  if (!a) { free(order); free(N); return -1; }
  for (;;) {
    /* all channel propensities, recomputed each event (tiny meshes only) */
    double a0 = 0.0;
    int64_t c = 0;
    for (int32_t i = 0; i < T; ++i) {
      for (int s = 0; s < S; ++s) N[s] = counts[(size_t)s * T + i];
      for (int r = 0; r < R; ++r) {
        double k = kcst[(size_t)(region ? region[i] : 0) * R + r];
        a[c] = rs_prop(S, lhs + r * S, k, order[r], nav[i], N);
        a0 += a[c++];
      }
      for (int s = 0; s < S; ++s)
        for (int k = 0; k < 4; ++k) {
          a[c] = nbr[4 * i + k] >= 0 ? D[s] * g[4 * i + k] * (double)N[s] : 0.0;
          a0 += a[c++];
        }
    }
    double dt = a0 > 0.0 ? -log(rs_uniform_oc(&rng)) / a0 : INFINITY;
    while (next_rec < n_rec && t + dt > t_rec[next_rec]) {
      for (int64_t x = 0; x < (int64_t)S * T; ++x) rec[(size_t)next_rec * S * T + x] = counts[x];
      next_rec++;
    }
    if (next_rec >= n_rec || !(a0 > 0.0) || events >= max_events) break;
    t += dt;
    double x = rs_uniform_oc(&rng) * a0;
    int64_t pick = -1;
    double acc = 0.0;
    for (int64_t j = 0; j < n_ch; ++j) {
      if (a[j] <= 0.0) continue;
      acc += a[j];
      pick = j;
      if (x <= acc) break;
    }
    if (pick < 0) break;
    int32_t i = (int32_t)(pick / (R + 4 * S));
    int64_t local = pick % (R + 4 * S);
    if (local < R) {
      for (int s = 0; s < S; ++s)
        counts[(size_t)s * T + i] += rhs[local * S + s] - lhs[local * S + s];
    } else {
      int64_t q = local - R;
      int s = (int)(q / 4), k = (int)(q % 4);
      counts[(size_t)s * T + i] -= 1;
      counts[(size_t)s * T + nbr[4 * i + k]] += 1;
    }
    events++;
  }
  free(a); free(order); free(N);
  return events;
}

/*
 * The same direct method with a selection that scales: the channels are
 * grouped by tet, a complete binary tree holds the per-tet propensity
 * totals, and an event first descends the tree to a tet (O(log T)), then
 * walks that tet's channels in the order above, recomputed from its counts,
 * in the same order that formed its total.  After an event only the totals
 * of the tets whose counts changed (one for a reaction, two for a jump) are
 * recomputed, with their tree paths.  Same law as rdme_direct; used to time
 * an exact serial SSA on meshes where rdme_direct's full recomputation per
 * event would take too long.  Same arguments and result as rdme_direct.
 */
static double rs_tet_total(int32_t i, int32_t T, int S, int R, const int32_t* nbr, const double* g,
                           const double* D, const int32_t* lhs, const int* order, const double* kcst,
                           const uint8_t* region, const double* nav, const int32_t* counts, int32_t* N)
{
  for (int s = 0; s < S; ++s) N[s] = counts[(size_t)s * T + i];
  double a = 0.0;
  for (int r = 0; r < R; ++r)
    a += rs_prop(S, lhs + r * S, kcst[(size_t)(region ? region[i] : 0) * R + r], order[r], nav[i], N);
  for (int s = 0; s < S; ++s)
    for (int k = 0; k < 4; ++k)
      a += nbr[4 * i + k] >= 0 ? D[s] * g[4 * i + k] * (double)N[s] : 0.0;
  return a;
}

int64_t rdme_tree(int32_t T, int32_t S, int32_t R, const int32_t* nbr, const double* g,
                  const double* D, const int32_t* lhs, const int32_t* rhs,
                  const double* kcst, const uint8_t* region, const double* nav,
                  int32_t* counts, int32_t n_rec, const double* t_rec, int32_t* rec,
                  uint64_t seed, int64_t max_events)
{
  if (T <= 0 || S <= 0 || R < 0) return -1;
  size_t leaves = 1;
  while (leaves < (size_t)T) leaves <<= 1;
  int* order = (int*)calloc((size_t)(R + 1), sizeof(int));
  int32_t* N = (int32_t*)malloc(sizeof(int32_t) * (size_t)S);
  double* tree = (double*)calloc(2 * leaves, sizeof(double));
  if (!order || !N || !tree) { free(order); free(N); free(tree); return -1; }
  for (int r = 0; r < R; ++r)
    for (int s = 0; s < S; ++s) order[r] += lhs[r * S + s];
  for (int32_t i = 0; i < T; ++i)
    tree[leaves + (size_t)i] = rs_tet_total(i, T, S, R, nbr, g, D, lhs, order, kcst, region, nav, counts, N);
  for (size_t k = leaves - 1; k >= 1; --k) tree[k] = tree[2 * k] + tree[2 * k + 1];
  uint64_t rng = seed;
  double t = 0.0;
  int64_t events = 0;
  int32_t next_rec = 0;
  for (;;) {
    double a0 = tree[1];
    double dt = a0 > 0.0 ? -log(rs_uniform_oc(&rng)) / a0 : INFINITY;
    while (next_rec < n_rec && t + dt > t_rec[next_rec]) {
      for (int64_t x = 0; x < (int64_t)S * T; ++x) rec[(size_t)next_rec * S * T + x] = counts[x];
      next_rec++;
    }
    if (next_rec >= n_rec || !(a0 > 0.0) || events >= max_events) break;
    t += dt;
    double x = rs_uniform_oc(&rng) * a0;
    size_t k = 1;
    while (k < leaves) {  /* to the left child unless x passes its total (or the right one is empty) */
      double left = tree[2 * k];
      if (x < left || !(tree[2 * k + 1] > 0.0)) k = 2 * k;
      else { x -= left; k = 2 * k + 1; }
    }
    int32_t i = (int32_t)(k - leaves);
    if (!(tree[k] > 0.0)) break;
    if (x >= tree[k]) x = tree[k] * 0.5;  /* rounding at the edge of the tet's share */
    for (int s = 0; s < S; ++s) N[s] = counts[(size_t)s * T + i];
    double acc = 0.0;
    int pick = -1;
    for (int r = 0; r < R && pick < 0; ++r) {
      double a = rs_prop(S, lhs + r * S, kcst[(size_t)(region ? region[i] : 0) * R + r], order[r], nav[i], N);
      acc += a;
      if (a > 0.0 && x < acc) pick = r;
    }
    int js = -1, jk = -1;
    for (int s = 0; s < S && pick < 0 && js < 0; ++s)
      for (int f = 0; f < 4; ++f) {
        double a = nbr[4 * i + f] >= 0 ? D[s] * g[4 * i + f] * (double)N[s] : 0.0;
        acc += a;
        if (a > 0.0 && x < acc) { js = s; jk = f; break; }
      }
    int32_t changed[2] = {i, -1};
    if (pick >= 0) {
      for (int s = 0; s < S; ++s)
        counts[(size_t)s * T + i] += rhs[pick * S + s] - lhs[pick * S + s];
    } else if (js >= 0) {
      int32_t j = nbr[4 * i + jk];
      counts[(size_t)js * T + i] -= 1;
      counts[(size_t)js * T + j] += 1;
      changed[1] = j;
    } else {
      break;  /* no channel found: cannot happen while the tet's total is positive */
    }
    for (int c = 0; c < 2; ++c) {
      if (changed[c] < 0) continue;
      size_t q = leaves + (size_t)changed[c];
      tree[q] = rs_tet_total(changed[c], T, S, R, nbr, g, D, lhs, order, kcst, region, nav, counts, N);
      for (q >>= 1; q >= 1; q >>= 1) tree[q] = tree[2 * q] + tree[2 * q + 1];
    }
    events++;
  }
  free(tree); free(order); free(N);
  return events;
}
