/*
 * os_oracle_par.c -- the serial oracle's window run over all host cores.
 *
 * TEST INFRASTRUCTURE ONLY (the all-core CPU baseline of the benchmark and
 * its bit-identity test).  It compiles the serial oracle's source unchanged
 * and adds one function: a window whose tet loop runs in parallel.  Every
 * tet's reaction SSA and leaver draws are the serial oracle's own functions
 * on the tet's own Philox streams, and all outflows are taken from the
 * post-reaction counts before any inflow is applied (the snapshot reading of
 * Algorithm 1's local and remote application), so the order in which tets
 * run cannot change a draw; the moves are integer adds into the next counts
 * (atomic here), whose sum does not depend on their order.  The result is
 * therefore bit for bit the serial oracle's, which a test checks.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -fopenmp -fPIC -shared.
 */
#include "os_oracle.c"

#include <omp.h>

static int os_window_par(const os_instance* I, uint64_t seed, double tau_k, uint32_t window,
                         int32_t* counts, int32_t* next, os_tallies* tal, int threads)
{
  int S = I->S;
  int32_t T = I->T;
  int status = OS_OK;
  int32_t status_tet = -1;   /* the serial loop keeps the error of the last tet */
  int64_t ev = 0, mv = 0, fm = 0;
  memset(next, 0, sizeof(int32_t) * (size_t)S * (size_t)T);
#pragma omp parallel for num_threads(threads) schedule(dynamic, 512) reduction(+ : ev, mv, fm)
  for (int32_t i = 0; i < T; ++i) {
    int32_t N[OS_MAX_S];
    double O[OS_MAX_S], tS[OS_MAX_S];
    int touched[OS_MAX_S];
    int64_t ev_i = 0;
    for (int s = 0; s < S; ++s) N[s] = counts[(size_t)s * T + i];
    int st_ssa = os_ssa_window(I, i, tau_k, seed, window, N, O, tS, touched, &ev_i);
    ev += ev_i;
    if (st_ssa != OS_OK) {
#pragma omp critical(os_par_status)
      if (i > status_tet) { status_tet = i; status = st_ssa; }
    }
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
#pragma omp atomic
      next[(size_t)s * T + i] += (int32_t)(N[s] - n);
      for (int k = 0; k < 4; ++k)
        if (out[k] > 0) {
#pragma omp atomic
          next[(size_t)s * T + I->nbr[4 * (size_t)i + k]] += (int32_t)out[k];
          mv += out[k];
          fm += 1;
        }
    }
  }
  tal->ssa_events += ev;
  tal->moves += mv;
  tal->face_moves += fm;
  for (size_t x = 0; x < (size_t)S * (size_t)T; ++x) {
    if (next[x] > OS_COUNT_CAP) status = OS_EOVERFLOW;
    counts[x] = next[x];
  }
  tal->windows += 1;
  tal->voxel_steps += T;
  return status;
}

/* n full windows of length tau on `threads` threads (as os_step). */
int os_step_par(const os_instance* I, uint64_t seed, int32_t* counts, double* t, int64_t n,
                int64_t* window, os_tallies* tal, int threads)
{
  int32_t* next = (int32_t*)malloc(sizeof(int32_t) * (size_t)I->S * (size_t)I->T);
  if (!next) return OS_ENOMEM;
  int status = OS_OK;
  for (int64_t k = 0; k < n; ++k) {
    int st = os_window_par(I, seed, I->tau, (uint32_t)*window, counts, next, tal, threads);
    *window += 1;
    *t = *t + I->tau;
    if (st != OS_OK) { status = st; break; }
  }
  free(next);
  return status;
}

int os_max_threads(void) { return omp_get_max_threads(); }
