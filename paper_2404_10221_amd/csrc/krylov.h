// Device-resident GMRES(m) state and the Arnoldi / least-squares kernels.
//
// GMRES (Lemma Krylov; Saad-Schultz) on the left-preconditioned system is run
// with classical Gram-Schmidt plus one re-orthogonalisation (CGS2), which spans
// the same Krylov space as the textbook modified Gram-Schmidt in exact
// arithmetic.  Basis columns are stored unnormalised with a scale factor
// vsc[k] (column k of V is vsc[k] * Vbar_k), so no sweep is spent on scaling.
// The Hessenberg column is reduced by Givens rotations on the device; the
// stopping rule |g_{j+1}| <= thr (Section 4) sets a flag that later kernels of
// a speculatively launched chunk read to exit early.
#pragma once
#include "common.h"

enum : int {
  GM_RUNNING = 0,
  GM_CONVERGED = 1,
  GM_CYCLE_FULL = 2,
  GM_BREAKDOWN = 3,
  GM_NONFINITE = -1
};

struct GmresSummary {
  int flag;       // GM_*
  int k;          // iterations of the finished cycle
  int applied;    // solution update done for this cycle
  int pad0;
  double beta0;   // ||z_0|| of the step
  double beta;    // ||z|| at the start of the current cycle
  double thr;     // stopping threshold on |g_{j+1}|
  double res;     // latest |g_{j+1}|
};

struct GmresState {
  GmresSummary sum;
  double g[RSFDE_MAX_RESTART + 1];
  double cs[RSFDE_MAX_RESTART], sn[RSFDE_MAX_RESTART];
  double Rm[RSFDE_MAX_RESTART * RSFDE_MAX_RESTART];  // R(i,j) at [j*MAX + i]
  double vsc[RSFDE_MAX_RESTART + 1];
  double h[RSFDE_MAX_RESTART + 1], h2[RSFDE_MAX_RESTART + 1];
  double y[RSFDE_MAX_RESTART];
};

// Grid size of the Krylov sweeps for an n-vector (fixed for a given n, so the
// reductions are deterministic).
inline int kry_blocks(int64_t n) {
  int64_t b = (n + 1023) / 1024;
  if (b > 1024) b = 1024;
  if (b < 1) b = 1;
  return (int)b;
}
#define RSFDE_KRY_THREADS 256

struct KryArgs {
  const double* V;    // basis, column k at V + k*ldv
  int64_t ldv;
  int64_t n;
  double* w;          // working vector (column j+1 of V)
  GmresState* st;
  double* partial;    // [blocks * (RSFDE_MAX_RESTART+1)]
  unsigned* counter;  // zero-initialised ticket counter
  int j;              // Arnoldi index (w = P^{-1} A v_j)
  int m;              // restart length
};

// Launchers (krylov.hip)
hipError_t kry_cycle_init(double* v0, int64_t n, GmresState* st, double* partial, unsigned* counter,
                          int first, double rtol, double inner_rtol, int mixed, hipStream_t s);
hipError_t kry_dots(const KryArgs& a, hipStream_t s);
hipError_t kry_orth_dots(const KryArgs& a, hipStream_t s);
hipError_t kry_orth_norm_givens(const KryArgs& a, hipStream_t s);
hipError_t kry_update(const double* V, int64_t ldv, int64_t n, double* x, GmresState* st,
                      unsigned* counter, hipStream_t s);
hipError_t kry_state_reset(GmresState* st, unsigned* counter, hipStream_t s);
