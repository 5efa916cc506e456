// Device-resident GMRES(m) state and the Arnoldi / least-squares machinery.
//
// GMRES (Lemma Krylov; Saad-Schultz) on the left-preconditioned system is run
// with classical Gram-Schmidt plus one re-orthogonalisation (CGS2), which spans
// the same Krylov space as the textbook modified Gram-Schmidt in exact
// arithmetic.  Basis columns are stored unnormalised with a scale factor
// vsc[k] (column k of V is vsc[k] * Vbar_k), so no sweep is spent on scaling.
//
// Kernel structure of one Arnoldi step j (no single-block "finish" kernels):
//   operator passes   w = (BP)^{-1} A v_j   (the first pass resolves step j-1)
//   sweep 1           partials of Vbar^T w
//   sweep 2           prologue: h = reduce(sweep-1 partials); w -= V h; partials of Vbar^T w
//   sweep 3           prologue: h2 = reduce(sweep-2 partials); w -= V h2; partials of ||w||^2
// Step j's Hessenberg column, Givens rotation and stopping test ("resolve j")
// run in the prologue of the next kernel that needs them: the first operator
// pass of step j+1, or the solution-update kernel that closes a launched
// chunk.  Every block of that kernel computes the same values from the same
// partials (fixed order, deterministic) and only block 0 stores them.  A kernel
// never reads a state field that a block of the same kernel writes: step
// status lives in FL[0..m] (FL[j] = status before step j, written once per
// cycle), so kernels launched speculatively past convergence see a non-running
// FL and exit.
#pragma once
#include "common.h"

enum : int {
  GM_RUNNING = 0,
  GM_CONVERGED = 1,
  GM_CYCLE_FULL = 2,
  GM_BREAKDOWN = 3,
  GM_UNSET = 7,       // FL entry not reached in this cycle
  GM_NONFINITE = -1
};

struct GmresSummary {
  int flag;       // GM_* of the latest resolve (or of the cycle start)
  int k;          // iterations of the finished cycle
  int pad0, pad1;
  double beta0;   // ||z_0|| of the step
  double beta;    // ||z|| at the start of the current cycle
  double thr;     // stopping threshold on |g_{j+1}|
  double res;     // latest |g_{j+1}|
};

struct GmresState {
  GmresSummary sum;
  int FL[RSFDE_MAX_RESTART + 1];
  int kfin;
  int pad;
  double gfin[RSFDE_MAX_RESTART];      // rotated right-hand side, final entries
  double gam[RSFDE_MAX_RESTART + 1];   // running entry before rotation j
  double cs[RSFDE_MAX_RESTART], sn[RSFDE_MAX_RESTART];
  double Rm[RSFDE_MAX_RESTART * RSFDE_MAX_RESTART];  // R(i,j) at [j*MAX + i]
  double vsc[RSFDE_MAX_RESTART + 1];
  double h[RSFDE_MAX_RESTART + 1], h2[RSFDE_MAX_RESTART + 1];
  double y[RSFDE_MAX_RESTART];
};

// Partial sums are stored value-major: partial[k * RSFDE_PVS + block].
#define RSFDE_PVS 256
#define RSFDE_KRY_BLOCKS 256

// Blocks of a Krylov sweep for an n-vector (fixed for a given n).
inline int kry_blocks(int64_t n) {
  int64_t b = (n / 2 + 511) / 512;
  if (b > RSFDE_KRY_BLOCKS) b = RSFDE_KRY_BLOCKS;
  if (b < 1) b = 1;
  return (int)b;
}

// Pending-resolve descriptor carried by the first operator pass of a step and
// by the update kernel.
struct GmRes {
  GmresState* st;
  const double* p3;  // sweep-3 partials of step `pend`
  int nb3;           // number of those partials
  int j;             // step this kernel belongs to
  int pend;          // step to resolve here, or -1
  int m;             // restart length
};

struct GmOut {
  int flag;          // status after this kernel's resolve (or the earlier one)
  int k;             // iterations of a finished cycle
  double sc;         // scale of column j (vsc[j])
};

// Deterministic block sum of one value per thread (any multiple-of-64 block).
__device__ __forceinline__ double gm_block_sum(double x, double* sh /* >= 16 */) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) sh[wv] = x;
  __syncthreads();
  double s = 0.0;
  const int nw = (blockDim.x + 63) >> 6;
  for (int w = 0; w < nw; ++w) s += sh[w];
  __syncthreads();
  return s;
}

// Prologue shared by the first operator pass and the update kernel.  All
// threads of the block must call it.  On return `o` (shared) holds the status
// and, when this kernel resolved a finishing step and want_y, y[0..k) is in ysh.
__device__ __forceinline__ void gm_prologue(const GmRes& g, GmOut* o, double* ysh, bool want_y) {
  __shared__ double sh[16];
  __shared__ double hc[RSFDE_MAX_RESTART + 1];  // Hessenberg column (LDS, not private memory)
  GmresState* st = g.st;
  const bool cand = g.pend >= 0;
  const int fl_prev = st->FL[cand ? g.pend : g.j];
  double part = 0.0;
  if (cand && fl_prev == GM_RUNNING)
    for (int b = threadIdx.x; b < g.nb3; b += blockDim.x) part += g.p3[b];
  const double nu = gm_block_sum(part, sh);
  if (threadIdx.x == 0) {
    if (!cand) {
      o->flag = fl_prev == GM_UNSET ? GM_CONVERGED : fl_prev;
      o->sc = st->vsc[g.j];
      o->k = st->kfin;
      if (fl_prev != GM_RUNNING && fl_prev != GM_NONFINITE && want_y)
        for (int i = 0; i < o->k; ++i) ysh[i] = st->y[i];
    } else if (fl_prev != GM_RUNNING) {
      // the cycle ended before step `pend`: its resolve stored kfin and y
      o->flag = fl_prev == GM_UNSET ? GM_CONVERGED : fl_prev;
      o->k = st->kfin;
      o->sc = 0.0;
      if (fl_prev != GM_NONFINITE && want_y)
        for (int i = 0; i < o->k; ++i) ysh[i] = st->y[i];
    } else {
      // resolve step j = pend: Hessenberg column, Givens rotation, stopping test
      const int j = g.pend;
      const int MX = RSFDE_MAX_RESTART;
      const bool writer = blockIdx.x == 0;
      for (int i = 0; i <= j; ++i) hc[i] = st->h[i] + st->h2[i];
      const double hn = sqrt(nu);
      double hsz = 0.0;
      for (int i = 0; i <= j; ++i) hsz = fmax(hsz, fabs(hc[i]));
      const bool breakdown = !(hn > 1e-14 * hsz);
      for (int i = 0; i < j; ++i) {
        const double p = hc[i], q = hc[i + 1];
        hc[i] = st->cs[i] * p + st->sn[i] * q;
        hc[i + 1] = -st->sn[i] * p + st->cs[i] * q;
      }
      const double r = hypot(hc[j], hn);
      const double c = r > 0.0 ? hc[j] / r : 1.0;
      const double s = r > 0.0 ? hn / r : 0.0;
      const double gj = c * st->gam[j];
      const double gn = -s * st->gam[j];
      const double rr = fabs(gn);
      const double vn = hn > 0.0 ? 1.0 / hn : 0.0;
      int flag;
      if (!isfinite(rr) || !isfinite(r)) flag = GM_NONFINITE;
      else if (rr <= st->sum.thr) flag = GM_CONVERGED;
      else if (breakdown) flag = GM_BREAKDOWN;
      else if (j + 1 >= g.m) flag = GM_CYCLE_FULL;
      else flag = GM_RUNNING;
      const int k = j + 1;
      const bool fin = flag != GM_RUNNING && flag != GM_NONFINITE;
      if (fin && (want_y || writer)) {
        // back substitution R y = g (column j of R is hc[0..j-1], r)
        for (int i = k - 1; i >= 0; --i) {
          double sacc = i == j ? gj : st->gfin[i];
          for (int l = i + 1; l < k; ++l) sacc -= (l == j ? hc[i] : st->Rm[l * MX + i]) * ysh[l];
          ysh[i] = sacc / (i == j ? r : st->Rm[i * MX + i]);
        }
      }
      if (writer) {
        st->cs[j] = c;
        st->sn[j] = s;
        for (int i = 0; i < j; ++i) st->Rm[j * MX + i] = hc[i];
        st->Rm[j * MX + j] = r;
        st->gfin[j] = gj;
        st->gam[j + 1] = gn;
        st->vsc[j + 1] = vn;
        st->FL[j + 1] = flag;
        st->sum.res = rr;
        st->sum.flag = flag;
        if (fin) {
          st->kfin = k;
          st->sum.k = k;
          for (int i = 0; i < k; ++i) st->y[i] = ysh[i];
        }
      }
      o->flag = flag;
      o->k = fin ? k : 0;
      o->sc = vn;
    }
  }
  __syncthreads();
}

struct KryArgs {
  const double* V;    // basis, column k at V + k*ldv
  int64_t ldv;
  int64_t n;
  double* w;          // working vector (column j+1 of V)
  GmresState* st;
  double* pa;         // sweep-1 partials
  double* pb;         // sweep-2 partials
  double* pc;         // sweep-3 partials
  int j;              // Arnoldi index (w = P^{-1} A v_j)
  int m;              // restart length
};

// Launchers (krylov.hip)
hipError_t kry_cycle_init(double* v0, int64_t n, GmresState* st, double* partial, int first,
                          double rtol, double inner_rtol, int mixed, int m, hipStream_t s);
// ea/eb: when non-null, HIP events stamped at the dispatch's start and end
hipError_t kry_sweep(int which, const KryArgs& a, hipStream_t s, hipEvent_t ea = nullptr,
                     hipEvent_t eb = nullptr);  // which = 1, 2, 3
hipError_t kry_update(const double* V, int64_t ldv, int64_t n, double* x, const GmRes& g,
                      hipStream_t s, hipEvent_t ea = nullptr, hipEvent_t eb = nullptr);
hipError_t kry_state_reset(GmresState* st, hipStream_t s);
