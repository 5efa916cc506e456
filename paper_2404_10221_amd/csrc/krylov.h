// Device-resident GMRES(m) state and the Arnoldi / least-squares machinery.
//
// GMRES (Lemma Krylov; Saad-Schultz) on the left-preconditioned system is run
// with classical Gram-Schmidt plus one re-orthogonalisation (CGS2), which spans
// the same Krylov space as the textbook modified Gram-Schmidt in exact
// arithmetic.  Basis columns are stored unnormalised with a scale factor
// vsc[k] (column k of V is vsc[k] * Vbar_k), so no sweep is spent on scaling.
//
// Kernel structure of one Arnoldi step j (no single-block "finish" kernels):
//   operator passes   w = (BP)^{-1} A qt_j  (the first pass resolves step j-1), where
//                     column j holds u_j, projected once against the final columns
//   sweep A           partials of Vbar^T w and Vbar^T u_j
//   sweep B           prologue: reduce sweep A's partials; per row: q_j = second
//                     projection of u_j (written over column j), u_{j+1} = first
//                     projection of w (written over w); partials of ||u_{j+1}||^2
// (CGS2 with the second projection of each basis vector delayed by one step;
// see krylov.hip).
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

// Blocks for an instance of a many-instance handle: at least 8192 entries per
// block.  Every block of a sweep first reduces the previous sweep's partials and
// forms the projection coefficients; with the single-instance count (one block
// per 1024 entries) that prologue outweighed the vector work of the small
// instances, and the batched launches already fill the GPU with many instances
// (64 instances of 127^2 to 511^2: 4096 entries per block gave 187.5, 8192
// gave 193, 16384 gave 191 steps/s).
inline int kry_blocks_many(int64_t n) {
  int64_t b = (n + 8191) / 8192;
  if (b > RSFDE_KRY_BLOCKS) b = RSFDE_KRY_BLOCKS;
  if (b < 1) b = 1;
  return (int)b;
}

// Pending-resolve descriptor carried by the first operator pass of a step and
// by the update kernel.
struct GmRes {
  GmresState* st;
  const double* p3;  // sweep-B partials of ||u_{j+1}||^2 of step `pend`
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

// Resolve outputs kept in LDS for the kernel that ran the prologue: the rotated
// Hessenberg column of the resolved step (R(0..j, j)) and its rotated
// right-hand-side entry, for a back substitution in the same kernel.
struct GmCol {
  double rc[RSFDE_MAX_RESTART + 1];
  double gj;
  int j;  // resolved step, or -1
};

// Lane i's value of x, broadcast to the whole wavefront (i uniform).
__device__ __forceinline__ double gm_lane(double x, int i) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)b, i);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), i);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Everything the resolve reads from the state, fetched by the first wavefront
// (lane i: Hessenberg entries h_i, h2_i and rotation i) in one round of
// unconditional loads at clamped indices: no branch and no use of a loaded value
// sits between the loads, so none of them waits for another (or for the tile
// loads issued after them).
struct GmIn {
  double pv[RSFDE_PVS / 64];  // sweep-B norm partials lane + 64 q
  double h, h2, cs, sn;
  double gam, thr, vsc;
  int fl, kfin;
};

__device__ __forceinline__ void gm_fetch(const GmRes& g, GmIn& in) {
  const GmresState* st = g.st;
  const int lane = threadIdx.x;
  const int j = g.pend;  // -1: nothing to resolve
  const int jj = j < 0 ? 0 : j;
  in.fl = st->FL[j >= 0 ? j : g.j];
  in.kfin = st->kfin;
  in.vsc = st->vsc[g.j];
  const double* p3 = j >= 0 ? g.p3 : st->h;
#pragma unroll
  for (int q = 0; q < RSFDE_PVS / 64; ++q) {
    const int b = lane + 64 * q;
    in.pv[q] = p3[j >= 0 && b < g.nb3 ? b : 0];
  }
  const int lh = lane <= jj ? lane : 0, lr = lane < jj ? lane : 0;
  in.h = st->h[lh];
  in.h2 = st->h2[lh];
  in.cs = st->cs[lr];
  in.sn = st->sn[lr];
  in.gam = st->gam[jj];
  in.thr = st->sum.thr;
}

// Resolve of step `pend` from the fetched values (first wavefront), then one
// barrier.  The earlier rotations are applied in order with values broadcast
// from their lanes, followed by the new Givens rotation and the stopping test
// (Lemma Krylov: |g_{j+1}| is the residual norm of the least-squares problem).
// On return `o` (shared) holds the status and `col` the resolved column.
__device__ __forceinline__ void gm_resolve(const GmRes& g, const GmIn& in, GmOut* o, GmCol* col,
                                           bool writer) {
  GmresState* st = g.st;
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    const bool cand = g.pend >= 0;
    const int j = g.pend;
    const int fl_prev = in.fl;
    if (!cand) {
      if (lane == 0) {
        o->flag = fl_prev == GM_UNSET ? GM_CONVERGED : fl_prev;
        o->sc = in.vsc;
        o->k = in.kfin;
        col->j = -1;
      }
    } else if (fl_prev != GM_RUNNING) {
      // the cycle ended before step `pend`: its resolve stored kfin
      if (lane == 0) {
        o->flag = fl_prev == GM_UNSET ? GM_CONVERGED : fl_prev;
        o->k = in.kfin;
        o->sc = 0.0;
        col->j = -1;
      }
    } else {
      const double hl = lane <= j ? in.h + in.h2 : 0.0;
      const double cl = lane < j ? in.cs : 0.0;
      const double sl = lane < j ? in.sn : 0.0;
      double part = 0.0;
#pragma unroll
      for (int q = 0; q < RSFDE_PVS / 64; ++q) part += lane + 64 * q < g.nb3 ? in.pv[q] : 0.0;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off, 64);
      double hsz = fabs(hl);
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) hsz = fmax(hsz, __shfl_xor(hsz, off, 64));
      const double nu = gm_lane(part, 0);  // one lane's sum: the same bits in every block
      const double hn = sqrt(nu);
      const bool breakdown = !(hn > 1e-14 * hsz);
      double p = gm_lane(hl, 0);
      double rcl = 0.0;  // lane i keeps R(i, j)
      for (int i = 0; i < j; ++i) {
        const double c = gm_lane(cl, i), sg = gm_lane(sl, i), q = gm_lane(hl, i + 1);
        const double ri = c * p + sg * q;
        p = -sg * p + c * q;
        if (lane == i) rcl = ri;
      }
      const double r = hypot(p, hn);
      const double c = r > 0.0 ? p / r : 1.0;
      const double sg = r > 0.0 ? hn / r : 0.0;
      const double gj = c * in.gam;
      const double gn = -sg * in.gam;
      const double rr = fabs(gn);
      const double vn = hn > 0.0 ? 1.0 / hn : 0.0;
      if (lane == j) rcl = r;
      int flag;
      if (!isfinite(rr) || !isfinite(r)) flag = GM_NONFINITE;
      else if (rr <= in.thr) flag = GM_CONVERGED;
      else if (breakdown) flag = GM_BREAKDOWN;
      else if (j + 1 >= g.m) flag = GM_CYCLE_FULL;
      else flag = GM_RUNNING;
      const bool fin = flag != GM_RUNNING && flag != GM_NONFINITE;
      if (lane <= j) col->rc[lane] = rcl;
      if (writer) {
        constexpr int MX = RSFDE_MAX_RESTART;
        if (lane <= j) st->Rm[j * MX + lane] = rcl;
        if (lane == 0) {
          st->cs[j] = c;
          st->sn[j] = sg;
          st->gfin[j] = gj;
          st->gam[j + 1] = gn;
          st->vsc[j + 1] = vn;
          st->FL[j + 1] = flag;
          st->sum.res = rr;
          st->sum.flag = flag;
          if (fin) {
            st->kfin = j + 1;
            st->sum.k = j + 1;
          }
        }
      }
      if (lane == 0) {
        col->gj = gj;
        col->j = j;
        o->flag = flag;
        o->k = fin ? j + 1 : 0;
        o->sc = vn;
      }
    }
  }
  __syncthreads();
}

// Fetch and resolve (for kernels with nothing to overlap the fetch with).
__device__ __forceinline__ void gm_prologue(const GmRes& g, GmOut* o, GmCol* col, bool writer) {
  GmIn in;
  if (threadIdx.x < 64) gm_fetch(g, in);
  gm_resolve(g, in, o, col, writer);
}


struct KryArgs {
  const double* V;    // basis, column k at V + k*ldv
  int64_t ldv;
  int64_t n;
  double* w;          // working vector (column j+1 of V)
  GmresState* st;
  double* pa;         // sweep-A partials (dot products of the basis with w and with u_j)
  double* pb;         // sweep-D partials (sums with column j, when sweep A splits)
  double* pc;         // sweep-B partials (||u_{j+1}||^2)
  int j;              // Arnoldi index (w = P^{-1} A v_j)
  int m;              // restart length
  int nb;             // blocks of the sweeps (kry_blocks or kry_blocks_many)
};

// Blocks of the solution-update kernel for an n-vector.
inline int upd_blocks(int64_t n) {
  int64_t b = (n / 2 + 1023) / 1024;
  if (b > 1024) b = 1024;
  if (b < 1) b = 1;
  return (int)b;
}

// ---- batched Krylov launches: per-instance arguments in device memory, the
// instance of a block from the block prefix sums (as for the batched passes).
struct KBatch {
  KryArgs k;           // as for Arnoldi step 0 (w = column 1); j and w follow the launch
  double* x;           // solution the update kernel adds V y to
  double* partial;     // cycle-start norm partials
  double rtol, inner_rtol;
  int nb;              // blocks of this instance's sweeps and norm (KryArgs::nb)
  int nbu;             // blocks of this instance's update (upd_blocks(n))
  int mixed;
  int overwrite;       // the update writes x = V y instead of adding it (two-sided form)
};
struct KLaunch {
  const KBatch* desc;  // slot order
  const int* start;    // block prefix sums of the launch (per-instance block counts)
  const int* mask;     // update: slot s adds V y only when mask[s] != 0 (NULL: all)
  int ninst;
  int j, pend, first;
};

// Launchers (krylov.hip)
hipError_t kry_cycle_init(double* v0, int64_t n, int nb, GmresState* st, double* partial, int first,
                          double rtol, double inner_rtol, int mixed, int m, hipStream_t s);
// ea/eb: when non-null, HIP events stamped at the dispatch's start and end
hipError_t kry_sweep(int which, const KryArgs& a, hipStream_t s, hipEvent_t ea = nullptr,
                     hipEvent_t eb = nullptr);  // which = 1, 2, 3
// x += V y once the cycle has finished (x = V y when overwrite is set)
hipError_t kry_update(const double* V, int64_t ldv, int64_t n, double* x, const GmRes& g,
                      hipStream_t s, hipEvent_t ea = nullptr, hipEvent_t eb = nullptr,
                      int overwrite = 0);
hipError_t kry_state_reset(GmresState* st, hipStream_t s);
// batched forms: `nblocks` = start[ninst]; sweeps and norms use KBatch::nb blocks
// per instance, the update KBatch::nbu, the cycle-start finish one block per instance
hipError_t kry_sweep_batched(int which, const KLaunch& kl, int64_t nblocks, hipStream_t s,
                             hipEvent_t ea = nullptr, hipEvent_t eb = nullptr);
hipError_t kry_update_batched(const KLaunch& kl, int64_t nblocks, hipStream_t s,
                              hipEvent_t ea = nullptr, hipEvent_t eb = nullptr);
hipError_t kry_norm_batched(const KLaunch& kl, int64_t nblocks, hipStream_t s);
hipError_t kry_cycle_fin_batched(const KLaunch& kl, hipStream_t s);
// out[i] = summary of slot i (desc in device memory, n slots)
hipError_t kry_gather_summaries(const KBatch* desc, int n, GmresSummary* out, hipStream_t s);
