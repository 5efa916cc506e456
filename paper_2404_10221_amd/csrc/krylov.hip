// Arnoldi (CGS2), Givens least-squares and solution-update kernels.
#include <math.h>

#include "krylov.h"

#define PST (RSFDE_MAX_RESTART + 1)  // partial-sum stride per block
#define NWAVE (RSFDE_KRY_THREADS / 64)

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

// Block-level sums of acc[0..nv) written to dst[0..nv) (fixed order).
template <int KM>
__device__ __forceinline__ void block_partials(const double (&acc)[KM], int nv, double* dst) {
  __shared__ double sh[NWAVE][KM];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < KM; ++k) {
    if (k < nv) {
      const double x = wave_sum(acc[k]);
      if (lane == 0) sh[wv][k] = x;
    }
  }
  __syncthreads();
  if ((int)threadIdx.x < nv) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NWAVE; ++w) s += sh[w][threadIdx.x];
    dst[threadIdx.x] = s;
  }
}

// True in the one block that finishes last; every block must call it.
__device__ __forceinline__ bool last_block(unsigned* counter) {
  __shared__ int amlast;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned tk = atomicAdd(counter, 1u);
    amlast = (tk == gridDim.x - 1);
  }
  __syncthreads();
  if (amlast) __threadfence();
  return amlast != 0;
}

// In the last block: out[k] = sum over blocks of partial[b*PST + k], k < nv, in a
// fixed order; result left in `res` (shared, length >= nv).  Resets the counter.
__device__ __forceinline__ void final_sums(const double* partial, int nblocks, int nv, double* res,
                                          unsigned* counter) {
  __shared__ double sh[RSFDE_KRY_THREADS];
  int KS = 1;
  while (KS < nv) KS <<= 1;
  const int ng = RSFDE_KRY_THREADS / KS;
  const int k = threadIdx.x % KS, g = threadIdx.x / KS;
  double s = 0.0;
  if (k < nv && g < ng) {
    for (int b = g; b < nblocks; b += ng) s += partial[(int64_t)b * PST + k];
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  if ((int)threadIdx.x < nv) {
    double t = 0.0;
    for (int gg = 0; gg < ng; ++gg) t += sh[gg * KS + threadIdx.x];
    res[threadIdx.x] = t;
  }
  if (threadIdx.x == 0) *counter = 0u;
  __syncthreads();
}

// ---- cycle start: beta = ||v0||, g = beta e_1, v0 scale 1/beta ---------------
__global__ void __launch_bounds__(RSFDE_KRY_THREADS)
k_cycle_init(const double* __restrict__ v0, int64_t n, GmresState* st, double* partial,
             unsigned* counter, int first, double rtol, double inner_rtol, int mixed) {
  double acc[1] = {0.0};
  const int64_t stride = (int64_t)gridDim.x * RSFDE_KRY_THREADS;
  for (int64_t i = (int64_t)blockIdx.x * RSFDE_KRY_THREADS + threadIdx.x; i < n; i += stride) {
    const double x = v0[i];
    acc[0] += x * x;
  }
  block_partials<1>(acc, 1, partial + (int64_t)blockIdx.x * PST);
  if (!last_block(counter)) return;
  __shared__ double res[RSFDE_MAX_RESTART + 1];
  final_sums(partial, gridDim.x, 1, res, counter);
  if (threadIdx.x == 0) {
    const double beta = sqrt(res[0]);
    GmresSummary& S = st->sum;
    if (first) S.beta0 = beta;
    S.beta = beta;
    S.res = beta;
    S.k = 0;
    S.applied = 0;
    S.thr = mixed ? inner_rtol * beta : rtol * S.beta0;
    st->g[0] = beta;
    st->vsc[0] = beta > 0.0 ? 1.0 / beta : 0.0;
    if (!isfinite(beta)) S.flag = GM_NONFINITE;
    else if (beta == 0.0 || (!first && beta <= rtol * S.beta0)) S.flag = GM_CONVERGED;
    else S.flag = GM_RUNNING;
  }
}

// ---- CGS2 sweep 1: h = V^T w --------------------------------------------------
template <int KM>
__global__ void __launch_bounds__(RSFDE_KRY_THREADS) k_dots(const KryArgs a) {
  GmresState* st = a.st;
  if (st->sum.flag != GM_RUNNING) return;
  const int nv = a.j + 1;
  double acc[KM];
#pragma unroll
  for (int k = 0; k < KM; ++k) acc[k] = 0.0;
  const double* __restrict__ w = a.w;
  const double* __restrict__ V = a.V;
  const int64_t stride = (int64_t)gridDim.x * RSFDE_KRY_THREADS;
  for (int64_t i = (int64_t)blockIdx.x * RSFDE_KRY_THREADS + threadIdx.x; i < a.n; i += stride) {
    const double wi = w[i];
#pragma unroll
    for (int k = 0; k < KM; ++k)
      if (k < nv) acc[k] += V[k * a.ldv + i] * wi;
  }
  block_partials<KM>(acc, nv, a.partial + (int64_t)blockIdx.x * PST);
  if (!last_block(a.counter)) return;
  __shared__ double res[RSFDE_MAX_RESTART + 1];
  final_sums(a.partial, gridDim.x, nv, res, a.counter);
  if ((int)threadIdx.x < nv) st->h[threadIdx.x] = res[threadIdx.x] * st->vsc[threadIdx.x];
}

// ---- CGS2 sweep 2: w -= V h ; h2 = V^T w ----------------------------------------
template <int KM>
__global__ void __launch_bounds__(RSFDE_KRY_THREADS) k_orth_dots(const KryArgs a) {
  GmresState* st = a.st;
  if (st->sum.flag != GM_RUNNING) return;
  const int nv = a.j + 1;
  __shared__ double cf[KM];
  if ((int)threadIdx.x < KM) cf[threadIdx.x] = (int)threadIdx.x < nv ? st->h[threadIdx.x] * st->vsc[threadIdx.x] : 0.0;
  __syncthreads();
  double acc[KM];
#pragma unroll
  for (int k = 0; k < KM; ++k) acc[k] = 0.0;
  double* __restrict__ w = a.w;
  const double* __restrict__ V = a.V;
  const int64_t stride = (int64_t)gridDim.x * RSFDE_KRY_THREADS;
  for (int64_t i = (int64_t)blockIdx.x * RSFDE_KRY_THREADS + threadIdx.x; i < a.n; i += stride) {
    double wi = w[i];
#pragma unroll
    for (int k = 0; k < KM; ++k)
      if (k < nv) wi -= cf[k] * V[k * a.ldv + i];
    w[i] = wi;
#pragma unroll
    for (int k = 0; k < KM; ++k)
      if (k < nv) acc[k] += V[k * a.ldv + i] * wi;
  }
  block_partials<KM>(acc, nv, a.partial + (int64_t)blockIdx.x * PST);
  if (!last_block(a.counter)) return;
  __shared__ double res[RSFDE_MAX_RESTART + 1];
  final_sums(a.partial, gridDim.x, nv, res, a.counter);
  if ((int)threadIdx.x < nv) st->h2[threadIdx.x] = res[threadIdx.x] * st->vsc[threadIdx.x];
}

// ---- CGS2 sweep 3: w -= V h2 ; ||w|| ; Givens update of the least-squares problem
template <int KM>
__global__ void __launch_bounds__(RSFDE_KRY_THREADS) k_orth_norm_givens(const KryArgs a) {
  GmresState* st = a.st;
  if (st->sum.flag != GM_RUNNING) return;
  const int nv = a.j + 1;
  __shared__ double cf[KM];
  if ((int)threadIdx.x < KM) cf[threadIdx.x] = (int)threadIdx.x < nv ? st->h2[threadIdx.x] * st->vsc[threadIdx.x] : 0.0;
  __syncthreads();
  double acc[1] = {0.0};
  double* __restrict__ w = a.w;
  const double* __restrict__ V = a.V;
  const int64_t stride = (int64_t)gridDim.x * RSFDE_KRY_THREADS;
  for (int64_t i = (int64_t)blockIdx.x * RSFDE_KRY_THREADS + threadIdx.x; i < a.n; i += stride) {
    double wi = w[i];
#pragma unroll
    for (int k = 0; k < KM; ++k)
      if (k < nv) wi -= cf[k] * V[k * a.ldv + i];
    w[i] = wi;
    acc[0] += wi * wi;
  }
  block_partials<1>(acc, 1, a.partial + (int64_t)blockIdx.x * PST);
  if (!last_block(a.counter)) return;
  __shared__ double res[RSFDE_MAX_RESTART + 1];
  final_sums(a.partial, gridDim.x, 1, res, a.counter);
  if (threadIdx.x != 0) return;
  const int j = a.j;
  const int MX = RSFDE_MAX_RESTART;
  double hc[RSFDE_MAX_RESTART + 1];
  for (int i = 0; i <= j; ++i) hc[i] = st->h[i] + st->h2[i];
  const double hn = sqrt(res[0]);
  double hsz = 0.0;
  for (int i = 0; i <= j; ++i) hsz = fmax(hsz, fabs(hc[i]));
  const bool breakdown = !(hn > 1e-14 * hsz);
  // previous rotations
  for (int i = 0; i < j; ++i) {
    const double p = hc[i], q = hc[i + 1];
    hc[i] = st->cs[i] * p + st->sn[i] * q;
    hc[i + 1] = -st->sn[i] * p + st->cs[i] * q;
  }
  const double r = hypot(hc[j], hn);
  const double c = r > 0.0 ? hc[j] / r : 1.0;
  const double sgiv = r > 0.0 ? hn / r : 0.0;
  st->cs[j] = c;
  st->sn[j] = sgiv;
  for (int i = 0; i < j; ++i) st->Rm[j * MX + i] = hc[i];
  st->Rm[j * MX + j] = r;
  const double gj = st->g[j];
  st->g[j] = c * gj;
  st->g[j + 1] = -sgiv * gj;
  st->vsc[j + 1] = hn > 0.0 ? 1.0 / hn : 0.0;
  GmresSummary& S = st->sum;
  const double rr = fabs(st->g[j + 1]);
  S.res = rr;
  int flag;
  if (!isfinite(rr) || !isfinite(r)) flag = GM_NONFINITE;
  else if (rr <= S.thr) flag = GM_CONVERGED;
  else if (breakdown) flag = GM_BREAKDOWN;
  else if (j + 1 >= a.m) flag = GM_CYCLE_FULL;
  else flag = GM_RUNNING;
  if (flag != GM_RUNNING && flag != GM_NONFINITE) {
    const int k = j + 1;
    // back substitution R y = g
    for (int i = k - 1; i >= 0; --i) {
      double s = st->g[i];
      for (int l = i + 1; l < k; ++l) s -= st->Rm[l * MX + i] * st->y[l];
      st->y[i] = s / st->Rm[i * MX + i];
    }
    S.k = k;
  }
  S.flag = flag;
}

// ---- x += V y (once per cycle) ---------------------------------------------------
__global__ void __launch_bounds__(RSFDE_KRY_THREADS)
k_update(const double* __restrict__ V, int64_t ldv, int64_t n, double* __restrict__ x,
         GmresState* st, unsigned* counter) {
  const GmresSummary S = st->sum;
  if (S.flag == GM_RUNNING || S.flag == GM_NONFINITE || S.applied) return;
  const int k = S.k;
  __shared__ double cf[RSFDE_MAX_RESTART];
  if ((int)threadIdx.x < k) cf[threadIdx.x] = st->y[threadIdx.x] * st->vsc[threadIdx.x];
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * RSFDE_KRY_THREADS;
  for (int64_t i = (int64_t)blockIdx.x * RSFDE_KRY_THREADS + threadIdx.x; i < n; i += stride) {
    double xi = x[i];
    for (int l = 0; l < k; ++l) xi += cf[l] * V[l * ldv + i];
    x[i] = xi;
  }
  if (!last_block(counter)) return;
  if (threadIdx.x == 0) {
    st->sum.applied = 1;
    *counter = 0u;
  }
}

__global__ void k_state_reset(GmresState* st, unsigned* counter) {
  if (threadIdx.x == 0) {
    st->sum.flag = GM_RUNNING;
    st->sum.k = 0;
    st->sum.applied = 1;
    st->sum.beta0 = 0.0;
    st->sum.beta = 0.0;
    st->sum.thr = 0.0;
    st->sum.res = 0.0;
    *counter = 0u;
  }
}

// ---- launchers --------------------------------------------------------------------
hipError_t kry_cycle_init(double* v0, int64_t n, GmresState* st, double* partial, unsigned* counter,
                          int first, double rtol, double inner_rtol, int mixed, hipStream_t s) {
  hipLaunchKernelGGL(k_cycle_init, dim3(kry_blocks(n)), dim3(RSFDE_KRY_THREADS), 0, s, v0, n, st,
                     partial, counter, first, rtol, inner_rtol, mixed);
  return hipGetLastError();
}

#define KRY_DISPATCH(KERNEL, a, s)                                                              \
  do {                                                                                          \
    const int nv = (a).j + 1;                                                                   \
    const dim3 g(kry_blocks((a).n)), b(RSFDE_KRY_THREADS);                                       \
    if (nv <= 8) hipLaunchKernelGGL(KERNEL<8>, g, b, 0, s, a);                                  \
    else if (nv <= 16) hipLaunchKernelGGL(KERNEL<16>, g, b, 0, s, a);                           \
    else if (nv <= 32) hipLaunchKernelGGL(KERNEL<32>, g, b, 0, s, a);                           \
    else hipLaunchKernelGGL(KERNEL<64>, g, b, 0, s, a);                                         \
  } while (0)

hipError_t kry_dots(const KryArgs& a, hipStream_t s) {
  KRY_DISPATCH(k_dots, a, s);
  return hipGetLastError();
}
hipError_t kry_orth_dots(const KryArgs& a, hipStream_t s) {
  KRY_DISPATCH(k_orth_dots, a, s);
  return hipGetLastError();
}
hipError_t kry_orth_norm_givens(const KryArgs& a, hipStream_t s) {
  KRY_DISPATCH(k_orth_norm_givens, a, s);
  return hipGetLastError();
}
hipError_t kry_update(const double* V, int64_t ldv, int64_t n, double* x, GmresState* st,
                      unsigned* counter, hipStream_t s) {
  hipLaunchKernelGGL(k_update, dim3(kry_blocks(n)), dim3(RSFDE_KRY_THREADS), 0, s, V, ldv, n, x, st,
                     counter);
  return hipGetLastError();
}
hipError_t kry_state_reset(GmresState* st, unsigned* counter, hipStream_t s) {
  hipLaunchKernelGGL(k_state_reset, dim3(1), dim3(64), 0, s, st, counter);
  return hipGetLastError();
}
