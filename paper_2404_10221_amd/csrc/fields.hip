// Field evaluation kernels (synthetic workloads) and the compact source operator.
#include <math.h>

#include "fields.h"
#include "rsfde.h"

__device__ __forceinline__ double sine_modes(const FieldDev& F, int d, const int* jc, const int* Ncl) {
  const int K = F.K;
  double acc = 0.0;
  if (d == 1) {
    for (int k1 = 0; k1 < K; ++k1) acc += F.amp[k1] * F.sintab[0][k1 * Ncl[0] + jc[0]];
  } else if (d == 2) {
    for (int k2 = 0; k2 < K; ++k2) {
      const double s2 = F.sintab[1][k2 * Ncl[1] + jc[1]];
      double inner = 0.0;
      for (int k1 = 0; k1 < K; ++k1) inner += F.amp[k1 + K * k2] * F.sintab[0][k1 * Ncl[0] + jc[0]];
      acc += inner * s2;
    }
  } else {
    for (int k3 = 0; k3 < K; ++k3) {
      const double s3 = F.sintab[2][k3 * Ncl[2] + jc[2]];
      for (int k2 = 0; k2 < K; ++k2) {
        const double s23 = s3 * F.sintab[1][k2 * Ncl[1] + jc[1]];
        double inner = 0.0;
        for (int k1 = 0; k1 < K; ++k1)
          inner += F.amp[k1 + K * (k2 + K * k3)] * F.sintab[0][k1 * Ncl[0] + jc[0]];
        acc += inner * s23;
      }
    }
  }
  return acc;
}

// The separable e families from their per-axis product p (one expression, shared
// by the generic and the grid-shaped kernels so that both round alike).
__device__ __forceinline__ double e_separable(const FieldDev& E, double p, double t, const TimeF& tf) {
  if (E.kind == RSFDE_FIELD_POLY_T) return E.c[0] + E.c[1] * (1.0 + E.c[2] * t) * p;
  return E.c[0] + E.c[1] * p * tf.cos_t;
}

__device__ __forceinline__ double e_value(const FieldDev& E, int d, const double* x, const int* jc,
                                          const int* Ncl, double t, const TimeF& tf) {
  switch (E.kind) {
    case RSFDE_FIELD_CONST:
      return E.c[0];
    case RSFDE_FIELD_SUMSQ_EXP: {
      double s = 0.0;
      for (int i = 0; i < d; ++i) s += x[i] * x[i];
      return (s + tf.exp_mt) / E.c[0];
    }
    case RSFDE_FIELD_POLY_T:       // p = prod_i x_i^c3 (table row AX_E)
    case RSFDE_FIELD_SINPROD_COS: {  // p = prod_i sin(pi x_i)
      double p = 1.0;
      for (int i = 0; i < d; ++i) p *= E.ax[i][AX_E * Ncl[i] + jc[i]];
      return e_separable(E, p, t, tf);
    }
    case RSFDE_FIELD_SINE_FIELD: {
      const double g = sine_modes(E, d, jc, Ncl);
      return E.c[0] + E.c[1] * 0.5 * (1.0 + g / E.norm);
    }
    default:
      return 0.0;
  }
}

__device__ __forceinline__ double poly_p(double x, int a) {
  const double b = x * (1.0 - x);
  double p = 1.0;
  for (int i = 0; i < a; ++i) p *= b;
  return p;
}

// Riesz derivative of x^a (1-x)^a from the Riemann-Liouville power rule; the
// coefficients (times the Gamma ratios) come from the host.
__device__ __forceinline__ double riesz_poly(const double* mc, double alpha, int a, double x) {
  double acc = 0.0;
  for (int k = 0; k <= 2 * a; ++k) {
    const double cl = mc[k], cr = mc[13 + k];
    if (cl != 0.0) acc += cl * pow(x, (double)k - alpha);
    if (cr != 0.0) acc += cr * pow(1.0 - x, (double)k - alpha);
  }
  return mc[26] * acc;
}

__device__ __forceinline__ void fields_eval_at(const FieldDev& E, const FieldDev& F, int which,
                                               const GridDev& g, double t, const TimeF& tf,
                                               double* __restrict__ out, int64_t idx) {
  if (idx >= g.size) return;
  const int d = g.d;
  int jc[3] = {0, 0, 0};
  int Ncl[3] = {1, 1, 1};
  double x[3] = {0.0, 0.0, 0.0};
  uint64_t r = (uint64_t)idx;
  for (int i = 0; i < d; ++i) {
    const unsigned ni = (unsigned)(g.closure ? g.N[i] + 2 : g.N[i]);
    unsigned ji;
    if (r < 0xffffffffull) {
      r = split_u32((unsigned)r, ni, g.inv[i], &ji);
    } else {
      ji = (unsigned)(r % ni);
      r /= ni;
    }
    jc[i] = (int)ji + (g.closure ? 0 : 1);
    Ncl[i] = g.N[i] + 2;
    x[i] = g.lo[i] + (double)jc[i] * g.h[i];
  }
  double v = 0.0;
  if (which == RSFDE_WHICH_E) {
    v = e_value(E, d, x, jc, Ncl, t, tf);
  } else if (which == RSFDE_WHICH_F) {
    if (F.kind == RSFDE_FIELD_SINE_MODES) {
      v = sine_modes(F, d, jc, Ncl);
    } else if (F.kind == RSFDE_FIELD_MANUFACTURED) {
      const double A = F.c[0] * tf.exp_mt;
      double pr[3];
      double u = A;
      for (int i = 0; i < d; ++i) {
        pr[i] = F.ax[i][AX_U * Ncl[i] + jc[i]];  // x_i^a (1 - x_i)^a
        u *= pr[i];
      }
      const double ev = e_value(E, d, x, jc, Ncl, t, tf);
      v = -ev * u;  // e u_t, u_t = -u
      for (int i = 0; i < d; ++i) {
        double other = A;
        for (int l = 0; l < d; ++l)
          if (l != i) other *= pr[l];
        v -= g.kappa[i] * other * F.ax[i][AX_RIESZ * Ncl[i] + jc[i]];
      }
    }
  } else {
    if (F.kind == RSFDE_FIELD_MANUFACTURED) {
      double u = F.c[0];
      for (int i = 0; i < d; ++i) u *= F.ax[i][AX_PSI * Ncl[i] + jc[i]];
      v = u;
    }
  }
  out[idx] = v;
}

__global__ void __launch_bounds__(256)
k_fields_eval(const FieldDev E, const FieldDev F, int which, const GridDev g, double t,
              const TimeF tf, double* __restrict__ out) {
  fields_eval_at(E, F, which, g, t, tf, out, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

// one launch for many instances: job[s] covers blocks start[s] .. start[s+1)
__global__ void __launch_bounds__(256)
k_fields_eval_b(const FieldJob* __restrict__ jobs, const int* __restrict__ start, int n, double t,
                const TimeF tf) {
  const int slot = batch_slot(start, n, blockIdx.x);
  const FieldJob& J = jobs[slot];
  fields_eval_at(J.e, J.f, J.which, J.g, t, tf, J.out,
                 (int64_t)((int)blockIdx.x - start[slot]) * blockDim.x + threadIdx.x);
}

// cos t and exp(-t), once per launch on the host
static TimeF time_factors(double t) { return TimeF{cos(t), exp(-t)}; }

hipError_t fields_eval_batched(const FieldJob* jobs, const int* start, int n, int64_t nblocks,
                               double t, hipStream_t s) {
  if (nblocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fields_eval_b, dim3((unsigned)nblocks), dim3(256), 0, s, jobs, start, n, t,
                     time_factors(t));
  return hipGetLastError();
}

// e of the separable families (POLY_T, SINPROD_COS) on a grid-shaped launch: x_1
// along the block's threads, x_2 and x_3 from the block indices, so no thread
// splits a flat index; p multiplies the axis factors in the order the generic
// kernel does.
template <int D>
__global__ void __launch_bounds__(256)
k_e_separable(const FieldDev E, const GridDev g, double t, const TimeF tf, double* __restrict__ out) {
  const int off = g.closure ? 0 : 1;
  const int n0 = g.closure ? g.N[0] + 2 : g.N[0];
  const int j0 = (int)blockIdx.x * 256 + (int)threadIdx.x;
  if (j0 >= n0) return;
  double p = 1.0;
  p *= E.ax[0][AX_E * (g.N[0] + 2) + j0 + off];
  int64_t row = 0;
  if constexpr (D >= 2) {
    const int j1 = (int)blockIdx.y;
    p *= E.ax[1][AX_E * (g.N[1] + 2) + j1 + off];
    row = j1;
  }
  if constexpr (D == 3) {
    const int j2 = (int)blockIdx.z;
    const int n1 = g.closure ? g.N[1] + 2 : g.N[1];
    p *= E.ax[2][AX_E * (g.N[2] + 2) + j2 + off];
    row += (int64_t)j2 * n1;
  }
  out[row * n0 + j0] = e_separable(E, p, t, tf);
}

hipError_t fields_eval(const FieldDev& e, const FieldDev& f, int which, const GridDev& g, double t,
                       double* out, hipStream_t s) {
  if (g.size == 0) return hipSuccess;
  if (which == RSFDE_WHICH_E && (e.kind == RSFDE_FIELD_POLY_T || e.kind == RSFDE_FIELD_SINPROD_COS)) {
    const int c = g.closure ? 2 : 0;
    const unsigned n0 = (unsigned)(g.N[0] + c);
    const unsigned n1 = g.d >= 2 ? (unsigned)(g.N[1] + c) : 1u;
    const unsigned n2 = g.d >= 3 ? (unsigned)(g.N[2] + c) : 1u;
    if (n1 <= 65535u && n2 <= 65535u) {
      const dim3 grid((n0 + 255) / 256, n1, n2);
      if (g.d == 1) hipLaunchKernelGGL(k_e_separable<1>, grid, dim3(256), 0, s, e, g, t, time_factors(t), out);
      else if (g.d == 2) hipLaunchKernelGGL(k_e_separable<2>, grid, dim3(256), 0, s, e, g, t, time_factors(t), out);
      else hipLaunchKernelGGL(k_e_separable<3>, grid, dim3(256), 0, s, e, g, t, time_factors(t), out);
      return hipGetLastError();
    }
  }
  hipLaunchKernelGGL(k_fields_eval, dim3((unsigned)((g.size + 255) / 256)), dim3(256), 0, s, e, f,
                     which, g, t, time_factors(t), out);
  return hipGetLastError();
}

__global__ void k_sintab(int K, int Ncl, double lo, double h, double* tab) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= K * Ncl) return;
  const int k = i / Ncl, j = i - k * Ncl;
  tab[i] = sinpi((double)(k + 1) * (lo + (double)j * h));
}

__global__ void k_axis_tables(const FieldDev E, const FieldDev F, const FieldDev P, const GridDev g,
                              int axis, double* __restrict__ tab) {
  const int Ncl = g.N[axis] + 2;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= Ncl) return;
  const double x = g.lo[axis] + (double)j * g.h[axis];
  double te = 0.0, tu = 0.0, tr = 0.0, tp = 0.0;
  if (E.kind == RSFDE_FIELD_POLY_T) te = pow(x, E.c[3]);
  else if (E.kind == RSFDE_FIELD_SINPROD_COS) te = sinpi(x);
  if (F.kind == RSFDE_FIELD_MANUFACTURED) {
    tu = poly_p(x, F.a);
    const double* mc = F.mc + axis * RSFDE_MC_STRIDE;
    tr = riesz_poly(mc, mc[27], F.a, x);
  }
  if (P.kind == RSFDE_FIELD_MANUFACTURED) tp = poly_p(x, P.a);
  tab[AX_E * Ncl + j] = te;
  tab[AX_U * Ncl + j] = tu;
  tab[AX_RIESZ * Ncl + j] = tr;
  tab[AX_PSI * Ncl + j] = tp;
}

hipError_t fields_axis_tables(const FieldDev& e, const FieldDev& f, const FieldDev& psi,
                              const GridDev& g, int axis, double* tab, hipStream_t s) {
  const int Ncl = g.N[axis] + 2;
  hipLaunchKernelGGL(k_axis_tables, dim3((Ncl + 255) / 256), dim3(256), 0, s, e, f, psi, g, axis, tab);
  return hipGetLastError();
}

hipError_t fields_sintab(int K, int Ncl, double lo, double h, double* tab, hipStream_t s) {
  hipLaunchKernelGGL(k_sintab, dim3((K * Ncl + 255) / 256), dim3(256), 0, s, K, Ncl, lo, h, tab);
  return hipGetLastError();
}

// F_J = sum over the 3^d neighbours of prod_i w_i(a_i) f_{J+a} on the closure
// grid, w(0) = 1 - alpha_i/12, w(+-1) = alpha_i/24 (every interior index lies
// inside the stencil's support, so H acts as the stencil on each axis).
template <int D>
__device__ __forceinline__ void compute_F_d(const double* __restrict__ fcl, const GridDev& g,
                                            const double (&al)[3], double* __restrict__ F,
                                            int64_t idx) {
  if (idx >= g.size) return;
  int j[3] = {0, 0, 0};
  int64_t sc[3] = {0, 0, 0};
  uint64_t r = (uint64_t)idx;
  int64_t stride = 1;
#pragma unroll
  for (int i = 0; i < D; ++i) {
    const unsigned ni = (unsigned)g.N[i];
    if (r < 0xffffffffull) {
      unsigned ji;
      r = split_u32((unsigned)r, ni, g.inv[i], &ji);
      j[i] = (int)ji + 1;
    } else {
      j[i] = (int)(r % ni) + 1;
      r /= ni;
    }
    sc[i] = stride;
    stride *= (g.N[i] + 2);
  }
  int64_t c0 = 0;
#pragma unroll
  for (int i = 0; i < D; ++i) c0 += (int64_t)j[i] * sc[i];
  double w[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const double a = i < D ? al[i] : 0.0;
    w[i][0] = a / 24.0;
    w[i][1] = i < D ? 1.0 - a / 12.0 : 1.0;
    w[i][2] = a / 24.0;
  }
  // all 3^D loads in flight together; the sums in the same order as written
  constexpr int n2 = D >= 2 ? 3 : 1, n3 = D >= 3 ? 3 : 1;
  double fv[n3][n2][3];
#pragma unroll
  for (int c = 0; c < n3; ++c)
#pragma unroll
    for (int b = 0; b < n2; ++b) {
      const int64_t off = c0 + (D >= 3 ? (int64_t)(c - 1) * sc[2] : 0) + (D >= 2 ? (int64_t)(b - 1) * sc[1] : 0);
      fv[c][b][0] = fcl[off - 1];
      fv[c][b][1] = fcl[off];
      fv[c][b][2] = fcl[off + 1];
    }
  double acc = 0.0;
#pragma unroll
  for (int c = 0; c < n3; ++c)
#pragma unroll
    for (int b = 0; b < n2; ++b) {
      const double wbc = (D >= 3 ? w[2][c] : 1.0) * (D >= 2 ? w[1][b] : 1.0);
      acc += wbc * (w[0][0] * fv[c][b][0] + w[0][1] * fv[c][b][1] + w[0][2] * fv[c][b][2]);
    }
  F[idx] = acc;
}

__device__ __forceinline__ void compute_F_at(const double* __restrict__ fcl, const GridDev& g,
                                             double a0, double a1, double a2,
                                             double* __restrict__ F, int64_t idx) {
  const double al[3] = {a0, a1, a2};
  if (g.d == 1) compute_F_d<1>(fcl, g, al, F, idx);
  else if (g.d == 2) compute_F_d<2>(fcl, g, al, F, idx);
  else compute_F_d<3>(fcl, g, al, F, idx);
}

__global__ void __launch_bounds__(256)
k_compute_F(const double* __restrict__ fcl, const GridDev g, double a0, double a1, double a2,
            double* __restrict__ F) {
  compute_F_at(fcl, g, a0, a1, a2, F, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

__global__ void __launch_bounds__(256)
k_compute_F_b(const FJob* __restrict__ jobs, const int* __restrict__ start, int n) {
  const int slot = batch_slot(start, n, blockIdx.x);
  const FJob& J = jobs[slot];
  compute_F_at(J.fcl, J.g, J.al[0], J.al[1], J.al[2], J.F,
               (int64_t)((int)blockIdx.x - start[slot]) * blockDim.x + threadIdx.x);
}

hipError_t compute_F_batched(const FJob* jobs, const int* start, int n, int64_t nblocks,
                             hipStream_t s) {
  if (nblocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_compute_F_b, dim3((unsigned)nblocks), dim3(256), 0, s, jobs, start, n);
  return hipGetLastError();
}

hipError_t compute_F(const double* fcl, const GridDev& g, const double* alpha, double* F,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_compute_F, dim3((unsigned)((g.size + 255) / 256)), dim3(256), 0, s, fcl, g,
                     alpha[0], alpha[1], alpha[2], F);
  return hipGetLastError();
}

__global__ void k_minmax_reset(double* mm) {
  mm[0] = INFINITY;
  mm[1] = -INFINITY;
}

hipError_t minmax_reset(double* mm, hipStream_t s) {
  hipLaunchKernelGGL(k_minmax_reset, dim3(1), dim3(1), 0, s, mm);
  return hipGetLastError();
}

// per-block extremes (no cross-block synchronisation)
__global__ void __launch_bounds__(256)
k_minmax_part(const double* __restrict__ e, int64_t n, double* __restrict__ partial) {
  double lo = INFINITY, hi = -INFINITY;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const double v = e[i];
    lo = fmin(lo, v);
    hi = fmax(hi, v);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, off, 64));
    hi = fmax(hi, __shfl_xor(hi, off, 64));
  }
  __shared__ double sl[4], sh[4];
  if ((threadIdx.x & 63) == 0) {
    sl[threadIdx.x >> 6] = lo;
    sh[threadIdx.x >> 6] = hi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 4; ++w) {
      lo = fmin(lo, sl[w]);
      hi = fmax(hi, sh[w]);
    }
    partial[2 * blockIdx.x] = lo;
    partial[2 * blockIdx.x + 1] = hi;
  }
}

// one workgroup folds the block extremes into the running mm[0..1]
__global__ void __launch_bounds__(256)
k_minmax_fin(const double* __restrict__ partial, int nblocks, double* mm) {
  double lo = INFINITY, hi = -INFINITY;
  for (int b = threadIdx.x; b < nblocks; b += blockDim.x) {
    lo = fmin(lo, partial[2 * b]);
    hi = fmax(hi, partial[2 * b + 1]);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, off, 64));
    hi = fmax(hi, __shfl_xor(hi, off, 64));
  }
  __shared__ double sl[4], sh[4];
  if ((threadIdx.x & 63) == 0) {
    sl[threadIdx.x >> 6] = lo;
    sh[threadIdx.x >> 6] = hi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double L = mm[0], H = mm[1];
    for (int w = 0; w < 4; ++w) {
      L = fmin(L, sl[w]);
      H = fmax(H, sh[w]);
    }
    mm[0] = L;
    mm[1] = H;
  }
}

hipError_t minmax_accum(const double* e, int64_t n, double* mm, double* partial, unsigned* counter,
                        hipStream_t s) {
  (void)counter;
  int64_t b = (n + 2047) / 2048;
  if (b > 512) b = 512;
  if (b < 1) b = 1;
  hipLaunchKernelGGL(k_minmax_part, dim3((unsigned)b), dim3(256), 0, s, e, n, partial);
  hipLaunchKernelGGL(k_minmax_fin, dim3(1), dim3(256), 0, s, partial, (int)b, mm);
  return hipGetLastError();
}

__global__ void k_f64_f32(const double* __restrict__ in, float* __restrict__ out, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) out[i] = (float)in[i];
}

hipError_t convert_f64_f32(const double* in, float* out, int64_t n, hipStream_t s) {
  int64_t b = (n + 1023) / 1024;
  if (b > 4096) b = 4096;
  if (b < 1) b = 1;
  hipLaunchKernelGGL(k_f64_f32, dim3((unsigned)b), dim3(256), 0, s, in, out, n);
  return hipGetLastError();
}

__global__ void k_fill(double* __restrict__ x, int64_t n, double v) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) x[i] = v;
}

hipError_t fill_f64(double* x, int64_t n, double v, hipStream_t s) {
  int64_t b = (n + 1023) / 1024;
  if (b > 4096) b = 4096;
  if (b < 1) b = 1;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)b), dim3(256), 0, s, x, n, v);
  return hipGetLastError();
}
