// Coefficient builder (runs once per setup; the preconditioner does not depend
// on the time step, Section 3 remark).
#include <math.h>

#include "setup.h"

// s_0..s_{N-1}: s_0 = Gamma(alpha+1)/Gamma(alpha/2+1)^2 and
// s_k = r_k s_{k-1}, r_k = 1 - (alpha+1)/(alpha/2+k) (eq. eq0 recurrence),
// computed as a prefix product: each of the 64 lanes multiplies the factors of
// its chunk, an exclusive multiplicative scan across lanes joins the chunks.
__global__ void __launch_bounds__(64) k_fcd_weights(double alpha, int N, double* __restrict__ s) {
  const int lane = threadIdx.x;
  const int C = (N + 63) / 64;
  const int k0 = lane * C, k1 = min(N, k0 + C);
  double chunk = 1.0;
  for (int k = max(k0, 1); k < k1; ++k) chunk *= 1.0 - (alpha + 1.0) / (alpha / 2.0 + (double)k);
  // exclusive product scan over lanes
  double incl = chunk;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const double o = __shfl_up(incl, off, 64);
    if (lane >= off) incl *= o;
  }
  double excl = __shfl_up(incl, 1, 64);
  if (lane == 0) excl = 1.0;
  const double g = tgamma(alpha / 2.0 + 1.0);
  double run = tgamma(alpha + 1.0) / (g * g) * excl;
  for (int k = k0; k < k1; ++k) {
    if (k > 0) run *= 1.0 - (alpha + 1.0) / (alpha / 2.0 + (double)k);
    s[k] = run;
  }
}

// exp(-2 pi i k / L) in FP64 and FP32.
__global__ void k_twiddles(int L, cpx<double>* __restrict__ t64, cpx<float>* __restrict__ t32) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= L) return;
  double sn, cs;
  sincospi(-2.0 * (double)k / (double)L, &sn, &cs);
  t64[k] = cpx<double>{cs, sn};
  t32[k] = cpx<float>{(float)cs, (float)sn};
}

// B eigenvalues (Lemma Heig) lambda_k = 1 - (alpha/6) sin^2(k pi / (2N+2)), k = 1..N
// stored at [k-1], and eta q_{k-1} / lambda_k for the 1/mu scaling.
__global__ void k_lam_wq(double alpha, int N, double eta, const double* __restrict__ q,
                         double* __restrict__ lam64, float* __restrict__ lam32,
                         double* __restrict__ wq64, float* __restrict__ wq32) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const double sp = sinpi((double)(i + 1) / (2.0 * (double)(N + 1)));
  const double lam = 1.0 - alpha / 6.0 * sp * sp;
  const double w = eta * q[i] / lam;
  lam64[i] = lam;
  lam32[i] = (float)lam;
  wq64[i] = w;
  wq32[i] = (float)w;
}

__global__ void __launch_bounds__(256)
k_strang_eigs(int N, double alpha, double eta, const double* __restrict__ s, double* __restrict__ lam,
              double* __restrict__ wq) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  double sig = 0.0;
  for (int k = 0; k < N; ++k) {
    const double c = k <= N / 2 ? s[k] : s[N - k];
    const long long r = ((long long)j * k) % N;  // angle 2 pi jk/N reduced mod 2 pi
    sig += c * cospi(2.0 * (double)r / (double)N);
  }
  const double b = (1.0 - alpha / 12.0) + alpha / 12.0 * cospi(2.0 * (double)j / (double)N);
  lam[j] = b;
  wq[j] = eta * sig / b;
}

hipError_t setup_strang_tables(int L, double alpha, int N, double eta, const double* s,
                               const cpx<double>* tw64, cpx<double>* chirp, cpx<double>* khat,
                               double* lam, double* wq, hipStream_t st) {
  hipLaunchKernelGGL(k_strang_eigs, dim3((N + 255) / 256), dim3(256), 0, st, N, alpha, eta, s, lam, wq);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_dht_tables(L, N, tw64, chirp, khat, st);
}

hipError_t setup_axis_tables(double alpha, int N, int L, double eta, double* s, cpx<double>* tw64,
                             cpx<float>* tw32, double* chat64, float* chat32, double* q,
                             double* lam64, float* lam32, double* wq64, float* wq32,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_fcd_weights, dim3(1), dim3(64), 0, st, alpha, N, s);
  hipLaunchKernelGGL(k_twiddles, dim3((L + 255) / 256), dim3(256), 0, st, L, tw64, tw32);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = launch_spectrum(L, s, N, tw64, chat64, chat32, q, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_lam_wq, dim3((N + 255) / 256), dim3(256), 0, st, alpha, N, eta, q, lam64,
                     lam32, wq64, wq32);
  return hipGetLastError();
}
