// One instantiation unit of the pencil pass kernels and the setup spectrum
// kernel; compiled once per transform length with -DRSFDE_PASS_L=<L> so the
// lengths build in parallel.
#include "dht.h"
#include "pass.h"
#include "setup.h"

#ifndef RSFDE_PASS_L
#error "RSFDE_PASS_L must be defined"
#endif

RSFDE_INSTANTIATE_PASS(double, RSFDE_PASS_L)
RSFDE_INSTANTIATE_PASS(float, RSFDE_PASS_L)
RSFDE_INSTANTIATE_DHT(RSFDE_PASS_L)

// Spectrum of the circulant embedding c = [t_0..t_{N-1}, 0, 0, 0, t_{N-1}..t_1]
// (length L = 2(N+1)) of the symmetric Toeplitz factor: FFT(c) is real and even,
// its entries 1..N are the tau eigenvalues q_0..q_{N-1} of eq. q, and FFT(c)/L is
// the multiplier of the circulant product (inverse FFT unnormalised).
template <int L>
__global__ void __launch_bounds__(FftPlan<L>::T)
k_spectrum(const double* __restrict__ s, int N, const cpx<double>* __restrict__ tw,
           double* __restrict__ chat64, float* __restrict__ chat32, double* __restrict__ q) {
  constexpr int T = FftPlan<L>::T;
  __shared__ cpx<double> bufs[LdsSeq<double, L>::size];
  const LdsSeq<double, L> buf{bufs};
  __shared__ cpx<double> twl[TwHalf<double, L>::size];
  const int t = threadIdx.x;
  double twr[TwFill<double, L, T>::C], twi[TwFill<double, L, T>::C];
  tw_load<double, L, T>(twr, twi, tw, t);
  tw_store<double, L, T>(twr, twi, twl, t);
  const TwHalf<double, L> twp{twl};
  for (int k = t; k < L; k += T) {
    double c = 0.0;
    if (k < N) c = s[k];
    else if (k >= N + 3) c = s[L - k];
    buf[k] = cpx<double>{c, 0.0};
  }
  __syncthreads();
  fft_lds<double, L, -1>(buf, t, twp);
  for (int k = t; k < L; k += T) {
    const double re = buf[k].x;
    chat64[k] = re / (double)L;
    chat32[k] = (float)(re / (double)L);
    if (k >= 1 && k <= N) q[k - 1] = re;
  }
}

template <>
hipError_t launch_spectrum_L<RSFDE_PASS_L>(const double* s, int N, const cpx<double>* tw64,
                                           double* chat64, float* chat32, double* q,
                                           hipStream_t st) {
  hipLaunchKernelGGL((k_spectrum<RSFDE_PASS_L>), dim3(1), dim3(FftPlan<RSFDE_PASS_L>::T), 0, st, s, N,
                     tw64, chat64, chat32, q);
  return hipGetLastError();
}
