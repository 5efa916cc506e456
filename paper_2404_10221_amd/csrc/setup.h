// Setup-time coefficient tables of one axis.
#pragma once
#include "common.h"

// Circulant spectrum of the Toeplitz factor by an LDS FFT of its embedding
// (defined per length in the pass instantiation units).
template <int L>
hipError_t launch_spectrum_L(const double* s, int N, const cpx<double>* tw64, double* chat64,
                             float* chat32, double* q, hipStream_t st);

hipError_t launch_spectrum(int L, const double* s, int N, const cpx<double>* tw64, double* chat64,
                           float* chat32, double* q, hipStream_t st);

// Strang circulant preconditioner of one axis: eigenvalues of the Strang
// circulants of B and S (Fourier order) and the Bluestein chirp tables.
hipError_t launch_dht_tables(int L, int N, const cpx<double>* tw64, cpx<double>* chirp,
                             cpx<double>* khat, hipStream_t st);
hipError_t setup_strang_tables(int L, double alpha, int N, double eta, const double* s,
                               const cpx<double>* tw64, cpx<double>* chirp, cpx<double>* khat,
                               double* lam, double* wq, hipStream_t st);

hipError_t setup_axis_tables(double alpha, int N, int L, double eta, double* s, cpx<double>* tw64,
                             cpx<float>* tw32, double* chat64, float* chat32, double* q,
                             double* lam64, float* lam32, double* wq64, float* wq32,
                             hipStream_t st);
