// Pencil passes of the Strang circulant preconditioner (the paper's comparison
// solver, Section 4): (ebar c(B) + c(S))^{-1} r.
//
// Every factor is a Strang circulant, so the operator is a d-level circulant whose
// eigenvalues m_J (discrete-Fourier order) are even in each index.  For such an
// operator the separable Hartley transform H (H_{jk} = cos + sin of 2 pi jk/N_l on
// each axis) diagonalises it as well: M^{-1} = (1/prod N_l) H diag(1/m) H, with H
// real and its own inverse up to N.  So the solve is a chain of real pencil
// passes like the sine-transform chain of the tau preconditioner: H along axes
// d-1..1, then H, 1/m, H along axis 0, then H along axes 1..d-1.
//
// The pencil length N_l is odd (N_l + 1 = 2^p or 3 2^p), so each length-N DFT is
// taken by Bluestein's chirp factorisation nk = (n^2 + k^2 - (k-n)^2)/2 as a
// cyclic convolution of length L = 2(N+1) >= 2N-1, on the same LDS FFT as the
// other passes.  Two real pencils travel as one complex sequence z = x + i y and
// are separated after the transform by Z_k and conj(Z_{N-k}).
#pragma once
#include "fft.h"
#include "krylov.h"

enum : int { DHT_PLAIN = 0, DHT_SCALE = 1 };

struct DhtArgs {
  int op;                     // DHT_PLAIN, or DHT_SCALE (axis 0: H, 1/m, H)
  int N, d, axis;
  int64_t inner;              // element stride of the pass axis
  int64_t npencil;            // pencils (= n / N)
  int64_t npairs;             // pencil pairs (workgroups that do work)
  int xcd_remap;              // strided axes: consecutive pairs on one XCD
  int pad;
  const double* in;
  double* out;
  const cpx<double>* chirp;   // w_n = exp(i pi n^2 / N), n < N
  const cpx<double>* khat;    // FFT_L of the chirp kernel, divided by L
  const cpx<double>* tw;      // exp(-2 pi i k / L), k < L
  const double* lam[3];       // Strang eigenvalues of B_{alpha_l} (Fourier order)
  const double* wq[3];        // eta_l sigma_l / b_l, sigma_l those of S_{alpha_l}
  int Nax[3];
  const double* ebar;
  double pscale;              // 1 / prod_l N_l
  const int* stop_fl;         // exit unless *stop_fl == running (NULL: always run)
};

// H of the two real pencils packed in buf (x in .x, y in .y, entries [0, N)),
// left in place packed the same way.  All threads of the workgroup call it.
template <int L>
__device__ __forceinline__ void dht_pair(const LdsSeq<double, L> buf, int t, const TwHalf<double, L>& tw,
                                         const DhtArgs& a) {
  constexpr int T = FftPlan<L>::T;
  constexpr int KS = (L + T - 1) / T;  // slots per thread over [0, L)
  const int N = a.N;
  // z_n conj(w_n), zero past N
#pragma unroll
  for (int i = 0; i < KS; ++i) {
    const int n = t + i * T;
    if (n < L) {
      cpx<double> z{0.0, 0.0};
      if (n < N) {
        const cpx<double> v = buf[n], w = a.chirp[n];
        z = cpx<double>{v.x * w.x + v.y * w.y, v.y * w.x - v.x * w.y};
      }
      buf[n] = z;
    }
  }
  __syncthreads();
  fft_lds<double, L, -1>(buf, t, tw);
#pragma unroll
  for (int i = 0; i < KS; ++i) {
    const int k = t + i * T;
    if (k < L) buf[k] = cmul(buf[k], a.khat[k]);
  }
  __syncthreads();
  fft_lds<double, L, 1>(buf, t, tw);
  // Z_k = conj(w_k) (conv)_k, k < N
#pragma unroll
  for (int i = 0; i < KS; ++i) {
    const int k = t + i * T;
    if (k < N) {
      const cpx<double> v = buf[k], w = a.chirp[k];
      buf[k] = cpx<double>{v.x * w.x + v.y * w.y, v.y * w.x - v.x * w.y};
    }
  }
  __syncthreads();
  // Hartley parts: with Z_k = p + iq and Z_{N-k} = r + is,
  // H x_k = (p + r - q + s)/2, H y_k = (p - r + q + s)/2
  cpx<double> h[KS];
#pragma unroll
  for (int i = 0; i < KS; ++i) {
    const int k = t + i * T;
    if (k < N) {
      const cpx<double> zk = buf[k], zr = buf[k == 0 ? 0 : N - k];
      h[i] = cpx<double>{0.5 * ((zk.x + zr.x) - (zk.y - zr.y)), 0.5 * ((zk.x - zr.x) + (zk.y + zr.y))};
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < KS; ++i) {
    const int k = t + i * T;
    if (k < N) buf[k] = h[i];
  }
  __syncthreads();
}

template <int L>
__device__ __forceinline__ void dht_body(const DhtArgs& a) {
  constexpr int T = FftPlan<L>::T;
  constexpr int KS = (L + T - 1) / T;
  __shared__ cpx<double> lds[LdsSeq<double, L>::size];
  __shared__ cpx<double> twl[TwHalf<double, L>::size];
  const int t = threadIdx.x;
  const LdsSeq<double, L> buf{lds};
  double twr[TwFill<double, L, T>::C], twi[TwFill<double, L, T>::C];
  tw_load<double, L, T>(twr, twi, a.tw, t);

  int64_t pair = blockIdx.x;
  if (a.xcd_remap) {
    const int64_t b = blockIdx.x, tpx = (a.npairs + 7) >> 3;
    pair = (b & 7) * tpx + (b >> 3);
  }
  if (pair >= a.npairs) return;                      // the same in every thread
  if (a.stop_fl && *a.stop_fl != GM_RUNNING) return;  // the same in every thread

  const int N = a.N;
  const int64_t inner = a.inner;
  const int64_t p0 = 2 * pair, p1 = 2 * pair + 1;
  const bool v1 = p1 < a.npencil;
  auto base = [&](int64_t p) -> int64_t {
    const int64_t o = p / inner, r = p - o * inner;
    return o * (int64_t)N * inner + r;
  };
  const int64_t b0 = base(p0), b1 = v1 ? base(p1) : b0;
  tw_store<double, L, T>(twr, twi, twl, t);
#pragma unroll
  for (int i = 0; i < KS; ++i) {
    const int n = t + i * T;
    if (n < N) {
      const double x = a.in[b0 + n * inner];
      const double y = v1 ? a.in[b1 + n * inner] : 0.0;
      buf[n] = cpx<double>{x, y};
    }
  }
  __syncthreads();
  const TwHalf<double, L> tw{twl};
  dht_pair<L>(buf, t, tw, a);
  if (a.op == DHT_SCALE) {
    // 1/(prod N_l m_J): axis 0 runs along the pencil, the other axes are already
    // transformed; m_J = (prod_l b_l) (ebar + sum_l eta_l sigma_l / b_l)
    double lam_o[2] = {1.0, 1.0}, sig_o[2] = {0.0, 0.0};
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      int64_t rr = c == 0 ? p0 : (v1 ? p1 : p0);
      for (int l = 1; l < a.d; ++l) {
        const int64_t j = rr % a.Nax[l];
        rr /= a.Nax[l];
        lam_o[c] *= a.lam[l][j];
        sig_o[c] += a.wq[l][j];
      }
    }
    const double eb = *a.ebar, ps = a.pscale;
#pragma unroll
    for (int i = 0; i < KS; ++i) {
      const int k = t + i * T;
      if (k < N) {
        const double l0 = a.lam[0][k], w0 = a.wq[0][k];
        const cpx<double> v = buf[k];
        buf[k] = cpx<double>{v.x * (ps / (lam_o[0] * l0 * (eb + w0 + sig_o[0]))),
                             v.y * (ps / (lam_o[1] * l0 * (eb + w0 + sig_o[1])))};
      }
    }
    __syncthreads();
    dht_pair<L>(buf, t, tw, a);
  }
#pragma unroll
  for (int i = 0; i < KS; ++i) {
    const int n = t + i * T;
    if (n < N) {
      const cpx<double> v = buf[n];
      a.out[b0 + n * inner] = v.x;
      if (v1) a.out[b1 + n * inner] = v.y;
    }
  }
}

template <int L>
__global__ void __launch_bounds__(FftPlan<L>::T) k_dht(const DhtArgs a) {
  dht_body<L>(a);
}

// Setup of one axis: the chirp w_n and the transform of its length-L cyclic
// kernel (w_m at m and L - m for |m| < N, zero between), divided by L.
template <int L>
__global__ void __launch_bounds__(FftPlan<L>::T)
k_dht_tables(int N, const cpx<double>* __restrict__ tw, cpx<double>* __restrict__ chirp,
             cpx<double>* __restrict__ khat) {
  constexpr int T = FftPlan<L>::T;
  __shared__ cpx<double> lds[LdsSeq<double, L>::size];
  __shared__ cpx<double> twl[TwHalf<double, L>::size];
  const LdsSeq<double, L> buf{lds};
  const int t = threadIdx.x;
  double twr[TwFill<double, L, T>::C], twi[TwFill<double, L, T>::C];
  tw_load<double, L, T>(twr, twi, tw, t);
  tw_store<double, L, T>(twr, twi, twl, t);
  const TwHalf<double, L> twp{twl};
  for (int k = t; k < L; k += T) {
    // the kernel index m = k or L - k; its chirp exp(i pi m^2 / N), angle reduced mod 2N
    const int m = k < N ? k : (k > L - N ? L - k : -1);
    cpx<double> w{0.0, 0.0};
    if (m >= 0) {
      const long long r = ((long long)m * m) % (2LL * N);
      double s, c;
      sincospi((double)r / (double)N, &s, &c);
      w = cpx<double>{c, s};
      if (k < N) chirp[k] = w;
    }
    buf[k] = w;
  }
  __syncthreads();
  fft_lds<double, L, -1>(buf, t, twp);
  for (int k = t; k < L; k += T) {
    const cpx<double> v = buf[k];
    khat[k] = cpx<double>{v.x / (double)L, v.y / (double)L};
  }
}

// Strang eigenvalues of one axis in Fourier order: b_j of B (closed form) into
// lam, eta sigma_j / b_j of S into wq; sigma_j = sum_k c_k cos(2 pi jk/N) over the
// Strang column c (central diagonals of S wrapped around).
__global__ void __launch_bounds__(256)
k_strang_eigs(int N, double alpha, double eta, const double* __restrict__ s, double* __restrict__ lam,
              double* __restrict__ wq);

template <int L>
hipError_t launch_dht_L(const DhtArgs& a, int64_t nblocks, hipStream_t st);
template <int L>
hipError_t launch_dht_tables_L(int N, const cpx<double>* tw, cpx<double>* chirp, cpx<double>* khat,
                               hipStream_t st);

#define RSFDE_INSTANTIATE_DHT(LL)                                                               \
  template <>                                                                                   \
  hipError_t launch_dht_L<LL>(const DhtArgs& a, int64_t nblocks, hipStream_t st) {              \
    hipLaunchKernelGGL((k_dht<LL>), dim3((unsigned)nblocks), dim3(FftPlan<LL>::T), 0, st, a);   \
    return hipGetLastError();                                                                   \
  }                                                                                             \
  template <>                                                                                   \
  hipError_t launch_dht_tables_L<LL>(int N, const cpx<double>* tw, cpx<double>* chirp,          \
                                     cpx<double>* khat, hipStream_t st) {                       \
    hipLaunchKernelGGL((k_dht_tables<LL>), dim3(1), dim3(FftPlan<LL>::T), 0, st, N, tw, chirp,  \
                       khat);                                                                   \
    return hipGetLastError();                                                                   \
  }
