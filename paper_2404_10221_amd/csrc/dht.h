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
#include "pass.h"  // LdsPitch, set_comp

enum : int { DHT_PLAIN = 0, DHT_SCALE = 1 };

struct DhtArgs {
  int op;                     // DHT_PLAIN, or DHT_SCALE (axis 0: H, 1/m, H)
  int N, d, axis;
  int64_t inner;              // element stride of the pass axis
  int64_t npencil;            // pencils (= n / N)
  int64_t tiles_inner;        // strided axes: tiles across the inner index range (launcher)
  int64_t ntiles;             // tiles of 2F pencils (set by the launcher)
  int xcd_remap;              // strided axes: consecutive tiles on one XCD
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

// Pencil pairs per workgroup of the Hartley passes: up to 512 threads, within
// the LDS left after the twiddle table.
template <int L>
struct DhtShape {
  static constexpr int T = FftPlan<L>::T;
  static constexpr int bytes_per_seq =
      (LdsSeq<double, L>::size + LdsPitch<double, L, 1>::M) * (int)sizeof(cpx<double>);
  static constexpr int cap = 160 * 1024 - TwHalf<double, L>::size * (int)sizeof(cpx<double>) - 2048;
  static constexpr int want = 512 / T > 1 ? 512 / T : 1;
  static constexpr int lim = cap / bytes_per_seq;
  static constexpr int F = want < lim ? want : (lim > 0 ? lim : 1);
  static constexpr int NT = F * T;
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

// One tile of 2F pencils (F packed pairs, one LDS sequence each).  Strided axes:
// the tile is 2F adjacent pencils of one outer index, loaded and stored as row
// segments across the pencils (lanes over pencils); the contiguous axis: 2F
// consecutive rows, each pair's thread group reading along its rows.
template <int L, int F, bool STRIDED>
__device__ __forceinline__ void dht_body(const DhtArgs& a, const int64_t bid) {
  constexpr int T = FftPlan<L>::T, NT = F * T, PT = 2 * F;
  constexpr int KS = (L + T - 1) / T;
  constexpr int LP = LdsPitch<double, L, F>::value;
  constexpr int NE = (L / 2 * PT + NT - 1) / NT;  // strided slots per thread (N < L/2)
  __shared__ cpx<double> lds[F * LP];
  __shared__ cpx<double> twl[TwHalf<double, L>::size];
  const int tid = threadIdx.x;
  const int f = tid / T, t = tid - f * T;
  const LdsSeq<double, L> buf{lds + f * LP};
  double twr[TwFill<double, L, NT>::C], twi[TwFill<double, L, NT>::C];
  tw_load<double, L, NT>(twr, twi, a.tw, tid);

  int64_t tile = bid;
  if (a.xcd_remap) {
    const int64_t tpx = (a.ntiles + 7) >> 3;
    tile = (bid & 7) * tpx + (bid >> 3);
  }
  if (tile >= a.ntiles) return;                       // the same in every thread
  if (a.stop_fl && *a.stop_fl != GM_RUNNING) return;  // the same in every thread

  const int N = a.N;
  const int64_t inner = a.inner;
  int64_t gbase = 0, row0 = 0;
  int nvalid;
  if constexpr (STRIDED) {
    const int64_t o = tile / a.tiles_inner;
    const int64_t pin0 = (tile - o * a.tiles_inner) * PT;
    const int64_t rem = inner - pin0;
    nvalid = rem < PT ? (int)rem : PT;
    gbase = o * (int64_t)N * inner + pin0;
  } else {
    row0 = tile * PT;
    const int64_t rem = a.npencil - row0;
    nvalid = rem < PT ? (int)rem : PT;
  }
  tw_store<double, L, NT>(twr, twi, twl, tid);
  if constexpr (STRIDED) {
#pragma unroll
    for (int i = 0; i < NE; ++i) {
      const int flat = tid + i * NT;
      const int p = flat / PT, pp = flat - p * PT;
      if (p < N) {
        const double x = pp < nvalid ? a.in[gbase + (int64_t)p * inner + pp] : 0.0;
        const LdsSeq<double, L> bb{lds + (pp >> 1) * LP};
        set_comp(bb[p], pp & 1, x);
      }
    }
  } else {
    const bool v0 = 2 * f < nvalid, v1 = 2 * f + 1 < nvalid;
    const int64_t b0 = (row0 + 2 * f) * N, b1 = (row0 + 2 * f + 1) * N;
#pragma unroll
    for (int i = 0; i < KS; ++i) {
      const int n = t + i * T;
      if (n < N) buf[n] = cpx<double>{v0 ? a.in[b0 + n] : 0.0, v1 ? a.in[b1 + n] : 0.0};
    }
  }
  __syncthreads();
  const TwHalf<double, L> tw{twl};
  dht_pair<L>(buf, t, tw, a);
  if constexpr (!STRIDED) {
    if (a.op == DHT_SCALE) {
      // 1/(prod N_l m_J): axis 0 runs along the pencil, the other axes are already
      // transformed; m_J = (prod_l b_l) (ebar + sum_l eta_l sigma_l / b_l)
      double lam_o[2] = {1.0, 1.0}, sig_o[2] = {0.0, 0.0};
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        int64_t rr = row0 + 2 * f + c;
        if (rr >= a.npencil) rr = row0 + 2 * f;
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
    const bool v0 = 2 * f < nvalid, v1 = 2 * f + 1 < nvalid;
    const int64_t b0 = (row0 + 2 * f) * N, b1 = (row0 + 2 * f + 1) * N;
#pragma unroll
    for (int i = 0; i < KS; ++i) {
      const int n = t + i * T;
      if (n < N) {
        const cpx<double> v = buf[n];
        if (v0) a.out[b0 + n] = v.x;
        if (v1) a.out[b1 + n] = v.y;
      }
    }
  } else {
#pragma unroll
    for (int i = 0; i < NE; ++i) {
      const int flat = tid + i * NT;
      const int p = flat / PT, pp = flat - p * PT;
      if (p < N && pp < nvalid) {
        const LdsSeq<double, L> bb{lds + (pp >> 1) * LP};
        a.out[gbase + (int64_t)p * inner + pp] = bb.comp(p, pp & 1);
      }
    }
  }
}

template <int L, int F, bool STRIDED>
__global__ void __launch_bounds__(F * FftPlan<L>::T) k_dht(const DhtArgs a) {
  dht_body<L, F, STRIDED>(a, blockIdx.x);
}

// Batched Hartley passes: one launch covers the same pass of many instances that
// share the transform length and axis kind (tile counts per instance in the
// descriptors, set by dht_tiles).  The output column and the status word move
// with the Arnoldi index j of the launch (BP_OUT_J, BP_STOP as for the pencil
// passes).
struct DBPass {
  DhtArgs a;     // arguments as for Arnoldi step 0
  int64_t ldv;   // basis leading dimension (element offset per step)
  int patch;     // BP_OUT_J, BP_STOP
  int pad;
};
struct DBLaunch {
  const DBPass* desc;  // per-instance descriptors, slot order
  const int* start;    // start[s] = first block of slot s; start[ninst] = grid size
  int ninst;
  int j;
};

template <int L, int F, bool STRIDED>
__global__ void __launch_bounds__(F * FftPlan<L>::T) k_dht_batched(const DBLaunch bl) {
  const int slot = batch_slot(bl.start, bl.ninst, blockIdx.x);
  const DBPass& d = bl.desc[slot];
  DhtArgs a = d.a;
  if (d.patch & BP_OUT_J) a.out = a.out + (int64_t)bl.j * d.ldv;
  if (d.patch & BP_STOP) a.stop_fl = a.stop_fl + bl.j;
  dht_body<L, F, STRIDED>(a, (int64_t)blockIdx.x - bl.start[slot]);
}

// Tile counts of a Hartley pass of length L (in place in a); returns the blocks
// of its launch (XCD rounds on strided axes).
template <int L>
inline int64_t dht_tiles_L(DhtArgs& a) {
  using S = DhtShape<L>;
  const bool strided = a.axis > 0;
  if (strided) {
    a.tiles_inner = (a.inner + 2 * S::F - 1) / (2 * S::F);
    a.ntiles = (a.npencil / a.inner) * a.tiles_inner;
  } else {
    a.tiles_inner = 1;
    a.ntiles = (a.npencil + 2 * S::F - 1) / (2 * S::F);
  }
  a.xcd_remap = strided ? 1 : 0;
  return strided ? (a.ntiles + 7) / 8 * 8 : a.ntiles;
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
hipError_t launch_dht_L(const DhtArgs& a, hipStream_t st);
template <int L>
hipError_t launch_dht_batched_L(const DBLaunch& bl, int64_t nblocks, bool strided, hipStream_t st);
template <int L>
hipError_t launch_dht_tables_L(int N, const cpx<double>* tw, cpx<double>* chirp, cpx<double>* khat,
                               hipStream_t st);

#define RSFDE_INSTANTIATE_DHT(LL)                                                               \
  template <>                                                                                   \
  hipError_t launch_dht_L<LL>(const DhtArgs& a0, hipStream_t st) {                              \
    using S = DhtShape<LL>;                                                                     \
    DhtArgs a = a0;                                                                             \
    const int64_t nb = dht_tiles_L<LL>(a);                                                      \
    if (nb <= 0) return hipSuccess;                                                             \
    if (nb > 0x7fffffffLL) return hipErrorInvalidValue;                                         \
    if (a.axis > 0)                                                                             \
      hipLaunchKernelGGL((k_dht<LL, S::F, true>), dim3((unsigned)nb), dim3(S::NT), 0, st, a);   \
    else                                                                                        \
      hipLaunchKernelGGL((k_dht<LL, S::F, false>), dim3((unsigned)nb), dim3(S::NT), 0, st, a);  \
    return hipGetLastError();                                                                   \
  }                                                                                             \
  template <>                                                                                   \
  hipError_t launch_dht_batched_L<LL>(const DBLaunch& bl, int64_t nblocks, bool strided,        \
                                      hipStream_t st) {                                         \
    using S = DhtShape<LL>;                                                                     \
    if (strided)                                                                                \
      hipLaunchKernelGGL((k_dht_batched<LL, S::F, true>), dim3((unsigned)nblocks), dim3(S::NT), \
                         0, st, bl);                                                            \
    else                                                                                        \
      hipLaunchKernelGGL((k_dht_batched<LL, S::F, false>), dim3((unsigned)nblocks),             \
                         dim3(S::NT), 0, st, bl);                                               \
    return hipGetLastError();                                                                   \
  }                                                                                             \
  template <>                                                                                   \
  hipError_t launch_dht_tables_L<LL>(int N, const cpx<double>* tw, cpx<double>* chirp,          \
                                     cpx<double>* khat, hipStream_t st) {                       \
    hipLaunchKernelGGL((k_dht_tables<LL>), dim3(1), dim3(FftPlan<LL>::T), 0, st, N, tw, chirp,  \
                       khat);                                                                   \
    return hipGetLastError();                                                                   \
  }
