// LDS-resident complex FFTs of length L = 2(N+1) for pencil batches (gfx950).
//
// One length-L transform is owned by T = L/E threads; each thread holds E
// complex values in registers per stage and runs E/R radix-R butterflies.
// Stages are Stockham auto-sort passes: stage s with radix R and Ns = product of
// the earlier radices reads x[j + r L/R], twiddles by W_{Ns R}^{r (j mod Ns)},
// applies a length-R DFT and writes y[(j/Ns) Ns R + (j mod Ns) + r Ns]; the
// result comes out in natural order, in place (reads finish before a barrier,
// writes follow it).
//
// The sizes carried are L = 2^p (8..4096) and 3*2^p (12..3072), i.e. the
// grid sizes N_i + 1 = 2^p or 3*2^p for which the same length serves the
// circulant embedding of the Toeplitz factors and the odd extension behind the
// type-I sine transform (Section 3, eq. diag).
#pragma once
#include <type_traits>

#include "common.h"

// Templates below are keyed by a plan code: the transform length L (its default
// radix plan) or L | RSFDE_PLAN_ALT (an alternative plan of the same length, for
// the lengths that carry one).  The tile autotuner times both.
#define RSFDE_PLAN_ALT (1 << 16)
constexpr int plan_len(int code) { return code & (RSFDE_PLAN_ALT - 1); }

template <int LC> struct FftPlan;
template <int L> struct HasAltPlan { static constexpr bool value = false; };

#define RSFDE_PLAN(L_, E_, ...)                                                  \
  template <> struct FftPlan<L_> {                                               \
    static constexpr int Lv = plan_len(L_), E = E_, T = plan_len(L_) / E_;        \
    static constexpr int R[] = {__VA_ARGS__};                                    \
    static constexpr int NS = sizeof(R) / sizeof(int);                           \
  };
#define RSFDE_ALT_PLAN(L_, E_, ...)                                              \
  RSFDE_PLAN(L_ | RSFDE_PLAN_ALT, E_, __VA_ARGS__)                               \
  template <> struct HasAltPlan<L_> { static constexpr bool value = true; };

RSFDE_PLAN(8, 8, 8)
RSFDE_PLAN(12, 12, 4, 3)
RSFDE_PLAN(16, 16, 16)
RSFDE_PLAN(24, 12, 4, 3, 2)
RSFDE_PLAN(32, 16, 16, 2)
RSFDE_PLAN(48, 12, 4, 4, 3)
RSFDE_PLAN(64, 16, 16, 4)
RSFDE_PLAN(96, 12, 4, 4, 3, 2)
RSFDE_PLAN(128, 16, 16, 8)
RSFDE_PLAN(192, 12, 4, 4, 4, 3)
RSFDE_PLAN(256, 16, 16, 16)
RSFDE_PLAN(384, 12, 4, 4, 4, 3, 2)
RSFDE_PLAN(512, 8, 8, 8, 8)
RSFDE_PLAN(768, 12, 4, 4, 4, 4, 3)
RSFDE_PLAN(1024, 8, 8, 8, 8, 2)
RSFDE_PLAN(1536, 24, 8, 8, 8, 3)
RSFDE_PLAN(2048, 8, 8, 8, 8, 4)
RSFDE_PLAN(3072, 24, 8, 8, 8, 3, 2)
RSFDE_PLAN(4096, 16, 16, 16, 16)
// alternatives: the other side of the trade between threads per transform (more
// wavefronts in flight) and radix (fewer LDS round trips)
RSFDE_ALT_PLAN(256, 8, 8, 8, 4)
RSFDE_ALT_PLAN(384, 24, 8, 8, 3, 2)
RSFDE_ALT_PLAN(512, 16, 16, 16, 2)
RSFDE_ALT_PLAN(768, 24, 8, 8, 4, 3)
RSFDE_ALT_PLAN(1024, 16, 16, 16, 4)
RSFDE_ALT_PLAN(1536, 12, 4, 4, 4, 4, 3, 2)
RSFDE_ALT_PLAN(2048, 16, 16, 16, 8)
RSFDE_ALT_PLAN(3072, 12, 4, 4, 4, 4, 4, 3)
RSFDE_ALT_PLAN(4096, 8, 8, 8, 8, 8)
#undef RSFDE_ALT_PLAN
#undef RSFDE_PLAN

constexpr int cgcd(int a, int b) { return b == 0 ? a : cgcd(b, a % b); }

// Layout of one transform's sequence in LDS.  Measured on gfx950 (rocprofv3 LDS
// bank-conflict counters on probe kernels): a wave-wide 16-byte store is served
// eight lanes at a time over 32 four-byte banks, so eight consecutive lanes
// writing the same 16-byte column conflict; a 16-byte load at unit stride is
// conflict-free, and costs about twice as much once the 16- or 8-lane groups of
// a 32-lane half are offset against each other (as a pad slot every 256 bytes
// does).
//
// FP64 sequences are therefore stored plainly (element i in slot i): every
// unit-stride access of the passes (loads, stencils, stage reads, stores) is
// conflict-free and its offsets are compile-time constants.  The one strided
// access is the first Stockham stage's write (element R t + r from thread t, a
// stride of R slots); between the first and the second stage only, the sequence
// is XOR-swizzled inside 128-byte rows, slot(i) = i ^ ((i >> K) & 7) with
// 2^K = min(R, 8) (StageSwz), which spreads eight consecutive lanes over eight
// columns (four for R = 16) and keeps the second stage's unit-stride reads
// whole-row, at offsets that fold into constants (K = 4 for R = 16 would not fold
// at 1024 points, and the per-read slot arithmetic cost a wave per SIMD).  FP32
// sequences (8-byte elements) keep one pad slot after every 256 bytes.
template <typename R, int L>
struct LdsSeq {
  static constexpr int BS = 256 / (int)sizeof(cpx<R>);  // elements per 256-byte row
  static constexpr bool PAD = sizeof(R) != 8;            // padded (FP32) or plain layout
  static constexpr int size = PAD ? plan_len(L) + plan_len(L) / BS : plan_len(L);  // slots
  // pos(i + d) = pos(i) + shift(d) for every i when d is a multiple of FOLD
  static constexpr int FOLD = PAD ? BS : 1;
  cpx<R>* p;
  __device__ __forceinline__ static constexpr int pos(int i) { return PAD ? i + i / BS : i; }
  __device__ __forceinline__ static constexpr int shift(int d) { return PAD ? d + d / BS : d; }
  __device__ __forceinline__ cpx<R>& operator[](int i) const { return p[pos(i)]; }
  // R-typed view of component c of element i
  __device__ __forceinline__ R& comp(int i, int c) const { return ((R*)(p + pos(i)))[c]; }
};

// Swizzle of the sequence between the first and the second Stockham stage (plain
// FP64 layouts whose first radix is a power of two and that have a second
// stage).  i ^ ((i >> K) & 7) is a bijection: bit b < 3 is XORed with bit b + K,
// which is recovered first from the top.
template <typename R, int L>
struct StageSwz {
  using P = FftPlan<L>;
  static constexpr int R0 = P::R[0];
  static constexpr int K = R0 == 2 ? 1 : R0 == 4 ? 2 : (R0 == 8 || R0 == 16) ? 3 : 0;
  static constexpr bool on = !LdsSeq<R, L>::PAD && K > 0 && P::NS > 1;
  // slot(i + d) = slot(i) + d for every i when d is a multiple of FOLD
  static constexpr int FOLD = 8 << K;
  __device__ __forceinline__ static constexpr int slot(int i) { return on ? i ^ ((i >> K) & 7) : i; }
};

template <int L, int S> struct StageNs {
  static constexpr int value = StageNs<L, S - 1>::value * FftPlan<L>::R[S - 1];
};
template <int L> struct StageNs<L, 0> { static constexpr int value = 1; };

// Twiddles W_L^m, m < L, from a half-length table in LDS: W_L^{m + L/2} = -W_L^m,
// so entries m < L/2 suffice.  The table carries the same one-slot-per-256-byte
// padding as the sequences, which spreads the strided twiddle reads of the last
// stages over the banks.  Used for the plans whose per-thread twiddles would take
// too many registers (TwReg below) and by the setup and Strang kernels.
template <typename R, int L>
struct TwHalf {
  static constexpr int H = plan_len(L) / 2;
  static constexpr int BS = 256 / (int)sizeof(cpx<R>);
  static constexpr int size = H + H / BS;
  const cpx<R>* tab;
  __device__ __forceinline__ static constexpr int pos(int m) { return m + m / BS; }
  __device__ __forceinline__ cpx<R> get(int m) const {
    const bool hi = m >= H;
    const cpx<R> w = tab[pos(hi ? m - H : m)];
    return hi ? -w : w;
  }
  // Twiddles w[r] = W^{r m} (conjugated for DIR = +1), r = 1..RAD-1, of one
  // butterfly: the table values at r = 1, 2, 4 (and 8, 12 for RAD = 16) and
  // products of two of them for the rest.  Three LDS reads instead of seven for
  // radix 8, five instead of fifteen for radix 16; every power is at most two
  // roundings from exact.  (S, B: stage and butterfly of the thread, unused here.)
  template <int RAD, int DIR, int S, int B>
  __device__ __forceinline__ void powers(int m, cpx<R>* w) const {
    static_assert(RAD == 2 || RAD == 3 || RAD == 4 || RAD == 8 || RAD == 16, "unsupported radix");
    auto rd = [&](int mm) {
      cpx<R> x = get(mm);
      if (DIR > 0) x.y = -x.y;
      return x;
    };
    w[1] = rd(m);
    if constexpr (RAD >= 3) w[2] = rd(2 * m);
    if constexpr (RAD >= 4) w[3] = cmul(w[2], w[1]);
    if constexpr (RAD >= 8) {
      w[4] = rd(4 * m);
#pragma unroll
      for (int r = 5; r < 8; ++r) w[r] = cmul(w[4], w[r - 4]);
    }
    if constexpr (RAD == 16) {
      w[8] = rd(8 * m);
      w[12] = rd(12 * m);
#pragma unroll
      for (int r = 9; r < 12; ++r) w[r] = cmul(w[8], w[r - 8]);
#pragma unroll
      for (int r = 13; r < 16; ++r) w[r] = cmul(w[12], w[r - 12]);
    }
  }
};

// Compile-time loop: f(integral_constant<int, Q>) for Q = 0 .. C-1 (constant
// indices keep small per-thread arrays in registers).
template <int C, int Q = 0, typename Fn>
__device__ __forceinline__ void static_for(Fn&& fn) {
  if constexpr (Q < C) {
    fn(std::integral_constant<int, Q>{});
    static_for<C, Q + 1>(fn);
  }
}

// This thread's share of the half table: loads (issued together) into v ...
template <typename R, int L, int NT>
struct TwFill {
  static constexpr int H = TwHalf<R, L>::H;
  static constexpr int C = (H + NT - 1) / NT;
};
// (real and imaginary parts in separate scalar arrays: they stay in registers)
template <typename R, int L, int NT>
__device__ __forceinline__ void tw_load(R* vr, R* vi, const cpx<R>* __restrict__ tw, int tid) {
  constexpr int H = TwHalf<R, L>::H;
  static_for<TwFill<R, L, NT>::C>([&](auto q) {
    const int m = tid + q.value * NT;
    const cpx<R> w = tw[m < H ? m : 0];
    vr[q.value] = w.x;
    vi[q.value] = w.y;
  });
}
// ... then stores into the LDS table (a barrier must follow before use)
template <typename R, int L, int NT>
__device__ __forceinline__ void tw_store(const R* vr, const R* vi, cpx<R>* tab, int tid) {
  constexpr int H = TwHalf<R, L>::H;
  static_for<TwFill<R, L, NT>::C>([&](auto q) {
    const int m = tid + q.value * NT;
    if (H % NT == 0 || m < H) tab[TwHalf<R, L>::pos(m)] = cpx<R>{vr[q.value], vi[q.value]};
  });
}

// ---- small DFTs; DIR = -1 forward (e^{-2 pi i nk/R}), +1 backward ----------

// multiply by e^{DIR i pi/2}: forward -i, backward +i
template <typename R, int DIR>
__device__ __forceinline__ cpx<R> rot90(cpx<R> a) {
  return DIR < 0 ? cpx<R>{a.y, -a.x} : cpx<R>{-a.y, a.x};
}

template <typename R, int DIR>
__device__ __forceinline__ void dft2(cpx<R>* v) {
  cpx<R> a = v[0], b = v[1];
  v[0] = a + b;
  v[1] = a - b;
}

template <typename R, int DIR>
__device__ __forceinline__ void dft3(cpx<R>* v) {
  const R s3 = (R)0.86602540378443864676;  // sin(2 pi/3)
  cpx<R> t1 = v[1] + v[2], t2 = v[1] - v[2];
  cpx<R> m = v[0] - t1 * (R)0.5;
  // forward: X1 = m - i s3 t2, X2 = m + i s3 t2 ; backward: signs swapped
  cpx<R> s = rot90<R, DIR>(t2) * s3;
  v[0] = v[0] + t1;
  v[1] = m + s;
  v[2] = m - s;
}

template <typename R, int DIR>
__device__ __forceinline__ void dft4(cpx<R>* v) {
  cpx<R> a0 = v[0] + v[2], a1 = v[0] - v[2];
  cpx<R> a2 = v[1] + v[3], a3 = rot90<R, DIR>(v[1] - v[3]);
  v[0] = a0 + a2;
  v[2] = a0 - a2;
  v[1] = a1 + a3;
  v[3] = a1 - a3;
}

template <typename R, int DIR>
__device__ __forceinline__ void dft8(cpx<R>* v) {
  const R h = (R)0.70710678118654752440;
  cpx<R> e[4] = {v[0], v[2], v[4], v[6]};
  cpx<R> o[4] = {v[1], v[3], v[5], v[7]};
  dft4<R, DIR>(e);
  dft4<R, DIR>(o);
  // W8^1 = (1 + DIR i) h, W8^2 = DIR i, W8^3 = (-1 + DIR i) h
  cpx<R> o1 = cpx<R>{(o[1].x - (R)DIR * o[1].y) * h, ((R)DIR * o[1].x + o[1].y) * h};
  cpx<R> o2 = rot90<R, DIR>(o[2]);
  cpx<R> o3 = cpx<R>{(-o[3].x - (R)DIR * o[3].y) * h, ((R)DIR * o[3].x - o[3].y) * h};
  v[0] = e[0] + o[0];
  v[4] = e[0] - o[0];
  v[1] = e[1] + o1;
  v[5] = e[1] - o1;
  v[2] = e[2] + o2;
  v[6] = e[2] - o2;
  v[3] = e[3] + o3;
  v[7] = e[3] - o3;
}

template <typename R, int DIR>
__device__ __forceinline__ void dft16(cpx<R>* v) {
  // 4 x 4 decomposition: inner length-4 DFTs over n2 (stride 4), twiddles
  // W16^{n1 k2}, outer length-4 DFTs over n1.
  const R c1 = (R)0.92387953251128675613, s1 = (R)0.38268343236508977173;
  const R h = (R)0.70710678118654752440;
  cpx<R> a[4][4];
#pragma unroll
  for (int n1 = 0; n1 < 4; ++n1) {
    cpx<R> q[4] = {v[n1], v[n1 + 4], v[n1 + 8], v[n1 + 12]};
    dft4<R, DIR>(q);
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) a[n1][k2] = q[k2];
  }
  // twiddles W16^{n1 k2} = cos(2 pi n1 k2/16) + DIR i sin(2 pi n1 k2/16)
  const R cs[10] = {(R)1, c1, h, s1, (R)0, -s1, -h, -c1, (R)-1, -c1};
  const R sn[10] = {(R)0, s1, h, c1, (R)1, c1, h, s1, (R)0, -s1};
#pragma unroll
  for (int n1 = 1; n1 < 4; ++n1) {
#pragma unroll
    for (int k2 = 1; k2 < 4; ++k2) {
      const int m = n1 * k2;  // 1..9
      cpx<R> w{cs[m], (R)DIR * sn[m]};
      a[n1][k2] = cmul(a[n1][k2], w);
    }
  }
#pragma unroll
  for (int k2 = 0; k2 < 4; ++k2) {
    cpx<R> q[4] = {a[0][k2], a[1][k2], a[2][k2], a[3][k2]};
    dft4<R, DIR>(q);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) v[k2 + 4 * k1] = q[k1];
  }
}

template <typename R, int RAD, int DIR>
__device__ __forceinline__ void dft(cpx<R>* v) {
  if constexpr (RAD == 2) dft2<R, DIR>(v);
  else if constexpr (RAD == 3) dft3<R, DIR>(v);
  else if constexpr (RAD == 4) dft4<R, DIR>(v);
  else if constexpr (RAD == 8) dft8<R, DIR>(v);
  else if constexpr (RAD == 16) dft16<R, DIR>(v);
  else static_assert(RAD == 2, "unsupported radix");
}

// Barrier inside one transform.  When the T threads of a transform lie in one
// wavefront (T divides 64), that wavefront's LDS accesses are performed in
// program order, so a wavefront-scope fence and a wave barrier (which only stops
// the compiler from moving memory accesses across it) take the place of the
// workgroup barrier: the wavefronts of a workgroup then run their transforms
// without waiting for each other.  `last` marks the barrier after the final
// stage, which stays a workgroup barrier: callers read other wavefronts'
// results there.
template <int L>
__device__ __forceinline__ void stage_sync(bool last) {
  if constexpr (64 % FftPlan<L>::T == 0) {
    if (!last) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      return;
    }
  }
  __syncthreads();
}

// One Stockham stage on the thread's part of one transform held in LDS, split
// into its LDS reads, its arithmetic and its LDS writes.  The thread holds E
// values in v: slot b R + r is element t + T (b + NB r) of the stage's input
// (before the arithmetic) and of its output (after it, for the last stage).
template <typename R, int L, int S>
struct StageGeom {
  using P = FftPlan<L>;
  static constexpr int RAD = P::R[S], Ns = StageNs<L, S>::value;
  static constexpr int T = P::T, E = P::E, NB = E / RAD, LR = P::Lv / RAD;
  static_assert(E % RAD == 0, "radix must divide the per-thread element count");
  // slot of element t + T m in the stage's register layout
  static constexpr int slot(int m) { return (m % NB) * RAD + m / NB; }
};

// Twiddles held in registers: per stage S >= 1 and per butterfly of the thread,
// the base twiddle W_L^m of that butterfly (m = (j mod Ns) L/(Ns R), j = t + b T),
// loaded once per kernel from the half table in global memory.  The powers come
// from it by squaring and products: w2 = w1^2, w4 = w2^2, w8 = w4^2 and
// w_{a+b} = w_a w_b for the rest, at most about a dozen roundings from exact for
// radix 16 (against 2^-52 per rounding, far below the transforms' own error
// growth).  When T is a multiple of Ns every butterfly of the thread shares one
// base.  No LDS table and no LDS reads: the table costs 8 KB (L = 1024, FP64) to
// 16 KB (L = 2048) per workgroup and its reads hit bank conflicts in the early
// stages, where the exponents step by large strides.
template <typename R, int L>
struct TwReg {
  using P = FftPlan<L>;
  template <int S>
  static constexpr int nb() {
    if constexpr (S == 0 || S >= P::NS) {
      return 0;
    } else {
      using G = StageGeom<R, L, S>;
      return G::T % G::Ns == 0 ? 1 : G::NB;
    }
  }
  template <int S>
  static constexpr int off() {
    if constexpr (S == 0) return 0;
    else return off<S - 1>() + nb<S - 1>();
  }
  static constexpr int count = off<P::NS>();
  cpx<R> base[count > 0 ? count : 1];

  // (the table holds W_L^m for m < L/2, and every base exponent is below L/R)
  __device__ __forceinline__ void load(const cpx<R>* __restrict__ tab, int t) {
    static_for<P::NS>([&](auto sq) {
      constexpr int S = decltype(sq)::value;
      if constexpr (nb<S>() > 0) {
        using G = StageGeom<R, L, S>;
        constexpr int step = plan_len(L) / (G::Ns * G::RAD);
        static_for<nb<S>()>([&](auto bq) {
          constexpr int b = decltype(bq)::value;
          base[off<S>() + b] = tab[((t + b * G::T) % G::Ns) * step];
        });
      }
    });
  }

  template <int RAD, int DIR, int S, int B>
  __device__ __forceinline__ void powers(int, cpx<R>* w) const {
    static_assert(RAD == 2 || RAD == 3 || RAD == 4 || RAD == 8 || RAD == 16, "unsupported radix");
    constexpr int bi = off<S>() + (nb<S>() == 1 ? 0 : B);
    cpx<R> w1 = base[bi];
    // (an empty asm that the compiler must assume changes w1: without it the
    // powers, pure functions of the bases, are hoisted to the kernel start and
    // shared by every transform, which keeps ~7 complex values per stage live)
    asm volatile("" : "+v"(w1.x), "+v"(w1.y));
    if (DIR > 0) w1.y = -w1.y;
    auto sq = [](cpx<R> a) { return cpx<R>{(a.x - a.y) * (a.x + a.y), (R)2 * a.x * a.y}; };
    w[1] = w1;
    if constexpr (RAD >= 3) w[2] = sq(w1);
    if constexpr (RAD >= 4) w[3] = cmul(w[2], w1);
    if constexpr (RAD >= 8) {
      w[4] = sq(w[2]);
#pragma unroll
      for (int r = 5; r < 8; ++r) w[r] = cmul(w[4], w[r - 4]);
    }
    if constexpr (RAD == 16) {
      w[8] = sq(w[4]);
#pragma unroll
      for (int r = 9; r < 16; ++r) w[r] = cmul(w[8], w[r - 8]);
    }
  }
};

// Register twiddles where they cost at most 6 complex values per thread (the
// 2^p plans of radix 8 and 16 up to 4096 points); the LDS table otherwise.
template <typename R, int L>
struct TwUseReg {
  static constexpr bool value = TwReg<R, L>::count <= 6;
};

// (slots r >= rmax are set to zero instead of read)
template <typename R, int L, int S>
__device__ __forceinline__ void stage_read(const LdsSeq<R, L> buf, int t, cpx<R>* v,
                                           const int rmax = StageGeom<R, L, S>::RAD) {
  using G = StageGeom<R, L, S>;
  using Q = LdsSeq<R, L>;
  using W = StageSwz<R, L>;
  constexpr int LR = G::LR;
  constexpr bool swz = S == 1 && W::on;  // reads the first stage's swizzled output
  // Reads x[j + r L/R]: when L/R is a multiple of the layout's fold distance,
  // the slot of j + r L/R is the slot of j plus a constant offset per r.
  constexpr bool rd_fold = swz ? LR % W::FOLD == 0 : LR % Q::FOLD == 0;
#pragma unroll
  for (int b = 0; b < G::NB; ++b) {
    const int j = t + b * G::T;
    const int pj = swz ? W::slot(j) : Q::pos(j);
#pragma unroll
    for (int r = 0; r < G::RAD; ++r) {
      cpx<R> x{0, 0};
      if (r < rmax) {
        if constexpr (rd_fold) x = buf.p[pj + (swz ? r * LR : Q::shift(r * LR))];
        else if constexpr (swz) x = buf.p[W::slot(j + r * LR)];
        else x = buf[j + r * LR];
      }
      v[b * G::RAD + r] = x;
    }
  }
}

template <typename R, int L, int DIR, int S, typename TW>
__device__ __forceinline__ void stage_math(int t, const TW& tw, cpx<R>* v) {
  using G = StageGeom<R, L, S>;
  constexpr int RAD = G::RAD, Ns = G::Ns;
  static_for<G::NB>([&](auto bq) {
    constexpr int b = decltype(bq)::value;
    const int j = t + b * G::T;
    if constexpr (Ns > 1) {
      const int k = j % Ns;
      constexpr int step = plan_len(L) / (Ns * RAD);
      cpx<R> w[RAD];
      tw.template powers<RAD, DIR, S, b>(k * step, w);
#pragma unroll
      for (int r = 1; r < RAD; ++r) v[b * RAD + r] = cmul(v[b * RAD + r], w[r]);
    }
    dft<R, RAD, DIR>(&v[b * RAD]);
  });
}

template <typename R, int L, int S>
__device__ __forceinline__ void stage_write(const LdsSeq<R, L> buf, int t, const cpx<R>* v) {
  using G = StageGeom<R, L, S>;
  using Q = LdsSeq<R, L>;
  using W = StageSwz<R, L>;
  constexpr int BS = Q::BS, RAD = G::RAD, Ns = G::Ns;
  if constexpr (S == 0 && W::on) {
    // first stage, swizzled: elements R j + r (the low bits of R j are zero, so
    // the slot arithmetic reduces to an XOR with a constant per r)
#pragma unroll
    for (int b = 0; b < G::NB; ++b) {
      const int base = (t + b * G::T) * RAD;
#pragma unroll
      for (int r = 0; r < RAD; ++r) buf.p[W::slot(base + r)] = v[b * RAD + r];
    }
    return;
  }
  // Writes y[base + r Ns], base = (j/Ns) Ns R + j mod Ns.  Plain layout: a
  // constant offset r Ns.  Padded layout: the row of base + r Ns is the row of
  // base plus (r Ns)/BS when Ns is a multiple of BS, or Ns divides BS and Ns R is
  // a multiple or a divisor of BS (no carry out of the row).
  constexpr bool wr_fold =
      !Q::PAD || (Ns % BS == 0 || (BS % Ns == 0 && ((Ns * RAD) % BS == 0 || BS % (Ns * RAD) == 0)));
#pragma unroll
  for (int b = 0; b < G::NB; ++b) {
    const int j = t + b * G::T;
    const int k = j % Ns;
    const int base = (j / Ns) * Ns * RAD + k;
    const int pb = Q::pos(base);
#pragma unroll
    for (int r = 0; r < RAD; ++r) {
      if constexpr (wr_fold) buf.p[pb + (Q::PAD ? r * Ns + (r * Ns) / BS : r * Ns)] = v[b * RAD + r];
      else buf[base + r * Ns] = v[b * RAD + r];
    }
  }
}

template <typename R, int L, int DIR, int S, typename TW>
__device__ __forceinline__ void fft_stage(const LdsSeq<R, L> buf, int t, const TW& tw) {
  cpx<R> v[FftPlan<L>::E];
  stage_read<R, L, S>(buf, t, v);
  stage_math<R, L, DIR, S>(t, tw, v);
  stage_sync<L>(false);
  stage_write<R, L, S>(buf, t, v);
  stage_sync<L>(S + 1 == FftPlan<L>::NS);
}

template <typename R, int L, int DIR, int S, typename TW>
__device__ __forceinline__ void fft_stages(const LdsSeq<R, L> buf, int t, const TW& tw) {
  if constexpr (S < FftPlan<L>::NS) {
    fft_stage<R, L, DIR, S>(buf, t, tw);
    fft_stages<R, L, DIR, S + 1>(buf, t, tw);
  }
}

// Full transform of the length-L sequence in `buf` (all threads of the
// workgroup must call it together: it contains barriers).  `tw` is a TwReg or
// TwHalf twiddle provider.
template <typename R, int L, int DIR, typename TW>
__device__ __forceinline__ void fft_lds(const LdsSeq<R, L> buf, int t, const TW& tw) {
  fft_stages<R, L, DIR, 0>(buf, t, tw);
}

// Stages 1 .. NS-2 of a transform whose first stage wrote to LDS.
template <typename R, int L, int DIR, int S, typename TW>
__device__ __forceinline__ void fft_mid_stages(const LdsSeq<R, L> buf, int t, const TW& tw) {
  if constexpr (S + 1 < FftPlan<L>::NS) {
    cpx<R> v[FftPlan<L>::E];
    stage_read<R, L, S>(buf, t, v);
    stage_math<R, L, DIR, S>(t, tw, v);
    stage_sync<L>(false);
    stage_write<R, L, S>(buf, t, v);
    stage_sync<L>(false);
    fft_mid_stages<R, L, DIR, S + 1>(buf, t, tw);
  }
}

// Transform with its input and output in registers: on entry c[m] is element
// t + T m of the sequence (m < E), on exit c[m] is element t + T m of its
// transform.  Those are the first stage's inputs and the last stage's outputs
// of thread t, so only the stages in between go through LDS.  FRESH: the LDS
// sequence has not been read since the last workgroup barrier, and an LDS
// twiddle table still needs one (taken after the first stage's writes);
// otherwise a previous register transform of the same threads has just read it.
template <typename R, int L, int DIR, bool FRESH, typename TW>
__device__ __forceinline__ void fft_regs(const LdsSeq<R, L> buf, int t, const TW& tw, cpx<R>* c) {
  using P = FftPlan<L>;
  constexpr int E = P::E, NS = P::NS;
  cpx<R> v[E];
#pragma unroll
  for (int m = 0; m < E; ++m) v[StageGeom<R, L, 0>::slot(m)] = c[m];
  stage_math<R, L, DIR, 0>(t, tw, v);
  if constexpr (NS > 1) {
    if constexpr (!FRESH) stage_sync<L>(false);
    stage_write<R, L, 0>(buf, t, v);
    if constexpr (FRESH) __syncthreads();
    else stage_sync<L>(false);
    fft_mid_stages<R, L, DIR, 1>(buf, t, tw);
    stage_read<R, L, NS - 1>(buf, t, v);
    stage_math<R, L, DIR, NS - 1>(t, tw, v);
  }
#pragma unroll
  for (int m = 0; m < E; ++m) c[m] = v[StageGeom<R, L, NS - 1>::slot(m)];
}

// Transform from LDS to registers: stages 0 .. NS-2 in LDS, the last stage's
// results left in c[m] (element t + T m, m < E).  The sequence must be visible
// to the transform's threads on entry (a barrier taken by the caller).
template <typename R, int L, int DIR, int S, typename TW>
__device__ __forceinline__ void fft_lds_stages_to(const LdsSeq<R, L> buf, int t, const TW& tw) {
  if constexpr (S + 1 < FftPlan<L>::NS) {
    cpx<R> v[FftPlan<L>::E];
    stage_read<R, L, S>(buf, t, v);
    stage_math<R, L, DIR, S>(t, tw, v);
    stage_sync<L>(false);
    stage_write<R, L, S>(buf, t, v);
    stage_sync<L>(false);
    fft_lds_stages_to<R, L, DIR, S + 1>(buf, t, tw);
  }
}
// ZU: entries L/2 .. L-1 of the sequence are zero and not read (the first
// stage takes zeros for r >= R/2, first radix even).
template <typename R, int L, int DIR, bool ZU = false, typename TW>
__device__ __forceinline__ void fft_lds_regs(const LdsSeq<R, L> buf, int t, const TW& tw, cpx<R>* c) {
  using P = FftPlan<L>;
  using G = StageGeom<R, L, 0>;
  constexpr int E = P::E, NS = P::NS;
  static_assert(!ZU || G::RAD % 2 == 0, "the first radix must be even");
  cpx<R> v[E];
  stage_read<R, L, 0>(buf, t, v, ZU ? G::RAD / 2 : G::RAD);
  stage_math<R, L, DIR, 0>(t, tw, v);
  if constexpr (NS > 1) {
    stage_sync<L>(false);
    stage_write<R, L, 0>(buf, t, v);
    stage_sync<L>(false);
    fft_lds_stages_to<R, L, DIR, 1>(buf, t, tw);
    stage_read<R, L, NS - 1>(buf, t, v);
    stage_math<R, L, DIR, NS - 1>(t, tw, v);
  }
#pragma unroll
  for (int m = 0; m < E; ++m) c[m] = v[StageGeom<R, L, NS - 1>::slot(m)];
}

// Transform from registers (c[m] = element t + T m) to LDS, natural order; the
// same threads have just read the sequence (fft_lds_regs).  Ends with a
// workgroup barrier, like fft_lds.
template <typename R, int L, int DIR, typename TW>
__device__ __forceinline__ void fft_regs_lds(const LdsSeq<R, L> buf, int t, const TW& tw, const cpx<R>* c) {
  using P = FftPlan<L>;
  constexpr int E = P::E, NS = P::NS;
  cpx<R> v[E];
#pragma unroll
  for (int m = 0; m < E; ++m) v[StageGeom<R, L, 0>::slot(m)] = c[m];
  stage_math<R, L, DIR, 0>(t, tw, v);
  stage_sync<L>(false);
  stage_write<R, L, 0>(buf, t, v);
  stage_sync<L>(NS == 1);
  fft_stages<R, L, DIR, 1>(buf, t, tw);
}

// Transform of an odd sequence z_{L-n} = -z_n of which only entries 0 .. L/2 are
// in LDS: the first stage reads x[j + r L/R] for r >= R/2 as -x[(R - r) L/R - j]
// (first radix even; j = 0, r = R/2 lands on z_{L/2} = 0).  The remaining
// stages run as in fft_lds; ends with a workgroup barrier.
template <typename R, int L, int DIR, typename TW>
__device__ __forceinline__ void fft_lds_odd(const LdsSeq<R, L> buf, int t, const TW& tw) {
  using G = StageGeom<R, L, 0>;
  constexpr int RAD = G::RAD, LR = G::LR;
  static_assert(RAD % 2 == 0, "the first radix must be even");
  cpx<R> v[FftPlan<L>::E];
#pragma unroll
  for (int b = 0; b < G::NB; ++b) {
    const int j = t + b * G::T;
#pragma unroll
    for (int r = 0; r < RAD; ++r) v[b * RAD + r] = r < RAD / 2 ? buf[j + r * LR] : -buf[(RAD - r) * LR - j];
  }
  stage_math<R, L, DIR, 0>(t, tw, v);
  stage_sync<L>(false);
  stage_write<R, L, 0>(buf, t, v);
  stage_sync<L>(FftPlan<L>::NS == 1);
  fft_stages<R, L, DIR, 1>(buf, t, tw);
}
