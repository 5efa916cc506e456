// Pencil pass kernels: one sweep over the grid along one axis that applies,
// per pencil and inside LDS, a fused combination of
//   * the B_{alpha_i} tridiagonal stencil (eq. Ha),
//   * the Toeplitz factor S_{alpha_i} (eq. eq0) by circulant embedding of length
//     L = 2(N_i+1): zero-pad, FFT, multiply by the real circulant spectrum,
//     inverse FFT, keep the first N_i entries,
//   * the type-I sine transform (Section 3, eq. diag) through the FFT of the odd
//     extension [0, x_1..x_N, 0, -x_N..-x_1] of length L,
//   * a diagonal scaling in the sine basis: 1/mu_K of the tau preconditioner,
//     or the factors of the two-sided form (eq. Pls).
// Two real pencils are packed as the real and imaginary parts of one complex
// transform.  Operators along different axes commute, so the d-dimensional
// matvec A v = B_alpha E v + S_alpha v and the preconditioner solve are chains of
// such passes (one sweep per axis and per transform direction).
#pragma once
#include <hip/hip_ext.h>

#include <type_traits>

#include "common.h"
#include "fft.h"
#include "krylov.h"

enum : int { OP_MV_FIRST = 0, OP_MV_MID = 1, OP_MV_LAST = 2, OP_DST = 3, OP_DSD = 4 };
// Diagonal of the scale phase in the sine basis, with Lambda_K the eigenvalues of
// B_alpha and mu_K = Lambda_K (ebar + sum_i eta_i q_i / lambda_i) those of B_alpha P_alpha:
//   PM_BP_INV     1/mu                  (B P)^{-1}            (eq. one-sided)
//   PM_PH_BINV    1/sqrt(Lambda mu)     P^{-1/2} B^{-1}       (eq. Pls, left factor)
//   PM_PH         sqrt(Lambda / mu)     P^{-1/2}              (eq. Pls, right factor)
enum : int { PM_BP_INV = 0, PM_PH_BINV = 1, PM_PH = 2 };
enum : int {
  FL_DST_AFTER = 1,      // MV_LAST: follow by a sine transform along the same axis
  FL_PREC_FULL = 2,      // MV_LAST (d = 1): follow by transform, 1/mu scaling, transform
  FL_IN64 = 4,           // in_c holds FP64 values (else the pass precision)
  FL_OUT64 = 8,          // out_a receives FP64 values (else the pass precision)
  FL_FIRST_IS_LAST = 16, // MV_LAST of a one-axis problem: stencil input is e .* v
  FL_NO_E = 32,          // first operator pass: the B (e .* v) term is dropped (S v alone)
  FL_ACCUM = 64          // OP_DST / OP_DSD: add the result to out_a instead of storing it
};

struct PassArgs {
  int op, flags;
  int N;                 // pencil length along the pass axis
  int d, axis;
  int64_t inner;         // element stride of the pass axis (prod of N_l, l < axis)
  int64_t npencil;       // pencils in the pass (= n / N)
  int64_t tiles_inner;   // strided passes: tiles across the inner index range
  int64_t ntiles;        // tiles (pencil groups) in the pass
  int64_t nlaunch;       // workgroups launched (>= ntiles)
  int xcd_remap;         // 1: block b takes tile (b mod 8) * ceil(ntiles/8) + b/8
  const void* in_c;      // Toeplitz / transform input (v for the first pass)
  const void* in_a;      // stencil input (e for the first pass)
  const double* in_x;    // MV_LAST: additive FP64 vector (b or F), may be NULL
  const double* sc_ptr;  // device scalar multiplying in_c, may be NULL
  void* out_a;           // a_i, w, or the transformed vector
  void* out_c;           // c_i = B_i c_{i-1} (MV_FIRST / MV_MID)
  double bd, bo;         // B stencil: 1 - alpha/12 and alpha/24
  double eta;            // signed eta_i of the Toeplitz term
  double gam;            // MV_LAST: multiplier of the operator part
  double xcoef;          // MV_LAST: multiplier of in_x
  const void* chat;      // circulant spectrum divided by L (precision R), length L
  const void* tw;        // exp(-2 pi i k/L), k < L (cpx<R>)
  int Nax[3];            // grid sizes per axis (for the mode indices of mu)
  const void* lam[3];    // B eigenvalues per axis (precision R), sine mode k+1 at [k]
  const void* wq[3];     // eta_i q_i / lambda_i per axis (precision R)
  const double* ebar;    // device scalar ebar
  double pscale;         // prod_i 1/L_i: normalisation of the two sine transforms
  int pmode;             // scaling of the scale phase (PM_*)
  int var;               // host only: workgroup-shape variant
  int use_gm;            // first operator pass of an Arnoldi step: resolve the previous step
  GmRes gm;              // (input scale = vsc[j] from that resolve; exit when the cycle ended)
  const int* stop_fl;    // other passes of the step: exit unless *stop_fl == running
};

template <typename R>
__device__ __forceinline__ R ld_any(const void* p, int64_t i, bool is64) {
  if constexpr (sizeof(R) == 8) {
    return ((const double*)p)[i];
  } else {
    return is64 ? (R)((const double*)p)[i] : ((const R*)p)[i];
  }
}

// NT: a non-temporal store (the nt cache policy).  The contiguous-axis passes of
// transform lengths up to 1024 store their pencils so (a compile-time choice: a
// branch between the two store forms is merged by the compiler, which drops the
// hint).  Measured per step with non-temporal stores in every contiguous pass:
// 3-D 255^3 (L = 512) 2 % faster (the passes' own stores get slower, the strided
// passes and the sweeps that follow them faster), 64 instances of 2-D (L = 256 ..
// 1024) 1.4 %, 3-D 511^3 and 1-D 511 (L = 1024) within noise; on 2-D 1023^2
// (L = 2048) the step rate did not move but the strided pass reading the
// non-temporal output slowed from 21 to 23 us, so L = 2048 and up keep plain
// stores.  Non-temporal stores in the strided passes were much slower (3-D 255^3
// sine-transform pass 78 -> 125 us), and in the Arnoldi sweeps made no difference.
template <typename R, bool NT = false>
__device__ __forceinline__ void st_any(void* p, int64_t i, R v, bool is64) {
  if constexpr (NT) {
    if constexpr (sizeof(R) == 8) {
      __builtin_nontemporal_store((double)v, ((double*)p) + i);
    } else {
      if (is64) __builtin_nontemporal_store((double)v, ((double*)p) + i);
      else __builtin_nontemporal_store(v, ((R*)p) + i);
    }
  } else if constexpr (sizeof(R) == 8) {
    ((double*)p)[i] = v;
  } else {
    if (is64) ((double*)p)[i] = (double)v;
    else ((R*)p)[i] = v;
  }
}

// out[i] += v, in out's precision (FL_ACCUM)
template <typename R>
__device__ __forceinline__ void st_acc(void* p, int64_t i, R v, bool is64) {
  if (is64) {
    double* q = (double*)p + i;
    *q = *q + (double)v;
  } else {
    R* q = (R*)p + i;
    *q = *q + v;
  }
}

template <typename R>
__device__ __forceinline__ R comp_of(cpx<R> z, int c) { return c ? z.y : z.x; }

template <typename R>
__device__ __forceinline__ void set_comp(cpx<R>& z, int c, R v) {
  if (c) z.y = v; else z.x = v;
}

// Pencils packed per workgroup: F complex transforms, i.e. 2F real pencils.
// Tile variant VAR halves F VAR times; the host picks a variant (tile width and
// radix plan) per axis by timing them at setup (the tile autotuner).

// Pitch (in elements) of the F sequences of a workgroup.  In a strided tile the
// lanes of a wavefront cover 2F pencils at consecutive positions, i.e. the same
// positions of F sequences, as 8-byte component accesses.  Consecutive sequences
// start W/F bytes apart modulo W, so that the F sequences x two components x the
// consecutive positions of a lane group fall on distinct banks: W = 128 bytes for
// the plain FP64 layout (the LDS serves a wave-wide access in 128-byte groups of
// 32 banks), W = 256 for the padded FP32 one.
template <typename R, int L, int F>
struct LdsPitch {
  static constexpr int S = LdsSeq<R, L>::size;
  static constexpr int EB = (int)sizeof(cpx<R>);
  static constexpr int W = LdsSeq<R, L>::PAD ? 256 : 128;
  static constexpr int M = 256 / EB;  // elements per 256 bytes
  static constexpr int want = F == 1 ? 0 : ((W / F) / EB > 1 ? (W / F) / EB : 1);
  static constexpr int value = S + ((want - S % M) % M + M) % M;
};

template <typename R, int L, bool STRIDED, int VAR>
struct PassShape {
  static constexpr int T = FftPlan<L>::T;
  // (sized for the largest pitch, S + M - 1)
  static constexpr int bytes_per_fft = (LdsSeq<R, L>::size + LdsPitch<R, L, 1>::M) * (int)sizeof(cpx<R>);
  // LDS left for the transforms: 160 KB minus the twiddle table (plans without
  // register twiddles), the circulant spectrum and 2 KB for the small shared arrays
  // (block sums, Givens column, y)
  static constexpr int cap = 160 * 1024 -
                             (TwUseReg<R, L>::value ? 0 : TwHalf<R, L>::size * (int)sizeof(cpx<R>)) -
                             plan_len(L) * (int)sizeof(R) - 2048;
  static constexpr int want = 512 / T > 1 ? 512 / T : 1;
  static constexpr int lim = cap / bytes_per_fft;
  static constexpr int F0a = want < lim ? want : lim;
  static constexpr int F0 = F0a * T > 1024 ? 1024 / T : F0a;
  static constexpr int F1 = F0 >> VAR;
  static constexpr int F = F1 < 1 ? 1 : F1;
  static constexpr int NT = F * T;
};

// Which ops a kernel carries: the operator passes or the sine-transform passes
// (two kernels, each with the registers of its own path).
enum : int { PK_MV = 1, PK_TR = 2 };

// Scale-phase factors of the two pencils of a packed pair, from g = mu / Lambda
// and Lambda (lam0, lam1) of each pencil: ps/(Lambda g) = ps/mu for PM_BP_INV
// (SQ false); for the two-sided forms (SQ true) ps/(Lambda sqrt g) =
// ps/sqrt(Lambda mu) for PM_PH_BINV and ps/sqrt g = ps sqrt(Lambda/mu) for PM_PH.
// One division for the pair: ps/(d0 d1) times d1 and d0.
template <typename R, bool SQ>
__device__ __forceinline__ void scale_pair(R g0, R g1, R lam0, R lam1, R ps, int pm, R& s0, R& s1) {
  if constexpr (SQ) {
    g0 = sqrt(g0);
    g1 = sqrt(g1);
  }
  const R d0 = SQ && pm == PM_PH ? g0 : lam0 * g0;
  const R d1 = SQ && pm == PM_PH ? g1 : lam1 * g1;
  const R r = ps / (d0 * d1);
  s0 = r * d1;
  s1 = r * d0;
}

// The pass on one tile; `bid` is the workgroup's index within the pass (the
// block index of a single-instance launch, the local index in a batched one).
template <typename R, int L, int F, bool STRIDED, int MODE>
__device__ __forceinline__ void pass_body(const PassArgs& a, const int64_t bid) {
  constexpr bool mv_op = MODE == PK_MV;  // (the launcher picks the kernel by op)
  using P = FftPlan<L>;
  constexpr int T = P::T, E = P::E, NT = F * T, PT = 2 * F;
  constexpr int LP = LdsPitch<R, L, F>::value;
  constexpr int NE = STRIDED ? E : E / 2;  // element slots per thread
  constexpr bool twreg = TwUseReg<R, L>::value;
  __shared__ cpx<R> lds[F * LP];
  __shared__ cpx<R> twl[twreg ? 1 : TwHalf<R, L>::size];
  // circulant spectrum / L (operator passes), or the axis-0 tables of OP_DSD;
  // not used by the strided sine-transform kernel
  __shared__ R chs[STRIDED && MODE == PK_TR ? 1 : plan_len(L)];

  const int tid = threadIdx.x;
  std::conditional_t<twreg, TwReg<R, L>, TwHalf<R, L>> tw;
  if constexpr (!twreg) tw.tab = twl;
  const int f = tid / T;
  const int t = tid - f * T;
  const LdsSeq<R, L> buf{lds + f * LP};
  const int N = a.N;
  const bool in64 = (a.flags & FL_IN64) != 0;
  const bool out64 = (a.flags & FL_OUT64) != 0;
  constexpr bool NT_ST = !STRIDED && plan_len(L) <= 1024;  // (see st_any)

  // ---- tile geometry.  Blocks are dispatched round-robin over the 8 XCDs
  // (each with its own L2); for strided passes every XCD takes a contiguous run
  // of tiles, so neighbouring tiles (which share cache lines) meet in one L2.
  int64_t tile = bid;
  if (a.xcd_remap) {
    const int64_t b = bid, tpx = (a.ntiles + 7) >> 3;
    tile = (b & 7) * tpx + (b >> 3);
  }
  if (tile >= a.ntiles) return;  // launches are rounded up to whole XCD rounds
  int64_t row0 = 0, gbase = 0;
  int nvalid;
  if constexpr (!STRIDED) {
    row0 = tile * PT;
    const int64_t rem = a.npencil - row0;
    nvalid = rem < PT ? (int)rem : PT;
  } else {
    const int64_t o = tile / a.tiles_inner;
    const int64_t pin0 = (tile - o * a.tiles_inner) * PT;
    const int64_t rem = a.inner - pin0;
    nvalid = rem < PT ? (int)rem : PT;
    gbase = o * (int64_t)N * a.inner + pin0;
  }
  const int64_t inner = a.inner;

  // element (slot i) -> position p, pencil-in-tile pp (strided) ; validity
  // Strided slots: lanes run over the tile's pencils (coalesced row segments).
  // The sine-transform kernel spreads a thread's slots along the pencil
  // (position tid/PT + i NT/PT); the operator kernel gives each thread a run of
  // NE consecutive positions of one pencil, so its B stencils need only the
  // run's two neighbours besides the run itself.
  // Runs need an even T (T/2 threads per pencil); they are used where they
  // measured faster, for transforms of one wavefront (T = 64: 3-D 255^3 axis-2
  // operator pass 18 % faster), and not at T = 128 (3-D 511^3, 9 % slower) or
  // T = 256 (2-D 1023^2, no change).
  constexpr bool runs = STRIDED && mv_op && T == 64;
  auto s_pos = [&](int i, int& p, int& pp) {
    if constexpr (runs) {
      pp = tid % PT;
      p = (tid / PT) * NE + i;
    } else {
      const int flat = tid + i * NT;
      p = flat / PT;
      pp = flat - p * PT;
    }
  };
  auto c_row = [&](int comp) -> int64_t { return row0 + 2 * f + comp; };

  // ---- the first wavefront fetches the state of the pending Givens resolve
  // before the tile's loads are issued, so the resolve can start while they fly
  GmIn gin;
  if (a.use_gm && tid < 64) gm_fetch(a.gm, gin);

  // ---- issue every global load of the tile first, at clamped addresses and
  // with no branch around them: one memory latency then covers the whole load
  // phase, and it overlaps the prologue below (slots past the pencil end or the
  // tile's last pencil are loaded from a valid address and discarded).
  // Contiguous sine-transform passes load elements t + T m of the odd extension
  // instead (see the register-staged transforms below): lc gets x_{p-1} and la
  // the mirrored x_{N-p}, p = t + T i < L/2.
  constexpr int NL = STRIDED ? NE : 2 * NE;  // values per input array per thread
  R lc[NL], la[NL];
  R nbc[2], nba[2];  // strided operator passes: the run's neighbours
  (void)nbc;
  (void)nba;
  {
    const bool ld_a = mv_op;
    if constexpr (!STRIDED) {
      const int64_t r0 = 2 * f < nvalid ? c_row(0) : 0;
      const int64_t r1 = 2 * f + 1 < nvalid ? c_row(1) : 0;
#pragma unroll
      for (int i = 0; i < NE; ++i) {
        const int p = t + i * T;
        if (ld_a) {
          const int pc = p < N ? p : 0;
          lc[2 * i] = ld_any<R>(a.in_c, r0 * N + pc, in64);
          lc[2 * i + 1] = ld_any<R>(a.in_c, r1 * N + pc, in64);
          la[2 * i] = ld_any<R>(a.in_a, r0 * N + pc, false);
          la[2 * i + 1] = ld_any<R>(a.in_a, r1 * N + pc, false);
        } else {
          const int pc = p >= 1 ? p - 1 : 0;  // p <= N here
          lc[2 * i] = ld_any<R>(a.in_c, r0 * N + pc, in64);
          lc[2 * i + 1] = ld_any<R>(a.in_c, r1 * N + pc, in64);
          la[2 * i] = ld_any<R>(a.in_c, r0 * N + (N - 1 - pc), in64);
          la[2 * i + 1] = ld_any<R>(a.in_c, r1 * N + (N - 1 - pc), in64);
        }
      }
    } else {
#pragma unroll
      for (int i = 0; i < NE; ++i) {
        int p, pp;
        s_pos(i, p, pp);
        const int64_t g = gbase + (int64_t)(p < N ? p : 0) * inner + (pp < nvalid ? pp : 0);
        lc[i] = ld_any<R>(a.in_c, g, in64);
        if (ld_a) la[i] = ld_any<R>(a.in_a, g, false);
      }
      if constexpr (runs) {
        // the run's neighbours p0 - 1 and p0 + NE (clamped; zero outside [0, N))
        const int pp = tid % PT, p0 = (tid / PT) * NE;
        const int64_t col = pp < nvalid ? pp : 0;
        const int64_t gm = gbase + (int64_t)(p0 >= 1 ? p0 - 1 : 0) * inner + col;
        const int64_t gq = gbase + (int64_t)(p0 + NE < N ? p0 + NE : 0) * inner + col;
        nbc[0] = ld_any<R>(a.in_c, gm, in64);
        nbc[1] = ld_any<R>(a.in_c, gq, in64);
        nba[0] = ld_any<R>(a.in_a, gm, false);
        nba[1] = ld_any<R>(a.in_a, gq, false);
      }
    }
  }
  // Tables for LDS (chs) join the batch: the circulant spectrum of the operator
  // passes, or the axis-0 eigenvalue tables lambda (first N entries) and
  // eta q / lambda (next N) of the transform-scale-transform pass, plus that
  // pass's per-pencil factors from the other (already transformed) axes.
  constexpr int Lv = plan_len(L);  // transform length (L is the plan code)
  constexpr int CH = (Lv + NT - 1) / NT;
  // (the 1/mu scaling runs along the contiguous axis only)
  const bool is_dsd = !STRIDED && !mv_op && a.op == OP_DSD;
  R lt[CH];
  R twr[twreg ? 1 : TwFill<R, L, NT>::C], twi[twreg ? 1 : TwFill<R, L, NT>::C];
  if constexpr (twreg) tw.load((const cpx<R>*)a.tw, t);
  else tw_load<R, L, NT>(twr, twi, (const cpx<R>*)a.tw, tid);
  R rl[2][2], rw[2][2];  // [pencil of the pair][axis 1, 2]: lambda and eta q / lambda
  R ebv = (R)0;
  if (mv_op) {
    const R* __restrict__ cg = (const R*)a.chat;
    static_for<CH>([&](auto q) {
      const int k = tid + q.value * NT;
      lt[q.value] = cg[k < Lv ? k : 0];
    });
  } else if (is_dsd) {
    const R* __restrict__ l0 = (const R*)a.lam[0];
    const R* __restrict__ w0 = (const R*)a.wq[0];
    static_for<CH>([&](auto q) {
      const int k = tid + q.value * NT;
      const R lv = l0[k < N ? k : 0];  // both loads in bounds
      const R wv = w0[k >= N && k < 2 * N ? k - N : 0];
      lt[q.value] = k < N ? lv : wv;
    });
    if constexpr (!STRIDED) {
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        int64_t rr = c_row(c);
        if (rr >= a.npencil) rr = 0;
#pragma unroll
        for (int l = 1; l < 3; ++l) {
          if (l < a.d) {
            const int64_t k = rr % a.Nax[l];
            rr /= a.Nax[l];
            rl[c][l - 1] = ((const R*)a.lam[l])[k];
            rw[c][l - 1] = ((const R*)a.wq[l])[k];
          } else {
            rl[c][l - 1] = (R)1;
            rw[c][l - 1] = (R)0;
          }
        }
      }
    }
    ebv = (R)(*a.ebar);
  }

  R sc = (R)1;
  if (a.use_gm) {
    __shared__ GmOut go;
    __shared__ GmCol gcol;
    gm_resolve(a.gm, gin, &go, &gcol, bid == 0);
    if (go.flag != GM_RUNNING) return;  // same value in every thread
    sc = (R)go.sc;
  } else {
    if (a.stop_fl && *a.stop_fl != GM_RUNNING) return;
    if (a.sc_ptr) sc = (R)(*a.sc_ptr);
  }
  const R bd = (R)a.bd, bo = (R)a.bo, eta = (R)a.eta;
  const R* __restrict__ chat = chs;
  if constexpr (!twreg) tw_store<R, L, NT>(twr, twi, twl, tid);
  if (mv_op || is_dsd) {
    static_for<CH>([&](auto q) {
      const int k = tid + q.value * NT;
      if (Lv % NT == 0 || k < Lv) chs[k] = lt[q.value];
    });
  }

  cpx<R> ra[STRIDED ? 1 : NE];  // contiguous: packed pair per slot
  R rs[STRIDED ? NE : 1];       // strided: one value per slot
  (void)ra;
  (void)rs;

  const int op = a.op;
  const bool is_mv = mv_op;
  bool scale_phase = is_dsd;  // a 1/mu scaling + second sine transform follow the first

  if constexpr (!STRIDED && !mv_op) {
    // ---- register-staged sine transforms along a contiguous axis.  Thread t
    // holds elements k = t + T m (m < E) of its packed pair; the odd extension
    // z_k = x_{k-1} (1 <= k <= N), z_{L-k} = -z_k, z_0 = z_{N+1} = 0 comes
    // straight from the loads, and fft_regs leaves Z_k at the same k.
    cpx<R> c[E];
    {
      const bool v0 = 2 * f < nvalid, v1 = 2 * f + 1 < nvalid;
#pragma unroll
      for (int i = 0; i < NE; ++i) {
        const bool live = t + i * T >= 1;
        const R x0 = live && v0 ? lc[2 * i] : (R)0, x1 = live && v1 ? lc[2 * i + 1] : (R)0;
        const R y0 = live && v0 ? la[2 * i] : (R)0, y1 = live && v1 ? la[2 * i + 1] : (R)0;
        c[i] = cpx<R>{x0, x1};             // k = p = t + T i
        c[NE + i] = cpx<R>{-y0, -y1};      // k = L/2 + p: -z_{N+1-p}
      }
    }
    fft_regs<R, L, -1, true>(buf, t, tw, c);
    if (scale_phase) {
      // 1/mu_K (or a two-sided factor) on the sine coefficients, as in the LDS
      // form below.  The coefficients of the odd extension satisfy
      // Z_{L-k} = -Z_k, so applying the factor of index L-k to Z_k at k > L/2
      // gives the odd extension of the scaled sequence in place.
      const R ps = (R)a.pscale;
      const int pm = a.pmode;
      R Lam[2], Sig[2];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        Lam[q] = ((R)1 * rl[q][0]) * rl[q][1];
        Sig[q] = ((R)0 + rw[q][0]) + rw[q][1];
      }
      // (one loop per form, chosen by a uniform branch: the square roots of the
      // two-sided factors are not computed, and then discarded, for the one-sided one)
      auto scale = [&](auto sqc) {
        constexpr bool SQ = decltype(sqc)::value;
#pragma unroll
        for (int m = 0; m < E; ++m) {
          const int p = t + (m % NE) * T;             // distance from 0 or from L/2
          const bool live = p >= 1;
          const int idx = live ? (m < NE ? p - 1 : N - p) : 0;  // sine index, < N
          const R l0 = chs[idx], w0 = chs[N + idx];
          R s0, s1;
          scale_pair<R, SQ>(ebv + w0 + Sig[0], ebv + w0 + Sig[1], Lam[0] * l0, Lam[1] * l0, ps,
                            pm, s0, s1);
          const cpx<R> Z = c[m];
          c[m] = live ? cpx<R>{-Z.y * s0, Z.x * s1} : cpx<R>{0, 0};
        }
      };
      if (pm == PM_BP_INV) scale(std::false_type{});
      else scale(std::true_type{});
      fft_regs<R, L, -1, false>(buf, t, tw, c);
    }
    // 2 DST(x0) = -Im Z_k, 2 DST(x1) = Re Z_k at k = t + T i (1 <= k <= N)
    const bool v0 = 2 * f < nvalid, v1 = 2 * f + 1 < nvalid;
    const int64_t b0 = c_row(0) * N - 1, b1 = c_row(1) * N - 1;
    if (a.flags & FL_ACCUM) {
#pragma unroll
      for (int i = 0; i < NE; ++i) {
        const int k = t + i * T;
        if (k >= 1) {
          if (v0) st_acc<R>(a.out_a, b0 + k, -c[i].y, out64);
          if (v1) st_acc<R>(a.out_a, b1 + k, c[i].x, out64);
        }
      }
      return;
    }
#pragma unroll
    for (int i = 0; i < NE; ++i) {
      const int k = t + i * T;
      if (k >= 1) {
        if (v0) st_any<R, NT_ST>(a.out_a, b0 + k, -c[i].y, out64);
        if (v1) st_any<R, NT_ST>(a.out_a, b1 + k, c[i].x, out64);
      }
    }
    return;
  }

  if (is_mv) {
    const bool ev_mode = op == OP_MV_FIRST || (a.flags & FL_FIRST_IS_LAST);
    const bool no_e = (a.flags & FL_NO_E) != 0;
    // ---- load (contiguous axis): Toeplitz input c into slots [0,N), stencil
    // input into [N+1, 2N+1); entry N stays zero (the Toeplitz input's padding)
    if (t == 0) {
      buf[N] = cpx<R>{0, 0};
      buf[2 * N + 1] = cpx<R>{0, 0};
    }
    if constexpr (!STRIDED) {
      const bool v0 = 2 * f < nvalid, v1 = 2 * f + 1 < nvalid;
#pragma unroll
      for (int i = 0; i < NE; ++i) {
        const int p = t + i * T;
        if (p < N) {
          R c0 = v0 ? lc[2 * i] * sc : (R)0;
          R c1 = v1 ? lc[2 * i + 1] * sc : (R)0;
          R a0 = v0 ? la[2 * i] : (R)0;
          R a1 = v1 ? la[2 * i + 1] : (R)0;
          if (ev_mode) {
            a0 = no_e ? (R)0 : a0 * c0;
            a1 = no_e ? (R)0 : a1 * c1;
          }
          buf[p] = cpx<R>{c0, c1};
          buf[N + 1 + p] = cpx<R>{a0, a1};
        }
      }
    } else if constexpr (!runs) {
      // (strided, one thread per transform) c and the stencil input into LDS
#pragma unroll
      for (int i = 0; i < NE; ++i) {
        int p, pp;
        s_pos(i, p, pp);
        if (p < N) {
          const bool v = pp < nvalid;
          R c = v ? lc[i] * sc : (R)0;
          R av = v ? la[i] : (R)0;
          if (ev_mode) av = no_e ? (R)0 : av * c;
          LdsSeq<R, L> bb{lds + (pp >> 1) * LP};
          set_comp(bb[p], pp & 1, c);
          set_comp(bb[N + 1 + p], pp & 1, av);
        }
      }
    } else {
      // ---- the thread's run p0 .. p0+NE-1 of pencil pp with its two neighbours
      // (zero outside [0, N)): c into LDS for the Toeplitz product; both stencils
      // in registers
      const int pp = tid % PT, p0 = (tid / PT) * NE;
      const bool v = pp < nvalid;
      const bool store_c = op != OP_MV_LAST;
      R cr[NE + 2], ar[NE + 2];
      cr[0] = v && p0 >= 1 ? nbc[0] * sc : (R)0;
      ar[0] = v && p0 >= 1 ? nba[0] : (R)0;
      cr[NE + 1] = v && p0 + NE < N ? nbc[1] * sc : (R)0;
      ar[NE + 1] = v && p0 + NE < N ? nba[1] : (R)0;
#pragma unroll
      for (int i = 0; i < NE; ++i) {
        const bool in = v && p0 + i < N;
        cr[i + 1] = in ? lc[i] * sc : (R)0;
        ar[i + 1] = in ? la[i] : (R)0;
      }
      if (ev_mode) {
#pragma unroll
        for (int k = 0; k < NE + 2; ++k) ar[k] = no_e ? (R)0 : ar[k] * cr[k];
      }
      const LdsSeq<R, L> bb{lds + (pp >> 1) * LP};
#pragma unroll
      for (int i = 0; i < NE; ++i) {
        const int p = p0 + i;
        if (p < N) {
          set_comp(bb[p], pp & 1, cr[i + 1]);
          const R bc = cr[i + 1] * bd + (cr[i] + cr[i + 2]) * bo;
          rs[i] = ar[i + 1] * bd + (ar[i] + ar[i + 2]) * bo;
          if (store_c && v) st_any<R>(a.out_c, gbase + (int64_t)p * inner + pp, bc, false);
        }
      }
    }
    __syncthreads();
    if constexpr (!STRIDED) {
      // ---- stencils: keep B a in registers, store c_out = B c
      const bool store_c = op != OP_MV_LAST;
      const bool v0 = 2 * f < nvalid, v1 = 2 * f + 1 < nvalid;
      const int64_t b0 = c_row(0) * N, b1 = c_row(1) * N;
#pragma unroll
      for (int i = 0; i < NE; ++i) {
        const int p = t + i * T;
        if (p < N) {
          cpx<R> cm = p > 0 ? buf[p - 1] : cpx<R>{0, 0};
          cpx<R> bc = buf[p] * bd + (cm + buf[p + 1]) * bo;
          cpx<R> ba = buf[N + 1 + p] * bd + (buf[N + p] + buf[N + 2 + p]) * bo;
          ra[i] = ba;
          if (store_c) {
            if (v0) st_any<R, NT_ST>(a.out_c, b0 + p, bc.x, false);
            if (v1) st_any<R, NT_ST>(a.out_c, b1 + p, bc.y, false);
          }
        }
      }
      __syncthreads();
    } else if constexpr (!runs) {
      const bool store_c = op != OP_MV_LAST;
#pragma unroll
      for (int i = 0; i < NE; ++i) {
        int p, pp;
        s_pos(i, p, pp);
        if (p < N) {
          const int c = pp & 1;
          const LdsSeq<R, L> bb{lds + (pp >> 1) * LP};
          R cm = p > 0 ? comp_of(bb[p - 1], c) : (R)0;
          R bc = comp_of(bb[p], c) * bd + (cm + comp_of(bb[p + 1], c)) * bo;
          R ba = comp_of(bb[N + 1 + p], c) * bd + (comp_of(bb[N + p], c) + comp_of(bb[N + 2 + p], c)) * bo;
          rs[i] = ba;
          if (store_c && pp < nvalid) st_any<R>(a.out_c, gbase + (int64_t)p * inner + pp, bc, false);
        }
      }
      __syncthreads();
    }
    // ---- Toeplitz product by circulant embedding.  The zero padding is not
    // stored: entry N is zero and the first stage takes entries L/2 .. L-1 as
    // zeros.  The spectrum multiplies the forward transform's last-stage results
    // in registers, which feed the inverse transform's first stage (elements
    // t + T m on both sides); on the contiguous axis the inverse transform's
    // results stay in registers for the combine below.
    cpx<R> z[E];
    fft_lds_regs<R, L, -1, true>(buf, t, tw, z);
#pragma unroll
    for (int m = 0; m < E; ++m) z[m] = z[m] * chat[t + T * m];
    if constexpr (STRIDED) fft_regs_lds<R, L, +1>(buf, t, tw, z);
    else fft_regs<R, L, +1, false>(buf, t, tw, z);
    // ---- combine
    const bool last = op == OP_MV_LAST;
    const bool want_dst = last && (a.flags & (FL_DST_AFTER | FL_PREC_FULL));
    const R gam = (R)a.gam, xcoef = (R)a.xcoef;
    const double* __restrict__ xin = a.in_x;
    // additive vector (right-hand side chains only): all loads issued together
    R lx[NL];
    if (last && xin) {
      if constexpr (!STRIDED) {
        const int64_t r0 = 2 * f < nvalid ? c_row(0) : 0;
        const int64_t r1 = 2 * f + 1 < nvalid ? c_row(1) : 0;
#pragma unroll
        for (int i = 0; i < NE; ++i) {
          const int p = t + i * T;
          const int pc = p < N ? p : 0;
          lx[2 * i] = (R)xin[r0 * N + pc];
          lx[2 * i + 1] = (R)xin[r1 * N + pc];
        }
      } else {
#pragma unroll
        for (int i = 0; i < NE; ++i) {
          int p, pp;
          s_pos(i, p, pp);
          lx[i] = (R)xin[gbase + (int64_t)(p < N ? p : 0) * inner + (pp < nvalid ? pp : 0)];
        }
      }
    }
    if constexpr (!STRIDED) {
      const bool v0 = 2 * f < nvalid, v1 = 2 * f + 1 < nvalid;
      const int64_t b0 = c_row(0) * N, b1 = c_row(1) * N;
#pragma unroll
      for (int i = 0; i < NE; ++i) {
        const int p = t + i * T;
        if (p < N) {
          cpx<R> w = ra[i] + z[i] * eta;  // z[i]: element p of T c
          if (last) {
            w = w * gam;
            if (xin) {
              R x0 = v0 ? lx[2 * i] : (R)0;
              R x1 = v1 ? lx[2 * i + 1] : (R)0;
              w = w + cpx<R>{x0, x1} * xcoef;
            }
          }
          if (want_dst) {
            ra[i] = w;
          } else {
            if (v0) st_any<R, NT_ST>(a.out_a, b0 + p, w.x, out64 && last);
            if (v1) st_any<R, NT_ST>(a.out_a, b1 + p, w.y, out64 && last);
          }
        }
      }
    } else {
#pragma unroll
      for (int i = 0; i < NE; ++i) {
        int p, pp;
        s_pos(i, p, pp);
        if (p < N) {
          const int c = pp & 1;
          const LdsSeq<R, L> bb{lds + (pp >> 1) * LP};
          const int64_t g = gbase + (int64_t)p * inner + pp;
          const bool v = pp < nvalid;
          R w = rs[i] + comp_of(bb[p], c) * eta;
          if (last) {
            w = w * gam;
            if (xin && v) w += lx[i] * xcoef;
          }
          if (want_dst) {
            rs[i] = w;
          } else if (v) {
            st_any<R>(a.out_a, g, w, out64 && last);
          }
        }
      }
    }
    if (!want_dst) return;  // uniform across the workgroup
    scale_phase = (a.flags & FL_PREC_FULL) != 0;
    __syncthreads();
    // ---- w for the sine transform: entries 0 .. N+1 of its odd extension (the
    // transform reads the other half mirrored)
    if (t == 0) {
      buf[0] = cpx<R>{0, 0};
      buf[N + 1] = cpx<R>{0, 0};
    }
    if constexpr (!STRIDED) {
#pragma unroll
      for (int i = 0; i < NE; ++i) {
        const int p = t + i * T;
        if (p < N) buf[p + 1] = ra[i];
      }
    } else {
#pragma unroll
      for (int i = 0; i < NE; ++i) {
        int p, pp;
        s_pos(i, p, pp);
        if (p < N) {
          LdsSeq<R, L> bb{lds + (pp >> 1) * LP};
          set_comp(bb[p + 1], pp & 1, rs[i]);
        }
      }
    }
    __syncthreads();
  } else {
    // ---- OP_DST / OP_DSD along a strided axis (the contiguous form returned
    // above): entries 0 .. N+1 of the odd extension of the input
    if (t == 0) {
      buf[0] = cpx<R>{0, 0};
      buf[N + 1] = cpx<R>{0, 0};
    }
    if constexpr (STRIDED) {
#pragma unroll
      for (int i = 0; i < NE; ++i) {
        int p, pp;
        s_pos(i, p, pp);
        if (p < N) {
          const bool v = pp < nvalid;
          R x = v ? lc[i] : (R)0;
          LdsSeq<R, L> bb{lds + (pp >> 1) * LP};
          set_comp(bb[p + 1], pp & 1, x);
        }
      }
    }
    __syncthreads();
  }

  // ---- sine transform(s): FFT of the odd extension; for z = x0 + i x1 the
  // transforms are 2 DST(x0) = -Im Z_k, 2 DST(x1) = Re Z_k (k = 1..N).
  fft_lds_odd<R, L, -1>(buf, t, tw);
  if (scale_phase) {
    // 1/mu_K in the sine basis (eq. Pa, Lemma le:eig, Lemma Heig, eq. q), or a
    // two-sided factor (PM_*); the pass runs along axis 0, the other axes are
    // already transformed.
    const R ps = (R)a.pscale;
    const int pm = a.pmode;
    if constexpr (!STRIDED) {
      // one-axis operator pass followed by the preconditioner (the contiguous
      // OP_DSD returned above): chs holds the circulant spectrum, the tables come
      // from global memory
      const R eb = (R)(*a.ebar);
      const R Lam[2] = {(R)1, (R)1}, Sig[2] = {(R)0, (R)0};
      R l0v[NE], w0v[NE];
      const R* __restrict__ lam0 = (const R*)a.lam[0];
      const R* __restrict__ wq0 = (const R*)a.wq[0];
#pragma unroll
      for (int i = 0; i < NE; ++i) {
        const int pc = t + i * T < N ? t + i * T : 0;
        l0v[i] = lam0[pc];
        w0v[i] = wq0[pc];
      }
      auto scale = [&](auto sqc) {
        constexpr bool SQ = decltype(sqc)::value;
#pragma unroll
        for (int i = 0; i < NE; ++i) {
          const int p = t + i * T;
          if (p < N) {
            const cpx<R> Z = buf[p + 1];
            const R l0 = l0v[i], w0 = w0v[i];
            R s0, s1;
            scale_pair<R, SQ>(eb + w0 + Sig[0], eb + w0 + Sig[1], Lam[0] * l0, Lam[1] * l0, ps, pm,
                              s0, s1);
            ra[i] = cpx<R>{-Z.y * s0, Z.x * s1};
          }
        }
      };
      if (pm == PM_BP_INV) scale(std::false_type{});
      else scale(std::true_type{});
      __syncthreads();
      if (t == 0) {
        buf[0] = cpx<R>{0, 0};
        buf[N + 1] = cpx<R>{0, 0};
      }
#pragma unroll
      for (int i = 0; i < NE; ++i) {
        const int p = t + i * T;
        if (p < N) buf[p + 1] = ra[i];
      }
      __syncthreads();
      fft_lds_odd<R, L, -1>(buf, t, tw);
    }
    // (the host only requests the scaling on the contiguous axis)
  }
  // ---- store the transformed pencils
  if constexpr (!STRIDED) {
    const bool v0 = 2 * f < nvalid, v1 = 2 * f + 1 < nvalid;
    const int64_t b0 = c_row(0) * N, b1 = c_row(1) * N;
#pragma unroll
    for (int i = 0; i < NE; ++i) {
      const int p = t + i * T;
      if (p < N) {
        const cpx<R> Z = buf[p + 1];
        if (v0) st_any<R, NT_ST>(a.out_a, b0 + p, -Z.y, out64);
        if (v1) st_any<R, NT_ST>(a.out_a, b1 + p, Z.x, out64);
      }
    }
  } else {
    const bool acc = (a.flags & FL_ACCUM) != 0;
#pragma unroll
    for (int i = 0; i < NE; ++i) {
      int p, pp;
      s_pos(i, p, pp);
      if (p < N && pp < nvalid) {
        const LdsSeq<R, L> bb{lds + (pp >> 1) * LP};
        // component pp&1 of the packed transform: -Im for the first pencil, Re for the second
        const R z = bb.comp(p + 1, (pp & 1) ^ 1);
        const int64_t g = gbase + (int64_t)p * inner + pp;
        if (acc) st_acc<R>(a.out_a, g, (pp & 1) ? z : -z, out64);
        else st_any<R>(a.out_a, g, (pp & 1) ? z : -z, out64);
      }
    }
  }
}

// Register budget of 128 VGPRs (4 waves per SIMD): measured faster on HBM-bound
// grids than the unconstrained allocation (3 waves per SIMD) despite a few spills.
// The operator passes (OP_MV_*) ...
template <typename R, int L, int F, bool STRIDED>
__global__ void __launch_bounds__(F * FftPlan<L>::T) __attribute__((amdgpu_waves_per_eu(4)))
rsfde_pass_kernel(const PassArgs a) {
  pass_body<R, L, F, STRIDED, PK_MV>(a, blockIdx.x);
}

// ... and the sine-transform passes (OP_DST, OP_DSD).
template <typename R, int L, int F, bool STRIDED>
__global__ void __launch_bounds__(F * FftPlan<L>::T) __attribute__((amdgpu_waves_per_eu(4)))
rsfde_dst_kernel(const PassArgs a) {
  pass_body<R, L, F, STRIDED, PK_TR>(a, blockIdx.x);
}

// ---- batched passes: one launch covers the same pass of many instances that
// share the transform length and tile shape.  Each instance's arguments sit in
// device memory; the fields that move with the Arnoldi index j are patched in
// the kernel from the launch's j (the basis column read or written, the step of
// the Givens resolve, the status word that stops speculative launches).
// BP_STOP_PEND: passes that run before the step's resolve (the two-sided form's
// right factor) stop on the status of the pending step, or of step j without one.
enum : int { BP_IN_J = 1, BP_OUT_J = 2, BP_GM = 4, BP_STOP = 8, BP_STOP_PEND = 16 };
struct BPass {
  PassArgs a;    // arguments as for Arnoldi step 0
  int64_t ldv;   // basis leading dimension (element offset per step)
  int patch;     // BP_* bits
  int pad;
};
struct BLaunch {
  const BPass* desc;   // per-instance descriptors of this launch, slot order
  const int* start;    // start[s] = first block of slot s; start[ninst] = grid size
  int ninst;
  int j, pend;         // Arnoldi step and pending resolve of this launch
  int mv;              // every slot runs the same op: an operator pass (1) or a sine transform (0)
};

template <typename R, int L, int F, bool STRIDED, int MODE>
__global__ void __launch_bounds__(F * FftPlan<L>::T) __attribute__((amdgpu_waves_per_eu(4)))
rsfde_pass_batched(const BLaunch bl) {
  const int slot = batch_slot(bl.start, bl.ninst, blockIdx.x);
  const BPass& d = bl.desc[slot];
  PassArgs a = d.a;
  const int64_t jo = (int64_t)bl.j * d.ldv;
  if (d.patch & BP_IN_J) a.in_c = (const double*)a.in_c + jo;
  if (d.patch & BP_OUT_J) a.out_a = (double*)a.out_a + jo;
  if (d.patch & BP_GM) {
    a.gm.j = bl.j;
    a.gm.pend = bl.pend;
  }
  if (d.patch & BP_STOP) a.stop_fl = a.stop_fl + bl.j;
  if (d.patch & BP_STOP_PEND) a.stop_fl = a.stop_fl + (bl.pend >= 0 ? bl.pend : bl.j);
  pass_body<R, L, F, STRIDED, MODE>(a, (int64_t)blockIdx.x - bl.start[slot]);
}

// Host launcher for one (precision, length); defined in the per-length
// instantiation units.  Returns a hipError_t.
// ea/eb: when non-null, HIP events stamped at the dispatch's start and end.
template <typename R, int L>
hipError_t launch_pass_L(const PassArgs& a, bool strided, int var, hipStream_t s, hipEvent_t ea,
                         hipEvent_t eb);

template <typename R, int L>
hipError_t launch_pass_batched_L(const BLaunch& bl, int64_t nblocks, bool strided, int var,
                                 hipStream_t s, hipEvent_t ea, hipEvent_t eb);

// Variants of a length: 0 .. 2 run the default radix plan with F, F/2, F/4
// transforms per workgroup, 3 .. 5 the alternative plan (where the length has
// one) with the same three tile widths.
#define RSFDE_PASS_VARIANTS 6

// Workgroup shape of a variant (threads, pencils per tile); 0 threads for a
// variant the length does not have.
template <typename R, int L>
inline void pass_shape(bool strided, int var, int* nt, int* pencils_per_tile) {
#define RSFDE_SHAPE_CASE(LC, V, VI)                                \
  if (var == VI) {                                                 \
    if (strided) {                                                 \
      *nt = PassShape<R, LC, true, V>::NT;                         \
      *pencils_per_tile = 2 * PassShape<R, LC, true, V>::F;        \
    } else {                                                       \
      *nt = PassShape<R, LC, false, V>::NT;                        \
      *pencils_per_tile = 2 * PassShape<R, LC, false, V>::F;       \
    }                                                              \
    return;                                                        \
  }
  RSFDE_SHAPE_CASE(L, 0, 0)
  RSFDE_SHAPE_CASE(L, 1, 1)
  RSFDE_SHAPE_CASE(L, 2, 2)
  if constexpr (HasAltPlan<L>::value) {
    RSFDE_SHAPE_CASE((L | RSFDE_PLAN_ALT), 0, 3)
    RSFDE_SHAPE_CASE((L | RSFDE_PLAN_ALT), 1, 4)
    RSFDE_SHAPE_CASE((L | RSFDE_PLAN_ALT), 2, 5)
  }
#undef RSFDE_SHAPE_CASE
  *nt = 0;
  *pencils_per_tile = 0;
}

// Radices of the plan a variant runs (radix[0..*nstage)); false for a variant the
// length does not have.
template <int L>
inline bool pass_plan(int var, int* code, int* radix, int* nstage) {
  auto fill = [&](auto plan, int c) {
    using P = decltype(plan);
    *code = c;
    *nstage = P::NS;
    for (int k = 0; k < P::NS; ++k) radix[k] = P::R[k];
  };
  if (var >= 0 && var < 3) {
    fill(FftPlan<L>{}, L);
    return true;
  }
  if constexpr (HasAltPlan<L>::value) {
    if (var >= 3 && var < 6) {
      fill(FftPlan<L | RSFDE_PLAN_ALT>{}, L | RSFDE_PLAN_ALT);
      return true;
    }
  }
  return false;
}

// One launch of kernel K<R, LC, F, STRIDED> in the tile shape of tile variant V.
#define RSFDE_LAUNCH_ONE(K, R, LC, V, STR)                                                      \
  {                                                                                             \
    using S = PassShape<R, LC, STR, V>;                                                         \
    if (ea) hipExtLaunchKernelGGL((K<R, LC, S::F, STR>), dim3((unsigned)a.nlaunch), dim3(S::NT),\
                                  0, s, ea, eb, 0, a);                                          \
    else hipLaunchKernelGGL((K<R, LC, S::F, STR>), dim3((unsigned)a.nlaunch), dim3(S::NT), 0, s,\
                            a);                                                                 \
  }

#define RSFDE_LAUNCH_VARIANT(R, LC, V, VI)                                                      \
  if (var == VI) {                                                                              \
    const bool mv = a.op <= OP_MV_LAST;                                                         \
    if (strided) {                                                                              \
      if (mv) RSFDE_LAUNCH_ONE(rsfde_pass_kernel, R, LC, V, true)                               \
      else RSFDE_LAUNCH_ONE(rsfde_dst_kernel, R, LC, V, true)                                   \
    } else {                                                                                    \
      if (mv) RSFDE_LAUNCH_ONE(rsfde_pass_kernel, R, LC, V, false)                              \
      else RSFDE_LAUNCH_ONE(rsfde_dst_kernel, R, LC, V, false)                                  \
    }                                                                                           \
    return hipGetLastError();                                                                   \
  }

#define RSFDE_LAUNCH_BATCHED_ONE(R, LC, V, STR, MODE)                                          \
  {                                                                                             \
    using S = PassShape<R, LC, STR, V>;                                                         \
    hipExtLaunchKernelGGL((rsfde_pass_batched<R, LC, S::F, STR, MODE>), dim3((unsigned)nblocks),\
                          dim3(S::NT), 0, s, ea, eb, 0, bl);                                    \
  }

#define RSFDE_LAUNCH_BATCHED_VARIANT(R, LC, V, VI)                                              \
  if (var == VI) {                                                                              \
    if (strided) {                                                                              \
      if (bl.mv) RSFDE_LAUNCH_BATCHED_ONE(R, LC, V, true, PK_MV)                                \
      else RSFDE_LAUNCH_BATCHED_ONE(R, LC, V, true, PK_TR)                                      \
    } else {                                                                                    \
      if (bl.mv) RSFDE_LAUNCH_BATCHED_ONE(R, LC, V, false, PK_MV)                               \
      else RSFDE_LAUNCH_BATCHED_ONE(R, LC, V, false, PK_TR)                                     \
    }                                                                                           \
    return hipGetLastError();                                                                   \
  }

// Variants 0 .. 2 of plan code LC (returns hipErrorInvalidValue for others).
template <typename R, int LC>
inline hipError_t launch_pass_plan(const PassArgs& a, bool strided, int var, hipStream_t s,
                                   hipEvent_t ea, hipEvent_t eb) {
  RSFDE_LAUNCH_VARIANT(R, LC, 0, 0)
  RSFDE_LAUNCH_VARIANT(R, LC, 1, 1)
  RSFDE_LAUNCH_VARIANT(R, LC, 2, 2)
  return hipErrorInvalidValue;
}
template <typename R, int LC>
inline hipError_t launch_pass_batched_plan(const BLaunch& bl, int64_t nblocks, bool strided,
                                           int var, hipStream_t s, hipEvent_t ea, hipEvent_t eb) {
  RSFDE_LAUNCH_BATCHED_VARIANT(R, LC, 0, 0)
  RSFDE_LAUNCH_BATCHED_VARIANT(R, LC, 1, 1)
  RSFDE_LAUNCH_BATCHED_VARIANT(R, LC, 2, 2)
  return hipErrorInvalidValue;
}
// All six variants of length L (the alternative plan only where L has one).
template <typename R, int L>
inline hipError_t launch_pass_all(const PassArgs& a, bool strided, int var, hipStream_t s,
                                  hipEvent_t ea, hipEvent_t eb) {
  if (var < 3) return launch_pass_plan<R, L>(a, strided, var, s, ea, eb);
  if constexpr (HasAltPlan<L>::value)
    return launch_pass_plan<R, L | RSFDE_PLAN_ALT>(a, strided, var - 3, s, ea, eb);
  return hipErrorInvalidValue;
}
template <typename R, int L>
inline hipError_t launch_pass_batched_all(const BLaunch& bl, int64_t nblocks, bool strided,
                                          int var, hipStream_t s, hipEvent_t ea, hipEvent_t eb) {
  if (var < 3) return launch_pass_batched_plan<R, L>(bl, nblocks, strided, var, s, ea, eb);
  if constexpr (HasAltPlan<L>::value)
    return launch_pass_batched_plan<R, L | RSFDE_PLAN_ALT>(bl, nblocks, strided, var - 3, s, ea, eb);
  return hipErrorInvalidValue;
}

#define RSFDE_INSTANTIATE_PASS(R, L)                                                         \
  template <>                                                                                \
  hipError_t launch_pass_L<R, L>(const PassArgs& a, bool strided, int var, hipStream_t s,   \
                                 hipEvent_t ea, hipEvent_t eb) {                           \
    return launch_pass_all<R, L>(a, strided, var, s, ea, eb);                                \
  }                                                                                          \
  template <>                                                                                \
  hipError_t launch_pass_batched_L<R, L>(const BLaunch& bl, int64_t nblocks, bool strided,  \
                                         int var, hipStream_t s, hipEvent_t ea,             \
                                         hipEvent_t eb) {                                   \
    return launch_pass_batched_all<R, L>(bl, nblocks, strided, var, s, ea, eb);              \
  }
