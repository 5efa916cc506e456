// Arnoldi (CGS2) sweeps, cycle start and solution update.
//
// Each sweep writes one partial sum per block and value (value-major, no
// cross-block synchronisation).  The next sweep adds those partials in a fixed
// order in its prologue (every block redundantly; the sum is deterministic),
// so no single-block finish kernel sits between sweeps.
#include <hip/hip_ext.h>
#include <math.h>

#include <type_traits>

#include "krylov.h"

// compile-time loop (constant indices keep per-thread arrays in registers)
template <int C, int Q = 0, typename Fn>
__device__ __forceinline__ void static_for(Fn&& fn) {
  if constexpr (Q < C) {
    fn(std::integral_constant<int, Q>{});
    static_for<C, Q + 1>(fn);
  }
}

// threads per block for a sweep handling up to KM values (sweep A: sums; sweep B:
// basis columns with their coefficients)
template <int W, int KM> struct SweepNT {
  static constexpr int value = W == 2 ? (KM <= 8 ? 1024 : (KM <= 16 ? 512 : 256))
                                      : (KM <= 16 ? 1024 : (KM <= 32 ? 512 : 256));
};

constexpr int ilog2c(int v) { return v <= 1 ? 0 : 1 + ilog2c(v / 2); }

// Wavefront sums of KM values at once by recursive halving: at the step with
// lane offset o, each lane keeps half of its values (the upper half when its
// lane bit o is set) and adds the partner lane's copy of that half; after
// log2(KM) steps lane l holds value l >> (6 - log2 KM), summed over the lanes
// that agree in those top bits, and plain butterflies over the remaining low
// bits finish the sum.  KM - 1 + 6 - log2(KM) shuffles instead of 6 KM; pairs
// add in symmetric order, so every lane holding a value gets the same bits.
template <int KM, int S = 0>
__device__ __forceinline__ void wave_halve(double (&a)[KM], int lane) {
  constexpr int Q = ilog2c(KM);
  if constexpr (S < Q) {
    constexpr int off = 32 >> S;
    constexpr int half = KM >> (S + 1);
    const bool up = (lane & off) != 0;
    static_for<half>([&](auto ic) {
      constexpr int i = decltype(ic)::value;
      const double send = up ? a[i] : a[i + half];
      const double keep = up ? a[i + half] : a[i];
      a[i] = keep + __shfl_xor(send, off, 64);
    });
    wave_halve<KM, S + 1>(a, lane);
  }
}

template <int KM>
__device__ __forceinline__ double wave_sums(double (&a)[KM], int lane) {
  constexpr int Q = ilog2c(KM);
  static_assert((1 << Q) == KM && Q <= 6, "KM must be a power of two <= 64");
  wave_halve<KM>(a, lane);
  double x = a[0];
#pragma unroll
  for (int off = 32 >> Q; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

// Block sums of acc[0..nv) (fixed order); result in res[0..nv) (shared).
template <int KM, int NT>
__device__ __forceinline__ void block_sums(double (&acc)[KM], int nv, double* res) {
  constexpr int NW = NT / 64;
  constexpr int Q = ilog2c(KM);
  __shared__ double sh[NW][KM];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  (void)nv;
  const double x = wave_sums<KM>(acc, lane);
  if ((lane & ((64 >> Q) - 1)) == 0) sh[wv][lane >> (6 - Q)] = x;
  __syncthreads();
  if ((int)threadIdx.x < nv) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) s += sh[w][threadIdx.x];
    res[threadIdx.x] = s;
  }
  __syncthreads();
}

// res[k] = sum over the nb blocks' partials of value k (requires nb <= NT).
template <int KM, int NT>
__device__ __forceinline__ void reduce_partials(const double* __restrict__ part, int nb, int nv,
                                                double* res) {
  double acc[KM];
  const int b = (int)threadIdx.x < nb ? (int)threadIdx.x : 0;
#pragma unroll
  for (int k = 0; k < KM; ++k) {
    const double v = part[(k < nv ? k : 0) * RSFDE_PVS + b];  // all loads in flight together
    acc[k] = ((int)threadIdx.x < nb && k < nv) ? v : 0.0;
  }
  block_sums<KM, NT>(acc, nv, res);
}

// ---- ||v||^2 partials and cycle start -------------------------------------------------
__device__ __forceinline__ void norm_part_body(const double* __restrict__ v0, int64_t n,
                                               double* __restrict__ partial, int bid, int nblk) {
  double acc[1] = {0.0};
  const int64_t stride = (int64_t)nblk * blockDim.x;
  const double2* __restrict__ v2 = (const double2*)v0;
  const int64_t n2 = n >> 1;
  for (int64_t i = (int64_t)bid * blockDim.x + threadIdx.x; i < n2; i += stride) {
    const double2 x = v2[i];
    acc[0] += x.x * x.x + x.y * x.y;
  }
  if ((n & 1) && bid == 0 && threadIdx.x == 0) acc[0] += v0[n - 1] * v0[n - 1];
  __shared__ double res[1];
  block_sums<1, 1024>(acc, 1, res);
  if (threadIdx.x == 0) partial[bid] = res[0];
}

__global__ void __launch_bounds__(1024)
k_norm_part(const double* __restrict__ v0, int64_t n, double* __restrict__ partial) {
  norm_part_body(v0, n, partial, blockIdx.x, gridDim.x);
}

// beta = ||v0||, gamma_0 = beta, vsc[0] = 1/beta, FL[0] = status, FL[1..m] unset
__device__ __forceinline__ void cycle_init_body(const double* __restrict__ partial, int nblocks,
                                                GmresState* st, int first, double rtol,
                                                double inner_rtol, int mixed, int m) {
  __shared__ double res[1];
  reduce_partials<1, 256>(partial, nblocks, 1, res);
  if ((int)threadIdx.x >= 1 && (int)threadIdx.x <= m) st->FL[threadIdx.x] = GM_UNSET;
  if (threadIdx.x == 0) {
    const double beta = sqrt(res[0]);
    GmresSummary& S = st->sum;
    const double beta0 = first ? beta : S.beta0;
    S.beta0 = beta0;
    S.beta = beta;
    S.res = beta;
    S.k = 0;
    S.thr = mixed ? inner_rtol * beta : rtol * beta0;
    st->kfin = 0;
    st->gam[0] = beta;
    st->vsc[0] = beta > 0.0 ? 1.0 / beta : 0.0;
    int flag;
    if (!isfinite(beta)) flag = GM_NONFINITE;
    else if (beta == 0.0 || (!first && beta <= rtol * beta0)) flag = GM_CONVERGED;
    else flag = GM_RUNNING;
    S.flag = flag;
    st->FL[0] = flag;
  }
}

__global__ void __launch_bounds__(256)
k_cycle_init_fin(const double* __restrict__ partial, int nblocks, GmresState* st, int first,
                 double rtol, double inner_rtol, int mixed, int m) {
  cycle_init_body(partial, nblocks, st, first, rtol, inner_rtol, mixed, m);
}

// Basis entries are loaded in chunks of up to 8 columns with no use between the
// loads of a chunk, so a chunk costs one memory latency; columns past nv read
// column nv - 1 (valid memory) and are discarded.
template <int C, typename T>
__device__ __forceinline__ void ld_cols(T (&v)[C], const T* __restrict__ V, int64_t ld, int64_t i,
                                        int k0, int nv) {
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const int k = k0 + c < nv ? k0 + c : nv - 1;
    v[c] = V[k * ld + i];
  }
}

// ---- partials of Vbar^T w (the body of sweep D) -----------------------------------------
template <int KM>
__device__ __forceinline__ void sweepD_body(const KryArgs& a, int bid, int nblk) {
  constexpr int NT = SweepNT<1, KM>::value;
  constexpr int CH = KM < 8 ? KM : 8;
  if (a.st->FL[a.j] != GM_RUNNING) return;
  const int nv = a.j + 1;
  double acc[KM];
#pragma unroll
  for (int k = 0; k < KM; ++k) acc[k] = 0.0;
  const double* __restrict__ w = a.w;
  const double* __restrict__ V = a.V;
  const int64_t stride = (int64_t)nblk * NT;
  const int64_t n2 = a.n >> 1, ld2 = a.ldv >> 1;
  const double2* __restrict__ w2 = (const double2*)w;
  const double2* __restrict__ V2 = (const double2*)V;
  for (int64_t i = (int64_t)bid * NT + threadIdx.x; i < n2; i += stride) {
    const double2 wi = w2[i];
#pragma unroll
    for (int kb = 0; kb < KM; kb += CH)
      if (kb < nv) {
        double2 v[CH];
        ld_cols<CH>(v, V2, ld2, i, kb, nv);
#pragma unroll
        for (int c = 0; c < CH; ++c)
          if (kb + c < nv) acc[kb + c] += v[c].x * wi.x + v[c].y * wi.y;
      }
  }
  if ((a.n & 1) && bid == 0 && threadIdx.x == 0) {
    const int64_t i = a.n - 1;
    const double wi = w[i];
#pragma unroll
    for (int kb = 0; kb < KM; kb += CH)
      if (kb < nv) {
        double v[CH];
        ld_cols<CH>(v, V, a.ldv, i, kb, nv);
#pragma unroll
        for (int c = 0; c < CH; ++c)
          if (kb + c < nv) acc[kb + c] += v[c] * wi;
      }
  }
  __shared__ double res[KM];
  block_sums<KM, NT>(acc, nv, res);
  if ((int)threadIdx.x < nv) a.pa[threadIdx.x * RSFDE_PVS + bid] = res[threadIdx.x];
}


// ---- Arnoldi step j: CGS2 with the second projection delayed by one step ---------------
//
// On entry column j holds u_j, the once-orthogonalised candidate for q_j (scale
// vsc[j] = 1/||u_j||, so qt = vsc[j] Vbar_j has unit norm) and column j+1 holds
// w = K qt (the operator of step j applied to qt).  With Q = [q_0 .. q_{j-1}] final:
//   sweep A   partials of Vbar_k . w and Vbar_k . Vbar_j (k <= j), one pass
//   sweep B   s = Q^T qt, t = Q^T w, tau = qt . w, r = sqrt(|qt|^2 - |s|^2),
//             q_j = (qt - Q s) / r                 (second projection of column j)
//             u_{j+1} = (I - P_{j+1}) w / r = (w - Q (t - c s) - c qt) / r,
//             c = (tau - s.t) / r^2,
//             q_j written over column j, u_{j+1} over w, partials of |u_{j+1}|^2.
// Projecting w and projecting K q_j = (w - K Q s)/r leave the same vector because
// K Q s lies in the span of Q and q_j (Arnoldi relation).  The Hessenberg column j
// is t/r (entries < j) and c (entry j); the terms K Q s / r dropped from it are of
// the size of s, the loss of orthogonality after one projection, as are the
// second-projection coefficients of plain CGS2.  Two sweeps per Arnoldi step
// instead of three, and 2j + 6 vector reads and writes instead of 3j + 7.
// Sweep A holds 2(j+1) sums; past 64 (j >= 32) the sums Vbar_k . Vbar_j come from
// a third sweep (sweep D, the same sums on column j) into the second partial buffer.

// Sweep A: partials of Vbar_k . w (values 0..j) and, for j >= 1, Vbar_k . Vbar_j
// (values j+1 .. 2j+1).
template <int KM>
__device__ __forceinline__ void sweepA_body(const KryArgs& a, int bid, int nblk) {
  constexpr int NT = SweepNT<1, KM>::value;
  constexpr int CH = KM < 8 ? KM : 8;
  if (a.st->FL[a.j] != GM_RUNNING) return;
  const int j = a.j;
  const int nv = j + 1;
  const bool dual = j >= 1 && 2 * nv <= KM;  // (else the column sums come from sweep D)
  const int nvals = dual ? 2 * nv : nv;
  double acc[KM];
#pragma unroll
  for (int k = 0; k < KM; ++k) acc[k] = 0.0;
  const double* __restrict__ w = a.w;
  const double* __restrict__ V = a.V;
  const int64_t stride = (int64_t)nblk * NT;
  const int64_t n2 = a.n >> 1, ld2 = a.ldv >> 1;
  const double2* __restrict__ w2 = (const double2*)w;
  const double2* __restrict__ V2 = (const double2*)V;
  for (int64_t i = (int64_t)bid * NT + threadIdx.x; i < n2; i += stride) {
    const double2 wi = w2[i];
    const double2 uj = V2[(int64_t)j * ld2 + i];
#pragma unroll
    for (int kb = 0; kb < KM; kb += CH)
      if (kb < nv) {
        double2 v[CH];
        ld_cols<CH>(v, V2, ld2, i, kb, nv);
#pragma unroll
        for (int c = 0; c < CH; ++c) {
          const int k = kb + c;
          if (k < nv && k < KM) acc[k] += v[c].x * wi.x + v[c].y * wi.y;
          if (dual && k < nv && KM / 2 + k < KM && k < KM / 2)
            acc[KM / 2 + k] += v[c].x * uj.x + v[c].y * uj.y;
        }
      }
  }
  if ((a.n & 1) && bid == 0 && threadIdx.x == 0) {
    const int64_t i = a.n - 1;
    const double wi = w[i], uj = V[(int64_t)j * a.ldv + i];
#pragma unroll
    for (int k = 0; k < KM; ++k) {
      if (k < nv) {
        const double v = V[(int64_t)k * a.ldv + i];
        acc[k] += v * wi;
        if (dual && k < KM / 2) acc[KM / 2 + k] += v * uj;
      }
    }
  }
  // values 0..j and KM/2 .. KM/2 + j hold the sums; compact them to 0..j, j+1..2j+1
  __shared__ double res[KM];
  block_sums<KM, NT>(acc, KM, res);
  if ((int)threadIdx.x < nvals) {
    const int src = (int)threadIdx.x < nv ? (int)threadIdx.x : KM / 2 + ((int)threadIdx.x - nv);
    a.pa[threadIdx.x * RSFDE_PVS + bid] = res[src];
  }
}

template <int KM>
__global__ void __launch_bounds__((SweepNT<1, KM>::value)) k_sweepA(const KryArgs a) {
  sweepA_body<KM>(a, blockIdx.x, gridDim.x);
}

// Sweep D: partials of Vbar_k . Vbar_j (k <= j) into pb, when sweep A cannot hold both sets.
template <int KM>
__global__ void __launch_bounds__((SweepNT<1, KM>::value)) k_sweepD(const KryArgs a) {
  KryArgs d = a;
  d.w = const_cast<double*>(a.V) + (int64_t)a.j * a.ldv;
  d.pa = a.pb;
  sweepD_body<KM>(d, blockIdx.x, gridDim.x);
}

// Sweep B.  `split`: the sums Vbar_k . Vbar_j are in pb (values 0..j) instead of pa
// (values j+1 .. 2j+1).
template <int KM>
__device__ __forceinline__ void sweepB_body(const KryArgs& a, int bid, int nblk) {
  constexpr int NT = SweepNT<2, KM>::value;
  constexpr int CH = KM < 8 ? KM : 8;
  GmresState* st = a.st;
  if (st->FL[a.j] != GM_RUNNING) return;
  const int j = a.j;
  const int nv = j + 1;  // columns 0 .. j are read
  const bool split = 2 * nv > 64;
  __shared__ double tb[KM], db[KM];
  __shared__ double cfq[KM], cfu[KM];
  __shared__ double invr_s;
  // The thread's first entry pair of w and of the first column chunk is loaded
  // before the prologue (reduction of sweep A's partials, coefficients), so that
  // its memory latency overlaps the prologue instead of following it.
  double* __restrict__ w = a.w;
  double* __restrict__ V = const_cast<double*>(a.V);
  const int64_t stride = (int64_t)nblk * NT;
  const int64_t n2 = a.n >> 1, ld2 = a.ldv >> 1;
  double2* __restrict__ w2 = (double2*)w;
  double2* __restrict__ V2 = (double2*)V;
  const int64_t i0 = (int64_t)bid * NT + threadIdx.x;
  const int64_t ip = i0 < n2 ? i0 : 0;  // (a valid address; unused past the end)
  const double2 w_pre = w2[ip];
  double2 v_pre[CH];
  ld_cols<CH>(v_pre, (const double2*)V2, ld2, ip, 0, nv);
  asm volatile("" ::: "memory");  // (keeps those loads ahead of the prologue's)
  reduce_partials<KM, NT>(a.pa, nblk, nv, tb);
  if (j >= 1)
    reduce_partials<KM, NT>(split ? a.pb : a.pa + (int64_t)nv * RSFDE_PVS, nblk, nv, db);
  if (threadIdx.x < 64) {
    const int k = threadIdx.x;
    const double vj = st->vsc[j];
    const double vk = k <= j ? st->vsc[k] : 0.0;
    const double sk = k < j ? vk * vj * db[k] : 0.0;
    const double tk = k <= j ? vk * tb[k] : 0.0;
    double ss = sk * sk, stt = k < j ? sk * tk : 0.0;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      ss += __shfl_xor(ss, off, 64);
      stt += __shfl_xor(stt, off, 64);
    }
    const double sig = j >= 1 ? vj * vj * db[j] : 1.0;
    const double r = sqrt(fmax(sig - gm_lane(ss, 0), 1e-300));
    const double ir = 1.0 / r;
    const double tau = gm_lane(tk, j < 64 ? j : 0);
    const double c = (tau - gm_lane(stt, 0)) * ir * ir;
    if (k < j) {
      cfq[k] = sk * vk / vj * ir;
      cfu[k] = (tk - c * sk) * vk * ir;
    } else if (k == j) {
      cfu[k] = c * vj * ir;
    }
    if (bid == 0 && k <= j) {
      st->h[k] = k < j ? tk * ir : c;
      st->h2[k] = 0.0;
    }
    if (k == 0) invr_s = ir;
  }
  __syncthreads();
  const double ir = invr_s;
  double acc[1] = {0.0};
  // one entry pair: column chunk 0 comes in v0, the later chunks are loaded here
  auto row = [&](const int64_t i, const double2 wi, const double2 (&v0)[CH]) {
    double2 qn = {0.0, 0.0}, u = {wi.x * ir, wi.y * ir};
#pragma unroll
    for (int kb = 0; kb < KM; kb += CH)
      if (kb < nv) {
        double2 v[CH];
        if (kb == 0) {
#pragma unroll
          for (int cc = 0; cc < CH; ++cc) v[cc] = v0[cc];
        } else {
          ld_cols<CH>(v, (const double2*)V2, ld2, i, kb, nv);
        }
#pragma unroll
        for (int cc = 0; cc < CH; ++cc) {
          const int k = kb + cc;
          if (k < nv) {
            const double fu = cfu[k];
            u.x -= fu * v[cc].x;
            u.y -= fu * v[cc].y;
            const double fq = k < j ? -cfq[k] : ir;
            if (k <= j) {
              qn.x += fq * v[cc].x;
              qn.y += fq * v[cc].y;
            }
          }
        }
      }
    if (j >= 1) V2[(int64_t)j * ld2 + i] = qn;
    w2[i] = u;
    acc[0] += u.x * u.x + u.y * u.y;
  };
  if (i0 < n2) row(i0, w_pre, v_pre);
  for (int64_t i = i0 + stride; i < n2; i += stride) {
    const double2 wi = w2[i];
    double2 v0[CH];
    ld_cols<CH>(v0, (const double2*)V2, ld2, i, 0, nv);
    row(i, wi, v0);
  }
  if ((a.n & 1) && bid == 0 && threadIdx.x == 0) {
    const int64_t i = a.n - 1;
    const double wi = w[i];
    double qn = 0.0, u = wi * ir;
    for (int k = 0; k < nv; ++k) {
      const double v = V[(int64_t)k * a.ldv + i];
      u -= cfu[k] * v;
      qn += (k < j ? -cfq[k] : ir) * v;
    }
    if (j >= 1) V[(int64_t)j * a.ldv + i] = qn;
    w[i] = u;
    acc[0] += u * u;
  }
  __shared__ double res[1];
  block_sums<1, NT>(acc, 1, res);
  if (threadIdx.x == 0) a.pc[bid] = res[0];
}

template <int KM>
__global__ void __launch_bounds__((SweepNT<2, KM>::value)) k_sweepB(const KryArgs a) {
  sweepB_body<KM>(a, blockIdx.x, gridDim.x);
}

// ---- resolve the last launched step; x += V y (or x = V y) when the cycle has finished -------
__device__ __forceinline__ void update_body(const double* __restrict__ V, int64_t ldv, int64_t n,
                                            double* __restrict__ x, const GmRes& g, int bid, int nblk,
                                            bool overwrite) {
  constexpr int MX = RSFDE_MAX_RESTART;
  __shared__ GmOut o;
  __shared__ GmCol col;
  __shared__ double Rs[MX * MX];  // R(i, l) at [l * MX + i], columns l < k
  __shared__ double gs[MX];
  __shared__ double cf[MX];
  gm_prologue(g, &o, &col, bid == 0);
  const int flag = o.flag, k = o.k;
  if (flag == GM_RUNNING || flag == GM_NONFINITE || k <= 0) return;
  // stage the triangular factor and the rotated right-hand side: column k-1 comes
  // from this kernel's resolve when it ran here, the others from the state
  const GmresState* st = g.st;
  const int jr = col.j;
  for (int idx = threadIdx.x; idx < k * MX; idx += blockDim.x) {
    const int l = idx / MX, i = idx - l * MX;
    if (i <= l) Rs[idx] = l == jr ? col.rc[i] : st->Rm[idx];
  }
  for (int i = threadIdx.x; i < k; i += blockDim.x) gs[i] = i == jr ? col.gj : st->gfin[i];
  __syncthreads();
  // back substitution R y = g by columns, one wavefront: lane i holds g_i
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    double gl = lane < k ? gs[lane] : 0.0;
    for (int i = k - 1; i >= 0; --i) {
      const double yi = __shfl(gl, i, 64) / Rs[i * MX + i];
      if (lane < i) gl -= Rs[i * MX + lane] * yi;
      if (lane == i) cf[i] = yi * st->vsc[i];
    }
  }
  __syncthreads();
  const int64_t stride = (int64_t)nblk * blockDim.x;
  const int64_t n2 = n >> 1, ld2 = ldv >> 1;
  double2* __restrict__ x2 = (double2*)x;
  const double2* __restrict__ V2 = (const double2*)V;
  for (int64_t i = (int64_t)bid * blockDim.x + threadIdx.x; i < n2; i += stride) {
    double2 xi = overwrite ? double2{0.0, 0.0} : x2[i];
    for (int lb = 0; lb < k; lb += 8) {
      double2 v[8];
      ld_cols<8>(v, V2, ld2, i, lb, k);
#pragma unroll
      for (int c = 0; c < 8; ++c)
        if (lb + c < k) {
          xi.x += cf[lb + c] * v[c].x;
          xi.y += cf[lb + c] * v[c].y;
        }
    }
    x2[i] = xi;
  }
  if ((n & 1) && bid == 0 && threadIdx.x == 0) {
    double xi = overwrite ? 0.0 : x[n - 1];
    for (int lb = 0; lb < k; lb += 8) {
      double v[8];
      ld_cols<8>(v, V, ldv, n - 1, lb, k);
#pragma unroll
      for (int c = 0; c < 8; ++c)
        if (lb + c < k) xi += cf[lb + c] * v[c];
    }
    x[n - 1] = xi;
  }
}

__global__ void __launch_bounds__(256)
k_update(const double* __restrict__ V, int64_t ldv, int64_t n, double* __restrict__ x,
         const GmRes g, int overwrite) {
  update_body(V, ldv, n, x, g, blockIdx.x, gridDim.x, overwrite != 0);
}

__global__ void k_state_reset(GmresState* st) {
  if (threadIdx.x == 0) {
    st->sum.flag = GM_RUNNING;
    st->sum.k = 0;
    st->sum.beta0 = 0.0;
    st->sum.beta = 0.0;
    st->sum.thr = 0.0;
    st->sum.res = 0.0;
    st->kfin = 0;
  }
  if (threadIdx.x <= RSFDE_MAX_RESTART) st->FL[threadIdx.x] = GM_UNSET;
}

// ---- launchers ---------------------------------------------------------------------------
hipError_t kry_cycle_init(double* v0, int64_t n, int nb, GmresState* st, double* partial, int first,
                          double rtol, double inner_rtol, int mixed, int m, hipStream_t s) {
  hipLaunchKernelGGL(k_norm_part, dim3(nb), dim3(1024), 0, s, v0, n, partial);
  hipLaunchKernelGGL(k_cycle_init_fin, dim3(1), dim3(256), 0, s, partial, nb, st, first, rtol,
                     inner_rtol, mixed, m);
  return hipGetLastError();
}

#define KRY_SWEEP(KERNEL, W, nv, g, a, s)                                                       \
  do {                                                                                          \
    if ((nv) <= 8) hipExtLaunchKernelGGL(KERNEL<8>, g, dim3(SweepNT<W, 8>::value), 0, s, ea, eb, 0, a); \
    else if ((nv) <= 16) hipExtLaunchKernelGGL(KERNEL<16>, g, dim3(SweepNT<W, 16>::value), 0, s, ea, eb, 0, a); \
    else if ((nv) <= 32) hipExtLaunchKernelGGL(KERNEL<32>, g, dim3(SweepNT<W, 32>::value), 0, s, ea, eb, 0, a); \
    else hipExtLaunchKernelGGL(KERNEL<64>, g, dim3(SweepNT<W, 64>::value), 0, s, ea, eb, 0, a);    \
  } while (0)

hipError_t kry_sweep(int which, const KryArgs& a, hipStream_t s, hipEvent_t ea, hipEvent_t eb) {
  const int nv = a.j + 1;
  const dim3 g(a.nb);
  if (which == 1) {
    if (a.j >= 1 && 2 * nv <= 64) {
      KRY_SWEEP(k_sweepA, 1, 2 * nv, g, a, s);
    } else {
      KRY_SWEEP(k_sweepA, 1, nv, g, a, s);  // (j = 0, or the sums over columns split off:)
      if (a.j >= 1) {
        hipEvent_t ea = nullptr, eb = nullptr;
        KRY_SWEEP(k_sweepD, 1, nv, g, a, s);
      }
    }
  } else if (which == 2) {
    KRY_SWEEP(k_sweepB, 2, nv, g, a, s);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t kry_update(const double* V, int64_t ldv, int64_t n, double* x, const GmRes& g,
                      hipStream_t s, hipEvent_t ea, hipEvent_t eb, int overwrite) {
  const int nb = upd_blocks(n);
  hipExtLaunchKernelGGL(k_update, dim3((unsigned)nb), dim3(256), 0, s, ea, eb, 0, V, ldv, n, x, g,
                        overwrite);
  return hipGetLastError();
}

// ---- batched kernels ---------------------------------------------------------------------
__device__ __forceinline__ KryArgs kb_args(const KBatch& d, int j) {
  KryArgs a = d.k;
  a.j = j;
  a.w = d.k.w + (int64_t)j * d.k.ldv;
  return a;
}

template <int W, int KM>
__global__ void __launch_bounds__((SweepNT<W, KM>::value)) k_sweep_b(const KLaunch kl) {
  const int slot = batch_slot(kl.start, kl.ninst, blockIdx.x);
  const KBatch& d = kl.desc[slot];
  const KryArgs a = kb_args(d, kl.j);
  const int bid = (int)blockIdx.x - kl.start[slot];
  if constexpr (W == 1) {
    sweepA_body<KM>(a, bid, d.nb);
  } else if constexpr (W == 3) {
    KryArgs dd = a;  // sums of the columns with column j, into pb (j >= 32)
    dd.w = const_cast<double*>(a.V) + (int64_t)a.j * a.ldv;
    dd.pa = a.pb;
    sweepD_body<KM>(dd, bid, d.nb);
  } else {
    sweepB_body<KM>(a, bid, d.nb);
  }
}

__global__ void __launch_bounds__(256) k_update_b(const KLaunch kl) {
  const int slot = batch_slot(kl.start, kl.ninst, blockIdx.x);
  if (kl.mask && kl.mask[slot] == 0) return;  // this instance's update was added earlier
  const KBatch& d = kl.desc[slot];
  GmRes g;
  g.st = d.k.st;
  g.p3 = d.k.pc;
  g.nb3 = d.nb;
  g.j = kl.j;
  g.pend = kl.pend;
  g.m = d.k.m;
  update_body(d.k.V, d.k.ldv, d.k.n, d.x, g, (int)blockIdx.x - kl.start[slot], d.nbu, d.overwrite != 0);
}

__global__ void __launch_bounds__(1024) k_norm_part_b(const KLaunch kl) {
  const int slot = batch_slot(kl.start, kl.ninst, blockIdx.x);
  const KBatch& d = kl.desc[slot];
  norm_part_body(d.k.V, d.k.n, d.partial, (int)blockIdx.x - kl.start[slot], d.nb);
}

__global__ void __launch_bounds__(256) k_cycle_init_fin_b(const KLaunch kl) {
  const KBatch& d = kl.desc[blockIdx.x];
  cycle_init_body(d.partial, d.nb, d.k.st, kl.first, d.rtol, d.inner_rtol, d.mixed, d.k.m);
}

#define KRY_SWEEP_B(W, nv, g, kl, s)                                                              \
  do {                                                                                            \
    if ((nv) <= 8) hipExtLaunchKernelGGL((k_sweep_b<W, 8>), g, dim3(SweepNT<W, 8>::value), 0, s, ea, eb, 0, kl); \
    else if ((nv) <= 16) hipExtLaunchKernelGGL((k_sweep_b<W, 16>), g, dim3(SweepNT<W, 16>::value), 0, s, ea, eb, 0, kl); \
    else if ((nv) <= 32) hipExtLaunchKernelGGL((k_sweep_b<W, 32>), g, dim3(SweepNT<W, 32>::value), 0, s, ea, eb, 0, kl); \
    else hipExtLaunchKernelGGL((k_sweep_b<W, 64>), g, dim3(SweepNT<W, 64>::value), 0, s, ea, eb, 0, kl); \
  } while (0)

hipError_t kry_sweep_batched(int which, const KLaunch& kl, int64_t nblocks, hipStream_t s,
                             hipEvent_t ea, hipEvent_t eb) {
  const int nv = kl.j + 1;
  const dim3 g((unsigned)nblocks);
  if (which == 1) {
    if (kl.j >= 1 && 2 * nv <= 64) {
      KRY_SWEEP_B(1, 2 * nv, g, kl, s);
    } else {
      KRY_SWEEP_B(1, nv, g, kl, s);
      if (kl.j >= 1) {
        hipEvent_t ea = nullptr, eb = nullptr;
        KRY_SWEEP_B(3, nv, g, kl, s);
      }
    }
  } else if (which == 2) {
    KRY_SWEEP_B(2, nv, g, kl, s);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t kry_update_batched(const KLaunch& kl, int64_t nblocks, hipStream_t s, hipEvent_t ea,
                              hipEvent_t eb) {
  hipExtLaunchKernelGGL(k_update_b, dim3((unsigned)nblocks), dim3(256), 0, s, ea, eb, 0, kl);
  return hipGetLastError();
}

hipError_t kry_norm_batched(const KLaunch& kl, int64_t nblocks, hipStream_t s) {
  hipLaunchKernelGGL(k_norm_part_b, dim3((unsigned)nblocks), dim3(1024), 0, s, kl);
  return hipGetLastError();
}

__global__ void k_gather_sum(const KBatch* __restrict__ desc, int n, GmresSummary* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = desc[i].k.st->sum;
}

hipError_t kry_gather_summaries(const KBatch* desc, int n, GmresSummary* out, hipStream_t s) {
  hipLaunchKernelGGL(k_gather_sum, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, s, desc, n, out);
  return hipGetLastError();
}

hipError_t kry_cycle_fin_batched(const KLaunch& kl, hipStream_t s) {
  hipLaunchKernelGGL(k_cycle_init_fin_b, dim3((unsigned)kl.ninst), dim3(256), 0, s, kl);
  return hipGetLastError();
}

hipError_t kry_state_reset(GmresState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_state_reset, dim3(1), dim3(128), 0, s, st);
  return hipGetLastError();
}
