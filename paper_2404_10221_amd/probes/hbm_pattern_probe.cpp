// HBM access-pattern probe for gfx950 (not part of the library).  It times, with
// HIP events, kernels that only move data in the patterns of the pencil passes,
// to give each pass a ceiling that has no transform in it:
//  * strided tiles: a workgroup of NT threads loads a tile of W adjacent pencils
//    (rows of W * 8 bytes) x N positions along an axis of element stride `inner`
//    (all loads issued first, as in the passes) and stores it to the same places
//    of a second array; tile order plain or XCD-aware (block b takes tile
//    (b mod 8) * ceil(tiles / 8) + b / 8);
//  * a streaming copy in 32 KiB chunks after another copy that wrote its input,
//    in the same chunk order or reversed (does the second pass find the end of the
//    first one's output in the Infinity Cache?).
// Build: hipcc --offload-arch=gfx950 -O3 -o hbm_pattern_probe hbm_pattern_probe.cpp
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <vector>

#define CK(x)                                                                        \
  do {                                                                               \
    hipError_t e_ = (x);                                                             \
    if (e_ != hipSuccess) {                                                          \
      printf("HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__);         \
      return 1;                                                                      \
    }                                                                                \
  } while (0)

// ---- strided tiles ----------------------------------------------------------
template <int W, int NT, int NE>
__global__ void __launch_bounds__(NT) tile_copy(const double* __restrict__ x, double* __restrict__ y, int N,
                                                long inner, long tiles_inner, long ntiles, int xcd) {
  long tile = blockIdx.x;
  if (xcd) {
    const long tpx = (ntiles + 7) >> 3;
    tile = (tile & 7) * tpx + (tile >> 3);
  }
  if (tile >= ntiles) return;
  const long o = tile / tiles_inner;
  const long pin0 = (tile - o * tiles_inner) * W;
  const long rem = inner - pin0;
  const int nvalid = rem < W ? (int)rem : W;
  const long gbase = o * (long)N * inner + pin0;
  double v[NE];
#pragma unroll
  for (int i = 0; i < NE; ++i) {  // clamped addresses: every slot loads in bounds
    const int flat = threadIdx.x + i * NT;
    const int p = flat / W, pp = flat - p * W;
    v[i] = x[gbase + (long)(p < N ? p : 0) * inner + (pp < nvalid ? pp : 0)];
  }
#pragma unroll
  for (int i = 0; i < NE; ++i) {
    const int flat = threadIdx.x + i * NT;
    const int p = flat / W, pp = flat - p * W;
    if (p < N && pp < nvalid) y[gbase + (long)p * inner + pp] = v[i] * 1.0000001;
  }
}

template <int W, int NT>
int run_tiles(const char* name, double* x, double* y, int N, long inner, long outer) {
  constexpr int NE = (512 * W + NT - 1) / NT;  // N <= 512
  if ((long)N * W > (long)NE * NT) return 1;
  const long tiles_inner = (inner + W - 1) / W;
  const long ntiles = tiles_inner * outer;
  const long nlaunch = (ntiles + 7) / 8 * 8;
  hipEvent_t e0, e1;
  CK(hipEventCreate(&e0));
  CK(hipEventCreate(&e1));
  for (int xcd = 0; xcd < 2; ++xcd) {
    std::vector<float> t;
    for (int rep = 0; rep < 9; ++rep) {
      tile_copy<W, NT, NE><<<nlaunch, NT>>>(y, x, N, inner, tiles_inner, ntiles, xcd);
      CK(hipEventRecord(e0));
      tile_copy<W, NT, NE><<<nlaunch, NT>>>(x, y, N, inner, tiles_inner, ntiles, xcd);
      CK(hipEventRecord(e1));
      CK(hipEventSynchronize(e1));
      float ms;
      CK(hipEventElapsedTime(&ms, e0, e1));
      t.push_back(ms);
    }
    std::sort(t.begin(), t.end());
    const double bytes = 2.0 * 8.0 * (double)N * inner * outer;
    printf("tiles %-12s W=%2d (%3d B rows) NT=%d %s: %8.1f us  %.2f TB/s\n", name, W, W * 8, NT,
           xcd ? "XCD-aware" : "plain    ", t[4] * 1e3, bytes / (t[4] * 1e-3) / 1e12);
    fflush(stdout);
  }
  CK(hipEventDestroy(e0));
  CK(hipEventDestroy(e1));
  return 0;
}

// ---- chunked streaming copy, forward or reversed ----------------------------
constexpr int CNT = 256, CPER = 8;  // one chunk: CNT * CPER 16-byte values
__global__ void __launch_bounds__(CNT) chunk_copy(const double2* __restrict__ a, double2* __restrict__ b, long nch,
                                                  int rev) {
  long c = blockIdx.x;
  if (c >= nch) return;
  if (rev) c = nch - 1 - c;
  const long base = c * (CNT * CPER);
  double2 v[CPER];
#pragma unroll
  for (int i = 0; i < CPER; ++i) v[i] = a[base + i * CNT + threadIdx.x];
#pragma unroll
  for (int i = 0; i < CPER; ++i) b[base + i * CNT + threadIdx.x] = v[i];
}

int main() {
  for (int n : {255, 511}) {
    const long tot = (long)n * n * n;
    double *x, *y;
    CK(hipMalloc(&x, tot * 8));
    CK(hipMalloc(&y, tot * 8));
    CK(hipMemset(x, 0, tot * 8));
    CK(hipMemset(y, 0, tot * 8));
    char nm[64];
    for (int ax = 2; ax <= 3; ++ax) {  // axis 2: stride n, n planes; axis 3: stride n^2
      const long inner = ax == 2 ? n : (long)n * n, outer = ax == 2 ? n : 1;
      snprintf(nm, sizeof nm, "%d^3 ax%d", n, ax);
      if (run_tiles<8, 256>(nm, x, y, n, inner, outer)) return 1;
      if (run_tiles<16, 512>(nm, x, y, n, inner, outer)) return 1;
      if (run_tiles<32, 512>(nm, x, y, n, inner, outer)) return 1;
    }
    CK(hipFree(x));
    CK(hipFree(y));
  }
  for (long mb : {64L, 128L, 192L, 256L, 1024L}) {
    const long n2 = mb * 1024 * 1024 / 16, nch = n2 / (CNT * CPER);
    double2 *x, *y, *z;
    CK(hipMalloc(&x, n2 * 16));
    CK(hipMalloc(&y, n2 * 16));
    CK(hipMalloc(&z, n2 * 16));
    CK(hipMemset(x, 0, n2 * 16));
    CK(hipMemset(y, 0, n2 * 16));
    CK(hipMemset(z, 0, n2 * 16));
    hipEvent_t e0, e1;
    CK(hipEventCreate(&e0));
    CK(hipEventCreate(&e1));
    std::vector<float> t[2];
    for (int rep = 0; rep < 12; ++rep)
      for (int rev = 0; rev < 2; ++rev) {
        chunk_copy<<<nch, CNT>>>(x, y, nch, 0);
        CK(hipEventRecord(e0));
        chunk_copy<<<nch, CNT>>>(y, z, nch, rev);
        CK(hipEventRecord(e1));
        CK(hipEventSynchronize(e1));
        float ms;
        CK(hipEventElapsedTime(&ms, e0, e1));
        t[rev].push_back(ms);
      }
    for (auto& v : t) std::sort(v.begin(), v.end());
    const double bytes = 2.0 * n2 * 16;
    printf("copy after copy %5ld MiB: same order %.1f us (%.2f TB/s), reversed %.1f us (%.2f TB/s)\n", mb,
           t[0][6] * 1e3, bytes / (t[0][6] * 1e-3) / 1e12, t[1][6] * 1e3, bytes / (t[1][6] * 1e-3) / 1e12);
    fflush(stdout);
    CK(hipEventDestroy(e0));
    CK(hipEventDestroy(e1));
    CK(hipFree(x));
    CK(hipFree(y));
    CK(hipFree(z));
  }
  printf("hbm pattern probe done\n");
  return 0;
}
