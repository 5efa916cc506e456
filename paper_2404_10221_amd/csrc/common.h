// Shared device/host helpers of the rsfde library (gfx950 only).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

template <typename R>
struct alignas(2 * sizeof(R)) cpx {
  R x, y;
};

template <typename R>
__host__ __device__ __forceinline__ cpx<R> operator+(cpx<R> a, cpx<R> b) {
  return {a.x + b.x, a.y + b.y};
}
template <typename R>
__host__ __device__ __forceinline__ cpx<R> operator-(cpx<R> a, cpx<R> b) {
  return {a.x - b.x, a.y - b.y};
}
template <typename R>
__host__ __device__ __forceinline__ cpx<R> operator-(cpx<R> a) {
  return {-a.x, -a.y};
}
template <typename R>
__host__ __device__ __forceinline__ cpx<R> operator*(cpx<R> a, R s) {
  return {a.x * s, a.y * s};
}
template <typename R>
__host__ __device__ __forceinline__ cpx<R> cmul(cpx<R> a, cpx<R> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

// Largest restart length the device-side Givens/Hessenberg storage supports.
#define RSFDE_MAX_RESTART 64
// Vectors a Krylov sweep kernel touches at once (CGS2 dots / updates).
#define RSFDE_KCHUNK 8

// ---- batched launches: the slot (instance) of a block from block prefix sums
// Slot of block `bid`: the number of slots s >= 1 with start[s] <= bid (one
// ballot per 64 slots, identical in every wavefront).
__device__ __forceinline__ int batch_slot(const int* __restrict__ start, int n, int bid) {
  int slot = 0;
  const int lane = threadIdx.x & 63;
  for (int base = 0; base < n; base += 64) {
    const int i = base + lane;
    const bool le = i < n && start[i + 1] <= bid;
    slot += __popcll(__ballot(le));
  }
  return __builtin_amdgcn_readfirstlane(slot);
}
